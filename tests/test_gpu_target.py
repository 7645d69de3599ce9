"""Parity at the target sizes, over a whole refresh period.

* 160-orbital H-chain-like system (80 + 80 electrons, eps = 1e-5, 8192
  walkers): after 100 moves of burn-in, 56 more moves cross a re-inversion
  (in the sweep for general orbitals, in the refresh kernel for spin-blocked
  ones).  Sixteen sampled walkers are followed teacher-forced: the oracle
  evaluates every state the GPU visited (E_L before each move, t, the pick)
  and the states the sweep ends on.  FP64: |dE_L| within 1e-10 + 1e-13 T,
  picks identical.  Mixed: within 1e-6 per electron plus 1e-8 T, and the
  residence-time weighted error (the energy's) within 1e-6 per electron.
* 10 x 10 Hubbard lattice, mixed form, general and spin-blocked orbitals:
  moves 40-49 after a fresh inversion and the state after move 50.
* Batch of the 40/80/160-orbital systems in the mixed form: equal to separate
  launches, and E_L against the oracle 49 moves after the inversion.
Section "Local energy and Gradient ratios" (the Sherman-Morrison updates and
the FP32 form of R) and Eq. eloc:hci.
"""
import os

import numpy as np
import pytest

from oracle.core import ORC_LEMMA, OracleSystem
from workloads import make_config

from gpu_common import (MIXED_TOL, ST_STALE, el_tol, field, gpu_system, mixed_tol, occ_of, run_sweep,
                        teacher_forced_batch)

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def orc160():
    wl = make_config("hchain160", n_walkers=1)
    return OracleSystem.from_workload(wl)


def _mixed_report(res, n_elec):
    dE, T = res["dE"], res["T"]
    t = 1.0 / T
    weighted = float(np.sum(t * dE) / np.sum(t)) / n_elec
    plain = float(np.mean(dE <= MIXED_TOL * n_elec))
    return weighted, plain


@pytest.mark.timeout(900)
@pytest.mark.parametrize("orbitals,prec", [("ghf", "fp64"), ("ghf", "mixed"), ("uhf", "mixed")])
def test_hchain160_teacher_forced_across_reinversion(torch, orc160, orbitals, prec):
    from paper_1807_10633_amd.vmc import VMC_FP64, VMC_MIXED, vmc_local_energy

    W, burn, steps, sample = 8192, 100, 56, 16
    wl = make_config("hchain160", n_walkers=W, orbitals=orbitals)
    _say(f"[hchain160 {orbitals} {prec}] W={W} burn={burn} steps={steps} sample={sample}")
    sysm = gpu_system(wl, precision=VMC_MIXED if prec == "mixed" else VMC_FP64)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, burn)
    occ0 = occ_of(sysm, walkers)
    step0 = walkers.step
    eh, th, ph = run_sweep(sysm, walkers, steps)
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    el_end = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    assert np.all((st & ~ST_STALE) == 0)
    orc160.set_params(wl.jastrow, wl.theta)
    idx = np.unique(np.linspace(0, W - 1, sample).astype(int))
    res = teacher_forced_batch(orc160, wl.ctmc_seed, occ0, step0, eh, th, ph, idx, el_final=el_end,
                               threads=THREADS)
    dE, T, k = res["dE"], res["T"], res["k"]
    late = (k >= 40) & (k < 50)
    _say(f"    states {res['states']}, max |dE| {dE.max():.3g} (moves 40-49: {dE[late].max():.3g}), median T "
         f"{np.median(T):.3g}, picks compared {res['picks_compared']}, exempt {res['picks_exempt']}, "
         f"mismatches {len(res['mismatches'])}")
    assert res["states"] == idx.size * (steps + 1)
    if prec == "fp64":
        scaled = dE / el_tol(T)
        _say(f"    max |dE|/tol {scaled.max():.3g}, max rel dt {res['dt_rel'].max():.3g}")
        assert scaled.max() <= 1.0
        assert res["dt_rel"].max() <= 1e-10
        assert not res["mismatches"], res["mismatches"][:5]
        assert res["picks_compared"] > 0.99 * idx.size * steps
    else:
        scaled = dE / mixed_tol(T, wl.n_elec)
        weighted, plain = _mixed_report(res, wl.n_elec)
        _say(f"    max |dE|/N_e {dE.max() / wl.n_elec:.3g}, max scaled {scaled.max():.3g}, t-weighted |dE|/N_e "
             f"{weighted:.3g}, states within 1e-6/N_e {plain:.4f}")
        assert scaled.max() <= 1.0
        assert weighted <= MIXED_TOL


@pytest.mark.parametrize("orbitals", ["ghf", "uhf"])
def test_hubbard10x10_mixed_full_refresh_period(torch, orbitals):
    from paper_1807_10633_amd.vmc import VMC_MIXED, vmc_local_energy, vmc_walkers_refresh

    W, burn, steps, sample = 16384, 60, 50, 8
    wl = make_config("hubbard10x10", n_walkers=W, orbitals=orbitals)
    _say(f"[hubbard10x10 {orbitals} mixed] W={W} moves 40-49 and 50 after a fresh inversion")
    sysm = gpu_system(wl, precision=VMC_MIXED)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, burn)
    vmc_walkers_refresh(sysm.handle, walkers)  # fresh inverses: the next 50 moves run on them
    occ0 = occ_of(sysm, walkers)
    step0 = walkers.step
    eh, th, ph = run_sweep(sysm, walkers, steps)
    assert walkers.since_inv == steps
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    el_end = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    orc = OracleSystem.from_workload(wl)
    idx = np.unique(np.linspace(0, W - 1, sample).astype(int))
    res = teacher_forced_batch(orc, wl.ctmc_seed, occ0, step0, eh, th, ph, idx, k_range=range(40, 50),
                               el_final=el_end, threads=THREADS)
    dE, T = res["dE"], res["T"]
    weighted, plain = _mixed_report(res, wl.n_elec)
    _say(f"    states {res['states']}, max |dE|/N_e {dE.max() / wl.n_elec:.3g}, median T {np.median(T):.3g}, "
         f"t-weighted |dE|/N_e {weighted:.3g}, within 1e-6/N_e {plain:.4f}")
    assert res["states"] == idx.size * 11
    assert np.all(dE <= mixed_tol(T, wl.n_elec))
    assert weighted <= MIXED_TOL


def test_batch_mixed_equals_separate_and_matches_oracle(torch):
    from paper_1807_10633_amd.vmc import (VMC_MIXED, vmc_batch_create, vmc_batch_ctmc_step, vmc_batch_destroy,
                                          vmc_batch_local_energy, vmc_ctmc_step, vmc_local_energy)

    names, Wb = ("hchain40", "hchain80", "hchain160"), 256
    wls = [make_config(n, n_walkers=Wb) for n in names]
    systems = [gpu_system(wl, precision=VMC_MIXED) for wl in wls]
    _say(f"[batch mixed] {names} x {Wb}")
    sep = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    bat = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    for s, wk in zip(systems, sep):
        vmc_ctmc_step(s.handle, wk, 3)
        vmc_local_energy(s.handle, wk)
    b = vmc_batch_create([s.handle for s in systems])
    try:
        vmc_batch_ctmc_step(b, bat, 3)
        vmc_batch_local_energy(b, bat)
        torch.cuda.synchronize()
        for s, a, c in zip(systems, sep, bat):
            for f, dt, per in (("eloc", torch.float64, 1), ("pick", torch.int64, 1), ("ainv", torch.float64, s.ne ** 2),
                               ("r", torch.float32, s.ne * s.n_so)):
                assert np.array_equal(field(s, a, f, dt, per), field(s, c, f, dt, per)), f
            assert np.array_equal(occ_of(s, a), occ_of(s, c))
        # 46 more moves: 49 updates since the inversion of vmc_walkers_init
        vmc_batch_ctmc_step(b, bat, 46)
        vmc_batch_local_energy(b, bat)
    finally:
        vmc_batch_destroy(b)
    torch.cuda.synchronize()
    for wl, s, wk in zip(wls, systems, bat):
        el = field(s, wk, "eloc", torch.float64, 1)[:, 0]
        occ = occ_of(s, wk)
        orc = OracleSystem.from_workload(wl)
        idx = np.arange(0, Wb, Wb // 8)
        e_o, T_o, _, st = orc.local_energy_batch(occ[idx], ORC_LEMMA, THREADS)
        assert np.all(st == 0)
        d = np.abs(el[idx] - e_o)
        _say(f"    {wl.name}: max |dE|/N_e {d.max() / wl.n_elec:.3g}, max scaled "
             f"{np.max(d / mixed_tol(T_o, wl.n_elec)):.3g}")
        assert np.all(d <= mixed_tol(T_o, wl.n_elec))
