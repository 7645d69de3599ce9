"""Spin-blocked (unrestricted) orbitals on the GPU, through the C ABI.

With VMC_UHF the library keeps R per slot over its own spin's n orbitals only,
B block diagonal, forms an opposite-spin double as the product of the two
spins' ratios, and updates only the blocks of the spin that moves (section
"Local energy and Gradient ratios", Eq. eq:R; the unrestricted determinant of
the sections "Performance of the optimizer" and "2-D Hubbard Model Benchmark").
The oracle is the same general-orbital oracle as everywhere, given the
spin-blocked theta: every result is compared with it as for the general form.
"""
import numpy as np
import pytest

from oracle.core import ORC_LEMMA, OracleSystem, list_to_occ
from workloads import make_config

from gpu_common import EL_TOL, el_tol, field, gpu_system, mixed_tol, occ_of, run_sweep, teacher_forced_check

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-6  # per electron


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(*a):
    print(*a, flush=True)


def _uhf(name, W, **kw):
    return make_config(name, n_walkers=W, orbitals="uhf", **kw)


@pytest.mark.parametrize("name,W,burn,steps,sample", [("hubbard8", 64, 0, 120, 16), ("hchain20", 512, 20, 60, 8),
                                                      ("hubbard10x10", 16384, 0, 3, 3)])
def test_uhf_ctmc_teacher_forced(torch, name, W, burn, steps, sample):
    """FP64: E_L, t and the pick of every step against the oracle, across
    re-inversions (every 50 moves)."""
    from paper_1807_10633_amd.vmc import vmc_launch_info

    wl = _uhf(name, W)
    _say(f"[uhf ctmc] {name} W={W} burn={burn} steps={steps} sample={sample}")
    sysm = gpu_system(wl)
    info = vmc_launch_info(sysm.handle)
    assert not info["state_in_lds"] and info["refresh_kernel"]
    walkers = sysm.walkers(wl.occ)
    if burn:
        run_sweep(sysm, walkers, burn)
    occ0 = occ_of(sysm, walkers)
    step0 = walkers.step
    eh, th, ph = run_sweep(sysm, walkers, steps)
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    assert np.all((st & 1) == 0)
    orc = OracleSystem.from_workload(wl)
    idx = np.unique(np.linspace(0, W - 1, sample).astype(int))
    res = teacher_forced_check(orc, wl.ctmc_seed, occ0, step0, eh, th, ph, idx)
    _say("    " + str({k: v for k, v in res.items() if k not in ("dE_all", "T_all")}))
    scaled = res["dE_all"] / (el_tol(res["T_all"]))
    assert scaled.max() <= 1.0, res["max_dE"]
    assert res["max_dt_rel"] <= 1e-10, res
    assert not res["mismatches"], res["mismatches"][:5]
    assert res["picks_compared"] > 0.99 * len(idx) * steps


@pytest.mark.parametrize("na,nb", [(5, 2), (3, 0), (0, 4)])
def test_uhf_uneven_spins(torch, na, nb):
    """Spin blocks of different sizes, one of them possibly empty (10-site
    ring, U = 4): E_L, t and picks against the oracle over 70 moves (one
    re-inversion of each block on the way)."""
    from workloads import Workload, hubbard_ring, init_jastrow, init_theta, init_walkers, spin_blocked

    L, W = 10, 48
    h1, ei, ev = hubbard_ring(L, 1.0, 4.0)
    wl = Workload(name=f"ring{L}_{na}_{nb}", n_orb=L, n_alpha=na, n_beta=nb, h1=h1, eri_idx=ei, eri_val=ev, eps=0.0,
                  theta=spin_blocked(init_theta(h1, na, nb, 0.05, 5), L, na, nb), jastrow=init_jastrow(2 * L, 0.05, 5),
                  occ=init_walkers(L, na, nb, W, 6), ctmc_seed=7, orbitals="uhf")
    _say(f"[uhf uneven] ring10 {na}+{nb}")
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    occ0 = occ_of(sysm, walkers)
    eh, th, ph = run_sweep(sysm, walkers, 70)
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    assert np.all((st & 1) == 0)
    orc = OracleSystem.from_workload(wl)
    res = teacher_forced_check(orc, wl.ctmc_seed, occ0, 0, eh, th, ph, range(0, W, 6))
    scaled = res["dE_all"] / (el_tol(res["T_all"]))
    assert scaled.max() <= 1.0 and not res["mismatches"], res["mismatches"][:3]


def test_uhf_state_after_updates(torch):
    """After 37 moves without re-inversion: B equals a fresh inverse of
    theta[N] in slot order and is exactly block diagonal, slots [0, na) hold
    the alpha electrons, and the stored R (own spin only) equals theta B."""
    wl = _uhf("hchain20", 64)
    sysm = gpu_system(wl, refresh_period=1000)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, 37)
    n, na, ne, n_so = wl.n_orb, wl.n_alpha, wl.n_elec, wl.n_so
    slot = field(sysm, walkers, "slot_orb", torch.int32, ne)
    B = field(sysm, walkers, "ainv", torch.float64, ne * ne)
    R = field(sysm, walkers, "r", torch.float64, ne * n)
    worst_b = worst_r = 0.0
    for w in range(64):
        assert np.all(slot[w][:na] < n) and np.all(slot[w][na:] >= n)
        A = wl.theta[slot[w]][:, :ne]
        Binv = np.linalg.inv(A)  # Binv[x, p]
        Bg = B[w].reshape(ne, ne).T  # stored column by slot
        assert np.all(Bg[:na, na:] == 0.0) and np.all(Bg[na:, :na] == 0.0)
        worst_b = max(worst_b, np.max(np.abs(Bg - Binv)) / np.max(np.abs(Binv)))
        Rf = wl.theta[:, :ne] @ Binv  # R[a, p] over every orbital
        Rg = R[w].reshape(ne, n)  # row p: orbitals of p's spin
        own = np.concatenate([Rf[:n, :na].T, Rf[n:, na:].T], axis=0)
        worst_r = max(worst_r, np.max(np.abs(Rg - own)) / np.max(np.abs(own)))
        # the entries the layout leaves out are zero
        assert np.max(np.abs(Rf[n:, :na])) <= 1e-12 and np.max(np.abs(Rf[:n, na:])) <= 1e-12
    _say(f"    37 updates: max rel |dB| {worst_b:.2e}, |dR| {worst_r:.2e}")
    assert worst_b < 1e-9 and worst_r < 1e-9


def test_uhf_agrees_with_general_form_on_the_same_theta(torch):
    """The same spin-blocked theta run in both forms: E_L and t of the same
    states agree to the FP64 bar."""
    from paper_1807_10633_amd.vmc import VMC_GHF, vmc_local_energy

    wl = _uhf("hchain20", 256)
    u = gpu_system(wl)
    g = gpu_system(wl, orbitals=VMC_GHF)
    wu = u.walkers(wl.occ)
    run_sweep(u, wu, 30)
    occ = occ_of(u, wu)
    wg = g.walkers(occ)
    vmc_local_energy(u.handle, wu)
    vmc_local_energy(g.handle, wg)
    torch.cuda.synchronize()
    eu = field(u, wu, "eloc", torch.float64, 1)[:, 0]
    eg = field(g, wg, "eloc", torch.float64, 1)[:, 0]
    tu = field(u, wu, "tres", torch.float64, 1)[:, 0]
    tg = field(g, wg, "tres", torch.float64, 1)[:, 0]
    T = 1.0 / tg
    assert np.all(np.abs(eu - eg) <= el_tol(T))
    assert np.all(np.abs(tu - tg) <= 1e-10 * tg)


@pytest.mark.parametrize("name,W,burn,steps,sample", [("hchain20", 512, 20, 60, 6), ("hubbard10x10", 2048, 0, 4, 2)])
def test_uhf_mixed_trajectory(torch, name, W, burn, steps, sample):
    """Mixed form (FP32 R): E_L of every visited state within 1e-6 per electron
    (plus 1e-9 T near nodes), picks mostly identical."""
    from paper_1807_10633_amd.vmc import VMC_MIXED

    wl = _uhf(name, W)
    _say(f"[uhf mixed] {name} W={W} burn={burn} steps={steps}")
    sysm = gpu_system(wl, precision=VMC_MIXED)
    walkers = sysm.walkers(wl.occ)
    if burn:
        run_sweep(sysm, walkers, burn)
    occ0 = occ_of(sysm, walkers)
    step0 = walkers.step
    eh, th, ph = run_sweep(sysm, walkers, steps)
    orc = OracleSystem.from_workload(wl)
    idx = np.unique(np.linspace(0, W - 1, sample).astype(int))
    res = teacher_forced_check(orc, wl.ctmc_seed, occ0, step0, eh, th, ph, idx)
    n_all = res["picks_compared"] + res["picks_exempt"]
    dE, T = res["dE_all"], res["T_all"]
    scaled = dE / (mixed_tol(T, wl.n_elec))
    _say(f"    max |dE| {res['max_dE']:.3g}, max scaled {scaled.max():.3g}, "
         f"pick agreement {1 - len(res['mismatches']) / max(1, n_all):.4f}")
    assert scaled.max() <= 1.0
    assert len(res["mismatches"]) <= 0.01 * n_all


def test_uhf_gradient_ratios(torch):
    """O_k against the oracle; the theta entries outside the spin blocks have
    exactly zero gradient, so AMSGrad never moves them."""
    from paper_1807_10633_amd.vmc import vmc_logderiv

    wl = _uhf("hchain20", 32)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, 23)
    O = torch.zeros((32, sysm.n_params), dtype=torch.float64, device="cuda")
    vmc_logderiv(sysm.handle, walkers, None, O)
    torch.cuda.synchronize()
    O = O.cpu().numpy()
    occ = occ_of(sysm, walkers)
    orc = OracleSystem.from_workload(wl)
    n, na, ne, n_so = wl.n_orb, wl.n_alpha, wl.n_elec, wl.n_so
    nj = n_so * (n_so + 1) // 2
    off = np.zeros((n_so, n_so), dtype=bool)
    off[:n, na:ne] = True
    off[n:, :na] = True
    for w in range(32):
        ref = orc.logderiv(occ[w])
        assert np.array_equal(O[w, :nj], ref[:nj])
        scale = np.max(np.abs(ref[nj:]))
        assert np.max(np.abs(O[w, nj:] - ref[nj:])) <= 1e-10 * scale
        assert np.all(O[w, nj:].reshape(n_so, n_so)[off] == 0.0)


def test_uhf_wrong_alpha_count_is_flagged(torch):
    """A determinant with 11 alpha and 9 beta electrons has no place in the
    spin-blocked layout: flagged SINGULAR, never moved; the others are fine."""
    from paper_1807_10633_amd.vmc import vmc_local_energy

    wl = _uhf("hchain20", 8)
    occ = wl.occ.copy()
    n = wl.n_orb
    orbs = [p for p in range(wl.n_so) if (int(occ[3][0]) >> p) & 1]
    beta = [p for p in orbs if p >= n]
    free_alpha = [p for p in range(n) if p not in orbs]
    orbs.remove(beta[0])
    orbs.append(free_alpha[0])
    occ[3] = list_to_occ(orbs, wl.n_so)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(occ)
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    assert st[3] & 1 and np.isnan(el[3])
    good = [w for w in range(8) if w != 3]
    assert np.all((st[good] & 1) == 0) and np.all(np.isfinite(el[good]))
    before = occ_of(sysm, walkers)
    eh, th, ph = run_sweep(sysm, walkers, 10)
    assert np.array_equal(before[3], occ_of(sysm, walkers)[3]) and np.all(ph[:, 3] == 0)
    orc = OracleSystem.from_workload(wl)
    after = occ_of(sysm, walkers)
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    for w in good[:3]:
        r = orc.local_energy(after[w], ORC_LEMMA, with_candidates=False)
        assert abs(el[w] - r["eloc"]) <= el_tol(r["T"])


def test_uhf_optimizer_keeps_the_spin_blocks(torch):
    """Five iterations of the optimisation loop: the parameters outside the
    spin blocks stay zero, and E_L of the final states at the final parameters
    matches the oracle."""
    from paper_1807_10633_amd.optimize import Optimizer
    from paper_1807_10633_amd.vmc import vmc_local_energy

    wl = _uhf("hubbard8", 256)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    opt = Optimizer(sysm, walkers, torch.as_tensor(wl.jastrow, device="cuda"), torch.as_tensor(wl.theta, device="cuda"),
                    moves=20)
    opt.run(5)
    n, na, ne, n_so = wl.n_orb, wl.n_alpha, wl.n_elec, wl.n_so
    p = opt.params.cpu().numpy()
    th = p[opt.nj:].reshape(n_so, n_so)
    assert np.all(th[:n, na:ne] == 0.0) and np.all(th[n:, :na] == 0.0)
    assert not np.array_equal(th, wl.theta)  # the blocks did move
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    orc = OracleSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, wl.eri_idx, wl.eri_val, wl.eps)
    orc.set_params(p[:opt.nj], th)
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    occ = occ_of(sysm, walkers)
    for w in (0, 100, 255):
        r = orc.local_energy(occ[w], ORC_LEMMA, with_candidates=False)
        assert abs(el[w] - r["eloc"]) <= el_tol(r["T"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_uhf_hchain160_full_size_sampled(torch, prec):
    """160 orbitals, 80+80 electrons (above the 128 a general-orbital inverse
    fits in registers; each spin block has 80), eps = 1e-5, 8192 walkers: E_L of
    sampled walkers, fresh and after a short sweep, against the oracle."""
    from paper_1807_10633_amd.vmc import VMC_FP64, VMC_MIXED, vmc_local_energy

    wl = _uhf("hchain160", 8192)
    _say(f"[uhf hchain160 {prec}] W=8192")
    sysm = gpu_system(wl, precision=VMC_MIXED if prec == "mixed" else VMC_FP64)
    walkers = sysm.walkers(wl.occ)
    tol = MIXED_TOL * wl.n_elec if prec == "mixed" else EL_TOL
    orc = OracleSystem.from_workload(wl)
    idx = [0, 4095, 8191]
    for sweep in (0, 3):
        if sweep:
            run_sweep(sysm, walkers, sweep)
        vmc_local_energy(sysm.handle, walkers)
        torch.cuda.synchronize()
        st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
        assert np.all((st & 1) == 0)
        el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
        occ = occ_of(sysm, walkers)
        for w in idx[: 3 if sweep == 0 else 2]:
            r = orc.local_energy(occ[w], ORC_LEMMA, with_candidates=False)
            tol = mixed_tol(r["T"], wl.n_elec) if prec == "mixed" else el_tol(r["T"])
            assert abs(el[w] - r["eloc"]) <= tol, (w, el[w], r["eloc"], r["T"])


@pytest.mark.parametrize("name,nw", [("hubbard8", 4), ("hchain20", 4)])
def test_uhf_excitation_lists(torch, name, nw):
    """The diagnostic candidate list reads the spin-blocked R: candidates
    bit-exact, H * ratio and |ratio| against the oracle, after some moves."""
    from paper_1807_10633_amd.vmc import vmc_excitations

    wl = _uhf(name, nw)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, 7)
    occ = occ_of(sysm, walkers)
    orc = OracleSystem.from_workload(wl)
    cap = 200000
    ijab = torch.zeros((cap, 5), dtype=torch.int32, device="cuda")
    hv = torch.zeros(cap, dtype=torch.float64, device="cuda")
    rv = torch.zeros(cap, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for w in range(nw):
        vmc_excitations(sysm.handle, walkers, w, ijab, hv, rv, cap, cnt)
        torch.cuda.synchronize()
        n = int(cnt.item())
        ref = orc.local_energy(occ[w], ORC_LEMMA)["cand"]
        assert n == ref.size
        exp = np.stack([ref["type"], ref["i"], ref["j"], ref["a"], ref["b"]], axis=1)
        assert np.array_equal(ijab[:n].cpu().numpy(), exp)
        h, r = hv[:n].cpu().numpy(), rv[:n].cpu().numpy()
        scale = np.abs(ref["ratio"]).sum() + 1.0
        assert np.max(np.abs(h * r - ref["h"] * ref["ratio"])) <= 1e-12 * scale
        assert np.allclose(np.abs(r), np.abs(ref["ratio"]), rtol=1e-10, atol=1e-13 * scale)


def test_uhf_systems_batch_in_stream_mode_only(torch):
    from paper_1807_10633_amd.vmc import (VMC_BATCH_STREAMS, VmcError, vmc_batch_create, vmc_batch_ctmc_step,
                                          vmc_batch_destroy, vmc_batch_set_mode)

    wl = _uhf("hubbard8", 8)
    sysm = gpu_system(wl)
    wk = sysm.walkers(wl.occ)
    b = vmc_batch_create([sysm.handle])
    try:
        with pytest.raises(VmcError):  # the fused launch is for the general form only
            vmc_batch_ctmc_step(b, [wk], 1)
        assert wk.step == 0
        vmc_batch_set_mode(b, VMC_BATCH_STREAMS)
        vmc_batch_ctmc_step(b, [wk], 2)
    finally:
        vmc_batch_destroy(b)
    torch.cuda.synchronize()
    assert wk.step == 2
