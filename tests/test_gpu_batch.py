"""Uneven batch in one launch: H-chain-like systems of 40, 80 and 160 orbitals
(half filled, eps = 1e-5), 2048 walkers each, swept by one kernel launch.

* The batch computes exactly what separate per-system launches of the same
  variant compute (bitwise: occupations, E_L, t, picks, B and R).
* The stream mode (one stream per system, each system with its own variant,
  spin-blocked systems included) computes exactly what the separate calls
  compute; the fused mode refuses spin-blocked systems.
* E_L of sampled walkers of every system against the oracle.
* The hand-written O_k backward over all parameters of the three systems
  (201,880), contracted with the estimator weights, against the oracle on
  sampled parameters; O_k against finite differences of the oracle's log|psi|;
  one AMSGrad step over the concatenated parameters against the oracle's.
"""
import numpy as np
import pytest

from oracle.core import ORC_LEMMA, OracleSystem
from oracle.optim import AMSGrad
from workloads import make_config

from gpu_common import EL_TOL, ST_STALE, el_tol, field, gpu_system, occ_of

pytestmark = pytest.mark.gpu

NAMES = ("hchain40", "hchain80", "hchain160")
W = 2048


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def batch_setup(torch):
    wls = [make_config(n, n_walkers=W) for n in NAMES]
    systems = [gpu_system(wl) for wl in wls]
    return wls, systems


def _state(torch, sysm, wk):
    ne, n_so = sysm.ne, sysm.r_row
    return {
        "occ": occ_of(sysm, wk),
        "eloc": field(sysm, wk, "eloc", torch.float64, 1),
        "tres": field(sysm, wk, "tres", torch.float64, 1),
        "pick": field(sysm, wk, "pick", torch.int64, 1),
        "B": field(sysm, wk, "ainv", torch.float64, ne * ne),
        "R": field(sysm, wk, "r", torch.float64, ne * n_so),
        "status": field(sysm, wk, "status", torch.int32, 1),
    }


def test_batch_equals_separate_launches(torch, batch_setup):
    from paper_1807_10633_amd.vmc import (vmc_batch_create, vmc_batch_ctmc_step, vmc_batch_destroy,
                                          vmc_batch_local_energy, vmc_ctmc_step, vmc_launch_info,
                                          vmc_local_energy)

    wls, systems = batch_setup
    for s in systems:
        assert not vmc_launch_info(s.handle)["state_in_lds"]  # same variant as the batch
    sep = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    bat = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    for s, wk in zip(systems, sep):
        vmc_ctmc_step(s.handle, wk, 3)
        vmc_local_energy(s.handle, wk)
    b = vmc_batch_create([s.handle for s in systems])
    try:
        vmc_batch_ctmc_step(b, bat, 3)
        vmc_batch_local_energy(b, bat)
    finally:
        vmc_batch_destroy(b)
    torch.cuda.synchronize()
    for name, s, a, c in zip(NAMES, systems, sep, bat):
        assert a.step == c.step == 3
        sa, sc = _state(torch, s, a), _state(torch, s, c)
        # the separate launches re-invert in their own kernel and mark moved
        # walkers stale; the batch re-inverts in place: the mark is scheduling
        sa["status"] = sa["status"] & ~ST_STALE
        sc["status"] = sc["status"] & ~ST_STALE
        for k in sa:
            assert np.array_equal(sa[k], sc[k]), f"{name}: field {k} differs between batch and separate launches"
        assert np.all((sa["status"] & 1) == 0)
        _say(f"    {name}: batch == separate launches (3 moves + E_L), mean E_L {np.mean(sa['eloc']):.6f}")


def test_batch_local_energy_matches_oracle(torch, batch_setup):
    from paper_1807_10633_amd.vmc import vmc_batch_create, vmc_batch_destroy, vmc_batch_local_energy

    wls, systems = batch_setup
    wks = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    b = vmc_batch_create([s.handle for s in systems])
    try:
        vmc_batch_local_energy(b, wks)
    finally:
        vmc_batch_destroy(b)
    torch.cuda.synchronize()
    for wl, s, wk in zip(wls, systems, wks):
        el = field(s, wk, "eloc", torch.float64, 1)[:, 0]
        orc = OracleSystem.from_workload(wl)
        worst = 0.0
        for w in (0, W // 2, W - 1):
            r = orc.local_energy(wl.occ[w], ORC_LEMMA, with_candidates=False)
            tol = el_tol(r["T"])
            d = abs(el[w] - r["eloc"])
            worst = max(worst, d / tol)
            assert d <= tol, (wl.name, w, el[w], r["eloc"], r["T"])
        _say(f"    {wl.name}: worst |dE|/tol {worst:.3g}")


def test_batch_gradient_and_amsgrad_all_parameters(torch, batch_setup):
    from paper_1807_10633_amd.vmc import vmc_amsgrad, vmc_estimate, vmc_local_energy, vmc_logderiv

    wls, systems = batch_setup
    rng = np.random.default_rng(5)
    Gs, params = [], []
    for wl, s in zip(wls, systems):
        wk = s.walkers(wl.occ)
        vmc_local_energy(s.handle, wk)
        est = torch.zeros(4, dtype=torch.float64, device="cuda")
        g = torch.zeros(W, dtype=torch.float64, device="cuda")
        vmc_estimate(s.handle, wk, est, g)
        G = torch.zeros(s.n_params, dtype=torch.float64, device="cuda")
        vmc_logderiv(s.handle, wk, g, G)
        torch.cuda.synchronize()
        Gh, gh = G.cpu().numpy(), g.cpu().numpy()
        # oracle: G_k = sum_w g_w O_w,k on sampled k
        orc = OracleSystem.from_workload(wl)
        nj = s.n_so * (s.n_so + 1) // 2
        ne = wl.n_elec
        ks = np.concatenate([rng.integers(0, nj, 24),
                             nj + rng.integers(0, s.n_so, 24) * s.n_so + rng.integers(0, ne, 24)])
        ref = np.zeros(ks.size)
        for w in range(W):
            if gh[w] != 0.0:
                ref += gh[w] * orc.logderiv(wl.occ[w])[ks]
        np.testing.assert_allclose(Gh[ks], ref, rtol=1e-9, atol=1e-12 * np.max(np.abs(ref)))
        # O_k of one walker against central differences of the oracle's log|psi|
        O = torch.zeros((1, s.n_params), dtype=torch.float64, device="cuda")
        one = s.walkers(wl.occ[:1])
        vmc_logderiv(s.handle, one, None, O)
        torch.cuda.synchronize()
        O0 = O[0].cpu().numpy()
        J0, th0 = wl.jastrow.copy(), wl.theta.copy()
        h = 1e-6
        for k in ks[::8]:
            fd = []
            for sgn in (1, -1):
                J, th = J0.copy(), th0.copy()
                if k < nj:
                    J[k] += sgn * h
                else:
                    th.reshape(-1)[k - nj] += sgn * h
                orc.set_params(J, th)
                fd.append(orc.log_psi(wl.occ[0])[0])
            d = (fd[0] - fd[1]) / (2 * h)
            assert abs(d - O0[k]) <= 1e-6 * max(1.0, abs(d)), (wl.name, int(k), d, O0[k])
        orc.set_params(J0, th0)
        Gs.append(Gh)
        params.append(np.concatenate([J0, th0.reshape(-1)]))
    # one AMSGrad step over all parameters of the batch (~2e5)
    Gall = np.concatenate(Gs)
    pall = np.concatenate(params)
    _say(f"    parameters in the batch: {pall.size}")
    assert pall.size == 201880
    p_d = torch.as_tensor(pall, device="cuda").clone()
    m = torch.zeros_like(p_d)
    v = torch.zeros_like(p_d)
    vh = torch.zeros_like(p_d)
    vmc_amsgrad(p_d, m, v, vh, torch.as_tensor(Gall, device="cuda"), 1e-3, 0.9, 0.99, 1e-8, False)
    torch.cuda.synchronize()
    opt = AMSGrad(pall.size, lr=1e-3, beta1=0.9, beta2=0.99)
    ref = opt.step(pall.copy(), Gall)
    np.testing.assert_allclose(p_d.cpu().numpy(), ref, rtol=0, atol=1e-15)


def test_batch_stream_mode_equals_separate_calls(torch):
    """Spin-blocked hubbard8, hchain20 (state in LDS) and hchain80 (state in
    HBM), 256 walkers each, in VMC_BATCH_STREAMS mode: every field after 4
    moves and E_L equals what the separate calls leave, bit for bit."""
    from paper_1807_10633_amd.vmc import (VMC_BATCH_FUSED, VMC_BATCH_STREAMS, VmcError, vmc_batch_create,
                                          vmc_batch_ctmc_step, vmc_batch_destroy, vmc_batch_info,
                                          vmc_batch_local_energy, vmc_batch_set_mode, vmc_ctmc_step,
                                          vmc_launch_info, vmc_local_energy)

    wls = [make_config("hubbard8", n_walkers=256, orbitals="uhf"), make_config("hchain20", n_walkers=256),
           make_config("hchain80", n_walkers=256)]
    systems = [gpu_system(wl) for wl in wls]
    lds = [vmc_launch_info(s.handle)["state_in_lds"] for s in systems]
    assert lds[1] and not lds[2], lds
    sep = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    bat = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    for s, wk in zip(systems, sep):
        vmc_ctmc_step(s.handle, wk, 4)
        vmc_local_energy(s.handle, wk)
    b = vmc_batch_create([s.handle for s in systems])
    try:
        assert vmc_batch_info(b)["mode"] == VMC_BATCH_FUSED
        with pytest.raises(VmcError):  # the fused launch holds no spin-blocked system
            vmc_batch_ctmc_step(b, bat, 1)
        with pytest.raises(VmcError):
            vmc_batch_set_mode(b, 7)
        vmc_batch_set_mode(b, VMC_BATCH_STREAMS)
        assert vmc_batch_info(b)["mode"] == VMC_BATCH_STREAMS
        vmc_batch_ctmc_step(b, bat, 4)
        vmc_batch_local_energy(b, bat)
    finally:
        vmc_batch_destroy(b)
    torch.cuda.synchronize()
    for wl, s, a, c in zip(wls, systems, sep, bat):
        assert a.step == c.step == 4
        sa, sc = _state(torch, s, a), _state(torch, s, c)
        for k in sa:
            assert np.array_equal(sa[k], sc[k]), f"{wl.name}: field {k} differs between stream mode and separate calls"
        el = sc["eloc"][:, 0]
        orc = OracleSystem.from_workload(wl)
        r = orc.local_energy(occ_of(s, c)[7], ORC_LEMMA, with_candidates=False)
        assert abs(el[7] - r["eloc"]) <= el_tol(r["T"]), (wl.name, el[7], r["eloc"])
        _say(f"    {wl.name}: stream mode == separate calls (4 moves + E_L), mean E_L {np.mean(el):.6f}")


def test_batch_autotune(torch):
    from paper_1807_10633_amd.vmc import (VMC_BATCH_FUSED, VMC_BATCH_STREAMS, vmc_batch_autotune, vmc_batch_create,
                                          vmc_batch_destroy, vmc_batch_info, vmc_batch_local_energy, vmc_launch_info)

    wls = [make_config(n, n_walkers=128) for n in ("hchain40", "hchain80")]
    systems = [gpu_system(wl) for wl in wls]
    wks = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    b = vmc_batch_create([s.handle for s in systems])
    try:
        nt = vmc_batch_autotune(b, wks, 2)
        info = vmc_batch_info(b)
        vmc_batch_local_energy(b, wks)
    finally:
        vmc_batch_destroy(b)
    torch.cuda.synchronize()
    if nt == 0:
        assert info["mode"] == VMC_BATCH_STREAMS
    else:
        assert info["mode"] == VMC_BATCH_FUSED and info["threads"] == nt and nt in (64, 128, 256, 512)
    for wl, s, wk in zip(wls, systems, wks):
        # 2 timed sweeps of 2 moves per shape: 8 fused shapes, then the
        # system's own shapes (4, or 8 with the occupancy targets where the
        # state stays in HBM), then the stream mode once
        own = 4 if vmc_launch_info(s.handle)["state_in_lds"] else 8
        assert wk.step == 4 * (8 + own + 1), (wl.name, wk.step)
        el = field(s, wk, "eloc", torch.float64, 1)[:, 0]
        orc = OracleSystem.from_workload(wl)
        r = orc.local_energy(occ_of(s, wk)[5], ORC_LEMMA, with_candidates=False)
        assert abs(el[5] - r["eloc"]) <= el_tol(r["T"])
    _say(f"    batch autotune: mode {info['mode']}, workgroup {info['threads']}, waves {info['waves']}")
