"""GPU gradient path: gradient ratios O_k, the contracted backward, the
autograd wrapper and the AMSGrad kernel, against the oracle, the brute force
and finite differences."""
import numpy as np
import pytest

from oracle.brute import BruteSystem
from oracle.core import ORC_DET, ORC_LEMMA, OracleSystem
from oracle.optim import AMSGrad, contraction_weights, gradient, weighted_energy
from workloads import eri_dense_spatial, make_config

from gpu_common import field, gpu_system, occ_of, run_sweep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available()
    return torch


def _dense_O(torch, sysm, walkers):
    from paper_1807_10633_amd.vmc import vmc_logderiv

    out = torch.zeros((walkers.n_walkers, sysm.n_params), dtype=torch.float64, device="cuda")
    vmc_logderiv(sysm.handle, walkers, None, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("burn", [0, 23])
def test_logderiv_dense_matches_oracle(torch, burn):
    wl = make_config("hchain20", n_walkers=32)
    print(f"[logderiv] hchain20 W=32 after {burn} moves", flush=True)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    if burn:
        run_sweep(sysm, walkers, burn)
    O = _dense_O(torch, sysm, walkers)
    occ = occ_of(sysm, walkers)
    orc = OracleSystem.from_workload(wl)
    nj = wl.n_so * (wl.n_so + 1) // 2
    for w in range(32):
        ref = orc.logderiv(occ[w])
        assert np.array_equal(O[w, :nj], ref[:nj])
        scale = np.max(np.abs(ref[nj:]))
        assert np.max(np.abs(O[w, nj:] - ref[nj:])) <= 1e-10 * scale


def test_contracted_backward_equals_dense_contraction(torch):
    from paper_1807_10633_amd.vmc import vmc_logderiv

    wl = make_config("hchain20", n_walkers=1000)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, 10)
    O = _dense_O(torch, sysm, walkers)
    g = np.random.default_rng(0).normal(size=1000)
    G = torch.zeros(sysm.n_params, dtype=torch.float64, device="cuda")
    vmc_logderiv(sysm.handle, walkers, torch.as_tensor(g, device="cuda"), G)
    torch.cuda.synchronize()
    ref = g @ O
    assert np.allclose(G.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(g).sum())


def test_exact_gradient_of_hubbard8_matches_fd_of_exact_energy(torch):
    """Every determinant of the sector as a walker, weights rho: the GPU
    backward gives the exact gradient, checked against finite differences of
    the brute-force energy <psi|H|psi>/<psi|psi>."""
    from paper_1807_10633_amd.vmc import vmc_local_energy, vmc_logderiv

    wl = make_config("hubbard8", n_walkers=1)
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    occ = np.stack([br.det_bits(k) for k in range(len(br.dets))])
    sysm = gpu_system(wl)
    walkers = sysm.walkers(occ)
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    psi = br.psi(wl.theta, wl.jastrow)
    rho = psi ** 2 / np.sum(psi ** 2)
    g = contraction_weights(el, rho)
    G = torch.zeros(sysm.n_params, dtype=torch.float64, device="cuda")
    vmc_logderiv(sysm.handle, walkers, torch.as_tensor(g, device="cuda"), G)
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    n_so = wl.n_so
    nj = n_so * (n_so + 1) // 2
    rng = np.random.default_rng(3)
    for k in list(rng.choice(nj, 8, replace=False)) + list(nj + rng.choice(n_so * n_so, 16, replace=False)):
        h = 1e-6
        Jp, Jm, tp, tm = wl.jastrow.copy(), wl.jastrow.copy(), wl.theta.copy(), wl.theta.copy()
        if k < nj:
            Jp[k] += h
            Jm[k] -= h
        else:
            tp.flat[k - nj] += h
            tm.flat[k - nj] -= h
        fd = (br.energy(br.psi(tp, Jp)) - br.energy(br.psi(tm, Jm))) / (2 * h)
        assert G[k] == pytest.approx(fd, abs=1e-6), k


def test_autograd_backward_is_the_vmc_estimator(torch):
    from paper_1807_10633_amd.autograd import vmc_energy

    wl = make_config("hchain20", n_walkers=256)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, 40)
    J = sysm.J.clone().requires_grad_(True)
    th = sysm.theta.clone().requires_grad_(True)
    E = vmc_energy(sysm, walkers, J, th)
    E.backward()
    occ = occ_of(sysm, walkers)
    orc = OracleSystem.from_workload(wl)
    el_o, T_o, _, st = orc.local_energy_batch(occ, ORC_LEMMA)
    assert np.all(st == 0)
    t_o = 1.0 / T_o
    assert float(E) == pytest.approx(weighted_energy(el_o, t_o), abs=1e-10)
    O = np.stack([orc.logderiv(o) for o in occ])
    G_ref = gradient(O, el_o, t_o)
    nj = wl.n_so * (wl.n_so + 1) // 2
    G = np.concatenate([J.grad.cpu().numpy().ravel(), th.grad.cpu().numpy().ravel()])
    assert np.max(np.abs(G - G_ref)) <= 1e-9 * (np.max(np.abs(G_ref)) + 1.0)
    assert np.all(G[nj:].reshape(wl.n_so, wl.n_so)[:, wl.n_elec:] == 0.0)


@pytest.mark.parametrize("literal", [False, True])
def test_amsgrad_kernel_matches_oracle(torch, literal):
    from paper_1807_10633_amd.vmc import vmc_amsgrad

    n = 100003
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=n)
    opt = AMSGrad(n, lr=1e-3, beta1=0.9, beta2=0.99, paper_literal=literal)
    p_ref = p0.copy()
    P = torch.as_tensor(p0.copy(), device="cuda")
    m = torch.zeros(n, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(m)
    vh = torch.zeros_like(m)
    for it in range(6):
        G = rng.normal(size=n) * (1 + it)
        p_ref = opt.step(p_ref, G)
        vmc_amsgrad(P, m, v, vh, torch.as_tensor(G, device="cuda"), 1e-3, 0.9, 0.99, 1e-8, literal)
    torch.cuda.synchronize()
    assert np.allclose(P.cpu().numpy(), p_ref, rtol=1e-14, atol=1e-15)
    assert np.allclose(vh.cpu().numpy(), opt.vhat, rtol=1e-14, atol=0)


def test_estimate_kernel_matches_oracle_weights(torch):
    """vmc_estimate: the t-weighted energy and the gradient weights, against the
    oracle's definitions, on the walkers' own E_L and t after a sweep, and with
    flagged entries (t = 0, non-finite E_L) that must carry no weight."""
    from paper_1807_10633_amd.vmc import vmc_estimate

    wl = make_config("hchain20", n_walkers=1000)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    run_sweep(sysm, walkers, 20)
    W = walkers.n_walkers
    el_t = walkers.view("eloc", torch.float64)[:W]
    t_t = walkers.view("tres", torch.float64)[:W]
    for flagged in (False, True):
        if flagged:
            el_t[3] = float("nan")
            t_t[7] = 0.0
            el_t[11] = float("inf")
        out = torch.zeros(4, dtype=torch.float64, device="cuda")
        g = torch.zeros(W, dtype=torch.float64, device="cuda")
        vmc_estimate(sysm.handle, walkers, out, g)
        torch.cuda.synchronize()
        el, t = el_t.cpu().numpy(), t_t.cpu().numpy()
        keep = (t > 0) & np.isfinite(el)
        E = weighted_energy(el[keep], t[keep])
        o = out.cpu().numpy()
        assert o[3] == np.count_nonzero(keep)
        assert o[2] == pytest.approx(E, rel=1e-13, abs=1e-13)
        gw = np.zeros(W)
        gw[keep] = contraction_weights(el[keep], t[keep])
        np.testing.assert_allclose(g.cpu().numpy(), gw, rtol=1e-11, atol=1e-16)
