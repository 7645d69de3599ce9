"""Pins of the CPU oracle against things other than itself.

Brute force over whole sectors (operator algebra, no Slater-Condon rules),
closed forms, invariants, library routines and finite differences.  Each test
names the passage of the paper whose quantity it pins.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.brute import BruteSystem, jastrow_dense
from oracle.core import ORC_DET, ORC_LEMMA, OracleSystem, list_to_occ, occ_to_list, philox4x64_10, uniform
from oracle.optim import AMSGrad, contraction_weights, gradient, weighted_energy
from workloads import (eri_dense_spatial, hchain_like, hubbard_2d, hubbard_ring, init_jastrow, init_theta,
                       make_config)

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _tol(T, hmax):
    """Absolute E_L tolerance: 1e-10, widened for near-node determinants
    where every ratio (and so the rounding of both sides) scales like T."""
    return 1e-10 + 1e-12 * hmax * np.asarray(T)


def _tiny_hchain(n, na, nb, seed, eps, jstd=0.05, noise=0.01):
    h, ei, ev = hchain_like(n, seed)
    theta = init_theta(h, na, nb, noise, seed + 1)
    J = init_jastrow(2 * n, jstd, seed + 2)
    orc = OracleSystem(n, na, nb, h, ei, ev, eps)
    orc.set_params(J, theta)
    return h, ei, ev, theta, J, orc


def _rotated(h, g, seed):
    n = h.shape[0]
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    h2 = Q.T @ h @ Q
    g2 = np.einsum("pqrs,pa,qb,rc,sd->abcd", g, Q, Q, Q, Q)
    return h2, g2


def _canonical_list(g, cut=0.0):
    n = g.shape[0]
    idx, val = [], []
    for p in range(n):
        for q in range(p + 1):
            for r in range(n):
                for s in range(r + 1):
                    if p * (p + 1) // 2 + q < r * (r + 1) // 2 + s:
                        continue
                    if abs(g[p, q, r, s]) > cut:
                        idx.append((p, q, r, s))
                        val.append(g[p, q, r, s])
    return np.array(idx, dtype=np.int32).reshape(-1, 4), np.array(val)


# --------------------------------------------------------------------------
# The brute force itself (pins the second-quantised Hamiltonian matrix)
# --------------------------------------------------------------------------
def test_brute_hubbard_dimer_closed_form():
    h, ei, ev = hubbard_ring(2, 1.0, 4.0)
    # a 2-ring built as a ring double counts the bond; use the plain dimer
    h = np.array([[0.0, -1.0], [-1.0, 0.0]])
    g = eri_dense_spatial(2, ei, ev)
    br = BruteSystem(2, 1, 1, h, g)
    assert br.ground_energy() == pytest.approx(GOLDEN["hubbard_dimer_U4_1a1b"]["value"], abs=1e-12)


def test_brute_single_electron_spectrum():
    h, ei, ev = hchain_like(5, 77)
    g = eri_dense_spatial(5, ei, ev)
    br = BruteSystem(5, 1, 0, h, g)
    assert np.allclose(np.linalg.eigvalsh(br.H), np.linalg.eigvalsh(h), atol=1e-12)


def test_brute_spectrum_invariant_under_orbital_rotation():
    """FCI energies do not depend on the orbital basis: a wrong index order,
    a missing exchange term or a wrong fermionic sign in the operator algebra
    would break the covariance."""
    n, na, nb = 4, 2, 1
    h, ei, ev = hchain_like(n, 91)
    g = eri_dense_spatial(n, ei, ev)
    e1 = np.linalg.eigvalsh(BruteSystem(n, na, nb, h, g).H)
    h2, g2 = _rotated(h, g, 5)
    e2 = np.linalg.eigvalsh(BruteSystem(n, na, nb, h2, g2).H)
    assert np.allclose(e1, e2, atol=1e-10)


def test_brute_diagonal_is_textbook_determinant_energy():
    n, na, nb = 4, 2, 2
    h, ei, ev = hchain_like(n, 13)
    g = eri_dense_spatial(n, ei, ev)
    br = BruteSystem(n, na, nb, h, g)
    for k in range(len(br.dets)):
        occ = [p for p in range(2 * n) if (br.dets[k] >> p) & 1]
        e = 0.0
        for i in occ:
            e += h[i % n, i % n]
        for x in range(len(occ)):
            for y in range(x + 1, len(occ)):
                i, j = occ[x], occ[y]
                e += g[i % n, i % n, j % n, j % n]
                if (i < n) == (j < n):
                    e -= g[i % n, j % n, j % n, i % n]
        assert br.H[k, k] == pytest.approx(e, abs=1e-12)


# --------------------------------------------------------------------------
# Local energy (Eq. eloc:hci): epsilon = 0 equals the unscreened sum
# --------------------------------------------------------------------------
def test_oracle_eloc_equals_brute_hubbard8_all_determinants():
    wl = make_config("hubbard8")
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    psi = br.psi(wl.theta, wl.jastrow)
    el = br.local_energies(psi)
    orc = OracleSystem.from_workload(wl)
    occ = np.stack([br.det_bits(k) for k in range(len(br.dets))])
    el_o, T_o, nc, st = orc.local_energy_batch(occ, ORC_DET)
    assert np.all(st == 0)
    # rounding in both E_L computations grows like 1/|psi(N)|, i.e. like T
    assert np.all(np.abs(el_o - el) <= _tol(T_o, 4.0))
    # exact energy identity E = sum_N rho_N E_L(N)  (Eq. eq:vmc)
    rho = psi ** 2 / np.sum(psi ** 2)
    assert np.sum(rho * el_o) == pytest.approx(br.energy(psi), abs=1e-10)
    assert br.energy(psi) >= br.ground_energy() - 1e-12


@pytest.mark.parametrize("n,na,nb,seed", [(4, 2, 2, 3), (5, 2, 3, 4), (6, 3, 2, 8)])
def test_oracle_eps0_equals_unscreened_hchain(n, na, nb, seed):
    h, ei, ev, theta, J, orc = _tiny_hchain(n, na, nb, seed, eps=0.0)
    br = BruteSystem(n, na, nb, h, eri_dense_spatial(n, ei, ev))
    psi = br.psi(theta, J)
    el = br.local_energies(psi)
    for k in range(len(br.dets)):
        r = orc.local_energy(br.det_bits(k), ORC_DET, with_candidates=False)
        assert r["eloc"] == pytest.approx(el[k], abs=_tol(r["T"], 1.0))
        r2 = orc.local_energy(br.det_bits(k), ORC_LEMMA, with_candidates=False)
        assert r2["eloc"] == pytest.approx(el[k], abs=_tol(r["T"], 1.0))


def test_oracle_rotated_dense_integrals_match_brute():
    """Dense rotated integrals exercise every symmetric image of the list."""
    n, na, nb = 4, 2, 2
    h, ei, ev = hchain_like(n, 21)
    h2, g2 = _rotated(h, eri_dense_spatial(n, ei, ev), 9)
    idx, val = _canonical_list(g2)
    theta = init_theta(h2, na, nb, 0.05, 3)
    J = init_jastrow(2 * n, 0.1, 4)
    orc = OracleSystem(n, na, nb, h2, idx, val, 0.0)
    orc.set_params(J, theta)
    br = BruteSystem(n, na, nb, h2, g2)
    el = br.local_energies(br.psi(theta, J))
    for k in range(len(br.dets)):
        r = orc.local_energy(br.det_bits(k), ORC_LEMMA, False)
        assert r["eloc"] == pytest.approx(el[k], abs=_tol(r["T"], 1.0))


def test_screened_sets_follow_the_paper_bounds():
    """Singles kept iff S_ia > eps, with S_ia >= |H_NM| for every N; doubles
    kept iff |H_NM| = |<ab|ij>-<ab|ji>| > eps (section 'Reduced scaling
    evaluation of the local energy')."""
    n, na, nb = 5, 2, 2
    eps = 2e-3
    h, ei, ev, theta, J, orc = _tiny_hchain(n, na, nb, 33, eps)
    br = BruteSystem(n, na, nb, h, eri_dense_spatial(n, ei, ev))
    S = orc.singles_bound()
    n_dropped = 0
    for k in range(len(br.dets)):
        N = br.dets[k]
        conn = br.connected(k)
        cands = orc.local_energy(br.det_bits(k), ORC_DET)["cand"]
        kept = set()
        for c in cands:
            M = N & ~(1 << int(c["i"])) | (1 << int(c["a"]))
            if c["type"] == 2:
                M = M & ~(1 << int(c["j"])) | (1 << int(c["b"]))
            kept.add(br.index[M])
            assert c["h"] == pytest.approx(conn.get(br.index[M], 0.0), abs=1e-12)
        for m, hnm in conn.items():
            diff = N ^ br.dets[m]
            removed = [p for p in range(2 * n) if (N >> p) & 1 and (diff >> p) & 1]
            added = [p for p in range(2 * n) if (br.dets[m] >> p) & 1 and (diff >> p) & 1]
            if len(removed) == 1:
                i, a = removed[0], added[0]
                assert S[i, a] >= abs(hnm) - 1e-15
                assert (m in kept) == (S[i, a] > eps)
            else:
                assert (m in kept) == (abs(hnm) > eps)
            n_dropped += m not in kept
    assert n_dropped > 0  # the threshold really screens something here


# --------------------------------------------------------------------------
# Zero variance (closed forms)
# --------------------------------------------------------------------------
def test_zero_variance_ring8_all_determinants():
    h, ei, ev = hubbard_ring(8, 1.0, 0.0)
    theta = init_theta(h, 4, 4, 0.0, 0)
    J = np.zeros(16 * 17 // 2)
    orc = OracleSystem(8, 4, 4, h, ei, ev, 0.0)
    orc.set_params(J, theta)
    br = BruteSystem(8, 4, 4, h, np.zeros((8, 8, 8, 8)))
    psi = br.psi(theta, J)
    e0 = GOLDEN["hubbard_ring8_U0_4a4b"]["value"]
    n_checked = 0
    for k in range(len(br.dets)):
        if abs(psi[k]) < 1e-8:
            continue
        r = orc.local_energy(br.det_bits(k), ORC_DET, False)
        assert r["eloc"] == pytest.approx(e0, abs=1e-9)
        n_checked += 1
    assert n_checked > 100


def test_zero_variance_10x10_lemma_mode():
    h, ei, ev = hubbard_2d(10, 10, 1.0, 0.0)
    theta = init_theta(h, 50, 50, 0.0, 0)
    J = np.zeros(200 * 201 // 2)
    orc = OracleSystem(100, 50, 50, h, ei, ev, 0.0)
    orc.set_params(J, theta)
    rng = np.random.default_rng(0)
    e0 = GOLDEN["hubbard_10x10_U0_50a50b"]["value"]
    for _ in range(3):
        orbs = list(rng.permutation(100)[:50]) + list(100 + rng.permutation(100)[:50])
        r = orc.local_energy(list_to_occ(orbs, 200), ORC_LEMMA, False)
        assert r["eloc"] == pytest.approx(e0, abs=1e-8)


# --------------------------------------------------------------------------
# Philox (the counter-based generator drawn for every CTMC pick)
# --------------------------------------------------------------------------
def test_philox_matches_numpy():
    M = (1 << 64) - 1
    for seed, walker, step in [(4001, 0, 1), (4001, 63, 999), (7, 123456, 2 ** 40), (0, 0, 5)]:
        bg = np.random.Philox(key=[seed, walker], counter=[step - 1, 0, 0, 0])
        ref = bg.random_raw(4)
        got = philox4x64_10([step, 0, 0, 0], [seed, walker])
        assert np.array_equal(got, ref)
        assert uniform(seed, walker, step) == (int(ref[0]) >> 11) * 2.0 ** -53
    # step 0: numpy increments an all-ones counter to zero
    bg = np.random.Philox(key=[3, 4], counter=[M, M, M, M])
    assert np.array_equal(philox4x64_10([0, 0, 0, 0], [3, 4]), bg.random_raw(4))


# --------------------------------------------------------------------------
# CTMC (section "Continuous time Monte Carlo")
# --------------------------------------------------------------------------
def test_ctmc_pick_is_the_direct_method():
    wl = make_config("hchain20", n_walkers=4)
    orc = OracleSystem.from_workload(wl)
    for w in range(4):
        occ = wl.occ[w]
        r = orc.local_energy(occ, ORC_LEMMA)
        rates = np.abs(r["cand"]["ratio"])
        for step in (1, 2, 3):
            new, el, t, pick, margin, rc = orc.ctmc_step(occ, wl.ctmc_seed, w, step, ORC_LEMMA)
            assert rc == 0
            assert t == pytest.approx(1.0 / rates.sum(), rel=1e-12)
            assert el == pytest.approx(r["eloc"], abs=1e-12)
            u = uniform(wl.ctmc_seed, w, step)
            k = int(np.searchsorted(np.cumsum(rates), u * rates.sum(), side="right"))
            c = r["cand"][k]
            assert pick == (int(c["type"]), int(c["i"]), int(c["j"]), int(c["a"]), int(c["b"]))


def test_ctmc_detailed_balance_and_stationarity_hubbard8():
    """r(M<-N)/r(N<-M) = rho_M/rho_N elementwise, and the embedded jump chain
    P(M|N) = r/T_N has stationary vector proportional to rho_N T_N, so the
    residence-time-weighted visits sample rho."""
    wl = make_config("hubbard8")
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    psi = br.psi(wl.theta, wl.jastrow)
    rho = psi ** 2 / np.sum(psi ** 2)
    orc = OracleSystem.from_workload(wl)
    D = len(br.dets)
    Rm = np.zeros((D, D))
    for k in range(D):
        N = br.dets[k]
        for c in orc.local_energy(br.det_bits(k), ORC_DET)["cand"]:
            M = N & ~(1 << int(c["i"])) | (1 << int(c["a"]))
            if c["type"] == 2:
                M = M & ~(1 << int(c["j"])) | (1 << int(c["b"]))
            Rm[k, br.index[M]] = abs(c["ratio"])
    # detailed balance rho_N r(M<-N) = rho_M r(N<-M)
    F = rho[:, None] * Rm
    assert np.max(np.abs(F - F.T)) < 1e-14
    T = Rm.sum(axis=1)
    P = Rm / T[:, None]
    pi = rho * T / np.sum(rho * T)
    assert np.max(np.abs(pi @ P - pi)) < 1e-14
    # residence-time weighting of pi recovers rho
    w = pi / T
    assert np.allclose(w / w.sum(), rho, atol=1e-14)


# --------------------------------------------------------------------------
# Gradient ratios and the gradient estimator (Eq. eq:grad)
# --------------------------------------------------------------------------
def test_logderiv_matches_finite_differences():
    n, na, nb = 5, 2, 3
    h, ei, ev, theta, J, orc = _tiny_hchain(n, na, nb, 55, 0.0, jstd=0.1, noise=0.05)
    n_so, ne = 2 * n, na + nb
    occ = list_to_occ([0, 3, 5, 7, 9], n_so)
    O = orc.logderiv(occ)
    nj = n_so * (n_so + 1) // 2
    rng = np.random.default_rng(1)
    hstep = 1e-6
    for k in list(rng.choice(nj, 12, replace=False)) + list(nj + rng.choice(n_so * n_so, 30, replace=False)):
        Jp, Jm, tp, tm = J.copy(), J.copy(), theta.copy(), theta.copy()
        if k < nj:
            Jp[k] += hstep
            Jm[k] -= hstep
        else:
            tp.flat[k - nj] += hstep
            tm.flat[k - nj] -= hstep
        orc.set_params(Jp, tp)
        lp, _ = orc.log_psi(occ)
        orc.set_params(Jm, tm)
        lm, _ = orc.log_psi(occ)
        fd = (lp - lm) / (2 * hstep)
        assert O[k] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    orc.set_params(J, theta)
    # orbital columns >= Ne never enter the determinant
    th = O[nj:].reshape(n_so, n_so)
    assert np.all(th[:, ne:] == 0.0)
    # unoccupied rows carry no derivative
    occ_l = occ_to_list(occ, n_so)
    for k in range(n_so):
        if k not in occ_l:
            assert np.all(th[k] == 0.0)


def test_exact_gradient_matches_fd_of_exact_energy():
    """2 sum_N rho_N O(N) (E_L(N) - E) with oracle O_k and E_L equals the
    finite-difference derivative of the brute-force <psi|H|psi>/<psi|psi>."""
    n, na, nb = 4, 2, 1
    h, ei, ev, theta, J, orc = _tiny_hchain(n, na, nb, 71, 0.0, jstd=0.1, noise=0.05)
    br = BruteSystem(n, na, nb, h, eri_dense_spatial(n, ei, ev))
    psi = br.psi(theta, J)
    rho = psi ** 2 / np.sum(psi ** 2)
    occs = np.stack([br.det_bits(k) for k in range(len(br.dets))])
    el, _, _, _ = orc.local_energy_batch(occs, ORC_DET)
    O = np.stack([orc.logderiv(o) for o in occs])
    G = gradient(O, el, rho)  # rho as the weights: an exact expectation
    n_so = 2 * n
    nj = n_so * (n_so + 1) // 2
    rng = np.random.default_rng(2)
    for k in list(rng.choice(nj, 6, replace=False)) + list(nj + rng.choice(n_so * n_so, 10, replace=False)):
        hstep = 1e-6
        Jp, Jm, tp, tm = J.copy(), J.copy(), theta.copy(), theta.copy()
        if k < nj:
            Jp[k] += hstep
            Jm[k] -= hstep
        else:
            tp.flat[k - nj] += hstep
            tm.flat[k - nj] -= hstep
        fd = (br.energy(br.psi(tp, Jp)) - br.energy(br.psi(tm, Jm))) / (2 * hstep)
        assert G[k] == pytest.approx(fd, abs=2e-7)
    g = contraction_weights(el, rho)
    assert np.allclose(g @ O, G, atol=1e-14)
    assert weighted_energy(el, rho) == pytest.approx(br.energy(psi), abs=1e-10)


def test_amsgrad_closed_form_constant_gradient():
    """Constant gradient g: m_t = g(1-b1^t), v_t = vhat_t = g^2(1-b2^t)."""
    g = np.array([0.3, -2.0, 1e-3])
    opt = AMSGrad(3, lr=1e-3, beta1=0.9, beta2=0.99)
    p = np.zeros(3)
    for t in range(1, 8):
        p_new = opt.step(p, g)
        m = g * (1 - 0.9 ** t)
        v = g * g * (1 - 0.99 ** t)
        assert np.allclose(opt.m, m, rtol=1e-14)
        assert np.allclose(opt.vhat, v, rtol=1e-14)
        assert np.allclose(p_new - p, -1e-3 * m / (np.sqrt(v) + 1e-8), rtol=1e-13)
        p = p_new


def test_amsgrad_paper_literal_closed_form_constant_gradient():
    """Paper-literal second moment n <- max(n, b2 n + (1-b2) g^2) (Eq. eq:m2
    with the paper's beta' = 1 - beta): for a constant gradient the moving
    average never falls below n, so n_t = g^2 (1 - b2^t), m_t = g (1 - b1^t)."""
    g = np.array([0.3, -2.0, 1e-3, 7.5])
    b1, b2, lr = 0.9, 0.99, 1e-2
    opt = AMSGrad(4, lr=lr, beta1=b1, beta2=b2, paper_literal=True)
    p = np.zeros(4)
    for t in range(1, 12):
        p_new = opt.step(p, g)
        m = g * (1 - b1 ** t)
        n = g * g * (1 - b2 ** t)
        assert np.allclose(opt.m, m, rtol=1e-14)
        assert np.allclose(opt.vhat, n, rtol=1e-14)
        assert np.allclose(p_new - p, -lr * m / (np.sqrt(n) + 1e-8), rtol=1e-13)
        p = p_new


def test_amsgrad_forms_differ_where_the_max_sits():
    """A gradient G at step 1, zero for k steps, then H.  Written out by hand:
    paper-literal (EMA of the maxed n): n = (1-b2) G^2 through the zeros, then
    max(n, b2 n + (1-b2) H^2).  Reddi form (EMA v kept apart, vhat = max):
    v = b2^k (1-b2) G^2 after the zeros, then b2 v + (1-b2) H^2, vhat the
    larger of that and (1-b2) G^2.  The two differ, which pins where each
    branch takes the maximum."""
    b1, b2, G, H, k = 0.9, 0.99, 1.0, 1.0, 200
    seq = [G] + [0.0] * k + [H]
    lit = AMSGrad(1, beta1=b1, beta2=b2, paper_literal=True)
    red = AMSGrad(1, beta1=b1, beta2=b2, paper_literal=False)
    p = np.zeros(1)
    for x in seq:
        lit.step(p, np.array([x]))
        red.step(p, np.array([x]))
    n1 = (1 - b2) * G * G
    lit_ref = max(n1, b2 * n1 + (1 - b2) * H * H)
    v_ref = b2 ** (k + 1) * (1 - b2) * G * G + (1 - b2) * H * H
    red_ref = max(n1, v_ref)
    assert lit.vhat[0] == pytest.approx(lit_ref, rel=1e-13)
    assert red.vhat[0] == pytest.approx(red_ref, rel=1e-13)
    assert red.v[0] == pytest.approx(v_ref, rel=1e-13)
    assert abs(lit_ref - red_ref) > 1e-3  # the sequence separates the forms
    m_ref = b1 ** (k + 1) * (1 - b1) * G + (1 - b1) * H
    assert lit.m[0] == pytest.approx(m_ref, rel=1e-13) and red.m[0] == pytest.approx(m_ref, rel=1e-13)


def test_amsgrad_second_moment_is_monotone():
    rng = np.random.default_rng(0)
    for literal in (False, True):
        opt = AMSGrad(50, paper_literal=literal)
        prev = opt.vhat.copy()
        p = np.zeros(50)
        for _ in range(30):
            p = opt.step(p, rng.normal(size=50) * rng.uniform(0, 3))
            assert np.all(opt.vhat >= prev)
            prev = opt.vhat.copy()


def test_jastrow_packing_roundtrip():
    n_so = 6
    Jp = np.arange(n_so * (n_so + 1) // 2, dtype=float)
    Jd = jastrow_dense(Jp, n_so)
    assert np.array_equal(Jd, Jd.T)
    assert Jd[0, 0] == 0 and Jd[0, 1] == 1 and Jd[1, 1] == n_so
