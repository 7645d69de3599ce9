"""Pins of the oracle's correlator product state (section "Correlator product
states and Slater determinant"; ratio and gradient ratio of section "Local
energy and Gradient ratios") against things other than its own code.

* Brute force: with two- and three-site correlators on the 8-site ring, the
  oracle's screened E_L (eps = 0, both ratio modes) equals
  sum_M H_NM psi(M)/psi(N) of the full-sector Hamiltonian, where the brute
  amplitude multiplies the coefficients read site by site off each bitstring.
* The Jastrow factor is a two-site correlator with c_11 = e^J: correlators
  built from a Jastrow matrix (one-site correlators for the pairs on one site,
  two-site correlators for the pairs across two sites) reproduce log|psi| and
  E_L of that Jastrow factor on every determinant.
* Gradient ratios: O_c = [n_l(N) = n] / c equals the central finite difference
  of log|psi| in each coefficient; coefficients of states not present in N
  have zero derivative.
"""
import itertools

import numpy as np
import pytest

from oracle.brute import BruteSystem, jastrow_dense
from oracle.core import ORC_DET, ORC_LEMMA, OracleSystem
from workloads import cps_chain_windows, cps_pack, eri_dense_spatial, init_cps, make_config


def _tol(T, hmax):
    return 1e-10 + 1e-12 * hmax * np.asarray(T)


def _ring_cps(n, seed, noise=0.3):
    sites = cps_chain_windows(n, 2, periodic=True) + cps_chain_windows(n, 3, periodic=True)[::2]
    coeffs = init_cps(sites, noise, seed)
    return sites, coeffs


def _split(sites, coeffs):
    out, o = [], 0
    for st in sites:
        out.append(coeffs[o:o + 4 ** len(st)])
        o += 4 ** len(st)
    return out


def test_cps_eloc_equals_brute_hubbard8_all_determinants():
    wl = make_config("hubbard8")
    sites, coeffs = _ring_cps(wl.n_orb, 11)
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    psi = br.psi(wl.theta, wl.jastrow, (sites, _split(sites, coeffs)))
    el = br.local_energies(psi)
    orc = OracleSystem.from_workload(wl)
    assert orc.set_cps(cps_pack(sites), coeffs) == coeffs.size
    occ = np.stack([br.det_bits(k) for k in range(len(br.dets))])
    for mode in (ORC_DET, ORC_LEMMA):
        el_o, T_o, nc, st = orc.local_energy_batch(occ, mode)
        assert np.all(st == 0)
        assert np.all(np.abs(el_o - el) <= _tol(T_o, 4.0)), mode
    # log|psi| and its sign against the brute amplitude (up to one global factor)
    lp = np.array([orc.log_psi(o)[0] for o in occ])
    sg = np.array([orc.log_psi(o)[1] for o in occ])
    ref = np.log(np.abs(psi))
    assert np.allclose(lp - ref, (lp - ref)[0], atol=1e-10)
    assert np.all(sg * np.sign(psi) == sg[0] * np.sign(psi[0]))
    # the correlators change the energy: they are not inert
    psi0 = br.psi(wl.theta, wl.jastrow)
    assert abs(br.energy(psi) - br.energy(psi0)) > 1e-3


def _cps_from_jastrow(J, n):
    """Correlators equal to exp(sum_{p<=q} J_pq n_p n_q): a one-site
    correlator per site (alpha-alpha, beta-beta, alpha-beta of that site) and a
    two-site correlator per pair of sites (the four cross pairs)."""
    sites, coeffs = [], []
    for s in range(n):
        a, b = s, n + s
        c = np.zeros(4)
        for st in range(4):
            na, nb = st & 1, st >> 1
            c[st] = np.exp(J[a, a] * na + J[b, b] * nb + J[a, b] * na * nb)
        sites.append([s])
        coeffs.append(c)
    for s, t in itertools.combinations(range(n), 2):
        orb_s, orb_t = (s, n + s), (t, n + t)
        c = np.zeros(16)
        for st in range(16):
            occ_s = (st & 1, (st >> 1) & 1)  # site s is digit 0
            occ_t = ((st >> 2) & 1, (st >> 3) & 1)
            e = 0.0
            for u in range(2):
                for v in range(2):
                    e += J[orb_s[u], orb_t[v]] * occ_s[u] * occ_t[v]
            c[st] = np.exp(e)
        sites.append([s, t])
        coeffs.append(c)
    return sites, np.concatenate(coeffs)


def test_two_site_correlators_reproduce_the_jastrow_factor():
    wl = make_config("hubbard8")
    n, n_so = wl.n_orb, wl.n_so
    J = jastrow_dense(wl.jastrow, n_so)
    sites, coeffs = _cps_from_jastrow(J, n)
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    occ = np.stack([br.det_bits(k) for k in range(0, len(br.dets), 7)])
    with_j = OracleSystem.from_workload(wl)
    with_c = OracleSystem.from_workload(wl)
    with_c.set_params(np.zeros_like(wl.jastrow), wl.theta)
    with_c.set_cps(cps_pack(sites), coeffs)
    for o in occ:
        lj, sj = with_j.log_psi(o)
        lc, sc = with_c.log_psi(o)
        assert sj == sc and lc == pytest.approx(lj, abs=1e-12)
    for mode in (ORC_DET, ORC_LEMMA):
        ej, Tj, _, st1 = with_j.local_energy_batch(occ, mode)
        ec, Tc, _, st2 = with_c.local_energy_batch(occ, mode)
        assert np.all(st1 == 0) and np.all(st2 == 0)
        assert np.all(np.abs(ej - ec) <= _tol(Tj, 4.0))
        assert np.allclose(Tj, Tc, rtol=1e-12)


def test_cps_gradient_ratios_match_finite_differences():
    wl = make_config("hchain20", n_walkers=3, cps="chain3", cps_noise=0.2)
    orc = OracleSystem.from_workload(wl)
    n_cps = orc.num_cps_params()
    assert n_cps == wl.cps_coeffs.size == 18 * 64
    base = orc.n_params - n_cps
    rng = np.random.default_rng(5)
    for w in range(3):
        occ = wl.occ[w]
        O = orc.logderiv(occ)
        Oc = O[base:]
        # exactly one nonzero per correlator, 1/c at the state it sees
        nz = np.flatnonzero(Oc)
        assert nz.size == len(wl.cps_sites)
        assert np.allclose(Oc[nz], 1.0 / wl.cps_coeffs[nz], rtol=0, atol=0)
        for k in list(nz[:6]) + list(rng.choice(n_cps, 6, replace=False)):
            hstep = 1e-6
            cp, cm = wl.cps_coeffs.copy(), wl.cps_coeffs.copy()
            cp[k] += hstep
            cm[k] -= hstep
            orc.set_cps(wl.cps_sites, cp)
            lp, _ = orc.log_psi(occ)
            orc.set_cps(wl.cps_sites, cm)
            lm, _ = orc.log_psi(occ)
            fd = (lp - lm) / (2 * hstep)
            assert Oc[k] == pytest.approx(fd, rel=1e-6, abs=1e-9), k
        orc.set_cps(wl.cps_sites, wl.cps_coeffs)


def test_cps_site_list_validation():
    wl = make_config("hubbard8")
    orc = OracleSystem.from_workload(wl)
    with pytest.raises(ValueError):
        orc.set_cps(np.array([[0, 0, -1, -1, -1]]), np.ones(16))  # repeated site
    with pytest.raises(ValueError):
        orc.set_cps(np.array([[8, -1, -1, -1, -1]]), np.ones(4))  # site out of range
    assert orc.set_cps(np.zeros((0, 5)), np.zeros(0)) == 0
