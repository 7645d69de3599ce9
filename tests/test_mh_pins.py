"""Pins of the Metropolis-Hastings comparator (oracle/mh.py), on the CPU.

* Its transition matrix on the 8-site ring (all 4900 determinants, built from
  the oracle's candidate lists) satisfies detailed balance with rho = |psi|^2
  from the brute-force wave function, so rho is stationary.
* The sampled walk on a 4-site ring (36 determinants) visits the determinants
  with frequencies rho and averages E_L to the exact <psi|H|psi>.
"""
import numpy as np

from oracle.brute import BruteSystem
from oracle.core import ORC_LEMMA, OracleSystem
from oracle.mh import acceptance, mh_walk
from workloads import Workload, eri_dense_spatial, hubbard_ring, init_jastrow, init_theta, init_walkers, make_config


def _transition_matrix(br, orc):
    D = len(br.dets)
    K = np.zeros(D, dtype=np.int64)
    cands = []
    for k in range(D):
        r = orc.local_energy(br.det_bits(k), ORC_LEMMA)
        K[k] = r["n_cand"]
        cands.append(r["cand"])
    P = np.zeros((D, D))
    for k in range(D):
        N = br.dets[k]
        for c in cands[k]:
            M = N & ~(1 << int(c["i"])) | (1 << int(c["a"]))
            if c["type"] == 2:
                M = M & ~(1 << int(c["j"])) | (1 << int(c["b"]))
            m = br.index[M]
            P[k, m] += acceptance(float(c["ratio"]), int(K[k]), int(K[m])) / K[k]
        P[k, k] += 1.0 - P[k].sum()
    return P, K


def test_mh_transition_matrix_satisfies_detailed_balance_hubbard8():
    wl = make_config("hubbard8")
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    psi = br.psi(wl.theta, wl.jastrow)
    rho = psi ** 2 / np.sum(psi ** 2)
    orc = OracleSystem.from_workload(wl)
    P, K = _transition_matrix(br, orc)
    assert np.min(K) > 0 and np.max(K) > np.min(K)  # the proposal is not symmetric: the K ratio matters
    assert np.all(P >= -1e-15) and np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
    F = rho[:, None] * P
    assert np.max(np.abs(F - F.T)) < 1e-15
    assert np.max(np.abs(rho @ P - rho)) < 1e-14


def test_mh_walk_samples_rho_on_a_small_ring():
    L, na, nb = 4, 2, 2
    h1, ei, ev = hubbard_ring(L, 1.0, 4.0)
    wl = Workload(name="ring4", n_orb=L, n_alpha=na, n_beta=nb, h1=h1, eri_idx=ei, eri_val=ev, eps=0.0,
                  theta=init_theta(h1, na, nb, 0.05, 3), jastrow=init_jastrow(2 * L, 0.2, 3),
                  occ=init_walkers(L, na, nb, 4, 4), ctmc_seed=5)
    br = BruteSystem(L, na, nb, h1, eri_dense_spatial(L, ei, ev))
    psi = br.psi(wl.theta, wl.jastrow)
    rho = psi ** 2 / np.sum(psi ** 2)
    e_exact = br.energy(psi)
    orc = OracleSystem.from_workload(wl)
    counts = np.zeros(len(br.dets))
    means = []
    n = 20000
    for w in range(4):
        occ = wl.occ[w]
        occ, el, acc = mh_walk(orc, occ, 77, w, n)
        assert 0 < acc < n
        means.append(el[1000:].reshape(-1, 950).mean(axis=1))  # block means after a burn-in
    blocks = np.concatenate(means)
    err = blocks.std(ddof=1) / np.sqrt(blocks.size)
    assert abs(blocks.mean() - e_exact) < 5 * err, (blocks.mean(), e_exact, err)
    # visit frequencies: the final states of 400 independent 60-step walks
    for w in range(400):
        occ, _, _ = mh_walk(orc, wl.occ[w % 4], 91, w, 60)
        counts[br.index[sum(1 << p for p in range(2 * L) if (int(occ[0]) >> p) & 1)]] += 1
    freq = counts / counts.sum()
    assert np.max(np.abs(freq - rho)) < 0.06
