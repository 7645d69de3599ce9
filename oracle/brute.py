"""Brute force over a whole (N_alpha, N_beta) sector, for tiny systems only.

TEST INFRASTRUCTURE ONLY.  This is the oracle's own pin: it never uses
Slater-Condon rules, screening, ratios or determinant lemmas.  The Hamiltonian
matrix comes from the second-quantised operator

    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps),
    E_pq = sum_sigma a+_{p sigma} a_{q sigma},

with each one-body operator E^sigma_pq applied to every determinant of the
sector (Jordan-Wigner signs counted on the bitstring).  From it:

* E_L(N) = sum_M H_NM psi(M) / psi(N)  (the unscreened local energy of
  Eq. eloc:hci's parent expression),
* E = <psi|H|psi>/<psi|psi> = sum_N rho_N E_L(N)  (Eq. eq:vmc),
* the exact ground-state energy by diagonalisation,
* psi(N) = C[N] exp(sum_{p<=q} J_pq n_p n_q) det(theta[occ(N), 0:Ne]) with
  numpy's determinant, C[N] the correlator product: for each correlator (a
  list of sites, i.e. spatial orbitals) the coefficient of the site
  occupations it sees, read off the bitstring site by site (alpha and beta
  occupation of site s_m giving digit n_alpha + 2 n_beta in place m of a base-4
  number).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp


def sector_basis(n: int, na: int, nb: int) -> Tuple[List[int], Dict[int, int]]:
    """Determinants as Python-int bitstrings (alpha bits 0..n-1, beta n..2n-1)."""
    dets = []
    for ca in itertools.combinations(range(n), na):
        ma = 0
        for p in ca:
            ma |= 1 << p
        for cb in itertools.combinations(range(n), nb):
            mb = 0
            for p in cb:
                mb |= 1 << (p + n)
            dets.append(ma | mb)
    dets.sort()
    return dets, {d: k for k, d in enumerate(dets)}


def _popcount_below(d: int, p: int) -> int:
    return bin(d & ((1 << p) - 1)).count("1")


def one_body_ops(n: int, dets: List[int], index: Dict[int, int]):
    """Spin-summed E_pq as a dict (p, q) -> scipy CSR matrix (D x D)."""
    D = len(dets)
    ops = {}
    for p in range(n):
        for q in range(n):
            rows, cols, vals = [], [], []
            for sigma in (0, 1):
                ps, qs = p + sigma * n, q + sigma * n
                for k, d in enumerate(dets):
                    if not (d >> qs) & 1:
                        continue
                    sgn = -1 if _popcount_below(d, qs) & 1 else 1
                    d1 = d ^ (1 << qs)
                    if (d1 >> ps) & 1:
                        continue
                    if _popcount_below(d1, ps) & 1:
                        sgn = -sgn
                    d2 = d1 | (1 << ps)
                    rows.append(index[d2])
                    cols.append(k)
                    vals.append(float(sgn))
            ops[(p, q)] = sp.csr_matrix((vals, (rows, cols)), shape=(D, D))
    return ops


def hamiltonian_matrix(h1: np.ndarray, g: np.ndarray, dets: List[int], index: Dict[int, int]) -> np.ndarray:
    """Dense H over the sector; g is the dense chemist-notation (pq|rs)."""
    n = h1.shape[0]
    D = len(dets)
    E = one_body_ops(n, dets, index)
    H = sp.csr_matrix((D, D))
    for (p, q), op in E.items():
        if h1[p, q] != 0.0:
            H = H + h1[p, q] * op
    for p in range(n):
        for q in range(n):
            F = sp.csr_matrix((D, D))
            any_term = False
            for r in range(n):
                for s in range(n):
                    if g[p, q, r, s] != 0.0:
                        F = F + g[p, q, r, s] * E[(r, s)]
                        any_term = True
            if any_term:
                H = H + 0.5 * (E[(p, q)] @ F)
            for s in range(n):
                if g[p, q, q, s] != 0.0:
                    H = H - 0.5 * g[p, q, q, s] * E[(p, s)]
    return np.asarray(H.todense())


def occ_list(d: int, n_so: int) -> List[int]:
    return [p for p in range(n_so) if (d >> p) & 1]


def jastrow_dense(J_packed: np.ndarray, n_so: int) -> np.ndarray:
    J = np.zeros((n_so, n_so))
    iu = np.triu_indices(n_so)
    J[iu] = J_packed
    J[(iu[1], iu[0])] = J_packed
    return J


def correlator_product(d: int, n: int, sites, coeffs) -> float:
    """C[N] for the bitstring d: sites is a list of site lists, coeffs a list
    of coefficient arrays (4^len(sites[l]) each)."""
    c = 1.0
    for lam, vals in zip(sites, coeffs):
        digits = []
        for s in lam:
            up = (d >> s) & 1
            dn = (d >> (n + s)) & 1
            digits.append(up + 2 * dn)
        state = 0
        for m in reversed(range(len(digits))):
            state = 4 * state + digits[m]
        c *= float(vals[state])
    return c


def psi_vector(theta: np.ndarray, J_packed: np.ndarray, dets: List[int], n_so: int, ne: int, cps=None) -> np.ndarray:
    """cps: None, or (sites, coeffs) as for correlator_product."""
    J = jastrow_dense(J_packed, n_so)
    out = np.zeros(len(dets))
    for k, d in enumerate(dets):
        occ = occ_list(d, n_so)
        logj = 0.0
        for x in range(len(occ)):
            for y in range(x, len(occ)):
                logj += J[occ[x], occ[y]]
        out[k] = np.exp(logj) * np.linalg.det(theta[np.array(occ)][:, :ne])
        if cps is not None:
            out[k] *= correlator_product(d, n_so // 2, cps[0], cps[1])
    return out


class BruteSystem:
    """Full-sector brute force for one small workload."""

    def __init__(self, n: int, na: int, nb: int, h1: np.ndarray, g: np.ndarray):
        self.n, self.na, self.nb = n, na, nb
        self.n_so = 2 * n
        self.ne = na + nb
        self.dets, self.index = sector_basis(n, na, nb)
        self.H = hamiltonian_matrix(h1, g, self.dets, self.index)

    def psi(self, theta: np.ndarray, J_packed: np.ndarray, cps=None) -> np.ndarray:
        return psi_vector(theta, J_packed, self.dets, self.n_so, self.ne, cps)

    def local_energies(self, psi: np.ndarray) -> np.ndarray:
        return (self.H @ psi) / psi

    def energy(self, psi: np.ndarray) -> float:
        return float(psi @ self.H @ psi / (psi @ psi))

    def ground_energy(self) -> float:
        return float(np.linalg.eigvalsh(self.H)[0])

    def det_bits(self, k: int) -> np.ndarray:
        d = self.dets[k]
        nw = (self.n_so + 63) // 64
        return np.array([(d >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(nw)], dtype=np.uint64)

    def connected(self, k: int) -> Dict[int, float]:
        """{M index: H_MN} for all M != N with a non-zero element."""
        col = self.H[:, k]
        return {m: float(col[m]) for m in np.nonzero(col)[0] if m != k}
