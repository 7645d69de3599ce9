"""Metropolis-Hastings comparator for the CTMC sampler.

TEST INFRASTRUCTURE ONLY: a plain sampler that the tests run beside the CTMC
walk to compare autocorrelation, never part of the library.

The paper contrasts its rejection-free CTMC walk with Metropolis-Hastings
(section "Continuous time Monte Carlo for sampling determinants") and reports a
shorter autocorrelation time for CTMC.  The comparator here uses the same
connected set as the CTMC walk (the screened singles and doubles of N, in the
oracle's canonical order) with a uniform proposal:
    propose M uniformly among the K(N) connected determinants,
    accept with probability min(1, |psi(M)/psi(N)|^2 K(N) / K(M)),
which is the Metropolis-Hastings acceptance for the proposal q(M|N) = 1/K(N),
so |psi|^2 is stationary (pinned exactly on a small space in the tests).  Each
step draws two uniforms from Philox4x64-10 with key (seed, walker) and counter
(step, 1, 0, 0): words 0 and 1, 53 high bits each, a stream disjoint from the
CTMC draws (counter word 1 = 0).
"""
from __future__ import annotations

import numpy as np

from .core import ORC_LEMMA, OracleSystem, philox4x64_10


def mh_uniforms(seed: int, walker: int, step: int):
    w = philox4x64_10([step, 1, 0, 0], [seed, walker])
    return float(int(w[0]) >> 11) * 2.0 ** -53, float(int(w[1]) >> 11) * 2.0 ** -53


def apply_excitation(occ: np.ndarray, c) -> np.ndarray:
    """The determinant reached by candidate c (fields type, i, j, a, b)."""
    m = np.array(occ, dtype=np.uint64, copy=True)

    def flip(p):
        m[p >> 6] ^= np.uint64(1) << np.uint64(p & 63)

    flip(int(c["i"]))
    flip(int(c["a"]))
    if int(c["type"]) == 2:
        flip(int(c["j"]))
        flip(int(c["b"]))
    return m


def acceptance(ratio: float, k_from: int, k_to: int) -> float:
    """min(1, |ratio|^2 K(from) / K(to)); a determinant with no connection
    cannot be proposed back to, so a move into one is refused."""
    if k_to == 0:
        return 0.0
    return min(1.0, ratio * ratio * k_from / k_to)


def mh_walk(orc: OracleSystem, occ0: np.ndarray, seed: int, walker: int, n_steps: int, step0: int = 0):
    """n_steps Metropolis-Hastings steps of one walker.  Returns (final occ,
    E_L of the state after each step, number of accepted moves)."""
    occ = np.array(occ0, dtype=np.uint64, copy=True)
    cur = orc.local_energy(occ, ORC_LEMMA, with_candidates=True)
    eloc = np.zeros(n_steps)
    accepted = 0
    for k in range(n_steps):
        u1, u2 = mh_uniforms(seed, walker, step0 + k)
        K = cur["n_cand"]
        if K > 0:
            c = cur["cand"][min(int(u1 * K), K - 1)]
            m = apply_excitation(occ, c)
            nxt = orc.local_energy(m, ORC_LEMMA, with_candidates=True)
            if u2 < acceptance(float(c["ratio"]), K, nxt["n_cand"]):
                occ, cur = m, nxt
                accepted += 1
        eloc[k] = cur["eloc"]
    return occ, eloc, accepted
