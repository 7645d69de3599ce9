"""Seeded generators for Hamiltonians, wavefunction parameters and walkers.

Every routine is deterministic given its seed.  Nothing here evaluates the
VMC method itself.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

_MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


# ---------------------------------------------------------------------------
# Counter-based uniform numbers for O(1)-access integral draws (SplitMix64,
# Steele, Lea and Flood, OOPSLA 2014: the finaliser applied to a Weyl sequence).
# ---------------------------------------------------------------------------
def _splitmix64_mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed: int, tag: int, idx) -> np.ndarray:
    """Uniform [0,1) numbers addressed by (seed, tag, idx).

    z = mix(mix(seed XOR tag<<56) + idx); u = (z >> 11) * 2**-53.
    """
    base = _splitmix64_mix(np.uint64(seed) ^ (np.uint64(tag) << np.uint64(56)))
    with np.errstate(over="ignore"):
        z = _splitmix64_mix(base + np.asarray(idx, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---------------------------------------------------------------------------
# Canonical index helpers for 8-fold symmetric integrals
# ---------------------------------------------------------------------------
def canonical_pair(p, q):
    """pair(p,q) = max(p,q)*(max+1)/2 + min(p,q)."""
    p = np.asarray(p, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    hi = np.maximum(p, q)
    lo = np.minimum(p, q)
    return hi * (hi + 1) // 2 + lo


def canonical_quad(p, q, r, s):
    """Compound index of the class of (pq|rs) under the 8-fold symmetry."""
    a = canonical_pair(p, q)
    b = canonical_pair(r, s)
    hi = np.maximum(a, b)
    lo = np.minimum(a, b)
    return hi * (hi + 1) // 2 + lo


@dataclasses.dataclass
class Workload:
    """One synthetic system plus its initial wavefunction and walkers."""

    name: str
    n_orb: int
    n_alpha: int
    n_beta: int
    h1: np.ndarray  # (n, n) float64, symmetric
    eri_idx: np.ndarray  # (n_nz, 4) int32: p>=q, r>=s, pair(p,q)>=pair(r,s)
    eri_val: np.ndarray  # (n_nz,) float64
    eps: float
    theta: np.ndarray  # (n_so, n_so) float64, row-major
    jastrow: np.ndarray  # (n_so(n_so+1)/2,) float64, packed upper triangle
    occ: np.ndarray  # (W, n_words) uint64 occupation bitstrings
    ctmc_seed: int
    notes: str = ""
    orbitals: str = "ghf"  # "ghf" general, "uhf" spin-blocked theta
    # correlator product state: sites (n_corr, 5) int32 padded with -1, and the
    # 4^k coefficients of each correlator concatenated; empty = no correlators
    cps_sites: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 5), dtype=np.int32))
    cps_coeffs: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))

    @property
    def n_so(self) -> int:
        return 2 * self.n_orb

    @property
    def n_elec(self) -> int:
        return self.n_alpha + self.n_beta

    @property
    def n_walkers(self) -> int:
        return int(self.occ.shape[0])

    @property
    def n_words(self) -> int:
        return (self.n_so + 63) // 64


# ---------------------------------------------------------------------------
# Hamiltonians
# ---------------------------------------------------------------------------
def _hubbard_from_hopping(hop: np.ndarray, U: float):
    n = hop.shape[0]
    idx = np.array([[i, i, i, i] for i in range(n)], dtype=np.int32)
    val = np.full(n, float(U)) if U != 0.0 else np.zeros(0)
    if U == 0.0:
        idx = np.zeros((0, 4), dtype=np.int32)
    return hop.astype(np.float64), idx, val.astype(np.float64)


def hubbard_ring(L: int, t: float = 1.0, U: float = 4.0):
    """1-D ring with periodic boundary: h_{i,i+-1} = -t, (ii|ii) = U."""
    hop = np.zeros((L, L))
    for i in range(L):
        j = (i + 1) % L
        hop[i, j] -= t
        hop[j, i] -= t
    return _hubbard_from_hopping(hop, U)


def hubbard_2d(Lx: int, Ly: int, t: float = 1.0, U: float = 4.0):
    """Periodic Lx x Ly square lattice, site index = x*Ly + y."""
    n = Lx * Ly
    hop = np.zeros((n, n))
    for x in range(Lx):
        for y in range(Ly):
            i = x * Ly + y
            for (dx, dy) in ((1, 0), (0, 1)):
                j = ((x + dx) % Lx) * Ly + (y + dy) % Ly
                if j != i:
                    hop[i, j] -= t
                    hop[j, i] -= t
    return _hubbard_from_hopping(hop, U)


def hchain_like(n: int, seed: int, eri_cut: float = 0.0):
    """Synthetic H-chain-like ab initio Hamiltonian.

    h_pq = -exp(-|p-q|/1.5) * u_pq and
    (pq|rs) = exp(-(|p-q|+|r-s|)/1.2) * exp(-|p-r|/3) * v_pqrs,
    u, v = 0.5 + 0.5*U[0,1) drawn by SplitMix64 from (seed, index).  The
    two-electron formula is evaluated at the canonical representative
    (p>=q, r>=s, pair(p,q)>=pair(r,s)), which makes the list 8-fold symmetric.
    Entries with |value| <= eri_cut are left out of the list.
    """
    p, q = np.tril_indices(n)  # p >= q
    u = 0.5 + 0.5 * splitmix64_uniform(seed, 1, canonical_pair(p, q))
    h = np.zeros((n, n))
    vals = -np.exp(-np.abs(p - q) / 1.5) * u
    h[p, q] = vals
    h[q, p] = vals

    pairs_p, pairs_q = np.tril_indices(n)  # ordered by pair index (row-major tril)
    pair_id = canonical_pair(pairs_p, pairs_q)
    order = np.argsort(pair_id)
    pairs_p = pairs_p[order]
    pairs_q = pairs_q[order]
    npair = pairs_p.size
    idx_chunks = []
    val_chunks = []
    for A in range(npair):
        P, Q = pairs_p[A], pairs_q[A]
        R = pairs_p[: A + 1]
        S = pairs_q[: A + 1]
        val = np.exp(-((P - Q) + (R - S)) / 1.2) * np.exp(-np.abs(P - R) / 3.0)
        keep = val * 1.0 > eri_cut  # v <= 1: a cheap pre-filter
        if not np.any(keep):
            continue
        R = R[keep]
        S = S[keep]
        comp = canonical_quad(np.full(R.shape, P), np.full(R.shape, Q), R, S)
        v = 0.5 + 0.5 * splitmix64_uniform(seed, 2, comp)
        val = val[keep] * v
        keep2 = np.abs(val) > eri_cut
        if not np.any(keep2):
            continue
        quad = np.stack([np.full(R.shape, P), np.full(R.shape, Q), R, S], axis=1)[keep2]
        idx_chunks.append(quad.astype(np.int32))
        val_chunks.append(val[keep2])
    eri_idx = np.concatenate(idx_chunks, axis=0) if idx_chunks else np.zeros((0, 4), np.int32)
    eri_val = np.concatenate(val_chunks) if val_chunks else np.zeros(0)
    return h, eri_idx, eri_val.astype(np.float64)


def eri_dense_spatial(n: int, eri_idx: np.ndarray, eri_val: np.ndarray) -> np.ndarray:
    """Expand a canonical list to a dense (n,n,n,n) chemist-notation array."""
    g = np.zeros((n, n, n, n))
    for (p, q, r, s), v in zip(eri_idx.tolist(), eri_val.tolist()):
        for (a, b, c, d) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                             (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
            g[a, b, c, d] = v
    return g


# ---------------------------------------------------------------------------
# Wavefunction parameters and walkers
# ---------------------------------------------------------------------------
def init_theta(h1: np.ndarray, n_alpha: int, n_beta: int, noise: float, seed: int) -> np.ndarray:
    """GHF-form orbital matrix from the eigenvectors of h1.

    Columns: the n_alpha lowest alpha MOs, the n_beta lowest beta MOs, then the
    remaining alpha and beta MOs; N(0, noise) is added to every entry.
    """
    n = h1.shape[0]
    _, C = np.linalg.eigh(h1)
    n_so = 2 * n
    theta = np.zeros((n_so, n_so))
    col = 0
    for k in range(n_alpha):
        theta[:n, col] = C[:, k]
        col += 1
    for k in range(n_beta):
        theta[n:, col] = C[:, k]
        col += 1
    for k in range(n_alpha, n):
        theta[:n, col] = C[:, k]
        col += 1
    for k in range(n_beta, n):
        theta[n:, col] = C[:, k]
        col += 1
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        theta = theta + rng.normal(0.0, noise, size=theta.shape)
    return np.ascontiguousarray(theta)


def spin_blocked(theta: np.ndarray, n: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """Unrestricted (spin-blocked) form of an init_theta matrix: entries whose
    orbital row and column have different spins set to zero.  Column spins
    follow init_theta's layout: [0, na) alpha, [na, Ne) beta, then n - na alpha
    and n - nb beta virtual columns."""
    ne = n_alpha + n_beta
    col_beta = np.zeros(2 * n, dtype=bool)
    col_beta[n_alpha:ne] = True
    col_beta[ne + n - n_alpha:] = True
    row_beta = np.arange(2 * n) >= n
    out = np.array(theta, dtype=np.float64, copy=True)
    out[row_beta[:, None] != col_beta[None, :]] = 0.0
    return np.ascontiguousarray(out)


def init_jastrow(n_so: int, std: float, seed: int) -> np.ndarray:
    """Packed upper-triangular J (p<=q, row by row), entries N(0, std)."""
    m = n_so * (n_so + 1) // 2
    if std <= 0.0:
        return np.zeros(m)
    rng = np.random.default_rng(seed + 7919)
    return rng.normal(0.0, std, size=m)


def init_walkers(n: int, n_alpha: int, n_beta: int, n_walkers: int, seed: int) -> np.ndarray:
    """Uniformly random occupations per spin, as (W, n_words) uint64 bitstrings."""
    rng = np.random.default_rng(seed)
    n_so = 2 * n
    n_words = (n_so + 63) // 64
    occ = np.zeros((n_walkers, n_words), dtype=np.uint64)
    pa = np.argsort(rng.random((n_walkers, n)), axis=1)[:, :n_alpha]
    pb = np.argsort(rng.random((n_walkers, n)), axis=1)[:, :n_beta] + n
    orbs = np.concatenate([pa, pb], axis=1)
    for w in range(n_walkers):
        for o in orbs[w]:
            occ[w, o >> 6] |= np.uint64(1) << np.uint64(o & 63)
    return occ


# ---------------------------------------------------------------------------
# Correlator layouts (sites are spatial orbitals) and coefficients
# ---------------------------------------------------------------------------
def cps_chain_windows(n: int, k: int, periodic: bool = False):
    """k consecutive sites starting at every site of a chain (n - k + 1
    correlators) or of a ring (n correlators, wrapping round)."""
    starts = range(n) if periodic else range(n - k + 1)
    return [[(s0 + m) % n for m in range(k)] for s0 in starts]


def cps_square_plus(Lx: int, Ly: int):
    """One five-site correlator centred on each site of a periodic Lx x Ly
    square lattice (site index x*Ly + y): the site and its four neighbours."""
    out = []
    for x in range(Lx):
        for y in range(Ly):
            c = x * Ly + y
            nb = [((x + 1) % Lx) * Ly + y, ((x - 1) % Lx) * Ly + y, x * Ly + (y + 1) % Ly, x * Ly + (y - 1) % Ly]
            sites = [c]
            for t in nb:
                if t not in sites:
                    sites.append(t)
            out.append(sites)
    return out


def cps_pack(site_lists) -> np.ndarray:
    """(n_corr, 5) int32 site array, -1 after the last site of each correlator."""
    out = np.full((len(site_lists), 5), -1, dtype=np.int32)
    for l, st in enumerate(site_lists):
        if not 1 <= len(st) <= 5:
            raise ValueError("a correlator has 1 to 5 sites")
        out[l, : len(st)] = st
    return out


def init_cps(site_lists, noise: float, seed: int) -> np.ndarray:
    """Coefficients 1 + N(0, noise), 4^k per correlator, concatenated."""
    n = sum(4 ** len(st) for st in site_lists)
    rng = np.random.default_rng(seed + 104729)
    return 1.0 + rng.normal(0.0, noise, size=n) if noise > 0.0 else np.ones(n)


# ---------------------------------------------------------------------------
# Named configurations
# ---------------------------------------------------------------------------
CONFIG_NAMES = ("hubbard8", "hchain20", "hubbard10x10", "hchain160", "hchain40", "hchain80")


def make_config(name: str, n_walkers: Optional[int] = None, *, theta_noise: float = 0.01,
                jastrow_std: float = 0.05, U: Optional[float] = None, eps: Optional[float] = None,
                seed_offset: int = 0, orbitals: str = "ghf", cps: Optional[str] = None,
                cps_noise: float = 0.1) -> Workload:
    """Build one of the named workloads.

    hubbard8      8-site ring, t=1, U=4, 4+4 electrons, eps=0, 64 walkers
    hchain20      H-chain-like, 20 orbitals, 10+10, eps=1e-6, 4096 walkers
    hubbard10x10  10x10 periodic square lattice, U=4, 50+50, eps=0, 16384 walkers
    hchain160     H-chain-like, 160 orbitals, 80+80, eps=1e-5, 8192 walkers
    hchain40/80   members of the uneven batch (half filled, eps=1e-5, 2048 walkers)
    Seeds for configuration k: integrals 1000+k, psi 2000+k, walkers 3000+k,
    CTMC 4000+k.  orbitals="uhf" gives the spin-blocked (unrestricted) form of
    the same theta (spin_blocked).  cps adds correlators with coefficients
    1 + N(0, cps_noise): "chainK" (K consecutive sites from every site; a ring
    for hubbard8), or "plus5" (five-site crosses centred on every site of the
    10x10 lattice).
    """
    if orbitals not in ("ghf", "uhf"):
        raise ValueError(f"orbitals must be 'ghf' or 'uhf', not {orbitals!r}")
    table = {
        "hubbard8": (1, 64),
        "hchain20": (2, 4096),
        "hubbard10x10": (3, 16384),
        "hchain160": (4, 8192),
        "hchain40": (5, 2048),
        "hchain80": (6, 2048),
    }
    if name not in table:
        raise ValueError(f"unknown configuration {name!r}; known: {CONFIG_NAMES}")
    k, W = table[name]
    k += seed_offset
    if n_walkers is not None:
        W = n_walkers
    if name == "hubbard8":
        h1, ei, ev = hubbard_ring(8, 1.0, 4.0 if U is None else U)
        n, na, nb, e = 8, 4, 4, 0.0
    elif name == "hubbard10x10":
        h1, ei, ev = hubbard_2d(10, 10, 1.0, 4.0 if U is None else U)
        n, na, nb, e = 100, 50, 50, 0.0
    elif name == "hchain20":
        h1, ei, ev = hchain_like(20, 1000 + k, eri_cut=0.0)
        n, na, nb, e = 20, 10, 10, 1e-6
    else:
        n = {"hchain160": 160, "hchain40": 40, "hchain80": 80}[name]
        h1, ei, ev = hchain_like(n, 1000 + k, eri_cut=1e-10)
        na = nb = n // 2
        e = 1e-5
    if eps is not None:
        e = eps
    n_so = 2 * n
    theta = init_theta(h1, na, nb, theta_noise, 2000 + k)
    if orbitals == "uhf":
        theta = spin_blocked(theta, n, na, nb)
    jas = init_jastrow(n_so, jastrow_std, 2000 + k)
    occ = init_walkers(n, na, nb, W, 3000 + k)
    wl = Workload(name=name, n_orb=n, n_alpha=na, n_beta=nb, h1=h1, eri_idx=ei, eri_val=ev,
                  eps=e, theta=theta, jastrow=jas, occ=occ, ctmc_seed=4000 + k, orbitals=orbitals)
    if cps:
        if cps.startswith("chain"):
            sites = cps_chain_windows(n, int(cps[5:]), periodic=(name == "hubbard8"))
        elif cps == "plus5" and name == "hubbard10x10":
            sites = cps_square_plus(10, 10)
        else:
            raise ValueError(f"unknown correlator layout {cps!r} for {name}")
        wl.cps_sites = cps_pack(sites)
        wl.cps_coeffs = init_cps(sites, cps_noise, 2000 + k)
        wl.notes = f"correlators {cps}"
    return wl
