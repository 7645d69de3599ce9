"""Seeded synthetic workloads for screened orbital-space VMC.

This module only *generates inputs*: model Hamiltonians (one-electron matrix and
a canonical list of two-electron integrals), initial wavefunction parameters and
walker occupations.  It contains none of the method's arithmetic (no local
energies, ratios, screening or sampling), so it can feed both the CPU oracle and
the GPU library without coupling them.

Conventions shared by every consumer of these inputs
----------------------------------------------------
* Spatial orbitals are numbered 0..n-1.  Spin-orbitals are block ordered:
  alpha = 0..n-1, beta = n..2n-1.
* Two-electron integrals are real, in chemist notation (pq|rs), with the 8-fold
  permutational symmetry.  They are passed as a *canonical list*: one entry per
  class of equivalent index quadruples, represented by p>=q, r>=s and
  pair(p,q) >= pair(r,s), where pair(p,q) = p(p+1)/2 + q for p>=q.
* The Jastrow matrix J is passed packed: the upper triangle (p<=q) row by row.
* The orbital matrix theta is n_so x n_so, row-major (row = spin-orbital,
  column = molecular orbital); the determinant uses columns 0..N_e-1.
* Occupations are little-endian bitstrings in 64-bit words, ceil(n_so/64) words
  per walker.
* Correlators (optional): each is a list of at most five sites (spatial
  orbitals), passed as an (n_corr, 5) int32 array padded with -1, with the 4^k
  coefficients of each correlator concatenated in correlator order.

The Hubbard and H-chain-like models stand in for the paper's benchmark systems
(2-D Hubbard lattices and sto-6g hydrogen chains), whose integrals cannot be
produced here; `make_config` documents the recipe of each configuration.
"""
from .generators import (  # noqa: F401
    Workload,
    canonical_pair,
    canonical_quad,
    hubbard_ring,
    hubbard_2d,
    hchain_like,
    splitmix64_uniform,
    init_theta,
    spin_blocked,
    init_jastrow,
    init_walkers,
    eri_dense_spatial,
    make_config,
    CONFIG_NAMES,
    cps_chain_windows,
    cps_square_plus,
    cps_pack,
    init_cps,
)
