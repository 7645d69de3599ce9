"""Pins of the oracle on spin-blocked (unrestricted) orbitals, the determinant
form of the paper's benchmarks (sections "Performance of the optimizer" and
"2-D Hubbard Model Benchmark").

With theta[a][x] = 0 wherever orbital a and occupied column x differ in spin,
theta[N] (rows in ascending orbital order, alpha first) is block diagonal, so
det theta[N] = det theta_alpha[N_alpha] * det theta_beta[N_beta].  The oracle
itself knows nothing of spin blocks (it forms and factors the full N_e x N_e
matrices); these tests hold its ratios and log|psi| to that factorisation,
computed here with numpy on the two blocks separately, and check the host-side
layout of workloads.spin_blocked."""
import numpy as np
import pytest

from oracle.core import ORC_DET, ORC_LEMMA, OracleSystem, occ_to_list
from workloads import init_theta, make_config, spin_blocked


def _block_dets(theta, rows, n, na, nb):
    """det of the alpha and beta blocks of theta[rows] (rows sorted)."""
    rows = sorted(rows)
    ra = [o for o in rows if o < n]
    rb = [o for o in rows if o >= n]
    assert len(ra) == na and len(rb) == nb
    da = np.linalg.det(theta[np.array(ra, dtype=int)][:, :na]) if na else 1.0
    db = np.linalg.det(theta[np.array(rb, dtype=int)][:, na:na + nb]) if nb else 1.0
    return da, db


@pytest.mark.parametrize("name,W", [("hubbard8", 6), ("hchain20", 4)])
@pytest.mark.parametrize("mode", [ORC_DET, ORC_LEMMA])
def test_ratios_factor_over_the_two_spins(name, W, mode):
    wl = make_config(name, n_walkers=W, orbitals="uhf")
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    orc = OracleSystem.from_workload(wl)
    orc.set_params(np.zeros_like(wl.jastrow), wl.theta)  # no Jastrow: the ratio is the determinant ratio
    seen = set()
    worst = 0.0
    for w in range(W):
        occ = occ_to_list(wl.occ[w], wl.n_so)
        da0, db0 = _block_dets(wl.theta, occ, n, na, nb)
        r = orc.local_energy(wl.occ[w], mode, with_candidates=True)
        for c in r["cand"]:
            rows = list(occ)
            rows[rows.index(int(c["i"]))] = int(c["a"])
            if c["type"] == 2:
                rows[rows.index(int(c["j"]))] = int(c["b"])
            da, db = _block_dets(wl.theta, rows, n, na, nb)
            ref = (da / da0) * (db / db0)
            worst = max(worst, abs(c["ratio"] - ref) / max(1.0, abs(ref)))
            spins = (int(c["i"]) >= n, int(c["j"]) >= n) if c["type"] == 2 else (int(c["i"]) >= n,)
            seen.add((int(c["type"]), spins))
            if c["type"] == 2 and spins == (False, True):
                # opposite spins: the product of the two single-spin ratios
                ra = list(occ)
                ra[ra.index(int(c["i"]))] = int(c["a"])
                rb = list(occ)
                rb[rb.index(int(c["j"]))] = int(c["b"])
                s_a = _block_dets(wl.theta, ra, n, na, nb)[0] / da0
                s_b = _block_dets(wl.theta, rb, n, na, nb)[1] / db0
                assert abs(c["ratio"] - s_a * s_b) <= 1e-10 * max(1.0, abs(s_a * s_b))
    assert worst <= 1e-10, worst
    # every kind of move was exercised: alpha and beta singles, and for the
    # H-chain doubles of both same-spin kinds and of opposite spins
    assert {(1, (False,)), (1, (True,))} <= seen
    if name == "hchain20":
        assert {(2, (False, False)), (2, (True, True)), (2, (False, True))} <= seen


def test_log_psi_is_the_sum_of_the_two_spins():
    wl = make_config("hchain20", n_walkers=5, orbitals="uhf")
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    orc = OracleSystem.from_workload(wl)
    orc.set_params(np.zeros_like(wl.jastrow), wl.theta)
    for w in range(5):
        occ = occ_to_list(wl.occ[w], wl.n_so)
        da, db = _block_dets(wl.theta, occ, n, na, nb)
        lp, sg = orc.log_psi(wl.occ[w])
        assert abs(lp - (np.log(abs(da)) + np.log(abs(db)))) <= 1e-10
        assert sg == int(np.sign(da * db))


def test_spin_blocked_layout():
    """Entries kept: alpha rows in columns [0, na) and the na..n-1 alpha virtual
    columns; beta rows in [na, Ne) and the beta virtual columns."""
    from workloads import hubbard_ring

    h1, _, _ = hubbard_ring(6, 1.0, 4.0)
    n, na, nb = 6, 3, 2
    th = init_theta(h1, na, nb, 0.1, 3)
    ub = spin_blocked(th, n, na, nb)
    ne = na + nb
    alpha_cols = list(range(na)) + list(range(ne, ne + n - na))
    for a in range(2 * n):
        for x in range(2 * n):
            same = (a < n) == (x in alpha_cols)
            assert ub[a, x] == (th[a, x] if same else 0.0)
    # every column is one spin's orbital: n - na + na alpha, the rest beta
    assert len(alpha_cols) == n
