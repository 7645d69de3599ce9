"""Degenerate and boundary cases of the hot path on the GPU, through the C ABI:
one electron (no pair groups), a single walker, an empty screened set (T = 0),
walkers at a node of the determinant and with a wrong electron count (flagged,
never moved, no weight in the estimator), and the largest supported space
(512 spatial orbitals); the small Sherman-Morrison denominator flag and its
in-place re-inversion."""
import numpy as np
import pytest

from oracle.core import ORC_LEMMA, OracleSystem, list_to_occ
from workloads import Workload, hubbard_ring, init_jastrow, init_theta, init_walkers, make_config

from gpu_common import EL_TOL, el_tol, field, gpu_system, occ_of, run_sweep, teacher_forced_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _ring(L, na, nb, W, seed=11, U=4.0, eps=0.0):
    h1, ei, ev = hubbard_ring(L, 1.0, U)
    n_so = 2 * L
    return Workload(name=f"ring{L}_{na}_{nb}", n_orb=L, n_alpha=na, n_beta=nb, h1=h1, eri_idx=ei, eri_val=ev,
                    eps=eps, theta=init_theta(h1, na, nb, 0.01, seed), jastrow=init_jastrow(n_so, 0.05, seed),
                    occ=init_walkers(L, na, nb, W, seed + 1), ctmc_seed=seed + 2)


def test_one_electron_has_no_pair_groups(torch):
    wl = _ring(8, 1, 0, 64)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    occ0 = occ_of(sysm, walkers)
    eh, th, ph = run_sweep(sysm, walkers, 40)
    orc = OracleSystem.from_workload(wl)
    res = teacher_forced_check(orc, wl.ctmc_seed, occ0, 0, eh, th, ph, range(0, 64, 8))
    scaled = res["dE_all"] / (el_tol(res["T_all"]))
    assert scaled.max() <= 1.0 and not res["mismatches"], res["mismatches"][:3]


def test_single_walker(torch):
    wl = make_config("hchain20", n_walkers=1)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    occ0 = occ_of(sysm, walkers)
    eh, th, ph = run_sweep(sysm, walkers, 20)
    orc = OracleSystem.from_workload(wl)
    res = teacher_forced_check(orc, wl.ctmc_seed, occ0, 0, eh, th, ph, [0])
    # the walker starts from a random determinant: the bar scales with T there
    scaled = res["dE_all"] / (el_tol(res["T_all"]))
    assert scaled.max() <= 1.0 and not res["mismatches"]


def test_empty_screened_set_gives_no_move(torch):
    """eps above every bound: only H_NN remains, T = 0, t = 0, status EMPTY,
    and CTMC leaves the walkers where they are."""
    from paper_1807_10633_amd.vmc import vmc_local_energy

    wl = make_config("hchain20", n_walkers=32, eps=1e6)
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    hnn = field(sysm, walkers, "hnn", torch.float64, 1)[:, 0]
    tr = field(sysm, walkers, "tres", torch.float64, 1)[:, 0]
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    orc = OracleSystem.from_workload(wl)
    for w in (0, 31):
        r = orc.local_energy(wl.occ[w], ORC_LEMMA, with_candidates=False)
        assert r["T"] == 0.0 and abs(el[w] - r["eloc"]) <= EL_TOL
    assert np.all(el == hnn) and np.all(tr == 0.0) and np.all(st & 2)
    before = occ_of(sysm, walkers)
    eh, th, ph = run_sweep(sysm, walkers, 5)
    assert np.array_equal(before, occ_of(sysm, walkers)) and np.all(ph == 0)


def test_flagged_walkers_never_move_and_carry_no_weight(torch):
    """A walker on a node of the determinant (theta row of an occupied orbital
    zeroed) and a walker whose bits hold the wrong number of electrons are
    flagged SINGULAR at initialisation, get E_L = NaN and t = 0, are never moved,
    and vmc_estimate gives them no weight; the other walkers are unaffected."""
    from paper_1807_10633_amd.vmc import vmc_estimate, vmc_local_energy

    wl = make_config("hchain20", n_walkers=8)
    theta = wl.theta.copy()
    theta[0, :] = 0.0  # orbital 0 can never be occupied in a nonzero determinant
    occ = wl.occ.copy()
    orbs = [p for p in range(wl.n_so) if (int(occ[1][0]) >> p) & 1]
    if 0 not in orbs:  # put orbital 0 into walker 1 (alpha spin, swap one alpha electron)
        alpha = [p for p in orbs if p < wl.n_orb]
        orbs.remove(alpha[-1])
        orbs.append(0)
    occ[1] = list_to_occ(orbs, wl.n_so)
    occ[2] = occ[2] | np.uint64(1) << np.uint64(int([p for p in range(wl.n_so)
                                                      if not (int(occ[2][0]) >> p) & 1][0]))
    sysm = gpu_system(wl)
    sysm.set_params(torch.as_tensor(wl.jastrow, device="cuda"), torch.as_tensor(theta, device="cuda"))
    walkers = sysm.walkers(occ)
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    tr = field(sysm, walkers, "tres", torch.float64, 1)[:, 0]
    assert st[1] & 1 and st[2] & 1
    assert np.isnan(el[1]) and np.isnan(el[2]) and tr[1] == 0.0 and tr[2] == 0.0
    has0 = [w for w in range(8) if int(occ[w][0]) & 1]  # orbital 0 occupied: on the node as well
    good = [w for w in range(8) if w not in (1, 2) and w not in has0]
    assert len(good) >= 2
    assert np.all((st[good] & 1) == 0) and np.all(np.isfinite(el[good]))
    before = occ_of(sysm, walkers)
    eh, th, ph = run_sweep(sysm, walkers, 10)
    after = occ_of(sysm, walkers)
    assert np.array_equal(before[1:3], after[1:3]) and np.all(ph[:, 1:3] == 0)
    vmc_local_energy(sysm.handle, walkers)  # E_L of the post-move states
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    g = torch.zeros(8, dtype=torch.float64, device="cuda")
    vmc_estimate(sysm.handle, walkers, out, g)
    torch.cuda.synchronize()
    assert out[3].item() == 8 - len(set(has0) | {1, 2}) and g[1].item() == 0.0 and g[2].item() == 0.0
    orc = OracleSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, wl.eri_idx, wl.eri_val, wl.eps)
    orc.set_params(wl.jastrow, theta)
    for w in good[:3]:
        r = orc.local_energy(after[w], ORC_LEMMA, with_candidates=False)
        e = field(sysm, walkers, "eloc", torch.float64, 1)[w, 0]
        assert abs(e - r["eloc"]) <= el_tol(r["T"])


def test_largest_space_512_orbitals(torch):
    """n = 512 spatial orbitals (1024 spin-orbitals, 16 occupancy words), 2+2
    electrons, walker state in HBM.  The oracle's dense integral array does not
    reach this size, so the pin is the zero-variance identity: U = 0, J = 0 and
    exact ring orbitals give E_L = E0 = 2(-2 - 2 cos(2 pi/512)) for every
    determinant with psi != 0, before and after CTMC moves."""
    from paper_1807_10633_amd.vmc import System, vmc_launch_info, vmc_local_energy

    L = 512
    h1, ei, ev = hubbard_ring(L, 1.0, 0.0)
    theta = init_theta(h1, 2, 2, 0.0, 0)
    e0 = 2.0 * (-2.0 - 2.0 * np.cos(2.0 * np.pi / L))
    sysm = System(L, 2, 2, h1, ei, ev, 0.0, seed=5)
    sysm.set_params(torch.zeros(2 * L * (2 * L + 1) // 2, dtype=torch.float64, device="cuda"),
                    torch.as_tensor(theta, device="cuda"))
    assert not vmc_launch_info(sysm.handle)["state_in_lds"]
    walkers = sysm.walkers(init_walkers(L, 2, 2, 256, 29))
    vmc_local_energy(sysm.handle, walkers)
    torch.cuda.synchronize()
    el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
    tr = field(sysm, walkers, "tres", torch.float64, 1)[:, 0]
    st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
    ok = (st & 1) == 0
    T = 1.0 / np.where(tr > 0, tr, np.inf)
    # random determinants of plane-wave orbitals include a few that sit within
    # ~1e-10 of a node (T ~ 1e10-1e11, A conditioned like 1/T): there every FP64
    # ratio carries rounding of order 1e-12 T or more.  Those numerically nodal
    # states (T > 1e9) are only required to be finite and rare; the others are
    # held to 1e-10 + 1e-13 T, the well-conditioned majority (T < 1e3) to 1e-10.
    well = ok & (T < 1e3)
    nodal = ok & (T > 1e9)
    assert np.count_nonzero(well) > 200 and np.count_nonzero(nodal) <= 5
    assert np.all(np.abs(el[well] - e0) <= 1e-10)
    rest = ok & ~nodal
    assert np.all(np.abs(el[rest] - e0) <= 1e-10 + 1e-13 * T[rest])
    assert np.all(np.isfinite(el[ok]))
    eh, th, ph = run_sweep(sysm, walkers, 6)
    # a walker that started numerically nodal carries that inverse's rounding
    # through its Sherman-Morrison updates until the next refresh: the moves
    # are checked on the others
    live = np.isfinite(eh) & (th > 1e-9) & ~nodal[None, :]
    assert np.all(np.abs(eh[live] - e0) <= 1e-10 + 1e-13 / th[live])


@pytest.mark.parametrize("name,W,moves", [("hchain20", 64, 7), ("hchain160", 8, 2)])
def test_small_denominator_flags_and_reinverts(torch, name, W, moves):
    """The small Sherman-Morrison denominator threshold (the Sherman-Morrison
    paragraph of section "Local energy and Gradient ratios"): at the default
    1e-8 none of these moves is flagged; at +inf every move is flagged
    VMC_ST_SMALLDEN.  Where the sweep re-inverts in place (state in LDS: the
    20-orbital chain) the walker is re-inverted right after the move; walkers
    re-inverted by the separate kernel (the 160-orbital chain) wait for their
    next re-inversion.  Either way the state left behind inverts theta[N] for
    the walker's own slot order (against numpy) and E_L matches the oracle."""
    from paper_1807_10633_amd.vmc import VmcError, vmc_launch_info, vmc_local_energy, vmc_set_small_denominator

    ST_SMALLDEN = 8
    wl = make_config(name, n_walkers=W)
    sysm = gpu_system(wl)
    info = vmc_launch_info(sysm.handle)
    assert info["state_in_lds"] == (name == "hchain20")
    with pytest.raises(VmcError):
        vmc_set_small_denominator(sysm.handle, -1.0)
    ne = wl.n_elec
    for thr in (1e-8, float("inf")):
        vmc_set_small_denominator(sysm.handle, thr)
        walkers = sysm.walkers(wl.occ)
        run_sweep(sysm, walkers, moves)
        vmc_local_energy(sysm.handle, walkers)
        torch.cuda.synchronize()
        st = field(sysm, walkers, "status", torch.int32, 1)[:, 0]
        moved = field(sysm, walkers, "pick", torch.int64, 1)[:, 0] != 0
        assert np.all((st & 1) == 0)
        if thr == 1e-8:
            assert not np.any(st & ST_SMALLDEN)
            continue
        assert moved.any() and np.all((st[moved] & ST_SMALLDEN) != 0)
        B = field(sysm, walkers, "ainv", torch.float64, ne * ne).reshape(W, ne, ne)
        so = field(sysm, walkers, "slot_orb", torch.int32, ne)
        for w in range(min(W, 4)):
            A = wl.theta[so[w], :ne]
            # B[p][x] = (A^-1)[x][p]: A B^T = I
            res = np.abs(A @ B[w].T - np.eye(ne)).max()
            assert res <= 1e-9, (w, res)
        el = field(sysm, walkers, "eloc", torch.float64, 1)[:, 0]
        orc = OracleSystem.from_workload(wl)
        occ = occ_of(sysm, walkers)
        idx = np.arange(0, W, max(1, W // 8))
        e_o, T_o, _, sto = orc.local_energy_batch(occ[idx], ORC_LEMMA, 16)
        assert np.all(sto == 0)
        assert np.all(np.abs(el[idx] - e_o) <= el_tol(T_o))
    vmc_set_small_denominator(sysm.handle, 1e-8)
