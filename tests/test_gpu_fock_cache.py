"""The walkers' singles elements H_ia = h_ia + sum_j V_ia[j], kept in the
scratch between launches (walker state in HBM) with a tag naming the
occupation and the system they belong to.

* After a CTMC sweep, E_L with the kept elements equals E_L on a twin walker
  set whose scratch was zero-filled (elements rebuilt), to rounding, and the
  oracle's on sampled walkers.
* Walkers re-initialised to other determinants, and walkers carrying the
  scratch of another system with the same tables (the Hamiltonian doubled),
  do not reuse stale elements: E_L matches the oracle.
"""
import dataclasses

import numpy as np
import pytest

from oracle.core import ORC_LEMMA, OracleSystem
from workloads import make_config

from gpu_common import el_tol, field, gpu_system, occ_of

pytestmark = pytest.mark.gpu

W = 256


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(*a):
    print(*a, flush=True)


def _check_oracle(wl, s, wk, torch, idx):
    el = field(s, wk, "eloc", torch.float64, 1)[:, 0]
    occ = occ_of(s, wk)
    orc = OracleSystem.from_workload(wl)
    worst = 0.0
    for w in idx:
        r = orc.local_energy(occ[w], ORC_LEMMA, with_candidates=False)
        d = abs(el[w] - r["eloc"])
        worst = max(worst, d / el_tol(r["T"]))
        assert d <= el_tol(r["T"]), (wl.name, w, el[w], r["eloc"])
    return worst


def test_kept_singles_elements_match_rebuilt_ones(torch):
    from paper_1807_10633_amd.vmc import vmc_ctmc_step, vmc_launch_info, vmc_local_energy

    wl = make_config("hchain40", n_walkers=W)
    s = gpu_system(wl)
    assert not vmc_launch_info(s.handle)["state_in_lds"]
    _say("[fock cache] hchain40: kept vs rebuilt")
    a, b = s.walkers(wl.occ), s.walkers(wl.occ)
    for wk in (a, b):
        vmc_ctmc_step(s.handle, wk, 30)
    b.view("scratch", torch.uint8).zero_()  # clears every tag: b rebuilds its elements
    vmc_local_energy(s.handle, a)
    vmc_local_energy(s.handle, b)
    torch.cuda.synchronize()
    assert np.array_equal(occ_of(s, a), occ_of(s, b))
    ea = field(s, a, "eloc", torch.float64, 1)[:, 0]
    eb = field(s, b, "eloc", torch.float64, 1)[:, 0]
    scale = np.maximum(1.0, np.abs(eb))
    assert np.max(np.abs(ea - eb) / scale) <= 1e-12, np.max(np.abs(ea - eb) / scale)
    worst = _check_oracle(wl, s, a, torch, (0, W // 3, W - 1))
    # a second sweep continues from the kept elements
    vmc_ctmc_step(s.handle, a, 20)
    vmc_local_energy(s.handle, a)
    torch.cuda.synchronize()
    worst = max(worst, _check_oracle(wl, s, a, torch, (1, W // 2)))
    _say(f"    max |E_L kept - E_L rebuilt| / max(1, |E_L|) = {np.max(np.abs(ea - eb) / scale):.3g}; "
         f"worst |dE|/tol vs oracle {worst:.3g}")


def test_stale_singles_elements_are_not_reused(torch):
    from paper_1807_10633_amd.vmc import vmc_ctmc_step, vmc_local_energy, vmc_walkers_init

    wl = make_config("hchain40", n_walkers=W)
    s = gpu_system(wl)
    a = s.walkers(wl.occ)
    vmc_ctmc_step(s.handle, a, 25)
    torch.cuda.synchronize()
    # other determinants written into the same walker set (its scratch still
    # holds the elements of the swept occupations)
    other = np.roll(wl.occ, 7, axis=0)
    a.view("occ_bits", torch.int64)[: other.size].copy_(torch.from_numpy(other.view(np.int64).reshape(-1)))
    vmc_walkers_init(s.handle, a)
    vmc_local_energy(s.handle, a)
    torch.cuda.synchronize()
    assert np.array_equal(occ_of(s, a), other)
    w1 = _check_oracle(wl, s, a, torch, (0, 5, W - 2))
    # a second system with the Hamiltonian and the threshold doubled: the
    # same screened tables (so the same scratch layout), singles elements
    # twice as large; its walkers get the first system's scratch bytes
    wl2 = dataclasses.replace(wl, h1=2.0 * wl.h1, eri_val=2.0 * wl.eri_val, eps=2.0 * wl.eps)
    s2 = gpu_system(wl2)
    b = s.walkers(wl.occ)
    vmc_ctmc_step(s.handle, b, 10)
    torch.cuda.synchronize()
    b2 = s2.walkers(occ_of(s, b))
    assert b2.view("scratch", torch.uint8).numel() == b.view("scratch", torch.uint8).numel()
    b2.view("scratch", torch.uint8).copy_(b.view("scratch", torch.uint8))
    vmc_local_energy(s2.handle, b2)
    torch.cuda.synchronize()
    w2 = _check_oracle(wl2, s2, b2, torch, (2, W // 2, W - 1))
    _say(f"[fock cache] re-initialised walkers: worst |dE|/tol {w1:.3g}; other system: {w2:.3g}")
