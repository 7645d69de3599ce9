"""CTMC against Metropolis-Hastings on the 8-site ring (section "Continuous time
Monte Carlo for sampling determinants": the CTMC walk is rejection free and
reported to decorrelate faster).

The CTMC walk runs on the GPU (vmc_ctmc_step with E_L and residence-time
histories), the Metropolis-Hastings comparator in the oracle (oracle/mh.py),
both over the same connected set.  Both estimates must agree with the exact
<psi|H|psi> of the brute-force wave function.  The statistical inefficiency
(block variance over sample variance, about twice the integrated
autocorrelation time) and the error of the mean per square root of steps are
printed for the comparison.
"""
import numpy as np
import pytest

from oracle.brute import BruteSystem
from oracle.core import OracleSystem
from oracle.mh import mh_walk
from workloads import eri_dense_spatial, make_config

from gpu_common import gpu_system, run_sweep

pytestmark = pytest.mark.gpu

BLOCK = 100


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _blocks(e, t):
    """Block means (t-weighted) of per-walker series e, t of shape (steps, W)."""
    n = (e.shape[0] // BLOCK) * BLOCK
    e, t = e[:n], t[:n]
    eb = (e * t).reshape(-1, BLOCK, e.shape[1]).sum(axis=1) / t.reshape(-1, BLOCK, e.shape[1]).sum(axis=1)
    return eb.reshape(-1)


def test_ctmc_and_metropolis_hastings_sample_the_same_energy(torch):
    wl = make_config("hubbard8", n_walkers=64)
    br = BruteSystem(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, eri_dense_spatial(wl.n_orb, wl.eri_idx, wl.eri_val))
    e_exact = br.energy(br.psi(wl.theta, wl.jastrow))
    # CTMC on the GPU: 64 walkers x 4200 moves, the first 200 dropped
    sysm = gpu_system(wl)
    walkers = sysm.walkers(wl.occ)
    eh, th, _ = run_sweep(sysm, walkers, 4200)
    eh, th = eh[200:], th[200:]
    e_ctmc = float(np.sum(eh * th) / np.sum(th))
    var_ctmc = float(np.sum(th * (eh - e_ctmc) ** 2) / np.sum(th))
    b = _blocks(eh, th)
    err_ctmc = b.std(ddof=1) / np.sqrt(b.size)
    s_ctmc = BLOCK * b.var(ddof=1) / var_ctmc
    # Metropolis-Hastings in the oracle: 16 walkers x 4200 steps
    orc = OracleSystem.from_workload(wl)
    series, acc = [], 0
    for w in range(16):
        _, el, a = mh_walk(orc, wl.occ[w], wl.ctmc_seed, w, 4200)
        series.append(el[200:])
        acc += a
    em = np.array(series).T
    e_mh = float(em.mean())
    bm = _blocks(em, np.ones_like(em))
    err_mh = bm.std(ddof=1) / np.sqrt(bm.size)
    s_mh = BLOCK * bm.var(ddof=1) / em.var()
    n_ctmc, n_mh = eh.size, em.size
    print(f"    exact <H> {e_exact:.5f}; CTMC {e_ctmc:.5f} +- {err_ctmc:.5f} ({n_ctmc} steps, inefficiency "
          f"{s_ctmc:.2f}, error x sqrt(steps) {err_ctmc * np.sqrt(n_ctmc):.3f}); MH {e_mh:.5f} +- {err_mh:.5f} "
          f"({n_mh} steps, acceptance {acc / (16 * 4200):.3f}, inefficiency {s_mh:.2f}, error x sqrt(steps) "
          f"{err_mh * np.sqrt(n_mh):.3f})", flush=True)
    assert abs(e_ctmc - e_exact) < 5 * err_ctmc
    assert abs(e_mh - e_exact) < 5 * err_mh
