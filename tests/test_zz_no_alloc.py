"""The allocation-free CTMC entry point (vmc_ctmc_step_static) through the C
ABI: its moves equal vmc_ctmc_step's bit for bit on identical walker copies,
on two calls in a row, the second with fewer walkers, with the walkers'
own workspace field left NULL; a walker set too large for the static
workspace is refused before any work."""
import ctypes as C

import numpy as np
import pytest

from workloads import make_config

from gpu_common import field, gpu_system, occ_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _state(torch, s, wk):
    return {"occ": occ_of(s, wk), "eloc": field(s, wk, "eloc", torch.float64, 1),
            "tres": field(s, wk, "tres", torch.float64, 1), "pick": field(s, wk, "pick", torch.int64, 1),
            "B": field(s, wk, "ainv", torch.float64, s.ne * s.ne), "R": field(s, wk, "r", torch.float64, s.ne * s.n_so),
            "status": field(s, wk, "status", torch.int32, 1)}


@pytest.mark.parametrize("name", ["hchain40", "hchain20"])
def test_static_workspace_step_equals_ctmc_step(torch, name):
    from paper_1807_10633_amd.vmc import VmcError, vmc_ctmc_step, vmc_ctmc_step_static, vmc_walker_bytes

    print(f"[static workspace] {name}", flush=True)
    for W, moves in ((64, 57), (32, 23)):  # the second call with a smaller input
        wl = make_config(name, n_walkers=W)
        sysm = gpu_system(wl)
        ref = sysm.walkers(wl.occ)
        sta = sysm.walkers(wl.occ)
        sta.cstruct.scratch = None  # the static entry point does not read it
        n = moves * W
        eh_r = torch.zeros(n, dtype=torch.float64, device="cuda")
        eh_s = torch.zeros(n, dtype=torch.float64, device="cuda")
        ph_r = torch.zeros(n, dtype=torch.int64, device="cuda")
        ph_s = torch.zeros(n, dtype=torch.int64, device="cuda")
        vmc_ctmc_step(sysm.handle, ref, moves, eh_r, None, ph_r)
        vmc_ctmc_step_static(sysm.handle, sta, moves, eh_s, None, ph_s)
        torch.cuda.synchronize()
        assert ref.step == sta.step == moves and ref.since_inv == sta.since_inv
        a, b = _state(torch, sysm, ref), _state(torch, sysm, sta)
        for k in a:
            assert np.array_equal(a[k], b[k]), (name, W, k)
        assert torch.equal(eh_r, eh_s) and torch.equal(ph_r, ph_s)
        assert np.all((a["status"] & 1) == 0)
    # a walker set beyond the 64 MiB workspace is refused on the host
    per = vmc_walker_bytes(sysm.handle, 1)["scratch"]
    big = (64 << 20) // per + 1
    wl = make_config(name, n_walkers=1)
    w1 = sysm.walkers(wl.occ)
    w1.cstruct.n_walkers = big  # checked before any launch: nothing is read
    with pytest.raises(VmcError):
        vmc_ctmc_step_static(sysm.handle, w1, 1)
    w1.cstruct.n_walkers = 1
