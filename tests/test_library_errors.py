"""Host-side argument validation of the C ABI (no GPU needed: every case is
rejected before any device call)."""
import ctypes as C

import numpy as np
import pytest

from paper_1807_10633_amd import vmc


def _init(n, na, nb, precision=0, refresh=50, orbitals=0, eps=1e-6, h1=None):
    lib = vmc.load_library()
    desc = vmc.SystemDesc(n, na, nb, precision, refresh, orbitals, 0)
    h = np.zeros((max(n, 1), max(n, 1))) if h1 is None else h1
    idx = np.zeros((0, 4), dtype=np.int32)
    val = np.zeros(0)
    eri = vmc.EriList(0, idx.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p))
    out = C.c_void_p()
    rc = lib.vmc_init(C.byref(desc), h.ctypes.data_as(C.c_void_p), C.byref(eri), eps, None, C.byref(out))
    return rc, lib.vmc_last_error(None).decode()


@pytest.mark.parametrize("args,code,msg", [
    ((0, 1, 0), -1, "n_orb"),
    ((513, 1, 1), -1, "n_orb"),
    ((4, 5, 0), -1, "electron counts"),
    ((4, 0, 0), -1, "electron counts"),
    ((2, 2, 2), -1, "empty spin-orbital"),
    ((4, 1, 1, 7), -1, "precision"),
    ((4, 1, 1, 0, 0), -1, "refresh_period"),
    ((4, 1, 1, 0, 50, 3), -1, "orbitals"),
])
def test_init_rejects_bad_descriptions(args, code, msg):
    rc, err = _init(*args)
    assert rc == code and msg in err, (rc, err)


def test_init_rejects_unsupported_spin_blocked_systems():
    # spin-blocked orbitals need at most 128 electrons of each spin
    rc, err = _init(130, 129, 1, orbitals=1)
    assert rc == -6 and "128" in err, (rc, err)


def test_init_rejects_bad_threshold_and_hamiltonian():
    rc, err = _init(4, 1, 1, eps=-1.0)
    assert rc == -1 and "eps" in err
    h = np.zeros((4, 4))
    h[0, 1] = 1.0  # not symmetric
    rc, err = _init(4, 1, 1, h1=h)
    assert rc == -1 and "symmetric" in err


def test_batch_create_rejects_empty_and_oversized():
    lib = vmc.load_library()
    out = C.c_void_p()
    assert lib.vmc_batch_create(None, 1, C.byref(out)) == -1
    arr = (C.c_void_p * 9)()
    assert lib.vmc_batch_create(arr, 9, C.byref(out)) == -1
    assert lib.vmc_batch_create(arr, 0, C.byref(out)) == -1


def test_calls_reject_null_handles():
    lib = vmc.load_library()
    assert lib.vmc_local_energy(None, None, None) == -1
    assert lib.vmc_ctmc_step(None, None, 1, None, None, None, None) == -1
    assert lib.vmc_ctmc_step_dev(None, None, 1, None, None) == -1
    assert lib.vmc_logderiv(None, None, None, None, None) == -1
    assert lib.vmc_estimate(None, None, None, None, None) == -1
    assert lib.vmc_autotune(None, None, 1, None, None) == -1
    assert lib.vmc_set_launch(None, 256) == -1
    assert lib.vmc_amsgrad(0, None, None, None, None, None, 1e-3, 0.9, 0.99, 1e-8, 0, None) == -1
