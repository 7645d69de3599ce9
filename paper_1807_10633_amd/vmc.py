"""ctypes binding of libvmc.so: the C ABI declared in include/vmc.h.

Argument marshalling only: every step of the hot path runs in the library's
gfx950 kernels.  PyTorch provides device memory and streams.  There is no CPU
fallback: if libvmc.so is missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvmc.so")

VMC_OK = 0
VMC_FP64 = 0
VMC_MIXED = 1
VMC_GHF = 0
VMC_UHF = 1
ST_SINGULAR, ST_EMPTY, ST_NONFINITE, ST_SMALLDEN = 1, 2, 4, 8

FIELDS = ("occ_bits", "slot_orb", "orb_slot", "ainv", "r", "rlo", "jsum", "hnn", "eloc", "tres", "pick", "status", "scratch")
NFIELDS = len(FIELDS)

EXPORTED = (
    "vmc_init", "vmc_set_params", "vmc_walker_bytes", "vmc_walkers_init", "vmc_local_energy", "vmc_ctmc_step",
    "vmc_logderiv", "vmc_amsgrad", "vmc_excitations", "vmc_uniforms", "vmc_decode_pick", "vmc_table_info",
    "vmc_destroy", "vmc_last_error", "vmc_host_tables_build", "vmc_host_tables_sizes", "vmc_host_tables_get",
    "vmc_host_tables_free", "vmc_set_launch", "vmc_launch_info", "vmc_estimate", "vmc_batch_create",
    "vmc_batch_set_launch", "vmc_batch_local_energy", "vmc_batch_ctmc_step", "vmc_batch_destroy", "vmc_autotune",
    "vmc_batch_autotune", "vmc_ctmc_step_dev", "vmc_walkers_refresh", "vmc_cps_init", "vmc_set_cps", "vmc_cps_info",
    "vmc_ctmc_step_static",
    "vmc_set_small_denominator", "vmc_set_occupancy", "vmc_batch_set_occupancy", "vmc_snapshot_weights",
    "vmc_logderiv_accumulate", "vmc_gradient_combine", "vmc_batch_set_mode", "vmc_batch_info",
)


class VmcError(RuntimeError):
    pass


class SystemDesc(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32), ("precision", C.c_int32),
                ("refresh_period", C.c_int32), ("orbitals", C.c_int32), ("seed", C.c_uint64)]


class EriList(C.Structure):
    _fields_ = [("n_nz", C.c_int64), ("pqrs", C.c_void_p), ("val", C.c_void_p)]


class WalkersStruct(C.Structure):
    _fields_ = ([("n_walkers", C.c_int64)] + [(f, C.c_void_p) for f in FIELDS] +
                [("step", C.c_uint64), ("since_inv", C.c_uint64)])


_lib = None


def load_library() -> C.CDLL:
    """Load libvmc.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise VmcError(f"{LIB_PATH} is missing: build it with `python -m paper_1807_10633_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "vmc_init": ([P, P, P, d, P, P], i32),
        "vmc_set_params": ([P, P, P, P], i32),
        "vmc_cps_init": ([P, i32, P], i32),
        "vmc_set_cps": ([P, P, P], i32),
        "vmc_cps_info": ([P, P], i32),
        "vmc_walker_bytes": ([P, i64, P], i32),
        "vmc_walkers_init": ([P, P, P], i32),
        "vmc_walkers_refresh": ([P, P, P], i32),
        "vmc_local_energy": ([P, P, P], i32),
        "vmc_ctmc_step": ([P, P, i32, P, P, P, P], i32),
        "vmc_ctmc_step_static": ([P, P, i32, P, P, P, P], i32),
        "vmc_set_small_denominator": ([P, C.c_double], i32),
        "vmc_logderiv": ([P, P, P, P, P], i32),
        "vmc_amsgrad": ([i64, P, P, P, P, P, d, d, d, d, i32, P], i32),
        "vmc_excitations": ([P, P, i64, P, P, P, i64, P, P], i32),
        "vmc_uniforms": ([u64, i64, u64, P, P], i32),
        "vmc_decode_pick": ([i64, P], None),
        "vmc_table_info": ([P, P], i32),
        "vmc_launch_info": ([P, P], i32),
        "vmc_estimate": ([P, P, P, P, P], i32),
        "vmc_batch_create": ([P, i32, P], i32),
        "vmc_batch_set_launch": ([P, i32], i32),
        "vmc_set_occupancy": ([P, i32], i32),
        "vmc_snapshot_weights": ([P, P, P, P, P, i32, P], i32),
        "vmc_logderiv_accumulate": ([P, P, P, P, P], i32),
        "vmc_gradient_combine": ([C.c_int64, P, P, P, P, P], i32),
        "vmc_batch_set_occupancy": ([P, i32], i32),
        "vmc_batch_set_mode": ([P, i32], i32),
        "vmc_batch_info": ([P, P], i32),
        "vmc_batch_local_energy": ([P, P, P], i32),
        "vmc_batch_ctmc_step": ([P, P, i32, P], i32),
        "vmc_batch_destroy": ([P], i32),
        "vmc_autotune": ([P, P, i32, P, P], i32),
        "vmc_ctmc_step_dev": ([P, P, i32, P, P], i32),
        "vmc_batch_autotune": ([P, P, i32, P, P], i32),
        "vmc_set_launch": ([P, i32], i32),
        "vmc_destroy": ([P], i32),
        "vmc_last_error": ([P], C.c_char_p),
        "vmc_host_tables_build": ([P, P, P, d, P], i32),
        "vmc_host_tables_sizes": ([P, P], i32),
        "vmc_host_tables_get": ([P, P, P, P, P, P, P, P], i32),
        "vmc_host_tables_free": ([P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int, handle=None, what: str = "") -> None:
    if rc != VMC_OK:
        msg = load_library().vmc_last_error(handle)
        raise VmcError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


# ----------------------------------------------------------------------------
# Thin wrappers, same names as the C ABI
# ----------------------------------------------------------------------------
def vmc_init(n_orb: int, n_alpha: int, n_beta: int, h1: np.ndarray, eri_idx: np.ndarray, eri_val: np.ndarray,
             eps: float, *, precision: int = VMC_FP64, refresh_period: int = 50, seed: int = 0,
             orbitals: int = VMC_GHF, stream=None):
    lib = load_library()
    desc = SystemDesc(n_orb, n_alpha, n_beta, precision, refresh_period, orbitals, seed)
    h = np.ascontiguousarray(h1, dtype=np.float64)
    ei = np.ascontiguousarray(eri_idx, dtype=np.int32).reshape(-1, 4)
    ev = np.ascontiguousarray(eri_val, dtype=np.float64)
    lst = EriList(ei.shape[0], ei.ctypes.data, ev.ctypes.data)
    out = C.c_void_p()
    rc = lib.vmc_init(C.byref(desc), _np_ptr(h), C.byref(lst), float(eps), _stream_ptr(stream), C.byref(out))
    _check(rc, None, "vmc_init")
    return out


def vmc_set_params(handle, J_dev, theta_dev, stream=None) -> None:
    _check(load_library().vmc_set_params(handle, _dev_ptr(J_dev), _dev_ptr(theta_dev), _stream_ptr(stream)), handle,
           "vmc_set_params")


def vmc_cps_init(handle, sites: np.ndarray) -> None:
    """Correlators: sites (n_corr, 5) int32 spatial orbitals, -1 padded."""
    st = np.ascontiguousarray(sites, dtype=np.int32).reshape(-1, 5)
    _check(load_library().vmc_cps_init(handle, st.shape[0], _np_ptr(st)), handle, "vmc_cps_init")


def vmc_set_cps(handle, coeffs_dev, stream=None) -> None:
    _check(load_library().vmc_set_cps(handle, _dev_ptr(coeffs_dev), _stream_ptr(stream)), handle, "vmc_set_cps")


def vmc_cps_info(handle):
    out = (C.c_int64 * 2)()
    _check(load_library().vmc_cps_info(handle, out), handle, "vmc_cps_info")
    return {"correlators": int(out[0]), "coefficients": int(out[1])}


def vmc_walker_bytes(handle, n_walkers: int) -> Dict[str, int]:
    arr = (C.c_size_t * NFIELDS)()
    _check(load_library().vmc_walker_bytes(handle, int(n_walkers), arr), handle, "vmc_walker_bytes")
    return {f: int(arr[k]) for k, f in enumerate(FIELDS)}


def vmc_walkers_init(handle, walkers: "Walkers", stream=None) -> None:
    _check(load_library().vmc_walkers_init(handle, C.byref(walkers.cstruct), _stream_ptr(stream)), handle,
           "vmc_walkers_init")


def vmc_walkers_refresh(handle, walkers: "Walkers", stream=None) -> None:
    _check(load_library().vmc_walkers_refresh(handle, C.byref(walkers.cstruct), _stream_ptr(stream)), handle,
           "vmc_walkers_refresh")


def vmc_local_energy(handle, walkers: "Walkers", stream=None) -> None:
    _check(load_library().vmc_local_energy(handle, C.byref(walkers.cstruct), _stream_ptr(stream)), handle,
           "vmc_local_energy")


def vmc_ctmc_step(handle, walkers: "Walkers", n_steps: int, eloc_hist=None, t_hist=None, pick_hist=None,
                  stream=None) -> None:
    _check(load_library().vmc_ctmc_step(handle, C.byref(walkers.cstruct), int(n_steps), _dev_ptr(eloc_hist),
                                        _dev_ptr(t_hist), _dev_ptr(pick_hist), _stream_ptr(stream)), handle,
           "vmc_ctmc_step")


def vmc_ctmc_step_static(handle, walkers: "Walkers", n_steps: int, eloc_hist=None, t_hist=None, pick_hist=None,
                         stream=None) -> None:
    """vmc_ctmc_step with the kernels' workspace in the library's static array (no allocation)."""
    _check(load_library().vmc_ctmc_step_static(handle, C.byref(walkers.cstruct), int(n_steps), _dev_ptr(eloc_hist),
                                               _dev_ptr(t_hist), _dev_ptr(pick_hist), _stream_ptr(stream)), handle,
           "vmc_ctmc_step_static")


def vmc_set_small_denominator(handle, threshold: float) -> None:
    """Threshold of the small Sherman-Morrison denominator flag (and in-place re-inversion)."""
    _check(load_library().vmc_set_small_denominator(handle, float(threshold)), handle, "vmc_set_small_denominator")


def vmc_ctmc_step_dev(handle, walkers: "Walkers", n_steps: int, step_dev, stream=None) -> None:
    """CTMC moves with the step counter in device memory (graph-capturable)."""
    _check(load_library().vmc_ctmc_step_dev(handle, C.byref(walkers.cstruct), int(n_steps), _dev_ptr(step_dev),
                                            _stream_ptr(stream)), handle, "vmc_ctmc_step_dev")


def vmc_logderiv(handle, walkers: "Walkers", g_dev, out_dev, stream=None) -> None:
    _check(load_library().vmc_logderiv(handle, C.byref(walkers.cstruct), _dev_ptr(g_dev), _dev_ptr(out_dev),
                                       _stream_ptr(stream)), handle, "vmc_logderiv")


def vmc_estimate(handle, walkers: "Walkers", out_dev, g_dev=None, stream=None) -> None:
    """out_dev (4 FP64, device) <- {sum t, sum t E_L, E, count}; g_dev (W FP64) <- gradient weights."""
    _check(load_library().vmc_estimate(handle, C.byref(walkers.cstruct), _dev_ptr(out_dev),
                                       _dev_ptr(g_dev) if g_dev is not None else None, _stream_ptr(stream)),
           handle, "vmc_estimate")


def vmc_snapshot_weights(handle, walkers: "Walkers", acc, g_te, g_t, reset: bool, stream=None) -> None:
    """Gradient weights t E_L and t of the walkers' current states, and running sums acc (4 doubles)."""
    _check(load_library().vmc_snapshot_weights(handle, C.byref(walkers.cstruct), _dev_ptr(acc), _dev_ptr(g_te),
                                               _dev_ptr(g_t), 1 if reset else 0, _stream_ptr(stream)), handle,
           "vmc_snapshot_weights")


def vmc_logderiv_accumulate(handle, walkers: "Walkers", g, out, stream=None) -> None:
    """out += sum_w g_w O_w (the contracted backward, accumulated)."""
    _check(load_library().vmc_logderiv_accumulate(handle, C.byref(walkers.cstruct), _dev_ptr(g), _dev_ptr(out),
                                                  _stream_ptr(stream)), handle, "vmc_logderiv_accumulate")


def vmc_gradient_combine(a, b, acc, out, stream=None) -> None:
    """out = 2 (a - E b) / sum t with E, sum t from acc."""
    _check(load_library().vmc_gradient_combine(int(out.numel()), _dev_ptr(a), _dev_ptr(b), _dev_ptr(acc),
                                               _dev_ptr(out), _stream_ptr(stream)), None, "vmc_gradient_combine")


def vmc_estimate_arrays(handle, eloc_dev, tres_dev, n: int, out_dev, g_dev=None, stream=None) -> None:
    """vmc_estimate over n (E_L, t) pairs held in any device arrays (e.g. the
    histories of a sweep): the walker record passed carries only those two."""
    ws = WalkersStruct(int(n), *([None] * NFIELDS), 0, 0)
    ws.eloc = _dev_ptr(eloc_dev)
    ws.tres = _dev_ptr(tres_dev)
    _check(load_library().vmc_estimate(handle, C.byref(ws), _dev_ptr(out_dev),
                                       _dev_ptr(g_dev) if g_dev is not None else None, _stream_ptr(stream)),
           handle, "vmc_estimate")


def vmc_amsgrad(params, m, v, vhat, grad, lr: float, beta1: float, beta2: float, delta: float = 1e-8,
                paper_literal: bool = False, stream=None) -> None:
    n = params.numel()
    _check(load_library().vmc_amsgrad(n, _dev_ptr(params), _dev_ptr(m), _dev_ptr(v), _dev_ptr(vhat), _dev_ptr(grad),
                                      lr, beta1, beta2, delta, int(paper_literal), _stream_ptr(stream)), None,
           "vmc_amsgrad")


def vmc_excitations(handle, walkers: "Walkers", walker: int, ijab, hval, ratio, cap: int, count, stream=None) -> None:
    _check(load_library().vmc_excitations(handle, C.byref(walkers.cstruct), int(walker), _dev_ptr(ijab),
                                          _dev_ptr(hval), _dev_ptr(ratio), int(cap), _dev_ptr(count),
                                          _stream_ptr(stream)), handle, "vmc_excitations")


def vmc_uniforms(seed: int, n: int, step: int, out_dev, stream=None) -> None:
    _check(load_library().vmc_uniforms(seed, int(n), step, _dev_ptr(out_dev), _stream_ptr(stream)), None,
           "vmc_uniforms")


def vmc_decode_pick(code: int):
    out = (C.c_int32 * 5)()
    load_library().vmc_decode_pick(int(code), out)
    return tuple(int(x) for x in out)


def vmc_table_info(handle):
    out = (C.c_int64 * 3)()
    _check(load_library().vmc_table_info(handle, out), handle, "vmc_table_info")
    return {"double_entries": int(out[0]), "single_entries": int(out[1]), "groups": int(out[2])}


def vmc_launch_info(handle):
    out = (C.c_int64 * 5)()
    _check(load_library().vmc_launch_info(handle, out), handle, "vmc_launch_info")
    return {"threads": int(out[0]), "state_in_lds": bool(out[1]), "lds_bytes": int(out[2]),
            "refresh_kernel": bool(out[3]), "waves": int(out[4])}


def vmc_set_occupancy(handle, waves: int) -> None:
    """Occupancy target (waves per SIMD: 3, 4, or 0 for the library's choice) of the HBM-layout sweep."""
    _check(load_library().vmc_set_occupancy(handle, int(waves)), handle, "vmc_set_occupancy")


def vmc_set_launch(handle, block_threads: int) -> None:
    _check(load_library().vmc_set_launch(handle, int(block_threads)), handle, "vmc_set_launch")


def vmc_destroy(handle) -> None:
    if handle:
        _check(load_library().vmc_destroy(handle), None, "vmc_destroy")


def vmc_host_tables(n_orb: int, n_alpha: int, n_beta: int, h1: np.ndarray, eri_idx: np.ndarray, eri_val: np.ndarray,
                    eps: float):
    """Host-only table build (no GPU needed); returns a dict of numpy arrays."""
    lib = load_library()
    desc = SystemDesc(n_orb, n_alpha, n_beta, VMC_FP64, 50, 0, 0)
    h = np.ascontiguousarray(h1, dtype=np.float64)
    ei = np.ascontiguousarray(eri_idx, dtype=np.int32).reshape(-1, 4)
    ev = np.ascontiguousarray(eri_val, dtype=np.float64)
    lst = EriList(ei.shape[0], ei.ctypes.data, ev.ctypes.data)
    t = C.c_void_p()
    _check(lib.vmc_host_tables_build(C.byref(desc), _np_ptr(h), C.byref(lst), float(eps), C.byref(t)), None,
           "vmc_host_tables_build")
    try:
        sizes = (C.c_int64 * 2)()
        _check(lib.vmc_host_tables_sizes(t, sizes), None, "vmc_host_tables_sizes")
        E, S = int(sizes[0]), int(sizes[1])
        n_so = 2 * n_orb
        out = {
            "row_off": np.zeros(n_so * n_so + 1, dtype=np.int64),
            "dab": np.zeros((max(E, 1), 2), dtype=np.int32),
            "dv": np.zeros(max(E, 1)),
            "s_off": np.zeros(n_so + 1, dtype=np.int64),
            "sa": np.zeros(max(S, 1), dtype=np.int32),
            "sS": np.zeros(max(S, 1)),
            "sh": np.zeros(max(S, 1)),
        }
        _check(lib.vmc_host_tables_get(t, *(_np_ptr(out[k]) for k in ("row_off", "dab", "dv", "s_off", "sa", "sS",
                                                                         "sh"))), None, "vmc_host_tables_get")
        out["dab"], out["dv"] = out["dab"][:E], out["dv"][:E]
        out["sa"], out["sS"], out["sh"] = out["sa"][:S], out["sS"][:S], out["sh"][:S]
        return out
    finally:
        lib.vmc_host_tables_free(t)


def vmc_batch_create(handles) -> int:
    arr = (C.c_void_p * len(handles))(*handles)
    out = C.c_void_p()
    _check(load_library().vmc_batch_create(arr, len(handles), C.byref(out)), None, "vmc_batch_create")
    return out.value


def vmc_batch_set_launch(batch, block_threads: int) -> None:
    _check(load_library().vmc_batch_set_launch(batch, int(block_threads)), None, "vmc_batch_set_launch")


def vmc_batch_set_occupancy(batch, waves: int) -> None:
    _check(load_library().vmc_batch_set_occupancy(batch, int(waves)), None, "vmc_batch_set_occupancy")


VMC_BATCH_FUSED, VMC_BATCH_STREAMS = 0, 1


def vmc_batch_set_mode(batch, mode: int) -> None:
    _check(load_library().vmc_batch_set_mode(batch, int(mode)), None, "vmc_batch_set_mode")


def vmc_batch_info(batch) -> dict:
    out = (C.c_int64 * 3)()
    _check(load_library().vmc_batch_info(batch, out), None, "vmc_batch_info")
    return {"mode": int(out[0]), "threads": int(out[1]), "waves": int(out[2])}


def _walker_array(walkers):
    return (C.c_void_p * len(walkers))(*[C.cast(C.pointer(w.cstruct), C.c_void_p) for w in walkers])


def vmc_batch_local_energy(batch, walkers, stream=None) -> None:
    _check(load_library().vmc_batch_local_energy(batch, _walker_array(walkers), _stream_ptr(stream)), None,
           "vmc_batch_local_energy")


def vmc_batch_ctmc_step(batch, walkers, n_steps: int, stream=None) -> None:
    _check(load_library().vmc_batch_ctmc_step(batch, _walker_array(walkers), int(n_steps), _stream_ptr(stream)), None,
           "vmc_batch_ctmc_step")


def vmc_autotune(handle, walkers: "Walkers", n_moves: int = 5, stream=None) -> int:
    out = C.c_int32(0)
    _check(load_library().vmc_autotune(handle, C.byref(walkers.cstruct), int(n_moves), C.byref(out),
                                       _stream_ptr(stream)), handle, "vmc_autotune")
    return int(out.value)


def vmc_batch_autotune(batch, walkers, n_moves: int = 5, stream=None) -> int:
    out = C.c_int32(0)
    _check(load_library().vmc_batch_autotune(batch, _walker_array(walkers), int(n_moves), C.byref(out),
                                             _stream_ptr(stream)), None, "vmc_batch_autotune")
    return int(out.value)


def vmc_batch_destroy(batch) -> None:
    _check(load_library().vmc_batch_destroy(batch), None, "vmc_batch_destroy")


# ----------------------------------------------------------------------------
# Device-memory owners (torch tensors), no compute
# ----------------------------------------------------------------------------
class Walkers:
    """Caller-owned walker buffers allocated as torch uint8 tensors on a device."""

    def __init__(self, handle, n_walkers: int, device="cuda"):
        import torch

        self.n_walkers = int(n_walkers)
        sizes = vmc_walker_bytes(handle, self.n_walkers)
        self.buffers = {f: torch.empty(max(sizes[f], 16), dtype=torch.uint8, device=device) for f in FIELDS}
        self.cstruct = WalkersStruct(self.n_walkers, *[self.buffers[f].data_ptr() for f in FIELDS], 0, 0)

    @property
    def step(self) -> int:
        return int(self.cstruct.step)

    @step.setter
    def step(self, v: int) -> None:
        self.cstruct.step = int(v)

    @property
    def since_inv(self) -> int:
        return int(self.cstruct.since_inv)

    def view(self, field: str, dtype):
        return self.buffers[field].view(dtype)


class System:
    """One Hamiltonian on the device: tables (library-owned) and parameters."""

    def __init__(self, n_orb, n_alpha, n_beta, h1, eri_idx, eri_val, eps, *, refresh_period=50, seed=0,
                 precision=VMC_FP64, orbitals=VMC_GHF, device="cuda"):
        self.n_orb, self.n_alpha, self.n_beta = int(n_orb), int(n_alpha), int(n_beta)
        self.n_so = 2 * self.n_orb
        self.ne = self.n_alpha + self.n_beta
        self.n_words = (self.n_so + 63) // 64
        self.n_base_params = self.n_so * (self.n_so + 1) // 2 + self.n_so * self.n_so
        self.n_cps = 0
        self.cps = None
        self._pvec = None
        self.device = device
        self.precision = int(precision)
        self.orbitals = int(orbitals)
        # length of one slot's row of R: every orbital, or the slot's own spin
        self.r_row = self.n_orb if self.orbitals == VMC_UHF else self.n_so
        self.handle = vmc_init(n_orb, n_alpha, n_beta, h1, eri_idx, eri_val, eps, precision=precision,
                               refresh_period=refresh_period, seed=seed, orbitals=orbitals)

    @classmethod
    def from_workload(cls, wl, **kw):
        import torch

        if getattr(wl, "orbitals", "ghf") == "uhf":
            kw.setdefault("orbitals", VMC_UHF)
        s = cls(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, wl.eri_idx, wl.eri_val, wl.eps, seed=wl.ctmc_seed, **kw)
        s.set_params(torch.as_tensor(wl.jastrow, device=s.device), torch.as_tensor(wl.theta, device=s.device))
        if getattr(wl, "cps_sites", None) is not None and len(wl.cps_sites):
            s.set_cps(wl.cps_sites, torch.as_tensor(wl.cps_coeffs, device=s.device))
        return s

    @property
    def n_params(self) -> int:
        return self.n_base_params + self.n_cps

    def set_params(self, J_packed, theta) -> None:
        self.J = J_packed.contiguous().to(dtype=__import__("torch").float64)
        self.theta = theta.contiguous().to(dtype=__import__("torch").float64)
        vmc_set_params(self.handle, self.J, self.theta)

    def set_cps(self, sites, coeffs) -> None:
        """Correlators (vmc_cps_init on first use) and their coefficients."""
        if self.n_cps == 0:
            vmc_cps_init(self.handle, sites)
            self.n_cps = vmc_cps_info(self.handle)["coefficients"]
            self.cps_sites = np.ascontiguousarray(sites, dtype=np.int32).reshape(-1, 5)
        self.cps = coeffs.contiguous().to(dtype=__import__("torch").float64)
        assert self.cps.numel() == self.n_cps
        vmc_set_cps(self.handle, self.cps)

    def param_vector(self):
        """All parameters in the order of vmc_logderiv: J, theta, correlators."""
        import torch

        parts = [self.J, self.theta.reshape(-1)] + ([self.cps] if self.n_cps else [])
        return torch.cat(parts)

    def set_param_vector(self, p, stream=None) -> None:
        """Hand a vector in param_vector's order to the library (views, no copy
        here: the library copies on `stream`); keeps a reference for host_params."""
        nj = self.n_so * (self.n_so + 1) // 2
        nt = self.n_so * self.n_so
        vmc_set_params(self.handle, p[:nj], p[nj:nj + nt], stream=stream)
        if self.n_cps:
            vmc_set_cps(self.handle, p[nj + nt:], stream=stream)
        self._pvec = p

    def host_params(self):
        """(J packed, theta) of the parameters last handed over, as numpy."""
        nj = self.n_so * (self.n_so + 1) // 2
        if self._pvec is None:
            return self.J.cpu().numpy(), self.theta.cpu().numpy()
        p = self._pvec.cpu().numpy()
        return p[:nj], p[nj:nj + self.n_so * self.n_so].reshape(self.n_so, self.n_so)

    def host_cps(self):
        nj = self.n_so * (self.n_so + 1) // 2
        if self._pvec is None:
            return self.cps.cpu().numpy()
        return self._pvec.cpu().numpy()[nj + self.n_so * self.n_so:]

    def walkers(self, occ: np.ndarray) -> Walkers:
        import torch

        occ = np.ascontiguousarray(occ, dtype=np.uint64).reshape(-1, self.n_words)
        w = Walkers(self.handle, occ.shape[0], device=self.device)
        w.view("occ_bits", torch.int64)[: occ.size].copy_(torch.from_numpy(occ.view(np.int64).reshape(-1)))
        vmc_walkers_init(self.handle, w)
        return w

    @property
    def r_dtype(self):
        """Element type of the walkers' R buffer: float32 in the mixed form."""
        import torch

        return torch.float32 if self.precision == VMC_MIXED else torch.float64

    def table_info(self):
        return vmc_table_info(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            vmc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
