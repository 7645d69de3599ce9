"""ctypes wrapper around the plain C oracle ``vmc_oracle.c``.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every quantity is the
plain definition from the paper; the C source documents which passage each
routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vmc_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ORC_DET = 0
ORC_LEMMA = 1


class _Cand(C.Structure):
    _fields_ = [("type", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("a", C.c_int32), ("b", C.c_int32),
                ("h", C.c_double), ("ratio", C.c_double)]


def build_oracle_library(force: bool = True) -> str:
    """Compile vmc_oracle.c with gcc (plain -O2, OpenMP over walkers only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", _SRC,
               "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle_library(force=True)
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, P, C.c_int64, P, P, C.c_double]
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_params.argtypes = [P, P, P]
    lib.orc_num_double_entries.restype = C.c_int64
    lib.orc_num_double_entries.argtypes = [P]
    lib.orc_singles_bound.argtypes = [P, P]
    lib.orc_pair_doubles.restype = C.c_int64
    lib.orc_pair_doubles.argtypes = [P, C.c_int, C.c_int, P, P, C.c_int64]
    lib.orc_hdiag.restype = C.c_double
    lib.orc_hdiag.argtypes = [P, P]
    lib.orc_log_psi.restype = C.c_double
    lib.orc_log_psi.argtypes = [P, P, P]
    lib.orc_local_energy.restype = C.c_int
    lib.orc_local_energy.argtypes = [P, P, C.c_int, P, P, P, P, C.c_int64, P]
    lib.orc_local_energy_batch.argtypes = [P, C.c_int64, P, C.c_int, P, P, P, P, C.c_int]
    lib.orc_max_threads.restype = C.c_int
    lib.orc_philox4x64_10.argtypes = [P, P, P]
    lib.orc_uniform.restype = C.c_double
    lib.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
    lib.orc_ctmc_step.restype = C.c_int
    lib.orc_ctmc_step.argtypes = [P, P, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, P, P, P, P]
    lib.orc_logderiv.restype = C.c_int
    lib.orc_logderiv.argtypes = [P, P, P]
    lib.orc_ctmc_batch.argtypes = [P, C.c_int64, P, C.c_int, C.c_uint64, C.c_uint64, C.c_int, P, P, P, C.c_int]
    lib.orc_eval_states.argtypes = [P, C.c_int64, P, C.c_int, C.c_uint64, P, P, P, P, P, P, P, C.c_int]
    lib.orc_set_cps.restype = C.c_int64
    lib.orc_set_cps.argtypes = [P, C.c_int, P, P]
    lib.orc_num_cps_params.restype = C.c_int64
    lib.orc_num_cps_params.argtypes = [P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox4x64_10(counter, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, walker: int, step: int) -> float:
    return float(_load().orc_uniform(seed, walker, step))


class OracleSystem:
    """One Hamiltonian + screening threshold + wavefunction parameters."""

    def __init__(self, n_orb: int, n_alpha: int, n_beta: int, h1: np.ndarray, eri_idx: np.ndarray,
                 eri_val: np.ndarray, eps: float):
        lib = _load()
        self.n = int(n_orb)
        self.n_so = 2 * self.n
        self.na = int(n_alpha)
        self.nb = int(n_beta)
        self.ne = self.na + self.nb
        self.nw = (self.n_so + 63) // 64
        if self.nw > 16:
            raise ValueError("oracle supports at most 1024 spin-orbitals")
        self.eps = float(eps)
        h = np.ascontiguousarray(h1, dtype=np.float64)
        ei = np.ascontiguousarray(eri_idx, dtype=np.int32).reshape(-1, 4)
        ev = np.ascontiguousarray(eri_val, dtype=np.float64)
        self._h = lib.orc_create(self.n, self.na, self.nb, _ptr(h), ei.shape[0], _ptr(ei), _ptr(ev), self.eps)
        self._lib = lib

    @classmethod
    def from_workload(cls, wl, eps: Optional[float] = None) -> "OracleSystem":
        s = cls(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, wl.eri_idx, wl.eri_val, wl.eps if eps is None else eps)
        s.set_params(wl.jastrow, wl.theta)
        if getattr(wl, "cps_sites", None) is not None and len(wl.cps_sites):
            s.set_cps(wl.cps_sites, wl.cps_coeffs)
        return s

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    # ------------------------------------------------------------------
    def set_params(self, jastrow_packed: np.ndarray, theta: np.ndarray) -> None:
        self._J = np.ascontiguousarray(jastrow_packed, dtype=np.float64)
        self._theta = np.ascontiguousarray(theta, dtype=np.float64)
        assert self._J.size == self.n_so * (self.n_so + 1) // 2
        assert self._theta.shape == (self.n_so, self.n_so)
        self._lib.orc_set_params(self._h, _ptr(self._J), _ptr(self._theta))

    def set_cps(self, sites, coeffs) -> int:
        """Correlators: sites (n_corr, 5) int, spatial orbitals padded with -1;
        coeffs: the 4^k coefficients of each correlator, concatenated.  An
        empty site list removes the correlator factor."""
        sites = np.ascontiguousarray(sites, dtype=np.int32).reshape(-1, 5)
        self._cps_sites = sites
        self._cps_coeffs = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(-1)
        n = int(self._lib.orc_set_cps(self._h, sites.shape[0], _ptr(sites), _ptr(self._cps_coeffs)))
        if n < 0:
            raise ValueError("malformed correlator site list")
        if n != self._cps_coeffs.size:
            raise ValueError(f"expected {n} correlator coefficients, got {self._cps_coeffs.size}")
        return n

    def num_cps_params(self) -> int:
        return int(self._lib.orc_num_cps_params(self._h))

    @property
    def n_params(self) -> int:
        return self.n_so * (self.n_so + 1) // 2 + self.n_so * self.n_so + self.num_cps_params()

    def num_double_entries(self) -> int:
        return int(self._lib.orc_num_double_entries(self._h))

    def singles_bound(self) -> np.ndarray:
        out = np.zeros((self.n_so, self.n_so))
        self._lib.orc_singles_bound(self._h, _ptr(out))
        return out

    def pair_doubles(self, i: int, j: int):
        """Doubles of the pair (i<j) with |v| > eps, sorted by (-|v|, a, b)."""
        m = int(self._lib.orc_pair_doubles(self._h, i, j, None, None, 0))
        ab = np.zeros((max(m, 1), 2), dtype=np.int32)
        v = np.zeros(max(m, 1))
        self._lib.orc_pair_doubles(self._h, i, j, _ptr(ab), _ptr(v), m)
        return ab[:m], v[:m]

    def _bits(self, occ) -> np.ndarray:
        b = np.ascontiguousarray(occ, dtype=np.uint64).reshape(-1)
        assert b.size == self.nw
        return b

    def hdiag(self, occ) -> float:
        return float(self._lib.orc_hdiag(self._h, _ptr(self._bits(occ))))

    def log_psi(self, occ):
        sg = C.c_int(0)
        v = self._lib.orc_log_psi(self._h, _ptr(self._bits(occ)), C.byref(sg))
        return float(v), int(sg.value)

    def local_energy(self, occ, mode: int = ORC_DET, with_candidates: bool = True):
        """Returns dict(eloc, T, n_cand, hnn, cand) for one walker."""
        bits = self._bits(occ)
        el = C.c_double(0.0)
        T = C.c_double(0.0)
        nc = C.c_int64(0)
        hnn = C.c_double(0.0)
        rc = self._lib.orc_local_energy(self._h, _ptr(bits), mode, C.byref(el), C.byref(T), C.byref(nc), None, 0,
                                        C.byref(hnn))
        if rc != 0:
            raise RuntimeError(f"oracle local energy failed with code {rc}")
        res = {"eloc": el.value, "T": T.value, "n_cand": int(nc.value), "hnn": hnn.value, "cand": None}
        if with_candidates:
            n = int(nc.value)
            arr = (_Cand * max(n, 1))()
            self._lib.orc_local_energy(self._h, _ptr(bits), mode, C.byref(el), C.byref(T), C.byref(nc),
                                       C.cast(arr, C.c_void_p), n, None)
            cands = np.zeros(n, dtype=[("type", "i4"), ("i", "i4"), ("j", "i4"), ("a", "i4"), ("b", "i4"),
                                       ("h", "f8"), ("ratio", "f8")])
            for k in range(n):
                c = arr[k]
                cands[k] = (c.type, c.i, c.j, c.a, c.b, c.h, c.ratio)
            res["cand"] = cands
        return res

    def local_energy_batch(self, occ: np.ndarray, mode: int = ORC_DET, threads: int = 0):
        occ = np.ascontiguousarray(occ, dtype=np.uint64).reshape(-1, self.nw)
        W = occ.shape[0]
        el = np.zeros(W)
        T = np.zeros(W)
        nc = np.zeros(W, dtype=np.int64)
        st = np.zeros(W, dtype=np.int32)
        self._lib.orc_local_energy_batch(self._h, W, _ptr(occ), mode, _ptr(el), _ptr(T), _ptr(nc), _ptr(st),
                                         int(threads))
        return el, T, nc, st

    def ctmc_step(self, occ, seed: int, walker: int, step: int, mode: int = ORC_DET):
        """One CTMC move.  Returns (new_occ, eloc, t, pick(type,i,j,a,b), margin, rc)."""
        bits = self._bits(occ).copy()
        el = C.c_double(0.0)
        t = C.c_double(0.0)
        pick = np.zeros(5, dtype=np.int32)
        margin = C.c_double(0.0)
        rc = self._lib.orc_ctmc_step(self._h, _ptr(bits), mode, seed, walker, step, C.byref(el), C.byref(t),
                                     _ptr(pick), C.byref(margin))
        return bits, el.value, t.value, tuple(int(x) for x in pick), margin.value, int(rc)

    def ctmc_batch(self, occ: np.ndarray, seed: int, step0: int, n_steps: int, mode: int = ORC_LEMMA,
                   threads: int = 0):
        """n_steps moves of every walker (walker index = row), OpenMP over walkers."""
        occ = np.ascontiguousarray(occ, dtype=np.uint64).reshape(-1, self.nw).copy()
        W = occ.shape[0]
        el = np.zeros((W, n_steps))
        t = np.zeros((W, n_steps))
        st = np.zeros(W, dtype=np.int32)
        self._lib.orc_ctmc_batch(self._h, W, _ptr(occ), mode, seed, step0, n_steps, _ptr(el), _ptr(t), _ptr(st),
                                 int(threads))
        return occ, el, t, st

    def eval_states(self, occ: np.ndarray, seed: int, walker, step, mode: int = ORC_LEMMA, threads: int = 0):
        """Teacher-forced evaluation of independent states (OpenMP over states):
        state k is occ[k] of walker walker[k] at step step[k].  Returns
        (eloc, t, picks (n, 5), margin, rc) as orc_ctmc_step would, no move applied."""
        occ = np.ascontiguousarray(occ, dtype=np.uint64).reshape(-1, self.nw)
        n = occ.shape[0]
        wk = np.ascontiguousarray(np.broadcast_to(np.asarray(walker, dtype=np.int64), (n,)))
        sk = np.ascontiguousarray(np.broadcast_to(np.asarray(step, dtype=np.int64), (n,)))
        el = np.zeros(n)
        t = np.zeros(n)
        pick = np.zeros((n, 5), dtype=np.int32)
        margin = np.zeros(n)
        rc = np.zeros(n, dtype=np.int32)
        self._lib.orc_eval_states(self._h, n, _ptr(occ), mode, seed, _ptr(wk), _ptr(sk), _ptr(el), _ptr(t),
                                  _ptr(pick), _ptr(margin), _ptr(rc), int(threads))
        return el, t, pick, margin, rc

    def logderiv(self, occ) -> np.ndarray:
        n_p = self.n_params
        out = np.zeros(n_p)
        rc = self._lib.orc_logderiv(self._h, _ptr(self._bits(occ)), _ptr(out))
        if rc != 0:
            raise RuntimeError(f"oracle logderiv failed with code {rc}")
        return out

    @staticmethod
    def max_threads() -> int:
        return int(_load().orc_max_threads())


def occ_to_list(occ_row: np.ndarray, n_so: int) -> List[int]:
    out = []
    for p in range(n_so):
        if (int(occ_row[p >> 6]) >> (p & 63)) & 1:
            out.append(p)
    return out


def list_to_occ(orbs, n_so: int) -> np.ndarray:
    nw = (n_so + 63) // 64
    b = np.zeros(nw, dtype=np.uint64)
    for p in orbs:
        b[p >> 6] |= np.uint64(1) << np.uint64(p & 63)
    return b
