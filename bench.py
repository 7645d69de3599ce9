#!/usr/bin/env python3
"""Throughput of the screened VMC hot path on one MI355X.

Default workload: the synthetic H-chain-like Hamiltonian with 160 spatial
orbitals, 80 alpha + 80 beta electrons, eps = 1e-5, 8192 walkers, with the
Jastrow-Slater wavefunction (51,360 Jastrow + 102,400 orbital parameters,
random-init), synthetic integrals.  The headline is the mixed-precision form
(FP32 R, FP64 inverse, denominators and accumulations); the plain FP64 form
is measured beside it (`other_form`).

One timed step is one optimisation iteration of the hot path:
  * vmc_ctmc_step: a persistent sweep of `--sweep` (= the refresh period, 50)
    CTMC moves of every walker -- screened singles/doubles enumeration,
    ratios, local energy, rates, pick, Sherman-Morrison updates;
  * vmc_local_energy of the post-sweep states, and vmc_estimate: their
    residence-time weighted energy and the contraction weights;
  * vmc_logderiv (contracted backward), vmc_amsgrad, vmc_set_params (Jastrow
    factors folded into the tables) and vmc_walkers_refresh (fresh inverses
    for the new parameters).
value = walker-steps/s = walkers * sweep * steps / wall time of the timed steps.

E_L is checked against the FP64 oracle on the states a sweep leaves before
any re-inversion: the last ten moves of a refresh period and the final
states, on a sample of walkers (teacher forced: the oracle evaluates the
GPU's own trajectory).

Prints one JSON line (see --help for knobs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walker-steps/s (E_L+CTMC) at stated E_L error vs FP64 oracle; % HBM/MFMA peak"
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

# HBM bytes per sweep launch (the timed 50-move sweeps, mean of two) from
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of `bench.py --steps 2 --warmup 1
# --no-cpu-baseline --no-check --no-other-form --no-graph`, scaled by the
# readings of a plain 1 GiB device copy (FETCH_SIZE reads 0.5 KiB per KiB
# moved, WRITE_SIZE 1 KiB per KiB).  Keyed by the SHA-256 of the kernel sources
# and the workload (config, walkers, moves per sweep, threads per walker,
# form): any other kernel source or workload reports null.
KERNEL_SOURCES = ("paper_1807_10633_amd/csrc/vmc.hip", "paper_1807_10633_amd/csrc/device.hpp",
                  "paper_1807_10633_amd/csrc/tables.cpp")
_SRC = ("ecebd9598f8ddc59f3a4a99104d30bebc01774b07f12dee8c1c08c31765475ff",
        "34612a5fdacc07521f2c4a2be434138557890b663234c3daf1567a7241d1ca55",
        "b71e869fe74a959896df20f208b4336cf4a33be250449d90fe9120f44388047d")
COUNTED_TRAFFIC = {
    _SRC + ("hchain160", 8192, 50, 512, "mixed"):
        {"fetch_kib": 1636928178.12, "fetch_factor": 2.0, "write_kib": 235131567.73, "write_factor": 1.0},
    _SRC + ("hubbard10x10", 16384, 50, 256, "mixed"):
        {"fetch_kib": 100650311.31, "fetch_factor": 2.0, "write_kib": 160297958.50, "write_factor": 1.0},
    _SRC + ("hubbard10x10", 16384, 50, 256, "fp64"):
        {"fetch_kib": 113866261.94, "fetch_factor": 2.0, "write_kib": 192131068.98, "write_factor": 1.0},
    _SRC + ("hubbard10x10:uhf", 16384, 50, 128, "mixed"):
        {"fetch_kib": 33707762.03, "fetch_factor": 2.0, "write_kib": 40722610.92, "write_factor": 1.0},
    _SRC + ("hubbard10x10:uhf", 16384, 50, 128, "fp64"):
        {"fetch_kib": 39151712.72, "fetch_factor": 2.0, "write_kib": 48711148.83, "write_factor": 1.0},
}


# Instruction counts per sweep launch (rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES
# SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_WAIT_INST_ANY and
# one more SQ counter, on the same bench command as the HBM counters; hchain20
# with --config hchain20 --precision fp64), keyed like COUNTED_TRAFFIC.  The
# issue peak is one wave64 VALU instruction per SIMD every 4 cycles (16 lanes):
# 256 CUs x 4 SIMDs x 2.4 GHz / 4.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
COUNTED_ISSUE = {
    _SRC + ("hchain160", 8192, 50, 512, "mixed"):
        {"valu_insts": 159128644210.0, "salu_insts": 65886576204.5, "lds_insts": 33176019209.5,
         "vmem_rd_insts": 7602248022.0},
    _SRC + ("hchain20", 4096, 50, 256, "fp64"):
        {"valu_insts": 4833229787.0, "salu_insts": 2676674381.0, "lds_insts": 550167940.0,
         "vmem_rd_insts": 174519680.0},
}


def _source_key():
    import hashlib

    return tuple(hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest() for f in KERNEL_SOURCES)


def counted_issue(config, walkers, sweep, threads, precision, sweep_s):
    rec = COUNTED_ISSUE.get(_source_key() + (config, walkers, sweep, threads, precision))
    if rec is None:
        return None
    rate = rec["valu_insts"] / sweep_s
    return {"valu_insts_per_launch": rec["valu_insts"], "salu_insts_per_launch": rec["salu_insts"],
            "lds_insts_per_launch": rec["lds_insts"], "vmem_rd_insts_per_launch": rec["vmem_rd_insts"],
            "valu_issue_per_s": rate, "valu_issue_peak_per_s": VALU_ISSUE_PEAK,
            "valu_issue_frac": rate / VALU_ISSUE_PEAK}


def counted_traffic(config, walkers, sweep, threads, precision):
    rec = COUNTED_TRAFFIC.get(_source_key() + (config, walkers, sweep, threads, precision))
    if rec is None:
        return None, None
    fetch = rec["fetch_kib"] * 1024 * rec["fetch_factor"]
    write = rec["write_kib"] * 1024 * rec["write_factor"]
    return fetch + write, {"fetch_bytes": fetch, "write_bytes": write}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walkers", type=int, default=0, help="walkers (0 = the workload's own: 8192 for hchain160)")
    ap.add_argument("--sweep", type=int, default=50, help="CTMC moves per step (= refresh period)")
    ap.add_argument("--config", default="hchain160",
                    help="hchain160 (default), hchain20, hubbard8, hubbard10x10, hchain40, hchain80, or batch "
                         "(40/80/160 orbitals swept together)")
    ap.add_argument("--threads", type=int, default=0, help="workgroup size of the sweep kernel (0 = autotuned)")
    ap.add_argument("--waves", type=int, default=0,
                    help="with --threads: occupancy target of the HBM-layout sweep, 3 or 4 waves per SIMD "
                         "(0 = the library's choice)")
    ap.add_argument("--batch-mode", choices=("auto", "fused", "streams"), default="auto",
                    help="batch: one fused launch, one stream per system, or the faster of the two (autotuned)")
    ap.add_argument("--eps", type=float, default=None, help="screening threshold (default: the workload's own)")
    ap.add_argument("--orbitals", choices=("ghf", "uhf"), default="ghf",
                    help="general or spin-blocked (unrestricted) orbitals of the same workload")
    ap.add_argument("--cps", default=None, help="add correlators to the wavefunction (chainK, plus5)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the E_L check against the oracle")
    ap.add_argument("--check-walkers", type=int, default=16, help="walkers sampled for the E_L check")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="mixed",
                    help="form of the headline number (the other form is measured beside it)")
    ap.add_argument("--no-other-form", action="store_true", help="do not measure the other precision form")
    ap.add_argument("--no-graph", action="store_true", help="do not time the hipGraph-replayed iteration")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (reference kernel for the HBM byte "
                         "counters) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    readings give the factor that turns those counters into bytes."""
    import torch

    n = mib * (1 << 20) // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8}), flush=True)


class HipTimer:
    """HIP events on the stream the library launches on (the current torch
    stream is passed to every call), averaged over the recorded intervals."""

    def __init__(self, stream):
        self.stream = stream
        self.ev = []

    def start(self):
        import torch

        e = torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self._e0 = e

    def stop(self):
        import torch

        e = torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self.ev.append((self._e0, e))

    def mean_ms(self):
        import numpy as np

        return float(np.mean([a.elapsed_time(b) for a, b in self.ev])) if self.ev else None


def cpu_oracle_baseline(wl, seconds, oracle_sys=None):
    """The plain oracle (fresh-inverse ratios, OpenMP over walkers) timed on a
    bounded sample of the same workload: walker-steps/s and the thread count."""
    from oracle.core import ORC_LEMMA, OracleSystem

    orc0 = oracle_sys or OracleSystem.from_workload(wl)
    threads = min(16, os.cpu_count() or 1)
    c0 = time.perf_counter()
    orc0.ctmc_batch(wl.occ[:threads], wl.ctmc_seed, 0, 1, ORC_LEMMA, threads)
    per = (time.perf_counter() - c0) / threads  # wall s per walker-step at full thread use
    n_ws = max(threads, int(seconds / max(per, 1e-9)))
    n_w = max(threads, min(wl.n_walkers, (n_ws // 5 // threads) * threads))
    n_steps_cpu = max(2, n_ws // n_w)
    c0 = time.perf_counter()
    orc0.ctmc_batch(wl.occ[:n_w], wl.ctmc_seed, 0, n_steps_cpu, ORC_LEMMA, threads)
    cpu_wall = time.perf_counter() - c0
    return {"value": n_w * n_steps_cpu / cpu_wall, "unit": "walker-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_w} walkers x {n_steps_cpu} CTMC moves of the same workload (oracle, fresh-inverse "
                      f"ratios, OpenMP over walkers), {cpu_wall:.1f} s"}


def batch_bench(args):
    """The uneven batch: H-chain-like systems of 40, 80 and 160 orbitals (half
    filled, eps = 1e-5), 2048 walkers each, swept together by
    vmc_batch_ctmc_step, either in one fused launch (every state in HBM) or
    with one stream per system (each system in its own variant).  value =
    walker-steps/s summed over the three systems.  The roofline is HBM: R and B
    read and written once per move where the state stays in HBM, once per
    sweep where it is held in LDS."""
    import numpy as np
    import torch

    from paper_1807_10633_amd import vmc
    from workloads import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    names = ("hchain40", "hchain80", "hchain160")
    Wb = 2048
    S = args.sweep
    prec = vmc.VMC_MIXED if args.precision == "mixed" else vmc.VMC_FP64
    wls = [make_config(n, n_walkers=Wb) for n in names]
    systems = [vmc.System.from_workload(wl, refresh_period=S, precision=prec) for wl in wls]
    walkers = [s.walkers(wl.occ) for s, wl in zip(systems, wls)]
    b = vmc.vmc_batch_create([s.handle for s in systems])
    stream = torch.cuda.current_stream()
    timer = HipTimer(stream)
    try:
        # burn-in from the random initial determinants, then the launch shapes
        # and the mode are tuned on equilibrated walkers with sweeps as long
        # as the timed ones
        vmc.vmc_batch_ctmc_step(b, walkers, 100, stream=stream)
        if args.batch_mode != "fused" or not args.threads:
            vmc.vmc_batch_autotune(b, walkers, S)
        if args.batch_mode != "auto":
            vmc.vmc_batch_set_mode(b, vmc.VMC_BATCH_STREAMS if args.batch_mode == "streams" else vmc.VMC_BATCH_FUSED)
        if args.threads:
            vmc.vmc_batch_set_launch(b, args.threads)
            vmc.vmc_batch_set_occupancy(b, args.waves)
        info = vmc.vmc_batch_info(b)
        streams = info["mode"] == vmc.VMC_BATCH_STREAMS
        shapes = [vmc.vmc_launch_info(s.handle) for s in systems]
        nt = [sh["threads"] for sh in shapes] if streams else info["threads"]
        for _ in range(args.warmup):
            vmc.vmc_batch_ctmc_step(b, walkers, S, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            timer.start()
            vmc.vmc_batch_ctmc_step(b, walkers, S, stream=stream)
            timer.stop()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = timer.mean_ms()
        vmc.vmc_batch_local_energy(b, walkers, stream=stream)
        torch.cuda.synchronize()
        el_err = None
        if not args.no_check:
            from oracle.core import ORC_LEMMA, OracleSystem

            errs = []
            for s, w, wl in zip(systems, walkers, wls):
                el = w.view("eloc", torch.float64)[:Wb].cpu().numpy()
                occ = w.view("occ_bits", torch.int64)[: Wb * s.n_words].cpu().numpy().view(np.uint64)
                occ = occ.reshape(Wb, s.n_words)
                idx = np.arange(0, Wb, Wb // 4)
                orc = OracleSystem.from_workload(wl)
                e_o, _, _, _ = orc.local_energy_batch(occ[idx], ORC_LEMMA)
                errs.append(float(np.max(np.abs(e_o - el[idx])) / (wl.n_elec if prec == vmc.VMC_MIXED else 1)))
            el_err = max(errs)
    finally:
        vmc.vmc_batch_destroy(b)
    total_w = Wb * len(names)
    # mixed form with the state in HBM: FP32 R plus its bfloat16 remainder
    rb = 6 if prec == vmc.VMC_MIXED else 8
    in_lds = [streams and sh["state_in_lds"] for sh in shapes]
    bytes_per_sweep = sum(2.0 * (s.n_so * s.ne * rb + s.ne * s.ne * 8) * Wb * (1 if lds else S)
                          for s, lds in zip(systems, in_lds))
    gbs = bytes_per_sweep / (ms * 1e-3) / 1e9
    flagged = sum(int(np.count_nonzero(w.view("status", torch.int32)[:Wb].cpu().numpy() & 1)) for w in walkers)
    traffic, split = (None, None) if streams else counted_traffic("batch", total_w, S, nt, args.precision)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on each system for a third of the time, summed as walker-steps per second of all three
        parts = [cpu_oracle_baseline(wl, args.cpu_seconds / 3) for wl in wls]
        per_ws = sum(1.0 / p["value"] for p in parts) / len(parts)  # mean CPU seconds per walker-step
        cpu = {"value": 1.0 / per_ws, "unit": "walker-steps/s", "cores": parts[0]["cores"], "kind": "oracle",
               "sample": "; ".join(f"{n}: {p['sample']}" for n, p in zip(names, parts))}
    out = {
        "metric": METRIC, "value": total_w * S * args.steps / wall, "unit": "walker-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "uneven batch: H-chain-like 40/80/160 orbitals, half filled, eps=1e-5",
                   "walkers": [Wb] * len(names), "ctmc_moves_per_step": S, "threads": nt,
                   "mode": "streams" if streams else "fused", "precision": args.precision},
        "flagged_walkers": flagged,
        ("el_max_abs_err_per_electron" if prec == vmc.VMC_MIXED else "el_max_abs_err_vs_oracle"): el_err,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "traffic_split": split,
                     "kernel": ("k_sweep per system, one stream each (time from fork to join)" if streams
                                else "k_sweep_batch (one launch)"), "sweep_kernel_ms": ms,
                     "bytes_per_sweep_all_walkers": bytes_per_sweep, "state_in_lds": in_lds},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU: walkers are independent and a multi-GPU run "
                                   "would shard them with one gradient all-reduce per iteration, which is not "
                                   "implemented here; run with --gpus 1"}), flush=True)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.config == "batch":
        batch_bench(args)
        return

    import numpy as np
    import torch

    from paper_1807_10633_amd import vmc
    from workloads import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = make_config(args.config, n_walkers=(args.walkers or None), eps=args.eps, orbitals=args.orbitals,
                     cps=args.cps)
    uhf = args.orbitals == "uhf"
    W, S = wl.n_walkers, args.sweep
    head_prec = vmc.VMC_MIXED if args.precision == "mixed" else vmc.VMC_FP64
    stream = torch.cuda.current_stream()

    def run_form(precision, steps, warmup, check):
        """One optimisation iteration per step, as described in the module docstring."""
        mixed = precision == vmc.VMC_MIXED
        sysm = vmc.System.from_workload(wl, refresh_period=S, precision=precision)
        walkers = sysm.walkers(wl.occ)
        # burn-in of the walkers (not timed, not counted), then the launch
        # shape: the project autotuner times sweeps of equilibrated walkers
        # at every workgroup size and occupancy target (more burn-in), each
        # as long as the timed ones, since a launch also carries a fixed
        # set-up cost that depends on the shape
        vmc.vmc_ctmc_step(sysm.handle, walkers, 100, stream=stream)
        if args.threads:
            vmc.vmc_set_launch(sysm.handle, args.threads)
            vmc.vmc_set_occupancy(sysm.handle, args.waves)
        else:
            vmc.vmc_autotune(sysm.handle, walkers, S)
        npar = sysm.n_params
        params = sysm.param_vector().clone()
        m = torch.zeros_like(params)
        v = torch.zeros_like(params)
        vh = torch.zeros_like(params)
        G = torch.zeros_like(params)
        est = torch.zeros(4, dtype=torch.float64, device=dev)
        g = torch.zeros(W, dtype=torch.float64, device=dev)
        sweep_t, eloc_t = HipTimer(stream), HipTimer(stream)

        def iteration(st):
            vmc.vmc_local_energy(sysm.handle, walkers, stream=st)
            vmc.vmc_estimate(sysm.handle, walkers, est, g, stream=st)
            vmc.vmc_logderiv(sysm.handle, walkers, g, G, stream=st)
            vmc.vmc_amsgrad(params, m, v, vh, G, 1e-3, 0.9, 0.99, 1e-8, False, stream=st)
            sysm.set_param_vector(params, stream=st)
            vmc.vmc_walkers_refresh(sysm.handle, walkers, stream=st)

        def one_step(timed):
            if timed:
                sweep_t.start()
            vmc.vmc_ctmc_step(sysm.handle, walkers, S, stream=stream)
            if timed:
                sweep_t.stop()
            # E_L and t of the post-sweep states, so that O_k and E_L refer to the same determinant
            iteration(stream)
            return est[2]

        for _ in range(warmup):
            one_step(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E = None
        for _ in range(steps):
            E = one_step(True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # E_L evaluations alone (vmc_local_energy over every walker)
        for _ in range(3):
            eloc_t.start()
            vmc.vmc_local_energy(sysm.handle, walkers, stream=stream)
            eloc_t.stop()
        torch.cuda.synchronize()
        # the same iteration captured once in a HIP graph and replayed (CTMC
        # moves with the device-resident step counter)
        graph_value = None
        if not args.no_graph:
            step_dev = torch.tensor([walkers.step], dtype=torch.int64, device=dev)
            graph = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs):
                with torch.cuda.graph(graph, stream=cs):
                    st = torch.cuda.current_stream()
                    vmc.vmc_ctmc_step_dev(sysm.handle, walkers, S, step_dev, stream=st)
                    iteration(st)
            torch.cuda.current_stream().wait_stream(cs)
            graph.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                graph.replay()
            torch.cuda.synchronize()
            graph_value = W * S * steps / (time.perf_counter() - t0)
            walkers.step = int(step_dev.item())
        res = {"sysm": sysm, "walkers": walkers, "params": params, "wall": wall, "E": float(E),
               "graph_value": graph_value, "value": W * S * steps / wall, "sweep_ms": sweep_t.mean_ms(),
               "eloc_ms": eloc_t.mean_ms(), "status": walkers.view("status", torch.int32)[:W].cpu().numpy()}
        res["check"] = check_eloc(sysm, walkers, mixed) if check else None
        return res

    def check_eloc(sysm, walkers, mixed):
        """One more refresh period from fresh inverses with histories; the
        oracle evaluates the sampled walkers' states of its last ten moves
        (E_L before each move) and the states it ends on (E_L by
        vmc_local_energy), all before any re-inversion."""
        from oracle.core import ORC_LEMMA, OracleSystem

        nw = sysm.n_words
        vmc.vmc_walkers_refresh(sysm.handle, walkers, stream=stream)
        occ0 = walkers.view("occ_bits", torch.int64)[: W * nw].cpu().numpy().view(np.uint64).reshape(W, nw).copy()
        step0 = walkers.step
        eh = torch.zeros((S, W), dtype=torch.float64, device=dev)
        ph = torch.zeros((S, W), dtype=torch.int64, device=dev)
        vmc.vmc_ctmc_step(sysm.handle, walkers, S, eh, None, ph, stream=stream)
        vmc.vmc_local_energy(sysm.handle, walkers, stream=stream)
        torch.cuda.synchronize()
        el_end = walkers.view("eloc", torch.float64)[:W].cpu().numpy()
        eh, ph = eh.cpu().numpy(), ph.cpu().numpy()
        idx = np.unique(np.linspace(0, W - 1, args.check_walkers).astype(int))
        states, ref, wk, sk = [], [], [], []
        k0 = max(0, S - 10)
        for w in idx:
            bits = occ0[w].copy()
            for k in range(S):
                if k >= k0:
                    states.append(bits.copy())
                    ref.append(eh[k, w])
                    wk.append(w)
                    sk.append(step0 + k)
                t, i, j, a, b = vmc.vmc_decode_pick(int(ph[k, w]))
                if t:
                    bits[i >> 6] &= ~np.uint64(1 << (i & 63))
                    bits[a >> 6] |= np.uint64(1 << (a & 63))
                    if t == 2:
                        bits[j >> 6] &= ~np.uint64(1 << (j & 63))
                        bits[b >> 6] |= np.uint64(1 << (b & 63))
            states.append(bits.copy())
            ref.append(el_end[w])
            wk.append(w)
            sk.append(step0 + S)
        orc = OracleSystem.from_workload(wl)
        orc.set_params(*sysm.host_params())
        if len(wl.cps_sites):
            orc.set_cps(wl.cps_sites, sysm.host_cps())
        e_o, t_o, _, _, rc = orc.eval_states(np.stack(states), wl.ctmc_seed, np.array(wk), np.array(sk), ORC_LEMMA,
                                             min(16, os.cpu_count() or 1))
        ok = rc == 0
        d = np.abs(e_o - np.array(ref))[ok]
        T = 1.0 / t_o[ok]
        tol = (1e-6 * wl.n_elec + 1e-9 * T) if mixed else (1e-10 + 1e-13 * T)
        return {"states": int(ok.sum()), "walkers": int(idx.size), "moves_since_inversion": [k0, S],
                "max_abs_err": float(d.max()), "max_abs_err_per_electron": float(d.max() / wl.n_elec),
                "max_err_over_tol": float(np.max(d / tol)), "median_T": float(np.median(T))}

    head = run_form(head_prec, args.steps, args.warmup, not args.no_check)
    sysm, walkers = head["sysm"], head["walkers"]
    value, wall, sweep_ms, E, status = head["value"], head["wall"], head["sweep_ms"], head["E"], head["status"]
    other = None
    if not args.no_other_form:
        o_prec = vmc.VMC_FP64 if head_prec == vmc.VMC_MIXED else vmc.VMC_MIXED
        o = run_form(o_prec, args.steps, args.warmup, not args.no_check)
        other = {"precision": "fp64" if o_prec == vmc.VMC_FP64 else "mixed", "value": o["value"],
                 "unit": "walker-steps/s", "sweep_kernel_ms": o["sweep_ms"],
                 "eloc_evals_per_s": W / (o["eloc_ms"] * 1e-3), "eloc_check": o["check"],
                 "energy": o["E"], "flagged_walkers": int(np.count_nonzero(o["status"] & 1)),
                 "graph_replay_value": o["graph_value"], "headline_over_this": value / o["value"],
                 "launch": vmc.vmc_launch_info(o["sysm"].handle)}
        o["sysm"].close()

    # --- algorithmic work of the sweep kernel, from candidate counts of a
    #     sample of the final walker states (library diagnostic entry point)
    ne, n_so = sysm.ne, sysm.n_so
    cap = 400000
    ijab = torch.zeros((cap, 5), dtype=torch.int32, device=dev)
    hv = torch.zeros(cap, dtype=torch.float64, device=dev)
    rv = torch.zeros(cap, dtype=torch.float64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ks, kd = [], []
    for w in range(0, W, max(1, W // 32)):
        vmc.vmc_excitations(sysm.handle, walkers, w, ijab, hv, rv, cap, cnt)
        n = int(cnt.item())
        types = ijab[: min(n, cap), 0].cpu().numpy()
        ks.append(int(np.count_nonzero(types == 1)))
        kd.append(int(np.count_nonzero(types == 2)))
    K_s, K_d = float(np.mean(ks)), float(np.mean(kd))
    # FP64 flops per walker-step: doubles 10 (2x2 minor 3, Jastrow 4, E_L 2,
    # rate 1); singles Ne + 7; H_NN Ne(Ne-1)/2 + Ne; update 2*1.5*(|R|+|B|)
    # (1.5 = mean electrons moved: the single/double pick mix is not tracked,
    # the midpoint is used); Jastrow sums 3 n_so; refresh amortised over the
    # sweep: GJ 2 Ne^3 + R 2 n_so Ne^2.
    # Spin-blocked orbitals: the update touches one spin's blocks, R n x N_s
    # and B N_s x N_s (N_s = N_e / 2 on average).
    upd = (sysm.n_orb * ne / 2 + ne * ne / 4) if uhf else (n_so * ne + ne * ne)
    flops = (10.0 * K_d + (ne + 7.0) * K_s + ne * (ne - 1) / 2 + ne + 2 * 1.5 * upd + 3 * n_so
             + (2.0 * ne ** 3 + 2.0 * n_so * ne * ne) / S)
    info = vmc.vmc_launch_info(sysm.handle)
    # mixed form: FP32 R, plus its bfloat16 remainder where the state is in HBM
    rbytes = (4 if info["state_in_lds"] else 6) if args.precision == "mixed" else 8
    # HBM bytes per walker-step when the state stays in HBM: R and B read and
    # written once per move.  Spin-blocked: the moving spin's blocks, averaged
    # over the two spins (exact for single moves and same-spin doubles; an
    # opposite-spin double touches both spins' blocks)
    if uhf:
        na, nb, n = sysm.n_alpha, sysm.n_beta, sysm.n_orb
        state_bytes = (n * na * rbytes + na * na * 8) + (n * nb * rbytes + nb * nb * 8)
    else:
        state_bytes = 2.0 * (n_so * ne * rbytes + ne * ne * 8)
    sweep_s = sweep_ms * 1e-3
    achieved_tflops = flops * W * S / sweep_s / 1e12
    # counted figures belong to the workload as defined, not to another screening threshold
    ckey = args.config if args.eps is None else f"{args.config}:eps={args.eps:g}"
    if uhf:
        ckey += ":uhf"
    if args.cps:
        ckey += f":cps={args.cps}"
    traffic, traffic_split = counted_traffic(ckey, W, S, info["threads"], args.precision)
    common = {
        "kernel": ("k_sweep (persistent E_L + CTMC + Sherman-Morrison, walker state in LDS)" if info["state_in_lds"]
                   else "k_sweep (walker state in HBM), one vmc_ctmc_step; the re-inversion after each parameter "
                        "update is outside the timed sweep but inside the step"),
        "traffic": traffic,
        "traffic_split": traffic_split,
        "hbm_gbs_measured": (traffic / sweep_s / 1e9) if traffic else None,
        "flop_per_walker_step": flops,
        "K_singles": K_s,
        "K_doubles": K_d,
        "sweep_kernel_ms": sweep_ms,
        "issue": counted_issue(ckey, W, S, info["threads"], args.precision, sweep_s),
        "launch": info,
    }
    if info["state_in_lds"]:
        roofline = {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved_tflops / FP64_VECTOR_PEAK_TFLOPS, **common}
    else:
        gbs = state_bytes * W * S / sweep_s / 1e9
        roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                    "bytes_per_walker_step": state_bytes, "fp64_tflops": achieved_tflops, **common}

    cpu = None if args.no_cpu_baseline else cpu_oracle_baseline(wl, args.cpu_seconds)
    chk = head["check"]
    workload = {
        "hchain160": "hchain160: H-chain-like 160 orbitals, 80a+80b, eps=1e-5, 8192 walkers",
        "hchain20": "hchain20: H-chain-like 20 orbitals, 10a+10b, eps=1e-6, 4096 walkers",
        "hubbard10x10": "hubbard10x10: 2-D Hubbard 10x10 periodic, U=4, 50a+50b, 16384 walkers",
    }.get(args.config, args.config)
    if args.eps is not None or args.walkers or uhf or args.cps:
        workload = f"{args.config} (eps={wl.eps:g}, {W} walkers, {args.orbitals}, cps={args.cps})"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload, "walkers": W, "ctmc_moves_per_step": S, "refresh_period": S,
                   "precision": args.precision, "eps": wl.eps, "orbitals": args.orbitals,
                   "correlators": args.cps},
        "eloc_evals_per_s": W / (head["eloc_ms"] * 1e-3),
        "eloc_kernel_ms": head["eloc_ms"],
        "graph_replay_value": head["graph_value"],
        "el_max_abs_err_vs_oracle": chk["max_abs_err"] if chk else None,
        "el_max_abs_err_per_electron": chk["max_abs_err_per_electron"] if chk else None,
        "eloc_check": chk,
        "energy": E,
        "other_form": other,
        "flagged_walkers": int(np.count_nonzero(status & 1)),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
