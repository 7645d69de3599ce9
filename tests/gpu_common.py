"""Helpers shared by the GPU tests: run the library through its C ABI and
compare with the CPU oracle on the same seeded inputs."""
import numpy as np

from oracle.core import ORC_LEMMA, OracleSystem

EL_TOL = 1e-10  # |Delta E_L| bar for the FP64 path (Hartree, or units of t)
PICK_MARGIN = 1e-12  # picks within this relative distance of a boundary are exempt


def torch_mod():
    import torch

    return torch


def gpu_system(wl, **kw):
    from paper_1807_10633_amd.vmc import System

    return System.from_workload(wl, **kw)


def occ_of(sysm, walkers):
    torch = torch_mod()
    a = walkers.view("occ_bits", torch.int64)[: walkers.n_walkers * sysm.n_words].cpu().numpy()
    return a.view(np.uint64).reshape(walkers.n_walkers, sysm.n_words).copy()


def field(sysm, walkers, name, dtype, per_walker):
    torch = torch_mod()
    return walkers.view(name, dtype)[: walkers.n_walkers * per_walker].cpu().numpy().reshape(walkers.n_walkers,
                                                                                            per_walker)


def apply_pick(bits, code):
    from paper_1807_10633_amd.vmc import vmc_decode_pick

    t, i, j, a, b = vmc_decode_pick(int(code))
    bits = bits.copy()
    if t == 0:
        return bits
    bits[i >> 6] &= ~np.uint64(1 << (i & 63))
    bits[a >> 6] |= np.uint64(1 << (a & 63))
    if t == 2:
        bits[j >> 6] &= ~np.uint64(1 << (j & 63))
        bits[b >> 6] |= np.uint64(1 << (b & 63))
    return bits


def run_sweep(sysm, walkers, n_steps):
    """One persistent launch of n_steps moves; returns host histories."""
    torch = torch_mod()
    W = walkers.n_walkers
    eh = torch.zeros((n_steps, W), dtype=torch.float64, device="cuda")
    th = torch.zeros((n_steps, W), dtype=torch.float64, device="cuda")
    ph = torch.zeros((n_steps, W), dtype=torch.int64, device="cuda")
    from paper_1807_10633_amd.vmc import vmc_ctmc_step

    vmc_ctmc_step(sysm.handle, walkers, n_steps, eh, th, ph)
    torch.cuda.synchronize()
    return eh.cpu().numpy(), th.cpu().numpy(), ph.cpu().numpy()


def teacher_forced_check(orc: OracleSystem, seed, occ0, step0, eh, th, ph, walkers_idx, mode=ORC_LEMMA):
    """Replay each sampled walker's trajectory through the oracle.

    At every step the oracle starts from the GPU's pre-move determinant and
    computes E_L, t and its own pick; returns a dict of statistics.
    """
    from paper_1807_10633_amd.vmc import vmc_decode_pick

    n_steps = eh.shape[0]
    dE = []
    T_or = []
    dt_rel = []
    n_pick = 0
    n_exempt = 0
    mismatches = []
    for w in walkers_idx:
        bits = occ0[w].copy()
        for k in range(n_steps):
            new, el, t, pick, margin, rc = orc.ctmc_step(bits, seed, int(w), int(step0 + k), mode)
            assert rc == 0, f"oracle failed on walker {w} step {k} ({rc})"
            dE.append(abs(el - eh[k, w]))
            T_or.append(1.0 / t)
            dt_rel.append(abs(t - th[k, w]) / t)
            gpu_pick = vmc_decode_pick(int(ph[k, w]))
            if margin < PICK_MARGIN:
                n_exempt += 1
            else:
                n_pick += 1
                if tuple(gpu_pick) != tuple(pick):
                    mismatches.append((int(w), k, pick, gpu_pick, margin))
            bits = apply_pick(bits, ph[k, w])
    dE = np.array(dE)
    return {
        "max_dE": float(dE.max()),
        "p999_dE": float(np.quantile(dE, 0.999)),
        "max_dt_rel": float(np.max(dt_rel)),
        "picks_compared": n_pick,
        "picks_exempt": n_exempt,
        "mismatches": mismatches,
        "dE_all": dE,
        "T_all": np.array(T_or),
    }
