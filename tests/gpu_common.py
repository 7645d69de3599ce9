"""Helpers shared by the GPU tests: run the library through its C ABI and
compare with the CPU oracle on the same seeded inputs."""
import numpy as np

from oracle.core import ORC_LEMMA, OracleSystem

EL_TOL = 1e-10  # |Delta E_L| bar for the FP64 path (Hartree, or units of t)
MIXED_TOL = 1e-6  # per electron, the mixed form's bar
PICK_MARGIN = 1e-12  # picks within this relative distance of a boundary are exempt
ST_STALE = 16  # status bit: moved since the last inversion (not an error)


def el_tol(T):
    """FP64 bar near nodes: 1e-10 + 1e-13 T, T = sum |psi(M)/psi(N)| of the
    state.  The fresh-LU and lemma ratios of oracle and GPU round at a level
    that grows with the conditioning of theta[N], which T measures; for T below
    about 1e3 this is the plain 1e-10."""
    return EL_TOL + 1e-13 * np.asarray(T, dtype=np.float64)


def mixed_tol(T, n_elec):
    """Mixed-form bar: 1e-6 per electron, plus a T-scaled term 1e-8 T for
    states near a node, where the FP32 storage of R (unit roundoff 6e-8)
    enters every ratio relative to the walker's scale T."""
    return MIXED_TOL * n_elec + 1e-8 * np.asarray(T, dtype=np.float64)


def trajectory_states(occ0, ph, idx, k_range=None):
    """The determinants a sweep visited: for each sampled walker w in idx, the
    state before move k (k in k_range, default all) rebuilt from its start
    occ0[w] and the packed picks ph[:, w].  Also returns the state after the
    last move.  Returns (states, walker, k) arrays, with k = n_steps for the
    final states."""
    n_steps = ph.shape[0]
    ks = set(range(n_steps)) if k_range is None else set(k_range)
    states, wk, kk = [], [], []
    for w in idx:
        bits = occ0[w].copy()
        for k in range(n_steps):
            if k in ks:
                states.append(bits.copy())
                wk.append(int(w))
                kk.append(k)
            bits = apply_pick(bits, ph[k, w])
        states.append(bits.copy())
        wk.append(int(w))
        kk.append(n_steps)
    return np.stack(states), np.array(wk), np.array(kk)


def teacher_forced_batch(orc, seed, occ0, step0, eh, th, ph, idx, k_range=None, el_final=None, threads=0):
    """teacher_forced_check with every state evaluated in one parallel oracle
    call (orc.eval_states).  The final states are compared with el_final (E_L
    of vmc_local_energy after the sweep) when given.  Returns arrays per state
    (dE, T, dt_rel, k) and the pick statistics."""
    from paper_1807_10633_amd.vmc import vmc_decode_pick

    states, wk, kk = trajectory_states(occ0, ph, idx, k_range)
    n_steps = eh.shape[0]
    e_o, t_o, pick, margin, rc = orc.eval_states(states, seed, wk, step0 + kk, ORC_LEMMA, threads)
    sel = kk < n_steps if el_final is None else np.ones(kk.size, dtype=bool)
    assert np.all(rc[sel] == 0), "oracle failed on a visited state"
    gpu_el = np.where(kk < n_steps, eh[np.minimum(kk, n_steps - 1), wk], np.nan)
    if el_final is not None:
        gpu_el = np.where(kk == n_steps, el_final[wk], gpu_el)
    gpu_t = np.where(kk < n_steps, th[np.minimum(kk, n_steps - 1), wk], np.nan)
    dE = np.abs(e_o - gpu_el)[sel]
    T = 1.0 / t_o[sel]
    mv = kk < n_steps
    dt_rel = np.abs(t_o[mv] - gpu_t[mv]) / t_o[mv]
    n_pick = n_exempt = 0
    mismatches = []
    for s in np.flatnonzero(mv):
        g = vmc_decode_pick(int(ph[kk[s], wk[s]]))
        if margin[s] < PICK_MARGIN:
            n_exempt += 1
        else:
            n_pick += 1
            if tuple(g) != tuple(int(x) for x in pick[s]):
                mismatches.append((int(wk[s]), int(kk[s]), tuple(pick[s]), g, float(margin[s])))
    return {"dE": dE, "T": T, "k": kk[sel], "dt_rel": dt_rel, "picks_compared": n_pick, "picks_exempt": n_exempt,
            "mismatches": mismatches, "states": int(sel.sum())}


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
