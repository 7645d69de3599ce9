"""The energy-minimisation loop: sample, estimate, backward, AMSGrad, repeat.

Each iteration (section "AMSGrad algorithm for optimizing the energy") is
  1. `moves` CTMC moves of every walker (vmc_ctmc_step), keeping E_L and t of
     every visited state;
  2. the energy estimate over every visited state, E = sum t E_L / sum t
     (vmc_estimate over the W x moves histories, Eq. eq:vmc with
     residence-time weights);
  3. E_L and t of the final states (vmc_local_energy), their weighted mean and
     the gradient weights g_w (vmc_estimate);
  4. the gradient G = sum_w g_w O_w over the final states (vmc_logderiv,
     Eq. eq:grad);
  5. one AMSGrad step (vmc_amsgrad, Eqs. eq:m1, eq:m2) with the step size of
     the schedule;
  6. the new parameters into the tables (vmc_set_params, vmc_set_cps) and the
     walkers' inverses recomputed for them (vmc_walkers_refresh).
The gradient needs the O_k of a state, hence its inverse, which the sweep
does not keep for the states it passes through.  By default it uses the
final state of each walker; with grad_every = K it uses the walkers every K
moves (moves / K snapshots per iteration): A = sum t E_L O and B = sum t O are
accumulated per snapshot by the contracted backward and G = 2 (A - E B) /
sum t (vmc_snapshot_weights, vmc_logderiv_accumulate, vmc_gradient_combine).
With many parameters the extra states matter: the gradient of one state per
walker fits the noise of those states.  The energy uses every visited state.

Every step runs in the library's kernels; this module only sequences the calls
on one stream and holds the device buffers.  The default schedule is the
paper's for its larger chains (section "Performance of the optimizer"):
alpha = 0.001 for the first 5 iterations, then 0.01.  beta1 = 0.9 and beta2 =
0.99 in the standard convention are the paper's beta1 = 0.1, beta2 = 0.01;
`paper_literal` selects the paper's own form of Eq. eq:m2.

    python -m paper_1807_10633_amd.optimize --config hubbard8 --iters 40
prints one JSON line per iteration.

`evaluate` gives the energy of fixed parameters at another screening
threshold: the paper optimises with a loose eps and computes the final energy
in one shot with a tighter one (section "Accuracy and scaling"); `--eval-eps`
runs that after the iterations.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Callable, List, Optional

import torch

from . import vmc as _vmc


def paper_schedule(i: int) -> float:
    """Step size of iteration i (0-based): 0.001 for 5 iterations, then 0.01."""
    return 0.001 if i < 5 else 0.01


class Optimizer:
    """Energy minimisation of one system's Jastrow, orbital and (when the
    system has them) correlator parameters.

    system: a vmc.System; walkers: its vmc.Walkers (initialised); J, theta
    (and cps): device float64 tensors (packed Jastrow upper triangle, n_so x
    n_so theta, correlator coefficients), copied into one parameter vector,
    in the order of vmc_logderiv, that the optimiser owns.
    """

    def __init__(self, system, walkers, J, theta, *, cps=None, moves: int = 50, grad_every: int = 0,
                 schedule: Callable[[int], float] = paper_schedule, beta1: float = 0.9, beta2: float = 0.99,
                 delta: float = 1e-8, paper_literal: bool = False, stream=None):
        if not J.is_cuda or not theta.is_cuda:
            raise RuntimeError("the optimiser runs on the GPU only")
        self.system, self.walkers = system, walkers
        self.moves, self.schedule = int(moves), schedule
        # gradient states: the walkers every grad_every moves (default: the
        # final states only)
        self.grad_every = int(grad_every) or self.moves
        if self.grad_every < 1 or self.moves % self.grad_every:
            raise ValueError("grad_every must divide moves")
        self.n_snap = self.moves // self.grad_every
        self.beta1, self.beta2, self.delta, self.paper_literal = beta1, beta2, delta, paper_literal
        self.stream = stream
        dev = J.device
        self.nj = system.n_so * (system.n_so + 1) // 2
        self.nt = system.n_so * system.n_so
        parts = [J.reshape(-1).to(torch.float64), theta.reshape(-1).to(torch.float64)]
        if system.n_cps:
            parts.append((cps if cps is not None else system.cps).reshape(-1).to(torch.float64))
        self.params = torch.cat(parts).contiguous()
        assert self.params.numel() == system.n_params
        W = walkers.n_walkers
        self.eh = torch.zeros((self.moves, W), dtype=torch.float64, device=dev)
        self.th = torch.zeros((self.moves, W), dtype=torch.float64, device=dev)
        self.est_all = torch.zeros(4, dtype=torch.float64, device=dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.vhat = torch.zeros_like(self.params)
        self.G = torch.zeros_like(self.params)
        self.est = torch.zeros(4, dtype=torch.float64, device=dev)
        self.g = torch.zeros(walkers.n_walkers, dtype=torch.float64, device=dev)
        if self.n_snap > 1:
            self.A = torch.zeros_like(self.params)
            self.B = torch.zeros_like(self.params)
            self.acc = torch.zeros(4, dtype=torch.float64, device=dev)
            self.g_t = torch.zeros(walkers.n_walkers, dtype=torch.float64, device=dev)
        self.iteration = 0
        self._apply()

    @property
    def J(self):
        return self.params[: self.nj]

    @property
    def theta(self):
        return self.params[self.nj:self.nj + self.nt].view(self.system.n_so, self.system.n_so)

    @property
    def cps(self):
        return self.params[self.nj + self.nt:]

    def _apply(self) -> None:
        h, st = self.system.handle, self.stream
        self.system.set_param_vector(self.params, stream=st)
        _vmc.vmc_walkers_refresh(h, self.walkers, stream=st)

    def step(self) -> torch.Tensor:
        """One iteration; returns the device scalar E of the gradient's states
        (the final states, or every grad_every-th), estimated before the
        parameter update.  est_all then holds {sum t, sum t E_L, E, count}
        over every state the iteration visited."""
        h, st, w = self.system.handle, self.stream, self.walkers
        if self.n_snap == 1:
            _vmc.vmc_ctmc_step(h, w, self.moves, self.eh, self.th, stream=st)
            _vmc.vmc_estimate_arrays(h, self.eh, self.th, self.eh.numel(), self.est_all, stream=st)
            _vmc.vmc_local_energy(h, w, stream=st)
            _vmc.vmc_estimate(h, w, self.est, self.g, stream=st)
            _vmc.vmc_logderiv(h, w, self.g, self.G, stream=st)
        else:
            # G over the states every grad_every moves: A = sum t E_L O and
            # B = sum t O accumulated per snapshot, G = 2 (A - E B) / sum t
            K = self.grad_every
            for s in range(self.n_snap):
                _vmc.vmc_ctmc_step(h, w, K, self.eh[s * K:(s + 1) * K], self.th[s * K:(s + 1) * K], stream=st)
                _vmc.vmc_local_energy(h, w, stream=st)
                _vmc.vmc_snapshot_weights(h, w, self.acc, self.g, self.g_t, s == 0, stream=st)
                if s == 0:
                    _vmc.vmc_logderiv(h, w, self.g, self.A, stream=st)
                    _vmc.vmc_logderiv(h, w, self.g_t, self.B, stream=st)
                else:
                    _vmc.vmc_logderiv_accumulate(h, w, self.g, self.A, stream=st)
                    _vmc.vmc_logderiv_accumulate(h, w, self.g_t, self.B, stream=st)
            _vmc.vmc_estimate_arrays(h, self.eh, self.th, self.eh.numel(), self.est_all, stream=st)
            _vmc.vmc_gradient_combine(self.A, self.B, self.acc, self.G, stream=st)
            self.est.copy_(self.acc)
        _vmc.vmc_amsgrad(self.params, self.m, self.v, self.vhat, self.G, self.schedule(self.iteration), self.beta1,
                         self.beta2, self.delta, self.paper_literal, stream=st)
        self._apply()
        self.iteration += 1
        return self.est[2].clone()

    def run(self, n_iter: int) -> List[float]:
        return [float(self.step().item()) for _ in range(n_iter)]

    def run_all_states(self, n_iter: int) -> List[float]:
        """As run, returning the energies over every visited state."""
        out = []
        for _ in range(n_iter):
            self.step()
            out.append(float(self.est_all[2].item()))
        return out


def evaluate(wl, J, theta, occ, *, eps: float, rounds: int = 10, moves: int = 50, burn: int = 100,
             precision: int = _vmc.VMC_FP64, orbitals: int = _vmc.VMC_GHF, stream=None) -> dict:
    """Energy of fixed parameters (device tensors J, theta) on the Hamiltonian of
    workload wl screened at eps, from walkers starting at occupations occ.

    After `burn` CTMC moves, each of `rounds` rounds makes `moves` moves and
    estimates E from the residence-time weighted local energies of the final
    states (vmc_estimate).  Returns the mean over rounds, its standard error
    (rounds taken as independent) and the per-round values.
    """
    system = _vmc.System(wl.n_orb, wl.n_alpha, wl.n_beta, wl.h1, wl.eri_idx, wl.eri_val, eps, seed=wl.ctmc_seed + 1,
                         refresh_period=moves, precision=precision, orbitals=orbitals)
    system.set_params(J, theta)
    walkers = system.walkers(occ)
    est = torch.zeros(4, dtype=torch.float64, device=J.device)
    g = torch.zeros(walkers.n_walkers, dtype=torch.float64, device=J.device)
    if burn:
        _vmc.vmc_ctmc_step(system.handle, walkers, burn, stream=stream)
    energies = []
    for _ in range(rounds):
        _vmc.vmc_ctmc_step(system.handle, walkers, moves, stream=stream)
        _vmc.vmc_local_energy(system.handle, walkers, stream=stream)
        _vmc.vmc_estimate(system.handle, walkers, est, g, stream=stream)
        energies.append(float(est[2].item()))
    e = torch.tensor(energies, dtype=torch.float64)
    err = float(e.std(unbiased=True).item() / len(energies) ** 0.5) if len(energies) > 1 else float("nan")
    return {"energy": float(e.mean().item()), "stderr": err, "rounds": energies, "eps": eps,
            "system": system, "walkers": walkers}


def plateau(energies: List[float], window: int, block: int = 10) -> dict:
    """Mean energy of the last two windows of `window` iterations, each with
    the standard error of its means over blocks of `block` iterations (the
    iterations' estimates are correlated through the walkers and the slowly
    moving parameters), and their difference in units of the combined error."""
    import numpy as np

    out = {}
    for name, seg in (("previous", energies[-2 * window:-window]), ("last", energies[-window:])):
        seg = np.asarray(seg, dtype=np.float64)
        nb = max(1, seg.size // block)
        means = seg[: nb * block].reshape(nb, -1).mean(axis=1)
        err = float(means.std(ddof=1) / np.sqrt(nb)) if nb > 1 else float("nan")
        out[name] = {"mean": float(seg.mean()), "stderr": err}
    d = out["last"]["mean"] - out["previous"]["mean"]
    out["difference"] = d
    out["difference_in_sigma"] = d / float(np.hypot(out["last"]["stderr"], out["previous"]["stderr"]))
    return out


def _main(argv: Optional[List[str]] = None) -> int:
    from workloads import make_config

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="hubbard8")
    ap.add_argument("--walkers", type=int, default=0, help="0: the configuration's walker count")
    ap.add_argument("--iters", type=int, default=40)
    ap.add_argument("--moves", type=int, default=50)
    ap.add_argument("--grad-every", type=int, default=10,
                    help="gradient states: the walkers every this many moves (moves: the final states only)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--orbitals", choices=("ghf", "uhf"), default="ghf",
                    help="general or spin-blocked (unrestricted) orbitals")
    ap.add_argument("--paper-literal", action="store_true")
    ap.add_argument("--eps", type=float, default=None, help="screening threshold of the optimisation "
                    "(default: the configuration's own)")
    ap.add_argument("--eval-eps", type=float, default=None,
                    help="after the iterations, evaluate the final parameters at this threshold")
    ap.add_argument("--eval-rounds", type=int, default=20)
    ap.add_argument("--cps", default=None, help="correlators (chainK, plus5)")
    ap.add_argument("--window", type=int, default=0,
                    help="after the iterations, compare the mean energy of the last two windows of this many "
                         "iterations (blocks of 10 iterations for the error bars)")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "needs a GPU"}))
        return 2
    wl = make_config(args.config, n_walkers=args.walkers or None, eps=args.eps, orbitals=args.orbitals,
                     cps=args.cps)
    prec = _vmc.VMC_MIXED if args.precision == "mixed" else _vmc.VMC_FP64
    system = _vmc.System.from_workload(wl, precision=prec, refresh_period=args.moves)
    walkers = system.walkers(wl.occ)
    opt = Optimizer(system, walkers, torch.as_tensor(wl.jastrow, device="cuda"),
                    torch.as_tensor(wl.theta, device="cuda"), moves=args.moves, grad_every=args.grad_every,
                    paper_literal=args.paper_literal)
    history = []
    for i in range(args.iters):
        t0 = time.perf_counter()
        E = float(opt.step().item())  # .item() waits for the iteration
        ea = opt.est_all.cpu().numpy()
        history.append(float(ea[2]))
        print(json.dumps({"iteration": i, "alpha": paper_schedule(i), "energy": E,
                          "energy_all_states": float(ea[2]), "states": int(ea[3]),
                          "energy_per_electron": float(ea[2]) / wl.n_elec, "ms": (time.perf_counter() - t0) * 1e3}),
              flush=True)
    if args.window > 0 and len(history) >= 2 * args.window:
        print(json.dumps({"plateau": plateau(history, args.window), "n_elec": wl.n_elec}), flush=True)
    if args.eval_eps is not None:
        occ = walkers.view("occ_bits", torch.int64)[: walkers.n_walkers * system.n_words].cpu().numpy()
        ev = evaluate(wl, opt.J.clone(), opt.theta.clone(), occ.view("uint64").reshape(walkers.n_walkers, -1),
                      eps=args.eval_eps, rounds=args.eval_rounds, moves=args.moves, precision=prec,
                      orbitals=system.orbitals)
        print(json.dumps({"eval_eps": args.eval_eps, "energy": ev["energy"], "stderr": ev["stderr"],
                          "energy_per_electron": ev["energy"] / wl.n_elec}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(_main())
