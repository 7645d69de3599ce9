"""Estimators and AMSGrad, written from their definitions.

TEST INFRASTRUCTURE ONLY.

* Energy (Eq. eq:vmc with CTMC residence-time weights): E = sum_w t_w E_L,w / sum_w t_w.
* Gradient (Eq. eq:grad): G_k = 2 < O_k (E_L - E) >, the average weighted by t,
  with E the same-sample weighted mean.
* AMSGrad (section "AMSGrad algorithm for optimizing the energy"), in the form
  of Reddi, Kale and Kumar (2018) with the standard beta convention:
      m <- b1 m + (1-b1) G ;  v <- b2 v + (1-b2) G^2 ;  vhat <- max(vhat, v)
      p <- p - alpha m / (sqrt(vhat) + delta)
  The paper's own equations use beta' = 1 - beta and put the max inside the
  moving average; ``paper_literal=True`` gives n <- max(n, (1-b2') n + b2' G^2)
  with b1' = 1 - b1, b2' = 1 - b2.
"""
from __future__ import annotations

import numpy as np


def weighted_energy(eloc: np.ndarray, t: np.ndarray) -> float:
    eloc = np.asarray(eloc, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return float(np.sum(t * eloc) / np.sum(t))


def gradient(O: np.ndarray, eloc: np.ndarray, t: np.ndarray) -> np.ndarray:
    """O is (W, N_p); returns G (N_p,)."""
    O = np.asarray(O, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    E = weighted_energy(eloc, t)
    g = 2.0 * t * (np.asarray(eloc) - E) / np.sum(t)
    return g @ O


def contraction_weights(eloc: np.ndarray, t: np.ndarray) -> np.ndarray:
    """g_w = 2 t_w (E_L,w - E) / sum t, so that G = sum_w g_w O_w."""
    t = np.asarray(t, dtype=np.float64)
    E = weighted_energy(eloc, t)
    return 2.0 * t * (np.asarray(eloc, dtype=np.float64) - E) / np.sum(t)


class AMSGrad:
    def __init__(self, n_params: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.99,
                 delta: float = 1e-8, paper_literal: bool = False):
        self.m = np.zeros(n_params)
        self.v = np.zeros(n_params)
        self.vhat = np.zeros(n_params)
        self.lr, self.b1, self.b2, self.delta = lr, beta1, beta2, delta
        self.paper_literal = paper_literal

    def step(self, params: np.ndarray, G: np.ndarray) -> np.ndarray:
        G = np.asarray(G, dtype=np.float64)
        if self.paper_literal:
            self.m = self.b1 * self.m + (1.0 - self.b1) * G
            self.vhat = np.maximum(self.vhat, self.b2 * self.vhat + (1.0 - self.b2) * G * G)
        else:
            self.m = self.b1 * self.m + (1.0 - self.b1) * G
            self.v = self.b2 * self.v + (1.0 - self.b2) * G * G
            self.vhat = np.maximum(self.vhat, self.v)
        return params - self.lr * self.m / (np.sqrt(self.vhat) + self.delta)
