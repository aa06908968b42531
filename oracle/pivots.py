"""Weight-scaled, fixed-rank pivoted Cholesky and pivot fusion.

Follows the ISDF section (pivot selection by pivoted Cholesky, Alg. 1) and the
matrix-free pivot search of the numerical-implementation notes:
  scalar channel   d_g = w_g^2 (sum_p phi_p(g)^2)^2,
                   s_g = w_g w_* (sum_p phi_p(g) phi_p(*))^2;
  gradient channel d_g = w_g^2 (sum_p phi_p(g)^2)(sum_{p,c} d_c phi_p(g)^2),
                   s_g = w_g w_* (sum_p phi_p(g) phi_p(*)) (sum_{p,c} d_c phi_p(g) d_c phi_p(*)).
Each step: g* = argmax_g d_g, L_{g,mu} = (s_g - sum_{lambda<mu} L_{g,lambda} L_{g*,lambda}) / sqrt(d_{g*}),
d_g <- max(d_g - L_{g,mu}^2, 0).

Readings where the paper is silent (also listed in the design notes):
  * ties in the argmax go to the lowest grid index;
  * the selected point's own residual is set to its exact-arithmetic value 0
    after its update (the update gives d_{g*} - d_{g*});
  * the fixed-rank loop stops early, reporting rank deficiency, once
    max_g d_g <= 1e-14 * max_g D_g (the division by sqrt(d_{g*}) would
    otherwise divide by zero after the clamp);
  * fusion "fill-to-target": the gradient channel runs to ceil(N_mu / 2)
    pivots, then the scalar channel is extended one pivot at a time until the
    union holds N_mu points; the fused order is the scalar pivots in selection
    order followed by the gradient-only pivots in theirs.

Pinned by: equality with LAPACK's column-pivoted QR (scipy.linalg.qr with
pivoting) on an explicit weighted pair matrix for tiny inputs, the projection
residual identity sum_g d_g = ||M_w - P_S M_w||_F^2, monotone pivot values and
termination exactly at the numerical rank.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

RANK_TOL = 1e-14


def diagonal(phi4: np.ndarray, w: np.ndarray, channel: str) -> np.ndarray:
    n2 = np.einsum("pg,pg->g", phi4[0], phi4[0])
    if channel == "scalar":
        return w * w * n2 * n2
    g2 = np.einsum("cpg,cpg->g", phi4[1:4], phi4[1:4])
    return w * w * n2 * g2


def column(phi4: np.ndarray, w: np.ndarray, gstar: int, channel: str) -> np.ndarray:
    a = phi4[0].T @ phi4[0][:, gstar]
    if channel == "scalar":
        return w * w[gstar] * a * a
    b = np.einsum("cpg,cp->g", phi4[1:4], phi4[1:4][:, :, gstar])
    return w * w[gstar] * a * b


@dataclass
class CholeskyState:
    """Incremental state of one channel's pivoted Cholesky (Alg. 1)."""
    phi4: np.ndarray
    w: np.ndarray
    channel: str
    d: np.ndarray = None
    d0max: float = 0.0
    L: list = field(default_factory=list)
    pivots: list = field(default_factory=list)
    pivot_values: list = field(default_factory=list)
    gaps: list = field(default_factory=list)
    deficient: bool = False

    def __post_init__(self):
        self.d = diagonal(self.phi4, self.w, self.channel)
        self.d0max = float(self.d.max()) if self.d.size else 0.0

    def step(self) -> bool:
        """One pivot; returns False (and marks rank deficiency) if none is left."""
        gstar = int(np.argmax(self.d))          # first maximum = lowest index
        dmax = float(self.d[gstar])
        if not dmax > RANK_TOL * self.d0max:
            self.deficient = True
            return False
        rest = np.delete(self.d, gstar)
        second = float(rest.max()) if rest.size else 0.0
        self.gaps.append((dmax - second) / dmax)
        s = column(self.phi4, self.w, gstar, self.channel)
        if self.L:
            Lm = np.asarray(self.L)
            s = s - Lm.T @ Lm[:, gstar]
        col = s / np.sqrt(dmax)
        self.d = np.maximum(self.d - col * col, 0.0)
        self.d[gstar] = 0.0
        self.L.append(col)
        self.pivots.append(gstar)
        self.pivot_values.append(dmax)
        return True


def pivoted_cholesky(phi4, w, n_steps: int, channel: str = "scalar") -> CholeskyState:
    st = CholeskyState(phi4, w, channel)
    for _ in range(n_steps):
        if not st.step():
            break
    return st


@dataclass
class FusedPivots:
    pivots: np.ndarray          # int64 [n], fused order
    scalar: list
    grad: list
    deficient: bool
    scalar_state: CholeskyState
    grad_state: CholeskyState


def select_fused(phi4, w, n_mu: int) -> FusedPivots:
    """Fill-to-target union of the gradient and scalar channels."""
    n_grad = (n_mu + 1) // 2
    gs = pivoted_cholesky(phi4, w, n_grad, "grad")
    gset = set(gs.pivots)
    ss = CholeskyState(phi4, w, "scalar")
    union = len(gset)
    while union < n_mu:
        if not ss.step():
            break
        if ss.pivots[-1] not in gset:
            union += 1
    sset = set(ss.pivots)
    fused = list(ss.pivots) + [g for g in gs.pivots if g not in sset]
    deficient = len(fused) < n_mu
    return FusedPivots(np.asarray(fused, np.int64), list(ss.pivots), list(gs.pivots),
                       deficient, ss, gs)
