"""Weight-scaled, fixed-rank pivoted Cholesky and pivot fusion (ISDF section,
pivot selection, Alg. 1; the matrix-free pivot search of the numerical notes).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is factorised. For one channel, let m_g be the weighted pair-product
vector of grid point g: the scalar channel's m_g has the entries
w_g phi_p(g) phi_q(g) over all ordered pairs (p, q); the gradient channel's has
w_g phi_p(g) d_c phi_q(g) over (p, c, q). The pair matrix S_{gh} = m_g . m_h is
positive semidefinite, and the method never forms it: its entries follow from
orbital dot products,
  scalar    S_{gh} = w_g w_h (Phi_g . Phi_h)^2,
  gradient  S_{gh} = w_g w_h (Phi_g . Phi_h) (sum_c dPhi_g^c . dPhi_h^c),
with Phi_g the vector of orbital values at g. Selecting interpolation points is
the greedy (diagonally pivoted) Cholesky factorisation of S: after k pivots
S ~ L^T L with L [k][N_g], and the residual diagonal d_g = S_gg - sum_k L_kg^2 is
the squared norm of m_g outside the span of the selected vectors, so each new
pivot is the point the current points represent worst. The next row of L is the
residual (Schur-complement) column of S at that pivot, normalised by the square
root of its diagonal entry.

Readings where the paper is silent (also listed in the design notes):
  * ties in the argmax go to the lowest grid index;
  * the selected point's own residual is set to its exact-arithmetic value 0;
  * the fixed-rank loop stops early, reporting rank deficiency, once
    max_g d_g <= 1e-14 * max_g S_gg (the normalisation would divide by ~0);
  * fusion "fill-to-target": the gradient channel runs to ceil(N_mu / 2)
    pivots, then the scalar channel is extended one pivot at a time until the
    union holds N_mu points; the fused order is the scalar pivots in selection
    order followed by the gradient-only pivots in theirs.

Pinned by: equality with LAPACK's column-pivoted QR (scipy.linalg.qr with
pivoting) of the explicit matrix [m_g] on tiny inputs, the projection residual
identity sum_g d_g = ||M - P_S M||_F^2, non-increasing pivot values, and
termination exactly at the numerical rank.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

RANK_TOL = 1e-14


def diagonal(phi4: np.ndarray, w: np.ndarray, channel: str) -> np.ndarray:
    """S_gg for every grid point."""
    n2 = np.einsum("pg,pg->g", phi4[0], phi4[0])
    if channel == "scalar":
        return w * w * n2 * n2
    g2 = np.einsum("cpg,cpg->g", phi4[1:4], phi4[1:4])
    return w * w * n2 * g2


def column(phi4: np.ndarray, w: np.ndarray, gstar: int, channel: str) -> np.ndarray:
    """S_{g, g*} for every grid point g."""
    a = phi4[0].T @ phi4[0][:, gstar]
    if channel == "scalar":
        return w * w[gstar] * a * a
    b = np.einsum("cpg,cp->g", phi4[1:4], phi4[1:4][:, :, gstar])
    return w * w[gstar] * a * b


@dataclass
class CholeskyState:
    """Incremental state of one channel's pivoted Cholesky (Alg. 1). The factor's
    rows live in a preallocated array that doubles when full."""
    phi4: np.ndarray
    w: np.ndarray
    channel: str
    d: np.ndarray = None
    d0max: float = 0.0
    pivots: list = field(default_factory=list)
    pivot_values: list = field(default_factory=list)
    gaps: list = field(default_factory=list)
    deficient: bool = False
    _rows: np.ndarray = None

    def __post_init__(self):
        self.d = diagonal(self.phi4, self.w, self.channel)
        self.d0max = float(self.d.max()) if self.d.size else 0.0
        self._rows = np.empty((16, self.d.size))

    @property
    def L(self) -> np.ndarray:
        """The Cholesky factor's rows [k][N_g] (S ~ L^T L)."""
        return self._rows[: len(self.pivots)]

    def step(self) -> bool:
        """One pivot; returns False (and marks rank deficiency) if none is left."""
        gstar = int(np.argmax(self.d))          # first maximum = lowest index
        dmax = float(self.d[gstar])
        if not dmax > RANK_TOL * self.d0max:
            self.deficient = True
            return False
        keep = self.d[gstar]
        self.d[gstar] = -np.inf
        second = max(float(self.d.max()), 0.0) if self.d.size > 1 else 0.0
        self.d[gstar] = keep
        self.gaps.append((dmax - second) / dmax)
        k = len(self.pivots)
        # residual column of S at g*: S[:, g*] minus what the current factor explains
        resid = column(self.phi4, self.w, gstar, self.channel)
        if k:
            resid = resid - self.L.T @ self.L[:, gstar]
        row = resid / np.sqrt(dmax)
        if k == self._rows.shape[0]:
            grown = np.empty((2 * k, self.d.size))
            grown[:k] = self._rows
            self._rows = grown
        self._rows[k] = row
        self.d = np.maximum(self.d - row * row, 0.0)
        self.d[gstar] = 0.0
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
