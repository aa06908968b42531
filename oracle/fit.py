"""ISDF least-squares fit of the auxiliary vectors (ISDF section, eq. isdf-rho and
the normal equations that follow it; auxiliary-fit robustness note).

Scalar:   A = G o G with G = Phi_mu^T Phi_mu,   B = P o P with P = Phi_mu^T Phi,
          A xi = B.
Gradient: A_c = (dPhi_mu^T dPhi_mu)_c o G,   B_c = P o (dPhi_mu^T dPhi)_c,   A_c xi~^c = B_c.
(o is the Hadamard product; Phi_mu = Phi restricted to the pivot columns.)

The normal equations are solved through a Cholesky factorisation of A. Reading
of the adaptive Tikhonov retry (constants absent from the paper): first no
shift, then shift_k = 1e-14 * 10^k * mean(diag A) for k = 0..8; after that the
fit fails. The fit residual is reported weighted by w_g^2, matching the
weight-scaled pivot selection: R = sum_g w_g^2 (|m_g|^2 - xi(g) . B(g)), where
m_g is the pair-product column at g (|m_g|^2 = (sum_p phi_p^2)^2 for the scalar
channel, (sum_p phi_p^2)(sum_q d_c phi_q^2) for component c).

Pinned by: the interpolation property xi_mu(r_nu) = delta_{mu nu}, exact
reproduction of every pair product once N_mu reaches the pair rank, equality
with scipy.linalg.lstsq on the explicit pair matrix, and equality of the
weighted residual with the pivoted-Cholesky residual trace.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import cho_factor, cho_solve, LinAlgError

N_JITTER = 9


def gram(phi4, piv):
    """(A [N_mu, N_mu], A_c [3, N_mu, N_mu], G)."""
    Pm = phi4[:, :, piv]                       # [4, N_orb, N_mu]
    G = Pm[0].T @ Pm[0]
    A = G * G
    Ac = np.stack([(Pm[1 + c].T @ Pm[1 + c]) * G for c in range(3)])
    return A, Ac, G


def rhs(phi4, piv, scalar: bool = True, grad: bool = True, cols=None):
    """(B [N_mu, N_g], B_c [3, N_mu, N_g]); a part not asked for is None. cols: the grid
    columns to form (default all)."""
    Pm = phi4[:, :, piv]
    ph = phi4 if cols is None else phi4[:, :, np.asarray(cols)]
    P = Pm[0].T @ ph[0]
    B = P * P if scalar else None
    Bc = np.stack([P * (Pm[1 + c].T @ ph[1 + c]) for c in range(3)]) if grad else None
    return B, Bc


def chol_with_jitter(A):
    """Cholesky of A with the adaptive shift schedule; returns (factor, k) with
    k = -1 for no shift, or raises LinAlgError after the last retry."""
    try:
        return cho_factor(A, lower=True), -1
    except LinAlgError:
        pass
    scale = float(np.mean(np.diag(A)))
    for k in range(N_JITTER):
        shift = 1e-14 * 10.0 ** k * scale
        try:
            return cho_factor(A + shift * np.eye(A.shape[0]), lower=True), k
        except LinAlgError:
            continue
    raise LinAlgError("Gram matrix not positive definite after the last Tikhonov shift")


@dataclass
class FitResult:
    xi: np.ndarray          # [N_mu, N_g]
    xigrad: np.ndarray      # [3, N_mu, N_g]
    jitter: np.ndarray      # int [4]: -1 = none, else shift index k
    resid: np.ndarray       # [4] weighted residuals (scalar, x, y, z)
    resid_rel: np.ndarray   # [4] residual / sum_g w^2 |m_g|^2


def pair_norms(phi4):
    n2 = np.einsum("pg,pg->g", phi4[0], phi4[0])
    g2 = np.einsum("cpg,cpg->cg", phi4[1:4], phi4[1:4])
    return n2 * n2, n2[None, :] * g2


def fit(phi4, w, piv, with_grad: bool = True, cols=None, grad_cols=None) -> FitResult:
    """xi and xi~ from the normal equations. The system of every grid point (one column of
    B) is solved on its own with the same factor of A, so the fit is column-separable:
    cols (grid indices, default all) selects the columns of xi and grad_cols (default
    cols) those of xi~, giving exactly those columns of the full solution; the residuals
    then cover the selected columns only."""
    piv = np.asarray(piv)
    A, Ac, _ = gram(phi4, piv)
    B, Bc = rhs(phi4, piv, grad=with_grad and grad_cols is None, cols=cols)
    jit = np.full(4, -1)
    res = np.zeros(4)
    rel = np.zeros(4)
    D, Dcol = pair_norms(phi4 if cols is None else phi4[:, :, np.asarray(cols)])
    w_c = w if cols is None else w[np.asarray(cols)]
    cf, jit[0] = chol_with_jitter(A)
    xi = cho_solve(cf, B)
    w2 = w_c * w_c
    res[0] = float(np.sum(w2 * (D - np.einsum("mg,mg->g", xi, B))))
    rel[0] = res[0] / float(np.sum(w2 * D))
    del B
    xig = None
    if with_grad:
        if Bc is None:
            Bc = rhs(phi4, piv, scalar=False, cols=grad_cols)[1]
            _, Dc = pair_norms(phi4[:, :, np.asarray(grad_cols)])
            wg = w[np.asarray(grad_cols)]
        else:
            Dc, wg = Dcol, w_c
        w2 = wg * wg
        xig = np.empty(Bc.shape)
        for c in range(3):
            cf, jit[1 + c] = chol_with_jitter(Ac[c])
            xig[c] = cho_solve(cf, Bc[c])
            res[1 + c] = float(np.sum(w2 * (Dc[c] - np.einsum("mg,mg->g", xig[c], Bc[c]))))
            rel[1 + c] = res[1 + c] / float(np.sum(w2 * Dc[c]))
    return FitResult(xi, xig, jit, res, rel)
