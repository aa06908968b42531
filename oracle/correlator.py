"""Correlators and their analytic derivatives (Jastrow correlator section,
eqs. bh-scaled and bh-u; the K-kernel section fixes that the gradient acts on
electron 1, i.e. on the bra point).

Two forms are supported.
  EE: u(r1, r2) = sum_k c_k rbar^{o_k}, rbar = d r / (1 + d r), r = |r1 - r2|
      (the electron-electron part of eq. bh-u without the nuclear sum; the
      workloads' correlator uses o_k = 2k, d = 1).
  BH: u = sum_I sum_k c_k^{type(I)} [a_1I^m a_2I^n + a_2I^m a_1I^n] e^o with
      a_iI = b r_iI / (1 + b r_iI) and e = rbar_12 (eq. bh-u, taken literally,
      so (0,0,o) terms carry the factor 2 N_nuc).

Derivatives, with t = 1/(1 + d r): d rbar/dr = d t^2, d^2 rbar/dr^2 = -2 d^2 t^3;
  u'(r) = sum c o rbar^{o-1} d t^2,
  grad_1 u = (u'/r) (r1 - r2), |grad_1 u|^2 = u'^2, lap_1 u = u'' + 2 u'/r.
For o >= 2, u'/r = sum c o d^2 t^3 rbar^{o-2} is regular at r = 0.

Reading for coincident pairs (r12 = 0), where odd powers o make the direction
of grad_1 rbar^o undefined: the vector channel drops the r12-direction part,
the squared channel keeps |N|^2 + S^2 (N the nuclear part, S the radial
electron-electron derivative), and the Laplacian drops odd-o terms.

Pinned by: closed forms at r = 0, symmetry u(1,2) = u(2,1), antisymmetry of
grad_1 u for EE, and central finite differences of u against grad_1 u and of
grad_1 u against the Laplacian.
"""
from __future__ import annotations

import numpy as np

FORM_EE = 0
FORM_BH = 1


def _diff(X1, X2):
    D = X1[:, :, None] - X2[:, None, :]            # [3, b, k], formed in FP64
    r = np.sqrt(np.einsum("ibk,ibk->bk", D, D))
    return D, r


def u_value(corr, X1, X2):
    """u(g, g') for bra points X1 [3, b] and ket points X2 [3, k]."""
    D, r = _diff(X1, X2)
    d = corr.d
    e = d * r / (1.0 + d * r)
    if corr.form == FORM_EE:
        out = np.zeros_like(r)
        for k in range(corr.n_terms):
            out += corr.c[0, k] * e ** int(corr.mno[k, 2])
        return out
    out = np.zeros_like(r)
    for I in range(corr.nuc_xyz.shape[0]):
        ty = int(corr.nuc_type[I])
        b = corr.b[ty]
        R = corr.nuc_xyz[I]
        r1 = np.linalg.norm(X1 - R[:, None], axis=0)
        r2 = np.linalg.norm(X2 - R[:, None], axis=0)
        a1 = (b * r1 / (1.0 + b * r1))[:, None]
        a2 = (b * r2 / (1.0 + b * r2))[None, :]
        for k in range(corr.n_terms):
            m, n, o = (int(v) for v in corr.mno[k])
            out += corr.c[ty, k] * (a1 ** m * a2 ** n + a2 ** m * a1 ** n) * e ** o
    return out


def _poly(coef, x):
    """sum_j coef[j] x^j by Horner's rule."""
    out = np.full_like(x, coef[-1])
    for cj in coef[-2::-1]:
        out = out * x + cj
    return out


def _ee(corr, D, r, want_lap):
    d = corr.d
    t = 1.0 / (1.0 + d * r)
    e = d * r * t
    o = corr.mno[:, 2].astype(int)
    c = corr.c[0]
    omax = int(o.max())
    # u' = d t^2 sum c o e^{o-1};  (u'/r)_{o>=2} = d^2 t^3 sum c o e^{o-2};
    # u'' = d^2 t^4 sum c o (o-1) e^{o-2} - 2 d^2 t^3 sum c o e^{o-1}
    p1 = np.zeros(max(omax, 1))
    p2 = np.zeros(max(omax - 1, 1))
    p3 = np.zeros(max(omax - 1, 1))
    c1 = 0.0                           # coefficient of the o = 1 terms
    for ck, ok in zip(c, o):
        if ok >= 1:
            p1[ok - 1] += ck * ok
        if ok >= 2:
            p2[ok - 2] += ck * ok
            p3[ok - 2] += ck * ok * (ok - 1)
        if ok == 1:
            c1 += ck
    t2 = t * t
    t3 = t2 * t
    up = d * t2 * _poly(p1, e)
    f = d * d * t3 * _poly(p2, e) if omax >= 2 else np.zeros_like(r)
    upp = d * d * t2 * t2 * _poly(p3, e) if omax >= 2 else np.zeros_like(r)
    upp = upp - 2.0 * d * d * t3 * _poly(p1, e)
    if c1 != 0.0:
        zero = r == 0.0
        rs = np.where(zero, 1.0, r)
        f = f + np.where(zero, 0.0, c1 * d * t2 / rs)
        upp = np.where(zero, upp + 2.0 * d * d * t3 * c1, upp)   # drop the o = 1 term at r = 0
    zero = r == 0.0
    rhat = np.where(zero[None], 0.0, D / np.where(zero, 1.0, r)[None])
    out = {"gx": f * D[0], "gy": f * D[1], "gz": f * D[2], "sq": up * up,
           "_N": np.zeros_like(D), "_S": up, "_rhat": rhat}
    if want_lap:
        out["lap"] = upp + 2.0 * f
    return out


def _bh(corr, X1, X2, D, r):
    d = corr.d
    t = 1.0 / (1.0 + d * r)
    e = d * r * t
    zero = r == 0.0
    rs = np.where(zero, 1.0, r)
    # sums take the type of d and b: a complex step in either is carried through
    dt = np.result_type(float, d, np.asarray(corr.b))
    N = np.zeros((3,) + r.shape, dt)
    S = np.zeros(r.shape, dt)
    for I in range(corr.nuc_xyz.shape[0]):
        ty = int(corr.nuc_type[I])
        b = corr.b[ty]
        R = corr.nuc_xyz[I]
        v1 = X1 - R[:, None]
        r1 = np.linalg.norm(v1, axis=0)
        r2 = np.linalg.norm(X2 - R[:, None], axis=0)
        t1 = 1.0 / (1.0 + b * r1)
        a1 = (b * r1 * t1)[:, None]
        a2 = (b * r2 / (1.0 + b * r2))[None, :]
        da1 = (b * t1 * t1 / r1)[None, :, None] * v1[:, :, None]    # grad_1 a_1I  [3, b, 1]
        for k in range(corr.n_terms):
            m, n, o = (int(v) for v in corr.mno[k])
            c = corr.c[ty, k]
            P = a1 ** m * a2 ** n + a2 ** m * a1 ** n
            dP = (m * a1 ** max(m - 1, 0) * a2 ** n if m > 0 else 0.0) + \
                 (n * a2 ** m * a1 ** max(n - 1, 0) if n > 0 else 0.0)
            eo = e ** o
            N += c * dP * eo * da1
            if o >= 1:
                S += c * P * o * e ** (o - 1) * d * t * t
    rhat = np.where(zero[None], 0.0, D / rs[None])
    G = N + S[None] * rhat
    sq = np.where(zero, np.einsum("ibk,ibk->bk", N, N) + S * S, np.einsum("ibk,ibk->bk", G, G))
    return {"gx": G[0], "gy": G[1], "gz": G[2], "sq": sq, "_N": N, "_S": S, "_rhat": rhat}


def pair_kernels(corr, X1, X2, want_lap: bool = False):
    """Grid-pair kernel channels for bra X1 [3, b] and ket X2 [3, k]:
    gx, gy, gz = grad_1 u; sq = |grad_1 u|^2; lap = lap_1 u (EE only)."""
    D, r = _diff(X1, X2)
    if corr.form == FORM_EE:
        return _ee(corr, D, r, want_lap)
    if want_lap:
        raise NotImplementedError("Laplacian channel is defined for the EE form only")
    return _bh(corr, X1, X2, D, r)


def sq_bilinear(corr_a, corr_b, X1, X2):
    """Symmetric bilinear form B(a, b) with B(c, c) = |grad_1 u_c|^2 (the squared
    channel, including the coincident-pair reading): with grad_1 u = N + S rhat,
    B = N_a . N_b + S_a S_b + (S_b N_a + S_a N_b) . rhat, rhat = 0 at r12 = 0."""
    Ka = pair_kernels(corr_a, X1, X2)
    Kb = pair_kernels(corr_b, X1, X2)
    Na, Nb, Sa, Sb, rh = Ka["_N"], Kb["_N"], Ka["_S"], Kb["_S"], Ka["_rhat"]
    return (np.einsum("ibk,ibk->bk", Na, Nb) + Sa * Sb
            + np.einsum("ibk,ibk->bk", Sb[None] * Na + Sa[None] * Nb, rh))
