"""Grid-pair kernels and xTC D terms (K-kernel section, eqs. K1-isdf and
K3-isdf; xTC section, eqs. deltaU-fields and deltaU-isdf-map, Terms 1 and 4).

For bra points g and ket points g' (grad acting on the bra point):
  calG^c_{mu,g} = sum_g' w_g' xi_mu(g') d_c u(g, g')                (c = x, y, z)
  T3_{mu,g}     = sum_g' w_g' xi_mu(g') |grad u(g, g')|^2
  TL_{mu,g}     = sum_g' w_g' xi_mu(g') lap u(g, g')
  u1^c_{mu,nu}  = sum_g w_g xi~^c_mu(g) calG^c_{nu,g}
                = sum_{g,g'} w_g w_g' xi~^c_mu(g) xi_nu(g') d_c u(g, g')
  u3_{mu,nu}    = sum_g w_g xi_mu(g) T3_{nu,g},  ulap likewise with TL
  wt_g          = w_g sum_lambda G_lambda xi_lambda(g)
  H_{g,c}       = sum_lambda G_lambda calG^c_{lambda,g}
  V_{nu,g}      = sum_c H_{g,c} calG^c_{nu,g}
  D4_{mu,nu}    = sum_g wt_g sum_c calG^c_{mu,g} calG^c_{nu,g}
  D1_{mu,nu}    = sum_g w_g xi_mu(g) V_{nu,g}
  field^c(g)    = A_gamma(g) = sum_g' w_g' rho_gamma(g') d_c u(g, g')     (exact, no ISDF)
Energy-scale scalars (FP64):
  E3 = G^T u3 G, E4 = G^T D4 G, E1 = 2 G^T D1 G and their ISDF-free counterparts
  E3x = sum_{g,g'} w w' rho rho' |grad u|^2, E4x = sum_g w rho |A_gamma|^2, E1x = 2 E4x.
G_nu = sum_tu C^t_u(r_nu) gamma^u_t equals rho_gamma(r_nu) for the occupied projector.

Order of work: stage 1 (sum over ket g' for a block of bra points), then
stage 2 (sum over bra g). The brute-force pin in the tests contracts in the
opposite order over a dense kernel.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from threadpoolctl import threadpool_limits

from .correlator import pair_kernels

U1, U3, ULAP, D1, D4, FIELD, ESCALE = 1, 2, 4, 8, 16, 32, 64


def contract(xyz, w, corr, xi, xigrad, G, rho, channels: int,
             bra_block: int = 128, ket_block: int = 2048, bra_range=None):
    """All outputs of the docstring above. bra_range = (start, stop) restricts the
    sum over bra points g to that range (used to time a sample of the work)."""
    n_mu, n_g = xi.shape
    # accumulators take the type of the correlator's d and b: a complex value carries a
    # complex step through every sum (the derivatives in d and b, see adjoint.dL_dnl)
    dt = np.result_type(float, corr.d, np.asarray(corr.b if corr.b is not None else 0.0))
    lap = bool(channels & ULAP)
    need_g = bool(channels & (U1 | D1 | D4))
    wxi = xi * w[None, :]
    wrho = w * rho
    out = {}
    u1 = np.zeros((3, n_mu, n_mu), dt) if channels & U1 else None
    u3 = np.zeros((n_mu, n_mu), dt) if channels & U3 else None
    ul = np.zeros((n_mu, n_mu), dt) if lap else None
    d1 = np.zeros((n_mu, n_mu), dt) if channels & D1 else None
    d4 = np.zeros((n_mu, n_mu), dt) if channels & D4 else None
    field = np.zeros((3, n_g), dt)
    t3rho = np.zeros(n_g, dt)
    def stage1(b0):
        """Stage 1 for one bra block: sums over every ket point."""
        b1 = min(hi, b0 + bra_block)
        nb = b1 - b0
        calG = np.zeros((3, n_mu, nb), dt)
        T3 = np.zeros((n_mu, nb), dt)
        TL = np.zeros((n_mu, nb), dt) if lap else None
        fld = np.zeros((3, nb), dt)
        t3r = np.zeros(nb, dt)
        for k0 in range(0, n_g, ket_block):
            k1 = min(n_g, k0 + ket_block)
            K = pair_kernels(corr, xyz[:, b0:b1], xyz[:, k0:k1], want_lap=lap)
            for c, key in enumerate(("gx", "gy", "gz")):
                calG[c] += wxi[:, k0:k1] @ K[key].T
                fld[c] += K[key] @ wrho[k0:k1]
            T3 += wxi[:, k0:k1] @ K["sq"].T
            t3r += K["sq"] @ wrho[k0:k1]
            if lap:
                TL += wxi[:, k0:k1] @ K["lap"].T
        return calG, T3, TL, fld, t3r

    lo, hi = (0, n_g) if bra_range is None else bra_range
    starts = list(range(lo, hi, bra_block))
    workers = max(1, min(len(starts), int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))))
    # one BLAS thread per worker: the workers already use every core
    with threadpool_limits(1 if workers > 1 else None), ThreadPoolExecutor(workers) as ex:
        # blocks are consumed in bra order, so every sum below has a fixed order
        for b0, (calG, T3, TL, fld, t3r) in zip(starts, ex.map(stage1, starts)):
            b1 = min(hi, b0 + bra_block)
            field[:, b0:b1] = fld
            t3rho[b0:b1] = t3r
            wb = w[b0:b1]
            if u1 is not None:
                for c in range(3):
                    u1[c] += (xigrad[c][:, b0:b1] * wb[None, :]) @ calG[c].T
            if u3 is not None:
                u3 += wxi[:, b0:b1] @ T3.T
            if ul is not None:
                ul += wxi[:, b0:b1] @ TL.T
            if d1 is not None or d4 is not None:
                wt = wb * (G @ xi[:, b0:b1])
                H = np.einsum("l,clg->gc", G, calG)
                if d4 is not None:
                    for c in range(3):
                        d4 += (calG[c] * wt[None, :]) @ calG[c].T
                if d1 is not None:
                    V = np.einsum("gc,cng->ng", H, calG)
                    d1 += wxi[:, b0:b1] @ V.T
    out.update(u1=u1, u3=u3, ulap=ul, D1=d1, D4=d4)
    if channels & FIELD:
        out["field"] = field
    if channels & ESCALE:
        e = np.zeros(6, dt)
        if u3 is not None:
            e[0] = G @ u3 @ G
        if d4 is not None:
            e[1] = G @ d4 @ G
        if d1 is not None:
            e[2] = 2.0 * (G @ d1 @ G)
        e[3] = np.dot(wrho, t3rho)
        e[4] = np.dot(wrho, np.einsum("cg,cg->g", field, field))
        e[5] = 2.0 * e[4]
        out["escale"] = e
    return out
