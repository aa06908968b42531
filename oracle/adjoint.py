"""Derivatives of the contracted outputs with respect to the linear correlator
coefficients c (every parameter of eq. bh-u that enters linearly).

The scalar is L = sum_c <Lu1_c, u1_c> + <Lu3, u3> + <Lul, ulap> + <LD1, D1>
+ <LD4, D4> + <Lf, field> for given cotangents (any may be absent). This
oracle differentiates the definitions in forward mode, one coefficient at a
time: the kernels are linear in c (grad u, lap u) or quadratic (|grad u|^2,
through d|grad u|^2/dc_j = 2 B(e_j, c), B the symmetric bilinear form of the
squared channel, i.e. 2 grad u_j . grad u away from coincident pairs, with u_j
the correlator with c = e_j), and D4, D1 are quadratic in calG, so
  dD4/dc_j = sum_g wt_g sum_c (calG_j^c calG^c^T + calG^c calG_j^c^T),
  dV/dc_j  = sum_c (H_j,c calG^c + H_c calG_j^c).
Pinned by: central finite differences, which are exact up to rounding here
because every output is a polynomial of degree <= 2 in c.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from threadpoolctl import threadpool_limits

from .correlator import pair_kernels, sq_bilinear


def _unit(corr, j):
    c = np.zeros(corr.c.size)
    c[j] = 1.0
    return corr.with_c(c)


def dL_dc(xyz, w, corr, xi, xigrad, G, rho, cot: dict, bra_block: int = 128, ket_block: int = 2048,
          bra_range=None, params=None):
    """dL/dc_j for j in params (default every coefficient). bra_range = (start, stop): the
    outputs are the partial sums over those bra points (the ket sums cover the whole grid)."""
    n_mu, n_g = xi.shape
    lo, hi = (0, n_g) if bra_range is None else bra_range
    wxi = xi * w[None, :]
    wrho = w * rho
    lap = cot.get("ulap") is not None
    need_calG = any(cot.get(k) is not None for k in ("u1", "D1", "D4"))
    units = [_unit(corr, j) for j in (range(corr.c.size) if params is None else params)]

    def block(b0):
        b1 = min(hi, b0 + bra_block)
        nb = b1 - b0
        P = len(units)
        calG = np.zeros((3, n_mu, nb))
        dcalG = np.zeros((P, 3, n_mu, nb))
        dT3 = np.zeros((P, n_mu, nb))
        dTL = np.zeros((P, n_mu, nb)) if lap else None
        dfld = np.zeros((P, 3, nb))
        for k0 in range(0, n_g, ket_block):
            k1 = min(n_g, k0 + ket_block)
            K = pair_kernels(corr, xyz[:, b0:b1], xyz[:, k0:k1])
            if need_calG:
                for c, key in enumerate(("gx", "gy", "gz")):
                    calG[c] += wxi[:, k0:k1] @ K[key].T
            for j, cj in enumerate(units):
                Kj = pair_kernels(cj, xyz[:, b0:b1], xyz[:, k0:k1], want_lap=lap)
                dot = sq_bilinear(cj, corr, xyz[:, b0:b1], xyz[:, k0:k1])
                for c, key in enumerate(("gx", "gy", "gz")):
                    dcalG[j, c] += wxi[:, k0:k1] @ Kj[key].T
                    dfld[j, c] += Kj[key] @ wrho[k0:k1]
                dT3[j] += wxi[:, k0:k1] @ (2.0 * dot).T
                if lap:
                    dTL[j] += wxi[:, k0:k1] @ Kj["lap"].T
        return calG, dcalG, dT3, dTL, dfld

    starts = list(range(lo, hi, bra_block))
    grad = np.zeros(len(units))
    workers = max(1, min(len(starts), int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))))
    with threadpool_limits(1 if workers > 1 else None), ThreadPoolExecutor(workers) as ex:
        for b0, (calG, dcalG, dT3, dTL, dfld) in zip(starts, ex.map(block, starts)):
            b1 = min(hi, b0 + bra_block)
            wb = w[b0:b1]
            wt = wb * (G @ xi[:, b0:b1])
            H = np.einsum("l,clg->gc", G, calG)
            for j in range(len(units)):
                s = 0.0
                if cot.get("u1") is not None:
                    for c in range(3):
                        du1 = (xigrad[c][:, b0:b1] * wb[None, :]) @ dcalG[j, c].T
                        s += np.sum(cot["u1"][c] * du1)
                if cot.get("u3") is not None:
                    s += np.sum(cot["u3"] * (wxi[:, b0:b1] @ dT3[j].T))
                if lap:
                    s += np.sum(cot["ulap"] * (wxi[:, b0:b1] @ dTL[j].T))
                if cot.get("D4") is not None:
                    dD4 = np.zeros((n_mu, n_mu))
                    for c in range(3):
                        dD4 += (dcalG[j, c] * wt[None, :]) @ calG[c].T
                        dD4 += (calG[c] * wt[None, :]) @ dcalG[j, c].T
                    s += np.sum(cot["D4"] * dD4)
                if cot.get("D1") is not None:
                    Hj = np.einsum("l,clg->gc", G, dcalG[j])
                    dV = np.einsum("gc,cng->ng", Hj, calG) + np.einsum("gc,cng->ng", H, dcalG[j])
                    s += np.sum(cot["D1"] * (wxi[:, b0:b1] @ dV.T))
                if cot.get("field") is not None:
                    s += np.sum(cot["field"][:, b0:b1] * dfld[j])
                grad[j] += s
    return grad


def loss(out: dict, cot: dict) -> complex:
    """L = sum over the cotangent keys of <cot[k], out[k]>."""
    return sum(np.sum(cot[k] * out[k]) for k in ("u1", "u3", "ulap", "D1", "D4", "field")
               if cot.get(k) is not None)


def dL_dnl(xyz, w, corr, xi, xigrad, G, rho, cot: dict, h: float = 1e-30):
    """Derivatives of L with respect to the nonlinear correlator parameters, by the complex
    step: L(p + i h) = L(p) + i h L'(p) - h^2 L''(p)/2 + ..., so L'(p) = Im L(p + i h) / h
    with no subtractive cancellation; the contraction is carried in complex arithmetic.
    Returns [dL/dd] for the EE form (rbar = d r / (1 + d r)) and
    [dL/dd, dL/db_0, ..., dL/db_{n_types - 1}] for the BH form (a_I = b r_I / (1 + b r_I))."""
    from dataclasses import replace

    from .contract import contract
    ch = 0
    for k, bit in (("u1", 1), ("u3", 2), ("ulap", 4), ("D1", 8), ("D4", 16), ("field", 32)):
        if cot.get(k) is not None:
            ch |= bit

    def step(c):
        out = contract(xyz, w, c, xi, xigrad, G, rho, ch)
        return float(np.imag(loss(out, cot)) / h)

    res = [step(replace(corr, d=corr.d + 1j * h))]
    if corr.form != 0:
        for t in range(len(corr.b)):
            b = np.asarray(corr.b, dtype=complex).copy()
            b[t] += 1j * h
            res.append(step(replace(corr, b=b)))
    return np.array(res)


def dL_dd(xyz, w, corr, xi, xigrad, G, rho, cot: dict, h: float = 1e-30):
    """dL/dd alone (dL_dnl's first entry)."""
    from dataclasses import replace

    from .contract import contract
    ch = 0
    for k, bit in (("u1", 1), ("u3", 2), ("ulap", 4), ("D1", 8), ("D4", 16), ("field", 32)):
        if cot.get(k) is not None:
            ch |= bit
    out = contract(xyz, w, replace(corr, d=corr.d + 1j * h), xi, xigrad, G, rho, ch)
    return float(np.imag(loss(out, cot)) / h)
