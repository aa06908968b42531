"""Analytic one-electron integrals over the synthetic Cartesian Gaussian basis.

Input preparation only: they produce the molecular-orbital coefficients that the
method starts from (the paper takes Hartree-Fock orbitals from PySCF; here the
orbitals are eigenvectors of a model core Hamiltonian, see ``core_orbitals``).
Nothing here evaluates a function on the integration grid, so none of it is
shared with the grid arithmetic of the method.

1-D Gaussian moments follow the Obara-Saika recurrences:
  I(i+1, j) = X_PA I(i, j) + (i I(i-1, j) + j I(i, j-1)) / (2p)
  I(i, j+1) = X_PB I(i, j) + (i I(i-1, j) + j I(i, j-1)) / (2p)
for int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2 - c(x-C)^2) dx.
"""
from __future__ import annotations

import numpy as np

from .basis import Basis, cart_components


def _tables(a, A, b, B, c, C, imax, jmax):
    """Obara-Saika tables; batch arrays a, b, c [...], centres [..., 3].

    Returns T[d][i][j] with shape [3, imax+1, jmax+1, ...].
    """
    p = a + b + c
    P = (a[..., None] * A + b[..., None] * B + c[..., None] * C) / p[..., None]
    inv2p = 0.5 / p
    out = np.zeros((3, imax + 1, jmax + 1) + p.shape)
    for d in range(3):
        Ad, Bd, Cd = A[..., d], B[..., d], C[..., d]
        k = np.exp(-(a * b * (Ad - Bd) ** 2 + a * c * (Ad - Cd) ** 2 + b * c * (Bd - Cd) ** 2) / p)
        T = out[d]
        T[0, 0] = k * np.sqrt(np.pi / p)
        PA = P[..., d] - Ad
        PB = P[..., d] - Bd
        for i in range(imax):
            T[i + 1, 0] = PA * T[i, 0] + (inv2p * i * T[i - 1, 0] if i > 0 else 0.0)
        for j in range(jmax):
            for i in range(imax + 1):
                v = PB * T[i, j]
                if i > 0:
                    v = v + inv2p * i * T[i - 1, j]
                if j > 0:
                    v = v + inv2p * j * T[i, j - 1]
                T[i, j + 1] = v
    return out


def coulomb_gaussian_expansion(h: float = 0.45, tau_lo: float = -4.5, tau_hi: float = 4.5):
    """1/r ~= sum_t beta_t exp(-gamma_t r^2): trapezoid rule of
    1/r = (2/sqrt(pi)) int exp(tau) exp(-exp(2 tau) r^2) dtau (model potential)."""
    tau = np.arange(tau_lo, tau_hi + 1e-12, h)
    gamma = np.exp(2.0 * tau)
    beta = 2.0 * h / np.sqrt(np.pi) * np.exp(tau)
    return beta, gamma


def one_electron(basis: Basis, charges: np.ndarray, with_potential: bool = True):
    """Overlap S, kinetic T and model nuclear attraction V over the AOs."""
    n = basis.n_ao
    S = np.zeros((n, n))
    T = np.zeros((n, n))
    V = np.zeros((n, n))
    beta, gamma = coulomb_gaussian_expansion()
    R = basis.atom_xyz
    nuc_c = np.repeat(gamma[None, :], R.shape[0], 0).ravel()            # [n_atom * n_t]
    nuc_w = (charges[:, None] * beta[None, :]).ravel()
    nuc_C = np.repeat(R, gamma.shape[0], axis=0)                       # [n_atom * n_t, 3]
    shells = range(basis.n_shell)
    for sa in shells:
        la = int(basis.shell_l[sa])
        A = R[basis.shell_center[sa]]
        pa = slice(basis.shell_prim_start[sa], basis.shell_prim_start[sa + 1])
        for sb in range(sa, basis.n_shell):
            lb = int(basis.shell_l[sb])
            B = R[basis.shell_center[sb]]
            pb = slice(basis.shell_prim_start[sb], basis.shell_prim_start[sb + 1])
            blkS = np.zeros((len(cart_components(la)), len(cart_components(lb))))
            blkT = np.zeros_like(blkS)
            blkV = np.zeros_like(blkS)
            for ea, ca in zip(basis.prim_exp[pa], basis.prim_coef[pa]):
                for eb, cb in zip(basis.prim_exp[pb], basis.prim_coef[pb]):
                    one = np.ones(1)
                    tab = _tables(ea * one, A[None], eb * one, B[None], 0.0 * one, A[None], la, lb + 2)[..., 0]
                    if with_potential:
                        m = nuc_c.shape[0]
                        vt = _tables(np.full(m, ea), np.broadcast_to(A, (m, 3)),
                                     np.full(m, eb), np.broadcast_to(B, (m, 3)),
                                     nuc_c, nuc_C, la, lb)
                    for u, (ia, ja, ka) in enumerate(cart_components(la)):
                        for v, (ib, jb, kb) in enumerate(cart_components(lb)):
                            sx, sy, sz = tab[0, ia, ib], tab[1, ja, jb], tab[2, ka, kb]
                            blkS[u, v] += ca * cb * sx * sy * sz

                            def d2(t, i, j):
                                r = -2.0 * eb * (2 * j + 1) * t[i, j] + 4.0 * eb * eb * t[i, j + 2]
                                if j >= 2:
                                    r += j * (j - 1) * t[i, j - 2]
                                return r
                            lap = d2(tab[0], ia, ib) * sy * sz + sx * d2(tab[1], ja, jb) * sz + sx * sy * d2(tab[2], ka, kb)
                            blkT[u, v] += -0.5 * ca * cb * lap
                            if with_potential:
                                blkV[u, v] -= ca * cb * np.dot(nuc_w, vt[0, ia, ib] * vt[1, ja, jb] * vt[2, ka, kb])
            oa = slice(basis.shell_ao_start[sa], basis.shell_ao_start[sa + 1])
            ob = slice(basis.shell_ao_start[sb], basis.shell_ao_start[sb + 1])
            fa = basis.comp_factor[oa][:, None]
            fb = basis.comp_factor[ob][None, :]
            for M, blk in ((S, blkS), (T, blkT), (V, blkV)):
                M[oa, ob] = blk * fa * fb
                M[ob, oa] = (blk * fa * fb).T
    return S, T, V


def core_orbitals(basis: Basis, charges: np.ndarray, n_orb: int):
    """Lowest n_orb eigenvectors of the model core Hamiltonian T + V in the S metric.

    Returns (C [n_ao, n_orb], eps [n_orb], S). Column signs are fixed so that the
    largest-magnitude coefficient of every orbital is positive (deterministic).
    """
    from scipy.linalg import eigh

    S, T, V = one_electron(basis, charges)
    H = T + V
    eps, C = eigh(H, S)
    C = C[:, :n_orb]
    eps = eps[:n_orb]
    idx = np.argmax(np.abs(C), axis=0)
    sgn = np.sign(C[idx, np.arange(C.shape[1])])
    sgn[sgn == 0] = 1.0
    return np.ascontiguousarray(C * sgn[None, :]), eps, S
