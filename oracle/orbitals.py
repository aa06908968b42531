"""Orbital and orbital-gradient values on the grid (Alg. 2, grid step).

chi_a(r) = f_a x^i y^j z^k sum_p c_p exp(-alpha_p |r - R|^2), (x, y, z) = r - R,
phi_p(r) = sum_a chi_a(r) C[a, p]. Gradients are the analytic derivatives:
d/dx [x^i e^{-alpha r^2}] = (i x^{i-1} - 2 alpha x^{i+1}) e^{-alpha r^2}.

Laplacians (for the local energy of the variational Monte Carlo section): with
chi = f P(x, y, z) g(s), P = x^i y^j z^k of degree l, g(s) = sum_p c_p e^{-alpha_p s},
s = r^2: lap chi = f [g lap P + P (4 l g' + 6 g' + 4 s g'')] (Euler: r . grad P = l P).

Pinned by: the grid quadrature of chi_a chi_b against the analytic overlap
matrix, central finite differences of phi against grad phi, and of grad chi
against lap chi.
"""
from __future__ import annotations

import numpy as np


def eval_ao(basis, xyz: np.ndarray) -> np.ndarray:
    """AO values and gradients, [4, n_ao, n_g] (value, d/dx, d/dy, d/dz)."""
    n_g = xyz.shape[1]
    out = np.zeros((4, basis.n_ao, n_g))
    for s in range(basis.n_shell):
        R = basis.atom_xyz[basis.shell_center[s]]
        d = xyz - R[:, None]                                   # [3, n_g]
        r2 = np.einsum("ig,ig->g", d, d)
        p0, p1 = basis.shell_prim_start[s], basis.shell_prim_start[s + 1]
        rad = np.zeros(n_g)      # sum_p c e^{-a r2}
        drad = np.zeros(n_g)     # sum_p c (-2 a) e^{-a r2}
        for p in range(p0, p1):
            e = basis.prim_coef[p] * np.exp(-basis.prim_exp[p] * r2)
            rad += e
            drad += -2.0 * basis.prim_exp[p] * e
        for a in range(basis.shell_ao_start[s], basis.shell_ao_start[s + 1]):
            i, j, k = (int(v) for v in basis.ao_pow[a])
            f = basis.comp_factor[a]
            pw = [d[0] ** i, d[1] ** j, d[2] ** k]
            ang = pw[0] * pw[1] * pw[2]
            out[0, a] = f * ang * rad
            # d/dx (x^i R(r)) = i x^{i-1} R + x^i x dR/d(x) where dR/dx = x * drad
            for c, n in enumerate((i, j, k)):
                lower = n * d[c] ** (n - 1) if n > 0 else 0.0
                others = np.prod([pw[e] for e in range(3) if e != c], axis=0)
                out[1 + c, a] = f * others * (lower * rad + pw[c] * d[c] * drad)
    return out


def eval_ao_lap(basis, xyz: np.ndarray) -> np.ndarray:
    """AO values, gradients and Laplacians, [5, n_ao, n] (value, d/dx, d/dy, d/dz, lap)."""
    out = np.zeros((5, basis.n_ao, xyz.shape[1]))
    out[:4] = eval_ao(basis, xyz)
    for s in range(basis.n_shell):
        R = basis.atom_xyz[basis.shell_center[s]]
        d = xyz - R[:, None]
        r2 = np.einsum("ig,ig->g", d, d)
        g0 = np.zeros_like(r2)
        g1 = np.zeros_like(r2)       # dg/ds
        g2 = np.zeros_like(r2)       # d2g/ds2
        for p in range(basis.shell_prim_start[s], basis.shell_prim_start[s + 1]):
            a = basis.prim_exp[p]
            e = basis.prim_coef[p] * np.exp(-a * r2)
            g0 += e
            g1 -= a * e
            g2 += a * a * e
        for ao in range(basis.shell_ao_start[s], basis.shell_ao_start[s + 1]):
            i, j, k = (int(v) for v in basis.ao_pow[ao])
            l = i + j + k
            P = d[0] ** i * d[1] ** j * d[2] ** k
            lapP = np.zeros_like(r2)
            for c, n in enumerate((i, j, k)):
                if n >= 2:
                    lapP += n * (n - 1) * d[c] ** (n - 2) * np.prod(
                        [d[e] ** (i, j, k)[e] for e in range(3) if e != c], axis=0)
            out[4, ao] = basis.comp_factor[ao] * (g0 * lapP + P * (4 * l * g1 + 6 * g1 + 4 * r2 * g2))
    return out


def eval_orbitals(basis, C_mo: np.ndarray, xyz: np.ndarray) -> np.ndarray:
    """phi4[4, n_orb, n_g] = AO4^T C: values and Cartesian gradients of the MOs."""
    ao = eval_ao(basis, xyz)
    return np.ascontiguousarray(np.einsum("cag,ap->cpg", ao, C_mo, optimize=True))


def density(phi4: np.ndarray, n_occ: int) -> np.ndarray:
    """One-spin reference density rho_gamma(g) = sum_{i in occ} phi_i(g)^2 (xTC section,
    eq. deltaU-fields, with gamma the occupied projector)."""
    return np.einsum("pg,pg->g", phi4[0, :n_occ], phi4[0, :n_occ])
