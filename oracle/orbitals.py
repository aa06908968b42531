"""Orbital and orbital-gradient values on the grid (Alg. 2, grid step).

chi_a(r) = f_a x^i y^j z^k sum_p c_p exp(-alpha_p |r - R|^2), (x, y, z) = r - R,
phi_p(r) = sum_a chi_a(r) C[a, p]. Gradients are the analytic derivatives:
d/dx [x^i e^{-alpha r^2}] = (i x^{i-1} - 2 alpha x^{i+1}) e^{-alpha r^2}.

Pinned by: the grid quadrature of chi_a chi_b against the analytic overlap
matrix, and central finite differences of phi against grad phi.
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


def eval_orbitals(basis, C_mo: np.ndarray, xyz: np.ndarray) -> np.ndarray:
    """phi4[4, n_orb, n_g] = AO4^T C: values and Cartesian gradients of the MOs."""
    ao = eval_ao(basis, xyz)
    return np.ascontiguousarray(np.einsum("cag,ap->cpg", ao, C_mo, optimize=True))


def density(phi4: np.ndarray, n_occ: int) -> np.ndarray:
    """One-spin reference density rho_gamma(g) = sum_{i in occ} phi_i(g)^2 (xTC section,
    eq. deltaU-fields, with gamma the occupied projector)."""
    return np.einsum("pg,pg->g", phi4[0, :n_occ], phi4[0, :n_occ])
