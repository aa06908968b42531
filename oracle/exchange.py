"""xTC Terms 2 and 3: the exchange-kernel intermediates X2 and X3 (xTC section,
"Terms 2 and 3 (non-factorizable)" and "Low-rank projector for Terms 2 and 3";
pre-ISDF forms in eq. deltaU-preisdf with the fields of eq. deltaU-fields).

Test infrastructure: plain FP64 NumPy, sharing no code with the GPU library.

Notation. Pivots r_nu; orbitals phi_p; pivot tensor C^p_q(nu) = phi_p(r_nu) phi_q(r_nu);
gamma^u_t the one-spin reference density in the MO basis; L^u_{s nu} =
sum_t gamma^u_t C^t_s(nu); calG^c_{mu,g} = sum_g' w_g' xi_mu(g') d_c u(g, g').

Direct form, literally as written in the paper:
  Y^u_{s,g,c} = sum_nu L^u_{s nu} calG^c_{nu,g}      Z^q_{u,g,c} = sum_nu C^q_u(nu) calG^c_{nu,g}
  Lt^u_{s,g}  = sum_nu L^u_{s nu} xi_nu(g)           Ch^q_{u,g}  = sum_nu C^q_u(nu) xi_nu(g)
  X2_{qs mu}  = sum_g w_g xi_mu(g) sum_{u,c} Y^u_{s,g,c} Z^q_{u,g,c}
  X31_{qs mu} = sum_{g,c} w_g calG^c_{mu,g} sum_u Lt^u_{s,g} Z^q_{u,g,c}
  X32_{qs mu} = sum_{g,c} w_g calG^c_{mu,g} sum_u Y^u_{s,g,c} Ch^q_{u,g}
  X3 = X31 + X32.
Projector form: with gamma = L_Q L_Q^T, sum_u L^u_{s nu} C^q_u(lambda) = sum_a P_{s nu,a} P_{q lambda,a},
P_{s nu,a} = sum_t C^t_s(nu) (L_Q)_{t a}. With R^c_{s a}(g) = sum_nu P_{s nu,a} calG^c_{nu,g} and
Q_{s a}(g) = sum_nu P_{s nu,a} xi_nu(g):
  X2_{qs mu} = sum_g w_g xi_mu(g) sum_{a,c} R^c_{s a}(g) R^c_{q a}(g)
  X3_{qs mu} = sum_{g,c} w_g calG^c_{mu,g} sum_a [Q_{s a}(g) R^c_{q a}(g) + R^c_{s a}(g) Q_{q a}(g)]
Both are symmetric in (q, s). The terms are Term2^{pq}_{rs} = -sum_mu C^p_r(mu) X2_{qs mu} and
Term3^{pq}_{rs} = -sum_mu C^p_r(mu) X3_{qs mu}.

Pinned by: the direct and projector forms agreeing; the (q, s) symmetry; the full-rank ISDF
Terms 2 and 3 equal to the pre-ISDF four-index brute force (fourindex.direct); quadratic
scaling in the correlator coefficients.
"""
from __future__ import annotations

import numpy as np

from .correlator import pair_kernels


def occupied_gamma(n_orb: int, n_occ: int) -> np.ndarray:
    """One-spin reference density of the closed-shell reference in the MO basis."""
    g = np.zeros((n_orb, n_orb))
    g[np.arange(n_occ), np.arange(n_occ)] = 1.0
    return g


def density_projector(gamma: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """L_Q with gamma = L_Q L_Q^T (gamma symmetric positive semidefinite)."""
    lam, V = np.linalg.eigh(gamma)
    keep = lam > tol * max(1.0, lam.max())
    return V[:, keep] * np.sqrt(lam[keep])[None, :]


def calG(xyz, w, corr, xi, bra_block: int = 256, bra=None):
    """calG[c, mu, g] = sum_g' w_g' xi_mu(g') d_c u(g, g') (bra-blocked); with bra = (b, e)
    only the bra points b <= g < e (columns g - b), the ket sum still over the whole grid."""
    n_mu, n_g = xi.shape
    lo, hi = (0, n_g) if bra is None else bra
    wxi = xi * w[None, :]
    out = np.zeros((3, n_mu, hi - lo))
    for b0 in range(lo, hi, bra_block):
        b1 = min(hi, b0 + bra_block)
        K = pair_kernels(corr, xyz[:, b0:b1], xyz)
        for c, key in enumerate(("gx", "gy", "gz")):
            out[c, :, b0 - lo:b1 - lo] = wxi @ K[key].T
    return out


def pivot_tensor(phi, piv):
    Pm = phi[:, piv]
    return np.einsum("pm,qm->pqm", Pm, Pm)


def x_terms_direct(phi, piv, xi, cG, w, gamma):
    """X2, X3 (and X31, X32) from the literal definitions. phi [n_orb, n_g]. Small inputs."""
    C = pivot_tensor(phi, piv)                                # C[p, q, nu]
    L = np.einsum("ut,tsn->usn", gamma, C)                    # L[u, s, nu]
    Y = np.einsum("usn,cng->usgc", L, cG, optimize=True)      # Y[u, s, g, c]
    Z = np.einsum("qun,cng->qugc", C, cG, optimize=True)      # Z[q, u, g, c]
    Lt = np.einsum("usn,ng->usg", L, xi)
    Ch = np.einsum("qun,ng->qug", C, xi)
    X2 = np.einsum("g,mg,usgc,qugc->qsm", w, xi, Y, Z, optimize=True)
    X31 = np.einsum("g,cmg,usg,qugc->qsm", w, cG, Lt, Z, optimize=True)
    X32 = np.einsum("g,cmg,usgc,qug->qsm", w, cG, Y, Ch, optimize=True)
    return dict(X2=X2, X31=X31, X32=X32, X3=X31 + X32)


def x_terms(phi, piv, xi, cG, w, LQ):
    """X2, X3 through the low-rank projector: the formulas of the module docstring as
    einsums over P, R^c and Q, each bracketed sum taken in turn (the inner sum over the
    projector index a and channel c at every grid point, then the grid sum)."""
    C = pivot_tensor(phi, piv)                                          # C[t, s, nu]
    P = np.einsum("tsn,ta->san", C, LQ)                                 # P[s, a, nu]
    R = np.einsum("san,cng->cgsa", P, cG, optimize=True)                # R^c[s, a](g)
    Q = np.einsum("san,ng->gsa", P, xi, optimize=True)                  # Q[s, a](g)
    # inner sums at each grid point
    T2 = np.einsum("cgsa,cgqa->gqs", R, R)                              # sum_{a,c} R^c_s R^c_q
    T3 = np.einsum("gsa,cgqa->cgqs", Q, R) + np.einsum("cgsa,gqa->cgqs", R, Q)
    # grid sums
    X2 = np.einsum("g,mg,gqs->qsm", w, xi, T2, optimize=True)
    X3 = np.einsum("g,cmg,cgqs->qsm", w, cG, T3, optimize=True)
    return dict(X2=X2, X3=X3)


def terms23_isdf(phi, piv, X2, X3):
    """Term2, Term3 [p, q, r, s] from the intermediates."""
    C = pivot_tensor(phi, piv)
    return dict(T2=-np.einsum("prm,qsm->pqrs", C, X2, optimize=True),
                T3=-np.einsum("prm,qsm->pqrs", C, X3, optimize=True))
