"""Four-index brute force on tiny inputs (K-kernel section, eqs. K1-isdf and
K3-isdf; xTC section, eqs. deltaU-fields and deltaU-preisdf, Terms 1 to 4).

Direct grid forms (no ISDF):
  K1^{pq}_{rs} = sum_{g,g'} w w' phi_p(g) grad phi_r(g) . grad_1 u(g,g') phi_q(g') phi_s(g')
  K3^{pq}_{rs} = sum_{g,g'} w w' phi_p phi_r(g) |grad_1 u(g,g')|^2 phi_q phi_s(g')
  Term4 = sum_g w rho_gamma A^p_r . A^q_s,  Term1 = 2 sum_g w rho^p_r A_gamma . A^q_s,
  Term2 = -sum_g w rho^p_r sum_u B^u_s . A^q_u,
  Term3 = -sum_g w A^p_r . sum_u [beta^u_s A^q_u + B^u_s rho^q_u],
  A^a_b(g) = sum_g' w' rho^a_b(g') grad_1 u(g, g'), beta^u_s = sum_t gamma^u_t rho^t_s,
  B^u_s(g) = sum_g' w' beta^u_s(g') grad_1 u(g, g'), gamma the occupied projector.
ISDF forms: K1 = sum_{mu nu} u1_{mu nu} . C~^p_r(mu) C^q_s(nu), K3 = sum u3 C C,
  Term4 = sum C D4 C, Term1 = 2 sum C D1 C.
At full pair rank the two agree up to rounding (the low-rank argument of the
ISDF section). Only for tiny inputs: the dense pair kernel is materialised.
"""
from __future__ import annotations

import numpy as np

from .correlator import pair_kernels


def dense_kernels(corr, xyz):
    K = pair_kernels(corr, xyz, xyz)
    return np.stack([K["gx"], K["gy"], K["gz"]]), K["sq"]


def direct(phi4, w, corr, xyz, n_occ):
    Kv, Ks = dense_kernels(corr, xyz)
    phi = phi4[0]
    rho_pr = np.einsum("pg,rg->prg", phi, phi)
    grad_pr = np.einsum("pg,crg->cprg", phi, phi4[1:4])
    ww = w[:, None] * w[None, :]
    K1 = np.einsum("cprg,cgh,gh,qsh->pqrs", grad_pr, Kv, ww, rho_pr, optimize=True)
    K3 = np.einsum("prg,gh,gh,qsh->pqrs", rho_pr, Ks, ww, rho_pr, optimize=True)
    rho = np.einsum("pg,pg->g", phi[:n_occ], phi[:n_occ])
    A = np.einsum("cgh,h,abh->cabg", Kv, w, rho_pr, optimize=True)      # A^a_b(g)
    Ag = np.einsum("cgh,h->cg", Kv, w * rho)
    T4 = np.einsum("g,cprg,cqsg->pqrs", w * rho, A, A, optimize=True)
    T1 = 2.0 * np.einsum("g,prg,cg,cqsg->pqrs", w, rho_pr, Ag, A, optimize=True)
    gam = np.zeros((phi.shape[0], phi.shape[0]))
    gam[np.arange(n_occ), np.arange(n_occ)] = 1.0
    beta = np.einsum("ut,tsg->usg", gam, rho_pr)                       # beta^u_s(g)
    B = np.einsum("cgh,h,ush->cusg", Kv, w, beta, optimize=True)       # B^u_s(g)
    T2 = -np.einsum("g,prg,cusg,cqug->pqrs", w, rho_pr, B, A, optimize=True)
    T3 = -(np.einsum("g,cprg,usg,cqug->pqrs", w, A, beta, A, optimize=True)
           + np.einsum("g,cprg,cusg,qug->pqrs", w, A, B, rho_pr, optimize=True))
    return dict(K1=K1, K3=K3, T1=T1, T2=T2, T3=T3, T4=T4)


def isdf(phi4, piv, u1, u3, D1, D4):
    Pm = phi4[:, :, piv]
    C = np.einsum("pm,rm->prm", Pm[0], Pm[0])
    Ct = np.einsum("pm,crm->cprm", Pm[0], Pm[1:4])
    K1 = np.einsum("cmn,cprm,qsn->pqrs", u1, Ct, C, optimize=True)
    K3 = np.einsum("mn,prm,qsn->pqrs", u3, C, C, optimize=True)
    T4 = np.einsum("mn,prm,qsn->pqrs", D4, C, C, optimize=True)
    T1 = 2.0 * np.einsum("mn,prm,qsn->pqrs", D1, C, C, optimize=True)
    return dict(K1=K1, K3=K3, T1=T1, T4=T4)


def p12(T):
    """Electron-1 <-> 2 exchange P12 T^{pq}_{rs} = T^{pq}_{rs} + T^{qp}_{sr}."""
    return T + T.transpose(1, 0, 3, 2)
