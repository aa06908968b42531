"""Four-index assembly of the transcorrelated two-body corrections and the xTC one-body
pieces from the ISDF intermediates.

Test infrastructure: plain FP64 NumPy on full four-index arrays (tiny inputs only),
sharing no code with the GPU library. Index convention: T[p, q, r, s] = T^{pq}_{rs}
(physicists' order: (p, r) is electron 1's bra-ket pair, (q, s) electron 2's).

  K-kernel section, eq. K-recombine-final:
    K = 1/2 P12 [K1 - K1swap + K3],  K1swap^{pq}_{rs} = K1^{rs}_{pq},
    K1^{pq}_{rs} = sum_{mu nu c} u1^c_{mu nu} C~^{p,c}_r(mu) C^q_s(nu)      (eq. K1-isdf)
    K3^{pq}_{rs} = sum_{mu nu} u3_{mu nu} C^p_r(mu) C^q_s(nu)               (eq. K3-isdf)
    with C^p_r(mu) = phi_p phi_r (r_mu), C~^{p,c}_r(mu) = phi_p d_c phi_r (r_mu),
    P12 T^{pq}_{rs} = T^{pq}_{rs} + T^{qp}_{sr}.
  xTC section, eq. delta-u-dx-kernels and the final assembly:
    D = D4 + 2 D1, X = X2 + X3,
    dU^{pq}_{rs} = -P12 [ sum_{mu nu} C^p_r(mu) D_{mu nu} C^q_s(nu) - sum_mu C^p_r(mu) X_{qs mu} ].
  Hamiltonian assembly section:
    W = -K + dU                                                    (effective two-body correction)
    dh_{pq} = -1/2 sum_{o in occ} (2 dU^{po}_{qo} - dU^{po}_{oq})  (eq. xtc-deltah)
    f_{pq}  = dh_{pq} + sum_{i in occ} (2 W^{pi}_{qi} - W^{pi}_{iq})  (eq. xtc-fock)
    E0      = -2/3 sum_{i in occ} dh_{ii} + E_nuc                 (eq. xtc-const)

Pinned by: the full-rank ISDF K and dU equal to the pre-ISDF four-index brute force
(fourindex.direct); the P12 exchange symmetry; the one-body contractions of an outer-
product tensor in closed matrix form.
"""
from __future__ import annotations

import numpy as np


def p12(T):
    """Electron-1 <-> 2 exchange: T^{pq}_{rs} + T^{qp}_{sr}."""
    return T + T.transpose(1, 0, 3, 2)


def pivot_factors(phi4, piv):
    """C[p, r, mu] = phi_p phi_r (r_mu); Ct[c, p, r, mu] = phi_p d_c phi_r (r_mu)."""
    Pm = phi4[:, :, piv]
    C = np.einsum("pm,rm->prm", Pm[0], Pm[0])
    Ct = np.einsum("pm,crm->cprm", Pm[0], Pm[1:4])
    return C, Ct


def k_tensor(phi4, piv, u1, u3):
    C, Ct = pivot_factors(phi4, piv)
    K1 = np.einsum("cmn,cprm,qsn->pqrs", u1, Ct, C, optimize=True)
    K3 = np.einsum("mn,prm,qsn->pqrs", u3, C, C, optimize=True)
    K1swap = K1.transpose(2, 3, 0, 1)          # K1swap^{pq}_{rs} = K1^{rs}_{pq}
    return 0.5 * p12(K1 - K1swap + K3)


def du_tensor(phi4, piv, D1, D4, X2, X3):
    C, _ = pivot_factors(phi4, piv)
    D = D4 + 2.0 * D1
    X = (0.0 if X2 is None else X2) + (0.0 if X3 is None else X3)
    CDC = np.einsum("prm,mn,qsn->pqrs", C, D, C, optimize=True)
    CX = np.einsum("prm,qsm->pqrs", C, X, optimize=True) if not np.isscalar(X) else 0.0
    return -p12(CDC - CX)


def w_tensor(K, dU):
    return -K + dU


def delta_h(dU, n_occ):
    coul = sum(dU[:, o, :, o] for o in range(n_occ))      # [p, q] = sum_o dU^{po}_{qo}
    exch = sum(dU[:, o, o, :] for o in range(n_occ))      # [p, q] = sum_o dU^{po}_{oq}
    return -0.5 * (2.0 * coul - exch)


def fock_xtc(dh, W, n_occ):
    coul = sum(W[:, i, :, i] for i in range(n_occ))       # [p, q] = sum_i W^{pi}_{qi}
    exch = sum(W[:, i, i, :] for i in range(n_occ))       # [p, q] = sum_i W^{pi}_{iq}
    return dh + 2.0 * coul - exch


def e0_xtc(dh, n_occ, e_nuc):
    return -2.0 / 3.0 * float(np.trace(dh[:n_occ, :n_occ])) + e_nuc


def _k1_entry(Pm, u1, p, q, r, s):
    """K1^{pq}_{rs} = sum_{c mu nu} u1^c_{mu nu} phi_p d_c phi_r (mu) phi_q phi_s (nu)."""
    a = Pm[0, p] * Pm[1:4, r]                 # [c, mu]
    b = Pm[0, q] * Pm[0, s]                   # [nu]
    return float(np.einsum("cm,cmn,n->", a, u1, b))


def _pair_entry(Pm, M, p, r, q, s):
    """sum_{mu nu} C^p_r(mu) M_{mu nu} C^q_s(nu)."""
    return float((Pm[0, p] * Pm[0, r]) @ M @ (Pm[0, q] * Pm[0, s]))


def w_entry(phi4_piv, u1, u3, D1, D4, X, p, q, r, s):
    """One element W^{pq}_{rs} = -K^{pq}_{rs} + dU^{pq}_{rs} from the definitions (for
    sampled checks at sizes where the tensors are not formed). phi4_piv [4][n_orb][n_mu],
    X [n_orb][n_orb][n_mu] or None."""
    Pm = phi4_piv
    D = D4 + 2.0 * D1

    def s_part(p, q, r, s):      # K1 - K1swap + K3 at (p, q, r, s)
        return (_k1_entry(Pm, u1, p, q, r, s) - _k1_entry(Pm, u1, r, s, p, q)
                + _pair_entry(Pm, u3, p, r, q, s))

    def t_part(p, q, r, s):      # C D C - C X at (p, q, r, s)
        v = _pair_entry(Pm, D, p, r, q, s)
        if X is not None:
            v -= float((Pm[0, p] * Pm[0, r]) @ X[q, s])
        return v

    K = 0.5 * (s_part(p, q, r, s) + s_part(q, p, s, r))
    dU = -(t_part(p, q, r, s) + t_part(q, p, s, r))
    return -K + dU


def w_panel(phi4_piv, u1, u3, D1, D4, X, p0, p1):
    """W^{pq}_{rs} for p0 <= p < p1 from the definitions (array [p - p0, q, r, s]), at sizes
    where the full tensors are not formed. phi4_piv [4][n_orb][n_mu], X [n_orb][n_orb][n_mu]
    or None."""
    C = np.einsum("pm,rm->prm", phi4_piv[0], phi4_piv[0])
    Ct = np.einsum("pm,crm->cprm", phi4_piv[0], phi4_piv[1:4])
    Cp, Ctp = C[p0:p1], Ct[:, p0:p1]                       # p restricted
    D = D4 + 2.0 * D1
    # S^{pq}_{rs} = K1^{pq}_{rs} - K1^{rs}_{pq} + K3^{pq}_{rs}
    S = (np.einsum("cmn,cprm,qsn->pqrs", u1, Ctp, C, optimize=True)
         - np.einsum("cmn,crpm,sqn->pqrs", u1, Ct[:, :, p0:p1], C, optimize=True)
         + np.einsum("mn,prm,qsn->pqrs", u3, Cp, C, optimize=True))
    # S^{qp}_{sr} = K1^{qp}_{sr} - K1^{sr}_{qp} + K3^{qp}_{sr}
    Sx = (np.einsum("cmn,cqsm,prn->pqrs", u1, Ct, Cp, optimize=True)
          - np.einsum("cmn,csqm,rpn->pqrs", u1, Ct, C[:, p0:p1], optimize=True)
          + np.einsum("mn,qsm,prn->pqrs", u3, C, Cp, optimize=True))
    T = np.einsum("mn,prm,qsn->pqrs", D, Cp, C, optimize=True)
    Tx = np.einsum("mn,qsm,prn->pqrs", D, C, Cp, optimize=True)
    if X is not None:
        T = T - np.einsum("prm,qsm->pqrs", Cp, X, optimize=True)
        Tx = Tx - np.einsum("qsm,prm->pqrs", C, X[p0:p1], optimize=True)
    return -0.5 * (S + Sx) - (T + Tx)
