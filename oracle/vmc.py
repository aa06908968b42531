"""Reference-variance optimisation of the correlator by variational Monte Carlo
(the VMC section: sampling from the reference determinant, eq. Eloc, the fixed-batch
objective eq. var-loss with its MAD clipping, and the Gauss-Newton update eq. gn).

Test infrastructure: plain FP64 NumPy, sharing no code with the GPU library.

Trial function (eq. tau-def): Psi_T(R) = F(R) Phi_0(R), F = prod_{i<j} exp(u(r_i, r_j)),
so log F = J = sum_{i<j} u(r_i, r_j). Phi_0 is the closed-shell reference
determinant: electrons 0 .. n_occ - 1 spin up, n_occ .. 2 n_occ - 1 spin down,
Phi_0 = det[phi_k(r_i)]_up det[phi_k(r_i)]_down over the occupied orbitals k.

Local energy (eq. Eloc) with H = -1/2 sum_i lap_i - sum_{i,I} Z_I / r_iI
+ sum_{i<j} 1 / r_ij + E_nuc:
  lap_i Psi_T / Psi_T = lap_i J + |grad_i J|^2 + 2 grad_i J . D_i + S_i,
  D_i = grad_i Phi_0 / Phi_0 = sum_k grad phi_k(r_i) [A^-1]_{k i},
  S_i = lap_i Phi_0 / Phi_0 = sum_k lap phi_k(r_i) [A^-1]_{k i}
(Jacobi's formula; A the spin block holding electron i). For the EE form
u = sum_k c_k rbar^{o_k}, rbar = d r / (1 + d r): grad_i J = sum_{j != i} (u'/r) (r_i - r_j),
lap_i J = sum_{j != i} (u'' + 2 u' / r). For the BH form (eq. bh-u) with
a = a(r_iI), a' = a(r_jI), e = rbar(r_ij) and P = a^m a'^n + a'^m a^n:
  grad_i f = c [P_a e^o grad a + P o e^{o-1} grad e],
  lap_i f = c [P_aa e^o |grad a|^2 + P_a e^o lap a + 2 P_a o e^{o-1} grad a . grad e
               + P (o (o-1) e^{o-2} |grad e|^2 + o e^{o-1} lap e)],
P_a, P_aa the derivatives in a; for s = x r / (1 + x r): s' = x t^2, s'' = -2 x^2 t^3,
grad s = s' rhat, lap s = s'' + 2 s' / r.

Readings (the paper leaves the sampler's details and the schedule to its supporting
information):
  * Metropolis sweeps move the electrons one at a time in index order with a
    symmetric Gaussian proposal r_i' = r_i + step * eta; the move is accepted when a
    uniform draw is below |Phi_0(R') / Phi_0(R)|^2. The draws are inputs.
  * The clip bounds m_s +- 5 d_s are functions of the parameters and are
    differentiated with them (sign(0) = 0 in the MAD's derivative).
  * Parameters theta = (c_0 .. c_{n_terms - 1}, d) of the EE form; for the BH form
    theta = (c[type][term] type-major, d, b_0 .. b_{n_types - 1}).

Pinned by: the AO Laplacian against central differences; the local energy
against a finite-difference Laplacian of Psi_T built from values alone; the
parameter derivatives (complex step) against Richardson differences; the sampler's
moments against grid quadrature of |phi|^2 for a two-electron system, and its
acceptance rule against brute-force determinants; the Gauss-Newton step against
the least-squares minimiser of a linear residual model.
"""
from __future__ import annotations

import numpy as np

from .orbitals import eval_ao, eval_ao_lap


def _occ_values(basis, C_occ, X, lap=False):
    """[5 or 1, n, n_occ]: occupied orbitals (and gradients, Laplacians) at points X [3, n]."""
    ao = eval_ao_lap(basis, X) if lap else eval_ao(basis, X)[:1]
    return np.einsum("can,ak->cnk", ao, C_occ, optimize=True)


def coulomb(R, nuc_xyz, nuc_Z, e_nuc):
    """V(R) for walkers R [n_w, n_el, 3]."""
    n_el = R.shape[1]
    V = np.full(R.shape[0], float(e_nuc))
    for i in range(n_el):
        for I in range(nuc_xyz.shape[0]):
            V -= nuc_Z[I] / np.linalg.norm(R[:, i] - nuc_xyz[I], axis=1)
        for j in range(i + 1, n_el):
            V += 1.0 / np.linalg.norm(R[:, i] - R[:, j], axis=1)
    return V


def _radial(corr, r):
    """u'(r) and u''(r) of the EE form u = sum_k c_k rbar^{o_k} (types of c and d kept)."""
    d = corr.d
    t = 1.0 / (1.0 + d * r)
    e = d * r * t
    up = 0.0
    upp = 0.0
    for k in range(corr.n_terms):
        o = int(corr.mno[k, 2])
        c = corr.c[0, k]
        # d rbar / dr = d t^2, d^2 rbar / dr^2 = -2 d^2 t^3
        up = up + c * o * e ** (o - 1) * d * t * t
        second = o * (o - 1) * e ** (o - 2) * (d * t * t) ** 2 if o >= 2 else 0.0
        upp = upp + c * (second - o * e ** (o - 1) * 2.0 * d * d * t ** 3)
    return up, upp


def _scaled(x, r):
    """s = x r / (1 + x r) and its first two derivatives in r."""
    t = 1.0 / (1.0 + x * r)
    return x * r * t, x * t * t, -2.0 * x * x * t ** 3


def _bh_grad_lap(corr, R):
    """grad_i J and lap_i J for the BH form (eq. bh-u), summed over nuclei and terms
    (arrays over walkers x nuclei x terms; types of c, d and b kept)."""
    n_w, n_el, _ = R.shape
    dt = np.result_type(float, corr.d, np.asarray(corr.b), corr.c)
    G = np.zeros((n_w, n_el, 3), dt)
    L = np.zeros((n_w, n_el), dt)
    m = corr.mno[:, 0].astype(int)[None, None, :]
    n = corr.mno[:, 1].astype(int)[None, None, :]
    o = corr.mno[:, 2].astype(int)[None, None, :]
    ty = np.asarray(corr.nuc_type, int)
    b = np.asarray(corr.b)[ty][None, :]                      # [1, I]
    c = corr.c[ty][None, :, :]                               # [1, I, k]
    X = corr.nuc_xyz                                         # [I, 3]

    def pw(x, k):          # x^k for integer k >= 0 (0 where k < 0)
        return np.where(k >= 0, x ** np.maximum(k, 0), 0.0)

    for i in range(n_el):
        Di = R[:, i, None, :] - X[None, :, :]                # [w, I, 3]
        ri = np.linalg.norm(Di, axis=2)                      # [w, I]
        a, a1, a2 = _scaled(b, ri)
        ga = (a1 / ri)[:, :, None] * Di                      # grad_i a   [w, I, 3]
        la = a2 + 2.0 * a1 / ri                              # lap_i a    [w, I]
        A = a[:, :, None]
        for j in range(n_el):
            if j == i:
                continue
            Dv = R[:, i] - R[:, j]
            r = np.linalg.norm(Dv, axis=1)
            e, e1, e2 = _scaled(corr.d, r)
            ge = (e1 / r)[:, None] * Dv                      # grad_i e  [w, 3]
            le = e2 + 2.0 * e1 / r
            aj = _scaled(b, np.linalg.norm(R[:, j, None, :] - X[None, :, :], axis=2))[0]
            Aj = aj[:, :, None]
            P = pw(A, m) * pw(Aj, n) + pw(Aj, m) * pw(A, n)
            Pa = m * pw(A, m - 1) * pw(Aj, n) + n * pw(Aj, m) * pw(A, n - 1)
            Paa = m * (m - 1) * pw(A, m - 2) * pw(Aj, n) + n * (n - 1) * pw(Aj, m) * pw(A, n - 2)
            E = e[:, None, None]
            E0, E1, E2 = pw(E, o), o * pw(E, o - 1), o * (o - 1) * pw(E, o - 2)
            ga_ge = np.einsum("wic,wc->wi", ga, ge)[:, :, None]
            ga2 = np.einsum("wic,wic->wi", ga, ga)[:, :, None]
            ge2 = np.einsum("wc,wc->w", ge, ge)[:, None, None]
            # gradient: sum over (I, k) of c [Pa E0 grad a + P E1 grad e]
            wa = (c * Pa * E0).sum(axis=2)                   # [w, I]
            we = (c * P * E1).sum(axis=(1, 2))               # [w]
            G[:, i] += np.einsum("wi,wic->wc", wa, ga) + we[:, None] * ge
            L[:, i] += (c * (Paa * E0 * ga2 + Pa * E0 * la[:, :, None] + 2.0 * Pa * E1 * ga_ge
                             + P * (E2 * ge2 + E1 * le[:, None, None]))).sum(axis=(1, 2))
    return G, L


def jastrow_grad_lap(corr, R):
    """grad_i J [n_w, n_el, 3] and lap_i J [n_w, n_el]."""
    if corr.form != 0:
        return _bh_grad_lap(corr, R)
    n_w, n_el, _ = R.shape
    dt = np.result_type(float, corr.d, corr.c)
    G = np.zeros((n_w, n_el, 3), dt)
    L = np.zeros((n_w, n_el), dt)
    for i in range(n_el):
        for j in range(n_el):
            if j == i:
                continue
            Dv = R[:, i] - R[:, j]
            r = np.linalg.norm(Dv, axis=1)
            up, upp = _radial(corr, r)
            G[:, i] += (up / r)[:, None] * Dv
            L[:, i] += upp + 2.0 * up / r
    return G, L


def slater_terms(basis, C_occ, R):
    """D_i = grad_i Phi_0 / Phi_0 [n_w, n_el, 3] and S_i = lap_i Phi_0 / Phi_0 [n_w, n_el]."""
    n_w, n_el, _ = R.shape
    n_occ = C_occ.shape[1]
    assert n_el == 2 * n_occ
    phi = _occ_values(basis, C_occ, R.reshape(-1, 3).T, lap=True).reshape(5, n_w, n_el, n_occ)
    D = np.zeros((n_w, n_el, 3))
    S = np.zeros((n_w, n_el))
    for s in range(2):
        sl = slice(s * n_occ, (s + 1) * n_occ)
        Ainv = np.linalg.inv(phi[0][:, sl, :])            # [n_w, k, i]
        for c in range(3):
            D[:, sl, c] = np.einsum("wik,wki->wi", phi[1 + c][:, sl, :], Ainv)
        S[:, sl] = np.einsum("wik,wki->wi", phi[4][:, sl, :], Ainv)
    return D, S


def local_energy(basis, C_occ, nuc_xyz, nuc_Z, e_nuc, corr, R):
    """E_loc(R; theta) for walkers R [n_w, n_el, 3] (eq. Eloc)."""
    D, S = slater_terms(basis, C_occ, R)
    G, L = jastrow_grad_lap(corr, R)
    lap = L + np.einsum("wic,wic->wi", G, G) + 2.0 * np.einsum("wic,wic->wi", G, D) + S
    return -0.5 * lap.sum(axis=1) + coulomb(R, nuc_xyz, nuc_Z, e_nuc)


def local_energy_grad(basis, C_occ, nuc_xyz, nuc_Z, e_nuc, corr, R, h=1e-30):
    """E [n_w] and dE/dtheta by the complex step Im E(theta + i h e_p) / h:
    theta = (c_0 .. c_{n-1}, d) for the EE form and (c[type][term] type-major, d,
    b_0 .. b_{n_types - 1}) for the BH form."""
    from dataclasses import replace
    E = local_energy(basis, C_occ, nuc_xyz, nuc_Z, e_nuc, corr, R)
    nt, n = corr.c.shape
    n_b = 0 if corr.form == 0 else len(corr.b)
    dE = np.zeros((R.shape[0], nt * n + 1 + n_b))
    f = lambda cr: np.imag(local_energy(basis, C_occ, nuc_xyz, nuc_Z, e_nuc, cr, R)) / h
    for t in range(nt):
        for p in range(n):
            c = corr.c.astype(complex)
            c[t, p] += 1j * h
            dE[:, t * n + p] = f(replace(corr, c=c))
    dE[:, nt * n] = f(replace(corr, d=corr.d + 1j * h))
    for t in range(n_b):
        b = np.asarray(corr.b, dtype=complex).copy()
        b[t] += 1j * h
        dE[:, nt * n + 1 + t] = f(replace(corr, b=b))
    return E, dE


def metropolis(basis, C_occ, R0, step, normals, uniforms):
    """Sweeps of single-electron Metropolis moves sampling |Phi_0|^2.
    normals [n_sweeps, n_el, n_w, 3], uniforms [n_sweeps, n_el, n_w].
    Returns (R [n_w, n_el, 3], accepted [n_w], margins) where margins holds
    |u - ratio^2| / max(ratio^2, u) of every decision (how far each was from a tie)."""
    R = np.array(R0, np.float64, copy=True)
    n_w, n_el, _ = R.shape
    n_occ = C_occ.shape[1]
    phi = _occ_values(basis, C_occ, R.reshape(-1, 3).T)[0].reshape(n_w, n_el, n_occ)
    acc = np.zeros(n_w, np.int64)
    margins = []
    for s in range(normals.shape[0]):
        for i in range(n_el):
            sl = slice((i // n_occ) * n_occ, (i // n_occ + 1) * n_occ)
            rp = R[:, i] + step * normals[s, i]
            php = _occ_values(basis, C_occ, rp.T)[0]                  # [n_w, n_occ]
            A = phi[:, sl]
            Ap = A.copy()
            Ap[:, i % n_occ] = php
            ratio = np.linalg.det(Ap) / np.linalg.det(A)
            p = ratio * ratio
            u = uniforms[s, i]
            ok = u < p
            margins.append(np.abs(u - p) / np.maximum(np.maximum(p, u), 1e-300))
            R[ok, i] = rp[ok]
            phi[ok, i] = php[ok]
            acc += ok
    return R, acc, np.concatenate(margins) if margins else np.zeros(0)


def clipped_objective(E):
    """Raw mean m, MAD d, clipped energies, their mean and the variance (eq. var-loss)."""
    E = np.asarray(E)
    n = E.shape[0]
    m = E.sum() / n
    mad = np.abs(E - m).sum() / n
    Et = np.clip(E, m - 5.0 * mad, m + 5.0 * mad)
    mean = Et.sum() / n
    var = ((Et - mean) ** 2).sum() / (n - 1)
    return {"m": m, "mad": mad, "Et": Et, "mean": mean, "var": var}


def gn_step(E, dE, lam, eta):
    """One Newton step with Gauss-Newton curvature (eq. gn) on the fixed batch:
    r_k = Et_k - mean(Et), C = (1/N) sum_k dr_k dr_k^T + lam I,
    grad sigma^2 = 2/(N - 1) sum_k r_k dr_k, delta = -eta C^-1 grad (Cholesky).
    The derivatives of the clipped energies follow the clip bounds m +- 5 d as
    functions of theta. Returns (delta, grad, C, stats)."""
    E = np.asarray(E, np.float64)
    dE = np.asarray(dE, np.float64)
    n, n_th = dE.shape
    st = clipped_objective(E)
    m, mad = st["m"], st["mad"]
    dm = dE.sum(axis=0) / n
    dmad = (np.sign(E - m)[:, None] * (dE - dm[None, :])).sum(axis=0) / n
    lo = E < m - 5.0 * mad
    hi = E > m + 5.0 * mad
    dEt = np.where(lo[:, None], (dm - 5.0 * dmad)[None, :],
                   np.where(hi[:, None], (dm + 5.0 * dmad)[None, :], dE))
    r = st["Et"] - st["mean"]
    dr = dEt - dEt.sum(axis=0)[None, :] / n
    grad = 2.0 / (n - 1) * (dr.T @ r)
    C = dr.T @ dr / n + lam * np.eye(n_th)
    Lc = np.linalg.cholesky(C)
    delta = -eta * np.linalg.solve(Lc.T, np.linalg.solve(Lc, grad))
    st = dict(st, n_clipped=int(lo.sum() + hi.sum()))
    return delta, grad, C, st
