"""Pins of the oracle's reference-variance VMC pieces (the VMC section: eq. Eloc,
eq. var-loss, eq. gn) against what the mathematics fixes independently of the
formulas the oracle uses: finite differences of values, grid quadrature of the
sampled density, brute-force determinants and the least-squares minimiser."""
import numpy as np
import pytest

from oracle import correlator, orbitals, vmc
from workloads import nuclear_repulsion, vmc_draws, vmc_walkers


def _occ(wl):
    return np.ascontiguousarray(wl.C_mo[:, :wl.n_occ])


def test_ao_laplacian_equals_richardson_differences_of_the_gradient(h6_small):
    wl = h6_small
    X = np.random.default_rng(0).normal(size=(3, 9)) * 1.5
    lap = orbitals.eval_ao_lap(wl.basis, X)[4]

    def fd(h):
        out = np.zeros_like(lap)
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[c] += h
            Xm[c] -= h
            out += (orbitals.eval_ao(wl.basis, Xp)[1 + c] - orbitals.eval_ao(wl.basis, Xm)[1 + c]) / (2 * h)
        return out

    rich = (4.0 * fd(1e-3) - fd(2e-3)) / 3.0
    assert np.abs(rich - lap).max() <= 1e-8 * np.abs(lap).max()


def _psi(wl, corr, R):
    """Psi_T = exp(sum_{i<j} u(r_i, r_j)) det_up det_down from values alone."""
    n_occ = wl.n_occ
    n_w, n_el, _ = R.shape
    C = _occ(wl)
    phi = np.einsum("an,ak->nk", orbitals.eval_ao(wl.basis, R.reshape(-1, 3).T)[0], C).reshape(n_w, n_el, n_occ)
    det = np.linalg.det(phi[:, :n_occ]) * np.linalg.det(phi[:, n_occ:])
    J = np.zeros(n_w)
    for i in range(n_el):
        for j in range(i + 1, n_el):
            J += np.array([correlator.u_value(corr, R[w, i][:, None], R[w, j][:, None])[0, 0]
                           for w in range(n_w)])
    return np.exp(J) * det


@pytest.mark.parametrize("name", ["h4", "h6_small"])
def test_local_energy_equals_finite_difference_laplacian_of_psi(name, h4, h6_small):
    """E_loc = -1/2 sum_i lap_i Psi / Psi + V with the Laplacian from fourth-order
    differences of Psi values (no derivative formula of the oracle involved)."""
    wl = {"h4": h4, "h6_small": h6_small}[name]
    corr = wl.corr
    R = vmc_walkers(wl, 3, seed=5)
    e_nuc = nuclear_repulsion(wl)
    E = vmc.local_energy(wl.basis, _occ(wl), wl.atom_xyz, wl.atom_Z.astype(float), e_nuc, corr, R)
    psi0 = _psi(wl, corr, R)

    def lap_fd(h):
        tot = np.zeros(R.shape[0])
        for i in range(R.shape[1]):
            for c in range(3):
                Rp, Rm = R.copy(), R.copy()
                Rp[:, i, c] += h
                Rm[:, i, c] -= h
                tot += (_psi(wl, corr, Rp) - 2.0 * psi0 + _psi(wl, corr, Rm)) / (h * h)
        return tot

    lap = (4.0 * lap_fd(1e-3) - lap_fd(2e-3)) / 3.0
    E_fd = -0.5 * lap / psi0 + vmc.coulomb(R, wl.atom_xyz, wl.atom_Z.astype(float), e_nuc)
    assert np.abs(E_fd - E).max() <= 1e-5 * max(1.0, np.abs(E).max()), (E, E_fd)
    # the correlator changes E_loc (a dropped Jastrow term would not be seen otherwise)
    E0 = vmc.local_energy(wl.basis, _occ(wl), wl.atom_xyz, wl.atom_Z.astype(float), e_nuc,
                          corr.with_c(0.0 * corr.c), R)
    assert np.abs(E0 - E).max() > 1e-2


def test_parameter_derivatives_equal_richardson_differences(h4):
    from dataclasses import replace
    wl = h4
    corr = wl.corr
    R = vmc_walkers(wl, 5, seed=6)
    args = (wl.basis, _occ(wl), wl.atom_xyz, wl.atom_Z.astype(float), nuclear_repulsion(wl))
    E, dE = vmc.local_energy_grad(*args, corr, R)
    n = corr.n_terms

    def moved(p, v):
        if p == n:
            return replace(corr, d=corr.d + v)
        c = corr.c.copy()
        c[0, p] += v
        return replace(corr, c=c)

    for p in range(n + 1):
        f = lambda v: vmc.local_energy(*args, moved(p, v), R)
        h = 1e-3
        rich = (4.0 * (f(h) - f(-h)) / (2 * h) - (f(2 * h) - f(-2 * h)) / (4 * h)) / 3.0
        assert np.abs(rich - dE[:, p]).max() <= 1e-8 * max(1.0, np.abs(dE[:, p]).max()), p


def test_sampler_moments_equal_quadrature_of_the_orbital_density(h2_tiny):
    """Two electrons in one doubly occupied orbital: |Phi_0|^2 = phi(r1)^2 phi(r2)^2, so
    every electron's marginal is phi^2 / int phi^2, whose moments the grid gives."""
    wl = h2_tiny
    assert wl.n_occ == 1
    n_w, burn, keep = 1500, 30, 40
    R0 = vmc_walkers(wl, n_w, seed=1)
    normals, uniforms = vmc_draws(burn + keep, 2, n_w, seed=2)
    C = _occ(wl)
    R, acc, _ = vmc.metropolis(wl.basis, C, R0, 0.9, normals[:burn], uniforms[:burn])
    samples = []
    for s in range(keep):
        R, a, _ = vmc.metropolis(wl.basis, C, R, 0.9, normals[burn + s:burn + s + 1],
                                 uniforms[burn + s:burn + s + 1])
        samples.append(R.copy())
    S = np.stack(samples)                                  # [keep, n_w, 2, 3]
    phi = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)[0, 0]
    rho = wl.grid_w * phi * phi
    for f in (lambda X: X[2] ** 2, lambda X: X[0] ** 2 + X[1] ** 2, lambda X: np.abs(X[2])):
        ref = float((rho * f(wl.grid_xyz)).sum() / rho.sum())
        per_walker = f(np.moveaxis(S, -1, 0)).mean(axis=(0, 2))     # [n_w]
        se = per_walker.std(ddof=1) / np.sqrt(n_w)
        assert abs(per_walker.mean() - ref) < 5.0 * se, (per_walker.mean(), ref, se)
        assert se < 0.05 * ref


def test_sampler_acceptance_rule_matches_brute_force_determinants(h4):
    wl = h4
    n_w = 40
    R0 = vmc_walkers(wl, n_w, seed=3)
    normals, uniforms = vmc_draws(1, 4, n_w, seed=4)
    C = _occ(wl)
    R, acc, _ = vmc.metropolis(wl.basis, C, R0, 0.8, normals, uniforms)
    # replay with full determinants of the whole configuration
    def phi0(Rw):
        v = np.einsum("an,ak->nk", orbitals.eval_ao(wl.basis, Rw.T)[0], C)
        return np.linalg.det(v[:2]) * np.linalg.det(v[2:])
    n_acc = np.zeros(n_w, int)
    for w in range(n_w):
        cur = R0[w].copy()
        for i in range(4):
            prop = cur.copy()
            prop[i] += 0.8 * normals[0, i, w]
            if uniforms[0, i, w] < (phi0(prop) / phi0(cur)) ** 2:
                cur = prop
                n_acc[w] += 1
        assert np.allclose(cur, R[w], rtol=0, atol=0)
    assert np.array_equal(n_acc, acc)
    assert 0 < acc.sum() < 4 * n_w


def test_gauss_newton_step_reaches_the_least_squares_minimum_of_a_linear_model():
    """E_k(theta) = a_k + B_k . theta without clipping: the variance is quadratic, and the
    step with lambda = 0, eta = (N - 1) / (2N) is exactly the Newton step to its minimum."""
    rng = np.random.default_rng(9)
    n, p = 400, 5
    a = rng.uniform(-1, 1, size=n)
    B = rng.uniform(-1, 1, size=(n, p))
    delta, grad, C, st = vmc.gn_step(a, B, 0.0, (n - 1) / (2.0 * n))
    assert st["n_clipped"] == 0
    Bc = B - B.mean(axis=0)
    ac = a - a.mean()
    ref = np.linalg.lstsq(Bc, -ac, rcond=None)[0]
    assert np.allclose(delta, ref, rtol=1e-12, atol=1e-13)
    var_new = vmc.clipped_objective(a + B @ delta)["var"]
    var_min = ((ac + Bc @ ref) ** 2).sum() / (n - 1)
    assert var_new == pytest.approx(var_min, rel=1e-12)
    assert np.allclose(C, Bc.T @ Bc / n, rtol=1e-13, atol=1e-15)


def test_variance_gradient_with_active_clipping_equals_central_differences():
    rng = np.random.default_rng(10)
    n, p = 300, 4
    a = rng.standard_cauchy(size=n)                   # heavy tails: points beyond 5 MAD
    B = rng.normal(size=(n, p))
    _, grad, _, st = vmc.gn_step(a, B, 0.1, 1.0)
    assert st["n_clipped"] > 0
    var = lambda th: vmc.clipped_objective(a + B @ th)["var"]
    h = 1e-6
    for q in range(p):
        e = np.zeros(p)
        e[q] = h
        fd = (var(e) - var(-e)) / (2 * h)
        assert fd == pytest.approx(grad[q], rel=1e-6, abs=1e-8)


def _bh_two_type(wl):
    from workloads import Correlator, bh_correlator
    base = bh_correlator(wl.atom_xyz)
    n = base.nuc_xyz.shape[0]
    c = np.random.default_rng(12).uniform(-0.5, 0.5, size=(2, base.n_terms)) / n
    return Correlator(base.form, base.mno, c, 0.9, np.array([1.1, 0.8]), base.nuc_xyz,
                      (np.arange(n) % 2).astype(np.int32))


def test_bh_local_energy_equals_finite_difference_laplacian_of_psi(h4):
    """The BH form (eq. bh-u, two nucleus types): E_loc against fourth-order differences of
    Psi_T values built from u itself (correlator.u_value) and the determinants."""
    wl = h4
    corr = _bh_two_type(wl)
    R = vmc_walkers(wl, 3, seed=15)
    e_nuc = nuclear_repulsion(wl)
    Z = wl.atom_Z.astype(float)
    E = vmc.local_energy(wl.basis, _occ(wl), wl.atom_xyz, Z, e_nuc, corr, R)
    psi0 = _psi(wl, corr, R)

    def lap_fd(h):
        tot = np.zeros(R.shape[0])
        for i in range(R.shape[1]):
            for c in range(3):
                Rp, Rm = R.copy(), R.copy()
                Rp[:, i, c] += h
                Rm[:, i, c] -= h
                tot += (_psi(wl, corr, Rp) - 2.0 * psi0 + _psi(wl, corr, Rm)) / (h * h)
        return tot

    lap = (4.0 * lap_fd(1e-3) - lap_fd(2e-3)) / 3.0
    E_fd = -0.5 * lap / psi0 + vmc.coulomb(R, wl.atom_xyz, Z, e_nuc)
    assert np.abs(E_fd - E).max() <= 1e-5 * max(1.0, np.abs(E).max()), (E, E_fd)
    E0 = vmc.local_energy(wl.basis, _occ(wl), wl.atom_xyz, Z, e_nuc, corr.with_c(0.0 * corr.c), R)
    assert np.abs(E0 - E).max() > 1e-2


def test_bh_parameter_derivatives_equal_richardson_differences(h4):
    """Complex-step dE/dc[t][k], dE/dd and dE/db_t of the BH form against Richardson
    differences (a sample of the linear coefficients, every nonlinear parameter)."""
    from dataclasses import replace
    wl = h4
    corr = _bh_two_type(wl)
    R = vmc_walkers(wl, 4, seed=16)
    args = (wl.basis, _occ(wl), wl.atom_xyz, wl.atom_Z.astype(float), nuclear_repulsion(wl))
    E, dE = vmc.local_energy_grad(*args, corr, R)
    nt, n = corr.c.shape
    assert dE.shape == (4, nt * n + 1 + nt)

    def moved(p, v):
        if p < nt * n:
            c = corr.c.copy()
            c[p // n, p % n] += v
            return replace(corr, c=c)
        if p == nt * n:
            return replace(corr, d=corr.d + v)
        b = np.asarray(corr.b, np.float64).copy()
        b[p - nt * n - 1] += v
        return replace(corr, b=b)

    for p in (0, 7, 30, n + 5, 2 * n - 1, nt * n, nt * n + 1, nt * n + 2):
        f = lambda v: vmc.local_energy(*args, moved(p, v), R)
        h = 1e-3
        rich = (4.0 * (f(h) - f(-h)) / (2 * h) - (f(2 * h) - f(-2 * h)) / (4 * h)) / 3.0
        assert np.abs(rich - dE[:, p]).max() <= 1e-8 * max(1.0, np.abs(dE[:, p]).max()), p
