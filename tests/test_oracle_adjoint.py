"""Pins of the oracle's coefficient derivatives: central finite differences are
exact up to rounding because every output is a polynomial of degree <= 2 in c."""
import numpy as np
import pytest

from oracle import adjoint, contract, fit, orbitals, pivots
from workloads import bh_correlator

ALL = contract.U1 | contract.U3 | contract.ULAP | contract.D1 | contract.D4 | contract.FIELD


def _problem(wl, n_points, n_mu, seed=0):
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(seed).choice(wl.n_g, n_points, replace=False))
    xyz, w, phi4 = wl.grid_xyz[:, idx], wl.grid_w[idx], phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, n_mu)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    return xyz, w, fr.xi, fr.xigrad, rho[fp.pivots], rho


def _cotangents(n_mu, n_g, seed, lap=True):
    rng = np.random.default_rng(seed)
    cot = {"u1": rng.normal(size=(3, n_mu, n_mu)) / n_mu, "u3": rng.normal(size=(n_mu, n_mu)) / n_mu,
           "D1": rng.normal(size=(n_mu, n_mu)) / n_mu, "D4": rng.normal(size=(n_mu, n_mu)) / n_mu,
           "field": rng.normal(size=(3, n_g)) / np.sqrt(n_g)}
    if lap:
        cot["ulap"] = rng.normal(size=(n_mu, n_mu)) / n_mu
    return cot


def _loss(out, cot):
    return sum(float(np.sum(cot[k] * out[k])) for k in cot)


@pytest.mark.parametrize("form", ["ee", "bh"])
def test_adjoint_matches_central_differences(h6_small, form):
    xyz, w, xi, xig, G, rho = _problem(h6_small, 500 if form == "ee" else 260, 30 if form == "ee" else 16)
    corr = h6_small.corr if form == "ee" else bh_correlator(h6_small.atom_xyz)
    lap = form == "ee"
    cot = _cotangents(xi.shape[0], xi.shape[1], 33, lap)
    chans = ALL if lap else ALL & ~contract.ULAP
    g = adjoint.dL_dc(xyz, w, corr, xi, xig, G, rho, cot)
    c0 = corr.c.ravel()
    h = 1e-4
    idx = range(c0.size) if form == "ee" else [0, 5, 17, 38, 39, 47]
    for j in idx:
        cp, cm = c0.copy(), c0.copy()
        cp[j] += h
        cm[j] -= h
        lp = _loss(contract.contract(xyz, w, corr.with_c(cp), xi, xig, G, rho, chans), cot)
        lm = _loss(contract.contract(xyz, w, corr.with_c(cm), xi, xig, G, rho, chans), cot)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_scale_derivative_complex_step_equals_richardson_differences(h2_tiny):
    """The oracle's dL/dd (complex step through its contraction, every channel) against
    Richardson-extrapolated central differences of real contractions (O(h^4))."""
    from dataclasses import replace
    from oracle import adjoint, contract, fit, orbitals, pivots
    wl = h2_tiny
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    fp = pivots.select_fused(phi4, wl.grid_w, 10)
    fr = fit.fit(phi4, wl.grid_w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    G = rho[fp.pivots]
    n = len(fp.pivots)
    rng = np.random.default_rng(3)
    cot = {"u1": rng.normal(size=(3, n, n)), "u3": rng.normal(size=(n, n)),
           "ulap": rng.normal(size=(n, n)), "D1": rng.normal(size=(n, n)),
           "D4": rng.normal(size=(n, n)), "field": rng.normal(size=(3, wl.n_g))}
    cs = adjoint.dL_dd(wl.grid_xyz, wl.grid_w, wl.corr, fr.xi, fr.xigrad, G, rho, cot)

    def L(d):
        out = contract.contract(wl.grid_xyz, wl.grid_w, replace(wl.corr, d=d), fr.xi, fr.xigrad,
                                G, rho, 1 | 2 | 4 | 8 | 16 | 32)
        return adjoint.loss(out, cot)

    d0, h = wl.corr.d, 1e-3
    fd1 = (L(d0 + h) - L(d0 - h)) / (2 * h)
    fd2 = (L(d0 + 2 * h) - L(d0 - 2 * h)) / (4 * h)
    rich = (4.0 * fd1 - fd2) / 3.0
    assert abs(rich - cs) <= 1e-10 * abs(cs)
    # a real d gives real outputs (the complex path leaves the real one unchanged)
    out = contract.contract(wl.grid_xyz, wl.grid_w, wl.corr, fr.xi, fr.xigrad, G, rho, 1 | 2)
    assert out["u1"].dtype == np.float64


def test_bh_nonlinear_derivatives_complex_step_equal_richardson_differences(h6_small):
    """The oracle's [dL/dd, dL/db_0, dL/db_1] for the BH form (eq. bh-u) on two nucleus
    types with distinct b: complex step against Richardson-extrapolated central
    differences of real contractions, each parameter moved on its own."""
    from dataclasses import replace
    from workloads import Correlator
    xyz, w, xi, xig, G, rho = _problem(h6_small, 200, 14, seed=4)
    base = bh_correlator(h6_small.atom_xyz)
    n = base.nuc_xyz.shape[0]
    c = np.random.default_rng(11).uniform(-0.5, 0.5, size=(2, base.n_terms)) / n
    corr = Correlator(base.form, base.mno, c, base.d, np.array([1.0, 1.3]), base.nuc_xyz,
                      (np.arange(n) % 2).astype(np.int32))
    cot = _cotangents(xi.shape[0], xi.shape[1], 35, lap=False)
    chans = ALL & ~contract.ULAP
    cs = adjoint.dL_dnl(xyz, w, corr, xi, xig, G, rho, cot)
    assert cs.shape == (3,)

    def moved(k, v):
        if k == 0:
            return replace(corr, d=corr.d + v)
        b = corr.b.copy()
        b[k - 1] += v
        return replace(corr, b=b)

    h = 1e-3
    for k in range(3):
        L = lambda v: _loss(contract.contract(xyz, w, moved(k, v), xi, xig, G, rho, chans), cot)
        fd1 = (L(h) - L(-h)) / (2 * h)
        fd2 = (L(2 * h) - L(-2 * h)) / (4 * h)
        rich = (4.0 * fd1 - fd2) / 3.0
        assert abs(rich - cs[k]) <= 1e-9 * np.abs(cs).max(), (k, rich, cs[k])
    # the EE form returns dL/dd alone, equal to dL_dd
    assert adjoint.dL_dnl(xyz, w, h6_small.corr, xi, xig, G, rho, cot).shape == (1,)
