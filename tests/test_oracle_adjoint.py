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
