"""Pins of the oracle's orbital evaluation (Alg. 2, grid step) against the
analytic Gaussian overlap and against finite differences."""
import numpy as np
import pytest

from oracle import orbitals
from workloads.basis import build_basis
from workloads.grid import atom_grid
from workloads.integrals import one_electron


def _two_atom_basis():
    xyz = np.array([[0.0, 0.0, -0.7], [0.3, -0.2, 0.8]])
    shells = [[(0, 1.3), (1, 0.9), (2, 0.7), (3, 0.6)], [(0, 0.5), (1, 1.1), (2, 0.8)]]
    return build_basis(xyz, shells)


def test_ao_quadrature_matches_analytic_overlap():
    basis = _two_atom_basis()
    gxyz, gw = atom_grid(basis.atom_xyz, np.array([0.8, 0.8]), 120, 302, seed=7)
    ao = orbitals.eval_ao(basis, gxyz)
    S_grid = np.einsum("ag,bg,g->ab", ao[0], ao[0], gw)
    S, _, _ = one_electron(basis, np.zeros(2), with_potential=False)
    # normalised Cartesian Gaussians: unit diagonal for pure-power components
    assert np.abs(S_grid - S).max() < 2e-5
    # kinetic energy: 1/2 sum w grad chi . grad chi equals the analytic T
    _, T, _ = one_electron(basis, np.zeros(2), with_potential=False)
    T_grid = 0.5 * np.einsum("cag,cbg,g->ab", ao[1:4], ao[1:4], gw)
    assert np.abs(T_grid - T).max() < 1e-4


def test_orbital_gradients_match_central_differences(h4):
    rng = np.random.default_rng(0)
    idx = rng.choice(h4.n_g, 200, replace=False)
    X = h4.grid_xyz[:, idx]
    phi4 = orbitals.eval_orbitals(h4.basis, h4.C_mo, X)
    h = 1e-5
    for c in range(3):
        e = np.zeros((3, 1))
        e[c] = h
        fp = orbitals.eval_orbitals(h4.basis, h4.C_mo, X + e)[0]
        fm = orbitals.eval_orbitals(h4.basis, h4.C_mo, X - e)[0]
        fd = (fp - fm) / (2 * h)
        scale = np.abs(phi4[1 + c]).max()
        assert np.abs(fd - phi4[1 + c]).max() < 1e-7 * max(scale, 1.0)


def test_density_is_occupied_sum(h2_tiny):
    phi4 = orbitals.eval_orbitals(h2_tiny.basis, h2_tiny.C_mo, h2_tiny.grid_xyz)
    rho = orbitals.density(phi4, 1)
    assert np.array_equal(rho, phi4[0, 0] ** 2)
    # one electron per spin in the occupied orbital: integrates to ~1 on the grid
    assert abs(np.dot(h2_tiny.grid_w, rho) - 1.0) < 5e-2
