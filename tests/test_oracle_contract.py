"""Pins of the oracle's grid-pair kernels and xTC D terms (eqs. K1-isdf,
K3-isdf; xTC section, Terms 1 and 4): dense brute force in the opposite
contraction order, invariances, and the four-index brute force at full rank."""
import numpy as np
import pytest

from oracle import contract, fit, fourindex, orbitals, pivots
from oracle.correlator import pair_kernels
from workloads import ee_correlator

ALL = contract.U1 | contract.U3 | contract.ULAP | contract.D1 | contract.D4 | contract.FIELD | contract.ESCALE


def _setup(wl, n_points=None, n_mu=None, seed=0):
    xyz, w = wl.grid_xyz, wl.grid_w
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, xyz)
    if n_points is not None:
        idx = np.sort(np.random.default_rng(seed).choice(wl.n_g, n_points, replace=False))
        xyz, w, phi4 = xyz[:, idx], w[idx], phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, n_mu or wl.n_mu)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    return dict(xyz=xyz, w=w, phi4=phi4, piv=fp.pivots, xi=fr.xi, xig=fr.xigrad, rho=rho,
                G=rho[fp.pivots])


@pytest.fixture(scope="module")
def sub(h6_small):
    s = _setup(h6_small, n_points=1500, n_mu=90)
    s["corr"] = h6_small.corr
    s["out"] = contract.contract(s["xyz"], s["w"], s["corr"], s["xi"], s["xig"], s["G"], s["rho"], ALL,
                                 bra_block=200, ket_block=700)
    return s


def test_brute_force_dense_kernel_other_order(sub):
    xyz, w, xi, xig, corr, out = sub["xyz"], sub["w"], sub["xi"], sub["xig"], sub["corr"], sub["out"]
    K = pair_kernels(corr, xyz, xyz, want_lap=True)
    wxi = xi * w
    for c, key in enumerate(("gx", "gy", "gz")):
        ref = ((xig[c] * w) @ K[key]) @ wxi.T          # sum over bra g first, then ket g'
        assert np.allclose(out["u1"][c], ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    ref3 = (wxi @ K["sq"]) @ wxi.T
    assert np.allclose(out["u3"], ref3, rtol=1e-11, atol=1e-12 * np.abs(ref3).max())
    refl = (wxi @ K["lap"]) @ wxi.T
    assert np.allclose(out["ulap"], refl, rtol=1e-11, atol=1e-12 * np.abs(refl).max())
    wr = w * sub["rho"]
    for c, key in enumerate(("gx", "gy", "gz")):
        assert np.allclose(out["field"][c], K[key] @ wr, rtol=1e-11, atol=1e-13)
    # energy-scale scalars
    e = out["escale"]
    G = sub["G"]
    assert np.isclose(e[0], G @ ref3 @ G, rtol=1e-11)
    assert np.isclose(e[3], wr @ K["sq"] @ wr, rtol=1e-11)


def test_zero_correlator_gives_exact_zeros(sub):
    z = sub["corr"].with_c(np.zeros_like(sub["corr"].c))
    out = contract.contract(sub["xyz"], sub["w"], z, sub["xi"], sub["xig"], sub["G"], sub["rho"], ALL)
    for k in ("u1", "u3", "ulap", "D1", "D4", "field", "escale"):
        assert np.all(out[k] == 0.0)


def test_scaling_in_c_and_symmetries(sub):
    c2 = sub["corr"].with_c(2.0 * sub["corr"].c)
    out2 = contract.contract(sub["xyz"], sub["w"], c2, sub["xi"], sub["xig"], sub["G"], sub["rho"], ALL)
    out = sub["out"]
    for k, f in (("u1", 2), ("ulap", 2), ("field", 2), ("u3", 4), ("D1", 4), ("D4", 4)):
        assert np.allclose(out2[k], f * out[k], rtol=1e-12, atol=1e-14 * np.abs(out[k]).max())
    assert np.allclose(out["D4"], out["D4"].T, rtol=1e-12, atol=1e-14 * np.abs(out["D4"]).max())
    assert np.allclose(out["u3"], out["u3"].T, rtol=1e-11, atol=1e-13 * np.abs(out["u3"]).max())


def test_translation_invariance_and_rotation_covariance(sub):
    xyz, w, xi, corr = sub["xyz"], sub["w"], sub["xi"], sub["corr"]
    xig3 = np.stack([xi, xi, xi])       # component-independent xi~ makes u1 a Cartesian vector
    base = contract.contract(xyz, w, corr, xi, xig3, sub["G"], sub["rho"], ALL)
    shifted = contract.contract(xyz + np.array([[0.37], [-1.1], [2.3]]), w, corr, xi, xig3,
                                sub["G"], sub["rho"], ALL)
    for k in ("u1", "u3", "D1", "D4", "field"):
        assert np.allclose(shifted[k], base[k], rtol=1e-9, atol=1e-11 * np.abs(base[k]).max())
    q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    rot = contract.contract(q @ xyz, w, corr, xi, xig3, sub["G"], sub["rho"], ALL)
    assert np.allclose(rot["u1"], np.einsum("cd,dmn->cmn", q, base["u1"]), rtol=1e-9,
                       atol=1e-11 * np.abs(base["u1"]).max())
    assert np.allclose(rot["field"], q @ base["field"], rtol=1e-9, atol=1e-12)
    for k in ("u3", "D1", "D4"):
        assert np.allclose(rot[k], base[k], rtol=1e-9, atol=1e-11 * np.abs(base[k]).max())


def test_block_sizes_do_not_change_the_result(sub):
    out = contract.contract(sub["xyz"], sub["w"], sub["corr"], sub["xi"], sub["xig"], sub["G"],
                            sub["rho"], ALL, bra_block=333, ket_block=1024)
    for k in ("u1", "u3", "D1", "D4"):
        assert np.allclose(out[k], sub["out"][k], rtol=1e-11, atol=1e-13 * np.abs(out[k]).max())


@pytest.fixture(scope="module")
def fullrank(h2_tiny):
    wl = h2_tiny
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    w = wl.grid_w
    # enough fused points to span both the scalar (10) and gradient pair spaces
    fp = pivots.select_fused(phi4, w, 40)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    out = contract.contract(wl.grid_xyz, w, wl.corr, fr.xi, fr.xigrad, rho[fp.pivots], rho, ALL)
    return wl, phi4, fp, fr, out


def test_full_rank_isdf_equals_four_index_brute_force(fullrank):
    wl, phi4, fp, fr, out = fullrank
    assert fr.resid_rel.max() < 1e-11
    ref = fourindex.direct(phi4, wl.grid_w, wl.corr, wl.grid_xyz, wl.n_occ)
    got = fourindex.isdf(phi4, fp.pivots, out["u1"], out["u3"], out["D1"], out["D4"])
    # at full rank the fit reproduces every pair product to its residual (~1e-13 here), so
    # the ISDF tensors equal the four-index ones to rounding (measured <= 7.4e-13)
    for k in ("K1", "K3", "T1", "T4"):
        scale = np.abs(ref[k]).max()
        assert np.abs(got[k] - ref[k]).max() < 1e-10 * scale, k
    # particle-exchange symmetry of the symmetrised kernels (I1)
    K = 0.5 * fourindex.p12(ref["K1"] + ref["K3"])
    assert np.allclose(K, K.transpose(1, 0, 3, 2), rtol=1e-12, atol=1e-14)


def test_full_rank_energy_scale_equals_exact(fullrank):
    e = fullrank[4]["escale"]
    assert np.allclose(e[:3], e[3:], rtol=1e-10)


def test_integration_by_parts_to_quadrature_accuracy(h2_tiny):
    """K2 = -K1 - K1swap holds only to quadrature accuracy (the surface terms vanish
    for the exact integrals, not for the grid sums)."""
    from workloads.grid import atom_grid
    wl = h2_tiny
    res = []
    for n_rad, n_ang in ((10, 26), (40, 86)):
        xyz, w = atom_grid(wl.atom_xyz, np.array([0.8, 0.8]), n_rad, n_ang, seed=11)
        res.append(_ibp_defect(wl, xyz, w))
    # the defect is a quadrature error: it shrinks as the grid is refined
    assert res[1] < 0.2 * res[0] and res[1] < 0.01


def _ibp_defect(wl, xyz, w):
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, xyz)
    K = pair_kernels(wl.corr, xyz, xyz, want_lap=True)
    phi = phi4[0]
    ww = w[:, None] * w[None, :]
    # diagonal p = r, q = s elements with the occupied orbital
    p = 0
    lhs = np.einsum("g,gh,gh,h->", phi[p] ** 2, K["lap"], ww, phi[p] ** 2)
    k1 = sum(np.einsum("g,gh,gh,h->", phi[p] * phi4[1 + c, p], K[key], ww, phi[p] ** 2)
             for c, key in enumerate(("gx", "gy", "gz")))
    return abs(lhs + 2.0 * k1) / abs(lhs)
