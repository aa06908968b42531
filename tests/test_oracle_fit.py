"""Pins of the oracle's ISDF fit (ISDF section: auxiliary basis fitting,
eq. isdf-rho and its normal equations; auxiliary-fit robustness)."""
import numpy as np
import pytest

from oracle import fit, orbitals, pivots


@pytest.fixture(scope="module")
def tiny(h2_tiny):
    phi4 = orbitals.eval_orbitals(h2_tiny.basis, h2_tiny.C_mo, h2_tiny.grid_xyz)
    return h2_tiny, phi4


@pytest.fixture(scope="module")
def small(h6_small):
    phi4 = orbitals.eval_orbitals(h6_small.basis, h6_small.C_mo, h6_small.grid_xyz)
    fp = pivots.select_fused(phi4, h6_small.grid_w, h6_small.n_mu)
    return h6_small, phi4, fp, fit.fit(phi4, h6_small.grid_w, fp.pivots)


def test_interpolation_property(small):
    wl, phi4, fp, fr = small
    n = len(fp.pivots)
    assert np.abs(fr.xi[:, fp.pivots] - np.eye(n)).max() < 1e-9
    for c in range(3):
        assert np.abs(fr.xigrad[c][:, fp.pivots] - np.eye(n)).max() < 1e-9


def test_matches_lstsq_on_explicit_pair_matrix(tiny):
    wl, phi4 = tiny
    st = pivots.pivoted_cholesky(phi4, wl.grid_w, 6, "scalar")
    piv = np.asarray(st.pivots)
    fr = fit.fit(phi4, wl.grid_w, piv)
    phi = phi4[0]
    M = np.einsum("pg,qg->pqg", phi, phi).reshape(-1, wl.n_g)
    Cm = M[:, piv]
    ref, *_ = np.linalg.lstsq(Cm, M, rcond=None)
    assert np.allclose(fr.xi, ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    for c in range(3):
        Mc = np.einsum("pg,qg->pqg", phi, phi4[1 + c]).reshape(-1, wl.n_g)
        refc, *_ = np.linalg.lstsq(Mc[:, piv], Mc, rcond=None)
        assert np.allclose(fr.xigrad[c], refc, rtol=1e-7, atol=1e-8 * np.abs(refc).max())


def test_weighted_residual_equals_cholesky_trace(tiny, small):
    for wl, phi4 in (tiny, small[:2]):
        st = pivots.pivoted_cholesky(phi4, wl.grid_w, 7, "scalar")
        fr = fit.fit(phi4, wl.grid_w, np.asarray(st.pivots), with_grad=False)
        assert np.isclose(fr.resid[0], st.d.sum(), rtol=1e-7)


def test_full_rank_reproduces_every_pair_product(tiny):
    wl, phi4 = tiny
    st = pivots.pivoted_cholesky(phi4, wl.grid_w, 50, "scalar")
    assert st.deficient and len(st.pivots) == 10
    piv = np.asarray(st.pivots)
    fr = fit.fit(phi4, wl.grid_w, piv, with_grad=False)
    phi = phi4[0]
    rho = np.einsum("pg,qg->pqg", phi, phi)
    approx = np.einsum("mg,pqm->pqg", fr.xi, rho[:, :, piv])
    assert np.abs(approx - rho).max() < 1e-10 * np.abs(rho).max()
    assert abs(fr.resid_rel[0]) < 1e-12


def test_jitter_retry_on_singular_gram(tiny):
    wl, phi4 = tiny
    st = pivots.pivoted_cholesky(phi4, wl.grid_w, 10, "scalar")
    rng = np.random.default_rng(5)
    extra = [g for g in rng.permutation(wl.n_g) if g not in st.pivots][:6]
    piv = np.asarray(st.pivots + extra)        # 16 points, pair rank 10: singular Gram
    fr = fit.fit(phi4, wl.grid_w, piv, with_grad=False)
    assert fr.jitter[0] >= 0
    # several xi are correct for a singular Gram: compare the reproduced products
    phi = phi4[0]
    rho = np.einsum("pg,qg->pqg", phi, phi)
    a = np.einsum("mg,pqm->pqg", fr.xi, rho[:, :, piv])
    assert np.abs(a - rho).max() < 1e-6 * np.abs(rho).max()


def test_column_restricted_fit_equals_full_columns(h6_small):
    """The fit is column-separable: solving only some grid columns gives exactly those
    columns of the full solution (xi and xi~ restricted separately)."""
    phi4 = orbitals.eval_orbitals(h6_small.basis, h6_small.C_mo, h6_small.grid_xyz)
    fp = pivots.select_fused(phi4, h6_small.grid_w, 80)
    full = fit.fit(phi4, h6_small.grid_w, fp.pivots)
    cols = np.arange(1000, 1700)
    gcols = np.arange(4000, 4123)
    part = fit.fit(phi4, h6_small.grid_w, fp.pivots, cols=cols, grad_cols=gcols)
    assert np.allclose(part.xi, full.xi[:, cols], rtol=0, atol=1e-12 * np.abs(full.xi).max())
    assert np.allclose(part.xigrad, full.xigrad[:, :, gcols], rtol=0,
                       atol=1e-12 * np.abs(full.xigrad).max())
    assert np.array_equal(part.jitter, full.jitter)
