"""Pins of the oracle's xTC Terms 2 and 3 (exchange intermediates X2, X3): the literal
and low-rank-projector forms agree, X is symmetric in its orbital pair, the full-rank
ISDF terms equal the pre-ISDF four-index brute force, and X is quadratic in c."""
import numpy as np
import pytest

from oracle import exchange, fit, fourindex, orbitals, pivots


@pytest.fixture(scope="module")
def fullrank(h2_tiny):
    wl = h2_tiny
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    w = wl.grid_w
    fp = pivots.select_fused(phi4, w, 40)
    fr = fit.fit(phi4, w, fp.pivots)
    cG = exchange.calG(wl.grid_xyz, w, wl.corr, fr.xi)
    return wl, phi4, fp, fr, cG


def test_projector_form_equals_direct_form(fullrank):
    wl, phi4, fp, fr, cG = fullrank
    gam = exchange.occupied_gamma(phi4.shape[1], wl.n_occ)
    d = exchange.x_terms_direct(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, gam)
    p = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, exchange.density_projector(gam))
    for k in ("X2", "X3"):
        assert np.abs(p[k] - d[k]).max() <= 1e-12 * np.abs(d[k]).max(), k
    # a non-diagonal reference density: the projector is its square-root factor
    rng = np.random.default_rng(3)
    V = np.linalg.qr(rng.normal(size=(phi4.shape[1], phi4.shape[1])))[0][:, :wl.n_occ]
    gam2 = V @ V.T
    d2 = exchange.x_terms_direct(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, gam2)
    p2 = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, exchange.density_projector(gam2))
    for k in ("X2", "X3"):
        assert np.abs(p2[k] - d2[k]).max() <= 1e-12 * np.abs(d2[k]).max(), k


def test_x_is_symmetric_in_the_orbital_pair(fullrank):
    wl, phi4, fp, fr, cG = fullrank
    LQ = exchange.density_projector(exchange.occupied_gamma(phi4.shape[1], wl.n_occ))
    x = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, LQ)
    for k in ("X2", "X3"):
        assert np.allclose(x[k], x[k].transpose(1, 0, 2), rtol=1e-12, atol=1e-15 * np.abs(x[k]).max())
    # X31 alone is not symmetric; X32 is its transpose in (q, s)
    gam = exchange.occupied_gamma(phi4.shape[1], wl.n_occ)
    d = exchange.x_terms_direct(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, gam)
    assert np.allclose(d["X32"], d["X31"].transpose(1, 0, 2), rtol=1e-12,
                       atol=1e-15 * np.abs(d["X31"]).max())


def test_full_rank_isdf_terms_equal_four_index_brute_force(fullrank):
    wl, phi4, fp, fr, cG = fullrank
    assert fr.resid_rel.max() < 1e-9
    ref = fourindex.direct(phi4, wl.grid_w, wl.corr, wl.grid_xyz, wl.n_occ)
    LQ = exchange.density_projector(exchange.occupied_gamma(phi4.shape[1], wl.n_occ))
    x = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, LQ)
    got = exchange.terms23_isdf(phi4[0], fp.pivots, x["X2"], x["X3"])
    for k in ("T2", "T3"):
        scale = np.abs(ref[k]).max()
        assert scale > 0.0
        assert np.abs(got[k] - ref[k]).max() < 1e-7 * scale, k


def test_x_is_quadratic_in_the_correlator(fullrank):
    wl, phi4, fp, fr, cG = fullrank
    LQ = exchange.density_projector(exchange.occupied_gamma(phi4.shape[1], wl.n_occ))
    x1 = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, wl.grid_w, LQ)
    cG2 = exchange.calG(wl.grid_xyz, wl.grid_w, wl.corr.with_c(2.0 * wl.corr.c), fr.xi)
    x2 = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG2, wl.grid_w, LQ)
    for k in ("X2", "X3"):
        assert np.allclose(x2[k], 4.0 * x1[k], rtol=1e-11, atol=1e-14 * np.abs(x1[k]).max())
    z = exchange.calG(wl.grid_xyz, wl.grid_w, wl.corr.with_c(0.0 * wl.corr.c), fr.xi)
    x0 = exchange.x_terms(phi4[0], fp.pivots, fr.xi, z, wl.grid_w, LQ)
    assert not np.any(x0["X2"]) and not np.any(x0["X3"])


def test_bra_range_of_calG_and_x_is_the_restricted_sum(fullrank):
    """calG over a bra range equals those columns of the whole-grid calG, and X over
    two complementary bra ranges adds up to the whole-grid X."""
    wl, phi4, fp, fr, cG = fullrank
    w, n = wl.grid_w, wl.grid_w.shape[0]
    cut = n // 3
    part = exchange.calG(wl.grid_xyz, w, wl.corr, fr.xi, bra=(cut, n))
    assert np.abs(part - cG[:, :, cut:]).max() <= 1e-14 * np.abs(cG).max()
    LQ = exchange.density_projector(exchange.occupied_gamma(phi4.shape[1], wl.n_occ))
    whole = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, w, LQ)
    a = exchange.x_terms(phi4[0], fp.pivots, fr.xi[:, :cut], cG[:, :, :cut], w[:cut], LQ)
    b = exchange.x_terms(phi4[0], fp.pivots, fr.xi[:, cut:], part, w[cut:], LQ)
    for k in ("X2", "X3"):
        assert np.abs(a[k] + b[k] - whole[k]).max() <= 1e-12 * np.abs(whole[k]).max(), k
