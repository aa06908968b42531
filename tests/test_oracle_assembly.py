"""Pins of the oracle's four-index assembly (K, dU, W) and the xTC one-body pieces
(dh, f, E0): at full pair rank the ISDF assembly equals the pre-ISDF four-index brute
force; the particle-exchange symmetry; closed matrix forms of the one-body contractions."""
import numpy as np
import pytest

from oracle import assembly, contract, exchange, fit, fourindex, orbitals, pivots

ALL = 1 | 2 | 8 | 16 | 32 | 64


@pytest.fixture(scope="module")
def fullrank(h2_tiny):
    wl = h2_tiny
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    w = wl.grid_w
    fp = pivots.select_fused(phi4, w, 40)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    out = contract.contract(wl.grid_xyz, w, wl.corr, fr.xi, fr.xigrad, rho[fp.pivots], rho, ALL)
    cG = exchange.calG(wl.grid_xyz, w, wl.corr, fr.xi)
    LQ = exchange.density_projector(exchange.occupied_gamma(phi4.shape[1], wl.n_occ))
    x = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, w, LQ)
    ref = fourindex.direct(phi4, w, wl.corr, wl.grid_xyz, wl.n_occ)
    return wl, phi4, fp, fr, out, x, ref


def _close(got, ref, tol):
    scale = np.abs(ref).max()
    assert scale > 0.0
    return np.abs(got - ref).max() <= tol * scale


def test_full_rank_k_and_du_equal_four_index_brute_force(fullrank):
    wl, phi4, fp, fr, out, x, ref = fullrank
    assert fr.resid_rel.max() < 1e-9
    K = assembly.k_tensor(phi4, fp.pivots, out["u1"], out["u3"])
    K1 = ref["K1"]
    Kref = 0.5 * assembly.p12(K1 - K1.transpose(2, 3, 0, 1) + ref["K3"])
    assert _close(K, Kref, 1e-7)
    dU = assembly.du_tensor(phi4, fp.pivots, out["D1"], out["D4"], x["X2"], x["X3"])
    dUref = -assembly.p12(ref["T1"] + ref["T2"] + ref["T3"] + ref["T4"])
    assert _close(dU, dUref, 1e-7)
    # X2, X3 carry a non-negligible part of dU here (the test would miss a dropped term)
    dU_d = assembly.du_tensor(phi4, fp.pivots, out["D1"], out["D4"], None, None)
    assert not _close(dU_d, dUref, 1e-3)


def test_exchange_symmetry_of_the_two_body_corrections(fullrank):
    wl, phi4, fp, fr, out, x, ref = fullrank
    K = assembly.k_tensor(phi4, fp.pivots, out["u1"], out["u3"])
    dU = assembly.du_tensor(phi4, fp.pivots, out["D1"], out["D4"], x["X2"], x["X3"])
    W = assembly.w_tensor(K, dU)
    for T in (K, dU, W):
        assert np.allclose(T, T.transpose(1, 0, 3, 2), rtol=1e-12, atol=1e-14 * np.abs(T).max())
    # the corrections are not Hermitian (stored without symmetrisation)
    assert not np.allclose(K, K.transpose(2, 3, 0, 1), rtol=1e-6, atol=1e-10 * np.abs(K).max())


def test_one_body_pieces_of_an_outer_product_tensor():
    """For T^{pq}_{rs} = a_{pr} b_{qs}: sum_o T^{po}_{qo} = a_{pq} tr_occ(b) and
    sum_o T^{po}_{oq} = (a[:, occ] b[occ, :])_{pq}."""
    rng = np.random.default_rng(5)
    n, n_occ = 7, 3
    a, b = rng.normal(size=(n, n)), rng.normal(size=(n, n))
    T = np.einsum("pr,qs->pqrs", a, b)
    tr = np.trace(b[:n_occ, :n_occ])
    ax = a[:, :n_occ] @ b[:n_occ, :]
    dh = assembly.delta_h(T, n_occ)
    assert np.allclose(dh, -0.5 * (2.0 * a * tr - ax), rtol=1e-13, atol=1e-13)
    c, d = rng.normal(size=(n, n)), rng.normal(size=(n, n))
    W = np.einsum("pr,qs->pqrs", c, d)
    f = assembly.fock_xtc(dh, W, n_occ)
    assert np.allclose(f, dh + 2.0 * c * np.trace(d[:n_occ, :n_occ]) - c[:, :n_occ] @ d[:n_occ, :],
                       rtol=1e-13, atol=1e-13)
    assert assembly.e0_xtc(np.eye(n), n_occ, 1.25) == pytest.approx(-2.0 / 3.0 * n_occ + 1.25)


def test_single_element_form_equals_the_tensors(fullrank):
    """assembly.w_entry (used for sampled checks at large sizes) reproduces the tensor
    assembly element by element."""
    wl, phi4, fp, fr, out, x, ref = fullrank
    K = assembly.k_tensor(phi4, fp.pivots, out["u1"], out["u3"])
    dU = assembly.du_tensor(phi4, fp.pivots, out["D1"], out["D4"], x["X2"], x["X3"])
    W = assembly.w_tensor(K, dU)
    X = x["X2"] + x["X3"]
    Pm = np.ascontiguousarray(phi4[:, :, fp.pivots])
    n = phi4.shape[1]
    rng = np.random.default_rng(8)
    for _ in range(40):
        p, q, r, s = (int(v) for v in rng.integers(n, size=4))
        got = assembly.w_entry(Pm, out["u1"], out["u3"], out["D1"], out["D4"], X, p, q, r, s)
        assert got == pytest.approx(W[p, q, r, s], rel=1e-12, abs=1e-14 * np.abs(W).max())


def test_panel_form_equals_the_tensors(fullrank):
    """assembly.w_panel (the bounded-sample form) reproduces the tensor assembly."""
    wl, phi4, fp, fr, out, x, ref = fullrank
    K = assembly.k_tensor(phi4, fp.pivots, out["u1"], out["u3"])
    dU = assembly.du_tensor(phi4, fp.pivots, out["D1"], out["D4"], x["X2"], x["X3"])
    W = assembly.w_tensor(K, dU)
    Pm = np.ascontiguousarray(phi4[:, :, fp.pivots])
    got = assembly.w_panel(Pm, out["u1"], out["u3"], out["D1"], out["D4"], x["X2"] + x["X3"], 1, 3)
    assert np.abs(got - W[1:3]).max() <= 1e-12 * np.abs(W).max()
