"""Pins of the oracle's correlators and analytic derivatives (eqs. bh-scaled
and bh-u): closed forms at r12 = 0, exchange symmetry and finite differences."""
import numpy as np
import pytest

from oracle.correlator import pair_kernels, u_value
from workloads import Correlator, FORM_EE, bh_correlator, ee_correlator


def _pts(n, seed, scale=2.0):
    return np.random.default_rng(seed).normal(size=(3, n)) * scale


CORRS = {
    "ee": ee_correlator(),
    "ee_odd": Correlator(FORM_EE, np.array([[0, 0, 1], [0, 0, 2], [0, 0, 3]], np.int32),
                         np.array([[0.5, -0.3, 0.2]]), 1.3),
    "bh": bh_correlator(np.array([[0.0, 0.0, -1.0], [0.2, 0.1, 1.1], [-0.5, 0.4, 2.3]])),
}


def test_closed_forms_at_coincidence():
    corr = CORRS["ee"]
    X = _pts(7, 1)
    K = pair_kernels(corr, X, X, want_lap=True)
    for k in ("gx", "gy", "gz", "sq"):
        assert np.all(np.diag(K[k]) == 0.0)
    # lap u(g, g) = 6 c_1 d^2 for u = sum c_k rbar^{2k}
    assert np.allclose(np.diag(K["lap"]), 6.0 * corr.c[0, 0] * corr.d ** 2, rtol=1e-13)
    # o = 1 convention: vector dropped, square keeps u'(0)^2 = (c d)^2, Laplacian drops the term
    co = CORRS["ee_odd"]
    K = pair_kernels(co, X, X, want_lap=True)
    assert np.all(np.diag(K["gx"]) == 0.0)
    assert np.allclose(np.diag(K["sq"]), (0.5 * 1.3) ** 2)
    assert np.allclose(np.diag(K["lap"]), 6.0 * (-0.3) * 1.3 ** 2)


@pytest.mark.parametrize("name", ["ee", "ee_odd", "bh"])
def test_exchange_symmetry(name):
    corr = CORRS[name]
    X1, X2 = _pts(5, 2), _pts(6, 3)
    assert np.allclose(u_value(corr, X1, X2), u_value(corr, X2, X1).T, rtol=1e-13)
    if corr.form == FORM_EE:
        K12 = pair_kernels(corr, X1, X2)
        K21 = pair_kernels(corr, X2, X1)
        for k in ("gx", "gy", "gz"):
            assert np.allclose(K12[k], -K21[k].T, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("name", ["ee", "ee_odd", "bh"])
def test_gradient_matches_central_differences(name):
    corr = CORRS[name]
    X1, X2 = _pts(6, 4), _pts(5, 5)
    K = pair_kernels(corr, X1, X2)
    h = 1e-5
    for c, key in enumerate(("gx", "gy", "gz")):
        e = np.zeros((3, 1))
        e[c] = h
        fd = (u_value(corr, X1 + e, X2) - u_value(corr, X1 - e, X2)) / (2 * h)
        assert np.abs(fd - K[key]).max() < 1e-8
    sq = K["gx"] ** 2 + K["gy"] ** 2 + K["gz"] ** 2
    assert np.allclose(sq, K["sq"], rtol=1e-12)


@pytest.mark.parametrize("name", ["ee", "ee_odd"])
def test_laplacian_matches_divergence_of_gradient(name):
    corr = CORRS[name]
    X1, X2 = _pts(6, 6), _pts(5, 7)
    K = pair_kernels(corr, X1, X2, want_lap=True)
    h = 1e-4
    div = np.zeros_like(K["lap"])
    for c, key in enumerate(("gx", "gy", "gz")):
        e = np.zeros((3, 1))
        e[c] = h
        div += (pair_kernels(corr, X1 + e, X2)[key] - pair_kernels(corr, X1 - e, X2)[key]) / (2 * h)
    assert np.abs(div - K["lap"]).max() < 1e-7


def test_linear_in_coefficients():
    corr = CORRS["bh"]
    X1, X2 = _pts(4, 8), _pts(4, 9)
    K = pair_kernels(corr, X1, X2)
    K2 = pair_kernels(corr.with_c(2.0 * corr.c), X1, X2)
    assert np.allclose(K2["gx"], 2 * K["gx"], rtol=1e-13)
    assert np.allclose(K2["sq"], 4 * K["sq"], rtol=1e-13)
