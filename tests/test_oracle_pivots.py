"""Pins of the oracle's pivoted Cholesky (Alg. 1; matrix-free pivot search)
and of the fill-to-target pivot fusion."""
import numpy as np
import pytest
from scipy.linalg import qr

from oracle import orbitals, pivots


def _pair_matrix(phi4, w, channel):
    """Explicit weighted pair matrix M_w whose Gram is the channel's S."""
    phi = phi4[0]
    if channel == "scalar":
        M = np.einsum("pg,qg->pqg", phi, phi).reshape(-1, phi.shape[1])
    else:
        M = np.einsum("pg,cqg->pcqg", phi, phi4[1:4]).reshape(-1, phi.shape[1])
    return M * w[None, :]


@pytest.fixture(scope="module")
def tiny_phi(h2_tiny):
    return orbitals.eval_orbitals(h2_tiny.basis, h2_tiny.C_mo, h2_tiny.grid_xyz)


@pytest.mark.parametrize("channel", ["scalar", "grad"])
def test_pivots_equal_lapack_qrcp(tiny_phi, h2_tiny, channel):
    w = h2_tiny.grid_w
    M = _pair_matrix(tiny_phi, w, channel)
    _, _, perm = qr(M, pivoting=True, mode="economic")
    st = pivots.pivoted_cholesky(tiny_phi, w, 40, channel)
    n = len(st.pivots)
    # compare while the greedy choice is well separated (near-tie rule)
    upto = next((i for i, gap in enumerate(st.gaps) if gap < 1e-8), n)
    assert upto >= 5
    assert list(perm[:upto]) == st.pivots[:upto]


@pytest.mark.parametrize("channel", ["scalar", "grad"])
def test_residual_trace_is_projection_residual(tiny_phi, h2_tiny, channel):
    w = h2_tiny.grid_w
    M = _pair_matrix(tiny_phi, w, channel)
    for k in (1, 3, 6):
        st = pivots.pivoted_cholesky(tiny_phi, w, k, channel)
        Q, _ = np.linalg.qr(M[:, st.pivots])
        R = M - Q @ (Q.T @ M)
        assert np.isclose(st.d.sum(), np.sum(R * R), rtol=1e-9, atol=1e-14 * np.sum(M * M))
        # the Cholesky columns reproduce S on the pivot columns
        Lm = np.asarray(st.L)
        S_cols = (M.T @ M)[:, st.pivots]
        assert np.allclose(Lm.T @ Lm[:, st.pivots], S_cols, rtol=1e-9, atol=1e-12 * np.abs(S_cols).max())


def test_pivot_values_nonincreasing_and_stop_at_rank(tiny_phi, h2_tiny):
    w = h2_tiny.grid_w
    M = _pair_matrix(tiny_phi, w, "scalar")
    sv = np.linalg.svd(M, compute_uv=False)
    rank = int(np.sum(sv > 1e-7 * sv[0]))
    st = pivots.pivoted_cholesky(tiny_phi, w, 60, "scalar")
    v = np.asarray(st.pivot_values)
    assert np.all(np.diff(v) <= 1e-12 * v[0])
    assert st.deficient
    assert len(st.pivots) == rank == 10     # 4 orbitals: 4*5/2 distinct pair products
    assert len(set(st.pivots)) == len(st.pivots)


def test_diagonal_matches_explicit(tiny_phi, h2_tiny):
    w = h2_tiny.grid_w
    for ch in ("scalar", "grad"):
        M = _pair_matrix(tiny_phi, w, ch)
        assert np.allclose(pivots.diagonal(tiny_phi, w, ch), np.sum(M * M, axis=0), rtol=1e-12)
        g = 17
        assert np.allclose(pivots.column(tiny_phi, w, g, ch), M.T @ M[:, g], rtol=1e-12, atol=1e-300)


def test_fusion_fill_to_target(h6_small):
    phi4 = orbitals.eval_orbitals(h6_small.basis, h6_small.C_mo, h6_small.grid_xyz)
    fp = pivots.select_fused(phi4, h6_small.grid_w, 120)
    assert len(fp.pivots) == 120 and len(set(fp.pivots.tolist())) == 120
    assert len(fp.grad) == 60
    ns = len(fp.scalar)
    assert fp.pivots[:ns].tolist() == fp.scalar
    assert fp.pivots[ns:].tolist() == [g for g in fp.grad if g not in set(fp.scalar)]
    # the last scalar pivot is the one that completed the union
    assert fp.scalar[-1] not in set(fp.grad)
    # independence from the correlator: pivots depend on orbitals and weights only
    fp2 = pivots.select_fused(phi4, h6_small.grid_w, 120)
    assert np.array_equal(fp.pivots, fp2.pivots)
