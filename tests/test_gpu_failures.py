"""Failure and warning paths of the boundary, forced from the host with valid launches:
rejected weights (negative, NaN, infinite) before any stage runs; Alg. 1's stop at the
pair rank (XTC_WARN_RANK_DEFICIENT); the auxiliary fit's Tikhonov retry
(XTC_WARN_JITTER when every orbital vanishes at one pivot) and its failure (XTC_ERR_NOT_SPD when every
orbital vanishes at the pivots, so that the Gram matrix and every shift are zero).
The oracle takes the same decisions on the same inputs."""
import numpy as np
import pytest

from gpu_common import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny(h2_tiny):
    import torch
    from oracle import fit, orbitals, pivots
    from paper_2607_17314_amd import api
    wl = h2_tiny
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    fp = pivots.select_fused(phi4, wl.grid_w, 8)
    fr = fit.fit(phi4, wl.grid_w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return dict(wl=wl, phi4=phi4, piv=fp.pivots, fr=fr, rho=rho, t=t, api=api)


@pytest.mark.parametrize("bad", [-1e-3, float("nan"), float("inf")])
def test_bad_weights_are_rejected_before_any_stage(tiny, bad):
    import torch
    from paper_2607_17314_amd import _lib as L
    api, wl, t = tiny["api"], tiny["wl"], tiny["t"]
    w = wl.grid_w.copy()
    w[123] = bad
    grid = api.DeviceGrid.from_host(wl.grid_xyz, w)
    phi4, xi, xig, rho = t(tiny["phi4"]), t(tiny["fr"].xi), t(tiny["fr"].xigrad), t(tiny["rho"])
    piv = tiny["piv"]
    n = len(piv)
    calls = {
        "isdf_select_points": lambda: api.select_points(phi4, grid, 6, wl.n_occ),
        "isdf_fit": lambda: api.fit(phi4, grid, piv),
        "xtc_kernel_contract": lambda: api.kernel_contract(grid, wl.corr, xi, xig, rho, piv),
        "xtc_grad": lambda: api.grad(grid, wl.corr, xi, xig, rho, piv,
                                     {"u3": torch.ones((n, n), dtype=torch.float64, device="cuda")}),
        "xtc_exchange_terms": lambda: api.exchange_terms(grid, wl.corr, xi, phi4[0][:, piv].contiguous(),
                                                         torch.eye(4, 1, dtype=torch.float64,
                                                                   device="cuda").contiguous()),
        "xtc_mlp_features": lambda: api.features(phi4, grid, wl.n_occ, wl.atom_xyz),
    }
    for name, call in calls.items():
        with pytest.raises(api.XtcError) as ei:
            call()
        assert ei.value.status == L.XTC_ERR_INVALID_ARG, name
        assert "weights" in str(ei.value), name
        note(f"  {name} with weight {bad}: {ei.value}")
    torch.cuda.synchronize()
    # a zero weight is valid (Becke partitions underflow to 0)
    w[123] = 0.0
    api.fit(phi4, api.DeviceGrid.from_host(wl.grid_xyz, w), piv)


def test_rank_deficiency_is_reported(tiny):
    """Asking for more points than the pair products span: Alg. 1 stops at the rank with
    XTC_WARN_RANK_DEFICIENT, and the points equal the oracle's."""
    from oracle import pivots
    from paper_2607_17314_amd import _lib as L
    api, wl, t = tiny["api"], tiny["wl"], tiny["t"]
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    ref = pivots.select_fused(tiny["phi4"], wl.grid_w, 40)
    assert ref.deficient
    piv, info, st = api.select_points(t(tiny["phi4"]), grid, 40, wl.n_occ)
    note(f"rank deficiency: device {len(piv)} points (scalar {info[0]:.0f}, gradient {info[1]:.0f}), "
         f"oracle {len(ref.pivots)} (scalar {len(ref.scalar)}, gradient {len(ref.grad)})")
    assert st == L.XTC_WARN_RANK_DEFICIENT
    assert len(piv) < 40
    assert np.array_equal(piv, ref.pivots)


def test_orbital_free_pivot_takes_the_tikhonov_retry(tiny):
    """All orbitals vanishing at one pivot give its Gram row and column exactly zero, so the
    unshifted Cholesky fails in every system and the first shift (k = 0) restores positive
    definiteness: XTC_WARN_JITTER with k = 0 for the scalar and the three gradient systems,
    the oracle's choice too; the fit then reproduces the pair products as well as the other
    pivots alone do."""
    from oracle import fit
    from paper_2607_17314_amd import _lib as L
    api, wl, t = tiny["api"], tiny["wl"], tiny["t"]
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    piv = np.asarray(tiny["piv"])
    phi4 = tiny["phi4"].copy()
    phi4[:, :, piv[2]] = 0.0
    xi, xig, info, st = api.fit(t(phi4), grid, piv)
    ref = fit.fit(phi4, wl.grid_w, piv)
    note(f"orbital-free pivot: status {st}, shift indices {info[:4]} (oracle {ref.jitter}), "
         f"residuals {info[4:]} (oracle {ref.resid_rel})")
    assert st == L.XTC_WARN_JITTER
    assert np.array_equal(info[:4], [0, 0, 0, 0]) and np.array_equal(ref.jitter, [0, 0, 0, 0])
    assert np.all(np.abs(info[4:] - ref.resid_rel) <= 1e-9 + 1e-9 * np.abs(ref.resid_rel))
    assert bool(np.isfinite(xi.cpu().numpy()).all() and np.isfinite(xig.cpu().numpy()).all())


def test_duplicated_pivot_is_singular_only_up_to_rounding(tiny):
    """A duplicated pivot makes the Gram matrix singular in exact arithmetic; in floating
    point the last Cholesky pivot is a rounding-level number of either sign, so some systems
    may need a shift (XTC_WARN_JITTER) and others not. Either way the fit reproduces the
    pair products as well as the pivots without the duplicate."""
    from oracle import fit
    from paper_2607_17314_amd import _lib as L
    api, wl, t = tiny["api"], tiny["wl"], tiny["t"]
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    piv = np.asarray(tiny["piv"])
    dup = np.concatenate([piv, piv[2:3]])
    xi, xig, info, st = api.fit(t(tiny["phi4"]), grid, dup)
    note(f"duplicated pivot: status {st}, shift indices {info[:4]}, residuals {info[4:]}")
    assert st in (L.XTC_OK, L.XTC_WARN_JITTER)
    assert (st == L.XTC_WARN_JITTER) == bool(np.any(info[:4] >= 0))
    base = fit.fit(tiny["phi4"], wl.grid_w, piv)
    assert np.all(np.abs(info[4:] - base.resid_rel) <= 1e-6 + 1e-6 * np.abs(base.resid_rel))


def test_vanishing_orbitals_fail_with_not_spd(tiny):
    """Orbitals that vanish at every pivot give a zero Gram matrix, whose mean diagonal
    makes every Tikhonov shift zero: the fit fails with XTC_ERR_NOT_SPD, as the oracle's
    does (LinAlgError)."""
    import torch
    from scipy.linalg import LinAlgError
    from oracle import fit
    from paper_2607_17314_amd import _lib as L
    api, wl, t = tiny["api"], tiny["wl"], tiny["t"]
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    phi4 = tiny["phi4"].copy()
    piv = np.asarray(tiny["piv"])
    phi4[:, :, piv] = 0.0
    with pytest.raises(LinAlgError):
        fit.fit(phi4, wl.grid_w, piv)
    with pytest.raises(api.XtcError) as ei:
        api.fit(t(phi4), grid, piv)
    note(f"vanishing orbitals: {ei.value}")
    assert ei.value.status == L.XTC_ERR_NOT_SPD
    torch.cuda.synchronize()
