"""xTC Terms 2 and 3 on the GPU (xtc_exchange_terms): the exchange intermediates X2, X3
through the low-rank projector against the oracle's projector form, on a ragged H6 grid
subset (two pair-product chunks, the second ragged) with 150 orbital functions (three
64-orbital blocks, the last ragged) and non-diagonal reference densities of rank 5 and 20."""
import numpy as np
import pytest

from gpu_common import note, rel_err

pytestmark = pytest.mark.gpu

N_SUB = 2300      # bra points: chunks of 2048 + 252
N_MU = 60
N_FUN = 150


@pytest.fixture(scope="module")
def ex_problem(h6_small):
    from oracle import exchange, fit, orbitals, pivots
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(21).choice(wl.n_g, N_SUB, replace=False))
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, N_MU)
    fr = fit.fit(phi4, w, fp.pivots)
    # 150 orbital functions: seeded mixtures of the 60 orbitals (only their pivot values enter)
    mix = np.random.default_rng(22).normal(size=(N_FUN, phi4.shape[1])) / np.sqrt(phi4.shape[1])
    phi = mix @ phi4[0]
    cG = exchange.calG(xyz, w, wl.corr, fr.xi)
    return wl, xyz, w, fp.pivots, fr, phi, cG


def _projector(n_q, seed):
    from oracle import exchange
    rng = np.random.default_rng(seed)
    V = np.linalg.qr(rng.normal(size=(N_FUN, N_FUN)))[0][:, :n_q]
    lam = rng.uniform(0.5, 1.0, n_q)
    return exchange.density_projector((V * lam) @ V.T)


def _run(api, wl, xyz, w, xi, phi_piv, LQ, precision, corr=None):
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(xyz, w)
    out = api.exchange_terms(grid, corr if corr is not None else wl.corr, t(xi), t(phi_piv), t(LQ),
                             precision)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("n_q,precision,tol", [(5, 0, 1e-10), (20, 0, 1e-10), (5, 2, 1e-6),
                                               (20, 2, 1e-6)])
def test_exchange_matches_oracle(ex_problem, n_q, precision, tol):
    from oracle import exchange
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, phi, cG = ex_problem
    LQ = _projector(n_q, 30 + n_q)
    note(f"exchange: n_g={len(w)} n_mu={len(piv)} n_orb={N_FUN} n_q={LQ.shape[1]} "
         f"precision={precision}")
    ref = exchange.x_terms(phi, piv, fr.xi, cG, w, LQ)
    got = _run(api, wl, xyz, w, fr.xi, phi[:, piv], LQ, precision)
    for k in ("X2", "X3"):
        e = rel_err(got[k], ref[k])
        fro = np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])
        note(f"  {k}: rel max err {e:.2e}, rel Frobenius {fro:.2e}")
        assert e < tol and fro < tol, k
        assert np.array_equal(got[k], got[k].transpose(1, 0, 2)), k


def test_exchange_single_output(ex_problem):
    """X3 alone equals the X3 of the joint call, bit for bit."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, phi, cG = ex_problem
    LQ = _projector(4, 41)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(xyz, w)
    both = api.exchange_terms(grid, wl.corr, t(fr.xi), t(phi[:, piv]), t(LQ), L.XTC_FP64)
    only = api.exchange_terms(grid, wl.corr, t(fr.xi), t(phi[:, piv]), t(LQ), L.XTC_FP64,
                              want=("X3",))
    torch.cuda.synchronize()
    assert only["X2"] is None
    assert torch.equal(only["X3"], both["X3"])


def test_exchange_bh_matches_oracle(h6_small):
    """The 48-term Boys-Handy correlator on the FP64 path (900 points, 70 orbital
    functions in two blocks); its split path is refused."""
    import torch
    from oracle import exchange, fit, orbitals, pivots
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    from workloads import bh_correlator
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(23).choice(wl.n_g, 900, replace=False))
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, 40)
    fr = fit.fit(phi4, w, fp.pivots)
    mix = np.random.default_rng(24).normal(size=(70, phi4.shape[1])) / np.sqrt(phi4.shape[1])
    phi = mix @ phi4[0]
    LQ = np.linalg.qr(np.random.default_rng(25).normal(size=(70, 70)))[0][:, :3]
    corr = bh_correlator(wl.atom_xyz)
    ref = exchange.x_terms(phi, fp.pivots, fr.xi, exchange.calG(xyz, w, corr, fr.xi), w, LQ)
    got = _run(api, wl, xyz, w, fr.xi, phi[:, fp.pivots], LQ, L.XTC_FP64, corr=corr)
    for k in ("X2", "X3"):
        e = rel_err(got[k], ref[k])
        note(f"  BH {k}: rel max err {e:.2e}")
        assert e < 1e-10, k
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(xyz, w)
    with pytest.raises(api.XtcError) as ei:
        api.exchange_terms(grid, corr, t(fr.xi), t(phi[:, fp.pivots]), t(LQ), L.XTC_SPLIT_F16)
    assert ei.value.status == L.XTC_ERR_UNSUPPORTED


def test_exchange_bra_ranges_add_up(ex_problem):
    """Partial sums over disjoint bra ranges (a ragged split across a chunk boundary)
    add up to the whole-grid result; an empty range gives zeros."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, phi, cG = ex_problem
    LQ = _projector(3, 43)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(xyz, w)
    args = (grid, wl.corr, t(fr.xi), t(phi[:, piv]), t(LQ), L.XTC_FP64)
    full = api.exchange_terms(*args)
    cut = 1111
    lo = api.exchange_terms(*args, bra=(0, cut))
    hi = api.exchange_terms(*args, bra=(cut, len(w)))
    none = api.exchange_terms(*args, bra=(cut, cut))
    torch.cuda.synchronize()
    for k in ("X2", "X3"):
        e = float((lo[k] + hi[k] - full[k]).abs().max() / full[k].abs().max())
        note(f"  {k}: split-range sum vs whole grid {e:.2e}")
        assert e < 1e-12, k
        assert float(none[k].abs().max()) == 0.0
