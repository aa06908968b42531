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
    return wl, xyz, w, fp.pivots, fr, phi, cG, orbitals.density(phi4, wl.n_occ)


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
    wl, xyz, w, piv, fr, phi, cG, rho = ex_problem
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
    wl, xyz, w, piv, fr, phi, cG, rho = ex_problem
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
    wl, xyz, w, piv, fr, phi, cG, rho = ex_problem
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


@pytest.mark.parametrize("precision", [0, 2])
def test_fused_contraction_pass_gives_the_same_x(ex_problem, precision):
    """X2, X3 formed inside xtc_kernel_contract from its own calG panels equal the
    standalone call's, bit for bit, and the contraction outputs are unchanged."""
    import torch
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, phi, cG, rho = ex_problem
    LQ = _projector(6, 44)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(xyz, w)
    ch = 1 | 2 | 8 | 16 | 32 | 64
    xi, xig, rh = t(fr.xi), t(fr.xigrad), t(rho)
    alone = api.exchange_terms(grid, wl.corr, xi, t(phi[:, piv]), t(LQ), precision)
    plain = api.kernel_contract(grid, wl.corr, xi, xig, rh, piv, ch, precision)
    fused = api.kernel_contract(grid, wl.corr, xi, xig, rh, piv, ch, precision,
                                exchange={"phi_piv": t(phi[:, piv]), "lq": t(LQ)})
    torch.cuda.synchronize()
    for k in ("X2", "X3"):
        assert torch.equal(fused[k], alone[k]), k
    for k in ("u1", "u3", "D1", "D4", "field"):
        assert torch.equal(fused[k], plain[k]), k
    assert np.array_equal(fused["escale"], plain["escale"])


@pytest.fixture(scope="module")
def h20_exchange():
    """The H20 grid (194,000 points) with N_mu = 3000 seeded interpolation vectors,
    300 orbital functions at the pivots and the closed-shell projector of 10
    occupied orbitals: the shapes the benchmark runs."""
    from workloads import make_config
    wl = make_config("h20")
    rng = np.random.default_rng(52)
    xi = rng.standard_normal((wl.n_mu, wl.n_g))
    phi_piv = rng.standard_normal((wl.n_orb, wl.n_mu)) / np.sqrt(wl.n_orb)
    LQ = np.zeros((wl.n_orb, wl.n_occ))
    LQ[np.arange(wl.n_occ), np.arange(wl.n_occ)] = 1.0
    return wl, xi, phi_piv, LQ


H20_BRA = (70001, 72101)    # a 2048-point chunk and a 52-point tail


def test_full_size_fp64_exchange_on_a_bra_range_matches_oracle(h20_exchange):
    """FP64 X2, X3 at the full H20 shape over a ragged bra range against the oracle's
    restricted sums (calG of those bra points over all 194,000 ket points)."""
    import torch
    from oracle import exchange
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, xi, phi_piv, LQ = h20_exchange
    b0, b1 = H20_BRA
    note(f"h20 exchange: bra range [{b0}, {b1}), n_mu={wl.n_mu}, n_orb={wl.n_orb}, n_q={LQ.shape[1]}")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    got = api.exchange_terms(grid, wl.corr, t(xi), t(phi_piv), t(LQ), L.XTC_FP64, bra=(b0, b1))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    note("  oracle calG over the bra range")
    cG = exchange.calG(wl.grid_xyz, wl.grid_w, wl.corr, xi, bra=(b0, b1))
    # the oracle's x_terms reads phi only at the pivots: pass phi_piv as the "grid" values
    note("  oracle X over the bra range")
    ref = exchange.x_terms(phi_piv, np.arange(wl.n_mu), xi[:, b0:b1], cG, wl.grid_w[b0:b1], LQ)
    for k in ("X2", "X3"):
        e = rel_err(got[k], ref[k])
        fro = np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k])
        note(f"  {k}: rel max err {e:.2e}, rel Frobenius {fro:.2e}")
        assert e < 1e-10 and fro < 1e-10, k


@pytest.fixture(scope="module")
def h20_fitted():
    """The H20 workload's own interpolation vectors (orbitals, fused pivots and fit on
    the device): the value structure the split bound is stated for."""
    import torch
    from paper_2607_17314_amd import api
    from workloads import make_config
    wl = make_config("h20")
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    phi4, rho = api.eval_orbitals(wl.basis, grid, torch.as_tensor(wl.C_mo).cuda(), wl.n_occ)
    piv, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ)
    xi, xig, _, _ = api.fit(phi4, grid, piv)
    phi_piv = phi4[0][:, torch.as_tensor(piv, device="cuda")].contiguous()
    lq = torch.zeros((wl.n_orb, wl.n_occ), dtype=torch.float64, device="cuda")
    lq[torch.arange(wl.n_occ), torch.arange(wl.n_occ)] = 1.0
    del phi4
    return wl, grid, xi, xig, rho, piv, phi_piv, lq


def test_full_size_split_exchange_vs_fp64(h20_fitted):
    """Split vs FP64 X2, X3 at the full H20 size on the workload's fitted interpolation
    vectors, over a ragged bra range."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, grid, xi, xig, rho, piv, phi_piv, lq = h20_fitted
    note(f"h20 fitted: split vs fp64 exchange over {H20_BRA}")
    f = api.exchange_terms(grid, wl.corr, xi, phi_piv, lq, L.XTC_FP64, bra=H20_BRA)
    s = api.exchange_terms(grid, wl.corr, xi, phi_piv, lq, L.XTC_SPLIT_F16, bra=H20_BRA)
    torch.cuda.synchronize()
    for k in ("X2", "X3"):
        e = float((s[k] - f[k]).abs().max() / f[k].abs().max())
        fro = float(torch.linalg.norm(s[k] - f[k]) / torch.linalg.norm(f[k]))
        note(f"  {k}: split vs fp64 rel max err {e:.2e}, rel Frobenius {fro:.2e}")
        assert e < 1e-6 and fro < 1e-6, k


def test_full_size_fused_pass_equals_standalone(h20_fitted):
    """At the full H20 size, X from the fused contraction pass equals the standalone
    call over the whole grid bit for bit, and X is symmetric in its orbital pair."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, grid, xi, xig, rho, piv, phi_piv, lq = h20_fitted
    note("h20: fused contraction + exchange")
    fused = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, 1 | 2 | 8 | 16, L.XTC_SPLIT_F16,
                                exchange={"phi_piv": phi_piv, "lq": lq})
    note("h20: standalone exchange")
    alone = api.exchange_terms(grid, wl.corr, xi, phi_piv, lq, L.XTC_SPLIT_F16)
    torch.cuda.synchronize()
    for k in ("X2", "X3"):
        assert torch.equal(fused[k], alone[k]), k
        assert torch.equal(fused[k], fused[k].transpose(0, 1)), k
        assert bool(torch.isfinite(fused[k]).all()), k


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (2, 1e-6)])
def test_exchange_matches_literal_direct_form(h6_small, precision, tol):
    """X2, X3 against the paper's literal Y, Z, Lt, Ch form (x_terms_direct, no projector)
    on a small case: 700 points, 40 interpolation points, 40 orbital functions, a
    non-diagonal reference density of rank 7."""
    from oracle import exchange, fit, orbitals, pivots
    from paper_2607_17314_amd import api
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(24).choice(wl.n_g, 700, replace=False))
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, 40)
    fr = fit.fit(phi4, w, fp.pivots)
    n_fun = 40
    mix = np.random.default_rng(25).normal(size=(n_fun, phi4.shape[1])) / np.sqrt(phi4.shape[1])
    phi = mix @ phi4[0]
    rng = np.random.default_rng(26)
    V = np.linalg.qr(rng.normal(size=(n_fun, n_fun)))[0][:, :7]
    gamma = (V * rng.uniform(0.5, 1.0, 7)) @ V.T
    cG = exchange.calG(xyz, w, wl.corr, fr.xi)
    ref = exchange.x_terms_direct(phi, fp.pivots, fr.xi, cG, w, gamma)
    LQ = exchange.density_projector(gamma)
    note(f"exchange vs literal form: n_g={len(w)} n_mu={len(fp.pivots)} n_orb={n_fun} "
         f"n_q={LQ.shape[1]} precision={precision}")
    got = _run(api, wl, xyz, w, fr.xi, phi[:, fp.pivots], LQ, precision)
    for k in ("X2", "X3"):
        e = rel_err(got[k], ref[k])
        note(f"  {k}: rel max err {e:.2e}")
        assert e < tol, k
