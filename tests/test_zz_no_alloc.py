"""xtc_kernel_contract_noalloc (the contraction without a workspace, for callers that
cannot allocate) against xtc_kernel_contract, through the C ABI: two calls in a row on
the static scratch, the second with a smaller problem (so it runs on the first call's
leftovers), on the FP64 and split paths; a problem whose scratch needs narrower
super-blocks; and one that cannot fit."""
import numpy as np
import pytest

from gpu_common import OracleCase, note

pytestmark = pytest.mark.gpu

CH = 1 | 2 | 8 | 16 | 32 | 64


@pytest.fixture(scope="module")
def cases(h4, h6_small):
    return [OracleCase(h4), OracleCase(h6_small, n_mu=150, subset=4963, seed=3)]


def _inputs(case):
    import torch
    from paper_2607_17314_amd import api
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return (api.DeviceGrid.from_host(case.xyz, case.w), t(case.fit.xi), t(case.fit.xigrad),
            t(case.rho), case.piv)


def _compare(got, ref, bitwise, tol, what):
    for k in ("u1", "u3", "D1", "D4", "field"):
        g, r = got[k], ref[k]
        e = float((g - r).abs().max() / r.abs().max())
        note(f"  {what} {k}: rel err {e:.2e}, bitwise {bool(g.equal(r))}")
        assert e <= tol, k
        if bitwise:
            assert g.equal(r), k
    ee = np.abs(got["escale"] - ref["escale"]) / np.abs(ref["escale"])
    assert ee.max() <= tol
    if bitwise:
        assert np.array_equal(got["escale"], ref["escale"])


@pytest.mark.parametrize("prec", [0, 2])
def test_noalloc_matches_regular_call_twice_in_a_row(cases, prec):
    """Call 1 on the larger problem (H4, 17,200 points, N_mu = 240), call 2 on a smaller
    one (a ragged 4,963-point subset, N_mu = 150) right after it on the same static
    scratch; both fit the scratch at the regular super-block width, so they equal the
    regular call bit for bit."""
    import torch
    from paper_2607_17314_amd import api
    tol = 1e-6 if prec else 1e-12
    for i, case in enumerate(cases):
        grid, xi, xig, rho, piv = _inputs(case)
        note(f"no-alloc call {i + 1}: n_g={case.w.shape[0]} n_mu={len(piv)} precision={prec}")
        got = api.kernel_contract(grid, case.wl.corr, xi, xig, rho, piv, CH, prec, noalloc=True)
        torch.cuda.synchronize()
        ref = api.kernel_contract(grid, case.wl.corr, xi, xig, rho, piv, CH, prec)
        torch.cuda.synchronize()
        _compare(got, ref, True, tol, f"call {i + 1}")


def test_noalloc_narrows_super_blocks_to_fit(h6_small):
    """N_mu = 2000 on the 9,000-point grid needs ~590 MB of panel at the regular width; the
    no-alloc call narrows the super-blocks until its scratch fits, which reorders only the
    stage-2 sums (seeded xi rows: the comparison is of two device paths on one input)."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl = h6_small
    n_mu = 2000
    rng = np.random.default_rng(61)
    piv = np.sort(rng.choice(wl.n_g, n_mu, replace=False))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    xi, xig = t(rng.normal(size=(n_mu, wl.n_g))), t(rng.normal(size=(3, n_mu, wl.n_g)))
    rho = t(rng.random(wl.n_g))
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    need = api.workspace_bytes(L.XTC_CALL_CONTRACT, wl.n_g, 0, n_mu, 0, CH)
    note(f"narrowed: regular workspace {need / 2**20:.0f} MiB, static scratch "
         f"{(256 << 20) / 2**20:.0f} MiB")
    assert need > (256 << 20)
    got = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, CH, L.XTC_FP64, noalloc=True)
    ref = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, CH, L.XTC_FP64)
    torch.cuda.synchronize()
    _compare(got, ref, False, 1e-12, "narrowed")


def test_noalloc_bh_split_narrows_to_fit(cases):
    """The BH form in split precision on H4 (17,200 points): its pair-value buffer (256 KiB
    per bra point of a super-block, 4.3 GB at the regular width) makes the no-alloc call
    narrow the super-blocks; stage 1 is the same per bra point at any width, so only the
    stage-2 sums are reordered."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    from workloads import bh_correlator
    case = cases[0]
    corr = bh_correlator(case.wl.atom_xyz)
    grid, xi, xig, rho, piv = _inputs(case)
    need = api.workspace_bytes(L.XTC_CALL_CONTRACT, case.w.shape[0], 0, len(piv), 0,
                               CH | (L.XTC_SPLIT_F16 << 16) | L.XTC_WS_BH)
    note(f"BH split no-alloc: regular workspace {need / 2**20:.0f} MiB")
    assert need > (256 << 20)
    got = api.kernel_contract(grid, corr, xi, xig, rho, piv, CH, L.XTC_SPLIT_F16, noalloc=True)
    ref = api.kernel_contract(grid, corr, xi, xig, rho, piv, CH, L.XTC_SPLIT_F16)
    torch.cuda.synchronize()
    _compare(got, ref, False, 1e-6, "BH split narrowed")


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    """The split operand of 3072 rows x 194,048 points (2.4 GB) cannot fit: the call returns
    XTC_ERR_NO_WORKSPACE before launching anything."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    from workloads import ee_correlator
    n_g, n_mu = 194000, 3000
    xyz = np.zeros((3, n_g))
    xyz[0] = np.arange(n_g) * 1e-3
    grid = api.DeviceGrid.from_host(xyz, np.ones(n_g))
    xi = torch.empty((n_mu, n_g), dtype=torch.float64, device="cuda")
    rho = torch.zeros(n_g, dtype=torch.float64, device="cuda")
    with pytest.raises(api.XtcError) as ei:
        api.kernel_contract(grid, ee_correlator(), xi, None, rho, np.arange(n_mu), 2 | 8 | 16,
                            L.XTC_SPLIT_F16, noalloc=True)
    note(f"beyond the scratch: {ei.value}")
    assert ei.value.status == L.XTC_ERR_NO_WORKSPACE
