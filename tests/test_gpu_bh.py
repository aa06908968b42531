"""The multi-centre Boys-Handy correlator (eq. bh-u, 48 terms) on the GPU: the FP64 and
split-precision contractions against the oracle on a ragged H6 grid subset, the adjoint,
and the combinations the split path refuses."""
import numpy as np
import pytest

from gpu_common import note, rel_err

pytestmark = pytest.mark.gpu

CH = 1 | 2 | 8 | 16 | 32 | 64   # u1, u3, D1, D4, field, escale (no Laplacian for BH)
TOL = 1e-10


@pytest.fixture(scope="module")
def bh_problem(h6_small):
    from oracle import fit, orbitals, pivots
    from workloads import bh_correlator
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(7).choice(wl.n_g, 1100, replace=False))   # ragged size
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, 60)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    corr = bh_correlator(wl.atom_xyz)
    return wl, xyz, w, fp.pivots, fr, rho, corr


def _device(api, xyz, w, fr, rho):
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return api.DeviceGrid.from_host(xyz, w), t(fr.xi), t(fr.xigrad), t(rho)


def test_bh_contract_matches_oracle(bh_problem):
    import torch
    from oracle import contract
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr = bh_problem
    note(f"BH contract: n_g={w.shape[0]} n_mu={len(piv)} nuclei={corr.nuc_xyz.shape[0]} "
         f"terms={corr.n_terms}")
    ref = contract.contract(xyz, w, corr, fr.xi, fr.xigrad, rho[piv], rho, CH)
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    out = api.kernel_contract(grid, corr, xi, xig, rh, piv, CH)
    torch.cuda.synchronize()
    for k in ("u1", "u3", "D1", "D4", "field"):
        e = rel_err(out[k].cpu().numpy(), ref[k])
        note(f"  {k}: rel err {e:.2e}")
        assert e < TOL, k
    e = np.max(np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"]))
    note(f"  escale rel err {e:.2e}; {out['escale']}")
    assert e < TOL


@pytest.mark.parametrize("types", [1, 2])
def test_bh_split_matches_oracle(bh_problem, types):
    """Split precision (pair values generated in FP64, stored as FP16 pairs, split MFMA
    products) on the ragged 1,100-point grid: 35 bra tiles (the last of 12 points), ten ket
    chunks in two generation groups. Within the mixed path's 1e-6 of the oracle per block;
    the density rows come from the FP64 pair values, so the field stays within 1e-10; the
    split result is also within 1e-6 of the device's FP64 form."""
    import torch
    from oracle import contract
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr = bh_problem
    if types == 2:
        corr = _two_type(corr)
    ref = contract.contract(xyz, w, corr, fr.xi, fr.xigrad, rho[piv], rho, CH)
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    out = api.kernel_contract(grid, corr, xi, xig, rh, piv, CH, precision=L.XTC_SPLIT_F16)
    f64 = api.kernel_contract(grid, corr, xi, xig, rh, piv, CH)
    torch.cuda.synchronize()
    note(f"BH split contract, {types} type(s): n_g={w.shape[0]} n_mu={len(piv)}")
    for k in ("u1", "u3", "D1", "D4", "field"):
        e = rel_err(out[k].cpu().numpy(), ref[k])
        ed = float((out[k] - f64[k]).abs().max() / f64[k].abs().max())
        note(f"  {k}: vs oracle {e:.2e}, vs FP64 device {ed:.2e}")
        assert e < (1e-10 if k == "field" else 1e-6), k
        assert ed < (1e-10 if k == "field" else 1e-6), k
    e = np.max(np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"]))
    note(f"  escale rel err {e:.2e}")
    assert e < 1e-6


def test_bh_split_exchange_outputs_are_refused(bh_problem):
    """The BH form's exchange intermediates are formed on the FP64 path only."""
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr = bh_problem
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    n_orb, n_mu = wl.n_orb, len(piv)
    ex = {"phi_piv": torch.zeros((n_orb, n_mu), dtype=torch.float64, device="cuda"),
          "lq": torch.eye(n_orb, wl.n_occ, dtype=torch.float64, device="cuda")}
    with pytest.raises(api.XtcError) as ei:
        api.kernel_contract(grid, corr, xi, xig, rh, piv, CH, precision=L.XTC_SPLIT_F16,
                            exchange=ex)
    assert ei.value.status == L.XTC_ERR_UNSUPPORTED
    with pytest.raises(api.XtcError) as ei:
        api.kernel_contract(grid, corr, xi, xig, rh, piv, CH | L.XTC_ULAP,
                            precision=L.XTC_SPLIT_F16)
    assert ei.value.status == L.XTC_ERR_UNSUPPORTED


def _two_type(corr):
    """The same 48 terms on alternating nucleus types with distinct b and c."""
    from workloads import Correlator
    n = corr.nuc_xyz.shape[0]
    rng = np.random.default_rng(11)
    c = rng.uniform(-0.5, 0.5, size=(2, corr.n_terms)) / n
    return Correlator(corr.form, corr.mno, c, corr.d, np.array([1.0, 1.3]), corr.nuc_xyz,
                      (np.arange(n) % 2).astype(np.int32))


@pytest.fixture(scope="module")
def bh_small(h6_small):
    """A smaller ragged subset for the adjoint (the oracle differentiates 48-96 units)."""
    from oracle import fit, orbitals, pivots
    from workloads import bh_correlator
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(8).choice(wl.n_g, 700, replace=False))
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, 40)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    n = len(fp.pivots)
    rng = np.random.default_rng(34)
    cot = {"u1": rng.normal(size=(3, n, n)) / n, "u3": rng.normal(size=(n, n)) / n,
           "D1": rng.normal(size=(n, n)) / n, "D4": rng.normal(size=(n, n)) / n,
           "field": rng.normal(size=(3, len(w))) / np.sqrt(len(w))}
    return wl, xyz, w, fp.pivots, fr, rho, bh_correlator(wl.atom_xyz), cot


@pytest.mark.parametrize("types", [1, 2])
def test_bh_adjoint_matches_oracle(bh_small, types):
    import torch
    from oracle import adjoint
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr, cot = bh_small
    if types == 2:
        corr = _two_type(corr)
    ref = adjoint.dL_dc(xyz, w, corr, fr.xi, fr.xigrad, rho[piv], rho, cot)
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    got = api.grad(grid, corr, xi, xig, rh, piv, {k: t(v) for k, v in cot.items()}).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    note(f"BH adjoint, {types} type(s), {got.size} parameters: rel err {err:.2e}")
    assert got.shape == ref.shape
    assert err < 1e-10


@pytest.mark.parametrize("types", [1, 2])
def test_bh_autograd_matches_central_differences_on_every_coefficient(bh_small, types):
    """Through XtcContract (torch.autograd, backward = xtc_grad): the gradient of a random
    linear functional of every output with respect to all 48 (one nucleus type) or 96 (two
    types) linear coefficients, against central differences of the device forward. Every
    output is a polynomial of degree <= 2 in c, so central differences are exact up to
    rounding."""
    import torch
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr, cot = bh_small
    if types == 2:
        corr = _two_type(corr)
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    dc = {k: t(v) for k, v in cot.items()}
    ch = CH & ~64
    theta = torch.tensor(corr.c.ravel(), dtype=torch.float64, requires_grad=True)
    outs = api.contract_autograd(theta, grid, corr, xi, xig, rh, piv, ch)
    assert set(outs) == set(dc)
    loss = sum((outs[k] * dc[k]).sum() for k in outs)
    loss.backward()
    g = theta.grad.numpy().copy()

    def L(c):
        out = api.kernel_contract(grid, corr, xi, xig, rh, piv, ch, c=c)
        return sum(float(torch.sum(dc[k] * out[k])) for k in dc)

    c0 = corr.c.ravel().copy()
    h = 1e-4
    fd = np.zeros_like(g)
    for j in range(c0.size):
        cp, cm = c0.copy(), c0.copy()
        cp[j] += h
        cm[j] -= h
        fd[j] = (L(cp) - L(cm)) / (2 * h)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    note(f"BH autograd, {types} type(s), {g.size} coefficients vs central differences: rel err {err:.2e}")
    assert g.size == 48 * types
    assert err < 1e-7


@pytest.mark.parametrize("types", [1, 2])
def test_bh_nonlinear_derivatives_match_oracle(bh_small, types):
    """dL/dd and dL/db_t (eq. bh-u) against the oracle's complex-step derivatives of its own
    contraction; dL/dc is unchanged by asking for them (a separate kernel variant)."""
    import torch
    from oracle import adjoint
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr, cot = bh_small
    if types == 2:
        corr = _two_type(corr)
    ref = adjoint.dL_dnl(xyz, w, corr, fr.xi, fr.xigrad, rho[piv], rho, cot)
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    dc = {k: t(v) for k, v in cot.items()}
    g_c, g_nl = api.grad(grid, corr, xi, xig, rh, piv, dc, want_d=True)
    g_only = api.grad(grid, corr, xi, xig, rh, piv, dc)
    torch.cuda.synchronize()
    got = g_nl.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    note(f"BH nonlinear derivatives, {types} type(s): device {got}, oracle {ref}, rel err {err:.2e}")
    assert got.shape == (1 + types,)
    assert err < 1e-10
    assert torch.allclose(g_c, g_only, rtol=1e-13, atol=1e-15 * float(g_only.abs().max()))


def test_bh_nonlinear_derivatives_match_richardson_differences(bh_small):
    """dL/db_0 and dL/dd against Richardson-extrapolated central differences of the
    device forward pass."""
    import torch
    from dataclasses import replace
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr, cot = bh_small
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    dc = {k: t(v) for k, v in cot.items()}
    _, g_nl = api.grad(grid, corr, xi, xig, rh, piv, dc, want_d=True)
    got = g_nl.cpu().numpy()

    def L(cr):
        out = api.kernel_contract(grid, cr, xi, xig, rh, piv, CH & ~64)
        return sum(float(torch.sum(dc[k] * out[k])) for k in ("u1", "u3", "D1", "D4", "field"))

    h = 1e-3
    for k in range(2):
        mv = (lambda v: replace(corr, d=corr.d + v)) if k == 0 else \
             (lambda v: replace(corr, b=np.asarray(corr.b, np.float64) + v))
        fd1 = (L(mv(h)) - L(mv(-h))) / (2 * h)
        fd2 = (L(mv(2 * h)) - L(mv(-2 * h))) / (4 * h)
        rich = (4.0 * fd1 - fd2) / 3.0
        note(f"  parameter {k}: adjoint {got[k]:.12e}, Richardson difference {rich:.12e}")
        assert abs(rich - got[k]) <= 1e-8 * np.abs(got).max()
