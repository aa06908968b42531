"""GPU adjoint (xtc_grad) against the oracle's forward-mode derivatives and
against central finite differences of the device forward pass, through the
C ABI and through the torch.autograd.Function."""
import numpy as np
import pytest

from gpu_common import note

pytestmark = pytest.mark.gpu

ALL = 1 | 2 | 4 | 8 | 16 | 32


@pytest.fixture(scope="module")
def problem(h6_small):
    from oracle import fit, orbitals, pivots
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(5).choice(wl.n_g, 1300, replace=False))   # ragged size
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, 70)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    rng = np.random.default_rng(33)
    n = len(fp.pivots)
    cot = {"u1": rng.normal(size=(3, n, n)) / n, "u3": rng.normal(size=(n, n)) / n,
           "ulap": rng.normal(size=(n, n)) / n, "D1": rng.normal(size=(n, n)) / n,
           "D4": rng.normal(size=(n, n)) / n, "field": rng.normal(size=(3, len(w))) / np.sqrt(len(w))}
    return wl, xyz, w, fp.pivots, fr, rho, cot


def _device(api, problem):
    import torch
    wl, xyz, w, piv, fr, rho, cot = problem
    grid = api.DeviceGrid.from_host(xyz, w)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return grid, t(fr.xi), t(fr.xigrad), t(rho), {k: t(v) for k, v in cot.items()}


@pytest.mark.parametrize("subset", ["all", "u1u3", "D-only"])
def test_adjoint_matches_oracle(problem, subset):
    import torch
    from oracle import adjoint
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, cot = problem
    keys = {"all": list(cot), "u1u3": ["u1", "u3", "field"], "D-only": ["D1", "D4"]}[subset]
    c_sub = {k: cot[k] for k in keys}
    ref = adjoint.dL_dc(xyz, w, wl.corr, fr.xi, fr.xigrad, rho[piv], rho, c_sub)
    grid, xi, xig, rh, dcot = _device(api, problem)
    got = api.grad(grid, wl.corr, xi, xig, rh, piv, {k: dcot[k] for k in keys}).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    note(f"adjoint {subset}: device {got}, oracle {ref}, rel err {err:.2e}")
    assert err < 1e-10


def test_adjoint_matches_central_differences_and_autograd(problem):
    import torch
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, cot = problem
    grid, xi, xig, rh, dcot = _device(api, problem)
    theta = torch.tensor(wl.corr.c.ravel(), dtype=torch.float64, requires_grad=True)
    outs = api.contract_autograd(theta, grid, wl.corr, xi, xig, rh, piv, ALL)
    loss = sum((outs[k] * dcot[k]).sum() for k in outs)
    loss.backward()
    g_auto = theta.grad.numpy().copy()
    h = 1e-4
    fd = np.zeros_like(g_auto)
    for j in range(theta.numel()):
        vals = []
        for s in (+1, -1):
            c = wl.corr.c.ravel().copy()
            c[j] += s * h
            o = api.kernel_contract(grid, wl.corr, xi, xig, rh, piv, ALL, c=c)
            vals.append(sum(float((o[k] * dcot[k]).sum()) for k in ("u1", "u3", "ulap", "D1", "D4", "field")))
        fd[j] = (vals[0] - vals[1]) / (2 * h)
    err = np.abs(g_auto - fd).max() / np.abs(fd).max()
    note(f"autograd {g_auto} vs central FD {fd}: rel err {err:.2e}")
    # every output is a polynomial of degree <= 2 in c: central differences are exact up to rounding
    assert err < 1e-7


@pytest.mark.parametrize("subset", ["all", "u1u3", "D-only"])
def test_scale_derivative_matches_oracle(problem, subset):
    """dL/dd for the nonlinear scale d of rbar against the oracle's complex-step
    derivative of its own contraction, and against Richardson-extrapolated central
    differences of the device forward pass; dL/dc is unchanged by asking for dL/dd."""
    import torch
    from dataclasses import replace
    from oracle import adjoint
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, cot = problem
    keys = {"all": list(cot), "u1u3": ["u1", "u3", "field"], "D-only": ["D1", "D4"]}[subset]
    c_sub = {k: cot[k] for k in keys}
    ref = adjoint.dL_dd(xyz, w, wl.corr, fr.xi, fr.xigrad, rho[piv], rho, c_sub)
    grid, xi, xig, rh, dcot = _device(api, problem)
    dc = {k: dcot[k] for k in keys}
    g_c, g_d = api.grad(grid, wl.corr, xi, xig, rh, piv, dc, want_d=True)
    g_only = api.grad(grid, wl.corr, xi, xig, rh, piv, dc)
    torch.cuda.synchronize()
    got = float(g_d.cpu()[0])
    err = abs(got - ref) / abs(ref)
    note(f"dL/dd {subset}: device {got:.15e}, oracle {ref:.15e}, rel err {err:.2e}")
    assert err < 1e-10
    assert torch.equal(g_c, g_only)
    if subset != "all":
        return
    bits = {"u1": 1, "u3": 2, "ulap": 4, "D1": 8, "D4": 16, "field": 32}
    ch = sum(bits[k] for k in keys)

    def L(d):
        out = api.kernel_contract(grid, replace(wl.corr, d=d), xi, xig, rh, piv, ch)
        return sum(float(torch.sum(dc[k] * out[k])) for k in keys)

    d0, h = wl.corr.d, 1e-3
    fd1 = (L(d0 + h) - L(d0 - h)) / (2 * h)
    fd2 = (L(d0 + 2 * h) - L(d0 - 2 * h)) / (4 * h)
    rich = (4.0 * fd1 - fd2) / 3.0
    note(f"  Richardson central difference {rich:.15e}")
    assert abs(rich - got) <= 1e-8 * abs(got)


def test_adjoint_bra_ranges_add_up_and_match_oracle(problem):
    """xtc_grad on a bra range is the derivative of that range's partial sums: two disjoint
    ranges add up to the whole grid's derivative, and one range matches the oracle's."""
    from oracle import adjoint
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, cot = problem
    grid, xi, xig, rh, dcot = _device(api, problem)
    n_g = len(w)
    cut = 517
    whole = api.grad(grid, wl.corr, xi, xig, rh, piv, dcot).cpu().numpy()
    a = api.grad(grid, wl.corr, xi, xig, rh, piv, dcot, bra=(0, cut)).cpu().numpy()
    b = api.grad(grid, wl.corr, xi, xig, rh, piv, dcot, bra=(cut, n_g)).cpu().numpy()
    e = np.abs(a + b - whole).max() / np.abs(whole).max()
    ref = adjoint.dL_dc(xyz, w, wl.corr, fr.xi, fr.xigrad, rho[piv], rho, cot, bra_range=(cut, n_g))
    eo = np.abs(b - ref).max() / np.abs(ref).max()
    note(f"adjoint bra ranges: sum vs whole {e:.2e}, range vs oracle {eo:.2e}")
    assert e < 1e-12
    assert eo < 1e-10
