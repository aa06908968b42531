"""GPU parity of the split-FP16 contraction (XTC_SPLIT_F16): against the FP64
oracle on seeded cases spanning several tiles and a ragged tail, and at the full
H20 size (the benchmark's launch configuration) against the FP64 GPU form and
against exact field values the oracle computes point by point."""
import numpy as np
import pytest

from gpu_common import OracleCase, note, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-6     # max |got - ref| / max |ref| per output block
CH = 1 | 2 | 8 | 16 | 32 | 64


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_2607_17314_amd import api
    return api


@pytest.fixture(scope="module")
def cases(h4, h6_small):
    return {"h4": OracleCase(h4), "ragged": OracleCase(h6_small, n_mu=150, subset=4963, seed=3)}


@pytest.mark.parametrize("which", ["h4", "ragged"])
def test_split_matches_oracle(api, cases, which):
    import torch
    from paper_2607_17314_amd import XTC_SPLIT_F16
    case = cases[which]
    note(f"split contract {which}")
    ref = case.contract(CH)
    grid = api.DeviceGrid.from_host(case.xyz, case.w)
    out = api.kernel_contract(grid, case.wl.corr, torch.as_tensor(case.fit.xi).cuda(),
                              torch.as_tensor(case.fit.xigrad).cuda(), torch.as_tensor(case.rho).cuda(),
                              case.piv, CH, XTC_SPLIT_F16)
    torch.cuda.synchronize()
    for k in ("u1", "u3", "D1", "D4", "field"):
        e = rel_err(out[k].cpu().numpy(), ref[k])
        note(f"  {k}: rel err {e:.2e}")
        assert e < TOL, k
    er = np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"])
    note(f"  escale rel err {er.max():.2e}")
    assert er.max() < TOL


def test_split_odd_powers_match_oracle(api, cases):
    """A correlator with odd powers of rbar (an o = 1 term, so u'/r carries a 1/r part, and
    no even-power compaction) on the ragged case: the split stage 1 takes its general
    polynomial form and the FP64 density rows their o = 1 branch."""
    import torch
    from oracle import contract
    from paper_2607_17314_amd import XTC_SPLIT_F16
    from workloads import FORM_EE, Correlator
    case = cases["ragged"]
    corr = Correlator(FORM_EE, np.array([[0, 0, 1], [0, 0, 2], [0, 0, 3], [0, 0, 5]], np.int32),
                      np.array([[0.3, -0.4, 0.25, -0.1]]), 0.8)
    ref = contract.contract(case.xyz, case.w, corr, case.fit.xi, case.fit.xigrad,
                            case.rho[case.piv], case.rho, CH)
    grid = api.DeviceGrid.from_host(case.xyz, case.w)
    out = api.kernel_contract(grid, corr, torch.as_tensor(case.fit.xi).cuda(),
                              torch.as_tensor(case.fit.xigrad).cuda(), torch.as_tensor(case.rho).cuda(),
                              case.piv, CH, XTC_SPLIT_F16)
    torch.cuda.synchronize()
    for k in ("u1", "u3", "D1", "D4", "field"):
        e = rel_err(out[k].cpu().numpy(), ref[k])
        note(f"  odd powers {k}: rel err {e:.2e}")
        assert e < (1e-12 if k == "field" else TOL), k
    er = np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"])
    note(f"  odd powers escale rel err {er.max():.2e}")
    assert er.max() < TOL


@pytest.fixture(scope="module")
def h20_device(api):
    import torch
    from workloads import make_config
    wl = make_config("h20")
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    phi4, rho = api.eval_orbitals(wl.basis, grid, wl.C_mo, wl.n_occ)
    piv, info, st = api.select_points(phi4, grid, wl.n_mu, wl.n_occ)
    assert len(piv) == wl.n_mu
    xi, xig, finfo, _ = api.fit(phi4, grid, piv)
    note(f"h20: pivots {len(piv)} (scalar {info[0]:.0f}, grad {info[1]:.0f}), fit info {finfo}")
    return wl, grid, rho, piv, xi, xig


def test_full_size_split_vs_fp64_and_sampled_field(api, h20_device):
    import torch
    from oracle.correlator import pair_kernels
    from paper_2607_17314_amd import XTC_FP64, XTC_SPLIT_F16
    wl, grid, rho, piv, xi, xig = h20_device
    note("h20 full size: split contraction")
    sp = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, CH, XTC_SPLIT_F16)
    torch.cuda.synchronize()
    note("h20 full size: fp64 contraction")
    fp = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, CH, XTC_FP64)
    torch.cuda.synchronize()
    for k in ("u1", "u3", "D1", "D4", "field"):
        e = float((sp[k] - fp[k]).abs().max() / fp[k].abs().max())
        note(f"  {k}: split vs fp64 rel err {e:.2e}")
        assert e < TOL, k
    er = np.abs(sp["escale"] - fp["escale"]) / np.abs(fp["escale"])
    note(f"  escale split vs fp64 rel err {er.max():.2e}; escale {fp['escale']}")
    assert er.max() < TOL
    # exact field at sampled bra points, one O(N_g) sum each, in the oracle
    rng = np.random.default_rng(7)
    gs = np.sort(rng.choice(wl.n_g, 64, replace=False))
    wr = wl.grid_w * rho.cpu().numpy()
    K = pair_kernels(wl.corr, wl.grid_xyz[:, gs], wl.grid_xyz)
    ref = np.stack([K["gx"] @ wr, K["gy"] @ wr, K["gz"] @ wr])
    got = fp["field"].cpu().numpy()[:, gs]
    e = rel_err(got, ref)
    note(f"  sampled exact field vs fp64 device: rel err {e:.2e}")
    assert e < 1e-10
    # properties that hold at any size
    d4 = fp["D4"]
    assert float((d4 - d4.T).abs().max() / d4.abs().max()) < 1e-12
    u3 = fp["u3"]
    assert float((u3 - u3.T).abs().max() / u3.abs().max()) < 1e-10
