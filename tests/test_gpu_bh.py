"""The multi-centre Boys-Handy correlator (eq. bh-u, 48 terms) on the GPU FP64
path: the contraction against the oracle on a ragged H6 grid subset, and the
split path's explicit refusal."""
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


def test_bh_split_path_is_refused(bh_problem):
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, xyz, w, piv, fr, rho, corr = bh_problem
    grid, xi, xig, rh = _device(api, xyz, w, fr, rho)
    with pytest.raises(api.XtcError) as ei:
        api.kernel_contract(grid, corr, xi, xig, rh, piv, CH, precision=L.XTC_SPLIT_F16)
    assert ei.value.status == L.XTC_ERR_UNSUPPORTED
