"""Parity at the shapes the benchmark and the multi-centre configuration run: the H20
workload (194,000 grid points, 300 orbitals, N_mu = 3000).

* Interpolation points: the GPU selection equals, index for index, the oracle's fused
  pivots stored in tests/golden/h20_pivots.txt (written by the committed script beside
  it, which calls only the oracle), up to the first step whose top-two gap is below
  1e-10 (none at this size).
* The contraction (eqs. K1-isdf, K3-isdf; xTC Terms 1 and 4), split and FP64, on a bra
  range that crosses a 16,384-point super-block boundary, with every ket point of the
  grid and the oracle's own xi and xi~ (fitted on those pivots) fed to both sides,
  against the oracle's contraction restricted to the same bra range.
* The 48-term multi-centre correlator (eq. bh-u, 20 nuclei): the forward on the FP64 and
  split paths, and the FP64 adjoint, on a bra range across the same boundary, against the
  oracle; and every
  one of the 48 coefficients by central differences (step 1e-4) of the device forward,
  which are exact up to rounding because every output is at most quadratic in c.
"""
import os

import numpy as np
import pytest

from gpu_common import note, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "h20_pivots.txt")
BRA = (16000, 16700)         # 700 bra points across the 16,384-point super-block boundary
BRA_BH = (16368, 16400)      # 32 bra points across the same boundary (BH oracle is slow)
BRA_BH_ADJ = (16376, 16392)  # 16 of them for the oracle's adjoint
CH = 1 | 2 | 8 | 16 | 32 | 64


def read_golden(path=GOLDEN):
    """(scalar pivots, scalar gaps, gradient pivots, gradient gaps) in selection order."""
    seq = {"s": ([], []), "g": ([], [])}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            ch, _, g, gap = line.split()
            seq[ch][0].append(int(g))
            seq[ch][1].append(float(gap))
    return seq["s"][0], np.array(seq["s"][1]), seq["g"][0], np.array(seq["g"][1])


def fused_order(scalar, grad, n_mu):
    ss = set(scalar)
    out = list(scalar) + [g for g in grad if g not in ss]
    return np.asarray(out[:n_mu], np.int64)


@pytest.fixture(scope="module")
def h20():
    """The oracle's H20 state: orbitals, the stored fused pivots, xi on every grid point
    and xi~ on the bra range (the fit is column-separable)."""
    from oracle import fit, orbitals
    from workloads import make_config
    wl = make_config("h20")
    sc, sg, gr, gg = read_golden()
    piv = fused_order(sc, gr, wl.n_mu)
    assert len(piv) == wl.n_mu
    note(f"h20 oracle: orbitals on {wl.n_g} points")
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    rho = orbitals.density(phi4, wl.n_occ)
    note("h20 oracle: fit of xi (all columns) and xi~ (bra columns)")
    cols = np.arange(BRA[0], BRA[1])
    fr = fit.fit(phi4, wl.grid_w, piv, with_grad=True, grad_cols=cols)
    note(f"h20 oracle: fit done, jitter {fr.jitter}, residuals {fr.resid_rel}")
    return dict(wl=wl, phi4=phi4, rho=rho, piv=piv, xi=fr.xi, xig_bra=fr.xigrad, golden=(sc, sg, gr, gg))


@pytest.fixture(scope="module")
def dev(h20):
    import torch
    from paper_2607_17314_amd import api
    wl = h20["wl"]
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    xi = t(h20["xi"])
    xig = torch.zeros((3, wl.n_mu, wl.n_g), dtype=torch.float64, device="cuda")
    xig[:, :, BRA[0]:BRA[1]] = t(h20["xig_bra"])
    return dict(api=api, grid=grid, xi=xi, xig=xig, rho=t(h20["rho"]))


def xig_host(h20):
    """xi~ as a full-size host array that is zero outside the bra range (np.zeros maps
    untouched pages lazily, so only the bra columns take memory)."""
    wl = h20["wl"]
    x = np.zeros((3, wl.n_mu, wl.n_g))
    x[:, :, BRA[0]:BRA[1]] = h20["xig_bra"]
    return x


def test_h20_orbitals_and_pivot_indices_match_oracle(h20, dev):
    import torch
    api, grid = dev["api"], dev["grid"]
    wl = h20["wl"]
    note("h20: device orbitals and fused selection")
    phi4, rho = api.eval_orbitals(wl.basis, grid, wl.C_mo, wl.n_occ)
    gs = np.sort(np.random.default_rng(5).choice(wl.n_g, 4096, replace=False))
    e = rel_err(phi4[:, :, torch.as_tensor(gs).cuda()].cpu().numpy(), h20["phi4"][:, :, gs])
    note(f"  sampled orbital values and gradients: rel err {e:.2e}")
    assert e < 1e-12
    piv, info, st = api.select_points(phi4, grid, wl.n_mu, wl.n_occ)
    sc, sg, gr, gg = h20["golden"]
    ks = int(np.argmax(sg < 1e-10)) if np.any(sg < 1e-10) else len(sc)
    kg = int(np.argmax(gg < 1e-10)) if np.any(gg < 1e-10) else len(gr)
    note(f"  device: {len(piv)} pivots, scalar steps {info[0]:.0f}, gradient steps {info[1]:.0f}; "
         f"oracle: {len(sc)} scalar, {len(gr)} gradient; first near tie at scalar step {ks}, "
         f"gradient step {kg}; smallest gaps {sg.min():.2e}, {gg.min():.2e}")
    assert np.array_equal(piv[:ks], np.asarray(sc[:ks]))
    if ks == len(sc) and kg == len(gr):
        assert int(info[0]) == len(sc) and int(info[1]) == len(gr)
        assert np.array_equal(piv, h20["piv"])


@pytest.mark.parametrize("prec", ["split", "fp64"])
def test_h20_contraction_on_bra_range_matches_oracle(h20, dev, prec):
    import torch
    from oracle import contract
    from paper_2607_17314_amd import XTC_FP64, XTC_SPLIT_F16
    api, wl, piv = dev["api"], h20["wl"], h20["piv"]
    tol = 1e-6 if prec == "split" else 1e-10
    note(f"h20 {prec} contraction on bra points [{BRA[0]}, {BRA[1]})")
    out = api.kernel_contract(dev["grid"], wl.corr, dev["xi"], dev["xig"], dev["rho"], piv, CH,
                              XTC_SPLIT_F16 if prec == "split" else XTC_FP64, bra=BRA)
    torch.cuda.synchronize()
    if "ref" not in h20:
        note("  oracle contraction on the same bra range")
        rho = h20["rho"]
        h20["ref"] = contract.contract(wl.grid_xyz, wl.grid_w, wl.corr, h20["xi"], xig_host(h20),
                                       rho[piv], rho, CH, bra_block=44, bra_range=BRA)
    ref = h20["ref"]
    for k in ("u1", "u3", "D1", "D4"):
        e = rel_err(out[k].cpu().numpy(), ref[k])
        note(f"  {k}: rel err {e:.2e}")
        assert e < tol, k
    fld = out["field"].cpu().numpy()
    e = rel_err(fld[:, BRA[0]:BRA[1]], ref["field"][:, BRA[0]:BRA[1]])
    note(f"  field on the range: rel err {e:.2e}")
    assert e < tol
    assert not fld[:, :BRA[0]].any() and not fld[:, BRA[1]:].any()
    er = np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"])
    note(f"  escale rel err {er.max():.2e}")
    assert er.max() < tol


@pytest.fixture(scope="module")
def bh(h20, dev):
    """Config-3 shape: the same H20 system, pivots and xi with the 48-term BH correlator
    on its 20 nuclei, and seeded cotangents."""
    from workloads import bh_correlator
    wl = h20["wl"]
    corr = bh_correlator(wl.atom_xyz)
    n = wl.n_mu
    rng = np.random.default_rng(35)
    cot = {"u1": rng.normal(size=(3, n, n)) / n, "u3": rng.normal(size=(n, n)) / n,
           "D1": rng.normal(size=(n, n)) / n, "D4": rng.normal(size=(n, n)) / n,
           "field": rng.normal(size=(3, wl.n_g)) / np.sqrt(wl.n_g)}
    return corr, cot


@pytest.fixture(scope="module")
def bh_ref(h20, bh):
    """The oracle's config-3 contraction on the bra range (the pivots and xi of the H20 fit)."""
    from oracle import contract
    wl, piv, rho = h20["wl"], h20["piv"], h20["rho"]
    corr, _ = bh
    return contract.contract(wl.grid_xyz, wl.grid_w, corr, h20["xi"], xig_host(h20), rho[piv],
                             rho, CH, bra_block=2, ket_block=16384, bra_range=BRA_BH)


@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_config3_bh_forward_on_bra_range_matches_oracle(h20, dev, bh, bh_ref, prec):
    """The BH contraction at the config-3 shape on 32 bra points across the super-block
    boundary. Split: twelve ket launches of pair values (the density-row sums carried across
    them), twelve 256-row tiles; blocks within 1e-6, the field (FP64 density rows) within
    1e-10."""
    import torch
    from paper_2607_17314_amd import XTC_FP64, XTC_SPLIT_F16
    api, wl, piv = dev["api"], h20["wl"], h20["piv"]
    corr, _ = bh
    note(f"config-3 shape BH forward ({prec}) on bra points [{BRA_BH[0]}, {BRA_BH[1]}), "
         f"{corr.nuc_xyz.shape[0]} nuclei, {corr.n_terms} terms")
    out = api.kernel_contract(dev["grid"], corr, dev["xi"], dev["xig"], dev["rho"], piv, CH,
                              XTC_SPLIT_F16 if prec == "split" else XTC_FP64, bra=BRA_BH)
    torch.cuda.synchronize()
    ref = bh_ref
    tol = 1e-6 if prec == "split" else 1e-10
    for k in ("u1", "u3", "D1", "D4"):
        e = rel_err(out[k].cpu().numpy(), ref[k])
        note(f"  {k}: rel err {e:.2e}")
        assert e < tol, k
    e = rel_err(out["field"].cpu().numpy()[:, BRA_BH[0]:BRA_BH[1]], ref["field"][:, BRA_BH[0]:BRA_BH[1]])
    note(f"  field: rel err {e:.2e}")
    assert e < 1e-10
    er = np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"])
    note(f"  escale rel err {er.max():.2e}")
    assert er.max() < tol


def test_config3_bh_adjoint_on_bra_range(h20, dev, bh):
    """xtc_grad on the bra range against the oracle's derivative for four coefficients, and
    against central differences (step 1e-4) of the device forward for all 48."""
    import torch
    from oracle import adjoint
    api, wl, piv = dev["api"], h20["wl"], h20["piv"]
    corr, cot = bh
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    dc = {k: t(v) for k, v in cot.items()}
    note("config-3 shape BH adjoint on the bra range")
    g = api.grad(dev["grid"], corr, dev["xi"], dev["xig"], dev["rho"], piv, dc, bra=BRA_BH)
    g = g.cpu().numpy()
    assert g.shape == (48,)
    sel = [0, 40]
    rho = h20["rho"]
    ga = api.grad(dev["grid"], corr, dev["xi"], dev["xig"], dev["rho"], piv, dc, bra=BRA_BH_ADJ)
    ga = ga.cpu().numpy()
    ref = adjoint.dL_dc(wl.grid_xyz, wl.grid_w, corr, h20["xi"], xig_host(h20), rho[piv], rho, cot,
                        bra_block=2, ket_block=16384, bra_range=BRA_BH_ADJ, params=sel)
    e = np.abs(ga[sel] - ref).max() / np.abs(ref).max()
    note(f"  oracle on [{BRA_BH_ADJ[0]}, {BRA_BH_ADJ[1]}), coefficients {sel}: rel err {e:.2e}")
    assert e < 1e-10

    def L(c):
        out = api.kernel_contract(dev["grid"], corr, dev["xi"], dev["xig"], dev["rho"], piv, CH & ~64,
                                  c=c, bra=BRA_BH)
        return sum(float(torch.sum(dc[k] * out[k])) for k in ("u1", "u3", "D1", "D4", "field"))

    c0 = corr.c.ravel().copy()
    h = 1e-4
    fd = np.zeros(c0.size)
    for j in range(c0.size):
        cp, cm = c0.copy(), c0.copy()
        cp[j] += h
        cm[j] -= h
        fd[j] = (L(cp) - L(cm)) / (2 * h)
    e = np.abs(fd - g).max() / np.abs(g).max()
    note(f"  central differences, all {c0.size} coefficients: max rel err {e:.2e}")
    assert e < 1e-7
