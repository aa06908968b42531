"""Four-index assembly on the GPU (xtc_assembly_prepare / xtc_assembly_panel) and the
xTC one-body pieces (xtc_one_body) against the oracle: full K, dU, W tensors on a ragged
H6 case (60 orbitals in 7-wide panels, the last one ragged; intermediates from the
oracle's contraction and exchange), and sampled elements at the full H20 shape."""
import numpy as np
import pytest

from gpu_common import note, rel_err

pytestmark = pytest.mark.gpu

ALL = 1 | 2 | 8 | 16 | 32 | 64


@pytest.fixture(scope="module")
def asm_problem(h6_small):
    from oracle import assembly, contract, exchange, fit, orbitals, pivots
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    idx = np.sort(np.random.default_rng(31).choice(wl.n_g, 1500, replace=False))
    xyz, w, phi4 = np.ascontiguousarray(wl.grid_xyz[:, idx]), wl.grid_w[idx].copy(), phi4[:, :, idx]
    fp = pivots.select_fused(phi4, w, 100)
    fr = fit.fit(phi4, w, fp.pivots)
    rho = orbitals.density(phi4, wl.n_occ)
    out = contract.contract(xyz, w, wl.corr, fr.xi, fr.xigrad, rho[fp.pivots], rho, ALL)
    cG = exchange.calG(xyz, w, wl.corr, fr.xi)
    LQ = exchange.density_projector(exchange.occupied_gamma(phi4.shape[1], wl.n_occ))
    x = exchange.x_terms(phi4[0], fp.pivots, fr.xi, cG, w, LQ)
    piv = fp.pivots
    K = assembly.k_tensor(phi4, piv, out["u1"], out["u3"])
    dU = assembly.du_tensor(phi4, piv, out["D1"], out["D4"], x["X2"], x["X3"])
    W = assembly.w_tensor(K, dU)
    return wl, phi4, piv, out, x, dict(K=K, dU=dU, W=W)


def _dev(a):
    import torch
    return None if a is None else torch.as_tensor(np.ascontiguousarray(a)).cuda()


def test_assembly_panels_match_oracle(asm_problem):
    import torch
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, phi4, piv, out, x, ref = asm_problem
    n = phi4.shape[1]
    note(f"assembly: n_orb={n} n_mu={len(piv)}, panels of 7")
    asm = api.Assembly(_dev(phi4[:, :, piv]), _dev(out["u1"]), _dev(out["u3"]), _dev(out["D1"]),
                       _dev(out["D4"]), _dev(x["X2"]), _dev(x["X3"]),
                       outputs=L.XTC_ASM_K | L.XTC_ASM_DU | L.XTC_ASM_W)
    got = {k: np.empty((n, n, n, n)) for k in ("K", "dU", "W")}
    for p0 in range(0, n, 7):
        p1 = min(n, p0 + 7)
        o = asm.panel(p0, p1)
        torch.cuda.synchronize()
        for k in got:
            got[k][p0:p1] = o[k].cpu().numpy()       # [p][r][q][s]
    for k in ("K", "dU", "W"):
        r = ref[k].transpose(0, 2, 1, 3)             # [p][q][r][s] -> [p][r][q][s]
        e = rel_err(got[k], r)
        note(f"  {k}: rel max err {e:.2e}")
        assert e < 1e-12, k


def test_assembly_without_exchange_terms(asm_problem):
    import torch
    from oracle import assembly
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    wl, phi4, piv, out, x, ref = asm_problem
    asm = api.Assembly(_dev(phi4[:, :, piv]), _dev(out["u1"]), _dev(out["u3"]), _dev(out["D1"]),
                       _dev(out["D4"]), None, None, outputs=L.XTC_ASM_DU)
    o = asm.panel(11, 29)
    torch.cuda.synchronize()
    r = assembly.du_tensor(phi4, piv, out["D1"], out["D4"], None, None).transpose(0, 2, 1, 3)[11:29]
    e = rel_err(o["dU"].cpu().numpy(), r)
    note(f"  dU without X: rel max err {e:.2e}")
    assert e < 1e-12


def test_one_body_matches_oracle(asm_problem):
    from oracle import assembly
    from paper_2607_17314_amd import api
    wl, phi4, piv, out, x, ref = asm_problem
    dh_ref = assembly.delta_h(ref["dU"], wl.n_occ)
    f_ref = assembly.fock_xtc(dh_ref, ref["W"], wl.n_occ)
    e0_ref = assembly.e0_xtc(dh_ref, wl.n_occ, 3.5)
    dh, f, e0 = api.one_body(_dev(phi4[:, :, piv]), _dev(out["u1"]), _dev(out["u3"]),
                             _dev(out["D1"]), _dev(out["D4"]), _dev(x["X2"]), _dev(x["X3"]),
                             wl.n_occ, 3.5)
    for k, g, r in (("dh", dh, dh_ref), ("f", f, f_ref)):
        e = rel_err(g.cpu().numpy(), r)
        note(f"  {k}: rel max err {e:.2e}")
        assert e < 1e-12, k
    note(f"  e0: {e0!r} vs {e0_ref!r}")
    assert abs(e0 - e0_ref) <= 1e-12 * max(1.0, abs(e0_ref))


def test_full_size_assembly_sampled_elements():
    """A W panel at the H20 shape (300 orbitals, N_mu = 3000) on seeded inputs, checked
    element by element against the definitions, plus the particle-exchange symmetry
    across two panels."""
    import torch
    from oracle import assembly
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    n, n_mu = 300, 3000
    rng = np.random.default_rng(61)
    phi = rng.standard_normal((4, n, n_mu)) / np.sqrt(n)
    u1 = rng.standard_normal((3, n_mu, n_mu)) / n_mu
    sym = lambda m: 0.5 * (m + m.T)
    u3 = sym(rng.standard_normal((n_mu, n_mu))) / n_mu
    D1 = rng.standard_normal((n_mu, n_mu)) / n_mu
    D4 = sym(rng.standard_normal((n_mu, n_mu))) / n_mu
    X = rng.standard_normal((n, n, n_mu)) / n_mu
    X = 0.5 * (X + X.transpose(1, 0, 2))
    note("h20 shape: assembly prepare")
    asm = api.Assembly(_dev(phi), _dev(u1), _dev(u3), _dev(D1), _dev(D4), _dev(X), None,
                       outputs=L.XTC_ASM_W)
    pa, pb = (17, 21), (140, 143)
    Wa = asm.panel(*pa)["W"].cpu().numpy()
    Wb = asm.panel(*pb)["W"].cpu().numpy()
    torch.cuda.synchronize()
    picks = [(int(rng.integers(*pa)), int(rng.integers(n)), int(rng.integers(n)), int(rng.integers(n)))
             for _ in range(24)]
    errs, scale = [], np.abs(Wa).max()
    for p, q, r, s in picks:
        ref = assembly.w_entry(phi, u1, u3, D1, D4, X, p, q, r, s)
        errs.append(abs(Wa[p - pa[0], r, q, s] - ref))
    e = max(errs) / scale
    note(f"  sampled W elements: max abs err / max |W| = {e:.2e}")
    assert e < 1e-12
    # W^{pq}_{rs} = W^{qp}_{sr}: p in panel a, q in panel b
    d = 0.0
    for p in range(*pa):
        for q in range(*pb):
            d = max(d, float(np.abs(Wa[p - pa[0], :, q, :] - Wb[q - pb[0], :, p, :].T).max()))
    note(f"  exchange symmetry across panels: {d / scale:.2e}")
    assert d <= 1e-13 * scale
