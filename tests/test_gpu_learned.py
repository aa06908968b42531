"""GPU parity of the learned interpolation-point proposer: features, MLP
forward, loss gradient and Adam against the oracle; the learned selection
(candidates: the best scores and every stride-th point) against the oracle's
pivoting on the same candidates (bit-exact); the judge's fallback on a corrupted
network; and a small training run on three chains, scored on two held-out chains,
showing what the trained network gains over the untrained one and over random
points, and that the judge accepts its proposal."""
import time

import numpy as np
import pytest

from gpu_common import note, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(h6_small):
    import torch
    from oracle import orbitals
    from paper_2607_17314_amd import api
    wl = h6_small
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    return wl, phi4, grid, torch.as_tensor(phi4).cuda()


def _model(api, feats_np, seed=0, hidden=64, kappa=3.0, nuclei=None, zero=False, judge=0,
           stride=0):
    from oracle import mlp
    p = np.zeros(mlp.n_params(hidden)) if zero else mlp.init_params(hidden, seed)
    shift = feats_np.mean(axis=1)
    scale = feats_np.std(axis=1) + 1e-3
    return api.MlpModel(p.astype(np.float32), shift.astype(np.float32), scale.astype(np.float32),
                        hidden, kappa, nuclei, judge=judge, stride=stride), p, \
        shift.astype(np.float32), scale.astype(np.float32)


def test_features_forward_grad_adam(case):
    import torch
    from oracle import mlp
    from paper_2607_17314_amd import api
    wl, phi4, grid, phi4_d = case
    f = api.features(phi4_d, grid, wl.n_occ, wl.atom_xyz)
    ref = mlp.features(phi4, wl.grid_w, wl.n_occ, wl.grid_xyz, wl.atom_xyz)
    got = f.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max()
    note(f"features: max abs err {err:.2e}")
    assert err < 2e-5
    model, p, sh, sc = _model(api, got, seed=3, nuclei=wl.atom_xyz)
    x = (got - sh[:, None].astype(np.float64)) / sc[:, None].astype(np.float64)
    pf = model.params.cpu().numpy().astype(np.float64)
    s_ref, _ = mlp.forward(pf, 64, x)
    s_gpu = api.mlp_forward(model, f).cpu().numpy()
    e = np.abs(s_gpu - s_ref).max() / np.abs(s_ref).max()
    note(f"forward: rel err {e:.2e}")
    assert e < 1e-4
    rng = np.random.default_rng(1)
    idx = rng.choice(wl.n_g, 4096, replace=False)
    y = (rng.random(4096) < 0.1).astype(np.float32)
    fb = f[:, torch.as_tensor(idx).cuda()].contiguous()
    loss, grad = api.mlp_loss_grad(model, fb, torch.as_tensor(y).cuda(), 9.0)
    l_ref, g_ref = mlp.loss_grad(pf, 64, x[:, idx], y.astype(np.float64), 9.0)
    eg = rel_err(grad.cpu().numpy(), g_ref)
    note(f"loss {float(loss):.6f} vs {l_ref:.6f}; grad rel err {eg:.2e}")
    assert abs(float(loss) - l_ref) < 1e-4 * abs(l_ref)
    assert eg < 1e-3
    m = torch.zeros_like(model.params)
    v = torch.zeros_like(model.params)
    p0 = model.params.clone()
    api.adam_step(model.params, grad, m, v, 1, lr=1e-3)
    pa, _, _ = mlp.adam(p0.cpu().numpy().astype(np.float64), grad.cpu().numpy().astype(np.float64),
                        np.zeros(p0.numel()), np.zeros(p0.numel()), 1, lr=1e-3)
    assert np.abs(model.params.cpu().numpy() - pa).max() < 1e-6


@pytest.mark.parametrize("stride", [0, 7])
def test_learned_selection_matches_oracle_pivoting_on_the_same_candidates(case, stride):
    from oracle import mlp, pivots
    from paper_2607_17314_amd import XTC_SELECT_LEARNED, api
    wl, phi4, grid, phi4_d = case
    f = api.features(phi4_d, grid, wl.n_occ, wl.atom_xyz)
    model, *_ = _model(api, f.cpu().numpy().astype(np.float64), seed=5, kappa=2.5, nuclei=wl.atom_xyz,
                       stride=stride)
    n_mu = 150
    piv, info, st = api.select_points(phi4_d, grid, n_mu, wl.n_occ, XTC_SELECT_LEARNED, model)
    logits = api.mlp_forward(model, f).cpu().numpy().astype(np.float64)
    K = int(np.ceil(2.5 * n_mu))
    cand = mlp.candidates(logits, K, stride)
    assert int(info[6]) == len(cand)
    fp = pivots.select_fused(np.ascontiguousarray(phi4[:, :, cand]), wl.grid_w[cand], n_mu)
    ref = cand[fp.pivots]
    note(f"learned selection (stride {stride}): {len(piv)} pivots from {len(cand)} candidates; "
         f"identical: {np.array_equal(piv, ref)}")
    assert np.array_equal(piv, ref)


def test_bf16_forward_matches_the_oracle_emulation(case):
    """The BF16 matrix-core scoring against the oracle's forward with the same operands
    rounded to BF16 (the two differ only in the order and precision of the FP32 sums),
    and the learned selection scored in BF16 against the oracle's on its own BF16
    candidates."""
    import torch
    from oracle import mlp, pivots
    from paper_2607_17314_amd import XTC_SELECT_LEARNED, api
    wl, phi4, grid, phi4_d = case
    f = api.features(phi4_d, grid, wl.n_occ, wl.atom_xyz)
    fn = f.cpu().numpy()
    model, *_ = _model(api, fn.astype(np.float64), seed=3, nuclei=wl.atom_xyz, stride=7, kappa=2.5)
    model.bf16 = True
    s_bf = api.mlp_forward(model, f).cpu().numpy().astype(np.float64)
    pf = model.params.cpu().numpy().astype(np.float64)
    sh, sc = model.shift.cpu().numpy(), model.scale.cpu().numpy()
    x = ((fn - sh[:, None]) / sc[:, None]).astype(np.float32)      # z-scoring in FP32, as the device
    ref = mlp.forward_bf16(pf, 64, x)
    s32, _ = mlp.forward(pf, 64, x.astype(np.float64))
    e = np.abs(s_bf - ref).max() / np.abs(ref).max()
    e32 = np.abs(s_bf - s32).max() / np.abs(s32).max()
    note(f"BF16 scoring: vs the oracle's BF16 emulation {e:.2e}, vs the FP32 network {e32:.2e}")
    # sum order only, unless a hidden activation lands on the other side of a BF16 rounding
    # boundary (one such flip moves a score by ~1e-5 of the largest)
    assert e < 2e-4
    n_mu = 150
    piv, info, st = api.select_points(phi4_d, grid, n_mu, wl.n_occ, XTC_SELECT_LEARNED, model)
    K = int(np.ceil(2.5 * n_mu))
    cand_dev = mlp.candidates(s_bf, K, 7)
    cand_ref = mlp.candidates(ref, K, 7)
    diff = np.array(sorted(set(cand_dev.tolist()) ^ set(cand_ref.tolist())), np.int64)
    note(f"BF16 candidates: {len(cand_dev)} from the device scores, {len(diff)} differ from the "
         f"oracle emulation's")
    assert int(info[6]) == len(cand_dev)
    # a candidate may differ only where the two score sets cross the K-th score within the bound
    kth = np.sort(ref)[::-1][K - 1]
    assert np.all(np.abs(ref[diff] - kth) <= 4e-3 * np.abs(ref).max())
    fp = pivots.select_fused(np.ascontiguousarray(phi4[:, :, cand_dev]), wl.grid_w[cand_dev], n_mu)
    assert np.array_equal(piv, cand_dev[fp.pivots])
    torch.cuda.synchronize()


def test_corrupted_network_falls_back_to_qr(case):
    from paper_2607_17314_amd import XTC_SELECT_LEARNED_JUDGED, XTC_SELECT_QR, api
    wl, phi4, grid, phi4_d = case
    f = api.features(phi4_d, grid, wl.n_occ, wl.atom_xyz)
    model, *_ = _model(api, f.cpu().numpy().astype(np.float64), zero=True, nuclei=wl.atom_xyz, judge=1)
    n_mu = 150
    piv, info, st = api.select_points(phi4_d, grid, n_mu, wl.n_occ, XTC_SELECT_LEARNED_JUDGED, model, 1.25)
    qr, _, _ = api.select_points(phi4_d, grid, n_mu, wl.n_occ, XTC_SELECT_QR)
    note(f"corrupted: status {st}, residual learned {info[3]:.3e} vs QR {info[4]:.3e}, fallback {info[2]}")
    assert st == 3 and info[2] == 1.0
    assert np.array_equal(piv, qr)


def test_training_gains_over_untrained_and_random_proposals():
    """Train on three small chains (labels: the library's QR selection at N_mu = 10 N_orb),
    score two held-out chains with candidates = the 3 N_mu best scores and every 32nd point:
    the trained proposal's judge residual (the mean of the four relative fit residuals) beats
    random points and the untrained network on the same candidate rule, and the judge
    (validation mode: against the QR selection's residual) accepts it at f = 1.25."""
    import torch
    from paper_2607_17314_amd import XTC_SELECT_LEARNED, XTC_SELECT_LEARNED_JUDGED, XTC_SELECT_QR, api
    from workloads import make_config
    train_ids, test_ids = (7, 22, 26), (46, 47)
    stride, kappa = 32, 3.0

    def prep(i):
        wl = make_config("chain", i)
        grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
        phi4, rho = api.eval_orbitals(wl.basis, grid, wl.C_mo, wl.n_occ)
        return wl, grid, phi4

    def resid(phi4, grid, piv):
        _, _, info, _ = api.fit(phi4, grid, piv)
        return float(np.mean(info[4:8]))

    feats, labels = [], []
    for i in train_ids:
        wl, grid, phi4 = prep(i)
        qr, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, XTC_SELECT_QR)
        f = api.features(phi4, grid, wl.n_occ, wl.atom_xyz)
        y = torch.zeros(wl.n_g, dtype=torch.float32, device="cuda")
        y[torch.as_tensor(qr).cuda()] = 1.0
        feats.append(f)
        labels.append(y)
    F = torch.cat(feats, dim=1)
    Y = torch.cat(labels)
    Fn = F.cpu().numpy().astype(np.float64)
    from oracle import mlp as omlp
    p0 = omlp.init_params(64, 0)
    sh, sc = Fn.mean(1).astype(np.float32), (Fn.std(1) + 1e-3).astype(np.float32)
    model = api.MlpModel(p0.astype(np.float32), sh, sc, 64, kappa, None, stride=stride)
    untrained = api.MlpModel(p0.astype(np.float32), sh, sc, 64, kappa, None, stride=stride)
    hist = api.train_mlp(model, F, Y, epochs=8, batch=4096, lr=2e-3, log=note)
    assert hist[-1] < hist[0]
    for tid in test_ids:
        wl, grid, phi4 = prep(tid)
        torch.cuda.synchronize()
        t = time.perf_counter()
        qr, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, XTC_SELECT_QR)
        torch.cuda.synchronize()
        t_qr = time.perf_counter() - t
        res = {}
        for name, mdl in (("trained", model), ("untrained", untrained)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            piv, info, st = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, XTC_SELECT_LEARNED,
                                              mdl.with_nuclei(wl.atom_xyz))
            torch.cuda.synchronize()
            res[name] = (piv, time.perf_counter() - t, int(info[6]))
        rand = np.random.default_rng(0).choice(wl.n_g, wl.n_mu, replace=False)
        r_qr, r_tr, r_un, r_rd = (resid(phi4, grid, p) for p in
                                  (qr, res["trained"][0], res["untrained"][0], rand))
        note(f"held-out chain {tid} (n_g {wl.n_g}, N_mu {wl.n_mu}): judge residual QR {r_qr:.3e} "
             f"({t_qr * 1e3:.0f} ms); trained {r_tr:.3e} ({res['trained'][1] * 1e3:.0f} ms, "
             f"{res['trained'][2]} candidates); untrained {r_un:.3e}; random {r_rd:.3e}")
        assert r_tr < r_rd and r_tr < r_un
        jm = model.with_nuclei(wl.atom_xyz)
        jm.judge = 1
        piv, info, st = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, XTC_SELECT_LEARNED_JUDGED,
                                          jm, 1.25)
        note(f"  judged (validation): status {st}, fallback {info[2]:.0f}, R_L {info[3]:.3e}, "
             f"R_QR {info[4]:.3e}, ratio {info[3] / info[4]:.3f}")
        assert st == 0 and info[2] == 0.0
        assert info[3] <= 1.25 * info[4]
