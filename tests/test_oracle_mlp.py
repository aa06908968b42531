"""Pins of the learned-point oracle: finite-difference gradients, the Adam
closed form on a quadratic, feature definitions and top-k selection."""
import numpy as np

from oracle import mlp, orbitals


def test_loss_gradient_matches_central_differences():
    h = 6
    rng = np.random.default_rng(0)
    p = mlp.init_params(h, 1) + 0.1 * rng.normal(size=mlp.n_params(h))
    x = rng.normal(size=(8, 40))
    y = (rng.random(40) < 0.3).astype(float)
    loss, g = mlp.loss_grad(p, h, x, y, 2.5)
    fd = np.zeros_like(p)
    eps = 1e-6
    for j in range(p.size):
        e = np.zeros_like(p)
        e[j] = eps
        fd[j] = (mlp.loss_grad(p + e, h, x, y, 2.5)[0] - mlp.loss_grad(p - e, h, x, y, 2.5)[0]) / (2 * eps)
    assert np.abs(fd - g).max() < 1e-7 * max(1.0, np.abs(g).max())
    assert mlp.n_params(64) == 4801


def test_adam_on_a_quadratic():
    # for f = 0.5 |p|^2 the first Adam step moves every coordinate by lr (bias-corrected)
    p = np.array([1.0, -2.0, 3.0])
    p1, m, v = mlp.adam(p, p.copy(), np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(p), rtol=1e-6)


def test_features_definitions(h2_tiny):
    phi4 = orbitals.eval_orbitals(h2_tiny.basis, h2_tiny.C_mo, h2_tiny.grid_xyz)
    f = mlp.features(phi4, h2_tiny.grid_w, 1, h2_tiny.grid_xyz, h2_tiny.atom_xyz)
    assert f.shape == (8, h2_tiny.n_g)
    assert np.allclose(np.exp(f[3]), phi4[0, 0] ** 2 + 1e-30)
    # grad rho by central differences at a few points
    idx = [3, 77, 300]
    hh = 1e-5
    for g in idx:
        gr = []
        for c in range(3):
            e = np.zeros((3, 1))
            e[c] = hh
            xp = orbitals.eval_orbitals(h2_tiny.basis, h2_tiny.C_mo, h2_tiny.grid_xyz[:, [g]] + e)[0, 0, 0] ** 2
            xm = orbitals.eval_orbitals(h2_tiny.basis, h2_tiny.C_mo, h2_tiny.grid_xyz[:, [g]] - e)[0, 0, 0] ** 2
            gr.append((xp - xm) / (2 * hh))
        assert np.isclose(np.exp(f[4, g]), np.linalg.norm(gr), rtol=1e-6)
    # the two-nuclei case repeats the farther distance for the third slot
    assert np.allclose(f[6], f[7])


def test_top_candidates_ties_and_order():
    s = np.array([0.5, 2.0, 2.0, -1.0, 2.0, 0.7])
    assert mlp.top_candidates(s, 2).tolist() == [1, 2]
    assert mlp.top_candidates(s, 4).tolist() == [1, 2, 4, 5]


def test_candidates_are_top_scores_and_coverage_points():
    """Candidate rule of the learned proposal: the k best scores (ties to the lowest index)
    united with every stride-th point, sorted; stride 0 is the top-k set alone."""
    from oracle import mlp
    rng = np.random.default_rng(2)
    s = rng.normal(size=1000)
    s[[10, 20, 30]] = 5.0                      # a three-way tie at the top
    c = mlp.candidates(s, 2, 0)
    assert c.tolist() == [10, 20]
    c = mlp.candidates(s, 50, 7)
    top = set(np.argsort(-s, kind="stable")[:50].tolist())
    assert set(c.tolist()) == top | set(range(0, 1000, 7))
    assert np.all(np.diff(c) > 0)
    assert mlp.judge_residual([1.0, 2.0, 3.0, 6.0]) == 3.0


def test_bf16_rounding_matches_torch_and_ties_to_even():
    """to_bf16 against torch's float32 -> bfloat16 conversion (round to nearest even), on
    random values and on exact halfway cases."""
    import torch
    from oracle import mlp
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, size=5000),
                        1.0 + np.array([1, 3, 5, 7]) * 2.0 ** -8]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.to_bf16(x), ref)
    # halfway between 1 and 1 + 2^-7 goes down (even), between 1 + 2^-7 and 1 + 2^-6 up
    assert mlp.to_bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert mlp.to_bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_bf16_forward_is_the_fp32_forward_to_bf16_precision():
    from oracle import mlp
    rng = np.random.default_rng(8)
    p = mlp.init_params(64, 3)
    x = rng.normal(size=(8, 2000))
    s, _ = mlp.forward(p, 64, x)
    sb = mlp.forward_bf16(p, 64, x)
    e = np.abs(sb - s).max() / np.abs(s).max()
    assert 1e-4 < e < 5e-2
