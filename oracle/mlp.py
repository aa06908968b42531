"""Learned interpolation-point scorer (not part of the paper: the method's
interpolation points come from pivoted Cholesky; this proposer is trained on
those selections and judged against them).

Features of grid point g (natural logarithms, eps = 1e-30):
  f0 = log(w_g), f1 = log(sum_p phi_p^2), f2 = log(sum_{p,c} (d_c phi_p)^2),
  f3 = log(rho_gamma), f4 = log|grad rho_gamma| with grad rho_gamma = 2 sum_occ phi_i grad phi_i,
  f5..f7 = log of the distances to the three nearest nuclei (repeating the last
  one when there are fewer than three nuclei);
z-scored with a shift and scale fitted on the training points.
Network: x -> h1 = silu(W1 x + b1) -> h2 = silu(W2 h1 + b2) -> s = W3 . h2 + b3 (a logit).
Loss: weighted binary cross-entropy on the logit,
  L = mean_g [ pw y_g softplus(-s_g) + (1 - y_g) softplus(s_g) ],  pw = N_neg / N_pos.
Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8).
Parameter packing (4801 for hidden 64): W1[h][8], b1[h], W2[h][h], b2[h], W3[h], b3.

Pinned by: central finite differences of the loss gradient (FP64) and the
closed-form Adam update of a quadratic.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-30
N_FEAT = 8


def n_params(h: int) -> int:
    return N_FEAT * h + h + h * h + h + h + 1


def unpack(p, h):
    o = 0
    W1 = p[o:o + h * N_FEAT].reshape(h, N_FEAT); o += h * N_FEAT
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + h]; o += h
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def init_params(h: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(h, N_FEAT)) / np.sqrt(N_FEAT)
    W2 = rng.normal(size=(h, h)) / np.sqrt(h)
    W3 = rng.normal(size=h) / np.sqrt(h)
    return np.concatenate([W1.ravel(), np.zeros(h), W2.ravel(), np.zeros(h), W3, [0.0]])


def features(phi4, w, n_occ, xyz, nuc):
    phi, dphi = phi4[0], phi4[1:4]
    n2 = np.einsum("pg,pg->g", phi, phi)
    g2 = np.einsum("cpg,cpg->g", dphi, dphi)
    rho = np.einsum("pg,pg->g", phi[:n_occ], phi[:n_occ])
    grho = 2.0 * np.einsum("pg,cpg->cg", phi[:n_occ], dphi[:, :n_occ])
    grn = np.sqrt(np.einsum("cg,cg->g", grho, grho))
    dist = np.linalg.norm(xyz[:, :, None] - np.asarray(nuc).T[:, None, :], axis=0)   # [n_g, n_nuc]
    dist = np.sort(dist, axis=1)
    if dist.shape[1] < 3:
        dist = np.concatenate([dist] + [dist[:, -1:]] * (3 - dist.shape[1]), axis=1)
    f = np.stack([w, n2, g2, rho, grn, dist[:, 0], dist[:, 1], dist[:, 2]])
    return np.log(f + EPS)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, h, x):
    """x: normalised features [8, n]; returns logits [n] and the pre-activations."""
    W1, b1, W2, b2, W3, b3 = unpack(p, h)
    z1 = W1 @ x + b1[:, None]
    a1 = silu(z1)
    z2 = W2 @ a1 + b2[:, None]
    a2 = silu(z2)
    s = W3 @ a2 + b3
    return s, (z1, a1, z2, a2)


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned in float64: BF16 keeps the
    upper 16 bits of the FP32 word (8 exponent bits, 7 stored significand bits)."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, h, x):
    """The scores with the weights and the inputs of each product rounded to BF16 (the
    z-scored features, W1, SiLU(z1), W2; FP32 values in, products and sums exact in FP64),
    biases, SiLU and the last layer in full precision: the arithmetic of the BF16
    matrix-core scoring, up to the order and precision of its FP32 sums."""
    W1, b1, W2, b2, W3, b3 = unpack(p, h)
    z1 = to_bf16(W1) @ to_bf16(x) + b1[:, None]
    a1 = to_bf16(silu(z1))
    z2 = to_bf16(W2) @ a1 + b2[:, None]
    return W3 @ silu(z2) + b3


def softplus(x):
    return np.logaddexp(0.0, x)


def loss_grad(p, h, x, y, pw):
    """Weighted BCE loss and its gradient w.r.t. the packed parameters."""
    n = x.shape[1]
    s, (z1, a1, z2, a2) = forward(p, h, x)
    loss = float(np.mean(pw * y * softplus(-s) + (1.0 - y) * softplus(s)))
    sig = 1.0 / (1.0 + np.exp(-s))
    ds = (-pw * y * (1.0 - sig) + (1.0 - y) * sig) / n          # dL/ds
    W1, b1, W2, b2, W3, b3 = unpack(p, h)
    dW3 = a2 @ ds
    db3 = ds.sum()
    dz2 = (W3[:, None] * ds[None, :]) * dsilu(z2)
    dW2 = dz2 @ a1.T
    db2 = dz2.sum(1)
    dz1 = (W2.T @ dz2) * dsilu(z1)
    dW1 = dz1 @ x.T
    db1 = dz1.sum(1)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3]])
    return loss, g


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t starts at 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def top_candidates(scores, k):
    """Indices of the k largest scores, ties to the lowest index, in ascending index order."""
    order = np.lexsort((np.arange(scores.shape[0]), -scores))
    return np.sort(order[:k])


def candidates(scores, k, stride):
    """The learned proposal's candidate set: the k largest scores (ties to the lowest index)
    and every stride-th grid point (coverage; stride 0: none), in ascending index order."""
    top = top_candidates(scores, k)
    if stride <= 0:
        return top
    return np.union1d(top, np.arange(0, scores.shape[0], stride))


def judge_residual(resid_rel):
    """The judge's residual: the mean of the four relative fit residuals (scalar, x, y, z)."""
    r = np.asarray(resid_rel, np.float64)
    return 0.25 * ((r[0] + r[1]) + (r[2] + r[3]))
