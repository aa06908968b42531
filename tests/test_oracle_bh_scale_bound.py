"""The a-priori bound behind the split path's BH channel scales (eq. bh-u): with
a = b r / (1 + b r) in [0, 1), |grad a| = b / (1 + b r)^2 <= b, rbar in [0, 1) and
t = 1 / (1 + d r) <= 1, every pair satisfies |grad_1 u| <= N_b + S_b with

    N_b = sum_I b_I sum_{o, m, n} m |C_t[m][n][o]|,
    S_b = d (sum_I sum_{o, m, n} o |C_t[m][n][o]| + sum_o o |c_ee[o]|),

where C_t[m][n][o] is the summed coefficient of the terms (m, n, o) and (n, m, o) of the
nucleus' type t ((m, n) != (0, 0)) and c_ee[o] = sum_t 2 N_t c_t of the (0, 0, o) terms.
The split path scales the gradient channels by 2^(14 - e) and |grad_1 u|^2 by
2^(14 - 2 e), N_b + S_b < 2^e, so no scaled value reaches the FP16 range. Checked on the
oracle's own channels (not on the kernels) at grid points, points within ~1e-3 of the
nuclei and coincident pairs, for one and two nucleus types."""
import numpy as np

from oracle import correlator
from workloads import Correlator, bh_correlator, make_config


def bound(corr):
    n_types = corr.c.shape[0]
    C = np.zeros((n_types, 4, 4, 4))
    cee = np.zeros(64)
    counts = np.bincount(corr.nuc_type, minlength=n_types)
    for k, (m, n, o) in enumerate(corr.mno):
        for t in range(n_types):
            if m == 0 and n == 0:
                cee[o] += 2.0 * counts[t] * corr.c[t, k]
            else:
                C[t, m, n, o] += corr.c[t, k]
                C[t, n, m, o] += corr.c[t, k]
    m_idx = np.arange(4)[None, :, None, None]
    o_idx = np.arange(4)[None, None, None, :]
    nb = sum(corr.b[t] * np.sum(m_idx[0] * np.abs(C[t])) for t in corr.nuc_type)
    sb = sum(np.sum(o_idx[0] * np.abs(C[t])) for t in corr.nuc_type)
    sb = corr.d * (sb + np.sum(np.arange(64) * np.abs(cee)))
    return nb + sb


def _points(wl, rng):
    g = wl.grid_xyz[:, rng.choice(wl.n_g, 300, replace=False)]
    near = np.repeat(wl.atom_xyz.T, 3, axis=1) + rng.normal(scale=1e-3, size=(3, 3 * len(wl.atom_xyz)))
    return np.concatenate([g, near], axis=1)   # grids hold no point at a nucleus itself


def _two_types(corr):
    rng = np.random.default_rng(5)
    n = corr.nuc_xyz.shape[0]
    c = rng.uniform(-0.5, 0.5, size=(2, corr.n_terms)) / n
    return Correlator(corr.form, corr.mno, c, 0.8, np.array([1.0, 2.5]), corr.nuc_xyz,
                      (np.arange(n) % 2).astype(np.int32))


def test_bh_channels_stay_below_the_scale_bound():
    rng = np.random.default_rng(17)
    for name in ("h4", "h6_small"):
        wl = make_config(name)
        X = _points(wl, rng)
        for corr in (bh_correlator(wl.atom_xyz), _two_types(bh_correlator(wl.atom_xyz))):
            B = bound(corr)
            k = correlator.pair_kernels(corr, X, X)
            g = np.sqrt(k["gx"] ** 2 + k["gy"] ** 2 + k["gz"] ** 2)
            # coincident pairs (the diagonal) keep |N|^2 + S^2 in the squared channel
            assert np.all(np.isfinite(k["sq"]))
            assert g.max() <= B, (name, g.max(), B)
            assert k["sq"].max() <= B * B, (name, k["sq"].max(), B * B)
            # the bound is not vacuous: within a few hundred of the largest channel
            assert g.max() > B / 500.0, (name, g.max(), B)
