"""Shared fixtures of the GPU parity tests: oracle results on seeded workloads
and a relative max-abs metric (max |got - ref| / max |ref|)."""
import sys

import numpy as np


def rel_err(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = np.abs(ref).max()
    if scale == 0.0:
        return float(np.abs(got).max())
    return float(np.abs(got - ref).max() / scale)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class OracleCase:
    """Oracle pipeline on one workload (optionally a grid subset)."""

    def __init__(self, wl, n_mu=None, subset=None, seed=0, channels=None):
        from oracle import contract, fit, orbitals, pivots
        self.wl = wl
        xyz, w = wl.grid_xyz, wl.grid_w
        if subset is not None:
            idx = np.sort(np.random.default_rng(seed).choice(wl.n_g, subset, replace=False))
            xyz, w = np.ascontiguousarray(xyz[:, idx]), np.ascontiguousarray(w[idx])
        self.xyz, self.w = xyz, w
        self.n_mu = n_mu or wl.n_mu
        self.phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, xyz)
        self.rho = orbitals.density(self.phi4, wl.n_occ)
        self.fused = pivots.select_fused(self.phi4, w, self.n_mu)
        self.piv = self.fused.pivots
        self.fit = fit.fit(self.phi4, w, self.piv)
        self._contract = {}

    def contract(self, channels):
        from oracle import contract
        if channels not in self._contract:
            self._contract[channels] = contract.contract(
                self.xyz, self.w, self.wl.corr, self.fit.xi, self.fit.xigrad, self.rho[self.piv],
                self.rho, channels)
        return self._contract[channels]
