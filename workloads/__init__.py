"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

A workload is everything the method takes as given: nuclei, a Cartesian
Gaussian basis, molecular-orbital coefficients, an integration grid, a
correlator and the target ISDF rank. None of the method's own arithmetic lives
here (no grid evaluation of orbitals, no pivoting, no fit, no kernels); see the
per-module docstrings for the readings taken where the paper's inputs (PySCF
grids, Dunning bases, VMC-optimised Jastrows) are not available.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass

import numpy as np

from .basis import Basis, build_basis, shells_from_counts
from .grid import atom_grid
from .integrals import core_orbitals

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903

FORM_EE = 0   # u = sum_k c_k rbar12^{o_k}
FORM_BH = 1   # multi-centre Boys-Handy form (scaled-distance correlator section)


@dataclass
class Correlator:
    form: int
    mno: np.ndarray          # int32 [n_terms, 3]
    c: np.ndarray            # f64 [n_types, n_terms]
    d: float = 1.0
    b: np.ndarray = None     # f64 [n_types]
    nuc_xyz: np.ndarray = None   # f64 [n_nuc, 3]
    nuc_type: np.ndarray = None  # int32 [n_nuc]

    @property
    def n_terms(self) -> int:
        return int(self.mno.shape[0])

    @property
    def n_params(self) -> int:
        return int(self.c.size)

    def with_c(self, c) -> "Correlator":
        return Correlator(self.form, self.mno, np.asarray(c, np.float64).reshape(self.c.shape),
                          self.d, self.b, self.nuc_xyz, self.nuc_type)


@dataclass
class Workload:
    name: str
    atom_Z: np.ndarray
    atom_xyz: np.ndarray
    basis: Basis
    C_mo: np.ndarray         # [n_ao, n_orb]
    n_occ: int
    grid_xyz: np.ndarray     # [3, n_g] SoA
    grid_w: np.ndarray       # [n_g]
    corr: Correlator
    n_mu: int

    @property
    def n_g(self) -> int:
        return int(self.grid_w.shape[0])

    @property
    def n_orb(self) -> int:
        return int(self.C_mo.shape[1])

    @property
    def n_ao(self) -> int:
        return int(self.C_mo.shape[0])


def ee_correlator(n_terms: int = 4, seed: int = 1234, lo: float = -0.5, hi: float = 0.5) -> Correlator:
    """u(r12) = sum_{k=1..n} c_k rbar^{2k}, rbar = r/(1+r), c_k ~ U[lo, hi] (seeded)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo, hi, size=n_terms)
    mno = np.array([[0, 0, 2 * k] for k in range(1, n_terms + 1)], np.int32)
    return Correlator(FORM_EE, mno, c[None, :].copy(), 1.0)


def bh_terms_48():
    """(m, n, o) with 0 <= m <= n <= 3, 0 <= o <= 3, except (0,0,0); then (0,0,o) for o = 4..12."""
    t = [(m, n, o) for m in range(4) for n in range(m, 4) for o in range(4) if (m, n, o) != (0, 0, 0)]
    t += [(0, 0, o) for o in range(4, 13)]
    return np.asarray(t, np.int32)


def bh_correlator(atom_xyz, seed: int = 3) -> Correlator:
    mno = bh_terms_48()
    n_nuc = atom_xyz.shape[0]
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5, 0.5, size=(1, mno.shape[0])) / n_nuc
    return Correlator(FORM_BH, mno, c, 1.0, np.ones(1), np.asarray(atom_xyz, np.float64),
                      np.zeros(n_nuc, np.int32))


def chain(n: int, spacing=None, seed=None, lo=1.4, hi=3.6):
    if spacing is None:
        rng = np.random.default_rng(seed)
        bonds = rng.uniform(lo, hi, size=n - 1)
    else:
        bonds = np.full(n - 1, spacing)
    z = np.concatenate([[0.0], np.cumsum(bonds)])
    z -= z.mean()
    xyz = np.zeros((n, 3))
    xyz[:, 2] = z
    return xyz


def benzene():
    rc = 1.39 * BOHR_PER_ANGSTROM
    rh = (1.39 + 1.09) * BOHR_PER_ANGSTROM
    ang = np.arange(6) * np.pi / 3.0
    C = np.stack([rc * np.cos(ang), rc * np.sin(ang), np.zeros(6)], 1)
    H = np.stack([rh * np.cos(ang), rh * np.sin(ang), np.zeros(6)], 1)
    return np.concatenate([C, H]), np.array([6] * 6 + [1] * 6)


# Per-element shell ladders (l -> count, l -> exponent range); uncontracted.
H_C1 = ({0: 5, 1: 3}, {0: (0.1, 30.0), 1: (0.1, 30.0)})
H_TINY = ({0: 2, 1: 1}, {0: (0.3, 3.0), 1: (0.8, 0.8)})
H_3S2P1D = ({0: 3, 1: 2, 2: 1}, {0: (0.1, 10.0), 1: (0.25, 1.6), 2: (0.7, 0.7)})
C_BIG = ({0: 8, 1: 6, 2: 4, 3: 3, 4: 2, 5: 1},
         {0: (0.08, 3000.0), 1: (0.06, 40.0), 2: (0.15, 4.0), 3: (0.3, 2.0), 4: (0.5, 1.5), 5: (0.9, 0.9)})
H_BIG = ({0: 6, 1: 4, 2: 3, 3: 2, 4: 1},
         {0: (0.05, 80.0), 1: (0.1, 3.0), 2: (0.25, 2.0), 3: (0.5, 1.5), 4: (1.0, 1.0)})

_CACHE = os.environ.get("XTC_WORKLOAD_CACHE",
                        os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                     ".workload_cache"))


def _orbitals_cached(tag: str, basis: Basis, Z: np.ndarray, n_orb: int):
    key = hashlib.sha1(repr((tag, basis.atom_xyz.tobytes(), basis.prim_exp.tobytes(),
                             basis.shell_l.tobytes(), n_orb)).encode()).hexdigest()[:16]
    path = os.path.join(_CACHE, f"orb_{tag}_{key}.npz")
    if os.path.exists(path):
        with np.load(path) as f:
            return f["C"]
    C, _, _ = core_orbitals(basis, Z.astype(np.float64), n_orb)
    try:
        os.makedirs(_CACHE, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, C=C)
        os.replace(tmp, path)
    except OSError:
        pass
    return C


def _molecule(name, xyz, Z, shells_by_Z, n_orb, n_occ, n_rad, n_ang, radii_by_Z, grid_seed, corr, n_mu):
    atom_shells = [shells_from_counts(*shells_by_Z[int(z)]) for z in Z]
    basis = build_basis(xyz, atom_shells)
    C = _orbitals_cached(name, basis, Z, n_orb)
    radii = np.array([radii_by_Z[int(z)] for z in Z])
    gxyz, gw = atom_grid(xyz, radii, n_rad, n_ang, grid_seed)
    return Workload(name, np.asarray(Z), xyz, basis, C, n_occ, gxyz, gw, corr, n_mu)


def make_config(name: str, index: int = 0) -> Workload:
    """Named seeded workloads.

    h2_tiny  : H2 (1.4 bohr), 10 AO -> 4 orbitals, 10 x 26 grid per atom, full pair rank 10.
    h4       : linear H4, 1.8 bohr; 5s3p per atom -> 24 orbitals (2 occ); 50 x 86 grid; N_mu 240.
    h6_small : linear H6, 1.8 bohr; 3s2p1d -> 60 orbitals (3 occ); 30 x 50 grid; N_mu 200.
    h20      : linear H20, bonds U[1.4, 3.6] (seed 2); 3s2p1d -> 300 orbitals (10 occ);
               50 x 194 grid; N_mu 3000.
    h20_bh   : h20 with the 48-term multi-centre Boys-Handy correlator.
    chain    : the index-th of 64 chains H_n, n in [10, 30] (seed 4); N_mu = 10 N_orb.
    benzene  : planar C6H6; 1212 AO -> 1200 orbitals (21 occ); 100 x 974 grid; N_mu 12000.
    """
    H = {1: 0.8, 6: 1.1}   # Treutler-Ahlrichs xi per element
    if name == "h2_tiny":
        xyz = chain(2, 1.4)
        return _molecule(name, xyz, np.array([1, 1]), {1: H_TINY}, 4, 1, 10, 26, H, 11,
                         ee_correlator(), 10)
    if name == "h4":
        xyz = chain(4, 1.8)
        return _molecule(name, xyz, np.array([1] * 4), {1: H_C1}, 24, 2, 50, 86, H, 1,
                         ee_correlator(), 240)
    if name == "h6_small":
        xyz = chain(6, 1.8)
        return _molecule(name, xyz, np.array([1] * 6), {1: H_3S2P1D}, 60, 3, 30, 50, H, 6,
                         ee_correlator(), 200)
    if name in ("h20", "h20_bh"):
        xyz = chain(20, seed=2)
        corr = ee_correlator() if name == "h20" else bh_correlator(xyz)
        return _molecule(name, xyz, np.array([1] * 20), {1: H_3S2P1D}, 300, 10, 50, 194, H, 2,
                         corr, 3000)
    if name == "chain":
        rng = np.random.default_rng(4)
        ns = rng.integers(10, 31, size=64)
        n = int(ns[index])
        xyz = chain(n, seed=1000 + index)
        n_orb = 15 * n
        return _molecule(f"chain{index}", xyz, np.array([1] * n), {1: H_3S2P1D}, n_orb, n // 2,
                         30 + (n - 10), 194, H, 100 + index, ee_correlator(), 10 * n_orb)
    if name == "benzene":
        xyz, Z = benzene()
        return _molecule(name, xyz, Z, {6: C_BIG, 1: H_BIG}, 1200, 21, 100, 974, H, 5,
                         ee_correlator(), 12000)
    raise KeyError(name)


def nuclear_repulsion(wl: Workload) -> float:
    """E_nuc = sum_{I<J} Z_I Z_J / |R_I - R_J| (a constant of the Hamiltonian)."""
    Z, X = wl.atom_Z.astype(np.float64), wl.atom_xyz
    e = 0.0
    for i in range(len(Z)):
        for j in range(i + 1, len(Z)):
            e += Z[i] * Z[j] / float(np.linalg.norm(X[i] - X[j]))
    return e


def vmc_walkers(wl: Workload, n_w: int, seed: int = 0) -> np.ndarray:
    """Initial walkers [n_w, 2 n_occ, 3]: electron i sits near nucleus i mod n_atom (both
    spins), displaced by N(0, 0.7^2) per coordinate (seeded)."""
    rng = np.random.default_rng(seed)
    n_el = 2 * wl.n_occ
    owner = np.arange(n_el) % wl.atom_xyz.shape[0]
    R = wl.atom_xyz[owner][None, :, :] + 0.7 * rng.normal(size=(n_w, n_el, 3))
    return np.ascontiguousarray(R)


def vmc_draws(n_sweeps: int, n_el: int, n_w: int, seed: int = 0):
    """Metropolis draws: standard normals [n_sweeps, n_el, n_w, 3] for the proposals and
    uniforms [n_sweeps, n_el, n_w] on [0, 1) for the acceptance tests (seeded)."""
    rng = np.random.default_rng(seed)
    normals = rng.normal(size=(n_sweeps, n_el, n_w, 3))
    uniforms = rng.random(size=(n_sweeps, n_el, n_w))
    return np.ascontiguousarray(normals), np.ascontiguousarray(uniforms)


__all__ = ["Workload", "Correlator", "make_config", "ee_correlator", "bh_correlator",
           "FORM_EE", "FORM_BH", "Basis", "nuclear_repulsion", "vmc_walkers", "vmc_draws"]
