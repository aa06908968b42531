"""Synthetic Cartesian Gaussian basis sets for the seeded workloads.

The paper builds its orbitals from Dunning correlation-consistent bases through
PySCF (Computational Details; Alg. 2, first two steps). Neither is available
here, so each workload uses uncontracted Cartesian Gaussians with geometric
exponent ladders. This module only *describes* the basis (centres, angular
powers, exponents, normalisation constants). Evaluating it on grid points is
part of the method and lives in the oracle and in the HIP library separately.

AO ordering: shell-major; inside a shell of angular momentum l the Cartesian
components (i, j, k), i + j + k = l, run with i descending, then j descending.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import factorial, pi, sqrt

import numpy as np


def cart_components(l: int):
    """Cartesian powers (i, j, k) of one shell, in the library's AO order."""
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def _dfact(n: int) -> int:
    """Double factorial with (-1)!! = 0!! = 1."""
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def radial_norm(alpha: float, l: int) -> float:
    """Normalisation of x^l exp(-alpha r^2) up to the per-component factor."""
    return (2.0 * alpha / pi) ** 0.75 * (4.0 * alpha) ** (l / 2.0)


def component_factor(i: int, j: int, k: int) -> float:
    """Per-component factor that completes the Cartesian normalisation."""
    return 1.0 / sqrt(_dfact(2 * i - 1) * _dfact(2 * j - 1) * _dfact(2 * k - 1))


@dataclass
class Basis:
    """Flat, device-friendly description of a Cartesian Gaussian basis.

    chi_a(r) = comp_factor[a] * x^i y^j z^k * sum_p prim_coef[p] exp(-prim_exp[p] |r - R|^2)
    with (x, y, z) = r - R_{shell_center}, primitives p of the AO's shell.
    """

    atom_xyz: np.ndarray            # [n_atom, 3] bohr
    shell_center: np.ndarray        # int32 [n_shell]
    shell_l: np.ndarray             # int32 [n_shell]
    shell_prim_start: np.ndarray    # int32 [n_shell + 1]
    prim_exp: np.ndarray            # f64 [n_prim]
    prim_coef: np.ndarray           # f64 [n_prim], includes radial_norm
    ao_shell: np.ndarray = field(default=None)    # int32 [n_ao]
    ao_pow: np.ndarray = field(default=None)      # int32 [n_ao, 3]
    comp_factor: np.ndarray = field(default=None)  # f64 [n_ao]
    shell_ao_start: np.ndarray = field(default=None)  # int32 [n_shell + 1]

    def __post_init__(self):
        ao_shell, ao_pow, comp, starts = [], [], [], [0]
        for s, l in enumerate(self.shell_l):
            for (i, j, k) in cart_components(int(l)):
                ao_shell.append(s)
                ao_pow.append((i, j, k))
                comp.append(component_factor(i, j, k))
            starts.append(len(ao_shell))
        self.ao_shell = np.asarray(ao_shell, np.int32)
        self.ao_pow = np.asarray(ao_pow, np.int32).reshape(-1, 3)
        self.comp_factor = np.asarray(comp, np.float64)
        self.shell_ao_start = np.asarray(starts, np.int32)

    @property
    def n_ao(self) -> int:
        return int(self.ao_shell.shape[0])

    @property
    def n_shell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def max_l(self) -> int:
        return int(self.shell_l.max())


def build_basis(atom_xyz: np.ndarray, atom_shells: list) -> Basis:
    """atom_shells[a] = list of (l, exponent) uncontracted shells of atom a."""
    centers, ls, starts, exps, coefs = [], [], [0], [], []
    for a, shells in enumerate(atom_shells):
        for (l, alpha) in shells:
            centers.append(a)
            ls.append(l)
            exps.append(alpha)
            coefs.append(radial_norm(alpha, l))
            starts.append(len(exps))
    return Basis(
        atom_xyz=np.asarray(atom_xyz, np.float64).reshape(-1, 3),
        shell_center=np.asarray(centers, np.int32),
        shell_l=np.asarray(ls, np.int32),
        shell_prim_start=np.asarray(starts, np.int32),
        prim_exp=np.asarray(exps, np.float64),
        prim_coef=np.asarray(coefs, np.float64),
    )


def ladder(lo: float, hi: float, n: int) -> list:
    """Geometric exponent ladder from lo to hi with n entries (n = 1: geometric mean)."""
    if n == 1:
        return [float(np.sqrt(lo * hi))]
    return [float(x) for x in np.geomspace(lo, hi, n)]


def shells_from_counts(counts: dict, ranges: dict) -> list:
    """counts = {l: n_shells}; ranges = {l: (lo, hi)} exponent ladders per l."""
    out = []
    for l in sorted(counts):
        for alpha in ladder(*ranges[l], counts[l]):
            out.append((l, alpha))
    return out


def n_cart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


__all__ = ["Basis", "build_basis", "cart_components", "ladder", "shells_from_counts",
           "radial_norm", "component_factor", "n_cart", "factorial"]
