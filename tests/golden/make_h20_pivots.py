"""Writes tests/golden/h20_pivots.txt: the oracle's fused interpolation points of the
H20 workload (194,000 grid points, 300 orbitals, N_mu = 3000), for the full-size
index-parity test of the GPU selection and as the pivots of the full-size contraction
parity tests. Calls only the oracle and the seeded workload generator.

    python tests/golden/make_h20_pivots.py      (about 10-20 minutes on 8 cores)

File format: comment lines start with '#'; then one line per selection step,
"<channel> <step> <grid index> <relative top-two gap>", channel s (scalar) or g
(gradient), each channel in selection order; the fused order is the scalar pivots,
then the gradient-only pivots (fill-to-target reading of the ISDF section's fusion).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import orbitals, pivots  # noqa: E402
from workloads import make_config  # noqa: E402


def main(name="h20"):
    wl = make_config(name)
    t0 = time.perf_counter()
    phi4 = orbitals.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
    t1 = time.perf_counter()
    fp = pivots.select_fused(phi4, wl.grid_w, wl.n_mu)
    t2 = time.perf_counter()
    out = os.path.join(HERE, f"{name}_pivots.txt")
    with open(out, "w") as f:
        f.write(f"# oracle fused pivots of workload {name}: n_g={wl.n_g} n_orb={wl.n_orb} "
                f"n_mu={wl.n_mu}\n")
        f.write(f"# written by tests/golden/make_h20_pivots.py (oracle.pivots.select_fused); "
                f"orbitals {t1 - t0:.0f} s, selection {t2 - t1:.0f} s\n")
        f.write(f"# scalar steps {len(fp.scalar)}, gradient steps {len(fp.grad)}, "
                f"fused {len(fp.pivots)}, deficient {fp.deficient}\n")
        for ch, st in (("s", fp.scalar_state), ("g", fp.grad_state)):
            for k, (g, gap) in enumerate(zip(st.pivots, st.gaps)):
                f.write(f"{ch} {k} {g} {gap:.6e}\n")
    print(f"wrote {out}: {len(fp.pivots)} pivots in {t2 - t1:.0f} s", flush=True)


if __name__ == "__main__":
    main(*sys.argv[1:])
