"""Benchmark of the ISDF-xTC hot path on one MI355X.

One step = the whole path over the H20 workload (194,000 grid points, 300
orbitals, N_mu = 3000): orbital values and gradients on the grid, fused
interpolation-point selection, ISDF fit of xi and xi~, and the grid-pair
contraction with every channel (u1, u3, D1, D4, field, energy-scale sums),
with inputs resident in HBM. Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision split|fp64] [--no-fp64-form]

After the timed region (not timed with it) the metric's comparison runs: one whole
step of the plain FP64 GPU form on the same inputs, its time-to-V, the speedup and the
per-block error of the timed form against it (gate 1e-6); and the CPU oracle on a
bounded bra sample with its own orbitals, stored pivots and fit, whose outputs the
device reproduces on the same inputs (gates 1e-6 split, 1e-10 FP64). A failed gate
exits with status 1 after the JSON line.

The roofline object is for the dominant kernel, the stage-1 pair kernel: its
algorithmic flops per launch (8 per row per grid pair, rows = the N_mu
interpolation vectors, plus the two density rows on the FP64 path) over its
average launch duration, timed with HIP events on the launching stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"fp64": 78.6, "f16": 2500.0,   # TFLOP/s, dense MFMA (MI355X datasheet)
         "fp64_vector": 78.6}            # FP64 vector ALU: 256 CUs x 128 FLOP/clk x 2.4 GHz


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", default="h20")
    p.add_argument("--precision", default="split", choices=["fp64", "split"])
    p.add_argument("--no-fp64-form", action="store_true",
                   help="skip the plain FP64 form (by default one whole FP64 step runs after the "
                        "timed region: its time-to-V, the speedup and the per-block error gate)")
    p.add_argument("--xi-fp32", action="store_true",
                   help="store xi in FP32 (split path; default for benzene)")
    p.add_argument("--xigrad-blocks", action="store_true",
                   help="form xi~ per bra super-block from the fit's kept factors instead of "
                        "storing it (default for benzene)")
    p.add_argument("--bra-calls", type=int, default=None,
                   help="split the timed contraction into this many bra-range calls whose partial "
                        "sums add up, each reported as it completes (default 8 for benzene, else 1)")
    p.add_argument("--field-oracle", action="store_true",
                   help="check the device field against the oracle's exact field at sampled bra "
                        "points (default for workloads too large for the oracle's own fit)")
    p.add_argument("--fp64-sample-blocks", type=int, default=None,
                   help="time the plain FP64 form's contraction on this many bra super-blocks "
                        "and extrapolate it to the whole grid (0: one whole FP64 step; default 2 "
                        "for benzene, 0 otherwise); the error gate then compares both forms on "
                        "that bra range")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-bra", type=int, default=1024, help="bra points in the CPU-oracle sample")
    p.add_argument("--exchange", action="store_true",
                   help="also time one step with the xTC Terms 2-3 intermediates X2, X3 formed in the "
                        "same contraction pass (low-rank projector of the occupied orbitals)")
    p.add_argument("--assembly", action="store_true",
                   help="also time the four-index assembly of W = -K + dU in orbital panels and the "
                        "xTC one-body pieces (implies --exchange)")
    p.add_argument("--panel", type=int, default=20, help="orbital panel width of the assembly")
    p.add_argument("--kernel-sample", default=None, metavar="CONFIG",
                   help="also time the split contraction (u3, D1, D4, field) of CONFIG (e.g. benzene) "
                        "on a bra shard of --sample-blocks super-blocks against the full ket range, "
                        "with seeded interpolation vectors of that shape")
    p.add_argument("--sample-blocks", type=int, default=2)
    p.add_argument("--vmc", action="store_true",
                   help="also time one reference-variance VMC optimisation step (sampling, local "
                        "energies with derivatives, Gauss-Newton) on the workload's determinant")
    p.add_argument("--vmc-bh", action="store_true",
                   help="with --vmc, also time the step for the 48-term BH correlator on the "
                        "workload's nuclei (c, d and b per type)")
    p.add_argument("--learned", action="store_true",
                   help="run only the learned-points protocol of the chain configuration: 64 "
                        "seeded chains, the network trained on 48 (QR labels at N_mu = 10 N_orb), "
                        "scored on the 16 held out against QR, the untrained network and random "
                        "points, with both judges, time-to-points and time-to-V")
    p.add_argument("--learned-epochs", type=int, default=6)
    p.add_argument("--learned-stride", type=int, default=32)
    p.add_argument("--learned-kappa", type=float, default=3.0)
    p.add_argument("--walkers", type=int, default=16384)
    p.add_argument("--vmc-sweeps", type=int, default=20)
    p.add_argument("--copy-probe", action="store_true",
                   help="copy 1 GiB device to device once before the timed region (the known-size "
                        "kernel that calibrates the HBM byte counters)")
    p.add_argument("--grad", action="store_true",
                   help="also time the adjoint (xtc_grad) once, with seeded cotangents for u1, u3 "
                        "and the field (D1/D4 cotangents add one recomputation of stage 1)")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the path is single-GPU in this build); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if a.learned:
        learned_protocol(a)
        return
    import numpy as np
    import torch

    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    from workloads import make_config

    wl = make_config(a.config)
    big = a.config == "benzene"
    xi_fp32 = a.xi_fp32 or big
    blocks = a.xigrad_blocks or big
    sample_blocks = a.fp64_sample_blocks if a.fp64_sample_blocks is not None else (2 if big else 0)
    bra_calls = a.bra_calls if a.bra_calls is not None else (8 if big else 1)
    field_oracle = a.field_oracle or big
    if a.grad and blocks:
        print("--grad needs the stored xi~ (no --xigrad-blocks)", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    C_mo = torch.as_tensor(wl.C_mo, device=dev)
    prec = L.XTC_SPLIT_F16 if a.precision == "split" else L.XTC_FP64
    if xi_fp32 and prec != L.XTC_SPLIT_F16:
        print("FP32 xi is read by the split path only", file=sys.stderr)
        sys.exit(2)
    chans = api.ALL_CHANNELS
    torch.cuda.synchronize()

    last = {}

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def step(precision, xp=L.XTC_FP64, piv=None, bra=None):
        """One pass of the path: orbitals, points (unless given), fit, contraction."""
        phi4, rho = api.eval_orbitals(wl.basis, grid, C_mo, wl.n_occ)
        if piv is None:
            piv, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ)
            if big:
                torch.cuda.empty_cache()
                log(f"  points selected ({len(piv)})")
        if blocks:
            xi, _, _, chol, _, rhot = api.fit_ex(phi4, grid, piv, xi_prec=xp, xigrad=False,
                                                 keep_chol=True, rho=rho)
            xig, src = None, api.XiSource(phi4=phi4, chol=chol, xi_prec=xp, rhot=rhot)
        else:
            xi, xig, _, _ = api.fit(phi4, grid, piv)
            src = None
        if big:
            torch.cuda.empty_cache()
            log("  fit done")
        if bra_calls > 1 and bra is None:
            # the bra range in several calls whose partial sums add up (the bra sharding of the
            # design), so that each call's completion is reported as it happens
            per = 16384 * -(-wl.n_g // (bra_calls * 16384))
            out = None
            for b0 in range(0, wl.n_g, per):
                b1 = min(wl.n_g, b0 + per)
                part = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, chans, precision,
                                           src=src, bra=(b0, b1))
                torch.cuda.synchronize()
                log(f"  bra points [{b0}, {b1}) contracted")
                if out is None:
                    out = part
                else:
                    for k in ("u1", "u3", "D1", "D4", "field"):
                        out[k] += part[k]
                    out["escale"] = out["escale"] + part["escale"]
                del part
        else:
            out = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, chans, precision, src=src,
                                      bra=bra)
        last.update(xi=xi, xig=xig, rho=rho, phi4=phi4, src=src)
        return out, piv

    if a.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 1 GiB device-to-device copy done")
    xp_timed = L.XTC_FP32 if xi_fp32 else L.XTC_FP64
    for i in range(a.warmup):
        step(prec, xp_timed)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{a.warmup} done")
    with api.KernelTimer() as kt:
        t0 = time.perf_counter()
        for i in range(a.steps):
            out, piv = step(prec, xp_timed)
            log(f"timed step {i + 1}/{a.steps} enqueued")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
    tm = kt.result
    n_g, n_mu = wl.n_g, len(piv)
    pairs = float(n_g) * n_g
    alg_stage1 = 8.0 * (n_mu + 1) * pairs          # 4 channels x 2 flops x (N_mu + rho row) per pair
    value = alg_stage1 / dt / 1e12

    # dominant kernel: the stage-1 pair kernel, per launch
    s1 = tm["stage1_kernel"]
    launches = max(1, s1["launches"])
    launch_ms = s1["ms"] / launches
    rows_k = n_mu if prec == L.XTC_SPLIT_F16 else n_mu + 2
    per_launch_flops = 8.0 * rows_k * pairs / (launches / a.steps)
    achieved = per_launch_flops / (launch_ms * 1e-3) / 1e12
    peak = PEAKS["f16"] if prec == L.XTC_SPLIT_F16 else PEAKS["fp64"]

    corr_desc = ("4-term e-e correlator" if wl.corr.form == 0 else
                 f"{wl.corr.n_terms}-term multi-centre Boys-Handy correlator ({wl.corr.nuc_xyz.shape[0]} nuclei)")
    system = {"h20": "linear H20 chain", "h20_bh": "linear H20 chain", "h4": "linear H4 chain",
              "benzene": "planar C6H6"}.get(a.config, a.config)
    res = {
        "metric": "ISDF-xTC build time & grid-pair TFLOP/s vs FP64 GPU form at 1e-6 rel err, 1 GPU",
        "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(dt * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f16x2-split/f32acc/f64" if prec == L.XTC_SPLIT_F16 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {system}, {n_g} grid points, {wl.n_orb} orbitals, "
                               f"N_mu={n_mu}, {corr_desc}; time-to-V = orbitals + pivots + fit + "
                               f"contraction (u1,u3,D1,D4,field,escale)",
                   "n_g": n_g, "n_orb": wl.n_orb, "n_mu": n_mu, "precision": a.precision,
                   "xi_storage": "fp32" if xi_fp32 else "fp64",
                   "xigrad": "per bra super-block from the kept factors" if blocks else "stored"},
        "time_to_V_s": round(dt, 4),
        "stage_ms": {k: round(v["ms"] / a.steps, 2) for k, v in tm.items() if v["launches"]},
        "roofline": {"bound": "mfma", "kernel": s1_kernel_name(prec == L.XTC_SPLIT_F16,
                                                              wl.corr.form != 0),
                     "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": (recorded_traffic("stage1_split_h20_hbm_traffic.md")
                                 if prec == L.XTC_SPLIT_F16 and a.config == "h20" else None),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "launch_ms": round(launch_ms, 3), "launches_per_step": launches // a.steps},
    }
    if prec == L.XTC_SPLIT_F16:
        # three FP16 products per algorithmic product (hi.hi, hi.lo, lo.hi)
        res["roofline"]["executed_mfma_frac"] = round(3.0 * achieved / peak, 4)
    if a.grad:
        n = n_mu
        rng = np.random.default_rng(33)
        cot = {k: torch.as_tensor(v, device=dev) for k, v in (
            ("u1", rng.normal(size=(3, n, n)) / n), ("u3", rng.normal(size=(n, n)) / n),
            ("field", rng.normal(size=(3, n_g)) / np.sqrt(n_g)))}
        log("timing the adjoint")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = api.grad(grid, wl.corr, last["xi"], last["xig"], last["rho"], piv, cot)
        torch.cuda.synchronize()
        res["adjoint_s"] = round(time.perf_counter() - t0, 4)
        res["adjoint_n_params"] = int(g.numel())
        res["adjoint_cotangents"] = "u1, u3, field"
        log(f"adjoint done in {res['adjoint_s']} s")
    if a.exchange or a.assembly:
        res["exchange"], inter = exchange_bench(wl, grid, C_mo, chans, prec, log)
        if a.assembly:
            res["assembly"] = assembly_bench(wl, inter, a.panel, log)
        del inter
        if not a.no_cpu_baseline:
            log("timing the CPU oracle sample of the exchange intermediates")
            res["exchange"]["cpu_baseline"] = exchange_cpu_baseline(wl, 128)
            if a.assembly:
                log("timing the CPU oracle sample of the assembly")
                res["assembly"]["cpu_baseline"] = assembly_cpu_baseline(wl, 1)
    if a.vmc:
        res["vmc"] = vmc_bench(wl, a.walkers, a.vmc_sweeps, log)
        if not a.no_cpu_baseline:
            log("timing the CPU oracle sample of the VMC step")
            res["vmc"]["cpu_baseline"] = vmc_cpu_baseline(wl)
        if a.vmc_bh:
            res["vmc"]["bh"] = vmc_bh_bench(wl, a.walkers, log)
            if not a.no_cpu_baseline:
                log("timing the CPU oracle sample of the BH local energies")
                res["vmc"]["bh"]["cpu_baseline"] = vmc_bh_cpu_baseline(wl)
    if a.kernel_sample:
        res["kernel_sample"] = kernel_sample(a.kernel_sample, a.sample_blocks, log)
    gate_ok = True
    field_full = out["field"]
    if not a.no_fp64_form and prec != L.XTC_FP64 and sample_blocks == 0:
        # the metric's comparison: the plain FP64 GPU form, one whole step (same inputs, so
        # the same pivots), and the per-block error of the timed form against it
        log("plain FP64 form: one whole step")
        torch.cuda.synchronize()
        with api.KernelTimer() as kt64:
            t0 = time.perf_counter()
            ref, piv64 = step(L.XTC_FP64)
            torch.cuda.synchronize()
            t64 = time.perf_counter() - t0
        errs = block_errors(out, ref)
        gate_ok = bool(np.array_equal(piv, piv64)) and max(errs.values()) <= GATE
        res["fp64_form"] = {"time_to_V_s": round(t64, 4),
                            "stage_ms": {k: round(v["ms"], 2) for k, v in kt64.result.items()
                                         if v["launches"]}}
        res["speedup_vs_fp64_form"] = round(t64 / dt, 3)
        res["max_rel_err_vs_fp64"] = errs
        res["accuracy_gate"] = {"bound": GATE, "per": "output block, max|got - ref| / max|ref|",
                                "pass": gate_ok}
        log(f"FP64 form {t64:.2f} s ({t64 / dt:.2f}x the timed form); worst block error "
            f"{max(errs.values()):.2e}")
        del ref
    elif not a.no_fp64_form and prec != L.XTC_FP64:
        # the plain FP64 form's contraction is timed on the first sample_blocks bra
        # super-blocks (its cost is linear in the bra points) after its own FP64 fit on the
        # same points; orbitals and point selection are the same work as the timed step's
        nb = min(n_g, sample_blocks * 16384)
        bra = (0, nb)
        escale_full = out["escale"]
        del out
        log(f"timed form on the bra sample [0, {nb})")
        sp = api.kernel_contract(grid, wl.corr, last["xi"], last["xig"], last["rho"], piv, chans, prec,
                                 src=last["src"], bra=bra)
        torch.cuda.synchronize()
        sp = {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in sp.items()}
        last["xi"] = last["xig"] = last["src"] = None
        torch.cuda.empty_cache()
        phi4, rho = last["phi4"], last["rho"]
        log("plain FP64 form: FP64 fit")
        with api.KernelTimer() as kt64:
            t0 = time.perf_counter()
            if blocks:
                xi64, _, _, chol64, _, rhot64 = api.fit_ex(phi4, grid, piv, xigrad=False,
                                                           keep_chol=True, rho=rho)
                xig64, src64 = None, api.XiSource(phi4=phi4, chol=chol64, rhot=rhot64)
            else:
                xi64, xig64, _, _ = api.fit(phi4, grid, piv)
                src64 = None
            torch.cuda.synchronize()
            t_fit = time.perf_counter() - t0
            log(f"plain FP64 form: contraction on the bra sample [0, {nb})")
            t0 = time.perf_counter()
            ref = api.kernel_contract(grid, wl.corr, xi64, xig64, rho, piv, chans, L.XTC_FP64,
                                      src=src64, bra=bra)
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t0
        ref = {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in ref.items()}
        del xi64, xig64, src64
        t_shared = (tm["orbitals"]["ms"] + tm["select"]["ms"]) * 1e-3 / a.steps
        t64 = t_shared + t_fit + t_s * n_g / nb
        errs = block_errors(sp, ref, cols=bra)
        gate_ok = max(errs.values()) <= GATE
        res["fp64_form"] = {"time_to_V_s": round(t64, 2), "extrapolated": True,
                            "how": f"orbitals + points of the timed step ({t_shared:.2f} s) + its own "
                                   f"FP64 fit ({t_fit:.2f} s) + its contraction timed on {nb} of "
                                   f"{n_g} bra points ({t_s:.2f} s) scaled by {n_g / nb:.2f}",
                            "stage_ms": {k: round(v["ms"], 2) for k, v in kt64.result.items()
                                         if v["launches"]}}
        res["speedup_vs_fp64_form"] = round(t64 / dt, 3)
        res["max_rel_err_vs_fp64"] = errs
        res["accuracy_gate"] = {"bound": GATE, "per": "output block, max|got - ref| / max|ref|, "
                                f"both forms on bra points [0, {nb})", "pass": gate_ok}
        res["escale"] = [float(x) for x in escale_full]
        log(f"FP64 form {t64:.1f} s extrapolated ({t64 / dt:.2f}x the timed form); worst block "
            f"error on the sample {max(errs.values()):.2e}")
        del ref, sp
    if not a.no_cpu_baseline and field_oracle:
        log("timing the CPU oracle's exact field on sampled bra points")
        res["cpu_baseline"], ferr = field_oracle_sample(wl, last["rho"], field_full, log)
        res["max_rel_err_vs_oracle"] = {"field": ferr}
        ok = ferr <= 1e-10
        res["oracle_gate"] = {"bounds": {"field": 1e-10}, "pass": ok}
        gate_ok = gate_ok and ok
    elif not a.no_cpu_baseline:
        log("timing the CPU oracle sample")
        res["cpu_baseline"], oerr = cpu_baseline(wl, n_mu, a.cpu_bra, a.config, grid, piv, log)
        if oerr is not None:
            res["max_rel_err_vs_oracle"] = oerr
            ok = max(oerr["split"].values()) <= GATE and max(oerr["fp64"].values()) <= 1e-10
            res["oracle_gate"] = {"bounds": {"split": GATE, "fp64": 1e-10}, "pass": ok}
            gate_ok = gate_ok and ok
    print(json.dumps(res), flush=True)
    if not gate_ok:
        print("accuracy gate failed", file=sys.stderr, flush=True)
        sys.exit(1)


GATE = 1e-6   # the mixed path's bound per output block (max |got - ref| / max |ref|)


def s1_kernel_name(split, bh):
    if not split:
        if bh:
            return ("stage-1 FP64 products (k_stage1_f64_pv; the FP64 pair values of "
                    "k_bh_pairs_f64 are timed under stage_ms.bh_pairs)")
        return "stage-1 pair kernel (k_stage1_f64)"
    if bh:
        return ("stage-1 split products (k_stage1_split_pv; the FP64 pair values of k_bh_pairs "
                "are timed under stage_ms.bh_pairs)")
    return "stage-1 pair kernel (k_stage1_split)"


def block_errors(out, ref, cols=None):
    """max |got - ref| / max |ref| for every output block (the field on cols, if given) and
    the largest relative error of the energy-scale scalars."""
    import numpy as np
    errs = {}
    for k in ("u1", "u3", "D1", "D4", "field"):
        g, r = out[k], ref[k]
        if not isinstance(g, np.ndarray):
            g = g.cpu().numpy()
        if not isinstance(r, np.ndarray):
            r = r.cpu().numpy()
        if k == "field" and cols is not None:
            g, r = g[:, cols[0]:cols[1]], r[:, cols[0]:cols[1]]
        errs[k] = float(np.abs(g - r).max() / np.abs(r).max())
    errs["escale"] = float(np.max(np.abs(out["escale"] - ref["escale"]) / np.abs(ref["escale"])))
    return errs


def exchange_bench(wl, grid, C_mo, chans, prec, log):
    """One whole step with X2 and X3 formed in the contraction pass from the same calG
    panels. Algorithmic flops of the X part: the X products, 2 N_pair N_mu per grid
    point and product (one for X2, three for X3; N_pair = the q <= s orbital pairs),
    plus the projections R, Q (8 N_orb N_occ N_mu per grid point)."""
    import torch

    from paper_2607_17314_amd import api
    n_orb, n_q = wl.n_orb, wl.n_occ
    lq = torch.zeros((n_orb, n_q), dtype=torch.float64, device="cuda")
    lq[torch.arange(n_q), torch.arange(n_q)] = 1.0     # closed-shell projector: occupied columns
    log("timing one step with the exchange intermediates")
    torch.cuda.synchronize()
    with api.KernelTimer() as kt:
        t0 = time.perf_counter()
        phi4, rho = api.eval_orbitals(wl.basis, grid, C_mo, wl.n_occ)
        piv, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ)
        xi, xig, _, _ = api.fit(phi4, grid, piv)
        phi_piv = phi4[0][:, torch.as_tensor(piv, device="cuda")].contiguous()
        out = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, chans, prec,
                                  exchange={"phi_piv": phi_piv, "lq": lq})
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    tm = kt.result
    n_mu = len(piv)
    npair = n_orb * (n_orb + 1) // 2
    fx = 2.0 * npair * n_mu * wl.n_g * 4
    frq = 8.0 * n_orb * n_q * n_mu * wl.n_g
    x_ms = tm["x_pairs"]["ms"] + tm["x_gemm"]["ms"]
    res = {"time_to_V_with_X_s": round(dt, 4), "n_q": n_q, "n_pair": npair,
           "x_part_s": round(x_ms * 1e-3, 4),
           "x_products_tflops": round(fx / (tm["x_gemm"]["ms"] * 1e-3) / 1e12, 2),
           "x_part_tflops": round((fx + frq) / (x_ms * 1e-3) / 1e12, 2),
           "stage_ms": {k: round(v["ms"], 2) for k, v in tm.items() if v["launches"]},
           "x_abs_max": [float(out["X2"].abs().max()), float(out["X3"].abs().max())]}
    xm = tm["x_mfma"]
    if xm["launches"]:
        ach = fx / (xm["ms"] * 1e-3) / 1e12
        res["roofline"] = {"bound": "mfma", "kernel": "split X-product kernel (k_gemm_split_nt)",
                           "achieved": round(ach, 2), "peak": PEAKS["f16"], "unit": "TFLOP/s",
                           "frac": round(ach / PEAKS["f16"], 4),
                           "executed_mfma_frac": round(3.0 * ach / PEAKS["f16"], 4), "traffic": None,
                           "launch_ms": round(xm["ms"] / xm["launches"], 3),
                           "launches": xm["launches"]}
    log(f"step with exchange done in {dt:.3f} s")
    inter = {"phi4_piv": phi4[:, :, torch.as_tensor(piv, device="cuda")].contiguous(),
             "u1": out["u1"], "u3": out["u3"], "D1": out["D1"], "D4": out["D4"],
             "X2": out["X2"], "X3": out["X3"]}
    return res, inter


def assembly_bench(wl, inter, width, log):
    """W = -K + dU for every p in panels of `width` orbitals into one reused panel buffer
    (FP64), after one prepare; then dh, f and E0. Per panel the product has
    2 (width N_orb) N_orb^2 (4 N_mu) flops and writes width N_orb^3 FP64 elements."""
    import torch

    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    n, n_mu = wl.n_orb, inter["u3"].shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    asm = api.Assembly(inter["phi4_piv"], inter["u1"], inter["u3"], inter["D1"], inter["D4"],
                       inter["X2"], inter["X3"], outputs=L.XTC_ASM_W)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    buf = None
    with api.KernelTimer() as kt:
        t0 = time.perf_counter()
        for p0 in range(0, n, width):
            p1 = min(n, p0 + width)
            buf = asm.panel(p0, p1, out=buf if buf is not None and p1 - p0 == width else None)
        torch.cuda.synchronize()
        t_pan = time.perf_counter() - t0
    wmax = float(buf["W"].abs().max())
    del asm, buf
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dh, f, e0 = api.one_body(inter["phi4_piv"], inter["u1"], inter["u3"], inter["D1"], inter["D4"],
                             inter["X2"], inter["X3"], wl.n_occ, 0.0)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    flops = 2.0 * n * n * n * n * 4 * n_mu
    res = {"panel_width": width, "prepare_s": round(t_prep, 4), "panels_s": round(t_pan, 4),
           "one_body_s": round(t_one, 4), "w_elements": n ** 4,
           "panel_tflops": round(flops / t_pan / 1e12, 2),
           "panel_write_gbs": round(8.0 * n ** 4 / t_pan / 1e9, 1),
           "e0_minus_enuc": e0, "w_abs_max_last_panel": wmax,
           "f_abs_max": float(f.abs().max())}
    ap = kt.result["asm_panel"]
    if ap["launches"]:
        ach = flops / (ap["ms"] * 1e-3) / 1e12
        res["roofline"] = {"bound": "mfma", "kernel": "assembly panel kernel (k_asm_panel)",
                           "achieved": round(ach, 2), "peak": PEAKS["fp64"], "unit": "TFLOP/s",
                           "frac": round(ach / PEAKS["fp64"], 4), "traffic": None,
                           "launch_ms": round(ap["ms"] / ap["launches"], 3),
                           "launches": ap["launches"]}
    log(f"assembly: prepare {t_prep:.3f} s, panels {t_pan:.3f} s, one-body {t_one:.3f} s")
    return res


def recorded_traffic(summary: str):
    """Calibrated HBM bytes per launch from a committed counter summary under profiles/,
    or None when the summary is missing or the kernel source has changed since (the SHA-1
    of its source files, concatenated in the order listed, differs from the one recorded
    with the counters)."""
    import hashlib
    import re
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(root, "profiles", summary)).read()
    except OSError:
        return None
    t = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    src = re.search(r"^source: (.+)$", text, re.M)
    sha = re.search(r"^source_sha1: ([0-9a-f]{40})$", text, re.M)
    if not (t and src and sha):
        return None
    try:
        h = hashlib.sha1()
        for f in src.group(1).split(", "):
            h.update(open(os.path.join(root, f.strip()), "rb").read())
        now = h.hexdigest()
    except OSError:
        return None
    return int(t.group(1)) if now == sha.group(1) else None


def _vmc_flops(wl, n_el):
    """Algorithmic FP64 work of the VMC kernels (exp counted as one operation):
    per proposal, the AO row (4 per primitive: r^2 term, exp, scale, sum; 3 per AO),
    the occupied-orbital row (2 n_ao n_occ), the ratio row (2 n_occ^2) and, when accepted,
    the Sherman-Morrison update (2 n_occ^2); per walker for the local energy, five AO
    quantities (12 per primitive, 30 per AO) and five orbital rows per electron, two
    inverses (2 n_occ^3 each), the Slater ratios (8 n_occ per electron) and the Jastrow
    pair sums (about 40 + 30 n_terms per ordered pair)."""
    n_prim = int(wl.basis.shell_prim_start[-1])
    n_ao, n = wl.n_ao, wl.n_occ
    move = 4 * n_prim + 3 * n_ao + 2 * n_ao * n + 2 * n * n
    update = 2 * n * n
    energy = (n_el * (12 * n_prim + 30 * n_ao + 10 * n_ao * n + 8 * n) + 2 * 2 * n ** 3
              + n_el * (n_el - 1) * (40 + 30 * wl.corr.n_terms))
    return move, update, energy


def vmc_bench(wl, n_w, n_sweeps, log):
    """One optimisation step of the VMC section at the workload's reference determinant:
    n_sweeps Metropolis sweeps of every electron of n_w walkers, the local energies with
    their (c, d) derivatives, and the Gauss-Newton step. Draws come from a seeded device
    generator before the timed region."""
    import numpy as np
    import torch

    from paper_2607_17314_amd import api
    from workloads import nuclear_repulsion, vmc_walkers
    sysv = api.VmcSystem.from_workload(wl, nuclear_repulsion(wl))
    n_el = sysv.n_el
    R = torch.as_tensor(vmc_walkers(wl, n_w, seed=1), device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    nrm = torch.randn((n_sweeps, n_el, n_w, 3), dtype=torch.float64, device="cuda", generator=g)
    uni = torch.rand((n_sweeps, n_el, n_w), dtype=torch.float64, device="cuda", generator=g)
    api.vmc_sample(sysv, R, n_sweeps, 0.6, nrm, uni)          # warm-up and equilibration
    E, dE = api.vmc_local_energy(sysv, wl.corr, R)
    api.vmc_gn_step(E, dE, 1e-3, 0.5)
    torch.cuda.synchronize()
    with api.KernelTimer() as kt:
        t0 = time.perf_counter()
        acc = api.vmc_sample(sysv, R, n_sweeps, 0.6, nrm, uni)
        E, dE = api.vmc_local_energy(sysv, wl.corr, R)
        delta, stats = api.vmc_gn_step(E, dE, 1e-3, 0.5)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    tm = kt.result
    st = stats.cpu().numpy()
    rate = float(acc.sum()) / (n_w * n_el * n_sweeps)
    moves = float(n_w) * n_el * n_sweeps
    f_move, f_upd, f_en = _vmc_flops(wl, n_el)
    samp_ms, en_ms, gn_ms = tm["vmc_sample"]["ms"], tm["vmc_energy"]["ms"], tm["vmc_gn"]["ms"]
    samp_flops = moves * (f_move + rate * f_upd)
    res = {"walkers": n_w, "sweeps": n_sweeps, "electrons": n_el, "n_ao": wl.n_ao,
           "step_s": round(dt, 4), "sample_ms": round(samp_ms, 2), "energy_ms": round(en_ms, 2),
           "gn_ms": round(gn_ms, 3), "acceptance": round(rate, 4),
           "moves_per_s": round(moves / (samp_ms * 1e-3), 1),
           "local_energies_per_s": round(n_w / (en_ms * 1e-3), 1),
           "clipped_mean": float(st[2]), "clipped_variance": float(st[3]), "n_clipped": int(st[4])}
    # the dominant kernel of the step (sampling or energies), FP64 vector ALU roofline
    if samp_ms >= en_ms:
        ach = samp_flops / (samp_ms * 1e-3) / 1e12
        kern, launch_ms = "VMC sampler (k_vmc_sweeps)", samp_ms
    else:
        ach = n_w * f_en / (en_ms * 1e-3) / 1e12
        kern, launch_ms = "VMC local energy (k_vmc_energy)", en_ms
    res["roofline"] = {"bound": "alu", "kernel": kern, "achieved": round(ach, 3),
                       "peak": PEAKS["fp64_vector"], "unit": "TFLOP/s",
                       "frac": round(ach / PEAKS["fp64_vector"], 4), "traffic": None,
                       "launch_ms": round(launch_ms, 3), "launches": 1}
    res["energy_tflops"] = round(n_w * f_en / (en_ms * 1e-3) / 1e12, 3)
    res["sample_tflops"] = round(samp_flops / (samp_ms * 1e-3) / 1e12, 3)
    log(f"vmc: step {dt:.3f} s (sample {samp_ms:.1f} ms, energies {en_ms:.1f} ms, GN {gn_ms:.2f} ms), "
        f"acceptance {rate:.3f}")
    return res


def vmc_bh_bench(wl, n_w, log):
    """Local energies with every (c, d, b) derivative and the Gauss-Newton step for the
    48-term BH correlator on the workload's nuclei, on n_w equilibrated walkers."""
    import torch

    from paper_2607_17314_amd import api
    from workloads import bh_correlator, nuclear_repulsion, vmc_walkers
    corr = bh_correlator(wl.atom_xyz)
    sysv = api.VmcSystem.from_workload(wl, nuclear_repulsion(wl))
    R = torch.as_tensor(vmc_walkers(wl, n_w, seed=1), device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    nrm = torch.randn((20, sysv.n_el, n_w, 3), dtype=torch.float64, device="cuda", generator=g)
    uni = torch.rand((20, sysv.n_el, n_w), dtype=torch.float64, device="cuda", generator=g)
    api.vmc_sample(sysv, R, 20, 0.6, nrm, uni)
    E, dE = api.vmc_local_energy(sysv, corr, R)
    torch.cuda.synchronize()
    with api.KernelTimer() as kt:
        t0 = time.perf_counter()
        E, dE = api.vmc_local_energy(sysv, corr, R)
        delta, stats = api.vmc_gn_step(E, dE, 1e-2, 0.5)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    en_ms, gn_ms = kt.result["vmc_energy"]["ms"], kt.result["vmc_gn"]["ms"]
    st = stats.cpu().numpy()
    log(f"vmc bh: energies {en_ms:.1f} ms, GN {gn_ms:.2f} ms for {dE.shape[1]} parameters")
    return {"correlator": f"{corr.n_terms}-term BH, {corr.nuc_xyz.shape[0]} nuclei",
            "parameters": int(dE.shape[1]), "energy_ms": round(en_ms, 2), "gn_ms": round(gn_ms, 3),
            "step_s": round(dt, 4), "local_energies_per_s": round(n_w / (en_ms * 1e-3), 1),
            "clipped_variance": float(st[3])}


def vmc_bh_cpu_baseline(wl, n_en=3):
    """The oracle's BH local energies with complex-step derivatives in every parameter."""
    import numpy as np

    from oracle import vmc
    from workloads import bh_correlator, nuclear_repulsion, vmc_walkers
    corr = bh_correlator(wl.atom_xyz)
    R = vmc_walkers(wl, n_en, seed=1)
    t0 = time.perf_counter()
    vmc.local_energy_grad(wl.basis, np.ascontiguousarray(wl.C_mo[:, :wl.n_occ]), wl.atom_xyz,
                          wl.atom_Z.astype(np.float64), nuclear_repulsion(wl), corr, R)
    t = time.perf_counter() - t0
    return {"kind": "oracle", "local_energies_per_s": round(n_en / t, 3), "cores": 1,
            "unit": "local energies (with every derivative) per second",
            "sample": f"{n_en} walkers, complex step over {corr.c.size + 2} parameters"}


def vmc_cpu_baseline(wl, n_w=1024, n_sweeps=2, n_en=256):
    """The oracle's sampler (n_sweeps sweeps of n_w walkers) and local energies with
    complex-step derivatives (n_en walkers) on the host."""
    import numpy as np

    from oracle import vmc
    from workloads import nuclear_repulsion, vmc_draws, vmc_walkers
    n_el = 2 * wl.n_occ
    C_occ = np.ascontiguousarray(wl.C_mo[:, :wl.n_occ])
    R0 = vmc_walkers(wl, n_w, seed=1)
    nrm, uni = vmc_draws(n_sweeps, n_el, n_w, seed=2)
    t0 = time.perf_counter()
    vmc.metropolis(wl.basis, C_occ, R0, 0.6, nrm, uni)
    t_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    vmc.local_energy_grad(wl.basis, C_occ, wl.atom_xyz, wl.atom_Z.astype(np.float64),
                          nuclear_repulsion(wl), wl.corr, R0[:n_en])
    t_e = time.perf_counter() - t0
    return {"kind": "oracle", "moves_per_s": round(n_w * n_el * n_sweeps / t_s, 1),
            "local_energies_per_s": round(n_en / t_e, 2), "unit": "moves/s, local energies/s",
            "cores": 1, "sample": f"{n_w} walkers x {n_sweeps} sweep(s); {n_en} walkers' "
                                  f"energies with {wl.corr.n_terms + 1} derivatives (element-wise "
                                  f"NumPy on small arrays: one thread)"}


def kernel_sample(config, nblk, log):
    """Stage 1 + stage 2 of the split contraction at another workload's shape on a bra
    shard of nblk super-blocks of 16,384 points against every ket point: the work one
    GPU does when the bra index is sharded. The interpolation vectors are seeded N(0,1)
    rows of the right shape (the kernels' cost does not depend on their values)."""
    import numpy as np
    import torch

    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    from workloads import make_config
    log(f"building the {config} workload")
    wl = make_config(config)
    n_g, n_mu = wl.n_g, wl.n_mu
    grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    xi = torch.randn((n_mu, n_g), dtype=torch.float64, device="cuda", generator=gen)
    rho = torch.rand(n_g, dtype=torch.float64, device="cuda", generator=gen)
    piv = np.sort(np.random.default_rng(7).choice(n_g, n_mu, replace=False))
    nb = min(n_g, nblk * 16384)
    ch = L.XTC_U3 | L.XTC_D1 | L.XTC_D4 | L.XTC_FIELD
    log(f"{config}: split contraction over bra points [0, {nb}) of {n_g}, N_mu={n_mu}")
    torch.cuda.synchronize()
    with api.KernelTimer() as kt:
        t0 = time.perf_counter()
        api.kernel_contract(grid, wl.corr, xi, None, rho, piv, ch, L.XTC_SPLIT_F16, bra=(0, nb))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    tm = kt.result
    s1 = tm["stage1_kernel"]
    pairs = float(nb) * n_g
    per_launch = 8.0 * n_mu * pairs / s1["launches"]
    ach = per_launch / (s1["ms"] / s1["launches"] * 1e-3) / 1e12
    res = {"workload": f"{config}: {n_g} grid points, {wl.n_orb} orbitals, N_mu={n_mu}",
           "bra_points": nb, "ket_points": n_g, "time_s": round(dt, 3),
           "stage_ms": {k: round(v["ms"], 2) for k, v in tm.items() if v["launches"]},
           "stage1_full_grid_estimate_s": round(tm["stage1"]["ms"] * 1e-3 * n_g / nb, 1),
           "roofline": {"bound": "mfma", "kernel": "stage-1 pair kernel (k_stage1_split)",
                        "achieved": round(ach, 2), "peak": PEAKS["f16"], "unit": "TFLOP/s",
                        "frac": round(ach / PEAKS["f16"], 4),
                        "executed_mfma_frac": round(3.0 * ach / PEAKS["f16"], 4), "traffic": None,
                        "launch_ms": round(s1["ms"] / s1["launches"], 3),
                        "launches": s1["launches"]}}
    log(f"{config} sample done in {dt:.2f} s")
    del xi
    return res


def exchange_cpu_baseline(wl, n_bra):
    """The oracle's exchange intermediates on a bounded sample: calG of n_bra bra points
    over every ket point and X2, X3 over those bra points, on seeded inputs of the
    workload's shapes. Work counted as on the GPU: the X products (8 N_pair N_mu per bra
    point) and calG (6 N_mu per grid pair)."""
    import numpy as np

    from oracle import exchange as oex
    n_mu, n, nq = wl.n_mu, wl.n_orb, wl.n_occ
    rng = np.random.default_rng(0)
    xi = rng.standard_normal((n_mu, wl.n_g))
    phi = rng.standard_normal((n, n_mu)) / np.sqrt(n)
    LQ = np.zeros((n, nq))
    LQ[np.arange(nq), np.arange(nq)] = 1.0
    cores = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    cG = oex.calG(wl.grid_xyz, wl.grid_w, wl.corr, xi, bra=(0, n_bra))
    oex.x_terms(phi, np.arange(n_mu), xi[:, :n_bra], cG, wl.grid_w[:n_bra], LQ)
    dt = time.perf_counter() - t0
    npair = n * (n + 1) // 2
    flops = (8.0 * npair * n_mu + 6.0 * n_mu * wl.n_g) * n_bra
    return {"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"calG and X2, X3 over {n_bra} bra points x {wl.n_g} ket points, N_mu={n_mu}, "
                      f"{n} orbitals, n_q={nq}; {dt:.1f} s"}


def assembly_cpu_baseline(wl, n_p=1):
    """The oracle's W panel for n_p orbitals (assembly.w_panel, from the definitions) on
    seeded inputs of the workload's shapes; work counted as on the GPU,
    2 n_p N_orb^3 4 N_mu flops."""
    import numpy as np

    from oracle import assembly as oasm
    n_mu, n = wl.n_mu, wl.n_orb
    rng = np.random.default_rng(1)
    phi = rng.standard_normal((4, n, n_mu)) / np.sqrt(n)
    u1 = rng.standard_normal((3, n_mu, n_mu)) / n_mu
    u3, D1, D4 = (rng.standard_normal((n_mu, n_mu)) / n_mu for _ in range(3))
    X = rng.standard_normal((n, n, n_mu)) / n_mu
    cores = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oasm.w_panel(phi, u1, u3, D1, D4, X, 0, n_p)
    dt = time.perf_counter() - t0
    flops = 2.0 * n_p * n ** 3 * 4 * n_mu
    return {"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"W panel of {n_p} of {n} orbitals, N_mu={n_mu}; {dt:.1f} s"}


def field_oracle_sample(wl, rho_dev, field_dev, log, n_blk=4, width=256, seed=9):
    """The exact field A_gamma(g) = sum_g' w' rho(g') grad_1 u(g, g') (the density row of
    stage 1, over every ket point) at n_blk seeded runs of `width` bra points, from the
    oracle's own orbitals and density, against the device field of the timed step; also
    the device density against the oracle's at those points. Returns (cpu_baseline, max
    relative error of the field)."""
    import numpy as np

    from oracle import contract as oc
    from oracle import orbitals as oorb
    rng = np.random.default_rng(seed)
    starts = np.sort(rng.choice(wl.n_g // width, n_blk, replace=False)) * width
    t0 = time.perf_counter()
    C_occ = np.ascontiguousarray(wl.C_mo[:, :wl.n_occ])
    rho = np.empty(wl.n_g)
    for g0 in range(0, wl.n_g, 65536):      # orbital values are pointwise: chunks are exact
        g1 = min(wl.n_g, g0 + 65536)
        phi_occ = oorb.eval_orbitals(wl.basis, C_occ, np.ascontiguousarray(wl.grid_xyz[:, g0:g1]))
        rho[g0:g1] = oorb.density(phi_occ, wl.n_occ)
    log(f"  oracle density on {wl.n_g} points in {time.perf_counter() - t0:.1f} s")
    zero = np.zeros((1, wl.n_g))
    fld = field_dev.cpu().numpy()
    rd = rho_dev.cpu().numpy()
    errs, erho = [], []
    cores = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    for b in starts:
        r = oc.contract(wl.grid_xyz, wl.grid_w, wl.corr, zero, None, np.zeros(1), rho, 32,
                        bra_block=16, bra_range=(int(b), int(b) + width))
        ref = r["field"][:, b:b + width]
        got = fld[:, b:b + width]
        errs.append(float(np.abs(got - ref).max() / np.abs(ref).max()))
        erho.append(float(np.abs(rd[b:b + width] - rho[b:b + width]).max() / np.abs(rho).max()))
    dt = time.perf_counter() - t0
    flops = 6.0 * n_blk * width * wl.n_g          # the field's 3 channels x 2 flops per pair
    log(f"  field at {n_blk} x {width} bra points: worst rel err {max(errs):.2e} ({dt:.1f} s)")
    return ({"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
             "sample": f"exact field of {n_blk} x {width} bra points (starts {starts.tolist()}) x "
                       f"{wl.n_g} ket points from the oracle's density; {dt:.1f} s",
             "density_max_rel_err": max(erho)}, max(errs))


def _chain_workload(i):
    from workloads import make_config
    return make_config("chain", i)


def learned_protocol(a):
    """The chain configuration's protocol for the learned proposer. The 64 workloads are
    built on the host by a small pool of worker processes (started before the GPU is
    touched; they do no GPU work). Training: QR labels, features and the four-system QR
    residual of chains 0..47; Adam on the pooled points (the library's kernels); judge 0's
    reference log R_ref = a + b log(N_mu / N_orb) fitted on those residuals (every chain has
    N_mu = 10 N_orb, so b = 0 and a is the mean of log R_QR). Held out, chains 48..63:
    QR, the trained and untrained proposals (candidates: the kappa N_mu best scores and
    every stride-th point), random points, judge 0 (production) and judge 1 (validation),
    time-to-points, and time-to-V (orbitals, points, fit, split contraction) with and
    without the network, with the ISDF error of the energy-scale scalar E3 against its
    exact counterpart."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    os.environ["OMP_NUM_THREADS"] = "2"
    pool = ProcessPoolExecutor(8, mp_context=mp.get_context("spawn"))
    jobs = [pool.submit(_chain_workload, i) for i in range(64)]   # workers start here
    import numpy as np
    import torch

    from oracle import mlp as omlp   # only the network's seeded initial parameters
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def sync():
        torch.cuda.synchronize()

    def judge_resid(phi4, grid, piv):
        _, _, info, _ = api.fit(phi4, grid, piv)
        return float(np.mean(info[4:8]))

    t_start = time.perf_counter()
    feats, labels, logr = [], [], []
    for i in range(48):
        wl = jobs[i].result()
        grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
        phi4, _ = api.eval_orbitals(wl.basis, grid, wl.C_mo, wl.n_occ)
        qr, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, L.XTC_SELECT_QR)
        feats.append(api.features(phi4, grid, wl.n_occ, wl.atom_xyz))
        y = torch.zeros(wl.n_g, dtype=torch.float32, device="cuda")
        y[torch.as_tensor(qr).cuda()] = 1.0
        labels.append(y)
        r = judge_resid(phi4, grid, qr)
        logr.append((np.log(wl.n_mu / wl.n_orb), np.log(r)))
        del phi4, grid
        torch.cuda.empty_cache()
        log(f"train chain {i}: H{wl.atom_xyz.shape[0]}, {wl.n_g} points, N_mu {wl.n_mu}, R_QR {r:.3e}")
    F = torch.cat(feats, dim=1)
    Y = torch.cat(labels)
    del feats, labels
    Fn = F.cpu().numpy().astype(np.float64)
    sh, sc = Fn.mean(1).astype(np.float32), (Fn.std(1) + 1e-3).astype(np.float32)
    del Fn
    p0 = omlp.init_params(64, 0).astype(np.float32)
    x = np.array([v[0] for v in logr]); lr_ = np.array([v[1] for v in logr])
    if np.ptp(x) < 1e-12:
        ref_a, ref_b = float(lr_.mean()), 0.0
    else:
        ref_b, ref_a = (float(v) for v in np.polyfit(x, lr_, 1))
    kw = dict(hidden=64, kappa=a.learned_kappa, stride=a.learned_stride)
    model = api.MlpModel(p0, sh, sc, ref_a=ref_a, ref_b=ref_b, **kw)
    untrained = api.MlpModel(p0, sh, sc, **kw)
    sync()
    t0 = time.perf_counter()
    hist = api.train_mlp(model, F, Y, epochs=a.learned_epochs, batch=4096, lr=2e-3, log=log)
    sync()
    t_train = time.perf_counter() - t0
    n_train_points, n_pos = int(Y.numel()), int(Y.sum())
    del F, Y
    torch.cuda.empty_cache()
    rows = []
    for i in range(48, 64):
        wl = jobs[i].result()
        grid = api.DeviceGrid.from_host(wl.grid_xyz, wl.grid_w)
        phi4, rho = api.eval_orbitals(wl.basis, grid, wl.C_mo, wl.n_occ)
        sync()
        t0 = time.perf_counter()
        qr, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, L.XTC_SELECT_QR)
        sync()
        t_qr = time.perf_counter() - t0
        m0 = model.with_nuclei(wl.atom_xyz)
        t0 = time.perf_counter()
        p0_, i0, s0 = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, L.XTC_SELECT_LEARNED_JUDGED, m0, 1.25)
        sync()
        t_l0 = time.perf_counter() - t0
        m1 = model.with_nuclei(wl.atom_xyz)
        m1.judge = 1
        _, i1, s1 = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, L.XTC_SELECT_LEARNED_JUDGED, m1, 1.25)
        t0 = time.perf_counter()
        pl, il, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, L.XTC_SELECT_LEARNED, m0)
        sync()
        t_l = time.perf_counter() - t0
        pu, _, _ = api.select_points(phi4, grid, wl.n_mu, wl.n_occ, L.XTC_SELECT_LEARNED,
                                     untrained.with_nuclei(wl.atom_xyz))
        rand = np.random.default_rng(i).choice(wl.n_g, wl.n_mu, replace=False)
        r_qr, r_l, r_u, r_r = (judge_resid(phi4, grid, p) for p in (qr, pl, pu, rand))

        def to_v(piv):
            sync()
            t = time.perf_counter()
            xi, xig, _, _ = api.fit(phi4, grid, piv)
            out = api.kernel_contract(grid, wl.corr, xi, xig, rho, piv, api.ALL_CHANNELS,
                                      L.XTC_SPLIT_F16)
            sync()
            e = out["escale"]
            return time.perf_counter() - t, abs(e[0] - e[3]) / abs(e[3])

        t_fc_qr, e3_qr = to_v(qr)
        t_fc_l, e3_l = to_v(p0_)
        row = {"chain": i, "atoms": int(wl.atom_xyz.shape[0]), "n_g": wl.n_g, "n_mu": wl.n_mu,
               "R_qr": r_qr, "R_trained": r_l, "R_untrained": r_u, "R_random": r_r,
               "ratio_trained": r_l / r_qr, "candidates": int(il[6]),
               "judge0_accept": s0 == 0, "judge1_accept": s1 == 0,
               "t_points_qr_s": t_qr, "t_points_learned_s": t_l, "t_points_judged0_s": t_l0,
               "time_to_V_qr_s": t_qr + t_fc_qr, "time_to_V_learned_s": t_l0 + t_fc_l,
               "E3_isdf_err_qr": e3_qr, "E3_isdf_err_learned": e3_l}
        rows.append(row)
        del phi4, rho, grid
        torch.cuda.empty_cache()
        log(f"held-out chain {i}: H{row['atoms']}, R_L/R_QR {row['ratio_trained']:.3f} (untrained "
            f"{r_u / r_qr:.1f}, random {r_r / r_qr:.1f}), judges {int(row['judge0_accept'])}"
            f"{int(row['judge1_accept'])}, points {t_qr * 1e3:.0f} -> {t_l * 1e3:.0f} ms "
            f"(judged {t_l0 * 1e3:.0f} ms)")
    pool.shutdown()
    ratios = np.array([r["ratio_trained"] for r in rows])
    agree = np.mean([r["judge0_accept"] == r["judge1_accept"] for r in rows])
    summ = {
        "protocol": "64 seeded chains H10-H30; trained on chains 0-47, scored on 48-63; "
                    f"candidates = {a.learned_kappa} N_mu best scores + every "
                    f"{a.learned_stride}th point; judge f = 1.25 on the mean of the four relative "
                    "fit residuals",
        "train_points": n_train_points, "train_positives": n_pos, "epochs": a.learned_epochs,
        "train_s": round(t_train, 2), "loss_history": [round(h, 4) for h in hist],
        "judge0_reference": {"a": ref_a, "b": ref_b},
        "ratio_trained_median": float(np.median(ratios)), "ratio_trained_max": float(ratios.max()),
        "ratio_untrained_median": float(np.median([r["R_untrained"] / r["R_qr"] for r in rows])),
        "ratio_random_median": float(np.median([r["R_random"] / r["R_qr"] for r in rows])),
        "judge1_accept_rate": float(np.mean([r["judge1_accept"] for r in rows])),
        "judge0_accept_rate": float(np.mean([r["judge0_accept"] for r in rows])),
        "judge_agreement_rate": float(agree),
        "t_points_qr_s": float(np.sum([r["t_points_qr_s"] for r in rows])),
        "t_points_learned_s": float(np.sum([r["t_points_learned_s"] for r in rows])),
        "t_points_judged0_s": float(np.sum([r["t_points_judged0_s"] for r in rows])),
        "time_to_V_qr_s": float(np.sum([r["time_to_V_qr_s"] for r in rows])),
        "time_to_V_learned_s": float(np.sum([r["time_to_V_learned_s"] for r in rows])),
        "E3_isdf_err_ratio_median": float(np.median([r["E3_isdf_err_learned"] / r["E3_isdf_err_qr"]
                                                     for r in rows])),
        "wall_s": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps({"learned": summ, "held_out": rows}), flush=True)


def read_pivots(config):
    """The oracle's fused pivots of a workload, stored under tests/golden/ by the committed
    script there (fused order: scalar pivots, then gradient-only pivots), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{config}_pivots.txt")
    if not os.path.exists(path):
        return None
    sc, gr = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            ch, _, g, _ = line.split()
            (sc if ch == "s" else gr).append(int(g))
    ss = set(sc)
    return sc + [g for g in gr if g not in ss]


def cpu_baseline(wl, n_mu, n_bra, config, grid, gpu_piv, log):
    """The FP64 CPU oracle's contraction on a bounded sample (n_bra bra points against every
    ket point, all channels) on the oracle's own inputs: its orbitals, its stored fused
    pivots and its fit of xi (all columns) and xi~ (the sample's columns). The same inputs go
    to the device (split and FP64) on the same bra range, and the per-block errors against
    the oracle are returned. Workloads without stored pivots use seeded N(0, 1) rows of the
    right shape and no error check."""
    import numpy as np
    import torch

    from oracle import contract as oc
    from oracle import fit as ofit
    from oracle import orbitals as oorb
    from paper_2607_17314_amd import _lib as L
    from paper_2607_17314_amd import api
    cores = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    piv = read_pivots(config)
    chans = 1 | 2 | 8 | 16 | 32 | 64
    if piv is None:
        rng = np.random.default_rng(0)
        xi = rng.standard_normal((n_mu, wl.n_g))
        xig = rng.standard_normal((3, n_mu, wl.n_g))
        rho = rng.random(wl.n_g)
        pv = np.arange(n_mu)
        kind = "seeded N(0,1) interpolation vectors"
    else:
        pv = np.asarray(piv, np.int64)
        log("  oracle orbitals and fit on the stored pivots (not timed)")
        phi4 = oorb.eval_orbitals(wl.basis, wl.C_mo, wl.grid_xyz)
        rho = oorb.density(phi4, wl.n_occ)
        fr = ofit.fit(phi4, wl.grid_w, pv, grad_cols=np.arange(n_bra))
        del phi4
        xi = fr.xi
        xig = np.zeros((3, n_mu, wl.n_g))        # untouched pages stay unmapped
        xig[:, :, :n_bra] = fr.xigrad
        kind = "the oracle's xi and xi~ on its own fused pivots"
    t0 = time.perf_counter()
    ref = oc.contract(wl.grid_xyz, wl.grid_w, wl.corr, xi, xig, rho[pv], rho, chans,
                      bra_range=(0, n_bra))
    dt = time.perf_counter() - t0
    flops = 8.0 * (n_mu + 1) * n_bra * wl.n_g
    res = {"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"stage 1 + stage 2 of {n_bra} bra points x {wl.n_g} ket points, N_mu={n_mu}, "
                     f"all channels, {kind}; {dt:.1f} s"}
    if piv is None:
        return res, None
    res["gpu_pivots_equal_oracle"] = bool(np.array_equal(np.asarray(gpu_piv), pv))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    xi_d, rho_d = t(xi), t(rho)
    xig_d = torch.zeros((3, n_mu, wl.n_g), dtype=torch.float64, device="cuda")
    xig_d[:, :, :n_bra] = t(fr.xigrad)
    errs = {}
    for name, prec in (("split", L.XTC_SPLIT_F16), ("fp64", L.XTC_FP64)):
        out = api.kernel_contract(grid, wl.corr, xi_d, xig_d, rho_d, pv, chans, prec, bra=(0, n_bra))
        torch.cuda.synchronize()
        errs[name] = block_errors(out, ref, cols=(0, n_bra))
        log(f"  {name} vs oracle on the sample: worst block {max(errs[name].values()):.2e}")
    del xig_d, xi_d
    return res, errs


if __name__ == "__main__":
    main()
