"""Benchmark: mode-amplitude Langevin steps of 4096 dsDNA chains of 256 bp.

One step = the whole hot path over the batch: bond-mode transform, bond
forces, coupling transform, per-mode update with Philox noise, centre of
mass in FP64, plus the observable sampling every 100 steps.  Inputs are
synthetic (straight chains, random orientation, jitter 0.01 a, seed 1) and
resident in HBM before the timed region.

Prints one JSON line.  ``value`` is chain-steps/s of the mixed-precision
path (default split-BF16); the same-GPU FP64 plain form is timed beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"bf16x3": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}  # dense MFMA, MI355X


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="modes",
                    choices=["modes", "uneven", "shear", "mc", "dtmax", "dtmax_t", "wlc", "euler",
                             "stats", "fp64", "coarse"],
                    help="modes: 4096 x 256 bp (the headline line); uneven: 8192 chains of "
                         "64..512 bp in one launch; shear: 2048 x 256 bp under simple shear "
                         "at Wi = 1, 10, 100 (tumbling and extension, FP32 vs FP64); mc: "
                         "Metropolis sweeps of 4096 x 256 bp; dtmax: equilibrium values of the "
                         "mode dynamics against Monte Carlo over a range of time steps")
    ap.add_argument("--shear-steps", type=int, default=1000000)
    ap.add_argument("--coarse-chains", type=int, default=2048)
    ap.add_argument("--coarse-samples", type=int, default=32768)
    ap.add_argument("--stats-steps", type=int, default=100000,
                    help="steps of each run of the stats workload")
    ap.add_argument("--profile-launches", type=int, default=0, metavar="N",
                    help="only run N fused launches of 200 steps of the default workload "
                         "(for hardware-counter passes) and exit")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "fp32"])
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--dtmax-lengths", default="64,128,256",
                    help="chain lengths (beads) of the dtmax workload; 512 is N = 511")
    ap.add_argument("--dtmax-dtaus", default="",
                    help="time steps of the dtmax workload (comma list), instead of each "
                         "length's default bracket")
    ap.add_argument("--uneven-chains", type=int, default=8192,
                    help="chains of the uneven workload (1024: one GPU's share of 8192 on 8)")
    ap.add_argument("--beads", type=int, default=256)
    ap.add_argument("--dtau", type=float, default=100.0)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--no-graphs", action="store_true", help="eager launches instead of "
                    "replayed graphs of the sampling blocks")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--table-mode", default="auto",
                    choices=["auto", "resident", "streamed", "split", "split8"],
                    help="force a tile shape of the fused launch where it exists (modes and "
                         "uneven workloads; overrides the autotuner)")
    ap.add_argument("--fp64-steps", type=int, default=0,
                    help="steps of the FP64 plain-form leg (0: the same window as the timed "
                         "mixed-precision steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024,
                    help="chains in the oracle's timed sample")
    ap.add_argument("--cpu-steps", type=int, default=600)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def time_steps(ctx, torch, n, stream):
    """HIP-event time of ctx.step_modes(n) on the context's stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.step_modes(n)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


# the sources the fused kernel is compiled from
FUSED_SOURCES = ("dm_fused.hip", "dm_fused.h", "dm_rng.h")


def fused_source_sha256():
    """SHA-256 of the fused kernel's sources, concatenated in FUSED_SOURCES order."""
    import hashlib
    h = hashlib.sha256()
    for name in FUSED_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_3487_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(precision, B, M):
    """HBM bytes per fused launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes, or None if the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "fused_kernel_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    sha = fused_source_sha256()
    key = f"{precision}-{B}x{M}"
    if rec.get("source_sha256") != sha or key not in rec.get("workloads", {}):
        return None
    return rec["workloads"][key]["hbm_bytes_per_launch"]


def executed_flops(precision, M, jc):
    """Matrix flops the fused kernel executes per chain-step (padding
    excluded): u = chi R as two M/2 x M/2 products per component (3 M^2),
    the coupling product over the kept mode rows p <= 32 jc (3 rows M), and
    three BF16 products per FP32 product on the split-BF16 path."""
    rows = min(32 * jc, M - 1)
    return (3.0 if precision == "bf16x3" else 1.0) * (3.0 * M * M + 3.0 * rows * M)


def host_cpu():
    """CPU model name and logical CPU count of this host (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(args, nu, ts):
    """The oracle on a sample of the same workload: the first --cpu-sample
    chains of the library's initial state (the oracle's own generator of the
    same recipe, seed 1), --cpu-steps mode steps."""
    import numpy as np
    import oracle
    sub = oracle.config_chains(args.beads, args.cpu_sample, nu, seed=1)
    R = oracle.modes_from_positions(sub)
    oracle.step_modes(R[:2], nu, ts, args.dtau, 1, seed=1)  # load + warm
    t0 = time.perf_counter()
    oracle.step_modes(R, nu, ts, args.dtau, args.cpu_steps, seed=1,
                      chain_ids=np.arange(sub.shape[0]))
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    host = host_cpu()
    # one core: the figure to set beside the paper's single-chain desktop runs
    one = sub[:32]
    R1 = oracle.modes_from_positions(one)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.step_modes(R1, nu, ts, args.dtau, 50, seed=1, chain_ids=np.arange(32))
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": sub.shape[0] * args.cpu_steps / dt, "unit": "chain-steps/s",
            "cores": cores, "kind": "oracle", "cpu_model": host["model"],
            "host_logical_cpus": host["logical_cpus"],
            "sample": f"{sub.shape[0]} chains x {args.beads} beads x {args.cpu_steps} mode "
                      f"steps (FP64 plain C, OpenMP over chains), {dt:.1f} s",
            "single_core": {"value": 32 * 50 / dt1, "unit": "chain-steps/s",
                            "sample": f"32 chains x 50 steps on one thread, {dt1:.1f} s"}}


LENGTHS = [64, 96, 128, 192, 256, 384, 512]
DTAU_OF = {64: 10.0, 96: 10.0, 128: 50.0, 192: 50.0, 256: 100.0, 384: 100.0, 512: 100.0}


def uneven_workload(args):
    """--uneven-chains chains (8192) with lengths uniform over LENGTHS (seed
    2), each at its length's time step, advanced in one fused launch per
    sampling block."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    B = args.uneven_chains
    beads = inputs.mixed_lengths(B, LENGTHS, seed=2)
    chains = inputs.mixed_chains(beads, b, seed=2)
    steps = args.steps if args.steps != 20000 else 4000
    dts = [DTAU_OF[m] for m in LENGTHS]
    ctx = Context(chains, seed=2, precision=args.precision, stream=stream)
    ctx.set_params(LENGTHS, dts, T_star=T_STAR_DSDNA, nu=NU_DSDNA,
                   sample_every=args.sample_every, use_graphs=not args.no_graphs,
                   autotune=not args.no_autotune, table_mode=args.table_mode)
    tiling, report = ctx.tiling(), ctx.tuning_report()
    ctx.step_modes(min(args.warmup, 500))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step_modes(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    finite = bool(np.all(np.isfinite(ctx.chain_observables())))
    ctx.close()
    c64 = Context(chains, seed=2, precision="fp64", stream=stream)
    c64.set_params(LENGTHS, dts, T_star=T_STAR_DSDNA, nu=NU_DSDNA, sample_every=args.sample_every,
                   use_graphs=not args.no_graphs)
    c64.step_modes(args.sample_every)
    t64 = time_steps(c64, torch, 2 * args.sample_every, stream)
    c64.close()
    rate = B * steps / wall
    out = {
        "metric": "chain-steps/s, uneven ensemble (one launch for all lengths)",
        "value": rate, "unit": "chain-steps/s", "n_gpus": 1, "steps": steps,
        "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16x3": "bf16x3-f32acc", "fp32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{B} chains, lengths uniform over {LENGTHS} bp (seed 2), "
                               f"dtau {dts}, observables every {args.sample_every} steps",
                   "graphs": not args.no_graphs, "autotune": not args.no_autotune,
                   "table_mode": args.table_mode},
        "bead_steps_per_s": rate * float(np.mean(beads)),
        "fp64_plain_chain_steps_per_s": B * 2 * args.sample_every / t64,
        "speedup_vs_fp64_plain": rate / (B * 2 * args.sample_every / t64),
        "state_finite": finite,
        "tiling": [{k: (float(v) if k == "item_us" else int(v)) for k, v in t.items()}
                   for t in tiling],
        "tuning_report": report.strip().splitlines(),
    }
    print(json.dumps(out))


def shear_workload(args):
    """2048 chains of 256 bp under simple shear at Wi = 1, 10, 100 relative
    to the slowest mode (gamma_dot = Wi zeta_1), dtau = 100: tumbling times
    and mean extension of the reduced-precision path against FP64 on the
    GPU, same initial state and Philox streams."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    B, M, dtau, se = 2048, 256, 100.0, 1000
    z1 = 16 * NU_DSDNA * np.sin(np.pi / (2 * M)) ** 4
    pos = inputs.straight_chains(B, M, b, seed=1, random_orientation=True)
    prec = args.precision if args.precision != "bf16x3" else "fp32"
    res = []
    for wi in (1.0, 10.0, 100.0):
        row = {"Wi": wi, "gamma_dot": wi * z1}
        for p in (prec, "fp64"):
            ctx = Context(pos, seed=7, precision=p, stream=stream)
            ctx.set_params([M], [dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA, gamma_dot=wi * z1,
                           sample_every=se, use_graphs=p != "fp64")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            left = args.shear_steps
            while left > 0:  # progress lines for long runs
                n = min(left, 100000)
                ctx.step_modes(n)
                left -= n
                torch.cuda.synchronize()
                print(f"# Wi={wi:g} {p}: {args.shear_steps - left} steps", file=sys.stderr,
                      flush=True)
            wall = time.perf_counter() - t0
            a = ctx.accumulators()[0]
            ctx.close()
            ns = a["n_samples"]
            row[p] = {
                "chain_steps_per_s": B * args.shear_steps / wall,
                "mean_extension": a["xspan"] / ns / B / ((M - 1) * b),
                "L2_over_contour2": a["L2"] / ns / B / ((M - 1) * b) ** 2,
                "tumbles": a["tumbles"],
                "tumbling_times": a["n_tau"],
                "mean_tumbling_time_tau": (a["tau"] / a["n_tau"] * dtau) if a["n_tau"] else None,
                "tumble_hist_octaves_of_steps": [int(x) for x in a["tumble_hist"]],
            }
        r, f = row[prec], row["fp64"]
        row["extension_rel_diff"] = r["mean_extension"] / f["mean_extension"] - 1
        res.append(row)
    print(json.dumps({"workload": f"shear: {B} chains x {M} bp, dtau = {dtau:g}, "
                                  f"{args.shear_steps} steps, samples every {se}",
                      "precision": prec, "results": res}))


def stats_workload(args):
    """Statistics of the reduced-precision paths against the FP64 plain form
    on the GPU at the batched configurations (1024 x 128 bp at dtau 50,
    4096 x 256 and 1024 x 512 bp at dtau 100; random orientation plus
    jitter, seed 1), --stats-steps steps each (default 1e5), observables
    every 100 steps, paired runs on identical Philox streams.  Per
    observable: the relative difference of its time and ensemble average
    from FP64 (the target is 2 %), and the centre-of-mass diffusion
    coefficient against D = T*/M (Sec. VII.B)."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    n, se = args.stats_steps, 100
    confs = [(1024, 128, 50.0), (4096, 256, 100.0), (1024, 512, 100.0)]
    out = []
    for B, M, dtau in confs:
        pos = inputs.straight_chains(B, M, b, seed=1, random_orientation=True)
        acc, wall = {}, {}
        for p in ("fp64", "fp32", "bf16x3"):
            t0 = time.perf_counter()
            with Context(pos, seed=1, precision=p) as ctx:
                ctx.set_params([M], [dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA, sample_every=se,
                               use_graphs=True, autotune=p != "fp64")
                steps_with_progress(ctx, n, f"{B}x{M} {p}", chunk=20000)
                acc[p] = ctx.accumulators()[0]
            wall[p] = time.perf_counter() - t0
            print(f"# {B}x{M} {p}: {n} steps in {wall[p]:.1f} s", file=sys.stderr, flush=True)
        ns = acc["fp64"]["n_samples"]
        t = dtau * se * np.arange(1, ns + 1)
        row = {"chains": B, "beads": M, "dtau": dtau, "steps": n, "samples": int(ns),
               "seconds": wall}
        for p in ("fp64", "fp32", "bf16x3"):
            a = acc[p]
            D = a["msd_cm"] / B / (6.0 * t.sum())
            row[p] = {"bond": a["bond"] / ns / B, "bond2": a["bond2"] / ns / B,
                      "L2": a["L2"] / ns / B, "dmid2": a["dmid2"] / ns / B,
                      "D_over_TstarM": D / (T_STAR_DSDNA / M)}
        ref = acc["fp64"]
        for p in ("fp32", "bf16x3"):
            a = acc[p]
            rel = {k: a[k] / ref[k] - 1 for k in ("bond", "bond2", "L2", "dmid2", "msd_cm")}
            rel["end_to_end_rms"] = np.sqrt(a["L2"] / ref["L2"]) - 1
            mrel = a["modes"][1:] / ref["modes"][1:] - 1
            rel["modes_max_abs"] = float(np.abs(mrel).max())
            rel["modes_p1_to_p5"] = [float(x) for x in mrel[:5]]
            rel["within_2pct"] = bool(all(abs(v) < 0.02 for k, v in rel.items()
                                          if isinstance(v, float)))
            row[f"{p}_rel_diff_vs_fp64"] = rel
        out.append(row)
        print(f"# {B}x{M}: {row['bf16x3_rel_diff_vs_fp64']}", file=sys.stderr, flush=True)
    print(json.dumps({"workload": f"reduced precision vs FP64 GPU statistics, {n} steps, "
                                  f"observables every {se} steps",
                      "results": out}))


def fp64_workload(args):
    """The FP64 plain form alone on the default workload (--chains x --beads,
    --dtau), --steps timed steps (whole sampling blocks, replayed as graphs
    unless --no-graphs) with HIP events after --warmup: the denominator of
    the mixed-precision speed-up, for profiling its kernels."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    B, M = args.chains, args.beads
    pos = inputs.straight_chains(B, M, b, seed=1, random_orientation=True)
    se = args.sample_every
    steps = -(-args.steps // se) * se if se > 0 else args.steps
    with Context(pos, seed=1, precision="fp64", stream=stream) as c64:
        c64.set_params([M], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA, sample_every=se,
                       use_graphs=not args.no_graphs)
        c64.step_modes(-(-args.warmup // se) * se if se > 0 else args.warmup)
        sec = time_steps(c64, torch, steps, stream)
        finite = bool(np.all(np.isfinite(c64.modes())))
    print(json.dumps({"metric": "chain-steps/s, FP64 plain form", "value": B * steps / sec,
                      "unit": "chain-steps/s", "us_per_step": sec / steps * 1e6,
                      "state_finite": finite,
                      "config": {"workload": f"{B} chains x {M} bp, dtau {args.dtau:g}, "
                                             f"{steps} steps, observables every {se} steps",
                                 "graphs": not args.no_graphs}}))


def coarse_workload(args):
    """Sec. VI, Fig. 5: the end-to-end vector's mean square displacement
    against real time for a chain of 256 basepairs (256 beads, k = 1) and for
    the same chain as 128 dimerised basepairs (128 beads, k = 2), both with
    the parameters of Eq. (x4) for r = l_p/a = 120, y = l_p K_0/kT = 12000
    (k = 1: T* = 0.034, nu = 6/17; k = 2: T*_2 = 0.008, nu_2 = 0.1875), so
    that both follow the same force-extension curve.  Real time t = c_k tau_k
    with c_k = k^3 T*_k (1 - 2 nu_k)^2 a^2 xi / kT (Eq. g2 with a_k = k a and
    xi_k = k xi); lengths in basepairs a via d_k = k a (1 - 2 nu_k).  Each
    chain relaxes from the library's straight initial state for 4 / zeta_1
    (same real time for both), then samples every 100 steps on a common
    real-time grid; the msd of L at lag l is 2 (<L.L> at lag 0 - <L.L> at lag
    l) from the lag correlators.  k = 2 runs at two time steps (the one that
    matches the k = 1 grid with 100 steps per sample, and a quarter of it
    with 400) to show its curve is converged in the time step."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, coarse_grain
    from paper_1411_3487_amd._lib import coarse_grain_time
    torch.cuda.set_device(0)
    r, y, B, K = 120.0, 12000.0, args.coarse_chains, 14
    nsamp = args.coarse_samples
    runs = [(1, 256, 100.0, 100), (2, 128, None, 100), (2, 128, None, 400)]
    c1 = coarse_grain_time(r, y, 1)
    grid = 100 * 100.0 * c1                      # real time between samples, a^2 xi / kT
    out = []
    for k, M, dtau, se in runs:
        T, nu = coarse_grain(r, y, k)
        ck = coarse_grain_time(r, y, k)
        if dtau is None:
            dtau = grid / (se * ck)
        z1 = 16 * nu * np.sin(np.pi / (2 * M)) ** 4
        relax = int(round(4.0 / z1 / dtau / se)) * se
        t0 = time.perf_counter()
        with Context(None, seed=5, precision=args.precision, beads=[M] * B) as ctx:
            ctx.set_params([M], [dtau], T_star=T, nu=nu, sample_every=se, corr_lags=K,
                           use_graphs=True, autotune=True)
            steps_with_progress(ctx, relax, f"k={k} dtau={dtau:.4g} relax", chunk=200 * se * 100)
            ctx.accumulators(reset=True)
            steps_with_progress(ctx, nsamp * se, f"k={k} dtau={dtau:.4g} sample",
                                chunk=200 * se * 100)
            a = ctx.accumulators()[0]
        d2 = (k * (1.0 - 2.0 * nu)) ** 2          # (d_k / a)^2
        c = a["corr"][:K]
        LL = c[:, 0] / np.maximum(c[:, 3], 1)
        msd = 2.0 * (LL[0] - LL) * d2
        lags = np.array([0] + [2 ** (j - 1) for j in range(1, K)])
        out.append({"k": k, "beads": M, "T_star": T, "nu": nu, "dtau": dtau,
                    "steps_per_sample": se, "c_k_ps": ck * 52.0,
                    "relax_steps": relax, "sample_steps": nsamp * se,
                    "L2_a2": a["L2"] / a["n_samples"] / B * d2,
                    "lag_samples": lags.tolist(), "msd_L_a2": msd.tolist(),
                    "seconds": round(time.perf_counter() - t0, 1)})
        print(f"# k={k} M={M} dtau={dtau:.4g}: <L^2> = {out[-1]['L2_a2']:.1f} a^2, "
              f"{out[-1]['seconds']} s", file=sys.stderr, flush=True)
    ref = np.array(out[0]["msd_L_a2"])
    t_us = np.array(out[0]["lag_samples"]) * grid * 52.0e-6
    rows = []
    for o in out[1:]:
        m = np.array(o["msd_L_a2"])
        ratio = [float(m[j] / ref[j]) if ref[j] > 0 else None for j in range(K)]
        ok = all(abs(x - 1) <= 0.05 for x in ratio[1:] if x is not None)
        rows.append({"k": o["k"], "dtau": o["dtau"], "ratio_to_k1": ratio, "within_5pct": ok,
                     "L2_ratio_to_k1": o["L2_a2"] / out[0]["L2_a2"]})
    print(json.dumps({"workload": f"Fig. 5: end-to-end msd, {B} chains of 256 bp (k = 1) vs "
                                  f"128 dimers (k = 2), {nsamp} samples, {args.precision}",
                      "real_time_per_sample_ns": grid * 52.0e-3, "lag_time_us": t_us.tolist(),
                      "runs": out, "comparison": rows}))


def profile_launches(args):
    """N launches of 200 mode steps of the default workload, no sampling, on
    the untimed default tile shape or the one --table-mode forces."""
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    pos = inputs.straight_chains(args.chains, args.beads, b, seed=1, random_orientation=True)
    ctx = Context(pos, seed=1, precision=args.precision, stream=torch.cuda.current_stream())
    ctx.set_params([args.beads], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA,
                   table_mode=args.table_mode)
    for _ in range(args.profile_launches):
        ctx.step_modes(200)
    torch.cuda.synchronize()
    print(json.dumps({"profile_launches": args.profile_launches, "steps_per_launch": 200,
                      "tiling": {k: float(v) for k, v in ctx.tiling()[0].items()}}))
    ctx.close()


def mc_workload(args):
    """Metropolis sweeps (dm_step_mc, FP64) of 4096 chains x 256 bp."""
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    B, M = args.chains, args.beads
    pos = inputs.straight_chains(B, M, b, seed=1, random_orientation=True)
    ctx = Context(pos, seed=1, precision="fp64", stream=torch.cuda.current_stream())
    ctx.set_params([M], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA)
    ctx.step_mc(2)
    sweeps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = ctx.step_mc(sweeps)
    wall = time.perf_counter() - t0
    R0 = ctx.modes()
    ctx.close()
    props = B * sweeps * 3 * (M - 1)
    flops = MC_FLOPS_PER_BOND * (M - 1)          # per proposal
    out = {"metric": "Metropolis proposals/s (mode representation, FP64)",
           "value": props / wall, "unit": "proposals/s",
           "chain_sweeps_per_s": B * sweeps / wall, "acceptance": acc / props,
           "config": {"workload": f"{B} chains x {M} bp, {sweeps} sweeps, step_scale 3"},
           "roofline": {"bound": "alu", "achieved": props / wall * flops / 1e12, "peak": 78.6,
                        "unit": "TFLOP/s", "frac": props / wall * flops / 78.6e12,
                        "flops_per_proposal": flops}}
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        t0 = time.perf_counter()
        oracle.mc_sweeps(R0[:256], NU_DSDNA, T_STAR_DSDNA, 3.0, 10, seed=1, step0=22,
                         chain_ids=np.arange(256))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 256 * 10 * 3 * (M - 1) / dt, "unit": "proposals/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                           os.cpu_count() or 1)),
                               "kind": "oracle", "sample": f"256 chains x 10 sweeps, {dt:.1f} s"}
    print(json.dumps(out))


# Floating-point operations of one Metropolis proposal per bond (the change
# of H' of Eq. b3 when one mode component moves): the new bond length 10,
# two square roots and the stretching terms 8, the bending cross terms 12.
MC_FLOPS_PER_BOND = 30
# Of one Euler step per bead (Eqs. b3-b5): bond vector and length 9, the
# stretching and bending gradient 21, the bead update with noise and shear
# 15, and the Box-Muller share of the noise 15.
EULER_FLOPS_PER_BEAD = 60


def euler_workload(args):
    """The bead-space Euler baseline (Eqs. b3-b5, FP64) on 4096 chains x 256 bp
    at the paper's safe time step dtau = 0.1: bead-steps/s and simulated time,
    beside the mode scheme's step of dtau = 100 at the same chain length."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    B, M, dtau, n = args.chains, args.beads, 0.1, 2000
    pos = inputs.straight_chains(B, M, b, seed=1, random_orientation=True)
    stream = torch.cuda.current_stream()
    with Context(pos, seed=1, precision="fp64", stream=stream) as ctx:
        ctx.set_params([M], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA)
        ctx.step_euler(20, dtau)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.step_euler(n, dtau)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        x = ctx.positions()
    rate = B * M * n / sec
    out = {"metric": "bead-steps/s, bead-space Euler (FP64)", "value": rate,
           "unit": "bead-steps/s", "chain_steps_per_s": B * n / sec,
           "simulated_ns_per_s_per_chain": n / sec * dtau * 0.159119 * 1e-3,
           "state_finite": bool(np.all(np.isfinite(x))),
           "config": {"workload": f"{B} chains x {M} bp, dtau 0.1, {n} steps in one launch"},
           "roofline": {"bound": "alu", "achieved": rate * EULER_FLOPS_PER_BEAD / 1e12,
                        "peak": 78.6, "unit": "TFLOP/s",
                        "frac": rate * EULER_FLOPS_PER_BEAD / 78.6e12,
                        "flops_per_bead_step": EULER_FLOPS_PER_BEAD}}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.step_euler(pos[:256], NU_DSDNA, T_STAR_DSDNA, dtau, 1000, seed=1)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 256 * M * 1000 / dt, "unit": "bead-steps/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                           os.cpu_count() or 1)),
                               "kind": "oracle", "sample": f"256 chains x 1000 steps, {dt:.1f} s"}
    print(json.dumps(out))


def steps_with_progress(ctx, n, label, chunk=2_000_000):
    """ctx.step_modes(n) in pieces, with a progress line to stderr after
    each (long runs at N = 511 take minutes)."""
    import torch
    t0, done = time.perf_counter(), 0
    while done < n:
        k = min(chunk, n - done)
        ctx.step_modes(k)
        done += k
        if n > chunk:
            torch.cuda.synchronize()
            print(f"# {label}: {done}/{n} steps, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)


def dtmax_workload(args):
    """Equilibrium values Q(0) of the mode dynamics (Sec. V.B: <L^2>, middle
    bead about the centre of mass, bond moments) for several time steps,
    each divided by its Metropolis value; the paper accepts a time step
    while all ratios stay within 5 %.  Chains are equilibrated by Monte
    Carlo first, and every dynamics run starts from that state."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, dtmax, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    # time steps bracketing the paper's Table 1 (50, 100, 100, 100 at N = 63,
    # 127, 255, 511); Monte Carlo burn-in and sampling sweeps
    plan = {64: ([1, 10, 20, 50, 100, 200, 500], 3000, 6000),
            128: ([10, 50, 100, 200, 500, 1000], 8000, 12000),
            256: ([100, 200, 500, 1000, 2000], 20000, 20000),
            512: ([100, 200, 500], 20000, 20000)}
    lengths = [int(x) for x in args.dtmax_lengths.split(",") if x]
    if any(M not in plan for M in lengths):
        raise SystemExit(f"dtmax lengths must be among {sorted(plan)}")
    B = 1024
    keys = ("L2", "dmid2", "bond", "bond2")
    out = []
    for M in lengths:
        dts, burn, samp = plan[M]
        if args.dtmax_dtaus:
            dts = [float(x) for x in args.dtmax_dtaus.split(",") if x]
        pos = inputs.straight_chains(B, M, b, seed=M, random_orientation=True)
        t0 = time.perf_counter()
        mc = Context(pos, seed=M, precision="fp64")
        mc.set_params([M], [1.0], T_star=T_STAR_DSDNA, nu=NU_DSDNA, sample_every=20)
        for phase, sweeps in (("burn-in", burn), ("sampling", samp)):
            if phase == "sampling":
                state = mc.positions()
                mc.accumulators(reset=True)
            for k0 in range(0, sweeps, 5000):
                mc.step_mc(min(5000, sweeps - k0))
                torch.cuda.synchronize()
                print(f"# M={M}: Monte Carlo {phase} {min(k0 + 5000, sweeps)}/{sweeps} sweeps, "
                      f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
        a = mc.accumulators()[0]
        ref = {k: a[k] / a["n_samples"] for k in keys}
        mc.close()
        z1 = 16 * NU_DSDNA * np.sin(np.pi / (2 * M)) ** 4
        rows = []
        for dt in dts:
            # relax 2/zeta_1 from the Monte Carlo state, then average 2/zeta_1
            n = max(2000, int(round(2.0 / z1 / dt)))
            ctx = Context(state, seed=M + 1, precision=args.precision)
            ctx.set_params([M], [float(dt)], T_star=T_STAR_DSDNA, nu=NU_DSDNA,
                           sample_every=max(1, n // 400), use_graphs=True)
            steps_with_progress(ctx, n, f"M={M} dtau={dt} relax")
            ctx.accumulators(reset=True)
            steps_with_progress(ctx, n, f"M={M} dtau={dt} average")
            d = ctx.accumulators()[0]
            ctx.close()
            ratio = {k: d[k] / d["n_samples"] / ref[k] for k in keys}
            rows.append({"dtau": dt, "steps": 2 * n, "ratios": ratio,
                         "within_5pct": dtmax.q0_passes(ratio.values())})
            print(f"# M={M} dtau={dt}: {ratio}", file=sys.stderr, flush=True)
        out.append({"M": M, "N": M - 1, "mc_reference": ref, "runs": rows,
                    "dtau_max_from_Q0": dtmax.contiguous_dtau_max(
                        [r["dtau"] for r in rows], [r["within_5pct"] for r in rows])})
    print(json.dumps({"workload": f"dtau_max from equilibrium values, {B} chains per length, "
                                  f"{args.precision} mode dynamics vs FP64 Monte Carlo",
                      "results": out}))


def dtmax_t_workload(args):
    """Dynamical group of the time-step test (Sec. V.B): the time correlations
    Q(t) (end-to-end vector, middle bond: autocorrelations; middle bead about
    the centre of mass: msd) at several time steps, from Monte Carlo
    equilibrated chains.  At fixed times tau the effective decay constant
    Q~ = (1/Q) dQ/dtau (central differences over the power-of-two lags) is
    divided by its value at the smallest time step; the paper accepts a time
    step while these ratios stay within 10 %.  Autocorrelations that have
    decayed below 5 % of their start are left out (noise)."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, dtmax, inputs, NU_DSDNA, T_STAR_DSDNA
    torch.cuda.set_device(0)
    b = 1.0 / (1.0 - 2.0 * NU_DSDNA)
    B, K = 1024, 14
    # M: (time steps, sampling interval in tau, run length in tau, test times,
    #     Monte Carlo burn-in sweeps)
    plan = {64: ([0.1, 1, 10, 20, 50, 100], 100.0, 2.0e6, [100, 1e3, 1e4, 1e5], 3000),
            128: ([1, 10, 50, 100, 200], 1000.0, 2.0e7, [1e3, 1e4, 1e5, 1e6], 8000),
            256: ([1, 10, 100, 200, 500], 1.0e4, 1.0e8, [1e4, 1e5, 1e6, 1e7], 20000),
            512: ([10, 100, 200, 500], 1.0e5, 5.0e8, [1e5, 1e6, 1e7, 1e8], 20000)}
    lengths = [int(x) for x in args.dtmax_lengths.split(",") if x]
    if any(M not in plan for M in lengths):
        raise SystemExit(f"dtmax_t lengths must be among {sorted(plan)}")
    names = ("L", "umid", "msd")
    out = []
    for M in lengths:
        dts, ts, run, times, burn = plan[M]
        if args.dtmax_dtaus:  # the first one is the reference
            dts = [float(x) for x in args.dtmax_dtaus.split(",") if x]
        pos = inputs.straight_chains(B, M, b, seed=M, random_orientation=True)
        mc = Context(pos, seed=M, precision="fp64")
        mc.set_params([M], [1.0], T_star=T_STAR_DSDNA, nu=NU_DSDNA)
        t0 = time.perf_counter()
        for k0 in range(0, burn, 5000):
            mc.step_mc(min(5000, burn - k0))
            torch.cuda.synchronize()
            print(f"# M={M}: Monte Carlo {min(k0 + 5000, burn)}/{burn} sweeps, "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
        state = mc.positions()
        mc.close()
        lags = np.array([0.0] + [ts * 2 ** (j - 1) for j in range(1, K)])
        curves = {}
        for dt in dts:
            se = int(round(ts / dt))
            n = int(round(run / dt))
            t0 = time.perf_counter()
            ctx = Context(state, seed=M + 2, precision=args.precision)
            ctx.set_params([M], [float(dt)], T_star=T_STAR_DSDNA, nu=NU_DSDNA,
                           sample_every=se, corr_lags=K, use_graphs=True)
            steps_with_progress(ctx, n, f"M={M} dtau={dt}", chunk=max(se, 2_000_000 // se * se))
            c = ctx.accumulators()[0]["corr"][:K]
            ctx.close()
            q = c[:, :3] / np.maximum(c[:, 3:4], 1)
            curves[dt] = q
            print(f"# M={M} dtau={dt}: {n} steps, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
        ref = curves[dts[0]]
        rows = []
        for dt in dts[1:]:
            ratios, ok = dtmax.qt_ratios(curves[dt], ref, lags, times, names)
            rows.append({"dtau": dt, "ratios": ratios, "within_10pct": ok})
            print(f"# M={M} dtau={dt}: ok={ok} {ratios}", file=sys.stderr, flush=True)
        best = dtmax.contiguous_dtau_max([r["dtau"] for r in rows],
                                         [r["within_10pct"] for r in rows])
        out.append({"M": M, "N": M - 1, "dtau_min": dts[0], "runs": rows,
                    "lags_tau": lags.tolist(),
                    "Q_ref": {n: ref[:, i].tolist() for i, n in enumerate(names)},
                    "dtau_max_from_Qt": best})
    print(json.dumps({"workload": f"dtau_max from time correlations, {B} chains per length, "
                                  f"{args.precision} mode dynamics",
                      "results": out}))


# Floating-point operations of one tension cycle per bond of the inextensible
# stepper (Eqs. y9-y14), counted as written with a Thomas solve: midpoint
# bond 13 (sqrt and divide counted as one), bending displacements 12, the
# tridiagonal row 27, its solve 8, the bond update 25.
WLC_FLOPS_PER_BOND_ITER = 85


def wlc_workload(args):
    """Sec. VII.A: the largest time step of the inextensible limit (Eqs.
    y2-y14) for N = 63 at the persistence length of dsDNA (T-bar = a / l_p =
    1/114.4), for two forms of the tension cycle (forces at the midpoint
    bonds iterated to convergence; forces at the bonds of the start of the
    step with three fixed passes).  From exact discrete-wormlike-chain
    starts, each time step runs to tau-bar = 1.024 and is accepted while
    every check stays within 5 %: the time averages of <L^2> and of the
    middle bead's squared distance from the centre of mass against their
    closed forms (set by slow modes, which these runs do not relax: they
    only show that the step keeps the ensemble), the local bending
    <1 - cos> (it relaxes within the run) and the middle bead's msd about
    the centre of mass at tau-bar = 0.002 * 2^k against the smallest step's,
    and the bonds within 1 % of unit length.  The extensible model under the
    bead Euler scheme is safe at dtau = 0.1 (Sec. III.A), i.e. at dtau-bar =
    nu dtau = 0.035."""
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, NU_DSDNA, dtmax
    from paper_1411_3487_amd.inputs import unit_chains
    torch.cuda.set_device(0)
    B, M, T = 8192, 64, 1.0 / 114.4
    c = 1 / np.tanh(1 / T) - T                     # <u_n . u_(n+1)>, bond angles independent
    f = lambda m: m + 2 * sum((m - k) * c ** k for k in range(1, m))   # <|r_i - r_(i+m)|^2>
    mid = (M - 1) // 2
    L2 = f(M - 1)
    d2 = (sum(f(abs(mid - j)) for j in range(M)) / M
          - sum(f(abs(j - k)) for j in range(M) for k in range(M)) / (2 * M * M))
    pos0 = unit_chains(B, M, seed=11, T_bar=T)
    times = [0.002 * 2 ** k for k in range(10)]

    def rel_mid(x):
        return x[:, :, mid] - x.mean(axis=2)
    dm0 = rel_mid(pos0)
    grid = [2e-5, 5e-5, 1e-4, 2e-4, 5e-4, 1e-3, 2e-3, 4e-3, 8e-3, 1.6e-2, 3.2e-2, 6.4e-2,
            0.128, 0.256]
    # the two forms of the tension cycle: forces and tensions along the
    # midpoint bonds (Eq. y14), iterated to convergence; and along the bonds
    # of the start of the step with three fixed passes (the cycle as first
    # written, "typically two or three steps")
    variants = {"midpoint_converged": dict(midpoint=True, iters=16, tol=1e-12),
                "start_bonds_3_passes": dict(midpoint=False, iters=3, tol=0.0)}
    scans = {}
    for vname, kw in variants.items():
        rows, ref, bend_ref = [], None, None
        for dt in grid:
            t0 = time.perf_counter()
            l2, dm, bend, msd, fin, done = [], [], [], {}, True, 0
            with Context(pos0, seed=13, precision="fp64") as ctx:
                for t in times:
                    n = int(round(t / dt)) - done
                    if n <= 0:
                        continue
                    ctx.step_wlc(n, dt, T, **kw)
                    done += n
                    x = ctx.positions()
                    fin = fin and bool(np.all(np.isfinite(x)))
                    L = x[:, :, -1] - x[:, :, 0]
                    d = rel_mid(x)
                    u = np.diff(x, axis=2)
                    bend.append(1 - (u[:, :, 1:] * u[:, :, :-1]).sum(axis=1).mean())
                    l2.append((L * L).sum(axis=1).mean())
                    dm.append((d * d).sum(axis=1).mean())
                    msd[t] = float(((d - dm0) ** 2).sum(axis=1).mean())
                bond_err = float(np.abs(np.linalg.norm(np.diff(x, axis=2), axis=1) - 1).max())
            if ref is None:
                ref, bend_ref = msd, float(np.mean(bend))
            r = {"dtau_bar": dt, "steps": done, "L2_ratio": float(np.mean(l2) / L2),
                 "dmid2_ratio": float(np.mean(dm) / d2),
                 "bend_ratio_to_theory": float(np.mean(bend) / (1 - c)),
                 "bend_ratio_to_smallest_step": float(np.mean(bend) / bend_ref),
                 "msd_mid_ratio": {f"{t:g}": msd[t] / ref[t] for t in msd},
                 "bond_err": bond_err, "finite": fin,
                 "seconds": round(time.perf_counter() - t0, 2)}
            checks = [r["L2_ratio"], r["dmid2_ratio"], r["bend_ratio_to_smallest_step"],
                      *r["msd_mid_ratio"].values()]
            r["within_5pct"] = bool(fin and bond_err < 0.01
                                    and all(abs(v - 1) < 0.05 for v in checks))
            rows.append(r)
            print(f"# {vname} dt_bar={dt}: {r}", file=sys.stderr, flush=True)
        scans[vname] = {"rows": rows, "dtau_bar_max": dtmax.contiguous_dtau_max(
            [r["dtau_bar"] for r in rows], [r["within_5pct"] for r in rows])}
    rows = scans["midpoint_converged"]["rows"]
    wlc_max = scans["midpoint_converged"]["dtau_bar_max"]
    ext = 0.1 * NU_DSDNA
    # throughput of the stepper: HIP events around one call on the context's stream
    stream = torch.cuda.current_stream()
    n_t, iters = 2000, 8
    with Context(pos0, seed=13, precision="fp64", stream=stream) as ctx:
        ctx.step_wlc(10, 1e-4, T, iters=iters)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.step_wlc(n_t, 1e-4, T, iters=iters)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        e0.record(stream)
        ctx.step_wlc(n_t, 1e-4, T, iters=16, tol=1e-12)
        e1.record(stream)
        torch.cuda.synchronize()
        sec_conv = e0.elapsed_time(e1) * 1e-3
    flops = WLC_FLOPS_PER_BOND_ITER * iters * (M - 1)      # per chain-step
    peak = 78.6e12
    perf = {"chain_steps_per_s": B * n_t / sec, "us_per_step": sec / n_t * 1e6,
            "iters": iters, "us_per_step_converged_1e-12": sec_conv / n_t * 1e6,
            "roofline": {"bound": "alu", "achieved": flops * B * n_t / sec / 1e12,
                         "peak": peak / 1e12, "unit": "TFLOP/s",
                         "frac": flops * B * n_t / sec / peak,
                         "flops_per_chain_step": flops}}
    if not args.no_cpu_baseline:
        import oracle
        sample = pos0[:16]
        t0 = time.perf_counter()
        oracle.step_wlc(sample, T, 1e-4, 200, iters=iters, seed=13)
        cs = time.perf_counter() - t0
        perf["cpu_baseline"] = {"value": 16 * 200 / cs, "unit": "chain-steps/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "16 of the chains, 200 steps at dtau-bar = 1e-4"}
    print(f"# stepper: {perf}", file=sys.stderr, flush=True)
    print(json.dumps({"workload": f"inextensible limit, {B} chains of {M} beads, T_bar = 1/114.4",
                      "theory": {"L2": L2, "dmid2": d2, "bond_cos": c},
                      "msd_mid_ref": {f"{t:g}": v for t, v in ref.items()},
                      "scans": scans, "stepper": perf, "dtau_bar_max_wlc": wlc_max,
                      "dtau_bar_max_start_bonds": scans["start_bonds_3_passes"]["dtau_bar_max"],
                      "dtau_bar_max_extensible_euler": ext,
                      "gain": (ext / wlc_max) if wlc_max else None}))


def main():
    args = parse()
    if args.workload == "wlc" and args.gpus == 1:
        return wlc_workload(args)
    if args.workload == "dtmax_t" and args.gpus == 1:
        return dtmax_t_workload(args)
    if args.workload == "mc" and args.gpus == 1:
        return mc_workload(args)
    if args.workload == "euler" and args.gpus == 1:
        return euler_workload(args)
    if args.workload == "dtmax" and args.gpus == 1:
        return dtmax_workload(args)
    if args.workload == "stats" and args.gpus == 1:
        return stats_workload(args)
    if args.workload == "fp64" and args.gpus == 1:
        return fp64_workload(args)
    if args.workload == "coarse" and args.gpus == 1:
        return coarse_workload(args)
    if args.profile_launches:
        return profile_launches(args)
    if args.workload != "modes" and args.gpus == 1:
        return uneven_workload(args) if args.workload == "uneven" else shear_workload(args)
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(chains are independent: a multi-GPU run is the same "
                                   "kernel on each GPU's share)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1411_3487_amd import Context, inputs, NU_DSDNA, T_STAR_DSDNA

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    B, M = args.chains, args.beads
    # the library's own initial state (straight chains, Philox-uniform
    # directions, jitter 0.01 a; seed 1), built at set_params
    beads = [M] * B

    # ---- mixed precision: the measured path.  Warm-up and timed steps are
    # rounded up to whole sampling blocks, so the timed region starts on a
    # block boundary and is made of replayed sampling blocks, each with its
    # observable sample, whatever --steps and --warmup say.
    se = args.sample_every
    blocks = lambda n: -(-n // se) * se if se > 0 else n
    warmup, steps = blocks(args.warmup), blocks(max(args.steps, 1))
    ctx = Context(None, seed=1, precision=args.precision, stream=stream, beads=beads)
    ctx.set_params([M], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA,
                   sample_every=se, use_graphs=not args.no_graphs,
                   autotune=not args.no_autotune, table_mode=args.table_mode)
    tiling, report = ctx.tiling()[0], ctx.tuning_report()
    shape = {0: "resident" if tiling["resident"] else "streamed", 1: "split",
             2: "split8"}[int(tiling["split"])]
    ctx.step_modes(warmup)
    torch.cuda.synchronize()
    n0 = ctx.accumulators()[0]["n_samples"]
    s0 = ctx.step
    t0 = time.perf_counter()
    ctx.step_modes(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    samples_timed = int(ctx.accumulators()[0]["n_samples"] - n0)
    graphs_used = (not args.no_graphs) and se > 0 and s0 % se == 0 and steps >= se
    obs = ctx.chain_observables()
    finite = bool(np.all(np.isfinite(obs)))
    # dominant kernel alone, in the launch shape of the timed loop: one fused
    # launch covers the steps between two observable samples
    ctx.set_params([M], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA, sample_every=0,
                   tiles_per_wg=int(tiling["tpw"]), table_mode=shape)
    k_launch = se if se > 0 else 100
    # launch durations settle over the first ~20 launches after the
    # autotuner (about 830 -> 750 us at 4096 x 256): 20 untimed launches of
    # the same shape back to back, then the median of 9 timed ones
    for _ in range(20):
        ctx.step_modes(k_launch)
    kern = sorted(time_steps(ctx, torch, k_launch, stream) for _ in range(9))[4]
    ctx.close()

    # ---- FP64 plain form on the same GPU and workload, over the same kind
    # of window: whole sampling blocks from a block boundary
    c64 = Context(None, seed=1, precision="fp64", stream=stream, beads=beads)
    c64.set_params([M], [args.dtau], T_star=T_STAR_DSDNA, nu=NU_DSDNA, sample_every=se,
                   use_graphs=not args.no_graphs)
    fp64_steps = steps if args.fp64_steps <= 0 else blocks(args.fp64_steps)
    c64.step_modes(blocks(20))
    t64 = time_steps(c64, torch, fp64_steps, stream)
    c64.close()

    chain_steps = B * steps / wall
    fp64_rate = B * fp64_steps / t64
    exec_flops = executed_flops(args.precision, M, int(tiling["JC"]))  # per chain-step
    achieved = exec_flops * B * k_launch / kern
    traffic = measured_traffic(args.precision, B, M)
    peak = PEAKS[args.precision]
    dt_ps = args.dtau * 0.159119  # (T*/b^2) a^2 xi/kT, Eq. (g2)
    out = {
        "metric": "chain-steps/s (bead-steps/s) at 256 bp, mixed precision vs FP64 on GPU",
        "value": chain_steps,
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3-f32acc", "fp32": "f32"}[args.precision],
        "data": "synthetic: straight chains, Philox-uniform directions, jitter 0.01 a (seed 1)",
        "config": {"workload": f"{B} chains x {M} bp dsDNA (nu=0.35, T*=0.034), "
                               f"dtau={args.dtau:g} ({dt_ps:.3g} ps), observables every "
                               f"{se} steps",
                   "chains": B, "beads": M, "parallelism": "1 GPU, chains data-parallel",
                   "timed_region": {"steps_requested": args.steps, "warmup_requested": args.warmup,
                                    "steps": steps, "warmup": warmup,
                                    "samples_in_timed_region": samples_timed,
                                    "graph_replays": steps // se if graphs_used else 0,
                                    "fp64_steps": fp64_steps,
                                    "fp64_samples": fp64_steps // se if se > 0 else 0},
                   "launch": {"graphs": graphs_used, "autotune": not args.no_autotune,
                              "tables": shape, "tiles_per_wg": int(tiling["tpw"]),
                              "coupling_row_tiles": int(tiling["JC"]), "row_tiles": int(tiling["RT"]),
                              "tuning_report": report.strip().splitlines()}},
        "bead_steps_per_s": chain_steps * M,
        "simulated_ns_per_s": chain_steps / B * dt_ps * 1e-3,
        "fp64_plain_chain_steps_per_s": fp64_rate,
        "speedup_vs_fp64_plain": chain_steps / fp64_rate,
        "state_finite": finite,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"{'split_wide_kernel' if shape == 'split8' else 'fused_kernel'} "
                               f"({args.precision}), {k_launch} steps per launch",
                     "kernel_ms": kern * 1e3, "flops_per_chain_step": exec_flops},
    }
    # Table 2 context: simulated time per hour of computing for one chain
    # (the paper's desktop: 0.56 ms per hour at 256 bp, Delta t = 15.9 ps)
    per_hour = lambda rate: rate * dt_ps * 3600.0 * 1e-9
    out["paper_context"] = {"unit": "ms simulated per hour, one chain",
                            "paper_desktop_table2": {64: 0.23, 128: 0.56, 256: 0.56,
                                                     512: 0.26}.get(M),
                            "this_gpu_per_chain": per_hour(chain_steps / B),
                            "this_gpu_all_chains": per_hour(chain_steps)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, NU_DSDNA, T_STAR_DSDNA)
        out["paper_context"]["oracle_one_core"] = per_hour(
            out["cpu_baseline"]["single_core"]["value"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
