"""Benchmark of the VLBM Mach-2000 jet ensemble hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision both|fp64|mixed]

The default workload is the largest configuration that fits one GPU: the
5056 x 2528 level with its 2528 x 1264 partner on the same seeds (the pair
whose one-point W1 the refinement study needs), M = 1000 realizations streamed
through HBM in batches.  One benchmark step is one slice of that job on one
batch of B realizations (B the largest batch HBM holds next to the job's
sample stores): a fixed block of step launches (fused collide-stream kernel
with the kinetic-speed reduction and the boundary layers, both levels in each
launch, hipGraph replays), then the batch's statistics -- moments and
conservative restriction of both levels to the 2528 x 1264 grid, Chan merge
into the running mean/std accumulators, scatter of the restricted densities
into the M = 1000 sample stores at the batch's rows, the per-cell sort of
those rows and the one-point W1 between the levels.

Both storage precisions run by default: FP64 gives the headline value, the
mixed variant (populations' rho, rho v in FP32) is reported beside it, and the
statistics of a mixed ensemble are compared with an FP64 ensemble of the same
seeds (640 x 320, M = 64, t = 1e-5, 1e-4, 1e-3) next to the round-off floor:
an FP64 ensemble whose inlet densities are moved by one ulp.

Prints one JSON line.  `value` is ensemble GLUPS: node updates summed over
realizations and levels per second of the timed steps.  `roofline` reports the
step kernel: algorithmic 320 B per FP64 node update (224 B mixed) over its
average launch duration, measured with HIP events on the stream the kernels
run on.  `cpu_baseline` times the CPU oracle on a bounded sample of the same
grid on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ensemble GLUPS (cell-updates/s summed over realizations) + % HBM roofline, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0
from paper_2605_25282_amd.rocprof_summary import BYTES_PER_LUP, kernel_source_hash  # noqa: E402


def measured_traffic(precision: str, workload: str, node_updates_per_launch: float | None = None):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary of this workload, if it was taken on the current kernel
    sources (null for a workload without one), scaled to this run's node
    updates per launch when the record states its own (a different batch)."""
    path = os.path.join(ROOT, "profiles", f"traffic_step_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    per_launch = d.get("bytes_per_launch")
    rec = d.get("node_updates_per_launch")
    if per_launch is not None and rec and node_updates_per_launch:
        per_launch = per_launch * node_updates_per_launch / rec
    return per_launch


def cpu_baseline(name, nx, ny, dx, y_min, steps=None, seconds_target: float = 15.0,
                 mem_budget: float = 120e9):
    """The oracle, as it stands, on a bounded sample of the same grid: the first
    realizations of the ensemble for a fixed number of steps, one realization per
    host thread (the oracle parallelizes over realizations only).  Threads: the
    host share of one GPU (OMP_NUM_THREADS, at most 16), fewer if one
    realization's oracle working set (state, step copy and per-node Maxwellians,
    about 820 B per node) times the threads would exceed mem_budget bytes."""
    import oracle as O
    from paper_2605_25282_amd import inputs

    share = min(int(os.environ.get("OMP_NUM_THREADS", "8") or 8), os.cpu_count() or 1, 16)
    per_real = 820.0 * nx * ny
    threads = max(1, min(share, int(mem_budget // per_real)))
    p = O.Params()
    g = O.Grid(nx, ny, dx, y_min)
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, threads)
    if steps is None:
        # size the sample from a short probe so that it takes ~seconds_target
        t0 = time.perf_counter()
        O.run(p, g, O.init(p, g, coefs[0]), 1e30, max_steps=2)
        per_step = (time.perf_counter() - t0) / 2
        steps = int(max(4, min(200, seconds_target / max(per_step, 1e-6))))
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        st0 = list(ex.map(lambda m: O.init(p, g, coefs[m]), range(threads)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        n = list(ex.map(lambda m: O.run(p, g, st0[m], 1e30, max_steps=steps)[2], range(threads)))
    el = time.perf_counter() - t0
    del st0
    lups = float(sum(n)) * nx * ny
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": lups / el / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"{threads} realizations x {steps} steps of the {nx}x{ny} {name} grid on "
                      f"{threads} host threads, the stepping timed ({el:.1f} s, "
                      f"{lups:.3e} node updates)"}


def decomposition(vlbm, h, n_levels: int, autotuned: bool) -> dict:
    """The step kernel's decomposition in use on handle h (vlbm_get_tuning)."""
    chunks, wpb, order, deal = vlbm.vlbm_get_tuning(h, n_levels)
    return {"rows_per_wave": chunks, "waves_per_block": wpb,
            "item_order": "strip fastest" if order == 0 else "realization fastest",
            "dealing": "static round-robin" if deal == 0 else "per-XCD work queues",
            "autotuned": autotuned}


def progress(msg: str) -> None:
    """One line per finished stage on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--workload", default="jet5056pair",
                    help="jet5056pair (default): the 5056x2528 level and its 2528x1264 partner, M = 1000 "
                         "streamed in batches; or the name of a single-level jet workload "
                         "(jet128, jet320, jet640, jet1280), one step = one whole pass to t_final")
    ap.add_argument("--launches", type=int, default=60,
                    help="jet5056pair: step launches per benchmark step")
    ap.add_argument("--batch", type=int, default=0,
                    help="jet5056pair: realizations per batch (0: the largest that fits in HBM, at most 64)")
    ap.add_argument("--chunk", type=int, default=240, help="launches per vlbm_step call (whole passes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed-error", action="store_true",
                    help="jet5056pair: skip the mixed-vs-FP64 statistics comparison")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuning pass (with --chunk-rows: a fixed step-kernel "
                         "configuration, e.g. for a profiler run of this same command)")
    ap.add_argument("--chunk-rows", type=int, default=0,
                    help="rows per wave of the step kernel (0: autotuned / default)")
    ap.add_argument("--decomposition", default="",
                    help="with --no-tune: the step kernel's whole decomposition as "
                         "CHUNKS:WAVES_PER_BLOCK:ITEM_ORDER:DEALING, CHUNKS comma-separated per level "
                         "(jet5056pair: coarse, fine), e.g. 79,79:4:0:1 (a profiler run of a tuned configuration)")
    ap.add_argument("--mixed-error", action="store_true",
                    help="instead of the default line: statistics of a mixed and of a one-ulp-"
                         "perturbed FP64 ensemble against an FP64 ensemble of the same seeds, at "
                         "several times (--workload jet640 or jet1280)")
    ap.add_argument("--study", action="store_true",
                    help="instead of the default line: the three-level ensemble (320x160, "
                         "640x320, 1280x640, M=128, t=1e-3) advanced by one launch per step, "
                         "then the Cauchy / reference convergence tables and rates")
    ap.add_argument("--study-geometry", default="config", choices=["config", "paper"],
                    help="paper: the paper's domain [0,2.5]x[-1,1] with grids 500x400, 1000x800, "
                         "2000x1600 and the study at t = 0.0005 k, k = 1..7")
    ap.add_argument("--study-m", type=int, default=0, help="realizations (0: 128 config, 32 paper)")
    ap.add_argument("--study-levels", type=int, default=3, choices=[3, 4],
                    help="paper geometry: 4 adds the 4000x3200 level (the paper's full hierarchy)")
    ap.add_argument("--pair-full", action="store_true",
                    help="instead of the default line: the largest level (5056x2528) with its "
                         "2528x1264 partner on the same seeds, whole batches streamed to t=1e-3 with "
                         "running mean/std and sample stores, then the one-point W1 between the levels")
    ap.add_argument("--pair-batches", type=int, default=1)
    ap.add_argument("--pair-batch-m", type=int, default=45)
    ap.add_argument("--w12", action="store_true",
                    help="instead of the default line: time the two-point W_{1,2} at the paper's "
                         "scale (1000 samples, 10 x 10 subsampled cells, 10^4 exact assignments) on "
                         "seeded synthetic samples of a 500 x 400 common grid")
    ap.add_argument("--centerline", type=int, default=0, metavar="NX",
                    help="instead of the default line: the paper's geometry at NX x 0.8 NX (500, 1000, "
                         "2000 or 4000), --study-m realizations (default 64) to t = 0.0035, then the "
                         "centerline quantile diagnostics of Sec. 4 (p5..p95, width ratio, skewness "
                         "of the bands, shear-layer onset, leading fringe)")
    ap.add_argument("--profile-launches", type=int, default=0,
                    help="profiling mode: initial datum and this many step launches of the "
                         "workload (jet5056pair: one batch, both levels), no statistics and no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not "
                                   "supported (--gpus must be 1)"}))
        return 2

    import torch

    from paper_2605_25282_amd import inputs, vlbm

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    vlbm.lib()  # fails loudly if the HIP library was not built
    if args.study:
        return run_study(args, torch, vlbm, inputs)
    if args.pair_full:
        return run_pair_full(args, torch, vlbm, inputs)
    if args.w12:
        return run_w12(args, torch, vlbm)
    if args.centerline:
        return run_centerline(args, torch, vlbm, inputs)
    if args.mixed_error:
        w = inputs.WORKLOADS["jet640" if args.workload == "jet5056pair" else args.workload]
        out = mixed_error_study(torch, vlbm, inputs, w, (0.01, 0.1, 1.0), args.chunk)
        print(json.dumps({"mixed_error_study": out}), flush=True)
        return 0
    if args.workload == "jet5056pair":
        return run_headline(args, torch, vlbm, inputs)
    return run_pass(args, torch, vlbm, inputs)


def copy_bandwidth(torch, nbytes: int = 1 << 31, reps: int = 5) -> float:
    """Device-to-device copy rate (bytes read + written per second) of torch's
    copy kernel, the practical HBM ceiling the step kernel is compared with."""
    stream = torch.cuda.current_stream()
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def stat_errors(torch, vlbm, a, b, ncell_w1, R):
    """mean/std rel. L1 per field and W1 / mean density between two ensembles'
    statistics (a is the reference); sorted restricted density samples for W1."""
    rel = lambda x, y: float((x - y).abs().sum() / y.abs().sum())
    w1c = torch.empty(ncell_w1, dtype=torch.float64, device="cuda")
    w1m = torch.zeros(1, dtype=torch.float64, device="cuda")
    vlbm.vlbm_w1(a["sorted"], b["sorted"], ncell_w1, R, w1c, w1m)
    torch.cuda.synchronize()
    sig = lambda x: float(f"{x:.4g}")
    return {"mean_rel_l1": [sig(rel(b["mean"][f], a["mean"][f])) for f in range(3)],
            "std_rel_l1": [sig(rel(b["std"][f], a["std"][f])) for f in range(3)],
            "w1_over_mean_rho": sig(float(w1m.item()) / float(a["mean"][0].mean())),
            "fields": ["rho", "|v|", "p"]}


def mixed_error_study(torch, vlbm, inputs, w, fracs, chunk):
    """Ensemble statistics of the mixed variant against an FP64 ensemble of the
    same seeds at t = frac * t_final, next to two references for the size of such
    differences: the round-off floor (FP64 ensembles of the same seeds whose
    inlet density, or inlet energy, is moved by one ulp up or down, which the
    Dirichlet inlet keeps feeding in: four perturbations, their spread and
    maximum reported) and the sampling floor (an FP64 ensemble on the next M
    seeds).  Statistics: mean and std of (rho, |v|, p) on the nodes, W1 of the
    2 x 2 restricted density."""
    R, r_w1 = w.m, 2
    ncell, ncell_w1 = w.nx * w.ny, (w.nx // r_w1) * (w.ny // r_w1)
    dev = dict(dtype=torch.float64, device="cuda")

    def run(precision, t_end, first_seed=0, ulp=None):
        coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, first_seed, R)
        ens = vlbm.Ensemble(vlbm.Params.jet(precision=precision), [(w.nx, w.ny, w.dx, w.y_min)], coefs, R)
        if ulp is not None:  # (variable, direction): one ulp on the inlet column's u
            var, sign = ulp
            st = ens.state(0)  # [4 var][5 slot][R][ny][nx]
            col = st[var, 0, :, :, 0]
            st[var, 0, :, :, 0] = torch.nextafter(col, torch.full_like(col, sign * float("inf")))
            t, s, a, _ = ens.times(0)
            ens.set_state(0, st, t, s, a)
            del st
        ens.run(t_end, chunk=chunk)
        t, s, a, status = ens.times(0)
        if (status != 0).any() or (t != t_end).any():
            raise RuntimeError(f"{precision} ensemble did not reach t = {t_end:g} cleanly")
        acc = torch.empty((3, 2, ncell), **dev)
        mean, std = torch.empty((3, ncell), **dev), torch.empty((3, ncell), **dev)
        sacc = torch.empty((3, 2, ncell_w1), **dev)
        smp = torch.empty((R, ncell_w1), **dev)
        vlbm.vlbm_ensemble_stats(ens.h, 0, 1, acc, 0, None, 0)
        vlbm.vlbm_stats_finalize(acc, ncell, R, mean, std)
        vlbm.vlbm_ensemble_stats(ens.h, 0, r_w1, sacc, 0, smp, 0)
        vlbm.vlbm_sort_samples(smp, ncell_w1, R)
        ens.close()
        progress(f"mixed-error study: {precision} ensemble (first seed {first_seed}, perturbation {ulp}) "
                 f"at t={t_end:g}")
        return {"mean": mean, "std": std, "sorted": smp, "steps": [int(s.min()), int(s.max())]}

    out = []
    for frac in fracs:
        t_e = w.t_final * frac
        ref = run("fp64", t_e)
        mixed = stat_errors(torch, vlbm, ref, run("mixed", t_e), ncell_w1, R)
        floors = {f"{name}{'+' if sign > 0 else '-'}1ulp": stat_errors(torch, vlbm, ref,
                                                                       run("fp64", t_e, ulp=(var, sign)),
                                                                       ncell_w1, R)
                  for name, var in (("rho", 0), ("E", 3)) for sign in (1, -1)}
        worst = {"w1_over_mean_rho": max(f["w1_over_mean_rho"] for f in floors.values()),
                 "mean_rel_l1": [max(f["mean_rel_l1"][k] for f in floors.values()) for k in range(3)],
                 "std_rel_l1": [max(f["std_rel_l1"][k] for f in floors.values()) for k in range(3)]}
        row = {"t": t_e, "time_steps_per_realization": ref["steps"],
               "mixed_vs_fp64": mixed,
               "fp64_one_ulp_inlet_vs_fp64": floors,
               "roundoff_floor_max": worst,
               "mixed_over_floor_max": {
                   "w1": round(mixed["w1_over_mean_rho"] / worst["w1_over_mean_rho"], 3),
                   "mean": [round(mixed["mean_rel_l1"][k] / worst["mean_rel_l1"][k], 3) for k in range(3)],
                   "std": [round(mixed["std_rel_l1"][k] / worst["std_rel_l1"][k], 3) for k in range(3)]},
               "fp64_independent_seeds_vs_fp64": stat_errors(torch, vlbm, ref, run("fp64", t_e, first_seed=R),
                                                             ncell_w1, R)}
        out.append(row)
        progress(f"mixed-error study: t={t_e:g} done")
        torch.cuda.empty_cache()
    return {"workload": f"{w.name}: {w.nx}x{w.ny}, M={R}, same seeds", "rows": out}


PAIR_M_TOTAL = 1000          # realizations of the whole job
PAIR_HEADROOM = 6 << 30      # device bytes left free next to the batch


def pair_works(inputs):
    fine = inputs.WORKLOADS["jet5056"]
    coarse = inputs.JetWorkload("jet2528", fine.nx // 2, fine.ny // 2, fine.m, fine.t_final)
    return [coarse, fine]


def run_headline(args, torch, vlbm, inputs) -> int:
    """The largest single-GPU configuration, one benchmark step = one slice of the
    M = 1000 job on one batch: `launches` step launches of both levels, then the
    batch's restriction, Chan merge, sample scatter, per-cell sort and the W1
    between the levels."""
    import numpy as np

    works = pair_works(inputs)
    coarse, fine = works
    t_final = fine.t_final
    levels = [(w.nx, w.ny, w.dx, w.y_min) for w in works]
    ncx, ncy = coarse.nx, coarse.ny
    ncell = ncx * ncy
    stream = torch.cuda.current_stream()
    dev = dict(dtype=torch.float64, device="cuda")
    variants = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    per_real = max(sum(2 * vlbm.vlbm_state_bytes(vlbm.Params.jet(precision=v), w.nx, w.ny, 1) for w in works)
                   for v in variants)
    lup_per_launch_per_real = sum(w.nx * w.ny for w in works)

    if args.profile_launches > 0:
        B = args.batch or 16
        prec = variants[0]
        ens = vlbm.Ensemble(vlbm.Params.jet(precision=prec), levels,
                            vlbm.vlbm_kl_coefficients(inputs.DEFAULT_SEED, 0, B), B)
        if args.decomposition:
            ch, wpb, order, deal = args.decomposition.split(":")
            ens.set_tuning([int(c) for c in ch.split(",")], int(wpb), int(order), int(deal))
        elif args.chunk_rows:
            ens.tune("march", args.chunk_rows)
        ens.step(t_final, args.profile_launches, want_done=True)
        ens.close()
        # a plain 2 GiB device copy: what FETCH_SIZE / WRITE_SIZE read for bytes of known size
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"profiled {args.profile_launches} step launches of the 5056x2528 + 2528x1264 pair, "
              f"{B} realizations, {prec}, and one 2 GiB copy", flush=True)
        return 0

    # the job's statistics: running accumulators and the sample stores of all M realizations
    stores = [torch.zeros((PAIR_M_TOTAL, ncell), **dev) for _ in works]
    acc = [torch.empty((3, 2, ncell), **dev) for _ in works]
    mean = [torch.empty((3, ncell), **dev) for _ in works]
    std = [torch.empty((3, ncell), **dev) for _ in works]
    w1c = torch.empty(ncell, **dev)
    w1m = torch.zeros(1, **dev)
    B = args.batch
    if B <= 0:
        free, _ = torch.cuda.mem_get_info()
        B = int(max(1, min(64, (free - PAIR_HEADROOM) // per_real)))
    slots = PAIR_M_TOTAL // B
    L = args.launches
    progress(f"jet5056pair: batch of {B} realizations ({per_real / 1e9:.2f} GB each), {L} launches per step")

    def variant(prec):
        params = vlbm.Params.jet(precision=prec)
        coefs = vlbm.vlbm_kl_coefficients(inputs.DEFAULT_SEED, 0, B)
        ens = vlbm.Ensemble(params, levels, coefs, B)
        if not args.no_tune:
            ens.autotune(t_final, 8)  # live steps, counted toward t_final
        elif args.decomposition:
            ch, wpb, order, deal = args.decomposition.split(":")
            ens.set_tuning([int(c) for c in ch.split(",")], int(wpb), int(order), int(deal))
        elif args.chunk_rows:
            ens.tune("march", args.chunk_rows)
        chunks, wpb, order, deal = ens.get_tuning()
        tuned = {"rows_per_wave": chunks, "waves_per_block": wpb,
                 "item_order": "strip fastest" if order == 0 else "realization fastest",
                 "dealing": "static round-robin" if deal == 0 else "per-XCD work queues",
                 "autotuned": not args.no_tune}
        progress(f"{prec}: step kernel decomposition {tuned}")
        acc_step = {"step_ms": 0.0, "stats_s": 0.0}

        def one_step(k, timed):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ens.step(t_final, L, want_done=False)
            e1.record(stream)
            e1.synchronize()
            c0 = time.perf_counter()
            slot = k % slots
            subs = []
            for l, w in enumerate(works):
                vlbm.vlbm_ensemble_stats(ens.h, l, w.nx // ncx, acc[l], slot * B, stores[l], slot * B)
                sub = stores[l][slot * B:(slot + 1) * B]
                vlbm.vlbm_sort_samples(sub, ncell, B, stream)
                vlbm.vlbm_stats_finalize(acc[l], ncell, (slot + 1) * B, mean[l], std[l], stream)
                subs.append(sub)
            vlbm.vlbm_w1(subs[0], subs[1], ncell, B, w1c, w1m, stream)
            torch.cuda.synchronize()
            if timed:
                acc_step["step_ms"] += e0.elapsed_time(e1)
                acc_step["stats_s"] += time.perf_counter() - c0

        for k in range(args.warmup):
            one_step(k, False)
            progress(f"{prec}: warmup step {k + 1}/{args.warmup} done")
        s0 = [ens.times(l)[1].copy() for l in range(len(works))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            one_step(args.warmup + k, True)
            progress(f"{prec}: timed step {k + 1}/{args.steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        lups, steps_range = 0.0, []
        for l, w in enumerate(works):
            t, s, a, status = ens.times(l)
            if np.any(status != 0):
                raise RuntimeError(f"{prec}: level {l} latched a failure")
            lups += float((s - s0[l]).sum()) * w.nx * w.ny
            steps_range.append([int(s.min()), int(s.max())])
        t_reached = float(ens.times(1)[0].min())
        ens.close()
        del ens
        torch.cuda.empty_cache()
        n_launch = args.steps * L
        achieved = BYTES_PER_LUP[prec] * lups / (acc_step["step_ms"] / 1e3) / 1e9 if acc_step["step_ms"] else 0.0
        return {"value": lups / elapsed / 1e9 if elapsed > 0 else 0.0,
                "ms_per_step": elapsed / max(args.steps, 1) * 1e3,
                "achieved": achieved,
                "avg_launch_ms": acc_step["step_ms"] / max(n_launch, 1),
                "phases_ms": {"step_launches": round(acc_step["step_ms"] / max(args.steps, 1), 3),
                              "statistics": round(acc_step["stats_s"] * 1e3 / max(args.steps, 1), 3)},
                "tuned": tuned, "steps": steps_range, "t_reached": t_reached,
                "w1_between_levels": float(w1m.item())}

    res = {}
    for v in variants:
        res[v] = variant(v)
    # once per job (untimed): sort of the whole M = 1000 store of each level and the W1
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for l in range(len(works)):
        vlbm.vlbm_sort_samples(stores[l], ncell, PAIR_M_TOTAL, stream)
    vlbm.vlbm_w1(stores[0], stores[1], ncell, PAIR_M_TOTAL, w1c, w1m, stream)
    e1.record(stream)
    e1.synchronize()
    final_ms = e0.elapsed_time(e1)
    del stores, acc, mean, std
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth(torch)

    head = variants[0]
    r0 = res[head]
    bpl = BYTES_PER_LUP[head]
    out = {
        "metric": METRIC, "value": round(r0["value"], 4), "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r0["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"jet5056pair: Mach-2000 jet, the 5056x2528 level with its 2528x1264 partner on the same "
                               f"seeds (domain [0,1]x[-0.25,0.25], t_final={t_final:g}), M={PAIR_M_TOTAL} "
                               f"streamed in batches of {B}; one step = {L} step launches of both levels "
                               f"on one batch + its restriction to 2528x1264, Chan merge, scatter into the "
                               f"M={PAIR_M_TOTAL} sample stores, per-cell sort and W1 between the levels, {head}",
                   "precision": head, "levels": [[w.nx, w.ny] for w in works], "batch": B,
                   "realizations_total": PAIR_M_TOTAL, "launches_per_step": L, "t_final": t_final,
                   "seed": inputs.DEFAULT_SEED, "time_steps_reached": r0["steps"],
                   "t_reached": r0["t_reached"],
                   "node_updates_per_launch": B * lup_per_launch_per_real,
                   "step_kernel_decomposition": r0["tuned"],
                   "phases_ms_per_step": r0["phases_ms"],
                   "once_per_job_sort_and_w1_of_the_full_stores_ms": round(final_ms, 1)},
        "roofline": {"bound": "hbm", "achieved": round(r0["achieved"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(r0["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(head, "jet5056pair", B * lup_per_launch_per_real),
                     "kernel": "vlbm step kernel (both levels per launch)", "bytes_per_node_update": bpl,
                     "avg_launch_ms": round(r0["avg_launch_ms"], 4),
                     "device_copy_GBs": round(copy_gbs, 1),
                     "frac_of_device_copy": round(r0["achieved"] / copy_gbs, 4)},
        "w1_between_levels_batch": r0["w1_between_levels"],
    }
    if "mixed" in res and head == "fp64":
        rm = res["mixed"]
        out["mixed"] = {
            "value": round(rm["value"], 4), "unit": "GLUPS", "dtype": "f32+f64",
            "ms_per_step": round(rm["ms_per_step"], 3),
            "speedup_vs_fp64": round(rm["value"] / r0["value"], 4),
            "roofline": {"bound": "hbm", "achieved": round(rm["achieved"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(rm["achieved"] / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic("mixed", "jet5056pair", B * lup_per_launch_per_real),
                         "bytes_per_node_update": BYTES_PER_LUP["mixed"],
                         "avg_launch_ms": round(rm["avg_launch_ms"], 4),
                         "frac_of_device_copy": round(rm["achieved"] / copy_gbs, 4)},
            "time_steps_reached": rm["steps"], "step_kernel_decomposition": rm["tuned"],
            "phases_ms_per_step": rm["phases_ms"],
        }
        if not args.no_mixed_error:
            out["mixed"]["error_vs_fp64"] = mixed_error_study(torch, vlbm, inputs, inputs.WORKLOADS["jet640"],
                                                              (0.01, 0.1, 1.0), 240)
    rooflines = [(out["roofline"], bpl)]
    if "mixed" in out:
        rooflines.append((out["mixed"]["roofline"], BYTES_PER_LUP["mixed"]))
    for roof, alg in rooflines:
        tr = roof.get("traffic")
        if tr:
            per_lup = tr / (B * lup_per_launch_per_real)
            roof["hbm_bytes_per_node_update"] = round(per_lup, 1)
            roof["hbm_GBs_implied"] = round(roof["achieved"] * per_lup / alg, 1)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fine.name, fine.nx, fine.ny, fine.dx, fine.y_min, steps=3)
    print(json.dumps(out), flush=True)
    return 0


def run_pass(args, torch, vlbm, inputs) -> int:
    """Single-level workload, one benchmark step = one whole pass to t_final."""
    import numpy as np

    w = inputs.WORKLOADS[args.workload]
    R, r_stats, r_w1 = w.m, 1, 2
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    stream = torch.cuda.current_stream()
    ncell = w.nx * w.ny
    ncell_w1 = (w.nx // r_w1) * (w.ny // r_w1)

    def make_level(params):
        nbytes = vlbm.vlbm_state_bytes(params, w.nx, w.ny, R)
        bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
        lv = vlbm.Level(w.nx, w.ny, w.dx, w.y_min,
                        (vlbm._VP * 2)(bufs[0].data_ptr(), bufs[1].data_ptr()))
        return lv, bufs

    def fixed_tuning(h):
        """--decomposition (whole) or --chunk-rows (item height) on handle h."""
        if args.decomposition:
            ch, wpb, order, deal = args.decomposition.split(":")
            vlbm.vlbm_set_tuning(h, [int(c) for c in ch.split(",")], int(wpb), int(order), int(deal))
        elif args.chunk_rows:
            vlbm.vlbm_tune(h, "march", args.chunk_rows)

    if args.profile_launches > 0:
        params = vlbm.Params.jet(precision=args.precision if args.precision != "both" else "fp64")
        level, bufs = make_level(params)
        h = vlbm.vlbm_init_ensemble(params, [level], coefs, R, stream)
        fixed_tuning(h)
        vlbm.vlbm_step(h, w.t_final, args.profile_launches, want_done=True)
        vlbm.vlbm_destroy(h)
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"profiled {args.profile_launches} step launches of {w.name} "
              f"({R} x {w.nx} x {w.ny}) and one 2 GiB copy", flush=True)
        return 0

    def run_variant(precision: str, first_seed: int = 0, timed_steps=None, warmup=None, tune=True):
        params = vlbm.Params.jet(precision=precision)
        coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, first_seed, R)
        level, bufs = make_level(params)
        acc = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
        mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
        std = torch.empty_like(mean)
        sacc = torch.empty((3, 2, ncell_w1), dtype=torch.float64, device="cuda")
        samples = [torch.empty((R, ncell_w1), dtype=torch.float64, device="cuda") for _ in range(2)]
        w1c = torch.empty(ncell_w1, dtype=torch.float64, device="cuda")
        w1m = torch.zeros(1, dtype=torch.float64, device="cuda")
        # Autotune on live steps of a first ensemble (outside the timed region);
        # later ensembles of the same shape reuse the cached choice.
        tuned = [args.decomposition or args.chunk_rows]
        tune = tune and not args.no_tune
        if tune:
            h = vlbm.vlbm_init_ensemble(params, [level], coefs, R, stream)
            vlbm.vlbm_autotune(h, w.t_final, 4, 1)
            tuned = [decomposition(vlbm, h, 1, True)]
            vlbm.vlbm_destroy(h)
            progress(f"{precision}: step kernel decomposition {tuned[0]}")
        n_timed = args.steps if timed_steps is None else timed_steps
        n_warm = args.warmup if warmup is None else warmup
        step_ms, step_launches, totals = [0.0], [0], {"lups": 0.0}
        phases = {"init": 0.0, "step": 0.0, "stats": 0.0}
        last = {}

        def one_step(k: int, timed: bool):
            # phases timed on the host: each ends with a synchronization
            # (initialisation and vlbm_destroy synchronize the stream, the last
            # vlbm_step reads the completion flag back)
            c0 = time.perf_counter()
            h = vlbm.vlbm_init_ensemble(params, [level], coefs, R, stream)
            fixed_tuning(h)
            c1 = time.perf_counter()
            done = False
            while not done:
                if timed:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                done = vlbm.vlbm_step(h, w.t_final, args.chunk, want_done=True)
                if timed:
                    e1.record(stream)
                    e1.synchronize()
                    step_ms[0] += e0.elapsed_time(e1)
                    step_launches[0] += args.chunk
            c2 = time.perf_counter()
            t, s, a, status = vlbm.vlbm_times(h, 0, R)
            vlbm.vlbm_ensemble_stats(h, 0, r_stats, acc, 0, None, 0)
            vlbm.vlbm_stats_finalize(acc, ncell, R, mean, std, stream)
            cur, prev = samples[k % 2], samples[(k + 1) % 2]
            vlbm.vlbm_ensemble_stats(h, 0, r_w1, sacc, 0, cur, 0)
            vlbm.vlbm_sort_samples(cur, ncell_w1, R, stream)
            if k > 0:
                vlbm.vlbm_w1(cur, prev, ncell_w1, R, w1c, w1m, stream)
            vlbm.vlbm_destroy(h)
            c3 = time.perf_counter()
            if timed:
                totals["lups"] += float(s.sum()) * w.nx * w.ny
                for key, dt in (("init", c1 - c0), ("step", c2 - c1), ("stats", c3 - c2)):
                    phases[key] += dt
            last["steps"], last["sorted"] = s, cur
            return s

        for k in range(n_warm):
            one_step(k, False)
            progress(f"{precision}: warmup pass {k + 1}/{n_warm} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_timed):
            one_step(n_warm + k, True)
            progress(f"{precision}: timed pass {k + 1}/{n_timed} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        steps_r = last["steps"]
        lup_pass = float(steps_r.sum()) * w.nx * w.ny
        achieved = (BYTES_PER_LUP[precision] * lup_pass / (step_ms[0] / n_timed / 1e3) / 1e9
                    if step_ms[0] > 0 else 0.0)
        return {
            "value": totals["lups"] / elapsed / 1e9 if n_timed > 0 else 0.0,
            "ms_per_step": elapsed / max(n_timed, 1) * 1e3,
            "achieved": achieved,
            "avg_launch_ms": step_ms[0] / max(step_launches[0], 1),
            "launches_per_pass": step_launches[0] / max(n_timed, 1),
            "tuned_rows": tuned[0],
            "steps": [int(steps_r.min()), int(steps_r.max())],
            "w1_rerun": float(w1m.item()) if n_warm + n_timed > 1 else None,
            "phases_ms": {key: round(v * 1e3 / max(n_timed, 1), 3) for key, v in phases.items()},
            "mean": mean.clone(), "std": std.clone(), "sorted": last["sorted"].clone(),
        }

    variants = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {v: run_variant(v) for v in variants}

    def copy_bandwidth(nbytes: int = 1 << 31, reps: int = 5) -> float:
        """Device-to-device copy rate (bytes read + written per second), the
        practical HBM ceiling the step kernel is compared with."""
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
        e1.synchronize()
        gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
        del src, dst
        torch.cuda.empty_cache()
        return gbs

    copy_gbs = copy_bandwidth()
    head = variants[0]
    r0 = res[head]
    out = {
        "metric": METRIC, "value": round(r0["value"], 4), "unit": "GLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r0["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: Mach-2000 jet, {w.nx}x{w.ny} nodes on [0,1]x[-0.25,0.25], "
                               f"M={R} realizations to t={w.t_final:g}, {head}",
                   "precision": head, "nx": w.nx, "ny": w.ny, "realizations": R,
                   "t_final": w.t_final, "seed": inputs.DEFAULT_SEED,
                   "time_steps_per_realization": r0["steps"],
                   "step_kernel_decomposition": r0["tuned_rows"],
                   "phases_ms_per_step": r0["phases_ms"]},
        "roofline": {"bound": "hbm", "achieved": round(r0["achieved"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(r0["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(head, w.name),
                     "kernel": "vlbm step kernel", "bytes_per_node_update": BYTES_PER_LUP[head],
                     "avg_launch_ms": round(r0["avg_launch_ms"], 5),
                     "launches_per_pass": r0["launches_per_pass"],
                     "device_copy_GBs": round(copy_gbs, 1),
                     "frac_of_device_copy": round(r0["achieved"] / copy_gbs, 4)},
        "w1_rerun": r0["w1_rerun"],
    }

    def add_hbm(roof, precision):
        """Measured HBM bytes per node update (counters, per launch of all R x nx x
        ny updates) and the HBM rate they imply at the measured kernel speed."""
        tr = roof.get("traffic")
        if tr:
            per_lup = tr / (R * w.nx * w.ny)
            roof["hbm_bytes_per_node_update"] = round(per_lup, 1)
            roof["hbm_GBs_implied"] = round(roof["achieved"] * per_lup / BYTES_PER_LUP[precision], 1)

    add_hbm(out["roofline"], head)

    def stat_errors(a, b):
        """mean/std rel. L1 per field and W1 / mean density between two runs' final
        ensembles (a is the reference)."""
        rel = lambda x, y: float((x - y).abs().sum() / y.abs().sum())
        w1c = torch.empty(ncell_w1, dtype=torch.float64, device="cuda")
        w1m = torch.zeros(1, dtype=torch.float64, device="cuda")
        vlbm.vlbm_w1(a["sorted"], b["sorted"], ncell_w1, R, w1c, w1m, stream)
        torch.cuda.synchronize()
        sig = lambda x: float(f"{x:.4g}")
        return {"mean_rel_l1": [sig(rel(b["mean"][f], a["mean"][f])) for f in range(3)],
                "std_rel_l1": [sig(rel(b["std"][f], a["std"][f])) for f in range(3)],
                "w1_over_mean_rho": sig(float(w1m.item()) / float(a["mean"][0].mean())),
                "fields": ["rho", "|v|", "p"]}

    def early_stats(precision: str, t_early: float, first_seed: int = 0):
        """Ensemble statistics of a fresh run to t_early (untimed)."""
        params = vlbm.Params.jet(precision=precision)
        level, bufs = make_level(params)
        cf = inputs.kl_coefficients(inputs.DEFAULT_SEED, first_seed, R)
        h = vlbm.vlbm_init_ensemble(params, [level], cf, R, stream)
        while not vlbm.vlbm_step(h, t_early, args.chunk, want_done=True):
            pass
        acc = torch.empty((3, 2, ncell), dtype=torch.float64, device="cuda")
        mean = torch.empty((3, ncell), dtype=torch.float64, device="cuda")
        std = torch.empty_like(mean)
        sacc = torch.empty((3, 2, ncell_w1), dtype=torch.float64, device="cuda")
        smp = torch.empty((R, ncell_w1), dtype=torch.float64, device="cuda")
        vlbm.vlbm_ensemble_stats(h, 0, r_stats, acc, 0, None, 0)
        vlbm.vlbm_stats_finalize(acc, ncell, R, mean, std, stream)
        vlbm.vlbm_ensemble_stats(h, 0, r_w1, sacc, 0, smp, 0)
        vlbm.vlbm_sort_samples(smp, ncell_w1, R, stream)
        vlbm.vlbm_destroy(h)
        return {"mean": mean, "std": std, "sorted": smp}

    if "mixed" in res and head == "fp64":
        rm = res["mixed"]
        # the same comparison at earlier times, next to two FP64 ensembles on
        # disjoint seeds: while the mixed run's difference stays below the
        # latter the realizations have not yet decorrelated pathwise
        early = []
        for frac in (0.01, 0.1):
            t_e = w.t_final * frac
            ref = early_stats("fp64", t_e)
            early.append({"t": t_e, "mixed_vs_fp64": stat_errors(ref, early_stats("mixed", t_e)),
                          "fp64_independent": stat_errors(ref, early_stats("fp64", t_e, first_seed=R))})
            progress(f"early comparison at t={t_e:g} done")
        # sampling-noise scale: an independent FP64 ensemble (the next R seeds)
        other = run_variant("fp64", first_seed=R, timed_steps=0, warmup=1, tune=False)
        out["mixed"] = {
            "value": round(rm["value"], 4), "unit": "GLUPS", "dtype": "f32+f64",
            "ms_per_step": round(rm["ms_per_step"], 3),
            "speedup_vs_fp64": round(rm["value"] / r0["value"], 4),
            "roofline": {"bound": "hbm", "achieved": round(rm["achieved"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(rm["achieved"] / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic("mixed", w.name),
                         "bytes_per_node_update": BYTES_PER_LUP["mixed"],
                         "avg_launch_ms": round(rm["avg_launch_ms"], 5),
                         "frac_of_device_copy": round(rm["achieved"] / copy_gbs, 4)},
            "error_vs_fp64": stat_errors(res["fp64"], rm),
            "fp64_independent_ensemble_difference": stat_errors(res["fp64"], other),
            "error_vs_fp64_earlier_times": early,
            "time_steps_per_realization": rm["steps"],
            "step_kernel_decomposition": rm["tuned_rows"],
            "phases_ms_per_step": rm["phases_ms"],
        }
        add_hbm(out["mixed"]["roofline"], "mixed")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.name, w.nx, w.ny, w.dx, w.y_min)
    print(json.dumps(out), flush=True)
    return 0


def run_study(args, torch, vlbm, inputs) -> int:
    """Nested levels of the jet with the same seeds in one ensemble: one step of
    all levels is one launch; at each checkpoint the convergence study of
    Sec. 3.3-3.4 on the coarsest (common) grid."""
    import numpy as np

    from paper_2605_25282_amd import convergence

    precision = args.precision if args.precision != "both" else "fp64"
    if args.study_geometry == "paper":
        works = [inputs.PAPER_GRIDS[f"paper{nx}"] for nx in (500, 1000, 2000, 4000)[:args.study_levels]]
        R = args.study_m or 32
        checkpoints = list(inputs.PAPER_CHECKPOINTS)
        geometry = "the paper's domain [0,2.5]x[-1,1]"
    else:
        works = [inputs.WORKLOADS[n] for n in ("jet320", "jet640", "jet1280")]
        R = args.study_m or 128
        checkpoints = [1e-3]
        geometry = "[0,1]x[-0.25,0.25]"
    shapes = [(w.nx, w.ny) for w in works]
    levels = [(w.nx, w.ny, w.dx, w.y_min) for w in works]
    dx = [w.dx for w in works]
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, R)
    params = vlbm.Params.jet(precision=precision)
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_tune:
        ens = vlbm.Ensemble(params, levels, coefs, R)
        ens.autotune(checkpoints[0], 4)
        tuned = decomposition(vlbm, ens.h, len(levels), True)
        ens.close()
        del ens  # release the tuning ensemble's state before the measured one allocates its own
    ens = vlbm.Ensemble(params, levels, coefs, R)
    if args.chunk_rows:
        ens.tune("march", args.chunk_rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s, launches, lups, rows = 0.0, 0, 0.0, []
    prev = np.zeros((len(levels), R))
    for tc in checkpoints:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        launches += ens.run(tc, chunk=args.chunk)
        e1.record(stream)
        e1.synchronize()
        step_s += e0.elapsed_time(e1) / 1e3
        steps = []
        for l, (nx, ny) in enumerate(shapes):
            t, s, a, status = ens.times(l)
            if np.any(status != 0) or np.any(t != tc):
                print(json.dumps({"error": f"level {l} did not reach t = {tc:g} cleanly"}))
                return 1
            lups += float((s - prev[l]).sum()) * nx * ny
            prev[l] = s
            steps.append([int(s.min()), int(s.max())])
        st = convergence.study(ens, dx, 10, stream)
        progress(f"study: checkpoint t={tc:g} done ({launches} launches)")
        rows.append({"t": tc, "time_steps_per_realization": steps,
                     "errors": {f"{p}/{o}": [float(f"{x:.6g}") for x in v] for (p, o), v in st.errors.items()},
                     "rates": {f"{p}/{o}": round(v, 4) for (p, o), v in st.rates.items()}})
    elapsed = time.perf_counter() - t0
    ens.close()
    bpl = BYTES_PER_LUP[precision]
    grids = ", ".join(f"{nx}x{ny}" for nx, ny in shapes)
    out = {
        "metric": METRIC, "value": round(lups / elapsed / 1e9, 4), "unit": "GLUPS", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(elapsed * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"nested levels of the Mach-2000 jet ({grids} on {geometry}), M={R} "
                               f"realizations each with the same seeds, to t={checkpoints[-1]:g}, one "
                               f"launch per step of all levels, {precision}",
                   "launches": launches, "step_kernel_decomposition": tuned},
        "roofline": {"bound": "hbm", "achieved": round(bpl * lups / step_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(bpl * lups / step_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "vlbm step kernel (all levels per launch)",
                     "bytes_per_node_update": bpl, "avg_launch_ms": round(step_s * 1e3 / launches, 5)},
        "study": {"common_grid": list(shapes[0]), "dx": dx, "n_pd": 10,
                  "pairs": {p: [[shapes[c][0], shapes[f][0]] for c, f, _ in v]
                            for p, v in (("cauchy", convergence.cauchy_pairs(len(shapes) - 1)),
                                         ("reference", convergence.reference_pairs(len(shapes) - 1)))},
                  "checkpoints": rows},
    }
    print(json.dumps(out), flush=True)
    return 0


def run_centerline(args, torch, vlbm, inputs) -> int:
    """Centerline diagnostics of Sec. 4 on the paper's geometry at t = 0.0035:
    per node of the row next to the axis (y = +dx/2) the ensemble mean and
    std, the empirical quantiles p5, p16, p50, p84, p95 (eq:empcdf) and the
    width ratio Q (eq:widthratio), all from the library's kernels; then the
    summary numbers the paper quotes: the onset of the shear-layer spread
    (first x where the std exceeds three times the inlet's 0.30), the peak std
    and the mean there, the leading fringe (last x where p95 exceeds twice the
    ambient density) with the largest Q near it, and, over the mixing region
    (std > 1 and p16 > twice the ambient density), the medians of Q and of
    (p95 - mean) / (mean - p5)."""
    import numpy as np

    w = inputs.PAPER_GRIDS[f"paper{args.centerline}"]
    M = args.study_m or 64
    t_final = inputs.PAPER_CHECKPOINTS[-1]
    precision = args.precision if args.precision != "both" else "fp64"
    params = vlbm.Params.jet(precision=precision)
    stream = torch.cuda.current_stream()
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, M)
    level = [(w.nx, w.ny, w.dx, w.y_min)]
    if not args.no_tune:
        ens = vlbm.Ensemble(params, level, coefs, M)
        ens.autotune(t_final, 4)
        ens.close()
        del ens
    ens = vlbm.Ensemble(params, level, coefs, M)
    t0 = time.perf_counter()
    launches = 0
    while launches == 0 or not done:
        done = ens.step(t_final, args.chunk)
        launches += args.chunk
        progress(f"centerline: {launches} launches")
    t, s, a, status = ens.times(0)
    if np.any(status != 0) or np.any(t != t_final):
        print(json.dumps({"error": "the ensemble did not reach t_final cleanly"}))
        return 1
    step_s = time.perf_counter() - t0
    ncell = w.nx * w.ny
    dev = dict(dtype=torch.float64, device="cuda")
    acc = torch.empty((3, 2, ncell), **dev)
    smp = torch.empty((M, ncell), **dev)
    vlbm.vlbm_ensemble_stats(ens.h, 0, 1, acc, 0, smp, 0)
    ens.close()
    mean = torch.empty((3, ncell), **dev)
    std = torch.empty_like(mean)
    vlbm.vlbm_stats_finalize(acc, ncell, M, mean, std, stream)
    j = w.ny // 2  # y = y_min + (j + 1/2) dx = +dx/2
    row = smp[:, j * w.nx:(j + 1) * w.nx].contiguous()
    del smp
    vlbm.vlbm_sort_samples(row, w.nx, M, stream)
    pct = [5, 16, 50, 84, 95]
    qs = torch.empty((len(pct), w.nx), **dev)
    vlbm.vlbm_quantiles(row, w.nx, M, pct, qs, stream)
    q = torch.empty(w.nx, **dev)
    vlbm.vlbm_width_ratio(row, w.nx, M, q, stream)
    torch.cuda.synchronize()
    mu = mean[0, j * w.nx:(j + 1) * w.nx].cpu().numpy()
    sd = std[0, j * w.nx:(j + 1) * w.nx].cpu().numpy()
    p5, p16, p50, p84, p95 = qs.cpu().numpy()
    Q = q.cpu().numpy()
    x = (np.arange(w.nx) + 0.5) * w.dx
    rho_amb = params.rho_amb
    onset = np.nonzero(sd > 3 * 0.30)[0]
    fringe = np.nonzero(p95 > 2 * rho_amb)[0]
    i_f = int(fringe.max()) if fringe.size else -1
    near = slice(max(i_f - 40, 0), min(i_f + 41, w.nx)) if i_f >= 0 else slice(0, 0)
    Qn = Q[near]
    mix = (sd > 1.0) & (p16 > 2 * rho_amb)
    with np.errstate(divide="ignore", invalid="ignore"):
        skew = (p95 - mu) / (mu - p5)
    step = max(w.nx // 40, 1)
    out = {
        "metric": "centerline quantile diagnostics (Sec. 4)", "value": None, "unit": None, "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(step_s * 1e3, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: the paper's domain [0,2.5]x[-1,1] at {w.nx}x{w.ny}, M={M}, "
                               f"t={t_final:g}, alpha={params.alpha:.4g}, row y=+dx/2", "launches": launches,
                   "time_steps_per_realization": [int(s.min()), int(s.max())]},
        "diagnostics": {
            "shear_layer_onset_x": float(x[onset[0]]) if onset.size else None,
            "peak_std": float(sd.max()), "mean_at_peak_std": float(mu[int(sd.argmax())]),
            "x_peak_std": float(x[int(sd.argmax())]),
            "leading_fringe_x": float(x[i_f]) if i_f >= 0 else None,
            "max_Q_near_fringe": float(np.nanmax(Qn[np.isfinite(Qn)])) if np.any(np.isfinite(Qn)) else None,
            "mixing_region_nodes": int(mix.sum()),
            "median_Q_mixing_region": float(np.median(Q[mix])) if mix.any() else None,
            "median_band_skew_mixing_region": float(np.median(skew[mix])) if mix.any() else None,
            "laminar_core_std_x_0.2_to_0.8": float(sd[(x > 0.2) & (x < 0.8)].mean()),
            "laminar_core_mean_x_0.2_to_0.8": float(mu[(x > 0.2) & (x < 0.8)].mean()),
        },
        "profile": {"x": [round(float(v), 4) for v in x[::step]],
                    "mean": [round(float(v), 4) for v in mu[::step]], "std": [round(float(v), 4) for v in sd[::step]],
                    **{f"p{k}": [round(float(v), 4) for v in arr[::step]]
                       for k, arr in zip(pct, (p5, p16, p50, p84, p95))},
                    "Q": [None if not np.isfinite(v) else round(float(v), 4) for v in Q[::step]]},
    }
    print(json.dumps(out), flush=True)
    return 0


def run_w12(args, torch, vlbm) -> int:
    """Time vlbm_w12 at the paper's scale: M = 1000 samples per cell, n_pd = 10
    subsampled points per direction (10^4 ordered cell pairs, one exact
    assignment each) on a 500 x 400 common grid of seeded synthetic samples."""
    m, ncx, ncy, n_pd = 1000, 500, 400, 10
    g = torch.Generator(device="cuda")
    g.manual_seed(2605)
    a = 0.1 + 9.9 * torch.rand((m, ncy * ncx), dtype=torch.float64, device="cuda", generator=g)
    b = a * (1.0 + 0.3 * (2 * torch.rand((m, ncy * ncx), dtype=torch.float64, device="cuda",
                                         generator=g) - 1))
    wp = torch.empty(n_pd ** 4, dtype=torch.float64, device="cuda")
    wm = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    vlbm.vlbm_w12(a, b, ncx, ncy, m, n_pd, wp, wm, stream)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(max(args.steps, 1)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        vlbm.vlbm_w12(a, b, ncx, ncy, m, n_pd, wp, wm, stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
        progress(f"w12: {times[-1]:.1f} ms")
    ms = sorted(times)[len(times) // 2]
    print(json.dumps({"metric": "exact two-point W_{1,2} assignments per second", "value": round(n_pd ** 4 / (ms / 1e3), 1),
                      "unit": "assignments/s", "n_gpus": 1, "steps": len(times), "warmup": 1,
                      "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"W_(1,2) of {m} samples, n_pd = {n_pd} on a {ncx} x {ncy} grid "
                                             f"({n_pd ** 4} ordered cell pairs)"},
                      "w12_mean": wm.item()}), flush=True)
    return 0


def run_pair_full(args, torch, vlbm, inputs) -> int:
    """The largest level of the study and its half-resolution partner in one
    ensemble per batch (same seeds on both levels), batches streamed through
    HBM: the running statistics merge each batch (vlbm_ensemble_stats with
    n_prev / m_offset); after the last batch the sample stores are sorted and
    the one-point W1 between the levels is taken on the 2528 x 1264 grid."""
    import numpy as np

    precision = args.precision if args.precision != "both" else "fp64"
    fine = inputs.WORKLOADS["jet5056"]
    coarse = inputs.JetWorkload("jet2528", fine.nx // 2, fine.ny // 2, fine.m, fine.t_final)
    works = [coarse, fine]
    levels = [(w.nx, w.ny, w.dx, w.y_min) for w in works]
    B, Mb = args.pair_batches, args.pair_batch_m
    M = B * Mb
    ncx, ncy = coarse.nx, coarse.ny
    ncell = ncx * ncy
    params = vlbm.Params.jet(precision=precision)
    stream = torch.cuda.current_stream()
    dev = dict(dtype=torch.float64, device="cuda")
    acc = [torch.empty((3, 2, ncell), **dev) for _ in works]
    smp = [torch.empty((M, ncell), **dev) for _ in works]
    # the fine level's statistics on its own nodes too (no restriction): the
    # share of the ensemble variance that sits at the grid scale
    acc_nodes = torch.empty((3, 2, fine.nx * fine.ny), **dev)
    # lups: every node update of the run (the autotuner's live steps included),
    # over the whole run's time; lups_timed: those of the stepping loops alone,
    # over their HIP-event time (the roofline)
    step_s, lups, lups_timed, launches, tuned = 0.0, 0.0, 0.0, 0, None
    t0 = time.perf_counter()
    for b in range(B):
        coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, b * Mb, Mb)
        ens = vlbm.Ensemble(params, levels, coefs, Mb)
        if b == 0 and not args.no_tune:
            ens.autotune(fine.t_final, 4)  # live steps, cached for later batches
            tuned = decomposition(vlbm, ens.h, 2, True)
        steps_before = [ens.times(l)[1].astype(np.float64) for l in range(len(works))]
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        done, last = False, time.perf_counter()
        while not done:
            done = ens.step(fine.t_final, args.chunk)
            launches += args.chunk
            if time.perf_counter() - last > 30:
                progress(f"batch {b + 1}/{B}: stepping, level steps {ens.times(1)[1].min()}")
                last = time.perf_counter()
        e1.record(stream)
        e1.synchronize()
        step_s += e0.elapsed_time(e1) / 1e3
        for l, w in enumerate(works):
            t, s, a, status = ens.times(l)
            if np.any(status != 0) or np.any(t != w.t_final):
                print(json.dumps({"error": f"batch {b}, level {l} did not reach t_final cleanly"}))
                return 1
            lups += float(s.sum()) * w.nx * w.ny
            lups_timed += float((s - steps_before[l]).sum()) * w.nx * w.ny
            vlbm.vlbm_ensemble_stats(ens.h, l, w.nx // ncx, acc[l], b * Mb, smp[l], b * Mb)
        vlbm.vlbm_ensemble_stats(ens.h, 1, 1, acc_nodes, b * Mb, None, 0)
        ens.close()
        del ens  # release this batch's state before the next batch allocates its own
        progress(f"batch {b + 1}/{B} done ({step_s:.1f} s of stepping so far)")
    mean = [torch.empty((3, ncell), **dev) for _ in works]
    std = [torch.empty((3, ncell), **dev) for _ in works]
    for l in range(2):
        vlbm.vlbm_stats_finalize(acc[l], ncell, M, mean[l], std[l], stream)
        vlbm.vlbm_sort_samples(smp[l], ncell, M, stream)
    std_nodes = torch.empty((3, fine.nx * fine.ny), **dev)
    vlbm.vlbm_stats_finalize(acc_nodes, fine.nx * fine.ny, M, None, std_nodes, stream)
    w1c = torch.empty(ncell, **dev)
    w1m = torch.zeros(1, **dev)
    vlbm.vlbm_w1(smp[0], smp[1], ncell, M, w1c, w1m, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    bpl = BYTES_PER_LUP[precision]
    out = {
        "metric": METRIC, "value": round(lups / elapsed / 1e9, 4), "unit": "GLUPS", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(elapsed * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"largest level 5056x2528 with 2528x1264 on the same seeds, {B} "
                               f"batch{'es' if B > 1 else ''} of {Mb} realizations streamed to "
                               f"t={fine.t_final:g} (the study's M = 1000 would be {-(-1000 // Mb)} such "
                               f"batches), {precision}",
                   "launches": launches, "step_kernel_decomposition": tuned,
                   "extrapolated_s_for_m1000": round(elapsed / M * 1000, 1)},
        "roofline": {"bound": "hbm", "achieved": round(bpl * lups_timed / step_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(bpl * lups_timed / step_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "vlbm step kernel (both levels per launch)",
                     "bytes_per_node_update": bpl},
        "statistics": {"w1_between_levels_mean": w1m.item(),
                       "mean_rho_domain_average": [float(m[0].mean().item()) for m in mean],
                       "std_rho_domain_average": [float(s[0].mean().item()) for s in std],
                       "std_rho_domain_average_fine_level_own_nodes": float(std_nodes[0].mean().item())},
        "note": "one launch per step advances both levels of a batch; the roofline is taken over the stepping "
                "loops (HIP events) with the node updates they made, the autotuner's live steps excluded; value "
                "is over the whole run, autotuner, statistics merge, sample sorts and W1 included. "
                "std_rho_domain_average is on the 2528x1264 grid (the fine level restricted 2x2); "
                "std_rho_domain_average_fine_level_own_nodes is the fine level without restriction.",
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
