#!/usr/bin/env python3
"""Benchmark of the fused anisotropic-equilibrium BGK stream-collide step on one MI355X.

Workload: D3Q19 256^3 periodic, FP32 deviations, seeded random SPD tensor (seed 0),
tau = 0.7, 3-D Taylor-Green initial state u0 = 0.02 -- one "step" is one fused
stream-and-collide pass over the whole grid. Prints ONE JSON line:

  value        whole-job MLUPS (cells * steps / time / 1e6), inputs resident in HBM
  roofline     the step kernel against the 8 TB/s HBM peak: achieved = algorithmic bytes per
               launch (2 q sizeof(float) = 152 B per cell) / mean kernel time from HIP events
               on the launch stream; traffic = HBM bytes per launch from rocprofv3 counters
               (profiles/), null if the kernel source changed since they were taken; beside
               it the plain copy kernel's bandwidth and the time of free streaming with the
               step's own loads and stores (its data-movement floor)
  cpu_baseline the FP64 oracle on the host cores, a bounded sample of the same workload
  variants     FP16 / BF16 shifted-deviation storage and FP64 storage of the same workload:
               MLUPS, roofline fraction and the per-field error against the FP64 path; the
               FP32 step with the second-order equilibrium (cost of the third-order term)
  adjoint      gradient workload (D2Q9 512^2 and D3Q19 128^3 channels with gray obstacles,
               2000 steps, checkpoints every 100, FP32): time of lbm_grad (forward + reverse
               sweep) over the time of the forward pass alone; adjoint_fwd_ratio = D3Q19's
  porous       D3Q27 porous medium (ellipsoid mask, porosity 0.6, halfway bounce-back, body
               force 1e-6, tensor cs^2 diag(1.5, 1, 0.5), tau = 0.9), FP64 / FP32 / FP16 / BF16:
               MLUPS, fraction of peak on the useful bytes (fluid cells' populations plus the
               link words) and each precision's error against the FP64 path after 1000 steps
  batched      512 independent D3Q19 domains (edges 16..64, own tensor and tau each), FP32,
               500 steps: the autotuned schedule's MLUPS and fraction of the 8 TB/s peak, beside
               fixed step-per-launch and persistent schedules

  d2q9_64_shear_wave  the D2Q9 64^2 FP64 shear wave (1000 steps): the oracle's wall time, with the
               GPU's time for the same steps as context

The headline is the median of --runs timed runs of exactly --steps steps (after --warmup
steps); every storage variant is timed over at least 200 steps after at least 50 warm-up steps.

Usage: python bench.py [--steps K] [--warmup W] [--runs R] [--gpus 1] [--no-cpu-baseline] [--no-variants]
                       [--no-adjoint] [--no-batched] [--batched-steps N] [--no-porous] [--porous-n N]
                       [--leg LEG]   (one timed leg alone, for profilers; see LEGS)
"""
import argparse
import hashlib
import json
import os
import sys
import time

# the oracle's OpenMP runtime reads these when it starts: all host threads, pinned close
os.environ.setdefault("OMP_PROC_BIND", "close")
os.environ.setdefault("OMP_PLACES", "cores")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBPS = 8000.0  # MI355X HBM3E
METRIC = "MLUPS & % of HBM peak, D3Q19 256^3 fp32 vs fp16-shifted; adjoint/fwd ratio"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_d3q19_f32_256.txt")
# the step kernel's source: the kernel file and the per-cell header it instantiates
KERNEL_SRCS = [os.path.join(ROOT, "paper_2605_27004_amd", "csrc", f)
               for f in ("kernels.hip", "cell.hpp", "common.hpp", "lattice.hpp")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-porous", action="store_true")
    ap.add_argument("--porous-n", type=int, default=512)
    ap.add_argument("--batched-stepwise-only", action="store_true",
                    help="batched block: time the step-per-launch schedule only (no autotune, no cooperative launch)")
    ap.add_argument("--batched-steps", type=int, default=0, help="steps of the batched block (0: the workload's 500)")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--runs", type=int, default=5, help="timed runs of --steps steps each; the median is reported")
    ap.add_argument("--leg", choices=sorted(LEGS), default=None,
                    help="run one timed leg alone (for profilers) and print its figures instead of the bench line")
    return ap.parse_args()


# One timed leg each, for running under a profiler: the kernel named in the leg's record is
# launched `--steps` times after `--warmup` steps on that leg's workload.
LEGS = {
    "step-f32": ("D3Q19 256^3 FP32 step (the headline kernel)", "step", "f32"),
    "step-f16": ("D3Q19 256^3 FP16-shifted step", "step", "f16"),
    "step-bf16": ("D3Q19 256^3 BF16-shifted step", "step", "bf16"),
    "step-f64": ("D3Q19 256^3 FP64 step", "step", "f64"),
    "porous-f32": ("D3Q27 porous medium 512^3, FP32 (links step with body force)", "porous", "f32"),
    "porous-f16": ("D3Q27 porous medium 512^3, FP16-shifted (links step with body force)", "porous", "f16"),
    "porous-bf16": ("D3Q27 porous medium 512^3, BF16-shifted (links step with body force)", "porous", "bf16"),
    "porous-f64": ("D3Q27 porous medium 512^3, FP64 (links step with body force)", "porous", "f64"),
    "adjoint-d3q19": ("gradient workload D3Q19 128^3, FP32: lbm_grad over --steps steps", "adjoint", "f32"),
    "batched": ("512 batched D3Q19 domains, FP32, step per launch (domain-major tiles)", "batched", "f32"),
    "batched-xcd": ("512 batched D3Q19 domains, FP32, step per launch (each domain's tiles on one XCD)", "batched",
                    "f32"),
    "batched-persistent": ("512 batched D3Q19 domains, FP32, one cooperative launch (2 work-groups per CU, "
                           "64 Ki-cell items, XCD placement)", "batched", "f32"),
}


def run_leg(args):
    """One leg alone: prints {leg, what, us_per_step, ...} as one JSON line."""
    import numpy as np
    import torch

    import paper_2605_27004_amd as lbm
    import workloads as W

    torch.cuda.init()
    what, kind, storage = LEGS[args.leg]
    rec = {"leg": args.leg, "what": what, "steps": args.steps, "warmup": args.warmup}
    if kind == "step":
        wl = W.config2(n=args.n)
        p = lbm.make_params(wl.lattice, storage, wl.shape, wl.tensor, wl.tensor_kind, wl.tau)
        sim = lbm.Simulation(p, wl.rho, wl.s)
        t = timed_steps(sim, args.steps, args.warmup, torch)
        rec["us_per_step"] = round(t / args.steps * 1e6, 2)
    elif kind == "porous":
        wl3 = W.config3(n=args.porous_n)
        mask = torch.as_tensor(wl3.meta["mask"]).cuda()
        p3 = lbm.make_params("D3Q27", storage, wl3.shape, wl3.tensor, "theta", wl3.tau, force=wl3.meta["force"],
                             masked=True)
        sim = lbm.Simulation(p3, wl3.rho, wl3.s, mask=mask)
        t = timed_steps(sim, args.steps, args.warmup, torch)
        rec["us_per_step"] = round(t / args.steps * 1e6, 2)
        rec["fluid_cells"] = int((wl3.meta["mask"] == 0).sum())
    elif kind == "adjoint":
        wl4 = W.config4("D3Q19")
        gray = torch.as_tensor(wl4.meta["gray"].astype(np.float32), device="cuda")
        p4 = lbm.make_params("D3Q19", storage, wl4.shape, wl4.tensor, "theta", wl4.tau, force=wl4.meta["force"],
                             gray=True)
        sim = lbm.Simulation(p4, wl4.rho, wl4.s, mask=gray)
        sim.grad("flux", args.warmup, 10, wl4.meta["outlet_plane"], want_dmask=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.grad("flux", args.steps, 10, wl4.meta["outlet_plane"], want_dmask=True)
        torch.cuda.synchronize()
        rec["us_per_step"] = round((time.perf_counter() - t0) / args.steps * 1e6, 2)
    else:
        wl5 = W.config5()
        bt = lbm.Batch(wl5.lattice, storage, wl5.domains)
        if args.leg == "batched-persistent":
            bt.set_schedule(mode="persistent", xcd_group=1, wg_per_cu=2, chunk_cells=65536, group_bytes=0)
        elif args.leg == "batched-xcd":
            bt.set_schedule(mode="stepwise", xcd_group=1)
        bt.step(args.warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(bt.stream)
        bt.step(args.steps)
        e1.record(bt.stream)
        torch.cuda.synchronize()
        bt.status()
        rec["us_per_step"] = round(e0.elapsed_time(e1) * 1e3 / args.steps, 2)
        bt.close()
    print(json.dumps(rec), flush=True)


def progress(msg):
    """One progress line on stderr after each block (the JSON result stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per step launch from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by the copy-kernel calibration), or None when the kernel source has
    changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(ln.split(None, 1) for ln in fh if ln.strip() and not ln.startswith("#"))
    except (OSError, ValueError):
        return None
    if kv.get("kernel_sha", "").strip() != kernel_sha():
        return None
    return int(kv["bytes_per_launch"])


def timed_steps(sim, steps, warmup, torch, runs=1):
    """Seconds for `steps` steps after `warmup` untimed ones, timed with HIP events on the stream
    the kernels run on. With runs > 1: (median over `runs` timed runs back to back, all runs)."""
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream
    times = []
    for _ in range(runs):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    med = sorted(times)[len(times) // 2]
    return (med, times) if runs > 1 else med


# Every storage variant is timed over at least this much work, whatever --steps / --warmup say:
# on a freshly created context the first steps run slower while clocks ramp up.
VARIANT_WARMUP, VARIANT_STEPS = 50, 200


def field_errors(a, b, u0):
    """e(f), e(rho), e(s) of run a against reference run b (dicts of torch tensors)."""
    ef = ((a["f"] - b["f"]).abs().max() / b["f"].abs().max()).item()
    er = ((a["rho"] - b["rho"]).abs().max() / b["rho"].abs().max()).item()
    es = ((a["s"] - b["s"]).abs().max() / u0).item()
    return {"f": ef, "rho": er, "s": es}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the library runs on "
              "one GPU (the multi-GPU slab decomposition is described, not implemented).", file=sys.stderr)
        sys.exit(2)
    if args.leg:
        run_leg(args)
        return

    import numpy as np
    import torch

    import paper_2605_27004_amd as lbm
    import workloads as W

    torch.cuda.init()
    wl = W.config2(n=args.n)
    cells = wl.cells
    q = 19

    def make(storage, order=3):
        p = lbm.make_params(wl.lattice, storage, wl.shape, wl.tensor, wl.tensor_kind, wl.tau, order)
        return lbm.Simulation(p, wl.rho, wl.s)

    # the headline context first: its set-up (fields from the host, init kernel) leaves the GPU
    # idle for a while, so the copy-kernel calibration below runs between it and the timed steps
    sim = make("f32")

    # ---- plain copy kernel over the same bytes (practical ceiling; also brings the clocks up) ----
    nbytes = q * 4 * cells
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(20):
        lbm.lbm_stream_copy(dst, src, nbytes, stream.cuda_stream)
    torch.cuda.synchronize()
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lbm.lbm_stream_copy(dst, src, nbytes, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()

    # ---- headline: FP32 storage, median of --runs timed runs of exactly --steps steps ----
    runs = max(1, args.runs)
    if runs > 1:
        secs, run_secs = timed_steps(sim, args.steps, args.warmup, torch, runs=runs)
    else:
        secs, run_secs = timed_steps(sim, args.steps, args.warmup, torch), None
    mlups = cells * args.steps / secs / 1e6
    kernel_s = secs / args.steps
    alg_bytes = 2 * q * 4 * cells
    achieved = alg_bytes / kernel_s / 1e9
    _, _, tot = sim.moments(fields=False)
    # data-movement floor: the same loads and stores without the collision
    nfl = max(args.steps, VARIANT_STEPS)
    sim.stream_floor(max(args.warmup, VARIANT_WARMUP))
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(sim.stream)
    sim.stream_floor(nfl)
    f1.record(sim.stream)
    torch.cuda.synchronize()
    floor_s = f0.elapsed_time(f1) / 1e3 / nfl
    del sim
    torch.cuda.empty_cache()

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(kernel_s * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 {args.n}^3 periodic, FP32 shifted deviations, seeded SPD tensor "
                               "(eigenvalues U[0.6,1.4] cs^2, seed 0), tau=0.7, 3-D Taylor-Green u0=0.02",
                   "lattice": "D3Q19", "grid": list(wl.shape), "storage": "f32", "order": 3, "tau": wl.tau,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_GBPS, 4), "traffic": traffic_per_launch(),
                     "algorithmic_bytes_per_launch": alg_bytes, "kernel": "k_step<D3Q19, float, order 3, plain>",
                     "copy_kernel_GBps": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4),
                     "stream_floor_us": round(floor_s * 1e6, 1), "frac_of_stream_floor": round(floor_s / kernel_s, 4)},
        "mass_total": tot[0],
        "timing": {"runs": runs, "statistic": "median",
                   "run_ms_per_step": None if run_secs is None else [round(t / args.steps * 1e3, 5) for t in run_secs]},
    }

    progress(f"headline done: {kernel_s * 1e6:.1f} us per step")
    # ---- storage variants: speed and error against the FP64 path at full size ----
    if not args.no_variants:
        def run_fields(storage, steps):
            s_ = make(storage)
            s_.step(steps)
            rho, sv, _ = s_.moments()
            out = {"f": s_.f64(), "rho": rho, "s": sv}
            torch.cuda.synchronize()
            return out

        ref = run_fields("f64", wl.steps)
        variants = {}
        n_ = max(args.steps, VARIANT_STEPS)
        w_ = max(args.warmup, VARIANT_WARMUP)
        for storage, sz in (("f16", 2), ("bf16", 2), ("f64", 8)):
            s_ = make(storage)
            t_ = timed_steps(s_, n_, w_, torch)
            del s_
            torch.cuda.empty_cache()
            v = {"MLUPS": round(cells * n_ / t_ / 1e6, 1),
                 "frac": round(2 * q * sz * cells / (t_ / n_) / 1e9 / PEAK_GBPS, 4),
                 "us_per_step": round(t_ / n_ * 1e6, 2), "timed_steps": n_, "warmup_steps": w_}
            if storage != "f64":
                got = run_fields(storage, wl.steps)
                v["err_vs_f64_after_%d_steps" % wl.steps] = field_errors(got, ref, wl.u0)
                del got
                torch.cuda.empty_cache()
            variants[storage + ("_shifted" if storage != "f64" else "")] = v
        got = run_fields("f32", wl.steps)
        variants["f32_shifted"] = {"err_vs_f64_after_%d_steps" % wl.steps: field_errors(got, ref, wl.u0)}
        # cost of the third-order term: the same FP32 step with the second-order equilibrium
        s_ = make("f32", order=2)
        t_ = timed_steps(s_, n_, w_, torch)
        del s_
        variants["f32_order2"] = {"MLUPS": round(cells * n_ / t_ / 1e6, 1),
                                  "frac": round(2 * q * 4 * cells / (t_ / n_) / 1e9 / PEAK_GBPS, 4),
                                  "us_per_step": round(t_ / n_ * 1e6, 2), "timed_steps": n_, "warmup_steps": w_}
        del got, ref
        torch.cuda.empty_cache()
        line["variants"] = variants
        progress("storage variants done")
    # ---- gradient workload: adjoint/forward time ratio ----
    if not args.no_adjoint:
        adj = {}
        for lat in ("D2Q9", "D3Q19"):
            wl4 = W.config4(lat)
            gray = torch.as_tensor(wl4.meta["gray"].astype(np.float32), device="cuda")
            p4 = lbm.make_params(lat, "f32", wl4.shape, wl4.tensor, "theta", wl4.tau, force=wl4.meta["force"],
                                 gray=True)
            sim4 = lbm.Simulation(p4, wl4.rho, wl4.s, mask=gray)
            sim4.grad("flux", 20, 10, wl4.meta["outlet_plane"], want_dmask=True)   # warm-up
            t_fwd = timed_steps(sim4, wl4.steps, 100, torch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            jv, _, _, _ = sim4.grad("flux", wl4.steps, wl4.meta["checkpoint_every"], wl4.meta["outlet_plane"])
            torch.cuda.synchronize()
            t_grad = time.perf_counter() - t0
            adj[lat] = {"grid": list(wl4.shape), "steps": wl4.steps, "checkpoint_every": wl4.meta["checkpoint_every"],
                        "forward_s": round(t_fwd, 4), "forward_plus_adjoint_s": round(t_grad, 4),
                        "ratio_total": round(t_grad / t_fwd, 3), "ratio_backward": round((t_grad - t_fwd) / t_fwd, 3),
                        "objective": jv}
            sim4.close()
            del sim4, gray
            torch.cuda.empty_cache()
        line["adjoint"] = adj
        line["adjoint_fwd_ratio"] = adj["D3Q19"]["ratio_total"]
        progress("gradient workload done")
    else:
        line["adjoint_fwd_ratio"] = None

    # ---- porous medium: walls, body force, reduced-precision storage ----
    if not args.no_porous:
        wl3 = W.config3(n=args.porous_n)
        mask = torch.as_tensor(wl3.meta["mask"]).cuda()
        fluid = int((wl3.meta["mask"] == 0).sum())
        por = {"grid": list(wl3.shape), "solid_fraction": round(1 - fluid / wl3.cells, 4), "steps": wl3.steps}
        ref3 = None
        for storage, sz in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)):
            p3 = lbm.make_params("D3Q27", storage, wl3.shape, wl3.tensor, "theta", wl3.tau, force=wl3.meta["force"],
                                 masked=True)
            s3 = lbm.Simulation(p3, wl3.rho, wl3.s, mask=mask)
            n3 = 50
            t3 = timed_steps(s3, n3, 10, torch) / n3
            useful = fluid * 2 * 27 * sz + wl3.cells * 4
            rec = {"MLUPS": round(wl3.cells / t3 / 1e6, 1), "fluid_MLUPS": round(fluid / t3 / 1e6, 1),
                   "frac": round(useful / t3 / 1e9 / PEAK_GBPS, 4), "ms_per_step": round(t3 * 1e3, 4)}
            s3.step(wl3.steps - n3 - 10)
            rho3, sv3, _ = s3.moments()
            torch.cuda.synchronize()
            if ref3 is None:
                ref3 = (rho3, sv3)
                rec["max_s"] = sv3.abs().max().item()
            else:
                fl = mask == 0
                rec["err_vs_f64_after_%d_steps" % wl3.steps] = {
                    "rho": ((rho3 - ref3[0])[fl].abs().max() / ref3[0][fl].abs().max()).item(),
                    "s": ((sv3 - ref3[1]).abs().max() / ref3[1].abs().max()).item()}
                del rho3, sv3
            por[storage] = rec
            s3.close()
            del s3
            torch.cuda.empty_cache()
        del ref3, mask
        torch.cuda.empty_cache()
        line["porous"] = por
        progress("porous medium done")

    # ---- batched small domains: one schedule picked by the autotuner ----
    if not args.no_batched:
        wl5 = W.config5()
        if args.batched_steps > 0:
            wl5.steps = args.batched_steps
        bt = lbm.Batch(wl5.lattice, "f32", wl5.domains)
        if args.batched_stepwise_only:
            chosen, tune_ms = bt.schedule(), float("nan")
        else:
            chosen, tune_ms = bt.autotune(trial_steps=20)

        def time_batch(steps):
            bt.step(5)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(bt.stream)
            bt.step(steps)
            e1.record(bt.stream)
            torch.cuda.synchronize()
            bt.status()
            return e0.elapsed_time(e1) / 1e3

        def figures(sec):
            return {"MLUPS": round(wl5.cells * wl5.steps / sec / 1e6, 1),
                    "frac": round(152.0 * wl5.cells * wl5.steps / sec / 1e9 / PEAK_GBPS, 4),
                    "ms_per_step": round(sec / wl5.steps * 1e3, 4)}

        res = {"domains": len(wl5.domains), "cells": wl5.cells, "steps": wl5.steps, "storage": "f32",
               "autotuned": dict(schedule=chosen, trial_ms_per_step=round(tune_ms, 4), **figures(time_batch(wl5.steps)))}
        fixed = {"stepwise_xcd": dict(mode="stepwise", xcd_group=1),
                 "persistent_all": dict(mode="persistent", xcd_group=1, wg_per_cu=2, chunk_cells=65536, group_bytes=0),
                 "persistent_groups": dict(mode="persistent", xcd_group=1, wg_per_cu=2, chunk_cells=4096,
                                           group_bytes=192 << 20)}
        for name, sch in fixed.items():
            if args.batched_stepwise_only and sch["mode"] != "stepwise":
                continue
            bt.set_schedule(**sch)
            res[name] = figures(time_batch(wl5.steps))
        bt.close()
        del bt
        torch.cuda.empty_cache()
        line["batched"] = res
        progress("batched domains done")

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload ----
    if not args.no_cpu_baseline:
        import oracle

        ainv = oracle.tensor_to_ainv(wl.tensor, wl.tensor_kind, 3)
        f = oracle.init(wl.lattice, wl.shape, ainv, wl.rho, wl.s)
        t0 = time.perf_counter()
        oracle.steps(wl.lattice, wl.shape, ainv, wl.tau, f, args.cpu_steps)
        dt = time.perf_counter() - t0
        del f
        cpu_name = ""
        try:
            with open("/proc/cpuinfo") as fh:
                for ln in fh:
                    if ln.startswith("model name"):
                        cpu_name = ln.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        line["cpu_baseline"] = {"value": round(cells * args.cpu_steps / dt / 1e6, 3), "unit": "MLUPS",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"FP64 oracle, {args.cpu_steps} steps of the full {args.n}^3 D3Q19 "
                                          f"workload (init excluded), {dt:.1f} s on {cpu_name}, "
                                          f"OMP_PROC_BIND={os.environ.get('OMP_PROC_BIND')}"}
        # the D2Q9 64^2 shear wave (FP64, 1000 steps): its metric is the oracle's wall time, with the
        # GPU's time for the same steps as context (the grid is cache-resident, not an HBM test)
        wl1 = W.config1()
        ainv1 = oracle.tensor_to_ainv(wl1.tensor, wl1.tensor_kind, 2)
        f1 = oracle.init(wl1.lattice, wl1.shape, ainv1, wl1.rho, wl1.s)
        t0 = time.perf_counter()
        oracle.steps(wl1.lattice, wl1.shape, ainv1, wl1.tau, f1, wl1.steps)
        dt1 = time.perf_counter() - t0
        p1 = lbm.make_params(wl1.lattice, "f64", wl1.shape, wl1.tensor, wl1.tensor_kind, wl1.tau)
        g1 = lbm.Simulation(p1, wl1.rho, wl1.s)
        g1.step(20)
        torch.cuda.synchronize()
        g1.close()
        g1 = lbm.Simulation(p1, wl1.rho, wl1.s)
        tg1 = timed_steps(g1, wl1.steps, 0, torch)
        g1.close()
        line["d2q9_64_shear_wave"] = {"workload": "D2Q9 64^2 periodic shear wave, FP64, tau=0.8, 1000 steps",
                                      "oracle_wall_s": round(dt1, 4), "oracle_cores": oracle.num_threads(),
                                      "gpu_s": round(tg1, 5), "gpu_MLUPS": round(wl1.cells * wl1.steps / tg1 / 1e6, 1)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
