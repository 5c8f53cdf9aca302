"""Benchmark of the leap-frog hot path on one MI355X.

Default workload (one "step" of this benchmark): a forward-traces call on the 2D batched
case -- 1024^2 cells (1,050,625 nodes, 2,097,152 triangles), 64 monostatic sources on the
circle r = 1.4, 16,000 leap-frog steps, FP32 wave fields -- with the mesh and
permittivity already resident in HBM.  Metric: node-updates/s x sources (one node
advanced one step for one source).  The same JSON line carries sub-records for the other
workloads, each with its time and a roofline block: the same call in FP64, the plain
per-source FP64 stepper, the small 2D FP64 case (128^2 cells, one source, 4,000 steps) with
replayed graphs and with direct launches, the multigrid Jacobian of the 2D differentiation
case (coarse columns/s) with the TV solves that consume it, the 3D batched forward
(128^3 cells) and the 3D checkpointed misfit gradient (256^3 cells); also the FP64 CPU
oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs c2,c1,...]
    python bench.py --workload c1|c3|c4|c5 ... one workload as the headline, at full size
    python bench.py --workload c2pml ...    the 2D batched forward with the split-field PML
                                            and the lossy target
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LEGS_DEFAULT = ["direct", "fp64", "plain", "jacobian", "c1", "c4", "c5"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def step_kernel_bytes(n, nnz_off, B, esz):
    """Algorithmic HBM bytes of one stepping launch: per node and column read p_l, read
    p_{l-1}, write p_{l+1}; per node the stiffness row (int32 column + value per
    off-diagonal entry) and the beta coefficient."""
    return 3 * esz * n * B + nnz_off * (4 + esz) + esz * n


def kernel_source_hash():
    """Hash of the stepping kernels' source (the device code and its launch mapping);
    host-side changes (tuning, graph replay, shared host structures) leave it alone."""
    h = hashlib.sha256()
    for f in ("step_kernels.hpp",):
        h.update(open(os.path.join(ROOT, "paper_1707_04605_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(name, batch, variant):
    """HBM bytes per launch measured with rocprofv3 counters for this batch width and
    launch variant, if the committed summary was taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_hash:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    t = re.search(rf"hbm_bytes_per_launch_b{int(batch)}_v{int(variant)}:\s*([0-9.eE+]+)", txt)
    return float(t.group(1)) if t else None


def tuning(ctx):
    """Per-launch microseconds of the launch variants (0..15; 0 = not timed) from the
    tuning the last call ran (None if it ran none)."""
    t = ctx.last_timing()["tune_us"]
    return [round(x, 1) for x in t] if any(t) else None


def roofline(tm, n, esz, launches_ms, launches, counter_file=None, tune=None):
    """Stepping-kernel roofline: the library's algorithmic bytes of the last call's
    launches (which include velocity and accumulator traffic of adjoint sweeps) over the
    event-timed launch duration."""
    B = tm["batch"]
    nnz_off = int(round(tm["ell_mean_width"] * n))
    launch_bytes = step_kernel_bytes(n, nnz_off, B, esz)
    if tm.get("step_bytes", 0) > 0 and tm["step_launches"] > 0:
        launch_bytes = tm["step_bytes"] / tm["step_launches"]
    avg_launch_s = launches_ms / launches / 1e3
    achieved = launch_bytes / avg_launch_s / 1e9
    # the per-entry operator count (3 state words + stiffness row with one value per
    # entry + two diagonal coefficients, over B), for comparison
    entry_bytes = step_kernel_bytes(n, nnz_off, B, esz) + esz * n
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (traffic_from_profile(counter_file, B, tm["variant"])
                        if counter_file else None),
            "kernel": f"k_step (B={B}, {'FP32' if esz == 4 else 'FP64'}, variant {tm['variant']})",
            "bytes_per_launch": launch_bytes, "avg_launch_us": avg_launch_s * 1e6,
            "avg_launch_timing": ("HIP events on the library's stream around the replayed "
                                  "step graphs (and around each direct launch): kernel time "
                                  "plus the gaps between graph nodes, so at or above the "
                                  "profiler's kernel average"),
            "per_entry_bytes_per_launch": entry_bytes,
            "per_entry_frac": entry_bytes / avg_launch_s / 1e9 / HBM_PEAK_GBS,
            "bytes_per_node_update": launch_bytes / (n * B),
            "launch_variant_tuning_us": tune}


def base_result(args, metric, value, unit, ms_per_step, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic (seeded star-shaped body with voids; no dataset)",
            "config": config}


def value_and_roofline_calls(fn, ctx, steps):
    """`steps` calls of the production path (no per-launch events) give the wall time per
    call; one more call with HIP events around every stepping launch gives the launch
    durations for the roofline.  Returns (wall s per call, event ms sum, launches)."""
    wall, _, _ = timed_calls(lambda: fn(False), ctx, steps)
    _, ms, launches = timed_calls(lambda: fn(True), ctx, 1)
    return wall, ms, launches


def timed_calls(fn, ctx, steps):
    """Run fn() `steps` times between device synchronisations; return wall seconds per
    call and the summed event time and count of the stepping launches."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms, launches = 0.0, 0
    for _ in range(steps):
        fn()
        tm = ctx.last_timing()
        ms += tm["step_ms_total"]
        launches += tm["step_launches"]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, ms, launches


def copy_probe(args):
    """A device copy of known size (--copy-probe-gib) that calibrates the HBM byte
    counters of a profiled run."""
    if args.copy_probe_gib <= 0:
        return
    import torch
    nel = int(args.copy_probe_gib * (1 << 30)) // 4
    xa = torch.ones(nel, dtype=torch.float32, device="cuda")
    xb = torch.empty_like(xa)
    for _ in range(3):
        xb.copy_(xa)
    torch.cuda.synchronize()
    log(f"copy probe: {nel * 4} bytes read + {nel * 4} bytes written per copy")
    del xa, xb


def measure_forward(ctx, p, args, prec, n_steps=None, warmup=None, steps=None, **kw):
    """Forward-traces calls of problem p: warm-up calls (the first one times the batch
    widths and launch variants), `steps` production calls for the wall time, one call with
    event timing for the roofline.  The traces go to device memory (MGRT_F_DEVICE_OUT), so
    the timed calls move no output over PCIe.  Returns (traces of the last call as a NumPy
    array, wall s per call, event ms, launches, timing dict, launch-variant tuning or
    None)."""
    import torch
    n_steps = n_steps or p.n_steps
    warmup = args.warmup if warmup is None else warmup
    steps = args.steps if steps is None else steps
    if kw.get("variant", "batched") == "batched" and "out" not in kw:
        kw["out"] = torch.empty((p.src.shape[0], p.rec.shape[1], n_steps), dtype=torch.float64,
                                device="cuda")

    def run(timing=False):
        return ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, n_steps, precision=prec,
                                  timing=timing, **kw)

    tune = btune = None
    for _ in range(warmup):
        run()
        tune = tune or tuning(ctx)
        btune = btune or batch_tuning(ctx)
    wall, _, _ = timed_calls(run, ctx, steps)
    y = run(True)
    tm = ctx.last_timing()
    tm["batch_tuning"] = btune
    if hasattr(y, "cpu"):
        y = y.cpu().numpy()
    return y, wall, tm["step_ms_total"], tm["step_launches"], tm, tune


def bench_c2(args):
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    legs = LEGS_DEFAULT if args.legs is None else [x for x in args.legs.split(",") if x]
    if args.no_extra:
        legs = []
    p = configs.make("c2")
    n_steps = args.n_steps or p.n_steps
    n, n_src = p.mesh.n, p.src.shape[0]
    log(f"workload c2: n={n} m={p.mesh.m} sources={n_src} steps={n_steps} legs={legs}")
    ctx = context_for_problem(p)
    copy_probe(args)
    y, wall, ms, launches, tm, tune = measure_forward(ctx, p, args, 32, n_steps)
    updates = n * n_steps * n_src
    value = updates / wall
    log(f"fp32: {1e3 * wall:.1f} ms per call, {value:.3e} node-updates/s, batch {tm['batch']}, "
        f"{tm['graph_steps']} of {tm['step_launches']} steps replayed")
    result = base_result(
        args, "node-updates/s x sources (FP32 leap-frog, 2D batched)", value, "node-updates/s",
        1e3 * wall, "f32",
        {"workload": "2D batched forward: 1024^2 cells (1,050,625 nodes), 64 monostatic "
                     "sources, 16,000 steps, lumped mass, absorbing boundary",
         "nodes": n, "sources": n_src, "leapfrog_steps": n_steps, "batch": tm["batch"]})
    result["roofline"] = roofline(tm, n, 4, ms, launches, "step_fp32_c2_counters.md", tune)
    result["batch_tuning"] = tm["batch_tuning"]
    result["mall_note"] = mall_note(n, tm, 4)
    if "direct" in legs:
        # the same call with one direct launch per step instead of replayed step graphs
        wd, _, _ = timed_calls(lambda: ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, n_steps,
                                                          precision=32, graph=False), ctx, 1)
        result["direct_launches"] = {"value": updates / wd, "ms_per_call": 1e3 * wd,
                                     "graph_gain": wd / wall}
        # and with the traces returned to host memory (the 8 MB copy over PCIe inside the
        # call): not the headline value
        wh, _, _ = timed_calls(lambda: ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, n_steps,
                                                          precision=32), ctx, 1)
        result["host_output"] = {"value": updates / wh, "ms_per_call": 1e3 * wh,
                                 "note": "traces copied to host memory inside the call"}
        log(f"fp32 with host output: {1e3 * wh:.1f} ms per call")
        log(f"fp32 direct launches: {1e3 * wd:.1f} ms per call (graph replay gains "
            f"{wd / wall:.3f}x)")

    if "fp64" in legs:
        _, w64, ms64, l64, tm64, _ = measure_forward(ctx, p, args, 64, n_steps, warmup=1, steps=1)
        rf64 = roofline(tm64, n, 8, ms64, l64, "step_fp64_c2_counters.md")
        result["fp64"] = {"value": updates / w64, "unit": "node-updates/s",
                          "ms_per_call": 1e3 * w64, "batch": tm64["batch"],
                          "batch_tuning": tm64["batch_tuning"], "roofline": rf64,
                          "mall_note": mall_note(n, tm64, 8)}
        log(f"fp64: {updates / w64:.3e} node-updates/s, batch {tm64['batch']}")
    if "plain" in legs:
        # plain per-source FP64 CSR stepper, bounded sample: one source, 2,000 steps
        ns_plain = 2000
        ctx.forward_traces(p.src[:1], p.rec[:1], p.wavelet, p.dt, 50, precision=64,
                           variant="plain")
        wp, _, _ = timed_calls(lambda: ctx.forward_traces(p.src[:1], p.rec[:1], p.wavelet, p.dt,
                                                         ns_plain, precision=64, variant="plain"),
                               ctx, 1)
        result["plain_fp64"] = {"value": n * ns_plain / wp, "unit": "node-updates/s",
                                "ms_per_call": 1e3 * wp, "sample": "1 source x 2,000 steps"}
        result["speedup_fp32_vs_plain_fp64"] = value / result["plain_fp64"]["value"]
        log(f"plain fp64: {n * ns_plain / wp:.3e} node-updates/s")
    if "jacobian" in legs:
        # multigrid Jacobian (eq. approx_2) of the 2D differentiation case on the same mesh
        # and sources, and the TV solves that consume it; y are the traces at the true
        # permittivity from the headline call
        result.update(jacobian_tv_legs(ctx, configs.make("c3"), args, y, deconv=False))
    ctx.close()
    del ctx
    if "c1" in legs:
        result["c1"] = leg_c1(args)
    if "c4" in legs:
        result["c4"] = leg_c4(args)
    if "c5" in legs:
        result["c5"] = leg_c5(args)

    if not args.no_cpu:
        from oracle import Oracle
        o = Oracle.from_problem(p)
        ns_cpu = 3000
        t = time.perf_counter()
        o.forward(p.src[:1], p.rec[:1], p.wavelet, p.dt, ns_cpu)
        wc = time.perf_counter() - t
        result["cpu_baseline"] = {"value": n * ns_cpu / wc, "unit": "node-updates/s",
                                  "cores": o.threads, "kind": "oracle",
                                  "sample": f"1 source x {ns_cpu} steps of the same mesh "
                                            f"(FP64 mixed form), one run, {wc:.1f} s"}
        log(f"cpu oracle: {n * ns_cpu / wc:.3e} node-updates/s on {o.threads} threads")
        # the same on one core (a shorter sample)
        threads, ns1 = o.threads, 200
        o.set_threads(1)
        t = time.perf_counter()
        o.forward(p.src[:1], p.rec[:1], p.wavelet, p.dt, ns1)
        w1 = time.perf_counter() - t
        o.set_threads(threads)
        result["cpu_one_core"] = {"value": n * ns1 / w1, "unit": "node-updates/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"1 source x {ns1} steps of the same mesh "
                                            f"(FP64 mixed form), one run, {w1:.1f} s"}
        result["host"] = host_info()
        log(f"cpu oracle on one core: {n * ns1 / w1:.3e} node-updates/s")
        result["cpu_other"] = cpu_other_configs()
    return result


def cpu_other_configs():
    """The oracle on the small 2D case in full (all threads and one core) and on a short
    sample of the 3D batched mesh (all threads): per-node-update rates beside the GPU legs
    of the same configurations."""
    from oracle import Oracle
    from synth import configs

    out = {}
    p = configs.make("c1")
    o = Oracle.from_problem(p)
    rates = {}
    for threads in (o.threads, 1):
        keep = o.threads
        o.set_threads(threads)
        t = time.perf_counter()
        o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
        w = time.perf_counter() - t
        o.set_threads(keep)
        rates[threads] = (p.mesh.n * p.n_steps / w, w)
    out["c1"] = {"value": rates[o.threads][0], "cores": o.threads,
                 "one_core": rates[1][0], "unit": "node-updates/s", "kind": "oracle",
                 "sample": f"the whole case (1 source x {p.n_steps} steps), one run each, "
                           f"{rates[o.threads][1]:.2f} s / {rates[1][1]:.2f} s"}
    p4 = configs.make("c4")
    o4 = Oracle.from_problem(p4)
    ns4 = 30
    t = time.perf_counter()
    o4.forward(p4.src[:1], p4.rec[:1], p4.wavelet, p4.dt, ns4)
    w4 = time.perf_counter() - t
    out["c4"] = {"value": p4.mesh.n * ns4 / w4, "cores": o4.threads, "unit": "node-updates/s",
                 "kind": "oracle",
                 "sample": f"1 source x {ns4} steps of the 128^3 mesh, one run, {w4:.1f} s"}
    log(f"cpu oracle c1: {out['c1']['value']:.3e} ({o.threads} threads), "
        f"{out['c1']['one_core']:.3e} (one core); c4: {out['c4']['value']:.3e} node-updates/s")
    return out


def mall_note(n, tm, esz):
    """Whether one batch's working set (the two state fields and the per-node operator
    records) fits the 256 MB Infinity Cache, so that the roofline's HBM fraction may count
    traffic the cache serves."""
    ws = 2 * n * tm["batch"] * esz + (tm["step_bytes"] / tm["step_launches"]
                                      - 3 * n * tm["batch"] * esz if tm["step_launches"] else 0)
    return {"working_set_bytes": ws, "infinity_cache_bytes": 256 << 20,
            "fits": bool(ws <= (256 << 20))}


def batch_tuning(ctx):
    """Batch widths the last call timed and their per-launch microseconds (None if the
    call timed none)."""
    t = ctx.last_timing()
    out = {str(b): round(u, 1) for b, u in zip(t["tune_b"], t["tune_b_us"]) if b > 0}
    return out or None


def leg_c1(args):
    """The small 2D FP64 case (128^2 cells, 16,641 nodes, one source, 4,000 steps): a
    launch-bound run, with several steps per launch (each workgroup steps its tile and the
    tile's k-ring in LDS), with one launch per step (replayed step graphs, and direct
    launches) and with the plain per-source CSR stepper."""
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    p = configs.make("c1")
    n = p.mesh.n
    ctx = context_for_problem(p)
    reps = max(3, args.steps)
    _, wm, msm, lm, tmm, _ = measure_forward(ctx, p, args, 64, warmup=1, steps=reps)
    _, wg, msg, lg, tmg, _ = measure_forward(ctx, p, args, 64, warmup=1, steps=reps, one_step=True)
    _, wd, msd, ld, tmd, _ = measure_forward(ctx, p, args, 64, warmup=1, steps=reps, one_step=True,
                                             graph=False)
    _, wp, _, _, _, _ = measure_forward(ctx, p, args, 64, warmup=1, steps=reps, variant="plain")
    ctx.close()
    upd = n * p.n_steps
    rf = roofline(tmm, n, 8, msm, lm)
    rf["note"] = ("the 16,641-node state (133 KB per field) stays in the L2 caches and in LDS: "
                  "the step is bound by launch and synchronisation latency, not by HBM bandwidth")
    out = {"workload": "2D FP64: 128^2 cells (16,641 nodes, 32,768 triangles), 1 monostatic "
                       "source, 4,000 steps",
           "value": upd / wm, "unit": "node-updates/s", "ms_per_call": 1e3 * wm,
           "steps_per_launch": tmm["steps_per_launch"], "launches": lm,
           "one_step_replayed": {"value": upd / wg, "ms_per_call": 1e3 * wg,
                                 "steps_replayed": tmg["graph_steps"]},
           "one_step_direct": {"value": upd / wd, "ms_per_call": 1e3 * wd,
                               "avg_launch_us": 1e3 * msd / ld},
           "plain_fp64": {"value": upd / wp, "ms_per_call": 1e3 * wp},
           "multistep_gain": wg / wm, "graph_gain": wd / wg, "roofline": rf}
    log(f"c1: {tmm['steps_per_launch']} steps per launch {1e3 * wm:.1f} ms, one step per launch "
        f"replayed {1e3 * wg:.1f} ms, direct {1e3 * wd:.1f} ms, plain {1e3 * wp:.1f} ms per call "
        f"({upd / wm:.3e} node-updates/s)")
    return out


def leg_c4(args):
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    t = time.perf_counter()
    p = configs.make("c4")
    n, n_src = p.mesh.n, p.src.shape[0]
    log(f"c4: generated in {time.perf_counter() - t:.0f} s")
    ctx = context_for_problem(p)
    copy_probe(args)
    n_steps = args.n_steps or p.n_steps
    _, wall, ms, launches, tm, tune = measure_forward(ctx, p, args, 32, n_steps, warmup=1,
                                                      steps=max(1, args.steps - 1))
    bt = tm["batch_tuning"]
    ctx.close()
    value = n * n_steps * n_src / wall
    log(f"c4 fp32: {wall:.2f} s per call, {value:.3e} node-updates/s, batch {tm['batch']}")
    return {"workload": "3D batched forward: 128^3 cells (2,146,689 nodes, 12,582,912 tets), "
                        "32 monostatic sources, 6,000 steps, FP32",
            "value": value, "unit": "node-updates/s", "ms_per_call": 1e3 * wall,
            "batch": tm["batch"], "batch_tuning": bt,
            "roofline": roofline(tm, n, 4, ms, launches, "step_fp32_c4_counters.md", tune),
            "mall_note": mall_note(n, tm, 4)}


def leg_c5(args):
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    t = time.perf_counter()
    p = configs.make("c5")
    n_steps = args.n_steps or p.n_steps
    n, n_src = p.mesh.n, p.src.shape[0]
    log(f"c5: generated in {time.perf_counter() - t:.0f} s")
    ctx = context_for_problem(p)
    rho = np.random.default_rng(5).normal(size=(n_src, 2, n_steps)) * 1e-3
    # a short call first: it times the launch variants and batch widths once
    ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, 128, rho[..., :128], precision=32)
    tune, btune = tuning(ctx), batch_tuning(ctx)
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, n_steps, rho, precision=32, timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    tm = ctx.last_timing()
    ctx.close()
    value = n * n_steps * n_src / wall
    log(f"c5 gradient: {wall:.2f} s ({tm['step_launches']} launches, batch {tm['batch']})")
    return {"workload": "3D misfit gradient: 256^3 cells (16,974,593 nodes, 100,663,296 tets), "
                        "16 sources x 2 receivers, 12,000 steps, 32^3 coarse level, "
                        "checkpointed adjoint, FP32 fields with FP64 sums",
            "value": value, "unit": "node-updates/s (forward sweep)", "ms_per_call": 1e3 * wall,
            "batch": tm["batch"], "batch_tuning": btune, "stepping_launches": tm["step_launches"],
            "roofline": roofline(tm, n, 4, tm["step_ms_total"], tm["step_launches"], tune=tune),
            "mall_note": mall_note(n, tm, 4)}


def host_info():
    """CPU model and the cores this process may use, for the CPU baselines."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0))}


def bench_c2pml(args):
    """The 2D batched forward with the paper's boundary and losses (App. A split-field PML,
    Sec. III sigma = 5 eps_r in the target) instead of the first-order absorbing boundary,
    beside the same run with the absorbing boundary."""
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    p = configs.make("c2", pml=True)
    n_steps = args.n_steps or p.n_steps
    n, n_src = p.mesh.n, p.src.shape[0]
    xi, zeta = p.pml
    log(f"workload c2pml: n={n} sources={n_src} steps={n_steps} layer element-directions="
        f"{int((zeta > 0).sum())}")
    ctx = context_for_problem(p)
    import torch
    tr = torch.empty((n_src, p.rec.shape[1], n_steps), dtype=torch.float64, device="cuda")

    def run(timing=False):
        return ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, n_steps, precision=32,
                                  timing=timing, out=tr)

    tune = None
    for _ in range(args.warmup):
        run()
        tune = tune or tuning(ctx)
    wall, ms, launches = value_and_roofline_calls(run, ctx, args.steps)
    tm = ctx.last_timing()
    value = n * n_steps * n_src / wall
    log(f"pml fp32: {1e3 * wall:.1f} ms per call, {value:.3e} node-updates/s")
    result = base_result(
        args, "node-updates/s x sources (FP32 leap-frog, 2D batched)", value, "node-updates/s",
        1e3 * wall, "f32",
        {"workload": "2D batched forward: 1024^2 cells (1,050,625 nodes), 64 monostatic "
                     "sources, 16,000 steps, lumped mass, split-field PML [1.42, 1.5] "
                     "(varsigma 40), sigma = 5 eps_r in the target",
         "nodes": n, "sources": n_src, "leapfrog_steps": n_steps, "batch": tm["batch"]})
    rf = roofline(tm, n, 4, ms, launches, tune=tune)
    rf["kernel"] = f"k_step with the layer load and q update (B={tm['batch']}, FP32, variant {tm['variant']})"
    result["roofline"] = rf
    # the same workload with the first-order absorbing boundary instead
    pa = configs.make("c2")
    ctx2 = context_for_problem(pa)
    ctx2.forward_traces(pa.src, pa.rec, pa.wavelet, pa.dt, n_steps, precision=32, out=tr)
    wa, _, _ = timed_calls(lambda: ctx2.forward_traces(pa.src, pa.rec, pa.wavelet, pa.dt,
                                                       n_steps, precision=32, out=tr), ctx2, 1)
    result["absorbing_boundary"] = {"value": n * n_steps * n_src / wa, "ms_per_call": 1e3 * wa,
                                    "pml_cost": wall / wa}
    log(f"absorbing boundary: {1e3 * wa:.1f} ms per call; PML costs {wall / wa:.2f}x")
    return result


def jacobian_tv_legs(ctx, p, args, y_true, deconv):
    """Multigrid Jacobian of the 2D differentiation case (Sec. II-B eq. approx_2) on ctx
    (which holds the same mesh), then the TV-regularised step that consumes it (Sec. II-C
    eq. tv_iteration), the coarse-to-fine inversion (Sec. II-D/E) and the projected system
    (Sec. II-F).  y_true: traces at the true permittivity.  With deconv, also the paper's
    regularised-deconvolution route for a sweep of its Tikhonov parameter."""
    import torch
    from synth import acquisition as acq
    from synth import configs, levels, regularizer

    n, n_src, N = p.mesh.n, p.src.shape[0], p.n_steps
    ss = p.sample_steps
    M = p.mesh.n_coarse
    ctx.upload_permittivity(configs.prior_eps_fine(p))
    y0 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, N, precision=32)[..., ss]
    r = (acq.add_peak_noise(y_true[..., ss], configs.DATA_NOISE, configs.NOISE_SEED)
         - y0).reshape(-1)
    # J stays in HBM (caller-owned device output): the TV stages below consume it there
    J = torch.empty((n_src * ss.size, M), dtype=torch.float64, device="cuda")

    def jac(timing=False):
        return ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, N, ss, mode="mg", precision=32,
                                   timing=timing, out=J)

    tune = None
    for _ in range(max(1, args.warmup)):
        jac()
        tune = tune or tuning(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    jac(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ctx.last_timing()
    step_s = tm["step_ms_total"] / 1e3
    log(f"J2: {wall:.2f} s per call ({M / wall:.0f} cols/s), stepping {step_s:.2f} s, "
        f"batch {tm['batch']}, wavelet split {tm['jac_split']}, {tm['jac_runs']} run(s) per pair, "
        f"{tm['jac_sets']} history set(s)")
    out = {}
    out["jacobian"] = {
        "cols_per_s": M / wall, "unit": "coarse-cols/s", "ms_per_call": 1e3 * wall,
        "shape": list(J.shape), "output": "device memory", "batch": tm["batch"],
        "wavelet_split": bool(tm["jac_split"]), "runs_per_pair": tm["jac_runs"],
        "history_sets": tm["jac_sets"],
        "node_updates_per_s": tm["node_updates"] / wall,
        "stepping_s": step_s, "stepping_launches": tm["step_launches"],
        "workload": "multigrid Jacobian, 1024^2 cells, 64 sources x 512 samples, 64^2 coarse "
                    "level (8,192 columns), 16,000 steps, FP32 fields, FP64 sums",
        "roofline": roofline(tm, n, 4, tm["step_ms_total"], tm["step_launches"], tune=tune)}
    if deconv:
        dec = []
        nJ = float(torch.linalg.norm(J))
        Jd = torch.empty_like(J)
        for delta in (1e-1, 1e-2, 1e-3, 1e-4):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, N, ss, mode="deconv",
                                precision=32, deconv_delta=delta, out=Jd)
            torch.cuda.synchronize()
            wd = time.perf_counter() - t
            dec.append({"delta": delta, "seconds": wd,
                        "rel_error_vs_reciprocity": float(torch.linalg.norm(Jd - J)) / nJ})
            log(f"deconvolution route delta={delta:g}: {wd:.2f} s, relative difference from "
                f"J2 {dec[-1]['rel_error_vs_reciprocity']:.3f}")
        del Jd
        out["deconvolution_route"] = {
            "sweep": dec,
            "note": "App. A-2 route (source function at each receiver, Tikhonov deconvolution "
                    "of the recorded field, FP32 fields) against the reciprocity J2 of the "
                    "same call; relative Frobenius difference over the whole Jacobian"}
    rp, col, val = regularizer.tv_matrix(p.mesh.coords, p.mesh.coarse_verts, configs.TV_BETA)
    Ld = J.float()                                           # FP32 L resident in HBM
    lbytes = Ld.numel() * 4
    del J
    torch.cuda.synchronize()
    t = time.perf_counter()
    z, its = ctx.tv_invert_level(Ld, r, rp, col, val, configs.TV_ALPHA, iters=3, cg_rtol=1e-6,
                                 cg_maxit=5000)
    wtv = time.perf_counter() - t
    cg = int(np.sum(its))
    log(f"TV: {wtv:.2f} s, CG iterations {list(its)}")
    # coarse-to-fine inversion over 64^2 and 32^2 cells with the largest-third compression
    lv = levels.two_level(2, p.mesh.Nc)
    Dc = regularizer.tv_matrix(lv.coords, lv.verts2, configs.TV_BETA)
    t = time.perf_counter()
    tl = ctx.tv_invert_two_level(Ld, r, lv.verts1, lv.parent, lv.M2, Dc, (rp, col, val),
                                 configs.TV_ALPHA, iters=3, n_keep=levels.keep_third(lv.M2),
                                 cg_rtol=1e-6, cg_maxit=20000)
    wtl = time.perf_counter() - t
    log(f"two-level TV: {wtl:.2f} s, CG iterations {tl['cg_iters'].tolist()}")
    # projected data and Jacobian (Sec. II-F): 2 rows per trace, then the TV step with
    # alpha = 1e-7, beta = 1
    from paper_1707_04605_amd import projection_weights
    q = projection_weights(ss, p.dt, N)
    u = (r + y0.reshape(-1)).reshape(-1, ss.size)                # noisy measured samples
    proj = []
    for _ in range(1 + max(1, args.steps)):                      # first call warms up
        P = ctx.project_rows(Ld, u, q)
        proj.append(ctx.last_timing()["call_ms"])
    proj_ms = float(np.median(proj[1:]))
    yp = ctx.project_rows(u.reshape(-1, 1), u, q).reshape(-1)
    y0p = ctx.project_rows(y0.reshape(-1, 1), u, q).reshape(-1)
    rp1, col1, val1 = regularizer.tv_matrix(p.mesh.coords, p.mesh.coarse_verts, 1.0)
    t = time.perf_counter()
    zp, itp = ctx.tv_invert_level(P, yp - y0p, rp1, col1, val1, 1e-7, iters=3, cg_rtol=1e-6,
                                  cg_maxit=20000)
    wpj = time.perf_counter() - t
    log(f"projection of J: {proj_ms:.3f} ms ({lbytes / proj_ms / 1e6:.0f} GB/s; first call "
        f"{proj[0]:.3f} ms); projected TV "
        f"{wpj:.2f} s, CG iterations {list(itp)}")
    del Ld
    M2 = float(M) * M * 8
    # the normal matrix G = L^T L on the FP64 matrix cores dominates the direct solve
    out["tv"] = {"ms": 1e3 * wtv, "cg_iterations": [int(x) for x in its],
                 "L_bytes": lbytes, "normal_matrix_bytes": M2,
                 "solver": "dense Cholesky of L^T L + alpha D^T Gamma D per step" if cg == 0
                           else "preconditioned CG",
                 "roofline": {"bound": "mfma", "kernel": "k_syrk (G = L^T L, FP64 MFMA)",
                              "achieved": n_src * ss.size * float(M) * M / wtv / 1e12,
                              "peak": 78.6, "unit": "TFLOP/s",
                              "frac": n_src * ss.size * float(M) * M / wtv / 1e12 / 78.6,
                              "achieved_is_lower_bound": True,
                              "note": "rows x M^2 flops of G = L^T L (upper half) over the "
                                      "wall time of the whole 3-step solve"},
                 "note": "L resident in HBM; G = L^T L (FP64) formed once on the matrix "
                         "cores; each IRLS step factorises G + alpha D^T Gamma D = U^T U and "
                         "solves two triangular systems; wall time includes the host-side "
                         "Gamma and D^T Gamma D assembly"}
    out["tv_two_level"] = {
        "ms": 1e3 * wtl, "levels": [M, lv.M2], "kept_parents": levels.keep_third(lv.M2),
        "cg_iterations": tl["cg_iters"].tolist(),
        "note": "coarse-to-fine (T' 64^2 cells, T'' 32^2): L_c = L R_c and L_f = L R_f formed "
                "on the device, both levels solved directly (dense Cholesky) on their normal "
                "matrices formed on the matrix cores"}
    out["projected"] = {
        "projection_ms": proj_ms, "rows": [int(P.shape[0]), int(P.shape[1])],
        "tv_ms": 1e3 * wpj, "tv_cg_iterations": [int(x) for x in itp],
        "roofline": {"bound": "hbm", "kernel": "k_project_vec (one pass over the FP32 J)",
                     "achieved": lbytes / proj_ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": lbytes / proj_ms / 1e6 / HBM_PEAK_GBS},
        "note": "P = 2 time-weighted sums of every trace's 512 J rows; TV with alpha = 1e-7, "
                "beta = 1 on the 128-row system"}
    return out


def bench_c3(args):
    """The multigrid Jacobian of the 2D differentiation case as the headline, with the
    TV solves that consume it and the deconvolution-route sweep."""
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    p = configs.make("c3")
    n, n_src, N = p.mesh.n, p.src.shape[0], p.n_steps
    M = p.mesh.n_coarse
    log(f"workload c3: n={n} sources={n_src} steps={N} coarse columns={M}")
    ctx = context_for_problem(p)
    y = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, N, precision=32)
    legs = jacobian_tv_legs(ctx, p, args, y, deconv=not args.no_extra)
    jl = legs.pop("jacobian")
    result = base_result(
        args, "Jacobian coarse-cols/s (multigrid Jacobian, FP32 fields)", jl["cols_per_s"],
        "coarse-cols/s", jl["ms_per_call"], "f32",
        {"workload": "2D multigrid Jacobian: 1024^2 cells, 64 sources x 512 samples, 64^2 "
                     "coarse level (8,192 columns), 16,000 steps; then 3 TV-IRLS steps, one- and "
                     "two-level",
         "nodes": n, "sources": n_src, "leapfrog_steps": N, "batch": jl["batch"]})
    result["roofline"] = jl.pop("roofline")
    result["jacobian"] = jl
    result.update(legs)
    return result


def headline(args, leg, metric):
    """A sub-record of the default line as the headline of its own run."""
    result = base_result(args, metric, leg["value"], "node-updates/s", leg["ms_per_call"],
                         "f64" if "FP64" in leg["workload"] else "f32",
                         {"workload": leg["workload"]})
    result["roofline"] = leg.pop("roofline")
    result.update({k: v for k, v in leg.items() if k not in result and k != "workload"})
    return result


def bench_c1(args):
    return headline(args, leg_c1(args), "node-updates/s (FP64 leap-frog, 2D, one source)")


def bench_c4(args):
    return headline(args, leg_c4(args), "node-updates/s x sources (FP32 leap-frog, 3D batched)")


def bench_c5(args):
    return headline(args, leg_c5(args),
                    "node-updates/s x sources of the misfit gradient (FP32 fields, FP64 sums)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c2pml", "c3", "c4", "c5"])
    ap.add_argument("--legs", default=None,
                    help="comma-separated sub-records of the c2 line (default: "
                         + ",".join(LEGS_DEFAULT) + "); empty for none")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true", help="skip FP64, plain and Jacobian legs")
    ap.add_argument("--n-steps", type=int, default=None, help="override leap-frog steps")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the sources would "
              "shard over GPUs with no per-step exchange, but no multi-GPU path is built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    result = {"c1": bench_c1, "c2": bench_c2, "c3": bench_c3, "c4": bench_c4,
              "c5": bench_c5, "c2pml": bench_c2pml}[args.workload](args)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
