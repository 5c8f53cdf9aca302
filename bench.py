"""Benchmark of the leap-frog hot path on one MI355X.

Workload (one "step" of this benchmark): a forward-traces call on the 2D batched case --
1024^2 cells (1,050,625 nodes, 2,097,152 triangles), 64 monostatic sources on the circle
r = 1.4, 16,000 leap-frog steps, FP32 wave fields -- with the mesh and permittivity
already resident in HBM.  Metric: node-updates/s x sources (one node advanced one step
for one source).  Also reported: the same call in FP64, the plain per-source FP64
stepper on a bounded sample, the HBM roofline fraction of the stepping kernel
(algorithmic bytes per launch / event-timed launch duration) and the FP64 CPU oracle on
a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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


def step_kernel_bytes(n, nnz_off, B, esz):
    """Algorithmic HBM bytes of one stepping launch: per node and column read p_l, read
    p_{l-1}, write p_{l+1}; per node the stiffness row (int32 column + value per
    off-diagonal entry) and the alpha, beta coefficients."""
    return 3 * esz * n * B + nnz_off * (4 + esz) + 2 * esz * n


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("step.hip", "mgrt_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1707_04605_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(launch_bytes_alg):
    """HBM bytes per launch measured with rocprofv3 counters, if the committed summary
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_fp32_b64_c2_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_hash:\s*(\w+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extra", action="store_true", help="skip FP64 and plain legs")
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
    from paper_1707_04605_amd import context_for_problem
    from synth import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p = configs.make("c2")
    n_steps = args.n_steps or p.n_steps
    n, n_src = p.mesh.n, p.src.shape[0]
    print(f"[bench] workload c2: n={n} m={p.mesh.m} sources={n_src} steps={n_steps}",
          file=sys.stderr, flush=True)
    ctx = context_for_problem(p)
    stream = torch.cuda.current_stream()
    if args.copy_probe_gib > 0:
        nel = int(args.copy_probe_gib * (1 << 30)) // 4
        xa = torch.ones(nel, dtype=torch.float32, device="cuda")
        xb = torch.empty_like(xa)
        for _ in range(3):
            xb.copy_(xa)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {nel * 4} bytes read + {nel * 4} bytes written per copy",
              file=sys.stderr, flush=True)
        del xa, xb

    def run(prec, timing=False, **kw):
        return ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, n_steps, precision=prec,
                                  timing=timing, **kw)

    for _ in range(args.warmup):
        run(32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    step_ms = []
    launches = 0
    ev0.record(stream)
    for _ in range(args.steps):
        run(32, timing=True)
        tm = ctx.last_timing()
        step_ms.append(tm["step_ms_total"])
        launches += tm["step_launches"]
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    updates = n * n_steps * n_src
    value = updates / (wall / args.steps)
    print(f"[bench] fp32: {ms_per_step:.1f} ms per call, {value:.3e} node-updates/s",
          file=sys.stderr, flush=True)

    tm = ctx.last_timing()
    B = tm["batch"]
    nnz_off = int(round(tm["ell_mean_width"] * n))
    launch_bytes = step_kernel_bytes(n, nnz_off, B, 4)
    avg_launch_s = sum(step_ms) / launches / 1e3
    achieved = launch_bytes / avg_launch_s / 1e9
    traffic = traffic_from_profile(launch_bytes)
    result = {
        "metric": "node-updates/s x sources (FP32 leap-frog, 2D batched)",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded star-shaped body, 8 voids, eps noise)",
        "config": {"workload": "2D batched forward: 1024^2 cells (1,050,625 nodes), 64 "
                               "monostatic sources, 16,000 steps, lumped mass, absorbing "
                               "boundary",
                   "nodes": n, "sources": n_src, "leapfrog_steps": n_steps, "batch": B},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": f"k_step<float,4,16,4> (B={B})",
                     "bytes_per_launch": launch_bytes,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "bytes_per_node_update": launch_bytes / (n * B)},
    }

    if not args.no_extra:
        run(64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        run(64, timing=True)
        w64 = time.perf_counter() - t
        tm64 = ctx.last_timing()
        b64 = step_kernel_bytes(n, nnz_off, tm64["batch"], 8)
        result["fp64"] = {"value": updates / w64, "unit": "node-updates/s",
                          "ms_per_call": 1e3 * w64, "batch": tm64["batch"],
                          "hbm_frac": b64 / (tm64["step_ms_total"] / tm64["step_launches"] / 1e3)
                          / 1e9 / HBM_PEAK_GBS}
        # plain per-source FP64 CSR stepper, bounded sample: one source, 2,000 steps
        ns_plain = 2000
        ctx.forward_traces(p.src[:1], p.rec[:1], p.wavelet, p.dt, 50, precision=64,
                           variant="plain")
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.forward_traces(p.src[:1], p.rec[:1], p.wavelet, p.dt, ns_plain, precision=64,
                           variant="plain")
        wp = time.perf_counter() - t
        result["plain_fp64"] = {"value": n * ns_plain / wp, "unit": "node-updates/s",
                                "sample": "1 source x 2,000 steps"}
        result["speedup_fp32_vs_plain_fp64"] = value / result["plain_fp64"]["value"]

    if not args.no_cpu:
        from oracle import Oracle
        o = Oracle.from_problem(p)
        ns_cpu = 1500
        t = time.perf_counter()
        o.forward(p.src[:1], p.rec[:1], p.wavelet, p.dt, ns_cpu)
        wc = time.perf_counter() - t
        result["cpu_baseline"] = {"value": n * ns_cpu / wc, "unit": "node-updates/s",
                                  "cores": o.threads, "kind": "oracle",
                                  "sample": f"1 source x {ns_cpu} steps of the same mesh "
                                            f"(FP64 mixed form), {wc:.1f} s"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
