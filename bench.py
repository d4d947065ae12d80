#!/usr/bin/env python3
"""Throughput of PC-sample attribution on one GPU.

One step is one hpa_attribute call over the whole sample batch of the medium
plain-method workload (4 binaries, 20k functions, 2M instructions, 100k host
contexts, 256M samples): every sample's context, PC and stall reason are read,
samples are aggregated by (context, PC, stall) into keys sorted in that order,
and every key is labelled with its innermost scope through the structure map
(Section 4.2 sample records, Section 6.1 attribution).  The structure map is
built once before the timed region, as it is per set of binaries.  Inputs are
resident in device memory when the timed region starts.

Prints one JSON line.  `roofline` is for the dominant kernel (the unit sort and
reduce kernel, its launch over the units read through the run list), timed
with hipEvents on the call's stream through the library's stage timer; `cpu_baseline` times the CPU oracle on a bounded prefix of the
same samples.  `--copy-calibration BYTES` instead runs a plain device copy of
that size (the scale for hardware byte counters) and exits.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_units32_medium_traffic.json")
# the unit kernel's sources, in the order their hash is taken
UNITS_SRCS = [os.path.join(ROOT, "paper_2109_06931_amd", "csrc", f)
              for f in ("attribute.hip", "block_prims.h", "hpa_internal.h")]


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=256_000_000, help="samples per batch (default: the full workload)")
    ap.add_argument("--cpu-samples", type=int, default=8_000_000, help="oracle sample (prefix of the batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES")
    return ap.parse_args()


def _copy_calibration(nbytes: int) -> None:
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "launches": 3}), flush=True)


def _units_traffic():
    """HBM bytes per launch of the unit kernel from committed counter runs, or
    None when absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        h = hashlib.sha256()
        for src in UNITS_SRCS:
            with open(src, "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sha:
        return None
    return float(t["fetch_bytes_per_launch"]) + float(t["write_bytes_per_launch"])


def _cpu_baseline(w, n: int, target_s: float = 15.0, cap: int = 96_000_000):
    """The oracle on a prefix of the batch (whole kernel-invocation runs): one
    run of n samples, then, if that took under target_s / 2, one run sized for
    about target_s seconds (at most cap samples); the last run is reported."""
    import oracle
    oracle.build()
    m = oracle.build_map_workload(w)

    def run(k):
        t0 = time.perf_counter()
        a = oracle.attribute(m, w.pc[:k], w.ctx[:k], w.stall[:k], None if w.weight is None else w.weight[:k],
                             w.n_ctx)
        dt = time.perf_counter() - t0
        assert int(a.count.sum()) == (k if w.weight is None else int(w.weight[:k].sum()))
        return dt

    n = min(n, w.n_samples)
    dt = run(n)
    if dt < target_s / 2 and n < min(cap, w.n_samples):
        n = int(min(cap, w.n_samples, n * target_s / max(dt, 1e-3)))
        dt = run(n)
    return {"value": n / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} samples of the same batch (whole kernel-invocation runs), "
                      f"{dt:.1f} s single-threaded"}


def main():
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}); "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        _copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import paper_2109_06931_amd as hpa
    from workloads import config2

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    print(f"[bench] generating the medium workload ({args.samples} samples)", file=sys.stderr, flush=True)
    w = config2(n_samples=args.samples, threads=16)
    ctx = hpa.Context(0)
    t0 = time.perf_counter()
    m = hpa.build_structure_map_workload(ctx, w)
    torch.cuda.synchronize()
    map_ms = (time.perf_counter() - t0) * 1e3
    pc, cx, st, wt = hpa.samples_to_device(w)
    torch.cuda.synchronize()
    N = w.n_samples

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    U = 0
    for _ in range(args.warmup):
        a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
        U = a.n_keys
        del a
    # invariant check outside the timed region: every sample attributed once
    a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
    U = a.n_keys
    total = int(a.tensors()["count"].sum().item())
    assert total == (N if wt is None else int(w.weight.sum())), "attribution lost samples"
    del a

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
        del a
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.timing()
    ctx.set_timing(False)
    ms_step = dt * 1e3 / args.steps
    value = N * args.steps / dt

    M = m.n_intervals
    b_alg = 13.0 + 25.0 * U / N + 16.0 * M / N
    # the unit sort kernel (its launch over the units read through the run
    # list) reads its samples (13 B each by the record layout); its packed
    # output is staging for the write pass, so it is not counted
    u = stages.get("units_plain", {})
    u_ms = u.get("ms", 0.0) / max(u.get("calls", 1), 1)
    u_bytes = 13.0 * u.get("items_in", 0) / max(u.get("calls", 1), 1)
    achieved = u_bytes / (u_ms * 1e-3) / 1e9 if u_ms > 0 else 0.0
    traffic = _units_traffic()
    roofline = {"bound": "hbm", "kernel": "k_units32<false, false, false>", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic),
                "launch_ms": round(u_ms, 3), "algorithmic_bytes": round(u_bytes)}
    pipe_gbps = value * b_alg / 1e9
    pipeline = {"B_alg_bytes_per_sample": round(b_alg, 3), "achieved": round(pipe_gbps, 1), "unit": "GB/s",
                "frac": round(pipe_gbps / HBM_PEAK_GBPS, 4), "map_build_ms": round(map_ms, 1),
                "stages_ms": {k: round(v["ms"] / max(v["calls"], 1), 3) for k, v in stages.items()}}
    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] oracle on {min(args.cpu_samples, N)} samples", file=sys.stderr, flush=True)
        cpu = _cpu_baseline(w, args.cpu_samples)
    out = {
        "metric": "PC samples attributed/sec (frac of HBM BW)", "value": value, "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain method, medium: 4 binaries, 20k functions, 2M instructions, "
                               "200k line intervals, 5k loops, 100k host contexts, 256M samples",
                   "n_samples": N, "n_contexts": int(w.n_ctx), "unique_keys": int(U), "intervals": int(M),
                   "seed": int(w.seed)},
        "roofline": roofline, "pipeline": pipeline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
