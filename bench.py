#!/usr/bin/env python3
"""Throughput of PC-sample attribution on one GPU, plus the report lines of the
learned index, batched profiles, serving ingest and the calling-context tree.

One step is one hpa_attribute call over the whole sample batch of the medium
plain-method workload (4 binaries, 20k functions, 2M instructions, 100k host
contexts, 256M samples): every sample's context, PC and stall reason are read,
samples are aggregated by (context, PC, stall) into keys sorted in that order,
and every key is labelled with its innermost scope through the structure map
(Section 4.2 sample records, Section 6.1 attribution).  The structure map is
built once before the timed region.  Inputs are resident in device memory when
the timed region starts, and the timed steps run with the library's stage
timer off.

Prints one JSON line.  `roofline` is for the dominant kernel (the unit sort and
reduce kernel over the units read through the run list), timed with hipEvents
on the call's stream by the library's stage timer in separate calls after the
timed steps; `pipeline` prices the whole step against HBM peak and against a
device-to-device copy measured here; `cpu_baseline` times the CPU oracle on a
prefix of the same samples.  The other sections (each skippable):

  tiny      the tiny plain-method workload (1M samples), samples/s
  cct       the calling-context tree and derived metrics of the tiny workload
  learned   5e7 intervals, 1e9 queries: learned index vs plain binary search
  batched   4,096 profiles of lognormal size: one batched call per group of
            profiles vs one hpa_attribute call per profile
  serve     512 streams of buffers (4 KB-16 MB) at Poisson offered loads:
            latency percentiles and sustained samples/s

`--copy-calibration BYTES` instead runs a plain device copy of that size (the
scale for hardware byte counters) and exits.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_d_units_medium_traffic.json")
# the unit kernel's sources, in the order their hash is taken
UNITS_SRCS = [os.path.join(ROOT, "paper_2109_06931_amd", "csrc", f)
              for f in ("attribute_dense.hip", "unit_sort.h", "block_prims.h", "hpa_internal.h")]
SECTIONS = ("tiny", "cct", "learned", "batched", "serve")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=256_000_000, help="samples per batch (default: the full workload)")
    ap.add_argument("--cpu-samples", type=int, default=8_000_000, help="oracle sample (prefix of the batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip", default="", help="comma-separated sections to skip: " + ",".join(SECTIONS))
    ap.add_argument("--only-headline", action="store_true", help="skip every extra section")
    ap.add_argument("--learned-queries", type=int, default=1_000_000_000)
    ap.add_argument("--batched-groups", type=int, default=4, help="groups of profiles, one batched call each")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="offered-load duration per rate")
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


def _copy_ceiling(nbytes: int = 4 << 30, reps: int = 10) -> float:
    """Device-to-device copy rate (bytes read + written per second), GB/s."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


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


def _host_cpu():
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "model": model}


def _cpu_baseline(w, n: int, target_s: float = 15.0, cap: int = 96_000_000):
    """The oracle on a prefix of the batch: one run of n samples, then, if that
    took under target_s / 2, one run sized for about target_s seconds (at most
    cap samples); the last run is reported."""
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
            "sample": f"the first {n} samples of the same batch (a prefix of the record stream), "
                      f"{dt:.1f} s single-threaded", "host": _host_cpu()}


def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


# ---------------------------------------------------------------------------
# sections
# ---------------------------------------------------------------------------
def section_tiny(hpa, ctx):
    from workloads import config1
    w = config1()
    m = hpa.build_structure_map_workload(ctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    for _ in range(3):
        hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
    dt = _timed(lambda: hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx), reps=20)
    return {"workload": "plain method, tiny: 64 functions, 4,096 instructions, 32 placeholders, 1M samples",
            "samples_per_s": w.n_samples / dt, "ms_per_call": round(dt * 1e3, 3)}


def section_cct(hpa, ctx):
    import numpy as np
    import oracle
    from workloads import config1
    w = config1()
    m = hpa.build_structure_map_workload(ctx, w)
    pc, cx, st, wt = hpa.samples_to_device(w)
    a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
    plan = hpa.prepare_callgraph_workload(ctx, m, w)
    try:
        hpa.apportion_callpaths(ctx, plan, a)
    except hpa.HpaError as e:
        if e.code != hpa.E_UNSUPPORTED:
            raise
        return {"workload": "plain method, tiny (1M samples, 32 placeholders)", "status": "compiled out",
                "reason": str(e)}
    dt_a = _timed(lambda: hpa.apportion_callpaths(ctx, plan, a), reps=5)
    t = hpa.apportion_callpaths(ctx, plan, a)
    dt_d = _timed(lambda: hpa.derive_metrics(ctx, plan, a, t), reps=5)
    d = hpa.derive_metrics(ctx, plan, a, t)
    om, oa, ot, od = oracle.run_all(w)
    tt = t.numpy()
    exact = bool(np.array_equal(tt["node"], ot.node) and np.array_equal(tt["parent"], ot.parent))
    rel = float(np.max(np.abs(tt["excl"] - ot.excl) / np.maximum(np.abs(ot.excl), 1e-300))) if len(ot.excl) else 0.0
    return {"workload": "plain method, tiny (1M samples, 32 placeholders)", "cct_nodes": int(t.n_nodes),
            "apportion_ms": round(dt_a * 1e3, 3), "derive_ms": round(dt_d * 1e3, 3),
            "nodes_equal_oracle": exact, "max_rel_err_excl": rel}


def section_learned(hpa, ctx, n_queries):
    import torch
    from workloads import learned_intervals, learned_queries_gpu
    start, end = learned_intervals()
    m = hpa.build_structure_map(ctx, iv_start=start, iv_end=end)
    t0 = time.perf_counter()
    st_untrained = hpa.learned_train(ctx, m, train_steps=0)
    q = learned_queries_gpu(start, end, n_queries)
    out_p = torch.empty(n_queries, dtype=torch.uint32, device="cuda")
    out_l = torch.empty_like(out_p)
    one = q[: min(n_queries, 100_000_000)]
    # untrained root: counted lookup on the first 1e8 queries
    cnt = torch.zeros(2, dtype=torch.uint64, device="cuda")
    hpa.lookup_learned_counted(ctx, m, one, out_l[: one.numel()], cnt)
    ms_u = _timed(lambda: hpa.lookup_intervals(ctx, m, one, out_l[: one.numel()], mode=hpa.LOOKUP_LEARNED)) * 1e3
    cu = cnt.cpu().numpy().view("uint64")
    t1 = time.perf_counter()
    st = hpa.learned_train(ctx, m)
    train_s = time.perf_counter() - t1
    hpa.lookup_intervals(ctx, m, q, out_p, mode=hpa.LOOKUP_PLAIN)
    hpa.lookup_intervals(ctx, m, q, out_l, mode=hpa.LOOKUP_LEARNED)
    ms_plain = _timed(lambda: hpa.lookup_intervals(ctx, m, q, out_p, mode=hpa.LOOKUP_PLAIN), reps=3) * 1e3
    ms_learn = _timed(lambda: hpa.lookup_intervals(ctx, m, q, out_l, mode=hpa.LOOKUP_LEARNED), reps=3) * 1e3
    identical = bool(torch.equal(out_p, out_l))
    cnt.zero_()
    hpa.lookup_learned_counted(ctx, m, one, out_l[: one.numel()], cnt)
    ms_t1 = _timed(lambda: hpa.lookup_intervals(ctx, m, one, out_l[: one.numel()], mode=hpa.LOOKUP_LEARNED)) * 1e3
    ct = cnt.cpu().numpy().view("uint64")
    n_one = one.numel()
    del q, out_p, out_l, one
    torch.cuda.empty_cache()
    b_alg = 12.0 * n_queries
    return {"workload": f"{len(start)} sorted intervals (lognormal(4, 2) gaps), {n_queries} queries "
                        "(70% Zipf(1.05) over intervals, 30% uniform)",
            "plain_ms": round(ms_plain, 2), "learned_ms": round(ms_learn, 2),
            "speedup_learned_vs_plain": round(ms_plain / ms_learn, 3), "identical_ids": identical,
            "plain_frac_hbm": round(b_alg / (ms_plain * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "learned_frac_hbm": round(b_alg / (ms_learn * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "root_flop_per_lookup": 2 * (2 * 64 + 64 * 64 + 64),
            "trained": {"probes_per_lookup": round(float(ct[0]) / n_one if n_one else 0, 3),
                        "fallbacks": int(ct[1]), "mean_window": round(st["mean_window"], 1),
                        "train_mse": st["train_mse"], "train_s": round(train_s, 2),
                        "ms_per_1e8": round(ms_t1, 2)},
            "untrained": {"probes_per_lookup": round(float(cu[0]) / n_one if n_one else 0, 3),
                          "fallbacks": int(cu[1]), "mean_window": round(st_untrained["mean_window"], 1),
                          "ms_per_1e8": round(ms_u, 2)},
            "setup_s": round(time.perf_counter() - t0, 1)}


def section_batched(hpa, ctx, n_groups):
    import numpy as np
    import torch
    from workloads import batched_sizes, batched_structures, GpuSampler
    sizes = batched_sizes()
    structs = batched_structures()
    maps = [hpa.build_structure_map_workload(ctx, w) for w in structs]
    samplers = [GpuSampler(w) for w in structs]
    P = len(sizes)
    sidx = np.arange(P) % len(structs)
    groups = np.array_split(np.arange(P), n_groups)
    t_seq = t_bat = 0.0
    tune_ms = 0.0
    info = None
    checked = 0
    for gi, g in enumerate(groups):
        n = int(sizes[g].sum())
        pc = torch.empty(n, dtype=torch.int64, device="cuda")
        cx = torch.empty(n, dtype=torch.int32, device="cuda")
        st = torch.empty(n, dtype=torch.uint8, device="cuda")
        off = [0]
        for p in g:
            a, b = off[-1], off[-1] + int(sizes[p])
            samplers[sidx[p]].draw(2109069313 * 7919 + int(p), int(sizes[p]), pc[a:b], cx[a:b], st[a:b])
            off.append(b)
        pcu, cxu = pc.view(torch.uint64), cx.view(torch.uint32)
        gm = [maps[sidx[p]] for p in g]
        gn = [int(sizes[p]) for p in g]
        gc = [structs[sidx[p]].meta["n_ctx"] for p in g]
        if gi == 0:  # the autotuner's pilot and the tuned parameters, kept in the context
            t0 = time.perf_counter()
            b0 = hpa.attribute_batched(ctx, gm, gn, gc, pcu, cxu, st, autotune=True)
            tune_ms = b0.info()["tune_ms"]
            del b0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, p in enumerate(g):
            a, b = off[i], off[i + 1]
            r = hpa.attribute(ctx, gm[i], pcu[a:b], cxu[a:b], st[a:b], None, gc[i])
            del r
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        t0 = time.perf_counter()
        bt = hpa.attribute_batched(ctx, gm, gn, gc, pcu, cxu, st, autotune=True)
        torch.cuda.synchronize()
        t_bat += time.perf_counter() - t0
        info = bt.info()
        for i in (0, len(g) // 2, len(g) - 1):  # identity on a few profiles of every group
            a, b = off[i], off[i + 1]
            one = hpa.attribute(ctx, gm[i], pcu[a:b], cxu[a:b], st[a:b], None, gc[i]).numpy()
            got = bt.profile(i).numpy()
            assert all(np.array_equal(got[f], one[f]) for f in one), f"batched profile {g[i]} differs"
            checked += 1
        del bt, pc, cx, st, pcu, cxu
        torch.cuda.empty_cache()
        log(f"batched group {gi}: {len(g)} profiles, {n} samples")
    N = int(sizes.sum())
    return {"workload": f"{P} profiles, sizes lognormal(13, 1.5) clipped to [1e4, 2e7] ({N} samples), "
                        f"{len(structs)} program structures of 1e3-5e4 functions, in {n_groups} groups",
            "sequential_s": round(t_seq, 3), "batched_s": round(t_bat, 3),
            "speedup_batched_vs_sequential": round(t_seq / t_bat, 3),
            "batched_samples_per_s": N / t_bat, "sequential_samples_per_s": N / t_seq,
            "autotuned": {"merge_rounds": info["merge_rounds"], "scan_wg_per_cu": info["scan_wg_per_cu"],
                          "tune_ms": round(tune_ms, 1)},
            "rounds_per_group": info["n_rounds"], "identity_checked_profiles": checked}


def section_serve(hpa, ctx, seconds):
    import numpy as np
    import torch
    from workloads import config1
    w = config1(n_samples=3_000_000)
    m = hpa.build_structure_map_workload(ctx, w)
    r = np.random.default_rng(2109069315)
    # a pool of buffers with log-uniform sizes in [4 KB, 16 MB]
    pool, lo = [], 0
    for k in range(48):
        nbytes = math.exp(r.uniform(math.log(4 << 10), math.log(16 << 20)))
        n = max(1, int(nbytes // 13))
        if lo + n > w.n_samples:
            lo = 0
        pool.append(hpa.sample_buffer(w.pc[lo:lo + n], w.ctx[lo:lo + n], w.stall[lo:lo + n]))
        lo += n
    sizes = np.array([b.n_samples * 13 for b in pool], dtype=np.float64)
    srv = hpa.Server(ctx, m, n_profiles=512, n_ctx=w.n_ctx, table_slots=1 << 22, n_slots=6,
                     max_batch_bytes=64 << 20, hbm_budget=200 * 10 ** 9)
    rows = []
    for rate_gbs in (1.0, 5.0, 20.0):
        lam = rate_gbs * 1e9 / sizes.mean()  # buffers per second
        srv.stats(reset=True)
        t_end = time.perf_counter() + seconds
        t_next = time.perf_counter()
        n_sub = 0
        while True:
            now = time.perf_counter()
            if now >= t_end:
                break
            if now < t_next:
                time.sleep(min(t_next - now, 0.0005))
                continue
            b = pool[int(r.integers(0, len(pool)))]
            srv.submit(int(r.integers(0, 512)), b)
            n_sub += 1
            t_next += r.exponential(1.0 / lam)
        srv.drain()
        st = srv.stats()
        rows.append({"offered_GBps": rate_gbs, "buffers": int(st["buffers"]), "p50_us": round(st["p50_us"], 1),
                     "p99_us": round(st["p99_us"], 1), "max_us": round(st["max_us"], 1),
                     "sustained_samples_per_s": st["samples"] / max(st["span_s"], 1e-9),
                     "sustained_GBps": st["bytes"] / max(st["span_s"], 1e-9) / 1e9,
                     "errors": int(st["errors"])})
        log(f"serve {rate_gbs} GB/s: {n_sub} buffers, p99 {st['p99_us']:.0f} us")
    srv.close()
    return {"workload": "512 streams on the tiny workload's structure, buffers 4 KB-16 MB log-uniform, "
                        f"Poisson arrivals, {seconds} s per offered rate, pinned host buffers",
            "rates": rows}


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
    import paper_2109_06931_amd as hpa
    from workloads import config2

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    skip = set() if not args.only_headline else set(SECTIONS)
    skip |= {s for s in args.skip.split(",") if s}
    log(f"generating the medium workload ({args.samples} samples)")
    w = config2(n_samples=args.samples, threads=16)
    ctx = hpa.Context(0)
    t0 = time.perf_counter()
    m = hpa.build_structure_map_workload(ctx, w)
    torch.cuda.synchronize()
    map_ms = (time.perf_counter() - t0) * 1e3
    pc, cx, st, wt = hpa.samples_to_device(w)
    torch.cuda.synchronize()
    N = w.n_samples

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
        del a
    # invariant check outside the timed region: every sample attributed once
    a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
    U = a.n_keys
    total = int(a.tensors()["count"].sum().item())
    assert total == (N if wt is None else int(w.weight.sum())), "attribution lost samples"
    del a

    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
        del a
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    value = N * args.steps / dt

    # stage times from separate calls with the stage timer on
    ctx.set_timing(True)
    for _ in range(3):
        a = hpa.attribute(ctx, m, pc, cx, st, wt, w.n_ctx)
        del a
    torch.cuda.synchronize()
    stages = ctx.timing()
    ctx.set_timing(False)

    M = m.n_intervals
    b_alg = 13.0 + 25.0 * U / N + 16.0 * M / N
    if "units_dense" in stages:
        # the dense pipeline's unit kernel reads each 4-byte record (and its
        # 4-byte weight) once and writes each key once (25 B)
        u = stages["units_dense"]
        calls = max(u.get("calls", 1), 1)
        per_rec = 8.0 if wt is not None else 4.0
        u_bytes = (per_rec * u.get("items_in", 0) + 25.0 * u.get("items_out", 0)) / calls
        kname = "k_d_units<%s>" % ("true" if wt is not None else "false")
    else:
        # the general pipeline's unit sort kernel (its launch over the units
        # read through the run list) reads its samples (13 B each)
        u = stages.get("units_plain", {})
        calls = max(u.get("calls", 1), 1)
        u_bytes = 13.0 * u.get("items_in", 0) / calls
        kname = "k_units32<false, false, false>"
    u_ms = u.get("ms", 0.0) / calls
    achieved = u_bytes / (u_ms * 1e-3) / 1e9 if u_ms > 0 else 0.0
    traffic = _units_traffic()
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": None if traffic is None else round(traffic),
                "launch_ms": round(u_ms, 3), "algorithmic_bytes": round(u_bytes)}
    del pc, cx, st, wt
    torch.cuda.empty_cache()
    copy_gbps = _copy_ceiling()
    pipe_gbps = value * b_alg / 1e9
    pipeline = {"B_alg_bytes_per_sample": round(b_alg, 3), "achieved": round(pipe_gbps, 1), "unit": "GB/s",
                "frac": round(pipe_gbps / HBM_PEAK_GBPS, 4), "copy_ceiling_GBps": round(copy_gbps, 1),
                "frac_of_copy_ceiling": round(pipe_gbps / copy_gbps, 4), "map_build_ms": round(map_ms, 1),
                "stages_ms": {k: round(v["ms"] / max(v["calls"], 1), 3) for k, v in stages.items()}}
    extra = {}
    for name in SECTIONS:
        if name in skip:
            continue
        log(f"section {name}")
        try:
            if name == "tiny":
                extra[name] = section_tiny(hpa, ctx)
            elif name == "cct":
                extra[name] = section_cct(hpa, ctx)
            elif name == "learned":
                extra[name] = section_learned(hpa, ctx, args.learned_queries)
            elif name == "batched":
                extra[name] = section_batched(hpa, ctx, args.batched_groups)
            elif name == "serve":
                extra[name] = section_serve(hpa, ctx, args.serve_seconds)
        except hpa.HpaError as e:  # a library error in a report section is reported, not fatal
            extra[name] = {"error": str(e)}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        log(f"oracle on {min(args.cpu_samples, N)} samples")
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
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
