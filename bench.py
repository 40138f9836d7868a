"""Benchmark: strided tensor contraction on one MI355X.

Default workload: the coupled-cluster particle-particle ladder
C[a,b,i,j] += sum_{e,f} W[a,b,e,f] T[e,f,i,j] at v=128, o=32 (M=1024 x
N=16384 x K=16384 in the kernel view, 5.50e11 flop), W stored in mode order
(e,a,f,b), FP64 (headline) and FP32, synthetic U[-1,1] data.

A step is one contraction call (famlies_execute on a cached plan: gather ->
MFMA -> scatter-update) with inputs resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15}
HBM_PEAK = 8.0e12


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_ladder(v, o, dtype, seed=2):
    import synth
    npdt = np.float64 if dtype == "f64" else np.float32
    p = synth.ladder(v, o, seed=seed, dtype=npdt)
    return p


def run_one(p, dtype, compute, steps, warmup, sample_check=2048):
    import torch
    import paper_2604_07311_amd as fm
    dev = torch.device("cuda:0")
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    comp = fm.FAMLIES_BF16X3 if compute == "bf16x3" else fm.FAMLIES_NATIVE
    h = fm.handle(0)
    t0 = time.time()
    plan = fm.famlies_plan_contract(h, code, comp, fm.make_desc(p.a.extents, p.a.strides, p.la),
                                    fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                    fm.make_desc(p.c.extents, p.c.strides, p.lc))
    plan_s = time.time() - t0
    info = fm.famlies_plan_get_info(plan)
    a = torch.from_numpy(p.abuf).to(dev)
    b = torch.from_numpy(p.bbuf).to(dev)
    c0 = torch.from_numpy(p.cbuf).to(dev)
    c = c0.clone()
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    es = a.element_size()

    def step():
        fm.famlies_execute(plan, p.alpha, a.data_ptr() + es * p.a.base, b.data_ptr() + es * p.b.base,
                           p.beta, c.data_ptr() + es * p.c.base, sh)

    # correctness of the timed configuration: one call from C0, sampled
    # entries checked against the oracle (CPU, FP64)
    step()
    torch.cuda.synchronize()
    got = c.cpu().numpy().astype(np.float64)
    check = sample_parity(p, got, dtype, compute, sample_check)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    per = [e0.elapsed_time(e1) for e0, e1 in evs]
    fm.famlies_plan_destroy(plan)
    del a, b, c, c0
    torch.cuda.empty_cache()
    return {"info": info, "ms_per_step": total_ms / steps, "launch_ms_avg": float(np.mean(per)),
            "launch_ms_min": float(np.min(per)), "plan_s": plan_s, "check": check}


def sample_parity(p, got, dtype, compute, n):
    """Oracle on n random C entries of the timed configuration."""
    import oracle
    rng = np.random.default_rng(1234)
    idx = np.stack([rng.integers(0, e, size=n) for e in p.c.extents], axis=1)
    a = (p.abuf.astype(np.float64), p.a.base, p.a.extents, p.a.strides)
    b = (p.bbuf.astype(np.float64), p.b.base, p.b.extents, p.b.strides)
    c = (p.cbuf.astype(np.float64), p.c.base, p.c.extents, p.c.strides)
    want, d = oracle.contract_entries(p.alpha, a, p.la, b, p.lb, p.beta, c, p.lc, idx,
                                      want_cond=True)
    offs = p.c.base + idx @ np.array(p.c.strides)
    g = got[offs]
    rel = float(np.linalg.norm(g - want) / np.linalg.norm(want))
    comp = float(np.max(np.abs(g - want) / np.maximum(d, 1e-300)))
    return {"samples": int(n), "normwise_rel_err": rel, "max_err_over_D": comp}


def cpu_baseline(p, target_s=12.0):
    """The oracle, untuned, on a bounded sample of the same workload: a set of
    randomly chosen C entries, each a full K-term dot product in FP64."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    K = 1
    for ch, e in zip(p.la, p.a.extents):
        if ch in p.lb:
            K *= e
    a = (p.abuf.astype(np.float64), p.a.base, p.a.extents, p.a.strides)
    b = (p.bbuf.astype(np.float64), p.b.base, p.b.extents, p.b.strides)
    c = (p.cbuf.astype(np.float64), p.c.base, p.c.extents, p.c.strides)
    rng = np.random.default_rng(99)

    def timed(n):
        idx = np.stack([rng.integers(0, e, size=n) for e in p.c.extents], axis=1)
        t0 = time.perf_counter()
        oracle.contract_entries(p.alpha, a, p.la, b, p.lb, p.beta, c, p.lc, idx, nthreads=cores)
        return time.perf_counter() - t0

    n0 = 256 * cores
    t0 = timed(n0)
    n = int(max(n0, min(n0 * target_s / max(t0, 1e-3), 5e7)))
    t = timed(n)
    flops = 2.0 * K * n
    return {"value": flops / t / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "%d random C entries of the ladder (each a %d-term FP64 dot product), "
                      "%.1f s" % (n, K, t)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--v", type=int, default=128)
    ap.add_argument("--o", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["f64", "f32"], default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design for sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    log("device %s" % torch.cuda.get_device_name(0))
    results = {}
    problems = {}
    for dtype in (["f64", "f32"] if args.only is None else [args.only]):
        log("generating ladder v=%d o=%d %s" % (args.v, args.o, dtype))
        p = make_ladder(args.v, args.o, dtype)
        problems[dtype] = p
        log("running %s: %d warmup + %d timed steps" % (dtype, args.warmup, args.steps))
        results[dtype] = run_one(p, dtype, "native", args.steps, args.warmup)
        r = results[dtype]
        log("%s: %.3f ms/step, %.1f GFLOP/s, check %s" % (
            dtype, r["ms_per_step"], r["info"]["flops"] / r["ms_per_step"] / 1e6, r["check"]))
    head = "f64" if "f64" in results else list(results)[0]
    r = results[head]
    flops = r["info"]["flops"]
    value = flops / (r["ms_per_step"] * 1e-3) / 1e9
    achieved = flops / (r["launch_ms_avg"] * 1e-3) / 1e12
    out = {
        "metric": "contraction GFLOP/s & % MFMA peak (FP64/FP32/bf16x3) at stated err vs FP64",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "ccsd_ladder_v%d_o%d" % (args.v, args.o),
                   "contraction": "C[a,b,i,j] += sum_ef W[a,b,e,f] T[e,f,i,j], W stored (e,a,f,b)",
                   "m": r["info"]["m"], "n": r["info"]["n"], "k": r["info"]["k"],
                   "tile": [r["info"]["tile_m"], r["info"]["tile_n"], r["info"]["tile_k"]],
                   "split_k": r["info"]["split_k"], "parallelism": "single GPU"},
        "pct_mfma_peak": round(100.0 * value * 1e9 / PEAK[head], 2),
        "error_vs_fp64": r["check"],
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[head] / 1e12,
                     "unit": "TFLOP/s", "frac": round(achieved * 1e12 / PEAK[head], 4),
                     "traffic": None},
    }
    if len(results) > 1:
        out["secondary"] = {}
        for dt, rr in results.items():
            if dt == head:
                continue
            v = rr["info"]["flops"] / (rr["ms_per_step"] * 1e-3) / 1e9
            out["secondary"][dt] = {"value": round(v, 2), "unit": "GFLOP/s",
                                    "ms_per_step": round(rr["ms_per_step"], 4),
                                    "pct_mfma_peak": round(100.0 * v * 1e9 / PEAK[dt], 2),
                                    "error_vs_fp64": rr["check"]}
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(problems[head])
        out["cpu_baseline"]["cpu_model"] = cpu_model()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
