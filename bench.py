"""Benchmark: strided tensor contraction on one MI355X.

Workloads (synthetic, seeded):
  ladder    (default) C[a,b,i,j] += sum_{e,f} W[a,b,e,f] T[e,f,i,j], v=128, o=32,
            W stored in mode order (e,a,f,b); FP64 headline, FP32 secondary.
  ladder3   the same ladder at v=192, o=48 with outliers: bf16x3 against FP32,
            bf16x6 and FP64 on the same data.
  ring      C[a,i,b,j] = sum_{k,c} X[a,k,i,c] Y[c,b,k,j], o=48, v=192: the same
            four precisions.
  batched   20,000 random 4-index FP32 contractions, one persistent launch
            replayed from a HIP graph.
  autograd  forward + backward (dA, dB) of C[a,b,i,j] = sum A[a,e,i,f] B[e,b,f,j],
            o=24, v=96, FP32.
  plain16   C[a,b,i,j] = sum A[a,e,i,f] B[e,b,f,j], all extents 16, FP64: latency,
            single call and 1,000 calls replayed from a graph.

A step is one pass of the workload's contraction(s) with inputs resident in
HBM.  Prints one JSON line.
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

PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "int8": 5.0e15}
METRIC = "contraction GFLOP/s & % MFMA peak (FP64/FP32/bf16x3) at stated err vs FP64"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cores_used():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Timer:
    """HIP events on the stream the kernels are launched on."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream

    def run(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(self.stream)
        for e0, e1 in evs:
            e0.record(self.stream)
            fn()
            e1.record(self.stream)
        end.record(self.stream)
        torch.cuda.synchronize()
        per = [e0.elapsed_time(e1) for e0, e1 in evs]
        return start.elapsed_time(end) / steps, float(np.mean(per)), float(np.min(per))


# ------------------------------------------------------------ single problems
class Single:
    """One labelled contraction planned once and executed through the C ABI."""

    def __init__(self, p, dtype, compute="native"):
        import torch
        import paper_2604_07311_amd as fm
        self.p, self.dtype, self.compute = p, dtype, compute
        self.fm, self.torch = fm, torch
        code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
        comp = fm._compute_code(compute)
        t0 = time.perf_counter()
        self.plan = fm.famlies_plan_contract(fm.handle(0), code, comp,
                                             fm.make_desc(p.a.extents, p.a.strides, p.la),
                                             fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                             fm.make_desc(p.c.extents, p.c.strides, p.lc))
        self.plan_s = time.perf_counter() - t0
        self.info = fm.famlies_plan_get_info(self.plan)
        npdt = np.float64 if dtype == "f64" else np.float32
        dev = torch.device("cuda:0")
        self.a = torch.from_numpy(np.ascontiguousarray(p.abuf, dtype=npdt)).to(dev)
        self.b = torch.from_numpy(np.ascontiguousarray(p.bbuf, dtype=npdt)).to(dev)
        self.c0 = torch.from_numpy(np.ascontiguousarray(p.cbuf, dtype=npdt)).to(dev)
        self.c = self.c0.clone()
        self.stream = torch.cuda.current_stream(dev)
        es = self.a.element_size()
        self.ptrs = (self.a.data_ptr() + es * p.a.base, self.b.data_ptr() + es * p.b.base,
                     self.c.data_ptr() + es * p.c.base)

    def step(self):
        self.fm.famlies_execute(self.plan, self.p.alpha, self.ptrs[0], self.ptrs[1], self.p.beta,
                                self.ptrs[2], self.stream.cuda_stream)

    def packed(self, mask, steps, warmup):
        """Pack the operands in `mask` (bit 0: A, bit 1: B) once, then time
        famlies_execute_packed.  Returns (pack ms, ms per step, check input)."""
        torch, fm = self.torch, self.fm
        bufs, ptrs = {}, list(self.ptrs[:2])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(self.stream)
        for op in (0, 1):
            if mask & (1 << op):
                n = fm.famlies_pack_size(self.plan, op)
                bufs[op] = torch.empty(n // 4 + 4, dtype=torch.int32, device=self.c.device)
                fm.famlies_pack(self.plan, op, self.ptrs[op], bufs[op].data_ptr(), self.stream.cuda_stream)
                ptrs[op] = bufs[op].data_ptr()
        e1.record(self.stream)
        torch.cuda.synchronize()
        pack_ms = e0.elapsed_time(e1)

        def step():
            fm.famlies_execute_packed(self.plan, self.p.alpha, ptrs[0], ptrs[1], self.p.beta,
                                      self.ptrs[2], mask, self.stream.cuda_stream)

        self.c.copy_(self.c0)
        step()
        torch.cuda.synchronize()
        got = self.c.cpu().numpy().astype(np.float64)
        ms, launch, _ = Timer(self.stream).run(step, steps, warmup)
        del bufs
        return pack_ms, ms, launch, got

    def torch_permute_matmul(self, steps, warmup):
        """Context only: the route the method avoids.  The operands are
        permuted into GEMM order and copied (permute().contiguous()), multiplied
        with torch.matmul, and the product is scattered back into C's layout
        with beta*C added.  Returns (ms for the whole route, ms for the matmul
        alone, normwise difference from this library's C)."""
        torch, p = self.torch, self.p
        la, lb, lc = p.la, p.lb, p.lc
        I = [ch for ch in lc if ch in la]
        J = [ch for ch in lc if ch in lb]
        P = [ch for ch in la if ch in lb]
        ext = dict(zip(la + lb, list(p.a.extents) + list(p.b.extents)))
        M = int(np.prod([ext[ch] for ch in I])) if I else 1
        N = int(np.prod([ext[ch] for ch in J])) if J else 1
        K = int(np.prod([ext[ch] for ch in P])) if P else 1
        A = self.a.as_strided(p.a.extents, p.a.strides, p.a.base)
        B = self.b.as_strided(p.b.extents, p.b.strides, p.b.base)
        Cv = self.c.as_strided(p.c.extents, p.c.strides, p.c.base)
        pa = [la.index(ch) for ch in I + P]
        pb = [lb.index(ch) for ch in P + J]
        # product laid out (I..., J...) -> permutation into C's label order
        pc = [(I + J).index(ch) for ch in lc]
        alpha, beta = p.alpha, p.beta

        def route():
            Xm = A.permute(pa).contiguous().reshape(M, K)
            Ym = B.permute(pb).contiguous().reshape(K, N)
            prod = torch.matmul(Xm, Ym).reshape([ext[ch] for ch in I + J]).permute(pc)
            Cv.copy_(alpha * prod + beta * Cv)

        Xm = A.permute(pa).contiguous().reshape(M, K)
        Ym = B.permute(pb).contiguous().reshape(K, N)
        ms_gemm, _, _ = Timer(self.stream).run(lambda: torch.matmul(Xm, Ym), steps, warmup)
        del Xm, Ym
        mine = self.result_once()
        self.c.copy_(self.c0)
        route()
        torch.cuda.synchronize()
        theirs = self.c.cpu().numpy().astype(np.float64)
        diff = float(np.linalg.norm(theirs - mine) / max(np.linalg.norm(mine), 1e-300))
        ms_route, _, _ = Timer(self.stream).run(route, steps, warmup)
        self.c.copy_(self.c0)
        torch.cuda.empty_cache()
        return ms_route, ms_gemm, diff

    def result_once(self):
        """C after one call from C0 (float64 numpy storage)."""
        self.c.copy_(self.c0)
        self.step()
        self.torch.cuda.synchronize()
        return self.c.cpu().numpy().astype(np.float64)

    def close(self):
        self.fm.famlies_plan_destroy(self.plan)
        del self.a, self.b, self.c, self.c0
        self.torch.cuda.empty_cache()


def rounded(buf, dtype):
    return buf.astype(np.float32).astype(np.float64) if dtype != "f64" else buf.astype(np.float64)


def sample_check(p, got, dtype, n=2048, split=False, seed=1234):
    """Oracle (FP64) on n random C entries; returns error statistics."""
    import oracle
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, e, size=n) for e in p.c.extents], axis=1)
    a = (rounded(p.abuf, dtype), p.a.base, p.a.extents, p.a.strides)
    b = (rounded(p.bbuf, dtype), p.b.base, p.b.extents, p.b.strides)
    c = (rounded(p.cbuf, dtype), p.c.base, p.c.extents, p.c.strides)
    want, d = oracle.contract_entries(p.alpha, a, p.la, b, p.lb, p.beta, c, p.lc, idx,
                                      want_cond=True)
    offs = p.c.base + idx @ np.array(p.c.strides, dtype=np.int64)
    g = got[offs]
    return {"samples": int(n), "normwise_rel_err": float(np.linalg.norm(g - want) / np.linalg.norm(want)),
            "max_abs_err_over_D": float(np.max(np.abs(g - want) / np.maximum(d, 1e-300)))}


def cpu_baseline(p, target_s=12.0):
    """The oracle as it stands, on a bounded sample of the same workload:
    randomly chosen C entries, each a full K-term FP64 dot product, on all the
    host cores this process may use."""
    import oracle
    cores = cores_used()
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

    n0 = 64 * cores
    t0 = timed(n0)
    n = int(max(n0, min(n0 * target_s / max(t0, 1e-3), 5e7)))
    t = timed(n)
    return {"value": round(2.0 * K * n / t / 1e9, 3), "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d random C entries of %s, each a %d-term FP64 dot product (%.1f s)"
                      % (n, p.name, K, t)}


# HBM bytes per launch of a workload's dominant kernel, from two rocprofv3
# --pmc runs (FETCH_SIZE, then WRITE_SIZE: KiB per dispatch), each scaled by
# the ratio the same counter shows for a plain device copy of 1 GiB taken in
# the same run.  A record holds only for the kernel it was measured on: the
# plain kernel's own sources (`sources` = kernel_sources_sha() then) and the
# plan's launch shape (`plan` = plan_signature() then).  After a change to
# either the traffic is reported as null until the counters are taken again.
TRAFFIC = {
    # plain_contract<double,u32,128,128,8,3,3>, ladder v=128 o=32
    ("ladder", "f64", 128, 32): {"fetch_kib": 3.06707e6, "write_kib": 131072.0, "fetch_scale": 1.99989,
                                 "write_scale": 1.0, "sources": "89c222de133bcc5c",
                                 "plan": "128x128x8 split1/0 kernel49 bits32",
                                 "profile": "profiles/plain_contract_ladder_v128_o32_fetch_size.md, "
                                            "profiles/plain_contract_ladder_v128_o32_write_size.md"},
    # plain_contract<float,u32,128,128,32,3,3>, ladder v=128 o=32
    ("ladder", "f32", 128, 32): {"fetch_kib": 2.81782e6, "write_kib": 65536.0, "fetch_scale": 1.99989,
                                 "write_scale": 1.0, "sources": "89c222de133bcc5c",
                                 "plan": "128x128x32 split1/0 kernel49 bits32",
                                 "profile": "profiles/plain_contract_ladder_v128_o32_fetch_size.md, "
                                            "profiles/plain_contract_ladder_v128_o32_write_size.md"},
}


# Sources of the plain contraction kernels themselves; the planner enters a
# record through the plan's launch shape instead.
PLAIN_SOURCES = ("args.hpp", "device.hpp", "launch.hpp", "plain_kernels.hip", "tile.hpp")


def kernel_sources_sha():
    import hashlib
    d = os.path.join(ROOT, "paper_2604_07311_amd", "csrc")
    h = hashlib.sha256()
    for name in PLAIN_SOURCES:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def plan_signature(info):
    """The launch shape a traffic record depends on."""
    return "%dx%dx%d split%d/%d kernel%d bits%d" % (info["tile_m"], info["tile_n"], info["tile_k"],
                                                   info["split_k"], info["split_tiles"], info["kernel"],
                                                   info["index_bits"])


def traffic(key, info):
    rec = TRAFFIC.get(key)
    if rec is None or rec["sources"] != kernel_sources_sha() or rec["plan"] != plan_signature(info):
        return None
    return int(round(1024 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])))


def roofline(flops, launch_ms, peak, bound="mfma", key=None, info=None):
    achieved = flops / (launch_ms * 1e-3) / 1e12
    return {"bound": bound, "achieved": round(achieved, 3), "peak": round(peak / 1e12, 1),
            "unit": "TFLOP/s", "frac": round(achieved * 1e12 / peak, 4),
            "traffic": traffic(key, info) if key else None}


def base_record(args, value, ms, dtype, config, unit="GFLOP/s"):
    return {"metric": METRIC, "value": round(value, 2), "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def wl_ladder(args):
    import synth
    res = {}
    probs = {}
    for dtype in (["f64", "f32"] if args.only is None else [args.only]):
        log("ladder v=%d o=%d %s: generating" % (args.v, args.o, dtype))
        p = synth.ladder(args.v, args.o, seed=2,
                         dtype=np.float64 if dtype == "f64" else np.float32)
        probs[dtype] = p
        s = Single(p, dtype)
        check = sample_check(p, s.result_once(), dtype)
        ms, launch, lmin = Timer(s.stream).run(s.step, args.steps, args.warmup)
        res[dtype] = {"ms": ms, "launch": launch, "info": s.info, "check": check, "plan_s": s.plan_s}
        log("%s: %.3f ms/step (%.1f GFLOP/s) check %s" % (dtype, ms, s.info["flops"] / ms / 1e6, check))
        if args.context:
            rms, gms, diff = s.torch_permute_matmul(max(3, args.steps // 2), 1)
            res[dtype]["context_torch"] = {
                "permute_copy_matmul_scatter_ms": round(rms, 4), "matmul_only_ms": round(gms, 4),
                "gflops_route": round(s.info["flops"] / (rms * 1e-3) / 1e9, 2),
                "gflops_matmul_only": round(s.info["flops"] / (gms * 1e-3) / 1e9, 2),
                "normwise_diff_vs_this_library": diff}
            log("%s torch permute+matmul: %.3f ms (matmul alone %.3f ms)" % (dtype, rms, gms))
        if args.pack:
            # W (operand A) pre-packed once, as a CC code reusing it across iterations would
            pack_ms, pms, plaunch, got = s.packed(1, args.steps, args.warmup)
            res[dtype]["packed_W"] = {"pack_ms_once": round(pack_ms, 3), "ms_per_step": round(pms, 4),
                                      "value": round(s.info["flops"] / (pms * 1e-3) / 1e9, 2),
                                      "pct_mfma_peak": round(100 * s.info["flops"] / (pms * 1e-3) / PEAK[dtype], 2),
                                      "error_vs_fp64": sample_check(p, got, dtype, n=512)}
            log("%s packed W: pack %.2f ms once, %.3f ms/step" % (dtype, pack_ms, pms))
        s.close()
    head = "f64" if "f64" in res else list(res)[0]
    r = res[head]
    flops = r["info"]["flops"]
    out = base_record(args, flops / (r["ms"] * 1e-3) / 1e9, r["ms"], head,
                      {"workload": "ccsd_ladder_v%d_o%d" % (args.v, args.o),
                       "contraction": "C[a,b,i,j] += sum_ef W[a,b,e,f] T[e,f,i,j]; W stored (e,a,f,b)",
                       "m": r["info"]["m"], "n": r["info"]["n"], "k": r["info"]["k"],
                       "tile": [r["info"]["tile_m"], r["info"]["tile_n"], r["info"]["tile_k"]],
                       "split_k": r["info"]["split_k"]})
    out["pct_mfma_peak"] = round(100 * flops / (r["ms"] * 1e-3) / PEAK[head], 2)
    out["error_vs_fp64"] = r["check"]
    out["roofline"] = roofline(flops, r["launch"], PEAK[head], key=("ladder", head, args.v, args.o),
                               info=r["info"])
    if "packed_W" in r:
        out["packed_W"] = r["packed_W"]
    if "context_torch" in r:
        out["context_torch"] = r["context_torch"]
    for dt, rr in res.items():
        if dt == head:
            continue
        v = rr["info"]["flops"] / (rr["ms"] * 1e-3)
        out.setdefault("secondary", {})[dt] = {
            "value": round(v / 1e9, 2), "unit": "GFLOP/s", "ms_per_step": round(rr["ms"], 4),
            "pct_mfma_peak": round(100 * v / PEAK[dt], 2), "error_vs_fp64": rr["check"],
            "roofline": roofline(rr["info"]["flops"], rr["launch"], PEAK[dt], key=("ladder", dt, args.v, args.o),
                                 info=rr["info"])}
        if "packed_W" in rr:
            out["secondary"][dt]["packed_W"] = rr["packed_W"]
        if "context_torch" in rr:
            out["secondary"][dt]["context_torch"] = rr["context_torch"]
    if "f64" in probs and not args.no_int8:
        out.setdefault("secondary", {})["f64_on_int8"] = int8_emulation(args, probs["f64"], r["ms"])
    if not args.no_ring:
        out.setdefault("secondary", {})["ring_o48_v192"] = ring_precisions(args)
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(probs[head])
    return out


def int8_emulation(args, p, native_ms):
    """The same FP64 ladder with FP64 emulated on INT8 MFMA, six and seven
    digit slices (21 and 28 INT8 products per FP64 product): FP64-equivalent
    GFLOP/s (2MNK/t) for the whole call (slicing both operands, then the INT8
    GEMM), error against the FP64 oracle, speed-up over the native FP64
    kernel, and a roofline against the INT8 MFMA peak on the INT8 operations
    issued (products * 2MNK) over the whole call."""
    out = {}
    for slices in (6, 7):
        s = Single(p, "f64", "int8x%d" % slices)
        check = sample_check(p, s.result_once(), "f64")
        ms, launch, _ = Timer(s.stream).run(s.step, args.steps, args.warmup)
        flops = s.info["flops"]
        prods = slices * (slices + 1) // 2
        log("ladder f64 on int8x%d: %.3f ms (%.1f GFLOP/s) check %s" % (slices, ms, flops / ms / 1e6, check))
        s.close()
        out["int8x%d" % slices] = {
            "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s (FP64-equivalent, 2MNK/t)",
            "ms_per_step": round(ms, 4), "slices": slices, "int8_products_per_fp64_product": prods,
            "speedup_vs_native_fp64": round(native_ms / ms, 3), "error_vs_fp64": check,
            "pct_fp64_mfma_peak_equivalent": round(100 * flops / (ms * 1e-3) / PEAK["f64"], 2),
            "roofline": roofline(prods * flops, launch, PEAK["int8"])}
    return out


def ring_precisions(args):
    """The split-BF16 precision path beside plain FP32 and FP64 on one
    workload: the ring C[a,i,b,j] = sum_{k,c} X[a,k,i,c] Y[c,b,k,j], o=48,
    v=192, FP32 inputs N(0,1) with Bernoulli(1e-3) x 1e4 outliers.  Each
    precision: FP32-equivalent GFLOP/s (2MNK/t), error against the FP64
    oracle on sampled entries, speed-up over FP32, and a roofline against
    its own MFMA peak on the flops it issues (bf16x3: 3 * 2MNK, bf16x6:
    6 * 2MNK on BF16 MFMA)."""
    import synth
    log("ring o=48 v=192 with outliers: generating")
    p = synth.ring(48, 192, seed=4, dist="outliers", dtype=np.float32)
    res = {}
    for dtype, comp, issued, peak in (("f32", "native", 1, "f32"), ("f32", "bf16x3", 3, "bf16"),
                                      ("f32", "bf16x6", 6, "bf16"), ("f64", "native", 1, "f64")):
        s = Single(p, dtype, comp)
        check = sample_check(p, s.result_once(), dtype, n=1024)
        ms, launch, _ = Timer(s.stream).run(s.step, args.steps, args.warmup)
        flops = s.info["flops"]
        name = "fp64" if dtype == "f64" else ("fp32" if comp == "native" else comp)
        res[name] = {"value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s (2MNK/t)",
                     "ms_per_step": round(ms, 4), "error_vs_fp64": check,
                     "tile": [s.info["tile_m"], s.info["tile_n"], s.info["tile_k"]],
                     "split_k": s.info["split_k"], "kernel": s.info["kernel"],
                     "roofline": roofline(issued * flops, launch, PEAK[peak])}
        log("ring %s %s: %.3f ms (%.1f GFLOP/s) check %s" % (dtype, comp, ms, flops / ms / 1e6, check))
        s.close()
    for name in ("bf16x3", "bf16x6", "fp64"):
        res[name]["speedup_vs_fp32"] = round(res["fp32"]["ms_per_step"] / res[name]["ms_per_step"], 3)
    res["workload"] = "ccsd_ring_o48_v192_outliers"
    return res


def _fp32_vs_bf16x3(args, p, name):
    res = {}
    for comp in ("native", "bf16x3", "bf16x6"):
        s = Single(p, "f32", comp)
        check = sample_check(p, s.result_once(), "f32", n=1024)
        ms, launch, _ = Timer(s.stream).run(s.step, args.steps, args.warmup)
        res[comp] = {"ms": ms, "launch": launch, "info": s.info, "check": check}
        log("%s %s: %.3f ms (%.1f GFLOP/s) check %s" % (name, comp, ms, s.info["flops"] / ms / 1e6, check))
        if args.pack and comp == "bf16x3" and s.info["index_bits"] == 64:
            res[comp]["packed"] = {"skipped": "operands span more than 4 GiB: 64-bit offsets, no packed kernel"}
        elif args.pack and comp == "bf16x3":
            pack_ms, pms, plaunch, got = s.packed(3, args.steps, args.warmup)
            res[comp]["packed"] = {"pack_ms_once": round(pack_ms, 3), "ms_per_step": round(pms, 4),
                                   "gflops_fp32_equivalent": round(s.info["flops"] / (pms * 1e-3) / 1e9, 2),
                                   "error_vs_fp64": sample_check(p, got, "f32", n=512)}
            log("%s bf16x3 packed A and B: pack %.2f ms once, %.3f ms/step" % (name, pack_ms, pms))
        s.close()
    # the same data in FP64 (the FP32 values, exact in FP64) on the FP64 kernel
    s = Single(p, "f64", "native")
    check = sample_check(p, s.result_once(), "f64", n=1024)
    ms, launch, _ = Timer(s.stream).run(s.step, args.steps, args.warmup)
    res["f64"] = {"ms": ms, "launch": launch, "info": s.info, "check": check}
    log("%s f64: %.3f ms (%.1f GFLOP/s) check %s" % (name, ms, s.info["flops"] / ms / 1e6, check))
    s.close()
    r3, r32 = res["bf16x3"], res["native"]
    flops = r3["info"]["flops"]
    out = base_record(args, flops / (r3["ms"] * 1e-3) / 1e9, r3["ms"], "bf16x3",
                      {"workload": name, "m": r3["info"]["m"], "n": r3["info"]["n"],
                       "k": r3["info"]["k"]})
    out["gflops_fp32_equivalent"] = round(flops / (r3["ms"] * 1e-3) / 1e9, 2)
    out["pct_fp32_mfma_peak"] = round(100 * flops / (r3["ms"] * 1e-3) / PEAK["f32"], 2)
    out["issued_bf16_tflops"] = round(3 * flops / (r3["ms"] * 1e-3) / 1e12, 2)
    out["error_vs_fp64"] = r3["check"]
    out["fp32"] = {"ms_per_step": round(r32["ms"], 4),
                   "value": round(flops / (r32["ms"] * 1e-3) / 1e9, 2),
                   "pct_mfma_peak": round(100 * flops / (r32["ms"] * 1e-3) / PEAK["f32"], 2),
                   "error_vs_fp64": r32["check"]}
    out["speedup_vs_fp32"] = round(r32["ms"] / r3["ms"], 3)
    if "packed" in r3:
        out["packed_operands"] = r3["packed"]
    r6 = res["bf16x6"]
    out["bf16x6"] = {"ms_per_step": round(r6["ms"], 4),
                     "value": round(flops / (r6["ms"] * 1e-3) / 1e9, 2),
                     "speedup_vs_fp32": round(r32["ms"] / r6["ms"], 3),
                     "error_vs_fp64": r6["check"]}
    r64 = res["f64"]
    out["fp64"] = {"ms_per_step": round(r64["ms"], 4),
                   "value": round(flops / (r64["ms"] * 1e-3) / 1e9, 2),
                   "pct_mfma_peak": round(100 * flops / (r64["ms"] * 1e-3) / PEAK["f64"], 2),
                   "error_vs_fp64": r64["check"]}
    out["bf16x3_speedup_vs_fp64"] = round(r64["ms"] / r3["ms"], 3)
    out["roofline"] = roofline(3 * flops, r3["launch"], PEAK["bf16"])
    return out


def wl_ladder3(args):
    import synth
    log("ladder v=192 o=48 with outliers (FP32): generating")
    p = synth.ladder(192, 48, seed=3, dist="outliers", dtype=np.float32)
    return _fp32_vs_bf16x3(args, p, "ccsd_ladder_v192_o48_outliers")


def wl_ring(args):
    import synth
    log("ring o=48 v=192 with outliers (FP32): generating")
    p = synth.ring(48, 192, seed=4, dist="outliers", dtype=np.float32)
    return _fp32_vs_bf16x3(args, p, "ccsd_ring_o48_v192_outliers")


def wl_plain16(args):
    import torch
    import synth
    p = synth.plain16(seed=1)
    s = Single(p, "f64")
    check = sample_check(p, s.result_once(), "f64", n=4096)
    ms, launch, lmin = Timer(s.stream).run(s.step, args.steps, args.warmup)
    # 1,000 calls replayed from one graph
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        s.stream = cs
        with torch.cuda.graph(g, stream=cs):
            for _ in range(1000):
                s.step()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    per_call_graph = e0.elapsed_time(e1) / 1000
    flops = s.info["flops"]
    out = base_record(args, flops / (ms * 1e-3) / 1e9, ms, "f64",
                      {"workload": "plain16", "m": 256, "n": 256, "k": 256,
                       "tile": [s.info["tile_m"], s.info["tile_n"], s.info["tile_k"]],
                       "split_k": s.info["split_k"]})
    out["latency_us_single_call"] = round(ms * 1e3, 2)
    out["latency_us_per_call_in_graph"] = round(per_call_graph * 1e3, 2)
    out["gflops_in_graph"] = round(flops / (per_call_graph * 1e-3) / 1e9, 2)
    out["error_vs_fp64"] = check
    out["roofline"] = roofline(flops, launch, PEAK["f64"])
    del g
    out["batched_4096_instances"] = _plain16_batched(s, 4096, args)
    s.close()
    return out


def _plain16_batched(s, n, args):
    """The same 16^4 problem, n independent instances (read-only operands
    shared, outputs disjoint) in one persistent batched launch from a graph:
    what the shape reaches when the GPU is full."""
    import torch
    fm, p = s.fm, s.p
    desc = lambda lay, lab: fm.make_desc(lay.extents, lay.strides, lab)
    plan = fm.famlies_batch_plan(fm.handle(0), fm.FAMLIES_F64, [desc(p.a, p.la)] * n,
                                 [desc(p.b, p.lb)] * n, [desc(p.c, p.lc)] * n)
    C = s.c0.repeat(n)
    csz = s.c0.numel()
    pa = torch.full((n,), s.ptrs[0], dtype=torch.int64, device="cuda")
    pb = torch.full((n,), s.ptrs[1], dtype=torch.int64, device="cuda")
    pc = torch.tensor([C.data_ptr() + 8 * (i * csz + p.c.base) for i in range(n)], dtype=torch.int64,
                      device="cuda")
    stream = torch.cuda.Stream()

    def launch():
        fm.famlies_batch_execute(plan, p.alpha, p.beta, pa.data_ptr(), pb.data_ptr(), pc.data_ptr(),
                                 stream.cuda_stream)

    with torch.cuda.stream(stream):
        launch()
    torch.cuda.synchronize()
    one = s.result_once()
    got = C.reshape(n, csz)[[0, n // 2, n - 1]].cpu().numpy()
    # the batched tiles sum K in another order than the split-K single call
    diff = max(float(np.linalg.norm(g - one) / np.linalg.norm(one)) for g in got)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            launch()
    torch.cuda.synchronize()
    ms, _, _ = Timer(torch.cuda.current_stream()).run(g.replay, max(args.steps, 5), args.warmup)
    flops = n * s.info["flops"]
    fm.famlies_plan_destroy(plan)
    del g
    return {"instances": n, "ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 2),
            "pct_fp64_peak": round(100 * flops / (ms * 1e-3) / PEAK["f64"], 2),
            "normwise_diff_vs_single_call": diff}


def wl_autograd(args):
    import torch
    import paper_2604_07311_amd as fm
    import synth
    o, v = 24, 96
    p = synth.autograd_case(o, v, seed=6)
    A = torch.from_numpy(p.abuf.astype(np.float32)).cuda().as_strided((v, v, o, v), p.a.strides)
    B = torch.from_numpy(p.bbuf.astype(np.float32)).cuda().as_strided((v, v, v, o), p.b.strides)
    G = torch.from_numpy(p.meta["G"].astype(np.float32)).cuda().as_strided((v, v, o, o), p.c.strides)
    A.requires_grad_()
    B.requires_grad_()

    def step():
        A.grad = None
        B.grad = None
        C = fm.contract_ad(1.0, A, "aeif", B, "ebfj", 0.0, None, "abij")
        C.backward(G)

    step()
    torch.cuda.synchronize()
    ms, launch, _ = Timer(torch.cuda.current_stream()).run(step, args.steps, args.warmup)
    # forward: M = a*i = v*o, N = b*j = v*o, K = e*f = v*v; dA and dB have the same volume
    flops = 3 * 2.0 * (v * o) * (v * o) * (v * v)
    out = base_record(args, flops / (ms * 1e-3) / 1e9, ms, "f32",
                      {"workload": "autograd_o24_v96", "contractions_per_step": 3,
                       "m": v * o, "n": v * o, "k": v * v})
    out["pct_mfma_peak"] = round(100 * flops / (ms * 1e-3) / PEAK["f32"], 2)
    out["roofline"] = roofline(flops, launch, PEAK["f32"])
    return out


def wl_batched(args):
    import torch
    import paper_2604_07311_amd as fm
    import oracle
    import synth
    n = args.batch
    table = None
    if args.tile_table != "none":
        table = args.tile_table or os.path.join(os.path.dirname(fm.__file__), "tables", "batch_mi355x.txt")
        fm.famlies_load_tune_table(fm.handle(0), table)
        log("batched: tile classes from %s" % table)
    log("batched: planning %d problems" % n)
    probs = synth.batched(n, seed=5)
    # read-only operands alias into one shared pool; outputs are disjoint
    pool_n = max(max(p.a.size for p in probs), max(p.b.size for p in probs)) * 8
    gen = torch.Generator(device="cuda").manual_seed(5)
    pool = torch.rand(pool_n, generator=gen, device="cuda", dtype=torch.float32) * 2 - 1
    rng = np.random.default_rng(55)
    aoff = [int(rng.integers(0, pool_n - p.a.size + 1)) for p in probs]
    boff = [int(rng.integers(0, pool_n - p.b.size + 1)) for p in probs]
    coff = np.concatenate([[0], np.cumsum([p.c.size for p in probs])]).astype(np.int64)
    C0 = torch.rand(int(coff[-1]), generator=gen, device="cuda", dtype=torch.float32) * 2 - 1
    C = C0.clone()
    pa = torch.tensor([pool.data_ptr() + 4 * (aoff[i] + p.a.base) for i, p in enumerate(probs)],
                      dtype=torch.int64, device="cuda")
    pb = torch.tensor([pool.data_ptr() + 4 * (boff[i] + p.b.base) for i, p in enumerate(probs)],
                      dtype=torch.int64, device="cuda")
    pc = torch.tensor([C.data_ptr() + 4 * (int(coff[i]) + p.c.base) for i, p in enumerate(probs)],
                      dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    plan = fm.famlies_batch_plan(fm.handle(0), fm.FAMLIES_F32,
                                 [fm.make_desc(p.a.extents, p.a.strides, p.la) for p in probs],
                                 [fm.make_desc(p.b.extents, p.b.strides, p.lb) for p in probs],
                                 [fm.make_desc(p.c.extents, p.c.strides, p.lc) for p in probs])
    plan_s = time.perf_counter() - t0
    tiles = fm.famlies_batch_plan_tiles(plan, n)
    flops = sum(2.0 * np.prod(synth.sizes(p)) for p in probs)
    stream = torch.cuda.Stream()

    def launch(s):
        fm.famlies_batch_execute(plan, 1.0, 0.5, pa.data_ptr(), pb.data_ptr(), pc.data_ptr(),
                                 s.cuda_stream)

    # eager run from C0, then check sampled problems fully against the oracle
    with torch.cuda.stream(stream):
        launch(stream)
    torch.cuda.synchronize()
    pool_h = pool.cpu().numpy().astype(np.float64)
    C_h = C.cpu().numpy().astype(np.float64)
    C0_h = C0.cpu().numpy().astype(np.float64)
    worst = 0.0
    checked = 0
    for i in rng.choice(n, size=min(n, 24), replace=False):
        p = probs[i]
        a = (pool_h[aoff[i]:aoff[i] + p.a.size], p.a.base, p.a.extents, p.a.strides)
        b = (pool_h[boff[i]:boff[i] + p.b.size], p.b.base, p.b.extents, p.b.strides)
        c = (C0_h[coff[i]:coff[i + 1]], p.c.base, p.c.extents, p.c.strides)
        want, d = oracle.contract(1.0, a, p.la, b, p.lb, 0.5, c, p.lc, want_cond=True)
        got = C_h[coff[i]:coff[i + 1]]
        worst = max(worst, float(np.max(np.abs(got - want) / np.maximum(d, 1e-300))))
        checked += 1
    # graph capture of the single launch, replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            launch(stream)
    torch.cuda.synchronize()
    ms, launch_ms, _ = Timer(torch.cuda.current_stream()).run(g.replay, args.steps, args.warmup)
    out = base_record(args, flops / (ms * 1e-3) / 1e9, ms, "f32",
                      {"workload": "batched_%d_random_4index" % n, "problems": n,
                       "dims": "U{4..48}", "launch": "one persistent kernel, graph replay",
                       "tile_table": os.path.basename(table) if table else None})
    classes = {}
    for t in tiles:
        if t != (0, 0):
            classes["%dx%d" % t] = classes.get("%dx%d" % t, 0) + 1
    out["tile_classes"] = classes
    out["pct_mfma_peak"] = round(100 * flops / (ms * 1e-3) / PEAK["f32"], 2)
    out["plan_s"] = round(plan_s, 3)
    out["error_vs_fp64"] = {"problems_checked_fully": checked, "max_abs_err_over_D": worst}
    out["roofline"] = roofline(flops, launch_ms, PEAK["f32"])
    del g
    fm.famlies_plan_destroy(plan)
    return out


WORKLOADS = {"ladder": wl_ladder, "ladder3": wl_ladder3, "ring": wl_ring, "plain16": wl_plain16,
             "autograd": wl_autograd, "batched": wl_batched}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="ladder")
    ap.add_argument("--v", type=int, default=128)
    ap.add_argument("--o", type=int, default=32)
    ap.add_argument("--batch", type=int, default=20000)
    ap.add_argument("--only", choices=["f64", "f32"], default=None)
    ap.add_argument("--tile-table", default="",
                    help="batched: tile table to load (default: the package's measured MI355X table; "
                         "'none': the built-in rule)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-int8", action="store_true",
                    help="ladder: skip FP64 emulated on INT8 MFMA reported under 'secondary'")
    ap.add_argument("--no-ring", action="store_true",
                    help="ladder: skip the ring in FP32, bf16x3, bf16x6 and FP64 reported under 'secondary'")
    ap.add_argument("--pack", action="store_true",
                    help="also time the pre-packed path (ladder: W packed once; ring: both operands)")
    ap.add_argument("--context", action="store_true",
                    help="ladder: also time torch's permute().contiguous() + matmul route (context only)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain device copy of this many bytes (a known-size "
                         "reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run it "
              "with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    log("device %s, workload %s" % (torch.cuda.get_device_name(0), args.workload))
    if args.copy_bytes > 0:
        n = args.copy_bytes // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("reference copy: %d bytes read, %d bytes written" % (4 * n, 4 * n))
        del src, dst
    out = WORKLOADS[args.workload](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
