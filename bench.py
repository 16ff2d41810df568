"""Benchmark of the mixed-precision HODLR matrix-vector product on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2] [--only WORKLOAD]

A step is one full product Y = A_H X (contraction, reduction, expansion and
leaves) over one batch of right-hand sides, with the operator, X and Y
resident in HBM.  The headline workload is the 65536-point 2D
Gaussian-kernel operator (Morton order, leaf 256, depth 8, eps = 1e-6,
formats chosen by the adaptive rule from fp32/bf16/fp16) with one fp32
right-hand side.  Printed as one JSON line.

Timing protocol (cold cache, the headline):

* before every timed product a read sweep of a 2 GiB buffer (8x the 256 MB
  last-level cache) evicts the operator from every cache without leaving
  dirty lines; the sweep is outside the product's HIP event pair;
* W untimed warm-up steps, then K timed steps; ms_per_step is the mean of
  the K products' event times, value = B_alg / ms_per_step, where
  B_alg = 8 sum m_i^2 + sum_b (r_b + c_b) p_b s(f_b) + scaled columns
          + n nrhs (s_X + s_Y)
  (leaves, factor codes, scales, X read once, Y written once);
* the same products replayed back to back from a HIP graph (operator warm
  in the caches) are reported beside it as warm_cache_gbs.

roofline: the dominant kernel of the workload's path, its algorithmic bytes
(or, for the fp64 leaf GEMM above the fp64 ridge, its flops) over its mean
cold duration from HIP events the library records around each kernel on
its launch stream (hodlr_profile), against the published peak:

* nrhs = 1 (wave path): k_phase1, the contraction items plus the fp64 leaf
  tiles, 8 sum m_i^2 + sum_b c_b p_b s(f_b) + n nrhs s_X bytes;
* nrhs >= 8 (matrix cores): k_expand_w, the fp64 leaf GEMM plus the
  expansion (fp64 MFMA peak when the leaf GEMM is above the ridge);
* bf16 / fp16 working precision: k_expand_lp;
* batched: the whole batch.

traffic: HBM bytes per launch of that kernel from rocprofv3 counters
(profiles/traffic_*.txt), reported while the kernel's sources are unchanged.

The default run also measures, as keys of the same line, the 262144-point
fp8 operator with 128 right-hand sides (fp32 and bf16 working precision),
the 2^20-point fp64-accumulated operator with 16 right-hand sides and the
512-operator batch, each with its own timing, roofline and oracle check;
and, on the headline operator, its construction on the GPU from the kernel
(hodlr_build_kernel: time, and norms, formats and ranks against the host
compressor's) and its LU (factorization time on the host, GPU solve time,
and the solve's residual against Cor. "LU of mixed-precision HODLR
matrices").
speedup_vs_fp64: the same operators with every level stored in fp64 and
fp64 accumulation (the uniform-precision product on the same GPU).
storage_ratio: uniform-fp64 bits over the stored bits (Sect. 4 storage
experiment): leaves and factors, and factors alone.
cpu_baseline: the CPU oracle's fp64 product of the same stored operator on
the host's cores (median of 5 after a warm-up; also on 1 thread).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HODLR matvec GB/s & Gflop/s (% roofline); speedup mixed vs FP64 at fixed eps"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0     # dense bf16 / fp16 MFMA
FLUSH_BYTES = 2 << 30         # read sweep before each cold product: 8x the 256 MB last-level cache
CSRC = os.path.join(ROOT, "paper_2407_21637_amd", "csrc")
# device sources of each product path: a counter summary under profiles/
# holds only while the hash of its path's sources is unchanged
PATH_SOURCES = {"wave": ("hodlr_internal.h", "dev_common.h", "wave_path.h"),
                "wide": ("hodlr_internal.h", "dev_common.h", "wave_path.h", "wide_path.h"),
                "lowp": ("hodlr_internal.h", "dev_common.h", "wave_path.h", "wide_path.h", "lowp_path.h"),
                "batch": ("hodlr_internal.h", "dev_common.h", "wave_path.h", "wide_path.h", "kernels_batch.hip")}
SBYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2, "e4m3": 1, "e5m2": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(path):
    h = hashlib.sha256()
    for f in PATH_SOURCES[path]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(workload, nrhs):
    """key: value lines of the counter summary (HBM bytes per launch)."""
    out = {}
    f = os.path.join(ROOT, "profiles", f"traffic_{workload}_nrhs{nrhs}.txt")
    if os.path.exists(f):
        for line in open(f):
            k, sep, v = line.partition(":")
            if sep and k.strip() and " " not in k.strip():
                out[k.strip()] = v.strip()
    return out


def host_info():
    model, mem = platform.processor() or "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:  # pragma: no cover
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_gib": mem}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return 1


# ---------------------------------------------------------------------------
# inputs (host, untimed)
# ---------------------------------------------------------------------------
def build_operator(cfg, H):
    """Compress the workload over the library's partition (host, untimed)."""
    from hodlr_inputs.compress import compress
    from hodlr_inputs.configs import norm_a_2
    desc = H.tree_blocks(cfg.n, cfg.depth)
    lb = H.tree_bounds(cfg.n, cfg.depth)[cfg.depth]
    leaves = [(int(lb[i]), int(lb[i + 1] - lb[i])) for i in range(len(lb) - 1)]
    blocks = [(int(r0), int(nr), int(c0), int(nc)) for _, r0, nr, c0, nc in desc]
    P = cfg.points()
    t = time.time()
    op = compress(cfg.kernel, P, blocks, leaves, cfg.eps, cfg.rule, norm_a_2(cfg, P),
                  method=cfg.extra.get("compress", "random"))
    op.host_seconds = time.time() - t
    log(f"[bench] compressed {cfg.name}: n={cfg.n} depth={cfg.depth} in {op.host_seconds:.1f}s")
    return op


def build_batch(name):
    """Compress a batched workload over the library's partitions (host,
    untimed; spawned processes, before anything touches the GPU)."""
    from hodlr_inputs import batch as BT
    import paper_2407_21637_amd as H
    specs = BT.get(name)
    parts = []
    for sp in specs:
        desc = H.tree_blocks(sp.n, sp.depth)
        lb = H.tree_bounds(sp.n, sp.depth)[sp.depth]
        parts.append(([tuple(int(v) for v in d[1:]) for d in desc],
                      [(int(lb[i]), int(lb[i + 1] - lb[i])) for i in range(len(lb) - 1)]))
    t = time.time()
    ops = BT.build_all(specs, parts, log=log)
    log(f"[bench] compressed {name}: {len(specs)} operators, sum n = {sum(sp.n for sp in specs)} "
        f"in {time.time() - t:.1f}s")
    return specs, ops


# ---------------------------------------------------------------------------
# algorithmic work
# ---------------------------------------------------------------------------
def work(h, n, nrhs, xy_bytes):
    """Algorithmic bytes and flops of one product, the algorithmic bytes of
    the first and second launches, fp64 leaf flops, and the uniform-fp64
    storage of the same operator (for the storage ratio)."""
    inf = h.info()
    B = inf["leaf_bytes"] + inf["factor_bytes"] + inf["scale_bytes"] + n * nrhs * 2 * xy_bytes
    lr = ub = vb = 0
    for b in range(h.nblocks):
        bi = h.block(b)
        s = SBYTES[bi["dtype"]]
        lr += (bi["nrows"] + bi["ncols"]) * bi["rank"]
        ub += bi["nrows"] * bi["rank"] * s
        vb += bi["ncols"] * bi["rank"] * s
    F = 2 * nrhs * (inf["leaf_bytes"] // 8 + lr)
    leaf_flops = 2 * nrhs * (inf["leaf_bytes"] // 8)
    if nrhs >= 8:       # matrix-core path: contraction | expansion with the leaf GEMM
        first = vb + n * nrhs * xy_bytes
        second = inf["leaf_bytes"] + ub + n * nrhs * 2 * xy_bytes
    else:               # wave path: contraction and leaf GEMV tiles | expansion
        first = inf["leaf_bytes"] + vb + n * nrhs * xy_bytes
        second = ub + n * nrhs * xy_bytes
    store = {"stored_bytes": inf["leaf_bytes"] + inf["factor_bytes"] + inf["scale_bytes"],
             "fp64_bytes": inf["leaf_bytes"] + 8 * lr,
             "stored_factor_bytes": inf["factor_bytes"] + inf["scale_bytes"], "fp64_factor_bytes": 8 * lr}
    return dict(B=B, F=F, first=first, second=second, LF=leaf_flops, store=store)


def storage_ratio(st):
    """Uniform-fp64 bits over stored bits (Sect. 4 storage experiment)."""
    return {"with_leaves": round(st["fp64_bytes"] / st["stored_bytes"], 4),
            "factors_only": round(st["fp64_factor_bytes"] / max(st["stored_factor_bytes"], 1), 4)}


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------
class Flush:
    """A read sweep over FLUSH_BYTES: evicts everything from L2 and the
    last-level cache and leaves no dirty lines behind."""

    def __init__(self, torch):
        self.buf = torch.ones(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda:0")
        self.torch = torch

    def __call__(self):
        self.buf.amax()


def time_warm(fn, steps, warmup, torch):
    """ms per product, operator warm in the caches: K calls of fn captured
    in one HIP graph and replayed between two events."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(warmup, 1)):     # also sizes this stream's workspace (and plans a batch)
            fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(steps):
            fn()
    torch.cuda.synchronize()
    g.replay()                              # untimed: first replay of the graph
    torch.cuda.synchronize()
    cs = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cs)
    g.replay()                              # exactly `steps` products
    e1.record(cs)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    return ms


def time_cold(fn, steps, warmup, flush, torch):
    """Cold-cache products on the current stream: W untimed (flush,
    product) steps, then K timed ones, each product between its own event
    pair with the flush before it.  Returns (mean ms, median ms, wall ms of
    the K steps including the flushes)."""
    for _ in range(max(warmup, 1)):
        flush()
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0.record()
    for e0, e1 in ev:
        flush()
        e0.record()
        fn()
        e1.record()
    w1.record()
    torch.cuda.synchronize()
    t = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return float(t.mean()), float(np.median(t)), float(w0.elapsed_time(w1))


def time_phases(h, fn, reps, torch, flush=None):
    """Mean per-kernel durations (us) from the library's event hook, with a
    flush before each product when given (cold)."""
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    h.profile(reps)
    for _ in range(reps):
        if flush is not None:
            flush()
        fn()
    torch.cuda.synchronize()
    ph = h.profile_read()
    h.profile(0)
    return {k: v[0] / v[1] * 1e3 for k, v in ph.items() if v[1]}


# ---------------------------------------------------------------------------
# rooflines
# ---------------------------------------------------------------------------
def roofline_single(w, phases, nrhs, traffic):
    """Roofline line of the dominant kernel (see the module docstring)."""
    if nrhs >= 8:
        us = phases["expand"]
        gbs = w["second"] / (us * 1e-6) / 1e9
        ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        if w["LF"] / w["second"] >= ridge:
            ach = w["LF"] / (us * 1e-6) / 1e12
            return {"bound": "mfma", "kernel": "k_expand_w (fp64 MFMA leaf GEMM + low-rank MFMA, writes Y)",
                    "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                    "alg_flops_per_launch": int(w["LF"]), "alg_bytes_per_launch": int(w["second"]),
                    "hbm_gbs": round(gbs, 2), "mean_launch_us": round(us, 2)}
        return {"bound": "hbm", "kernel": "k_expand_w (fp64 MFMA leaf GEMM + low-rank MFMA, writes Y)",
                "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": int(w["second"]),
                "intensity_flop_per_byte": round(w["LF"] / w["second"], 3), "mean_launch_us": round(us, 2)}
    us = phases["contract"]
    gbs = w["first"] / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": "k_phase1 (contraction items + fp64 leaf GEMV tiles)",
            "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic, "alg_bytes_per_launch": int(w["first"]), "mean_launch_us": round(us, 2)}


def launches(w, ph, nrhs, tr=None):
    """Both launches of a product: algorithmic bytes, mean cold duration,
    achieved GB/s, and the counter traffic of the profiles (tr: the
    summary's keys, only when its kernel hash matches)."""
    wide = nrhs >= 8
    out = {"first": {"kernel": "k_contract_w" if wide else "k_phase1", "alg_bytes": int(w["first"])},
           "second": {"kernel": "k_expand_w" if wide else "k_expand", "alg_bytes": int(w["second"])}}
    for key, ph_name in (("first", "contract"), ("second", "expand")):
        if ph_name in ph:
            out[key]["mean_us"] = round(ph[ph_name], 2)
            out[key]["achieved_gbs"] = round(out[key]["alg_bytes"] / (ph[ph_name] * 1e-6) / 1e9, 2)
        out[key]["traffic"] = int(tr.get(f"{key}_launch_bytes", 0)) or None if tr else None
    return out


# ---------------------------------------------------------------------------
# oracle legs
# ---------------------------------------------------------------------------
def oracle_stored(cfg, op, level_fmt):
    from oracle import quantize as Q
    from oracle import tree as T
    oblocks = T.blocks(cfg.n, cfg.depth)
    U = [Q.quantize(u, level_fmt[b.level - 1]).values for b, u in zip(oblocks, op.U)]
    V = [Q.quantize(v, level_fmt[b.level - 1]).values for b, v in zip(oblocks, op.V)]
    return oblocks, T.leaves(cfg.n, cfg.depth), U, V


def cpu_baseline(cfg, op, level_fmt, B_alg, X):
    """The oracle's fp64 product of the same stored operator on the host:
    all cores and one thread (the paper's setting), median of 5 after a
    warm-up each."""
    from oracle import matvec as MV
    oblocks, lb, U, V = oracle_stored(cfg, op, level_fmt)

    def med5():
        MV.matvec(cfg.n, oblocks, lb, op.leaves, U, V, X)          # warm-up
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            y = MV.matvec(cfg.n, oblocks, lb, op.leaves, U, V, X)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), y

    cores = blas_threads()
    sec, y = med5()
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            one, _ = med5()
    except Exception:  # pragma: no cover
        pass
    cb = {"value": round(B_alg / sec / 1e9, 4), "unit": "GB/s", "cores": int(cores), "kind": "oracle",
          "sample": f"median of 5 full products (after a warm-up) of the oracle's fp64 HODLR_MATVEC on the same "
                    f"stored operator (n={cfg.n}, nrhs={X.shape[1]}): {sec * 1e3:.2f} ms each on {cores} threads",
          "ms_per_product": round(sec * 1e3, 3)}
    if one is not None:
        cb["one_thread"] = {"value": round(B_alg / one / 1e9, 4), "unit": "GB/s", "cores": 1,
                            "ms_per_product": round(one * 1e3, 3)}
    cb.update(host_info())
    return cb, y, oblocks, lb, U, V


def check_against_oracle(cfg, op, level_fmt, X, Yg, acc, xb, oracle=None):
    """Max componentwise error over the gate tau_prob (entries outside it are logged)."""
    from oracle import bounds as BD
    from oracle import matvec as MV
    if oracle is None:
        oblocks, lb, U, V = oracle_stored(cfg, op, level_fmt)
        y = MV.matvec(cfg.n, oblocks, lb, op.leaves, U, V, X)
    else:
        y, oblocks, lb, U, V = oracle
    z = MV.matvec_abs(cfg.n, oblocks, lb, op.leaves, U, V, X)
    M = BD.chain_length(oblocks, op.ranks, [m for _, m in lb], cfg.depth)
    u_acc = 2.0 ** -24 if acc == "fp32" else 2.0 ** -53
    tau = BD.tolerance_prob(z, y, M, u_acc, 2.0 ** -24 if xb == 4 else 2.0 ** -53)
    err = np.abs(Yg - y)
    bad = int((err > tau).sum())
    if bad:
        log(f"[bench] {cfg.name}: {bad} entries outside the tolerance")
    return {"max_err_over_tau_prob": float((err / tau).max()), "entries_outside": bad,
            "rel_err_vs_oracle": float(np.linalg.norm(err) / np.linalg.norm(y)), "columns_checked": int(X.shape[1])}


# ---------------------------------------------------------------------------
# one operator, one nrhs
# ---------------------------------------------------------------------------
def measure(h, cfg, nrhs, xdt, xb, Xh, args, flush, torch, H):
    dev = torch.device("cuda:0")
    X = H.colmajor_empty(cfg.n, nrhs, xdt, dev)
    X.copy_(torch.from_numpy(np.asfortranarray(Xh[:, :nrhs])).to(xdt))
    Y = H.colmajor_empty(cfg.n, nrhs, xdt, dev)
    w = work(h, cfg.n, nrhs, xb)
    fn = lambda: h.matvec(X, Y)  # noqa: E731
    cold, cold_med, wall = time_cold(fn, args.steps, args.warmup, flush, torch)
    warm = time_warm(fn, args.steps, args.warmup, torch)
    ph_cold = time_phases(h, fn, 20, torch, flush)
    ph_warm = time_phases(h, fn, 50, torch)
    log(f"[bench] {cfg.name} nrhs={nrhs}: cold {cold * 1e3:.1f} us ({w['B'] / cold / 1e6:.1f} GB/s), warm "
        f"{warm * 1e3:.1f} us ({w['B'] / warm / 1e6:.1f} GB/s); kernels cold {ph_cold} warm {ph_warm}")
    return dict(X=X, Y=Y, w=w, cold=cold, cold_med=cold_med, wall=wall, warm=warm, ph_cold=ph_cold,
                ph_warm=ph_warm)


def fp64_speedup(h, cfg, r, args, flush, torch, H, xb):
    """Same handle, every level fp64 with fp64 accumulation, cold and warm."""
    fn = lambda: h.matvec(r["X"], r["Y"])  # noqa: E731
    h.set_level_precisions(["fp64"] * cfg.depth, H.ACC_FP64)
    B64 = work(h, cfg.n, r["X"].shape[1], xb)["B"]
    c64 = time_cold(fn, args.steps, args.warmup, flush, torch)[0]
    w64 = time_warm(fn, args.steps, args.warmup, torch)
    return {"speedup_vs_fp64": round(c64 / r["cold"], 3), "speedup_vs_fp64_warm": round(w64 / r["warm"], 3),
            "fp64_gbs": round(B64 / (c64 * 1e-3) / 1e9, 2), "fp64_ms": round(c64, 5)}


def single_workload(name, nrhs_list, args, flush, torch, H, with_cpu, headline):
    """Measure one compressed workload at the given nrhs values."""
    from hodlr_inputs import configs as CF
    cfg = CF.get(name)
    op = build_operator(cfg, H)
    norms2 = np.concatenate([[op.norm2_all], op.norm2_blocks])
    h = H.Operator(cfg.n, cfg.depth, op.leaves, op.U, op.V, device=0)
    h.assign_precision(cfg.eps, cfg.allowed, norms2)
    fmts = [lv[0] for lv in h.levels()]
    acc = h.info()["acc_dtype"]
    log(f"[bench] {name}: formats {fmts}; accumulation {acc}")
    xdt = torch.float32 if cfg.x_dtype == "fp32" else torch.float64
    xb = 4 if cfg.x_dtype == "fp32" else 8
    Xh = cfg.X(max(nrhs_list))
    res = {k: measure(h, cfg, k, xdt, xb, Xh, args, flush, torch, H) for k in nrhs_list}
    n0 = nrhs_list[0]
    r = res[n0]
    tr = read_traffic(cfg.name, n0)
    path = "wide" if n0 >= 8 else "wave"
    traffic = None
    if tr.get("kernel_sha") == kernel_hash(path) and tr.get("workload") == cfg.name and tr.get("nrhs") == str(n0):
        traffic = int(tr.get("second_launch_bytes" if n0 >= 8 else "first_launch_bytes", 0)) or None
    else:
        tr = None
    w = r["w"]
    out = {
        "value": round(w["B"] / (r["cold"] * 1e-3) / 1e9, 2), "unit": "GB/s",
        "ms_per_step": round(r["cold"], 5), "ms_per_step_median": round(r["cold_med"], 5),
        "timed_region_ms_incl_flushes": round(r["wall"], 3),
        "config": {"workload": f"{cfg.name}: {cfg.description}; n={cfg.n}, leaf {-(-cfg.n >> cfg.depth)}, depth "
                               f"{cfg.depth}, eps={cfg.eps:g}, formats {fmts}, {cfg.x_dtype} X nrhs={n0}",
                   "n": cfg.n, "depth": cfg.depth, "eps": cfg.eps, "nrhs": n0, "formats": fmts, "accumulation": acc},
        "gflops": round(w["F"] / (r["cold"] * 1e-3) / 1e9, 2),
        "hbm_frac": round(w["B"] / (r["cold"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "alg_bytes": int(w["B"]), "alg_flops": int(w["F"]),
        "warm_cache_gbs": round(w["B"] / (r["warm"] * 1e-3) / 1e9, 2), "warm_ms_per_step": round(r["warm"], 5),
        "kernels_us_cold": {k: round(v, 2) for k, v in r["ph_cold"].items()},
        "kernels_us_warm": {k: round(v, 2) for k, v in r["ph_warm"].items()},
        "roofline": roofline_single(w, r["ph_cold"], n0, traffic),
        "roofline_warm": roofline_single(w, r["ph_warm"], n0, None),
        "launches": launches(w, r["ph_cold"], n0, tr),
        "storage_ratio": storage_ratio(w["store"]),
    }
    out["roofline"]["timing"] = "cold: 2 GiB read sweep before each product"
    for k in nrhs_list[1:]:
        rk = res[k]
        wk = rk["w"]
        out[f"nrhs{k}"] = {"gbs": round(wk["B"] / (rk["cold"] * 1e-3) / 1e9, 2),
                           "gflops": round(wk["F"] / (rk["cold"] * 1e-3) / 1e9, 2),
                           "ms_per_step": round(rk["cold"], 5),
                           "warm_cache_gbs": round(wk["B"] / (rk["warm"] * 1e-3) / 1e9, 2),
                           "kernels_us_cold": {q: round(v, 2) for q, v in rk["ph_cold"].items()},
                           "roofline": roofline_single(wk, rk["ph_cold"], k, None)}
    # accuracy of every measured product against the oracle, and the CPU leg
    oracle = None
    if with_cpu:
        cb, y, oblocks, lb, U, V = cpu_baseline(cfg, op, fmts, w["B"], Xh[:, :n0])
        out["cpu_baseline"] = cb
        oracle = (y, oblocks, lb, U, V)
    checks = {}
    for k in nrhs_list:
        rk = res[k]
        fn = lambda: h.matvec(rk["X"], rk["Y"])  # noqa: E731
        fn()
        torch.cuda.synchronize()
        Yg = rk["Y"].cpu().double().numpy()
        checks[k] = check_against_oracle(cfg, op, fmts, Xh[:, :k], Yg, acc, xb, oracle if k == n0 else None)
    out["check"] = checks[n0]
    for k in nrhs_list[1:]:
        out[f"nrhs{k}"]["check"] = checks[k]
    out.update(fp64_speedup(h, cfg, r, args, flush, torch, H, xb))
    h.assign_precision(cfg.eps, cfg.allowed, norms2)
    return out, (cfg, op, h, fmts, norms2)


# ---------------------------------------------------------------------------
# construction on the GPU and the LU solve, on the headline workload
# ---------------------------------------------------------------------------
# the library's description of each recipe's kernel matrix (hodlr_build_kernel)
LIB_KERNELS = {"c2": dict(kind="gaussian", a=0.04, diag_shift=0.01)}


def construct_lu_workload(state, torch, H, solves=10):
    """The headline operator built on the GPU from its kernel (compared with
    the host compressor's exact norms, formats and ranks), its LU on the
    host, and the GPU solve with the inverse factors (residual against
    Cor. "LU of mixed-precision HODLR matrices")."""
    cfg, op, h, fmts, norms2 = state
    if cfg.name not in LIB_KERNELS:
        return None
    P = cfg.points()
    torch.cuda.synchronize()
    t = time.time()
    hb, rep = H.build_kernel(P, cfg.depth, eps=cfg.eps, seed=7, **LIB_KERNELS[cfg.name])
    torch.cuda.synchronize()
    wall = time.time() - t
    got = hb.norms2()
    norm_rel = float(np.max(np.abs(got - norms2) / np.maximum(np.abs(norms2), 1e-300)))
    hb.assign_precision(cfg.eps, cfg.allowed)               # from the norms the construction kept
    gfmts = [lv[0] for lv in hb.levels()]
    dr = np.array(hb.query()["ranks"]) - np.array(op.ranks)
    log(f"[bench] {cfg.name} built on the GPU in {wall:.2f}s (host compressor "
        f"{getattr(op, 'host_seconds', float('nan')):.1f}s); norms rel diff {norm_rel:.1e}, "
        f"formats {gfmts}, rank diff [{dr.min()}, {dr.max()}]")
    out = {"construct": {"seconds": round(wall, 3), "report_ms": {k: round(rep[k], 1) for k in
                                                                   ("ms_norms", "ms_factors", "ms_total")},
                         "host_compressor_seconds": round(getattr(op, "host_seconds", float("nan")), 2),
                         "max_rank": rep["max_rank"],
                         "check": {"norms_max_rel_diff": norm_rel, "formats_equal": gfmts == fmts,
                                   "rank_diff_min": int(dr.min()), "rank_diff_max": int(dr.max())}}}
    t = time.time()
    lrep = hb.lu(cfg.eps)
    lu_wall = time.time() - t
    b = np.random.default_rng(21).standard_normal((cfg.n, 1))
    B = H.colmajor_empty(cfg.n, 1, torch.float64, "cuda:0")
    B.copy_(torch.from_numpy(np.asfortranarray(b)))
    X = H.colmajor_empty(cfg.n, 1, torch.float64, "cuda:0")
    hb.solve(B, X)                                          # workspaces
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(solves):
        hb.solve(B, X)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / solves
    res = float(torch.linalg.vector_norm(hb.matvec(X) - B)) / float(torch.linalg.vector_norm(X))
    # Cor. "LU of mixed-precision HODLR matrices": 2 (2^l - 1) eps ||H|| + 11 (2^l - 1) eps ||L|| ||U||
    c = 2 ** cfg.depth - 1
    bound = 2 * c * cfg.eps * float(np.sqrt(norms2[0])) + 11 * c * cfg.eps * lrep["norm_l"] * lrep["norm_u"]
    log(f"[bench] {cfg.name} LU on the host {lu_wall:.1f}s; GPU solve {ms:.3f} ms; ||Hx-b||/||x|| {res:.2e} "
        f"(bound {bound:.2e})")
    out["lu"] = {"factor_seconds": round(lu_wall, 2), "solve_ms": round(ms, 4), "nrhs": 1,
                 "max_rank": lrep["max_rank"], "norm_l": lrep["norm_l"], "norm_u": lrep["norm_u"],
                 "check": {"residual_over_norm_x": res, "corollary_bound": bound, "within": res <= bound}}
    hb.close()
    return out


# ---------------------------------------------------------------------------
# the product in a low working precision
# ---------------------------------------------------------------------------
def lowp_workload(state, w, nrhs, args, flush, torch, H):
    """The product in working precision w on an already built operator: the
    roofline is the expansion launch (the W leaf GEMM, HBM-bound below the W
    ridge of 2500 TFLOP/s / 8 TB/s ~ 312 flop/B)."""
    cfg, op, h, fmts, _ = state
    wdt = torch.bfloat16 if w == "bf16" else torch.float16
    inf = h.info()
    leaf_w = inf["leaf_bytes"] // 4                      # the W copy of the leaves
    ub = vb = lr = tw = 0
    for b in range(h.nblocks):
        bi = h.block(b)
        sb = SBYTES[bi["dtype"]]
        ub += bi["nrows"] * bi["rank"] * sb
        vb += bi["ncols"] * bi["rank"] * sb
        lr += (bi["nrows"] + bi["ncols"]) * bi["rank"]
        tw += -(-bi["rank"] // 32) * 32 * nrhs * 2
    n = cfg.n
    B = leaf_w + inf["factor_bytes"] + inf["scale_bytes"] + n * nrhs * 2 * 2
    LF = 2 * nrhs * (inf["leaf_bytes"] // 8)
    Fl = LF + 2 * nrhs * lr
    EB = leaf_w + ub + tw + n * nrhs * 2 * 2             # expansion: leaves, U, T, X, Y
    from oracle import formats as OF
    Xw = OF.round_rne(w, cfg.X(nrhs))
    X = H.colmajor_empty(n, nrhs, wdt, "cuda:0")
    X.copy_(torch.from_numpy(np.asfortranarray(Xw)).to(wdt))
    Y = H.colmajor_empty(n, nrhs, wdt, "cuda:0")
    fn = lambda: h.matvec(X, Y)  # noqa: E731
    cold, cold_med, _ = time_cold(fn, args.steps, args.warmup, flush, torch)
    warm = time_warm(fn, args.steps, args.warmup, torch)
    ph = time_phases(h, fn, 20, torch, flush)
    log(f"[bench] {cfg.name} {w} working precision, nrhs={nrhs}: cold {cold * 1e3:.1f} us, warm "
        f"{warm * 1e3:.1f} us, kernels cold {ph}")
    # the fp32/fp64 product on the same operator and X for the speedup
    xdt = torch.float32 if cfg.x_dtype == "fp32" else torch.float64
    Xf = H.colmajor_empty(n, nrhs, xdt, "cuda:0")
    Xf.copy_(torch.from_numpy(np.asfortranarray(Xw)).to(xdt))
    Yf = H.colmajor_empty(n, nrhs, xdt, "cuda:0")
    cold_full = time_cold(lambda: h.matvec(Xf, Yf), args.steps, args.warmup, flush, torch)[0]
    exp_us = ph["expand"]
    exp_gbs = EB / (exp_us * 1e-6) / 1e9
    intensity = LF / EB
    if intensity >= BF16_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        ach = LF / (exp_us * 1e-6) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / BF16_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(exp_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(exp_gbs / HBM_PEAK_GBS, 4)}
    tr = read_traffic(f"{cfg.name}_{w}", nrhs)
    traffic = None
    if tr.get("kernel_sha") == kernel_hash("lowp") and tr.get("nrhs") == str(nrhs):
        traffic = int(tr.get("second_launch_bytes", 0)) or None
    roof.update({"kernel": f"k_expand_lp ({w} MFMA leaf GEMM + low-rank, writes Y)", "traffic": traffic,
                 "alg_bytes_per_launch": int(EB), "intensity_flop_per_byte": round(intensity, 2),
                 "mfma_tflops": round(LF / (exp_us * 1e-6) / 1e12, 2), "mean_launch_us": round(exp_us, 2),
                 "timing": "cold: 2 GiB read sweep before each product"})
    out = {"value": round(B / (cold * 1e-3) / 1e9, 2), "unit": "GB/s", "ms_per_step": round(cold, 5),
           "dtype": w, "working_precision": w, "nrhs": nrhs, "formats": fmts,
           "gflops": round(Fl / (cold * 1e-3) / 1e9, 2), "alg_bytes": int(B), "alg_flops": int(Fl),
           "warm_cache_gbs": round(B / (warm * 1e-3) / 1e9, 2),
           "speedup_vs_full_precision_path": round(cold_full / cold, 3),
           "kernels_us_cold": {k: round(v, 2) for k, v in ph.items()}, "roofline": roof}
    # the oracle's W product on every column: the tolerance check
    from oracle import bounds as BD
    from oracle import lowp as LP
    from oracle import quantize as Q
    from oracle import tree as T
    oblocks = T.blocks(n, cfg.depth)
    lb = T.leaves(n, cfg.depth)
    QU = [Q.quantize(u, fmts[b.level - 1]) for b, u in zip(oblocks, op.U)]
    QV = [Q.quantize(v, fmts[b.level - 1]) for b, v in zip(oblocks, op.V)]
    k = nrhs
    prod = LP.matvec_lowp(n, oblocks, lb, op.leaves, QU, QV, Xw[:, :k], w)
    fn()
    torch.cuda.synchronize()
    yg = Y[:, :k].float().cpu().double().numpy()
    M = BD.chain_length(oblocks, op.ranks, [m for _, m in lb], cfg.depth)
    tol = LP.tolerance(prod, w, M, max(b.ncols for b in oblocks))
    err = np.abs(yg - prod.y)
    out["check"] = {"max_err_over_tol": float((err / np.where(tol > 0, tol, 1)).max()),
                    "entries_outside": int((err > tol).sum()), "columns_checked": k,
                    "rel_err_vs_oracle": float(np.linalg.norm(err) / np.linalg.norm(prod.y))}
    return out


# ---------------------------------------------------------------------------
# the batch
# ---------------------------------------------------------------------------
def batch_workload(name, batch, args, flush, torch, H, with_check):
    """The batched workload: all operators in one hodlr_matvec_batched call."""
    from hodlr_inputs import batch as BT
    specs, cops = batch
    dev = torch.device("cuda:0")
    t = time.time()
    hs, Xs, Ys, xbs = [], [], [], []
    for sp, c in zip(specs, cops):
        h = H.Operator(sp.n, sp.depth, c.leaves, c.U, c.V, device=0)
        h.assign_precision(sp.eps, BT.ALLOWED, np.concatenate([[c.norm2_all], c.norm2_blocks]))
        dt = torch.float64 if sp.x_dtype == "fp64" else torch.float32
        X = H.colmajor_empty(sp.n, sp.nrhs, dt, dev)
        X.copy_(torch.from_numpy(np.asfortranarray(sp.X())).to(dt))
        hs.append(h)
        Xs.append(X)
        Ys.append(H.colmajor_empty(sp.n, sp.nrhs, dt, dev))
        xbs.append(8 if sp.x_dtype == "fp64" else 4)
    log(f"[bench] {len(hs)} operators on GPU in {time.time() - t:.1f}s")

    def fn():
        H.matvec_batched(hs, Xs, Ys)

    t = time.time()
    fn()                                   # plan: work lists, autotuning, graph
    torch.cuda.synchronize()
    log(f"[bench] batch plan built and tuned in {time.time() - t:.2f}s")

    def totals():
        B = F = st64 = st = 0
        for h, sp, xb in zip(hs, specs, xbs):
            w = work(h, sp.n, sp.nrhs, xb)
            B += w["B"]
            F += w["F"]
            st64 += w["store"]["fp64_bytes"]
            st += w["store"]["stored_bytes"]
        return B, F, st64, st

    B, F, st64, st = totals()
    cold, cold_med, wall = time_cold(fn, args.steps, args.warmup, flush, torch)
    warm = time_warm(fn, args.steps, args.warmup, torch)
    log(f"[bench] batch: cold {cold * 1e3:.1f} us ({B / cold / 1e6:.1f} GB/s), warm {warm * 1e3:.1f} us")
    fm = [[lv[0] for lv in h.levels()] for h in hs]
    acc = [h.info()["acc_dtype"] for h in hs]
    for h, sp in zip(hs, specs):
        h.set_level_precisions(["fp64"] * sp.depth, H.ACC_FP64)
    B64 = totals()[0]
    cold64 = time_cold(fn, args.steps, args.warmup, flush, torch)[0]
    warm64 = time_warm(fn, args.steps, args.warmup, torch)
    for h, sp, c in zip(hs, specs, cops):
        h.assign_precision(sp.eps, BT.ALLOWED, np.concatenate([[c.norm2_all], c.norm2_blocks]))
    log(f"[bench] uniform fp64 batch: cold {cold64 * 1e3:.1f} us, warm {warm64 * 1e3:.1f} us")
    value = B / (cold * 1e-3) / 1e9
    fmt_count = {}
    for f in fm:
        for x in f:
            fmt_count[x] = fmt_count.get(x, 0) + 1
    out = {
        "value": round(value, 2), "unit": "GB/s", "ms_per_step": round(cold, 5),
        "config": {"workload": f"{name}: {len(specs)} independent operators, n log-uniform, kernels 1/(r+1e-3), "
                               f"exp(-r), exp(-r^2/0.08) in 1D/2D, eps 1e-4/1e-6/1e-8, nrhs 1/8/32, one "
                               f"hodlr_matvec_batched call", "operators": len(specs),
                   "sum_n": int(sum(sp.n for sp in specs)), "level_formats": fmt_count,
                   "fp64_accumulation_ops": int(sum(a == "fp64" for a in acc))},
        "gflops": round(F / (cold * 1e-3) / 1e9, 2), "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "alg_bytes": int(B), "alg_flops": int(F),
        "warm_cache_gbs": round(B / (warm * 1e-3) / 1e9, 2),
        "speedup_vs_fp64": round(cold64 / cold, 3), "speedup_vs_fp64_warm": round(warm64 / warm, 3),
        "fp64_gbs": round(B64 / (cold64 * 1e-3) / 1e9, 2),
        "storage_ratio": {"with_leaves": round(st64 / st, 4)},
        "roofline": {"bound": "hbm", "kernel": "whole batch (persistent launches of every kernel variant)",
                     "achieved": round(value, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(value / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": int(B), "mean_launch_us": round(cold * 1e3, 2),
                     "timing": "cold: 2 GiB read sweep before each batch"},
    }
    if with_check:
        from oracle import bounds as BD
        from oracle import matvec as MV
        from oracle import quantize as Q
        from oracle import tree as T
        fn()
        torch.cuda.synchronize()
        worst, bad, t0 = 0.0, 0, time.perf_counter()
        for k, (h, sp, c, xb) in enumerate(zip(hs, specs, cops, xbs)):
            blocks = T.blocks(sp.n, sp.depth)
            lb = T.leaves(sp.n, sp.depth)
            U = [Q.quantize(u, fm[k][b.level - 1]).values for b, u in zip(blocks, c.U)]
            V = [Q.quantize(v, fm[k][b.level - 1]).values for b, v in zip(blocks, c.V)]
            X = sp.X()
            y = MV.matvec(sp.n, blocks, lb, c.leaves, U, V, X)
            z = MV.matvec_abs(sp.n, blocks, lb, c.leaves, U, V, X)
            M = BD.chain_length(blocks, c.ranks, [m for _, m in lb], sp.depth)
            u_acc = 2.0 ** -24 if acc[k] == "fp32" else 2.0 ** -53
            tau = BD.tolerance_prob(z, y, M, u_acc, 2.0 ** -24 if xb == 4 else 2.0 ** -53)
            err = np.abs(Ys[k].cpu().double().numpy() - y)
            worst = max(worst, float((err / tau).max()))
            bad += int((err > tau).sum())
        out["check"] = {"max_err_over_tau_prob": worst, "entries_outside": bad, "operators_checked": len(hs),
                        "oracle_seconds": round(time.perf_counter() - t0, 1)}
    for h in hs:
        h.close()
    return out


# ---------------------------------------------------------------------------
# profiling mode: only the timed products (under rocprofv3)
# ---------------------------------------------------------------------------
def profile_run(args, torch, H, batch):
    flush = Flush(torch) if not args.warm else None
    if batch is not None:
        from hodlr_inputs import batch as BT
        specs, cops = batch
        hs, Xs, Ys = [], [], []
        for sp, c in zip(specs, cops):
            h = H.Operator(sp.n, sp.depth, c.leaves, c.U, c.V, device=0)
            if args.fp64:
                h.set_level_precisions(["fp64"] * sp.depth, H.ACC_FP64)
            else:
                h.assign_precision(sp.eps, BT.ALLOWED, np.concatenate([[c.norm2_all], c.norm2_blocks]))
            dt = torch.float64 if sp.x_dtype == "fp64" else torch.float32
            X = H.colmajor_empty(sp.n, sp.nrhs, dt, "cuda:0")
            X.copy_(torch.from_numpy(np.asfortranarray(sp.X())).to(dt))
            hs.append(h)
            Xs.append(X)
            Ys.append(H.colmajor_empty(sp.n, sp.nrhs, dt, "cuda:0"))
        fn = lambda: H.matvec_batched(hs, Xs, Ys)  # noqa: E731
    else:
        from hodlr_inputs import configs as CF
        cfg = CF.get(args.workload)
        op = build_operator(cfg, H)
        h = H.Operator(cfg.n, cfg.depth, op.leaves, op.U, op.V, device=0)
        if args.fp64:
            h.set_level_precisions(["fp64"] * cfg.depth, H.ACC_FP64)
        else:
            h.assign_precision(cfg.eps, cfg.allowed, np.concatenate([[op.norm2_all], op.norm2_blocks]))
        nrhs = args.nrhs if args.nrhs is not None else cfg.nrhs[0]
        if args.working:
            from oracle import formats as OF
            dt = torch.bfloat16 if args.working == "bf16" else torch.float16
            Xv = OF.round_rne(args.working, cfg.X(nrhs))
        else:
            dt = torch.float32 if cfg.x_dtype == "fp32" else torch.float64
            Xv = cfg.X(nrhs)
        X = H.colmajor_empty(cfg.n, nrhs, dt, "cuda:0")
        X.copy_(torch.from_numpy(np.asfortranarray(Xv)).to(dt))
        Y = H.colmajor_empty(cfg.n, nrhs, dt, "cuda:0")
        fn = lambda: h.matvec(X, Y)  # noqa: E731
    if flush is None:
        ms = time_warm(fn, args.steps, args.warmup, torch)
    else:
        ms = time_cold(fn, args.steps, args.warmup, flush, torch)[0]
    print(json.dumps({"profile_run": True, "workload": args.workload, "cold": flush is not None,
                      "us_per_step": ms * 1e3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nrhs", type=int, default=None, help="profile runs: default the workload's first nrhs")
    ap.add_argument("--workload", default="c2", help="headline workload (c2 by default)")
    ap.add_argument("--only", action="store_true", help="measure only the headline workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the timed products of --workload (for running under rocprofv3)")
    ap.add_argument("--warm", action="store_true", help="profile runs: warm graph replays instead of cold")
    ap.add_argument("--fp64", action="store_true",
                    help="profile runs: every level stored in fp64 with fp64 accumulation (the uniform baseline)")
    ap.add_argument("--working", choices=["bf16", "fp16"], default=None,
                    help="profile runs: the product in this low working precision")
    ap.add_argument("--kernel-hash", action="store_true",
                    help="print the source hash of each product path and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device-to-device copy 5 times (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the product runs on one GPU; a multi-GPU product would give each GPU "
                                   "a subtree (its leaves and blocks) and exchange the top levels' small "
                                   "T_b, which is not implemented; run with --gpus 1"}), flush=True)
        sys.exit(2)
    if args.kernel_hash:
        print(json.dumps({k: kernel_hash(k) for k in PATH_SOURCES}))
        return

    # torch first: the library then binds to the HIP runtime torch loaded
    import torch
    import paper_2407_21637_amd as H
    from hodlr_inputs.batch import BATCHES

    t_start = time.time()
    batch = None
    if not args.copy_calibration:
        # host-side, in spawned processes, before anything touches the GPU
        if args.workload in BATCHES:
            batch = build_batch(args.workload)
        elif not args.only and not args.profile_run:
            batch = build_batch("c4")

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda:0")
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "copies": 5}), flush=True)
        return
    H.lib()   # fail loudly if the HIP library is not built
    if args.profile_run:
        return profile_run(args, torch, H, batch if args.workload in BATCHES else None)
    flush = Flush(torch)
    common = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if args.workload in BATCHES:
        out = batch_workload(args.workload, batch, args, flush, torch, H, not args.no_cpu)
        out.update(common)
        out["dtype"] = "f32+f64"
        print(json.dumps(out), flush=True)
        return
    from hodlr_inputs import configs as CF
    cfg = CF.get(args.workload)
    head, state = single_workload(args.workload, list(cfg.nrhs), args, flush, torch, H, not args.no_cpu, True)
    out = dict(common)
    out.update(head)
    out["dtype"] = "f32+f64" if cfg.x_dtype == "fp32" else "f64"
    if not args.only:
        extra = {}
        cl = construct_lu_workload(state, torch, H)
        if cl is not None:
            extra[f"{cfg.name}_construct_lu"] = cl
        state[2].close()
        del state
        # the low-accuracy fp8 operator with 128 right-hand sides: fp32 X (fp64 MFMA leaves), then bf16 X
        r3, st3 = single_workload("c3", [128], args, flush, torch, H, False, False)
        extra["c3"] = r3
        extra["c3_bf16"] = lowp_workload(st3, "bf16", 128, args, flush, torch, H)
        st3[2].close()
        del st3
        # the 2^20-point high-accuracy operator (fp64 accumulation), 16 fp64 right-hand sides
        r5, st5 = single_workload("c5", [16], args, flush, torch, H, False, False)
        extra["c5"] = r5
        st5[2].close()
        del st5
        # the 512-operator batch
        extra["c4"] = batch_workload("c4", batch, args, flush, torch, H, not args.no_cpu)
        out["workloads"] = extra
    out["bench_wall_s"] = round(time.time() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
