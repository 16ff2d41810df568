"""Benchmark of the mixed-precision HODLR matrix-vector product on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs 1] [--workload c2]

A step is one full product Y = A_H X (contraction, reduction, expansion and
leaves) over one batch of right-hand sides, with the operator and X already
resident in HBM.  The default workload is the 65536-point 2D Gaussian-kernel
operator (Morton order, leaf 256, depth 8, eps = 1e-6, formats chosen by the
adaptive rule from fp32/bf16/fp16) with one fp32 right-hand side.  Printed
as one JSON line:

* value: algorithmic GB/s = B_alg / time per step, where
  B_alg = 8 sum m_i^2 + sum_b (r_b + c_b) p_b s(f_b) + scaled columns
          + n nrhs (s_X + s_Y)
  (leaves, factor codes, scales, X read once, Y written once);
* gflops: F_alg / time, F_alg = 2 nrhs (sum m_i^2 + sum_b (r_b + c_b) p_b);
* roofline: the dominant kernel, k_expand (fp64 leaves, U codes, X and Y:
  8 sum m_i^2 + sum_b r_b p_b s(f_b) + n nrhs (s_X + s_Y) bytes per
  launch), over its mean duration from HIP events the library records
  around it on its launch stream (an eager loop of the same products);
  k_contract (sum_b c_b p_b s(f_b) + n nrhs s_X bytes) is reported beside it;
* timing: the K timed products are captured once into a HIP graph and
  replayed between two events, so the timed region holds exactly K
  products and no Python launch latency;
* speedup_vs_fp64: same operator with every level stored in fp64 and fp64
  accumulation (the uniform-precision product on the same GPU);
* cpu_baseline: the CPU oracle's fp64 product of the same stored operator
  on the host's cores, over a bounded number of repetitions.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
CSRC = os.path.join(ROOT, "paper_2407_21637_amd", "csrc")
# device sources of each product path: a counter summary under profiles/
# holds only while the hash of its path's sources is unchanged
PATH_SOURCES = {"wave": ("hodlr_internal.h", "dev_common.h", "wave_path.h"),
                "wide": ("hodlr_internal.h", "dev_common.h", "wave_path.h", "wide_path.h"),
                "lowp": ("hodlr_internal.h", "dev_common.h", "wave_path.h", "wide_path.h", "lowp_path.h")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(path):
    h = hashlib.sha256()
    for f in PATH_SOURCES[path]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_file(workload, nrhs):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}_nrhs{nrhs}.txt")


def read_traffic(workload, nrhs):
    """key: value lines of the counter summary (HBM bytes per launch)."""
    out = {}
    f = traffic_file(workload, nrhs)
    if os.path.exists(f):
        for line in open(f):
            k, sep, v = line.partition(":")
            if sep and k.strip() and " " not in k.strip():
                out[k.strip()] = v.strip()
    return out


def build_operator(cfg, H):
    """Compress the workload over the library's partition (host, untimed)."""
    from hodlr_inputs.compress import compress
    desc = H.tree_blocks(cfg.n, cfg.depth)
    lb = H.tree_bounds(cfg.n, cfg.depth)[cfg.depth]
    leaves = [(int(lb[i]), int(lb[i + 1] - lb[i])) for i in range(len(lb) - 1)]
    blocks = [(int(r0), int(nr), int(c0), int(nc)) for _, r0, nr, c0, nc in desc]
    from hodlr_inputs.configs import norm_a_2
    P = cfg.points()
    t = time.time()
    op = compress(cfg.kernel, P, blocks, leaves, cfg.eps, cfg.rule, norm_a_2(cfg, P),
                  method=cfg.extra.get("compress", "random"))
    log(f"[bench] compressed {cfg.name}: n={cfg.n} depth={cfg.depth} in {time.time() - t:.1f}s")
    return P, blocks, leaves, op


SBYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2, "e4m3": 1, "e5m2": 1}


def work(h, n, nrhs, xy_bytes):
    """Algorithmic bytes and flops of one product; algorithmic bytes of the
    second (expansion) and first (contraction, with the leaf tiles on the wave
    path) launches; fp64 flops of the leaf products."""
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
    return B, F, second, first, leaf_flops


def time_steps(fn, steps, warmup, torch):
    """ms per product: K calls of fn (one product each, on the current
    stream) captured in one HIP graph, replayed."""
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
    torch.cuda.synchronize()
    e0.record(cs)
    g.replay()                              # exactly `steps` products
    e1.record(cs)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    return ms


def time_phases(h, X, Y, reps, torch):
    """Mean per-kernel durations (us) from the library's event hook, eager."""
    for _ in range(3):
        h.matvec(X, Y)
    torch.cuda.synchronize()
    h.profile(reps)
    for _ in range(reps):
        h.matvec(X, Y)
    torch.cuda.synchronize()
    ph = h.profile_read()
    h.profile(0)
    return {k: v[0] / v[1] * 1e3 for k, v in ph.items() if v[1]}


def time_cold(fn, reps, torch):
    """Per-product time with the caches flushed (1 GiB written) before each."""
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
    out = []
    for _ in range(reps):
        flush.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    del flush
    return float(np.median(out))


def cpu_baseline(cfg, blocks, leaves, op, level_fmt, B_alg, X, budget_s=12.0):
    """The oracle's product of the same stored operator, timed on the host."""
    from oracle import matvec as MV
    from oracle import quantize as Q
    from oracle import tree as T
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    oblocks = T.blocks(cfg.n, cfg.depth)
    U = [Q.quantize(u, level_fmt[b.level - 1]).values for b, u in zip(oblocks, op.U)]
    V = [Q.quantize(v, level_fmt[b.level - 1]).values for b, v in zip(oblocks, op.V)]
    lb = T.leaves(cfg.n, cfg.depth)
    MV.matvec(cfg.n, oblocks, lb, op.leaves, U, V, X)        # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        y = MV.matvec(cfg.n, oblocks, lb, op.leaves, U, V, X)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    sec = (time.perf_counter() - t0) / reps
    return {"value": round(B_alg / sec / 1e9, 4), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} full products (n={cfg.n}, nrhs={X.shape[1]}) of the oracle's fp64 HODLR_MATVEC "
                      f"on the same stored operator, {sec * 1e3:.1f} ms each"}, y, U, V, oblocks, lb


BF16_PEAK_TFLOPS = 2500.0     # dense bf16 / fp16 MFMA


def main_lowp(args, torch, H, cfg, h, op, fmts, nrhs):
    """The product in a low working precision W on the workload's operator:
    one JSON line; the roofline is the expansion launch (the W leaf GEMM,
    HBM-bound below the W ridge of 2500 TFLOP/s / 8 TB/s ~ 312 flop/B)."""
    w = args.working
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
    CB = vb + n * nrhs * 2                               # contraction: V, X
    Xh = cfg.X(nrhs)
    from oracle import formats as OF
    Xw = OF.round_rne(w, Xh)
    X = H.colmajor_empty(n, nrhs, wdt, "cuda:0")
    X.copy_(torch.from_numpy(np.asfortranarray(Xw)).to(wdt))
    Y = H.colmajor_empty(n, nrhs, wdt, "cuda:0")
    ms = time_steps(lambda: h.matvec(X, Y), args.steps, args.warmup, torch)
    ph = time_phases(h, X, Y, 50, torch)
    cold = time_cold(lambda: h.matvec(X, Y), 10, torch)
    log(f"[bench] {w} working precision, nrhs={nrhs}: {ms * 1e3:.1f} us/step, {B / ms / 1e6:.1f} GB/s, "
        f"cold {cold * 1e3:.1f} us, kernels (us) {ph}")
    # the fp32/fp64 path on the same operator and X for the speedup
    xdt = torch.float32 if cfg.x_dtype == "fp32" else torch.float64
    Xf = H.colmajor_empty(n, nrhs, xdt, "cuda:0")
    Xf.copy_(torch.from_numpy(np.asfortranarray(Xw)).to(xdt))
    Yf = H.colmajor_empty(n, nrhs, xdt, "cuda:0")
    ms_full = time_steps(lambda: h.matvec(Xf, Yf), args.steps, args.warmup, torch)
    log(f"[bench] same product with {cfg.x_dtype} X: {ms_full * 1e3:.1f} us/step")
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
                 "mfma_tflops": round(LF / (exp_us * 1e-6) / 1e12, 2), "mean_launch_us": round(exp_us, 2)})
    value = B / (ms * 1e-3) / 1e9
    out = {
        "metric": "HODLR matvec GB/s & Gflop/s (% roofline); speedup mixed vs FP64 at fixed eps",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": w, "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description}; n={n}, depth {cfg.depth}, eps={cfg.eps:g}, "
                               f"formats {fmts}, {w} working precision, nrhs={nrhs}",
                   "n": n, "depth": cfg.depth, "eps": cfg.eps, "nrhs": nrhs, "formats": fmts,
                   "working_precision": w},
        "gflops": round(Fl / (ms * 1e-3) / 1e9, 2), "alg_bytes": int(B), "alg_flops": int(Fl),
        "cold_cache_gbs": round(B / (cold * 1e-3) / 1e9, 2),
        "speedup_vs_full_precision_path": round(ms_full / ms, 3),
        "kernels_us": {k: round(v, 2) for k, v in ph.items()},
        "roofline": roof,
    }
    if not args.no_cpu:
        # the oracle's W product on a column sample: timing and the tolerance check
        from oracle import lowp as LP
        from oracle import quantize as Q
        from oracle import tree as T
        from oracle import bounds as BD
        oblocks = T.blocks(n, cfg.depth)
        lb = T.leaves(n, cfg.depth)
        QU = [Q.quantize(u, fmts[b.level - 1]) for b, u in zip(oblocks, op.U)]
        QV = [Q.quantize(v, fmts[b.level - 1]) for b, v in zip(oblocks, op.V)]
        k = min(nrhs, 4)
        t0 = time.perf_counter()
        prod = LP.matvec_lowp(n, oblocks, lb, op.leaves, QU, QV, Xw[:, :k], w)
        sec = time.perf_counter() - t0
        Bk = leaf_w + inf["factor_bytes"] + inf["scale_bytes"] + n * k * 2 * 2
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            threads = 1
        out["cpu_baseline"] = {"value": round(Bk / sec / 1e9, 4), "unit": "GB/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"one {w} product of the oracle (n={n}, nrhs={k}), {sec * 1e3:.1f} ms"}
        h.matvec(X, Y)
        torch.cuda.synchronize()
        yg = Y[:, :k].float().cpu().double().numpy()
        M = BD.chain_length(oblocks, op.ranks, [m for _, m in lb], cfg.depth)
        tol = LP.tolerance(prod, w, M, max(b.ncols for b in oblocks))
        err = np.abs(yg - prod.y)
        out["check"] = {"max_err_over_tol": float((err / np.where(tol > 0, tol, 1)).max()),
                        "rel_err_vs_oracle": float(np.linalg.norm(err) / np.linalg.norm(prod.y))}
        if (err > tol).any():
            log(f"[bench] {int((err > tol).sum())} entries outside the tolerance")
    print(json.dumps(out), flush=True)


def build_batch(name):
    """Compress a batched workload over the library's partitions (host, untimed)."""
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
    return specs, parts, ops


def main_batch(args, torch, H):
    """The batched workload: all operators in one hodlr_matvec_batched call."""
    from hodlr_inputs import batch as BT
    specs, parts, cops = args.batch_ops
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
        B = F = 0
        for h, sp, xb in zip(hs, specs, xbs):
            w = work(h, sp.n, sp.nrhs, xb)
            B += w[0]
            F += w[1]
        return B, F

    B, F = totals()
    ms = time_steps(fn, args.steps, args.warmup, torch)
    if args.profile_run:
        print(json.dumps({"profile_run": True, "us_per_step": ms * 1e3}), flush=True)
        return
    cold = time_cold(fn, 5, torch)
    log(f"[bench] batch: {ms * 1e3:.1f} us/step, {B / ms / 1e6:.1f} GB/s, cold {cold * 1e3:.1f} us")
    fm = [[lv[0] for lv in h.levels()] for h in hs]
    acc = [h.info()["acc_dtype"] for h in hs]
    # uniform fp64 on the same GPU (same ranks), then back
    for h, sp in zip(hs, specs):
        h.set_level_precisions(["fp64"] * sp.depth, H.ACC_FP64)
    B64, _ = totals()
    ms64 = time_steps(fn, args.steps, args.warmup, torch)
    for h, sp, c in zip(hs, specs, cops):
        h.assign_precision(sp.eps, BT.ALLOWED, np.concatenate([[c.norm2_all], c.norm2_blocks]))
    log(f"[bench] uniform fp64 batch: {ms64 * 1e3:.1f} us/step")
    value = B / (ms * 1e-3) / 1e9
    fmt_count = {}
    for f in fm:
        for x in f:
            fmt_count[x] = fmt_count.get(x, 0) + 1
    out = {
        "metric": "HODLR matvec GB/s & Gflop/s (% roofline); speedup mixed vs FP64 at fixed eps",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {len(specs)} independent operators, n log-uniform, kernels "
                               f"1/(r+1e-3), exp(-r), exp(-r^2/0.08) in 1D/2D, eps 1e-4/1e-6/1e-8, nrhs 1/8/32, "
                               f"one hodlr_matvec_batched call", "operators": len(specs),
                   "sum_n": int(sum(sp.n for sp in specs)), "level_formats": fmt_count,
                   "fp64_accumulation_ops": int(sum(a == "fp64" for a in acc))},
        "gflops": round(F / (ms * 1e-3) / 1e9, 2), "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "alg_bytes": int(B), "alg_flops": int(F),
        "cold_cache_gbs": round(B / (cold * 1e-3) / 1e9, 2),
        "speedup_vs_fp64": round(ms64 / ms, 3), "fp64_gbs": round(B64 / (ms64 * 1e-3) / 1e9, 2),
        "roofline": {"bound": "hbm", "kernel": "whole batch (persistent launches of every kernel variant)",
                     "achieved": round(value, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(value / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": int(B), "mean_launch_us": round(ms * 1e3, 2)},
    }
    if not args.no_cpu:
        from oracle import bounds as BD
        from oracle import matvec as MV
        from oracle import quantize as Q
        from oracle import tree as T
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            threads = 1
        fn()
        torch.cuda.synchronize()
        worst, done_b, t_cpu, k = 0.0, 0, 0.0, 0
        for k, (h, sp, c, xb) in enumerate(zip(hs, specs, cops, xbs)):
            blocks = T.blocks(sp.n, sp.depth)
            lb = T.leaves(sp.n, sp.depth)
            U = [Q.quantize(u, fm[k][b.level - 1]).values for b, u in zip(blocks, c.U)]
            V = [Q.quantize(v, fm[k][b.level - 1]).values for b, v in zip(blocks, c.V)]
            X = sp.X()
            t0 = time.perf_counter()
            y = MV.matvec(sp.n, blocks, lb, c.leaves, U, V, X)
            t_cpu += time.perf_counter() - t0
            done_b += work(h, sp.n, sp.nrhs, xb)[0]
            z = MV.matvec_abs(sp.n, blocks, lb, c.leaves, U, V, X)
            M = BD.chain_length(blocks, c.ranks, [m for _, m in lb], sp.depth)
            u_acc = 2.0 ** -24 if acc[k] == "fp32" else 2.0 ** -53
            tau = BD.tolerance_prob(z, y, M, u_acc, 2.0 ** -24 if xb == 4 else 2.0 ** -53)
            err = np.abs(Ys[k].cpu().double().numpy() - y)
            worst = max(worst, float((err / tau).max()))
            if t_cpu >= 12.0:
                break
        out["cpu_baseline"] = {"value": round(done_b / t_cpu / 1e9, 4), "unit": "GB/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"the oracle's fp64 HODLR_MATVEC of the first {k + 1} operators of the "
                                         f"batch (same stored operators and X), {t_cpu:.1f} s in total"}
        out["check"] = {"max_err_over_tau_prob": worst, "operators_checked": k + 1}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nrhs", type=int, default=None, help="default: the workload's first nrhs")
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the timed products (for running under rocprofv3)")
    ap.add_argument("--working", choices=["bf16", "fp16"], default=None,
                    help="time the product in this low working precision (X, Y, operands in W; fp32 sums)")
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
    from hodlr_inputs import configs as CF
    from hodlr_inputs.batch import BATCHES

    batch_ops = None
    if args.workload in BATCHES and not args.copy_calibration:
        # host-side, in spawned processes, before anything touches the GPU
        batch_ops = build_batch(args.workload)
    args.batch_ops = batch_ops

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
    if args.workload in BATCHES:
        return main_batch(args, torch, H)
    dev = torch.device("cuda:0")
    cfg = CF.get(args.workload)
    nrhs0 = args.nrhs if args.nrhs is not None else cfg.nrhs[0]
    P, blocks, leaves, op = build_operator(cfg, H)
    norms2 = np.concatenate([[op.norm2_all], op.norm2_blocks])
    t = time.time()
    h = H.Operator(cfg.n, cfg.depth, op.leaves, op.U, op.V, device=0)
    h.assign_precision(cfg.eps, cfg.allowed, norms2)
    fmts = [lv[0] for lv in h.levels()]
    acc = h.info()["acc_dtype"]
    log(f"[bench] operator on GPU in {time.time() - t:.1f}s; formats {fmts}; acc {acc}")

    if args.working:
        return main_lowp(args, torch, H, cfg, h, op, fmts, nrhs0)
    xdt = torch.float32 if cfg.x_dtype == "fp32" else torch.float64
    xb = 4 if cfg.x_dtype == "fp32" else 8
    nrhs_list = [nrhs0] if args.profile_run else [nrhs0] + [k for k in cfg.nrhs if k != nrhs0]
    Xh = cfg.X(max(nrhs_list))
    results = {}
    for nrhs in nrhs_list:
        X = H.colmajor_empty(cfg.n, nrhs, xdt, dev)
        X.copy_(torch.from_numpy(np.asfortranarray(Xh[:, :nrhs])).to(xdt))
        Y = H.colmajor_empty(cfg.n, nrhs, xdt, dev)
        B, Fl, EB, CB, LF = work(h, cfg.n, nrhs, xb)
        ms = time_steps(lambda: h.matvec(X, Y), args.steps, args.warmup, torch)
        ph = time_phases(h, X, Y, 50, torch)
        cold = time_cold(lambda: h.matvec(X, Y), 10, torch)
        results[nrhs] = dict(ms=ms, phases=ph, B=B, F=Fl, EB=EB, CB=CB, LF=LF, cold_ms=cold, X=X, Y=Y)
        log(f"[bench] nrhs={nrhs}: {ms * 1e3:.1f} us/step, {B / ms / 1e6:.1f} GB/s, {Fl / ms / 1e9:.2f} Tflop/s, "
            f"cold {cold * 1e3:.1f} us, kernels (us) {ph}")
    if args.profile_run:
        print(json.dumps({"profile_run": True, "us_per_step": results[nrhs0]["ms"] * 1e3}), flush=True)
        return

    # uniform-fp64 product on the same GPU, same ranks
    r = results[nrhs0]
    h.set_level_precisions(["fp64"] * cfg.depth, H.ACC_FP64)
    ms64 = time_steps(lambda: h.matvec(r["X"], r["Y"]), args.steps, args.warmup, torch)
    B64 = work(h, cfg.n, nrhs0, xb)[0]
    h.assign_precision(cfg.eps, cfg.allowed, norms2)
    log(f"[bench] uniform fp64: {ms64 * 1e3:.1f} us/step")

    exp_us = r["phases"]["expand"]
    con_us = r["phases"].get("contract", 0.0)
    wide = nrhs0 >= 8
    traffic = traffic_c = None
    tr = read_traffic(cfg.name, nrhs0)
    if tr.get("kernel_sha") == kernel_hash("wide" if wide else "wave") and tr.get("workload") == cfg.name and \
            tr.get("nrhs") == str(nrhs0):
        traffic = int(tr.get("second_launch_bytes", 0)) or None
        traffic_c = int(tr.get("first_launch_bytes", 0)) or None
    value = r["B"] / (r["ms"] * 1e-3) / 1e9
    exp_gbs = r["EB"] / (exp_us * 1e-6) / 1e9
    con_gbs = r["CB"] / (con_us * 1e-6) / 1e9 if con_us else 0.0
    # the matrix-core expansion is MFMA-bound only above the fp64 ridge
    # (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B); below it the HBM roofline applies
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if wide and r["LF"] / r["EB"] >= ridge:
        # matrix-core path: the fp64 leaf GEMM dominates the expansion's work
        achieved = r["LF"] / (exp_us * 1e-6) / 1e12
        roof = {"bound": "mfma", "kernel": "k_expand_w (fp64 MFMA leaf GEMM + low-rank MFMA, writes Y)",
                "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "alg_flops_per_launch": int(r["LF"]), "alg_bytes_per_launch": int(r["EB"]),
                "hbm_gbs": round(exp_gbs, 2), "mean_launch_us": round(exp_us, 2)}
    elif wide:
        roof = {"bound": "hbm", "kernel": "k_expand_w (fp64 MFMA leaf GEMM + low-rank MFMA, writes Y)",
                "achieved": round(exp_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(exp_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": int(r["EB"]), "intensity_flop_per_byte": round(r["LF"] / r["EB"], 3),
                "mean_launch_us": round(exp_us, 2)}
    else:
        # wave path: the first launch (contraction items + fp64 leaf GEMV tiles) moves most bytes
        roof = {"bound": "hbm", "kernel": "k_phase1 (contraction items + fp64 leaf GEMV tiles)",
                "achieved": round(con_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(con_gbs / HBM_PEAK_GBS, 4), "traffic": traffic_c,
                "alg_bytes_per_launch": int(r["CB"]), "mean_launch_us": round(con_us, 2)}
    out = {
        "metric": "HODLR matvec GB/s & Gflop/s (% roofline); speedup mixed vs FP64 at fixed eps",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if xb == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description}; n={cfg.n}, leaf {-(-cfg.n >> cfg.depth)}, "
                               f"depth {cfg.depth}, eps={cfg.eps:g}, formats {fmts}, {cfg.x_dtype} X nrhs={nrhs0}",
                   "n": cfg.n, "depth": cfg.depth, "eps": cfg.eps, "nrhs": nrhs0, "formats": fmts,
                   "accumulation": acc},
        "gflops": round(r["F"] / (r["ms"] * 1e-3) / 1e9, 2),
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "alg_bytes": int(r["B"]),
        "alg_flops": int(r["F"]),
        "cold_cache_gbs": round(r["B"] / (r["cold_ms"] * 1e-3) / 1e9, 2),
        "speedup_vs_fp64": round(ms64 / r["ms"], 3),
        "fp64_gbs": round(B64 / (ms64 * 1e-3) / 1e9, 2),
        "kernels_us": {k: round(v, 2) for k, v in r["phases"].items()},
        "roofline": roof,
        "launches": {
            "first": {"kernel": "k_contract_w" if wide else "k_phase1", "alg_bytes": int(r["CB"]),
                      "mean_us": round(con_us, 2), "achieved_gbs": round(con_gbs, 2), "traffic": traffic_c},
            "second": {"kernel": "k_expand_w" if wide else "k_expand", "alg_bytes": int(r["EB"]),
                       "mean_us": round(exp_us, 2), "achieved_gbs": round(exp_gbs, 2), "traffic": traffic}},
    }
    for k in nrhs_list[1:]:
        rk = results[k]
        out[f"nrhs{k}"] = {"gbs": round(rk["B"] / (rk["ms"] * 1e-3) / 1e9, 2),
                           "gflops": round(rk["F"] / (rk["ms"] * 1e-3) / 1e9, 2),
                           "ms_per_step": round(rk["ms"], 5),
                           "kernels_us": {q: round(v, 2) for q, v in rk["phases"].items()}}
        if k >= 8 and "expand" in rk["phases"]:
            out[f"nrhs{k}"]["leaf_fp64_mfma_tflops"] = round(rk["LF"] / (rk["phases"]["expand"] * 1e-6) / 1e12, 3)
    if not args.no_cpu:
        Xc = Xh[:, :nrhs0]
        cb, y_ora, U, V, oblocks, lb = cpu_baseline(cfg, blocks, leaves, op, fmts, r["B"], Xc)
        out["cpu_baseline"] = cb
        # accuracy of the timed product against the oracle
        from oracle import bounds as BD
        from oracle import matvec as MV
        h.matvec(r["X"], r["Y"])
        torch.cuda.synchronize()
        yg = r["Y"].cpu().double().numpy()
        z = MV.matvec_abs(cfg.n, oblocks, lb, op.leaves, U, V, Xc)
        M = BD.chain_length(oblocks, op.ranks, [m for _, m in lb], cfg.depth)
        u_acc = 2.0 ** -24 if acc == "fp32" else 2.0 ** -53
        tau = BD.tolerance_prob(z, y_ora, M, u_acc, 2.0 ** -24 if xb == 4 else 2.0 ** -53)
        err = np.abs(yg - y_ora)
        out["check"] = {"max_err_over_tau_prob": float((err / tau).max()),
                        "rel_err_vs_oracle": float(np.linalg.norm(err) / np.linalg.norm(y_ora))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
