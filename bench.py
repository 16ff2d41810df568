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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_expand_c2_nrhs1.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2407_21637_amd", "csrc", "kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def read_traffic():
    """key: value lines of the counter summary (HBM bytes per launch)."""
    out = {}
    if os.path.exists(TRAFFIC_FILE):
        for line in open(TRAFFIC_FILE):
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
    P = cfg.points()
    t = time.time()
    op = compress(cfg.kernel, P, blocks, leaves, cfg.eps, cfg.rule)
    log(f"[bench] compressed {cfg.name}: n={cfg.n} depth={cfg.depth} in {time.time() - t:.1f}s")
    return P, blocks, leaves, op


SBYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2, "e4m3": 1, "e5m2": 1}


def work(h, n, nrhs, xy_bytes):
    """Algorithmic bytes and flops of one product; bytes of the expansion and
    contraction launches; fp64 flops of the leaf products."""
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
    expand = inf["leaf_bytes"] + ub + n * nrhs * 2 * xy_bytes
    contract = vb + n * nrhs * xy_bytes
    leaf_flops = 2 * nrhs * (inf["leaf_bytes"] // 8)
    return B, F, expand, contract, leaf_flops


def time_steps(h, X, Y, steps, warmup, torch):
    """ms per product: K products captured in one HIP graph, replayed."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(warmup, 1)):     # also sizes this stream's workspace
            h.matvec(X, Y)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(steps):
            h.matvec(X, Y)
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


def time_cold(h, X, Y, reps, torch):
    """Per-product time with the caches flushed (1 GiB written) before each."""
    flush = torch.empty(1 << 28, dtype=torch.float32, device=X.device)
    out = []
    for _ in range(reps):
        flush.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        h.matvec(X, Y)
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device-to-device copy 5 times (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the product shards by subtree with a "
                                   "small exchange of T (see DESIGN.md), which is not implemented; "
                                   "run with --gpus 1"}), flush=True)
        sys.exit(2)

    import torch
    import paper_2407_21637_amd as H
    from hodlr_inputs import configs as CF

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
        ms = time_steps(h, X, Y, args.steps, args.warmup, torch)
        ph = time_phases(h, X, Y, 50, torch)
        cold = time_cold(h, X, Y, 10, torch)
        results[nrhs] = dict(ms=ms, phases=ph, B=B, F=Fl, EB=EB, CB=CB, LF=LF, cold_ms=cold, X=X, Y=Y)
        log(f"[bench] nrhs={nrhs}: {ms * 1e3:.1f} us/step, {B / ms / 1e6:.1f} GB/s, {Fl / ms / 1e9:.2f} Tflop/s, "
            f"cold {cold * 1e3:.1f} us, kernels (us) {ph}")
    if args.profile_run:
        print(json.dumps({"profile_run": True, "us_per_step": results[nrhs0]["ms"] * 1e3}), flush=True)
        return

    # uniform-fp64 product on the same GPU, same ranks
    r = results[nrhs0]
    h.set_level_precisions(["fp64"] * cfg.depth, H.ACC_FP64)
    ms64 = time_steps(h, r["X"], r["Y"], args.steps, args.warmup, torch)
    B64 = work(h, cfg.n, nrhs0, xb)[0]
    h.assign_precision(cfg.eps, cfg.allowed, norms2)
    log(f"[bench] uniform fp64: {ms64 * 1e3:.1f} us/step")

    exp_us = r["phases"]["expand"]
    con_us = r["phases"].get("contract", 0.0)
    traffic = traffic_c = None
    tr = read_traffic()
    if tr.get("kernel_sha") == kernel_hash() and tr.get("workload") == cfg.name and \
            tr.get("nrhs") == str(nrhs0) and "k_expand_bytes_per_launch" in tr:
        traffic = int(tr["k_expand_bytes_per_launch"])
        traffic_c = int(tr.get("k_contract_bytes_per_launch", 0)) or None
    value = r["B"] / (r["ms"] * 1e-3) / 1e9
    wide = nrhs0 >= 16
    exp_gbs = r["EB"] / (exp_us * 1e-6) / 1e9
    if wide:
        # matrix-core path: the fp64 leaf GEMM dominates the expansion's work
        achieved = r["LF"] / (exp_us * 1e-6) / 1e12
        roof = {"bound": "mfma", "kernel": "k_expand_w (fp64 MFMA leaf GEMM + low-rank MFMA, writes Y)",
                "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "alg_flops_per_launch": int(r["LF"]), "alg_bytes_per_launch": int(r["EB"]),
                "hbm_gbs": round(exp_gbs, 2), "mean_launch_us": round(exp_us, 2)}
    else:
        roof = {"bound": "hbm", "kernel": "k_expand (fp64 leaf GEMV + expansion, writes Y)",
                "achieved": round(exp_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(exp_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": int(r["EB"]), "mean_launch_us": round(exp_us, 2)}
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
        "contract_kernel": {"alg_bytes_per_launch": int(r["CB"]), "mean_launch_us": round(con_us, 2),
                            "achieved_gbs": round(r["CB"] / (con_us * 1e-6) / 1e9, 2) if con_us else None,
                            "traffic": traffic_c},
    }
    for k in nrhs_list[1:]:
        rk = results[k]
        out[f"nrhs{k}"] = {"gbs": round(rk["B"] / (rk["ms"] * 1e-3) / 1e9, 2),
                           "gflops": round(rk["F"] / (rk["ms"] * 1e-3) / 1e9, 2),
                           "ms_per_step": round(rk["ms"], 5),
                           "kernels_us": {q: round(v, 2) for q, v in rk["phases"].items()}}
        if k >= 16 and "expand" in rk["phases"]:
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
