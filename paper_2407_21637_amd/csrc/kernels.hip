// HIP kernels (gfx950) of the HODLR matrix-vector product
// Y = A_H X, following Alg. "HODLR_MATVEC" of Carson, Chen, Liu,
// "Mixed Precision HODLR Matrices" (arXiv 2407.21637):
//
//   b <- 0;  b_rows(b) += U_b (V_b^T x_cols(b)) for every off-diagonal block;
//   b_i += D_i x_i for every leaf.
//
// Wave path (nrhs < kWideMin = 8), two launches per product; one kernel boundary is
// the only synchronisation between phases (no work queue, no spin-waits):
//
//  * k_phase1: workgroups [0, ncitems) take contraction items, the others
//    the leaf tiles.  A contraction item (rows [r0, r0+nr) of the V panel of
//    one block) stores its partial sums of T_b = V_b^T X and counts itself
//    in the block's arrival counter; the last item of a block to arrive
//    adds the partials in item order (deterministic, no float atomics),
//    applies the column scales, stores T_b and clears the counter for the
//    next launch.  A leaf tile (64*RPL padded rows of one leaf) computes
//    W = D_i X_i in fp64.  Neither waits for the other, so the V and D
//    streams share the first launch.
//  * k_expand, one workgroup per tile: Y rows = W + U_b T_b over the tile's
//    depth ancestor blocks (each wave takes whole levels), the waves'
//    partial rows are added in LDS and Y is written once.
//
// Matrix-core path (nrhs >= 8): k_contract_w, k_reduce_w, k_expand_w (see
// wide_path.h).  Batched products run the same device code from persistent
// kernels (section "batched products" below).
//
// Low working precision (X and Y in bf16 or fp16): k_contract_lp,
// k_reduce_lp, k_expand_lp (lowp_path.h).
//
// Layout of the sources: dev_common.h (codecs, wave sums, coherent
// accesses), wave_path.h, wide_path.h, lowp_path.h, and this file (batched
// kernels and the launch entry points), one translation unit.
//
// Stored codes are converted in registers (Sect. 3.3: low-precision
// storage cast to the working precision on the fly).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hodlr_internal.h"

#include "dev_common.h"
#include "wave_path.h"
#include "wide_path.h"
#include "lowp_path.h"

namespace hodlr {
namespace {

// ---------------------------------------------------------------------------
// batched products: persistent kernels over a work list of many operators
// ---------------------------------------------------------------------------
// Each workgroup walks the list with stride gridDim.x (the list is sorted by
// the planner, longest first by default); every step runs the same device
// code as the single-operator launch for one (operator, unit) pair.  A
// barrier separates steps that use LDS.
template <typename XT>
__global__ __launch_bounds__(256) void kb_padx(const BatchOp* __restrict__ ops, const WorkItem* __restrict__ w,
                                               int nw) {
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        padx_leaf<XT>(o.kp, wi.idx, static_cast<const XT*>(o.X), o.ldx, o.nrhs);
    }
}

// wave-path first launch over many operators: idx is a contraction item
// (y == 0) or a leaf tile (y == 1) of operator op
template <typename XT, typename AT, int RG, int RPL>
__global__ __launch_bounds__(kThreads, HODLR_CONTRACT_MINW) void kb_phase1(const BatchOp* __restrict__ ops,
                                                                          const WorkItem* __restrict__ w, int nw,
                                                                          int stage_cap) {
    extern __shared__ double smem_d[];
    __shared__ int s_flag;
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_phase1<XT, AT, RG, RPL>(o.kp, wi.y ? o.kp.ncitems + wi.idx : wi.idx, static_cast<const XT*>(o.Xc), o.ldc,
                                    static_cast<const XT*>(o.X), o.ldx, o.nrhs, stage_cap,
                                    reinterpret_cast<unsigned char*>(smem_d), &s_flag);
        __syncthreads();
    }
}

template <typename XT, typename AT, int RG, int RPL>
__global__ __launch_bounds__(kThreads, HODLR_EXPAND_MINW) void kb_expand(const BatchOp* __restrict__ ops,
                                                                        const WorkItem* __restrict__ w, int nw) {
    extern __shared__ double smem_d[];
    __shared__ int s_off[kMaxDepth + 1];
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_expand<XT, AT, RG, RPL>(o.kp, wi.idx, static_cast<XT*>(o.Y), o.ldy, o.nrhs,
                                    reinterpret_cast<unsigned char*>(smem_d), s_off);
        __syncthreads();
    }
}

template <typename XT, typename AT, int NT>
__global__ __launch_bounds__(kThreads) void kb_contract_w(const BatchOp* __restrict__ ops,
                                                          const WorkItem* __restrict__ w, int nw) {
    extern __shared__ double smem_d[];
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_contract_w<XT, AT, NT>(o.kp, wi.idx, wi.y, static_cast<const XT*>(o.Xc), o.ldc, o.nrhs, smem_d);
        __syncthreads();
    }
}

template <typename AT>
__global__ __launch_bounds__(256) void kb_reduce_w(const BatchOp* __restrict__ ops, const WorkItem* __restrict__ w,
                                                   int nw) {
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_reduce_w<AT>(o.kp, wi.idx, wi.y, o.nrhs);
    }
}

template <typename XT, typename AT, int NT>
__global__ __launch_bounds__(kThreads) void kb_expand_w(const BatchOp* __restrict__ ops,
                                                        const WorkItem* __restrict__ w, int nw, int lds_bytes,
                                                        int jc) {
    extern __shared__ double smem_d[];
    __shared__ int s_off[kMaxDepth + 2];
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_expand_w<XT, AT, NT>(o.kp, wi.idx, wi.y, static_cast<const XT*>(o.Xc), o.ldc, static_cast<XT*>(o.Y),
                                 o.ldy, o.nrhs, lds_bytes, jc, smem_d, s_off);
        __syncthreads();
    }
}

template <typename XT, typename AT, int RG>
hipError_t batch_narrow(const BatchGroup& g, hipStream_t s) {
    if (g.n_padx)
        hipLaunchKernelGGL((kb_padx<XT>), dim3(g.grid[0]), dim3(256), 0, s, g.ops, g.padx, g.n_padx);
    if (g.n_contract)
        hipLaunchKernelGGL((kb_phase1<XT, AT, RG, kRPL>), dim3(g.grid[1]), dim3(kThreads), size_t(g.lds_contract), s,
                           g.ops, g.contract, g.n_contract, g.stage_cap);
    if (g.n_expand)
        hipLaunchKernelGGL((kb_expand<XT, AT, RG, kRPL>), dim3(g.grid[3]), dim3(kThreads), size_t(g.lds_expand), s,
                           g.ops, g.expand, g.n_expand);
    return hipGetLastError();
}

template <typename XT, typename AT, int NT>
hipError_t batch_wide(const BatchGroup& g, hipStream_t s) {
    constexpr int NTC = NT > 4 ? 4 : NT;                // as the single-operator launch
    if (g.n_padx)
        hipLaunchKernelGGL((kb_padx<XT>), dim3(g.grid[0]), dim3(256), 0, s, g.ops, g.padx, g.n_padx);
    if (g.n_contract)
        hipLaunchKernelGGL((kb_contract_w<XT, AT, NTC>), dim3(g.grid[1]), dim3(kThreads), size_t(g.lds_contract), s,
                           g.ops, g.contract, g.n_contract);
    if (g.n_reduce)
        hipLaunchKernelGGL((kb_reduce_w<AT>), dim3(g.grid[2]), dim3(256), 0, s, g.ops, g.reduce, g.n_reduce);
    if (g.n_expand)
        hipLaunchKernelGGL((kb_expand_w<XT, AT, NT>), dim3(g.grid[3]), dim3(kThreads), size_t(g.lds_expand), s,
                           g.ops, g.expand, g.n_expand, int(g.lds_expand), g.jc);
    return hipGetLastError();
}

template <typename XT, typename AT>
hipError_t batch_typed(const BatchGroup& g, hipStream_t s) {
    if (!g.wide) {
        switch (g.rg) {
            case 1: return batch_narrow<XT, AT, 1>(g, s);
            case 2: return batch_narrow<XT, AT, 2>(g, s);
            default: return batch_narrow<XT, AT, 4>(g, s);
        }
    }
    switch (g.rg) {
        case 1: return batch_wide<XT, AT, 1>(g, s);
        case 2: return batch_wide<XT, AT, 2>(g, s);
        default: return batch_wide<XT, AT, 4>(g, s);
    }
}

}  // namespace

int launch_matvec(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs,
                  bool xy_double, bool acc_double, void* stream, void* const* events, bool* ran) {
    const Timer tm{events, ran, static_cast<hipStream_t>(stream)};
    hipError_t e;
    if (nrhs >= kWideMin) {
        if (xy_double)
            e = acc_double ? launch_wide<double, double>(kp, X, ldx, Y, ldy, nrhs, tm)
                           : launch_wide<double, float>(kp, X, ldx, Y, ldy, nrhs, tm);
        else
            e = acc_double ? launch_wide<float, double>(kp, X, ldx, Y, ldy, nrhs, tm)
                           : launch_wide<float, float>(kp, X, ldx, Y, ldy, nrhs, tm);
    } else if (xy_double) {
        e = acc_double ? launch_rg<double, double>(kp, X, ldx, Y, ldy, nrhs, tm)
                       : launch_rg<double, float>(kp, X, ldx, Y, ldy, nrhs, tm);
    } else {
        e = acc_double ? launch_rg<float, double>(kp, X, ldx, Y, ldy, nrhs, tm)
                       : launch_rg<float, float>(kp, X, ldx, Y, ldy, nrhs, tm);
    }
    return int(e);
}


int launch_matvec_lp(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, int w,
                     void* stream, void* const* events, bool* ran) {
    const Timer tm{events, ran, static_cast<hipStream_t>(stream)};
    const hipError_t e = w == 0 ? launch_lp<__bf16>(kp, X, ldx, Y, ldy, nrhs, tm)
                                : launch_lp<_Float16>(kp, X, ldx, Y, ldy, nrhs, tm);
    return int(e);
}

int launch_build_aug(const KParams& kp, int w, void* stream) {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    return int(w == 0 ? launch_build_aug_w<__bf16>(kp, s) : launch_build_aug_w<_Float16>(kp, s));
}

int plan_launch(const KParams& kp, const void* X, int64_t ldx, int nrhs, bool xy_double, bool acc_double,
                OpLaunch* out) {
    OpLaunch o{};
    const size_t acc_bytes = acc_double ? 8 : 4;
    const size_t xbytes = xy_double ? 8 : 4;
    if (nrhs < kWideMin) {
        int rg = nrhs == 1 ? 1 : nrhs == 2 ? 2 : 4;
        auto fits = [&](int g) { return lds_expand(kp, g, acc_bytes) <= kMaxLds && lds_phase1(kp, g) <= kMaxLds; };
        while (rg > 1 && !fits(rg)) rg /= 2;
        if (!fits(rg)) return int(hipErrorInvalidConfiguration);
        o.wide = 0;
        o.rg = rg;
        o.padx = kp.padded && kp.ncitems > 0;
        o.stage_cap = stage_cap(kp, rg);
        o.lds_contract = int64_t(lds_phase1(kp, rg));
        o.lds_expand = int64_t(lds_expand(kp, rg, acc_bytes));
    } else {
        const int nt = nrhs <= 16 ? 1 : nrhs <= 32 ? 2 : 4;
        const int ntc = nt;
        const int cw = 16 * nt;
        const bool aligned = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((ldx * int64_t(xbytes)) % 16 == 0);
        o.wide = 1;
        o.rg = nt;
        o.ntc = ntc;
        o.padx = kp.padded || !aligned;
        o.lds_contract = int64_t(kWaves) * ntc * 256 * 8;
        int jc = 0;
        int64_t lds = 0;
        if (!wide_lds(kp, cw, xbytes, &jc, &lds)) return int(hipErrorInvalidConfiguration);
        o.jc = jc;
        o.lds_expand = lds;
        o.gy_contract = (nrhs + 16 * ntc - 1) / (16 * ntc);
        o.gy_expand = (nrhs + cw - 1) / cw;
    }
    *out = o;
    return 0;
}

int launch_batch_group(const BatchGroup& g, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (g.xy_double)
        e = g.acc_double ? batch_typed<double, double>(g, s) : batch_typed<double, float>(g, s);
    else
        e = g.acc_double ? batch_typed<float, double>(g, s) : batch_typed<float, float>(g, s);
    return int(e);
}

}  // namespace hodlr
