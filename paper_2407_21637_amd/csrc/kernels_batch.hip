// HIP kernels (gfx950) of the batched HODLR product: persistent launches
// over the work lists of many operators, running the same device code as
// the single-operator launches (wave_path.h, wide_path.h), so results are
// bit-identical to single calls.  One translation unit of the library (see
// kernels.hip).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hodlr_internal.h"

#include "dev_common.h"
#include "wave_path.h"
#include "wide_path.h"

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
__global__ __launch_bounds__(kExpandThreads) void kb_expand(const BatchOp* __restrict__ ops,
                                                          const WorkItem* __restrict__ w, int nw) {
    extern __shared__ double smem_d[];
    __shared__ int s_off[2 * (kMaxDepth + 1)];
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_expand<XT, AT, RG, RPL>(o.kp, wi.idx, static_cast<XT*>(o.Y), o.ldy, o.nrhs,
                                    reinterpret_cast<unsigned char*>(smem_d), s_off);
        __syncthreads();
    }
}

template <typename XT, typename AT, int NT, int STACK>
__global__ __launch_bounds__(kThreads) void kb_contract_w(const BatchOp* __restrict__ ops,
                                                          const WorkItem* __restrict__ w, int nw) {
    extern __shared__ double smem_d[];
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_contract_w<XT, AT, NT, STACK>(o.kp, wi.idx, wi.y, static_cast<const XT*>(o.Xc), o.ldc, o.nrhs, smem_d);
        __syncthreads();
    }
}

template <typename AT, bool STACK>
__global__ __launch_bounds__(256) void kb_reduce_w(const BatchOp* __restrict__ ops, const WorkItem* __restrict__ w,
                                                   int nw) {
    for (int i = blockIdx.x; i < nw; i += gridDim.x) {
        const WorkItem wi = w[i];
        const BatchOp o = ops[wi.op];                  // uniform: the step's operator
        run_reduce_w<AT, STACK>(o.kp, wi.idx, wi.y, o.nrhs);
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
        hipLaunchKernelGGL((kb_expand<XT, AT, RG, kRPL>), dim3(g.grid[3]), dim3(kExpandThreads), size_t(g.lds_expand),
                           s, g.ops, g.expand, g.n_expand);
    return hipGetLastError();
}

template <typename XT, typename AT, int NT>
hipError_t batch_wide(const BatchGroup& g, hipStream_t s) {
    constexpr int NTC = NT > 4 ? 4 : NT;                // as the single-operator launch
    if (g.n_padx)
        hipLaunchKernelGGL((kb_padx<XT>), dim3(g.grid[0]), dim3(256), 0, s, g.ops, g.padx, g.n_padx);
    if (g.n_contract) {
        if (g.stacked > 2)
            hipLaunchKernelGGL((kb_contract_w<XT, AT, NTC, 4>), dim3(g.grid[1]), dim3(kThreads),
                               size_t(g.lds_contract), s, g.ops, g.contract, g.n_contract);
        else if (g.stacked)
            hipLaunchKernelGGL((kb_contract_w<XT, AT, NTC, 2>), dim3(g.grid[1]), dim3(kThreads),
                               size_t(g.lds_contract), s, g.ops, g.contract, g.n_contract);
        else
            hipLaunchKernelGGL((kb_contract_w<XT, AT, NTC, 0>), dim3(g.grid[1]), dim3(kThreads),
                               size_t(g.lds_contract), s, g.ops, g.contract, g.n_contract);
    }
    if (g.n_reduce) {
        if (g.stacked)
            hipLaunchKernelGGL((kb_reduce_w<AT, true>), dim3(g.grid[2]), dim3(256), 0, s, g.ops, g.reduce, g.n_reduce);
        else
            hipLaunchKernelGGL((kb_reduce_w<AT, false>), dim3(g.grid[2]), dim3(256), 0, s, g.ops, g.reduce, g.n_reduce);
    }
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
