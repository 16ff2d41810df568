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
// wide_path.h).
//
// Layout of the device sources: dev_common.h (codecs, wave sums, coherent
// accesses), wave_path.h, wide_path.h, lowp_path.h; the translation units
// kernels.hip (single-operator launches in fp64/fp32), kernels_lowp.hip
// (low working precision), kernels_batch.hip (batched launches), built in
// parallel.
//
// Stored codes are converted in registers (Sect. 3.3: low-precision
// storage cast to the working precision on the fly).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "hodlr_internal.h"

#include "dev_common.h"
#include "wave_path.h"
#include "wide_path.h"

namespace hodlr {

// ---------------------------------------------------------------------------
// scratch of the allocation-free entry point
// ---------------------------------------------------------------------------
// One array per GPU, alive until the process ends.  In host code its name
// stands for a host-side shadow, not for device memory: host code uses only
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

__global__ __launch_bounds__(256) void k_zero_words(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) p[i] = 0;
}

}  // namespace

int scratch_address(int device, void** ptr) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return int(hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return int(e);
        if (!p) return int(hipErrorInvalidSymbol);
        addr[device] = p;
    }
    *ptr = addr[device];
    return 0;
}

int launch_zero_words(int32_t* p, int64_t n, void* stream) {
    if (n <= 0) return 0;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_words, dim3(unsigned(blocks < 1024 ? blocks : 1024)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p, n);
    return int(hipGetLastError());
}

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

}  // namespace hodlr
