// HIP kernel of the LU solves (Sect. 3.4, Alg. "HODLR_LU"): the solve
// applies the inverse factors L^-1 and U^-1 as two fp64 HODLR products
// (lu.cpp, on the product's kernels); this translation unit only moves an
// fp32 right-hand side into fp64 and the fp64 solution back to fp32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "lu_internal.h"

namespace hodlr {
namespace {

constexpr int kBT = 256;

__global__ __launch_bounds__(kBT) void k_lu_convert(const void* __restrict__ src, int64_t lds, int src_f64,
                                                    void* __restrict__ dst, int64_t ldd, int dst_f64, int64_t n,
                                                    int nrhs) {
    const int64_t i = int64_t(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n) return;
    for (int c = blockIdx.y; c < nrhs; c += gridDim.y) {
        const double v = src_f64 ? static_cast<const double*>(src)[int64_t(c) * lds + i]
                                 : double(static_cast<const float*>(src)[int64_t(c) * lds + i]);
        if (dst_f64)
            static_cast<double*>(dst)[int64_t(c) * ldd + i] = v;
        else
            static_cast<float*>(dst)[int64_t(c) * ldd + i] = float(v);
    }
}

}  // namespace

int launch_lu_convert(const void* src, int64_t lds, bool src_f64, void* dst, int64_t ldd, bool dst_f64, int64_t n,
                      int nrhs, void* stream) {
    const dim3 grid(unsigned((n + kBT - 1) / kBT), unsigned(std::min(nrhs, 65535)));
    hipLaunchKernelGGL(k_lu_convert, grid, dim3(kBT), 0, static_cast<hipStream_t>(stream), src, lds, int(src_f64),
                       dst, ldd, int(dst_f64), n, nrhs);
    return int(hipGetLastError());
}

}  // namespace hodlr
