// HIP kernels (gfx950) of the construction of an eps-HODLR operator from a
// kernel matrix A_ij = k(p_i, p_j) evaluated on the fly (never stored):
//
//  * squared Frobenius norms of every leaf and off-diagonal block (the
//    nrmAll and nrm_k steps of Alg. "Adaptive-precision HODLR Format"),
//    summed in fp64 over tiles in a fixed order;
//  * the heavy steps of a randomised truncated SVD of each block B (a range
//    finder: sketch Y = B Omega, projection M^T = B^T Q, and the exact
//    residual ||B - Q M||_F^2 when the rule needs it), batched over all the
//    blocks of a level; Omega is N(0,1) from a counter-based generator;
//  * the tall-skinny pieces: Gram matrices A^T A in row chunks (in
//    double-double) and the products A S with a small S (orthogonalisation
//    and the final factors);
//  * the leaves D_i.
//
// Everything is fp64.  One translation unit of the library (see kernels.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "build_internal.h"
#include "hodlr_internal.h"

namespace hodlr {
namespace {

constexpr int kBT = 256;          // threads per workgroup
constexpr int kRows = kBuildRows; // output rows of an on-the-fly product tile (64: one per lane)
constexpr int kChunk = 32;        // inner-dimension chunk staged in LDS

__device__ __forceinline__ double kernel_entry(const BuildKernel& K, const double* __restrict__ P, int64_t i,
                                               int64_t j) {
    double v;
    if (i == j && K.diag_given) {
        v = K.diag_value;
    } else {
        double d2;
        double dx = P[i * K.dim] - P[j * K.dim];
        if (K.dim == 1) {
            d2 = dx * dx;
        } else {
            const double dy = P[i * K.dim + 1] - P[j * K.dim + 1];
            d2 = dx * dx + dy * dy;
        }
        switch (K.kind) {
            case 0: v = exp(-d2 / K.a); break;                 // Gaussian exp(-r^2 / a)
            case 1: v = 1.0 / (sqrt(d2) + K.a); break;         // 1 / (r + a)
            case 2: v = log(sqrt(d2) + K.a); break;            // log(r + a)
            case 3: v = exp(-sqrt(d2)); break;                 // exp(-r)
            default: v = 1.0 / dx; break;                      // 1 / (x_i - x_j), 1D
        }
    }
    if (i == j) v += K.diag_shift;
    return v;
}

// ---------------------------------------------------------------------------
// squared Frobenius norms over tiles of the matrix
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBT) void k_norms(BuildKernel K, const double* __restrict__ P,
                                               const BuildTile* __restrict__ tiles, double* __restrict__ out) {
    const BuildTile t = tiles[blockIdx.x];
    double s = 0.0;
    const int64_t cnt = int64_t(t.nr) * t.nc;
    for (int64_t e = threadIdx.x; e < cnt; e += kBT) {
        const int64_t c = e / t.nr, r = e - c * t.nr;
        const double v = kernel_entry(K, P, t.r0 + r, t.c0 + c);
        s += v * v;
    }
    __shared__ double red[kBT];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Omega: N(0, 1) entries from a counter-based generator (splitmix64 of the
// seed, block and entry index, then Box-Muller)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBT) void k_omega(const BuildPanel* __restrict__ pans, uint64_t seed,
                                               double* __restrict__ W) {
    const BuildPanel pn = pans[blockIdx.y];
    const int64_t cnt = int64_t(pn.inner) * pn.s;
    for (int64_t e = blockIdx.x * int64_t(kBT) + threadIdx.x; e < cnt; e += int64_t(gridDim.x) * kBT) {
        const uint64_t h = mix64(seed ^ mix64(uint64_t(pn.block) * 0x100000001b3ull + uint64_t(e)));
        const double u1 = (double((h >> 11) & ((1ull << 26) - 1)) + 0.5) * (1.0 / 67108864.0);
        const double u2 = double(h >> 37) * (1.0 / 134217728.0);
        W[pn.w_off + e] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    }
}

// ---------------------------------------------------------------------------
// Out = B W (trans = 0) or B^T W (trans = 1) for one block per panel, with
// B(i, j) = k(p_{r0+i}, p_{c0+j}) generated on the fly.  A workgroup makes
// kRows output rows x s columns: the inner dimension goes through LDS in
// chunks of kChunk (the B chunk evaluated by the workgroup, the W chunk
// loaded), each thread accumulating s / 4 outputs of one row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBT) void k_apply(BuildKernel K, const double* __restrict__ P,
                                               const BuildPanel* __restrict__ pans, const BuildItem* __restrict__ items,
                                               const double* __restrict__ W, double* __restrict__ Out) {
    const BuildItem it = items[blockIdx.x];
    const BuildPanel pn = pans[it.panel];
    const int s = pn.s;                              // multiple of 4, at most kMaxSketch
    __shared__ double bt[kChunk][kRows + 1];         // B chunk, [inner][out row]
    __shared__ double wt[kChunk][kMaxSketch];
    const int row = threadIdx.x & (kRows - 1);
    const int q0 = threadIdx.x >> 6;                 // columns q0, q0 + 4, ...
    double acc[kMaxSketch / 4];
#pragma unroll
    for (int m = 0; m < kMaxSketch / 4; ++m) acc[m] = 0.0;
    const int orow = it.row0 + row;                  // output row of this thread (within the panel)
    for (int j0 = 0; j0 < pn.inner; j0 += kChunk) {
        const int jn = min(kChunk, pn.inner - j0);
        __syncthreads();
        for (int e = threadIdx.x; e < kChunk * kRows; e += kBT) {
            const int jj = e / kRows, rr = e - jj * kRows;
            double v = 0.0;
            if (jj < jn && it.row0 + rr < pn.outer) {
                const int64_t oi = it.row0 + rr, ij = j0 + jj;
                v = pn.trans ? kernel_entry(K, P, pn.r0 + ij, pn.c0 + oi) : kernel_entry(K, P, pn.r0 + oi, pn.c0 + ij);
            }
            bt[jj][rr] = v;
        }
        for (int e = threadIdx.x; e < kChunk * s; e += kBT) {
            const int q = e / kChunk, jj = e - q * kChunk;
            wt[jj][q] = jj < jn ? W[pn.w_off + int64_t(q) * pn.inner + j0 + jj] : 0.0;
        }
        __syncthreads();
        for (int jj = 0; jj < kChunk; ++jj) {
            const double b = bt[jj][row];
#pragma unroll
            for (int m = 0; m < kMaxSketch / 4; ++m)
                if (4 * m + q0 < s) acc[m] += b * wt[jj][4 * m + q0];
        }
    }
    if (orow < pn.outer)
#pragma unroll
        for (int m = 0; m < kMaxSketch / 4; ++m)
            if (4 * m + q0 < s) Out[pn.o_off + int64_t(4 * m + q0) * pn.outer + orow] = acc[m];
}

// ---------------------------------------------------------------------------
// partial Gram matrices A^T A over row chunks, in double-double: item
// (panel, row0) covers rows [row0, row0 + kGramRows) of panel A (outer x s,
// column-major at o_off).  Each product is split exactly with an FMA and
// the sums are carried as (hi, lo) pairs (Knuth's two-sum), so a chunk's
// Gram entries are accurate to about u^2 |A|^T |A|.
// out[(item * kMaxSketch^2 + a * s + b) * 2 + {0: hi, 1: lo}], b >= a
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum_acc(double& hi, double& lo, double x) {
    const double s = hi + x;
    const double bb = s - hi;
    const double err = (hi - (s - bb)) + (x - bb);
    hi = s;
    lo += err;
}

__global__ __launch_bounds__(kBT) void k_gram(const BuildPanel* __restrict__ pans, const BuildItem* __restrict__ items,
                                              const double* __restrict__ A, double* __restrict__ out) {
    const BuildItem it = items[blockIdx.x];
    const BuildPanel pn = pans[it.panel];
    const int s = pn.s;
    const int r1 = min(pn.outer, it.row0 + kGramRows);
    const double* Ap = A + pn.o_off;
    for (int e = threadIdx.x; e < s * s; e += kBT) {
        const int a = e / s, b = e - a * s;
        if (b < a) continue;
        double hi = 0.0, lo = 0.0;
        const double* ca = Ap + int64_t(a) * pn.outer;
        const double* cb = Ap + int64_t(b) * pn.outer;
        for (int r = it.row0; r < r1; ++r) {
            const double x = ca[r], y = cb[r];
            const double p = x * y;
            lo += fma(x, y, -p);                     // the product's rounding error, exactly
            two_sum_acc(hi, lo, p);
        }
        const int64_t o = (int64_t(blockIdx.x) * kMaxSketch * kMaxSketch + a * s + b) * 2;
        out[o] = hi;
        out[o + 1] = lo;
    }
}

// ---------------------------------------------------------------------------
// C = A S per panel: A (outer x s at a_off), S (s x p, column-major at the
// panel's w_off in Sbuf), C (outer x p at c_off, leading dimension outer)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBT) void k_small_gemm(const BuildPanel* __restrict__ pans,
                                                    const BuildItem* __restrict__ items, const double* __restrict__ A,
                                                    const double* __restrict__ S, double* __restrict__ Cm) {
    const BuildItem it = items[blockIdx.x];
    const BuildPanel pn = pans[it.panel];
    const int s = pn.s, p = pn.p;
    __shared__ double st[kMaxSketch * kMaxSketch / 4];   // a kMaxSketch x (kMaxSketch / 4) slice of S
    const int row = it.row0 + (threadIdx.x & (kRows - 1));
    const int q0 = threadIdx.x >> 6;
    for (int c0 = 0; c0 < p; c0 += kMaxSketch / 4) {
        const int cn = min(kMaxSketch / 4, p - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < s * cn; e += kBT) {
            const int c = e / s, k = e - c * s;
            st[c * kMaxSketch + k] = S[pn.w_off + int64_t(c0 + c) * s + k];
        }
        __syncthreads();
        if (row < pn.outer)
            for (int c = q0; c < cn; c += 4) {
                double acc = 0.0;
                for (int k = 0; k < s; ++k) acc += A[pn.o_off + int64_t(k) * pn.outer + row] * st[c * kMaxSketch + k];
                Cm[pn.c_off + int64_t(c0 + c) * pn.outer + row] = acc;
            }
    }
}

// ---------------------------------------------------------------------------
// ||B - Q M||_F^2 over a tile: item (panel, row0) covers kResRows rows and
// all columns of the block; Q (rows x s at o_off), Mt = M^T (cols x s at
// c_off).  The tile's Q rows and each kResCols-column chunk of Mt go
// through LDS; thread t takes row t % kResRows and columns t / kResRows and
// t / kResRows + 8 of each chunk.
// ---------------------------------------------------------------------------
constexpr int kResRows = kResidualRows;
constexpr int kResCols = 16;

__global__ __launch_bounds__(kBT) void k_residual(BuildKernel K, const double* __restrict__ P,
                                                  const BuildPanel* __restrict__ pans,
                                                  const BuildItem* __restrict__ items, const double* __restrict__ Q,
                                                  const double* __restrict__ Mt, double* __restrict__ out) {
    const BuildItem it = items[blockIdx.x];
    const BuildPanel pn = pans[it.panel];
    const int s = pn.s;
    __shared__ double qt[kMaxSketch][kResRows + 1];
    __shared__ double mt[kMaxSketch][kResCols + 1];
    __shared__ double red[kBT];
    for (int e = threadIdx.x; e < kResRows * s; e += kBT) {
        const int q = e / kResRows, rr = e - q * kResRows;
        qt[q][rr] = it.row0 + rr < pn.outer ? Q[pn.o_off + int64_t(q) * pn.outer + it.row0 + rr] : 0.0;
    }
    const int rr = threadIdx.x % kResRows, cc = threadIdx.x / kResRows;
    const bool live = it.row0 + rr < pn.outer;
    double acc = 0.0;
    for (int c0 = 0; c0 < pn.inner; c0 += kResCols) {
        __syncthreads();
        for (int e = threadIdx.x; e < kResCols * s; e += kBT) {
            const int q = e / kResCols, c = e - q * kResCols;
            mt[q][c] = c0 + c < pn.inner ? Mt[pn.c_off + int64_t(q) * pn.inner + c0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = cc + 8 * h;
            if (!live || c0 + c >= pn.inner) continue;
            double qm = 0.0;
            for (int q = 0; q < s; ++q) qm += qt[q][rr] * mt[q][c];
            const double d = kernel_entry(K, P, pn.r0 + it.row0 + rr, pn.c0 + c0 + c) - qm;
            acc += d * d;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// leaves: D_i = A(I_i, I_i), column-major, one after another
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBT) void k_leaves(BuildKernel K, const double* __restrict__ P,
                                                const BuildTile* __restrict__ leaves, double* __restrict__ D) {
    const BuildTile t = leaves[blockIdx.y];
    const int64_t cnt = int64_t(t.nr) * t.nc;
    for (int64_t e = blockIdx.x * int64_t(kBT) + threadIdx.x; e < cnt; e += int64_t(gridDim.x) * kBT) {
        const int64_t c = e / t.nr, r = e - c * t.nr;
        D[t.out + e] = kernel_entry(K, P, t.r0 + r, t.c0 + c);
    }
}

}  // namespace

int launch_build_norms(const BuildKernel& K, const double* P, const BuildTile* tiles, int ntiles, double* out,
                       void* stream) {
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL(k_norms, dim3(ntiles), dim3(kBT), 0, static_cast<hipStream_t>(stream), K, P, tiles, out);
    return int(hipGetLastError());
}

int launch_build_omega(const BuildPanel* pans, int npan, uint64_t seed, double* W, void* stream) {
    if (npan <= 0) return 0;
    hipLaunchKernelGGL(k_omega, dim3(64, npan), dim3(kBT), 0, static_cast<hipStream_t>(stream), pans, seed, W);
    return int(hipGetLastError());
}

int launch_build_apply(const BuildKernel& K, const double* P, const BuildPanel* pans, const BuildItem* items,
                       int nitems, const double* W, double* Out, void* stream) {
    if (nitems <= 0) return 0;
    hipLaunchKernelGGL(k_apply, dim3(nitems), dim3(kBT), 0, static_cast<hipStream_t>(stream), K, P, pans, items, W,
                       Out);
    return int(hipGetLastError());
}

int launch_build_gram(const BuildPanel* pans, const BuildItem* items, int nitems, const double* A, double* out,
                      void* stream) {
    if (nitems <= 0) return 0;
    hipLaunchKernelGGL(k_gram, dim3(nitems), dim3(kBT), 0, static_cast<hipStream_t>(stream), pans, items, A, out);
    return int(hipGetLastError());
}

int launch_build_small_gemm(const BuildPanel* pans, const BuildItem* items, int nitems, const double* A,
                            const double* S, double* C, void* stream) {
    if (nitems <= 0) return 0;
    hipLaunchKernelGGL(k_small_gemm, dim3(nitems), dim3(kBT), 0, static_cast<hipStream_t>(stream), pans, items, A, S,
                       C);
    return int(hipGetLastError());
}

int launch_build_residual(const BuildKernel& K, const double* P, const BuildPanel* pans, const BuildItem* items,
                          int nitems, const double* Q, const double* Mt, double* out, void* stream) {
    if (nitems <= 0) return 0;
    hipLaunchKernelGGL(k_residual, dim3(nitems), dim3(kBT), 0, static_cast<hipStream_t>(stream), K, P, pans, items, Q,
                       Mt, out);
    return int(hipGetLastError());
}

int launch_build_leaves(const BuildKernel& K, const double* P, const BuildTile* leaves, int nleaves, double* D,
                        void* stream) {
    if (nleaves <= 0) return 0;
    hipLaunchKernelGGL(k_leaves, dim3(64, nleaves), dim3(kBT), 0, static_cast<hipStream_t>(stream), K, P, leaves, D);
    return int(hipGetLastError());
}

}  // namespace hodlr
