// HIP kernels (gfx950) of the triangular solves X = U^-1 L^-1 B with the
// LU factors of a HODLR operator (Sect. 3.4, Alg. "HODLR_LU"; the solves
// are forward and back substitution over the tree).
//
// The host walks the steps in order on one stream: forward substitution
// (pending P = B, solved S = Z = L^-1 B), then back substitution (pending
// P = Z, solved S = X).  A leaf step is a dense product with the inverse of
// the leaf's triangular factor; a node step is a rank-r update of the
// pending rows of one child from the solved rows of the other, as three
// launches: partial sums of A^T S over row chunks, their sum T, and the
// update P -= Bm T.  Everything is fp64; the two conversions at the ends
// read fp32 or fp64 B and write fp32 (rounded to nearest) or fp64 X.
// One translation unit of the library (see kernels.hip).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lu_internal.h"

namespace hodlr {
namespace {

constexpr int kBT = 256;            // threads per workgroup
constexpr int kC = kLuCols;         // right-hand sides per workgroup
constexpr int kChunkRows = 64;      // rows of a reduction chunk
constexpr int kTileQ = 64;          // rank columns per reduction pass
constexpr int kExpandQ = 256;       // rank columns of T staged per expansion pass

// W (ld n) = B (ld ldb), fp64 or fp32 in.
__global__ __launch_bounds__(kBT) void k_lu_load(const void* __restrict__ B, int64_t ldb, int f64,
                                                 double* __restrict__ W, int64_t n, int nrhs) {
    const int64_t i = int64_t(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n) return;
    for (int c = blockIdx.y; c < nrhs; c += gridDim.y)
        W[int64_t(c) * n + i] = f64 ? static_cast<const double*>(B)[int64_t(c) * ldb + i]
                                    : double(static_cast<const float*>(B)[int64_t(c) * ldb + i]);
}

// X (ld ldx) = W (ld n), fp64 or fp32 out.
__global__ __launch_bounds__(kBT) void k_lu_store(const double* __restrict__ W, int64_t n, int nrhs,
                                                  void* __restrict__ X, int64_t ldx, int f64) {
    const int64_t i = int64_t(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n) return;
    for (int c = blockIdx.y; c < nrhs; c += gridDim.y) {
        const double v = W[int64_t(c) * n + i];
        if (f64)
            static_cast<double*>(X)[int64_t(c) * ldx + i] = v;
        else
            static_cast<float*>(X)[int64_t(c) * ldx + i] = float(v);
    }
}

// S[i, c] = sum_k M[k*m + i] P[k, c] for the block's 64 rows and up to kC
// columns; the four waves split k and meet in LDS.
__global__ __launch_bounds__(kBT) void k_lu_leaf(const double* __restrict__ M, int m, const double* __restrict__ P,
                                                 double* __restrict__ S, int64_t ld, int nrhs) {
    __shared__ double red[kBT / 64][64][kC + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int c0 = blockIdx.y * kC, nc = min(kC, nrhs - c0);
    double acc[kC];
#pragma unroll
    for (int c = 0; c < kC; ++c) acc[c] = 0.0;
    if (i < m) {
        for (int k = wv; k < m; k += kBT / 64) {
            const double a = M[int64_t(k) * m + i];
#pragma unroll
            for (int c = 0; c < kC; ++c)
                if (c < nc) acc[c] += a * P[int64_t(c0 + c) * ld + k];
        }
    }
#pragma unroll
    for (int c = 0; c < kC; ++c) red[wv][lane][c] = acc[c];
    __syncthreads();
    if (wv == 0 && i < m) {
        for (int c = 0; c < nc; ++c) {
            double s = red[0][lane][c];
#pragma unroll
            for (int w = 1; w < kBT / 64; ++w) s += red[w][lane][c];
            S[int64_t(c0 + c) * ld + i] = s;
        }
    }
}

// part[g][c][q] = sum over the rows i of chunks g, g + G, ... of
// A[q*m + i] S[c, i]  (A: m x r; S rows from the solved child).
__global__ __launch_bounds__(kBT) void k_lu_reduce(const double* __restrict__ A, int m, int r,
                                                   const double* __restrict__ S, int64_t ld, int nrhs,
                                                   double* __restrict__ part) {
    __shared__ double sa[kChunkRows][kTileQ + 1];
    __shared__ double ss[kChunkRows][kC + 1];
    const int c0 = blockIdx.y * kC, nc = min(kC, nrhs - c0);
    for (int q0 = 0; q0 < r; q0 += kTileQ) {
        const int nq = min(kTileQ, r - q0);
        double acc[kTileQ * kC / kBT];
#pragma unroll
        for (int t = 0; t < kTileQ * kC / kBT; ++t) acc[t] = 0.0;
        for (int64_t i0 = int64_t(blockIdx.x) * kChunkRows; i0 < m; i0 += int64_t(gridDim.x) * kChunkRows) {
            __syncthreads();
            for (int t = threadIdx.x; t < kChunkRows * kTileQ; t += kBT) {
                const int i = t % kChunkRows, q = t / kChunkRows;
                sa[i][q] = (i0 + i < m && q < nq) ? A[int64_t(q0 + q) * m + i0 + i] : 0.0;
            }
            for (int t = threadIdx.x; t < kChunkRows * kC; t += kBT) {
                const int i = t % kChunkRows, c = t / kChunkRows;
                ss[i][c] = (i0 + i < m && c < nc) ? S[int64_t(c0 + c) * ld + i0 + i] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < kTileQ * kC / kBT; ++t) {
                const int e = threadIdx.x + kBT * t, q = e % kTileQ, c = e / kTileQ;
                double s = 0.0;
#pragma unroll 8
                for (int i = 0; i < kChunkRows; ++i) s += sa[i][q] * ss[i][c];
                acc[t] += s;
            }
        }
#pragma unroll
        for (int t = 0; t < kTileQ * kC / kBT; ++t) {
            const int e = threadIdx.x + kBT * t, q = e % kTileQ, c = e / kTileQ;
            if (q < nq && c < nc) part[(int64_t(blockIdx.x) * nrhs + c0 + c) * r + q0 + q] = acc[t];
        }
        __syncthreads();
    }
}

// T[c][q] = sum over g < G of part[g][c][q].
__global__ __launch_bounds__(kBT) void k_lu_sum(const double* __restrict__ part, int G, int r, int nrhs,
                                                double* __restrict__ T) {
    const int64_t e = int64_t(blockIdx.x) * kBT + threadIdx.x;
    const int64_t total = int64_t(nrhs) * r;
    if (e >= total) return;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += part[int64_t(g) * total + e];
    T[e] = s;
}

// P[d0 + i, c] -= sum_q Bm[q*md + i] T[c][q] (Bm: md x r).
__global__ __launch_bounds__(kBT) void k_lu_expand(const double* __restrict__ Bm, int md, int r,
                                                   const double* __restrict__ T, double* __restrict__ P, int64_t ld,
                                                   int nrhs) {
    __shared__ double tq[kC][kExpandQ];
    const int i = blockIdx.x * kBT + threadIdx.x;
    const int c0 = blockIdx.y * kC, nc = min(kC, nrhs - c0);
    double acc[kC];
#pragma unroll
    for (int c = 0; c < kC; ++c) acc[c] = 0.0;
    for (int q0 = 0; q0 < r; q0 += kExpandQ) {
        const int nq = min(kExpandQ, r - q0);
        __syncthreads();
        for (int t = threadIdx.x; t < kC * kExpandQ; t += kBT) {
            const int q = t % kExpandQ, c = t / kExpandQ;
            tq[c][q] = (q < nq && c < nc) ? T[int64_t(c0 + c) * r + q0 + q] : 0.0;
        }
        __syncthreads();
        if (i < md) {
            for (int q = 0; q < nq; ++q) {
                const double b = Bm[int64_t(q0 + q) * md + i];
#pragma unroll
                for (int c = 0; c < kC; ++c) acc[c] += b * tq[c][q];
            }
        }
    }
    if (i < md)
        for (int c = 0; c < nc; ++c) P[int64_t(c0 + c) * ld + i] -= acc[c];
}

int run_steps(const double* img, const LuStep* st, int ns, int64_t n, int nrhs, double* P, double* S, double* part,
              double* T, hipStream_t stream) {
    const int gy = (nrhs + kC - 1) / kC;
    for (int s = 0; s < ns; ++s) {
        const LuStep& x = st[s];
        if (x.kind == 0) {
            hipLaunchKernelGGL(k_lu_leaf, dim3((x.m + 63) / 64, gy), dim3(kBT), 0, stream, img + x.a, x.m,
                               P + x.s0, S + x.s0, n, nrhs);
        } else {
            if (x.r == 0 || x.m == 0 || x.md == 0) continue;
            const int G = int(std::min<int64_t>(kLuParts, (int64_t(x.m) + kChunkRows - 1) / kChunkRows));
            hipLaunchKernelGGL(k_lu_reduce, dim3(G, gy), dim3(kBT), 0, stream, img + x.a, x.m, x.r, S + x.s0, n,
                               nrhs, part);
            const int64_t total = int64_t(nrhs) * x.r;
            hipLaunchKernelGGL(k_lu_sum, dim3(unsigned((total + kBT - 1) / kBT)), dim3(kBT), 0, stream, part, G,
                               x.r, nrhs, T);
            hipLaunchKernelGGL(k_lu_expand, dim3((x.md + kBT - 1) / kBT, gy), dim3(kBT), 0, stream, img + x.b,
                               x.md, x.r, T, P + x.d0, n, nrhs);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return int(e);
    }
    return 0;
}

}  // namespace

int launch_lu_solve(const double* img, const LuStep* fwd, int nfwd, const LuStep* bwd, int nbwd, int64_t n,
                    const void* B, int64_t ldb, void* X, int64_t ldx, int nrhs, bool f64, int rmax, double* ws,
                    void* stream_) {
    const hipStream_t stream = static_cast<hipStream_t>(stream_);
    double* P = ws;                                   // pending values
    double* Z = ws + n * nrhs;                        // L^-1 B
    double* part = ws + 2 * n * nrhs;
    double* T = part + int64_t(kLuParts) * nrhs * std::max(rmax, 1);
    const dim3 gconv(unsigned((n + kBT - 1) / kBT), unsigned(std::min(nrhs, 65535)));
    hipLaunchKernelGGL(k_lu_load, gconv, dim3(kBT), 0, stream, B, ldb, int(f64), P, n, nrhs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return int(e);
    int r = run_steps(img, fwd, nfwd, n, nrhs, P, Z, part, T, stream);     // P = B, S = Z
    if (r) return r;
    r = run_steps(img, bwd, nbwd, n, nrhs, Z, P, part, T, stream);         // P = Z, S = X (in P's memory)
    if (r) return r;
    hipLaunchKernelGGL(k_lu_store, gconv, dim3(kBT), 0, stream, P, n, nrhs, X, ldx, int(f64));
    return int(hipGetLastError());
}

}  // namespace hodlr
