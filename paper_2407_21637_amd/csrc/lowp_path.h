// Low working precision path of the HODLR product: X, Y, the leaf blocks,
// the generators and T_b all enter the arithmetic as bf16 or fp16 values
// (the working precision W), and every product is accumulated in fp32 on
// the matrix cores (v_mfma_f32_16x16x32_{bf16,f16}).  This is the product
// of Alg. "HODLR_MATVEC" computed in a working precision u = u_W, the
// setting of Thm. 3.5 and of the Sect. 4 matrix-vector experiment, with
// the hardware's rounding model: operands rounded to W, sums in fp32.
// Included by kernels.hip only.
//
// Rounding points (each round-to-nearest-even into W):
//   * the leaf blocks, once per operator (a W copy next to the fp64 one);
//   * each stored code value of U_b and V_b, in registers when loaded;
//   * T_b = tscale * (V_b^T X) after its fp32 sum (stored in W);
//   * Y once, after the fp32 sum of the leaf and all levels.
// X arrives in W.
#ifndef HODLR_LOWP_PATH_H
#define HODLR_LOWP_PATH_H

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "wide_path.h"

namespace hodlr {
namespace {

template <typename W>
struct LpMfma;
template <>
struct LpMfma<__bf16> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    __device__ static f32x4 mma(v8 a, v8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct LpMfma<_Float16> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    __device__ static f32x4 mma(v8 a, v8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// eight consecutive W values (16 bytes) as an MFMA operand
template <typename W>
__device__ __forceinline__ typename LpMfma<W>::v8 load_w8(const W* p) {
    typedef typename LpMfma<W>::v8 V8;
    return *reinterpret_cast<const V8*>(p);
}

// eight stored codes of one rank column (consecutive rows), rounded to W
// (fp64 codes are rounded to W directly, the others are exact in fp32 first)
template <int F>
using CodeT = typename std::conditional<F == F64, double, float>::type;

template <int F, typename W>
__device__ __forceinline__ typename LpMfma<W>::v8 codes_to_w8(const uint8_t* p) {
    CodeT<F> v[kKL];
    load_codes8<F, CodeT<F>>(p, v);
    typename LpMfma<W>::v8 r;
#pragma unroll
    for (int q = 0; q < kKL; ++q) r[q] = W(v[q]);
    return r;
}

// ---------------------------------------------------------------------------
// contraction: partial sums of V_b^T X per item, on the matrix cores
// ---------------------------------------------------------------------------
// Item rows [r0, r0+nr) of block b's V panel against X (W).  The waves
// split the rows in 32-row steps; lane group g of a step holds rows
// 8g..8g+7 (one 16-byte X load per column tile, eight codes per rank), so
// one MFMA covers the step.  PG rank tiles of 16 per pass; the waves'
// blocks are added in LDS and stored as the item's fp64 partial ([j][c]).
template <int F, typename W, int NT>
__device__ void contract_item_lp(const KParams& kp, const CItem& it, const BlockDesc& bd, const W* __restrict__ X,
                                 int64_t ldx, int nrhs, int c0, float* red) {
    typedef LpMfma<W> M;
    typedef typename M::v8 V8;
    constexpr int S = Codec<F>::kBytes;
    constexpr int PG = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int p = bd.rank;
    const uint8_t* Vp = kp.fac + bd.v_off + int64_t(it.r0) * p * S;
    const int64_t ld = it.nr;
    double* part = kp.partial + it.poff * nrhs;
    const W* Xr = X + int64_t(bd.vrow0) + it.r0;
    const int nstep = (it.nr + kStep - 1) / kStep;
    const V8 zero = {};
    for (int j0 = 0; j0 < p; j0 += 16 * PG) {
        f32x4 acc[PG][NT];
#pragma unroll
        for (int a = 0; a < PG; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
        for (int st = wave; st < nstep; st += kWaves) {
            const int row = st * kStep + g * kKL;       // nr and row are multiples of 8
            const bool ok = row < it.nr;
            V8 a[PG], b[NT];
#pragma unroll
            for (int pg = 0; pg < PG; ++pg) {
                const int j = j0 + 16 * pg + li;
                a[pg] = (ok && j < p) ? codes_to_w8<F, W>(Vp + (int64_t(j) * ld + row) * S) : zero;
            }
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int c = c0 + 16 * ct + li;
                b[ct] = (ok && c < nrhs) ? load_w8<W>(Xr + row + ldx * c) : zero;
            }
#pragma unroll
            for (int pg = 0; pg < PG; ++pg)
                if (j0 + 16 * pg < p)
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) acc[pg][ct] = M::mma(a[pg], b[ct], acc[pg][ct]);
        }
        // add the four waves' blocks, one rank tile at a time
#pragma unroll
        for (int pg = 0; pg < PG; ++pg) {
            if (j0 + 16 * pg >= p) break;
#pragma unroll
            for (int ct = 0; ct < NT; ++ct)
#pragma unroll
                for (int e = 0; e < 4; ++e) red[(wave * NT + ct) * 256 + (4 * g + e) * 16 + li] = acc[pg][ct][e];
            __syncthreads();
            for (int idx = threadIdx.x; idx < NT * 256; idx += kThreads) {
                const int ct = idx >> 8, jr = (idx >> 4) & 15, cl = idx & 15;
                const int j = j0 + 16 * pg + jr, c = c0 + 16 * ct + cl;
                float s = 0.0f;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) s += red[(w * NT) * 256 + idx];
                if (j < p && c < nrhs) part[int64_t(j) * nrhs + c] = double(s);
            }
            __syncthreads();
        }
    }
}

template <typename W, int NT>
__global__ __launch_bounds__(kThreads) void k_contract_lp(KParams kp, const W* __restrict__ X, int64_t ldx,
                                                          int nrhs) {
    extern __shared__ double smem_d[];
    const CItem it = kp.citems[blockIdx.x];
    const BlockDesc bd = kp.blocks[it.block];
    const int c0 = blockIdx.y * 16 * NT;
    float* red = reinterpret_cast<float*>(smem_d);
    switch (bd.fmt) {
        case F64: contract_item_lp<F64, W, NT>(kp, it, bd, X, ldx, nrhs, c0, red); break;
        case F32: contract_item_lp<F32, W, NT>(kp, it, bd, X, ldx, nrhs, c0, red); break;
        case BF16: contract_item_lp<BF16, W, NT>(kp, it, bd, X, ldx, nrhs, c0, red); break;
        case F16: contract_item_lp<F16, W, NT>(kp, it, bd, X, ldx, nrhs, c0, red); break;
        case E4M3: contract_item_lp<E4M3, W, NT>(kp, it, bd, X, ldx, nrhs, c0, red); break;
        default: contract_item_lp<E5M2, W, NT>(kp, it, bd, X, ldx, nrhs, c0, red); break;
    }
}

// T_b in W: thread o of block b makes entry (c, j) = (o / P, o % P) of the
// [c][j] array (P = rank rounded up to 32, zero past the rank), the item
// partials summed in fp32 in item order, scaled, rounded once
template <typename W>
__global__ __launch_bounds__(256) void k_reduce_lp(KParams kp, int nrhs) {
    const BlockDesc bd = kp.blocks[blockIdx.x];
    const int p = bd.rank;
    const int P = (p + 31) & ~31;
    const int o = blockIdx.y * 256 + threadIdx.x;
    if (o >= P * nrhs) return;
    const int c = o / P, j = o - (o / P) * P;
    W* Tw = static_cast<W*>(kp.Tw) + bd.tw_off * nrhs;
    if (j >= p) {
        Tw[o] = W(0.0f);
        return;
    }
    const double* src = kp.partial + kp.citems[bd.item0].poff * nrhs + int64_t(j) * nrhs + c;
    const int total = p * nrhs;
    float s = 0.0f;
    for (int i = 0; i < bd.nitems; ++i) s += float(src[int64_t(i) * total]);
    Tw[o] = W(double(s) * kp.tscale[bd.ts_off + j]);     // the scale is a power of two: one rounding
}

// ---------------------------------------------------------------------------
// expansion: leaf GEMM and U_b T_b on the matrix cores, Y written once
// ---------------------------------------------------------------------------
// One workgroup per (128-row tile, 16 NT right-hand sides); wave w owns
// tile rows 32w..32w+31 as two 16-row MFMA tiles (h).  The K index of the
// leaf GEMM (leaf columns) and of the low-rank products (ranks) runs in
// steps of 32: lane group g holds K = 8g..8g+7 of a step for both operands.
// The leaf's W copy is row-major (ld = mp), so a lane's eight K values are
// one 16-byte load; X (column-major) likewise; T_b in W is [c][j].
template <int F, typename W, int NT>
__device__ void expand_level_lp(const KParams& kp, const BlockDesc& bd, int chunk0, int ld, int c0, int nrhs,
                                int wave, int li, int g, f32x4 acc[2][NT]) {
    typedef LpMfma<W> M;
    typedef typename M::v8 V8;
    constexpr int S = Codec<F>::kBytes;
    const int p = bd.rank;
    const int P = (p + 31) & ~31;
    const uint8_t* Up = kp.fac + bd.u_off + int64_t(chunk0) * p * S;   // the tile's chunk: (j, row) at (j ld + row) S
    const W* Tw = static_cast<const W*>(kp.Tw) + bd.tw_off * nrhs;
    const V8 zero = {};
    for (int j0 = 0; j0 < P; j0 += kStep) {
        const int jg = j0 + kKL * g;                    // the lane's eight ranks
        V8 a[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = 32 * wave + 16 * h + li;      // tile row
            a[h] = zero;
            if (r < ld) {
#pragma unroll
                for (int q = 0; q < kKL; ++q) {
                    CodeT<F> v = 0;
                    if (jg + q < p) Codec<F>::template load<1, CodeT<F>>(Up + (int64_t(jg + q) * ld + r) * S, &v);
                    a[h][q] = W(v);
                }
            }
        }
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int c = c0 + 16 * ct + li;
            const V8 b = c < nrhs ? load_w8<W>(Tw + int64_t(c) * P + jg) : zero;
            acc[0][ct] = M::mma(a[0], b, acc[0][ct]);
            acc[1][ct] = M::mma(a[1], b, acc[1][ct]);
        }
    }
}

template <typename W, int NT>
__global__ __launch_bounds__(kThreads) void k_expand_lp(KParams kp, const W* __restrict__ Xw, int64_t ldw,
                                                        W* __restrict__ Y, int64_t ldy, int nrhs) {
    typedef LpMfma<W> M;
    typedef typename M::v8 V8;
    const ETile t = kp.etiles[blockIdx.x];
    const LeafDesc L = kp.leaves[t.leaf];
    const int c0 = blockIdx.y * 16 * NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int depth = kp.depth;
    f32x4 acc[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
    // leaf: rows of the tile (row-major W copy, ld = mp) times X_i
    {
        const W* Dw = static_cast<const W*>(kp.leafw) + L.d_off;
        const W* Xl = Xw + L.prow0;
        const V8 zero = {};
        // rows past the tile read tile row li instead (present: nr >= 16); their results are not written
        const int ra = t.r0 + (32 * wave + li < t.nr ? 32 * wave + li : li);
        const int rb = t.r0 + (32 * wave + 16 + li < t.nr ? 32 * wave + 16 + li : li);
        for (int k0 = 0; k0 < L.mp; k0 += kStep) {
            const int k = k0 + kKL * g;
            const bool ok = k < L.mp;                   // mp is a multiple of 16, k of 8
            const int kk = ok ? k : 0;
            const V8 a0 = load_w8<W>(Dw + int64_t(ra) * L.mp + kk);
            const V8 a1 = load_w8<W>(Dw + int64_t(rb) * L.mp + kk);
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int c = c0 + 16 * ct + li;
                const V8 b = (ok && c < nrhs) ? load_w8<W>(Xl + kk + ldw * c) : zero;
                acc[0][ct] = M::mma(a0, b, acc[0][ct]);
                acc[1][ct] = M::mma(a1, b, acc[1][ct]);
            }
        }
    }
    // the depth ancestors' blocks whose rows contain this leaf
    for (int k = 1; k <= depth; ++k) {
        const BlockDesc bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
        if (bd.rank == 0) continue;
        const int chunk0 = L.prow0 - bd.urow0 + t.r0;
        switch (bd.fmt) {
            case F64: expand_level_lp<F64, W, NT>(kp, bd, chunk0, t.nr, c0, nrhs, wave, li, g, acc); break;
            case F32: expand_level_lp<F32, W, NT>(kp, bd, chunk0, t.nr, c0, nrhs, wave, li, g, acc); break;
            case BF16: expand_level_lp<BF16, W, NT>(kp, bd, chunk0, t.nr, c0, nrhs, wave, li, g, acc); break;
            case F16: expand_level_lp<F16, W, NT>(kp, bd, chunk0, t.nr, c0, nrhs, wave, li, g, acc); break;
            case E4M3: expand_level_lp<E4M3, W, NT>(kp, bd, chunk0, t.nr, c0, nrhs, wave, li, g, acc); break;
            default: expand_level_lp<E5M2, W, NT>(kp, bd, chunk0, t.nr, c0, nrhs, wave, li, g, acc); break;
        }
    }
    // result element e of lane (li, g): tile row 16h + 4g + e of the wave, column li
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int c = c0 + 16 * ct + li;
            if (c >= nrhs) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = 32 * wave + 16 * h + 4 * g + e;
                const int pr = t.r0 + rr;
                if (rr < t.nr && pr < L.m) Y[L.row0 + pr + ldy * c] = W(acc[h][ct][e]);
            }
        }
}

template <typename W, int NT>
hipError_t launch_lp_nt(const KParams& kp, const W* Xw, int64_t ldw, W* Y, int64_t ldy, int nrhs, const Timer& tm) {
    hipStream_t s = tm.s;
    const int gy = (nrhs + 16 * NT - 1) / (16 * NT);
    if (kp.ncitems > 0) {
        tm.begin(1);
        hipLaunchKernelGGL((k_contract_lp<W, NT>), dim3(kp.ncitems, gy), dim3(kThreads),
                           size_t(kWaves) * NT * 256 * sizeof(float), s, kp, Xw, ldw, nrhs);
        tm.end(1);
        tm.begin(3);
        const int64_t rows_y = (int64_t((kp.max_block_rank + 31) & ~31) * nrhs + 255) / 256;
        hipLaunchKernelGGL((k_reduce_lp<W>), dim3(kp.nblocks, unsigned(rows_y)), dim3(256), 0, s, kp, nrhs);
        tm.end(3);
    }
    tm.begin(2);
    hipLaunchKernelGGL((k_expand_lp<W, NT>), dim3(kp.netiles, gy), dim3(kThreads), 0, s, kp, Xw, ldw, Y, ldy, nrhs);
    tm.end(2);
    return hipGetLastError();
}

template <typename W>
hipError_t launch_lp(const KParams& kp, const void* Xv, int64_t ldx, void* Yv, int64_t ldy, int nrhs,
                     const Timer& tm) {
    const W* X = static_cast<const W*>(Xv);
    W* Y = static_cast<W*>(Yv);
    // 16-byte loads of X need 16-byte aligned columns; padded leaves need the padded copy
    const bool aligned = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((ldx * int64_t(sizeof(W))) % 16 == 0);
    const W* Xw = X;
    int64_t ldw = ldx;
    if (kp.padded || !aligned) {
        tm.begin(0);
        hipLaunchKernelGGL((k_padx<W>), dim3(kp.nleaves), dim3(256), 0, tm.s, kp, X, ldx, nrhs);
        tm.end(0);
        Xw = static_cast<const W*>(kp.xpad);
        ldw = kp.npad;
    }
    if (nrhs <= 16) return launch_lp_nt<W, 1>(kp, Xw, ldw, Y, ldy, nrhs, tm);
    if (nrhs <= 32) return launch_lp_nt<W, 2>(kp, Xw, ldw, Y, ldy, nrhs, tm);
    return launch_lp_nt<W, 4>(kp, Xw, ldw, Y, ldy, nrhs, tm);
}

}  // namespace
}  // namespace hodlr

#endif  // HODLR_LOWP_PATH_H
