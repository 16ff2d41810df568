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
//   * the leaf blocks and each stored code value of U_b, once per precision
//     assignment (the augmented operand, k_build_aug);
//   * each stored code value of V_b, in registers when loaded;
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

// the type a stored code is decoded to before it is rounded to W (fp64
// codes are rounded to W directly, the others are exact in fp32 first)
template <int F>
using CodeT = typename std::conditional<F == F64, double, float>::type;

// ---------------------------------------------------------------------------
// contraction: partial sums of V_b^T X per item, on the matrix cores
// ---------------------------------------------------------------------------
// Item rows [r0, r0+nr) of block b's V panel against X (W).  The waves
// split the rows in 32-row steps; lane group g of a step holds rows
// 8g..8g+7 (one 16-byte X load per column tile, eight codes per rank), so
// one MFMA covers the step.  PG rank tiles of 16 per pass; the waves'
// blocks are added in LDS and stored as the item's fp64 partial ([j][c]).
template <int F, typename W, int NT>
__device__ void contract_item_lp(const KParams& kp, const CItem& it, const BlockDesc& bd, const W* __restrict__ X8,
                                 int nrhs, int c0, float* red) {
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
    const int64_t prow0 = int64_t(bd.vrow0) + it.r0;  // padded row of the item's first row
    const int nstep = (it.nr + kStep - 1) / kStep;
    const V8 zero = {};
    for (int j0 = 0; j0 < p; j0 += 16 * PG) {
        f32x4 acc[PG][NT];
#pragma unroll
        for (int a = 0; a < PG; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
        // two of the wave's steps per pass, both loaded before either is multiplied (the
        // accumulation order, step st then st + kWaves, is that of one step per pass)
        for (int st = wave; st < nstep; st += 2 * kWaves) {
            // the codes of both steps are loaded before any is decoded, from
            // addresses clamped into the item (rank -> j0, row -> 0), then
            // decoded, masked and rounded to W
            V8 a[2][PG], b[2][NT];
            RawCodes<F, kKL> rv[2][PG];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = (st + h * kWaves) * kStep + g * kKL;   // nr and row are multiples of 8
                const bool ok = row < it.nr;
#pragma unroll
                for (int pg = 0; pg < PG; ++pg) {
                    const int j = j0 + 16 * pg + li;
                    rv[h][pg].load(Vp + (int64_t(j < p ? j : j0) * ld + (ok ? row : 0)) * S);
                }
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const int c = c0 + 16 * ct + li;
                    b[h][ct] = (ok && c < nrhs) ? load_w8<W>(X8 + (((prow0 + row) >> 3) * nrhs + c) * 8) : zero;
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bool ok = (st + h * kWaves) * kStep + g * kKL < it.nr;
#pragma unroll
                for (int pg = 0; pg < PG; ++pg) {
                    CodeT<F> v[kKL];
                    rv[h][pg].template decode<CodeT<F>>(v, ok && j0 + 16 * pg + li < p);
#pragma unroll
                    for (int q = 0; q < kKL; ++q) a[h][pg][q] = W(v[q]);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int pg = 0; pg < PG; ++pg)
                    if (j0 + 16 * pg < p)
#pragma unroll
                        for (int ct = 0; ct < NT; ++ct) acc[pg][ct] = M::mma(a[h][pg], b[h][ct], acc[pg][ct]);
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
__global__ __launch_bounds__(kThreads) void k_contract_lp(KParams kp, const W* __restrict__ X8, int nrhs) {
    extern __shared__ double smem_d[];
    const CItem it = kp.citems[blockIdx.x];
    const BlockDesc bd = kp.blocks[it.block];
    const int c0 = blockIdx.y * 16 * NT;
    float* red = reinterpret_cast<float*>(smem_d);
    switch (bd.fmt) {
        case F64: contract_item_lp<F64, W, NT>(kp, it, bd, X8, nrhs, c0, red); break;
        case F32: contract_item_lp<F32, W, NT>(kp, it, bd, X8, nrhs, c0, red); break;
        case BF16: contract_item_lp<BF16, W, NT>(kp, it, bd, X8, nrhs, c0, red); break;
        case F16: contract_item_lp<F16, W, NT>(kp, it, bd, X8, nrhs, c0, red); break;
        case E4M3: contract_item_lp<E4M3, W, NT>(kp, it, bd, X8, nrhs, c0, red); break;
        default: contract_item_lp<E5M2, W, NT>(kp, it, bd, X8, nrhs, c0, red); break;
    }
}

// T_b in W: thread o of block b makes entry (c, j) = (o / P, o % P) of the
// [c][j] array (P = rank rounded up to 8, zero past the rank), the item
// partials summed in fp32 in item order, scaled, rounded once
template <typename W>
__global__ __launch_bounds__(256) void k_reduce_lp(KParams kp, int nrhs) {
    const BlockDesc bd = kp.blocks[blockIdx.x];
    const int p = bd.rank;
    const int P = (p + 7) & ~7;
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
    int i = 0;
    for (; i + 8 <= bd.nitems; i += 8) {         // eight loads in flight, summed in item order
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = src[int64_t(i + q) * total];
#pragma unroll
        for (int q = 0; q < 8; ++q) s += float(v[q]);
    }
    for (; i < bd.nitems; ++i) s += float(src[int64_t(i) * total]);
    Tw[o] = W(double(s) * kp.tscale[bd.ts_off + j]);     // the scale is a power of two: one rounding
}

// ---------------------------------------------------------------------------
// contraction on leaf-stacked tiles (operators whose every leaf is one
// contraction unit): X read once per leaf for all levels
// ---------------------------------------------------------------------------
// The partial T_b of every ancestor block of leaf `leaf` over the leaf's
// rows, right-hand sides [c0, c0 + 16 NT): the leaf's (block, rank) rows
// stacked 16 to a tile (STile, ng <= TG tiles of format F), the codes
// rounded to W as in contract_item_lp, X in W from the 8-row blocked
// layout.  The waves split the rows in 32-row steps, H steps per pass
// loaded before any is multiplied (the accumulation order is that of one
// step per pass); lane group g of a step holds rows 8g..8g+7.  The four
// waves' blocks are added in LDS and stored in fp32 as the leaf's slice of
// each block's partials ([j][c], ld nrhs).
template <int F, typename W, int NT, int TG, int H>
__device__ void contract_group_lp(const KParams& kp, const LeafDesc& L, int leaf, const STile* __restrict__ tiles,
                                  int ng, const W* __restrict__ X8, int nrhs, int c0, float* red) {
    typedef LpMfma<W> M;
    typedef typename M::v8 V8;
    constexpr int S = Codec<F>::kBytes;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    // the lane's row of each tile (see contract_group_s): tiles past ng
    // repeat tile 0 (valid addresses), rows past a tile's n its row 0
    const uint8_t* vb[TG];
    int vr0[TG], vch[TG], vrows[TG], vp[TG], vj[TG];
    bool vok[TG];
#pragma unroll
    for (int tg = 0; tg < TG; ++tg) {
        const int t = tg < ng ? tg : 0;
        const BlockDesc& bd = kp.blocks[tiles[t].blk[li]];
        vok[tg] = tg < ng && li < tiles[t].n;
        vb[tg] = kp.fac + bd.v_off;
        vr0[tg] = L.prow0 - bd.vrow0;
        vch[tg] = bd.pad_;
        vrows[tg] = bd.vrows;
        vp[tg] = bd.rank;
        vj[tg] = tiles[t].j[li];
    }
    f32x4 acc[TG][NT];
#pragma unroll
    for (int a = 0; a < TG; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
    const V8 zero = {};
    const int nstep = (L.mp + kStep - 1) / kStep;
    for (int st = wave; st < nstep; st += H * kWaves) {
        RawCodes<F, kKL> rv[H][TG];
        V8 b[H][NT];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int row = (st + h * kWaves) * kStep + g * kKL;   // mp and row are multiples of 8
            const bool ok = row < L.mp;
            const int rowc = ok ? row : 0;
#pragma unroll
            for (int tg = 0; tg < TG; ++tg) {
                const int r = vr0[tg] + rowc;                       // row in the panel
                const int cs = (r / vch[tg]) * vch[tg];             // its chunk: first row and rows
                const int rows_c = min(vch[tg], vrows[tg] - cs);
                rv[h][tg].load(vb[tg] + (int64_t(cs) * vp[tg] + int64_t(vj[tg]) * rows_c + (r - cs)) * S);
            }
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int c = c0 + 16 * ct + li;
                b[h][ct] = (ok && c < nrhs) ? load_w8<W>(X8 + (((int64_t(L.prow0) + row) >> 3) * nrhs + c) * 8)
                                            : zero;
            }
        }
        V8 a[H][TG];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const bool ok = (st + h * kWaves) * kStep + g * kKL < L.mp;
#pragma unroll
            for (int tg = 0; tg < TG; ++tg) {
                CodeT<F> v[kKL];
                rv[h][tg].template decode<CodeT<F>>(v, ok && vok[tg]);
#pragma unroll
                for (int q = 0; q < kKL; ++q) a[h][tg][q] = W(v[q]);
            }
        }
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int tg = 0; tg < TG; ++tg)
                if (tg < ng)
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) acc[tg][ct] = M::mma(a[h][tg], b[h][ct], acc[tg][ct]);
    }
    // add the four waves' blocks, one tile at a time, and store each row's
    // slice [c][j] (ld rank): the tile rows of one block are consecutive
    // ranks, so consecutive threads (row fastest) store consecutive words
    float* part = reinterpret_cast<float*>(kp.partial);
#pragma unroll
    for (int tg = 0; tg < TG; ++tg) {
        if (tg >= ng) break;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[(wave * NT + ct) * 256 + (4 * g + e) * 16 + li] = acc[tg][ct][e];
        __syncthreads();
        const int n = tiles[tg].n;
        for (int idx = threadIdx.x; idx < NT * 256; idx += kThreads) {
            const int ct = idx >> 8, cl = (idx >> 4) & 15, jr = idx & 15;
            const int c = c0 + 16 * ct + cl;
            const int ri = ct * 256 + jr * 16 + cl;
            float s = 0.0f;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += red[(w * NT) * 256 + ri];
            if (jr < n && c < nrhs) {
                const BlockDesc& bd = kp.blocks[tiles[tg].blk[jr]];
                part[(bd.s_off + int64_t(leaf - bd.sleaf0) * bd.rank) * nrhs + int64_t(c) * bd.rank + tiles[tg].j[jr]] = s;
            }
        }
        __syncthreads();
    }
}

// one contraction unit (blockIdx.x) for right-hand-side group blockIdx.y,
// at most TGM tiles to a unit (the launch takes 2 when no unit has more,
// which halves the accumulators); fp64 codes come at most two tiles to a
// unit, and four loads in flight per lane are enough for 4- and 8-byte codes
template <typename W, int NT, int TGM>
__global__ __launch_bounds__(kThreads) void k_contract_lp_stack(KParams kp, const W* __restrict__ X8, int nrhs) {
    extern __shared__ double smem_d[];
    const SUnit su = kp.sunits[blockIdx.x];
    const LeafDesc L = kp.leaves[su.leaf];
    const STile* tiles = kp.stiles + su.t0;
    const int c0 = blockIdx.y * 16 * NT;
    float* red = reinterpret_cast<float*>(smem_d);
    switch (tiles[0].fmt) {
        case F64: contract_group_lp<F64, W, NT, 2, 1>(kp, L, su.leaf, tiles, su.ng, X8, nrhs, c0, red); break;
        case F32: contract_group_lp<F32, W, NT, TGM, 1>(kp, L, su.leaf, tiles, su.ng, X8, nrhs, c0, red); break;
        case BF16: contract_group_lp<BF16, W, NT, TGM, 2>(kp, L, su.leaf, tiles, su.ng, X8, nrhs, c0, red); break;
        case F16: contract_group_lp<F16, W, NT, TGM, 2>(kp, L, su.leaf, tiles, su.ng, X8, nrhs, c0, red); break;
        case E4M3: contract_group_lp<E4M3, W, NT, TGM, 2>(kp, L, su.leaf, tiles, su.ng, X8, nrhs, c0, red); break;
        default: contract_group_lp<E5M2, W, NT, TGM, 2>(kp, L, su.leaf, tiles, su.ng, X8, nrhs, c0, red); break;
    }
}

// Slices of k_reduce_lp_stack at a level of `leaves` leaves per column
// node and at most pmax ranks per block (<= 64 on a stacked operator):
// stack_slices(leaves), halved until a slice's 256 / SL threads hold pmax
// outputs; and the columns of T_b per workgroup, (256 / SL) / pmax.
__host__ __device__ inline int lp_reduce_slices(int leaves, int pmax) {
    int sl = stack_slices(leaves);
    while (sl > 1 && 256 / sl < pmax) sl >>= 1;
    return sl;
}
__host__ __device__ inline int lp_reduce_cols(int sl, int pmax) {
    const int c = pmax > 0 ? (256 / sl) / pmax : 256 / sl;
    return c > 1 ? c : 1;
}

// T_b in W from the per-leaf fp32 partials ([c][j] slices), columns
// [c0, c0 + cw) of block b per workgroup (launch shape: ReduceShape by
// columns).  Output v = (c - c0) p + j (j < p) is summed by the threads
// (v, s), s < SL = lp_reduce_slices(leaves, pmax): slices s, s + SL, ... in order
// (eight loads issued before their adds), then the SL runs in order; the
// sum is scaled and rounded once.  The workgroup then writes its columns
// of the [c][j] array whole (ld P = rank rounded up to 8, zero past the
// rank), as k_reduce_lp stores it.
template <typename W>
__global__ __launch_bounds__(256) void k_reduce_lp_stack(KParams kp, int nrhs, ReduceShape rs) {
    __shared__ float sred[256];
    const int w = blockIdx.x;
    int k = 1;
    while (k < rs.depth && w >= rs.start[k]) ++k;
    const int rem = w - rs.start[k - 1];
    const int yg = rem % rs.chunks[k - 1];
    const BlockDesc bd = kp.blocks[(1 << k) - 2 + rem / rs.chunks[k - 1]];
    const int p = bd.rank, P = (p + 7) & ~7;
    const int pmax = kp.level_max_rank[k - 1];
    const int sl = lp_reduce_slices(bd.sleaves, pmax), out = 256 / sl;
    const int cw = lp_reduce_cols(sl, pmax);
    const int c0 = yg * cw;
    if (p == 0 || c0 >= nrhs) return;                   // whole workgroup: before the barrier
    const int ncol = min(cw, nrhs - c0);
    const int v = threadIdx.x % out, s = threadIdx.x / out;
    const int valid = p * nrhs;
    if (v < ncol * p) {                                 // ncol p <= cw pmax <= out
        const float* src = reinterpret_cast<const float*>(kp.partial) + bd.s_off * nrhs + int64_t(c0) * p + v;
        const int n = bd.sleaves;
        float acc = 0.0f;
        int l = s;
        for (; l + 7 * sl < n; l += 8 * sl) {
            float x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = src[int64_t(l + q * sl) * valid];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += x[q];
        }
        for (; l < n; l += sl) acc += src[int64_t(l) * valid];
        sred[threadIdx.x] = acc;
    }
    __syncthreads();
    W* Tw = static_cast<W*>(kp.Tw) + bd.tw_off * nrhs + int64_t(c0) * P;
    for (int i = threadIdx.x; i < ncol * P; i += 256) {
        const int cl = i / P, j = i - cl * P;
        W r = W(0.0f);
        if (j < p) {
            const int vi = cl * p + j;
            float a = sred[vi];
            for (int q = 1; q < sl; ++q) a += sred[q * out + vi];
            r = W(double(a) * kp.tscale[bd.ts_off + j]);    // the scale is a power of two: one rounding
        }
        Tw[i] = r;
    }
}

// ---------------------------------------------------------------------------
// the augmented operand: [D_i | U_1 | ... | U_depth] per leaf, in W
// ---------------------------------------------------------------------------
// Row r of leaf i's operand holds D_i's row r (mp columns, then zeros up to
// mp32 = round_up(mp, 32)), then for each level k the leaf's rows of the
// ancestor block's U panel (rank p_k codes, rounded to W, then zeros up to
// round_up(p_k, 8)), then zeros up to kp columns.  The expansion of a tile
// is then one GEMM over K = mp32 + kp
// against [X_i ; T_1 ; ... ; T_depth].  Built on the device from the packed
// codes, once per precision assignment; fp64 values (the leaves, fp64
// generators) are rounded to W directly, narrower codes through their
// exact fp32 value.
__device__ __forceinline__ int lp_code_bytes(int f) { return f == F64 ? 8 : f == F32 ? 4 : (f == BF16 || f == F16) ? 2 : 1; }

template <typename W>
__global__ __launch_bounds__(256) void k_build_aug(KParams kp) {
    const ETile t = kp.etiles[blockIdx.x];
    const LeafDesc L = kp.leaves[t.leaf];
    const int depth = kp.depth;
    const int mp32 = (L.mp + 31) & ~31;
    const int ld = mp32 + L.kp;
    W* A = static_cast<W*>(const_cast<void*>(kp.aug)) + L.aug_off + int64_t(t.r0) * ld;
    const double* Dt = kp.leafd + L.d_off + int64_t(t.r0) * L.mp;      // tile: column-major, ld = nr
    for (int64_t idx = threadIdx.x; idx < int64_t(t.nr) * ld; idx += 256) {
        const int r = int(idx / ld), c = int(idx - (idx / ld) * ld);
        W v = W(0.0f);
        if (c < L.mp) {
            v = W(Dt[int64_t(c) * t.nr + r]);
        } else if (c >= mp32) {
            int kk = c - mp32;
            for (int k = 1; k <= depth; ++k) {
                const BlockDesc bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
                const int seg = (bd.rank + 7) & ~7;
                if (kk < seg) {
                    if (kk < bd.rank) {
                        const int S = lp_code_bytes(bd.fmt);
                        const int chunk0 = L.prow0 - bd.urow0 + t.r0;
                        const uint8_t* q = kp.fac + bd.u_off + (int64_t(chunk0) * bd.rank + int64_t(kk) * t.nr + r) * S;
                        switch (bd.fmt) {
                            case F64: { double d; Codec<F64>::template load<1, double>(q, &d); v = W(d); } break;
                            case F32: { float f; Codec<F32>::template load<1, float>(q, &f); v = W(f); } break;
                            case BF16: { float f; Codec<BF16>::template load<1, float>(q, &f); v = W(f); } break;
                            case F16: { float f; Codec<F16>::template load<1, float>(q, &f); v = W(f); } break;
                            case E4M3: { float f; Codec<E4M3>::template load<1, float>(q, &f); v = W(f); } break;
                            default: { float f; Codec<E5M2>::template load<1, float>(q, &f); v = W(f); } break;
                        }
                    }
                    break;
                }
                kk -= seg;
            }
        }
        A[int64_t(r) * ld + c] = v;
    }
}

// ---------------------------------------------------------------------------
// expansion: one GEMM per tile over the augmented operand, Y written once
// ---------------------------------------------------------------------------
// One workgroup per (128-row tile, 16 NT right-hand sides); wave w owns
// tile rows 32w..32w+31 as two 16-row MFMA tiles (h).  K runs in steps of
// 32: lane group g holds K = 8g..8g+7 of a step for both operands (16
// bytes each: the operand is row-major, X and the staged T are
// column-major).  K < mp32 (mp rounded up to 32; the operand is zero in
// [mp, mp32)) multiplies X_i: the workgroup loads a step's 32 x 16 NT
// block of X once (thread t one 16-byte piece) into one of kLU LDS
// buffers, and every wave reads it from there after a barrier.  The rest
// of K multiplies the ancestors' T_b, staged at the start as an LDS copy
// [column][kp] in the operand's segment order.  The steps rotate through kLU register buffers: each is refilled
// with the step kLU ahead as soon as its MFMAs are issued, so kLU steps of
// operand loads stay in flight and no loaded value is tested.  The step
// numbering puts the low-rank steps at nsr = round_up(nsteps, kLU), so
// the leaf loop already fetches the first low-rank operands into the
// buffers the low-rank loop reads first (steps in [nsteps, nsr) do nothing).
constexpr int kLU = 4;

template <typename W, int NT>
struct LpStep {                                  // the lane's operands of one step
    typedef typename LpMfma<W>::v8 V8;
    V8 a[2];
    V8 xq;                                       // the thread's piece of the step's X block
};

// operand column of lane group g at step st (see above; steps outside both parts read column 0)
__device__ __forceinline__ int lp_col(int st, int nsteps, int nsr, int ntot, int g) {
    return st < nsteps ? kStep * st + kKL * g : (st >= nsr && st < ntot) ? kStep * (st - nsr + nsteps) + kKL * g : 0;
}

// step st of the leaf loop: the operand and, for threads t < 64 NT (whole
// waves), piece t of X's 32 x 16 NT block: rows 8 (t / 16 NT) .. + 7 of the
// step, column c0 + t mod 16 NT (rows of any other step read row 0 and are
// never used)
template <typename W, int NT>
__device__ __forceinline__ void lp_load(LpStep<W, NT>& o, const W* A0, const W* A1, const W* X8, int prow0,
                                        int st, int nsteps, int nsr, int ntot, int mp, int c0, int g,
                                        int nrhs) {
    constexpr int CW = 16 * NT;
    const int k = lp_col(st, nsteps, nsr, ntot, g);
    o.a[0] = load_w8<W>(A0 + k);
    o.a[1] = load_w8<W>(A1 + k);
    const int t = int(threadIdx.x);
    if (t < 4 * CW) {                            // uniform per wave
        const int kq = kStep * st + kKL * (t / CW);
        const int kx = st < nsteps && kq < mp ? kq : 0;    // rows of X past the leaf meet zero columns
        const int c = c0 + t % CW;
        o.xq = load_w8<W>(X8 + (int64_t((prow0 + kx) >> 3) * nrhs + (c < nrhs ? c : c0)) * 8);
    }
}

template <typename W, int NT>
__global__ __launch_bounds__(kThreads) void k_expand_lp(KParams kp, const W* __restrict__ X8, W* __restrict__ Y,
                                                        int64_t ldy, int nrhs) {
    typedef LpMfma<W> M;
    typedef typename M::v8 V8;
    constexpr int CW = 16 * NT;
    extern __shared__ double smem_d[];
    __shared__ int seg_k[kMaxDepth + 1];         // first operand column of each level's segment
    __shared__ int seg_p[kMaxDepth];             // each level's rank
    __shared__ int64_t seg_t[kMaxDepth];         // each level's T_b in W: element offset of column 0
    W* ts = reinterpret_cast<W*>(smem_d);        // staged T: [column][kp]
    W* xs = ts + int64_t(kp.max_kp) * CW;        // kLU X blocks of 4 CW pieces of 8 values
    // Each XCD (blocks b with the same b mod 8) takes a contiguous run of
    // (tile, column group) units, column groups innermost: the column groups
    // and the tiles of a leaf run back to back on one XCD, so the operand
    // rows and X rows they share are read from that XCD's L2.
    const int ncg = (nrhs + CW - 1) / CW;
    const int units = kp.netiles * ncg, per = (units + 7) / 8;
    const int u = int(blockIdx.x & 7) * per + int(blockIdx.x >> 3);
    if (u >= units) return;                      // whole block: before any barrier
    const ETile t = kp.etiles[u / ncg];
    const LeafDesc L = kp.leaves[t.leaf];
    const int c0 = (u % ncg) * CW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int depth = kp.depth;
    const int mp32 = (L.mp + 31) & ~31;
    const int ld = mp32 + L.kp;
    const int nsteps = mp32 / kStep;
    const int nsr = (nsteps + kLU - 1) / kLU * kLU;
    const int ntot = nsr + L.kp / kStep;         // kp is a multiple of 32
    // rows past the tile read tile row li instead (present: nr >= 16); their results are not written
    const W* A0 = static_cast<const W*>(kp.aug) + L.aug_off +
                  int64_t(t.r0 + (32 * wave + li < t.nr ? 32 * wave + li : li)) * ld;
    const W* A1 = static_cast<const W*>(kp.aug) + L.aug_off +
                  int64_t(t.r0 + (32 * wave + 16 + li < t.nr ? 32 * wave + 16 + li : li)) * ld;
    // the leaf's first kLU steps are fetched before the T staging
    LpStep<W, NT> ring[kLU];
#pragma unroll
    for (int u = 0; u < kLU; ++u)
        lp_load<W, NT>(ring[u], A0, A1, X8, L.prow0, u, nsteps, nsr, ntot, L.mp, c0, g, nrhs);
    if (threadIdx.x < depth) {                   // the ancestors' ranks and T_b offsets
        const int k = threadIdx.x + 1;
        const BlockDesc& bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
        seg_p[k - 1] = bd.rank;
        seg_t[k - 1] = bd.tw_off * nrhs + int64_t(c0) * ((bd.rank + 7) & ~7);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0;
        for (int k = 1; k <= depth; ++k) {
            seg_k[k - 1] = off;
            off += (seg_p[k - 1] + 7) & ~7;
        }
        seg_k[depth] = off;
    }
    __syncthreads();
    // stage T_b of the leaf's ancestors: ts[c][seg_k + j] = T_b[c0 + c][j], zero past the rank / nrhs / kp,
    // in 16-byte chunks (a segment is round_up(p, 8) wide and T_b is stored zero from p up to a multiple
    // of 8, so a chunk never crosses a column); each thread issues its loads before it stores any
    {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        constexpr int kB = 4;
        const W* Tw = static_cast<const W*>(kp.Tw);
        const int kc = L.kp / 8;                 // chunks per staged column
        const int tot = CW * kc;
        for (int base = 0; base < tot; base += kB * kThreads) {
            u32x4 v[kB];
#pragma unroll
            for (int i = 0; i < kB; ++i) {
                const int idx = base + i * kThreads + int(threadIdx.x);
                v[i] = u32x4{0u, 0u, 0u, 0u};
                if (idx < tot) {
                    const int c = idx / kc, kk = (idx - c * kc) * 8;
                    if (kk < seg_k[depth] && c0 + c < nrhs) {
                        int k = 1;
                        while (k < depth && kk >= seg_k[k]) ++k;
                        const int j = kk - seg_k[k - 1];
                        const int p = seg_p[k - 1];
                        if (j < p)
                            v[i] = *reinterpret_cast<const u32x4*>(Tw + seg_t[k - 1] + int64_t(c) * ((p + 7) & ~7) + j);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < kB; ++i) {
                const int idx = base + i * kThreads + int(threadIdx.x);
                if (idx < tot) *reinterpret_cast<u32x4*>(ts + idx * 8) = v[i];
            }
        }
    }
    __syncthreads();                             // the staged T is complete
    f32x4 acc[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
    // leaf: K in [0, mp32), X through LDS buffer u.  Buffer u is rewritten at
    // step st + kLU only after the barrier of step st + kLU - 1, which every
    // wave reaches after its reads of step st.
    for (int s0 = 0; s0 < nsr; s0 += kLU) {
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            if (s0 + u < nsteps) {                   // uniform: the barrier is reached by every thread
                W* xb = xs + u * (4 * CW * kKL);
                if (int(threadIdx.x) < 4 * CW) *reinterpret_cast<V8*>(xb + threadIdx.x * kKL) = ring[u].xq;
                __syncthreads();
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const V8 b = *reinterpret_cast<const V8*>(xb + (g * CW + 16 * ct + li) * kKL);
                    acc[0][ct] = M::mma(ring[u].a[0], b, acc[0][ct]);
                    acc[1][ct] = M::mma(ring[u].a[1], b, acc[1][ct]);
                }
            }
            lp_load<W, NT>(ring[u], A0, A1, X8, L.prow0, s0 + u + kLU, nsteps, nsr, ntot, L.mp, c0, g, nrhs);
        }
    }
    // low rank: K in [mp32, mp32 + kp), the staged T from LDS; only the operand part of the buffers is refilled
    for (int s0 = nsr; s0 < ntot; s0 += kLU) {
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int st = s0 + u;
            if (st < ntot) {
                const int j = (st - nsr) * kStep + kKL * g;
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const V8 b = *reinterpret_cast<const V8*>(ts + (16 * ct + li) * L.kp + j);
                    acc[0][ct] = M::mma(ring[u].a[0], b, acc[0][ct]);
                    acc[1][ct] = M::mma(ring[u].a[1], b, acc[1][ct]);
                }
            }
            const int k = lp_col(st + kLU, nsteps, nsr, ntot, g);
            ring[u].a[0] = load_w8<W>(A0 + k);
            ring[u].a[1] = load_w8<W>(A1 + k);
        }
    }
    // result element e of lane (li, g): tile row 16h + 4g + e of the wave,
    // column li -- four consecutive rows of one column, written as one
    // 8-byte store when they lie inside the leaf and are 8-byte aligned
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int c = c0 + 16 * ct + li;
            if (c >= nrhs) continue;
            const int rr = 32 * wave + 16 * h + 4 * g;
            const int pr = t.r0 + rr;
            W* dst = Y + L.row0 + pr + ldy * c;
            if (rr + 3 < t.nr && pr + 3 < L.m && (reinterpret_cast<uintptr_t>(dst) & 7) == 0) {
                typedef W w4 __attribute__((ext_vector_type(4)));
                w4 v;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = W(acc[h][ct][e]);
                *reinterpret_cast<w4*>(dst) = v;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (rr + e < t.nr && pr + e < L.m) dst[e] = W(acc[h][ct][e]);
            }
        }
}

// dynamic LDS of k_expand_lp: the staged T (max_kp x 16 NT values) and kLU
// X blocks (32 x 16 NT values each)
template <typename W>
size_t lp_expand_lds(const KParams& kp, int nt) {
    return (size_t(kp.max_kp) * 16 * nt + size_t(kLU) * 32 * 16 * nt) * sizeof(W);
}

template <typename W, int NT>
hipError_t launch_lp_nt(const KParams& kp, const W* X8, W* Y, int64_t ldy, int nrhs, const Timer& tm) {
    hipStream_t s = tm.s;
    const int gy = (nrhs + 16 * NT - 1) / (16 * NT);
    if (kp.ncitems > 0) {
        const size_t lds_c = size_t(kWaves) * NT * 256 * sizeof(float);
        tm.begin(1);
        if (kp.stacked > 2)
            hipLaunchKernelGGL((k_contract_lp_stack<W, NT, 4>), dim3(kp.nsunits, gy), dim3(kThreads), lds_c, s, kp,
                               X8, nrhs);
        else if (kp.stacked)
            hipLaunchKernelGGL((k_contract_lp_stack<W, NT, 2>), dim3(kp.nsunits, gy), dim3(kThreads), lds_c, s, kp,
                               X8, nrhs);
        else
            hipLaunchKernelGGL((k_contract_lp<W, NT>), dim3(kp.ncitems, gy), dim3(kThreads), lds_c, s, kp, X8, nrhs);
        tm.end(1);
        tm.begin(3);
        if (kp.stacked) {
            ReduceShape rs{};
            rs.depth = kp.depth;
            int64_t nwg = 0;
            for (int k = 1; k <= kp.depth; ++k) {           // chunks of lp_reduce_cols columns
                const int pmax = kp.level_max_rank[k - 1];
                const int cw = lp_reduce_cols(lp_reduce_slices(1 << (kp.depth - k), pmax), pmax);
                rs.start[k - 1] = int32_t(nwg);
                rs.chunks[k - 1] = (nrhs + cw - 1) / cw;
                nwg += (int64_t(1) << k) * rs.chunks[k - 1];
            }
            rs.start[kp.depth] = int32_t(nwg);
            hipLaunchKernelGGL((k_reduce_lp_stack<W>), dim3(unsigned(nwg)), dim3(256), 0, s, kp, nrhs, rs);
        } else {
            const int64_t rows_y = (int64_t((kp.max_block_rank + 7) & ~7) * nrhs + 255) / 256;
            hipLaunchKernelGGL((k_reduce_lp<W>), dim3(kp.nblocks, unsigned(rows_y)), dim3(256), 0, s, kp, nrhs);
        }
        tm.end(3);
    }
    tm.begin(2);
    hipLaunchKernelGGL((k_expand_lp<W, NT>), dim3(8 * ((kp.netiles * gy + 7) / 8)), dim3(kThreads),
                       lp_expand_lds<W>(kp, NT), s, kp, X8, Y, ldy, nrhs);
    tm.end(2);
    return hipGetLastError();
}

// X in the 8-row blocked layout of the W path: padded row r, column c at
// ((r / 8) nrhs + c) 8 + r mod 8, zero on padding rows, so that a lane's
// 8 consecutive rows of one column and the 16 columns of a lane group are
// one contiguous 256-byte run (the caller's column-major X, columns apart
// by ldx, made every load instruction touch 16 distant columns)
template <typename W>
__global__ __launch_bounds__(256) void k_x8(KParams kp, const W* __restrict__ X, int64_t ldx, int nrhs) {
    const LeafDesc L = kp.leaves[blockIdx.x];
    W* X8 = static_cast<W*>(kp.xpad);
    const int ng = L.mp >> 3;                           // 8-row groups of the leaf
    typedef W w8 __attribute__((ext_vector_type(8)));
    // units of 8 groups x 8 columns, one per wave: lane l takes group l % 8
    // and column l / 8, so the reads are 128-byte runs of one column and the
    // writes 128-byte runs of one group.  Blocks (leaf, y) take runs of 16
    // units (4 per wave, their loads issued before any store), strided by
    // gridDim.y
    constexpr int kU = 4;
    const int ug = (ng + 7) >> 3, uc = (nrhs + 7) >> 3, nu = ug * uc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int ub = int(blockIdx.y) * 4 * kU; ub < nu; ub += int(gridDim.y) * 4 * kU) {
        w8 v[kU];
        int64_t dst[kU];
#pragma unroll
        for (int i = 0; i < kU; ++i) {
            const int u = ub + wave * kU + i;
            const int grp = 8 * (u % ug) + (lane & 7), c = 8 * (u / ug) + (lane >> 3);
            dst[i] = -1;
            if (u >= nu || grp >= ng || c >= nrhs) continue;
            const W* src = X + L.row0 + 8 * grp + ldx * c;
            if (8 * grp + 7 < L.m && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
                v[i] = *reinterpret_cast<const w8*>(src);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) v[i][q] = 8 * grp + q < L.m ? src[q] : W(0.0f);
            }
            dst[i] = ((int64_t(L.prow0 >> 3) + grp) * nrhs + c) * 8;
        }
#pragma unroll
        for (int i = 0; i < kU; ++i)
            if (dst[i] >= 0) *reinterpret_cast<w8*>(X8 + dst[i]) = v[i];
    }
}

template <typename W>
hipError_t launch_lp(const KParams& kp, const void* Xv, int64_t ldx, void* Yv, int64_t ldy, int nrhs,
                     const Timer& tm) {
    const W* X = static_cast<const W*>(Xv);
    W* Y = static_cast<W*>(Yv);
    tm.begin(0);
    {
        // units of the largest leaf (mp <= max_leaf rounded up to 32), 16 per block
        const int64_t nu = int64_t((((kp.max_leaf + 31) & ~31) / 8 + 7) / 8) * ((nrhs + 7) / 8);
        const unsigned gy = unsigned(std::min<int64_t>((nu + 15) / 16, 4096));
        hipLaunchKernelGGL((k_x8<W>), dim3(kp.nleaves, std::max(gy, 1u)), dim3(256), 0, tm.s, kp, X, ldx, nrhs);
    }
    tm.end(0);
    const W* X8 = static_cast<const W*>(kp.xpad);
    auto fits = [&](int nt) { return int64_t(lp_expand_lds<W>(kp, nt)) <= int64_t(kMaxLds); };
    if (nrhs > 32 && fits(4)) return launch_lp_nt<W, 4>(kp, X8, Y, ldy, nrhs, tm);
    if (nrhs > 16 && fits(2)) return launch_lp_nt<W, 2>(kp, X8, Y, ldy, nrhs, tm);
    if (fits(1)) return launch_lp_nt<W, 1>(kp, X8, Y, ldy, nrhs, tm);
    return hipErrorInvalidConfiguration;
}

// the augmented operand of every tile (k_build_aug)
template <typename W>
hipError_t launch_build_aug_w(const KParams& kp, hipStream_t s) {
    hipLaunchKernelGGL((k_build_aug<W>), dim3(kp.netiles), dim3(256), 0, s, kp);
    return hipGetLastError();
}

}  // namespace
}  // namespace hodlr

#endif  // HODLR_LOWP_PATH_H
