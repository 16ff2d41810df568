// Matrix-core path of the HODLR product (nrhs >= kWideMin): MFMA
// contraction, reduction and expansion, and their launches.  Included by
// kernels.hip only.
#ifndef HODLR_WIDE_PATH_H
#define HODLR_WIDE_PATH_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "wave_path.h"

namespace hodlr {
namespace {

// ---------------------------------------------------------------------------
// many right-hand sides: MFMA tiles
// ---------------------------------------------------------------------------
// With nrhs >= kWideMin the leaf products are dense fp64 GEMMs and the
// low-rank products skinny GEMMs, so both phases run on the matrix cores:
// v_mfma_f64_16x16x4f64 for the leaves and fp64 levels, v_mfma_f32_16x16x4f32
// for levels decoded to fp32.  In both, A is 16x4 with A[l%16][l/16] in lane
// l and B is 4x16 with B[l/16][l%16] in lane l.  Element e of lane l of the
// 16x16 result is C[4*(l/16)+e][l%16] for fp32 but C[l/16+4e][l%16] for fp64
// (measured on gfx950; see acc_row).  The reduction index only has
// to agree between A and B, so lane l feeds its own kKL consecutive rows
// (one vector load) to kKL successive MFMAs: lane group g = l/16 of a 32-row
// step takes rows 8g..8g+7.
constexpr int kKL = 8;                      // consecutive rows per lane per step
constexpr int kStep = 4 * kKL;              // rows per MFMA step (4 lane groups)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    using acc_t = f32x4;
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    using acc_t = f64x4;
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// row of the 16x16 result held in element e by lane group g = l/16
template <typename CT>
__device__ __forceinline__ int acc_row(int g, int e) {
    return sizeof(CT) == 8 ? g + 4 * e : 4 * g + e;
}

// A-operand row that lane l%16 feeds so that an fp32 result lands in the
// fp64 layout: output row 4g+e of the MFMA then holds tile row g+4e.
__device__ __forceinline__ int f64_layout_row(int li) { return (li >> 2) + 4 * (li & 3); }

template <typename A>
__device__ __forceinline__ void zero_acc(A& a) {
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = 0;
}

// kKL consecutive codes of one column (8-element aligned)
template <int F, typename CT>
__device__ __forceinline__ void load_codes8(const uint8_t* p, CT v[kKL]) {
    constexpr int S = Codec<F>::kBytes;
    Codec<F>::template load<4, CT>(p, v);
    Codec<F>::template load<4, CT>(p + 4 * S, v + 4);
}

// kKL consecutive right-hand-side values (16-byte aligned)
template <typename XT, typename CT>
__device__ __forceinline__ void load_x8(const XT* p, CT v[kKL]) {
    if constexpr (sizeof(XT) == 4) {
        const float4 a = reinterpret_cast<const float4*>(p)[0];
        const float4 b = reinterpret_cast<const float4*>(p)[1];
        v[0] = CT(a.x); v[1] = CT(a.y); v[2] = CT(a.z); v[3] = CT(a.w);
        v[4] = CT(b.x); v[5] = CT(b.y); v[6] = CT(b.z); v[7] = CT(b.w);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double2 a = reinterpret_cast<const double2*>(p)[i];
            v[2 * i] = CT(a.x);
            v[2 * i + 1] = CT(a.y);
        }
    }
}

// Contraction on the matrix cores, one leaf at a time: the partial T_b of
// every ancestor block over the leaf's rows (the block of level k whose V
// panel covers them), for right-hand sides [c0, c0 + 16 NT).  The leaf's
// (block, rank) rows are stacked 16 to an MFMA tile (STile); a group of TG
// tiles of one format and arithmetic type is one pass over the leaf's rows
// (X comes from HBM for the first group, from the caches for the others).
// The waves split the rows in 32-row steps; lane group g of a step holds
// rows 8g..8g+7; every tile's codes are loaded before any is decoded; the
// four waves' blocks are added in LDS (`red`) and stored as the leaf's
// slice of each block's partials ([j][c], ld nrhs).
template <int F, typename CT, typename XT, int NT, int TG>
__device__ void contract_group_s(const KParams& kp, const LeafDesc& L, int leaf, const STile* __restrict__ tiles,
                                 int ng, const XT* __restrict__ X, int64_t ldx, int nrhs, int c0, CT* red) {
    using M = Mfma<CT>;
    constexpr int S = Codec<F>::kBytes;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    // the lane's row of each tile: its block's V panel (chunked every pad_
    // rows, see the packer) and the leaf's first row in it; rows past a
    // tile's n repeat its row 0 (valid addresses) and are masked
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
    typename M::acc_t acc[TG][NT];
#pragma unroll
    for (int a = 0; a < TG; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
    const XT* Xr = X + L.prow0;
    const int nstep = (L.mp + kStep - 1) / kStep;
    for (int st = wave; st < nstep; st += kWaves) {
        const int row = st * kStep + g * kKL;           // mp and row are multiples of 8
        const bool ok = row < L.mp;
        const int rowc = ok ? row : 0;
        RawCodes<F, kKL> rv[TG];
#pragma unroll
        for (int tg = 0; tg < TG; ++tg) {
            const int r = vr0[tg] + rowc;               // row in the panel
            const int cs = (r / vch[tg]) * vch[tg];     // its chunk: first row and rows
            const int rows_c = min(vch[tg], vrows[tg] - cs);
            rv[tg].load(vb[tg] + (int64_t(cs) * vp[tg] + int64_t(vj[tg]) * rows_c + (r - cs)) * S);
        }
        CT a[TG][kKL], b[NT][kKL];
        if constexpr (sizeof(XT) == sizeof(CT)) {
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int c = c0 + 16 * ct + li;
                if (ok && c < nrhs)
                    load_x8<XT, CT>(Xr + row + ldx * c, b[ct]);
                else
#pragma unroll
                    for (int q = 0; q < kKL; ++q) b[ct][q] = CT(0);
            }
        } else {
            // X converted to CT: loaded first (column -> c0, row -> 0), converted after
            RawX<XT, kKL> rx[NT];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int c = c0 + 16 * ct + li;
                rx[ct].load(Xr + rowc + ldx * (c < nrhs ? c : c0));
            }
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) rx[ct].template convert<CT>(b[ct], ok && c0 + 16 * ct + li < nrhs);
        }
#pragma unroll
        for (int tg = 0; tg < TG; ++tg) rv[tg].template decode<CT>(a[tg], ok && vok[tg]);
#pragma unroll
        for (int q = 0; q < kKL; ++q)
#pragma unroll
            for (int tg = 0; tg < TG; ++tg)
                if (tg < ng)
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) acc[tg][ct] = M::mma(a[tg][q], b[ct][q], acc[tg][ct]);
    }
    // add the four waves' blocks, one tile at a time, and store each row's slice
#pragma unroll
    for (int tg = 0; tg < TG; ++tg) {
        if (tg >= ng) break;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[(wave * NT + ct) * 256 + acc_row<CT>(g, e) * 16 + li] = acc[tg][ct][e];
        __syncthreads();
        const int n = tiles[tg].n;
        for (int idx = threadIdx.x; idx < NT * 256; idx += kThreads) {
            const int ct = idx >> 8, jr = (idx >> 4) & 15, cl = idx & 15;
            const int c = c0 + 16 * ct + cl;
            CT s = CT(0);
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += red[(w * NT) * 256 + idx];
            if (jr < n && c < nrhs) {
                const BlockDesc& bd = kp.blocks[tiles[tg].blk[jr]];
                const int64_t e = (bd.s_off + int64_t(leaf - bd.sleaf0) * bd.rank + tiles[tg].j[jr]) * nrhs + c;
                if constexpr (sizeof(CT) == 4) {
                    if (kp.part_f32)
                        reinterpret_cast<float*>(kp.partial)[e] = s;
                    else
                        kp.partial[e] = double(s);
                } else {
                    kp.partial[e] = double(s);
                }
            }
        }
        __syncthreads();
    }
}

template <typename CT, typename XT, int NT, int TG>
__device__ void contract_group_dispatch(int fmt, const KParams& kp, const LeafDesc& L, int leaf,
                                        const STile* tiles, int ng, const XT* X, int64_t ldx, int nrhs, int c0,
                                        CT* red) {
    switch (fmt) {
        case F64: contract_group_s<F64, CT, XT, NT, TG>(kp, L, leaf, tiles, ng, X, ldx, nrhs, c0, red); break;
        case F32: contract_group_s<F32, CT, XT, NT, TG>(kp, L, leaf, tiles, ng, X, ldx, nrhs, c0, red); break;
        case BF16: contract_group_s<BF16, CT, XT, NT, TG>(kp, L, leaf, tiles, ng, X, ldx, nrhs, c0, red); break;
        case F16: contract_group_s<F16, CT, XT, NT, TG>(kp, L, leaf, tiles, ng, X, ldx, nrhs, c0, red); break;
        case E4M3: contract_group_s<E4M3, CT, XT, NT, TG>(kp, L, leaf, tiles, ng, X, ldx, nrhs, c0, red); break;
        default: contract_group_s<E5M2, CT, XT, NT, TG>(kp, L, leaf, tiles, ng, X, ldx, nrhs, c0, red); break;
    }
}

// One contraction unit (a group of tiles of one leaf) for right-hand-side
// group yg; at most TGM tiles to a unit in fp32 arithmetic (2 when no unit
// has more, which halves the accumulators), 2 in fp64.
template <typename XT, typename AT, int NT, int TGM>
__device__ void run_contract_stack(const KParams& kp, int unit, int yg, const XT* __restrict__ Xc, int64_t ldc,
                               int nrhs, double* smem_d) {
    const SUnit su = kp.sunits[unit];
    const LeafDesc L = kp.leaves[su.leaf];
    const STile* tiles = kp.stiles + su.t0;
    const int fmt = tiles[0].fmt, dbl = tiles[0].dbl;
    const int c0 = yg * 16 * NT;
    if (dbl || sizeof(AT) == 8) {
        contract_group_dispatch<double, XT, NT, 2>(fmt, kp, L, su.leaf, tiles, su.ng, Xc, ldc, nrhs, c0,
                                                   reinterpret_cast<double*>(smem_d));
    } else if constexpr (sizeof(AT) == 4) {
        contract_group_dispatch<float, XT, NT, TGM>(fmt, kp, L, su.leaf, tiles, su.ng, Xc, ldc, nrhs, c0,
                                                  reinterpret_cast<float*>(smem_d));
    }
}


// Contraction by items (operators whose leaves need more than one pass of
// stacked tiles): item on the matrix cores, partial T_b over rows [r0, r0+nr)
// of the V panel for right-hand sides [c0, c0 + 16 NT).  The waves split
// the rows in 32-row steps; each keeps a (16 PG) x (16 NT) block of partial
// sums per pass over the rank and the four are added in LDS (`red`).  The
// partials ([j][c], ld nrhs) are summed over items by k_reduce_w after the
// launch; on this path T_b is stored [j][c] as well.
template <int F, typename CT, typename XT, int NT>
__device__ void contract_item_w(const KParams& kp, const CItem& it, const BlockDesc& bd,
                                const XT* __restrict__ X, int64_t ldx, int nrhs, int c0, CT* red) {
    using M = Mfma<CT>;
    constexpr int S = Codec<F>::kBytes;
    constexpr int PG = sizeof(CT) == 8 ? 2 : 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int p = bd.rank;
    const uint8_t* Vp = kp.fac + bd.v_off + int64_t(it.r0) * p * S;
    const int64_t ld = it.nr;
    double* part = kp.partial + it.poff * nrhs;
    const XT* Xr = X + int64_t(bd.vrow0) + it.r0;
    const int nstep = (it.nr + kStep - 1) / kStep;
    for (int j0 = 0; j0 < p; j0 += 16 * PG) {
        typename M::acc_t acc[PG][NT];
#pragma unroll
        for (int a = 0; a < PG; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) zero_acc(acc[a][b]);
        for (int st = wave; st < nstep; st += kWaves) {
            const int row = st * kStep + g * kKL;       // nr and row are multiples of 8
            const bool ok = row < it.nr;
            CT a[PG][kKL], b[NT][kKL];
            if constexpr (direct_codes<F, CT>()) {
#pragma unroll
                for (int pg = 0; pg < PG; ++pg) {
                    const int j = j0 + 16 * pg + li;
                    if (ok && j < p)
                        load_codes8<F, CT>(Vp + (int64_t(j) * ld + row) * S, a[pg]);
                    else
#pragma unroll
                        for (int q = 0; q < kKL; ++q) a[pg][q] = CT(0);
                }
            } else {
                // codes that need decoding: all loads first, from clamped
                // addresses (rank -> j0, row -> 0), then decoded and masked
                RawCodes<F, kKL> rv[PG];
#pragma unroll
                for (int pg = 0; pg < PG; ++pg) {
                    const int j = j0 + 16 * pg + li;
                    rv[pg].load(Vp + (int64_t(j < p ? j : j0) * ld + (ok ? row : 0)) * S);
                }
#pragma unroll
                for (int pg = 0; pg < PG; ++pg) rv[pg].template decode<CT>(a[pg], ok && j0 + 16 * pg + li < p);
            }
            if constexpr (sizeof(XT) == sizeof(CT)) {
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const int c = c0 + 16 * ct + li;
                    if (ok && c < nrhs)
                        load_x8<XT, CT>(Xr + row + ldx * c, b[ct]);
                    else
#pragma unroll
                        for (int q = 0; q < kKL; ++q) b[ct][q] = CT(0);
                }
            } else {
                // X converted to CT: loaded first (column -> c0, row -> 0), converted after
                RawX<XT, kKL> rx[NT];
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const int c = c0 + 16 * ct + li;
                    rx[ct].load(Xr + (ok ? row : 0) + ldx * (c < nrhs ? c : c0));
                }
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) rx[ct].template convert<CT>(b[ct], ok && c0 + 16 * ct + li < nrhs);
            }
#pragma unroll
            for (int q = 0; q < kKL; ++q)
#pragma unroll
                for (int pg = 0; pg < PG; ++pg)
                    if (j0 + 16 * pg < p)
#pragma unroll
                        for (int ct = 0; ct < NT; ++ct) acc[pg][ct] = M::mma(a[pg][q], b[ct][q], acc[pg][ct]);
        }
        // add the four waves' blocks, one rank tile at a time
#pragma unroll
        for (int pg = 0; pg < PG; ++pg) {
            if (j0 + 16 * pg >= p) break;
#pragma unroll
            for (int ct = 0; ct < NT; ++ct)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    red[(wave * NT + ct) * 256 + acc_row<CT>(g, e) * 16 + li] = acc[pg][ct][e];
            __syncthreads();
            for (int idx = threadIdx.x; idx < NT * 256; idx += kThreads) {
                const int ct = idx >> 8, jr = (idx >> 4) & 15, cl = idx & 15;
                const int j = j0 + 16 * pg + jr, c = c0 + 16 * ct + cl;
                CT s = CT(0);
#pragma unroll
                for (int w = 0; w < kWaves; ++w) s += red[(w * NT) * 256 + idx];
                if (j < p && c < nrhs) part[int64_t(j) * nrhs + c] = double(s);
            }
            __syncthreads();
        }
    }
}

template <typename XT, typename AT, int NT>
__device__ void run_contract_items(const KParams& kp, int item, int yg, const XT* __restrict__ Xc, int64_t ldc,
                               int nrhs, double* smem_d) {
    const CItem it = kp.citems[item];
    const BlockDesc bd = kp.blocks[it.block];
    const int c0 = yg * 16 * NT;
    switch (bd.fmt) {
        case F64: contract_item_w<F64, double, XT, NT>(kp, it, bd, Xc, ldc, nrhs, c0, reinterpret_cast<double*>(smem_d)); break;
        case F32: contract_item_w<F32, AT, XT, NT>(kp, it, bd, Xc, ldc, nrhs, c0, reinterpret_cast<AT*>(smem_d)); break;
        case BF16: contract_item_w<BF16, AT, XT, NT>(kp, it, bd, Xc, ldc, nrhs, c0, reinterpret_cast<AT*>(smem_d)); break;
        case F16: contract_item_w<F16, AT, XT, NT>(kp, it, bd, Xc, ldc, nrhs, c0, reinterpret_cast<AT*>(smem_d)); break;
        case E4M3: contract_item_w<E4M3, AT, XT, NT>(kp, it, bd, Xc, ldc, nrhs, c0, reinterpret_cast<AT*>(smem_d)); break;
        default: contract_item_w<E5M2, AT, XT, NT>(kp, it, bd, Xc, ldc, nrhs, c0, reinterpret_cast<AT*>(smem_d)); break;
    }
}

// T_b = tscale .* (sum of the block's item partials, in item order): one
// thread per output o = j * nrhs + c of block blockIdx.x, 256 outputs per
// workgroup along blockIdx.y.  fp64 blocks add in fp64, others in the
// accumulation type.
template <typename CT>
__device__ void reduce_block(const KParams& kp, const BlockDesc& bd, int o, int total, int nrhs) {
    const double* src = kp.partial + kp.citems[bd.item0].poff * nrhs + o;
    CT s = CT(0);
    int c = 0;
    for (; c + 8 <= bd.nitems; c += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = src[int64_t(c + q) * total];
#pragma unroll
        for (int q = 0; q < 8; ++q) s += CT(v[q]);
    }
    for (; c < bd.nitems; ++c) s += CT(src[int64_t(c) * total]);
    kp.T[bd.t_off * nrhs + o] = double(s) * kp.tscale[bd.ts_off + o / nrhs];
}

template <typename AT>
__device__ void run_reduce_items(const KParams& kp, int block, int yg, int nrhs) {
    const BlockDesc bd = kp.blocks[block];
    const int total = bd.rank * nrhs;
    const int o = yg * 256 + threadIdx.x;
    if (o >= total) return;
    if (bd.fmt == F64)
        reduce_block<double>(kp, bd, o, total, nrhs);
    else
        reduce_block<AT>(kp, bd, o, total, nrhs);
}

// T_b = tscale .* (sum over the leaves of the column node of their partial
// slices), outputs o = j * nrhs + c, 256 / SL per workgroup (chunk yg),
// SL = stack_slices(leaves): thread (o, s) adds the slices s, s + SL, ...
// in order (eight loads issued before their adds), then the SL runs are
// added in order.  fp64 blocks add in fp64, others in the accumulation type.
template <typename AT>
__device__ void run_reduce_stack(const KParams& kp, int block, int yg, int nrhs) {
    __shared__ double sred[256];
    const BlockDesc bd = kp.blocks[block];
    const int total = bd.rank * nrhs;
    const int sl = stack_slices(bd.sleaves), out = 256 / sl;
    if (yg * out >= total) return;                      // whole block: before the barrier
    const int ol = threadIdx.x % out, s = threadIdx.x / out;
    const int o = yg * out + ol;
    const bool f64 = bd.fmt == F64 || sizeof(AT) == 8;
    if (o < total) {
        const int n = bd.sleaves;
        double acc_d = 0.0;
        AT acc_a = AT(0);
        int l = s;
        if (kp.part_f32) {                              // fp32 partials: fp32 sums (never f64 here)
            const float* src = reinterpret_cast<const float*>(kp.partial) + bd.s_off * nrhs + o;
            for (; l + 7 * sl < n; l += 8 * sl) {
                float v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = src[int64_t(l + q * sl) * total];
#pragma unroll
                for (int q = 0; q < 8; ++q) acc_a += AT(v[q]);
            }
            for (; l < n; l += sl) acc_a += AT(src[int64_t(l) * total]);
        } else {
            const double* src = kp.partial + bd.s_off * nrhs + o;
            for (; l + 7 * sl < n; l += 8 * sl) {
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = src[int64_t(l + q * sl) * total];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (f64) acc_d += v[q];
                    else acc_a += AT(v[q]);
                }
            }
            for (; l < n; l += sl) {
                if (f64) acc_d += src[int64_t(l) * total];
                else acc_a += AT(src[int64_t(l) * total]);
            }
        }
        sred[threadIdx.x] = f64 ? acc_d : double(acc_a);
    }
    __syncthreads();
    if (s == 0 && o < total) {
        double r;
        if (f64) {
            double a = sred[ol];
            for (int q = 1; q < sl; ++q) a += sred[q * out + ol];
            r = a;
        } else {
            AT a = AT(sred[ol]);
            for (int q = 1; q < sl; ++q) a += AT(sred[q * out + ol]);
            r = double(a);
        }
        kp.T[bd.t_off * nrhs + o] = r * kp.tscale[bd.ts_off + o / nrhs];
    }
    __syncthreads();                                    // sred is reused by the next work item
}

// The contraction and the reduction of an operator: stacked (kp.stacked,
// work unit = SUnit, partials per leaf; STACK = the most tiles of a unit
// the kernel holds, 2 or 4) or by items (STACK = 0, work unit = CItem,
// partials per item).
// (a template parameter, not a run-time branch: one kernel holding both
// would take the larger register count for both)
template <typename XT, typename AT, int NT, int STACK>
__device__ void run_contract_w(const KParams& kp, int unit, int yg, const XT* __restrict__ Xc, int64_t ldc,
                               int nrhs, double* smem_d) {
    if constexpr (STACK > 0)
        run_contract_stack<XT, AT, NT, STACK>(kp, unit, yg, Xc, ldc, nrhs, smem_d);
    else
        run_contract_items<XT, AT, NT>(kp, unit, yg, Xc, ldc, nrhs, smem_d);
}

template <typename AT, bool STACK>
__device__ void run_reduce_w(const KParams& kp, int block, int yg, int nrhs) {
    if constexpr (STACK)
        run_reduce_stack<AT>(kp, block, yg, nrhs);
    else
        run_reduce_items<AT>(kp, block, yg, nrhs);
}

template <typename XT, typename AT, int NT, int STACK>
__global__ __launch_bounds__(kThreads) void k_contract_w(KParams kp, const XT* __restrict__ Xc, int64_t ldc,
                                                         int nrhs) {
    extern __shared__ double smem_d[];
    run_contract_w<XT, AT, NT, STACK>(kp, blockIdx.x, blockIdx.y, Xc, ldc, nrhs, smem_d);
}

// reduction by items: blockIdx.x the block, blockIdx.y its 256-output chunk
template <typename AT>
__global__ __launch_bounds__(256) void k_reduce_items(KParams kp, int nrhs) {
    run_reduce_items<AT>(kp, blockIdx.x, blockIdx.y, nrhs);
}

// Launch shape of the reduction of one product: levels one after another,
// level k holding 2^k blocks x chunks[k - 1] chunks (its largest rank x
// nrhs outputs in chunks of 256 / stack_slices(2^(depth - k))), from
// workgroup start[k - 1] on.
struct ReduceShape {
    int32_t depth;
    int32_t start[kMaxDepth + 1];
    int32_t chunks[kMaxDepth];
};

// The shape for a product with nrhs columns.  Returns the workgroups.
inline int64_t reduce_shape(const KParams& kp, int nrhs, ReduceShape* rs) {
    *rs = ReduceShape{};
    rs->depth = kp.depth;
    int64_t nwg = 0;
    for (int k = 1; k <= kp.depth; ++k) {
        const int out = 256 / stack_slices(1 << (kp.depth - k));
        rs->start[k - 1] = int32_t(nwg);
        rs->chunks[k - 1] = std::max(1, int((int64_t(kp.level_max_rank[k - 1]) * nrhs + out - 1) / out));
        nwg += (int64_t(1) << k) * rs->chunks[k - 1];
    }
    rs->start[kp.depth] = int32_t(nwg);
    return nwg;
}

template <typename AT>
__global__ __launch_bounds__(256) void k_reduce_stack(KParams kp, int nrhs, ReduceShape rs) {
    const int w = blockIdx.x;
    int k = 1;
    while (k < rs.depth && w >= rs.start[k]) ++k;
    const int rem = w - rs.start[k - 1];
    run_reduce_stack<AT>(kp, (1 << k) - 2 + rem / rs.chunks[k - 1], rem % rs.chunks[k - 1], nrhs);
}

// rows [j0, j0 + rows) of T_b (stored [j][c], ld nrhs) for right-hand
// sides [c0, c0 + CW), zero beyond the rank or nrhs, as ts[j][c] with row
// stride CW + 4 (the pad keeps the four lane groups' rows in different banks)
template <typename CT, int CW>
__device__ __forceinline__ void stage_t(const KParams& kp, const BlockDesc& bd, int j0, int rows, int c0, int nrhs,
                                        CT* ts) {
    const int p = bd.rank;
    const double* Tb = kp.T + bd.t_off * nrhs;
    for (int idx = threadIdx.x; idx < rows * CW; idx += kThreads) {
        const int jr = idx / CW, cl = idx - jr * CW;
        const int j = j0 + jr, c = c0 + cl;
        ts[jr * (CW + 4) + cl] = (j < p && c < nrhs) ? CT(Tb[int64_t(j) * nrhs + c]) : CT(0);
    }
}

__device__ __forceinline__ int round4(int v) { return (v + 3) & ~3; }

// One level's U_b T_b added to a wave's two 16-row tiles (accumulators in
// the fp64 row layout).  T_b comes from LDS as ts[j][c]: staged whole
// before the call (jc == 0; round_up(p, 4) rows), or here, jc rows at a
// time.  Within the staged rows the U operands of QG MFMA groups (4 ranks
// each: MFMA q takes ranks j0 + 4q + (l/16)) are loaded at once; groups
// past the rank are skipped.
template <int F, typename CT, int NT>
__device__ void expand_level_w(const KParams& kp, const BlockDesc& bd, int chunk0, int ld, int c0, int nrhs,
                               bool act0, bool act1, CT* ts, int jc, typename Mfma<CT>::acc_t acc[2][NT]) {
    using M = Mfma<CT>;
    constexpr int S = Codec<F>::kBytes;
    constexpr int CW = 16 * NT;
    constexpr int TS = CW + 4;
    constexpr int QG = (NT <= 2 && sizeof(CT) == 4) ? 2 * kKL : kKL;   // MFMA groups per batch of U loads
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int p = bd.rank;
    const uint8_t* Up = kp.fac + bd.u_off + int64_t(chunk0) * p * S;
    // fp32 results are steered into the fp64 row layout of the accumulators
    const int r0 = 32 * wave + (sizeof(CT) == 8 ? li : f64_layout_row(li)), r1 = r0 + 16;
    const int chunk = jc ? jc : p;
    for (int cr0 = 0; cr0 < p; cr0 += chunk) {
        const int crows = p - cr0 < chunk ? p - cr0 : chunk;
        if (jc) {
            __syncthreads();                            // previous users of ts are done
            stage_t<CT, CW>(kp, bd, cr0, round4(crows), c0, nrhs, ts);
            __syncthreads();
        }
        const CT* tc = ts + (jc ? 0 : cr0 * TS);
        for (int j0 = 0; j0 < crows; j0 += 4 * QG) {
            const int left = crows - j0 < 4 * QG ? crows - j0 : 4 * QG;
            const int qn = (left + 3) >> 2;             // MFMA groups holding some rank < p
            CT a0[QG], a1[QG];
            if constexpr (direct_codes<F, CT>()) {
#pragma unroll
                for (int q = 0; q < QG; ++q) {
                    const int jr = j0 + 4 * q + g;      // rank within the staged rows
                    a0[q] = CT(0);
                    a1[q] = CT(0);
                    if (q < qn && jr < crows) {
                        const uint8_t* col = Up + int64_t(cr0 + jr) * ld * S;
                        if (act0) Codec<F>::template load<1, CT>(col + int64_t(r0) * S, &a0[q]);
                        if (act1) Codec<F>::template load<1, CT>(col + int64_t(r1) * S, &a1[q]);
                    }
                }
            } else {
                // codes that need decoding: every group's codes are loaded
                // before any is decoded, from addresses clamped into the
                // panel (rank -> the chunk's first staged rank, inactive
                // rows -> row 0), and masked when decoded
                RawCodes<F, 1> u0[QG], u1[QG];
                auto issue = [&](int q) {
                    const int jr = j0 + 4 * q + g;
                    const uint8_t* col = Up + int64_t(cr0 + (jr < crows ? jr : 0)) * ld * S;
                    u0[q].load(col + int64_t(act0 ? r0 : 0) * S);
                    u1[q].load(col + int64_t(act1 ? r1 : 0) * S);
                };
#pragma unroll
                for (int q = 0; q < QG / 2; ++q) issue(q);
                if (__builtin_amdgcn_readfirstlane(qn) > QG / 2) {   // the second half only when used
#pragma unroll
                    for (int q = QG / 2; q < QG; ++q) issue(q);
                }
#pragma unroll
                for (int q = 0; q < QG; ++q) {
                    const bool okr = q < qn && j0 + 4 * q + g < crows;
                    u0[q].template decode<CT>(&a0[q], okr && act0);
                    u1[q].template decode<CT>(&a1[q], okr && act1);
                }
            }
#pragma unroll
            for (int q = 0; q < QG; ++q) {
                if (q >= qn) break;
#pragma unroll
                for (int ct = 0; ct < NT; ++ct) {
                    const CT bv = tc[(j0 + 4 * q + g) * TS + 16 * ct + li];
                    acc[0][ct] = M::mma(a0[q], bv, acc[0][ct]);
                    acc[1][ct] = M::mma(a1[q], bv, acc[1][ct]);
                }
            }
        }
    }
}

template <typename CT, int NT>
__device__ void expand_level_dispatch(const KParams& kp, const BlockDesc& bd, int chunk0, int ld, int c0, int nrhs,
                                      bool act0, bool act1, CT* ts, int jc, typename Mfma<CT>::acc_t acc[2][NT]) {
    switch (bd.fmt) {
        case F64: expand_level_w<F64, CT, NT>(kp, bd, chunk0, ld, c0, nrhs, act0, act1, ts, jc, acc); break;
        case F32: expand_level_w<F32, CT, NT>(kp, bd, chunk0, ld, c0, nrhs, act0, act1, ts, jc, acc); break;
        case BF16: expand_level_w<BF16, CT, NT>(kp, bd, chunk0, ld, c0, nrhs, act0, act1, ts, jc, acc); break;
        case F16: expand_level_w<F16, CT, NT>(kp, bd, chunk0, ld, c0, nrhs, act0, act1, ts, jc, acc); break;
        case E4M3: expand_level_w<E4M3, CT, NT>(kp, bd, chunk0, ld, c0, nrhs, act0, act1, ts, jc, acc); break;
        default: expand_level_w<E5M2, CT, NT>(kp, bd, chunk0, ld, c0, nrhs, act0, act1, ts, jc, acc); break;
    }
}

// Leaf GEMM operands.  X moves through LDS one 32-row step at a time
// (double-buffered, shared by the four waves): xs[c][k], row stride kXLD.
// The lane's D values for a step (its two 16-row tiles, its kKL columns)
// come straight from HBM into registers, one step ahead.
constexpr int kXLD = kStep + 4;

template <typename XT, int NT>
__device__ __forceinline__ int xs_bytes() { return 2 * 16 * NT * kXLD * int(sizeof(XT)); }

template <typename XT, int NT>
struct XStage {                                     // this thread's share of one X step
    static constexpr int CW = 16 * NT;
    static constexpr int N = (CW * (kStep / 4) + kThreads - 1) / kThreads;   // 4-element pieces
    XT v[N][4];
    bool in[N];
    // Every lane loads (pieces outside the leaf or the column range read
    // row 0 of column c0 instead and are zeroed when stored): with no
    // branch around the loads, and nothing using their values before the
    // MFMAs of the current step, the wait before those MFMAs leaves the
    // step fetched ahead in flight.
    __device__ __forceinline__ void load(const XT* Xl, int64_t ldw, int k0, int mp, int c0, int nrhs) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int e = threadIdx.x + kThreads * i;
            const int col = e >> 3, part = e & 7;    // 8 pieces of 4 rows per column
            const int k = k0 + 4 * part, c = c0 + col;
            in[i] = col < CW && k < mp && c < nrhs;
            const XT* src = Xl + (in[i] ? k + ldw * c : ldw * c0);
            if constexpr (sizeof(XT) == 4) {
                const float4 a = *reinterpret_cast<const float4*>(src);
                v[i][0] = a.x; v[i][1] = a.y; v[i][2] = a.z; v[i][3] = a.w;
            } else {
                const double2 a = reinterpret_cast<const double2*>(src)[0];
                const double2 b = reinterpret_cast<const double2*>(src)[1];
                v[i][0] = a.x; v[i][1] = a.y; v[i][2] = b.x; v[i][3] = b.y;
            }
        }
    }
    __device__ __forceinline__ void store(XT* xs) const {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int e = threadIdx.x + kThreads * i;
            const int col = e >> 3, part = e & 7;
            // (the test is needed only when the block has more pieces than the step)
            if (kThreads * N <= CW * 8 || col < CW) {
                XT* dst = xs + col * kXLD + 4 * part;
#pragma unroll
                for (int r = 0; r < 4; ++r) dst[r] = in[i] ? v[i][r] : XT(0);
            }
        }
    }
};

struct LeafD {                                      // the lane's D values of one step
    double a0[kKL], a1[kKL];
    // Branch-free like XStage::load, and the values are used as loaded:
    // lanes past the leaf's columns read columns 0..7 instead, which meet
    // the zero rows of the staged X; lanes of a row tile past the tile read
    // tile row r & 15 (present: nr >= 16), and those accumulator rows are
    // never written.  Either way the values are finite leaf entries.
    __device__ __forceinline__ void load(const double* Dp, int nr, int k, bool ok, bool act0, bool act1, int r0,
                                         int r1) {
        const int kk = ok ? k : 0;
        const int s0 = act0 ? r0 : (r0 & 15), s1 = act1 ? r1 : (r1 & 15);
#pragma unroll
        for (int q = 0; q < kKL; ++q) {
            a0[q] = Dp[int64_t(kk + q) * nr + s0];
            a1[q] = Dp[int64_t(kk + q) * nr + s1];
        }
    }
};

// one step of the leaf GEMM: B operands from the LDS X step, two column
// tiles at a time (four independent accumulators between dependent MFMAs)
template <typename XT, int NT>
__device__ __forceinline__ void leaf_mma(const XT* xs, const LeafD& d, int g, int li,
                                         typename Mfma<double>::acc_t acc[2][NT]) {
    constexpr int CP = NT >= 2 ? 2 : 1;
#pragma unroll
    for (int cp = 0; cp < NT; cp += CP) {
        double b[CP][kKL];
#pragma unroll
        for (int u = 0; u < CP; ++u) {
            const XT* src = xs + (16 * (cp + u) + li) * kXLD + kKL * g;
#pragma unroll
            for (int q = 0; q < kKL; ++q) b[u][q] = double(src[q]);
        }
#pragma unroll
        for (int q = 0; q < kKL; ++q)
#pragma unroll
            for (int u = 0; u < CP; ++u) {
                acc[0][cp + u] = Mfma<double>::mma(d.a0[q], b[u][q], acc[0][cp + u]);
                acc[1][cp + u] = Mfma<double>::mma(d.a1[q], b[u][q], acc[1][cp + u]);
            }
    }
}

// Expansion tile on the matrix cores: rows [r0, r0+nr) of leaf i (at most
// 128, a multiple of 16) for right-hand sides [c0, c0 + 16 NT).  Wave w
// owns tile rows 32w..32w+31 as two 16-row MFMA tiles.  The fp64 leaf GEMM
// and every fp64 level accumulate in fp64; levels decoded to fp32 (when AT
// is float) accumulate in fp32; the sum is rounded once into Y.  LDS: the
// two X steps, then T.  When the T of all the leaf's levels fits in the
// rest of lds_bytes it is staged once, before the leaf GEMM, and the levels
// need no barrier; otherwise it goes through jc-row chunks.
template <typename XT, typename AT, int NT>
__device__ void run_expand_w(const KParams& kp, int tile, int yg, const XT* __restrict__ Xw, int64_t ldw,
                             XT* __restrict__ Y, int64_t ldy, int nrhs, int lds_bytes, int jc, double* smem_d,
                             int* s_off) {
    using MD = Mfma<double>;
    constexpr int CW = 16 * NT;
    constexpr int TS = CW + 4;
    const ETile t = kp.etiles[tile];
    const LeafDesc L = kp.leaves[t.leaf];
    const int c0 = yg * CW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int r0 = 32 * wave + li, r1 = r0 + 16;        // tile rows of the lane's A operands
    const bool act0 = 32 * wave < t.nr, act1 = 32 * wave + 16 < t.nr;   // nr is a multiple of 16
    const int depth = kp.depth;
    unsigned char* lds = reinterpret_cast<unsigned char*>(smem_d);
    XT* xs0 = reinterpret_cast<XT*>(lds);
    XT* xs1 = xs0 + CW * kXLD;
    unsigned char* tl = lds + xs_bytes<XT, NT>();
    const int t_bytes = lds_bytes - xs_bytes<XT, NT>();
    // byte offsets of each level's staged T (level k at s_off[k-1])
    if (threadIdx.x < depth) {
        const int k = threadIdx.x + 1;
        const BlockDesc& bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
        const int w = (sizeof(AT) == 8 || bd.fmt == F64) ? 8 : 4;
        s_off[k] = round4(bd.rank) * TS * w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0;
        for (int k = 1; k <= depth; ++k) {
            const int sz = s_off[k];
            s_off[k - 1] = off;
            off += sz;
        }
        s_off[depth] = off;
    }
    __syncthreads();
    const bool staged = s_off[depth] <= t_bytes;
    if (staged) {
        for (int k = 1; k <= depth; ++k) {
            const BlockDesc& bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
            if (sizeof(AT) == 8 || bd.fmt == F64)
                stage_t<double, CW>(kp, bd, 0, round4(bd.rank), c0, nrhs, reinterpret_cast<double*>(tl + s_off[k - 1]));
            else
                stage_t<float, CW>(kp, bd, 0, round4(bd.rank), c0, nrhs, reinterpret_cast<float*>(tl + s_off[k - 1]));
        }
    }
    MD::acc_t accd[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) zero_acc(accd[a][b]);
    // leaf: D_i (tile rows, all mp columns; column-major, ld = nr) times X_i
    {
        const double* Dp = kp.leafd + L.d_off + int64_t(t.r0) * L.mp;
        const XT* Xl = Xw + L.prow0;
        const int nstep = (L.mp + kStep - 1) / kStep;
        XStage<XT, NT> xr;
        LeafD da, db;
        xr.load(Xl, ldw, 0, L.mp, c0, nrhs);
        da.load(Dp, t.nr, kKL * g, kKL * g < L.mp, act0, act1, r0, r1);   // mp and k are multiples of 8
        xr.store(xs0);
        __syncthreads();
        // Steps go in pairs (X step s in xs0 / xs1 by parity, D in da / db)
        // with one exit, and the step fetched ahead is issued
        // unconditionally (after the last pair it re-reads the last step
        // into buffers read again only by an odd count's final step), so
        // every iteration issues the same loads and the wait before the
        // MFMAs leaves the fetch ahead in flight.
        const int last = (nstep - 1) * kStep;
        int s = 0;
        for (; s + 1 < nstep; s += 2) {
            const int k1 = (s + 1) * kStep, k2 = min((s + 2) * kStep, last);
            xr.load(Xl, ldw, k1, L.mp, c0, nrhs);
            db.load(Dp, t.nr, k1 + kKL * g, k1 + kKL * g < L.mp, act0, act1, r0, r1);
            leaf_mma<XT, NT>(xs0, da, g, li, accd);
            __builtin_amdgcn_sched_barrier(0);          // keep the store's zeroing after the MFMAs
            xr.store(xs1);
            __syncthreads();
            xr.load(Xl, ldw, k2, L.mp, c0, nrhs);
            da.load(Dp, t.nr, k2 + kKL * g, k2 + kKL * g < L.mp, act0, act1, r0, r1);
            leaf_mma<XT, NT>(xs1, db, g, li, accd);
            __builtin_amdgcn_sched_barrier(0);
            xr.store(xs0);
            __syncthreads();
        }
        if (s < nstep) leaf_mma<XT, NT>(xs0, da, g, li, accd);   // odd count: the last step
    }
    // the depth ancestors' blocks whose rows contain this leaf (T staged
    // before the leaf GEMM is visible: its loop ended with a barrier)
    typename Mfma<AT>::acc_t accl[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) zero_acc(accl[a][b]);
    const int jcu = staged ? 0 : jc;
    for (int k = 1; k <= depth; ++k) {
        const BlockDesc bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
        if (bd.rank == 0) continue;
        const int chunk0 = L.prow0 - bd.urow0 + t.r0;   // the tile's chunk of the U panel
        unsigned char* ts = tl + (staged ? s_off[k - 1] : 0);
        if constexpr (sizeof(AT) == 8) {
            expand_level_dispatch<double, NT>(kp, bd, chunk0, t.nr, c0, nrhs, act0, act1,
                                              reinterpret_cast<double*>(ts), jcu, accd);
        } else {
            if (bd.fmt == F64)
                expand_level_dispatch<double, NT>(kp, bd, chunk0, t.nr, c0, nrhs, act0, act1,
                                                  reinterpret_cast<double*>(ts), jcu, accd);
            else
                expand_level_dispatch<float, NT>(kp, bd, chunk0, t.nr, c0, nrhs, act0, act1,
                                                 reinterpret_cast<float*>(ts), jcu, accl);
        }
    }
    // Y rows g+4e of each 16-row tile (fp64 layout), column li of each column tile
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            const int c = c0 + 16 * ct + li;
            if (c >= nrhs) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = 32 * wave + 16 * h + acc_row<double>(g, e);   // row within the tile
                const int pr = t.r0 + rr;                                     // padded row within the leaf
                if (rr < t.nr && pr < L.m)
                    Y[L.row0 + pr + ldy * c] = XT(accd[h][ct][e] + double(accl[h][ct][e]));
            }
        }
    }
}

// LDS of the matrix-core expansion: the two X steps, then T of all levels
// when it fits in 64 KB (jc = 0), else jc rows of T at a time, jc the
// largest multiple of 16 that fits (fp64 rows, the larger case)
bool wide_lds(const KParams& kp, int cw, size_t xbytes, int* jc, int64_t* lds) {
    const int64_t xb = 2 * int64_t(cw) * kXLD * int64_t(xbytes);
    const int64_t all = int64_t(kp.max_tstage) * (cw + 4);
    if (xb + all <= kMaxLds) {
        *jc = 0;
        *lds = xb + all;
        return true;
    }
    const int64_t rowb = int64_t(cw + 4) * 8;
    const int64_t rows = (kMaxLds - xb) / rowb / 16 * 16;
    if (rows < 16) return false;
    *jc = int(rows);
    *lds = xb + rows * rowb;
    return true;
}

template <typename XT, typename AT, int NT>
__global__ __launch_bounds__(kThreads) void k_expand_w(KParams kp, const XT* __restrict__ Xw, int64_t ldw,
                                                       XT* __restrict__ Y, int64_t ldy, int nrhs, int lds_bytes,
                                                       int jc) {
    extern __shared__ double smem_d[];
    __shared__ int s_off[kMaxDepth + 2];
    // Block b runs tile 8 (b / 8 ncg) + b % 8, column group (b / 8) % ncg:
    // consecutive blocks go to the 8 XCDs in turn, so the column groups of
    // a tile run one after another on the same XCD and the second reads
    // the tile's D from that XCD's L2.
    const int ncg = (nrhs + 16 * NT - 1) / (16 * NT);
    const int b = blockIdx.x;
    const int tile = (b / (8 * ncg)) * 8 + (b & 7), cg = (b >> 3) % ncg;
    if (tile >= kp.netiles) return;                     // whole block: before any barrier
    run_expand_w<XT, AT, NT>(kp, tile, cg, Xw, ldw, Y, ldy, nrhs, lds_bytes, jc, smem_d, s_off);
}

template <typename XT, typename AT, int NT>
hipError_t launch_wide_nt(const KParams& kp, const XT* Xw, int64_t ldw, XT* Y, int64_t ldy, int nrhs,
                          const Timer& tm) {
    hipStream_t s = tm.s;
    constexpr int NTC = NT > 4 ? 4 : NT;                // contraction: at most 64 columns per workgroup
    constexpr int CW = 16 * NT;
    if (kp.ncitems > 0) {                               // some block has a nonzero rank
        // the stacked contraction with at most two tiles to a unit takes 32
        // columns per workgroup: twice the workgroups of 64 at four waves
        // per SIMD instead of two
        constexpr int NTS = NTC > 2 ? 2 : NTC;
        const int gy = (nrhs + 16 * NTC - 1) / (16 * NTC), gys = (nrhs + 16 * NTS - 1) / (16 * NTS);
        tm.begin(1);
        const size_t lds_c = size_t(kWaves) * NTC * 256 * sizeof(double);
        if (kp.stacked > 2)
            hipLaunchKernelGGL((k_contract_w<XT, AT, NTC, 4>), dim3(kp.nsunits, gy), dim3(kThreads), lds_c, s, kp,
                               Xw, ldw, nrhs);
        else if (kp.stacked)
            hipLaunchKernelGGL((k_contract_w<XT, AT, NTS, 2>), dim3(kp.nsunits, gys), dim3(kThreads), lds_c, s, kp,
                               Xw, ldw, nrhs);
        else
            hipLaunchKernelGGL((k_contract_w<XT, AT, NTC, 0>), dim3(kp.ncitems, gy), dim3(kThreads), lds_c, s, kp,
                               Xw, ldw, nrhs);
        tm.end(1);
        tm.begin(3);
        if (kp.stacked) {
            ReduceShape rs;
            const int64_t nwg = reduce_shape(kp, nrhs, &rs);
            hipLaunchKernelGGL((k_reduce_stack<AT>), dim3(unsigned(nwg)), dim3(256), 0, s, kp, nrhs, rs);
        } else {
            // largest rank * nrhs of a block bounds the outputs per block
            const int64_t rows_y = (int64_t(kp.max_block_rank) * nrhs + 255) / 256;
            hipLaunchKernelGGL((k_reduce_items<AT>), dim3(kp.nblocks, unsigned(rows_y)), dim3(256), 0, s, kp, nrhs);
        }
        tm.end(3);
    }
    // LDS: two X steps, then T of all levels if it fits in 64 KB, else T
    // in chunks of as many rows as fit (a multiple of 16)
    int jc = 0;
    int64_t lds = 0;
    if (!wide_lds(kp, CW, sizeof(XT), &jc, &lds)) return hipErrorInvalidConfiguration;
    tm.begin(2);
    hipLaunchKernelGGL((k_expand_w<XT, AT, NT>), dim3(8 * ((nrhs + CW - 1) / CW) * ((kp.netiles + 7) / 8)),
                       dim3(kThreads),
                       size_t(lds), s, kp, Xw, ldw, Y, ldy, nrhs, int(lds), jc);
    tm.end(2);
    return hipGetLastError();
}

template <typename XT, typename AT>
hipError_t launch_wide(const KParams& kp, const void* Xv, int64_t ldx, void* Yv, int64_t ldy, int nrhs,
                       const Timer& tm) {
    const XT* X = static_cast<const XT*>(Xv);
    XT* Y = static_cast<XT*>(Yv);
    // vector loads of X need 16-byte aligned columns: otherwise use the padded copy
    const bool aligned = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((ldx * int64_t(sizeof(XT))) % 16 == 0);
    const XT* Xw = X;
    int64_t ldw = ldx;
    if (kp.padded || !aligned) {
        tm.begin(0);
        hipLaunchKernelGGL((k_padx<XT>), dim3(kp.nleaves), dim3(256), 0, tm.s, kp, X, ldx, nrhs);
        tm.end(0);
        Xw = static_cast<const XT*>(kp.xpad);
        ldw = kp.npad;
    }
    if (nrhs <= 16) return launch_wide_nt<XT, AT, 1>(kp, Xw, ldw, Y, ldy, nrhs, tm);
    if (nrhs <= 32) return launch_wide_nt<XT, AT, 2>(kp, Xw, ldw, Y, ldy, nrhs, tm);
    return launch_wide_nt<XT, AT, 4>(kp, Xw, ldw, Y, ldy, nrhs, tm);
}

}  // namespace
}  // namespace hodlr

#endif  // HODLR_WIDE_PATH_H
