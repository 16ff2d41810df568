// Wave path of the HODLR product (nrhs < kWideMin): contraction items,
// fp64 leaf tiles, expansion tiles, and their launches.  Included by
// kernels.hip only.
#ifndef HODLR_WAVE_PATH_H
#define HODLR_WAVE_PATH_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev_common.h"

namespace hodlr {
namespace {

// ---------------------------------------------------------------------------
// contraction item: partial T_b over rows [r0, r0+nr) of the V panel
// ---------------------------------------------------------------------------
// Lane l owns rows 4l..4l+3 of every 256-row slab of the item (at most 16
// slabs).  Wave w owns columns w, w+4, w+8, ...: for each group of CJ of
// its columns it issues the loads of every slab at once, accumulates per
// lane, sums across the wave (DPP) and lane 63 stores the column's partial
// (device-coherent).  No barrier inside the column loop.
template <int F, typename CT, typename XT, int RG>
__device__ void contract_item(const KParams& kp, const CItem& it, const BlockDesc& bd,
                              const XT* __restrict__ X, int64_t ldx, int nrhs) {
    constexpr int S = Codec<F>::kBytes;
    constexpr int GS = kItemRowsMax / 256;                          // slabs per item
    constexpr int CJ0 = (sizeof(CT) == 8 ? 8 : 16) / (GS / 4) / RG;   // loads in flight ~ CJ * slabs
    constexpr int CJ = CJ0 > 1 ? CJ0 : 1;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int p = bd.rank;
    const uint8_t* Vp = kp.fac + bd.v_off + int64_t(it.r0) * p * S;   // the item's chunk
    const int64_t ld = it.nr;
    double* part = kp.partial + it.poff * nrhs;
    const int nslab = (it.nr + 255) >> 8;
    const int64_t xrow0 = int64_t(bd.vrow0) + it.r0;
    for (int rb = 0; rb < nrhs; rb += RG) {
        for (int j0 = wave * CJ; j0 < p; j0 += kWaves * CJ) {
            CT acc[CJ][RG];
#pragma unroll
            for (int c = 0; c < CJ; ++c)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) acc[c][rg] = CT(0);
            for (int s0 = 0; s0 < nslab; s0 += GS / 4) {            // slab groups of GS/4
                CT xr[GS / 4][4][RG];
                CT v[GS / 4][CJ][4];
                if constexpr (direct_codes<F, CT>() && sizeof(XT) == sizeof(CT)) {
#pragma unroll
                    for (int q = 0; q < GS / 4; ++q) {
                        const int row = (s0 + q) * 256 + 4 * lane;
                        const bool ok = s0 + q < nslab && row < it.nr;
#pragma unroll
                        for (int c = 0; c < CJ; ++c) {
                            if (ok && j0 + c < p)
                                Codec<F>::template load<4, CT>(Vp + (int64_t(j0 + c) * ld + row) * S, v[q][c]);
                            else
                                v[q][c][0] = v[q][c][1] = v[q][c][2] = v[q][c][3] = CT(0);
                        }
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                xr[q][i][rg] = (ok && row + i < it.nr && rb + rg < nrhs)
                                                   ? CT(X[xrow0 + row + i + ldx * (rb + rg)]) : CT(0);
                    }
                } else {
                    // codes or X that need decoding: all loads of the slab
                    // group first, from addresses clamped into the item (rank
                    // -> j0 < p, row -> 0, column -> 0), then decoded and masked
                    RawCodes<F, 4> rv[GS / 4][CJ];
                    RawX<XT, 1> rx[GS / 4][4][RG];
#pragma unroll
                    for (int q = 0; q < GS / 4; ++q) {
                        const int row = (s0 + q) * 256 + 4 * lane;
                        const bool ok = s0 + q < nslab && row < it.nr;
#pragma unroll
                        for (int c = 0; c < CJ; ++c)
                            rv[q][c].load(Vp + (int64_t(j0 + c < p ? j0 + c : j0) * ld + (ok ? row : 0)) * S);
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const bool okx = ok && row + i < it.nr;
                                rx[q][i][rg].load(X + xrow0 + (okx ? row + i : 0) +
                                                  ldx * (rb + rg < nrhs ? rb + rg : 0));
                            }
                    }
#pragma unroll
                    for (int q = 0; q < GS / 4; ++q) {
                        const int row = (s0 + q) * 256 + 4 * lane;
                        const bool ok = s0 + q < nslab && row < it.nr;
#pragma unroll
                        for (int c = 0; c < CJ; ++c) rv[q][c].template decode<CT>(v[q][c], ok && j0 + c < p);
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                rx[q][i][rg].template convert<CT>(&xr[q][i][rg],
                                                                  ok && row + i < it.nr && rb + rg < nrhs);
                    }
                }
#pragma unroll
                for (int q = 0; q < GS / 4; ++q)
#pragma unroll
                    for (int c = 0; c < CJ; ++c)
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                            for (int i = 0; i < 4; ++i) acc[c][rg] += v[q][c][i] * xr[q][i][rg];
            }
#pragma unroll
            for (int c = 0; c < CJ; ++c)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    const CT r = wave_sum63(acc[c][rg]);
                    if (lane == 63 && j0 + c < p && rb + rg < nrhs)
                        st_coh(part + int64_t(rb + rg) * p + j0 + c, double(r));
                }
        }
    }
}

template <typename XT, typename AT, int RG>
__device__ void run_contract_item(const KParams& kp, const CItem& it, const BlockDesc& bd,
                                  const XT* __restrict__ X, int64_t ldx, int nrhs) {
    switch (bd.fmt) {
        case F64: contract_item<F64, double, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case F32: contract_item<F32, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case BF16: contract_item<BF16, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case F16: contract_item<F16, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case E4M3: contract_item<E4M3, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        default: contract_item<E5M2, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
    }
}

// The last item of block b to arrive adds the block's partials in item
// order: all of them are staged in LDS first (every load in flight), then
// each output is summed and scaled, and T_b is stored device-coherently.
template <typename CT>
__device__ void finish_block(const KParams& kp, const BlockDesc& bd, int nrhs, double* __restrict__ stage,
                             int stage_cap) {
    const int p = bd.rank;
    const int total = p * nrhs;                           // outputs, rhs-major
    const int nit = bd.nitems;
    const double* src = kp.partial + kp.citems[bd.item0].poff * nrhs;   // item c at src + c * total
    double* dst = kp.T + bd.t_off * nrhs;
    if (nit > stage_cap) {
        for (int r = threadIdx.x; r < total; r += kThreads) {
            CT s = CT(0);
#pragma unroll 8
            for (int c = 0; c < nit; ++c) s += CT(ld_coh(src + int64_t(c) * total + r));
            st_coh(dst + r, double(s) * kp.tscale[bd.ts_off + r % p]);
        }
        return;
    }
    const int oc_max = stage_cap / nit;
    for (int o0 = 0; o0 < total; o0 += oc_max) {
        const int oc = (total - o0) < oc_max ? (total - o0) : oc_max;
        for (int e = threadIdx.x; e < nit * oc; e += kThreads) {
            const int c = e / oc, r = e - c * oc;
            stage[e] = ld_coh(src + int64_t(c) * total + o0 + r);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < oc; r += kThreads) {
            CT s = CT(0);
            for (int c = 0; c < nit; ++c) s += CT(stage[c * oc + r]);
            st_coh(dst + o0 + r, double(s) * kp.tscale[bd.ts_off + (o0 + r) % p]);
        }
        __syncthreads();
    }
}

template <typename XT, typename AT, int RG>
__device__ void run_contract(const KParams& kp, int item, const XT* __restrict__ X, int64_t ldx, int nrhs,
                             unsigned char* smem, int* s_flag, int stage_cap) {
    const CItem it = kp.citems[item];
    const BlockDesc bd = kp.blocks[it.block];
    run_contract_item<XT, AT, RG>(kp, it, bd, X, ldx, nrhs);
    // publish: the partial's stores complete before the arrival is counted;
    // the last arrival reduces the block and clears the counter for the next
    // launch (nobody else touches it in this one)
    drain_and_sync();
    if (threadIdx.x == 0) *s_flag = (add_coh(arrivals(kp) + it.block, 1) == bd.nitems - 1);
    __syncthreads();
    if (*s_flag) {
        double* stage = reinterpret_cast<double*>(smem);
        if (bd.fmt == F64)
            finish_block<double>(kp, bd, nrhs, stage, stage_cap);
        else
            finish_block<AT>(kp, bd, nrhs, stage, stage_cap);
        if (threadIdx.x == 0) st_coh(arrivals(kp) + it.block, 0);
    }
}

// ---------------------------------------------------------------------------
// leaf tiles and expansion tiles: Y rows of one leaf = D_i x_i + sum_k U_b T_b
// ---------------------------------------------------------------------------
// Leaf tile of the first launch (wave path): W rows of the tile = D_i X_i,
// summed over the four waves in fp64 and stored once (padded row space,
// ld npad).  Lane l owns rows RPL*l.. of the tile; wave w walks columns
// w, w+4, ... of D_i with kLeafUnroll loads in flight; x_i is staged in LDS.
template <typename XT, int RG, int RPL>
__device__ void run_leaf(const KParams& kp, int tile, const XT* __restrict__ X, int64_t ldx, int nrhs,
                         unsigned char* smem) {
    constexpr int TR = 64 * RPL;                    // rows per tile
    const ETile t = kp.etiles[tile];
    const LeafDesc L = kp.leaves[t.leaf];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const bool act = RPL * lane < t.nr;
    // LDS: x of the leaf [m][RG] | wave sums [kWaves][TR]
    double* xs = reinterpret_cast<double*>(smem);
    double* red = xs + int64_t(L.m) * RG;
    for (int rb = 0; rb < nrhs; rb += RG) {
        for (int idx = threadIdx.x; idx < L.m * RG; idx += kThreads) {
            const int c = idx / RG, rg = idx % RG;
            xs[idx] = (rb + rg < nrhs) ? double(X[L.row0 + c + ldx * (rb + rg)]) : 0.0;
        }
        __syncthreads();
        double dacc[RPL][RG];
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) dacc[i][rg] = 0.0;
        // the tile's chunk of D_i: column-major, ld = t.nr
        const uint8_t* Dp = reinterpret_cast<const uint8_t*>(kp.leafd + L.d_off + int64_t(t.r0) * L.mp + RPL * lane);
        const int64_t ldb = int64_t(t.nr) * 8;
        int c = wave;
        for (; c + (kLeafUnroll - 1) * kWaves < L.m; c += kLeafUnroll * kWaves) {
            double d[kLeafUnroll][RPL];
#pragma unroll
            for (int q = 0; q < kLeafUnroll; ++q) {
                if (act)
                    Codec<F64>::template load<RPL, double>(Dp + int64_t(c + q * kWaves) * ldb, d[q]);
                else
#pragma unroll
                    for (int i = 0; i < RPL; ++i) d[q][i] = 0.0;
            }
#pragma unroll
            for (int q = 0; q < kLeafUnroll; ++q)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    const double xv = xs[(c + q * kWaves) * RG + rg];
#pragma unroll
                    for (int i = 0; i < RPL; ++i) dacc[i][rg] += d[q][i] * xv;
                }
        }
        for (; c < L.m; c += kWaves) {
            double d[RPL];
            if (act)
                Codec<F64>::template load<RPL, double>(Dp + int64_t(c) * ldb, d);
            else
#pragma unroll
                for (int i = 0; i < RPL; ++i) d[i] = 0.0;
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                const double xv = xs[c * RG + rg];
#pragma unroll
                for (int i = 0; i < RPL; ++i) dacc[i][rg] += d[i] * xv;
            }
        }
        // sum the waves' partial rows in fp64; store W once
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) red[wave * TR + RPL * lane + i] = dacc[i][rg];
            __syncthreads();
            for (int r = threadIdx.x; r < TR; r += kThreads) {
                double sum = red[r];
#pragma unroll
                for (int w = 1; w < kWaves; ++w) sum += red[w * TR + r];
                if (r < t.nr && rb + rg < nrhs) kp.W[int64_t(L.prow0) + t.r0 + r + kp.npad * (rb + rg)] = sum;
            }
            __syncthreads();
        }
    }
}

// Expansion tile of the second launch (wave path): Y rows of one leaf tile
// = W + sum_k U_b T_b over the tile's depth ancestor blocks.
//
// The tile's work is cut into units of (level k, group of kUnroll columns
// of level k's U chunk), numbered level by level, and unit u runs on wave
// u mod kExpandWaves: every wave streams about the same number of U
// columns whatever the ranks of the levels, so the chain of dependent
// loads a wave walks is about (sum of the ranks) / (kUnroll x waves) long.
// A unit's kUnroll column loads are all issued before its FMAs.  Each wave
// accumulates its units into per-row partials; the waves' partials are
// added in LDS in wave order, W (loaded before the units) is added and Y is
// written once (the order of every sum is fixed, so the result is
// deterministic).
constexpr int kExpandWaves = 8;
constexpr int kExpandThreads = 64 * kExpandWaves;

// columns of one unit of a level stored in format f (fp64 levels take half)
__device__ __forceinline__ int unit_cols(int f) { return f == F64 ? kUnroll / 2 : kUnroll; }

template <int F, typename CT, typename AT, int RG, int RPL>
__device__ __forceinline__ void expand_unit(const KParams& kp, const BlockDesc& bd, int j0, int chunk0, int rin,
                                            int ld, bool act, const double* __restrict__ ts, AT acc[RPL][RG]) {
    constexpr int S = Codec<F>::kBytes;
    constexpr int UN = F == F64 ? kUnroll / 2 : kUnroll;          // columns per unit (= unit_cols(F))
    const int p = bd.rank;
    CT u[UN][RPL];
    if constexpr (direct_codes<F, CT>()) {
        const uint8_t* Up = kp.fac + bd.u_off + (int64_t(chunk0) * p + rin) * S;
#pragma unroll
        for (int q = 0; q < UN; ++q) {
            if (act && j0 + q < p)
                Codec<F>::template load<RPL, CT>(Up + int64_t(j0 + q) * ld * S, u[q]);
            else
#pragma unroll
                for (int i = 0; i < RPL; ++i) u[q][i] = CT(0);
        }
    } else {
        // codes that need decoding: every column's codes are loaded before
        // any is decoded, from addresses clamped into the chunk (rank -> j0
        // < p, inactive lanes -> row 0)
        const uint8_t* Up = kp.fac + bd.u_off + (int64_t(chunk0) * p + (act ? rin : 0)) * S;
        RawCodes<F, RPL> ru[UN];
#pragma unroll
        for (int q = 0; q < UN; ++q) ru[q].load(Up + int64_t(j0 + q < p ? j0 + q : j0) * ld * S);
#pragma unroll
        for (int q = 0; q < UN; ++q) ru[q].template decode<CT>(u[q], act && j0 + q < p);
    }
    CT lacc[RPL][RG];
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) lacc[i][rg] = CT(0);
#pragma unroll
    for (int q = 0; q < UN; ++q) {
        if (j0 + q >= p) break;
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            const CT tv = CT(ts[rg * p + j0 + q]);
#pragma unroll
            for (int i = 0; i < RPL; ++i) lacc[i][rg] += u[q][i] * tv;
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) acc[i][rg] += AT(lacc[i][rg]);
}

template <typename XT, typename AT, int RG, int RPL>
__device__ void run_expand(const KParams& kp, int tile, XT* __restrict__ Y, int64_t ldy, int nrhs,
                           unsigned char* smem, int* s_off) {
    constexpr int TR = 64 * RPL;                    // rows per tile
    static_assert(TR <= kExpandThreads, "one Y row per thread");
    const ETile t = kp.etiles[tile];
    const LeafDesc L = kp.leaves[t.leaf];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const bool act = RPL * lane < t.nr;
    const int depth = kp.depth;
    // LDS: T of every level [sum p][RG] | wave sums [kExpandWaves][TR].
    // s_off[0..depth]: T offsets of the levels (level k at s_off[k-1]);
    // s_off[kMaxDepth+1 ..]: first unit of each level, then the unit count.
    int* s_u0 = s_off + kMaxDepth + 1;
    double* ts = reinterpret_cast<double*>(smem);
    if (threadIdx.x < depth) {
        const int k = threadIdx.x + 1;
        const BlockDesc& bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
        s_off[k] = bd.rank * RG;
        s_u0[k] = (bd.rank + unit_cols(bd.fmt) - 1) / unit_cols(bd.fmt);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0, u0 = 0;
        for (int k = 1; k <= depth; ++k) {
            const int r = s_off[k], nu = s_u0[k];
            s_off[k - 1] = off;
            s_u0[k - 1] = u0;
            off += r;
            u0 += nu;
        }
        s_off[depth] = off;
        s_u0[depth] = u0;
    }
    __syncthreads();
    const int nunits = s_u0[depth];
    AT* red = reinterpret_cast<AT*>(ts + s_off[depth]);
    for (int rb = 0; rb < nrhs; rb += RG) {
        // the leaf product W of the rows this thread writes, loaded before the units
        AT wv[RG];
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            const int lr = t.r0 + int(threadIdx.x);
            wv[rg] = (int(threadIdx.x) < TR && int(threadIdx.x) < t.nr && lr < L.m && rb + rg < nrhs)
                         ? AT(kp.W[int64_t(L.prow0) + lr + kp.npad * (rb + rg)])
                         : AT(0);
        }
        AT acc[RPL][RG];
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) acc[i][rg] = AT(0);
        // T of every level for right-hand sides [rb, rb+RG): one pass of loads
        for (int idx = threadIdx.x; idx < s_off[depth]; idx += kExpandThreads) {
            int k = 1;
            while (k < depth && s_off[k] <= idx) ++k;
            const BlockDesc& bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
            const int p = bd.rank;
            const int r = idx - s_off[k - 1];
            const int rg = r / p, j = r - rg * p;
            ts[idx] = (rb + rg < nrhs) ? kp.T[bd.t_off * nrhs + int64_t(rb + rg) * p + j] : 0.0;
        }
        __syncthreads();
        int k = 1;
        for (int u = wave; u < nunits; u += kExpandWaves) {
            while (s_u0[k] <= u) ++k;                // level of unit u (units ascend by level)
            const int b = (1 << k) - 2 + (t.leaf >> (depth - k));
            const BlockDesc bd = kp.blocks[b];
            const int j0 = (u - s_u0[k - 1]) * unit_cols(bd.fmt);
            const int c0 = L.prow0 - bd.urow0 + t.r0;
            const int rin = RPL * lane;
            const double* tk = ts + s_off[k - 1];
            switch (bd.fmt) {
                case F64: expand_unit<F64, double, AT, RG, RPL>(kp, bd, j0, c0, rin, t.nr, act, tk, acc); break;
                case F32: expand_unit<F32, AT, AT, RG, RPL>(kp, bd, j0, c0, rin, t.nr, act, tk, acc); break;
                case BF16: expand_unit<BF16, AT, AT, RG, RPL>(kp, bd, j0, c0, rin, t.nr, act, tk, acc); break;
                case F16: expand_unit<F16, AT, AT, RG, RPL>(kp, bd, j0, c0, rin, t.nr, act, tk, acc); break;
                case E4M3: expand_unit<E4M3, AT, AT, RG, RPL>(kp, bd, j0, c0, rin, t.nr, act, tk, acc); break;
                default: expand_unit<E5M2, AT, AT, RG, RPL>(kp, bd, j0, c0, rin, t.nr, act, tk, acc); break;
            }
        }
        // sum the waves' partial rows, add the leaf product; write Y once
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) red[wave * TR + RPL * lane + i] = acc[i][rg];
            __syncthreads();
            for (int r = threadIdx.x; r < TR; r += kExpandThreads) {
                AT sum = red[r];
#pragma unroll
                for (int w = 1; w < kExpandWaves; ++w) sum += red[w * TR + r];
                const int lr = t.r0 + r;
                if (r < t.nr && lr < L.m && rb + rg < nrhs) Y[L.row0 + lr + ldy * (rb + rg)] = XT(sum + wv[rg]);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// the two launches
// ---------------------------------------------------------------------------
// First launch: workgroups [0, ncitems) take contraction items, the rest
// the leaf tiles (nothing in it waits for anything else in it).
template <typename XT, typename AT, int RG, int RPL>
__device__ void run_phase1(const KParams& kp, int w, const XT* __restrict__ Xc, int64_t ldc,
                           const XT* __restrict__ X, int64_t ldx, int nrhs, int stage_cap, unsigned char* smem,
                           int* s_flag) {
    if (w < kp.ncitems)
        run_contract<XT, AT, RG>(kp, w, Xc, ldc, nrhs, smem, s_flag, stage_cap);
    else
        run_leaf<XT, RG, RPL>(kp, w - kp.ncitems, X, ldx, nrhs, smem);
}

template <typename XT, typename AT, int RG, int RPL>
__global__ __launch_bounds__(kThreads, HODLR_CONTRACT_MINW) void k_phase1(KParams kp, const XT* __restrict__ Xc,
                                                                         int64_t ldc, const XT* __restrict__ X,
                                                                         int64_t ldx, int nrhs, int stage_cap) {
    extern __shared__ double smem_d[];
    __shared__ int s_flag;
    run_phase1<XT, AT, RG, RPL>(kp, blockIdx.x, Xc, ldc, X, ldx, nrhs, stage_cap,
                                reinterpret_cast<unsigned char*>(smem_d), &s_flag);
}

template <typename XT, typename AT, int RG, int RPL>
__global__ __launch_bounds__(kExpandThreads) void k_expand(KParams kp, XT* __restrict__ Y, int64_t ldy, int nrhs) {
    extern __shared__ double smem_d[];
    __shared__ int s_off[2 * (kMaxDepth + 1)];
    run_expand<XT, AT, RG, RPL>(kp, blockIdx.x, Y, ldy, nrhs, reinterpret_cast<unsigned char*>(smem_d), s_off);
}

// ---------------------------------------------------------------------------
// padded copy of X (only when some leaf size is not a multiple of 16)
// ---------------------------------------------------------------------------
template <typename XT>
__device__ void padx_leaf(const KParams& kp, int leaf, const XT* __restrict__ X, int64_t ldx, int nrhs) {
    const LeafDesc L = kp.leaves[leaf];
    XT* Xp = static_cast<XT*>(kp.xpad);
    const int64_t total = int64_t(L.mp) * nrhs;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int64_t r = idx % L.mp, c = idx / L.mp;
        Xp[L.prow0 + r + kp.npad * c] = r < L.m ? X[L.row0 + r + ldx * c] : XT(0);
    }
}

template <typename XT>
__global__ __launch_bounds__(256) void k_padx(KParams kp, const XT* __restrict__ X, int64_t ldx, int nrhs) {
    padx_leaf<XT>(kp, blockIdx.x, X, ldx, nrhs);
}

struct Timer {            // optional event pair around each phase
    void* const* ev;
    bool* ran;
    hipStream_t s;
    void begin(int ph) const {
        if (ev) (void)hipEventRecord(static_cast<hipEvent_t>(ev[2 * ph]), s);
    }
    void end(int ph) const {
        if (ev) {
            (void)hipEventRecord(static_cast<hipEvent_t>(ev[2 * ph + 1]), s);
            ran[ph] = true;
        }
    }
};

constexpr int kRPL = kTileRows / 64;       // rows per lane in expansion tiles

constexpr int kStageMax = 4096;   // doubles of LDS for staging a block's partials

int stage_cap(const KParams& kp, int rg) {
    const int64_t need = int64_t(kp.max_items_rank) * rg;
    return int(need < kStageMax ? (need > 0 ? need : 1) : kStageMax);
}

// expansion tile LDS (wave path): T of its levels (doubles) | wave sums
size_t lds_expand(const KParams& kp, int rg, size_t acc_bytes) {
    return size_t(kp.max_rank_path) * rg * 8 + size_t(kExpandWaves) * kTileRows * acc_bytes;
}

// first launch LDS: the larger of a contraction item's staging and a leaf
// tile's x of the leaf plus wave sums (doubles)
size_t lds_phase1(const KParams& kp, int rg) {
    const size_t leaf = (size_t(kp.max_leaf) * rg + size_t(kWaves) * kTileRows) * 8;
    const size_t stage = size_t(stage_cap(kp, rg)) * 8;
    return leaf > stage ? leaf : stage;
}

template <typename XT, typename AT, int RG, int RPL>
hipError_t launch_typed(const KParams& kp, const void* Xv, int64_t ldx, void* Yv, int64_t ldy, int nrhs,
                        const Timer& tm) {
    hipStream_t s = tm.s;
    const XT* X = static_cast<const XT*>(Xv);
    XT* Y = static_cast<XT*>(Yv);
    const XT* Xc = X;
    int64_t ldc = ldx;
    if (kp.padded && kp.ncitems > 0) {
        tm.begin(0);
        hipLaunchKernelGGL((k_padx<XT>), dim3(kp.nleaves), dim3(256), 0, s, kp, X, ldx, nrhs);
        tm.end(0);
        Xc = static_cast<const XT*>(kp.xpad);
        ldc = kp.npad;
    }
    const int sc = stage_cap(kp, RG);
    tm.begin(1);
    hipLaunchKernelGGL((k_phase1<XT, AT, RG, RPL>), dim3(kp.ncitems + kp.netiles), dim3(kThreads),
                       lds_phase1(kp, RG), s, kp, Xc, ldc, X, ldx, nrhs, sc);
    tm.end(1);
    tm.begin(2);
    hipLaunchKernelGGL((k_expand<XT, AT, RG, RPL>), dim3(kp.netiles), dim3(kExpandThreads),
                       lds_expand(kp, RG, sizeof(AT)), s, kp, Y, ldy, nrhs);
    tm.end(2);
    return hipGetLastError();
}

template <typename XT, typename AT>
hipError_t launch_rg(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs,
                     const Timer& tm) {
    // the widest right-hand-side group (at most 4: wider ones spill registers)
    // whose LDS fits in 64 KB
    int rg = nrhs == 1 ? 1 : nrhs == 2 ? 2 : 4;
    auto fits = [&](int g) { return lds_expand(kp, g, sizeof(AT)) <= kMaxLds && lds_phase1(kp, g) <= kMaxLds; };
    while (rg > 1 && !fits(rg)) rg /= 2;
    if (!fits(rg)) return hipErrorInvalidConfiguration;
    if (rg == 1) return launch_typed<XT, AT, 1, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
    if (rg == 2) return launch_typed<XT, AT, 2, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
    return launch_typed<XT, AT, 4, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
}

}  // namespace
}  // namespace hodlr

#endif  // HODLR_WAVE_PATH_H
