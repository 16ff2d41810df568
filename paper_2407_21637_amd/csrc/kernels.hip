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
// the section "many right-hand sides").  Batched products run the same
// device code from persistent kernels (section "batched products").
//
// Stored codes are converted in registers (Sect. 3.3: low-precision
// storage cast to the working precision on the fly).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hodlr_internal.h"

namespace hodlr {
namespace {

// ---------------------------------------------------------------------------
// decoding N consecutive codes of one column (N rows a lane owns)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float half_bits_to_float(uint32_t h) {
    _Float16 v = __builtin_bit_cast(_Float16, uint16_t(h));
    return float(v);
}

// fp8 E4M3FN -> fp16 bits: sign to bit 15, the 7 magnitude bits to bits
// 7..13.  The fp16 number is the e4m3 value times 2^-8 (subnormals too); the
// 2^8 is folded into the block's column scales.
__device__ __forceinline__ float e4m3_scaled(uint32_t c) {
    return half_bits_to_float(((c & 0x80u) << 8) | ((c & 0x7fu) << 7));
}

// fp8 E5M2 is the top byte of an fp16.
__device__ __forceinline__ float e5m2(uint32_t c) { return half_bits_to_float((c & 0xffu) << 8); }

template <int F>
struct Codec;

template <>
struct Codec<F64> {
    static constexpr int kBytes = 8;
    template <int N, typename CT>
    __device__ static void load(const uint8_t* p, CT v[N]) {
        if constexpr (N == 4) {
            const double2 a = *reinterpret_cast<const double2*>(p);
            const double2 b = *reinterpret_cast<const double2*>(p + 16);
            v[0] = CT(a.x); v[1] = CT(a.y); v[2] = CT(b.x); v[3] = CT(b.y);
        } else if constexpr (N == 2) {
            const double2 a = *reinterpret_cast<const double2*>(p);
            v[0] = CT(a.x); v[1] = CT(a.y);
        } else {
            v[0] = CT(*reinterpret_cast<const double*>(p));
        }
    }
};

template <>
struct Codec<F32> {
    static constexpr int kBytes = 4;
    template <int N, typename CT>
    __device__ static void load(const uint8_t* p, CT v[N]) {
        if constexpr (N == 4) {
            const float4 a = *reinterpret_cast<const float4*>(p);
            v[0] = CT(a.x); v[1] = CT(a.y); v[2] = CT(a.z); v[3] = CT(a.w);
        } else if constexpr (N == 2) {
            const float2 a = *reinterpret_cast<const float2*>(p);
            v[0] = CT(a.x); v[1] = CT(a.y);
        } else {
            v[0] = CT(*reinterpret_cast<const float*>(p));
        }
    }
};

template <>
struct Codec<BF16> {   // bf16 is the top half of an fp32
    static constexpr int kBytes = 2;
    template <int N, typename CT>
    __device__ static void load(const uint8_t* p, CT v[N]) {
        if constexpr (N == 4) {
            const uint2 a = *reinterpret_cast<const uint2*>(p);
            v[0] = CT(__uint_as_float(a.x << 16));
            v[1] = CT(__uint_as_float(a.x & 0xffff0000u));
            v[2] = CT(__uint_as_float(a.y << 16));
            v[3] = CT(__uint_as_float(a.y & 0xffff0000u));
        } else if constexpr (N == 2) {
            const uint32_t a = *reinterpret_cast<const uint32_t*>(p);
            v[0] = CT(__uint_as_float(a << 16));
            v[1] = CT(__uint_as_float(a & 0xffff0000u));
        } else {
            v[0] = CT(__uint_as_float(uint32_t(*reinterpret_cast<const uint16_t*>(p)) << 16));
        }
    }
};

template <>
struct Codec<F16> {
    static constexpr int kBytes = 2;
    template <int N, typename CT>
    __device__ static void load(const uint8_t* p, CT v[N]) {
        if constexpr (N == 4) {
            const uint2 a = *reinterpret_cast<const uint2*>(p);
            v[0] = CT(half_bits_to_float(a.x & 0xffffu));
            v[1] = CT(half_bits_to_float(a.x >> 16));
            v[2] = CT(half_bits_to_float(a.y & 0xffffu));
            v[3] = CT(half_bits_to_float(a.y >> 16));
        } else if constexpr (N == 2) {
            const uint32_t a = *reinterpret_cast<const uint32_t*>(p);
            v[0] = CT(half_bits_to_float(a & 0xffffu));
            v[1] = CT(half_bits_to_float(a >> 16));
        } else {
            v[0] = CT(half_bits_to_float(*reinterpret_cast<const uint16_t*>(p)));
        }
    }
};

template <>
struct Codec<E4M3> {
    static constexpr int kBytes = 1;
    template <int N, typename CT>
    __device__ static void load(const uint8_t* p, CT v[N]) {
        uint32_t w;
        if constexpr (N == 4) w = *reinterpret_cast<const uint32_t*>(p);
        else if constexpr (N == 2) w = *reinterpret_cast<const uint16_t*>(p);
        else w = *p;
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = CT(e4m3_scaled(w >> (8 * i)));
    }
};

template <>
struct Codec<E5M2> {
    static constexpr int kBytes = 1;
    template <int N, typename CT>
    __device__ static void load(const uint8_t* p, CT v[N]) {
        uint32_t w;
        if constexpr (N == 4) w = *reinterpret_cast<const uint32_t*>(p);
        else if constexpr (N == 2) w = *reinterpret_cast<const uint16_t*>(p);
        else w = *p;
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = CT(e5m2(w >> (8 * i)));
    }
};

// ---------------------------------------------------------------------------
// wave64 sum; the total ends in lane 63
// ---------------------------------------------------------------------------
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, false);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dppf(float v) {
    return __int_as_float(dpp<CTRL, ROWMASK>(__float_as_int(v)));
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dppd(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = dpp<CTRL, ROWMASK>(int(uint32_t(b)));
    const int hi = dpp<CTRL, ROWMASK>(int(uint32_t(b >> 32)));
    return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

__device__ __forceinline__ float wave_sum63(float v) {
    v += dppf<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dppf<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dppf<0x141, 0xf>(v);   // row_half_mirror
    v += dppf<0x140, 0xf>(v);   // row_mirror
    v += dppf<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v += dppf<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    return v;
}

__device__ __forceinline__ double wave_sum63(double v) {
    v += dppd<0xb1, 0xf>(v);
    v += dppd<0x4e, 0xf>(v);
    v += dppd<0x141, 0xf>(v);
    v += dppd<0x140, 0xf>(v);
    v += dppd<0x142, 0xa>(v);
    v += dppd<0x143, 0xc>(v);
    return v;
}

// ---------------------------------------------------------------------------
// synchronisation words (int32 workspace, zero between launches)
// ---------------------------------------------------------------------------
//   sync[kSyncHead + b]: arrivals of block b's contraction items.

__device__ __forceinline__ int* arrivals(const KParams& kp) { return kp.sync + kSyncHead; }

// Data shared between workgroups of one launch (partials, T, counters) is
// written and read with device-coherent accesses (relaxed atomics at agent
// scope: loads/stores that go to the coherence point instead of an XCD's
// private L2), and published by waiting for the stores to complete before
// the counter or flag update.  This avoids device-wide fences, which write
// back and invalidate a whole L2 each time.
__device__ __forceinline__ void st_coh(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_coh(int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_coh(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// all of this workgroup's outstanding memory operations complete, then sync
__device__ __forceinline__ void drain_and_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}



constexpr int kWaves = 4;            // waves per workgroup
constexpr int kThreads = 64 * kWaves;
#ifndef HODLR_U_UNROLL
#define HODLR_U_UNROLL 8             // U columns in flight per wave in the expansion
#endif
#ifndef HODLR_LEAF_UNROLL
#define HODLR_LEAF_UNROLL 16         // leaf columns in flight per wave
#endif
#ifndef HODLR_EXPAND_MINW
#define HODLR_EXPAND_MINW 2          // k_expand: minimum resident waves per SIMD
#endif
#ifndef HODLR_CONTRACT_MINW
#define HODLR_CONTRACT_MINW 2
#endif
constexpr int kUnroll = HODLR_U_UNROLL;
constexpr int kLeafUnroll = HODLR_LEAF_UNROLL;

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
// expansion tile: Y rows of one leaf = D_i x_i + sum_k U_b T_b
// ---------------------------------------------------------------------------
// chunk0: node-relative padded row where the tile's chunk of the U panel
// starts; rin: the lane's first row within the tile; ld: tile rows.
template <int F, typename CT, typename AT, int RG, int RPL>
__device__ void expand_level(const KParams& kp, const BlockDesc& bd, int chunk0, int rin, int ld, bool act,
                             const double* __restrict__ ts, AT acc[RPL][RG]) {
    constexpr int S = Codec<F>::kBytes;
    constexpr int UN = sizeof(CT) == 8 ? kUnroll / 2 : kUnroll;   // columns in flight
    const int p = bd.rank;
    const uint8_t* Up = kp.fac + bd.u_off + (int64_t(chunk0) * p + rin) * S;
    CT lacc[RPL][RG];
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) lacc[i][rg] = CT(0);
    // every column of the level, UN loads in flight (the last group guarded)
    for (int j = 0; j < p; j += UN) {
        CT u[UN][RPL];
#pragma unroll
        for (int q = 0; q < UN; ++q) {
            if (act && j + q < p)
                Codec<F>::template load<RPL, CT>(Up + int64_t(j + q) * ld * S, u[q]);
            else
#pragma unroll
                for (int i = 0; i < RPL; ++i) u[q][i] = CT(0);
        }
#pragma unroll
        for (int q = 0; q < UN; ++q) {
            if (j + q >= p) break;
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                const CT tv = CT(ts[rg * p + j + q]);
#pragma unroll
                for (int i = 0; i < RPL; ++i) lacc[i][rg] += u[q][i] * tv;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) acc[i][rg] += AT(lacc[i][rg]);
}

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
// = W + sum_k U_b T_b over the tile's depth ancestor blocks; the waves'
// partial rows are added in LDS and Y is written once.
template <typename XT, typename AT, int RG, int RPL>
__device__ void run_expand(const KParams& kp, int tile, XT* __restrict__ Y, int64_t ldy, int nrhs,
                           unsigned char* smem, int* s_off) {
    constexpr int TR = 64 * RPL;                    // rows per tile
    const ETile t = kp.etiles[tile];
    const LeafDesc L = kp.leaves[t.leaf];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const bool act = RPL * lane < t.nr;
    const int depth = kp.depth;
    // LDS: T of every level [sum p][RG] | wave sums [kWaves][TR]
    double* ts = reinterpret_cast<double*>(smem);
    // level offsets of T in LDS: thread k-1 reads level k's rank, thread 0 adds up
    if (threadIdx.x < depth) {
        const int k = threadIdx.x + 1;
        s_off[k] = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))].rank * RG;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0;
        for (int k = 1; k <= depth; ++k) {
            const int r = s_off[k];
            s_off[k - 1] = off;
            off += r;
        }
        s_off[depth] = off;
    }
    __syncthreads();
    AT* red = reinterpret_cast<AT*>(ts + s_off[depth]);
    for (int rb = 0; rb < nrhs; rb += RG) {
        AT acc[RPL][RG];
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) acc[i][rg] = AT(0);
        // T of every level for right-hand sides [rb, rb+RG): one pass of loads
        for (int idx = threadIdx.x; idx < s_off[depth]; idx += kThreads) {
            int k = 1;
            while (k < depth && s_off[k] <= idx) ++k;
            const BlockDesc& bd = kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))];
            const int p = bd.rank;
            const int r = idx - s_off[k - 1];
            const int rg = r / p, j = r - rg * p;
            ts[idx] = (rb + rg < nrhs) ? kp.T[bd.t_off * nrhs + int64_t(rb + rg) * p + j] : 0.0;
        }
        __syncthreads();
        // the waves take whole levels (wave w: levels w+1, w+5, ...), so the
        // chain of dependent loads per wave is short
        for (int k = 1 + wave; k <= depth; k += kWaves) {
            const int b = (1 << k) - 2 + (t.leaf >> (depth - k));
            const BlockDesc bd = kp.blocks[b];
            if (bd.rank == 0) continue;
            const int c0 = L.prow0 - bd.urow0 + t.r0;
            const int rin = RPL * lane;
            const double* tk = ts + s_off[k - 1];
            switch (bd.fmt) {
                case F64: expand_level<F64, double, AT, RG, RPL>(kp, bd, c0, rin, t.nr, act, tk, acc); break;
                case F32: expand_level<F32, AT, AT, RG, RPL>(kp, bd, c0, rin, t.nr, act, tk, acc); break;
                case BF16: expand_level<BF16, AT, AT, RG, RPL>(kp, bd, c0, rin, t.nr, act, tk, acc); break;
                case F16: expand_level<F16, AT, AT, RG, RPL>(kp, bd, c0, rin, t.nr, act, tk, acc); break;
                case E4M3: expand_level<E4M3, AT, AT, RG, RPL>(kp, bd, c0, rin, t.nr, act, tk, acc); break;
                default: expand_level<E5M2, AT, AT, RG, RPL>(kp, bd, c0, rin, t.nr, act, tk, acc); break;
            }
        }
        // sum the waves' partial rows, add the leaf product; write Y once
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) red[wave * TR + RPL * lane + i] = acc[i][rg];
            __syncthreads();
            for (int r = threadIdx.x; r < TR; r += kThreads) {
                AT sum = red[r];
#pragma unroll
                for (int w = 1; w < kWaves; ++w) sum += red[w * TR + r];
                const int lr = t.r0 + r;
                if (r < t.nr && lr < L.m && rb + rg < nrhs)
                    Y[L.row0 + lr + ldy * (rb + rg)] =
                        XT(sum + AT(kp.W[int64_t(L.prow0) + lr + kp.npad * (rb + rg)]));
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
__global__ __launch_bounds__(kThreads, HODLR_EXPAND_MINW) void k_expand(KParams kp, XT* __restrict__ Y, int64_t ldy,
                                                                       int nrhs) {
    extern __shared__ double smem_d[];
    __shared__ int s_off[kMaxDepth + 1];
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
    return size_t(kp.max_rank_path) * rg * 8 + size_t(kWaves) * kTileRows * acc_bytes;
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
    hipLaunchKernelGGL((k_expand<XT, AT, RG, RPL>), dim3(kp.netiles), dim3(kThreads), lds_expand(kp, RG, sizeof(AT)),
                       s, kp, Y, ldy, nrhs);
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

// Contraction item on the matrix cores: partial T_b over rows [r0, r0+nr)
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
#pragma unroll
            for (int pg = 0; pg < PG; ++pg) {
                const int j = j0 + 16 * pg + li;
                if (ok && j < p)
                    load_codes8<F, CT>(Vp + (int64_t(j) * ld + row) * S, a[pg]);
                else
#pragma unroll
                    for (int q = 0; q < kKL; ++q) a[pg][q] = CT(0);
            }
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int c = c0 + 16 * ct + li;
                if (ok && c < nrhs)
                    load_x8<XT, CT>(Xr + row + ldx * c, b[ct]);
                else
#pragma unroll
                    for (int q = 0; q < kKL; ++q) b[ct][q] = CT(0);
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
__device__ void run_contract_w(const KParams& kp, int item, int yg, const XT* __restrict__ Xc, int64_t ldc,
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

template <typename XT, typename AT, int NT>
__global__ __launch_bounds__(kThreads) void k_contract_w(KParams kp, const XT* __restrict__ Xc, int64_t ldc,
                                                         int nrhs) {
    extern __shared__ double smem_d[];
    run_contract_w<XT, AT, NT>(kp, blockIdx.x, blockIdx.y, Xc, ldc, nrhs, smem_d);
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
__device__ void run_reduce_w(const KParams& kp, int block, int yg, int nrhs) {
    const BlockDesc bd = kp.blocks[block];
    const int total = bd.rank * nrhs;
    const int o = yg * 256 + threadIdx.x;
    if (o >= total) return;
    if (bd.fmt == F64)
        reduce_block<double>(kp, bd, o, total, nrhs);
    else
        reduce_block<AT>(kp, bd, o, total, nrhs);
}

template <typename AT>
__global__ __launch_bounds__(256) void k_reduce_w(KParams kp, int nrhs) {
    run_reduce_w<AT>(kp, blockIdx.x, blockIdx.y, nrhs);
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
#pragma unroll
            for (int q = 0; q < QG; ++q) {
                const int jr = j0 + 4 * q + g;          // rank within the staged rows
                a0[q] = CT(0);
                a1[q] = CT(0);
                if (q < qn && jr < crows) {
                    const uint8_t* col = Up + int64_t(cr0 + jr) * ld * S;
                    if (act0) Codec<F>::template load<1, CT>(col + int64_t(r0) * S, &a0[q]);
                    if (act1) Codec<F>::template load<1, CT>(col + int64_t(r1) * S, &a1[q]);
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
    if (kp.ncitems > 0) {
        tm.begin(1);
        hipLaunchKernelGGL((k_contract_w<XT, AT, NTC>), dim3(kp.ncitems, (nrhs + 16 * NTC - 1) / (16 * NTC)),
                           dim3(kThreads), size_t(kWaves) * NTC * 256 * sizeof(double), s, kp, Xw, ldw, nrhs);
        tm.end(1);
        // largest rank * nrhs of a block bounds the outputs per block
        tm.begin(3);
        const int64_t rows_y = (int64_t(kp.max_block_rank) * nrhs + 255) / 256;
        hipLaunchKernelGGL((k_reduce_w<AT>), dim3(kp.nblocks, unsigned(rows_y)), dim3(256), 0, s, kp, nrhs);
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
