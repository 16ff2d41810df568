// HIP kernels (gfx950) of the HODLR matrix-vector product
// Y = A_H X, following Alg. "HODLR_MATVEC" of Carson, Chen, Liu,
// "Mixed Precision HODLR Matrices" (arXiv 2407.21637):
//
//   b <- 0;  b_rows(b) += U_b (V_b^T x_cols(b)) for every off-diagonal block;
//   b_i += D_i x_i for every leaf.
//
// One launch does the whole product.  Its workgroups take tickets from a
// counter in launch order, so ticket t is only taken once every smaller
// ticket belongs to a running or finished workgroup:
//
//  * tickets [0, ncitems): contraction items.  Item = rows [r0, r0+nr) of
//    the V panel of one block; it writes the partial sums of T_b = V_b^T X
//    over its rows.  The last item of a block to finish (arrival counter)
//    adds the block's partials in item order, applies the column scales and
//    publishes T_b through a ready flag (deterministic, no float atomics).
//  * tickets [ncitems, ncitems+netiles): expansion tiles.  Tile = 64*RPL
//    padded rows of one leaf.  It first computes D_i X_i in fp64 (needs
//    only X), then waits for the T_b of its depth ancestors' blocks, adds
//    U_b T_b for each level, sums its waves' partial rows and writes Y once.
//    Tiles only wait on contraction items, which hold smaller tickets, so
//    the wait always ends; it is bounded anyway (a timed-out tile writes NaN).
//  * The last workgroup to finish resets the counters for the next launch.
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
//   sync[0] ticket counter, sync[1] finished workgroups, sync[2] timed-out
//   waits (sticky), sync[4 + b] arrivals of block b, sync[4 + nb + b] ready.
constexpr int kSyncHead = 4;
constexpr int kWaitSpins = 1 << 24;   // ~1 s of s_sleep(2)

__device__ __forceinline__ int* arrivals(const KParams& kp) { return kp.sync + kSyncHead; }
__device__ __forceinline__ int* ready(const KParams& kp) { return kp.sync + kSyncHead + kp.nblocks; }

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

__device__ bool wait_ready(int* flag) {
    for (int i = 0; i < kWaitSpins; ++i) {
        if (ld_coh(flag) != 0) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

constexpr int kWaves = 4;            // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kContractCols = 8;     // columns a contraction wave keeps in flight

// ---------------------------------------------------------------------------
// contraction item: partial T_b over rows [r0, r0+nr) of the V panel
// ---------------------------------------------------------------------------
// Lane l owns rows 4l..4l+3 of a 256-row slab; wave w takes slabs w, w+4, ...
// (at most 4 each), keeps their x values in registers and accumulates CJ
// columns at a time (CJ loads in flight per slab), then reduces each column
// across its lanes (DPP) into LDS; the four waves' sums make the item's
// partial.
template <int F, typename CT, typename XT, int RG>
__device__ void contract_item(const KParams& kp, const CItem& it, const BlockDesc& bd,
                              const XT* __restrict__ X, int64_t ldx, int nrhs, unsigned char* smem) {
    constexpr int CJ0 = kContractCols * 4 / int(sizeof(CT)) / RG;   // fp64 keeps half as many
    constexpr int CJ = CJ0 > 1 ? CJ0 : 2;
    constexpr int GS = 4;
    constexpr int S = Codec<F>::kBytes;
    CT* red = reinterpret_cast<CT*>(smem);          // [kWaves][CJ][RG]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int p = bd.rank;
    const uint8_t* Vp = kp.fac + bd.v_off + int64_t(it.r0) * S;
    const int64_t ld = bd.vrows;
    double* part = kp.partial + it.poff * nrhs;
    const int nslab = (it.nr + 255) >> 8;
    const int64_t xrow0 = int64_t(bd.vrow0) + it.r0;
    for (int rb = 0; rb < nrhs; rb += RG) {
        for (int j0 = 0; j0 < p; j0 += CJ) {
            CT acc[CJ][RG];
#pragma unroll
            for (int c = 0; c < CJ; ++c)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) acc[c][rg] = CT(0);
#pragma unroll 1
            for (int q = 0; q < GS; ++q) {
                const int row = (wave + kWaves * q) * 256 + 4 * lane;
                if ((wave + kWaves * q) < nslab && row < it.nr) {
                    CT v[CJ][4];
#pragma unroll
                    for (int c = 0; c < CJ; ++c) {
                        if (j0 + c < p)
                            Codec<F>::template load<4, CT>(Vp + (int64_t(j0 + c) * ld + row) * S, v[c]);
                        else
                            v[c][0] = v[c][1] = v[c][2] = v[c][3] = CT(0);
                    }
                    CT xr[4][RG];
#pragma unroll
                    for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            xr[i][rg] = (rb + rg < nrhs) ? CT(X[xrow0 + row + i + ldx * (rb + rg)]) : CT(0);
#pragma unroll
                    for (int c = 0; c < CJ; ++c)
#pragma unroll
                        for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                            for (int i = 0; i < 4; ++i) acc[c][rg] += v[c][i] * xr[i][rg];
                }
            }
#pragma unroll
            for (int c = 0; c < CJ; ++c)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    const CT r = wave_sum63(acc[c][rg]);
                    if (lane == 63) red[(wave * CJ + c) * RG + rg] = r;
                }
            __syncthreads();
            if (threadIdx.x < CJ * RG) {
                const int c = threadIdx.x / RG, rg = threadIdx.x % RG;
                if (j0 + c < p && rb + rg < nrhs) {
                    CT s = red[c * RG + rg];
#pragma unroll
                    for (int w = 1; w < kWaves; ++w) s += red[(w * CJ + c) * RG + rg];
                    st_coh(part + int64_t(rb + rg) * p + j0 + c, double(s));
                }
            }
            __syncthreads();
        }
    }
}

// The last item of block b adds the block's partials in item order.
template <typename CT>
__device__ void finish_block(const KParams& kp, const BlockDesc& bd, int nrhs) {
    const int p = bd.rank;
    const int64_t total = int64_t(p) * nrhs;
    const int64_t base = kp.citems[bd.item0].poff * nrhs;
    for (int64_t idx = threadIdx.x; idx < total; idx += kThreads) {
        const int j = int(idx % p);
        CT s = CT(0);
        int c = 0;
        for (; c + 4 <= bd.nitems; c += 4) {
            const double a0 = ld_coh(kp.partial + base + int64_t(c) * total + idx);
            const double a1 = ld_coh(kp.partial + base + int64_t(c + 1) * total + idx);
            const double a2 = ld_coh(kp.partial + base + int64_t(c + 2) * total + idx);
            const double a3 = ld_coh(kp.partial + base + int64_t(c + 3) * total + idx);
            s += CT(a0);
            s += CT(a1);
            s += CT(a2);
            s += CT(a3);
        }
        for (; c < bd.nitems; ++c) s += CT(ld_coh(kp.partial + base + int64_t(c) * total + idx));
        st_coh(kp.T + bd.t_off * nrhs + idx, double(s) * kp.tscale[bd.ts_off + j]);
    }
}

template <typename XT, typename AT, int RG>
__device__ void run_contract(const KParams& kp, int ticket, const XT* __restrict__ X, int64_t ldx, int nrhs,
                             unsigned char* smem, int* s_flag) {
    const CItem it = kp.citems[ticket];
    const BlockDesc bd = kp.blocks[it.block];
    switch (bd.fmt) {
        case F64: contract_item<F64, double, XT, RG>(kp, it, bd, X, ldx, nrhs, smem); break;
        case F32: contract_item<F32, AT, XT, RG>(kp, it, bd, X, ldx, nrhs, smem); break;
        case BF16: contract_item<BF16, AT, XT, RG>(kp, it, bd, X, ldx, nrhs, smem); break;
        case F16: contract_item<F16, AT, XT, RG>(kp, it, bd, X, ldx, nrhs, smem); break;
        case E4M3: contract_item<E4M3, AT, XT, RG>(kp, it, bd, X, ldx, nrhs, smem); break;
        default: contract_item<E5M2, AT, XT, RG>(kp, it, bd, X, ldx, nrhs, smem); break;
    }
    // publish the partial; the last arrival of the block reduces it
    drain_and_sync();
    if (threadIdx.x == 0) *s_flag = (add_coh(arrivals(kp) + it.block, 1) == bd.nitems - 1);
    __syncthreads();
    if (*s_flag) {
        if (bd.fmt == F64)
            finish_block<double>(kp, bd, nrhs);
        else
            finish_block<AT>(kp, bd, nrhs);
        drain_and_sync();
        if (threadIdx.x == 0) st_coh(ready(kp) + it.block, 1);
    }
}

// ---------------------------------------------------------------------------
// expansion tile: Y rows of one leaf = D_i x_i + sum_k U_b T_b
// ---------------------------------------------------------------------------
template <int F, typename CT, typename AT, int RG, int RPL>
__device__ void expand_level(const KParams& kp, const BlockDesc& bd, int prow, bool act,
                             const double* __restrict__ ts, AT acc[RPL][RG]) {
    constexpr int S = Codec<F>::kBytes;
    const int wave = threadIdx.x >> 6;
    const int p = bd.rank;
    const uint8_t* Up = kp.fac + bd.u_off + int64_t(prow) * S;
    const int64_t ld = bd.urows;
    CT lacc[RPL][RG];
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) lacc[i][rg] = CT(0);
    int j = wave;
    for (; j + 3 * kWaves < p; j += 4 * kWaves) {
        CT u[4][RPL];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (act)
                Codec<F>::template load<RPL, CT>(Up + int64_t(j + q * kWaves) * ld * S, u[q]);
            else
#pragma unroll
                for (int i = 0; i < RPL; ++i) u[q][i] = CT(0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int rg = 0; rg < RG; ++rg) {
                const CT tv = CT(ts[rg * p + j + q * kWaves]);
#pragma unroll
                for (int i = 0; i < RPL; ++i) lacc[i][rg] += u[q][i] * tv;
            }
    }
    for (; j < p; j += kWaves) {
        CT u[RPL];
        if (act)
            Codec<F>::template load<RPL, CT>(Up + int64_t(j) * ld * S, u);
        else
#pragma unroll
            for (int i = 0; i < RPL; ++i) u[i] = CT(0);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            const CT tv = CT(ts[rg * p + j]);
#pragma unroll
            for (int i = 0; i < RPL; ++i) lacc[i][rg] += u[i] * tv;
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) acc[i][rg] += AT(lacc[i][rg]);
}

template <typename XT, typename AT, int RG, int RPL>
__device__ void run_expand(const KParams& kp, int tile, const XT* __restrict__ X, int64_t ldx,
                           XT* __restrict__ Y, int64_t ldy, int nrhs, unsigned char* smem, int* s_off,
                           int* s_err) {
    constexpr int TR = 64 * RPL;                    // rows per tile
    const ETile t = kp.etiles[tile];
    const LeafDesc L = kp.leaves[t.leaf];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = t.r0 + RPL * lane;              // padded row within the leaf
    const bool act = RPL * lane < t.nr;
    const int depth = kp.depth;
    // LDS: x of the leaf [m][RG] | T of every level [sum p][RG] | wave sums [kWaves][TR]
    double* xs = reinterpret_cast<double*>(smem);
    double* ts = xs + int64_t(L.m) * RG;
    if (threadIdx.x == 0) {
        int off = 0;
        for (int k = 1; k <= depth; ++k) {
            s_off[k - 1] = off;
            off += kp.blocks[(1 << k) - 2 + (t.leaf >> (depth - k))].rank * RG;
        }
        s_off[depth] = off;
    }
    __syncthreads();
    AT* red = reinterpret_cast<AT*>(ts + s_off[depth]);
    bool waited_ok = true;
    for (int rb = 0; rb < nrhs; rb += RG) {
        for (int idx = threadIdx.x; idx < L.m * RG; idx += kThreads) {
            const int c = idx / RG, rg = idx % RG;
            xs[idx] = (rb + rg < nrhs) ? double(X[L.row0 + c + ldx * (rb + rg)]) : 0.0;
        }
        __syncthreads();
        AT acc[RPL][RG];
        {
            double dacc[RPL][RG];
#pragma unroll
            for (int i = 0; i < RPL; ++i)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) dacc[i][rg] = 0.0;
            const uint8_t* Dp = reinterpret_cast<const uint8_t*>(kp.leafd + L.d_off + row);
            const int64_t ldb = int64_t(L.mp) * 8;
            int c = wave;
            for (; c + 3 * kWaves < L.m; c += 4 * kWaves) {
                double d[4][RPL];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (act)
                        Codec<F64>::template load<RPL, double>(Dp + int64_t(c + q * kWaves) * ldb, d[q]);
                    else
#pragma unroll
                        for (int i = 0; i < RPL; ++i) d[q][i] = 0.0;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
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
#pragma unroll
            for (int i = 0; i < RPL; ++i)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) acc[i][rg] = AT(dacc[i][rg]);
        }
        if (rb == 0) {
            // T of every ancestor level: thread k-1 waits for level k's block
            if (threadIdx.x < depth) {
                const int k = threadIdx.x + 1;
                const int b = (1 << k) - 2 + (t.leaf >> (depth - k));
                if (kp.blocks[b].rank > 0 && !wait_ready(ready(kp) + b)) {
                    atomicOr(kp.sync + 2, 1);
                    *s_err = 1;
                }
            }
            __syncthreads();
            waited_ok = *s_err == 0;
        }
        for (int k = 1; k <= depth; ++k) {
            const int b = (1 << k) - 2 + (t.leaf >> (depth - k));
            const BlockDesc& bd = kp.blocks[b];
            const int p = bd.rank;
            for (int idx = threadIdx.x; idx < p * RG; idx += kThreads) {
                const int rg = idx / p, j = idx % p;
                ts[s_off[k - 1] + idx] = (rb + rg < nrhs) ? ld_coh(kp.T + bd.t_off * nrhs + int64_t(rb + rg) * p + j) : 0.0;
            }
        }
        __syncthreads();
        for (int k = 1; k <= depth; ++k) {
            const int b = (1 << k) - 2 + (t.leaf >> (depth - k));
            const BlockDesc bd = kp.blocks[b];
            if (bd.rank == 0) continue;
            const int prow = L.prow0 - bd.urow0 + row;
            const double* tk = ts + s_off[k - 1];
            switch (bd.fmt) {
                case F64: expand_level<F64, double, AT, RG, RPL>(kp, bd, prow, act, tk, acc); break;
                case F32: expand_level<F32, AT, AT, RG, RPL>(kp, bd, prow, act, tk, acc); break;
                case BF16: expand_level<BF16, AT, AT, RG, RPL>(kp, bd, prow, act, tk, acc); break;
                case F16: expand_level<F16, AT, AT, RG, RPL>(kp, bd, prow, act, tk, acc); break;
                case E4M3: expand_level<E4M3, AT, AT, RG, RPL>(kp, bd, prow, act, tk, acc); break;
                default: expand_level<E5M2, AT, AT, RG, RPL>(kp, bd, prow, act, tk, acc); break;
            }
        }
        // sum the waves' partial rows; write Y once
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) red[wave * TR + RPL * lane + i] = acc[i][rg];
            __syncthreads();
            for (int r = threadIdx.x; r < TR; r += kThreads) {
                AT s = red[r];
#pragma unroll
                for (int w = 1; w < kWaves; ++w) s += red[w * TR + r];
                const int lr = t.r0 + r;
                if (r < t.nr && lr < L.m && rb + rg < nrhs)
                    Y[L.row0 + lr + ldy * (rb + rg)] = waited_ok ? XT(s) : XT(__builtin_nan(""));
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// the fused launch
// ---------------------------------------------------------------------------
template <typename XT, typename AT, int RG, int RPL>
__global__ __launch_bounds__(kThreads, 4) void k_matvec(KParams kp, const XT* __restrict__ Xc, int64_t ldc,
                                                     const XT* __restrict__ X, int64_t ldx,
                                                     XT* __restrict__ Y, int64_t ldy, int nrhs) {
    extern __shared__ double smem_d[];
    unsigned char* smem = reinterpret_cast<unsigned char*>(smem_d);
    __shared__ int s_ticket, s_flag, s_err;
    __shared__ int s_off[kMaxDepth + 1];
    if (threadIdx.x == 0) {
        s_ticket = add_coh(kp.sync, 1);
        s_err = 0;
    }
    __syncthreads();
    const int ticket = s_ticket;
    if (ticket < kp.ncitems) {
        run_contract<XT, AT, RG>(kp, ticket, Xc, ldc, nrhs, smem, &s_flag);
    } else if (ticket < kp.ncitems + kp.netiles) {
        run_expand<XT, AT, RG, RPL>(kp, ticket - kp.ncitems, X, ldx, Y, ldy, nrhs, smem, s_off, &s_err);
    } else if (threadIdx.x == 0) {
        atomicOr(kp.sync + 2, 2);   // counters were not clear: flag it, touch nothing
    }
    // the last workgroup to finish clears the counters for the next launch
    __syncthreads();
    if (threadIdx.x == 0) s_flag = (add_coh(kp.sync + 1, 1) == kp.ncitems + kp.netiles - 1);
    __syncthreads();
    if (s_flag) {
        for (int i = threadIdx.x; i < 2 * kp.nblocks; i += kThreads) st_coh(kp.sync + kSyncHead + i, 0);
        if (threadIdx.x == 0) {
            st_coh(kp.sync, 0);
            st_coh(kp.sync + 1, 0);
        }
    }
}

// ---------------------------------------------------------------------------
// padded copy of X (only when some leaf size is not a multiple of 16)
// ---------------------------------------------------------------------------
template <typename XT>
__global__ __launch_bounds__(256) void k_padx(KParams kp, const XT* __restrict__ X, int64_t ldx, int nrhs) {
    const LeafDesc L = kp.leaves[blockIdx.x];
    XT* Xp = static_cast<XT*>(kp.xpad);
    const int64_t total = int64_t(L.mp) * nrhs;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int64_t r = idx % L.mp, c = idx / L.mp;
        Xp[L.prow0 + r + kp.npad * c] = r < L.m ? X[L.row0 + r + ldx * c] : XT(0);
    }
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

size_t lds_need(const KParams& kp, int rg, size_t acc_bytes) {
    const size_t cj = kContractCols / rg > 1 ? kContractCols / rg : 2;    // an upper bound
    const size_t c = kWaves * cj * rg * 8;
    const size_t e = (size_t(kp.max_leaf) + size_t(kp.max_rank_path)) * rg * 8 + kWaves * kTileRows * acc_bytes;
    return c > e ? c : e;
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
    // dynamic LDS: the larger of the contraction's wave sums and the tile's
    // x | T | wave-sum regions
    const size_t lds = lds_need(kp, RG, sizeof(AT));
    tm.begin(1);
    hipLaunchKernelGGL((k_matvec<XT, AT, RG, RPL>), dim3(kp.ncitems + kp.netiles), dim3(kThreads), lds, s, kp,
                       Xc, ldc, X, ldx, Y, ldy, nrhs);
    tm.end(1);
    return hipGetLastError();
}

template <typename XT, typename AT>
hipError_t launch_rg(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs,
                     const Timer& tm) {
    // the widest right-hand-side group whose LDS fits in 64 KB
    int rg = nrhs == 1 ? 1 : nrhs == 2 ? 2 : nrhs <= 4 ? 4 : 8;
    while (rg > 1 && lds_need(kp, rg, sizeof(AT)) > kMaxLds) rg /= 2;
    if (lds_need(kp, rg, sizeof(AT)) > kMaxLds) return hipErrorInvalidConfiguration;
    if (rg == 1) return launch_typed<XT, AT, 1, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
    if (rg == 2) return launch_typed<XT, AT, 2, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
    if (rg == 4) return launch_typed<XT, AT, 4, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
    return launch_typed<XT, AT, 8, kRPL>(kp, X, ldx, Y, ldy, nrhs, tm);
}

}  // namespace

int launch_matvec(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs,
                  bool xy_double, bool acc_double, void* stream, void* const* events, bool* ran) {
    const Timer tm{events, ran, static_cast<hipStream_t>(stream)};
    hipError_t e;
    if (xy_double)
        e = acc_double ? launch_rg<double, double>(kp, X, ldx, Y, ldy, nrhs, tm)
                       : launch_rg<double, float>(kp, X, ldx, Y, ldy, nrhs, tm);
    else
        e = acc_double ? launch_rg<float, double>(kp, X, ldx, Y, ldy, nrhs, tm)
                       : launch_rg<float, float>(kp, X, ldx, Y, ldy, nrhs, tm);
    return int(e);
}

}  // namespace hodlr
