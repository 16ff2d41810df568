// HIP kernels (gfx950) of the HODLR matrix-vector product
// Y = A_H X, following Alg. "HODLR_MATVEC" of Carson, Chen, Liu,
// "Mixed Precision HODLR Matrices" (arXiv 2407.21637):
//
//   b <- 0;  b_rows(b) += U_b (V_b^T x_cols(b)) for every off-diagonal block;
//   b_i += D_i x_i for every leaf.
//
// The product is split by data dependence into three launches:
//   1. contraction: T_b partials = V_b^T X over chunks of V-panel rows
//      (every level at once; wave64 reductions over rows);
//   2. reduction: T_b = sum of its partials in a fixed order, times the
//      per-column power-of-2 scales (deterministic, no atomics);
//   3. expansion + leaf: each tile of 256 rows of a leaf accumulates
//      D_i X_i (fp64) and U_b T_b of every level it belongs to, and writes
//      Y once.
// Stored codes are converted in registers (Sect. 3.3: low-precision
// storage cast to the working precision on the fly).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hodlr_internal.h"

namespace hodlr {
namespace {

// ---------------------------------------------------------------------------
// decoding 4 consecutive codes of one column (the 4 rows a lane owns)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float half_bits_to_float(uint32_t h) {
    _Float16 v = __builtin_bit_cast(_Float16, uint16_t(h));
    return float(v);
}

template <int F>
struct Codec;

template <>
struct Codec<F64> {
    static constexpr int kBytes = 8;
    template <typename CT>
    __device__ static void load4(const uint8_t* p, CT v[4]) {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 16);
        v[0] = CT(a.x); v[1] = CT(a.y); v[2] = CT(b.x); v[3] = CT(b.y);
    }
};

template <>
struct Codec<F32> {
    static constexpr int kBytes = 4;
    template <typename CT>
    __device__ static void load4(const uint8_t* p, CT v[4]) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        v[0] = CT(a.x); v[1] = CT(a.y); v[2] = CT(a.z); v[3] = CT(a.w);
    }
};

template <>
struct Codec<BF16> {   // bf16 is the top half of an fp32
    static constexpr int kBytes = 2;
    template <typename CT>
    __device__ static void load4(const uint8_t* p, CT v[4]) {
        const uint2 a = *reinterpret_cast<const uint2*>(p);
        v[0] = CT(__uint_as_float(a.x << 16));
        v[1] = CT(__uint_as_float(a.x & 0xffff0000u));
        v[2] = CT(__uint_as_float(a.y << 16));
        v[3] = CT(__uint_as_float(a.y & 0xffff0000u));
    }
};

template <>
struct Codec<F16> {
    static constexpr int kBytes = 2;
    template <typename CT>
    __device__ static void load4(const uint8_t* p, CT v[4]) {
        const uint2 a = *reinterpret_cast<const uint2*>(p);
        v[0] = CT(half_bits_to_float(a.x & 0xffffu));
        v[1] = CT(half_bits_to_float(a.x >> 16));
        v[2] = CT(half_bits_to_float(a.y & 0xffffu));
        v[3] = CT(half_bits_to_float(a.y >> 16));
    }
};

// fp8 E4M3FN -> fp16 bits by placing sign at bit 15 and the 7 magnitude bits
// at bits 7..13: the fp16 number equals the e4m3 value times 2^-8 (normal and
// subnormal alike); the 2^8 is folded into the block's column scales.
template <>
struct Codec<E4M3> {
    static constexpr int kBytes = 1;
    template <typename CT>
    __device__ static void load4(const uint8_t* p, CT v[4]) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t c = (w >> (8 * i)) & 0xffu;
            v[i] = CT(half_bits_to_float(((c & 0x80u) << 8) | ((c & 0x7fu) << 7)));
        }
    }
};

// fp8 E5M2 is exactly the top byte of an fp16.
template <>
struct Codec<E5M2> {
    static constexpr int kBytes = 1;
    template <typename CT>
    __device__ static void load4(const uint8_t* p, CT v[4]) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = CT(half_bits_to_float(((w >> (8 * i)) & 0xffu) << 8));
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
// 1. contraction: partial T_b over rows [r0, r0+nr) of the V panel
// ---------------------------------------------------------------------------
// Lane l of a pass owns rows 4l..4l+3 of a 256-row slab; the item's slabs
// are processed in groups of GX with the x values of the group in
// registers.  Waves split the columns; a wave owns its columns outright, so
// it accumulates their partials across slab groups without synchronisation.
template <int F, typename CT, typename XT, int RG>
__device__ void contract_item(const KParams& kp, const CItem& it, const BlockDesc& bd,
                              const XT* __restrict__ X, int64_t ldx, int nrhs) {
    constexpr int GX = (sizeof(CT) == 8 ? 8 : 16) / RG;
    constexpr int S = Codec<F>::kBytes;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const int p = bd.rank;
    const uint8_t* Vp = kp.fac + bd.v_off;
    const int64_t ld = bd.vrows;
    double* part = kp.partial + it.poff * nrhs;
    const int G = (it.nr + 255) >> 8;
    const int64_t xrow0 = int64_t(bd.vrow0) + it.r0;
    for (int rb = 0; rb < nrhs; rb += RG) {
        for (int g0 = 0; g0 < G; g0 += GX) {
            CT xr[GX][4][RG];
#pragma unroll
            for (int g = 0; g < GX; ++g) {
                const int row = (g0 + g) * 256 + 4 * lane;
#pragma unroll
                for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const bool ok = (g0 + g < G) && (row + i < it.nr) && (rb + rg < nrhs);
                        xr[g][i][rg] = ok ? CT(X[xrow0 + row + i + ldx * (rb + rg)]) : CT(0);
                    }
            }
            for (int j = wave; j < p; j += W) {
                CT acc[RG];
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) acc[rg] = CT(0);
                const uint8_t* col = Vp + (int64_t(j) * ld + it.r0) * S;
#pragma unroll
                for (int g = 0; g < GX; ++g) {
                    if (g0 + g < G) {
                        const int row = (g0 + g) * 256 + 4 * lane;
                        if (row < it.nr) {
                            CT v[4];
                            Codec<F>::template load4<CT>(col + int64_t(row) * S, v);
#pragma unroll
                            for (int rg = 0; rg < RG; ++rg)
#pragma unroll
                                for (int i = 0; i < 4; ++i) acc[rg] += v[i] * xr[g][i][rg];
                        }
                    }
                }
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    const CT r = wave_sum63(acc[rg]);
                    if (lane == 63 && rb + rg < nrhs) {
                        double* dst = part + int64_t(rb + rg) * p + j;
                        *dst = (g0 == 0) ? double(r) : double(CT(*dst) + r);
                    }
                }
            }
        }
    }
}

template <typename XT, typename AT, int RG>
__global__ __launch_bounds__(256) void k_contract(KParams kp, const XT* __restrict__ X, int64_t ldx,
                                                  int nrhs) {
    const CItem it = kp.citems[blockIdx.x];
    const BlockDesc bd = kp.blocks[it.block];
    switch (bd.fmt) {
        case F64: contract_item<F64, double, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case F32: contract_item<F32, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case BF16: contract_item<BF16, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case F16: contract_item<F16, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        case E4M3: contract_item<E4M3, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
        default: contract_item<E5M2, AT, XT, RG>(kp, it, bd, X, ldx, nrhs); break;
    }
}

// ---------------------------------------------------------------------------
// 2. reduction of partials, fixed order, times the column scales
// ---------------------------------------------------------------------------
template <typename CT>
__device__ void reduce_block(const KParams& kp, const BlockDesc& bd, int nrhs) {
    const int p = bd.rank;
    const int64_t total = int64_t(p) * nrhs;
    const int64_t base = kp.citems[bd.item0].poff * nrhs;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int j = int(idx % p);
        CT s = CT(0);
        for (int c = 0; c < bd.nitems; ++c) s += CT(kp.partial[base + int64_t(c) * total + idx]);
        kp.T[bd.t_off * nrhs + idx] = double(s) * kp.tscale[bd.ts_off + j];
    }
}

template <typename AT>
__global__ __launch_bounds__(256) void k_reduce(KParams kp, int nrhs) {
    const BlockDesc bd = kp.blocks[blockIdx.x];
    if (bd.rank == 0) return;
    if (bd.fmt == F64)
        reduce_block<double>(kp, bd, nrhs);
    else
        reduce_block<AT>(kp, bd, nrhs);
}

// ---------------------------------------------------------------------------
// 3. expansion + leaf
// ---------------------------------------------------------------------------
template <int F, typename CT, typename AT, int RG, int W>
__device__ void expand_level(const KParams& kp, const BlockDesc& bd, int prow, bool act, int rb,
                             int nrhs, AT acc[4][RG]) {
    constexpr int S = Codec<F>::kBytes;
    const int wave = threadIdx.x >> 6;
    const int p = bd.rank;
    const uint8_t* Up = kp.fac + bd.u_off + int64_t(prow) * S;
    const int64_t ld = bd.urows;
    const double* Tb = kp.T + bd.t_off * nrhs;
    CT lacc[4][RG];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) lacc[i][rg] = CT(0);
    for (int j = wave; j < p; j += W) {
        CT u[4] = {CT(0), CT(0), CT(0), CT(0)};
        if (act) Codec<F>::template load4<CT>(Up + int64_t(j) * ld * S, u);
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
            const CT tv = (rb + rg < nrhs) ? CT(Tb[int64_t(rb + rg) * p + j]) : CT(0);
#pragma unroll
            for (int i = 0; i < 4; ++i) lacc[i][rg] += u[i] * tv;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) acc[i][rg] += AT(lacc[i][rg]);
}

template <typename XT, typename AT, int RG, int W>
__global__ __launch_bounds__(64 * W) void k_expand(KParams kp, const XT* __restrict__ X, int64_t ldx,
                                                   XT* __restrict__ Y, int64_t ldy, int nrhs) {
    __shared__ AT red[W][256];
    const ETile t = kp.etiles[blockIdx.x];
    const LeafDesc L = kp.leaves[t.leaf];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int row = t.r0 + 4 * lane;           // padded row within the leaf
    const bool act = 4 * lane < t.nr;
    for (int rb = 0; rb < nrhs; rb += RG) {
        AT acc[4][RG];
        {
            double dacc[4][RG];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) dacc[i][rg] = 0.0;
            const double* Dp = kp.leafd + L.d_off + row;
            for (int c = wave; c < L.m; c += W) {
                double d[4] = {0.0, 0.0, 0.0, 0.0};
                if (act) Codec<F64>::template load4<double>(reinterpret_cast<const uint8_t*>(Dp + int64_t(c) * L.mp), d);
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) {
                    const double xv = (rb + rg < nrhs) ? double(X[L.row0 + c + ldx * (rb + rg)]) : 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) dacc[i][rg] += d[i] * xv;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int rg = 0; rg < RG; ++rg) acc[i][rg] = AT(dacc[i][rg]);
        }
        for (int k = 1; k <= kp.depth; ++k) {
            const int b = (1 << k) - 2 + (t.leaf >> (kp.depth - k));
            const BlockDesc bd = kp.blocks[b];
            if (bd.rank == 0) continue;
            const int prow = L.prow0 - bd.urow0 + row;
            switch (bd.fmt) {
                case F64: expand_level<F64, double, AT, RG, W>(kp, bd, prow, act, rb, nrhs, acc); break;
                case F32: expand_level<F32, AT, AT, RG, W>(kp, bd, prow, act, rb, nrhs, acc); break;
                case BF16: expand_level<BF16, AT, AT, RG, W>(kp, bd, prow, act, rb, nrhs, acc); break;
                case F16: expand_level<F16, AT, AT, RG, W>(kp, bd, prow, act, rb, nrhs, acc); break;
                case E4M3: expand_level<E4M3, AT, AT, RG, W>(kp, bd, prow, act, rb, nrhs, acc); break;
                default: expand_level<E5M2, AT, AT, RG, W>(kp, bd, prow, act, rb, nrhs, acc); break;
            }
        }
        // sum the waves' partial rows and write Y once
#pragma unroll
        for (int rg = 0; rg < RG; ++rg) {
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wave][4 * lane + i] = acc[i][rg];
            __syncthreads();
            for (int r = threadIdx.x; r < 256; r += 64 * W) {
                AT s = red[0][r];
#pragma unroll
                for (int w = 1; w < W; ++w) s += red[w][r];
                const int lr = t.r0 + r;
                if (r < t.nr && lr < L.m && rb + rg < nrhs) Y[L.row0 + lr + ldy * (rb + rg)] = XT(s);
            }
            __syncthreads();
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

template <typename XT, typename AT, int RG>
hipError_t launch_typed(const KParams& kp, const void* Xv, int64_t ldx, void* Yv, int64_t ldy, int nrhs,
                        const Timer& tm) {
    constexpr int W = 8;
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
    if (kp.ncitems > 0) {
        tm.begin(1);
        hipLaunchKernelGGL((k_contract<XT, AT, RG>), dim3(kp.ncitems), dim3(256), 0, s, kp, Xc, ldc, nrhs);
        tm.end(1);
        tm.begin(2);
        hipLaunchKernelGGL((k_reduce<AT>), dim3(kp.nblocks), dim3(256), 0, s, kp, nrhs);
        tm.end(2);
    }
    if (kp.netiles > 0) {
        tm.begin(3);
        hipLaunchKernelGGL((k_expand<XT, AT, RG, W>), dim3(kp.netiles), dim3(64 * W), 0, s, kp, X, ldx, Y,
                           ldy, nrhs);
        tm.end(3);
    }
    return hipGetLastError();
}

template <typename XT, typename AT>
hipError_t launch_rg(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs,
                     const Timer& tm) {
    if (nrhs == 1) return launch_typed<XT, AT, 1>(kp, X, ldx, Y, ldy, nrhs, tm);
    if (nrhs == 2) return launch_typed<XT, AT, 2>(kp, X, ldx, Y, ldy, nrhs, tm);
    if (nrhs <= 4) return launch_typed<XT, AT, 4>(kp, X, ldx, Y, ldy, nrhs, tm);
    return launch_typed<XT, AT, 8>(kp, X, ldx, Y, ldy, nrhs, tm);
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
