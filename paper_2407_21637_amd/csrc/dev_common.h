// Device helpers shared by the HODLR product kernels: format codecs, wave
// reductions, device-coherent accesses, workgroup shape.  Included by
// kernels.hip only (one translation unit).
#ifndef HODLR_DEV_COMMON_H
#define HODLR_DEV_COMMON_H

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
// loads whose use comes later
// ---------------------------------------------------------------------------
// A load through a global-address-space pointer: the generic pointers in the
// kernels' parameter structs would otherwise become flat loads, which also
// wait on the LDS counter.
template <typename T>
__device__ __forceinline__ T gload(const void* p) {
    return *(const __attribute__((address_space(1))) T*)(p);
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));   // plain vector types for gload
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// N consecutive codes of format F as raw bits.  The caller loads them from
// an address it has clamped into the buffer, with no branch around the
// load, and decodes (and masks) them after all the loads it has in flight
// are issued: a load inside a branch whose value is decoded inside the
// same branch makes the compiler wait for that load before issuing the
// next one.
template <int F, int N>
struct RawCodes {
    static constexpr int kBytes = N * Codec<F>::kBytes;
    static constexpr int kWords = kBytes < 4 ? 1 : kBytes / 4;
    uint32_t w[kWords];

    __device__ __forceinline__ void load(const uint8_t* p) {
        if constexpr (kBytes == 1) {
            w[0] = gload<uint8_t>(p);
        } else if constexpr (kBytes == 2) {
            w[0] = gload<uint16_t>(p);
        } else if constexpr (kBytes == 4) {
            w[0] = gload<uint32_t>(p);
        } else if constexpr (kBytes == 8) {
            const u32x2 a = gload<u32x2>(p);
            w[0] = a.x;
            w[1] = a.y;
        } else {
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i) {
                const u32x4 a = gload<u32x4>(p + 16 * i);
                w[4 * i] = a.x;
                w[4 * i + 1] = a.y;
                w[4 * i + 2] = a.z;
                w[4 * i + 3] = a.w;
            }
        }
    }

    // the values Codec<F>::load would give; zero where !keep
    template <typename CT>
    __device__ __forceinline__ void decode(CT v[N], bool keep) const {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            CT x;
            if constexpr (F == F64) {
                x = CT(__builtin_bit_cast(double, uint64_t(w[2 * i]) | (uint64_t(w[2 * i + 1]) << 32)));
            } else if constexpr (F == F32) {
                x = CT(__uint_as_float(w[i]));
            } else if constexpr (F == BF16) {
                x = CT(__uint_as_float(((w[i / 2] >> (16 * (i & 1))) & 0xffffu) << 16));
            } else if constexpr (F == F16) {
                x = CT(half_bits_to_float((w[i / 2] >> (16 * (i & 1))) & 0xffffu));
            } else if constexpr (F == E4M3) {
                x = CT(e4m3_scaled(w[i / 4] >> (8 * (i & 3))));
            } else {
                x = CT(e5m2(w[i / 4] >> (8 * (i & 3))));
            }
            v[i] = keep ? x : CT(0);
        }
    }
};

// Codes of format F read as CT with no decode (fp64 as fp64, fp32 as
// fp32): these keep the plain conditional loads, whose values the compiler
// leaves in flight; every other pairing takes the RawCodes pattern.
template <int F, typename CT>
constexpr bool direct_codes() {
    return (F == F64 && sizeof(CT) == 8) || (F == F32 && sizeof(CT) == 4);
}

// N consecutive values of a right-hand side (fp32 or fp64), loaded as
// RawCodes are and converted later.
template <typename XT, int N>
struct RawX {
    XT v[N];
    __device__ __forceinline__ void load(const XT* p) {
        if constexpr (sizeof(XT) * N % 16 == 0) {
#pragma unroll
            for (int i = 0; i < int(sizeof(XT)) * N / 16; ++i) {
                const u32x4 a = gload<u32x4>(reinterpret_cast<const uint8_t*>(p) + 16 * i);
                __builtin_memcpy(reinterpret_cast<uint8_t*>(v) + 16 * i, &a, 16);
            }
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = gload<XT>(p + i);
        }
    }
    template <typename CT>
    __device__ __forceinline__ void convert(CT out[N], bool keep) const {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = keep ? CT(v[i]) : CT(0);
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
#ifndef HODLR_CONTRACT_MINW
#define HODLR_CONTRACT_MINW 2
#endif
constexpr int kUnroll = HODLR_U_UNROLL;
constexpr int kLeafUnroll = HODLR_LEAF_UNROLL;

}  // namespace
}  // namespace hodlr

#endif  // HODLR_DEV_COMMON_H
