// Internal declarations of the LU solves (lu.cpp, kernels_lu.hip); not
// part of the public ABI.
#pragma once

#include <cstdint>

namespace hodlr {

// Dst (n x nrhs, ld ldd) = Src (ld lds), each fp64 or fp32 (src_f64,
// dst_f64); fp64 to fp32 rounds to nearest.  Launched on `stream`;
// returns a hipError_t as int.
int launch_lu_convert(const void* src, int64_t lds, bool src_f64, void* dst, int64_t ldd, bool dst_f64, int64_t n,
                      int nrhs, void* stream);

}  // namespace hodlr
