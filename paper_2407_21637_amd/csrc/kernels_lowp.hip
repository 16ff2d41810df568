// HIP kernels (gfx950) of the HODLR product in a low working precision
// (X and Y in bf16 or fp16): k_contract_lp, k_reduce_lp, k_expand_lp and
// the per-assignment build of the augmented operands (lowp_path.h).  One
// translation unit of the library (see kernels.hip).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hodlr_internal.h"

#include "dev_common.h"
#include "wave_path.h"
#include "wide_path.h"
#include "lowp_path.h"

namespace hodlr {

int launch_matvec_lp(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, int w,
                     void* stream, void* const* events, bool* ran) {
    const Timer tm{events, ran, static_cast<hipStream_t>(stream)};
    const hipError_t e = w == 0 ? launch_lp<__bf16>(kp, X, ldx, Y, ldy, nrhs, tm)
                                : launch_lp<_Float16>(kp, X, ldx, Y, ldy, nrhs, tm);
    return int(e);
}

int launch_build_aug(const KParams& kp, int w, void* stream) {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    return int(w == 0 ? launch_build_aug_w<__bf16>(kp, s) : launch_build_aug_w<_Float16>(kp, s));
}

}  // namespace hodlr
