// Host-side hooks shared by the library's C++ sources (host.cpp,
// construct.cpp).  Not part of the public ABI; hidden in the shared library.
#pragma once

#include <string>

#include "../../include/hodlr.h"

namespace hodlr {

// Set the calling thread's detail string (hodlr_last_error_message) and
// return s.
__attribute__((visibility("hidden"))) hodlr_status host_fail(hodlr_status s, const std::string& msg);

// Attach the squared Frobenius norms of the original matrix (||A||_F^2 and
// ||A_b||_F^2 of every off-diagonal block in canonical order) to an
// operator: hodlr_assign_precision then uses them when it is given neither
// xi nor norms2, and hodlr_get_norms returns them.
__attribute__((visibility("hidden"))) void attach_original_norms(hodlr_op op, double norm2_all,
                                                                  const double* norm2_blocks);

}  // namespace hodlr
