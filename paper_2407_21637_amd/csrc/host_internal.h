// Host-side hooks shared by the library's C++ sources (host.cpp,
// construct.cpp).  Not part of the public ABI; hidden in the shared library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

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

// The operator as stored: fp64 leaves and every generator decoded from its
// codes (the mixed-precision representation the product uses), with the
// tree (levels 0..depth of node boundaries, as hodlr_tree_bounds).
struct StoredView {
    int64_t n = 0;
    int depth = 0;
    std::vector<int64_t> bounds;
    std::vector<std::vector<double>> leaves;   // m_i x m_i, column-major
    std::vector<std::vector<double>> U, V;     // r_b x p_b, c_b x p_b, column-major
    std::vector<int32_t> rank;
};
__attribute__((visibility("hidden"))) hodlr_status stored_operator(hodlr_op op, StoredView* out);

// LU factors attached to an operator (hodlr_lu); freed by lu_free when the
// operator is destroyed or reassigned.
__attribute__((visibility("hidden"))) void* get_lu(hodlr_op op);
__attribute__((visibility("hidden"))) void set_lu(hodlr_op op, void* lu, void (*lu_free)(void*));
__attribute__((visibility("hidden"))) int op_device(hodlr_op op);

}  // namespace hodlr
