// Internal declarations of the LU solves (lu.cpp, kernels_lu.hip); not
// part of the public ABI.
#pragma once

#include <algorithm>
#include <cstdint>

namespace hodlr {

// ---------------------------------------------------------------------------
// triangular solves with the LU factors (hodlr_solve, kernels_lu.hip)
// ---------------------------------------------------------------------------
// One step of forward or back substitution over the tree.  The solve keeps
// two fp64 n x nrhs arrays: P (values still pending updates) and S (solved
// values).
//  * kind 0, a leaf: S[s0, s0+m) = M P[s0, s0+m), M the m x m inverse of the
//    leaf's triangular factor at image offset a;
//  * kind 1, a node: P[d0, d0+md) -= Bm (A^T S[s0, s0+m)), A (m x r) at
//    offset a, Bm (md x r) at offset b.
// Every matrix in the image is column-major with its row count as leading
// dimension.
struct LuStep {
    int32_t kind;
    int32_t m;
    int32_t md;
    int32_t r;
    int64_t s0;
    int64_t d0;
    int64_t a;
    int64_t b;
};

constexpr int kLuCols = 16;          // right-hand sides per workgroup of a solve step
constexpr int kLuParts = 32;         // workgroups of a node step's reduction

// Device memory of one solve with nrhs right-hand sides: P, S (n x nrhs
// each), the reduction's partial sums (kLuParts x nrhs x rmax) and T
// (nrhs x rmax), in doubles.
inline int64_t lu_workspace_doubles(int64_t n, int nrhs, int rmax) {
    return 2 * n * nrhs + int64_t(kLuParts + 1) * nrhs * std::max(rmax, 1);
}

// X = U^-1 L^-1 B on `stream`: B and X are fp64 (f64) or fp32, n x nrhs,
// column-major; fwd and bwd (host arrays) the forward and backward steps;
// img the device image of the factors; ws a device workspace of
// lu_workspace_doubles(n, nrhs, rmax).  Returns a hipError_t as int.
int launch_lu_solve(const double* img, const LuStep* fwd, int nfwd, const LuStep* bwd, int nbwd, int64_t n,
                    const void* B, int64_t ldb, void* X, int64_t ldx, int nrhs, bool f64, int rmax, double* ws,
                    void* stream);

}  // namespace hodlr
