// Internal declarations of the construction from a kernel matrix
// (construct.cpp, kernels_build.hip); not part of the public ABI.
#pragma once

#include <algorithm>
#include <cstdint>

namespace hodlr {

// ---------------------------------------------------------------------------
// construction from a kernel matrix (hodlr_build_kernel, kernels_build.hip)
// ---------------------------------------------------------------------------
constexpr int kMaxSketch = 128;      // widest sketch (columns of Omega) of the range finder
constexpr int kGramRows = 1024;      // rows of a partial Gram matrix
constexpr int kBuildRows = 64;       // output rows of an on-the-fly product tile
constexpr int kResidualRows = 32;    // rows of a residual tile

struct BuildKernel {                 // A_ij = k(p_i, p_j) (+ diag_shift if i == j)
    int32_t kind;                    // 0 exp(-r^2/a), 1 1/(r+a), 2 log(r+a), 3 exp(-r), 4 1/(x_i-x_j) (1D)
    int32_t dim;                     // coordinates per point (1 or 2)
    double a;
    double diag_shift;
    double diag_value;               // used at i == j when diag_given
    int32_t diag_given;
    int32_t pad_;
};

struct BuildTile {                   // rows [r0, r0+nr) x columns [c0, c0+nc) of A
    int64_t r0, c0;
    int32_t nr, nc;
    int64_t out;                     // leaves: element offset of D_i
};

// One block's panel of a batched tall-skinny operation:
//  * apply: Out (outer x s, at o_off) = B W (trans 0: outer = rows, inner =
//    cols) or B^T W (trans 1: outer = cols, inner = rows), W (inner x s, at
//    w_off), B the block whose first row and column are r0 and c0;
//  * Omega: W (inner x s, at w_off) drawn for `block`;
//  * Gram: A (outer x s, at o_off);
//  * small product: C (outer x p, at c_off) = A (outer x s, at o_off) S
//    (s x p, at w_off);
//  * residual: Q (rows x s, at o_off), M^T (cols x s, at c_off).
// Matrices are column-major with leading dimension = their row count.
struct BuildPanel {
    int64_t r0, c0;
    int32_t outer, inner;
    int32_t s, p;
    int32_t trans, block;
    int64_t w_off, o_off, c_off;
};

struct BuildItem {                   // a workgroup's part of a panel: rows from row0
    int32_t panel;
    int32_t row0;
};

// Launches on `stream`; each returns a hipError_t as int.
int launch_build_norms(const BuildKernel& K, const double* P, const BuildTile* tiles, int ntiles, double* out,
                       void* stream);
int launch_build_omega(const BuildPanel* pans, int npan, uint64_t seed, double* W, void* stream);
int launch_build_apply(const BuildKernel& K, const double* P, const BuildPanel* pans, const BuildItem* items,
                       int nitems, const double* W, double* Out, void* stream);
int launch_build_gram(const BuildPanel* pans, const BuildItem* items, int nitems, const double* A, double* out,
                      void* stream);
int launch_build_small_gemm(const BuildPanel* pans, const BuildItem* items, int nitems, const double* A,
                            const double* S, double* C, void* stream);
int launch_build_residual(const BuildKernel& K, const double* P, const BuildPanel* pans, const BuildItem* items,
                          int nitems, const double* Q, const double* Mt, double* out, void* stream);
int launch_build_leaves(const BuildKernel& K, const double* P, const BuildTile* leaves, int nleaves, double* D,
                        void* stream);

}  // namespace hodlr
