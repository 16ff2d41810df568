// LU factorization of the stored HODLR operator (hodlr_lu) and the
// triangular solves on the GPU (hodlr_solve).
//
// Method: Carson, Chen, Liu, "Mixed Precision HODLR Matrices"
// (arXiv 2407.21637), Sect. 3.4, Alg. "HODLR_LU", computed in fp64 (the
// working precision u, which meets u <~ eps / n for the eps of the
// representation) on the mixed-precision representation: fp64 leaves and
// every generator decoded from its stored codes.  For H = [[H11, H12],
// [H21, H22]] with H12 = U12 V12^T, H21 = U21 V21^T:
//   L11, U11 = LU(H11);
//   X12 = L11^-1 U12        (U's block (1,2) = X12 V12^T),
//   Y21 = U11^-T V21        (L's block (2,1) = U21 Y21^T),
//   S = H22 - U21 (Y21^T X12) V12^T, a low-rank update applied down H22's
//       tree: leaves updated densely, each off-diagonal block's generators
//       extended by the update's and truncated to the smallest rank with
//       ||B - U V^T||_F <= eps ||B||_F (the truncation assumption of
//       Sect. 3.4; eps = 0 keeps every nonzero singular value);
//   L22, U22 = LU(S).
// Leaves: LU without pivoting (Doolittle, unit lower L), as the algorithm
// performs no row exchanges.  Truncation: Householder QR of both factors
// and a one-sided Jacobi SVD of the small core.
//
// The solve X = U^-1 L^-1 B runs on the GPU as two HODLR products.  The
// inverse of a lower triangular HODLR matrix is lower triangular HODLR with
// the same tree and ranks: for L = [[L11, 0], [U21 Y21^T, L22]],
//   L^-1 = [[L11^-1, 0], [(-L22^-1 U21)(L11^-T Y21)^T, L22^-1]],
// and for U = [[U11, X12 V12^T], [0, U22]],
//   U^-1 = [[U11^-1, (-U11^-1 X12)(U22^-T V12)^T], [0, U22^-1]].
// After the factorization the generators of both inverses are formed on the
// host (triangular solves over the subtrees, in fp64) with the inverses of
// the leaves' triangular factors as their leaves; each inverse becomes an
// internal uniform-fp64 operator with fp64 accumulation (hodlr_create), and
// hodlr_solve applies them with hodlr_matvec: every solve is then two
// products on the product's kernels instead of a chain of dependent steps.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <atomic>
#include <future>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hodlr.h"
#include "lu_internal.h"
#include "host_internal.h"

using namespace hodlr;

namespace {

// column-major dense matrix
struct Mat {
    int64_t r = 0, c = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int64_t rr, int64_t cc) : r(rr), c(cc), a(size_t(rr * cc), 0.0) {}
    double& operator()(int64_t i, int64_t j) { return a[size_t(j * r + i)]; }
    double operator()(int64_t i, int64_t j) const { return a[size_t(j * r + i)]; }
};

Mat from_vec(const std::vector<double>& v, int64_t r, int64_t c) {
    Mat m(r, c);
    std::copy(v.begin(), v.begin() + r * c, m.a.begin());
    return m;
}

Mat mul(const Mat& A, const Mat& B) {                 // A B
    Mat C(A.r, B.c);
    for (int64_t j = 0; j < B.c; ++j)
        for (int64_t k = 0; k < A.c; ++k) {
            const double b = B(k, j);
            if (b == 0.0) continue;
            const double* ak = A.a.data() + k * A.r;
            double* cj = C.a.data() + j * C.r;
            for (int64_t i = 0; i < A.r; ++i) cj[i] += ak[i] * b;
        }
    return C;
}

Mat mul_tn(const Mat& A, const Mat& B) {              // A^T B
    Mat C(A.c, B.c);
    for (int64_t j = 0; j < B.c; ++j)
        for (int64_t i = 0; i < A.c; ++i) {
            const double* ai = A.a.data() + i * A.r;
            const double* bj = B.a.data() + j * B.r;
            double s = 0.0;
            for (int64_t k = 0; k < A.r; ++k) s += ai[k] * bj[k];
            C(i, j) = s;
        }
    return C;
}

void sub_mul_nt(Mat& D, const Mat& A, const Mat& B) {   // D -= A B^T
    for (int64_t j = 0; j < D.c; ++j)
        for (int64_t k = 0; k < A.c; ++k) {
            const double b = B(j, k);
            if (b == 0.0) continue;
            const double* ak = A.a.data() + k * A.r;
            double* dj = D.a.data() + j * D.r;
            for (int64_t i = 0; i < D.r; ++i) dj[i] -= ak[i] * b;
        }
}

Mat rows(const Mat& A, int64_t r0, int64_t nr) {
    Mat B(nr, A.c);
    for (int64_t j = 0; j < A.c; ++j) std::copy(A.a.begin() + j * A.r + r0, A.a.begin() + j * A.r + r0 + nr,
                                                B.a.begin() + j * nr);
    return B;
}

Mat hcat(const Mat& A, const Mat& B) {
    Mat C(A.r, A.c + B.c);
    std::copy(A.a.begin(), A.a.end(), C.a.begin());
    std::copy(B.a.begin(), B.a.end(), C.a.begin() + A.r * A.c);
    return C;
}

Mat vcat(const Mat& A, const Mat& B) {
    Mat C(A.r + B.r, A.c);
    for (int64_t j = 0; j < A.c; ++j) {
        std::copy(A.a.begin() + j * A.r, A.a.begin() + (j + 1) * A.r, C.a.begin() + j * C.r);
        std::copy(B.a.begin() + j * B.r, B.a.begin() + (j + 1) * B.r, C.a.begin() + j * C.r + A.r);
    }
    return C;
}

Mat scaled(const Mat& A, double s) {
    Mat B = A;
    for (double& x : B.a) x *= s;
    return B;
}

// Thin Householder QR: A (m x q) = Q R, Q m x k orthonormal, R k x q upper,
// k = min(m, q).  Reflectors H = I - tau [1; v] [1; v]^T with the leading
// entry normalised to 1 and the column norm taken with scaling, so that
// columns of tiny entries neither underflow to a zero norm nor divide by one.
void householder_qr(Mat A, Mat& Q, Mat& R) {
    const int64_t m = A.r, q = A.c, k = std::min(m, q);
    std::vector<std::vector<double>> vs;
    std::vector<double> taus;
    for (int64_t j = 0; j < k; ++j) {
        std::vector<double> v(static_cast<size_t>(m - j), 0.0);
        v[0] = 1.0;
        double scale = 0.0;
        for (int64_t i = j + 1; i < m; ++i) scale = std::max(scale, std::fabs(A(i, j)));
        double tau = 0.0;
        if (scale > 0.0) {
            double ss = 0.0;
            for (int64_t i = j + 1; i < m; ++i) ss += (A(i, j) / scale) * (A(i, j) / scale);
            const double alpha = A(j, j), xnorm = scale * std::sqrt(ss);
            const double beta = -std::copysign(std::hypot(alpha, xnorm), alpha);
            tau = (beta - alpha) / beta;
            const double inv = 1.0 / (alpha - beta);
            for (int64_t i = j + 1; i < m; ++i) v[size_t(i - j)] = A(i, j) * inv;
            for (int64_t c = j; c < q; ++c) {
                double t = A(j, c);
                for (int64_t i = j + 1; i < m; ++i) t += v[size_t(i - j)] * A(i, c);
                t *= tau;
                A(j, c) -= t;
                for (int64_t i = j + 1; i < m; ++i) A(i, c) -= t * v[size_t(i - j)];
            }
        }
        vs.push_back(std::move(v));
        taus.push_back(tau);
    }
    R = Mat(k, q);
    for (int64_t j = 0; j < q; ++j)
        for (int64_t i = 0; i <= std::min(j, k - 1); ++i) R(i, j) = A(i, j);
    Q = Mat(m, k);
    for (int64_t i = 0; i < k; ++i) Q(i, i) = 1.0;
    for (int64_t j = k - 1; j >= 0; --j) {
        const std::vector<double>& v = vs[size_t(j)];
        const double tau = taus[size_t(j)];
        if (tau == 0.0) continue;
        for (int64_t c = 0; c < k; ++c) {
            double t = 0.0;
            for (int64_t i = j; i < m; ++i) t += v[size_t(i - j)] * Q(i, c);
            t *= tau;
            for (int64_t i = j; i < m; ++i) Q(i, c) -= t * v[size_t(i - j)];
        }
    }
}

// SVD of a small matrix A (r x c) by one-sided Jacobi on its columns:
// A = W diag(s) Z^T with W r x c', Z c x c', c' = c (W columns of zero
// singular values are zero), singular values descending.
void jacobi_svd(Mat A, Mat& W, std::vector<double>& s, Mat& Z) {
    const int64_t r = A.r, c = A.c;
    Z = Mat(c, c);
    for (int64_t i = 0; i < c; ++i) Z(i, i) = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rot = false;
        for (int64_t p = 0; p + 1 < c; ++p)
            for (int64_t q = p + 1; q < c; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int64_t i = 0; i < r; ++i) {
                    al += A(i, p) * A(i, p);
                    be += A(i, q) * A(i, q);
                    ga += A(i, p) * A(i, q);
                }
                if (ga == 0.0 || std::fabs(ga) <= 1e-15 * std::sqrt(al * be)) continue;
                rot = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = std::copysign(1.0, zeta) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int64_t i = 0; i < r; ++i) {
                    const double x = A(i, p), y = A(i, q);
                    A(i, p) = cs * x - sn * y;
                    A(i, q) = sn * x + cs * y;
                }
                for (int64_t i = 0; i < c; ++i) {
                    const double x = Z(i, p), y = Z(i, q);
                    Z(i, p) = cs * x - sn * y;
                    Z(i, q) = sn * x + cs * y;
                }
            }
        if (!rot) break;
    }
    std::vector<double> nrm(static_cast<size_t>(c));
    for (int64_t j = 0; j < c; ++j) {
        double t = 0.0;
        for (int64_t i = 0; i < r; ++i) t += A(i, j) * A(i, j);
        nrm[size_t(j)] = std::sqrt(t);
    }
    std::vector<int64_t> ord(static_cast<size_t>(c));
    for (int64_t j = 0; j < c; ++j) ord[size_t(j)] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return nrm[size_t(x)] > nrm[size_t(y)]; });
    W = Mat(r, c);
    Mat Z2(c, c);
    s.assign(size_t(c), 0.0);
    for (int64_t jj = 0; jj < c; ++jj) {
        const int64_t j = ord[size_t(jj)];
        s[size_t(jj)] = nrm[size_t(j)];
        for (int64_t i = 0; i < r; ++i) W(i, jj) = nrm[size_t(j)] > 0.0 ? A(i, j) / nrm[size_t(j)] : 0.0;
        for (int64_t i = 0; i < c; ++i) Z2(i, jj) = Z(i, j);
    }
    Z = Z2;
}

// A B^T as U V^T, U orthonormal, the smallest rank with
// ||A B^T - U V^T||_F <= eps ||A B^T||_F (eps = 0: every nonzero singular value).
void truncate(const Mat& A, const Mat& B, double eps, Mat& U, Mat& V) {
    if (A.c == 0 || A.r == 0 || B.r == 0) {
        U = Mat(A.r, 0);
        V = Mat(B.r, 0);
        return;
    }
    Mat Qa, Ra, Qb, Rb;
    householder_qr(A, Qa, Ra);
    householder_qr(B, Qb, Rb);
    Mat core(Ra.r, Rb.r);                              // Ra Rb^T
    for (int64_t j = 0; j < Rb.r; ++j)
        for (int64_t i = 0; i < Ra.r; ++i) {
            double t = 0.0;
            for (int64_t k = 0; k < Ra.c; ++k) t += Ra(i, k) * Rb(j, k);
            core(i, j) = t;
        }
    // one-sided Jacobi on the columns of the core, or of its transpose when
    // it is wide, so that min(rows, cols) singular values come out
    Mat W, Z;
    std::vector<double> s;
    if (core.r >= core.c) {
        jacobi_svd(core, W, s, Z);                     // core = W diag(s) Z^T
    } else {
        Mat ct(core.c, core.r);
        for (int64_t j = 0; j < core.c; ++j)
            for (int64_t i = 0; i < core.r; ++i) ct(j, i) = core(i, j);
        jacobi_svd(ct, Z, s, W);                       // core^T = Z diag(s) W^T
    }
    double tot = 0.0;
    for (double x : s) tot += x * x;
    int64_t p = 0;
    if (eps > 0.0) {
        double tail = tot;
        for (p = 0; p < int64_t(s.size()); ++p) {
            if (tail <= eps * eps * tot) break;
            tail -= s[size_t(p)] * s[size_t(p)];
        }
        if (p == int64_t(s.size()) && !(tail <= eps * eps * tot)) p = int64_t(s.size());
    } else {
        while (p < int64_t(s.size()) && s[size_t(p)] > 0.0) ++p;
    }
    Mat Wp(W.r, p), Zp(Z.r, p);
    for (int64_t j = 0; j < p; ++j) {
        for (int64_t i = 0; i < W.r; ++i) Wp(i, j) = W(i, j);
        for (int64_t i = 0; i < Z.r; ++i) Zp(i, j) = Z(i, j) * s[size_t(j)];
    }
    U = mul(Qa, Wp);
    V = mul(Qb, Zp);
}

// ---------------------------------------------------------------------------
// the HODLR matrix being factored, and its factors
// ---------------------------------------------------------------------------
struct Tree {
    int depth = 0;
    std::vector<int64_t> b0, sz;      // per node id (2^k - 1 + j): first row, size
    int id(int k, int64_t j) const { return (1 << k) - 1 + int(j); }
};

struct Factors {
    Tree t;
    int64_t n = 0;
    // working matrix: leaves (dense) and per internal node the generators
    std::vector<Mat> D;                     // per leaf
    std::vector<Mat> U12, V12, U21, V21;    // per internal node id
    // factors
    std::vector<Mat> Lf, Uf;                // per leaf: unit lower, upper
    std::vector<Mat> X12, Y21;              // per internal node: U's (1,2) = X12 V12^T, L's (2,1) = U21 Y21^T
    double eps = 0.0;
    int32_t max_rank = 0;
    // the inverse factors as device operators, for the solve
    int device = -1;
    hodlr_op linv = nullptr, uinv = nullptr;
    std::mutex mu;                          // guards the solve workspace
    double* d_ws = nullptr;
    int64_t ws_doubles = 0;
};

void free_factors(void* p) {
    Factors* f = static_cast<Factors*>(p);
    if (f->linv) (void)hodlr_destroy(f->linv);
    if (f->uinv) (void)hodlr_destroy(f->uinv);
    if (f->d_ws) {
        (void)hipSetDevice(f->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(f->d_ws);
    }
    delete f;
}

void dense_lu(const Mat& A, Mat& L, Mat& U, bool* singular) {    // Doolittle, no pivoting
    const int64_t n = A.r;
    L = Mat(n, n);
    U = Mat(n, n);
    for (int64_t k = 0; k < n; ++k) {
        for (int64_t j = k; j < n; ++j) {
            double s = A(k, j);
            for (int64_t q = 0; q < k; ++q) s -= L(k, q) * U(q, j);
            U(k, j) = s;
        }
        L(k, k) = 1.0;
        if (U(k, k) == 0.0) *singular = true;
        for (int64_t i = k + 1; i < n; ++i) {
            double s = A(i, k);
            for (int64_t q = 0; q < k; ++q) s -= L(i, q) * U(q, k);
            L(i, k) = U(k, k) != 0.0 ? s / U(k, k) : 0.0;
        }
    }
}

Mat fwd_solve(const Mat& L, Mat B) {                 // L X = B, L lower
    for (int64_t c = 0; c < B.c; ++c)
        for (int64_t i = 0; i < L.r; ++i) {
            double s = B(i, c);
            for (int64_t j = 0; j < i; ++j) s -= L(i, j) * B(j, c);
            B(i, c) = s / L(i, i);
        }
    return B;
}

Mat fwd_solve_ut(const Mat& U, Mat B) {              // U^T X = B, U upper
    for (int64_t c = 0; c < B.c; ++c)
        for (int64_t i = 0; i < U.r; ++i) {
            double s = B(i, c);
            for (int64_t j = 0; j < i; ++j) s -= U(j, i) * B(j, c);
            B(i, c) = s / U(i, i);
        }
    return B;
}

// L X = B with the factored subtree at node (k, j) (B: the node's rows)
Mat solve_lower(const Factors& F, int k, int64_t j, const Mat& B) {
    if (k == F.t.depth) return fwd_solve(F.Lf[size_t(j)], B);
    const int id = F.t.id(k, j);
    const int64_t m1 = F.t.sz[size_t(F.t.id(k + 1, 2 * j))];
    Mat X1 = solve_lower(F, k + 1, 2 * j, rows(B, 0, m1));
    Mat B2 = rows(B, m1, B.r - m1);
    sub_mul_nt(B2, F.U21[size_t(id)], mul_tn(X1, F.Y21[size_t(id)]));   // B2 -= U21 (Y21^T X1)
    return vcat(X1, solve_lower(F, k + 1, 2 * j + 1, B2));
}

// U^T X = B with the factored subtree at node (k, j)
Mat solve_upper_t(const Factors& F, int k, int64_t j, const Mat& B) {
    if (k == F.t.depth) return fwd_solve_ut(F.Uf[size_t(j)], B);
    const int id = F.t.id(k, j);
    const int64_t m1 = F.t.sz[size_t(F.t.id(k + 1, 2 * j))];
    Mat X1 = solve_upper_t(F, k + 1, 2 * j, rows(B, 0, m1));
    Mat B2 = rows(B, m1, B.r - m1);
    sub_mul_nt(B2, F.V12[size_t(id)], mul_tn(X1, F.X12[size_t(id)]));   // B2 -= V12 (X12^T X1)
    return vcat(X1, solve_upper_t(F, k + 1, 2 * j + 1, B2));
}

Mat bwd_solve(const Mat& U, Mat B) {                 // U X = B, U upper
    for (int64_t c = 0; c < B.c; ++c)
        for (int64_t i = U.r - 1; i >= 0; --i) {
            double s = B(i, c);
            for (int64_t j = i + 1; j < U.r; ++j) s -= U(i, j) * B(j, c);
            B(i, c) = s / U(i, i);
        }
    return B;
}

Mat bwd_solve_lt(const Mat& L, Mat B) {              // L^T X = B, L lower
    for (int64_t c = 0; c < B.c; ++c)
        for (int64_t i = L.r - 1; i >= 0; --i) {
            double s = B(i, c);
            for (int64_t j = i + 1; j < L.r; ++j) s -= L(j, i) * B(j, c);
            B(i, c) = s / L(i, i);
        }
    return B;
}

// U X = B with the factored subtree at node (k, j): back substitution
Mat solve_upper(const Factors& F, int k, int64_t j, const Mat& B) {
    if (k == F.t.depth) return bwd_solve(F.Uf[size_t(j)], B);
    const int id = F.t.id(k, j);
    const int64_t m1 = F.t.sz[size_t(F.t.id(k + 1, 2 * j))];
    Mat X2 = solve_upper(F, k + 1, 2 * j + 1, rows(B, m1, B.r - m1));
    Mat B1 = rows(B, 0, m1);
    sub_mul_nt(B1, F.X12[size_t(id)], mul_tn(X2, F.V12[size_t(id)]));   // B1 -= X12 (V12^T X2)
    return vcat(solve_upper(F, k + 1, 2 * j, B1), X2);
}

// L^T X = B with the factored subtree at node (k, j): L^T's (1,2) block is Y21 U21^T
Mat solve_lower_t(const Factors& F, int k, int64_t j, const Mat& B) {
    if (k == F.t.depth) return bwd_solve_lt(F.Lf[size_t(j)], B);
    const int id = F.t.id(k, j);
    const int64_t m1 = F.t.sz[size_t(F.t.id(k + 1, 2 * j))];
    Mat X2 = solve_lower_t(F, k + 1, 2 * j + 1, rows(B, m1, B.r - m1));
    Mat B1 = rows(B, 0, m1);
    sub_mul_nt(B1, F.Y21[size_t(id)], mul_tn(X2, F.U21[size_t(id)]));   // B1 -= Y21 (U21^T X2)
    return vcat(solve_lower_t(F, k + 1, 2 * j, B1), X2);
}

// the working matrix of subtree (k, j) minus A B^T, blocks truncated
void subtract_lowrank(Factors& F, int k, int64_t j, const Mat& A, const Mat& B) {
    if (A.c == 0) return;
    if (k == F.t.depth) {
        sub_mul_nt(F.D[size_t(j)], A, B);
        return;
    }
    const int id = F.t.id(k, j);
    const int64_t m1 = F.t.sz[size_t(F.t.id(k + 1, 2 * j))], m2 = F.t.sz[size_t(id)] - m1;
    const Mat A1 = rows(A, 0, m1), A2 = rows(A, m1, m2), B1 = rows(B, 0, m1), B2 = rows(B, m1, m2);
    auto t12 = std::async(std::launch::async, [&] {
        Mat U, V;
        truncate(hcat(F.U12[size_t(id)], scaled(A1, -1.0)), hcat(F.V12[size_t(id)], B2), F.eps, U, V);
        F.U12[size_t(id)] = std::move(U);
        F.V12[size_t(id)] = std::move(V);
    });
    Mat U, V;
    truncate(hcat(F.U21[size_t(id)], scaled(A2, -1.0)), hcat(F.V21[size_t(id)], B1), F.eps, U, V);
    F.U21[size_t(id)] = std::move(U);
    F.V21[size_t(id)] = std::move(V);
    t12.wait();
    F.max_rank = std::max<int32_t>({F.max_rank, int32_t(F.U12[size_t(id)].c), int32_t(F.U21[size_t(id)].c)});
    subtract_lowrank(F, k + 1, 2 * j, A1, B1);
    subtract_lowrank(F, k + 1, 2 * j + 1, A2, B2);
}

bool factor(Factors& F, int k, int64_t j) {
    if (k == F.t.depth) {
        bool singular = false;
        dense_lu(F.D[size_t(j)], F.Lf[size_t(j)], F.Uf[size_t(j)], &singular);
        return !singular;
    }
    const int id = F.t.id(k, j);
    if (!factor(F, k + 1, 2 * j)) return false;
    F.X12[size_t(id)] = solve_lower(F, k + 1, 2 * j, F.U12[size_t(id)]);
    F.Y21[size_t(id)] = solve_upper_t(F, k + 1, 2 * j, F.V21[size_t(id)]);
    const Mat C = mul_tn(F.Y21[size_t(id)], F.X12[size_t(id)]);             // Y21^T X12
    subtract_lowrank(F, k + 1, 2 * j + 1, mul(F.U21[size_t(id)], C), F.V12[size_t(id)]);
    return factor(F, k + 1, 2 * j + 1);
}

Mat invert_lower(const Mat& L) {
    Mat I(L.r, L.r);
    for (int64_t i = 0; i < L.r; ++i) I(i, i) = 1.0;
    return fwd_solve(L, I);
}

Mat invert_upper(const Mat& U) {              // (U^-1) = ((U^T)^-1)^T
    Mat I(U.r, U.r);
    for (int64_t i = 0; i < U.r; ++i) I(i, i) = 1.0;
    Mat X = fwd_solve_ut(U, I);               // X = U^-T
    Mat Y(U.r, U.r);
    for (int64_t i = 0; i < U.r; ++i)
        for (int64_t j = 0; j < U.r; ++j) Y(i, j) = X(j, i);
    return Y;
}

// ||A B^T||_F^2 = sum_ij (A^T A)_ij (B^T B)_ij
double lowrank_norm2(const Mat& A, const Mat& B) {
    if (A.c == 0) return 0.0;
    const Mat Ga = mul_tn(A, A), Gb = mul_tn(B, B);
    double s = 0.0;
    for (size_t i = 0; i < Ga.a.size(); ++i) s += Ga.a[i] * Gb.a[i];
    return std::max(s, 0.0);
}

// Frobenius norms of L and U (the quantities of Cor. "LU of mixed-precision
// HODLR matrices"), without forming them.
void lu_norms(const Factors& F, double* nl, double* nu) {
    double l2 = 0.0, u2 = 0.0;
    for (size_t j = 0; j < F.Lf.size(); ++j) {
        for (double x : F.Lf[j].a) l2 += x * x;
        for (double x : F.Uf[j].a) u2 += x * x;
    }
    for (int id = 0; id < (1 << F.t.depth) - 1; ++id) {
        l2 += lowrank_norm2(F.U21[size_t(id)], F.Y21[size_t(id)]);
        u2 += lowrank_norm2(F.X12[size_t(id)], F.V12[size_t(id)]);
    }
    *nl = std::sqrt(l2);
    *nu = std::sqrt(u2);
}

// L^-1 and U^-1 as device operators (uniform fp64, fp64 accumulation)
hodlr_status make_inverses(Factors& F) {
    const Tree& t = F.t;
    const int depth = t.depth, nl = 1 << depth, ninner = nl - 1;
    std::vector<Mat> li(static_cast<size_t>(nl)), ui(static_cast<size_t>(nl));
    std::vector<Mat> lu_(size_t(std::max(ninner, 1))), lv_(lu_.size()), uu_(lu_.size()), uv_(lu_.size());
    // independent tasks: the leaves' inverses and each node's four generators
    const int ntasks = nl + ninner;
    std::atomic<int> next{0};
    auto work = [&] {
        for (int q = next++; q < ntasks; q = next++) {
            if (q < nl) {
                li[size_t(q)] = invert_lower(F.Lf[size_t(q)]);
                ui[size_t(q)] = invert_upper(F.Uf[size_t(q)]);
                continue;
            }
            const int id = q - nl;
            int k = 0;
            while (((1 << (k + 1)) - 1) <= id) ++k;
            const int64_t j = id - ((int64_t(1) << k) - 1);
            lu_[size_t(id)] = scaled(solve_lower(F, k + 1, 2 * j + 1, F.U21[size_t(id)]), -1.0);
            lv_[size_t(id)] = solve_lower_t(F, k + 1, 2 * j, F.Y21[size_t(id)]);
            uu_[size_t(id)] = scaled(solve_upper(F, k + 1, 2 * j, F.X12[size_t(id)]), -1.0);
            uv_[size_t(id)] = solve_upper_t(F, k + 1, 2 * j + 1, F.V12[size_t(id)]);
        }
    };
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned i = 1; i < nth; ++i) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    // the two operators in canonical block order: block (k, j) has rows node j, columns node j^1;
    // j even is the upper block of node (k-1, j/2), j odd the lower one
    const int nb = (1 << (depth + 1)) - 2;
    std::vector<int64_t> lb(size_t(nl) + 1);
    for (int j = 0; j < nl; ++j) lb[size_t(j)] = t.b0[size_t(t.id(depth, j))];
    lb[size_t(nl)] = F.n;
    std::vector<const double*> lp(static_cast<size_t>(nl)), up(static_cast<size_t>(nl));
    std::vector<int64_t> ld(static_cast<size_t>(nl));
    for (int j = 0; j < nl; ++j) {
        lp[size_t(j)] = li[size_t(j)].a.data();
        up[size_t(j)] = ui[size_t(j)].a.data();
        ld[size_t(j)] = std::max<int64_t>(1, li[size_t(j)].r);
    }
    std::vector<hodlr_lowrank> bl(size_t(std::max(nb, 1))), bu(bl.size());
    for (int k = 1; k <= depth; ++k)
        for (int64_t j = 0; j < (int64_t(1) << k); ++j) {
            const int b = (1 << k) - 2 + int(j), parent = t.id(k - 1, j / 2);
            const int64_t rr = std::max<int64_t>(1, t.sz[size_t(t.id(k, j))]);
            const int64_t cc = std::max<int64_t>(1, t.sz[size_t(t.id(k, j ^ 1))]);
            hodlr_lowrank none{0, nullptr, rr, nullptr, cc};
            if ((j & 1) == 0) {          // upper: zero in L^-1
                const Mat &Ug = uu_[size_t(parent)], &Vg = uv_[size_t(parent)];
                bl[size_t(b)] = none;
                bu[size_t(b)] = hodlr_lowrank{int32_t(Ug.c), Ug.a.data(), rr, Vg.a.data(), cc};
            } else {                     // lower: zero in U^-1
                const Mat &Ug = lu_[size_t(parent)], &Vg = lv_[size_t(parent)];
                bl[size_t(b)] = hodlr_lowrank{int32_t(Ug.c), Ug.a.data(), rr, Vg.a.data(), cc};
                bu[size_t(b)] = none;
            }
        }
    hodlr_status r = hodlr_create(&F.linv, F.n, depth, lb.data(), lp.data(), ld.data(), bl.data(), F.device);
    if (r == HODLR_OK) r = hodlr_create(&F.uinv, F.n, depth, lb.data(), up.data(), ld.data(), bu.data(), F.device);
    return r;
}

}  // namespace

extern "C" hodlr_status hodlr_lu(hodlr_op op, double eps, hodlr_lu_report* report) {
    if (!op) return host_fail(HODLR_E_ARG, "op is NULL");
    if (!(eps >= 0.0 && eps < 1.0)) return host_fail(HODLR_E_ARG, "eps must lie in [0, 1)");
    const auto t0 = std::chrono::steady_clock::now();
    StoredView sv;
    hodlr_status r = stored_operator(op, &sv);
    if (r != HODLR_OK) return r;
    std::unique_ptr<Factors> F(new Factors);
    F->n = sv.n;
    F->eps = eps;
    F->device = op_device(op);
    Tree& t = F->t;
    t.depth = sv.depth;
    const int nnodes = (1 << (sv.depth + 1)) - 1;
    t.b0.resize(size_t(nnodes));
    t.sz.resize(size_t(nnodes));
    for (int k = 0; k <= sv.depth; ++k) {
        const int64_t* lv = sv.bounds.data() + ((int64_t(1) << k) - 1) + k;
        for (int64_t j = 0; j < (int64_t(1) << k); ++j) {
            t.b0[size_t(t.id(k, j))] = lv[j];
            t.sz[size_t(t.id(k, j))] = lv[j + 1] - lv[j];
        }
    }
    const int nl = 1 << sv.depth, ninner = nl - 1;
    F->D.resize(size_t(nl));
    F->Lf.resize(size_t(nl));
    F->Uf.resize(size_t(nl));
    for (int j = 0; j < nl; ++j) {
        const int64_t m = t.sz[size_t(t.id(sv.depth, j))];
        F->D[size_t(j)] = from_vec(sv.leaves[size_t(j)], m, m);
    }
    F->U12.resize(size_t(std::max(ninner, 1)));
    F->V12.resize(F->U12.size());
    F->U21.resize(F->U12.size());
    F->V21.resize(F->U12.size());
    F->X12.resize(F->U12.size());
    F->Y21.resize(F->U12.size());
    // canonical block (k, j) (rows node j, cols node j^1) is H12 of node (k-1, j/2) when j is even, H21 when odd
    for (int k = 1; k <= sv.depth; ++k)
        for (int64_t j = 0; j < (int64_t(1) << k); ++j) {
            const int b = (1 << k) - 2 + int(j);
            const int parent = t.id(k - 1, j / 2);
            const int64_t rr = t.sz[size_t(t.id(k, j))], cc = t.sz[size_t(t.id(k, j ^ 1))];
            const int p = sv.rank[size_t(b)];
            Mat Ub = from_vec(sv.U[size_t(b)], rr, p), Vb = from_vec(sv.V[size_t(b)], cc, p);
            F->max_rank = std::max(F->max_rank, p);
            if ((j & 1) == 0) {
                F->U12[size_t(parent)] = std::move(Ub);
                F->V12[size_t(parent)] = std::move(Vb);
            } else {
                F->U21[size_t(parent)] = std::move(Ub);
                F->V21[size_t(parent)] = std::move(Vb);
            }
        }
    if (!factor(*F, 0, 0))
        return host_fail(HODLR_E_UNSUPPORTED, "a zero pivot in a leaf: LU without pivoting does not exist");
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (F->device >= 0 && (r = make_inverses(*F)) != HODLR_OK) {
        const std::string msg = hodlr_last_error_message();
        free_factors(F.release());
        return host_fail(r, "the inverse factors as device operators: " + msg);
    }
    if (report) {
        report->ms_factor = ms;
        lu_norms(*F, &report->norm_l, &report->norm_u);
        report->max_rank = F->max_rank;
        report->reserved_ = 0;
    }
    set_lu(op, F.release(), free_factors);
    return host_fail(HODLR_OK, "");
}

extern "C" hodlr_status hodlr_lu_dense(hodlr_op op, double* L, int64_t ldl, double* U, int64_t ldu) {
    if (!op) return host_fail(HODLR_E_ARG, "op is NULL");
    Factors* F = static_cast<Factors*>(get_lu(op));
    if (!F) return host_fail(HODLR_E_STATE, "no LU factors: call hodlr_lu first");
    const int64_t n = F->n;
    if ((L && ldl < n) || (U && ldu < n)) return host_fail(HODLR_E_ARG, "leading dimension below n");
    const Tree& t = F->t;
    const int depth = t.depth;
    for (int64_t c = 0; c < n; ++c) {
        if (L) std::fill(L + c * ldl, L + c * ldl + n, 0.0);
        if (U) std::fill(U + c * ldu, U + c * ldu + n, 0.0);
    }
    for (int64_t j = 0; j < (int64_t(1) << depth); ++j) {
        const int id = t.id(depth, j);
        const int64_t r0 = t.b0[size_t(id)], m = t.sz[size_t(id)];
        for (int64_t c = 0; c < m; ++c)
            for (int64_t i = 0; i < m; ++i) {
                if (L) L[(r0 + c) * ldl + r0 + i] = F->Lf[size_t(j)](i, c);
                if (U) U[(r0 + c) * ldu + r0 + i] = F->Uf[size_t(j)](i, c);
            }
    }
    for (int k = 0; k < depth; ++k)
        for (int64_t j = 0; j < (int64_t(1) << k); ++j) {
            const int id = t.id(k, j), c1 = t.id(k + 1, 2 * j), c2 = t.id(k + 1, 2 * j + 1);
            const int64_t a = t.b0[size_t(c1)], m1 = t.sz[size_t(c1)], b = t.b0[size_t(c2)], m2 = t.sz[size_t(c2)];
            if (L) {        // rows of c2, columns of c1: U21 Y21^T
                const Mat P = mul(F->U21[size_t(id)], [&] {
                    Mat T(F->Y21[size_t(id)].c, m1);
                    for (int64_t x = 0; x < m1; ++x)
                        for (int64_t q = 0; q < T.r; ++q) T(q, x) = F->Y21[size_t(id)](x, q);
                    return T;
                }());
                for (int64_t c = 0; c < m1; ++c)
                    for (int64_t i = 0; i < m2; ++i) L[(a + c) * ldl + b + i] = P(i, c);
            }
            if (U) {        // rows of c1, columns of c2: X12 V12^T
                const Mat P = mul(F->X12[size_t(id)], [&] {
                    Mat T(F->V12[size_t(id)].c, m2);
                    for (int64_t x = 0; x < m2; ++x)
                        for (int64_t q = 0; q < T.r; ++q) T(q, x) = F->V12[size_t(id)](x, q);
                    return T;
                }());
                for (int64_t c = 0; c < m2; ++c)
                    for (int64_t i = 0; i < m1; ++i) U[(b + c) * ldu + a + i] = P(i, c);
            }
        }
    return host_fail(HODLR_OK, "");
}

extern "C" hodlr_status hodlr_solve(hodlr_op op, const void* B, int64_t ldb, void* X, int64_t ldx, int32_t nrhs,
                                    int32_t xy_dtype, hipStream_t stream) {
    if (!op) return host_fail(HODLR_E_ARG, "op is NULL");
    Factors* F = static_cast<Factors*>(get_lu(op));
    if (!F) return host_fail(HODLR_E_STATE, "no LU factors: call hodlr_lu first");
    if (F->device < 0 || !F->linv) return host_fail(HODLR_E_STATE, "host-only handle: no solve");
    if (nrhs < 1) return host_fail(HODLR_E_ARG, "nrhs must be >= 1");
    if (xy_dtype != HODLR_FP64 && xy_dtype != HODLR_FP32)
        return host_fail(HODLR_E_UNSUPPORTED, "hodlr_solve takes HODLR_FP64 or HODLR_FP32 B and X");
    if (!B || !X) return host_fail(HODLR_E_ARG, "B or X is NULL");
    if (ldb < F->n || ldx < F->n) return host_fail(HODLR_E_ARG, "ldb and ldx must be >= n");
    hipError_t e = hipSetDevice(F->device);
    if (e != hipSuccess) return host_fail(HODLR_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(F->mu);
    const int64_t need = 2 * F->n * int64_t(nrhs);
    if (need > F->ws_doubles) {
        if (F->d_ws) {                       // earlier solves may still read it
            (void)hipDeviceSynchronize();
            (void)hipFree(F->d_ws);
            F->d_ws = nullptr;
            F->ws_doubles = 0;
        }
        void* p = nullptr;
        if (hipMalloc(&p, size_t(need) * 8) != hipSuccess) {
            (void)hipGetLastError();
            return host_fail(HODLR_E_NOMEM, "solve workspace");
        }
        F->d_ws = static_cast<double*>(p);
        F->ws_doubles = need;
    }
    // Z = L^-1 B and X = U^-1 Z in fp64 (fp32 B widened first, X rounded once at the end)
    double* W0 = F->d_ws;
    double* W1 = F->d_ws + F->n * nrhs;
    const bool f64 = xy_dtype == HODLR_FP64;
    hodlr_status r;
    if (f64) {
        r = hodlr_matvec(F->linv, B, ldb, W0, F->n, nrhs, HODLR_FP64, stream);
        if (r == HODLR_OK) r = hodlr_matvec(F->uinv, W0, F->n, X, ldx, nrhs, HODLR_FP64, stream);
    } else {
        int he = launch_lu_convert(B, ldb, false, W1, F->n, true, F->n, nrhs, static_cast<void*>(stream));
        if (he != 0) return host_fail(HODLR_E_DEVICE, std::string("solve: ") + hipGetErrorString(hipError_t(he)));
        r = hodlr_matvec(F->linv, W1, F->n, W0, F->n, nrhs, HODLR_FP64, stream);
        if (r == HODLR_OK) r = hodlr_matvec(F->uinv, W0, F->n, W1, F->n, nrhs, HODLR_FP64, stream);
        if (r == HODLR_OK) {
            he = launch_lu_convert(W1, F->n, true, X, ldx, false, F->n, nrhs, static_cast<void*>(stream));
            if (he != 0) return host_fail(HODLR_E_DEVICE, std::string("solve: ") + hipGetErrorString(hipError_t(he)));
        }
    }
    if (r != HODLR_OK) return host_fail(r, std::string("solve: ") + hodlr_last_error_message());
    return host_fail(HODLR_OK, "");
}
