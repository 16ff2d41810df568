// Construction of an eps-HODLR operator from a kernel matrix on the GPU
// (hodlr_build_kernel).
//
// Method: Carson, Chen, Liu, "Mixed Precision HODLR Matrices"
// (arXiv 2407.21637), Sect. 2-3: every off-diagonal block B of the tree is
// replaced by a truncated SVD U V^T with orthonormal U (eq. (3.1)) and the
// smallest rank p that keeps ||B - U V^T||_F <= eps ||B||_F (the Frobenius
// reading of Def. 2.2, which makes Lemma 2.4 hold); the squared norms
// ||A||_F^2 and ||A_b||_F^2 of the original matrix that the adaptive rule
// needs (Alg. "Adaptive-precision HODLR Format") are computed exactly.
//
// The truncated SVD is a randomised one (Halko, Martinsson, Tropp, SIAM
// Rev. 53 (2011)), all blocks of a level at once:
//   1. Y = B Omega (Omega c x s Gaussian), B evaluated on the fly;
//   2. the range of Y: Y^T Y is accumulated in double-double on the
//      device and eigen-decomposed in long double on the host; the k
//      directions with sigma_i > 1e-9 sigma_1 give Q0 = Y V_k Lambda_k^-1/2,
//      whose columns are close to orthonormal, and two Cholesky QR passes
//      make Q exactly so (Cholesky QR alone fails on the numerically
//      rank-deficient Y of a sketch wider than the block's rank);
//   3. M^T = B^T Q, B evaluated again; the residual ||B - Q M||_F^2 is
//      ||B||_F^2 - ||M||_F^2 (Q orthonormal), or computed exactly in a third
//      pass when eps < 1e-6 (where that difference would lose the digits
//      the rule needs);
//   4. M M^T = Z diag(mu) Z^T (the Gram of M^T in double-double, eigen in
//      long double): the singular values of M are sqrt(mu_i);
//   5. p = the smallest rank with sum_{i>p} mu_i + residual <= eps^2
//      ||B||_F^2; U = Q Z_p, V = M^T Z_p (= B^T U).
// A block whose rule is not met with p + 8 <= s (oversampling) goes round
// again with twice the sketch, up to kMaxSketch columns or min(r, c), or
// until Y has at least 8 fewer significant directions than columns (then
// the sketch saw the block's whole numerical range).
// The O(n^2 s) passes and the tall-skinny products run in the kernels of
// kernels_build.hip; only the s x s factorizations run here.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hodlr.h"
#include "build_internal.h"
#include "hodlr_internal.h"
#include "host_internal.h"

using namespace hodlr;

namespace {

// Directions of a sketch kept by the range step: sigma_i > kRangeTol sigma_1
// (eigenvalues of its Gram above kRangeTol^2 times the largest; the
// double-double Gram and the long double eigen-solver resolve them).
constexpr long double kRangeTol = 1e-9L;
constexpr long double kRangeTol2 = kRangeTol * kRangeTol;

// ---- small dense linear algebra (column-major, n x n) --------------------

// Upper triangular R with R^T R = G (G symmetric, upper part used);
// false if a pivot is not positive.
bool chol_upper(const std::vector<double>& G, int n, std::vector<double>& R) {
    R.assign(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i <= j; ++i) {
            double s = G[size_t(j) * n + i];
            for (int k = 0; k < i; ++k) s -= R[size_t(i) * n + k] * R[size_t(j) * n + k];
            if (i < j) {
                R[size_t(j) * n + i] = s / R[size_t(i) * n + i];
            } else {
                if (!(s > 0.0)) return false;
                R[size_t(j) * n + j] = std::sqrt(s);
            }
        }
    }
    return true;
}

// Inverse of an upper triangular matrix (column-major).
std::vector<double> inv_upper(const std::vector<double>& R, int n) {
    std::vector<double> X(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        X[size_t(j) * n + j] = 1.0 / R[size_t(j) * n + j];
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += R[size_t(k) * n + i] * X[size_t(j) * n + k];
            X[size_t(j) * n + i] = -s / R[size_t(i) * n + i];
        }
    }
    return X;
}

// ---- device buffers --------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hodlr_status reserve(size_t bytes, const char* what) {
        if (bytes <= cap) return HODLR_OK;
        if (p) {
            (void)hipDeviceSynchronize();             // nothing enqueued may still read the old buffer
            (void)hipFree(p);
        }
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return host_fail(HODLR_E_NOMEM, std::string("construction workspace: ") + what);
        }
        cap = std::max<size_t>(bytes, 256);
        return HODLR_OK;
    }
    double* d() const { return static_cast<double*>(p); }
};

hodlr_status dev_err(int e, const char* what) {
    if (e == 0) return HODLR_OK;
    return host_fail(HODLR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(hipError_t(e)));
}

template <typename T>
hodlr_status upload(DevBuf& b, const std::vector<T>& v, hipStream_t s, const char* what) {
    hodlr_status r = b.reserve(v.size() * sizeof(T), what);
    if (r != HODLR_OK) return r;
    if (v.empty()) return HODLR_OK;
    // waited for: the caller reuses the host vector right away
    r = dev_err(int(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s)), what);
    if (r != HODLR_OK) return r;
    return dev_err(int(hipStreamSynchronize(s)), what);
}

template <typename T>
hodlr_status download(std::vector<T>& v, const DevBuf& b, size_t count, hipStream_t s, const char* what) {
    v.resize(count);
    if (!count) return HODLR_OK;
    hodlr_status r = dev_err(int(hipMemcpyAsync(v.data(), b.p, count * sizeof(T), hipMemcpyDeviceToHost, s)), what);
    if (r != HODLR_OK) return r;
    return dev_err(int(hipStreamSynchronize(s)), what);
}

// Items of a batched panel operation: one per `rows` rows of each panel.
std::vector<BuildItem> panel_items(const std::vector<BuildPanel>& pans, int rows) {
    std::vector<BuildItem> it;
    for (size_t q = 0; q < pans.size(); ++q)
        for (int r = 0; r < pans[q].outer; r += rows) it.push_back(BuildItem{int32_t(q), r});
    return it;
}

struct Ctx {
    BuildKernel K{};
    double* P = nullptr;
    hipStream_t s = nullptr;
    DevBuf pans, items, gram, S;
};

// fn(i) for i in [0, n) on the host's cores
template <typename Fn>
void parallel_for(int n, Fn fn) {
    const int nt = std::max(1, std::min<int>(n, int(std::thread::hardware_concurrency())));
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (int i = next++; i < n; i = next++) fn(i);
        });
    for (auto& x : th) x.join();
}

// Eigen-decomposition G = V diag(lam) V^T of a symmetric n x n matrix
// (column-major) by cyclic Jacobi rotations in long double, eigenvalues
// descending.
void jacobi_eig(std::vector<long double> A, int n, std::vector<long double>& lam, std::vector<long double>& V) {
    V.assign(size_t(n) * n, 0.0L);
    for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0L;
    auto at = [&](int r, int c) -> long double& { return A[size_t(c) * n + r]; };
    for (int sweep = 0; sweep < 80; ++sweep) {
        long double off = 0.0L, diag = 0.0L;
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r) (r == q ? diag : off) += at(r, q) * at(r, q);
        if (off <= 1e-36L * diag || off == 0.0L) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const long double apq = at(p, q);
                if (apq == 0.0L) continue;
                const long double app = at(p, p), aqq = at(q, q);
                const long double theta = (aqq - app) / (2.0L * apq);
                const long double t = (theta >= 0.0L ? 1.0L : -1.0L) / (std::fabs(theta) + std::sqrt(1.0L + theta * theta));
                const long double c = 1.0L / std::sqrt(1.0L + t * t), sn = c * t;
                for (int k = 0; k < n; ++k) {            // columns p, q
                    const long double akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp - sn * akq;
                    at(k, q) = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {            // rows p, q
                    const long double apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk - sn * aqk;
                    at(q, k) = sn * apk + c * aqk;
                }
                at(p, q) = at(q, p) = 0.0L;
                for (int k = 0; k < n; ++k) {
                    const long double vkp = V[size_t(p) * n + k], vkq = V[size_t(q) * n + k];
                    V[size_t(p) * n + k] = c * vkp - sn * vkq;
                    V[size_t(q) * n + k] = sn * vkp + c * vkq;
                }
            }
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return at(x, x) > at(y, y); });
    std::vector<long double> V2(size_t(n) * n);
    lam.assign(n, 0.0L);
    for (int j = 0; j < n; ++j) {
        lam[j] = at(ord[j], ord[j]);
        for (int i = 0; i < n; ++i) V2[size_t(j) * n + i] = V[size_t(ord[j]) * n + i];
    }
    V.swap(V2);
}

// Gram matrices A^T A (s x s, symmetric) of every panel, accumulated in
// double-double on the device and summed over row chunks in long double.
hodlr_status gram_dd(Ctx& c, const std::vector<BuildPanel>& pans, const DevBuf& A,
                     std::vector<std::vector<long double>>& G) {
    const std::vector<BuildItem> gi = panel_items(pans, kGramRows);
    hodlr_status r;
    if ((r = upload(c.pans, pans, c.s, "panels")) != HODLR_OK) return r;
    if ((r = upload(c.items, gi, c.s, "items")) != HODLR_OK) return r;
    if ((r = c.gram.reserve(gi.size() * size_t(kMaxSketch) * kMaxSketch * 16, "Gram")) != HODLR_OK) return r;
    if ((r = dev_err(launch_build_gram(static_cast<BuildPanel*>(c.pans.p), static_cast<BuildItem*>(c.items.p),
                                       int(gi.size()), A.d(), c.gram.d(), c.s), "Gram")) != HODLR_OK)
        return r;
    std::vector<double> part;
    if ((r = download(part, c.gram, gi.size() * size_t(kMaxSketch) * kMaxSketch * 2, c.s, "Gram")) != HODLR_OK)
        return r;
    G.assign(pans.size(), {});
    size_t item = 0;
    for (size_t q = 0; q < pans.size(); ++q) {
        const int s = pans[q].s;
        G[q].assign(size_t(s) * s, 0.0L);
        for (; item < gi.size() && gi[item].panel == int32_t(q); ++item)
            for (int a = 0; a < s; ++a)
                for (int b = a; b < s; ++b) {
                    const size_t o = (item * size_t(kMaxSketch) * kMaxSketch + size_t(a) * s + b) * 2;
                    G[q][size_t(b) * s + a] += (long double)part[o] + (long double)part[o + 1];
                }
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < a; ++b) G[q][size_t(b) * s + a] = G[q][size_t(a) * s + b];
    }
    return HODLR_OK;
}

// C = A S for every panel (A outer x s at o_off; S_q s x p, uploaded here;
// C outer x p at c_off).
hodlr_status small_gemm(Ctx& c, std::vector<BuildPanel> pans, const std::vector<std::vector<double>>& S,
                        const DevBuf& A, DevBuf& Cbuf) {
    std::vector<double> Sh;
    for (size_t q = 0; q < pans.size(); ++q) {
        pans[q].w_off = int64_t(Sh.size());
        Sh.insert(Sh.end(), S[q].begin(), S[q].end());
    }
    const std::vector<BuildItem> mi = panel_items(pans, kBuildRows);
    hodlr_status r;
    if ((r = upload(c.S, Sh, c.s, "small factors")) != HODLR_OK) return r;
    if ((r = upload(c.pans, pans, c.s, "panels")) != HODLR_OK) return r;
    if ((r = upload(c.items, mi, c.s, "items")) != HODLR_OK) return r;
    return dev_err(launch_build_small_gemm(static_cast<BuildPanel*>(c.pans.p), static_cast<BuildItem*>(c.items.p),
                                           int(mi.size()), A.d(), c.S.d(), Cbuf.d(), c.s), "small product");
}

// Two plain Cholesky QR passes on panels whose columns are already close
// to orthonormal: afterwards they are orthonormal to working precision.
// The panels are in A (outer x s at o_off); T is scratch of the same size.
hodlr_status chol_qr2(Ctx& c, std::vector<BuildPanel> pans, DevBuf& A, DevBuf& T) {
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<std::vector<long double>> G;
        hodlr_status r = gram_dd(c, pans, A, G);
        if (r != HODLR_OK) return r;
        std::vector<std::vector<double>> S(pans.size());
        for (size_t q = 0; q < pans.size(); ++q) {
            const int s = pans[q].s;
            std::vector<double> Gd(size_t(s) * s), R;
            for (size_t i = 0; i < Gd.size(); ++i) Gd[i] = double(G[q][i]);
            if (!chol_upper(Gd, s, R))
                return host_fail(HODLR_E_DEVICE, "orthonormalisation: a Gram matrix that should be close to the "
                                                 "identity is not positive definite");
            S[q] = inv_upper(R, s);
            pans[q].p = s;
            pans[q].c_off = pans[q].o_off;
        }
        if ((r = small_gemm(c, pans, S, A, T)) != HODLR_OK) return r;
        std::swap(A.p, T.p);
        std::swap(A.cap, T.cap);
    }
    return HODLR_OK;
}

// ||B - Q M||_F^2 of every panel: Q (rows x s at o_off) in dQ, M^T (cols x s
// at c_off) in dMt, computed tile by tile with B evaluated on the fly.
hodlr_status residuals(Ctx& c, const std::vector<BuildPanel>& pr, const DevBuf& dQ, const DevBuf& dMt,
                       std::vector<double>& res2) {
    const auto it = panel_items(pr, kResidualRows);
    hodlr_status r;
    if ((r = upload(c.pans, pr, c.s, "panels")) != HODLR_OK) return r;
    if ((r = upload(c.items, it, c.s, "items")) != HODLR_OK) return r;
    DevBuf dR;
    if ((r = dR.reserve(it.size() * 8, "residual")) != HODLR_OK) return r;
    if ((r = dev_err(launch_build_residual(c.K, c.P, static_cast<BuildPanel*>(c.pans.p),
                                           static_cast<BuildItem*>(c.items.p), int(it.size()), dQ.d(), dMt.d(), dR.d(),
                                           c.s), "residual")) != HODLR_OK)
        return r;
    std::vector<double> rp;
    if ((r = download(rp, dR, it.size(), c.s, "residual")) != HODLR_OK) return r;
    res2.assign(pr.size(), 0.0);
    for (size_t t = 0; t < it.size(); ++t) res2[size_t(it[t].panel)] += rp[t];
    return HODLR_OK;
}

double elapsed_ms(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" hodlr_status hodlr_build_kernel(hodlr_op* out, int64_t n, int32_t depth, const double* points,
                                           const hodlr_kernel* kernel, double eps, uint64_t seed, int32_t device,
                                           hodlr_build_report* report) {
    if (!out) return host_fail(HODLR_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || depth < 0 || depth > 24) return host_fail(HODLR_E_ARG, "need n >= 1 and 0 <= depth <= 24");
    if (!points || !kernel) return host_fail(HODLR_E_ARG, "points or kernel is NULL");
    if (kernel->dim != 1 && kernel->dim != 2) return host_fail(HODLR_E_ARG, "kernel dim must be 1 or 2");
    if (kernel->kind < HODLR_KERNEL_GAUSSIAN || kernel->kind > HODLR_KERNEL_SIGNED_INV)
        return host_fail(HODLR_E_ARG, "unknown kernel kind");
    if (kernel->kind == HODLR_KERNEL_SIGNED_INV && (kernel->dim != 1 || !kernel->diag_given))
        return host_fail(HODLR_E_ARG, "the signed inverse kernel is 1D and needs diag_given");
    if (kernel->kind == HODLR_KERNEL_GAUSSIAN && !(kernel->a > 0.0))
        return host_fail(HODLR_E_ARG, "the Gaussian kernel needs a > 0");
    if (!(eps > 0.0 && eps < 1.0)) return host_fail(HODLR_E_ARG, "eps must lie in (0, 1)");
    if (device < 0) return host_fail(HODLR_E_ARG, "construction runs on a GPU: device must be >= 0");
    const auto t_all = std::chrono::steady_clock::now();
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return dev_err(int(e), "hipSetDevice");
    // tree and blocks (Def. 2.1, eq. (2.1))
    const int nleaves = 1 << depth, nb = (1 << (depth + 1)) - 2;
    std::vector<int64_t> bounds((size_t(1) << (depth + 1)) + depth), desc(size_t(std::max(nb, 1)) * 5);
    hodlr_status r = hodlr_tree_bounds(n, depth, nullptr, bounds.data());
    if (r == HODLR_OK && nb > 0) r = hodlr_tree_blocks(n, depth, nullptr, desc.data());
    if (r != HODLR_OK) return r;
    const int64_t* lb = bounds.data() + ((int64_t(1) << depth) - 1) + depth;

    Ctx c;
    c.K.kind = kernel->kind;
    c.K.dim = kernel->dim;
    c.K.a = kernel->a;
    c.K.diag_shift = kernel->diag_shift;
    c.K.diag_value = kernel->diag_value;
    c.K.diag_given = kernel->diag_given ? 1 : 0;
    struct StreamGuard {
        hipStream_t s = nullptr;
        ~StreamGuard() {
            if (s) (void)hipStreamDestroy(s);
        }
    } sg;
    if ((e = hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking)) != hipSuccess) return dev_err(int(e), "stream");
    c.s = sg.s;
    DevBuf dP;
    if ((r = upload(dP, std::vector<double>(points, points + n * kernel->dim), c.s, "points")) != HODLR_OK) return r;
    c.P = dP.d();

    // ---- squared norms of the leaves and blocks, tile by tile --------------
    const auto t_norms = std::chrono::steady_clock::now();
    std::vector<BuildTile> tiles;
    std::vector<int32_t> owner;                       // 0..nleaves-1 leaves, then nleaves + b
    auto add_tiles = [&](int64_t r0, int64_t nr, int64_t c0, int64_t nc, int32_t who) {
        const int64_t tr = 512, tc = 2048;
        for (int64_t a = 0; a < nr; a += tr)
            for (int64_t b = 0; b < nc; b += tc) {
                tiles.push_back(BuildTile{r0 + a, c0 + b, int32_t(std::min(tr, nr - a)), int32_t(std::min(tc, nc - b)), 0});
                owner.push_back(who);
            }
    };
    for (int i = 0; i < nleaves; ++i) add_tiles(lb[i], lb[i + 1] - lb[i], lb[i], lb[i + 1] - lb[i], i);
    for (int b = 0; b < nb; ++b) add_tiles(desc[size_t(b) * 5 + 1], desc[size_t(b) * 5 + 2], desc[size_t(b) * 5 + 3],
                                           desc[size_t(b) * 5 + 4], nleaves + b);
    DevBuf dT, dO;
    if ((r = upload(dT, tiles, c.s, "tiles")) != HODLR_OK) return r;
    if ((r = dO.reserve(tiles.size() * 8, "norm partials")) != HODLR_OK) return r;
    if ((r = dev_err(launch_build_norms(c.K, c.P, static_cast<BuildTile*>(dT.p), int(tiles.size()), dO.d(), c.s),
                     "norms")) != HODLR_OK)
        return r;
    std::vector<double> part;
    if ((r = download(part, dO, tiles.size(), c.s, "norms")) != HODLR_OK) return r;
    std::vector<double> nrm(size_t(nleaves + nb), 0.0);
    for (size_t t = 0; t < tiles.size(); ++t) nrm[size_t(owner[t])] += part[t];
    double norm2_all = 0.0;
    for (double v : nrm) norm2_all += v;
    // leaves
    std::vector<BuildTile> lt(nleaves);
    int64_t dtot = 0;
    for (int i = 0; i < nleaves; ++i) {
        const int64_t m = lb[i + 1] - lb[i];
        lt[i] = BuildTile{lb[i], lb[i], int32_t(m), int32_t(m), dtot};
        dtot += m * m;
    }
    DevBuf dL, dD;
    if ((r = upload(dL, lt, c.s, "leaf tiles")) != HODLR_OK) return r;
    if ((r = dD.reserve(size_t(std::max<int64_t>(dtot, 1)) * 8, "leaves")) != HODLR_OK) return r;
    if ((r = dev_err(launch_build_leaves(c.K, c.P, static_cast<BuildTile*>(dL.p), nleaves, dD.d(), c.s), "leaves")) !=
        HODLR_OK)
        return r;
    std::vector<double> Dall;
    if ((r = download(Dall, dD, size_t(dtot), c.s, "leaves")) != HODLR_OK) return r;
    const double ms_norms = elapsed_ms(t_norms);

    // ---- truncated SVD of every block, level by level ----------------------
    const auto t_fac = std::chrono::steady_clock::now();
    const bool exact_res = eps < 1e-6;
    std::vector<std::vector<double>> U(static_cast<size_t>(nb)), V(static_cast<size_t>(nb));
    std::vector<int32_t> rank(size_t(nb), 0);
    int rounds = 0, max_sketch = 0;
    DevBuf dW, dY, dY2, dM;
    for (int k = 1; k <= depth; ++k) {
        std::vector<int> pending;
        std::vector<int> sk(size_t(nb), 0);
        for (int j = 0; j < (1 << k); ++j) {
            const int b = (1 << k) - 2 + j;
            const int64_t rr = desc[size_t(b) * 5 + 2], cc = desc[size_t(b) * 5 + 4];
            const double nb2 = nrm[size_t(nleaves + b)];
            if (rr == 0 || cc == 0 || nb2 == 0.0) continue;    // rank 0
            pending.push_back(b);
            sk[size_t(b)] = int(std::min<int64_t>({rr, cc, 32}));      // never wider than the block
        }
        while (!pending.empty()) {
            ++rounds;
            // panels: Omega (cols x s), Y = B Omega (outer = rows), M^T = B^T Q (outer = cols)
            std::vector<BuildPanel> py, pm;
            int64_t wy = 0, wm = 0;
            for (int b : pending) {
                const int64_t rr = desc[size_t(b) * 5 + 2], cc = desc[size_t(b) * 5 + 4];
                const int s = sk[size_t(b)];
                max_sketch = std::max(max_sketch, s);
                BuildPanel a{};
                a.r0 = desc[size_t(b) * 5 + 1];
                a.c0 = desc[size_t(b) * 5 + 3];
                a.outer = int32_t(rr);
                a.inner = int32_t(cc);
                a.s = s;
                a.p = s;
                a.trans = 0;
                a.block = b + int32_t(nb) * rounds;
                a.w_off = wm;                          // Omega in dW (cols x s)
                a.o_off = wy;
                a.c_off = wy;
                py.push_back(a);
                BuildPanel m = a;
                m.outer = int32_t(cc);
                m.inner = int32_t(rr);
                m.trans = 1;
                m.w_off = wy;                          // Q in dY
                m.o_off = wm;
                m.c_off = wm;
                pm.push_back(m);
                wy += rr * s;
                wm += cc * s;
            }
            if ((r = dW.reserve(size_t(wm) * 8, "Omega")) != HODLR_OK) return r;
            if ((r = dY.reserve(size_t(wy) * 8, "Y")) != HODLR_OK) return r;
            if ((r = dY2.reserve(size_t(wy) * 8, "Y")) != HODLR_OK) return r;
            if ((r = dM.reserve(size_t(wm) * 8, "M")) != HODLR_OK) return r;
            // 1. Y = B Omega
            {
                std::vector<BuildPanel> po = pm;
                for (auto& q : po) {
                    q.inner = q.outer;
                    q.w_off = q.o_off;
                }
                if ((r = upload(c.pans, po, c.s, "panels")) != HODLR_OK) return r;
                if ((r = dev_err(launch_build_omega(static_cast<BuildPanel*>(c.pans.p), int(po.size()), seed, dW.d(), c.s),
                                 "Omega")) != HODLR_OK)
                    return r;
                const auto it = panel_items(py, kBuildRows);
                if ((r = upload(c.pans, py, c.s, "panels")) != HODLR_OK) return r;
                if ((r = upload(c.items, it, c.s, "items")) != HODLR_OK) return r;
                if ((r = dev_err(launch_build_apply(c.K, c.P, static_cast<BuildPanel*>(c.pans.p),
                                                    static_cast<BuildItem*>(c.items.p), int(it.size()), dW.d(), dY.d(),
                                                    c.s), "sketch")) != HODLR_OK)
                    return r;
            }
            // 2. the range of Y: its Gram in double-double, the eigenvectors with
            //    sigma_i > kRangeTol sigma_1, Q0 = Y V_k Lambda_k^(-1/2), then two
            //    Cholesky QR passes make Q orthonormal
            std::vector<int> kq(pending.size(), 0);
            {
                std::vector<std::vector<long double>> G;
                if ((r = gram_dd(c, py, dY, G)) != HODLR_OK) return r;
                std::vector<std::vector<double>> S(pending.size());
                parallel_for(int(pending.size()), [&](int q) {
                    const int s = py[size_t(q)].s;
                    std::vector<long double> lam, V;
                    jacobi_eig(G[size_t(q)], s, lam, V);
                    int k = 0;
                    while (k < s && lam[size_t(k)] > kRangeTol2 * lam[0] && lam[size_t(k)] > 0.0L) ++k;
                    kq[size_t(q)] = k;
                    S[size_t(q)].assign(size_t(s) * std::max(k, 1), 0.0);
                    for (int j = 0; j < k; ++j)
                        for (int i = 0; i < s; ++i)
                            S[size_t(q)][size_t(j) * s + i] = double(V[size_t(j) * s + i] / std::sqrt(lam[size_t(j)]));
                });
                std::vector<BuildPanel> pq = py;
                for (size_t q = 0; q < pq.size(); ++q) pq[q].p = std::max(kq[q], 1);
                if ((r = small_gemm(c, pq, S, dY, dY2)) != HODLR_OK) return r;
                std::swap(dY.p, dY2.p);
                std::swap(dY.cap, dY2.cap);
                for (size_t q = 0; q < py.size(); ++q) {
                    py[q].s = py[q].p = std::max(kq[q], 1);
                    pm[q].s = pm[q].p = std::max(kq[q], 1);
                }
                if ((r = chol_qr2(c, py, dY, dY2)) != HODLR_OK) return r;
            }
            // 3. M^T = B^T Q, and the exact residual ||B - Q M||_F^2 when needed
            {
                const auto it = panel_items(pm, kBuildRows);
                if ((r = upload(c.pans, pm, c.s, "panels")) != HODLR_OK) return r;
                if ((r = upload(c.items, it, c.s, "items")) != HODLR_OK) return r;
                if ((r = dev_err(launch_build_apply(c.K, c.P, static_cast<BuildPanel*>(c.pans.p),
                                                    static_cast<BuildItem*>(c.items.p), int(it.size()), dY.d(), dM.d(),
                                                    c.s), "projection")) != HODLR_OK)
                    return r;
            }
            std::vector<double> res2(pending.size(), 0.0);
            if (exact_res) {
                std::vector<BuildPanel> pr = py;       // Q (rows x k at o_off), M^T (cols x k at c_off)
                for (size_t q = 0; q < pr.size(); ++q) pr[q].c_off = pm[q].o_off;
                if ((r = residuals(c, pr, dY, dM, res2)) != HODLR_OK) return r;
            }
            // 4. M M^T = Z diag(mu) Z^T (Gram of M^T in double-double, eigen in long double):
            //    sigma_i^2 = mu_i, U = Q Z_p, V = M^T Z_p (= B^T U)
            std::vector<std::vector<long double>> G2;
            if ((r = gram_dd(c, pm, dM, G2)) != HODLR_OK) return r;
            std::vector<std::vector<long double>> mu(pending.size()), Zs(pending.size());
            std::vector<long double> m2(pending.size(), 0.0L);
            parallel_for(int(pending.size()), [&](int q) {
                const int k = pm[size_t(q)].s;
                for (int i = 0; i < k; ++i) m2[size_t(q)] += G2[size_t(q)][size_t(i) * k + i];
                jacobi_eig(G2[size_t(q)], k, mu[size_t(q)], Zs[size_t(q)]);
            });
            // 5. rank by the rule
            std::vector<int> again, done;
            for (size_t q = 0; q < pending.size(); ++q) {
                const int b = pending[q];
                const int s = sk[size_t(b)], k = pm[q].s;
                const int64_t rr = desc[size_t(b) * 5 + 2], cc = desc[size_t(b) * 5 + 4];
                const long double nb2 = nrm[size_t(nleaves + b)];
                const long double rs = exact_res ? (long double)res2[q] : std::max(0.0L, nb2 - m2[q]);
                const long double thr = (long double)eps * eps * nb2;
                // tail[p] = sum_{i >= p} mu_i + residual
                std::vector<long double> tl(size_t(k) + 1);
                tl[size_t(k)] = rs;
                for (int i = k - 1; i >= 0; --i) tl[size_t(i)] = tl[size_t(i) + 1] + std::max(0.0L, mu[q][size_t(i)]);
                int p = -1;
                for (int i = 0; i <= k; ++i)
                    if (tl[size_t(i)] <= thr) {
                        p = i;
                        break;
                    }
                // the sketch saw the block's whole numerical range if Y had at least 8
                // fewer significant directions than columns, or covered min(r, c)
                const bool whole = k + 8 <= s || int64_t(s) >= std::min(rr, cc);
                if (p >= 0 && (p + 8 <= s || whole || s >= kMaxSketch)) {
                    rank[size_t(b)] = p;
                    done.push_back(int(q));
                    continue;
                }
                if (whole || s >= kMaxSketch) {
                    char msg[320];
                    std::snprintf(msg, sizeof(msg),
                                  "block %d (%lld x %lld): no rank up to %d meets the rule (||B||_F^2 = %.6Le, "
                                  "captured %.6Le, residual %.3Le, limit %.3Le); below eps ~ 1e-8 the range of the "
                                  "sketch is resolved only to about %.0e of its largest singular value",
                                  b, (long long)rr, (long long)cc, k, nb2, m2[q], rs, thr, double(kRangeTol));
                    return host_fail(HODLR_E_UNSUPPORTED, msg);
                }
                sk[size_t(b)] = int(std::min<int64_t>({int64_t(2) * s, int64_t(kMaxSketch), rr, cc}));
                again.push_back(b);
            }
            // 6. the accepted blocks' factors: U = Q Z_p (rows x p), V = M^T Z_p (cols x p)
            for (int side = 0; side < 2; ++side) {
                std::vector<BuildPanel> pp;
                std::vector<std::vector<double>> S;
                std::vector<int> who;
                int64_t tot = 0;
                for (int q : done) {
                    const int b = pending[size_t(q)];
                    const int p = rank[size_t(b)];
                    if (p == 0) continue;
                    BuildPanel x = side == 0 ? py[size_t(q)] : pm[size_t(q)];
                    const int k = x.s;
                    x.p = p;
                    x.c_off = tot;
                    tot += int64_t(x.outer) * p;
                    std::vector<double> z(size_t(k) * p);
                    for (int j = 0; j < p; ++j)
                        for (int i = 0; i < k; ++i) z[size_t(j) * k + i] = double(Zs[size_t(q)][size_t(j) * k + i]);
                    S.push_back(std::move(z));
                    pp.push_back(x);
                    who.push_back(b);
                }
                if (pp.empty()) continue;
                DevBuf dOut;
                if ((r = dOut.reserve(size_t(tot) * 8, "factors")) != HODLR_OK) return r;
                if ((r = small_gemm(c, pp, S, side == 0 ? dY : dM, dOut)) != HODLR_OK) return r;
                std::vector<double> hostf;
                if ((r = download(hostf, dOut, size_t(tot), c.s, "factors")) != HODLR_OK) return r;
                for (size_t i = 0; i < pp.size(); ++i) {
                    const size_t cnt = size_t(pp[i].outer) * pp[i].p;
                    (side == 0 ? U : V)[size_t(who[i])].assign(hostf.begin() + pp[i].c_off,
                                                                  hostf.begin() + pp[i].c_off + cnt);
                }
            }
            pending = again;
        }
    }
    const double ms_fac = elapsed_ms(t_fac);

    // ---- the operator (uniform fp64), with the original matrix's norms -----
    std::vector<const double*> lp(static_cast<size_t>(nleaves));
    std::vector<int64_t> ld(static_cast<size_t>(nleaves));
    for (int i = 0; i < nleaves; ++i) {
        lp[size_t(i)] = Dall.data() + lt[size_t(i)].out;
        ld[size_t(i)] = std::max<int64_t>(1, lt[size_t(i)].nr);
    }
    std::vector<hodlr_lowrank> blk(size_t(std::max(nb, 1)));
    for (int b = 0; b < nb; ++b) {
        blk[size_t(b)].rank = rank[size_t(b)];
        blk[size_t(b)].U = U[size_t(b)].empty() ? nullptr : U[size_t(b)].data();
        blk[size_t(b)].ldu = std::max<int64_t>(1, desc[size_t(b) * 5 + 2]);
        blk[size_t(b)].V = V[size_t(b)].empty() ? nullptr : V[size_t(b)].data();
        blk[size_t(b)].ldv = std::max<int64_t>(1, desc[size_t(b) * 5 + 4]);
    }
    hodlr_op op = nullptr;
    if ((r = hodlr_create(&op, n, depth, nullptr, lp.data(), ld.data(), blk.data(), device)) != HODLR_OK) return r;
    attach_original_norms(op, norm2_all, nrm.data() + nleaves);
    *out = op;
    if (report) {
        report->ms_norms = ms_norms;
        report->ms_factors = ms_fac;
        report->ms_total = elapsed_ms(t_all);
        report->max_rank = rank.empty() ? 0 : *std::max_element(rank.begin(), rank.end());
        report->max_sketch = max_sketch;
        report->sketch_rounds = rounds;
        report->exact_residual = exact_res ? 1 : 0;
    }
    return host_fail(HODLR_OK, "");
}
