// Host core of the HODLR library: cluster tree, storage-format codecs,
// adaptive precision assignment, packing of the device image and the C ABI.
//
// Method: Carson, Chen, Liu, "Mixed Precision HODLR Matrices"
// (arXiv 2407.21637).  Section references are to that paper.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sys/stat.h>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hodlr.h"
#include "hodlr_internal.h"
#include "host_internal.h"

using namespace hodlr;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_last_error;

hodlr_status fail(hodlr_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

hodlr_status ok() {
    g_last_error.clear();
    return HODLR_OK;
}

// ---------------------------------------------------------------------------
// formats (Table 1.1, plus OCP fp8 E4M3FN)
// ---------------------------------------------------------------------------
struct FmtInfo {
    int t;          // significand bits incl. the implicit one; u = 2^-t
    int emin, emax;
    int ebits, bias;
    double maxf;    // largest finite value
};

const FmtInfo kFmt[NFMT] = {
    {53, -1022, 1023, 11, 1023, DBL_MAX},
    {24, -126, 127, 8, 127, FLT_MAX},
    {8, -126, 127, 8, 127, 0x1.fep127},
    {11, -14, 15, 5, 15, 65504.0},
    {4, -6, 8, 4, 7, 448.0},
    {3, -14, 15, 5, 15, 57344.0},
};

double unit_roundoff(int f) { return std::ldexp(1.0, -kFmt[f].t); }

bool scaled_format(int f) { return f == F16 || f == E4M3 || f == E5M2; }

// Round x (fp64) to format f with round-to-nearest-even, once, and return
// the bit pattern.  Works on the fp64 bit fields: the exact significand is
// shifted right to the target quantum 2^(max(lead, emin) - t + 1) (gradual
// underflow below 2^emin) with the discarded bits deciding the rounding.
// *overflow is set when the rounded value exceeds the largest finite value
// (or x is not finite).
uint64_t encode_rne(double x, int f, bool* overflow) {
    uint64_t bits;
    std::memcpy(&bits, &x, 8);
    if (f == F64) return bits;
    const FmtInfo& F = kFmt[f];
    const int nbits = 8 * fmt_bytes(f);
    const int mbits = F.t - 1;
    const uint64_t sgn = (bits >> 63) << (nbits - 1);
    const int E = int((bits >> 52) & 0x7ff);
    const uint64_t M = bits & ((uint64_t(1) << 52) - 1);
    if (E == 0x7ff) {
        *overflow = true;
        return sgn | (((uint64_t(1) << F.ebits) - 1) << mbits);
    }
    if (E == 0 && M == 0) return sgn;
    uint64_t sig;
    int e2, lead;
    if (E) {
        sig = M | (uint64_t(1) << 52);
        e2 = E - 1075;
        lead = E - 1023;
    } else {
        sig = M;
        e2 = -1074;
        lead = -1074 + (63 - __builtin_clzll(M));
    }
    int q = std::max(lead, F.emin) - mbits;
    const int shift = q - e2;  // >= 0: every target is narrower than fp64
    uint64_t r;
    if (shift >= 64) {
        r = 0;
    } else if (shift == 0) {
        r = sig;
    } else {
        r = sig >> shift;
        const uint64_t rem = sig & ((uint64_t(1) << shift) - 1);
        const uint64_t half = uint64_t(1) << (shift - 1);
        if (rem > half || (rem == half && (r & 1))) ++r;
    }
    if (r == 0) return sgn;
    const uint64_t hidden = uint64_t(1) << mbits;
    if (r >= hidden) {
        if (r == (hidden << 1)) {
            r >>= 1;
            ++q;
        }
        if (std::ldexp(double(r), q) > F.maxf) {
            *overflow = true;
            return sgn | (((uint64_t(1) << F.ebits) - 1) << mbits);
        }
        const uint64_t expf = uint64_t(q + mbits + F.bias);
        return sgn | (expf << mbits) | (r - hidden);
    }
    return sgn | r;  // subnormal: exponent field 0
}

// Largest integer e with amax * 2^e <= maxf (0 for amax == 0), from the
// binary exponents: amax = ma 2^ea, maxf = mf 2^ef with ma, mf in [0.5, 1).
int column_exponent(int f, double amax) {
    if (amax == 0.0) return 0;
    int ea, ef;
    const double ma = std::frexp(amax, &ea);
    const double mf = std::frexp(kFmt[f].maxf, &ef);
    return ef - ea - (ma > mf ? 1 : 0);
}

template <typename Fn>
void parallel_for(int64_t n, Fn fn) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 2 || nt == 1) {
        for (int64_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (int64_t i; (i = next.fetch_add(1)) < n;) fn(i);
        });
    for (auto& x : th) x.join();
}

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// tree (Def. 2.1; left child = ceil(parent / 2) as in Sect. 4)
// ---------------------------------------------------------------------------
// Fills all levels 0..depth, level k at offset (2^k - 1) + k with 2^k + 1
// values.  Returns false on inconsistent leaf bounds.
bool build_bounds(int64_t n, int depth, const int64_t* leaf_bounds, std::vector<int64_t>& out) {
    out.assign((size_t(1) << (depth + 1)) + depth, 0);
    auto lvl = [&](int k) { return out.data() + ((int64_t(1) << k) - 1) + k; };
    if (!leaf_bounds) {
        int64_t* l0 = lvl(0);
        l0[0] = 0;
        l0[1] = n;
        for (int k = 0; k < depth; ++k) {
            const int64_t* p = lvl(k);
            int64_t* c = lvl(k + 1);
            c[0] = 0;
            for (int64_t j = 0; j < (int64_t(1) << k); ++j) {
                const int64_t a = p[j], b = p[j + 1];
                c[2 * j + 1] = a + (b - a + 1) / 2;
                c[2 * j + 2] = b;
            }
        }
        return true;
    }
    const int64_t nl = int64_t(1) << depth;
    if (leaf_bounds[0] != 0 || leaf_bounds[nl] != n) return false;
    for (int64_t i = 0; i < nl; ++i)
        if (leaf_bounds[i] > leaf_bounds[i + 1]) return false;
    for (int k = 0; k <= depth; ++k) {
        const int64_t step = int64_t(1) << (depth - k);
        int64_t* c = lvl(k);
        for (int64_t j = 0; j <= (int64_t(1) << k); ++j) c[j] = leaf_bounds[j * step];
    }
    return true;
}

struct HBlock {
    int level;
    int64_t row0, nrows, col0, ncols;
};

std::vector<HBlock> build_blocks(int depth, const std::vector<int64_t>& bounds) {
    std::vector<HBlock> out;
    for (int k = 1; k <= depth; ++k) {
        const int64_t* b = bounds.data() + ((int64_t(1) << k) - 1) + k;
        for (int64_t j = 0; j < (int64_t(1) << k); ++j) {
            const int64_t c = j ^ 1;
            out.push_back({k, b[j], b[j + 1] - b[j], b[c], b[c + 1] - b[c]});
        }
    }
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
struct Workspace {
    double* partial = nullptr;
    double* T = nullptr;
    void* xpad = nullptr;
    double* W = nullptr;       // leaf products of the wave path
    void* Tw = nullptr;        // T_b in a low working precision
    int32_t* sync = nullptr;   // counters of the fused launch; zeroed once, self-resetting
    int64_t cap_partial = 0, cap_T = 0, cap_xpad = 0, cap_sync = 0, cap_W = 0, cap_Tw = 0;
    uint64_t gen = 0;          // bumped whenever a buffer is replaced (batched plans keep pointers)
    // buffers replaced by larger ones: a graph the caller captured earlier may
    // still name them, so they are freed only by hodlr_destroy
    std::vector<void*> retired;
};

struct hodlr_op_s {
    uint64_t uid = 0;          // unique per handle in this process
    uint64_t gen = 0;          // bumped by every pack (device image replaced)
    int64_t n = 0;
    int depth = 0;
    int nb = 0;
    int nleaves = 0;
    std::vector<int64_t> bounds;
    std::vector<HBlock> blocks;
    std::vector<int32_t> rank;
    std::vector<std::vector<double>> U, V, D;   // fp64, column-major, ld = rows

    // squared norms of the original matrix, when the operator was built from it
    bool have_orig = false;
    double orig_norm2_all = 0.0;
    std::vector<double> orig_norm2;            // per block

    // assignment
    std::vector<int32_t> level_fmt;            // per level k-1
    std::vector<int32_t> block_fmt;            // per block (HODLR_PER_BLOCK); empty: the level's
    std::vector<double> xi, uprime;
    std::vector<int32_t> insufficient;
    double eps = 0.0;
    bool acc_double = true;
    // LU factors of the stored operator (hodlr_lu), owned through lu_free
    void* lu = nullptr;
    void (*lu_free)(void*) = nullptr;
    bool scale_cols = true;

    // padded layout
    std::vector<int64_t> lprow0, lmp;          // per leaf
    int64_t npad = 0;
    bool padded = false;

    // host-side descriptors (mirrors of the device arrays)
    std::vector<BlockDesc> bdesc;
    std::vector<LeafDesc> ldesc;
    std::vector<CItem> citems;
    std::vector<ETile> etiles;
    int64_t fac_bytes = 0;     // device factor buffer size
    int64_t total_rank = 0;    // sum of ranks (T slots)
    int64_t total_rank8 = 0;   // sum of ranks rounded up to 8 (T slots in a low working precision)
    int64_t total_item_rank = 0;
    std::vector<STile> stiles;                 // matrix-core contraction tiles (see stack_tiles)
    std::vector<int32_t> stile_off;            // per leaf, nleaves + 1
    std::vector<SUnit> sunits;                 // contraction units (groups of tiles)
    int64_t total_stack_rank = 0;              // sum over blocks of rank x leaves of the column node
    bool stacked = false;                      // see stack_tiles
    int64_t codes_bytes = 0;   // sum (r+c) p s(f)
    int64_t scaled_cols = 0;
    int32_t max_leaf = 0;
    int32_t max_rank_path = 0;
    int32_t max_tstage = 0;      // see KParams::max_tstage
    int32_t max_block_rank = 0;
    int32_t max_items_rank = 0;

    // device
    int device = -1;
    uint8_t* d_fac = nullptr;
    double* d_leaf = nullptr;
    void* d_aug[2] = {nullptr, nullptr};       // augmented operands in bf16 / fp16 (LeafDesc::aug_off)
    uint64_t aug_gen[2] = {0, 0};              // pack generation each was built for (0: never)
    int64_t aug_total = 0;                     // elements of one augmented image
    int32_t max_kp = 0;
    BlockDesc* d_blocks = nullptr;
    LeafDesc* d_leaves = nullptr;
    CItem* d_citems = nullptr;
    STile* d_stiles = nullptr;
    int32_t* d_stile_off = nullptr;
    SUnit* d_sunits = nullptr;
    ETile* d_etiles = nullptr;
    double* d_tscale = nullptr;
    std::mutex ws_mu;
    std::map<void*, Workspace> ws;             // per stream
    std::mutex aug_mu;                         // builds of d_aug

    // per-phase timing (hodlr_profile)
    std::vector<hipEvent_t> prof_ev;           // 2 * kPhases per record
    std::vector<uint8_t> prof_ran;             // kPhases per record
    int32_t prof_cap = 0, prof_used = 0;
};

namespace {

void drop_lu(hodlr_op_s* op) {
    if (op->lu && op->lu_free) op->lu_free(op->lu);
    op->lu = nullptr;
    op->lu_free = nullptr;
}

int64_t node_of(const hodlr_op_s* op, int k, int64_t j, int64_t* b, int64_t* e) {
    const int64_t* lv = op->bounds.data() + ((int64_t(1) << k) - 1) + k;
    *b = lv[j];
    *e = lv[j + 1];
    return *e - *b;
}

// Padded row range of node j at level k: its leaves are
// [j 2^(depth-k), (j+1) 2^(depth-k)).
void node_padded(const hodlr_op_s* op, int k, int64_t j, int64_t* prow0, int64_t* prows) {
    const int64_t step = int64_t(1) << (op->depth - k);
    const int64_t l0 = j * step, l1 = (j + 1) * step;
    *prow0 = op->lprow0[l0];
    *prows = op->lprow0[l1 - 1] + op->lmp[l1 - 1] - *prow0;
}

void dev_free(void* p) {
    if (p) (void)hipFree(p);
}

void free_profile(hodlr_op_s* op) {
    for (hipEvent_t e : op->prof_ev) (void)hipEventDestroy(e);
    op->prof_ev.clear();
    op->prof_ran.clear();
    op->prof_cap = op->prof_used = 0;
}

void free_device(hodlr_op_s* op) {
    free_profile(op);
    dev_free(op->d_fac);
    dev_free(op->d_leaf);
    dev_free(op->d_aug[0]);
    dev_free(op->d_aug[1]);
    op->d_aug[0] = op->d_aug[1] = nullptr;
    op->aug_gen[0] = op->aug_gen[1] = 0;
    dev_free(op->d_blocks);
    dev_free(op->d_leaves);
    dev_free(op->d_citems);
    dev_free(op->d_stiles);
    dev_free(op->d_stile_off);
    dev_free(op->d_sunits);
    dev_free(op->d_etiles);
    dev_free(op->d_tscale);
    op->d_fac = nullptr;
    op->d_leaf = nullptr;
    op->d_blocks = nullptr;
    op->d_leaves = nullptr;
    op->d_citems = nullptr;
    op->d_stiles = nullptr;
    op->d_stile_off = nullptr;
    op->d_sunits = nullptr;
    op->d_etiles = nullptr;
    op->d_tscale = nullptr;
    for (auto& kv : op->ws) {
        dev_free(kv.second.partial);
        dev_free(kv.second.T);
        dev_free(kv.second.xpad);
        dev_free(kv.second.W);
        dev_free(kv.second.Tw);
        dev_free(kv.second.sync);
        for (void* p : kv.second.retired) dev_free(p);
    }
    op->ws.clear();
}

hodlr_status hip_fail(hipError_t e, const char* what) {
    return fail(HODLR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
hodlr_status upload(T** dst, const T* src, size_t count, const char* what) {
    dev_free(*dst);
    *dst = nullptr;
    if (count == 0) return HODLR_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), count * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        (void)hipGetLastError();
        return fail(HODLR_E_NOMEM, "hipMalloc %s (%zu bytes): %s", what, count * sizeof(T),
                    hipGetErrorString(e));
    }
    e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
    return HODLR_OK;
}

// Rows of a contraction work item: a multiple of 256 (one slab of 64 lanes
// x 4 rows), at least HODLR_ITEM_MIN_ROWS, aiming at HODLR_ITEM_KB of codes,
// at most kItemRowsMax.
int32_t item_rows(int rank, int f) {
    const int64_t per_row = int64_t(rank) * fmt_bytes(f);
    int64_t g = per_row > 0 ? (int64_t(HODLR_ITEM_KB) * 1024) / (256 * per_row) : kItemRowsMax / 256;
    g = std::max<int64_t>(HODLR_ITEM_MIN_ROWS / 256, std::min<int64_t>(kItemRowsMax / 256, g));
    return int32_t(256 * g);
}

// Quantise block b's factor F (rows x p, fp64, ld = rows) in format f;
// write codes at (code_of(i, j)) through `put` and the column exponents.
template <typename Put>
hodlr_status quantize_factor(const std::vector<double>& Fm, int64_t rows, int p, int f,
                             bool scale, int32_t* exps, Put put) {
    for (int j = 0; j < p; ++j) {
        const double* col = Fm.data() + int64_t(j) * rows;
        int e = 0;
        if (scale && scaled_format(f)) {
            double amax = 0.0;
            for (int64_t i = 0; i < rows; ++i) amax = std::max(amax, std::fabs(col[i]));
            e = column_exponent(f, amax);
            if (e < -128 || e > 127)
                return fail(HODLR_E_RANGE, "column scale exponent %d out of int8 range", e);
        }
        exps[j] = e;
        bool ovf = false;
        for (int64_t i = 0; i < rows; ++i) put(i, j, encode_rne(std::ldexp(col[i], e), f, &ovf));
        if (ovf)
            return fail(HODLR_E_RANGE, "a factor value overflows the storage format (column %d)", j);
    }
    return HODLR_OK;
}

void put_code(uint8_t* dst, int f, uint64_t code) {
    switch (fmt_bytes(f)) {
        case 8: std::memcpy(dst, &code, 8); break;
        case 4: { uint32_t c = uint32_t(code); std::memcpy(dst, &c, 4); } break;
        case 2: { uint16_t c = uint16_t(code); std::memcpy(dst, &c, 2); } break;
        default: *dst = uint8_t(code); break;
    }
}

// Where row r (unpadded, relative to the node's first index) of a factor
// panel lives.  A panel of node j at level k is cut into row chunks and each
// chunk is stored column-major on its own (chunk-contiguous layout), so that
// every work item streams one contiguous piece: U panels are cut at the
// expansion tiles of the node's leaves, V panels at the contraction items
// (every item_rows rows).  Element (r, col) of a rank-p panel is at
// chunk_start * p + col * chunk_rows + row_in_chunk.
struct RowLoc {
    int64_t cs;     // chunk start (padded rows, node-relative)
    int32_t ch;     // chunk rows
    int32_t in;     // row within the chunk
};

int64_t loc_index(const RowLoc& L, int64_t col, int64_t p) { return L.cs * p + col * L.ch + L.in; }

// chunk_rows = 0: chunks are the expansion tiles; else fixed chunks of that
// many rows (the last one shorter).
void node_rowlocs(const hodlr_op_s* op, int k, int64_t j, int64_t chunk_rows, std::vector<RowLoc>& out) {
    int64_t b, e;
    node_of(op, k, j, &b, &e);
    out.resize(size_t(e - b));
    const int64_t step = int64_t(1) << (op->depth - k);
    const int64_t p0 = op->lprow0[j * step];
    const int64_t l1 = (j + 1) * step;
    const int64_t rows = op->lprow0[l1 - 1] + op->lmp[l1 - 1] - p0;
    const int64_t* lb = op->bounds.data() + ((int64_t(1) << op->depth) - 1) + op->depth;
    int64_t idx = 0;
    for (int64_t l = j * step; l < l1; ++l) {
        const int64_t m = lb[l + 1] - lb[l];
        const int64_t lrel = op->lprow0[l] - p0;
        for (int64_t r = 0; r < m; ++r) {
            RowLoc L;
            const int64_t pr = lrel + r;
            if (chunk_rows == 0) {
                const int64_t t0 = (r / kTileRows) * kTileRows;
                L.cs = lrel + t0;
                L.ch = int32_t(std::min<int64_t>(kTileRows, op->lmp[l] - t0));
            } else {
                L.cs = (pr / chunk_rows) * chunk_rows;
                L.ch = int32_t(std::min<int64_t>(chunk_rows, rows - L.cs));
            }
            L.in = int32_t(pr - L.cs);
            out[size_t(idx++)] = L;
        }
    }
}

// Tiles of the matrix-core contraction (STile): for every leaf, the ranks
// of the depth blocks whose V panels cover its rows (level k: the block
// whose column node holds the leaf), grouped by arithmetic type and code
// format, 16 to a tile; and, per block, where its per-leaf partials go.
// Which other rows share a row's tile does not change that row's sums.
void stack_tiles(hodlr_op_s* op) {
    const int depth = op->depth, nl = op->nleaves;
    int64_t soff = 0;
    for (int b = 0; b < op->nb; ++b) {
        BlockDesc& d = op->bdesc[size_t(b)];
        const int k = d.level;
        const int64_t jrow = b - ((int64_t(1) << k) - 2);
        d.sleaves = int32_t(int64_t(1) << (depth - k));
        d.sleaf0 = int32_t((jrow ^ 1) << (depth - k));
        d.s_off = soff;
        soff += int64_t(d.rank) * d.sleaves;
    }
    op->total_stack_rank = soff;
    op->stiles.clear();
    op->stile_off.assign(size_t(nl) + 1, 0);
    for (int i = 0; i < nl; ++i) {
        op->stile_off[size_t(i)] = int32_t(op->stiles.size());
        // (arithmetic type, format) -> its rows, levels in order
        std::map<std::pair<int, int>, std::vector<std::pair<int32_t, int32_t>>> groups;
        for (int k = 1; k <= depth; ++k) {
            const int b = ((1 << k) - 2) + ((i >> (depth - k)) ^ 1);
            const BlockDesc& d = op->bdesc[size_t(b)];
            const int dbl = (op->acc_double || d.fmt == F64) ? 1 : 0;
            auto& rows = groups[{-dbl, d.fmt}];              // fp64 tiles first
            for (int j = 0; j < d.rank; ++j) rows.push_back({b, j});
        }
        for (const auto& g : groups) {
            const auto& rows = g.second;
            for (size_t r0 = 0; r0 < rows.size(); r0 += kStackRows) {
                STile t{};
                t.fmt = g.first.second;
                t.dbl = -g.first.first;
                t.n = int32_t(std::min<size_t>(kStackRows, rows.size() - r0));
                for (int q = 0; q < kStackRows; ++q) {
                    const auto& rw = rows[r0 + (q < t.n ? size_t(q) : 0)];
                    t.blk[q] = rw.first;
                    t.j[q] = rw.second;
                }
                op->stiles.push_back(t);
            }
        }
    }
    op->stile_off[size_t(nl)] = int32_t(op->stiles.size());
    // units: consecutive tiles of a leaf with one format and arithmetic type, up to 2 (fp64) or 4
    op->sunits.clear();
    for (int i = 0; i < nl; ++i) {
        const int t1 = op->stile_off[size_t(i) + 1];
        for (int t = op->stile_off[size_t(i)]; t < t1;) {
            const STile& a = op->stiles[size_t(t)];
            const int cap = a.dbl ? 2 : 4;
            int ng = 1;
            while (ng < cap && t + ng < t1 && op->stiles[size_t(t + ng)].fmt == a.fmt &&
                   op->stiles[size_t(t + ng)].dbl == a.dbl)
                ++ng;
            op->sunits.push_back(SUnit{i, t, ng, 0});
            t += ng;
        }
    }
    // The stacked contraction reads X once per leaf only when each leaf is
    // one unit (one pass); with more passes the per-level items, whose long
    // runs of rows keep more loads in flight, are faster (measured on the
    // 512-operator batch), so they are used instead.
    op->stacked = !op->sunits.empty() && op->sunits.size() == size_t(nl);
}

// Build descriptors, quantise every factor into a host staging image and
// (for device handles) upload it.  Called after create and after every
// precision change.
hodlr_status pack(hodlr_op_s* op) {
    ++op->gen;
    const int nb = op->nb;
    op->bdesc.assign(nb, BlockDesc{});
    op->citems.clear();
    int64_t off = 0, toff = 0, poff = 0, twoff = 0;
    op->codes_bytes = 0;
    op->scaled_cols = 0;
    std::vector<int64_t> ts_off(nb);
    int64_t ts_total = 0;
    for (int b = 0; b < nb; ++b) {
        const HBlock& hb = op->blocks[b];
        const int k = hb.level;
        const int64_t j = b - ((int64_t(1) << k) - 2);
        BlockDesc& d = op->bdesc[b];
        const int f = op->block_fmt.empty() ? op->level_fmt[k - 1] : op->block_fmt[b];
        const int p = op->rank[b];
        int64_t up0, upr, vp0, vpr;
        node_padded(op, k, j, &up0, &upr);
        node_padded(op, k, j ^ 1, &vp0, &vpr);
        d.rank = p;
        d.fmt = f;
        d.level = k;
        d.urow0 = int32_t(up0);
        d.urows = int32_t(upr);
        d.vrow0 = int32_t(vp0);
        d.vrows = int32_t(vpr);
        d.u_off = off;
        off = align_up(off + upr * p * fmt_bytes(f), kPanelAlign);
        d.v_off = off;
        off = align_up(off + vpr * p * fmt_bytes(f), kPanelAlign);
        d.t_off = toff;
        toff += p;
        d.tw_off = twoff;
        twoff += (p + 7) / 8 * 8;
        d.ts_off = ts_total;
        ts_off[b] = ts_total;
        ts_total += p;
        d.item0 = int32_t(op->citems.size());
        d.pad_ = p > 0 ? item_rows(p, f) : 0;     // V chunk rows (contraction item rows)
        if (p > 0) {
            const int32_t ch = d.pad_;
            for (int64_t r = 0; r < vpr; r += ch) {
                CItem it{};
                it.block = b;
                it.r0 = int32_t(r);
                it.nr = int32_t(std::min<int64_t>(ch, vpr - r));
                it.poff = poff;
                poff += p;
                op->citems.push_back(it);
            }
        }
        d.nitems = int32_t(op->citems.size()) - d.item0;
        op->codes_bytes += (hb.nrows + hb.ncols) * p * fmt_bytes(f);
        if (op->scale_cols && scaled_format(f)) op->scaled_cols += 2 * p;
    }
    stack_tiles(op);
    op->fac_bytes = std::max<int64_t>(off, kPanelAlign);
    op->total_rank = toff;
    op->total_rank8 = twoff;
    op->total_item_rank = poff;
    op->max_items_rank = 0;
    for (int b = 0; b < nb; ++b)
        op->max_items_rank = std::max(op->max_items_rank, op->bdesc[b].nitems * op->bdesc[b].rank);
    op->max_rank_path = 0;
    for (int i = 0; i < op->nleaves; ++i) {
        int32_t sum = 0;
        for (int k = 1; k <= op->depth; ++k) sum += op->rank[((1 << k) - 2) + (i >> (op->depth - k))];
        op->max_rank_path = std::max(op->max_rank_path, sum);
    }
    op->max_block_rank = 0;
    for (int b = 0; b < nb; ++b) op->max_block_rank = std::max(op->max_block_rank, op->rank[b]);
    op->max_tstage = 0;
    for (int i = 0; i < op->nleaves; ++i) {
        int32_t bytes = 0;
        for (int k = 1; k <= op->depth; ++k) {
            const int b = ((1 << k) - 2) + (i >> (op->depth - k));
            const int32_t w = (op->acc_double || op->bdesc[b].fmt == F64) ? 8 : 4;
            bytes += ((op->rank[b] + 3) / 4) * 4 * w;
        }
        op->max_tstage = std::max(op->max_tstage, bytes);
    }

    std::vector<uint8_t> img;
    try {
        img.assign(size_t(op->fac_bytes), 0);
    } catch (const std::bad_alloc&) {
        return fail(HODLR_E_NOMEM, "host staging image of %lld bytes", (long long)op->fac_bytes);
    }
    std::vector<double> tscale(size_t(std::max<int64_t>(ts_total, 1)), 1.0);
    std::vector<hodlr_status> st(nb, HODLR_OK);
    std::vector<std::string> msg(nb);
    parallel_for(nb, [&](int64_t b) {
        const HBlock& hb = op->blocks[b];
        const BlockDesc& d = op->bdesc[b];
        const int p = d.rank;
        if (p == 0) return;
        const int k = hb.level;
        const int64_t j = b - ((int64_t(1) << k) - 2);
        const int f = d.fmt;
        const int s = fmt_bytes(f);
        std::vector<RowLoc> umap, vmap;
        node_rowlocs(op, k, j, 0, umap);
        node_rowlocs(op, k, j ^ 1, d.pad_, vmap);
        std::vector<int32_t> eu(p), ev(p);
        uint8_t* ub = img.data() + d.u_off;
        uint8_t* vb = img.data() + d.v_off;
        hodlr_status r = quantize_factor(op->U[b], hb.nrows, p, f, op->scale_cols, eu.data(),
                                         [&](int64_t i, int jj, uint64_t c) {
                                             put_code(ub + loc_index(umap[i], jj, p) * s, f, c);
                                         });
        if (r == HODLR_OK)
            r = quantize_factor(op->V[b], hb.ncols, p, f, op->scale_cols, ev.data(),
                                [&](int64_t i, int jj, uint64_t c) {
                                    put_code(vb + loc_index(vmap[i], jj, p) * s, f, c);
                                });
        if (r != HODLR_OK) {
            st[b] = r;
            msg[b] = g_last_error;
            return;
        }
        // e4m3 codes are decoded through fp16 at 2^-8 of their value
        const int comp = (f == E4M3) ? 16 : 0;
        for (int jj = 0; jj < p; ++jj)
            tscale[size_t(ts_off[b] + jj)] = std::ldexp(1.0, comp - eu[jj] - ev[jj]);
    });
    for (int b = 0; b < nb; ++b)
        if (st[b] != HODLR_OK) return fail(st[b], "%s", msg[b].c_str());

    if (op->device < 0) return HODLR_OK;
    hipError_t e = hipSetDevice(op->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hodlr_status r;
    if ((r = upload(&op->d_fac, img.data(), img.size(), "factor image")) != HODLR_OK) return r;
    if ((r = upload(&op->d_blocks, op->bdesc.data(), op->bdesc.size(), "block table")) != HODLR_OK)
        return r;
    if ((r = upload(&op->d_citems, op->citems.data(), op->citems.size(), "work items")) != HODLR_OK)
        return r;
    if ((r = upload(&op->d_stiles, op->stiles.data(), op->stiles.size(), "contraction tiles")) != HODLR_OK)
        return r;
    if ((r = upload(&op->d_stile_off, op->stile_off.data(), op->stile_off.size(), "contraction tiles")) != HODLR_OK)
        return r;
    if ((r = upload(&op->d_sunits, op->sunits.data(), op->sunits.size(), "contraction units")) != HODLR_OK)
        return r;
    if ((r = upload(&op->d_tscale, tscale.data(), tscale.size(), "column scales")) != HODLR_OK)
        return r;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "upload");
    return HODLR_OK;
}

// Leaves and tiles: once per operator.
hodlr_status pack_leaves(hodlr_op_s* op) {
    const int nl = op->nleaves;
    const int64_t* lb = op->bounds.data() + ((int64_t(1) << op->depth) - 1) + op->depth;
    op->lprow0.assign(nl, 0);
    op->lmp.assign(nl, 0);
    int64_t pr = 0;
    op->padded = false;
    for (int i = 0; i < nl; ++i) {
        const int64_t m = lb[i + 1] - lb[i];
        op->lprow0[i] = pr;
        op->lmp[i] = align_up(m, kRowAlign);
        if (op->lmp[i] != m) op->padded = true;
        pr += op->lmp[i];
    }
    op->npad = pr;
    op->max_leaf = 0;
    for (int i = 0; i < nl; ++i) op->max_leaf = std::max<int32_t>(op->max_leaf, int32_t(lb[i + 1] - lb[i]));
    if (op->npad >= (int64_t(1) << 31))
        return fail(HODLR_E_UNSUPPORTED, "padded size %lld exceeds 2^31 rows", (long long)pr);
    op->ldesc.assign(nl, LeafDesc{});
    op->etiles.clear();
    int64_t doff = 0, aug = 0;
    op->max_kp = 0;
    for (int i = 0; i < nl; ++i) {
        LeafDesc& L = op->ldesc[i];
        L.d_off = doff;
        L.row0 = lb[i];
        L.m = int32_t(lb[i + 1] - lb[i]);
        L.mp = int32_t(op->lmp[i]);
        L.prow0 = int32_t(op->lprow0[i]);
        doff += int64_t(L.mp) * L.mp;
        // low working precision: the ancestors' ranks, each rounded up to 8, then the sum up to 32
        int32_t kpl = 0;
        for (int k = 1; k <= op->depth; ++k) kpl += (op->rank[size_t(((1 << k) - 2) + (i >> (op->depth - k)))] + 7) / 8 * 8;
        L.kp = (kpl + 31) / 32 * 32;
        L.aug_off = aug;
        aug += int64_t(L.mp) * ((L.mp + 31) / 32 * 32 + L.kp);
        op->max_kp = std::max(op->max_kp, L.kp);
        for (int32_t r = 0; r < L.mp; r += kTileRows) {
            ETile t{};
            t.leaf = i;
            t.r0 = r;
            t.nr = std::min<int32_t>(kTileRows, L.mp - r);
            op->etiles.push_back(t);
        }
    }
    op->aug_total = aug;
    if (op->device < 0) return HODLR_OK;
    std::vector<double> img;
    try {
        img.assign(size_t(std::max<int64_t>(doff, 1)), 0.0);
    } catch (const std::bad_alloc&) {
        return fail(HODLR_E_NOMEM, "host staging of leaves");
    }
    // leaf i is cut at its expansion tiles; tile rows [r0, r0+nr) are stored
    // column-major (ld = nr) at d_off + r0 * mp
    parallel_for(nl, [&](int64_t i) {
        const LeafDesc& L = op->ldesc[i];
        for (int64_t r0 = 0; r0 < L.mp; r0 += kTileRows) {
            const int64_t nr = std::min<int64_t>(kTileRows, L.mp - r0);
            double* chunk = img.data() + L.d_off + r0 * L.mp;
            for (int64_t c = 0; c < L.m; ++c)
                for (int64_t r = r0; r < std::min<int64_t>(r0 + nr, L.m); ++r)
                    chunk[c * nr + (r - r0)] = op->D[i][size_t(c * L.m + r)];
        }
    });
    hipError_t e = hipSetDevice(op->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hodlr_status r;
    if ((r = upload(&op->d_leaf, img.data(), img.size(), "leaf blocks")) != HODLR_OK) return r;
    if ((r = upload(&op->d_leaves, op->ldesc.data(), op->ldesc.size(), "leaf table")) != HODLR_OK)
        return r;
    if ((r = upload(&op->d_etiles, op->etiles.data(), op->etiles.size(), "tiles")) != HODLR_OK)
        return r;
    return HODLR_OK;
}

bool valid_fmt(int32_t f) { return f >= 0 && f < NFMT; }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t hodlr_depth_for_leaf(int64_t n, int64_t leaf) {
    if (n < 1 || leaf < 1) return -1;
    int32_t d = 0;
    while (leaf * (int64_t(1) << d) < n) ++d;
    return d;
}

hodlr_status hodlr_tree_bounds(int64_t n, int32_t depth, const int64_t* leaf_bounds,
                               int64_t* bounds_out) {
    if (n < 1 || depth < 0 || depth > 24 || !bounds_out)
        return fail(HODLR_E_ARG, "hodlr_tree_bounds: n >= 1, 0 <= depth <= 24, non-null output");
    std::vector<int64_t> b;
    if (!build_bounds(n, depth, leaf_bounds, b))
        return fail(HODLR_E_ARG, "leaf_bounds must run non-decreasing from 0 to n");
    std::memcpy(bounds_out, b.data(), b.size() * sizeof(int64_t));
    return ok();
}

hodlr_status hodlr_tree_blocks(int64_t n, int32_t depth, const int64_t* leaf_bounds,
                               int64_t* desc_out) {
    if (n < 1 || depth < 0 || depth > 24 || !desc_out)
        return fail(HODLR_E_ARG, "hodlr_tree_blocks: n >= 1, 0 <= depth <= 24, non-null output");
    std::vector<int64_t> b;
    if (!build_bounds(n, depth, leaf_bounds, b))
        return fail(HODLR_E_ARG, "leaf_bounds must run non-decreasing from 0 to n");
    const auto blks = build_blocks(depth, b);
    for (size_t i = 0; i < blks.size(); ++i) {
        desc_out[5 * i + 0] = blks[i].level;
        desc_out[5 * i + 1] = blks[i].row0;
        desc_out[5 * i + 2] = blks[i].nrows;
        desc_out[5 * i + 3] = blks[i].col0;
        desc_out[5 * i + 4] = blks[i].ncols;
    }
    return ok();
}

hodlr_status hodlr_create(hodlr_op* out, int64_t n, int32_t depth, const int64_t* leaf_bounds,
                          const double* const* leaves, const int64_t* ld_leaves,
                          const hodlr_lowrank* blocks, int32_t device) {
    if (!out) return fail(HODLR_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || depth < 0 || depth > 24)
        return fail(HODLR_E_ARG, "need n >= 1 and 0 <= depth <= 24");
    if (!leaves || !ld_leaves || (depth > 0 && !blocks))
        return fail(HODLR_E_ARG, "leaves, ld_leaves and blocks must be non-null");
    if (device < -1) return fail(HODLR_E_ARG, "device must be >= -1");
    std::unique_ptr<hodlr_op_s> op(new (std::nothrow) hodlr_op_s);
    if (!op) return fail(HODLR_E_NOMEM, "operator");
    static std::atomic<uint64_t> next_uid{1};
    op->uid = next_uid++;
    op->n = n;
    op->depth = depth;
    op->nleaves = 1 << depth;
    op->nb = (1 << (depth + 1)) - 2;
    if (!build_bounds(n, depth, leaf_bounds, op->bounds))
        return fail(HODLR_E_ARG, "leaf_bounds must run non-decreasing from 0 to n");
    op->blocks = build_blocks(depth, op->bounds);
    const int64_t* lb = op->bounds.data() + ((int64_t(1) << depth) - 1) + depth;
    try {
        op->D.resize(op->nleaves);
        for (int i = 0; i < op->nleaves; ++i) {
            const int64_t m = lb[i + 1] - lb[i];
            if (m > 0 && (!leaves[i] || ld_leaves[i] < m))
                return fail(HODLR_E_ARG, "leaf %d: NULL data or ld < m", i);
            op->D[i].resize(size_t(m * m));
            for (int64_t c = 0; c < m; ++c)
                std::memcpy(op->D[i].data() + c * m, leaves[i] + c * ld_leaves[i], sizeof(double) * m);
        }
        op->U.resize(op->nb);
        op->V.resize(op->nb);
        op->rank.resize(op->nb);
        for (int b = 0; b < op->nb; ++b) {
            const HBlock& hb = op->blocks[b];
            const hodlr_lowrank& L = blocks[b];
            if (L.rank < 0 || L.rank > std::min(hb.nrows, hb.ncols))
                return fail(HODLR_E_ARG, "block %d: rank %d outside [0, min(%lld, %lld)]", b,
                            L.rank, (long long)hb.nrows, (long long)hb.ncols);
            if (L.rank > 0 && (!L.U || !L.V || L.ldu < hb.nrows || L.ldv < hb.ncols))
                return fail(HODLR_E_ARG, "block %d: NULL factor or leading dimension too small", b);
            op->rank[b] = L.rank;
            op->U[b].resize(size_t(hb.nrows * L.rank));
            op->V[b].resize(size_t(hb.ncols * L.rank));
            for (int j = 0; j < L.rank; ++j) {
                std::memcpy(op->U[b].data() + j * hb.nrows, L.U + j * L.ldu, sizeof(double) * hb.nrows);
                std::memcpy(op->V[b].data() + j * hb.ncols, L.V + j * L.ldv, sizeof(double) * hb.ncols);
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(HODLR_E_NOMEM, "host copy of the operator");
    }
    op->level_fmt.assign(depth, F64);
    op->xi.assign(depth, 0.0);
    op->uprime.assign(depth, 0.0);
    op->insufficient.assign(depth, 0);
    op->acc_double = true;
    op->device = device;
    if (device >= 0) {
        int cnt = 0;
        hipError_t e = hipGetDeviceCount(&cnt);
        if (e != hipSuccess || device >= cnt)
            return fail(HODLR_E_DEVICE, "device %d not available (%d devices): %s", device, cnt,
                        hipGetErrorString(e));
    }
    hodlr_status r = pack_leaves(op.get());
    if (r == HODLR_OK) r = pack(op.get());
    if (r != HODLR_OK) {
        free_device(op.get());
        return r;
    }
    *out = op.release();
    return ok();
}

hodlr_status hodlr_assign_precision(hodlr_op op, double eps, const int32_t* allowed,
                                    int32_t n_allowed, const double* xi_in, const double* norms2,
                                    uint32_t flags) {
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (!(eps > 0.0 && eps < 1.0)) return fail(HODLR_E_ARG, "eps must lie in (0, 1)");
    if (n_allowed < 0 || (n_allowed > 0 && !allowed)) return fail(HODLR_E_ARG, "allowed set");
    for (int i = 0; i < n_allowed; ++i)
        if (!valid_fmt(allowed[i])) return fail(HODLR_E_ARG, "allowed[%d] = %d is no format", i, allowed[i]);
    if ((flags & HODLR_ACC_FP32) && (flags & HODLR_ACC_FP64))
        return fail(HODLR_E_ARG, "HODLR_ACC_FP32 and HODLR_ACC_FP64 both set");
    const int depth = op->depth;
    if (xi_in)
        for (int k = 0; k < depth; ++k)
            if (!(xi_in[k] >= 0.0) || std::isinf(xi_in[k]))
                return fail(HODLR_E_ARG, "xi[%d] is negative, infinite or NaN", k);
    // nrmAll, ||H_b||_F^2 and their per-level maxima: given, the original
    // matrix's (operators built by hodlr_build_kernel), or from the factors
    std::vector<double> tmp_norms;
    double all = 0.0;
    std::vector<double> lvl(depth, 0.0), bn2(op->nb, 0.0);
    if (!norms2 && op->have_orig) {
        tmp_norms.push_back(op->orig_norm2_all);
        tmp_norms.insert(tmp_norms.end(), op->orig_norm2.begin(), op->orig_norm2.end());
        norms2 = tmp_norms.data();
    }
    if (norms2) {
        all = norms2[0];
        for (int b = 0; b < op->nb; ++b) {
            const double v = norms2[1 + b];
            if (!(v >= 0.0)) return fail(HODLR_E_ARG, "norms2[%d] is negative or NaN", 1 + b);
            bn2[b] = v;
            lvl[op->blocks[b].level - 1] = std::max(lvl[op->blocks[b].level - 1], v);
        }
        if (!(all >= 0.0)) return fail(HODLR_E_ARG, "norms2[0] is negative or NaN");
    } else if (!xi_in || (flags & HODLR_PER_BLOCK)) {
        // ||U V^T||_F^2 = sum((U^T U) .* (V^T V)); ||H~||_F^2 adds the leaves
        std::vector<double> nb2(op->nb, 0.0);
        parallel_for(op->nb, [&](int64_t b) {
            const int p = op->rank[b];
            const int64_t r = op->blocks[b].nrows, c = op->blocks[b].ncols;
            double s = 0.0;
            for (int a = 0; a < p; ++a)
                for (int bb = 0; bb < p; ++bb) {
                    double gu = 0.0, gv = 0.0;
                    for (int64_t i = 0; i < r; ++i) gu += op->U[b][a * r + i] * op->U[b][bb * r + i];
                    for (int64_t i = 0; i < c; ++i) gv += op->V[b][a * c + i] * op->V[b][bb * c + i];
                    s += gu * gv;
                }
            nb2[b] = s;
        });
        for (int i = 0; i < op->nleaves; ++i)
            for (double v : op->D[i]) all += v * v;
        for (int b = 0; b < op->nb; ++b) {
            all += nb2[b];
            bn2[b] = nb2[b];
            lvl[op->blocks[b].level - 1] = std::max(lvl[op->blocks[b].level - 1], nb2[b]);
        }
    }
    // candidates: fp64 (the working precision) and the allowed set
    std::vector<int> cand = {F64};
    for (int i = 0; i < n_allowed; ++i) cand.push_back(allowed[i]);
    // the rule for xi at level k: (u', format or -1)
    auto choose = [&](double x, int k, double* u_out) {
        const double u1 = (x == 0.0) ? INFINITY : eps / (std::sqrt(std::ldexp(1.0, k)) * x);
        int best = -1;
        for (int f : cand)
            if (unit_roundoff(f) <= u1 && (best < 0 || unit_roundoff(f) > unit_roundoff(best))) best = f;
        *u_out = u1;
        return best;
    };
    auto xi_of = [&](double v) { return all > 0.0 ? std::sqrt(v / all) : 0.0; };
    std::vector<int32_t> fmt(depth), bad(depth);
    std::vector<double> xi(depth), up(depth);
    for (int k = 1; k <= depth; ++k) {
        xi[k - 1] = xi_in ? xi_in[k - 1] : xi_of(lvl[k - 1]);
        const int best = choose(xi[k - 1], k, &up[k - 1]);
        fmt[k - 1] = best < 0 ? F64 : best;
        bad[k - 1] = best < 0 ? 1 : 0;
    }
    std::vector<int32_t> bfmt;
    if (flags & HODLR_PER_BLOCK) {
        bfmt.assign(op->nb, F64);
        for (int b = 0; b < op->nb; ++b) {
            double u1;
            const int best = choose(xi_of(bn2[b]), op->blocks[b].level, &u1);
            bfmt[b] = best < 0 ? F64 : best;
        }
    }
    const auto old_fmt = op->level_fmt;
    const auto old_bfmt = op->block_fmt;
    const bool old_acc = op->acc_double, old_scale = op->scale_cols;
    op->level_fmt = fmt;
    op->block_fmt = bfmt;
    op->scale_cols = !(flags & HODLR_NO_COLUMN_SCALE);
    op->acc_double = (flags & HODLR_ACC_FP64) ? true : (flags & HODLR_ACC_FP32) ? false : (eps < 1e-7);
    hodlr_status r = pack(op);
    if (r != HODLR_OK) {
        std::string m = g_last_error;
        op->level_fmt = old_fmt;
        op->block_fmt = old_bfmt;
        op->acc_double = old_acc;
        op->scale_cols = old_scale;
        (void)pack(op);
        return fail(r, "%s", m.c_str());
    }
    op->xi = xi;
    op->uprime = up;
    op->insufficient = bad;
    op->eps = eps;
    drop_lu(op);                  // factors of the previous representation
    return ok();
}

hodlr_status hodlr_set_level_precisions(hodlr_op op, const int32_t* per_level, uint32_t flags) {
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (op->depth > 0 && !per_level) return fail(HODLR_E_ARG, "per_level is NULL");
    if ((flags & HODLR_ACC_FP32) && (flags & HODLR_ACC_FP64))
        return fail(HODLR_E_ARG, "HODLR_ACC_FP32 and HODLR_ACC_FP64 both set");
    bool all64 = true;
    for (int k = 0; k < op->depth; ++k) {
        if (!valid_fmt(per_level[k])) return fail(HODLR_E_ARG, "per_level[%d] = %d is no format", k, per_level[k]);
        all64 = all64 && per_level[k] == F64;
    }
    const auto old_fmt = op->level_fmt;
    const auto old_bfmt = op->block_fmt;
    const bool old_acc = op->acc_double, old_scale = op->scale_cols;
    op->level_fmt.assign(per_level, per_level + op->depth);
    op->block_fmt.clear();
    op->scale_cols = !(flags & HODLR_NO_COLUMN_SCALE);
    op->acc_double = (flags & HODLR_ACC_FP64) ? true : (flags & HODLR_ACC_FP32) ? false : all64;
    hodlr_status r = pack(op);
    if (r != HODLR_OK) {
        std::string m = g_last_error;
        op->level_fmt = old_fmt;
        op->block_fmt = old_bfmt;
        op->acc_double = old_acc;
        op->scale_cols = old_scale;
        (void)pack(op);
        return fail(r, "%s", m.c_str());
    }
    op->xi.assign(op->depth, 0.0);
    op->uprime.assign(op->depth, 0.0);
    op->insufficient.assign(op->depth, 0);
    op->eps = 0.0;
    drop_lu(op);
    return ok();
}

hodlr_status hodlr_get_level(hodlr_op op, int32_t level, int32_t* dtype, double* xi,
                             double* u_prime, int32_t* insufficient) {
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (level < 1 || level > op->depth) return fail(HODLR_E_ARG, "level %d outside 1..%d", level, op->depth);
    if (dtype) *dtype = op->level_fmt[level - 1];
    if (xi) *xi = op->xi[level - 1];
    if (u_prime) *u_prime = op->uprime[level - 1];
    if (insufficient) *insufficient = op->insufficient[level - 1];
    return ok();
}

hodlr_status hodlr_get_info(hodlr_op op, hodlr_info* info) {
    if (!op || !info) return fail(HODLR_E_ARG, "NULL argument");
    info->n = op->n;
    info->depth = op->depth;
    info->nblocks = op->nb;
    info->acc_dtype = op->acc_double ? HODLR_FP64 : HODLR_FP32;
    info->max_rank = 0;
    for (int32_t r : op->rank) info->max_rank = std::max(info->max_rank, r);
    info->on_device = op->device >= 0;
    info->device = op->device;
    info->eps = op->eps;
    int64_t lb = 0;
    for (auto& d : op->D) lb += int64_t(d.size()) * 8;
    info->leaf_bytes = lb;
    info->factor_bytes = op->codes_bytes;
    info->scale_bytes = op->scaled_cols;
    int64_t dl = 0;
    for (auto& L : op->ldesc) dl += int64_t(L.mp) * L.mp * 8;
    info->device_bytes = op->fac_bytes + dl;
    return ok();
}

hodlr_status hodlr_get_block(hodlr_op op, int32_t block, hodlr_block_info* info) {
    if (!op || !info) return fail(HODLR_E_ARG, "NULL argument");
    if (block < 0 || block >= op->nb) return fail(HODLR_E_ARG, "block %d outside 0..%d", block, op->nb - 1);
    const HBlock& hb = op->blocks[block];
    info->level = hb.level;
    info->rank = op->rank[block];
    info->row0 = hb.row0;
    info->nrows = hb.nrows;
    info->col0 = hb.col0;
    info->ncols = hb.ncols;
    info->dtype = op->block_fmt.empty() ? op->level_fmt[hb.level - 1] : op->block_fmt[block];
    info->scaled = (op->scale_cols && scaled_format(info->dtype)) ? 1 : 0;
    return ok();
}

hodlr_status hodlr_query(hodlr_op op, hodlr_query_info* q, int64_t* leaf_bounds, int32_t* ranks) {
    if (!op || !q) return fail(HODLR_E_ARG, "NULL argument");
    std::memset(q, 0, sizeof(*q));
    hodlr_status r = hodlr_get_info(op, &q->info);
    if (r != HODLR_OK) return r;
    for (int k = 0; k < op->depth; ++k) {
        q->level_dtype[k] = op->level_fmt[k];
        q->insufficient[k] = op->insufficient[k];
        q->xi[k] = op->xi[k];
        q->u_prime[k] = op->uprime[k];
    }
    q->per_block = op->block_fmt.empty() ? 0 : 1;
    q->leaf_stacked = op->stacked ? 1 : 0;
    if (leaf_bounds) {
        const int64_t* lb = op->bounds.data() + ((int64_t(1) << op->depth) - 1) + op->depth;
        std::memcpy(leaf_bounds, lb, sizeof(int64_t) * size_t(op->nleaves + 1));
    }
    if (ranks) std::memcpy(ranks, op->rank.data(), sizeof(int32_t) * size_t(op->nb));
    return ok();
}

hodlr_status hodlr_export_block(hodlr_op op, int32_t block, void* u_codes, int8_t* u_exp,
                                void* v_codes, int8_t* v_exp, int32_t from_device) {
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (block < 0 || block >= op->nb) return fail(HODLR_E_ARG, "block %d outside 0..%d", block, op->nb - 1);
    const HBlock& hb = op->blocks[block];
    const BlockDesc& d = op->bdesc[block];
    const int p = d.rank, f = d.fmt, s = fmt_bytes(f);
    const int k = hb.level;
    const int64_t j = block - ((int64_t(1) << k) - 2);
    std::vector<int32_t> eu(p), ev(p);
    std::vector<RowLoc> umap, vmap;
    node_rowlocs(op, k, j, 0, umap);
    node_rowlocs(op, k, j ^ 1, d.pad_, vmap);
    auto put_u = [&](int64_t i, int jj, uint64_t c) {
        if (u_codes) put_code(static_cast<uint8_t*>(u_codes) + (int64_t(jj) * hb.nrows + i) * s, f, c);
    };
    auto put_v = [&](int64_t i, int jj, uint64_t c) {
        if (v_codes) put_code(static_cast<uint8_t*>(v_codes) + (int64_t(jj) * hb.ncols + i) * s, f, c);
    };
    hodlr_status r = quantize_factor(op->U[block], hb.nrows, p, f, op->scale_cols, eu.data(), put_u);
    if (r == HODLR_OK) r = quantize_factor(op->V[block], hb.ncols, p, f, op->scale_cols, ev.data(), put_v);
    if (r != HODLR_OK) return r;
    if (from_device) {
        if (op->device < 0 || !op->d_fac) return fail(HODLR_E_STATE, "host-only handle has no device image");
        hipError_t e = hipSetDevice(op->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        std::vector<uint8_t> ub(size_t(d.urows) * p * s), vb(size_t(d.vrows) * p * s);
        if (p > 0) {
            e = hipMemcpy(ub.data(), op->d_fac + d.u_off, ub.size(), hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = hipMemcpy(vb.data(), op->d_fac + d.v_off, vb.size(), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "read back factor image");
        }
        for (int jj = 0; jj < p; ++jj) {
            if (u_codes)
                for (int64_t i = 0; i < hb.nrows; ++i)
                    std::memcpy(static_cast<uint8_t*>(u_codes) + (int64_t(jj) * hb.nrows + i) * s,
                                ub.data() + loc_index(umap[i], jj, p) * s, s);
            if (v_codes)
                for (int64_t i = 0; i < hb.ncols; ++i)
                    std::memcpy(static_cast<uint8_t*>(v_codes) + (int64_t(jj) * hb.ncols + i) * s,
                                vb.data() + loc_index(vmap[i], jj, p) * s, s);
        }
    }
    for (int jj = 0; jj < p; ++jj) {
        if (u_exp) u_exp[jj] = int8_t(eu[jj]);
        if (v_exp) v_exp[jj] = int8_t(ev[jj]);
    }
    return ok();
}

}  // extern "C"

namespace {

// The augmented operands [D_i | U of the ancestors] in the working
// precision w (HODLR_BF16 or HODLR_FP16), built on `stream` by the device
// from the current image when it is older than the last pack.  For fp16
// every leaf entry and every generator stored in a format wider than
// fp16's range (fp64, fp32, bf16) must be finite in fp16 (E_RANGE
// otherwise); the narrow stored formats are column-scaled into range.
//
// Built once per assignment under the handle's aug_mu: the first caller
// enqueues the build on its stream and waits for it before marking the
// operand ready, so a product on any other stream that finds it ready
// reads a finished operand.  The build allocates, so it cannot happen
// while `stream` is being captured (E_STATE: run one product outside the
// capture first).
hodlr_status ensure_aug(hodlr_op_s* op, int32_t w, const KParams& kp, void* stream) {
    const int slot = w == HODLR_BF16 ? 0 : 1;
    std::lock_guard<std::mutex> lk(op->aug_mu);
    if (op->d_aug[slot] && op->aug_gen[slot] == op->gen) return HODLR_OK;
    {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cap);
        if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
        if (cap != hipStreamCaptureStatusNone)
            return fail(HODLR_E_STATE, "the %s operand of this assignment is built on the first %s product, "
                        "which cannot run under stream capture; run one product outside the capture first",
                        w == HODLR_BF16 ? "bf16" : "fp16", w == HODLR_BF16 ? "bf16" : "fp16");
    }
    if (w == HODLR_FP16) {
        std::atomic<int> bad{-1};
        parallel_for(op->nleaves, [&](int64_t i) {
            for (double v : op->D[size_t(i)]) {
                bool ovf = false;
                (void)encode_rne(v, F16, &ovf);
                if (ovf) { bad.store(int(i)); return; }
            }
        });
        if (bad.load() >= 0) return fail(HODLR_E_RANGE, "leaf %d has an entry outside the fp16 range", bad.load());
        for (int b = 0; b < op->nb; ++b) {
            const int32_t bf = op->bdesc[size_t(b)].fmt;
            if (bf != F64 && bf != F32 && bf != BF16) continue;
            for (const std::vector<double>* Fm : {&op->U[size_t(b)], &op->V[size_t(b)]})
                for (double v : *Fm) {
                    bool ovf = false;
                    (void)encode_rne(v, F16, &ovf);
                    if (ovf) return fail(HODLR_E_RANGE, "block %d has a generator value outside the fp16 range", b);
                }
        }
    }
    if (!op->d_aug[slot]) {
        hipError_t e = hipMalloc(&op->d_aug[slot], size_t(std::max<int64_t>(op->aug_total, 1)) * 2);
        if (e != hipSuccess) {
            op->d_aug[slot] = nullptr;
            (void)hipGetLastError();
            return fail(HODLR_E_NOMEM, "augmented operand (%lld values)", (long long)op->aug_total);
        }
    }
    KParams k2 = kp;
    k2.aug = op->d_aug[slot];
    const int he = launch_build_aug(k2, slot, stream);
    if (he != 0) return fail(HODLR_E_DEVICE, "augmented operand: %s", hipGetErrorString(hipError_t(he)));
    const hipError_t se = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (se != hipSuccess) return hip_fail(se, "building the augmented operand");
    op->aug_gen[slot] = op->gen;
    return HODLR_OK;
}

// Bytes of each workspace buffer one product needs.
struct WsNeeds {
    int64_t partial, T, xpad, W, Tw, sync;
};

WsNeeds workspace_needs(const hodlr_op_s* op, int nrhs, int xy_bytes) {
    WsNeeds n{};
    // padded X: when some leaf is padded, and for the matrix-core path (nrhs >= kWideMin),
    // which reads X with 16-byte vector loads and copies it when it is not aligned
    // (the low working precision path, 2-byte X, always runs on the matrix cores)
    const bool lowp = xy_bytes == 2;
    // partials: per (block, leaf) for the leaf-stacked contraction (operators
    // whose leaves are one unit each, on the matrix cores: nrhs >= kWideMin
    // or the low working precision), else per contraction item
    n.partial = std::max<int64_t>(1, ((nrhs >= kWideMin || lowp) && op->stacked ? op->total_stack_rank
                                                                                  : op->total_item_rank) *
                                         nrhs) * 8;
    n.T = std::max<int64_t>(1, op->total_rank * nrhs) * 8;
    n.xpad = (op->padded || nrhs >= kWideMin || lowp) ? op->npad * nrhs * xy_bytes : 0;
    n.W = (nrhs < kWideMin && !lowp) ? op->npad * nrhs * 8 : 0;
    n.Tw = lowp ? std::max<int64_t>(1, op->total_rank8 * nrhs) * 2 : 0;
    n.sync = sync_words(op->nb) * int64_t(sizeof(int32_t));
    return n;
}

// The operator's part of the launch parameters (everything but the workspace).
void fill_kparams(const hodlr_op_s* op, KParams* kp) {
    kp->fac = op->d_fac;
    kp->leafd = op->d_leaf;
    kp->blocks = op->d_blocks;
    kp->leaves = op->d_leaves;
    kp->citems = op->d_citems;
    kp->stiles = op->d_stiles;
    kp->stile_off = op->d_stile_off;
    kp->sunits = op->d_sunits;
    kp->nsunits = int32_t(op->sunits.size());
    kp->stacked = 0;
    kp->part_f32 = op->stacked ? 1 : 0;
    if (op->stacked)
        for (const SUnit& su : op->sunits) {
            kp->stacked = std::max(kp->stacked, su.ng);
            if (op->stiles[size_t(su.t0)].dbl) kp->part_f32 = 0;
        }
    for (int k = 0; k < kMaxDepth; ++k) kp->level_max_rank[k] = 0;
    for (int b = 0; b < op->nb; ++b) {
        const int k = op->bdesc[size_t(b)].level;
        kp->level_max_rank[k - 1] = std::max(kp->level_max_rank[k - 1], op->rank[size_t(b)]);
    }
    kp->etiles = op->d_etiles;
    kp->tscale = op->d_tscale;
    kp->npad = op->npad;
    kp->max_leaf = op->max_leaf;
    kp->max_rank_path = op->max_rank_path;
    kp->max_tstage = op->max_tstage;
    kp->max_kp = op->max_kp;
    kp->max_block_rank = op->max_block_rank;
    kp->max_items_rank = op->max_items_rank;
    kp->depth = op->depth;
    kp->nblocks = op->nb;
    kp->nleaves = op->nleaves;
    kp->ncitems = int32_t(op->citems.size());
    kp->netiles = int32_t(op->etiles.size());
    kp->padded = op->padded ? 1 : 0;
}

hodlr_status prepare_workspace(hodlr_op_s* op, void* stream, int nrhs, int xy_bytes, KParams* kp,
                               uint64_t* ws_gen = nullptr) {
    std::lock_guard<std::mutex> lk(op->ws_mu);
    Workspace& w = op->ws[stream];
    const WsNeeds need = workspace_needs(op, nrhs, xy_bytes);
    auto grow = [&](void** ptr, int64_t* cap, int64_t bytes, const char* what) -> hodlr_status {
        if (bytes <= *cap) return HODLR_OK;
        if (*ptr) {
            // the old buffer stays allocated (retired): work already enqueued, and any graph
            // captured with it, keep reading valid memory; grow at least twofold so the
            // retired buffers never hold more than the current one
            w.retired.push_back(*ptr);
            bytes = std::max(bytes, 2 * *cap);
            *ptr = nullptr;
            *cap = 0;
        }
        hipError_t e = hipMalloc(ptr, size_t(bytes));
        if (e != hipSuccess) {
            *ptr = nullptr;
            (void)hipGetLastError();
            return fail(HODLR_E_NOMEM, "workspace %s (%lld bytes)", what, (long long)bytes);
        }
        *cap = bytes;
        ++w.gen;
        return HODLR_OK;
    };
    hodlr_status r;
    if ((r = grow(reinterpret_cast<void**>(&w.partial), &w.cap_partial, need.partial, "partials")) != HODLR_OK)
        return r;
    if ((r = grow(reinterpret_cast<void**>(&w.T), &w.cap_T, need.T, "T")) != HODLR_OK) return r;
    if (need.xpad && (r = grow(&w.xpad, &w.cap_xpad, need.xpad, "padded X")) != HODLR_OK) return r;
    if (need.W && (r = grow(reinterpret_cast<void**>(&w.W), &w.cap_W, need.W, "leaf products")) != HODLR_OK)
        return r;
    if (need.Tw && (r = grow(&w.Tw, &w.cap_Tw, need.Tw, "T in the working precision")) != HODLR_OK) return r;
    if (need.sync > w.cap_sync) {
        if ((r = grow(reinterpret_cast<void**>(&w.sync), &w.cap_sync, need.sync, "counters")) != HODLR_OK) return r;
        hipError_t e = hipMemset(w.sync, 0, size_t(w.cap_sync));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "clearing counters");
    }
    fill_kparams(op, kp);
    kp->partial = w.partial;
    kp->T = w.T;
    kp->xpad = w.xpad;
    kp->W = w.W;
    kp->Tw = w.Tw;
    kp->sync = w.sync;
    if (ws_gen) *ws_gen = w.gen;
    return HODLR_OK;
}

// ---------------------------------------------------------------------------
// batched products: plan, autotune, capture, replay
// ---------------------------------------------------------------------------
// A plan holds, for one batch signature (operators with their image and
// workspace generations, X/Y pointers and leading dimensions, nrhs, dtypes,
// stream), the device copies of the per-operator launch records and of the
// work lists of every kernel-variant group, the launch shape the autotuner
// chose for each launch, and a HIP graph of the launches.
//
// The autotuner picks, separately for every launch (one group's one
// phase), the work order (longest item first, or as the operators were
// given) and the persistent grid (1, 2, 4 or 8 workgroups per compute
// unit): each candidate launch runs alone, four times, on the caller's
// stream the first time a signature is seen (the groups run one after
// another, so the best launch of each is the best batch).  Choices are
// kept in a tuning cache keyed by the device's architecture and the
// launch's shape class (variant, phase, and the number of work items and
// their total cost rounded to powers of two), in memory and in a text
// file (HODLR_TUNE_CACHE, default $HOME/.cache/hodlr/batch_tune.txt;
// HODLR_TUNE_CACHE=off keeps it in memory only), so later plans of the
// same shapes skip the timing.  HODLR_BATCH_TUNE=0 skips tuning (longest
// first, 2 workgroups per compute unit).  Any choice gives the same
// result bit for bit: a work item's arithmetic does not depend on which
// workgroup runs it.
struct BatchPlan {
    std::vector<uint64_t> uids;
    void* d_buf = nullptr;
    std::vector<BatchGroup> groups[2];   // [order]: 0 longest first, 1 natural
    std::vector<BatchGroup> tuned;       // the launches as run: per phase its order's list and grid
    std::vector<std::array<std::string, 4>> shape;   // tuning-cache class of each group's phases
    float tuned_ms = 0.0f;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
    bool captured = false;   // recorded into a caller's graph: kept until an operator of it is destroyed
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_buf) (void)hipFree(d_buf);
    }
};

std::mutex g_batch_mu;
// Deliberately never destroyed: a static map would free its plans' graphs
// and device buffers from the library's static destructor, after the HIP
// runtime may already have shut down at process exit.  Plans of destroyed
// operators are freed by hodlr_destroy (batch_forget).
auto& g_plans = *new std::map<std::vector<uint64_t>, std::unique_ptr<BatchPlan>>();
uint64_t g_batch_clock = 0;
constexpr size_t kMaxPlans = 32;

void batch_forget(uint64_t uid) {      // plans that name a destroyed operator
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::find(it->second->uids.begin(), it->second->uids.end(), uid) != it->second->uids.end())
            it = g_plans.erase(it);
        else
            ++it;
    }
}

int compute_units(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

hipError_t launch_groups(const std::vector<BatchGroup>& gs, hipStream_t s) {
    // phase by phase across groups (each group's own launches stay in order)
    for (const auto& g : gs) {
        const int r = launch_batch_group(g, s);
        if (r) return hipError_t(r);
    }
    return hipSuccess;
}

struct GroupBuild {
    BatchGroup g{};
    std::vector<BatchOp> ops;
    std::vector<std::pair<int64_t, WorkItem>> work[4];   // (cost, item) per phase
};

hodlr_status build_plan(const hodlr_op* ops, int count, const void* const* X, const int64_t* ldx,
                        void* const* Y, const int64_t* ldy, const int32_t* nrhs, const int32_t* xy_dtype,
                        void* stream, BatchPlan* plan) {
    std::map<std::vector<int32_t>, GroupBuild> groups;
    for (int i = 0; i < count; ++i) {
        hodlr_op op = ops[i];
        const bool xyd = xy_dtype[i] == HODLR_FP64;
        KParams kp{};
        hodlr_status r = prepare_workspace(op, stream, nrhs[i], xyd ? 8 : 4, &kp);
        if (r != HODLR_OK) return r;
        OpLaunch ol{};
        if (plan_launch(kp, X[i], ldx[i], nrhs[i], xyd, op->acc_double, &ol) != 0)
            return fail(HODLR_E_UNSUPPORTED, "operator %d: leaf size %d with path rank %d needs more than 64 KB of LDS",
                        i, op->max_leaf, op->max_rank_path);
        const std::vector<int32_t> key = {xyd ? 1 : 0, op->acc_double ? 1 : 0, ol.wide, ol.rg,
                                          (ol.wide && op->stacked) ? 1 : 0};
        GroupBuild& gb = groups[key];
        BatchGroup& g = gb.g;
        if (gb.ops.empty()) {
            g.xy_double = key[0];
            g.acc_double = key[1];
            g.wide = ol.wide;
            g.rg = ol.rg;
            g.ntc = ol.ntc;
            g.jc = 0;
            g.stacked = 0;
        }
        if (key[4]) g.stacked = std::max(g.stacked, kp.stacked);   // the most tiles of a unit in the group
        g.stage_cap = std::max(g.stage_cap, ol.stage_cap);
        g.lds_contract = std::max(g.lds_contract, ol.lds_contract);
        g.lds_expand = std::max(g.lds_expand, ol.lds_expand);
        if (ol.jc) g.jc = g.jc ? std::min(g.jc, ol.jc) : ol.jc;
        const int32_t oi = int32_t(gb.ops.size());
        BatchOp bo{};
        bo.kp = kp;
        bo.X = X[i];
        bo.ldx = ldx[i];
        bo.Y = Y[i];
        bo.ldy = ldy[i];
        bo.nrhs = nrhs[i];
        bo.Xc = ol.padx ? kp.xpad : X[i];
        bo.ldc = ol.padx ? op->npad : ldx[i];
        gb.ops.push_back(bo);
        const int64_t s_rhs = nrhs[i];
        if (ol.padx)
            for (int l = 0; l < op->nleaves; ++l)
                gb.work[0].push_back({int64_t(op->ldesc[l].mp) * s_rhs, WorkItem{oi, l, 0, 0}});
        const int gyc = ol.wide ? ol.gy_contract : 1;
        if (ol.wide && op->stacked) {   // matrix cores, stacked: one work item per (unit, column group)
            for (int u = 0; u < int(op->sunits.size()); ++u) {
                const SUnit& su = op->sunits[size_t(u)];
                const int64_t mp = op->ldesc[size_t(su.leaf)].mp;
                int64_t cost = mp * 4 * s_rhs;
                for (int t = su.t0; t < su.t0 + su.ng; ++t)
                    cost += mp * op->stiles[size_t(t)].n * fmt_bytes(op->stiles[size_t(t)].fmt);
                for (int y = 0; y < gyc; ++y) gb.work[1].push_back({cost, WorkItem{oi, u, y, 0}});
            }
        } else {
            for (int c = 0; c < int(op->citems.size()); ++c) {
                const CItem& it = op->citems[c];
                const BlockDesc& bd = op->bdesc[it.block];
                const int64_t cost = int64_t(it.nr) * bd.rank * fmt_bytes(bd.fmt) + int64_t(it.nr) * 4 * s_rhs;
                for (int y = 0; y < gyc; ++y) gb.work[1].push_back({cost, WorkItem{oi, c, y, 0}});
            }
        }
        if (!ol.wide)             // the wave path's first launch also runs the leaf tiles (y = 1)
            for (int t = 0; t < int(op->etiles.size()); ++t) {
                const ETile& et = op->etiles[t];
                gb.work[1].push_back({int64_t(et.nr) * op->ldesc[et.leaf].mp * 8, WorkItem{oi, t, 1, 0}});
            }
        if (ol.wide && !op->citems.empty())
            for (int b = 0; b < op->nb; ++b) {
                const BlockDesc& bd = op->bdesc[b];
                const int64_t total = int64_t(bd.rank) * nrhs[i];
                const int out = op->stacked ? 256 / stack_slices(bd.sleaves) : 256;
                for (int64_t y = 0; y * out < total; ++y)
                    gb.work[2].push_back({op->stacked ? int64_t(bd.sleaves) : int64_t(bd.nitems),
                                          WorkItem{oi, b, int32_t(y), 0}});
            }
        const int gye = ol.wide ? ol.gy_expand : 1;
        for (int t = 0; t < int(op->etiles.size()); ++t) {
            const ETile& et = op->etiles[t];
            const LeafDesc& L = op->ldesc[et.leaf];
            int64_t cost = ol.wide ? int64_t(et.nr) * L.mp * 8 : int64_t(et.nr) * 8;
            for (int k = 1; k <= op->depth; ++k) {
                const BlockDesc& bd = op->bdesc[((1 << k) - 2) + (et.leaf >> (op->depth - k))];
                cost += int64_t(et.nr) * bd.rank * fmt_bytes(bd.fmt);
            }
            for (int y = 0; y < gye; ++y) gb.work[3].push_back({cost, WorkItem{oi, t, y, 0}});
        }
    }
    // device image: per group its ops, then the work lists in both orders
    size_t bytes = 0;
    auto reserve = [&](size_t n) {
        const size_t off = bytes;
        bytes = (bytes + n + 255) / 256 * 256;
        return off;
    };
    struct Offs { size_t ops, work[2][4]; };
    std::vector<Offs> offs;
    for (auto& kv : groups) {
        Offs o{};
        o.ops = reserve(kv.second.ops.size() * sizeof(BatchOp));
        for (int ord = 0; ord < 2; ++ord)
            for (int ph = 0; ph < 4; ++ph) o.work[ord][ph] = reserve(kv.second.work[ph].size() * sizeof(WorkItem));
        offs.push_back(o);
    }
    std::vector<uint8_t> img(std::max<size_t>(bytes, 256), 0);
    size_t gi = 0;
    for (auto& kv : groups) {
        GroupBuild& gb = kv.second;
        const Offs& o = offs[gi++];
        std::memcpy(img.data() + o.ops, gb.ops.data(), gb.ops.size() * sizeof(BatchOp));
        for (int ph = 0; ph < 4; ++ph) {
            auto& w = gb.work[ph];
            std::vector<WorkItem> natural(w.size()), sorted(w.size());
            for (size_t q = 0; q < w.size(); ++q) natural[q] = w[q].second;
            std::stable_sort(w.begin(), w.end(), [](const std::pair<int64_t, WorkItem>& a,
                                                    const std::pair<int64_t, WorkItem>& b) {
                return a.first > b.first;
            });
            for (size_t q = 0; q < w.size(); ++q) sorted[q] = w[q].second;
            std::memcpy(img.data() + o.work[0][ph], sorted.data(), sorted.size() * sizeof(WorkItem));
            std::memcpy(img.data() + o.work[1][ph], natural.data(), natural.size() * sizeof(WorkItem));
        }
    }
    hipError_t e = hipMalloc(&plan->d_buf, img.size());
    if (e != hipSuccess) {
        plan->d_buf = nullptr;
        (void)hipGetLastError();
        return fail(HODLR_E_NOMEM, "batch plan (%zu bytes)", img.size());
    }
    e = hipMemcpy(plan->d_buf, img.data(), img.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "uploading the batch plan");
    uint8_t* base = static_cast<uint8_t*>(plan->d_buf);
    gi = 0;
    for (auto& kv : groups) {
        const GroupBuild& gb = kv.second;
        const Offs& o = offs[gi++];
        for (int ord = 0; ord < 2; ++ord) {
            BatchGroup g = gb.g;
            g.ops = reinterpret_cast<const BatchOp*>(base + o.ops);
            g.padx = reinterpret_cast<const WorkItem*>(base + o.work[ord][0]);
            g.contract = reinterpret_cast<const WorkItem*>(base + o.work[ord][1]);
            g.reduce = reinterpret_cast<const WorkItem*>(base + o.work[ord][2]);
            g.expand = reinterpret_cast<const WorkItem*>(base + o.work[ord][3]);
            g.n_padx = int32_t(gb.work[0].size());
            g.n_contract = int32_t(gb.work[1].size());
            g.n_reduce = int32_t(gb.work[2].size());
            g.n_expand = int32_t(gb.work[3].size());
            plan->groups[ord].push_back(g);
        }
    }
    for (int i = 0; i < count; ++i) plan->uids.push_back(ops[i]->uid);
    // the tuning-cache class of every launch: variant, phase, work items and cost (powers of two)
    auto lg = [](int64_t v) { int b = 0; while ((int64_t(1) << b) < v) ++b; return b; };
    for (auto& kv : groups) {
        std::array<std::string, 4> cls;
        for (int ph = 0; ph < 4; ++ph) {
            int64_t cost = 0;
            for (auto& w : kv.second.work[ph]) cost += w.first;
            char buf[160];
            std::snprintf(buf, sizeof(buf), "x%d.a%d.w%d.r%d.s%d.ph%d.n%d.c%d", kv.first[0], kv.first[1],
                          kv.first[2], kv.first[3], kv.first[4], ph, lg(int64_t(kv.second.work[ph].size())),
                          lg(cost));
            cls[ph] = buf;
        }
        plan->shape.push_back(cls);
    }
    return ok();
}

// ---- tuning cache ---------------------------------------------------------
struct TuneChoice {
    int order, mult;
};
std::mutex g_tune_mu;
// never destroyed (see g_plans); loaded from the file on first use
auto& g_tune = *new std::map<std::string, TuneChoice>();
bool g_tune_loaded = false;

std::string tune_file() {
    const char* env = std::getenv("HODLR_TUNE_CACHE");
    if (env && std::strcmp(env, "off") == 0) return "";
    if (env && env[0]) return env;
    const char* home = std::getenv("HOME");
    if (!home || !home[0]) return "";
    return std::string(home) + "/.cache/hodlr/batch_tune.txt";
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string f = tune_file();
    if (f.empty()) return;
    std::ifstream in(f);
    std::string key;
    int o, m;
    while (in >> key >> o >> m)
        if ((o == 0 || o == 1) && (m == 1 || m == 2 || m == 4 || m == 8)) g_tune[key] = TuneChoice{o, m};
}

void tune_store_locked(const std::string& key, TuneChoice c) {
    g_tune[key] = c;
    const std::string f = tune_file();
    if (f.empty()) return;
    // create the file's directories (failures show up as an unwritable file, which is ignored)
    for (size_t q = f.find('/', 1); q != std::string::npos; q = f.find('/', q + 1))
        (void)::mkdir(f.substr(0, q).c_str(), 0755);
    std::ofstream out(f, std::ios::app);
    if (out) out << key << ' ' << c.order << ' ' << c.mult << '\n';
}

std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    for (char& ch : a)
        if (ch == ' ') ch = '_';
    char buf[32];
    std::snprintf(buf, sizeof(buf), ".cu%d", prop.multiProcessorCount);
    return a + buf;
}

// One group's launch of phase ph alone: the other phases' counts set to 0.
BatchGroup phase_only(const BatchGroup& g, int ph) {
    BatchGroup o = g;
    if (ph != 0) o.n_padx = 0;
    if (ph != 1) o.n_contract = 0;
    if (ph != 2) o.n_reduce = 0;
    if (ph != 3) o.n_expand = 0;
    return o;
}

int phase_count(const BatchGroup& g, int ph) {
    return ph == 0 ? g.n_padx : ph == 1 ? g.n_contract : ph == 2 ? g.n_reduce : g.n_expand;
}

// Set phase ph of `dst` to order `ord`'s work list with `mult` workgroups per CU.
void apply_choice(BatchGroup& dst, const BatchPlan* plan, size_t gi, int ph, TuneChoice c, int cus) {
    const BatchGroup& src = plan->groups[c.order][gi];
    if (ph == 0) dst.padx = src.padx;
    if (ph == 1) dst.contract = src.contract;
    if (ph == 2) dst.reduce = src.reduce;
    if (ph == 3) dst.expand = src.expand;
    dst.grid[ph] = std::max(1, std::min(phase_count(src, ph), cus * c.mult));
}

hodlr_status tune_plan(BatchPlan* plan, int device, hipStream_t s) {
    const int cus = compute_units(device);
    plan->tuned = plan->groups[0];
    const char* env = std::getenv("HODLR_BATCH_TUNE");
    const bool timing = !(env && env[0] == '0');
    const std::string arch = arch_name(device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return fail(HODLR_E_DEVICE, "events for the batch autotuner");
    }
    hodlr_status st = HODLR_OK;
    float total = 0.0f;
    for (size_t gi = 0; gi < plan->tuned.size() && st == HODLR_OK; ++gi)
        for (int ph = 0; ph < 4 && st == HODLR_OK; ++ph) {
            if (phase_count(plan->groups[0][gi], ph) == 0) continue;
            TuneChoice best{0, 2};
            const std::string key = arch + "|" + plan->shape[gi][ph];
            bool have = false;
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                tune_load_locked();
                auto it = g_tune.find(key);
                if (it != g_tune.end()) {
                    best = it->second;
                    have = true;
                }
            }
            if (timing && !have) {
                float best_ms = -1.0f;
                const int mults[4] = {1, 2, 4, 8};
                for (int ord = 0; ord < 2 && st == HODLR_OK; ++ord)
                    for (int m : mults) {
                        BatchGroup cand = plan->tuned[gi];
                        apply_choice(cand, plan, gi, ph, TuneChoice{ord, m}, cus);
                        const std::vector<BatchGroup> one = {phase_only(cand, ph)};
                        hipError_t e = launch_groups(one, s);                 // warm-up
                        if (e == hipSuccess) e = hipEventRecord(e0, s);
                        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) e = launch_groups(one, s);
                        if (e == hipSuccess) e = hipEventRecord(e1, s);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0.0f;
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        if (e != hipSuccess) {
                            st = hip_fail(e, "batch autotuner");
                            break;
                        }
                        if (best_ms < 0.0f || ms < best_ms) {
                            best_ms = ms;
                            best = TuneChoice{ord, m};
                        }
                    }
                if (st != HODLR_OK) break;
                total += best_ms / 4.0f;
                std::lock_guard<std::mutex> lk(g_tune_mu);
                tune_store_locked(key, best);
            }
            apply_choice(plan->tuned[gi], plan, gi, ph, best, cus);
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != HODLR_OK) return st;
    plan->tuned_ms = total;
    return ok();
}

// The chosen launches, in order, captured on a private stream.
hodlr_status capture_plan(BatchPlan* plan) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = launch_groups(plan->tuned, cs);
        e = hipStreamEndCapture(cs, &plan->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "capturing the batch graph");
    return ok();
}

hodlr_status batch_run(const hodlr_op* ops, int count, const void* const* X, const int64_t* ldx, void* const* Y,
                       const int64_t* ldy, const int32_t* nrhs, const int32_t* xy_dtype, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    const bool capturing = cap == hipStreamCaptureStatusActive;
    // signature (after making sure every workspace is large enough)
    std::vector<uint64_t> key;
    key.reserve(size_t(count) * 10 + 1);
    key.push_back(reinterpret_cast<uintptr_t>(stream));
    for (int i = 0; i < count; ++i) {
        KParams kp{};
        uint64_t wg = 0;
        if (capturing) {
            // nothing may be allocated while capturing: use the workspace as it is
            std::lock_guard<std::mutex> lk(ops[i]->ws_mu);
            auto it = ops[i]->ws.find(stream);
            if (it == ops[i]->ws.end())
                return fail(HODLR_E_STATE, "operator %d: no workspace on this stream; run the batch once "
                                           "outside capture first", i);
            wg = it->second.gen;
        } else {
            hodlr_status r = prepare_workspace(ops[i], stream, nrhs[i], xy_dtype[i] == HODLR_FP64 ? 8 : 4, &kp, &wg);
            if (r != HODLR_OK) return r;
        }
        key.insert(key.end(), {ops[i]->uid, ops[i]->gen, wg, uint64_t(reinterpret_cast<uintptr_t>(X[i])),
                               uint64_t(ldx[i]), uint64_t(reinterpret_cast<uintptr_t>(Y[i])), uint64_t(ldy[i]),
                               uint64_t(nrhs[i]), uint64_t(xy_dtype[i])});
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) {
        // a plan is built (allocated, uploaded, tuned, captured) outside capture only; the
        // signature pins the workspaces it was built with, so a capture that finds it is safe
        if (capturing)
            return fail(HODLR_E_STATE, "batch not seen before on this stream with these arguments; run it "
                                       "once outside capture first");
        if (g_plans.size() >= kMaxPlans) {            // drop the least recently used plan no graph of the
            auto lru = g_plans.end();                   // caller's holds (those stay until an operator goes)
            for (auto q = g_plans.begin(); q != g_plans.end(); ++q)
                if (!q->second->captured && (lru == g_plans.end() || q->second->last_use < lru->second->last_use))
                    lru = q;
            if (lru != g_plans.end()) {
                (void)hipDeviceSynchronize();
                g_plans.erase(lru);
            }
        }
        std::unique_ptr<BatchPlan> plan(new (std::nothrow) BatchPlan);
        if (!plan) return fail(HODLR_E_NOMEM, "batch plan");
        hodlr_status r = build_plan(ops, count, X, ldx, Y, ldy, nrhs, xy_dtype, stream, plan.get());
        if (r != HODLR_OK) return r;
        r = tune_plan(plan.get(), ops[0]->device, s);
        if (r == HODLR_OK) r = capture_plan(plan.get());
        if (r != HODLR_OK) return r;
        it = g_plans.emplace(key, std::move(plan)).first;
    }
    BatchPlan* plan = it->second.get();
    plan->last_use = ++g_batch_clock;
    if (capturing) plan->captured = true;
    if (capturing || !plan->exec)
        e = launch_groups(plan->tuned, s);                   // the caller's capture records the launches
    else
        e = hipGraphLaunch(plan->exec, s);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return ok();
}

}  // namespace

extern "C" {

hodlr_status hodlr_matvec(hodlr_op op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                          int32_t nrhs, int32_t xy_dtype, hipStream_t hstream) {
    void* stream = static_cast<void*>(hstream);
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (op->device < 0) return fail(HODLR_E_STATE, "host-only handle: no product");
    if (nrhs < 1) return fail(HODLR_E_ARG, "nrhs must be >= 1");
    const bool lowp = xy_dtype == HODLR_BF16 || xy_dtype == HODLR_FP16;
    if (xy_dtype != HODLR_FP32 && xy_dtype != HODLR_FP64 && !lowp)
        return fail(HODLR_E_UNSUPPORTED, "X/Y dtype must be HODLR_FP64, HODLR_FP32, HODLR_BF16 or HODLR_FP16");
    if (!X || !Y) return fail(HODLR_E_ARG, "X or Y is NULL");
    if (ldx < op->n || ldy < op->n) return fail(HODLR_E_ARG, "ldx and ldy must be >= n");
    hipError_t e = hipSetDevice(op->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    KParams kp{};
    const int xy_bytes = xy_dtype == HODLR_FP64 ? 8 : xy_dtype == HODLR_FP32 ? 4 : 2;
    hodlr_status r = prepare_workspace(op, stream, nrhs, xy_bytes, &kp);
    if (r != HODLR_OK) return r;
    if (lowp) {
        if ((r = ensure_aug(op, xy_dtype, kp, stream)) != HODLR_OK) return r;
        kp.aug = op->d_aug[xy_dtype == HODLR_BF16 ? 0 : 1];
    }
    void* const* ev = nullptr;
    bool ran[kPhases] = {false, false, false, false};
    int32_t slot = -1;
    if (op->prof_used < op->prof_cap) {
        slot = op->prof_used++;
        ev = reinterpret_cast<void* const*>(op->prof_ev.data() + size_t(slot) * 2 * kPhases);
    }
    const int he = lowp ? launch_matvec_lp(kp, X, ldx, Y, ldy, nrhs, xy_dtype == HODLR_BF16 ? 0 : 1, stream, ev, ran)
                        : launch_matvec(kp, X, ldx, Y, ldy, nrhs, xy_dtype == HODLR_FP64, op->acc_double, stream,
                                        ev, ran);
    if (he == int(hipErrorInvalidConfiguration))
        return fail(HODLR_E_UNSUPPORTED, "leaf size %d with path rank %d needs more than 64 KB of LDS",
                    op->max_leaf, op->max_rank_path);
    if (slot >= 0)
        for (int ph = 0; ph < kPhases; ++ph) op->prof_ran[size_t(slot) * kPhases + ph] = ran[ph] ? 1 : 0;
    if (he != 0) return fail(HODLR_E_DEVICE, "kernel launch: %s", hipGetErrorString(hipError_t(he)));
    return ok();
}

hodlr_status hodlr_matvec_noalloc(hodlr_op op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                  int32_t nrhs, int32_t xy_dtype, hipStream_t hstream) {
    void* stream = static_cast<void*>(hstream);
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (op->device < 0) return fail(HODLR_E_STATE, "host-only handle: no product");
    if (nrhs < 1) return fail(HODLR_E_ARG, "nrhs must be >= 1");
    if (xy_dtype != HODLR_FP32 && xy_dtype != HODLR_FP64)
        return fail(HODLR_E_UNSUPPORTED, "hodlr_matvec_noalloc takes HODLR_FP64 or HODLR_FP32 X and Y");
    if (!X || !Y) return fail(HODLR_E_ARG, "X or Y is NULL");
    if (ldx < op->n || ldy < op->n) return fail(HODLR_E_ARG, "ldx and ldy must be >= n");
    const int xy_bytes = xy_dtype == HODLR_FP64 ? 8 : 4;
    // the workspace carved from the scratch array: counters first, every buffer 256-byte aligned
    const WsNeeds need = workspace_needs(op, nrhs, xy_bytes);
    int64_t off = 0;
    auto carve = [&](int64_t bytes) {
        const int64_t o = off;
        off += align_up(std::max<int64_t>(bytes, 0), 256);
        return o;
    };
    const int64_t o_sync = carve(need.sync), o_part = carve(need.partial), o_T = carve(need.T);
    const int64_t o_x = carve(need.xpad), o_W = carve(need.W);
    if (off > int64_t(kScratchBytes))
        return fail(HODLR_E_ARG, "this product needs %lld bytes of workspace, more than the %lld bytes of "
                    "hodlr_matvec_noalloc's scratch; use hodlr_matvec", (long long)off, (long long)kScratchBytes);
    hipError_t e = hipSetDevice(op->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* base = nullptr;
    const int se = scratch_address(op->device, &base);
    if (se != 0) return fail(HODLR_E_DEVICE, "scratch address: %s", hipGetErrorString(hipError_t(se)));
    uint8_t* b8 = static_cast<uint8_t*>(base);
    KParams kp{};
    fill_kparams(op, &kp);
    kp.sync = reinterpret_cast<int32_t*>(b8 + o_sync);
    kp.partial = reinterpret_cast<double*>(b8 + o_part);
    kp.T = reinterpret_cast<double*>(b8 + o_T);
    kp.xpad = need.xpad ? static_cast<void*>(b8 + o_x) : nullptr;
    kp.W = need.W ? reinterpret_cast<double*>(b8 + o_W) : nullptr;
    // the array keeps the last call's contents: the arrival counters must start at zero
    int he = launch_zero_words(kp.sync, need.sync / int64_t(sizeof(int32_t)), stream);
    if (he == 0)
        he = launch_matvec(kp, X, ldx, Y, ldy, nrhs, xy_dtype == HODLR_FP64, op->acc_double, stream, nullptr,
                           nullptr);
    if (he == int(hipErrorInvalidConfiguration))
        return fail(HODLR_E_UNSUPPORTED, "leaf size %d with path rank %d needs more than 64 KB of LDS",
                    op->max_leaf, op->max_rank_path);
    if (he != 0) return fail(HODLR_E_DEVICE, "kernel launch: %s", hipGetErrorString(hipError_t(he)));
    return ok();
}

hodlr_status hodlr_matvec_batched(const hodlr_op* ops, int32_t count, const void* const* X,
                                  const int64_t* ldx, void* const* Y, const int64_t* ldy,
                                  const int32_t* nrhs, const int32_t* xy_dtype, hipStream_t hstream) {
    void* stream = static_cast<void*>(hstream);
    if (count < 0) return fail(HODLR_E_ARG, "count < 0");
    if (count == 0) return ok();
    if (!ops || !X || !ldx || !Y || !ldy || !nrhs || !xy_dtype) return fail(HODLR_E_ARG, "NULL array");
    for (int i = 0; i < count; ++i) {
        hodlr_op op = ops[i];
        if (!op) return fail(HODLR_E_ARG, "ops[%d] is NULL", i);
        if (op->device < 0) return fail(HODLR_E_STATE, "ops[%d] is a host-only handle", i);
        if (op->device != ops[0]->device) return fail(HODLR_E_STATE, "operators on different devices");
        if (nrhs[i] < 1) return fail(HODLR_E_ARG, "nrhs[%d] must be >= 1", i);
        if (xy_dtype[i] != HODLR_FP32 && xy_dtype[i] != HODLR_FP64 && xy_dtype[i] != HODLR_BF16 &&
            xy_dtype[i] != HODLR_FP16)
            return fail(HODLR_E_UNSUPPORTED, "xy_dtype[%d] must be HODLR_FP64, HODLR_FP32, HODLR_BF16 or HODLR_FP16",
                        i);
        if (!X[i] || !Y[i]) return fail(HODLR_E_ARG, "X[%d] or Y[%d] is NULL", i, i);
        if (ldx[i] < op->n || ldy[i] < op->n) return fail(HODLR_E_ARG, "ldx[%d] and ldy[%d] must be >= n", i, i);
    }
    {   // each operator's workspace serves one product at a time
        std::vector<hodlr_op> sorted(ops, ops + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(HODLR_E_ARG, "an operator appears more than once in the batch");
    }
    hipError_t e = hipSetDevice(ops[0]->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    // products in a low working precision (bf16 / fp16) run one after another
    // through the single-operator launches; the others as the planned batch
    std::vector<int> lp, hp;
    for (int i = 0; i < count; ++i)
        (xy_dtype[i] == HODLR_BF16 || xy_dtype[i] == HODLR_FP16 ? lp : hp).push_back(i);
    hodlr_status r;
    // the low-precision operands (range checks, one build per assignment)
    // are settled before any product is enqueued
    for (int i : lp) {
        KParams kp{};
        if ((r = prepare_workspace(ops[i], stream, nrhs[i], 2, &kp)) != HODLR_OK) return r;
        if ((r = ensure_aug(ops[i], xy_dtype[i], kp, stream)) != HODLR_OK) return r;
    }
    if (hp.size() == size_t(count)) return batch_run(ops, count, X, ldx, Y, ldy, nrhs, xy_dtype, stream);
    if (!hp.empty()) {
        const size_t m = hp.size();
        std::vector<hodlr_op> o(m);
        std::vector<const void*> x(m);
        std::vector<void*> y(m);
        std::vector<int64_t> lx(m), ly(m);
        std::vector<int32_t> nr(m), dt(m);
        for (size_t q = 0; q < m; ++q) {
            const int i = hp[q];
            o[q] = ops[i];
            x[q] = X[i];
            y[q] = Y[i];
            lx[q] = ldx[i];
            ly[q] = ldy[i];
            nr[q] = nrhs[i];
            dt[q] = xy_dtype[i];
        }
        if ((r = batch_run(o.data(), int(m), x.data(), lx.data(), y.data(), ly.data(), nr.data(), dt.data(),
                           stream)) != HODLR_OK)
            return r;
    }
    for (int i : lp)
        if ((r = hodlr_matvec(ops[i], X[i], ldx[i], Y[i], ldy[i], nrhs[i], xy_dtype[i], hstream)) != HODLR_OK)
            return r;
    return ok();
}

hodlr_status hodlr_profile(hodlr_op op, int32_t capacity) {
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (capacity < 0) return fail(HODLR_E_ARG, "capacity < 0");
    if (op->device < 0) return fail(HODLR_E_STATE, "host-only handle");
    hipError_t e = hipSetDevice(op->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    free_profile(op);
    if (capacity == 0) return ok();
    op->prof_ev.resize(size_t(capacity) * 2 * kPhases, nullptr);
    for (auto& ev : op->prof_ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            ev = nullptr;
            free_profile(op);
            return hip_fail(e, "hipEventCreate");
        }
    }
    op->prof_ran.assign(size_t(capacity) * kPhases, 0);
    op->prof_cap = capacity;
    op->prof_used = 0;
    return ok();
}

hodlr_status hodlr_profile_read(hodlr_op op, double* ms_per_phase, int64_t* launches_per_phase) {
    if (!op || !ms_per_phase || !launches_per_phase) return fail(HODLR_E_ARG, "NULL argument");
    for (int ph = 0; ph < kPhases; ++ph) {
        ms_per_phase[ph] = 0.0;
        launches_per_phase[ph] = 0;
    }
    for (int32_t i = 0; i < op->prof_used; ++i)
        for (int ph = 0; ph < kPhases; ++ph) {
            if (!op->prof_ran[size_t(i) * kPhases + ph]) continue;
            hipEvent_t a = op->prof_ev[(size_t(i) * kPhases + ph) * 2];
            hipEvent_t b = op->prof_ev[(size_t(i) * kPhases + ph) * 2 + 1];
            hipError_t e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) return hip_fail(e, "reading profile events");
            ms_per_phase[ph] += ms;
            launches_per_phase[ph] += 1;
        }
    op->prof_used = 0;
    std::fill(op->prof_ran.begin(), op->prof_ran.end(), 0);
    return ok();
}

hodlr_status hodlr_destroy(hodlr_op op) {
    if (!op) return fail(HODLR_E_ARG, "op is NULL");
    if (op->device >= 0) {
        (void)hipSetDevice(op->device);
        (void)hipDeviceSynchronize();
    }
    batch_forget(op->uid);
    drop_lu(op);
    free_device(op);
    delete op;
    return ok();
}

const char* hodlr_status_string(hodlr_status s) {
    switch (s) {
        case HODLR_OK: return "HODLR_OK";
        case HODLR_E_ARG: return "HODLR_E_ARG";
        case HODLR_E_STATE: return "HODLR_E_STATE";
        case HODLR_E_NOMEM: return "HODLR_E_NOMEM";
        case HODLR_E_DEVICE: return "HODLR_E_DEVICE";
        case HODLR_E_RANGE: return "HODLR_E_RANGE";
        case HODLR_E_UNSUPPORTED: return "HODLR_E_UNSUPPORTED";
    }
    return "HODLR_E_UNKNOWN";
}

hodlr_status hodlr_get_norms(hodlr_op op, double* norms2) {
    if (!op || !norms2) return fail(HODLR_E_ARG, "NULL argument");
    if (!op->have_orig) return fail(HODLR_E_STATE, "the operator carries no norms of an original matrix");
    norms2[0] = op->orig_norm2_all;
    std::memcpy(norms2 + 1, op->orig_norm2.data(), sizeof(double) * size_t(op->nb));
    return ok();
}

const char* hodlr_last_error(void) { return g_last_error.c_str(); }

const char* hodlr_last_error_message(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace hodlr {

hodlr_status host_fail(hodlr_status s, const std::string& msg) {
    if (s == HODLR_OK) return ok();
    return fail(s, "%s", msg.c_str());
}

void attach_original_norms(hodlr_op op, double norm2_all, const double* norm2_blocks) {
    op->have_orig = true;
    op->orig_norm2_all = norm2_all;
    op->orig_norm2.assign(norm2_blocks, norm2_blocks + op->nb);
}

}  // namespace hodlr

namespace hodlr {

namespace {
// The value of a code of format f (the inverse of encode_rne).
double decode_code(uint64_t code, int f) {
    if (f == F64) {
        double v;
        std::memcpy(&v, &code, 8);
        return v;
    }
    if (f == F32) {
        const uint32_t c = uint32_t(code);
        float v;
        std::memcpy(&v, &c, 4);
        return v;
    }
    const FmtInfo& F = kFmt[f];
    const int nbits = 8 * fmt_bytes(f), mbits = F.t - 1;
    const bool neg = (code >> (nbits - 1)) & 1;
    const int ex = int((code >> mbits) & ((uint64_t(1) << F.ebits) - 1));
    const double m = double(code & ((uint64_t(1) << mbits) - 1));
    const double v = ex == 0 ? std::ldexp(m, 1 - F.bias - mbits) : std::ldexp(1.0 + std::ldexp(m, -mbits), ex - F.bias);
    return neg ? -v : v;
}
}  // namespace

hodlr_status stored_operator(hodlr_op op, StoredView* out) {
    if (!op || !out) return fail(HODLR_E_ARG, "NULL argument");
    out->n = op->n;
    out->depth = op->depth;
    out->bounds = op->bounds;
    out->leaves = op->D;
    out->U.assign(size_t(op->nb), {});
    out->V.assign(size_t(op->nb), {});
    out->rank = op->rank;
    std::vector<hodlr_status> st(size_t(op->nb), HODLR_OK);
    parallel_for(op->nb, [&](int64_t b) {
        const HBlock& hb = op->blocks[size_t(b)];
        const int f = op->block_fmt.empty() ? op->level_fmt[size_t(hb.level - 1)] : op->block_fmt[size_t(b)];
        const int p = op->rank[size_t(b)];
        for (int side = 0; side < 2; ++side) {
            const std::vector<double>& Fm = side == 0 ? op->U[size_t(b)] : op->V[size_t(b)];
            const int64_t rows = side == 0 ? hb.nrows : hb.ncols;
            std::vector<double>& dst = side == 0 ? out->U[size_t(b)] : out->V[size_t(b)];
            dst.assign(size_t(rows) * p, 0.0);
            std::vector<int32_t> ex(size_t(std::max(p, 1)), 0);
            const hodlr_status r = quantize_factor(Fm, rows, p, f, op->scale_cols, ex.data(),
                                                   [&](int64_t i, int j, uint64_t code) {
                                                       dst[size_t(j) * rows + i] =
                                                           std::ldexp(decode_code(code, f), -ex[size_t(j)]);
                                                   });
            if (r != HODLR_OK) st[size_t(b)] = r;
        }
    });
    for (hodlr_status r : st)
        if (r != HODLR_OK) return r;
    return HODLR_OK;
}

void* get_lu(hodlr_op op) { return op->lu; }

void set_lu(hodlr_op op, void* lu, void (*lu_free)(void*)) {
    drop_lu(op);
    op->lu = lu;
    op->lu_free = lu_free;
}

int op_device(hodlr_op op) { return op->device; }

}  // namespace hodlr
