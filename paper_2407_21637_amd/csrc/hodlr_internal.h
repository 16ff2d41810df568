// Internal layout shared by the host core (host.cpp) and the HIP kernels
// (kernels.hip).  Not part of the public ABI.
//
// Device image of one operator
// ----------------------------
// Rows are addressed in a padded row space: leaf i occupies padded rows
// [lprow0_i, lprow0_i + mp_i) with mp_i = m_i rounded up to kRowAlign, and
// a node of any level is the concatenation of its leaves, so every node is
// one contiguous padded range.  Padding rows hold zeros in every factor
// panel and in the leaf blocks.
//
//  * leaves: fp64, leaf i (mp_i x mp_i) at element offset d_off, cut at its
//    expansion tiles: tile rows [r0, r0+nr) are column-major (ld = nr) at
//    d_off + r0 * mp_i.
//  * factor panels: for block b (rows = node j of level k, columns = node
//    j^1), the U panel covers the padded rows of node j and the V panel the
//    padded rows of node j^1, rank_b columns, codes of the level's format,
//    256-byte aligned.  Each panel is cut into row chunks stored
//    column-major one after another (chunk rows [c0, c0+h) at c0 * rank,
//    ld = h): U panels at the expansion tiles of the node's leaves, V panels
//    at the contraction items.  Every work item reads one contiguous chunk.
//  * tscale_b[j] = 2^-(eV_j + eU_j) times the decode compensation of the
//    format (fp8 e4m3 decodes through fp16 at 2^-8 of its value, once per
//    factor), applied once to T_b = V_b^T X.
//  * contraction work items split the V panel rows of each block into
//    chunks; partial results land in a workspace and are summed per block
//    in a fixed order (deterministic).
#pragma once

#include <cstddef>
#include <cstdint>

namespace hodlr {

enum Fmt : int32_t { F64 = 0, F32 = 1, BF16 = 2, F16 = 3, E4M3 = 4, E5M2 = 5, NFMT = 6 };

// Tuning parameters (compile-time; the build may override them).
#ifndef HODLR_TILE_ROWS
#define HODLR_TILE_ROWS 128          // padded rows of an expansion tile (64, 128 or 256)
#endif
#ifndef HODLR_ITEM_KB
#define HODLR_ITEM_KB 256            // target KB of codes per contraction item
#endif
#ifndef HODLR_ITEM_MIN_ROWS
#define HODLR_ITEM_MIN_ROWS 1024     // smallest contraction item (multiple of 256)
#endif

constexpr int kRowAlign = 16;        // padded rows per leaf are a multiple of this
constexpr int kPanelAlign = 256;     // byte alignment of every panel
constexpr int kTileRows = HODLR_TILE_ROWS;
constexpr int kItemRowsMax = 4096;   // rows of a contraction item (at most 16 slabs of 256)
constexpr int kMaxDepth = 24;
constexpr size_t kMaxLds = 65536;    // dynamic LDS per workgroup

inline int fmt_bytes(int f) {
    return f == F64 ? 8 : f == F32 ? 4 : (f == BF16 || f == F16) ? 2 : 1;
}

struct BlockDesc {        // one per off-diagonal block, canonical order
    int64_t u_off;        // byte offset of the U panel in the factor buffer
    int64_t v_off;        // byte offset of the V panel
    int64_t ts_off;       // offset of tscale (rank doubles)
    int64_t t_off;        // offset of T_b in units of rank (x nrhs doubles)
    int32_t rank;
    int32_t fmt;
    int32_t level;
    int32_t urow0;        // padded row start of the row node (U panel rows)
    int32_t urows;        // padded rows of the row node (= U panel ld)
    int32_t vrow0;        // padded row start of the column node
    int32_t vrows;        // padded rows of the column node (= V panel ld)
    int32_t item0;        // first contraction item of this block
    int32_t nitems;       // number of contraction items
    int32_t pad_;         // rows of a contraction item (V panel chunk)
    int64_t tw_off;       // low working precision: offset of T_b in W, in units of
                          // round_up(rank, 8) (x nrhs values, [c][j])
    int64_t s_off;        // matrix-core contraction: per-leaf partials of T_b, offset in units
                          // of rank (x nrhs doubles), one rank x nrhs slice per leaf of the
                          // column node
    int32_t sleaf0;       // first leaf of the column node
    int32_t sleaves;      // leaves of the column node
};

// Reduction of the per-leaf partials of a block with `leaves` leaves in its
// column node: the 256 threads of a workgroup take 256 / slices outputs and
// split the leaves into `slices` interleaved runs (at most 8 leaves a run
// up to 512 leaves), then add the runs in order.
constexpr int stack_slices(int leaves) {
    int s = 1;
    while (s * 8 < leaves && s < 64) s *= 2;
    return s;
}

// Matrix-core contraction (nrhs >= kWideMin): each leaf's work is cut into
// tiles of up to 16 MFMA rows, each row one rank j of one ancestor block
// whose V panel covers the leaf's rows (the block of level k whose column
// node holds the leaf).  A tile's rows share the code format and the
// arithmetic type (fp64 for fp64 codes or fp64 accumulation, else the
// accumulation type), so X is read once per leaf for all levels.
constexpr int kStackRows = 16;
struct STile {
    int32_t fmt;               // code format of every row
    int32_t dbl;               // 1: multiplied in fp64, 0: in the accumulation type
    int32_t n;                 // rows in use; rows n..15 repeat row 0 and are masked
    int32_t pad_;
    int32_t blk[kStackRows];   // block of each row
    int32_t j[kStackRows];     // rank of each row within its block
};

// A workgroup's share of the matrix-core contraction: ng consecutive tiles
// of one leaf with one format and arithmetic type (up to 2 in fp64, 4 in
// fp32), one pass over the leaf's rows.
struct SUnit {
    int32_t leaf;
    int32_t t0;                // first tile (index into the tiles)
    int32_t ng;
    int32_t pad_;
};

struct LeafDesc {
    int64_t d_off;        // element offset of D_i (doubles)
    int64_t row0;         // first (unpadded) row of the leaf
    int32_t m;            // real rows
    int32_t mp;           // padded rows (= ld of D_i)
    int32_t prow0;        // padded row start
    int32_t kp;           // low working precision: columns of the ancestors' U in the augmented
                          // operand (sum over levels of rank rounded up to 8, then up to 32)
    int64_t aug_off;      // low working precision: element offset of the leaf's augmented operand
                          // [D_i 0 | U_1 | ... | U_depth] (mp rows, row-major, ld = round_up(mp, 32) + kp)
};

struct CItem {            // contraction work item: rows [r0, r0+nr) of a V panel
    int32_t block;
    int32_t r0;
    int32_t nr;
    int32_t pad_;
    int64_t poff;         // partial offset in units of rank (x nrhs doubles)
};

struct ETile {            // expansion + leaf tile: padded rows [r0, r0+nr) of leaf
    int32_t leaf;
    int32_t r0;
    int32_t nr;
    int32_t pad_;
};

// Everything a launch needs, by value.
struct KParams {
    const uint8_t* fac;          // factor panels
    const double* leafd;         // leaf blocks
    const BlockDesc* blocks;
    const LeafDesc* leaves;
    const CItem* citems;
    const STile* stiles;         // matrix-core contraction tiles, leaf by leaf
    const int32_t* stile_off;    // first tile of each leaf (nleaves + 1 values)
    const SUnit* sunits;         // matrix-core contraction units (nsunits)
    const ETile* etiles;
    const double* tscale;
    const void* aug;             // low working precision: the augmented operands in W (LeafDesc::aug_off)
    void* Tw;                    // low working precision: T_b in W (sum of round_up(rank, 8) * nrhs)
    double* partial;             // workspace: sum over items of rank * nrhs
    double* T;                   // workspace: sum over blocks of rank * nrhs
    void* xpad;                  // workspace: padded copy of X (npad * nrhs), if needed
    double* W;                   // workspace (nrhs < kWideMin): leaf products D_i X_i, npad * nrhs
    int32_t* sync;               // workspace: sync_words(nblocks) counters, zero between launches
    int64_t npad;                // padded rows
    int32_t max_leaf;            // largest leaf (rows)
    int32_t max_rank_path;       // largest sum of ranks over the blocks of one leaf's ancestors
    int32_t max_items_rank;      // largest nitems * rank of a block (partials to add up)
    int32_t depth;
    int32_t nblocks;
    int32_t nleaves;
    int32_t ncitems;
    int32_t nsunits;
    int32_t stacked;             // matrix-core contraction by stacked tiles (SUnit): the most tiles of a unit; 0: by items
    int32_t part_f32;            // stacked, every tile in fp32 arithmetic: the per-leaf partials are
                                 // stored as fp32 (their values are fp32 sums), else fp64
    int32_t netiles;
    int32_t padded;              // 1 if any leaf has padding rows (X goes through xpad)
    int32_t max_block_rank;      // largest rank of a block
    int32_t max_tstage;          // matrix-core expansion: largest sum, over one leaf's ancestor
                                 // blocks, of round_up(rank, 4) * (8 if fp64 else 4) bytes
                                 // (T of every level staged in LDS, per LDS row element)
    int32_t max_kp;              // low working precision: largest LeafDesc::kp
    int32_t level_max_rank[kMaxDepth];   // largest rank of a block of level k (index k - 1)
};

// Counters of the contraction launch: kSyncHead reserved words, then one
// arrival counter per block (zero between launches).
constexpr int kSyncHead = 4;
constexpr int64_t sync_words(int64_t nblocks) { return kSyncHead + nblocks; }

// products with at least this many right-hand sides run on the matrix cores
constexpr int kWideMin = 8;

constexpr int kPhases = 4;     // padded X copy, contraction, expansion, reduction of partials

// Launch the whole product on `stream`.  xy_double: X/Y are fp64 (else fp32);
// acc_double: accumulation precision of Y.  events: NULL, or 2 * kPhases
// hipEvent_t recorded before/after each phase that runs (a phase that does
// not run leaves its pair unrecorded; `ran` reports which did).
// Returns a hipError_t as int.
int launch_matvec(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy,
                  int nrhs, bool xy_double, bool acc_double, void* stream, void* const* events,
                  bool* ran);

// low working precision (w = 0: bf16, 1: fp16): X and Y in W, every operand
// rounded to W, fp32 accumulation on the matrix cores
// build the augmented operands (LeafDesc::aug_off) of kp.aug in W (w = 0: bf16, 1: fp16)
int launch_build_aug(const KParams& kp, int w, void* stream);

int launch_matvec_lp(const KParams& kp, const void* X, int64_t ldx, void* Y, int64_t ldy, int nrhs, int w,
                     void* stream, void* const* events, bool* ran);

// ---------------------------------------------------------------------------
// allocation-free products (hodlr_matvec_noalloc)
// ---------------------------------------------------------------------------
// Every workspace buffer of such a product is carved from one file-scope
// device array (`scratch`, kernels.hip) of kScratchBytes on each GPU.
constexpr size_t kScratchBytes = size_t(64) << 20;

// Device address of the scratch array on `device`, which must be the
// current device.  Looked up once per device (hipGetSymbolAddress) and
// kept; returns a hipError_t as int.
int scratch_address(int device, void** ptr);

// Zero n int32 words at p on `stream` with a fill kernel (no memset node,
// so the call may be captured into a graph).  Returns a hipError_t as int.
int launch_zero_words(int32_t* p, int64_t n, void* stream);

// ---------------------------------------------------------------------------
// batched products: persistent launches over many operators
// ---------------------------------------------------------------------------
// How one product of one operator is launched (chosen as the
// single-operator path chooses it).
struct OpLaunch {
    int32_t wide;              // matrix-core path (nrhs >= kWideMin)
    int32_t rg;                // wave path: right-hand sides per pass; matrix-core path: 16-column tiles
    int32_t ntc;               // matrix-core contraction: 16-column tiles
    int32_t padx;              // X goes through the padded copy
    int32_t stage_cap;         // wave contraction: LDS doubles for the last arriver's staging
    int32_t jc;                // matrix-core expansion: T chunk rows when not staged whole
    int64_t lds_contract;
    int64_t lds_expand;
    int32_t gy_contract;       // matrix-core: right-hand-side groups of the contraction
    int32_t gy_expand;         // ... and of the expansion
};

struct BatchOp {               // one operator of a batched product (device array)
    KParams kp;
    const void* X;             // caller's X (ld ldx)
    const void* Xc;            // X as the contraction (and the matrix-core expansion) reads it
    void* Y;
    int64_t ldx, ldc, ldy;
    int32_t nrhs;
    int32_t pad_;
};

struct WorkItem {              // (operator, leaf / item / block / tile, right-hand-side group)
    int32_t op;
    int32_t idx;
    int32_t y;
    int32_t pad_;
};

// One persistent launch per phase for the operators sharing a kernel variant.
struct BatchGroup {
    int32_t xy_double, acc_double, wide, rg, ntc;
    int32_t stage_cap, jc;
    int32_t stacked;           // matrix cores: contraction by stacked tiles (every operator of the group),
                               // the most tiles of a unit over the group; 0: by items
    int32_t pad_;
    int64_t lds_contract, lds_expand;
    const BatchOp* ops;        // device
    const WorkItem* padx;      // device arrays and their lengths
    const WorkItem* contract;
    const WorkItem* reduce;
    const WorkItem* expand;
    int32_t n_padx, n_contract, n_reduce, n_expand;
    int32_t grid[4];           // workgroups of the four persistent launches
};

// 0 on success, else a hipError_t value (hipErrorInvalidConfiguration: LDS
// needs beyond 64 KB).
int plan_launch(const KParams& kp, const void* X, int64_t ldx, int nrhs, bool xy_double, bool acc_double,
                OpLaunch* out);
int launch_batch_group(const BatchGroup& g, void* stream);

}  // namespace hodlr
