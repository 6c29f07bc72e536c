// Host-side data structures of the FE step library: CSR pattern + element
// map, nested-dissection ordering, supernodal symbolic structure, and the
// FP64 numeric LDL^T factor in the explicit-inverse panel form used by the
// GPU triangular solves.  Pure C++ (no HIP); compiled with the host compiler.
#pragma once

#include <sys/mman.h>

#include <cstdint>
#include <cstdlib>
#include <functional>
#include <new>
#include <string>
#include <vector>

namespace fe {

// Allocator for the large host arrays of the set-up (triplets, map, pattern):
// blocks of 64 MiB and more are 2 MiB aligned and asked for transparent huge
// pages, which cuts the first-touch page faults of multi-GB arrays.
template <typename T>
struct HugeAlloc {
  using value_type = T;
  static constexpr size_t kBig = size_t(64) << 20, kAlign = size_t(2) << 20;
  HugeAlloc() = default;
  template <typename U>
  HugeAlloc(const HugeAlloc<U> &) {}
  T *allocate(size_t n) {
    const size_t bytes = n * sizeof(T);
    if (bytes < kBig) return static_cast<T *>(::operator new(bytes));
    const size_t al = (bytes + kAlign - 1) / kAlign * kAlign;
    void *p = std::aligned_alloc(kAlign, al);
    if (!p) throw std::bad_alloc();
    madvise(p, al, MADV_HUGEPAGE);
    return static_cast<T *>(p);
  }
  void deallocate(T *p, size_t n) {
    if (n * sizeof(T) < kBig) ::operator delete(p);
    else std::free(p);
  }
};
template <typename T, typename U>
bool operator==(const HugeAlloc<T> &, const HugeAlloc<U> &) { return true; }
template <typename T, typename U>
bool operator!=(const HugeAlloc<T> &, const HugeAlloc<U> &) { return false; }
template <typename T>
using hvec = std::vector<T, HugeAlloc<T>>;

// ---------------------------------------------------------------- pattern
struct Pattern {
  int32_t n_nodes = 0, n_elems = 0, nen = 0;
  int64_t n = 0;                          // DOFs
  std::vector<int32_t> conn;              // [E * nen] element-major copy
  std::vector<int32_t> row_ptr;           // CSR of A (structural, sorted)
  hvec<int32_t> col_idx;
  hvec<int32_t> tmap;                     // canonical map [E * (3 nen)^2]
  std::vector<int32_t> fixed_diag_slot;   // CSR slot of (d, d) per fixed DOF
  std::vector<int32_t> fixed_dofs;
  std::vector<uint8_t> fixed;             // [n]
  // compact map: slot[e * nen*nen + a*nen + b] = rank of node conn[e][b]
  // among the free neighbour nodes of conn[e][a] (0xFF: dropped).  Valid when
  // every node is fully free or fully fixed.
  bool compact_ok = false;
  std::vector<uint8_t> slot;
  std::vector<uint8_t> node_fixed;        // [n_nodes], 1 = all DOFs fixed
  // Inverse of the compact map, for an assembly without atomics: the 3 x 3
  // node blocks of the free rows of A (block = (row node, slot)), each with
  // the list of element contributions e * nen^2 + a * nen + b that fall on
  // it, in element order.  blk_pos = CSR position of the block's entry
  // (0, 0); blk_node = row node, with bit 31 set on diagonal blocks.
  std::vector<int32_t> blk_ptr, blk_pos, blk_node;
  hvec<int32_t> blk_src;
};

// Two counting-sort transposes + merge (paper Sec. 4.2, Sec. 6.1).
// Returns an error message or "" on success.
std::string build_pattern(int32_t n_nodes, int32_t n_elems, int32_t nen,
                          const int32_t *conn, const uint8_t *fixed_dof, Pattern &P);

// ------------------------------------------------- ordering and symbolic
// Device panels store column j of supernode s at dev_off + j * ld with ld a
// multiple of kPanelAlign entries, so that the sweeps' 256-row column runs of
// a tile start on cache-line boundaries.
constexpr int32_t kPanelAlign = 32;

struct Supernode {
  int32_t nc = 0;        // own columns (DOFs eliminated in this block)
  int32_t m = 0;         // rows of the panel: own columns first, then struct
  int64_t panel_off = 0; // offset (entries) of the m x nc column-major panel
                         // of the host factorisation (leading dimension m)
  int32_t ld = 0;        // leading dimension of the device panel: m rounded
                         // up to kPanelAlign entries, so that every column
                         // starts on a 128-byte boundary (FP32)
  int64_t dev_off = 0;   // offset (entries) of the device panel
  int64_t rows_off = 0;  // offset into Symbolic::rows
  int32_t parent = -1;   // enclosing supernode, -1 for a root
  int32_t level = 0;     // height above the leaves (dependency level)
  int32_t first = 0;     // position of the first own column in perm
};

// Tile of the GPU triangular solves: supernode s, row block r0, column
// block c0 (tile extents fixed by the kernels' tile sizes).
struct Tile {
  int32_t s, r0, c0, pad;
};

// One tile of the many-right-hand-side sweeps: supernode s, the first of the
// 64 panel rows (forward) or own columns (backward) it produces, and the
// range [lo, hi) of the contraction it covers (panel columns forward, panel
// rows backward).  A long contraction is split over several tiles whose
// results are summed with atomics.
struct MTile {
  int32_t s, b0, lo, hi;
};
constexpr int kMultiRows = 64;     // output rows (forward) / columns (backward) per tile

struct Symbolic {
  int64_t n = 0;                       // DOFs (incl. fixed)
  int64_t n_free = 0;
  std::vector<int32_t> perm;           // perm[k] = DOF eliminated k-th
  std::vector<int32_t> iperm;          // iperm[dof] (fixed DOFs >= n_free)
  std::vector<int32_t> sn_ptr;         // supernode s owns perm[sn_ptr[s]..)
  std::vector<Supernode> sn;           // in elimination (post)order
  std::vector<int32_t> rows;           // panel row DOFs per supernode
  std::vector<std::vector<int32_t>> children;
  int32_t n_levels = 0;
  int64_t panel_entries = 0, lower_entries = 0;
  int64_t dev_panel_entries = 0;  // device panels, columns padded to ld
  double flops = 0.0;
  // GPU schedules, grouped by level (forward: ascending, backward: descending)
  std::vector<Tile> fwd_tiles, bwd_tiles;
  std::vector<int32_t> fwd_level_ptr, bwd_level_ptr;
  // tile extents per level (index = level): forward columns, backward rows
  std::vector<int32_t> fwd_level_cols, fwd_level_groups, bwd_level_rows, bwd_level_cols;
  // many-right-hand-side schedules (same level order)
  std::vector<MTile> mfwd_tiles, mbwd_tiles;
  std::vector<int32_t> mfwd_level_ptr, mbwd_level_ptr;
  std::vector<double> level_lower;     // panel entries on/below the diagonal per level
  std::vector<int32_t> mbwd_dofs, mbwd_dof_ptr;  // own DOFs per backward level
};

// Tile extents shared with the device kernels.
constexpr int kFwdRows = 256;      // rows per forward tile (one per thread)
constexpr int kBwdColsPerWave = 4;  // backward tile: 4 columns per wavefront
// columns per forward tile: 16, 32, 64 or 128; rows per backward tile: 256,
// 512 or 1024 (compile-time extents of the sweep kernels).  A requested
// extent of 0 lets the analysis choose one per level from the level's
// supernode shapes (tile_extents_for_level).
inline bool valid_fwd_cols(int c) { return c == 16 || c == 32 || c == 64 || c == 128; }
inline bool valid_bwd_rows(int r) { return r == 256 || r == 512 || r == 1024; }
inline bool valid_bwd_cols(int c) { return c == 16 || c == 32 || c == 64; }

// Geometric nested dissection on the node graph, supernodes = ND blocks,
// relaxed (dense) supernodal structure from the assembly tree.
std::string analyse(const Pattern &P, const double *X, int32_t leaf_nodes, int32_t fwd_cols,
                    int32_t fwd_groups, int32_t bwd_rows, int32_t bwd_cols, Symbolic &S);

// ------------------------------------------- GPU factorisation plan
// One frontal matrix of the GPU multifrontal factorisation.  The front is
// eliminated with an augmented block X (m x nc, row-major, starts as the
// identity on the own rows): the row operations of the elimination turn it
// into [L11^{-1}; -L21 L11^{-1}], i.e. the explicit-inverse panel.
// Storage is split by lifetime: the own columns of F, X and W are needed
// only while the front's level is processed (a per-level arena), the update
// block (rows and columns >= nc) until the parent's extend-add.
struct GfFront {
  int32_t m, nc;       // front order and eliminated columns
  int64_t offF;        // own columns: m x nc column-major FP64 (lower part used)
  int64_t offU;        // update block: (m - nc) x (m - nc) column-major (lower)
  int64_t offX;        // m x nc row-major FP64 augmented block
  int64_t offW;        // m x kGfPanel column-major FP64 panel scratch
  int64_t rows_off;    // panel rows (DOF indices), as Symbolic::rows
  int64_t panel_off;   // output panel offset, as Supernode::dev_off
  int32_t ld, pad;     // output panel leading dimension, as Supernode::ld
};
// Square output tile of an update, kGfStepTile (regions 0/1) or kGfTile
// (regions 2-5; kGfStepTile where a launch would hold too few of them) wide
// (L: the front's scaled lower factor, d: its pivots, W = L D for the
// current panel, X: augmented block; the own columns are taken in blocks of
// kGfBlock, [K0, Ke) the block of the panel, Ke = min(K0 + kGfBlock, nc)):
//   region 0  F[i, j] -= sum_{k in panel} L[i, k] W[j, k]   k1 <= j < Ke, i >= j
//   region 1  X[i, j] -= sum_{k in panel} L[i, k] X[k, j]   k1 <= i < Ke, j < k1
//   region 4  F[i, j] -= sum_{K0 <= k < Ke} L[i, k] d_k L[j, k]   Ke <= j < nc, i >= j
//   region 5  X[i, j] -= sum_{K0 <= k < Ke} L[i, k] X[k, j]       Ke <= i < nc, j < Ke
//   region 2  F[i, j] -= sum_{k < nc} L[i, k] d_k L[j, k]   nc <= j <= i (Schur)
//   region 3  X[i, j] -= sum_{k < nc} L[i, k] X[k, j]       i >= nc, j < nc
// Regions 0/1 run after each panel step, 4/5 after the last panel step of a
// block, 2/3 once the own columns are done.
struct GfTile {
  int32_t s, region, i0, j0;
};
struct GfExt {         // 32 x 32 tile of a child's update matrix (extend-add)
  int32_t child, i0, j0, pad;
};
constexpr int kGfPanel = 64;   // panel width of the GPU factorisation
constexpr int kGfTile = 128;   // trailing-update tile (Schur complements)
constexpr int kGfStepTile = 64; // update tile of the panel steps (K = 64:
                                // smaller tiles, more of them in flight)
constexpr int kGfSchurMinTiles = 1024;  // fewer large Schur tiles than this
                                        // in a level: the level uses 64-wide
constexpr int kGfBlock = 256;  // own-column block of the panel steps (regions 4/5)
static_assert(kGfBlock % kGfTile == 0 && kGfBlock % kGfPanel == 0,
              "block updates cover whole tiles and whole panels");

struct GfPlan {
  std::vector<GfFront> fr;                   // by supernode
  int64_t doubles = 0;                       // front storage (FP64 entries)
  int64_t level_doubles = 0;                 // per-level arena (own columns, X, W)
  int64_t update_doubles = 0;                // update blocks (first fit)
  std::vector<int32_t> lvl_sn, lvl_ptr;      // supernodes of each level
  std::vector<int32_t> a_csr;                // A scatter: CSR slot ...
  std::vector<int64_t> a_off, a_ptr;         // ... -> front entry; per-level ranges
  std::vector<int32_t> parent;               // supernode -> parent (or -1)
  std::vector<int32_t> rel;                  // child struct row -> parent front row
  std::vector<int64_t> rel_off;              // by supernode, into rel
  std::vector<GfExt> ext;                    // extend-add tiles, by parent level
  std::vector<int64_t> ext_ptr;              //   and child rank: ext_pass bounds the
  std::vector<int64_t> ext_pass;             //   passes, ext_lvl_pass[L] is level L's
  std::vector<int32_t> ext_lvl_pass;         //   first pass (one child per parent)
  std::vector<int32_t> step_k0;              // panel steps: k0 of each step
  std::vector<int32_t> step_level;           // level of each step
  std::vector<int32_t> panel_sn;             // fronts with nc > k0, per step
  std::vector<int64_t> panel_ptr;
  std::vector<GfTile> upd;                   // update tiles (regions 0-5)
  std::vector<int64_t> upd_lo, upd_hi;       // regions 0/1 of each step
  std::vector<int64_t> blk_lo, blk_hi;       // regions 4/5 after each step (may be empty),
  std::vector<int32_t> blk_k0, blk_tile;     //   their block start K0 and tile width
  std::vector<int64_t> schur_lo, schur_hi;   // regions 2/3 of each level
  std::vector<int32_t> schur_tile;           // their tile width (per level)
  std::vector<int32_t> lvl_step_ptr;         // steps of each level
  double flops = 0.0;
};

std::string gpu_plan(const Pattern &P, const Symbolic &S, GfPlan &G);

// ------------------------------------------------------- numeric factor
// Parallel-for helper (dynamic scheduling on std::threads).
void parallel_for(int64_t n, int n_threads, const std::function<void(int64_t, int)> &fn);

// FP64 numeric factorisation of A (CSR values in the pattern's order,
// float or double) with the symbolic structure S.  Output per supernode:
// G_s = [L11^{-1}; L21 L11^{-1}] (m x nc, column-major) at panel_off in
// `panels`, and dinv[dof] = 1 / D for every free DOF (1 for fixed DOFs).
// Returns "" or an error message (non-positive pivot).
template <typename TA>
std::string factorize(const Pattern &P, const Symbolic &S, const TA *A, int n_threads,
                      std::vector<double> &panels, std::vector<double> &dinv);

}  // namespace fe
