// Nested-dissection ordering, supernodal symbolic structure and the GPU
// schedules of the triangular solves (paper Sec. 5.1).
//
// The paper reorders L with nested dissection so that the two diagonal
// domains a and b of Eq. "regional problem" can be solved independently and
// only the separator c depends on both; it recurses until the blocks are
// small, and assigns each block a parallelisation level.  Here the partition
// is geometric (the node coordinates are known): a block is split at the
// median along its longest axis and the boundary layer of one side against
// the other (the smaller of the two) is the vertex separator.  Every ND block
// (leaf domain or separator) becomes one supernode whose diagonal block is
// stored dense; its off-diagonal rows are the ancestor DOFs reached through
// the assembly tree, struct(s) = (adj(own(s)) U struct(children)) restricted
// to later columns.  The level of a supernode is its height above the leaves:
// all supernodes of one level are independent in both sweeps.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace fe {

namespace {

// Node adjacency of the mesh (every element couples all of its nodes).
void node_graph(const Pattern &P, std::vector<int64_t> &ptr, std::vector<int32_t> &adj) {
  const int32_t N = P.n_nodes, nen = P.nen;
  const int64_t E = P.n_elems;
  std::vector<int64_t> eptr(N + 1, 0);
  for (int64_t k = 0; k < E * nen; ++k) ++eptr[P.conn[k] + 1];
  for (int32_t i = 0; i < N; ++i) eptr[i + 1] += eptr[i];
  std::vector<int32_t> elems(eptr[N]);
  {
    std::vector<int64_t> fill(eptr.begin(), eptr.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int a = 0; a < nen; ++a) elems[fill[P.conn[e * nen + a]]++] = (int32_t)e;
  }
  ptr.assign(N + 1, 0);
  adj.clear();
  std::vector<int32_t> mark(N, -1);
  for (int32_t i = 0; i < N; ++i) {
    const size_t start = adj.size();
    for (int64_t k = eptr[i]; k < eptr[i + 1]; ++k) {
      const int64_t e = elems[k];
      for (int a = 0; a < nen; ++a) {
        const int32_t j = P.conn[e * nen + a];
        if (j != i && mark[j] != i) {
          mark[j] = i;
          adj.push_back(j);
        }
      }
    }
    std::sort(adj.begin() + start, adj.end());
    ptr[i + 1] = (int64_t)adj.size();
  }
}

struct NDTree {
  std::vector<std::vector<int32_t>> own;   // nodes owned by each tree node
  std::vector<int32_t> ch0, ch1;           // children, -1 = none
};

struct Dissector {
  const std::vector<int64_t> &ptr;
  const std::vector<int32_t> &adj;
  const double *X;
  int32_t leaf;
  NDTree T;
  std::vector<int32_t> side;  // scratch: 0 unset, 1 = A, 2 = B
  std::vector<int32_t> stamp;
  int32_t stamp_val = 0;

  Dissector(const std::vector<int64_t> &p, const std::vector<int32_t> &a, const double *x,
            int32_t lf, int32_t N)
      : ptr(p), adj(a), X(x), leaf(lf), side(N, 0), stamp(N, -1) {}

  int32_t make(std::vector<int32_t> own, int32_t c0, int32_t c1) {
    T.own.push_back(std::move(own));
    T.ch0.push_back(c0);
    T.ch1.push_back(c1);
    return (int32_t)T.own.size() - 1;
  }

  int32_t dissect(std::vector<int32_t> &S, int depth) {
    if (S.empty()) return -1;
    if ((int32_t)S.size() <= leaf || depth > 60) {
      std::sort(S.begin(), S.end());
      return make(std::move(S), -1, -1);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : S)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], X[3 * v + c]);
        hi[c] = std::max(hi[c], X[3 * v + c]);
      }
    int axes[3] = {0, 1, 2};
    std::sort(axes, axes + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    for (int ai = 0; ai < 3; ++ai) {
      const int ax = axes[ai];
      std::vector<double> c(S.size());
      for (size_t k = 0; k < S.size(); ++k) c[k] = X[3 * S[k] + ax];
      std::nth_element(c.begin(), c.begin() + c.size() / 2, c.end());
      const double med = c[c.size() / 2];
      // nodes within a small tolerance of the median plane go to B, so a
      // structured grid plane becomes the separator
      const double tol = 1e-9 * std::max(1e-300, hi[ax] - lo[ax]);
      std::vector<int32_t> A, B;
      for (int32_t v : S) (X[3 * v + ax] < med - tol ? A : B).push_back(v);
      if (A.empty() || B.empty()) continue;
      for (int32_t v : A) side[v] = 1;
      for (int32_t v : B) side[v] = 2;
      std::vector<int32_t> sepB, sepA, restA, restB;
      for (int32_t v : B) {
        bool touch = false;
        for (int64_t k = ptr[v]; k < ptr[v + 1] && !touch; ++k) touch = side[adj[k]] == 1;
        (touch ? sepB : restB).push_back(v);
      }
      for (int32_t v : A) {
        bool touch = false;
        for (int64_t k = ptr[v]; k < ptr[v + 1] && !touch; ++k) touch = side[adj[k]] == 2;
        (touch ? sepA : restA).push_back(v);
      }
      for (int32_t v : S) side[v] = 0;
      std::vector<int32_t> sep, p0, p1;
      if (sepB.size() <= sepA.size()) {
        sep = std::move(sepB);
        p0 = std::move(A);
        p1 = std::move(restB);
      } else {
        sep = std::move(sepA);
        p0 = std::move(restA);
        p1 = std::move(B);
      }
      if (sep.size() == S.size()) continue;
      S.clear();
      S.shrink_to_fit();
      const int32_t c0 = dissect(p0, depth + 1);
      const int32_t c1 = dissect(p1, depth + 1);
      std::sort(sep.begin(), sep.end());
      return make(std::move(sep), c0, c1);
    }
    std::sort(S.begin(), S.end());
    return make(std::move(S), -1, -1);
  }
};

}  // namespace

// Tiles of the many-right-hand-side sweeps.  Forward: one tile per 64 panel
// rows, contracting over the own columns that row block can touch (all nc
// for update rows, up to the diagonal for own rows).  Backward: one tile per
// 64 own columns, contracting over the panel rows from that column block
// down.  A level whose tiles are too few to fill the GPU has its contractions
// cut into pieces (multiples of the 16-wide staging chunk, at least 64 long)
// until it has about 512 tiles.
// Sweep tile extents of one level where the caller left them to the
// analysis (0).
//  * Forward columns: a level whose supernodes mostly have 65..128 own
//    columns takes 128-column tiles, one per row block instead of two
//    64-column tiles whose second is mostly empty, which halves the level's
//    tiles, input gathers and output atomics; other levels keep 64 (128
//    doubles the panel registers of a thread and so halves the tiles in
//    flight).
//  * Forward column groups: a level of wide supernodes (256-column tiles pad
//    its own columns by at most 10 % more than 64-column ones, and it keeps
//    kSweepMinTiles tiles) takes 4 groups of 64 columns per tile, whose row
//    sums meet in one atomic per row: a quarter of the atomics (forward
//    levels 8-12 of the hex block 3-4 % faster; on narrow supernodes the
//    empty groups only cost).
//  * Backward rows: 256-row tiles where they cover the level's panel rows
//    with clearly less padding than 512-row tiles (supernodes of a few
//    hundred rows), else 512.
//  * Backward columns: the widest of 64 and 32 (16 and 8 wavefronts sharing
//    the tile's gathered inputs) that pads the level's own columns by at
//    most 5 % more than 32 does and still gives the level kSweepMinTiles
//    workgroups (4 per compute unit), else 16: a small level is bound by the
//    latency of its tiles, and fewer, wider tiles only lengthen it (the
//    14,883-DOF beam ran 6 % slower with them).
// On the 1.39 M-DOF hex block: forward levels 2 and 3 100 -> 81 and 79 ->
// 67 us, backward level 2 113 -> 93 us; the backward sweep 2.22 -> 2.02 ms
// with 32-column instead of 16-column tiles, and about 0.03 ms less with 64
// columns on its wide levels.
constexpr double kSweepMinTiles = 1024;
static void tile_extents_for_level(const Symbolic &S, const std::vector<int32_t> &sns,
                                   int32_t &fwd_cols, int32_t &fwd_groups, int32_t &bwd_rows,
                                   int32_t &bwd_cols) {
  if (fwd_cols == 0) {
    size_t mid = 0;
    for (int32_t s : sns) mid += S.sn[s].nc > 64 && S.sn[s].nc <= 128;
    fwd_cols = 2 * mid >= sns.size() && !sns.empty() ? 128 : 64;
  }
  if (fwd_cols != 64) {
    fwd_groups = 1;  // column groups are groups of 64 columns
  } else if (fwd_groups == 0) {
    double pad64 = 0, pad256 = 0, tiles256 = 0;
    for (int32_t s : sns) {
      const double c = S.sn[s].nc, rb = std::ceil(S.sn[s].m / (double)kFwdRows);
      pad64 += 64.0 * std::ceil(c / 64.0);
      pad256 += 256.0 * std::ceil(c / 256.0);
      tiles256 += rb * std::ceil(c / 256.0);
    }
    fwd_groups = pad256 <= 1.1 * pad64 && tiles256 >= kSweepMinTiles ? 4 : 1;
  }
  if (bwd_rows == 0) {
    double m = 0, pad256 = 0, pad512 = 0;
    for (int32_t s : sns) {
      const double r = S.sn[s].m;
      m += r;
      pad256 += 256.0 * std::ceil(r / 256.0);
      pad512 += 512.0 * std::ceil(r / 512.0);
    }
    // fill(256) > 1.1 fill(512)  <=>  1.1 pad256 < pad512
    bwd_rows = m > 0 && 1.1 * pad256 < pad512 ? 256 : 512;
  }
  if (bwd_cols == 0) {
    double pad32 = 0, pad64 = 0, tiles32 = 0, tiles64 = 0;
    for (int32_t s : sns) {
      const double c = S.sn[s].nc, rb = std::ceil(S.sn[s].m / (double)bwd_rows);
      pad32 += 32.0 * std::ceil(c / 32.0);
      pad64 += 64.0 * std::ceil(c / 64.0);
      tiles32 += rb * std::ceil(c / 32.0);
      tiles64 += rb * std::ceil(c / 64.0);
    }
    // wide tiles only where the level still has kSweepMinTiles of them
    if (pad64 <= 1.05 * pad32 && tiles64 >= kSweepMinTiles) bwd_cols = 64;
    else if (tiles32 >= kSweepMinTiles) bwd_cols = 32;
    else bwd_cols = 16;
  }
}

static void build_multi_tiles(Symbolic &S, const std::vector<std::vector<int32_t>> &by_level) {
  constexpr int kTarget = 256, kMinChunk = 128, kStage = 32;
  const int nl = (int)by_level.size();
  struct Base { int32_t s, b0, lo, hi; };
  auto emit = [&](const std::vector<Base> &base, std::vector<MTile> &out) {
    int64_t longest = 0;
    for (const Base &b : base) longest = std::max<int64_t>(longest, b.hi - b.lo);
    int64_t chunk = std::max<int64_t>(longest, kMinChunk);
    auto count = [&](int64_t ch) {
      int64_t k = 0;
      for (const Base &b : base) k += (b.hi - b.lo + ch - 1) / ch;
      return k;
    };
    while (count(chunk) < kTarget && chunk > kMinChunk)
      chunk = std::max<int64_t>(kMinChunk, (chunk / 2 + kStage - 1) / kStage * kStage);
    for (const Base &b : base)
      for (int64_t lo = b.lo; lo < b.hi; lo += chunk)
        out.push_back({b.s, b.b0, (int32_t)lo, (int32_t)std::min<int64_t>(b.hi, lo + chunk)});
  };
  S.mfwd_tiles.clear();
  S.mbwd_tiles.clear();
  S.mfwd_level_ptr.assign(1, 0);
  S.mbwd_level_ptr.assign(1, 0);
  S.level_lower.assign(nl, 0.0);
  for (int L = 0; L < nl; ++L) {
    std::vector<Base> base;
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      S.level_lower[L] += (double)sn.m * sn.nc - 0.5 * (double)sn.nc * (sn.nc - 1);
      for (int32_t r0 = 0; r0 < sn.m; r0 += kMultiRows)
        base.push_back({s, r0, 0, r0 < sn.nc ? std::min(sn.nc, r0 + kMultiRows) : sn.nc});
    }
    emit(base, S.mfwd_tiles);
    S.mfwd_level_ptr.push_back((int32_t)S.mfwd_tiles.size());
  }
  S.mbwd_dofs.clear();
  S.mbwd_dof_ptr.assign(1, 0);
  for (int L = nl - 1; L >= 0; --L) {
    std::vector<Base> base;
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      for (int32_t j0 = 0; j0 < sn.nc; j0 += kMultiRows) base.push_back({s, j0, j0, sn.m});
      for (int32_t j = 0; j < sn.nc; ++j) S.mbwd_dofs.push_back(S.rows[sn.rows_off + j]);
    }
    emit(base, S.mbwd_tiles);
    S.mbwd_level_ptr.push_back((int32_t)S.mbwd_tiles.size());
    S.mbwd_dof_ptr.push_back((int32_t)S.mbwd_dofs.size());
  }
}

std::string analyse(const Pattern &P, const double *X, int32_t leaf_nodes, int32_t fwd_cols,
                    int32_t fwd_groups, int32_t bwd_rows, int32_t bwd_cols, Symbolic &S) {
  if (leaf_nodes <= 0) leaf_nodes = 48;
  if (fwd_groups < 0 || fwd_groups == 3 || fwd_groups > 4 ||
      (fwd_groups > 1 && fwd_cols != 0 && fwd_cols != 64))
    return "forward column groups: 0 (chosen per level), 1, 2 or 4 (groups of 64 columns)";
  if (fwd_cols < 0 || bwd_rows < 0 || bwd_cols < 0 || (fwd_cols && !valid_fwd_cols(fwd_cols)) ||
      (bwd_rows && !valid_bwd_rows(bwd_rows)) || (bwd_cols && !valid_bwd_cols(bwd_cols)))
    return "tile extents: forward width 0, 16, 32, 64 or 128; backward height 0, 256, 512 or "
           "1024; backward width 0, 16, 32 or 64 (0: chosen per level)";
  const int32_t N = P.n_nodes;
  S = Symbolic();
  S.n = P.n;

  std::vector<int64_t> gptr;
  std::vector<int32_t> gadj;
  node_graph(P, gptr, gadj);

  // active nodes: at least one free DOF
  std::vector<int32_t> active;
  for (int32_t i = 0; i < N; ++i)
    if (!(P.fixed[3 * i] && P.fixed[3 * i + 1] && P.fixed[3 * i + 2])) active.push_back(i);

  Dissector D(gptr, gadj, X, leaf_nodes, N);
  const int32_t root = D.dissect(active, 0);
  NDTree &T = D.T;

  // post-order of the ND tree; supernodes = tree nodes with own nodes
  const int32_t nt = (int32_t)T.own.size();
  std::vector<int32_t> order;
  order.reserve(nt);
  std::vector<int32_t> tree_parent(nt, -1);
  for (int32_t t = 0; t < nt; ++t) {
    if (T.ch0[t] >= 0) tree_parent[T.ch0[t]] = t;
    if (T.ch1[t] >= 0) tree_parent[T.ch1[t]] = t;
  }
  if (root >= 0) {
    std::vector<std::pair<int32_t, int>> st{{root, 0}};
    while (!st.empty()) {
      auto &[t, state] = st.back();
      if (state == 0) {
        state = 1;
        if (T.ch0[t] >= 0) st.push_back({T.ch0[t], 0});
      } else if (state == 1) {
        state = 2;
        if (T.ch1[t] >= 0) st.push_back({T.ch1[t], 0});
      } else {
        order.push_back(t);
        st.pop_back();
      }
    }
  }
  std::vector<int32_t> tree2sn(nt, -1);
  std::vector<int32_t> sn_tree;
  for (int32_t t : order)
    if (!T.own[t].empty()) {
      tree2sn[t] = (int32_t)sn_tree.size();
      sn_tree.push_back(t);
    }
  const int32_t ns = (int32_t)sn_tree.size();

  // node positions in elimination order
  std::vector<int32_t> node_pos(N, INT32_MAX);
  {
    int32_t pos = 0;
    for (int32_t t : sn_tree)
      for (int32_t v : T.own[t]) node_pos[v] = pos++;
  }

  // DOF permutation: each supernode's own nodes' free DOFs, in order
  S.iperm.assign(P.n, -1);
  S.sn.assign(ns, Supernode());
  S.sn_ptr.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    S.sn_ptr[s] = (int32_t)S.perm.size();
    for (int32_t v : T.own[sn_tree[s]])
      for (int c = 0; c < 3; ++c)
        if (!P.fixed[3 * v + c]) {
          S.iperm[3 * v + c] = (int32_t)S.perm.size();
          S.perm.push_back(3 * v + c);
        }
  }
  S.sn_ptr[ns] = (int32_t)S.perm.size();
  S.n_free = (int64_t)S.perm.size();
  for (int64_t d = 0; d < P.n; ++d)
    if (P.fixed[d]) {
      S.iperm[d] = (int32_t)S.perm.size();
      S.perm.push_back((int32_t)d);
    }

  // supernode tree: parent = nearest ancestor tree node that is a supernode
  S.children.assign(ns, {});
  for (int32_t s = 0; s < ns; ++s) {
    int32_t t = tree_parent[sn_tree[s]];
    while (t >= 0 && tree2sn[t] < 0) t = tree_parent[t];
    S.sn[s].parent = t >= 0 ? tree2sn[t] : -1;
    if (S.sn[s].parent >= 0) S.children[S.sn[s].parent].push_back(s);
  }

  // struct sets at node level, in post-order (children before parents)
  std::vector<std::vector<int32_t>> snode_struct(ns);
  std::vector<int32_t> mark(N, -1);
  int64_t panel = 0, lower = 0, dev_panel = 0;
  double flops = 0.0;
  S.rows.clear();
  for (int32_t s = 0; s < ns; ++s) {
    const auto &own = T.own[sn_tree[s]];
    int32_t last = -1;
    for (int32_t v : own) last = std::max(last, node_pos[v]);
    std::vector<int32_t> st;
    auto add = [&](int32_t u) {
      if (node_pos[u] > last && node_pos[u] != INT32_MAX && mark[u] != s) {
        mark[u] = s;
        st.push_back(u);
      }
    };
    for (int32_t v : own)
      for (int64_t k = gptr[v]; k < gptr[v + 1]; ++k) add(gadj[k]);
    for (int32_t c : S.children[s]) {
      for (int32_t u : snode_struct[c]) add(u);
      std::vector<int32_t>().swap(snode_struct[c]);
    }
    std::sort(st.begin(), st.end(), [&](int32_t a, int32_t b) { return node_pos[a] < node_pos[b]; });
    Supernode &sn = S.sn[s];
    sn.first = S.sn_ptr[s];
    sn.nc = S.sn_ptr[s + 1] - S.sn_ptr[s];
    sn.rows_off = (int64_t)S.rows.size();
    for (int32_t k = S.sn_ptr[s]; k < S.sn_ptr[s + 1]; ++k) S.rows.push_back(S.perm[k]);
    for (int32_t u : st)
      for (int c = 0; c < 3; ++c)
        if (!P.fixed[3 * u + c]) S.rows.push_back(3 * u + c);
    sn.m = (int32_t)((int64_t)S.rows.size() - sn.rows_off);
    sn.panel_off = panel;
    panel += (int64_t)sn.m * sn.nc;
    sn.ld = (sn.m + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
    sn.dev_off = dev_panel;
    dev_panel += (int64_t)sn.ld * sn.nc;
    lower += (int64_t)sn.m * sn.nc - (int64_t)sn.nc * (sn.nc - 1) / 2;
    // partial LDL^T + explicit inverse of L11 + W = L21 L11^{-1}
    const double m = sn.m, nc = sn.nc, nr = sn.m - sn.nc;
    flops += nc * m * m - m * nc * nc + nc * nc * nc / 3.0;  // ~ sum_k (m - k)^2
    flops += nc * nc * nc / 3.0 + 2.0 * nr * nc * nc;
    snode_struct[s] = std::move(st);
  }
  S.panel_entries = panel;
  S.dev_panel_entries = dev_panel;
  S.lower_entries = lower;
  S.flops = flops;

  // levels = height above the leaves
  int32_t nl = 0;
  for (int32_t s = 0; s < ns; ++s) {
    int32_t h = 0;
    for (int32_t c : S.children[s]) h = std::max(h, S.sn[c].level + 1);
    S.sn[s].level = h;
    nl = std::max(nl, h + 1);
  }
  S.n_levels = nl;

  // tile schedules
  std::vector<std::vector<int32_t>> by_level(nl);
  for (int32_t s = 0; s < ns; ++s) by_level[S.sn[s].level].push_back(s);
  S.fwd_tiles.clear();
  S.bwd_tiles.clear();
  S.fwd_level_ptr.assign(1, 0);
  S.bwd_level_ptr.assign(1, 0);
  S.fwd_level_cols.assign(nl, fwd_cols);
  S.fwd_level_groups.assign(nl, fwd_groups);
  S.bwd_level_rows.assign(nl, bwd_rows);
  S.bwd_level_cols.assign(nl, bwd_cols);
  for (int32_t L = 0; L < nl; ++L)
    tile_extents_for_level(S, by_level[L], S.fwd_level_cols[L], S.fwd_level_groups[L],
                           S.bwd_level_rows[L], S.bwd_level_cols[L]);
  for (int32_t L = 0; L < nl; ++L) {
    const int32_t fwd_cols_L = S.fwd_level_cols[L] * S.fwd_level_groups[L];
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      for (int32_t r0 = 0; r0 < sn.m; r0 += kFwdRows)
        for (int32_t c0 = 0; c0 < sn.nc; c0 += fwd_cols_L) {
          const int32_t r1 = std::min(sn.m, r0 + kFwdRows);
          if (r1 <= c0) continue;  // entirely above the diagonal of L11^{-1}
          S.fwd_tiles.push_back({s, r0, c0, 0});
        }
    }
    S.fwd_level_ptr.push_back((int32_t)S.fwd_tiles.size());
  }
  for (int32_t L = nl - 1; L >= 0; --L) {
    const int32_t bwd_rows_L = S.bwd_level_rows[L], bwd_cols_L = S.bwd_level_cols[L];
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      for (int32_t c0 = 0; c0 < sn.nc; c0 += bwd_cols_L)
        for (int32_t r0 = 0; r0 < sn.m; r0 += bwd_rows_L) {
          const int32_t r1 = std::min(sn.m, r0 + bwd_rows_L);
          if (r1 <= c0) continue;
          S.bwd_tiles.push_back({s, r0, c0, 0});
        }
    }
    S.bwd_level_ptr.push_back((int32_t)S.bwd_tiles.size());
  }
  build_multi_tiles(S, by_level);
  return "";
}

}  // namespace fe
