// Static plan of the GPU multifrontal factorisation: front storage, the A
// scatter lists, the extend-add index maps and tiles, and the per-panel-step
// tile lists of the trailing updates.  Built once per topology from the
// supernodal structure (the same assembly tree as the host factorisation).
#include <algorithm>
#include <map>

#include "host.hpp"

namespace fe {

namespace {

// Order the MFMA tiles [lo, end) of one front in super-blocks of 8 x 8 tiles
// (super-block columns, then super-block rows, then tile columns and rows):
// the update launches give each XCD runs of 64 consecutive tiles, which then
// share 8 row slabs and 8 column slabs of their operands in its L2.
void group_tiles(std::vector<GfTile> &upd, size_t lo, int32_t t) {
  const int32_t g = 8 * t;
  std::stable_sort(upd.begin() + lo, upd.end(), [g](const GfTile &a, const GfTile &b) {
    if (a.region != b.region) return a.region < b.region;
    if (a.j0 / g != b.j0 / g) return a.j0 / g < b.j0 / g;
    if (a.i0 / g != b.i0 / g) return a.i0 / g < b.i0 / g;
    if (a.j0 != b.j0) return a.j0 < b.j0;
    return a.i0 < b.i0;
  });
}

}  // namespace

std::string gpu_plan(const Pattern &P, const Symbolic &S, GfPlan &G) {
  G = GfPlan();
  const int32_t ns = (int32_t)S.sn.size();
  const int32_t nl = S.n_levels;
  G.fr.resize(ns);
  G.parent.resize(ns);
  std::vector<std::vector<int32_t>> by_level(nl);
  for (int32_t s = 0; s < ns; ++s) by_level[S.sn[s].level].push_back(s);

  // Storage.  The per-level arena holds the own columns of F, X and W of
  // the level's fronts (the next level reuses it: the launches are stream
  // ordered).  An update block lives from its front's level to its parent's
  // extend-add; blocks are placed first fit, allocated at the start of their
  // level and released once the parent level's extend-add has read them.
  auto round = [](int64_t x) { return (x + 31) / 32 * 32; };
  G.lvl_ptr.assign(1, 0);
  int64_t arena = 0;
  for (int32_t L = 0; L < nl; ++L) {
    int64_t cur = 0;
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      GfFront &f = G.fr[s];
      f.m = sn.m;
      f.nc = sn.nc;
      f.offF = cur;
      cur += round((int64_t)sn.m * sn.nc);
      f.offX = cur;
      cur += round((int64_t)sn.m * sn.nc);
      f.offW = cur;
      cur += round((int64_t)sn.m * kGfPanel);
      f.rows_off = sn.rows_off;
      f.panel_off = sn.dev_off;
      f.ld = sn.ld;
      G.lvl_sn.push_back(s);
      G.parent[s] = sn.parent;
    }
    arena = std::max(arena, cur);
    G.lvl_ptr.push_back((int32_t)G.lvl_sn.size());
  }
  std::map<int64_t, int64_t> free_blocks;  // offset -> size, coalesced
  int64_t top = 0;
  auto alloc = [&](int64_t n) -> int64_t {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it)
      if (it->second >= n) {
        const int64_t o = it->first, rest = it->second - n;
        free_blocks.erase(it);
        if (rest > 0) free_blocks[o + n] = rest;
        return o;
      }
    const int64_t o = top;
    top += n;
    return o;
  };
  auto release = [&](int64_t o, int64_t n) {
    auto it = free_blocks.emplace(o, n).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  };
  auto ublock = [&](int32_t s) { return round((int64_t)(S.sn[s].m - S.sn[s].nc) * (S.sn[s].m - S.sn[s].nc)); };
  for (int32_t L = 0; L < nl; ++L) {
    for (int32_t s : by_level[L]) G.fr[s].offU = arena + alloc(std::max<int64_t>(ublock(s), 32));
    for (int32_t s : by_level[L])
      for (int32_t c : S.children[s]) release(G.fr[c].offU - arena, std::max<int64_t>(ublock(c), 32));
  }
  G.level_doubles = arena;
  G.update_doubles = top;
  G.doubles = arena + top;

  // front position of every panel row, per supernode (DOF -> row)
  std::vector<int32_t> pos(P.n, -1);

  // extend-add maps: child struct row ii -> position in the parent's front
  G.rel_off.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    G.rel_off[s] = (int64_t)G.rel.size();
    const int32_t p = S.sn[s].parent;
    if (p < 0) continue;
    const Supernode &ps = S.sn[p];
    const int32_t *prow = S.rows.data() + ps.rows_off;
    for (int32_t i = 0; i < ps.m; ++i) pos[prow[i]] = i;
    const Supernode &cs = S.sn[s];
    const int32_t *crow = S.rows.data() + cs.rows_off;
    for (int32_t ii = cs.nc; ii < cs.m; ++ii) {
      const int32_t q = pos[crow[ii]];
      if (q < 0) return "child row missing from the parent front";
      G.rel.push_back(q);
    }
    for (int32_t i = 0; i < ps.m; ++i) pos[prow[i]] = -1;
  }
  G.rel_off[ns] = (int64_t)G.rel.size();

  G.a_ptr.assign(1, 0);
  G.ext_ptr.assign(1, 0);
  G.ext_pass.assign(1, 0);
  G.ext_lvl_pass.clear();
  G.lvl_step_ptr.assign(1, 0);
  G.panel_ptr.assign(1, 0);
  double flops = 0.0;
  for (int32_t L = 0; L < nl; ++L) {
    // A scatter: lower part of the own columns
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      const int32_t *rw = S.rows.data() + sn.rows_off;
      for (int32_t i = 0; i < sn.m; ++i) pos[rw[i]] = i;
      for (int32_t j = 0; j < sn.nc; ++j) {
        const int32_t d = rw[j];
        for (int32_t k = P.row_ptr[d]; k < P.row_ptr[d + 1]; ++k) {
          const int32_t r = pos[P.col_idx[k]];
          if (r >= j) {
            G.a_csr.push_back(k);
            G.a_off.push_back(G.fr[s].offF + (int64_t)j * sn.m + r);
          }
        }
      }
      for (int32_t i = 0; i < sn.m; ++i) pos[rw[i]] = -1;
    }
    G.a_ptr.push_back((int64_t)G.a_csr.size());
    // extend-add tiles of the children of this level's fronts, one pass per
    // child rank: within a pass every parent receives from one child only,
    // and a child's update block maps one to one into its parent's front, so
    // no two tiles of a pass add into the same entry
    G.ext_lvl_pass.push_back((int32_t)G.ext_pass.size() - 1);
    size_t maxch = 0;
    for (int32_t s : by_level[L]) maxch = std::max(maxch, S.children[s].size());
    for (size_t rank = 0; rank < maxch; ++rank) {
      for (int32_t s : by_level[L]) {
        if (rank >= S.children[s].size()) continue;
        const int32_t c = S.children[s][rank];
        const int32_t nr = S.sn[c].m - S.sn[c].nc;
        for (int32_t j0 = 0; j0 < nr; j0 += 32)
          for (int32_t i0 = j0; i0 < nr; i0 += 32) G.ext.push_back({c, i0, j0, 0});
      }
      G.ext_pass.push_back((int64_t)G.ext.size());
    }
    G.ext_ptr.push_back((int64_t)G.ext.size());
    // panel steps
    int32_t maxnc = 0;
    for (int32_t s : by_level[L]) maxnc = std::max(maxnc, S.sn[s].nc);
    for (int32_t k0 = 0; k0 < maxnc; k0 += kGfPanel) {
      G.step_k0.push_back(k0);
      G.upd_lo.push_back((int64_t)G.upd.size());
      G.step_level.push_back(L);
      const int32_t K0 = k0 / kGfBlock * kGfBlock;  // block of this panel
      for (int32_t s : by_level[L]) {
        const Supernode &sn = S.sn[s];
        if (sn.nc <= k0) continue;
        G.panel_sn.push_back(s);
        const int32_t k1 = std::min(k0 + kGfPanel, sn.nc);
        const int32_t kb = k1 - k0;
        const int32_t ke = std::min(K0 + kGfBlock, sn.nc);
        // the rest of the block's own columns (all rows below the diagonal)
        // and own rows of X; the columns and rows past the block wait for
        // the block's end, the Schur complement for the level's end
        for (int32_t j0 = k1; j0 < ke; j0 += kGfStepTile)
          for (int32_t i0 = j0; i0 < sn.m; i0 += kGfStepTile) G.upd.push_back({s, 0, i0, j0});
        for (int32_t i0 = k1; i0 < ke; i0 += kGfStepTile)
          for (int32_t j0 = 0; j0 < k1; j0 += kGfStepTile) G.upd.push_back({s, 1, i0, j0});
        const double t = sn.nc - k1;
        flops += 2.0 * kb * (t * (sn.m - k1 - t / 2.0) + t * k1);
      }
      G.panel_ptr.push_back((int64_t)G.panel_sn.size());
      G.upd_hi.push_back((int64_t)G.upd.size());
      // after the block's last panel step: the block applied to the own
      // columns and own rows of X past it (K = kGfBlock), in fronts that
      // have own columns past it
      G.blk_lo.push_back((int64_t)G.upd.size());
      G.blk_k0.push_back(K0);
      int32_t bt = kGfTile;
      if ((k0 + kGfPanel) % kGfBlock == 0) {
        const int32_t ke = K0 + kGfBlock;
        auto block_tiles = [&](int32_t t) {
          int64_t n = 0;
          for (int32_t s : by_level[L]) {
            const Supernode &sn = S.sn[s];
            if (sn.nc <= ke) continue;
            const int64_t c = (sn.nc - ke + t - 1) / t, r = (sn.m - ke + t - 1) / t;
            n += c * r - c * (c - 1) / 2 + c * (ke / t);
          }
          return n;
        };
        bt = block_tiles(kGfTile) >= kGfSchurMinTiles ? kGfTile : kGfStepTile;
        for (int32_t s : by_level[L]) {
          const Supernode &sn = S.sn[s];
          if (sn.nc <= ke) continue;
          const size_t lo = G.upd.size();
          for (int32_t j0 = ke; j0 < sn.nc; j0 += bt)
            for (int32_t i0 = j0; i0 < sn.m; i0 += bt) G.upd.push_back({s, 4, i0, j0});
          for (int32_t i0 = ke; i0 < sn.nc; i0 += bt)
            for (int32_t j0 = 0; j0 < ke; j0 += bt) G.upd.push_back({s, 5, i0, j0});
          group_tiles(G.upd, lo, bt);
        }
      }
      G.blk_tile.push_back(bt);
      G.blk_hi.push_back((int64_t)G.upd.size());
    }
    // Schur complement and struct rows of X, one pass each (K = nc), on
    // kGfTile tiles, or kGfStepTile tiles when the level has too few of the
    // large ones to fill the GPU
    auto schur_tiles = [&](int32_t t) {
      int64_t n = 0;
      for (int32_t s : by_level[L]) {
        const int64_t r = (S.sn[s].m - S.sn[s].nc + t - 1) / t, c = (S.sn[s].nc + t - 1) / t;
        n += r * (r + 1) / 2 + r * c;
      }
      return n;
    };
    const int32_t st = schur_tiles(kGfTile) >= kGfSchurMinTiles ? kGfTile : kGfStepTile;
    G.schur_tile.push_back(st);
    G.schur_lo.push_back((int64_t)G.upd.size());
    for (int32_t s : by_level[L]) {
      const Supernode &sn = S.sn[s];
      const size_t lo = G.upd.size();
      for (int32_t j0 = sn.nc; j0 < sn.m; j0 += st)
        for (int32_t i0 = j0; i0 < sn.m; i0 += st) G.upd.push_back({s, 2, i0, j0});
      for (int32_t i0 = sn.nc; i0 < sn.m; i0 += st)
        for (int32_t j0 = 0; j0 < sn.nc; j0 += st) G.upd.push_back({s, 3, i0, j0});
      group_tiles(G.upd, lo, st);
      const double r = sn.m - sn.nc, c = sn.nc;
      flops += r * r * c + r * c * c;
    }
    G.schur_hi.push_back((int64_t)G.upd.size());
    G.lvl_step_ptr.push_back((int32_t)G.step_k0.size());
  }
  G.flops = flops;
  return "";
}

}  // namespace fe
