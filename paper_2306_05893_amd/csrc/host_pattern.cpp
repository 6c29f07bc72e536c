// CSR pattern of A and the element-to-nonzero map, built the way the paper's
// "build matrix pattern" stage does it (Sec. 4.2, Table "build pattern"):
//
//   triplet keys in fill order  --(counting sort by column)-->  X^T in the
//   "uncompressed structure" (rows of X^T sorted and compressed, entries in
//   fill order)  --(counting sort by row)-->  X in the uncompressed structure
//   (rows and columns sorted, duplicates adjacent)  --(merge)-->  CSR + map.
//
// Projective constraints (Sec. 6.1) are applied while the map is built: the
// first transpose skips triplets whose column is fixed, the second skips
// triplets whose row is fixed, and each fixed row becomes a lone 1 on the
// diagonal.  The fill order is element-major: element e, local row
// i = 3a + r, local column j = 3b + c, row-major over (i, j).
#include "host.hpp"

#include <algorithm>
#include <cstdio>
#include <numeric>

namespace fe {

std::string build_pattern(int32_t n_nodes, int32_t n_elems, int32_t nen,
                          const int32_t *conn, const uint8_t *fixed_dof, Pattern &P) {
  if (n_nodes <= 0 || n_elems <= 0) return "empty mesh";
  if (nen != 4 && nen != 8) return "element type must be TET4 or HEX8";
  const int64_t n = 3LL * n_nodes;
  if (n > INT32_MAX / 2) return "too many DOFs for int32 indices";
  for (int64_t k = 0; k < (int64_t)n_elems * nen; ++k)
    if (conn[k] < 0 || conn[k] >= n_nodes) return "connectivity index out of range";

  P = Pattern();
  P.n_nodes = n_nodes;
  P.n_elems = n_elems;
  P.nen = nen;
  P.n = n;
  P.conn.assign(conn, conn + (int64_t)n_elems * nen);
  P.fixed.assign(n, 0);
  if (fixed_dof)
    for (int64_t d = 0; d < n; ++d) P.fixed[d] = fixed_dof[d] ? 1 : 0;
  for (int64_t d = 0; d < n; ++d)
    if (P.fixed[d]) P.fixed_dofs.push_back((int32_t)d);

  const int ne = 3 * nen;                 // element DOFs
  const int64_t per_elem = (int64_t)ne * ne;
  const int64_t T = per_elem * n_elems;   // triplets
  if (T > INT32_MAX) return "too many triplets for int32 indices";
  auto key_row = [&](int64_t t) {
    const int64_t e = t / per_elem, ij = t % per_elem;
    const int i = (int)(ij / ne);
    return 3 * conn[e * nen + i / 3] + i % 3;
  };
  auto key_col = [&](int64_t t) {
    const int64_t e = t / per_elem, ij = t % per_elem;
    const int j = (int)(ij % ne);
    return 3 * conn[e * nen + j / 3] + j % 3;
  };

  // ---- transpose 1: X -> X^T (count per column, skipping fixed columns)
  std::vector<int64_t> ptr1(n + 1, 0);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t c = key_col(t);
    if (!P.fixed[c]) ++ptr1[c + 1];
  }
  for (int64_t c = 0; c < n; ++c) ptr1[c + 1] += ptr1[c];
  const int64_t T1 = ptr1[n];
  hvec<int32_t> t1_row(T1);   // row of X for each entry of X^T
  hvec<int32_t> t1_id(T1);    // triplet index (fill order)
  {
    std::vector<int64_t> fill(ptr1.begin(), ptr1.end() - 1);
    for (int64_t t = 0; t < T; ++t) {
      const int32_t c = key_col(t);
      if (P.fixed[c]) continue;
      const int64_t pos = fill[c]++;
      t1_row[pos] = key_row(t);
      t1_id[pos] = (int32_t)t;
    }
  }

  // ---- transpose 2: X^T -> X (count per row, skipping fixed rows); walking
  // X^T row by row (= column by column of X) makes each row's columns sorted.
  std::vector<int64_t> ptr2(n + 1, 0);
  for (int64_t k = 0; k < T1; ++k)
    if (!P.fixed[t1_row[k]]) ++ptr2[t1_row[k] + 1];
  for (int64_t r = 0; r < n; ++r) ptr2[r + 1] += ptr2[r];
  const int64_t T2 = ptr2[n];
  hvec<int32_t> t2_col(T2);
  hvec<int32_t> t2_id(T2);
  {
    std::vector<int64_t> fill(ptr2.begin(), ptr2.end() - 1);
    for (int64_t c = 0; c < n; ++c)
      for (int64_t k = ptr1[c]; k < ptr1[c + 1]; ++k) {
        const int32_t r = t1_row[k];
        if (P.fixed[r]) continue;
        const int64_t pos = fill[r]++;
        t2_col[pos] = (int32_t)c;
        t2_id[pos] = t1_id[k];
      }
  }
  hvec<int32_t>().swap(t1_row);
  hvec<int32_t>().swap(t1_id);

  // ---- merge duplicates into CSR and record the map
  P.tmap.assign(T, -1);
  P.row_ptr.assign(n + 1, 0);
  P.col_idx.clear();
  P.col_idx.reserve(T2 / 4 + n);
  P.fixed_diag_slot.reserve(P.fixed_dofs.size());
  for (int64_t r = 0; r < n; ++r) {
    if (P.fixed[r]) {
      P.fixed_diag_slot.push_back((int32_t)P.col_idx.size());
      P.col_idx.push_back((int32_t)r);
    } else {
      int32_t last = -1;
      for (int64_t k = ptr2[r]; k < ptr2[r + 1]; ++k) {
        if (t2_col[k] != last) {
          last = t2_col[k];
          P.col_idx.push_back(last);
        }
        P.tmap[t2_id[k]] = (int32_t)(P.col_idx.size() - 1);
      }
    }
    if (P.col_idx.size() > (size_t)INT32_MAX) return "nnz exceeds int32 range";
    if (P.col_idx.size() == (size_t)P.row_ptr[r])
      return "a free DOF belongs to no element (its row of A would be empty)";
    P.row_ptr[r + 1] = (int32_t)P.col_idx.size();
  }

  // ---- compact 1-byte slot map (node-level Dirichlet only)
  P.node_fixed.assign(n_nodes, 0);
  bool node_level = true;
  for (int32_t i = 0; i < n_nodes; ++i) {
    const int s = P.fixed[3 * i] + P.fixed[3 * i + 1] + P.fixed[3 * i + 2];
    if (s == 3) P.node_fixed[i] = 1;
    else if (s != 0) node_level = false;
  }
  P.compact_ok = false;
  if (node_level) {
    const int nn = nen * nen;
    P.slot.assign((size_t)n_elems * nn, 0xFF);
    bool ok = true;
    for (int64_t e = 0; e < n_elems && ok; ++e)
      for (int a = 0; a < nen && ok; ++a)
        for (int b = 0; b < nen && ok; ++b) {
          const int32_t ga = conn[e * nen + a], gb = conn[e * nen + b];
          const int64_t t0 = e * per_elem + (int64_t)(3 * a) * ne + 3 * b;
          if (P.node_fixed[ga] || P.node_fixed[gb]) {
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) ok &= P.tmap[t0 + r * ne + c] == -1;
            continue;
          }
          const int64_t k0 = P.tmap[t0] - P.row_ptr[3 * ga];
          if (k0 < 0 || k0 % 3 != 0 || k0 / 3 > 254) { ok = false; break; }
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
              ok &= P.tmap[t0 + r * ne + c] == P.row_ptr[3 * ga + r] + (int32_t)k0 + c;
          P.slot[e * nn + a * nen + b] = (uint8_t)(k0 / 3);
        }
    P.compact_ok = ok;
    if (!ok) std::vector<uint8_t>().swap(P.slot);
  }

  // ---- inverse of the compact map: contributions per node block
  if (P.compact_ok) {
    std::vector<int32_t> blk0(n_nodes + 1, 0);  // first block of each row node
    for (int32_t g = 0; g < n_nodes; ++g)
      blk0[g + 1] = blk0[g] + (P.node_fixed[g] ? 0 : (P.row_ptr[3 * g + 1] - P.row_ptr[3 * g]) / 3);
    const int32_t nb = blk0[n_nodes];
    P.blk_pos.resize(nb);
    P.blk_node.resize(nb);
    for (int32_t g = 0; g < n_nodes; ++g)
      for (int32_t k = blk0[g]; k < blk0[g + 1]; ++k) {
        const int32_t pos = P.row_ptr[3 * g] + 3 * (k - blk0[g]);
        P.blk_pos[k] = pos;
        const bool diag = P.col_idx[pos] == 3 * g;
        P.blk_node[k] = (int32_t)((uint32_t)g | (diag ? 0x80000000u : 0u));
      }
    const int nn = nen * nen;
    P.blk_ptr.assign(nb + 1, 0);
    for (int64_t e = 0; e < n_elems; ++e)
      for (int ab = 0; ab < nn; ++ab) {
        const uint8_t s = P.slot[e * nn + ab];
        if (s != 0xFF) ++P.blk_ptr[blk0[conn[e * nen + ab / nen]] + s + 1];
      }
    for (int32_t k = 0; k < nb; ++k) P.blk_ptr[k + 1] += P.blk_ptr[k];
    P.blk_src.resize(P.blk_ptr[nb]);
    std::vector<int32_t> fill(P.blk_ptr.begin(), P.blk_ptr.end() - 1);
    for (int64_t e = 0; e < n_elems; ++e)
      for (int ab = 0; ab < nn; ++ab) {
        const uint8_t s = P.slot[e * nn + ab];
        if (s != 0xFF) P.blk_src[fill[blk0[conn[e * nen + ab / nen]] + s]++] = (int32_t)(e * nn + ab);
      }
  }
  return "";
}

}  // namespace fe
