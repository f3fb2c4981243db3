// Symbolic analysis (host): fill-reducing ordering, supernodes, the row
// structure of L, the factor storage layout and the gather/scatter maps.
//
// Paper, Sec. II.B: step 1 reorders rows and columns to reduce the fill of
// the LDL^T factor; step 2 (symbolic factorization) finds the nonzero
// locations of L; the elimination tree (eq. parent) has nodes that are blocks
// of contiguous columns (supernodes), traversed leaves-to-root by the
// factorization and root-to-leaves by selected inversion.
//
// Design (one GPU, batched shifts):
//   * nested dissection on the atom-block graph (geometric bisection when
//     coordinates are given, else level-structure bisection), leaves of at
//     most leaf_cols columns;
//   * every separator and every leaf is one supernode whose diagonal block is
//     stored dense; its rows below are the union of the column structures
//     (a relaxed supernodal pattern that contains the exact pattern of L);
//   * supernode J is stored as a dense column-major |E_J| x w_J panel, E_J =
//     its own columns followed by its sorted rows below;
//   * for every supernode a column map and per-segment relative row
//     positions locate any lower element (i, q) of E_J x E_J in the storage of
//     the supernode that owns column E_J[q] -- the scatter target of the
//     factor update and the gather source of selected inversion.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "pxs_internal.h"

namespace pxs {
namespace {

struct BlockGraph {
  int32_t nv = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  std::vector<int32_t> wgt;  // columns per block
};

class NestedDissection {
 public:
  NestedDissection(const BlockGraph& g, const double* coords, int leaf_cols, int sep_cols)
      : g_(g), coords_(coords), leaf_(leaf_cols), sep_(sep_cols), mark_(g.nv, -1), level_(g.nv, -1) {}

  // Appends the block order to `order` and one entry per supernode (its
  // blocks, in order) to `snodes`.
  void run(std::vector<int32_t>& order, std::vector<std::vector<int32_t>>& snodes) {
    order_ = &order;
    snodes_ = &snodes;
    std::vector<int32_t> all(g_.nv);
    std::iota(all.begin(), all.end(), 0);
    recurse(all, 0);
  }

 private:
  const BlockGraph& g_;
  const double* coords_;
  int leaf_;
  int sep_;
  std::vector<int32_t> mark_, level_;
  int32_t stamp_ = 0;
  std::vector<int32_t>* order_ = nullptr;
  std::vector<std::vector<int32_t>>* snodes_ = nullptr;

  int64_t weight(const std::vector<int32_t>& v) const {
    int64_t w = 0;
    for (int32_t x : v) w += g_.wgt[x];
    return w;
  }

  void emit(const std::vector<int32_t>& v) {
    if (v.empty()) return;
    for (int32_t x : v) order_->push_back(x);
    snodes_->push_back(v);
  }

  // A separator wider than sep_ columns becomes several supernodes of at
  // most sep_ columns, cut in slabs along its longest extent (coordinates)
  // or in its current order.  Each piece's rows below are the union of its
  // own columns' structures, which along a separator grow from the first
  // column to the last: one supernode over the whole separator stores the
  // last column's structure for every column.
  void emit_separator(std::vector<int32_t>& sep) {
    if (sep_ <= 0 || weight(sep) <= sep_) {
      emit(sep);
      return;
    }
    if (coords_) {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int32_t v : sep)
        for (int d = 0; d < 3; ++d) {
          lo[d] = std::min(lo[d], coords_[3 * v + d]);
          hi[d] = std::max(hi[d], coords_[3 * v + d]);
        }
      int ax = 0;
      for (int d = 1; d < 3; ++d)
        if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
      std::stable_sort(sep.begin(), sep.end(), [&](int32_t a, int32_t b) {
        return coords_[3 * a + ax] < coords_[3 * b + ax];
      });
    }
    std::vector<int32_t> piece;
    int64_t w = 0;
    for (int32_t v : sep) {
      if (!piece.empty() && w + g_.wgt[v] > sep_) {
        emit(piece);
        piece.clear();
        w = 0;
      }
      piece.push_back(v);
      w += g_.wgt[v];
    }
    emit(piece);
  }

  // BFS inside the vertex subset tagged with `tag`; returns visit order and
  // fills level_ for visited vertices.
  std::vector<int32_t> bfs(int32_t src, int32_t tag) {
    std::vector<int32_t> q;
    q.push_back(src);
    level_[src] = 0;
    mark_[src] = tag + 1;  // visited marker = tag + 1
    for (size_t h = 0; h < q.size(); ++h) {
      int32_t v = q[h];
      for (int64_t p = g_.xadj[v]; p < g_.xadj[v + 1]; ++p) {
        int32_t u = g_.adj[p];
        if (mark_[u] == tag) {
          mark_[u] = tag + 1;
          level_[u] = level_[v] + 1;
          q.push_back(u);
        }
      }
    }
    return q;
  }

  void recurse(std::vector<int32_t> verts, int depth) {
    if (verts.empty()) return;
    if (weight(verts) <= leaf_ || verts.size() <= 1 || depth > 200) {
      emit(verts);
      return;
    }
    std::vector<int32_t> L, R;
    bool have_split = coords_ ? split_geometric(verts, L, R) : split_graph(verts, L, R);
    if (!have_split) {
      emit(verts);
      return;
    }
    // vertex separator: the smaller of the two boundary layers
    int32_t tagL = (stamp_ += 2), tagR = (stamp_ += 2);
    for (int32_t v : L) mark_[v] = tagL;
    for (int32_t v : R) mark_[v] = tagR;
    std::vector<int32_t> bL, bR;
    int64_t wbL = 0, wbR = 0;
    for (int32_t v : L) {
      for (int64_t p = g_.xadj[v]; p < g_.xadj[v + 1]; ++p)
        if (mark_[g_.adj[p]] == tagR) { bL.push_back(v); wbL += g_.wgt[v]; break; }
    }
    for (int32_t v : R) {
      for (int64_t p = g_.xadj[v]; p < g_.xadj[v + 1]; ++p)
        if (mark_[g_.adj[p]] == tagL) { bR.push_back(v); wbR += g_.wgt[v]; break; }
    }
    std::vector<int32_t> sep;
    if (!bL.empty() || !bR.empty()) {
      const bool useL = (wbL <= wbR);
      sep = useL ? bL : bR;
      int32_t tagS = (stamp_ += 2);
      for (int32_t v : sep) mark_[v] = tagS;
      std::vector<int32_t>& side = useL ? L : R;
      std::vector<int32_t> keep;
      for (int32_t v : side)
        if (mark_[v] != tagS) keep.push_back(v);
      side.swap(keep);
    }
    if (L.empty() && R.empty()) {
      emit(sep);
      return;
    }
    recurse(std::move(L), depth + 1);
    recurse(std::move(R), depth + 1);
    emit_separator(sep);
  }

  bool split_geometric(std::vector<int32_t>& verts, std::vector<int32_t>& L,
                       std::vector<int32_t>& R) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : verts)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], coords_[3 * v + d]);
        hi[d] = std::max(hi[d], coords_[3 * v + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    if (!(hi[ax] > lo[ax])) return false;
    std::stable_sort(verts.begin(), verts.end(), [&](int32_t a, int32_t b) {
      double ca = coords_[3 * a + ax], cb = coords_[3 * b + ax];
      if (ca != cb) return ca < cb;
      return a < b;
    });
    const int64_t half = weight(verts) / 2;
    int64_t acc = 0;
    size_t cut = 0;
    while (cut < verts.size() && acc + g_.wgt[verts[cut]] <= half) acc += g_.wgt[verts[cut++]];
    if (cut == 0) cut = 1;
    // keep atoms at the same coordinate on one side
    while (cut < verts.size() && cut > 0 &&
           coords_[3 * verts[cut] + ax] == coords_[3 * verts[cut - 1] + ax])
      ++cut;
    if (cut >= verts.size()) {
      cut = 0;
      acc = 0;
      while (cut < verts.size() && acc + g_.wgt[verts[cut]] <= half) acc += g_.wgt[verts[cut++]];
      if (cut == 0) cut = 1;
      while (cut > 0 && coords_[3 * verts[cut] + ax] == coords_[3 * verts[cut - 1] + ax]) --cut;
      if (cut == 0) return false;
    }
    L.assign(verts.begin(), verts.begin() + cut);
    R.assign(verts.begin() + cut, verts.end());
    return true;
  }

  bool split_graph(std::vector<int32_t>& verts, std::vector<int32_t>& L, std::vector<int32_t>& R) {
    int32_t tag = (stamp_ += 2);
    for (int32_t v : verts) mark_[v] = tag;
    // pseudo-peripheral start: two sweeps
    std::vector<int32_t> q = bfs(verts[0], tag);
    int32_t far = q.back();
    for (int32_t v : verts) mark_[v] = tag;
    q = bfs(far, tag);
    if (q.size() < verts.size()) {
      // disconnected: the reached component against the rest, no separator
      int32_t vis = tag + 1;
      L.clear();
      R.clear();
      for (int32_t v : verts) (mark_[v] == vis ? L : R).push_back(v);
      std::sort(L.begin(), L.end(), [&](int32_t a, int32_t b) { return level_[a] < level_[b] || (level_[a] == level_[b] && a < b); });
      return !L.empty() && !R.empty();
    }
    // order by level, cut at half the weight: levels below, levels above;
    // the boundary layer becomes the separator
    std::stable_sort(q.begin(), q.end(), [&](int32_t a, int32_t b) { return level_[a] < level_[b]; });
    const int64_t half = weight(q) / 2;
    int64_t acc = 0;
    size_t cut = 0;
    while (cut < q.size() && acc + g_.wgt[q[cut]] <= half) acc += g_.wgt[q[cut++]];
    if (cut == 0) cut = 1;
    // move the cut to a level boundary
    int32_t lev = level_[q[cut - 1]];
    while (cut < q.size() && level_[q[cut]] == lev) ++cut;
    if (cut >= q.size()) {
      cut = 0;
      while (cut < q.size() && level_[q[cut]] < lev) ++cut;
      if (cut == 0) return false;
    }
    L.assign(q.begin(), q.begin() + cut);
    R.assign(q.begin() + cut, q.end());
    return true;
  }
};

bool validate_csc(int32_t n, const int64_t* colptr, const int32_t* rowind, std::string& msg) {
  if (n <= 0) { msg = "n must be positive"; return false; }
  if (colptr[0] != 0) { msg = "colptr[0] != 0"; return false; }
  for (int32_t j = 0; j < n; ++j) {
    if (colptr[j + 1] < colptr[j] + 1) { msg = "column " + std::to_string(j) + " is empty"; return false; }
    if (rowind[colptr[j]] != j) { msg = "column " + std::to_string(j) + " lacks its diagonal entry first"; return false; }
    for (int64_t p = colptr[j] + 1; p < colptr[j + 1]; ++p) {
      if (rowind[p] <= rowind[p - 1]) { msg = "rows not strictly increasing in column " + std::to_string(j); return false; }
      if (rowind[p] >= n) { msg = "row index out of range in column " + std::to_string(j); return false; }
    }
  }
  return true;
}

}  // namespace

int analyze(int32_t n, const int64_t* colptr, const int32_t* rowind, int32_t nblk,
            const int32_t* blkptr, const double* coords, const AnalyzeOptions& opt, Symbolic& S,
            std::string& msg) {
  if (!validate_csc(n, colptr, rowind, msg)) return -1;
  const int64_t nnz = colptr[n];
  // blocks
  std::vector<int32_t> bptr;
  if (blkptr) {
    if (nblk <= 0 || blkptr[0] != 0 || blkptr[nblk] != n) { msg = "bad blkptr"; return -1; }
    for (int32_t b = 0; b < nblk; ++b)
      if (blkptr[b + 1] <= blkptr[b]) { msg = "blkptr not strictly increasing"; return -1; }
    bptr.assign(blkptr, blkptr + nblk + 1);
  } else {
    if (coords && nblk != n) { msg = "coords without blkptr need nblk == n"; return -1; }
    nblk = n;
    bptr.resize(n + 1);
    std::iota(bptr.begin(), bptr.end(), 0);
  }
  std::vector<int32_t> blk_of(n);
  for (int32_t b = 0; b < nblk; ++b)
    for (int32_t c = bptr[b]; c < bptr[b + 1]; ++c) blk_of[c] = b;

  // block graph (symmetric, no self loops)
  BlockGraph g;
  g.nv = nblk;
  g.wgt.resize(nblk);
  for (int32_t b = 0; b < nblk; ++b) g.wgt[b] = bptr[b + 1] - bptr[b];
  {
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve((size_t)nnz / 4 + 16);
    for (int32_t j = 0; j < n; ++j) {
      int32_t bj = blk_of[j];
      int32_t last = -1;
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        int32_t bi = blk_of[rowind[p]];
        if (bi != bj && bi != last) {
          e.emplace_back(bi, bj);
          e.emplace_back(bj, bi);
          last = bi;
        }
      }
    }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    g.xadj.assign(nblk + 1, 0);
    for (auto& x : e) g.xadj[x.first + 1]++;
    for (int32_t b = 0; b < nblk; ++b) g.xadj[b + 1] += g.xadj[b];
    g.adj.resize(e.size());
    for (size_t t = 0; t < e.size(); ++t) g.adj[t] = e[t].second;
  }

  // ordering + supernode partition (both at block level)
  std::vector<int32_t> border;
  std::vector<std::vector<int32_t>> sblocks;
  if (opt.ordering == 1) {
    // natural order; supernodes = runs of at most leaf_cols columns
    std::vector<int32_t> cur;
    int64_t w = 0;
    for (int32_t b = 0; b < nblk; ++b) {
      if (!cur.empty() && w + g.wgt[b] > opt.leaf_cols) {
        sblocks.push_back(cur);
        cur.clear();
        w = 0;
      }
      cur.push_back(b);
      w += g.wgt[b];
      border.push_back(b);
    }
    if (!cur.empty()) sblocks.push_back(cur);
  } else {
    NestedDissection nd(g, coords, std::max(1, opt.leaf_cols), opt.sep_cols);
    nd.run(border, sblocks);
  }
  if ((int32_t)border.size() != nblk) { msg = "internal: ordering lost blocks"; return -1; }

  // new block index, block sizes in new order, new column numbering
  std::vector<int32_t> bnew(nblk);
  for (int32_t t = 0; t < nblk; ++t) bnew[border[t]] = t;
  std::vector<int32_t> nbptr(nblk + 1, 0);  // first new column of new block t
  for (int32_t t = 0; t < nblk; ++t) nbptr[t + 1] = nbptr[t] + g.wgt[border[t]];
  S.n = n;
  S.nnz_lower = nnz;
  S.perm.resize(n);
  S.iperm.resize(n);
  for (int32_t t = 0; t < nblk; ++t) {
    int32_t ob = border[t];
    for (int32_t c = 0; c < g.wgt[ob]; ++c) {
      S.perm[nbptr[t] + c] = bptr[ob] + c;
      S.iperm[bptr[ob] + c] = nbptr[t] + c;
    }
  }
  // supernodes in new block ranges
  const int32_t ns = (int32_t)sblocks.size();
  std::vector<int32_t> sbfirst(ns + 1, 0);  // first new block of each supernode
  {
    int32_t t = 0;
    for (int32_t J = 0; J < ns; ++J) {
      sbfirst[J] = t;
      for (int32_t ob : sblocks[J]) {
        if (bnew[ob] != t) { msg = "internal: supernode blocks not contiguous"; return -1; }
        ++t;
      }
    }
    sbfirst[ns] = t;
  }
  std::vector<int32_t> snode_of_blk(nblk);
  for (int32_t J = 0; J < ns; ++J)
    for (int32_t t = sbfirst[J]; t < sbfirst[J + 1]; ++t) snode_of_blk[t] = J;

  // new-order block adjacency (upper part: neighbours with larger index)
  std::vector<std::vector<int32_t>> nadj(nblk);
  for (int32_t ob = 0; ob < nblk; ++ob) {
    int32_t t = bnew[ob];
    for (int64_t p = g.xadj[ob]; p < g.xadj[ob + 1]; ++p) {
      int32_t u = bnew[g.adj[p]];
      if (u > t) nadj[t].push_back(u);
    }
  }

  // supernodal symbolic factorization at block level: below-block sets C_J
  std::vector<std::vector<int32_t>> Cb(ns);
  std::vector<std::vector<int32_t>> children(ns);
  S.sparent.assign(ns, -1);
  {
    std::vector<int32_t> mark(nblk, -1);
    for (int32_t J = 0; J < ns; ++J) {
      const int32_t last = sbfirst[J + 1];
      std::vector<int32_t>& C = Cb[J];
      for (int32_t t = sbfirst[J]; t < last; ++t)
        for (int32_t u : nadj[t])
          if (u >= last && mark[u] != J) { mark[u] = J; C.push_back(u); }
      for (int32_t K : children[J])
        for (int32_t u : Cb[K])
          if (u >= last && mark[u] != J) { mark[u] = J; C.push_back(u); }
      std::sort(C.begin(), C.end());
      if (!C.empty()) {
        int32_t P = snode_of_blk[C[0]];
        S.sparent[J] = P;
        children[P].push_back(J);
      }
    }
  }

  // Panels cut every supernode into column blocks of panel_width (the
  // numeric kernels' unit); pbase[J] is the index of J's first panel.
  const int32_t pwid = std::max(1, std::min(64, opt.panel_width));
  std::vector<int64_t> pbase(ns + 1, 0);
  for (int32_t J = 0; J < ns; ++J) {
    const int32_t w = nbptr[sbfirst[J + 1]] - nbptr[sbfirst[J]];
    pbase[J + 1] = pbase[J] + (w + pwid - 1) / pwid;
  }
  S.xm_panel.assign((size_t)pbase[ns], PanelMacs{});
  S.xm_update.assign(ns, 0.0);

  // exact block-level pattern of L (block elimination tree) for the flop
  // model and nnz(L): struct(t) = upper neighbours of t plus the structures
  // of its block-etree children, minus t itself.  The structure of column k
  // of block t is then the later columns of t plus every column of the
  // blocks in struct(t).
  //
  // Along the way the exact multiply-adds of every column are split by the
  // kernel that performs them (per shift; c = a + g + e off-diagonal
  // nonzeros of column k: a inside k's panel, g in the later panels of its
  // supernode, e below the supernode, b = g + e):
  //   factor  c(c+1)/2 = a(a+1)/2 [diagonal block] + a b [panel TRSM]
  //           + g(g+1)/2 + g e [internal updates of the later panels]
  //           + e(e+1)/2 [the supernode's update of its ancestors],
  //   SelInv  c^2 + c = b^2 [Z_BB times L-hat] + 2 a b [diagonal-block
  //           partials] + a^2 + a + b [diagonal block in LDS].
  {
    std::vector<std::vector<int32_t>> st(nblk);
    std::vector<std::vector<int32_t>> ch(nblk);
    std::vector<int32_t> mark(nblk, -1);
    std::vector<int64_t> rs, re, rc;   // ranges of struct(t) and their cumulative sizes
    double ff = 0.0, fs = 0.0;
    int64_t nnzx = 0;
    for (int32_t t = 0; t < nblk; ++t) {
      std::vector<int32_t>& s = st[t];
      for (int32_t u : nadj[t])
        if (mark[u] != t) { mark[u] = t; s.push_back(u); }
      for (int32_t c : ch[t]) {
        for (int32_t u : st[c])
          if (u > t && mark[u] != t) { mark[u] = t; s.push_back(u); }
        std::vector<int32_t>().swap(st[c]);
      }
      std::sort(s.begin(), s.end());
      int64_t below = 0;
      rs.clear();
      re.clear();
      rc.clear();
      for (int32_t u : s) {
        rs.push_back(nbptr[u]);
        re.push_back(nbptr[u + 1]);
        rc.push_back(below);
        below += nbptr[u + 1] - nbptr[u];
      }
      const int32_t o = nbptr[t + 1] - nbptr[t];
      for (int32_t c = 0; c < o; ++c) {
        double ck = (double)(o - 1 - c) + (double)below;
        ff += 8.0 * ck * (ck + 1.0) / 2.0;
        fs += 8.0 * (ck * ck + ck);
        nnzx += (int64_t)ck + 1;
      }
      // rows of struct(t)'s blocks below x
      auto fbelow = [&](int64_t x) -> int64_t {
        const size_t i = (size_t)(std::lower_bound(rs.begin(), rs.end(), x) - rs.begin());
        if (i == 0) return 0;
        return rc[i - 1] + std::min(x, re[i - 1]) - rs[i - 1];
      };
      const int32_t J = snode_of_blk[t];
      const int64_t sj0 = nbptr[sbfirst[J]], sj1 = nbptr[sbfirst[J + 1]];
      const int64_t bend = nbptr[t + 1];
      for (int64_t k = nbptr[t]; k < bend; ++k) {
        // structure rows of column k in [lo, hi)
        auto cnt = [&](int64_t lo, int64_t hi) -> double {
          if (hi <= lo) return 0.0;
          const int64_t inb = std::max<int64_t>(0, std::min(hi, bend) - std::max(lo, k + 1));
          return (double)(inb + fbelow(hi) - fbelow(lo));
        };
        const int64_t q = (k - sj0) / pwid;
        const int64_t fe = std::min(sj0 + (q + 1) * pwid, sj1);
        const double ck = (double)(bend - 1 - k) + (double)below;
        const double a = cnt(k + 1, fe), g = cnt(fe, sj1), e = ck - a - g, b = g + e;
        PanelMacs& pm = S.xm_panel[(size_t)(pbase[J] + q)];
        pm.diag += 0.5 * a * (a + 1.0);
        pm.trsm += a * b;
        pm.off += b * b;
        pm.sdiag += 2.0 * a * b;
        pm.sfinal += a * a + a + b;
        S.xm_update[J] += 0.5 * e * (e + 1.0);
        const int64_t nq = pbase[J + 1] - pbase[J];
        for (int64_t q2 = q + 1; q2 < nq; ++q2) {
          const int64_t f2 = sj0 + q2 * pwid, fe2 = std::min(f2 + pwid, sj1);
          const double s2 = cnt(f2, fe2);
          if (s2 > 0.0) S.xm_panel[(size_t)(pbase[J] + q2)].intu += 0.5 * s2 * (s2 + 1.0) + s2 * cnt(fe2, INT64_MAX / 4);
        }
      }
      if (!s.empty()) ch[s[0]].push_back(t);
    }
    S.flops_factor = ff;
    S.flops_selinv = fs;
    S.nnzL_exact = nnzx;
  }

  // scalar supernodes: columns, row lists, storage
  S.nsuper = ns;
  S.sfirst.resize(ns + 1);
  for (int32_t J = 0; J <= ns; ++J) S.sfirst[J] = nbptr[sbfirst[J]];
  S.snode_of_col.resize(n);
  for (int32_t J = 0; J < ns; ++J)
    for (int32_t c = S.sfirst[J]; c < S.sfirst[J + 1]; ++c) S.snode_of_col[c] = J;
  S.rowptr.assign(ns + 1, 0);
  S.ld.resize(ns);
  S.off.resize(ns);
  S.rows.clear();
  int64_t offs = 0, lower = 0;
  int32_t maxld = 0;
  for (int32_t J = 0; J < ns; ++J) {
    S.rowptr[J] = (int64_t)S.rows.size();
    for (int32_t c = S.sfirst[J]; c < S.sfirst[J + 1]; ++c) S.rows.push_back(c);
    for (int32_t u : Cb[J])
      for (int32_t c = nbptr[u]; c < nbptr[u + 1]; ++c) S.rows.push_back(c);
    const int32_t w = S.sfirst[J + 1] - S.sfirst[J];
    const int32_t l = (int32_t)((int64_t)S.rows.size() - S.rowptr[J]);
    S.ld[J] = l;
    S.off[J] = offs;
    offs += (int64_t)l * w;
    lower += (int64_t)w * (w + 1) / 2 + (int64_t)(l - w) * w;
    maxld = std::max(maxld, l);
  }
  S.rowptr[ns] = (int64_t)S.rows.size();
  S.nnzL_store = offs;
  S.nnzL_stored_lower = lower;
  S.max_front = maxld;

  // maps
  const int64_t nrows_total = S.rowptr[ns];
  S.colmap.assign(nrows_total, 0);
  S.colseg.assign(nrows_total, 0);
  S.relpos.clear();
  // shared identity segment for a supernode's own columns
  for (int32_t i = 0; i < maxld; ++i) S.relpos.push_back(i);
  for (int32_t J = 0; J < ns; ++J) {
    const int64_t rb = S.rowptr[J];
    const int32_t w = S.sfirst[J + 1] - S.sfirst[J];
    const int32_t l = S.ld[J];
    for (int32_t q = 0; q < w; ++q) {
      S.colmap[rb + q] = S.off[J] + (int64_t)q * l;
      S.colseg[rb + q] = 0;
    }
    int32_t q = w;
    while (q < l) {
      const int32_t A = S.snode_of_col[S.rows[rb + q]];
      int32_t qe = q;
      while (qe < l && S.snode_of_col[S.rows[rb + qe]] == A) ++qe;
      // positions in E_A of E_J[q .. l)
      const int64_t base = (int64_t)S.relpos.size();
      const int64_t ra = S.rowptr[A];
      const int32_t la = S.ld[A];
      int32_t pa = 0;
      for (int32_t i = q; i < l; ++i) {
        const int32_t r = S.rows[rb + i];
        while (pa < la && S.rows[ra + pa] < r) ++pa;
        if (pa >= la || S.rows[ra + pa] != r) {
          msg = "internal: row structure not nested in ancestor";
          return -1;
        }
        S.relpos.push_back(pa);
      }
      for (int32_t t = q; t < qe; ++t) {
        const int32_t col = S.rows[rb + t];
        S.colmap[rb + t] = S.off[A] + (int64_t)(col - S.sfirst[A]) * la;
        S.colseg[rb + t] = base - q;
      }
      q = qe;
    }
  }
  // input entries -> storage offsets
  S.entry_off.resize(nnz);
  S.entry_diag.resize(nnz);
  for (int32_t j = 0; j < n; ++j) {
    for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
      const int32_t a = S.iperm[rowind[p]], b = S.iperm[j];
      const int32_t lo = std::min(a, b), hi = std::max(a, b);
      const int32_t J = S.snode_of_col[lo];
      const int64_t rb = S.rowptr[J];
      const int32_t* first = S.rows.data() + rb;
      const int32_t* lastp = first + S.ld[J];
      const int32_t* it = std::lower_bound(first, lastp, hi);
      if (it == lastp || *it != hi) { msg = "internal: entry outside the pattern of L"; return -1; }
      S.entry_off[p] = S.off[J] + (int64_t)(lo - S.sfirst[J]) * S.ld[J] + (it - first);
      // 1: diagonal; 2: the entry's transpose is what is stored (its new
      // row index precedes its new column index); 0: stored as given
      S.entry_diag[p] = (rowind[p] == j) ? 1 : (a < b ? 2 : 0);
    }
  }

  // panels
  S.panel_width = std::max(1, std::min(64, opt.panel_width));
  S.pivot_tol = opt.pivot_tol;
  S.panels.clear();
  S.max_below = 0;
  S.max_split = 1;
  for (int32_t J = 0; J < ns; ++J) {
    const int32_t w = S.sfirst[J + 1] - S.sfirst[J];
    for (int32_t p0 = 0; p0 < w; p0 += S.panel_width) {
      Panel P;
      P.J = J;
      P.p0 = p0;
      P.wp = std::min(S.panel_width, w - p0);
      P.nb_rows = S.ld[J] - p0 - P.wp;
      S.max_below = std::max<int64_t>(S.max_below, P.nb_rows);
      S.max_split = std::max(S.max_split, split_count(P.nb_rows));
      S.panels.push_back(P);
    }
  }
  if (S.panels.size() != S.xm_panel.size()) { msg = "internal: panel count"; return -1; }
  // workspace (bytes): per shift the SelInv panel product L_hat
  // (max_below x panel_width complex), the split-K partials of the diagonal
  // block update (max_split x 64 x 64 complex) and the shift, weight and
  // status scalars; fixed: reduction partials.
  const int64_t pw = S.panel_width;
  S.work_per_shift = 16 * (S.max_below * pw + (int64_t)S.max_split * 64 * 64) + 16 * 8 + 256;
  S.work_per_shift = (S.work_per_shift + 255) / 256 * 256;
  S.work_fixed = 1 << 20;
  S.max_below_super = 0;
  for (int32_t J = 0; J < ns; ++J)
    S.max_below_super = std::max(S.max_below_super, S.ld[J] - (S.sfirst[J + 1] - S.sfirst[J]));
  S.gather_per_shift = (16 * (int64_t)S.max_below_super * S.max_below_super + 255) / 256 * 256;

  // streams for selected inversion: walking the supernodal tree from the
  // roots, a node's heaviest child stays on its stream, further children
  // open new streams while there are free ones, else join the least loaded
  {
    const int NS = std::max(1, std::min(8, opt.selinv_streams));
    std::vector<double> work(ns, 0.0), sub(ns, 0.0);
    for (const Panel& P : S.panels) work[P.J] += (double)P.nb_rows * P.nb_rows * P.wp;
    for (int32_t J = 0; J < ns; ++J) {
      sub[J] += work[J];
      if (S.sparent[J] >= 0) sub[S.sparent[J]] += sub[J];
    }
    S.sel_stream.assign(ns, 0);
    S.cross_child.assign(ns, 0);
    std::vector<double> load(NS, 0.0);
    int used = 0;
    std::vector<int32_t> roots;
    for (int32_t J = ns - 1; J >= 0; --J)
      if (S.sparent[J] < 0) roots.push_back(J);
    auto pick = [&](double w) {
      int s = 0;
      if (used < NS) {
        s = used++;
      } else {
        for (int t = 1; t < NS; ++t)
          if (load[t] < load[s]) s = t;
      }
      load[s] += w;
      return s;
    };
    for (int32_t r : roots) S.sel_stream[r] = pick(sub[r]);
    for (int32_t J = ns - 1; J >= 0; --J) {
      std::vector<int32_t> kids = children[J];
      std::sort(kids.begin(), kids.end(), [&](int32_t a, int32_t b) { return sub[a] > sub[b]; });
      for (size_t q = 0; q < kids.size(); ++q) {
        if (q == 0) {
          S.sel_stream[kids[q]] = S.sel_stream[J];
        } else {
          load[S.sel_stream[J]] -= sub[kids[q]];
          S.sel_stream[kids[q]] = pick(sub[kids[q]]);
        }
        if (S.sel_stream[kids[q]] != S.sel_stream[J]) S.cross_child[J] = 1;
      }
    }
    S.sel_nstreams = std::max(1, used);
    S.gather_bytes.assign(S.sel_nstreams, 0);
    for (int32_t J = 0; J < ns; ++J) {
      const int64_t c = S.ld[J] - (S.sfirst[J + 1] - S.sfirst[J]);
      int64_t& g = S.gather_bytes[S.sel_stream[J]];
      g = std::max(g, (16 * c * c + 255) / 256 * 256);
    }
  }
  {
    // factorization issue order (children are numbered before parents)
    std::vector<int32_t> height(ns, 0);
    for (int32_t J = 0; J < ns; ++J)
      if (S.sparent[J] >= 0) height[S.sparent[J]] = std::max(height[S.sparent[J]], height[J] + 1);
    S.fac_order.resize(ns);
    std::iota(S.fac_order.begin(), S.fac_order.end(), 0);
    std::stable_sort(S.fac_order.begin(), S.fac_order.end(),
                     [&](int32_t a, int32_t b) { return height[a] < height[b]; });
    std::vector<int32_t> seq(ns);
    for (int32_t i = 0; i < ns; ++i) seq[S.fac_order[i]] = i;
    S.fac_child.assign(ns, -1);
    for (int32_t J = 0; J < ns; ++J) {
      const int32_t q = S.sparent[J];
      if (q >= 0 && (S.fac_child[q] < 0 || seq[J] > seq[S.fac_child[q]])) S.fac_child[q] = J;
    }
  }
  S.selinv_chunk = std::max(0, opt.selinv_chunk);
  // Subtree lanes fused on one stream: on request, or, by default, when the
  // average supernode carries under FUSE_FLOPS_PER_SUPER flops per shift --
  // trees of many small supernodes (1D chains), whose launches are short
  // and latency-bound: one fused grid per step halves their density-matrix
  // time, while systems of a few large supernodes run at the same speed or
  // 1-3% slower (measured over 64 chain, sheet and bulk systems)
  if (opt.fused_lanes != 0) {
    S.fused_lanes = opt.fused_lanes > 0 ? 1 : 0;
  } else {
    const double per = (S.flops_factor + S.flops_selinv) / std::max(1, ns);
    S.fused_lanes = per < FUSE_FLOPS_PER_SUPER ? 1 : 0;
  }
  S.tile_rows = (opt.tile_rows == 128) ? 128 : 64;
  return 0;
}

}  // namespace pxs
