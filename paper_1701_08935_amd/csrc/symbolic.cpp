// Host nested dissection and symbolic analysis for the multifrontal LDL^T
// (pre-factorization phase of the direct solver, Sec. 2.3).
//
// Ordering.  A box grid (rows = x + nx*y + nx*ny*z, stencil reaching only
// distance-one neighbours, which covers 7- and 27-point stencils) is cut by
// grid planes normal to its longest side; other graphs are cut by the middle
// level of a breadth-first level structure rooted at a pseudo-peripheral
// vertex.  Subdomains of at most leaf_size vertices stay whole.  Vertices are
// numbered in post-order (left subtree, right subtree, separator), so each
// front's fully summed variables are a contiguous range and its other rows
// belong to ancestors.
//
// Fronts.  struct(f) = (adjacency of f's vertices  U  struct of f's
// children) restricted to ancestors, sorted.  The extend-add map of a child
// gives, for each child struct row, its position in the parent's row list
// [own vertices..., struct...].
#include <algorithm>
#include <cstring>
#include <deque>
#include <functional>

#include "zolo_internal.h"

namespace zolo {
namespace {

struct NDNode {
  std::vector<int32_t> verts;  // original vertex ids of this node's separator / leaf
  int left = -1, right = -1;
};

class NDBuilder {
 public:
  NDBuilder(int64_t n, const int64_t* rp, const int32_t* ci, int leaf) : n_(n), rp_(rp), ci_(ci), leaf_(leaf) {}

  // Geometric: box [x0,x1) x [y0,y1) x [z0,z1).
  int box(int nx, int ny, int x0, int x1, int y0, int y1, int z0, int z1) {
    int dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
    if (dx <= 0 || dy <= 0 || dz <= 0) return -1;
    int64_t vol = (int64_t)dx * dy * dz;
    int id = (int)nodes_.size();
    nodes_.emplace_back();
    if (vol <= leaf_ || (dx == 1 && dy == 1 && dz == 1)) {
      std::vector<int32_t> v;
      v.reserve(vol);
      for (int z = z0; z < z1; ++z)
        for (int y = y0; y < y1; ++y)
          for (int x = x0; x < x1; ++x) v.push_back((int32_t)(x + (int64_t)nx * y + (int64_t)nx * ny * z));
      nodes_[id].verts = std::move(v);
      return id;
    }
    int axis = 0;
    if (dy > dx && dy >= dz) axis = 1;
    if (dz > dx && dz > dy) axis = 2;
    int lo = axis == 0 ? x0 : axis == 1 ? y0 : z0;
    int hi = axis == 0 ? x1 : axis == 1 ? y1 : z1;
    int mid = lo + (hi - lo) / 2;
    int l, r;
    std::vector<int32_t> sep;
    if (axis == 0) {
      l = box(nx, ny, x0, mid, y0, y1, z0, z1);
      r = box(nx, ny, mid + 1, x1, y0, y1, z0, z1);
      for (int z = z0; z < z1; ++z)
        for (int y = y0; y < y1; ++y) sep.push_back((int32_t)(mid + (int64_t)nx * y + (int64_t)nx * ny * z));
    } else if (axis == 1) {
      l = box(nx, ny, x0, x1, y0, mid, z0, z1);
      r = box(nx, ny, x0, x1, mid + 1, y1, z0, z1);
      for (int z = z0; z < z1; ++z)
        for (int x = x0; x < x1; ++x) sep.push_back((int32_t)(x + (int64_t)nx * mid + (int64_t)nx * ny * z));
    } else {
      l = box(nx, ny, x0, x1, y0, y1, z0, mid);
      r = box(nx, ny, x0, x1, y0, y1, mid + 1, z1);
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) sep.push_back((int32_t)(x + (int64_t)nx * y + (int64_t)nx * ny * mid));
    }
    std::sort(sep.begin(), sep.end());
    nodes_[id].verts = std::move(sep);
    nodes_[id].left = l;
    nodes_[id].right = r;
    return id;
  }

  // General graph: vertices in `set` (original ids).  Returns the list of
  // subtree roots created (more than one if the induced subgraph is split).
  void graph(std::vector<int32_t> set, std::vector<int>* roots) {
    if (set.empty()) return;
    if ((int64_t)set.size() <= leaf_) {
      int id = (int)nodes_.size();
      nodes_.emplace_back();
      std::sort(set.begin(), set.end());
      nodes_[id].verts = std::move(set);
      roots->push_back(id);
      return;
    }
    for (int32_t v : set) mark_[v] = stamp_ + 1;
    ++stamp_;
    int cur = stamp_;
    // BFS from a pseudo-peripheral vertex (two sweeps)
    int32_t start = set[0];
    std::vector<int32_t> order;
    int nlev = 0;
    for (int sweep = 0; sweep < 2; ++sweep) {
      bfs(start, cur, &order, &nlev);
      start = order.back();
    }
    bfs(start, cur, &order, &nlev);
    if ((int64_t)order.size() < (int64_t)set.size()) {
      // disconnected: reached component and the rest are independent subtrees
      std::vector<int32_t> rest;
      for (int32_t v : set)
        if (mark2_[v] != bfs_stamp_) rest.push_back(v);
      std::vector<int32_t> comp(order.begin(), order.end());
      graph(std::move(comp), roots);
      graph(std::move(rest), roots);
      return;
    }
    // cumulative level sizes; separator = first level reaching half
    std::vector<int64_t> cnt(nlev, 0);
    for (int32_t v : order) cnt[dist_[v]]++;
    int64_t half = (int64_t)set.size() / 2, acc = 0;
    int sl = 0;
    for (sl = 0; sl < nlev; ++sl) {
      acc += cnt[sl];
      if (acc >= half) break;
    }
    if (sl == 0) sl = std::min(1, nlev - 1);
    std::vector<int32_t> L, Sp, R;
    for (int32_t v : order) {
      int d = dist_[v];
      if (d < sl)
        L.push_back(v);
      else if (d == sl)
        Sp.push_back(v);
      else
        R.push_back(v);
    }
    if (L.empty() && R.empty()) {
      int id = (int)nodes_.size();
      nodes_.emplace_back();
      std::sort(Sp.begin(), Sp.end());
      nodes_[id].verts = std::move(Sp);
      roots->push_back(id);
      return;
    }
    std::vector<int> lr, rr;
    graph(std::move(L), &lr);
    graph(std::move(R), &rr);
    // children of the separator node: all subtree roots found below it
    int id = (int)nodes_.size();
    nodes_.emplace_back();
    std::sort(Sp.begin(), Sp.end());
    nodes_[id].verts = std::move(Sp);
    extra_children_.resize(nodes_.size());
    for (int c : lr) extra_children_[id].push_back(c);
    for (int c : rr) extra_children_[id].push_back(c);
    roots->push_back(id);
  }

  void init_graph() {
    mark_.assign(n_, 0);
    mark2_.assign(n_, 0);
    dist_.assign(n_, -1);
  }

  std::vector<NDNode> nodes_;
  std::vector<std::vector<int>> extra_children_;

 private:
  void bfs(int32_t s, int setmark, std::vector<int32_t>* order, int* nlev) {
    ++bfs_stamp_;
    order->clear();
    std::deque<int32_t> q;
    q.push_back(s);
    mark2_[s] = bfs_stamp_;
    dist_[s] = 0;
    int maxd = 0;
    while (!q.empty()) {
      int32_t v = q.front();
      q.pop_front();
      order->push_back(v);
      for (int64_t e = rp_[v]; e < rp_[v + 1]; ++e) {
        int32_t w = ci_[e];
        if (mark_[w] != setmark || mark2_[w] == bfs_stamp_) continue;
        mark2_[w] = bfs_stamp_;
        dist_[w] = dist_[v] + 1;
        maxd = std::max(maxd, dist_[w]);
        q.push_back(w);
      }
    }
    *nlev = maxd + 1;
  }

  int64_t n_;
  const int64_t* rp_;
  const int32_t* ci_;
  int leaf_;
  std::vector<int> mark_, mark2_, dist_;
  int stamp_ = 0, bfs_stamp_ = 0;
};

}  // namespace

int symbolic_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind, const int32_t* grid, int leaf_size,
                     Symbolic* S) {
  if (leaf_size <= 0) leaf_size = 64;
  S->n = n;
  NDBuilder nd(n, rowptr, colind, leaf_size);
  std::vector<int> roots;
  bool geometric = grid && (int64_t)grid[0] * grid[1] * grid[2] == n && grid[0] > 0 && grid[1] > 0 && grid[2] > 0;
  if (geometric) {
    // a distance-one stencil is required for planes to separate
    for (int64_t i = 0; i < n && geometric; ++i) {
      int64_t xi = i % grid[0], yi = (i / grid[0]) % grid[1], zi = i / ((int64_t)grid[0] * grid[1]);
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        int64_t j = colind[e];
        int64_t xj = j % grid[0], yj = (j / grid[0]) % grid[1], zj = j / ((int64_t)grid[0] * grid[1]);
        if (std::llabs(xi - xj) > 1 || std::llabs(yi - yj) > 1 || std::llabs(zi - zj) > 1) {
          geometric = false;
          break;
        }
      }
    }
  }
  if (geometric) {
    roots.push_back(nd.box(grid[0], grid[1], 0, grid[0], 0, grid[1], 0, grid[2]));
  } else {
    nd.init_graph();
    std::vector<int32_t> all(n);
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    nd.graph(std::move(all), &roots);
  }
  nd.extra_children_.resize(nd.nodes_.size());
  // children lists
  const int nn = (int)nd.nodes_.size();
  std::vector<std::vector<int>> kids(nn);
  for (int i = 0; i < nn; ++i) {
    if (nd.nodes_[i].left >= 0) kids[i].push_back(nd.nodes_[i].left);
    if (nd.nodes_[i].right >= 0) kids[i].push_back(nd.nodes_[i].right);
    for (int c : nd.extra_children_[i]) kids[i].push_back(c);
  }
  // post-order traversal -> front ids and vertex numbering
  std::vector<int> post;
  post.reserve(nn);
  std::vector<int> front_of(nn, -1);
  {
    std::vector<std::pair<int, int>> st;
    for (int r : roots) {
      st.push_back({r, 0});
      while (!st.empty()) {
        auto& top = st.back();
        if (top.second < (int)kids[top.first].size()) {
          int c = kids[top.first][top.second++];
          st.push_back({c, 0});
        } else {
          front_of[top.first] = (int)post.size();
          post.push_back(top.first);
          st.pop_back();
        }
      }
    }
  }
  const int nf = (int)post.size();
  S->perm.assign(n, -1);
  S->iperm.assign(n, -1);
  S->fronts.assign(nf, Front());
  int32_t next = 0;
  for (int f = 0; f < nf; ++f) {
    const NDNode& nd_node = nd.nodes_[post[f]];
    S->fronts[f].first = next;
    S->fronts[f].ns = (int32_t)nd_node.verts.size();
    for (int32_t v : nd_node.verts) {
      S->perm[next] = v;
      S->iperm[v] = next;
      ++next;
    }
  }
  if (next != n) {
    set_error("nested dissection numbered %d of %lld vertices", (int)next, (long long)n);
    return ZOLO_EINVAL;
  }
  // parents / children in front ids
  S->children.clear();
  for (int f = 0; f < nf; ++f) {
    const auto& ks = kids[post[f]];
    S->fronts[f].child_begin = (int32_t)S->children.size();
    S->fronts[f].child_count = (int32_t)ks.size();
    S->max_children = std::max<int>(S->max_children, (int)ks.size());
    for (int c : ks) {
      S->children.push_back(front_of[c]);
      S->fronts[front_of[c]].parent = f;
    }
  }
  // permuted CSR (rows and columns in the new ordering, columns sorted)
  S->prow.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) S->prow[i + 1] = S->prow[i] + (rowptr[S->perm[i] + 1] - rowptr[S->perm[i]]);
  S->pcol.resize(S->prow[n]);
  S->psrc.resize(S->prow[n]);
  {
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t i = 0; i < n; ++i) {
      int64_t o = S->perm[i];
      row.clear();
      for (int64_t e = rowptr[o]; e < rowptr[o + 1]; ++e) row.push_back({S->iperm[colind[e]], e});
      std::sort(row.begin(), row.end());
      int64_t base = S->prow[i];
      for (size_t t = 0; t < row.size(); ++t) {
        S->pcol[base + t] = row[t].first;
        S->psrc[base + t] = row[t].second;
      }
    }
  }
  // struct lists, bottom-up (post-order = children first)
  std::vector<int32_t> mark(n, -1);
  std::vector<std::vector<int32_t>> st(nf);
  for (int f = 0; f < nf; ++f) {
    Front& F = S->fronts[f];
    int32_t last = F.first + F.ns - 1;
    std::vector<int32_t>& out = st[f];
    for (int32_t v = F.first; v <= last; ++v)
      for (int64_t e = S->prow[v]; e < S->prow[v + 1]; ++e) {
        int32_t w = S->pcol[e];
        if (w > last && mark[w] != f) {
          mark[w] = f;
          out.push_back(w);
        }
      }
    for (int t = 0; t < F.child_count; ++t) {
      int c = S->children[F.child_begin + t];
      for (int32_t w : st[c])
        if (w > last && mark[w] != f) {
          mark[w] = f;
          out.push_back(w);
        }
    }
    std::sort(out.begin(), out.end());
    F.nb = (int32_t)out.size();
  }
  // concatenate + parent maps + levels
  S->struct_rows.clear();
  S->parent_map.clear();
  for (int f = 0; f < nf; ++f) {
    Front& F = S->fronts[f];
    F.struct_off = (int64_t)S->struct_rows.size();
    for (int32_t w : st[f]) S->struct_rows.push_back(w);
  }
  S->parent_map.assign(S->struct_rows.size(), -1);
  for (int f = 0; f < nf; ++f) {
    const Front& F = S->fronts[f];
    if (F.parent < 0) {
      if (F.nb != 0) {
        set_error("symbolic: root front with nonempty struct");
        return ZOLO_EINVAL;
      }
      continue;
    }
    const Front& P = S->fronts[F.parent];
    const std::vector<int32_t>& ps = st[F.parent];
    for (int i = 0; i < F.nb; ++i) {
      int32_t w = st[f][i];
      int32_t loc;
      if (w >= P.first && w < P.first + P.ns) {
        loc = w - P.first;
      } else {
        auto it = std::lower_bound(ps.begin(), ps.end(), w);
        if (it == ps.end() || *it != w) {
          set_error("symbolic: child row %d missing from its parent front", (int)w);
          return ZOLO_EINVAL;
        }
        loc = P.ns + (int32_t)(it - ps.begin());
      }
      S->parent_map[F.struct_off + i] = loc;
    }
  }
  int maxlev = 0;
  for (int f = 0; f < nf; ++f) {
    Front& F = S->fronts[f];
    int h = 0;
    for (int t = 0; t < F.child_count; ++t) h = std::max(h, S->fronts[S->children[F.child_begin + t]].level + 1);
    F.level = h;
    maxlev = std::max(maxlev, h);
  }
  S->levels.assign(maxlev + 1, {});
  for (int f = 0; f < nf; ++f) S->levels[S->fronts[f].level].push_back(f);
  // assembly map: lower-triangle entries (i >= j) of each front's columns j
  S->asm_entry.clear();
  S->asm_pos.clear();
  for (int f = 0; f < nf; ++f) {
    Front& F = S->fronts[f];
    F.asm_begin = (int64_t)S->asm_entry.size();
    int64_t k = (int64_t)F.ns + F.nb;
    const std::vector<int32_t>& fs = st[f];
    for (int32_t j = F.first; j < F.first + F.ns; ++j)
      for (int64_t e = S->prow[j]; e < S->prow[j + 1]; ++e) {
        int32_t i = S->pcol[e];  // entry (j, i) == (i, j) by symmetry of the pattern
        if (i < j) continue;
        int64_t lr;
        if (i < F.first + F.ns) {
          lr = i - F.first;
        } else {
          auto it = std::lower_bound(fs.begin(), fs.end(), i);
          if (it == fs.end() || *it != i) {
            set_error("symbolic: entry (%d,%d) outside its front", (int)i, (int)j);
            return ZOLO_EINVAL;
          }
          lr = F.ns + (it - fs.begin());
        }
        S->asm_entry.push_back(e);
        S->asm_pos.push_back(lr + (int64_t)(j - F.first) * k);
      }
    F.asm_end = (int64_t)S->asm_entry.size();
  }
  // figures
  S->panel_entries = S->inv_entries = S->update_entries = S->struct_total = 0;
  S->max_front = 0;
  S->flops = 0.0;
  S->elim_flops = 0.0;
  for (const Front& F : S->fronts) {
    int64_t k = (int64_t)F.ns + F.nb;
    S->panel_entries += k * F.ns;
    S->inv_entries += (int64_t)F.ns * F.ns;
    S->update_entries += (int64_t)F.nb * F.nb;
    S->struct_total += F.nb;
    S->max_front = std::max(S->max_front, k);
    // complex LDL^T: eliminating column t updates the lower (k-t-1)^2/2 trailing
    // entries (one complex multiply-add = 8 real flops); the inverse of the
    // unit lower diagonal block costs about ns^3/6 complex multiply-adds.
    double kk = (double)k, nbb = (double)F.nb, nss = (double)F.ns;
    S->flops += 8.0 * ((kk * kk * kk - nbb * nbb * nbb) / 6.0) + 8.0 * nss * nss * nss / 6.0;
    S->elim_flops += 8.0 * ((kk * kk * kk - nbb * nbb * nbb) / 6.0);
  }
  return ZOLO_OK;
}

}  // namespace zolo
