// Hierarchical box decomposition (Sec. 1: overlapping subdomains split again
// recursively; Sec. 3: [m_x1 x m_y1, ...] notation, element-based partition
// extended outward by delta/2 cells per interface side).
#include "geometry.h"

#include <algorithm>
#include <cstdio>

static int cut(int n_cells, int M, int j) { return (int)(((long long)j * n_cells) / M); }

std::string build_geometry(int dim, int n_cells, int levels, const int (*m)[2], const int* overlap,
                           Geometry& g) {
  if (dim != 1 && dim != 2) return "dim must be 1 or 2";
  if (n_cells < 2) return "n_cells must be >= 2";
  if (levels < 1 || levels > 8) return "levels must be in 1..8";
  g.dim = dim;
  g.n_cells = n_cells;
  g.levels.clear();
  HBox root;
  root.level = 0;
  root.dx0 = 0; root.dx1 = n_cells;
  root.dy0 = 0; root.dy1 = dim == 2 ? n_cells : 0;
  root.p0 = 0; root.p1 = n_cells; root.q0 = 0; root.q1 = root.dy1;
  root.op0 = root.p0; root.op1 = root.p1; root.oq0 = root.q0; root.oq1 = root.q1;
  g.levels.push_back({root});
  long long Mx = 1, My = 1;
  for (int l = 1; l <= levels; ++l) {
    int mx = m[l - 1][0], my = dim == 2 ? m[l - 1][1] : 1;
    int ov = overlap[l - 1];
    if (mx < 1 || my < 1) return "m must be >= 1";
    if (ov < 0 || (ov & 1)) return "overlap must be a non-negative even number of cells";
    Mx *= mx;
    My *= my;
    if (Mx > n_cells || (dim == 2 && My > n_cells)) return "more boxes than cells";
    const int half = ov / 2;
    std::vector<HBox> boxes;
    std::vector<HBox>& prev = g.levels.back();
    for (size_t pi = 0; pi < prev.size(); ++pi) {
      HBox& par = prev[pi];
      for (int a = 0; a < mx; ++a) {
        for (int b = 0; b < my; ++b) {
          HBox c;
          c.level = l;
          c.index = (int)boxes.size();
          c.parent = (int)pi;
          c.a = a; c.b = b;
          c.I = par.I * mx + a;
          c.J = par.J * my + b;
          c.dx0 = cut(n_cells, (int)Mx, c.I);
          c.dx1 = cut(n_cells, (int)Mx, c.I + 1);
          if (dim == 2) {
            c.dy0 = cut(n_cells, (int)My, c.J);
            c.dy1 = cut(n_cells, (int)My, c.J + 1);
          }
          // sides on the parent's element-based boundary take the parent's extent
          c.p0 = a == 0 ? par.p0 : std::max(c.dx0 - half, par.p0);
          c.p1 = a == mx - 1 ? par.p1 : std::min(c.dx1 + half, par.p1);
          c.op0 = a == 0 ? par.p0 : c.dx0;
          c.op1 = a == mx - 1 ? par.p1 : c.dx1 - 1;
          if (dim == 2) {
            c.q0 = b == 0 ? par.q0 : std::max(c.dy0 - half, par.q0);
            c.q1 = b == my - 1 ? par.q1 : std::min(c.dy1 + half, par.q1);
            c.oq0 = b == 0 ? par.q0 : c.dy0;
            c.oq1 = b == my - 1 ? par.q1 : c.dy1 - 1;
          }
          if (c.nx() < 2 || (dim == 2 && c.ny() < 2)) return "a box has fewer than two nodes per side";
          if (c.op1 < c.op0 || c.oq1 < c.oq0) return "a box owns no node";
          par.children.push_back(c.index);
          boxes.push_back(c);
        }
      }
    }
    for (HBox& c : boxes) {
      const HBox& par = prev[c.parent];
      const bool lo_x = c.p0 > par.p0, hi_x = c.p1 < par.p1;
      const bool lo_y = dim == 2 && c.q0 > par.q0, hi_y = dim == 2 && c.q1 < par.q1;
      c.n_if = (int)lo_x + (int)hi_x + (int)lo_y + (int)hi_y;
      // node rows on an x side are interface nodes whole; the other rows hold
      // at most their two y ends (a 2D box has ny >= 2, so the ends differ)
      c.iface.reserve(2 * (c.nx() + c.ny()));
      for (int p = c.p0; p <= c.p1; ++p) {
        if ((lo_x && p == c.p0) || (hi_x && p == c.p1)) {
          for (int q = c.q0; q <= c.q1; ++q) c.iface.push_back(c.local(p, q));
        } else {
          if (lo_y) c.iface.push_back(c.local(p, c.q0));
          if (hi_y) c.iface.push_back(c.local(p, c.q1));
        }
      }
      for (int o : par.children) {
        if (o == c.index) continue;
        const HBox& d = boxes[o];
        if (d.p0 <= c.p1 && c.p0 <= d.p1 && d.q0 <= c.q1 && c.q0 <= d.q1) c.nbrs.push_back(o);
      }
    }
    g.levels.push_back(std::move(boxes));
  }
  return "";
}

std::string merge_geometries(const std::vector<Geometry>& parts, Geometry& g) {
  if (parts.empty()) return "no problems";
  const int depth = parts[0].depth();
  g = Geometry();
  g.dim = parts[0].dim;
  g.n_cells = parts[0].n_cells;
  g.levels.assign(depth + 1, {});
  std::vector<int> base(depth + 1, 0);
  for (size_t p = 0; p < parts.size(); ++p) {
    const Geometry& h = parts[p];
    if (h.dim != g.dim || h.depth() != depth) return "problems of a batch need the same dimension and depth";
    for (int l = 0; l <= depth; ++l) {
      for (HBox b : h.levels[l]) {
        b.prob = (int)p;
        b.index += base[l];
        if (b.parent >= 0) b.parent += base[l - 1];
        for (int& c : b.children) c += base[l + 1];
        for (int& o : b.nbrs) o += base[l];
        g.levels[l].push_back(std::move(b));
      }
    }
    for (int l = 0; l <= depth; ++l) base[l] += (int)h.levels[l].size();
  }
  return "";
}

void trace_tables(const Geometry& g, int level, int i, std::vector<TraceRow>& rows,
                  std::vector<AdjEntry>& adj) {
  rows.clear();
  adj.clear();
  const std::vector<HBox>& L = g.levels[level];
  const HBox& bi = L[i];
  static const int DP[5] = {0, -1, 1, 0, 0};
  static const int DQ[5] = {0, 0, 0, -1, 1};
  for (int j : bi.nbrs) {
    const HBox& bj = L[j];
    for (int xl : bj.iface) {
      const int xp = bj.p0 + xl / bj.ny(), xq = bj.q0 + xl % bj.ny();
      bool touches = false;
      for (int d = 0; d < 5; ++d) {
        int yp = xp + DP[d], yq = xq + DQ[d];
        if (g.dim == 1 && DQ[d] != 0) continue;
        if (bj.contains(yp, yq) && bi.owns(yp, yq)) touches = true;
      }
      if (!touches) continue;
      const int row = (int)rows.size();
      rows.push_back({j, xl});
      for (int d = 0; d < 5; ++d) {
        int yp = xp + DP[d], yq = xq + DQ[d];
        if (g.dim == 1 && DQ[d] != 0) continue;
        if (bj.contains(yp, yq) && bi.owns(yp, yq)) adj.push_back({bi.local(yp, yq), row, DP[d], DQ[d]});
      }
    }
  }
  std::stable_sort(adj.begin(), adj.end(), [](const AdjEntry& u, const AdjEntry& v) {
    return u.yl != v.yl ? u.yl < v.yl : u.row < v.row;
  });
}
