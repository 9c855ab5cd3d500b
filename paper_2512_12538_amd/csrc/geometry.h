// Host-side construction of the hierarchical overlapping box decomposition:
// nested element-based cuts per level, overlap extension, restricted-
// prolongation ownership, interface nodes, neighbours and the index tables of
// the interface map.  Integer work only.
#pragma once

#include <string>
#include <vector>

struct HBox {
  int level = 0, index = 0, parent = -1;
  int prob = 0;              // problem of a merged batch (merge_geometries)
  int a = 0, b = 0;          // position among the parent's children (x slow, y fast)
  int I = 0, J = 0;          // position among all boxes of the level
  int dx0 = 0, dx1 = 0, dy0 = 0, dy1 = 0;  // non-overlapping (element-based) box, in cells
  int p0 = 0, p1 = 0, q0 = 0, q1 = 0;      // inclusive node ranges of the overlapping box
  int op0 = 0, op1 = 0, oq0 = 0, oq1 = 0;  // inclusive node ranges owned under P_i
  int n_if = 0;                             // interface sides
  std::vector<int> iface;                   // interface nodes, local p-major index, ascending
  std::vector<int> nbrs;                    // sibling boxes whose closed boxes intersect
  std::vector<int> children;
  int nx() const { return p1 - p0 + 1; }
  int ny() const { return q1 - q0 + 1; }
  int n() const { return nx() * ny(); }
  int n_own() const { return (op1 - op0 + 1) * (oq1 - oq0 + 1); }
  bool owns(int p, int q) const { return p >= op0 && p <= op1 && q >= oq0 && q <= oq1; }
  bool contains(int p, int q) const { return p >= p0 && p <= p1 && q >= q0 && q <= q1; }
  int local(int p, int q) const { return (p - p0) * ny() + (q - q0); }
};

struct Geometry {
  int dim = 2, n_cells = 0;
  std::vector<std::vector<HBox>> levels;  // levels[0] = root
  int depth() const { return (int)levels.size() - 1; }
};

// Builds the boxes of every level.  m[l] = {m_x, m_y} for level l+1, overlap[l]
// in cells (even).  Returns an empty string on success or a message.
std::string build_geometry(int dim, int n_cells, int levels, const int (*m)[2], const int* overlap,
                           Geometry& g);

// Concatenates the hierarchies of independent problems (same dim and depth)
// level by level: problem p's boxes follow those of problems < p, with every
// box index (parent, children, neighbours) shifted and prob = p.  Returns an
// empty string on success or a message.
std::string merge_geometries(const std::vector<Geometry>& parts, Geometry& g);

// Rows of the interface map of box i at level l: (neighbour j, local node of j)
// for every interface node of every neighbour whose stencil row touches a node
// owned by i, neighbours ascending, nodes ascending.
struct TraceRow {
  int j;        // neighbour box index (same level)
  int xl;       // local node index in box j
};
// Adjoint entries: for an owned node y of box i, the rows whose stencil reaches y.
struct AdjEntry {
  int yl;       // local node index in box i
  int row;      // trace row index (within box i's rows)
  int dp, dq;   // y - x
};
void trace_tables(const Geometry& g, int level, int i, std::vector<TraceRow>& rows,
                  std::vector<AdjEntry>& adj);
