// Host-side discretization data built once per mesh: velocity/pressure DOF maps, CSR
// sparsity patterns of the IPCS matrices and the row-owner assembly maps.
//
// Row-owner assembly: every CSR row is produced by exactly one GPU thread,
// which visits the cells incident to its DOF and adds the cell's local row
// into the row's slots. The maps below give, per (row, incident cell) pair,
// the cell, the row's local index in the cell and the position (slot, < 256)
// of each local column inside the CSR row. No two threads write one value,
// so the scatter needs no atomics and is deterministic.
#pragma once
#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

namespace ipcs {

struct Pattern {
  int64_t nrows = 0, ncols = 0;
  std::vector<int32_t> rowptr, col;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// (row, incident cell) pairs of one row space, sorted by row then cell.
struct Incidence {
  std::vector<int32_t> ptr;   // [nrows+1]
  std::vector<int32_t> code;  // cell << 5 | local index of the row's DOF
};

// SELL-64 layout of a pattern (sliced ELLPACK): rows are grouped in slices of
// 64 consecutive rows (one wavefront, one row per lane); slice s holds
// width(s) = max row length in the slice columns of 64 entries, stored
// column-major, so entry k of row r sits at sptr[r/64] + 64 k + r%64. Padding
// entries carry value 0 and repeat the row's last column index.
struct Sell {
  int64_t nrows = 0, nslices = 0, nent = 0;
  int maxw = 0;
  std::vector<int32_t> sptr;   // [nslices+1], entry offsets
  std::vector<int32_t> col;    // [nent]
  int64_t index(int64_t row, int k) const { return sptr[row >> 6] + 64ll * k + (row & 63); }
};

// Per incidence pair, the slots of the cell's local columns in the row
// (stride bytes per pair, stride = local columns rounded up to 4).
struct SlotMap {
  int stride = 0;
  std::vector<uint8_t> slot;
};

// Rows of a square pattern partitioned into parts of at most rows_max rows
// (compact patches of DOFs), renumbered so that each part is contiguous
// ("part order": perm[i] is the original row of part-order row i), with a
// SELL-64 layout per part whose column indices are local to the part:
// 0 .. own-1 for its own rows, own + q for its q-th halo column (a column
// referenced by its rows and owned by another part, in part order). src maps
// each entry to the pattern's SELL-64 value index (-1: padding, value 0).
struct PartSell {
  int64_t n = 0, nent = 0;
  int rows_max = 0, nparts = 0, maxw = 0;
  int lds_max = 0;                  // largest own + halo count of a part
  std::vector<int32_t> perm;        // [n]
  std::vector<int32_t> part_ptr;    // [nparts+1] part-order rows
  std::vector<int32_t> halo_ptr;    // [nparts+1]
  std::vector<int32_t> halo;        // part-order rows
  std::vector<int32_t> slice_ptr;   // [nparts+1] first slice of each part
  std::vector<int32_t> sptr;        // [nslices+1] entry offsets
  std::vector<uint16_t> lcol;       // [nent]
  std::vector<int32_t> src;         // [nent]
  // depth 2 (two CG iterations per launch): the second ring halo2 (the
  // columns the halo rows reference outside the part and its halo, sorted,
  // local indices own + nhalo + q) and a SELL-64 layout of each part's halo
  // rows (local row q = the q-th halo row) with local columns over own, halo
  // and halo2; hsrc as src
  int depth = 1;
  int lds2_max = 0;                 // largest own + halo + halo2 count of a part
  int64_t hnent = 0;
  std::vector<int32_t> halo2_ptr;   // [nparts+1]
  std::vector<int32_t> halo2;       // part-order rows
  std::vector<int32_t> hslice_ptr;  // [nparts+1] first halo-row slice of each part
  std::vector<int32_t> hsptr;       // [nhslices+1] entry offsets
  std::vector<uint16_t> hlcol;      // [hnent]
  std::vector<int32_t> hsrc;        // [hnent]
};

// The Taylor-Hood pair fixes the two spaces. Names keep the P2-P1 pair's
// vocabulary: "2" is the velocity space, "1" the pressure space.
//   P2-P1 (triangles, tetrahedra): velocity P2 (vertices and edge midpoints),
//   pressure P1 (vertices).
//   P3-P2: velocity P3 (vertices; two nodes per edge, at (2 x_lo + x_hi)/3
//   and (x_lo + 2 x_hi)/3 for sorted vertices lo < hi; one node per cell at
//   its centroid (triangles) or per face at its centroid, the faces sorted by
//   their vertex triples (tetrahedra)), pressure P2 (vertices, then the edges
//   sorted by (lo, hi)).
// Velocity DOFs, internal numbering (every array below): the vertices in input
// order, then the other velocity nodes in lexicographic order of their
// coordinates (last coordinate most significant), so that neighbouring nodes
// have neighbouring indices. The interface numbering differs: the vertices,
// then the other nodes in listing order (P2: the edge midpoints with the edges
// sorted by (lo, hi); P3: two nodes per edge in edge order, then the cell or
// face centroids). v_out maps internal to interface ids, v_in back.
// A cell's local velocity DOFs start with its vertices. Kernels take the cell
// geometry from the pressure cell table, which starts with the vertex ids in
// both pairs (P1: the vertices; P2: vertices, then edges).
struct Mesh {
  int dim = 0;
  int pair = 0;                   // IPCS_PAIR_P2P1 or IPCS_PAIR_P3P2
  int64_t nv = 0, nc = 0, ne = 0;
  int nloc2 = 0, nloc1 = 0;
  std::vector<double> X;          // [nv][dim]
  std::vector<int32_t> c2d;       // [nc][nloc2] velocity DOFs (local order: vertices first)
  std::vector<int32_t> c2dp;      // [nc][nloc1] pressure DOFs; first dim+1 = vertex ids
  std::vector<int32_t> edges;     // [ne][2] sorted pairs
  int64_t n1 = 0, n2 = 0;
  std::vector<double> x2;         // [n2][dim] velocity node coordinates
  std::vector<double> xp;         // [n1][dim] pressure node coordinates
  std::vector<uint8_t> bmask;     // [n2]
  std::vector<int32_t> bidx;      // boundary velocity nodes, ascending
  std::vector<int32_t> v_out;     // [n2] internal velocity id -> interface id
  std::vector<int32_t> v_in;      // [n2] interface velocity id -> internal id
  Pattern p22, p11, p12, p21;
  Sell e22, e11, e12, e21;        // SELL-64 layouts of the four patterns
  Incidence inc2, inc1;
  SlotMap s22, s21, s11, s12;
  // Dirichlet lifting: for interior P2 rows, the entries of the P2P2 pattern
  // in boundary columns: (SELL index into P2P2 values, boundary column).
  std::vector<int32_t> lift_ptr;  // [n2+1]
  std::vector<int32_t> lift_slot, lift_col;
  int max_row22 = 0, max_row11 = 0, max_row12 = 0, max_row21 = 0;

  const Pattern& pattern(int which) const;
  const Sell& sell(int which) const;
  // partition of the pressure-pressure pattern by the pressure node
  // coordinates, built on first use for each part size and kept with the mesh
  // (depth 2: with the second halo ring, for two CG iterations per launch)
  std::shared_ptr<const PartSell> parts11(int rows_max, int depth = 1) const;

 private:
  mutable std::mutex parts_mu;
  mutable std::vector<std::shared_ptr<const PartSell>> parts_cache;
};

// SELL-64 layout of a CSR pattern (padding repeats a row's last column)
void build_sell(const Pattern& P, Sell& S);

std::shared_ptr<const PartSell> build_parts(const Pattern& P, const Sell& S, const double* X,
                                            int dim, int rows_max, int depth = 1);

// Builders. All throw ipcs::Error on invalid input.
Mesh* build_unit_square(int nx, int ny, int pair = 0);
Mesh* build_unit_cube(int nx, int ny, int nz, int pair = 0);
Mesh* build_from_arrays(int dim, int64_t nv, const double* x, int64_t nc, const int32_t* cells,
                        int pair = 0);

}  // namespace ipcs
