// Host-side discretization data built once per mesh: P1/P2 DOF maps, CSR
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
  std::vector<int32_t> code;  // cell << 4 | local index of the row's DOF
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

struct Mesh {
  int dim = 0;
  int64_t nv = 0, nc = 0, ne = 0;
  int nloc2 = 0, nloc1 = 0;
  std::vector<double> X;          // [nv][dim]
  std::vector<int32_t> c2d;       // [nc][nloc2]; first dim+1 entries = P1 DOFs
  std::vector<int32_t> edges;     // [ne][2] sorted pairs
  int64_t n1 = 0, n2 = 0;
  std::vector<double> x2;         // [n2][dim] P2 node coordinates
  std::vector<uint8_t> bmask;     // [n2]
  std::vector<int32_t> bidx;      // boundary P2 nodes, ascending
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
};

// Builders. All throw ipcs::Error on invalid input.
Mesh* build_unit_square(int nx, int ny);
Mesh* build_unit_cube(int nx, int ny, int nz);
Mesh* build_from_arrays(int dim, int64_t nv, const double* x, int64_t nc, const int32_t* cells);

}  // namespace ipcs
