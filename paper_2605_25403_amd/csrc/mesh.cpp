// Mesh generators, velocity/pressure DOF maps, CSR patterns and row-owner
// assembly maps. Integer work done once per mesh on the host (Section 2.2.1:
// conforming simplicial mesh, continuous Lagrange spaces of a Taylor-Hood pair:
// P2 velocity and P1 pressure, or on triangles P3 velocity and P2 pressure).
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <string>

#include "common.hpp"
#include "rules.hpp"

namespace ipcs {

const Pattern& Mesh::pattern(int which) const {
  switch (which) {
    case IPCS_PATTERN_P2P2: return p22;
    case IPCS_PATTERN_P1P1: return p11;
    case IPCS_PATTERN_P1P2: return p12;
    case IPCS_PATTERN_P2P1: return p21;
  }
  fail(IPCS_E_INVALID, "unknown pattern id " + std::to_string(which));
}

const Sell& Mesh::sell(int which) const {
  switch (which) {
    case IPCS_PATTERN_P2P2: return e22;
    case IPCS_PATTERN_P1P1: return e11;
    case IPCS_PATTERN_P1P2: return e12;
    case IPCS_PATTERN_P2P1: return e21;
  }
  fail(IPCS_E_INVALID, "unknown pattern id " + std::to_string(which));
}

void build_sell(const Pattern& P, Sell& S) {
  S.nrows = P.nrows;
  S.nslices = (P.nrows + 63) / 64;
  S.sptr.assign(S.nslices + 1, 0);
  S.maxw = 0;
  for (int64_t s = 0; s < S.nslices; ++s) {
    int w = 0;
    for (int64_t r = 64 * s; r < std::min<int64_t>(P.nrows, 64 * s + 64); ++r)
      w = std::max(w, P.rowptr[r + 1] - P.rowptr[r]);
    S.maxw = std::max(S.maxw, w);
    const int64_t next = (int64_t)S.sptr[s] + 64ll * w;
    if (next >= (int64_t(1) << 31)) fail(IPCS_E_INVALID, "SELL layout exceeds 2^31 entries");
    S.sptr[s + 1] = int32_t(next);
  }
  S.nent = S.sptr[S.nslices];
  S.col.assign(S.nent, 0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S.nslices; ++s) {
    const int w = (S.sptr[s + 1] - S.sptr[s]) / 64;
    for (int lane = 0; lane < 64; ++lane) {
      const int64_t r = 64 * s + lane;
      const int len = r < P.nrows ? P.rowptr[r + 1] - P.rowptr[r] : 0;
      const int32_t pad = len > 0 ? P.col[P.rowptr[r] + len - 1] : 0;
      for (int k = 0; k < w; ++k)
        S.col[S.sptr[s] + 64ll * k + lane] = k < len ? P.col[P.rowptr[r] + k] : pad;
    }
  }
}

namespace {

inline int edge_a(int dim, int e) { return dim == 2 ? Edges<2>::a(e) : Edges<3>::a(e); }
inline int edge_b(int dim, int e) { return dim == 2 ? Edges<2>::b(e) : Edges<3>::b(e); }

inline uint64_t edge_key(int32_t u, int32_t v) {
  if (u > v) std::swap(u, v);
  return (uint64_t(uint32_t(u)) << 32) | uint32_t(v);
}

// Row-wise union of the column DOFs of the cells incident to each row.
void build_pattern(const Incidence& inc, const std::vector<int32_t>& c2d, int nloc,
                   int ncolloc, int64_t nrows, int64_t ncols, Pattern& P, int& maxrow) {
  P.nrows = nrows;
  P.ncols = ncols;
  P.rowptr.assign(nrows + 1, 0);
  std::vector<int32_t> len(nrows);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < nrows; ++i) {
    int32_t buf[1024];
    int n = 0;
    for (int32_t p = inc.ptr[i]; p < inc.ptr[i + 1]; ++p) {
      int64_t c = inc.code[p] >> 5;
      for (int j = 0; j < ncolloc; ++j) {
        if (n < 1024) buf[n++] = c2d[c * nloc + j];
      }
    }
    std::sort(buf, buf + n);
    len[i] = int32_t(std::unique(buf, buf + n) - buf);
  }
  int64_t tot = 0;
  maxrow = 0;
  for (int64_t i = 0; i < nrows; ++i) {
    P.rowptr[i] = int32_t(tot);
    tot += len[i];
    maxrow = std::max(maxrow, len[i]);
  }
  if (tot >= (int64_t(1) << 31)) fail(IPCS_E_INVALID, "pattern exceeds 2^31 entries");
  P.rowptr[nrows] = int32_t(tot);
  P.col.resize(tot);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < nrows; ++i) {
    int32_t buf[1024];
    int n = 0;
    for (int32_t p = inc.ptr[i]; p < inc.ptr[i + 1]; ++p) {
      int64_t c = inc.code[p] >> 5;
      for (int j = 0; j < ncolloc; ++j) {
        if (n < 1024) buf[n++] = c2d[c * nloc + j];
      }
    }
    std::sort(buf, buf + n);
    int m = int(std::unique(buf, buf + n) - buf);
    std::copy(buf, buf + m, P.col.begin() + P.rowptr[i]);
  }
  if (maxrow > 255) fail(IPCS_E_INVALID, "a matrix row has more than 255 entries");
}

void build_slots(const Incidence& inc, const std::vector<int32_t>& c2d, int nloc, int ncolloc,
                 const Pattern& P, SlotMap& S) {
  S.stride = int((ncolloc + 3) / 4 * 4);
  const int64_t npairs = (int64_t)inc.code.size();
  S.slot.assign(npairs * S.stride, 0);
  const int64_t nrows = P.nrows;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < nrows; ++i) {
    const int32_t* b = P.col.data() + P.rowptr[i];
    const int32_t* e = P.col.data() + P.rowptr[i + 1];
    for (int32_t p = inc.ptr[i]; p < inc.ptr[i + 1]; ++p) {
      int64_t c = inc.code[p] >> 5;
      for (int j = 0; j < ncolloc; ++j) {
        const int32_t* f = std::lower_bound(b, e, c2d[c * nloc + j]);
        S.slot[(int64_t)p * S.stride + j] = uint8_t(f - b);
      }
    }
  }
}

void build_incidence(const std::vector<int32_t>& c2d, int64_t nc, int nloc, int nrowloc,
                     int64_t nrows, Incidence& I) {
  I.ptr.assign(nrows + 1, 0);
  for (int64_t c = 0; c < nc; ++c)
    for (int j = 0; j < nrowloc; ++j) I.ptr[c2d[c * nloc + j] + 1]++;
  for (int64_t i = 0; i < nrows; ++i) I.ptr[i + 1] += I.ptr[i];
  I.code.resize(I.ptr[nrows]);
  std::vector<int32_t> fill(I.ptr.begin(), I.ptr.end() - 1);
  for (int64_t c = 0; c < nc; ++c)
    for (int j = 0; j < nrowloc; ++j) I.code[fill[c2d[c * nloc + j]]++] = int32_t((c << 5) | j);
}

// Internal numbering of the velocity DOFs (the interface keeps the listing
// order; v_out and v_in map between the two): the vertices keep their
// numbers; every other velocity node is numbered in lexicographic order of its
// coordinates, last coordinate most
// significant (y, x in 2D; z, y, x in 3D), ties (none on a valid mesh) by the
// listing order. Rows that are neighbours in this order reference nearby
// columns, so a SELL-64 slice's gathers touch few cache lines; keeping the
// vertices apart keeps each slice to rows of one kind and length (one
// coordinate order over all nodes interleaves vertex and edge rows and was
// slower).
void renumber_velocity(Mesh& m) {
  const int d = m.dim;
  const int64_t nv = m.nv, n = m.n2;
  std::vector<int64_t> ord(n - nv);
  for (int64_t i = 0; i < n - nv; ++i) ord[i] = nv + i;
  const double* x = m.x2.data();
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    for (int r = d - 1; r >= 0; --r)
      if (x[a * d + r] != x[b * d + r]) return x[a * d + r] < x[b * d + r];
    return a < b;
  });
  std::vector<int32_t> nw(n);
  for (int64_t i = 0; i < nv; ++i) nw[i] = int32_t(i);
  for (int64_t k = 0; k < n - nv; ++k) nw[ord[k]] = int32_t(nv + k);
  for (auto& v : m.c2d) v = nw[v];
  m.v_in = nw;
  m.v_out.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) m.v_out[nw[i]] = int32_t(i);
  std::vector<double> x2(m.x2.size());
  std::vector<uint8_t> bm(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int r = 0; r < d; ++r) x2[(int64_t)nw[i] * d + r] = m.x2[i * d + r];
    bm[nw[i]] = m.bmask[i];
  }
  m.x2.swap(x2);
  m.bmask.swap(bm);
}

void finalize(Mesh& m) {
  const int d = m.dim;
  const int64_t nc = m.nc, nv = m.nv;
  const int ne_loc = d == 2 ? 3 : 6;
  if (m.pair != IPCS_PAIR_P2P1 && m.pair != IPCS_PAIR_P3P2)
    fail(IPCS_E_INVALID, "unknown Taylor-Hood pair " + std::to_string(m.pair));
  m.nloc1 = d + 1;
  m.nloc2 = d + 1 + ne_loc;
  if (nc >= (int64_t(1) << 26)) fail(IPCS_E_INVALID, "too many cells");
  if (nv >= (int64_t(1) << 31)) fail(IPCS_E_INVALID, "too many vertices");
  // --- edges: unique vertex pairs, sorted lexicographically
  std::vector<uint64_t> keys(nc * ne_loc);
#pragma omp parallel for
  for (int64_t c = 0; c < nc; ++c)
    for (int e = 0; e < ne_loc; ++e)
      keys[c * ne_loc + e] = edge_key(m.c2d[c * (d + 1) + edge_a(d, e)],
                                      m.c2d[c * (d + 1) + edge_b(d, e)]);
  std::vector<uint64_t> uk(keys);
  std::sort(uk.begin(), uk.end());
  uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
  m.ne = (int64_t)uk.size();
  m.n1 = nv;
  m.n2 = nv + m.ne;
  if (m.n2 >= (int64_t(1) << 31)) fail(IPCS_E_INVALID, "too many DOFs");
  m.edges.resize(2 * m.ne);
  for (int64_t e = 0; e < m.ne; ++e) {
    m.edges[2 * e] = int32_t(uk[e] >> 32);
    m.edges[2 * e + 1] = int32_t(uk[e] & 0xffffffffu);
  }
  // --- cell -> P2 dofs (c2d currently holds the vertices, stride d+1)
  std::vector<int32_t> c2d(nc * m.nloc2);
#pragma omp parallel for
  for (int64_t c = 0; c < nc; ++c) {
    for (int k = 0; k <= d; ++k) c2d[c * m.nloc2 + k] = m.c2d[c * (d + 1) + k];
    for (int e = 0; e < ne_loc; ++e) {
      uint64_t k = keys[c * ne_loc + e];
      c2d[c * m.nloc2 + d + 1 + e] =
          int32_t(nv + (std::lower_bound(uk.begin(), uk.end(), k) - uk.begin()));
    }
  }
  m.c2d.swap(c2d);
  // --- P2 node coordinates
  m.x2.resize(m.n2 * d);
  for (int64_t i = 0; i < nv * d; ++i) m.x2[i] = m.X[i];
  for (int64_t e = 0; e < m.ne; ++e)
    for (int k = 0; k < d; ++k)
      m.x2[(nv + e) * d + k] =
          0.5 * (m.X[(int64_t)m.edges[2 * e] * d + k] + m.X[(int64_t)m.edges[2 * e + 1] * d + k]);
  // --- boundary: facets owned by exactly one cell; their vertices and edges
  m.bmask.assign(m.n2, 0);
  if (d == 2) {
    std::vector<int32_t> cnt(m.ne, 0);
    for (int64_t c = 0; c < nc; ++c)
      for (int e = 0; e < 3; ++e) cnt[m.c2d[c * m.nloc2 + 3 + e] - nv]++;
    for (int64_t e = 0; e < m.ne; ++e)
      if (cnt[e] == 1) {
        m.bmask[m.edges[2 * e]] = 1;
        m.bmask[m.edges[2 * e + 1]] = 1;
        m.bmask[nv + e] = 1;
      }
  } else {
    std::vector<std::array<int32_t, 3>> faces(nc * 4);
    for (int64_t c = 0; c < nc; ++c)
      for (int k = 0; k < 4; ++k) {
        std::array<int32_t, 3> f;
        int n = 0;
        for (int j = 0; j < 4; ++j)
          if (j != k) f[n++] = m.c2d[c * m.nloc2 + j];
        std::sort(f.begin(), f.end());
        faces[c * 4 + k] = f;
      }
    std::sort(faces.begin(), faces.end());
    for (size_t i = 0; i < faces.size();) {
      size_t j = i + 1;
      while (j < faces.size() && faces[j] == faces[i]) ++j;
      if (j - i == 1) {
        const auto& f = faces[i];
        for (int a = 0; a < 3; ++a) {
          m.bmask[f[a]] = 1;
          for (int b = a + 1; b < 3; ++b) {
            uint64_t k = edge_key(f[a], f[b]);
            m.bmask[nv + (std::lower_bound(uk.begin(), uk.end(), k) - uk.begin())] = 1;
          }
        }
      }
      i = j;
    }
  }
  if (m.pair == IPCS_PAIR_P2P1) {
    // pressure P1: the vertices
    m.c2dp.resize(nc * m.nloc1);
    for (int64_t c = 0; c < nc; ++c)
      for (int k = 0; k <= d; ++k) m.c2dp[c * m.nloc1 + k] = m.c2d[c * m.nloc2 + k];
    m.xp = m.X;
  } else {
    // pressure P2: the P2 maps built above; velocity P3: vertices, two nodes
    // per edge, then one node per cell (triangles) or per face (tetrahedra)
    m.c2dp.swap(m.c2d);
    m.nloc1 = m.nloc2;
    m.xp.swap(m.x2);
    std::vector<uint8_t> bm2;
    bm2.swap(m.bmask);
    const int nl3 = d == 2 ? 10 : 20;
    const int nl2 = m.nloc1;
    m.nloc2 = nl3;
    m.n1 = m.n2;
    // faces (tetrahedra): unique sorted vertex triples, the face opposite
    // local vertex k of each cell; boundary faces are owned by one cell
    std::vector<uint64_t> fkeys, fu;
    std::vector<int32_t> fcnt;
    if (d == 3) {
      fkeys.resize(nc * 4);
      auto fkey = [](int32_t a, int32_t b, int32_t c) {
        int32_t v[3] = {a, b, c};
        std::sort(v, v + 3);
        return (uint64_t(uint32_t(v[0])) << 42) | (uint64_t(uint32_t(v[1])) << 21) |
               uint64_t(uint32_t(v[2]));
      };
      if (nv >= (int64_t(1) << 21)) fail(IPCS_E_INVALID, "too many vertices for P3 tetrahedra");
#pragma omp parallel for
      for (int64_t c = 0; c < nc; ++c)
        for (int f = 0; f < 4; ++f) {
          const int32_t* p = m.c2dp.data() + c * nl2;
          fkeys[c * 4 + f] = fkey(p[P3Tet::fv(f, 0)], p[P3Tet::fv(f, 1)], p[P3Tet::fv(f, 2)]);
        }
      fu = fkeys;
      std::sort(fu.begin(), fu.end());
      fcnt.assign(fu.size(), 0);
      {
        std::vector<uint64_t> tmp;
        tmp.reserve(fu.size());
        for (size_t i = 0; i < fu.size();) {
          size_t j = i + 1;
          while (j < fu.size() && fu[j] == fu[i]) ++j;
          tmp.push_back(fu[i]);
          i = j;
        }
        fcnt.assign(tmp.size(), 0);
        for (uint64_t k : fkeys) fcnt[std::lower_bound(tmp.begin(), tmp.end(), k) - tmp.begin()]++;
        fu.swap(tmp);
      }
    }
    const int64_t ncn = d == 2 ? nc : (int64_t)fu.size();   // cell or face nodes
    m.n2 = nv + 2 * m.ne + ncn;
    if (m.n2 >= (int64_t(1) << 31)) fail(IPCS_E_INVALID, "too many DOFs");
    m.c2d.resize(nc * nl3);
    const int ne_l = Edges<3>::NE;
#pragma omp parallel for
    for (int64_t c = 0; c < nc; ++c) {
      const int32_t* p = m.c2dp.data() + c * nl2;
      int32_t* o = m.c2d.data() + c * nl3;
      for (int k = 0; k <= d; ++k) o[k] = p[k];
      const int nel = d == 2 ? 3 : ne_l;
      for (int e = 0; e < nel; ++e) {
        const int64_t k = p[d + 1 + e] - nv;           // edge index
        const int ea = d == 2 ? Edges<2>::a(e) : Edges<3>::a(e);
        const int eb = d == 2 ? Edges<2>::b(e) : Edges<3>::b(e);
        const bool fwd = p[ea] < p[eb];
        o[d + 1 + 2 * e] = int32_t(nv + 2 * k + (fwd ? 0 : 1));
        o[d + 2 + 2 * e] = int32_t(nv + 2 * k + (fwd ? 1 : 0));
      }
      if (d == 2) {
        o[9] = int32_t(nv + 2 * m.ne + c);
      } else {
        for (int f = 0; f < 4; ++f)
          o[16 + f] = int32_t(nv + 2 * m.ne +
                              (std::lower_bound(fu.begin(), fu.end(), fkeys[c * 4 + f]) - fu.begin()));
      }
    }
    m.x2.resize(m.n2 * d);
    for (int64_t i = 0; i < nv * d; ++i) m.x2[i] = m.X[i];
    for (int64_t e = 0; e < m.ne; ++e)
      for (int r = 0; r < d; ++r) {
        const double lo = m.X[(int64_t)m.edges[2 * e] * d + r];
        const double hi = m.X[(int64_t)m.edges[2 * e + 1] * d + r];
        m.x2[(nv + 2 * e) * d + r] = (2.0 * lo + hi) / 3.0;
        m.x2[(nv + 2 * e + 1) * d + r] = (lo + 2.0 * hi) / 3.0;
      }
    if (d == 2) {
      for (int64_t c = 0; c < nc; ++c)
        for (int r = 0; r < 2; ++r)
          m.x2[(nv + 2 * m.ne + c) * 2 + r] =
              (m.X[(int64_t)m.c2d[c * 10] * 2 + r] + m.X[(int64_t)m.c2d[c * 10 + 1] * 2 + r] +
               m.X[(int64_t)m.c2d[c * 10 + 2] * 2 + r]) / 3.0;
    } else {
      for (int64_t f = 0; f < ncn; ++f) {
        const int32_t v[3] = {int32_t(fu[f] >> 42), int32_t((fu[f] >> 21) & 0x1fffff),
                              int32_t(fu[f] & 0x1fffff)};
        for (int r = 0; r < 3; ++r)
          m.x2[(nv + 2 * m.ne + f) * 3 + r] =
              (m.X[(int64_t)v[0] * 3 + r] + m.X[(int64_t)v[1] * 3 + r] + m.X[(int64_t)v[2] * 3 + r]) / 3.0;
      }
    }
    // boundary: boundary vertices, both nodes of boundary edges, the nodes of
    // boundary faces
    m.bmask.assign(m.n2, 0);
    for (int64_t i = 0; i < nv; ++i) m.bmask[i] = bm2[i];
    for (int64_t e = 0; e < m.ne; ++e)
      if (bm2[nv + e]) m.bmask[nv + 2 * e] = m.bmask[nv + 2 * e + 1] = 1;
    if (d == 3)
      for (int64_t f = 0; f < ncn; ++f)
        if (fcnt[f] == 1) m.bmask[nv + 2 * m.ne + f] = 1;
  }
  renumber_velocity(m);
  m.bidx.clear();
  for (int64_t i = 0; i < m.n2; ++i)
    if (m.bmask[i]) m.bidx.push_back(int32_t(i));
  // --- incidence, patterns, slot maps (velocity rows/columns from c2d,
  // pressure rows/columns from c2dp)
  build_incidence(m.c2d, nc, m.nloc2, m.nloc2, m.n2, m.inc2);
  build_incidence(m.c2dp, nc, m.nloc1, m.nloc1, m.n1, m.inc1);
  build_pattern(m.inc2, m.c2d, m.nloc2, m.nloc2, m.n2, m.n2, m.p22, m.max_row22);
  build_pattern(m.inc2, m.c2dp, m.nloc1, m.nloc1, m.n2, m.n1, m.p21, m.max_row21);
  build_pattern(m.inc1, m.c2dp, m.nloc1, m.nloc1, m.n1, m.n1, m.p11, m.max_row11);
  build_pattern(m.inc1, m.c2d, m.nloc2, m.nloc2, m.n1, m.n2, m.p12, m.max_row12);
  build_slots(m.inc2, m.c2d, m.nloc2, m.nloc2, m.p22, m.s22);
  build_slots(m.inc2, m.c2dp, m.nloc1, m.nloc1, m.p21, m.s21);
  build_slots(m.inc1, m.c2dp, m.nloc1, m.nloc1, m.p11, m.s11);
  build_slots(m.inc1, m.c2d, m.nloc2, m.nloc2, m.p12, m.s12);
  build_sell(m.p22, m.e22);
  build_sell(m.p21, m.e21);
  build_sell(m.p11, m.e11);
  build_sell(m.p12, m.e12);
  // --- Dirichlet lifting entries (interior rows, boundary columns)
  m.lift_ptr.assign(m.n2 + 1, 0);
  m.lift_slot.clear();
  m.lift_col.clear();
  for (int64_t i = 0; i < m.n2; ++i) {
    if (!m.bmask[i])
      for (int32_t s = m.p22.rowptr[i]; s < m.p22.rowptr[i + 1]; ++s)
        if (m.bmask[m.p22.col[s]]) {
          m.lift_slot.push_back(int32_t(m.e22.index(i, s - m.p22.rowptr[i])));
          m.lift_col.push_back(m.p22.col[s]);
        }
    m.lift_ptr[i + 1] = int32_t(m.lift_slot.size());
  }
}

}  // namespace

Mesh* build_unit_square(int nx, int ny, int pair) {
  if (nx < 1 || ny < 1) fail(IPCS_E_INVALID, "unit square needs nx, ny >= 1");
  if (int64_t(nx) * ny > (int64_t(1) << 26)) fail(IPCS_E_INVALID, "mesh too large");
  Mesh* m = new Mesh;
  m->dim = 2;
  m->pair = pair;
  m->nv = int64_t(nx + 1) * (ny + 1);
  m->nc = 2 * int64_t(nx) * ny;
  m->X.resize(m->nv * 2);
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i <= nx; ++i) {
      int64_t v = int64_t(j) * (nx + 1) + i;
      m->X[2 * v] = double(i) / nx;
      m->X[2 * v + 1] = double(j) / ny;
    }
  m->c2d.resize(m->nc * 3);
  int64_t c = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int32_t a = int32_t(int64_t(j) * (nx + 1) + i), b = a + 1, cc = a + (nx + 1) + 1,
              e = a + (nx + 1);
      int32_t t0[3] = {a, b, cc}, t1[3] = {a, cc, e};
      for (int k = 0; k < 3; ++k) m->c2d[3 * c + k] = t0[k];
      ++c;
      for (int k = 0; k < 3; ++k) m->c2d[3 * c + k] = t1[k];
      ++c;
    }
  try {
    finalize(*m);
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

Mesh* build_unit_cube(int nx, int ny, int nz, int pair) {
  if (nx < 1 || ny < 1 || nz < 1) fail(IPCS_E_INVALID, "unit cube needs nx, ny, nz >= 1");
  if (int64_t(nx) * ny * nz > (int64_t(1) << 23)) fail(IPCS_E_INVALID, "mesh too large");
  Mesh* m = new Mesh;
  m->dim = 3;
  m->pair = pair;
  m->nv = int64_t(nx + 1) * (ny + 1) * (nz + 1);
  m->nc = 6 * int64_t(nx) * ny * nz;
  m->X.resize(m->nv * 3);
  auto vid = [&](int i, int j, int k) {
    return int32_t((int64_t(k) * (ny + 1) + j) * (nx + 1) + i);
  };
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        int64_t v = vid(i, j, k);
        m->X[3 * v] = double(i) / nx;
        m->X[3 * v + 1] = double(j) / ny;
        m->X[3 * v + 2] = double(k) / nz;
      }
  m->c2d.resize(m->nc * 4);
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                  {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int64_t c = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        for (int p = 0; p < 6; ++p) {
          int q[3] = {i, j, k};
          m->c2d[4 * c] = vid(q[0], q[1], q[2]);
          for (int s = 0; s < 3; ++s) {
            q[perms[p][s]] += 1;
            m->c2d[4 * c + 1 + s] = vid(q[0], q[1], q[2]);
          }
          // positive orientation: the path e_a, e_b, e_c has det = sign of the
          // permutation (a,b,c); odd permutations swap the last two vertices
          if (p == 1 || p == 2 || p == 5) std::swap(m->c2d[4 * c + 2], m->c2d[4 * c + 3]);
          ++c;
        }
  try {
    finalize(*m);
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

Mesh* build_from_arrays(int dim, int64_t nv, const double* x, int64_t nc, const int32_t* cells,
                        int pair) {
  if (dim != 2 && dim != 3) fail(IPCS_E_INVALID, "dim must be 2 or 3");
  if (nv < dim + 1 || nc < 1 || !x || !cells) fail(IPCS_E_INVALID, "empty mesh");
  Mesh* m = new Mesh;
  m->dim = dim;
  m->pair = pair;
  m->nv = nv;
  m->nc = nc;
  m->X.assign(x, x + nv * dim);
  m->c2d.assign(cells, cells + nc * (dim + 1));
  for (int64_t i = 0; i < nc * (dim + 1); ++i)
    if (m->c2d[i] < 0 || m->c2d[i] >= nv) {
      delete m;
      fail(IPCS_E_INVALID, "cell vertex index out of range");
    }
  for (int64_t c = 0; c < nc; ++c) {
    double J[3][3] = {};
    for (int k = 0; k < dim; ++k)
      for (int r = 0; r < dim; ++r)
        J[r][k] = x[(int64_t)cells[c * (dim + 1) + k + 1] * dim + r] -
                  x[(int64_t)cells[c * (dim + 1)] * dim + r];
    double det = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                          : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(std::fabs(det) > 0)) {
      delete m;
      fail(IPCS_E_INVALID, "degenerate cell " + std::to_string(c));
    }
  }
  try {
    finalize(*m);
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

}  // namespace ipcs
