// Host-side mesh, pattern, partition and quadrature code of the library,
// built for the CPU alone with AddressSanitizer and UndefinedBehaviorSanitizer
// (no device code, no HIP calls). It builds every kind of mesh the library
// accepts (both Taylor-Hood pairs, triangles and tetrahedra, structured and
// relabelled, jittered meshes, the smallest ones), partitions their pressure
// patterns at several part sizes, builds the tetrahedral rule, and goes
// through the error paths; every internal structure is checked for
// consistency on the way. Any out-of-bounds access, use after free, leak,
// overflow or other undefined behaviour aborts with the sanitizer's report.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "mesh.hpp"
#include "rules.hpp"

using namespace ipcs;

static int g_checks = 0;

#define CHECK(c)                                                             \
  do {                                                                       \
    ++g_checks;                                                              \
    if (!(c)) {                                                              \
      std::fprintf(stderr, "check failed: %s (%s:%d)\n", #c, __FILE__, __LINE__); \
      std::exit(2);                                                          \
    }                                                                        \
  } while (0)

static void check_pattern(const Pattern& P) {
  CHECK((int64_t)P.rowptr.size() == P.nrows + 1);
  CHECK(P.rowptr[0] == 0 && P.rowptr[P.nrows] == (int32_t)P.col.size());
  for (int64_t i = 0; i < P.nrows; ++i) {
    CHECK(P.rowptr[i] < P.rowptr[i + 1]);
    for (int32_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k) {
      CHECK(P.col[k] >= 0 && P.col[k] < P.ncols);
      if (k > P.rowptr[i]) CHECK(P.col[k] > P.col[k - 1]);
    }
  }
}

static void check_sell(const Pattern& P, const Sell& S) {
  CHECK(S.nrows == P.nrows && S.nslices == (P.nrows + 63) / 64);
  CHECK((int64_t)S.col.size() == S.nent && S.sptr[S.nslices] == S.nent);
  for (int64_t i = 0; i < P.nrows; ++i)
    for (int k = 0; k < P.rowptr[i + 1] - P.rowptr[i]; ++k)
      CHECK(S.col[S.index(i, k)] == P.col[P.rowptr[i] + k]);
}

static void check_parts(const Mesh& m, int rows_max) {
  auto q = m.parts11(rows_max);
  const PartSell& Q = *q;
  CHECK(Q.n == m.n1 && Q.nparts >= 1);
  std::vector<int32_t> seen(Q.n, 0);
  for (int32_t r : Q.perm) {
    CHECK(r >= 0 && r < Q.n);
    seen[r]++;
  }
  for (int32_t c : seen) CHECK(c == 1);
  for (int p = 0; p < Q.nparts; ++p) {
    const int own = Q.part_ptr[p + 1] - Q.part_ptr[p];
    CHECK(own >= 1 && own <= Q.rows_max);
    const int nh = Q.halo_ptr[p + 1] - Q.halo_ptr[p];
    CHECK(own + nh <= Q.lds_max);
    for (int h = Q.halo_ptr[p]; h < Q.halo_ptr[p + 1]; ++h)
      CHECK(Q.halo[h] >= 0 && Q.halo[h] < Q.n &&
            (Q.halo[h] < Q.part_ptr[p] || Q.halo[h] >= Q.part_ptr[p + 1]));
  }
  for (int64_t e = 0; e < Q.nent; ++e) {
    CHECK(Q.src[e] >= -1 && Q.src[e] < m.e11.nent);
  }
  // the second ring (two CG iterations per launch): exactly the columns the
  // halo rows reference outside the part and its halo, and the halo rows'
  // SELL entries resolve to their CSR entries
  auto q2 = m.parts11(rows_max, 2);
  const PartSell& Q2 = *q2;
  CHECK(Q2.depth == 2 && Q2.nparts == Q.nparts && Q2.perm == Q.perm && Q2.halo == Q.halo);
  std::vector<int32_t> iperm(Q2.n);
  for (int64_t i = 0; i < Q2.n; ++i) iperm[Q2.perm[i]] = (int32_t)i;
  const Pattern& P = m.p11;
  for (int p = 0; p < Q2.nparts; ++p) {
    const int p0 = Q2.part_ptr[p], own = Q2.part_ptr[p + 1] - p0;
    const int h0 = Q2.halo_ptr[p], nh = Q2.halo_ptr[p + 1] - h0;
    const int g0 = Q2.halo2_ptr[p], nh2 = Q2.halo2_ptr[p + 1] - g0;
    CHECK(own + nh + nh2 <= Q2.lds2_max);
    auto inside = [&](int32_t c) {
      if (c >= p0 && c < p0 + own) return true;
      return std::binary_search(Q2.halo.begin() + h0, Q2.halo.begin() + h0 + nh, c);
    };
    std::vector<int32_t> want;
    for (int q = 0; q < nh; ++q) {
      const int32_t o = Q2.perm[Q2.halo[h0 + q]];
      for (int32_t k = P.rowptr[o]; k < P.rowptr[o + 1]; ++k)
        if (!inside(iperm[P.col[k]])) want.push_back(iperm[P.col[k]]);
    }
    std::sort(want.begin(), want.end());
    want.erase(std::unique(want.begin(), want.end()), want.end());
    CHECK((int)want.size() == nh2);
    for (int q = 0; q < nh2; ++q) CHECK(Q2.halo2[g0 + q] == want[q]);
    auto resolve = [&](int l) -> int32_t {
      if (l < own) return p0 + l;
      if (l < own + nh) return Q2.halo[h0 + l - own];
      return Q2.halo2[g0 + l - own - nh];
    };
    const int s0 = Q2.hslice_ptr[p], s1 = Q2.hslice_ptr[p + 1];
    CHECK(s1 - s0 == (nh + 63) / 64);
    for (int sl = s0; sl < s1; ++sl) {
      const int w = (Q2.hsptr[sl + 1] - Q2.hsptr[sl]) / 64;
      CHECK((Q2.hsptr[sl + 1] - Q2.hsptr[sl]) % 64 == 0);
      for (int lane = 0; lane < 64; ++lane) {
        const int q = 64 * (sl - s0) + lane;
        const int32_t o = q < nh ? Q2.perm[Q2.halo[h0 + q]] : -1;
        const int len = o >= 0 ? P.rowptr[o + 1] - P.rowptr[o] : 0;
        CHECK(len <= w);
        for (int k = 0; k < w; ++k) {
          const int64_t e = Q2.hsptr[sl] + 64ll * k + lane;
          CHECK(Q2.hlcol[e] < own + nh + nh2);
          if (k < len) {
            CHECK(resolve(Q2.hlcol[e]) == iperm[P.col[P.rowptr[o] + k]]);
            CHECK(Q2.hsrc[e] == m.e11.index(o, k));
          } else {
            CHECK(Q2.hsrc[e] == -1);
          }
        }
      }
    }
  }
  CHECK(Q2.hnent == Q2.hsptr.back());
}

static void check_mesh(const Mesh& m) {
  const int d = m.dim;
  CHECK(m.nloc1 == (m.pair == 0 ? d + 1 : (d == 2 ? 6 : 10)));
  CHECK(m.nloc2 == (m.pair == 0 ? (d == 2 ? 6 : 10) : (d == 2 ? 10 : 20)));
  CHECK((int64_t)m.c2d.size() == m.nc * m.nloc2 && (int64_t)m.c2dp.size() == m.nc * m.nloc1);
  for (int32_t v : m.c2d) CHECK(v >= 0 && v < m.n2);
  for (int32_t v : m.c2dp) CHECK(v >= 0 && v < m.n1);
  // velocity DOFs: every node belongs to a cell, the maps are inverse permutations
  std::vector<char> used(m.n2, 0);
  for (int32_t v : m.c2d) used[v] = 1;
  for (char u : used) CHECK(u);
  for (int64_t i = 0; i < m.n2; ++i) CHECK(m.v_in[m.v_out[i]] == i);
  CHECK((int64_t)m.x2.size() == m.n2 * d && (int64_t)m.xp.size() == m.n1 * d);
  for (double x : m.x2) CHECK(std::isfinite(x));
  for (int32_t b : m.bidx) CHECK(b >= 0 && b < m.n2 && m.bmask[b]);
  for (const Pattern* P : {&m.p22, &m.p11, &m.p12, &m.p21}) check_pattern(*P);
  check_sell(m.p22, m.e22);
  check_sell(m.p11, m.e11);
  check_sell(m.p12, m.e12);
  check_sell(m.p21, m.e21);
  // incidence codes point at cells that hold the row's DOF at that local index
  for (int64_t r = 0; r < m.n2; ++r)
    for (int32_t p = m.inc2.ptr[r]; p < m.inc2.ptr[r + 1]; ++p) {
      const int64_t c = m.inc2.code[p] >> 5;
      const int li = m.inc2.code[p] & 31;
      CHECK(c < m.nc && li < m.nloc2 && m.c2d[c * m.nloc2 + li] == r);
      for (int j = 0; j < m.nloc2; ++j) {
        const int s = m.s22.slot[(int64_t)p * m.s22.stride + j];
        CHECK(m.p22.col[m.p22.rowptr[r] + s] == m.c2d[c * m.nloc2 + j]);
      }
    }
  for (int64_t r = 0; r < m.n1; ++r)
    for (int32_t p = m.inc1.ptr[r]; p < m.inc1.ptr[r + 1]; ++p) {
      const int64_t c = m.inc1.code[p] >> 5;
      const int li = m.inc1.code[p] & 31;
      CHECK(c < m.nc && li < m.nloc1 && m.c2dp[c * m.nloc1 + li] == r);
    }
  for (int rows : {64, 384, 2048}) check_parts(m, rows);
}

// a seeded relabelled and jittered copy of the structured mesh: interior
// vertices moved by up to 0.2 h, vertex labels permuted, cells shuffled and
// every other cell's orientation flipped
static Mesh* jittered(int dim, int n, unsigned seed, int pair) {
  std::unique_ptr<Mesh> s(dim == 2 ? build_unit_square(n, n) : build_unit_cube(n, n, n));
  uint64_t st = 0x9e3779b97f4a7c15ull ^ seed;
  auto rnd = [&]() {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
  };
  const int64_t nv = s->nv, nc = s->nc;
  std::vector<double> X(s->X);
  for (int64_t v = 0; v < nv; ++v) {
    bool inner = true;
    for (int r = 0; r < dim; ++r) inner &= X[v * dim + r] > 1e-12 && X[v * dim + r] < 1 - 1e-12;
    if (inner)
      for (int r = 0; r < dim; ++r) X[v * dim + r] += (0.4 / n) * ((rnd() % 1001) / 1000.0 - 0.5);
  }
  std::vector<int32_t> perm(nv), inv(nv);
  std::iota(perm.begin(), perm.end(), 0);
  for (int64_t i = nv - 1; i > 0; --i) std::swap(perm[i], perm[rnd() % (i + 1)]);
  for (int64_t i = 0; i < nv; ++i) inv[perm[i]] = (int32_t)i;
  std::vector<double> Xp(X.size());
  for (int64_t v = 0; v < nv; ++v)
    for (int r = 0; r < dim; ++r) Xp[inv[v] * dim + r] = X[v * dim + r];
  std::vector<int64_t> order(nc);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t i = nc - 1; i > 0; --i) std::swap(order[i], order[rnd() % (i + 1)]);
  std::vector<int32_t> cells(nc * (dim + 1));
  for (int64_t c = 0; c < nc; ++c) {
    for (int k = 0; k <= dim; ++k)
      cells[c * (dim + 1) + k] = inv[s->c2dp[order[c] * s->nloc1 + k]];
    if (c & 1) std::swap(cells[c * (dim + 1)], cells[c * (dim + 1) + 1]);
  }
  return build_from_arrays(dim, nv, Xp.data(), nc, cells.data(), pair);
}

template <class F>
static void expect_error(F f) {
  bool threw = false;
  try {
    f();
  } catch (const Error& e) {
    threw = e.code != IPCS_OK;
  }
  CHECK(threw);
}

int main() {
  int meshes = 0;
  for (int pair : {0, 1}) {
    for (int n : {1, 2, 5, 16}) {
      std::unique_ptr<Mesh> m(build_unit_square(n, n, pair));
      check_mesh(*m);
      ++meshes;
    }
    std::unique_ptr<Mesh> r(build_unit_square(7, 3, pair));
    check_mesh(*r);
    for (int n : {1, 2, 4}) {
      std::unique_ptr<Mesh> m(build_unit_cube(n, n, n, pair));
      check_mesh(*m);
      ++meshes;
    }
    std::unique_ptr<Mesh> c(build_unit_cube(3, 2, 1, pair));
    check_mesh(*c);
    for (unsigned seed : {1u, 2u}) {
      std::unique_ptr<Mesh> a(jittered(2, 9, seed, pair));
      check_mesh(*a);
      std::unique_ptr<Mesh> b(jittered(3, 3, seed, pair));
      check_mesh(*b);
      meshes += 2;
    }
  }
  // the tetrahedral rule of the P3-P2 pair: positive weights summing to 1/6
  std::vector<double> lam(4 * RuleTet9::NQ), w(RuleTet9::NQ);
  tet_rule9(lam.data(), w.data());
  double sw = 0.0;
  for (int q = 0; q < RuleTet9::NQ; ++q) {
    CHECK(w[q] > 0.0);
    sw += w[q];
    double sl = 0.0;
    for (int k = 0; k < 4; ++k) sl += lam[4 * q + k];
    CHECK(std::fabs(sl - 1.0) < 1e-14);
  }
  CHECK(std::fabs(sw - 1.0 / 6.0) < 1e-15);
  // error paths
  expect_error([] { delete build_unit_square(0, 3); });
  expect_error([] { delete build_unit_cube(2, 0, 2); });
  expect_error([] { delete build_unit_square(2, 2, 7); });
  expect_error([] {
    const double x[6] = {0, 0, 1, 0, 0, 1};
    const int32_t cells[3] = {0, 1, 5};
    delete build_from_arrays(2, 3, x, 1, cells);
  });
  expect_error([] {
    const double x[6] = {0, 0, 1, 0, 2, 0};   // degenerate (zero-area) cell
    const int32_t cells[3] = {0, 1, 2};
    delete build_from_arrays(2, 3, x, 1, cells);
  });
  expect_error([] { delete build_from_arrays(4, 3, nullptr, 1, nullptr); });
  std::printf("host sanitizer run: %d meshes, %d checks, ok\n", meshes, g_checks);
  std::fflush(stdout);
  return 0;
}
