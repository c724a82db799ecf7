// The C ABI's host-side calls (mesh creation and queries, pattern, partition
// and quadrature exports, parameter defaults, workspace sizing of the
// transient and steady solvers, argument checks and error reporting) with the
// library's host translation units built under AddressSanitizer, LeakSanitizer
// and UndefinedBehaviorSanitizer. No call here reaches the device: the driver
// runs on a machine without a GPU. Any sanitizer report aborts the run.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ipcs.h"

static int g_checks = 0;

#define CHECK(c)                                                                   \
  do {                                                                             \
    ++g_checks;                                                                    \
    if (!(c)) {                                                                    \
      std::fprintf(stderr, "check failed: %s (%s:%d) last error: %s\n", #c, __FILE__, \
                   __LINE__, ipcs_last_error());                                   \
      std::exit(2);                                                                \
    }                                                                              \
  } while (0)

static void query_mesh(ipcs_mesh m, int dim, int pair) {
  int32_t pr = -1;
  CHECK(ipcs_mesh_pair(m, &pr) == IPCS_OK && pr == pair);
  ipcs_counts c;
  CHECK(ipcs_mesh_counts(m, &c) == IPCS_OK && c.dim == dim);
  std::vector<double> x2(c.n2 * dim), x1(c.n1 * dim);
  CHECK(ipcs_mesh_dof_coords(m, IPCS_SPACE_P2, x2.data(), (int64_t)x2.size()) == IPCS_OK);
  CHECK(ipcs_mesh_dof_coords(m, IPCS_SPACE_P1, x1.data(), (int64_t)x1.size()) == IPCS_OK);
  CHECK(ipcs_mesh_dof_coords(m, IPCS_SPACE_P2, x2.data(), (int64_t)x2.size() - 1) != IPCS_OK);
  const int nl2 = pair == IPCS_PAIR_P2P1 ? (dim == 2 ? 6 : 10) : (dim == 2 ? 10 : 20);
  const int nl1 = pair == IPCS_PAIR_P2P1 ? dim + 1 : (dim == 2 ? 6 : 10);
  std::vector<int32_t> c2(c.nc * nl2), c1(c.nc * nl1);
  CHECK(ipcs_mesh_cell_dofs(m, IPCS_SPACE_P2, c2.data(), (int64_t)c2.size()) == IPCS_OK);
  CHECK(ipcs_mesh_cell_dofs(m, IPCS_SPACE_P1, c1.data(), (int64_t)c1.size()) == IPCS_OK);
  CHECK(ipcs_mesh_cell_dofs(m, 9, c1.data(), (int64_t)c1.size()) != IPCS_OK);
  for (int32_t v : c2) CHECK(v >= 0 && v < c.n2);
  std::vector<uint8_t> b(c.n2);
  CHECK(ipcs_mesh_boundary(m, b.data(), (int64_t)b.size()) == IPCS_OK);
  int64_t nb = 0;
  for (uint8_t v : b) nb += v;
  CHECK(nb == c.nb2);
  for (int which = 0; which < 4; ++which) {
    const int64_t rows = (which == IPCS_PATTERN_P2P2 || which == IPCS_PATTERN_P2P1) ? c.n2 : c.n1;
    std::vector<int32_t> rp(rows + 1), col(c.nnz[which]);
    CHECK(ipcs_mesh_pattern(m, which, rp.data(), (int64_t)rp.size(), col.data(),
                            (int64_t)col.size()) == IPCS_OK);
    CHECK(rp[rows] == c.nnz[which]);
    CHECK(ipcs_mesh_pattern(m, which, rp.data(), (int64_t)rp.size(), col.data(),
                            (int64_t)col.size() - 1) != IPCS_OK);
  }
  for (int32_t rows_max : {64, 384}) {
    int64_t sz[5] = {};
    CHECK(ipcs_mesh_p1_partition(m, rows_max, sz, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, nullptr) == IPCS_OK);
    std::vector<int32_t> perm(c.n1), pp(sz[0] + 1), hp(sz[0] + 1), halo(sz[1]), slp(sz[0] + 1),
        sptr(sz[2] + 1), src(sz[3]);
    std::vector<uint16_t> lcol(sz[3]);
    CHECK(ipcs_mesh_p1_partition(m, rows_max, sz, perm.data(), pp.data(), hp.data(), halo.data(),
                                 slp.data(), sptr.data(), lcol.data(), src.data()) == IPCS_OK);
    CHECK(pp[sz[0]] == c.n1);
  }
  ipcs_params p;
  ipcs_params_default(&p);
  int64_t bytes = 0;
  CHECK(ipcs_run_workspace_bytes(m, &p, &bytes) == IPCS_OK && bytes > 0);
  p.precision = IPCS_MIXED;
  int64_t bytes32 = 0;
  CHECK(ipcs_run_workspace_bytes(m, &p, &bytes32) == IPCS_OK && bytes32 > 0);
  p.dt = -1.0;
  CHECK(ipcs_run_workspace_bytes(m, &p, &bytes) != IPCS_OK);
  ipcs_steady_params sp;
  ipcs_steady_params_default(&sp);
  int64_t sbytes = 0;
  const int rc = ipcs_steady_workspace_bytes(m, &sp, &sbytes);
  CHECK(pair == IPCS_PAIR_P2P1 ? (rc == IPCS_OK && sbytes > bytes32) : rc != IPCS_OK);
}

int main() {
  int meshes = 0;
  for (int pair : {IPCS_PAIR_P2P1, IPCS_PAIR_P3P2}) {
    for (int n : {1, 3, 8}) {
      ipcs_mesh m = nullptr;
      CHECK(ipcs_mesh_unit_square_pair(n, n + 1, pair, &m) == IPCS_OK);
      query_mesh(m, 2, pair);
      ipcs_mesh_destroy(m);
      ++meshes;
    }
    for (int n : {1, 2, 3}) {
      ipcs_mesh m = nullptr;
      CHECK(ipcs_mesh_unit_cube_pair(n, n, n + 1, pair, &m) == IPCS_OK);
      query_mesh(m, 3, pair);
      ipcs_mesh_destroy(m);
      ++meshes;
    }
    // one tetrahedron and two triangles given as arrays (one of them clockwise)
    const double xt[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
    const int32_t ct[4] = {0, 2, 1, 3};
    ipcs_mesh m = nullptr;
    CHECK(ipcs_mesh_from_arrays_pair(3, 4, xt, 1, ct, pair, &m) == IPCS_OK);
    query_mesh(m, 3, pair);
    ipcs_mesh_destroy(m);
    const double xs[8] = {0, 0, 1, 0, 1, 1, 0, 1};
    const int32_t cs[6] = {0, 1, 2, 0, 3, 2};
    CHECK(ipcs_mesh_from_arrays_pair(2, 4, xs, 2, cs, pair, &m) == IPCS_OK);
    query_mesh(m, 2, pair);
    ipcs_mesh_destroy(m);
    meshes += 2;
  }
  for (int dim : {2, 3})
    for (int pair : {IPCS_PAIR_P2P1, IPCS_PAIR_P3P2}) {
      int32_t nq = 0;
      CHECK(ipcs_quadrature_rule_pair(dim, pair, &nq, nullptr, nullptr, 0) == IPCS_OK && nq > 0);
      std::vector<double> lam(nq * (dim + 1)), w(nq);
      CHECK(ipcs_quadrature_rule_pair(dim, pair, &nq, lam.data(), w.data(),
                                      (int64_t)lam.size()) == IPCS_OK);
      CHECK(ipcs_quadrature_rule_pair(dim, pair, &nq, lam.data(), w.data(),
                                      (int64_t)lam.size() - 1) != IPCS_OK);
    }
  // argument checks and their messages
  ipcs_mesh m = nullptr;
  CHECK(ipcs_mesh_unit_square(0, 3, &m) != IPCS_OK && std::strlen(ipcs_last_error()) > 0);
  CHECK(ipcs_mesh_unit_cube_pair(2, 2, 2, 5, &m) != IPCS_OK);
  CHECK(ipcs_mesh_unit_square(2, 2, nullptr) != IPCS_OK);
  CHECK(ipcs_mesh_counts(nullptr, nullptr) != IPCS_OK);
  const double xbad[6] = {0, 0, 1, 0, 2, 0};
  const int32_t cbad[3] = {0, 1, 2};
  CHECK(ipcs_mesh_from_arrays(2, 3, xbad, 1, cbad, &m) != IPCS_OK);
  const int32_t cout_[3] = {0, 1, 3};
  CHECK(ipcs_mesh_from_arrays(2, 3, xbad, 1, cout_, &m) != IPCS_OK);
  CHECK(ipcs_quadrature_rule(4, nullptr, nullptr, nullptr, 0) != IPCS_OK);
  ipcs_mesh_destroy(nullptr);
  ipcs_run_destroy(nullptr);
  ipcs_steady_destroy(nullptr);
  std::printf("host C ABI sanitizer run: %d meshes, %d checks, ok\n", meshes, g_checks);
  std::fflush(stdout);
  return 0;
}
