// extern "C" entry points declared in include/ipcs.h. Every call converts
// exceptions into status codes and records a thread-local message.
#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "ipcs.h"
#include "mesh.hpp"
#include "rules.hpp"
#include "run.hpp"
#include "steady.hpp"

struct ipcs_mesh_s {
  std::shared_ptr<ipcs::Mesh> m;
};
struct ipcs_run_s {
  ipcs::Run r;
};
struct ipcs_steady_s {
  ipcs::Steady s;
};

namespace {
thread_local std::string g_err;

template <class F>
int guard(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const ipcs::Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return IPCS_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return IPCS_E_INVALID;
  } catch (...) {
    g_err = "unknown error";
    return IPCS_E_INVALID;
  }
}

void need(bool c, const char* msg) {
  if (!c) ipcs::fail(IPCS_E_INVALID, msg);
}

const ipcs::Mesh& M(ipcs_mesh m) {
  need(m && m->m, "null mesh handle");
  return *m->m;
}

ipcs::Run& R(ipcs_run r) {
  need(r != nullptr, "null run handle");
  return r->r;
}

ipcs::Steady& S(ipcs_steady s) {
  need(s != nullptr, "null steady handle");
  return s->s;
}

int wrap_mesh(ipcs::Mesh* raw, ipcs_mesh* out) {
  std::unique_ptr<ipcs::Mesh> own(raw);
  auto* h = new ipcs_mesh_s;
  h->m.reset(own.release());
  *out = h;
  return IPCS_OK;
}

void check_params(const ipcs_params* p) {
  need(p != nullptr, "null params");
  need(p->nu >= 0 && p->dt > 0 && p->rho > 0, "need nu >= 0, dt > 0, rho > 0");
  need(p->tol_mom > 0 && p->tol_p > 0 && p->tol_corr > 0, "tolerances must be positive");
  need(p->maxit > 0, "maxit must be positive");
  need(p->precision == IPCS_FP64 || p->precision == IPCS_MIXED, "unknown precision");
  need(p->convection == IPCS_CONV_EXPLICIT || p->convection == IPCS_CONV_SEMI_IMPLICIT,
       "unknown convection form");
  need(p->precision == IPCS_FP64 || p->tol_ir > 0, "the mixed form needs tol_ir > 0");
  need(p->poisson_s >= 0 && p->poisson_s <= 2, "poisson_s must be 0, 1 or 2");
  need(p->poisson_part_rows == 0 || p->poisson_part_rows == -1 ||
           (p->poisson_part_rows >= 64 && p->poisson_part_rows <= 2048),
       "poisson_part_rows must be 0, -1 or in [64, 2048]");
  need(p->scheme == IPCS_SCHEME_IPCS || p->scheme == IPCS_SCHEME_CHORIN, "unknown scheme");
  need(p->poisson_start == IPCS_START_ZERO || p->poisson_start == IPCS_START_PREVIOUS,
       "unknown Poisson start");
  need(p->momentum_start == IPCS_MSTART_EXTRAPOLATED || p->momentum_start == IPCS_MSTART_STATE,
       "unknown momentum start");
}

// The interface numbers velocity DOFs in listing order, the library
// internally in coordinate order (mesh.hpp: v_out, v_in). These convert the
// velocity-indexed data that crosses the interface.
// out[c][v_out[i]] = in[c][i] for ncomp components of n2 values
void vel_to_interface(const ipcs::Mesh& m, int ncomp, const double* in, double* out) {
  const int64_t n = m.n2;
  for (int c = 0; c < ncomp; ++c)
    for (int64_t i = 0; i < n; ++i) out[c * n + m.v_out[i]] = in[c * n + i];
}
// out[c][i] = in[c][v_out[i]]
void vel_to_internal(const ipcs::Mesh& m, int ncomp, const double* in, double* out) {
  const int64_t n = m.n2;
  for (int c = 0; c < ncomp; ++c)
    for (int64_t i = 0; i < n; ++i) out[c * n + i] = in[c * n + m.v_out[i]];
}
// A CSR pattern (and values, if val) of the internal numbering in the
// interface numbering: velocity rows and/or columns relabelled, rows in
// interface order, columns ascending within each row.
void csr_to_interface(const ipcs::Mesh& m, const ipcs::Pattern& P, bool vrows, bool vcols,
                      const double* val, int32_t* rowptr, int32_t* col, double* vout) {
  std::vector<int32_t> rp(P.nrows + 1, 0);
  for (int64_t e = 0; e < P.nrows; ++e) {
    const int64_t r = vrows ? m.v_in[e] : e;
    rp[e + 1] = rp[e] + (P.rowptr[r + 1] - P.rowptr[r]);
  }
  std::vector<std::pair<int32_t, int32_t>> row;   // (interface column, internal entry)
  for (int64_t e = 0; e < P.nrows; ++e) {
    const int64_t r = vrows ? m.v_in[e] : e;
    row.clear();
    for (int32_t k = P.rowptr[r]; k < P.rowptr[r + 1]; ++k)
      row.emplace_back(vcols ? m.v_out[P.col[k]] : P.col[k], k);
    std::sort(row.begin(), row.end());
    for (size_t q = 0; q < row.size(); ++q) {
      if (col) col[rp[e] + q] = row[q].first;
      if (vout) vout[rp[e] + q] = val[row[q].second];
    }
  }
  if (rowptr) std::memcpy(rowptr, rp.data(), sizeof(int32_t) * (P.nrows + 1));
}
bool velocity_rows(int pattern) {
  return pattern == IPCS_PATTERN_P2P2 || pattern == IPCS_PATTERN_P2P1;
}
bool velocity_cols(int pattern) {
  return pattern == IPCS_PATTERN_P2P2 || pattern == IPCS_PATTERN_P1P2;
}

}  // namespace

extern "C" {

const char* ipcs_last_error(void) { return g_err.c_str(); }

int ipcs_mesh_unit_square(int32_t nx, int32_t ny, ipcs_mesh* out) {
  return guard([&]() -> int {
    need(out != nullptr, "null output handle");
    return wrap_mesh(ipcs::build_unit_square(nx, ny), out);
  });
}

int ipcs_mesh_unit_square_pair(int32_t nx, int32_t ny, int32_t pair, ipcs_mesh* out) {
  return guard([&]() -> int {
    need(out != nullptr, "null output handle");
    return wrap_mesh(ipcs::build_unit_square(nx, ny, pair), out);
  });
}

int ipcs_mesh_unit_cube(int32_t nx, int32_t ny, int32_t nz, ipcs_mesh* out) {
  return guard([&]() -> int {
    need(out != nullptr, "null output handle");
    return wrap_mesh(ipcs::build_unit_cube(nx, ny, nz), out);
  });
}

int ipcs_mesh_unit_cube_pair(int32_t nx, int32_t ny, int32_t nz, int32_t pair, ipcs_mesh* out) {
  return guard([&]() -> int {
    need(out != nullptr, "null output handle");
    return wrap_mesh(ipcs::build_unit_cube(nx, ny, nz, pair), out);
  });
}

int ipcs_mesh_from_arrays(int32_t dim, int64_t nv, const double* x, int64_t nc,
                          const int32_t* cells, ipcs_mesh* out) {
  return guard([&]() -> int {
    need(out != nullptr, "null output handle");
    return wrap_mesh(ipcs::build_from_arrays(dim, nv, x, nc, cells), out);
  });
}

int ipcs_mesh_from_arrays_pair(int32_t dim, int64_t nv, const double* x, int64_t nc,
                               const int32_t* cells, int32_t pair, ipcs_mesh* out) {
  return guard([&]() -> int {
    need(out != nullptr, "null output handle");
    return wrap_mesh(ipcs::build_from_arrays(dim, nv, x, nc, cells, pair), out);
  });
}

int ipcs_mesh_pair(ipcs_mesh m, int32_t* pair) {
  return guard([&]() -> int {
    const ipcs::Mesh& mm = M(m);
    need(pair != nullptr, "null output");
    *pair = mm.pair;
    return IPCS_OK;
  });
}

int ipcs_mesh_counts(ipcs_mesh m, ipcs_counts* out) {
  return guard([&]() -> int {
    const ipcs::Mesh& mm = M(m);
    need(out != nullptr, "null output");
    std::memset(out, 0, sizeof(*out));
    out->dim = mm.dim;
    out->nv = mm.nv;
    out->nc = mm.nc;
    out->n1 = mm.n1;
    out->n2 = mm.n2;
    for (int k = 0; k < 4; ++k) out->nnz[k] = mm.pattern(k).nnz();
    out->nb2 = (int64_t)mm.bidx.size();
    return IPCS_OK;
  });
}

int ipcs_mesh_dof_coords(ipcs_mesh m, int32_t space, double* out, int64_t cap) {
  return guard([&]() -> int {
    const ipcs::Mesh& mm = M(m);
    need(space == IPCS_SPACE_P1 || space == IPCS_SPACE_P2, "unknown space");
    const int64_t n = (space == IPCS_SPACE_P1 ? mm.n1 : mm.n2) * mm.dim;
    need(out != nullptr && cap >= n, "output buffer too small");
    if (space == IPCS_SPACE_P1) {
      std::memcpy(out, mm.xp.data(), sizeof(double) * n);
    } else {
      for (int64_t i = 0; i < mm.n2; ++i)
        for (int a = 0; a < mm.dim; ++a) out[(int64_t)mm.v_out[i] * mm.dim + a] = mm.x2[i * mm.dim + a];
    }
    return IPCS_OK;
  });
}

int ipcs_mesh_cell_dofs(ipcs_mesh m, int32_t space, int32_t* out, int64_t cap) {
  return guard([&]() -> int {
    const ipcs::Mesh& mm = M(m);
    need(space == IPCS_SPACE_P1 || space == IPCS_SPACE_P2, "unknown space");
    const int nl = space == IPCS_SPACE_P1 ? mm.nloc1 : mm.nloc2;
    need(out != nullptr && cap >= mm.nc * nl, "output buffer too small");
    if (space == IPCS_SPACE_P1)
      for (int64_t i = 0; i < mm.nc * nl; ++i) out[i] = mm.c2dp[i];
    else
      for (int64_t i = 0; i < mm.nc * nl; ++i) out[i] = mm.v_out[mm.c2d[i]];
    return IPCS_OK;
  });
}

int ipcs_mesh_boundary(ipcs_mesh m, uint8_t* out, int64_t cap) {
  return guard([&]() -> int {
    const ipcs::Mesh& mm = M(m);
    need(out != nullptr && cap >= mm.n2, "output buffer too small");
    for (int64_t i = 0; i < mm.n2; ++i) out[mm.v_out[i]] = mm.bmask[i];
    return IPCS_OK;
  });
}

int ipcs_mesh_pattern(ipcs_mesh m, int32_t which, int32_t* rowptr, int64_t cap_rows,
                      int32_t* col, int64_t cap_nnz) {
  return guard([&]() -> int {
    const ipcs::Mesh& mm = M(m);
    const ipcs::Pattern& P = mm.pattern(which);
    need(rowptr != nullptr && cap_rows >= P.nrows + 1, "rowptr buffer too small");
    need(col != nullptr && cap_nnz >= P.nnz(), "col buffer too small");
    csr_to_interface(mm, P, velocity_rows(which), velocity_cols(which), nullptr, rowptr, col,
                     nullptr);
    return IPCS_OK;
  });
}

int ipcs_mesh_p1_partition(ipcs_mesh m, int32_t rows_max, int64_t sizes[5], int32_t* perm,
                           int32_t* part_ptr, int32_t* halo_ptr, int32_t* halo,
                           int32_t* slice_ptr, int32_t* sptr, uint16_t* lcol, int32_t* src) {
  return guard([&]() -> int {
    need(sizes != nullptr, "null sizes");
    need(rows_max >= 64 && rows_max <= 2048, "rows_max must be in [64, 2048]");
    const auto q = M(m).parts11(rows_max);
    sizes[0] = q->nparts;
    sizes[1] = (int64_t)q->halo.size();
    sizes[2] = (int64_t)q->sptr.size() - 1;
    sizes[3] = q->nent;
    sizes[4] = q->lds_max;
    const bool any = perm || part_ptr || halo_ptr || halo || slice_ptr || sptr || lcol || src;
    if (!any) return IPCS_OK;
    // an empty halo (one part) may come as NULL
    need(perm && part_ptr && halo_ptr && (halo || q->halo.empty()) && slice_ptr && sptr &&
             lcol && src,
         "partition arrays must be all NULL or all non-NULL");
    auto cp = [](auto* dst, const auto& v) {
      if (!v.empty()) std::memcpy(dst, v.data(), sizeof(v[0]) * v.size());
    };
    cp(perm, q->perm);
    cp(part_ptr, q->part_ptr);
    cp(halo_ptr, q->halo_ptr);
    cp(halo, q->halo);
    cp(slice_ptr, q->slice_ptr);
    cp(sptr, q->sptr);
    cp(lcol, q->lcol);
    cp(src, q->src);
    return IPCS_OK;
  });
}

int ipcs_quadrature_rule(int32_t dim, int32_t* nq, double* lam, double* w, int64_t cap) {
  return guard([&]() -> int {
    need(dim == 2 || dim == 3, "dim must be 2 or 3");
    const int n = dim == 2 ? ipcs::Rule<2>::NQ : ipcs::Rule<3>::NQ;
    if (nq) *nq = n;
    if (!lam && !w) return IPCS_OK;
    need(lam && w && cap >= (int64_t)n * (dim + 1), "output buffer too small");
    for (int q = 0; q < n; ++q) {
      w[q] = dim == 2 ? ipcs::Rule<2>::w(q) : ipcs::Rule<3>::w(q);
      for (int k = 0; k <= dim; ++k)
        lam[q * (dim + 1) + k] = dim == 2 ? ipcs::Rule<2>::lam(q, k) : ipcs::Rule<3>::lam(q, k);
    }
    return IPCS_OK;
  });
}

int ipcs_quadrature_rule_pair(int32_t dim, int32_t pair, int32_t* nq, double* lam, double* w,
                              int64_t cap) {
  if (pair == IPCS_PAIR_P2P1) return ipcs_quadrature_rule(dim, nq, lam, w, cap);
  return guard([&]() -> int {
    need(dim == 2 || dim == 3, "dim must be 2 or 3");
    need(pair == IPCS_PAIR_P3P2, "unknown Taylor-Hood pair");
    const int n = dim == 2 ? ipcs::RuleT9::NQ : ipcs::RuleTet9::NQ;
    if (nq) *nq = n;
    if (!lam && !w) return IPCS_OK;
    need(lam && w && cap >= (int64_t)n * (dim + 1), "output buffer too small");
    if (dim == 3) {
      ipcs::tet_rule9(lam, w);
      return IPCS_OK;
    }
    for (int q = 0; q < n; ++q) {
      w[q] = ipcs::RuleT9::w(q);
      for (int k = 0; k < 3; ++k) lam[q * 3 + k] = ipcs::RuleT9::lam(q, k);
    }
    return IPCS_OK;
  });
}

void ipcs_mesh_destroy(ipcs_mesh m) { delete m; }

void ipcs_params_default(ipcs_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nu = 0.01;
  p->rho = 1.0;
  p->dt = 1e-3;
  p->t0 = 0.0;
  p->precision = IPCS_FP64;
  p->convection = IPCS_CONV_EXPLICIT;
  p->tol_mom = p->tol_p = p->tol_corr = 1e-12;
  p->tol_ir = 1e-10;
  p->maxit = 20000;
  p->check_every = 16;
  p->callbacks = 0;
}

int ipcs_run_workspace_bytes(ipcs_mesh m, const ipcs_params* p, int64_t* bytes) {
  return guard([&]() -> int {
    check_params(p);
    need(bytes != nullptr, "null output");
    (void)M(m);
    ipcs::Run tmp;
    tmp.mesh = m->m;
    tmp.prm = *p;
    tmp.set_precision();   // the layout of the run's own form
    tmp.sizes_from_mesh();
    ipcs::Carver c;
    tmp.layout(c);
    *bytes = c.off;
    return IPCS_OK;
  });
}

int ipcs_run_create(ipcs_mesh m, const ipcs_params* p, void* dev_ws, int64_t ws_bytes,
                    void* hip_stream, ipcs_run* out) {
  return guard([&]() -> int {
    check_params(p);
    need(out != nullptr, "null output handle");
    (void)M(m);
    std::unique_ptr<ipcs_run_s> h(new ipcs_run_s);
    h->r.create(m->m, *p, dev_ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
    *out = h.release();
    return IPCS_OK;
  });
}

int ipcs_set_viscosity(ipcs_run r, double nu) {
  return guard([&]() -> int {
    need(nu >= 0, "nu must be >= 0");
    R(r).prm.nu = nu;
    R(r).A_dirty = true;
    R(r).clear_history();
    return IPCS_OK;
  });
}

int ipcs_set_time_step(ipcs_run r, double dt) {
  return guard([&]() -> int {
    need(dt > 0, "dt must be > 0");
    R(r).prm.dt = dt;
    R(r).A_dirty = true;
    R(r).clear_history();
    return IPCS_OK;
  });
}

int ipcs_set_forcing(ipcs_run r, ipcs_field_fn f, void* ctx) {
  return guard([&]() -> int {
    ipcs::Run& rr = R(r);
    if (f && !rr.prm.callbacks)
      ipcs::fail(IPCS_E_STATE, "forcing callbacks need a run created with params.callbacks = 1");
    rr.f_cb = f;
    rr.f_ctx = ctx;
    rr.clear_history();
    return IPCS_OK;
  });
}

int ipcs_set_dirichlet(ipcs_run r, ipcs_field_fn g, void* ctx) {
  return guard([&]() -> int {
    R(r).g_cb = g;
    R(r).g_ctx = ctx;
    R(r).clear_history();
    return IPCS_OK;
  });
}

int ipcs_set_builtin_solution(ipcs_run r, int32_t kind, const double* prm, int32_t nprm) {
  return guard([&]() -> int {
    need(nprm >= 0 && (nprm == 0 || prm != nullptr), "bad parameter array");
    R(r).set_builtin(kind, prm, nprm);
    return IPCS_OK;
  });
}

int ipcs_set_state(ipcs_run r, const double* u, const double* p, double t) {
  return guard([&]() -> int {
    need(u != nullptr && p != nullptr, "null state arrays");
    ipcs::Run& rr = R(r);
    std::vector<double> ui((size_t)rr.dim * rr.n2);
    vel_to_internal(*rr.mesh, rr.dim, u, ui.data());
    rr.set_state(ui.data(), p, t);
    return IPCS_OK;
  });
}

int ipcs_advance(ipcs_run r, int32_t nsteps, ipcs_step_stats* stats) {
  return guard([&]() -> int {
    need(nsteps >= 0, "nsteps must be >= 0");
    ipcs::Run& rr = R(r);
    for (int32_t k = 0; k < nsteps; ++k) {
      const int rc = rr.step(stats ? stats + k : nullptr);
      if (rc != IPCS_OK) {
        g_err = "step " + std::to_string(k) + " failed in solve " +
                std::to_string(stats ? stats[k].failed_solve : 0);
        return rc;
      }
    }
    return IPCS_OK;
  });
}

int ipcs_step_phase(ipcs_run r, int32_t phase, ipcs_step_stats* stats) {
  return guard([&]() -> int { return R(r).phase(phase, stats); });
}

static int copy_out(ipcs::Run& rr, const double* src, int64_t n, double* out, int64_t cap) {
  need(out != nullptr && cap >= n, "output buffer too small");
  HIP_OK(hipMemcpyAsync(out, src, sizeof(double) * n, hipMemcpyDeviceToHost, rr.stream));
  HIP_OK(hipStreamSynchronize(rr.stream));
  return IPCS_OK;
}

// a velocity field [dim][n2] of the run, in the interface numbering
static int copy_out_velocity(ipcs::Run& rr, const double* src, double* out, int64_t cap) {
  const int64_t n = (int64_t)rr.dim * rr.n2;
  need(out != nullptr && cap >= n, "output buffer too small");
  std::vector<double> h((size_t)n);
  HIP_OK(hipMemcpyAsync(h.data(), src, sizeof(double) * n, hipMemcpyDeviceToHost, rr.stream));
  HIP_OK(hipStreamSynchronize(rr.stream));
  vel_to_interface(*rr.mesh, rr.dim, h.data(), out);
  return IPCS_OK;
}

int ipcs_get_velocity(ipcs_run r, double* u, int64_t cap) {
  return guard([&]() -> int { ipcs::Run& rr = R(r); return copy_out_velocity(rr, rr.U, u, cap); });
}

int ipcs_get_pressure(ipcs_run r, double* p, int64_t cap) {
  return guard([&]() -> int { ipcs::Run& rr = R(r); return copy_out(rr, rr.P, rr.n1, p, cap); });
}

int ipcs_get_time(ipcs_run r, double* t) {
  return guard([&]() -> int {
    need(t != nullptr, "null output");
    *t = R(r).t;
    return IPCS_OK;
  });
}

int ipcs_get_field(ipcs_run r, int32_t which, double* out, int64_t cap) {
  return guard([&]() -> int {
    ipcs::Run& rr = R(r);
    switch (which) {
      case IPCS_FIELD_U: return copy_out_velocity(rr, rr.U, out, cap);
      case IPCS_FIELD_P: return copy_out(rr, rr.P, rr.n1, out, cap);
      case IPCS_FIELD_USTAR: return copy_out_velocity(rr, rr.Ustar, out, cap);
      case IPCS_FIELD_DP: return copy_out(rr, rr.dP, rr.n1, out, cap);
      case IPCS_FIELD_RHS_MOM: return copy_out_velocity(rr, rr.bU, out, cap);
      case IPCS_FIELD_RHS_P: return copy_out(rr, rr.rP, rr.n1, out, cap);
    }
    ipcs::fail(IPCS_E_INVALID, "unknown field id");
  });
}

int ipcs_export_matrix(ipcs_run r, int32_t which, int32_t* rowptr, int64_t cap_rows,
                       int32_t* col, double* val, int64_t cap_nnz) {
  return guard([&]() -> int {
    ipcs::Run& rr = R(r);
    const ipcs::Mesh& mm = *rr.mesh;
    const void* src = nullptr;
    int pat = IPCS_PATTERN_P2P2;
    if (which == IPCS_MAT_M) src = rr.M;
    else if (which == IPCS_MAT_K) src = rr.K;
    else if (which == IPCS_MAT_E) src = rr.E;
    else if (which == IPCS_MAT_A_ELIM) src = rr.Ael;
    else if (which == IPCS_MAT_M_ELIM) src = rr.Mel;
    else if (which == IPCS_MAT_KP) {
      src = rr.Kp;
      pat = IPCS_PATTERN_P1P1;
    } else if (which >= IPCS_MAT_D0 && which < IPCS_MAT_D0 + rr.dim) {
      src = rr.Dc[which - IPCS_MAT_D0];
      pat = IPCS_PATTERN_P1P2;
    } else if (which >= IPCS_MAT_G0 && which < IPCS_MAT_G0 + rr.dim) {
      src = rr.Gc[which - IPCS_MAT_G0];
      pat = IPCS_PATTERN_P2P1;
    } else if (which == IPCS_MAT_A) {
      ipcs::fail(IPCS_E_INVALID, "A is stored Dirichlet-eliminated: use IPCS_MAT_A_ELIM");
    } else {
      ipcs::fail(IPCS_E_INVALID, "unknown matrix id");
    }
    const ipcs::Pattern& P = mm.pattern(pat);
    if (rowptr) need(cap_rows >= P.nrows + 1, "rowptr buffer too small");
    need(val != nullptr && cap_nnz >= P.nnz(), "value buffer too small");
    if (rr.A_dirty) rr.reform_A();
    std::vector<double> v((size_t)P.nnz());
    rr.export_values(pat, src, pat == IPCS_PATTERN_P1P2 ? 8 : rr.vsz, v.data());
    csr_to_interface(mm, P, velocity_rows(pat), velocity_cols(pat), v.data(), rowptr, col, val);
    return IPCS_OK;
  });
}

int ipcs_batch_step(ipcs_run* runs, int32_t nruns, void* hip_stream, ipcs_step_stats* stats) {
  return guard([&]() -> int {
    need(runs != nullptr && nruns > 0, "need at least one run");
    std::vector<ipcs::Run*> rs((size_t)nruns);
    for (int i = 0; i < nruns; ++i) {
      need(runs[i] != nullptr, "null run in the batch");
      rs[i] = &R(runs[i]);
      for (int k = 0; k < i; ++k) need(rs[k] != rs[i], "a run appears twice in the batch");
    }
    return ipcs::batch_step(rs.data(), nruns, static_cast<hipStream_t>(hip_stream), stats);
  });
}

int ipcs_batch_step_noalloc(ipcs_run* runs, int32_t nruns, void* hip_stream,
                            ipcs_step_stats* stats) {
  return guard([&]() -> int {
    need(runs != nullptr && nruns > 0, "need at least one run");
    if (nruns > IPCS_BATCH_NOALLOC_MAX_RUNS)
      ipcs::fail(IPCS_E_CAPACITY, "more runs than IPCS_BATCH_NOALLOC_MAX_RUNS in one batch");
    std::vector<ipcs::Run*> rs((size_t)nruns);
    for (int i = 0; i < nruns; ++i) {
      need(runs[i] != nullptr, "null run in the batch");
      rs[i] = &R(runs[i]);
      for (int k = 0; k < i; ++k) need(rs[k] != rs[i], "a run appears twice in the batch");
    }
    ipcs::BatchMem mem;
    mem.dev = ipcs::batch_scratch(&mem.dev_cap);
    mem.host = ipcs::batch_host_staging(&mem.host_cap);
    const size_t bytes = ipcs::batch_descriptor_bytes(rs.data(), nruns);
    if (bytes > mem.dev_cap)
      ipcs::fail(IPCS_E_CAPACITY, "the batch's descriptors need " + std::to_string(bytes) +
                                      " bytes, more than IPCS_BATCH_SCRATCH_BYTES");
    return ipcs::batch_step(rs.data(), nruns, static_cast<hipStream_t>(hip_stream), stats, mem);
  });
}

int ipcs_profile_kernel(ipcs_run r, int32_t kernel, int32_t nlaunch, double* us_per_launch) {
  return guard([&]() -> int {
    need(nlaunch > 0 && us_per_launch != nullptr, "need nlaunch > 0 and an output");
    *us_per_launch = R(r).profile_kernel(kernel, nlaunch);
    return IPCS_OK;
  });
}

int ipcs_kernel_timing(ipcs_run r, uint32_t mask) {
  return guard([&]() -> int {
    need(mask < (1u << IPCS_NKERNEL), "kernel mask has bits beyond IPCS_NKERNEL");
    R(r).timer.reset(mask);
    return IPCS_OK;
  });
}

int ipcs_kernel_times(ipcs_run r, double* ms, int64_t* launches, int32_t cap) {
  return guard([&]() -> int {
    need(ms != nullptr && launches != nullptr && cap >= IPCS_NKERNEL,
         "need outputs with room for IPCS_NKERNEL entries");
    const ipcs::KTimer& T = R(r).timer;
    for (int k = 0; k < IPCS_NKERNEL; ++k) {
      ms[k] = T.ms[k];
      launches[k] = T.cnt[k];
    }
    return IPCS_OK;
  });
}

int ipcs_poisson_partition(ipcs_run r, int32_t* rows_max, int32_t* nparts, int64_t* halo_rows,
                           int32_t* lds_rows) {
  return guard([&]() -> int {
    const auto& pp = R(r).pp;
    if (rows_max) *rows_max = pp ? pp->rows_max : 0;
    if (nparts) *nparts = pp ? pp->nparts : 0;
    if (halo_rows) *halo_rows = pp ? (int64_t)pp->halo.size() : 0;
    if (lds_rows) *lds_rows = pp ? pp->lds_max : 0;
    return IPCS_OK;
  });
}

void ipcs_run_destroy(ipcs_run r) { delete r; }

void ipcs_steady_params_default(ipcs_steady_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nu = 1.0;
  p->tol = 1e-10;
  p->maxit = 10;
  p->restart = 60;
  p->lin_tol = 1e-12;
  p->lin_maxit = 3000;
  p->inner_maxit = 2000;
  p->inner_tol = 1e-2;
}

int ipcs_steady_workspace_bytes(ipcs_mesh m, const ipcs_steady_params* p, int64_t* bytes) {
  return guard([&]() -> int {
    need(p != nullptr && bytes != nullptr, "null argument");
    (void)M(m);
    ipcs::Steady tmp;
    *bytes = tmp.measure(m->m, *p);
    return IPCS_OK;
  });
}

int ipcs_steady_create(ipcs_mesh m, const ipcs_steady_params* p, void* dev_ws, int64_t ws_bytes,
                       void* hip_stream, ipcs_steady* out) {
  return guard([&]() -> int {
    need(p != nullptr && out != nullptr, "null argument");
    (void)M(m);
    auto h = std::make_unique<ipcs_steady_s>();
    h->s.create(m->m, *p, dev_ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
    *out = h.release();
    return IPCS_OK;
  });
}

int ipcs_steady_set_builtin(ipcs_steady s, int32_t kind, const double* prm, int32_t nprm) {
  return guard([&]() -> int {
    need(nprm >= 0 && (nprm == 0 || prm != nullptr), "bad parameter array");
    S(s).set_builtin(kind, prm, nprm);
    return IPCS_OK;
  });
}

int ipcs_steady_set_state(ipcs_steady s, const double* u, const double* p) {
  return guard([&]() -> int {
    need(u != nullptr && p != nullptr, "null field");
    ipcs::Steady& st = S(s);
    std::vector<double> ui((size_t)st.nu_rows);
    vel_to_internal(*st.run.mesh, st.dim, u, ui.data());
    st.set_state(ui.data(), p);
    return IPCS_OK;
  });
}

int ipcs_steady_step(ipcs_steady s, ipcs_steady_stats* stats) {
  return guard([&]() -> int {
    ipcs::Steady& st = S(s);
    st.lin_it = st.inner_it = 0;
    st.newton_step(stats);
    if (stats) stats->inner_it += st.inner_it;
    st.to_run();
    return IPCS_OK;
  });
}

int ipcs_steady_solve(ipcs_steady s, ipcs_steady_stats* stats) {
  return guard([&]() -> int {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    const int rc = S(s).solve(stats);
    if (stats) stats->status = rc;
    return rc;
  });
}

int ipcs_steady_get_velocity(ipcs_steady s, double* u, int64_t cap) {
  return guard([&]() -> int {
    ipcs::Steady& st = S(s);
    return copy_out_velocity(st.run, st.x, u, cap);
  });
}

int ipcs_steady_get_pressure(ipcs_steady s, double* p, int64_t cap) {
  return guard([&]() -> int {
    ipcs::Steady& st = S(s);
    return copy_out(st.run, st.x + st.nu_rows, st.n1, p, cap);
  });
}

int ipcs_steady_get_vector(ipcs_steady s, int32_t which, double* out, int64_t cap) {
  return guard([&]() -> int {
    ipcs::Steady& st = S(s);
    need(which == IPCS_STEADY_RESIDUAL || which == IPCS_STEADY_INCREMENT, "unknown vector id");
    need(out != nullptr && cap >= st.n, "output buffer too small");
    const double* src = which == IPCS_STEADY_RESIDUAL ? st.R : st.dx;
    copy_out_velocity(st.run, src, out, cap);
    return copy_out(st.run, src + st.nu_rows, st.n1, out + st.nu_rows, cap - st.nu_rows);
  });
}

void ipcs_steady_destroy(ipcs_steady s) { delete s; }

}  // extern "C"
