// IPCS run: workspace layout, constant-matrix assembly, the three sub-steps of
// eq. (9) (Section 2.2.1) and the host side of the Krylov solves.
#include "run.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "builtin.hpp"
#include "common.hpp"
#include "rules.hpp"

namespace ipcs {

constexpr int NBLK_MAX = 1024;

int lanes_for(double avg_row) {
  int g = 4;
  while (g < 64 && g < avg_row) g *= 2;
  return g;
}

int nblk_for(int64_t n, int G) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(div_up(n, BLOCK / G), NBLK_MAX));
}

void build_bmap(const std::vector<int>& nblk, std::vector<int2>& bmap) {
  bmap.clear();
  int mx = 0;
  for (int b : nblk) mx = std::max(mx, b);
  // interleave systems block by block so that systems sharing a matrix read it
  // at nearly the same time (cache reuse across velocity components)
  for (int b = 0; b < mx; ++b)
    for (size_t s = 0; s < nblk.size(); ++s)
      if (b < nblk[s]) bmap.push_back(make_int2((int)s, b));
}

static AsmCfg asm_cfg(const Pattern& P, int nout) {
  for (int bs : {256, 128, 64, 32}) {
    int64_t mx = 0;
    for (int64_t r0 = 0; r0 < P.nrows; r0 += bs) {
      const int64_t r1 = std::min<int64_t>(r0 + bs, P.nrows);
      mx = std::max<int64_t>(mx, P.rowptr[r1] - P.rowptr[r0]);
    }
    const size_t lds = (size_t)nout * mx * sizeof(double);
    if (lds <= 65536) return AsmCfg{bs, std::max<size_t>(lds, 8)};
  }
  fail(IPCS_E_INVALID, "matrix rows too long for the assembly kernel");
}

static int status_to_code(int s) {
  switch (s) {
    case KS_MAXIT: return IPCS_E_NOT_CONVERGED;
    case KS_BREAKDOWN: return IPCS_E_BREAKDOWN;
    case KS_NONFINITE: return IPCS_E_NONFINITE;
  }
  return IPCS_OK;
}

int krylov_solve(hipStream_t s, const SolveSet& S, KMethod m, int check_every,
                 std::vector<KState>& hs, KState* pinned) {
  const int n = S.nsys;
  hs.resize(n);
  auto fetch = [&]() {
    gather_states(s, S.d_sys, n, S.d_poll);
    HIP_OK(hipMemcpyAsync(pinned, S.d_poll, sizeof(KState) * n, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    std::memcpy(hs.data(), pinned, sizeof(KState) * n);
  };
  auto init = [&](int mode) {
    if (m == KMethod::PCG) pcg_init(s, S.G, S.d_sys, S.d_bmap, S.nblocks, mode);
    else bicg_init(s, S.G, S.d_sys, S.d_bmap, S.nblocks, mode);
  };
  init(0);
  int chunk = 2;
  const int cap = std::max(1, check_every);
  for (;;) {
    fetch();
    bool pend = false, run = false;
    for (const auto& k : hs) pend |= (k.status == KS_PENDING || k.status == KS_RESTART);
    if (pend) {
      init(1);
      fetch();
    }
    for (const auto& k : hs) run |= (k.status == KS_RUN);
    if (!run) break;
    for (int k = 0; k < chunk; ++k) {
      if (m == KMethod::PCG) pcg_iter(s, S.G, S.d_sys, S.d_bmap, S.nblocks);
      else bicg_iter(s, S.G, S.d_sys, S.d_bmap, S.nblocks);
    }
    chunk = std::min(chunk * 2, cap);
  }
  ksys_zero(s, S.d_sys, S.d_bmap, S.nblocks);
  for (const auto& k : hs) {
    const int c = status_to_code(k.status);
    if (c != IPCS_OK) return c;
  }
  return IPCS_OK;
}

// ------------------------------------------------------------------ layout
void Run::layout(Carver& c) {
  const Mesh& m = *mesh;
  const int nsys = 2 * dim + 1;
  X = c.take<double>(nv * dim);
  c2d = c.take<int32_t>(nc * m.nloc2);
  x2 = c.take<double>(n2 * dim);
  bmask = c.take<uint8_t>(n2);
  bidx = c.take<int32_t>(std::max<int64_t>(nb, 1));
  rp22 = c.take<int32_t>(n2 + 1);
  col22 = c.take<int32_t>(m.p22.nnz());
  rp21 = c.take<int32_t>(n2 + 1);
  col21 = c.take<int32_t>(m.p21.nnz());
  rp11 = c.take<int32_t>(n1 + 1);
  col11 = c.take<int32_t>(m.p11.nnz());
  rp12 = c.take<int32_t>(n1 + 1);
  col12 = c.take<int32_t>(m.p12.nnz());
  inc2p = c.take<int32_t>(n2 + 1);
  inc2 = c.take<int32_t>((int64_t)m.inc2.code.size());
  inc1p = c.take<int32_t>(n1 + 1);
  inc1 = c.take<int32_t>((int64_t)m.inc1.code.size());
  s22 = c.take<uint8_t>((int64_t)m.s22.slot.size());
  s21 = c.take<uint8_t>((int64_t)m.s21.slot.size());
  s11 = c.take<uint8_t>((int64_t)m.s11.slot.size());
  s12 = c.take<uint8_t>((int64_t)m.s12.slot.size());
  lift_ptr = c.take<int32_t>(n2 + 1);
  lift_slot = c.take<int32_t>(std::max<int64_t>(nlift, 1));
  lift_col = c.take<int32_t>(std::max<int64_t>(nlift, 1));
  const int64_t nnz22 = m.p22.nnz(), nnz11 = m.p11.nnz(), nnz12 = m.p12.nnz(),
                nnz21 = m.p21.nnz();
  M = c.take<double>(nnz22);
  K = c.take<double>(nnz22);
  E = c.take<double>(nnz22);
  Ael = c.take<double>(nnz22);
  Mel = c.take<double>(nnz22);
  Kp = c.take<double>(nnz11);
  for (int k = 0; k < 3; ++k) {
    Dc[k] = k < dim ? c.take<double>(nnz12) : nullptr;
    Gc[k] = k < dim ? c.take<double>(nnz21) : nullptr;
  }
  liftA = c.take<double>(std::max<int64_t>(nlift, 1));
  liftM = c.take<double>(std::max<int64_t>(nlift, 1));
  dinvA = c.take<double>(n2);
  dinvM = c.take<double>(n2);
  dinvKp = c.take<double>(n1);
  w = c.take<double>(n1);
  U = c.take<double>(dim * n2);
  Unew = c.take<double>(dim * n2);
  Ustar = c.take<double>(dim * n2);
  bU = c.take<double>(dim * n2);
  F = c.take<double>(dim * n2);
  gfull = c.take<double>(dim * n2);
  P = c.take<double>(n1);
  dP = c.take<double>(n1);
  rP = c.take<double>(n1);
  kv2 = c.take<double>(9 * dim * n2);
  kv1 = c.take<double>(5 * n1);
  kst = c.take<KState>(nsys);
  kcnt = c.take<uint32_t>(nsys);
  ksys = c.take<KSys>(nsys);
  kpart = c.take<double>((int64_t)nsys * NBLK_MAX * KPART);
  const int nb2 = nblk_for(n2, G22), nb1 = nblk_for(n1, G11);
  bmap_mom = c.take<int2>((int64_t)dim * nb2);
  bmap_p = c.take<int2>(nb1);
  bmap_corr = c.take<int2>((int64_t)dim * nb2);
  spart = c.take<double>(8192 * KPART);
  scnt = c.take<uint32_t>(4);
  scal = c.take<double>(8);
  poll = c.take<KState>(nsys);
  gb = c.take<double>(std::max<int64_t>(nb, 1) * dim);
  const int nq = dim == 2 ? Rule<2>::NQ : Rule<3>::NQ;
  fq = c.take<double>(prm.callbacks ? (int64_t)dim * nc * nq : 1);
}

Run::~Run() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (pinned) (void)hipHostFree(pinned);
}

template <class T>
static void up(hipStream_t s, T* dst, const std::vector<T>& src) {
  if (!src.empty())
    HIP_OK(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
}

void Run::upload_mesh() {
  const Mesh& m = *mesh;
  up(stream, X, m.X);
  up(stream, c2d, m.c2d);
  up(stream, x2, m.x2);
  up(stream, bmask, m.bmask);
  up(stream, bidx, m.bidx);
  up(stream, rp22, m.p22.rowptr);
  up(stream, col22, m.p22.col);
  up(stream, rp21, m.p21.rowptr);
  up(stream, col21, m.p21.col);
  up(stream, rp11, m.p11.rowptr);
  up(stream, col11, m.p11.col);
  up(stream, rp12, m.p12.rowptr);
  up(stream, col12, m.p12.col);
  up(stream, inc2p, m.inc2.ptr);
  up(stream, inc2, m.inc2.code);
  up(stream, inc1p, m.inc1.ptr);
  up(stream, inc1, m.inc1.code);
  up(stream, s22, m.s22.slot);
  up(stream, s21, m.s21.slot);
  up(stream, s11, m.s11.slot);
  up(stream, s12, m.s12.slot);
  up(stream, lift_ptr, m.lift_ptr);
  up(stream, lift_slot, m.lift_slot);
  up(stream, lift_col, m.lift_col);
}

void Run::assemble_constant() {
  const Mesh& m = *mesh;
  RowAsm a22{(int32_t)n2, rp22, inc2p, inc2, s22, m.s22.stride, c2d, m.nloc2, X, {M, K, nullptr}};
  asm_mass_stiff(dim, stream, a22, cfg_mk.bs, cfg_mk.lds);
  RowAsm a21{(int32_t)n2, rp21, inc2p, inc2, s21, m.s21.stride, c2d, m.nloc2, X,
             {Gc[0], Gc[1], Gc[2]}};
  asm_grad(dim, stream, a21, cfg_g.bs, cfg_g.lds);
  RowAsm a12{(int32_t)n1, rp12, inc1p, inc1, s12, m.s12.stride, c2d, m.nloc2, X,
             {Dc[0], Dc[1], Dc[2]}};
  asm_div(dim, stream, a12, cfg_d.bs, cfg_d.lds);
  RowAsm a11{(int32_t)n1, rp11, inc1p, inc1, s11, m.s11.stride, c2d, m.nloc2, X,
             {Kp, nullptr, nullptr}};
  asm_kp(dim, stream, a11, cfg_kp.bs, cfg_kp.lds);
  asm_lumped_p1(dim, stream, a11, w);
  inv_diagonal(stream, n1, rp11, col11, Kp, dinvKp);
  form_eliminated(stream, n2, rp22, col22, bmask, M, nullptr, 1.0, 0.0, Mel, dinvM);
  lift_values(stream, nlift, lift_slot, M, nullptr, 1.0, 0.0, liftM);
}

void Run::reform_A() {
  form_eliminated(stream, n2, rp22, col22, bmask, M, K, 1.0 / prm.dt, prm.nu, Ael, dinvA);
  lift_values(stream, nlift, lift_slot, M, K, 1.0 / prm.dt, prm.nu, liftA);
  bi.nu = prm.nu;
  A_dirty = false;
}

static KState fresh_state(double tol, int maxit) {
  KState k;
  std::memset(&k, 0, sizeof(k));
  k.tol2 = tol * tol;
  k.maxit = maxit;
  k.status = KS_DONE;
  return k;
}

void Run::setup_solvers() {
  const int nsys = 2 * dim + 1;
  const int nb2 = nblk_for(n2, G22), nb1 = nblk_for(n1, G11);
  std::vector<KSys> hs(nsys);
  std::vector<KState> st(nsys);
  for (int s = 0; s < nsys; ++s) {
    KSys& k = hs[s];
    std::memset(&k, 0, sizeof(k));
    k.st = kst + s;
    k.part = kpart + (size_t)s * NBLK_MAX * KPART;
    k.cnt = kcnt + s;
    const bool vel = s != dim;
    const int c = s < dim ? s : s - dim - 1;
    if (vel) {
      double* base = kv2 + (size_t)c * 9 * n2;
      k.rowptr = rp22;
      k.col = col22;
      k.n = (int32_t)n2;
      k.nblk = nb2;
      k.r = base;
      k.z = base + n2;
      k.p[0] = base + 2 * n2;
      k.p[1] = base + 3 * n2;
      k.q = base + 4 * n2;
      k.s = base + 5 * n2;
      k.t = base + 6 * n2;
      k.phat = base + 7 * n2;
      k.shat = base + 8 * n2;
      k.b = bU + (size_t)c * n2;
      if (s < dim) {   // momentum
        k.val = Ael;
        k.dinv = dinvA;
        k.x = Ustar + (size_t)c * n2;
        st[s] = fresh_state(prm.tol_mom, prm.maxit);
      } else {         // correction
        k.val = Mel;
        k.dinv = dinvM;
        k.x = Unew + (size_t)c * n2;
        st[s] = fresh_state(prm.tol_corr, prm.maxit);
      }
    } else {           // pressure Poisson
      k.rowptr = rp11;
      k.col = col11;
      k.val = Kp;
      k.dinv = dinvKp;
      k.n = (int32_t)n1;
      k.nblk = nb1;
      k.r = kv1;
      k.z = kv1 + n1;
      k.p[0] = kv1 + 2 * n1;
      k.p[1] = kv1 + 3 * n1;
      k.q = kv1 + 4 * n1;
      k.b = rP;
      k.x = dP;
      st[s] = fresh_state(prm.tol_p, prm.maxit);
    }
  }
  HIP_OK(hipMemcpyAsync(ksys, hs.data(), sizeof(KSys) * nsys, hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(kst, st.data(), sizeof(KState) * nsys, hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemsetAsync(kcnt, 0, sizeof(uint32_t) * nsys, stream));
  auto mk = [&](SolveSet& S, int first, int count, int G, int nblk, int2* dmap) {
    S.nsys = count;
    S.G = G;
    S.h_sys.assign(hs.begin() + first, hs.begin() + first + count);
    std::vector<int> nb(count, nblk);
    build_bmap(nb, S.h_bmap);
    S.nblocks = (int)S.h_bmap.size();
    S.d_sys = ksys + first;
    S.d_bmap = dmap;
    S.d_poll = poll + first;
    HIP_OK(hipMemcpyAsync(dmap, S.h_bmap.data(), sizeof(int2) * S.h_bmap.size(),
                          hipMemcpyHostToDevice, stream));
  };
  mk(set_mom, 0, dim, G22, nb2, bmap_mom);
  mk(set_p, dim, 1, G11, nb1, bmap_p);
  mk(set_corr, dim + 1, dim, G22, nb2, bmap_corr);
}

void Run::create(std::shared_ptr<const Mesh> m, const ipcs_params& p, void* ws, int64_t bytes,
                 hipStream_t s) {
  mesh = std::move(m);
  prm = p;
  stream = s;
  const Mesh& mm = *mesh;
  dim = mm.dim;
  n1 = mm.n1;
  n2 = mm.n2;
  nc = mm.nc;
  nv = mm.nv;
  nb = (int64_t)mm.bidx.size();
  nlift = (int64_t)mm.lift_slot.size();
  G22 = lanes_for(double(mm.p22.nnz()) / n2);
  G11 = lanes_for(double(mm.p11.nnz()) / n1);
  G12 = lanes_for(double(mm.p12.nnz()) / n1);
  cfg_mk = asm_cfg(mm.p22, 2);
  cfg_e = asm_cfg(mm.p22, 1);
  cfg_g = asm_cfg(mm.p21, dim);
  cfg_d = asm_cfg(mm.p12, dim);
  cfg_kp = asm_cfg(mm.p11, 1);
  Carver meas;
  layout(meas);
  if (!ws || bytes < meas.off)
    fail(IPCS_E_NOMEM, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Carver c;
  c.base = static_cast<char*>(ws);
  layout(c);
  ws_bytes = bytes;
  HIP_OK(hipHostMalloc((void**)&pinned, sizeof(KState) * (2 * dim + 1), hipHostMallocDefault));
  for (auto& e : ev) HIP_OK(hipEventCreate(&e));
  upload_mesh();
  const size_t vbytes = sizeof(double) * dim * n2;
  for (double* v : {U, Unew, Ustar, bU, F, gfull}) HIP_OK(hipMemsetAsync(v, 0, vbytes, stream));
  for (double* v : {P, dP, rP}) HIP_OK(hipMemsetAsync(v, 0, sizeof(double) * n1, stream));
  HIP_OK(hipMemsetAsync(scnt, 0, sizeof(uint32_t) * 4, stream));
  HIP_OK(hipMemsetAsync(scal, 0, sizeof(double) * 8, stream));
  assemble_constant();
  reform_A();
  setup_solvers();
  t = prm.t0;
  if (!prm.callbacks) {
    // keep host memory small when no callbacks are used
  } else {
    const int nq = dim == 2 ? Rule<2>::NQ : Rule<3>::NQ;
    h_xq.resize((size_t)nc * nq * dim);
    for (int64_t cc = 0; cc < nc; ++cc)
      for (int q = 0; q < nq; ++q)
        for (int r = 0; r < dim; ++r) {
          double x = 0.0;
          for (int k = 0; k <= dim; ++k) {
            const double l = dim == 2 ? Rule<2>::lam(q, k) : Rule<3>::lam(q, k);
            x += l * mm.X[(size_t)mm.c2d[cc * mm.nloc2 + k] * dim + r];
          }
          h_xq[((size_t)cc * nq + q) * dim + r] = x;
        }
  }
  h_xb.resize((size_t)nb * dim);
  for (int64_t k = 0; k < nb; ++k)
    for (int r = 0; r < dim; ++r) h_xb[k * dim + r] = mm.x2[(size_t)mm.bidx[k] * dim + r];
  HIP_OK(hipStreamSynchronize(stream));
}

void Run::normalize_pressure(double* Pdev) {
  weighted_mean(stream, n1, w, Pdev, spart, scnt, scal + 2);
  sub_scalar(stream, n1, scal + 2, Pdev);
}

void Run::set_builtin(int kind, const double* p, int np) {
  const bool ok2 = kind == IPCS_SOL_TAYLOR_GREEN_2D || kind == IPCS_SOL_JOHN_2D ||
                   kind == IPCS_SOL_POLY_STEADY_2D;
  const bool ok3 = kind == IPCS_SOL_BELTRAMI_3D || kind == IPCS_SOL_POLY_STEADY_3D;
  if (!((dim == 2 && ok2) || (dim == 3 && ok3)))
    fail(IPCS_E_INVALID, "built-in solution kind does not match the mesh dimension");
  Builtin b{};
  b.kind = kind;
  b.nu = prm.nu;
  if (kind == IPCS_SOL_TAYLOR_GREEN_2D) b.prm[0] = M_PI;
  if (kind == IPCS_SOL_BELTRAMI_3D) {
    b.prm[0] = M_PI / 4;
    b.prm[1] = M_PI / 2;
  }
  for (int i = 0; i < std::min(np, 4); ++i) b.prm[i] = p[i];
  bi = b;
  f_cb = g_cb = nullptr;
  eval_velocity(stream, dim, bi, x2, n2, t, U, n2);
  eval_pressure(stream, dim, bi, X, nv, t, P);
  normalize_pressure(P);
  phase_next = IPCS_PHASE_ASM;
  HIP_OK(hipStreamSynchronize(stream));
}

void Run::set_state(const double* u, const double* p, double tt) {
  HIP_OK(hipMemcpyAsync(U, u, sizeof(double) * dim * n2, hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(P, p, sizeof(double) * n1, hipMemcpyHostToDevice, stream));
  HIP_OK(hipStreamSynchronize(stream));
  t = tt;
  phase_next = IPCS_PHASE_ASM;
}

void fill_stats_solve(const std::vector<KState>& hs, int which, ipcs_step_stats* st) {
  if (!st) return;
  for (size_t c = 0; c < hs.size(); ++c) {
    const double res = hs[c].bb > 0 ? std::sqrt(hs[c].rr / hs[c].bb) : 0.0;
    if (which == 1) {
      st->it_mom[c] = hs[c].it;
      st->res_mom[c] = res;
    } else if (which == 2) {
      st->it_p = hs[c].it;
      st->res_p = res;
    } else {
      st->it_corr[c] = hs[c].it;
      st->res_corr[c] = res;
    }
  }
}

int Run::phase(int which, ipcs_step_stats* st) {
  if (which != phase_next)
    fail(IPCS_E_STATE, "IPCS phases must run in order; expected phase " +
                           std::to_string(phase_next) + ", got " + std::to_string(which));
  std::vector<KState> hs;
  int rc = IPCS_OK;
  switch (which) {
    case IPCS_PHASE_ASM: {
      if (A_dirty) reform_A();
      t1 = t + prm.dt;
      HIP_OK(hipEventRecord(ev[0], stream));
      if (g_cb) {
        std::vector<double> vals((size_t)nb * dim);
        g_cb(g_ctx, dim, nb, h_xb.data(), t1, vals.data());
        HIP_OK(hipMemcpyAsync(gb, vals.data(), sizeof(double) * vals.size(),
                              hipMemcpyHostToDevice, stream));
        dirichlet_scatter(stream, dim, gb, bidx, nb, gfull, n2);
        HIP_OK(hipStreamSynchronize(stream));
      } else if (bi.kind) {
        dirichlet_builtin(stream, dim, bi, x2, bidx, nb, t1, gfull, n2);
      }
      const Mesh& m = *mesh;
      RowAsm a22{(int32_t)n2, rp22, inc2p, inc2, s22, m.s22.stride, c2d, m.nloc2, X,
                 {E, nullptr, nullptr}};
      has_F = false;
      if (f_cb) {
        const int nq = dim == 2 ? Rule<2>::NQ : Rule<3>::NQ;
        std::vector<double> vals((size_t)nc * nq * dim), tr(vals.size());
        f_cb(f_ctx, dim, nc * nq, h_xq.data(), t1, vals.data());
        for (int64_t i = 0; i < nc * nq; ++i)
          for (int c = 0; c < dim; ++c) tr[(size_t)c * nc * nq + i] = vals[i * dim + c];
        HIP_OK(hipMemcpyAsync(fq, tr.data(), sizeof(double) * tr.size(), hipMemcpyHostToDevice,
                              stream));
        asm_forcing(dim, stream, a22, bi, fq, nc, t1, F, n2);
        HIP_OK(hipStreamSynchronize(stream));
        has_F = true;
      } else if (builtin_has_force(bi.kind)) {
        asm_forcing(dim, stream, a22, bi, nullptr, nc, t1, F, n2);
        has_F = true;
      }
      asm_conv_explicit(dim, stream, a22, cfg_e.bs, cfg_e.lds, U, n2, 1.0 / prm.dt);
      rhs_momentum(stream, dim, G22, n2, rp22, col22, E, U, rp21, col21, Gc, P,
                   has_F ? F : nullptr, lift_ptr, lift_col, liftA, bmask, gfull, bU);
      copy_with_bc(stream, dim, U, bmask, gfull, Ustar, n2);
      HIP_OK(hipEventRecord(ev[1], stream));
      phase_next = IPCS_PHASE_MOMENTUM;
      return IPCS_OK;
    }
    case IPCS_PHASE_MOMENTUM: {
      rc = krylov_solve(stream, set_mom, KMethod::BICG, prm.check_every, hs, pinned);
      fill_stats_solve(hs, 1, st);
      HIP_OK(hipEventRecord(ev[2], stream));
      if (rc != IPCS_OK) {
        if (st) st->failed_solve = 1;
        phase_next = IPCS_PHASE_ASM;
        return rc;
      }
      phase_next = IPCS_PHASE_PRESSURE;
      return IPCS_OK;
    }
    case IPCS_PHASE_PRESSURE: {
      rhs_pressure(stream, dim, G12, n1, rp12, col12, Dc, Ustar, n2, -prm.rho / prm.dt, rP, spart,
                   scnt, scal + 0);
      sub_scalar(stream, n1, scal + 0, rP);
      HIP_OK(hipMemsetAsync(dP, 0, sizeof(double) * n1, stream));
      rc = krylov_solve(stream, set_p, KMethod::PCG, prm.check_every, hs, pinned);
      fill_stats_solve(hs, 2, st);
      if (rc != IPCS_OK) {
        if (st) st->failed_solve = 2;
        phase_next = IPCS_PHASE_ASM;
        return rc;
      }
      weighted_mean(stream, n1, w, dP, spart, scnt, scal + 1);
      sub_scalar(stream, n1, scal + 1, dP);
      HIP_OK(hipEventRecord(ev[3], stream));
      phase_next = IPCS_PHASE_CORRECTION;
      return IPCS_OK;
    }
    case IPCS_PHASE_CORRECTION: {
      rhs_correction(stream, dim, G22, n2, rp22, col22, M, Ustar, rp21, col21, Gc, dP,
                     prm.dt / prm.rho, lift_ptr, lift_col, liftM, bmask, gfull, bU);
      HIP_OK(hipMemcpyAsync(Unew, Ustar, sizeof(double) * dim * n2, hipMemcpyDeviceToDevice,
                            stream));
      rc = krylov_solve(stream, set_corr, KMethod::PCG, prm.check_every, hs, pinned);
      fill_stats_solve(hs, 3, st);
      phase_next = IPCS_PHASE_ASM;
      if (rc != IPCS_OK) {
        if (st) st->failed_solve = 3;
        return rc;
      }
      axpy_inplace(stream, n1, 1.0, dP, P);
      HIP_OK(hipMemcpyAsync(U, Unew, sizeof(double) * dim * n2, hipMemcpyDeviceToDevice, stream));
      HIP_OK(hipEventRecord(ev[4], stream));
      HIP_OK(hipEventSynchronize(ev[4]));
      t = t1;
      if (st) {
        st->t = t;
        HIP_OK(hipEventElapsedTime(&st->ms_asm, ev[0], ev[1]));
        HIP_OK(hipEventElapsedTime(&st->ms_mom, ev[1], ev[2]));
        HIP_OK(hipEventElapsedTime(&st->ms_p, ev[2], ev[3]));
        HIP_OK(hipEventElapsedTime(&st->ms_corr, ev[3], ev[4]));
      }
      return IPCS_OK;
    }
  }
  fail(IPCS_E_INVALID, "unknown phase " + std::to_string(which));
}

int Run::step(ipcs_step_stats* st) {
  if (phase_next != IPCS_PHASE_ASM) fail(IPCS_E_STATE, "a step is in progress (phase API)");
  if (st) std::memset(st, 0, sizeof(*st));
  for (int ph = IPCS_PHASE_ASM; ph <= IPCS_PHASE_CORRECTION; ++ph) {
    const int rc = phase(ph, st);
    if (rc != IPCS_OK) {
      if (st) {
        st->status = rc;
        st->t = t;
      }
      return rc;
    }
  }
  return IPCS_OK;
}

}  // namespace ipcs
