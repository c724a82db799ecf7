// Steady Navier-Stokes by Newton's method: monolithic patterns, workspace,
// the Newton loop and its flexible GMRES (host side; kernels in
// kernels_asm.hip, kernels_steady.hip and the Krylov kernels of the velocity
// block).
#include "steady.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "builtin.hpp"
#include "common.hpp"

namespace ipcs {

void build_sell(const Pattern& P, Sell& S);   // mesh.cpp

MonoPattern build_mono(const Mesh& m, bool velocity_only) {
  const int d = m.dim;
  const int64_t n2 = m.n2, n1 = m.n1;
  const int64_t nrows = d * n2 + (velocity_only ? 0 : n1);
  Pattern P;
  P.nrows = P.ncols = nrows;
  P.rowptr.assign(nrows + 1, 0);
  // row lengths
  for (int c = 0; c < d; ++c)
    for (int64_t i = 0; i < n2; ++i) {
      int len = d * (m.p22.rowptr[i + 1] - m.p22.rowptr[i]);
      if (!velocity_only) len += m.p21.rowptr[i + 1] - m.p21.rowptr[i];
      P.rowptr[c * n2 + i + 1] = len;
    }
  if (!velocity_only)
    for (int64_t k = 0; k < n1; ++k)
      P.rowptr[d * n2 + k + 1] = d * (m.p12.rowptr[k + 1] - m.p12.rowptr[k]);
  for (int64_t r = 0; r < nrows; ++r) P.rowptr[r + 1] += P.rowptr[r];
  P.col.resize(P.rowptr[nrows]);
  std::vector<int32_t> src(P.col.size());
  std::vector<uint8_t> code(P.col.size());
  auto kode = [](int kind, int c, int e) { return (uint8_t)(kind | (c << 3) | (e << 5)); };
  for (int c = 0; c < d; ++c)
    for (int64_t i = 0; i < n2; ++i) {
      int64_t q = P.rowptr[c * n2 + i];
      for (int e = 0; e < d; ++e)
        for (int k = 0; k < m.p22.rowptr[i + 1] - m.p22.rowptr[i]; ++k, ++q) {
          P.col[q] = (int32_t)(e * n2 + m.p22.col[m.p22.rowptr[i] + k]);
          src[q] = (int32_t)m.e22.index(i, k);
          code[q] = kode(c == e ? MONO_UU_DIAG : MONO_UU_OFF, c, e);
        }
      if (!velocity_only)
        for (int k = 0; k < m.p21.rowptr[i + 1] - m.p21.rowptr[i]; ++k, ++q) {
          P.col[q] = (int32_t)(d * n2 + m.p21.col[m.p21.rowptr[i] + k]);
          src[q] = (int32_t)m.e21.index(i, k);
          code[q] = kode(MONO_G, c, 0);
        }
    }
  if (!velocity_only)
    for (int64_t kr = 0; kr < n1; ++kr) {
      int64_t q = P.rowptr[d * n2 + kr];
      for (int e = 0; e < d; ++e)
        for (int k = 0; k < m.p12.rowptr[kr + 1] - m.p12.rowptr[kr]; ++k, ++q) {
          P.col[q] = (int32_t)(e * n2 + m.p12.col[m.p12.rowptr[kr] + k]);
          src[q] = (int32_t)m.e12.index(kr, k);
          code[q] = kode(MONO_D, 0, e);
        }
    }
  MonoPattern out;
  build_sell(P, out.sell);
  const Sell& S = out.sell;
  out.src.assign(S.nent, 0);
  out.code.assign(S.nent, (uint8_t)MONO_PAD);
  for (int64_t r = 0; r < nrows; ++r)
    for (int k = 0; k < P.rowptr[r + 1] - P.rowptr[r]; ++k) {
      const int64_t e = S.index(r, k);
      out.src[e] = src[P.rowptr[r] + k];
      out.code[e] = code[P.rowptr[r] + k];
    }
  return out;
}

namespace {

ipcs_params run_params(const ipcs_steady_params& p) {
  ipcs_params r;
  ipcs_params_default(&r);
  r.nu = p.nu;
  r.dt = 1.0;                 // the run's time-dependent matrices are not used
  r.precision = IPCS_FP64;
  r.poisson_part_rows = -1;   // no Poisson partition (no IPCS step is taken)
  return r;
}

template <class T>
void up(hipStream_t s, T* dst, const std::vector<T>& src) {
  if (!src.empty())
    HIP_OK(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
}

}  // namespace

Steady::~Steady() {
  pinned_give(pinned);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
}

void Steady::layout(Carver& c) {
  const int m = sp.restart;
  const Sell &J = mj.sell, &A = ma.sell;
  j_sp = c.take<int32_t>(J.nslices + 1);
  j_col = c.take<int32_t>(J.nent);
  j_src = c.take<int32_t>(J.nent);
  j_code = c.take<uint8_t>(J.nent);
  a_sp = c.take<int32_t>(A.nslices + 1);
  a_col = c.take<int32_t>(A.nent);
  a_src = c.take<int32_t>(A.nent);
  a_code = c.take<uint8_t>(A.nent);
  Jv = c.take<double>(J.nent);
  Pv = c.take<double>(J.nent);
  Av = c.take<double>(A.nent);
  dinvA = c.take<double>(nu_rows);
  const int64_t ne22 = run.ne22;
  Cv = c.take<double>(ne22);
  Nv = c.take<double>((int64_t)dim * dim * ne22);
  x = c.take<double>(n);
  bvec = c.take<double>(n);
  R = c.take<double>(n);
  dx = c.take<double>(n);
  tmp = c.take<double>(n);
  V = c.take<double>((int64_t)(m + 1) * n);
  Z = c.take<double>((int64_t)m * n);
  h = c.take<double>(2 * (m + 2));
  part = c.take<double>((int64_t)(m + 2) * mdot_blocks(n));
  scal = c.take<double>(16);
  kva = c.take<double>(8 * nu_rows);
  ib = c.take<double>(nu_rows);
  ix = c.take<double>(nu_rows);
  kst = c.take<KState>(1);
  kgroup = c.take<KGroup>(1);
  const int nbm = nblk_m_for(nu_rows, 1), nbv = nblk_v_for(nu_rows, 1);
  pm = c.take<double>((int64_t)nbm * GMAX * KP);
  pv0 = c.take<double>((int64_t)nbv * GMAX * KP);
  pv1 = c.take<double>((int64_t)nbv * GMAX * KP);
  pfold = c.take<double>(GMAX * KP);
  bm = c.take<int2>(nbm);
  bv = c.take<int2>(nbv);
  poll = c.take<KState>(GMAX);
}

int64_t Steady::measure(std::shared_ptr<const Mesh> msh, const ipcs_steady_params& p) {
  if (msh->pair != IPCS_PAIR_P2P1) fail(IPCS_E_INVALID, "the steady solver uses the P2-P1 pair");
  if (!(p.nu > 0.0) || !(p.tol > 0.0) || p.maxit < 1 || p.restart < 2 || p.restart > 512 ||
      !(p.lin_tol > 0.0) || p.lin_maxit < 1 || p.inner_maxit < 1 || !(p.inner_tol > 0.0))
    fail(IPCS_E_INVALID, "invalid steady solver parameters");
  sp = p;
  dim = msh->dim;
  n2 = msh->n2;
  n1 = msh->n1;
  nu_rows = dim * n2;
  n = nu_rows + n1;
  mj = build_mono(*msh, false);
  ma = build_mono(*msh, true);
  // the run's own workspace first, then the steady solver's
  Run probe;
  probe.mesh = msh;
  probe.prm = run_params(p);
  probe.set_precision();
  probe.sizes_from_mesh();
  Carver cm;
  probe.layout(cm);
  ws_run = (cm.off + 255) / 256 * 256;
  run.ne22 = msh->e22.nent;
  Carver meas;
  layout(meas);
  return ws_run + meas.off;
}

void Steady::create(std::shared_ptr<const Mesh> msh, const ipcs_steady_params& p, void* ws,
                    int64_t bytes, hipStream_t s) {
  const int64_t need = measure(msh, p);
  if (!ws || bytes < need)
    fail(IPCS_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  const ipcs_params rp = run_params(p);
  run.create(msh, rp, ws, ws_run, s);
  Carver c;
  c.base = static_cast<char*>(ws) + ws_run;
  layout(c);
  hipStream_t st = run.stream;
  up(st, j_sp, mj.sell.sptr);
  up(st, j_col, mj.sell.col);
  up(st, j_src, mj.src);
  up(st, j_code, mj.code);
  up(st, a_sp, ma.sell.sptr);
  up(st, a_col, ma.sell.col);
  up(st, a_src, ma.src);
  up(st, a_code, ma.code);
  fill(st, n, 0.0, x);
  fill(st, n, 0.0, bvec);
  // inner Jacobi-BiCGStab on the velocity block
  KGroup g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.n = (int32_t)nu_rows;
  g.sptr = a_sp;
  g.col = a_col;
  g.val = Av;
  g.dinv = dinvA;
  g.nblk_m = nblk_m_for(nu_rows, 1);
  g.nblk_v = nblk_v_for(nu_rows, 1);
  g.maxit = sp.inner_maxit;
  g.part_m = pm;
  g.part_v[0] = pv0;
  g.part_v[1] = pv1;
  g.fold = pfold;
  KVecs& Vv = g.v[0];
  Vv.b = ib;
  Vv.x = ix;
  double* vk[8];
  for (int k = 0; k < 8; ++k) vk[k] = kva + (size_t)k * nu_rows;
  Vv.r = vk[0];
  Vv.u = vk[1];
  Vv.p = vk[2];
  Vv.s = vk[3];
  Vv.w = vk[4];
  Vv.t = vk[5];
  Vv.phat = vk[6];
  Vv.shat = vk[7];
  Vv.st = kst;
  KState k0;
  std::memset(&k0, 0, sizeof(k0));
  k0.tol2 = sp.inner_tol * sp.inner_tol;
  k0.status = KS_DONE;
  HIP_OK(hipMemcpyAsync(kgroup, &g, sizeof(g), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(kst, &k0, sizeof(k0), hipMemcpyHostToDevice, st));
  std::vector<int2> mm, mv;
  build_bmap({g.nblk_m}, mm);
  build_bmap({g.nblk_v}, mv);
  xcd_chunks(mm, 8);
  up(st, bm, mm);
  up(st, bv, mv);
  setA.h_groups = {g};
  setA.L = KLaunch{kgroup, 1, 1, kept_m_for(nu_rows, 1), 0, bm, (int)mm.size(), bv,
                   (int)mv.size(), fold_for(nu_rows, 1)};
  setA.d_poll = poll;
  pinned = pinned_take();
  for (auto& e : ev) HIP_OK(hipEventCreate(&e));
  // the host copies above are stack or member vectors: finish the transfers
  HIP_OK(hipStreamSynchronize(st));
}

void Steady::set_builtin(int kind, const double* prm, int nprm) {
  const bool ok2 = kind == IPCS_SOL_POLY_STEADY_2D || kind == IPCS_SOL_STEADY_PAPER_2D;
  const bool ok3 = kind == IPCS_SOL_POLY_STEADY_3D;
  if (!((dim == 2 && ok2) || (dim == 3 && ok3)))
    fail(IPCS_E_INVALID, "built-in steady solution kind does not match the mesh dimension");
  Builtin b{};
  b.kind = kind;
  b.nu = sp.nu;
  for (int i = 0; i < std::min(nprm, 4); ++i) b.prm[i] = prm[i];
  run.bi = b;
  hipStream_t s = run.stream;
  const Mesh& m = *run.mesh;
  dirichlet_builtin(s, dim, b, run.x2, run.bidx, run.nb, 0.0, run.gfull, n2);
  RowAsm a22{(int32_t)n2, run.sp22, run.inc2p, run.inc2, run.s22, m.s22.stride, run.c2d,
             m.nloc2, run.X, {nullptr, nullptr, nullptr}, m.pair, run.c2v, m.nloc1};
  if (builtin_has_force(kind)) asm_forcing(dim, s, a22, b, nullptr, run.nc, 0.0, run.F, n2);
  else fill(s, nu_rows, 0.0, run.F);
  // right-hand side: F on velocity rows off the boundary, 0 elsewhere
  fill(s, n, 0.0, tmp);
  copy_with_bc(s, dim, run.F, run.bmask, tmp, bvec, n2);
  // start: the Dirichlet data on the boundary, zero elsewhere; P = 0
  copy_with_bc(s, dim, tmp, run.bmask, run.gfull, x, n2);
  HIP_OK(hipStreamSynchronize(s));
  history.clear();
}

void Steady::set_state(const double* u, const double* p) {
  hipStream_t s = run.stream;
  HIP_OK(hipMemcpyAsync(x, u, sizeof(double) * nu_rows, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(x + nu_rows, p, sizeof(double) * n1, hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  history.clear();
}

void Steady::to_run() {
  copy_vec(run.stream, nu_rows, x, run.U);
  copy_vec(run.stream, n1, x + nu_rows, run.P);
  HIP_OK(hipStreamSynchronize(run.stream));
}

namespace {

// host copy of n doubles from the device (synchronizes the stream)
void fetch(hipStream_t s, const double* src, double* dst, int n) {
  HIP_OK(hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
}

}  // namespace

double Steady::newton_step(ipcs_steady_stats* st) {
  hipStream_t s = run.stream;
  const Mesh& m = *run.mesh;
  const int64_t ne22 = run.ne22;
  HIP_OK(hipEventRecord(ev[0], s));
  // blocks of the Newton matrix at the current iterate
  RowAsm a22{(int32_t)n2, run.sp22, run.inc2p, run.inc2, run.s22, m.s22.stride, run.c2d,
             m.nloc2, run.X, {Cv, nullptr, nullptr}, m.pair, run.c2v, m.nloc1};
  asm_conv(dim, false, s, a22, run.cfg_e.bs, run.cfg_e.lds, x, n2, 0.0, 1.0);   // C(U)
  for (int c = 0; c < dim; ++c)
    for (int e = 0; e < dim; ++e) {
      RowAsm an = a22;
      an.out[0] = Nv + (size_t)(c * dim + e) * ne22;
      asm_newton(dim, s, an, run.cfg_e.bs, run.cfg_e.lds, x, n2, c, e);
    }
  MonoCompose mc{};
  mc.nrows = n;
  mc.n2 = n2;
  mc.dim = dim;
  mc.sptr = j_sp;
  mc.col = j_col;
  mc.src = j_src;
  mc.code = j_code;
  mc.bmask = run.bmask;
  mc.nu = sp.nu;
  mc.K = static_cast<const double*>(run.K);
  mc.C = Cv;
  for (int k = 0; k < dim * dim; ++k) mc.N[k] = Nv + (size_t)k * ne22;
  for (int c = 0; c < dim; ++c) {
    mc.Gc[c] = static_cast<const double*>(run.Gc[c]);
    mc.Dc[c] = static_cast<const double*>(run.Dc[c]);
  }
  mc.J = Jv;
  mc.Pic = Pv;
  mono_compose(s, mc);
  MonoCompose ma_ = mc;
  ma_.nrows = nu_rows;
  ma_.sptr = a_sp;
  ma_.col = a_col;
  ma_.src = a_src;
  ma_.code = a_code;
  ma_.J = Av;
  ma_.Pic = nullptr;
  mono_compose(s, ma_);
  sell_inv_diag(s, nu_rows, a_sp, a_col, Av, dinvA);
  // residual R = b - Pic x, pressure rows projected to zero sum
  sell_axpby(s, n, j_sp, j_col, Pv, x, -1.0, 1.0, bvec, R);
  fill(s, n1, 1.0, tmp);
  mdot(s, n1, R + nu_rows, n1, tmp, 1, part, scal + 0, 0);
  sub_scaled(s, n1, scal + 0, 1.0 / (double)n1, R + nu_rows);
  mdot(s, n, R, n, R, 1, part, scal + 1, 0);
  double rr = 0.0;
  fetch(s, scal + 1, &rr, 1);
  const double beta0 = std::sqrt(rr);
  if (!std::isfinite(beta0)) fail(IPCS_E_NONFINITE, "non-finite Newton residual");
  if (st && st->newton_steps == 0) st->res0 = beta0;
  if (st) st->res = beta0;
  // FGMRES(m) for J dx = R, x0 = 0, right preconditioning by the block
  // upper-triangular [[A, G], [0, -S]]
  fill(s, n, 0.0, dx);
  const int M = sp.restart;
  const double* w1 = run.w;
  std::vector<double> H((size_t)(M + 1) * M), cs(M), sn(M), g(M + 1), hb(2 * (M + 1) + 1);
  double beta = beta0;
  int total = 0;
  KTimer none;
  std::vector<KState> hs;
  bool converged = beta0 == 0.0;
  while (!converged && total < sp.lin_maxit) {
    // v_0 = r / ||r||, r = R - J dx
    if (total == 0) {
      copy_vec(s, n, R, V);
    } else {
      sell_axpby(s, n, j_sp, j_col, Jv, dx, -1.0, 1.0, R, V);
      mdot(s, n, V, n, V, 1, part, scal + 1, 0);
      fetch(s, scal + 1, &rr, 1);
      beta = std::sqrt(rr);
      if (beta <= sp.lin_tol * beta0) {
        converged = true;
        break;
      }
    }
    mdot(s, n, V, n, V, 1, part, scal + 2, 0);
    scale_inv_norm(s, n, V, scal + 2, V);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (; k < M && total < sp.lin_maxit; ++k) {
      double* vk = V + (size_t)k * n;
      double* zk = Z + (size_t)k * n;
      double* w = V + (size_t)(k + 1) * n;
      // z_k: pressure part -nu v_p / (Mp 1), velocity part A^{-1} (v_u - G z_p)
      prec_pressure(s, n1, vk + nu_rows, w1, sp.nu, zk + nu_rows);
      fill(s, nu_rows, 0.0, tmp);
      copy_vec(s, n1, zk + nu_rows, tmp + nu_rows);
      sell_axpby(s, nu_rows, j_sp, j_col, Jv, tmp, -1.0, 1.0, vk, ib);
      fill(s, nu_rows, 0.0, ix);
      const int irc = krylov_solve(s, setA, KMethod::BICG, 64, hs, pinned, none);
      if (irc == IPCS_E_NONFINITE) fail(IPCS_E_NONFINITE, "non-finite inner solve");
      inner_it += hs[0].it;
      copy_vec(s, nu_rows, ix, zk);
      // w = J z_k, orthogonalized twice against v_0..v_k (classical Gram-Schmidt)
      sell_axpby(s, n, j_sp, j_col, Jv, zk, 1.0, 0.0, nullptr, w);
      mdot(s, n, V, n, w, k + 1, part, h, 0);
      maxpy(s, n, V, n, h, k + 1, -1.0, w);
      mdot(s, n, V, n, w, k + 1, part, h + (M + 1), 0);
      maxpy(s, n, V, n, h + (M + 1), k + 1, -1.0, w);
      mdot(s, n, w, n, w, 1, part, scal + 3, 0);
      scale_inv_norm(s, n, w, scal + 3, w);
      fetch(s, h, hb.data(), 2 * (M + 1));
      fetch(s, scal + 3, &rr, 1);
      ++total;
      for (int i = 0; i <= k; ++i) H[(size_t)i * M + k] = hb[i] + hb[M + 1 + i];
      H[(size_t)(k + 1) * M + k] = std::sqrt(rr);
      // Givens rotations
      for (int i = 0; i < k; ++i) {
        const double a = H[(size_t)i * M + k], b = H[(size_t)(i + 1) * M + k];
        H[(size_t)i * M + k] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * M + k] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[(size_t)k * M + k], b = H[(size_t)(k + 1) * M + k];
      const double rad = std::hypot(a, b);
      cs[k] = rad > 0.0 ? a / rad : 1.0;
      sn[k] = rad > 0.0 ? b / rad : 0.0;
      H[(size_t)k * M + k] = rad;
      H[(size_t)(k + 1) * M + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      if (!std::isfinite(g[k + 1])) fail(IPCS_E_NONFINITE, "non-finite GMRES residual");
      if (std::fabs(g[k + 1]) <= sp.lin_tol * beta0 || rr == 0.0) {
        ++k;
        break;
      }
    }
    // y = H^{-1} g, dx += Z y
    std::vector<double> y(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int j = i + 1; j < k; ++j) sacc -= H[(size_t)i * M + j] * y[j];
      y[i] = H[(size_t)i * M + i] != 0.0 ? sacc / H[(size_t)i * M + i] : 0.0;
    }
    HIP_OK(hipMemcpyAsync(h, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    maxpy(s, n, Z, n, h, k, 1.0, dx);
    HIP_OK(hipStreamSynchronize(s));   // y is a host vector about to go away
  }
  lin_it += total;
  // the true residual of the linear solve
  sell_axpby(s, n, j_sp, j_col, Jv, dx, -1.0, 1.0, R, tmp);
  mdot(s, n, tmp, n, tmp, 1, part, scal + 4, 0);
  fetch(s, scal + 4, &rr, 1);
  const double lin_res = beta0 > 0.0 ? std::sqrt(rr) / beta0 : 0.0;
  if (!(lin_res <= std::max(10.0 * sp.lin_tol, 1e-14)))
    fail(IPCS_E_NOT_CONVERGED, "Newton system not solved: relative residual " +
                                   std::to_string(lin_res));
  // x += dx, pressure shifted to zero integral mean
  axpy_inplace(s, n, 1.0, dx, x);
  sub_weighted_mean(s, n1, w1, x + nu_rows, part, scal + 5);
  mdot(s, n, dx, n, dx, 1, part, scal + 6, 0);
  mdot(s, n, x, n, x, 1, part, scal + 7, 0);
  double nn[2];
  fetch(s, scal + 6, nn, 2);
  HIP_OK(hipEventRecord(ev[1], s));
  HIP_OK(hipEventSynchronize(ev[1]));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
  const double rel = nn[1] > 0.0 ? std::sqrt(nn[0] / nn[1]) : 0.0;
  history.push_back(rel);
  if (st) {
    st->newton_steps += 1;
    st->lin_it += total;
    st->rel_change = rel;
    st->ms += ms;
  }
  return rel;
}

int Steady::solve(ipcs_steady_stats* st) {
  lin_it = inner_it = 0;
  for (int k = 0; k < sp.maxit; ++k) {
    const double rel = newton_step(st);
    if (st) st->inner_it = inner_it;
    if (rel <= sp.tol) {
      to_run();
      return IPCS_OK;
    }
  }
  to_run();
  return IPCS_E_NOT_CONVERGED;
}

}  // namespace ipcs
