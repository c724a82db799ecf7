// Jacobi-preconditioned CG with one kernel per iteration, for the pressure
// Poisson system (eq. (9), second line) on a row partition of its matrix.
//
// The iterates are those of the two-kernel Chronopoulos-Gear CG in
// kernels_krylov.hip (u = D^{-1} r, w = A u, s = A p):
//   [gamma = r.u, ||r||^2, delta = w.u] -> stop test;
//   beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old);
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = D^{-1} r;
//   w = A u; partials r.u, r.r, w.u
// but the vector update and the product w = A u share one launch. A block owns
// one part of the rows (a compact patch of DOFs, mesh.hpp PartSell): it updates
// its own rows, recomputes r and u on its halo rows (the columns its rows
// reference in other parts) from the previous launch's r, s, w, which no block
// of this launch writes (r, s, w are double-buffered by launch parity), keeps
// u for own and halo rows in LDS, and multiplies its rows by it with the
// part-local 16-bit column indices. The halo recomputation is bitwise the
// owner's computation (the same fused multiply-adds on the same inputs and
// scalars), so every block applies A to one and the same u. The only global
// synchronization is the kernel boundary, which also completes the
// reductions: as in kernels_krylov.hip, each block writes partial sums and
// every block of the next launch re-reduces all of them in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"
#include "launch.hpp"

namespace ipcs {

#define FGROUP_HEAD(BMAP)                \
  const int2 m_ = (BMAP)[blockIdx.x];    \
  const FGroup& g = groups[m_.x];        \
  const int lb = m_.y;                   \
  const int p0 = g.part_ptr[lb];         \
  const int own = g.part_ptr[lb + 1] - p0; \
  const int h0 = g.halo_ptr[lb];         \
  const int nh = g.halo_ptr[lb + 1] - h0;

// y[e] = sum_k A(l, k) loc[lcol(l, k)] for the part's local rows
// l = KBS e + tid (wavefront wv of the block takes local slices wv, wv + 4, ...).
// Entries are loaded eight at a time before the LDS gathers; the last chunk
// re-reads entry w-1 and discards it. Lanes past the part's rows give 0.
template <int EPT, class VT>
__device__ __forceinline__ void part_spmv(const FGroup& g, int lb, const double* loc,
                                          double (&y)[EPT]) {
  const VT* val = static_cast<const VT*>(g.val);
  const int s0 = g.slice_ptr[lb], s1 = g.slice_ptr[lb + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    y[e] = 0.0;
    const int sl = s0 + (KBS / 64) * e + wv;
    if (sl >= s1) continue;
    const int b0 = g.sptr[sl];
    const int w = (g.sptr[sl + 1] - b0) >> 6;
    const int base = b0 + lane;
    for (int k = 0; k < w; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
        c[q] = g.lcol[base + 64 * kk];
        a[q] = (double)val[base + 64 * kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) y[e] += k + q < w ? a[q] * loc[c[q]] : 0.0;
    }
  }
}

__device__ __forceinline__ bool fcg_active(const FGroup& g, int mode) {
  const int st = g.st->status;
  return mode == 0 || st == KS_PENDING || st == KS_RESTART;
}

// ------------------------------------------------------------------ start
// r = b - A x for the systems that start (mode 0: all; x and b are brought to
// part order here) or are confirmed (mode 1: PENDING or RESTART); p = s = 0.
// Partials r.r, b.b into part_s.
template <int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_fcg_resid(const FGroup* groups, const int2* bmap,
                                                   int mode, int par) {
  FGROUP_HEAD(bmap)
  extern __shared__ double loc[];
  __shared__ double sh[(KBS / 64) * 2];
  if (!fcg_active(g, mode)) return;   // uniform over the block
  for (int l = threadIdx.x; l < own; l += KBS)
    loc[l] = mode == 0 ? g.x[g.perm[p0 + l]] : g.xp[p0 + l];
  for (int q = threadIdx.x; q < nh; q += KBS) {
    const int c = g.halo[h0 + q];
    loc[own + q] = mode == 0 ? g.x[g.perm[c]] : g.xp[c];
  }
  __syncthreads();
  double y[EPT];
  part_spmv<EPT, VT>(g, lb, loc, y);
  double acc[2] = {};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    if (l >= own) continue;
    const int i = p0 + l;
    const double bi = mode == 0 ? g.b[g.perm[i]] : g.bp[i];
    if (mode == 0) {
      g.bp[i] = bi;
      g.xp[i] = loc[l];
    }
    const double r = bi - y[e];
    g.r[par][i] = r;
    g.p[i] = 0.0;
    g.s[par][i] = 0.0;
    acc[0] += r * r;
    acc[1] += bi * bi;
  }
  store_partials<1, 2>(acc, g.part_s, g.nparts, lb, sh);
}

// w = A u with u = D^{-1} r (own and halo rows from the start's r);
// partials gamma = r.u, r.r, delta = w.u for the first iteration.
template <int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_fcg_first(const FGroup* groups, const int2* bmap,
                                                   int mode, int par) {
  FGROUP_HEAD(bmap)
  extern __shared__ double loc[];
  __shared__ double sh[(KBS / 64) * 3];
  if (!fcg_active(g, mode)) return;
  const double* r = g.r[par];
  double ri[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    ri[e] = 0.0;
    if (l < own) {
      ri[e] = r[p0 + l];
      loc[l] = g.dinv[p0 + l] * ri[e];
    }
  }
  for (int q = threadIdx.x; q < nh; q += KBS) {
    const int c = g.halo[h0 + q];
    loc[own + q] = g.dinv[c] * r[c];
  }
  __syncthreads();
  double y[EPT];
  part_spmv<EPT, VT>(g, lb, loc, y);
  double acc[3] = {};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    if (l >= own) continue;
    const double u = loc[l];
    g.w[par][p0 + l] = y[e];
    acc[0] += ri[e] * u;
    acc[1] += ri[e] * ri[e];
    acc[2] += y[e] * u;
  }
  store_partials<1, 3>(acc, g.part[par], g.nparts, lb, sh);
}

// One block per group: status of the systems that were started or confirmed,
// and the scalars of a first iteration of launch parity par (beta = 0).
__global__ void __launch_bounds__(KBS) k_fcg_decide(const FGroup* groups, int mode, int par,
                                                    int launched) {
  const FGroup& g = groups[blockIdx.x];
  __shared__ double sh[(KBS / 64) * 2];
  if (!fcg_active(g, mode)) return;
  double tot[2];
  load_partials<1, 2>(g.part_s, g.nparts, tot);
  block_sum_t<KBS, 2>(tot, sh);
  if (threadIdx.x != 0) return;
  KState* st = g.st;
  if (mode == 0) {
    st->bb = tot[1];
    st->it = 0;
    st->nchecks = 0;
  } else {
    st->nchecks += 1;
  }
  const double bb = st->bb, rr = tot[0];
  st->rr = rr;
  int nst = KS_RUN;
  // b at or below the rounding level of the terms it was formed from
  // (zero2, set by the caller; 0 if none) carries no information: x = 0
  if (bb == 0.0 || bb <= st->zero2) nst = KS_ZERO;
  else if (!finite(rr)) nst = KS_NONFINITE;
  else if (rr <= st->tol2 * bb) nst = KS_DONE;
  else if (launched >= g.maxit) nst = KS_MAXIT;
  // true residuals that stop falling: the tolerance is below the
  // attainable accuracy
  if (mode == 0 || rr <= 0.81 * st->rr_best) {
    st->rr_best = rr;
    st->nstall = 0;
  } else {
    st->nstall += 1;
  }
  if (nst == KS_RUN && st->nstall >= KSTALL_CHECKS) nst = KS_STALL;
  if (nst == KS_RUN) {
    st->sc[par ^ 1] = INFINITY;   // beta = gamma / inf = 0
    st->alpha[par ^ 1] = 1.0;
  }
  st->status = nst;
}

// ------------------------------------------------------------------ iteration
// Load order: the index words first (slice offsets, the first halo row), then
// the bulk of independent loads (state, partial sums, own rows' vectors), then
// what depends on the indices (the first chunk of eight matrix entries of
// every row, the first halo row's vectors), all before the first wait, so that
// a block spends one memory latency before the reduction instead of several.
// PF: the first chunk is kept in registers (parts of at most 4 KBS rows).
// sb[e], sw[e]: entry offset (with the lane) and width of this wave's slice
// of rows e; c0: the halo row of this thread (row 0 past the halo).
template <int EPT, class VT>
__device__ __forceinline__ void fcg_iter_body(const FGroup& g, int lb, int p0, int own, int h0,
                                              int nh, const int (&sb)[EPT], const int (&sw)[EPT],
                                              int c0, int par, double* loc, double* sh) {
  constexpr bool PF = EPT <= 4;
  const bool h_in = (int)threadIdx.x < nh;
  const gptr<const VT> val = G(static_cast<const VT*>(g.val));
  // own rows (rows past the part's end read its first row and are discarded)
  const gptr<const double> r0 = G((const double*)(par ? g.r[1] : g.r[0])),
                           s0v = G((const double*)(par ? g.s[1] : g.s[0])),
                           w0 = G((const double*)(par ? g.w[1] : g.w[0])), dv = G(g.dinv);
  double di[EPT], xi[EPT], ri[EPT], pi[EPT], si[EPT], wi[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    const int i = p0 + (l < own ? l : 0);
    di[e] = dv[i];
    xi[e] = G(g.xp)[i];
    ri[e] = r0[i];
    pi[e] = G(g.p)[i];
    si[e] = s0v[i];
    wi[e] = w0[i];
  }
  const gptr<const KState> st = G((const KState*)g.st);
  const int status = st->status;
  const double g_old = st->sc[par ^ 1], a_old = st->alpha[par ^ 1];
  const double lim = st->tol2 * st->bb;
  const double* part_in = par ? g.part[1] : g.part[0];
  double px[4][3];
  partials_first<1, 3>(part_in, g.nparts, px);
  // what depends on the index words: the first chunk of matrix entries and
  // the first halo row's vectors, used after the reduction (issued before the
  // partial sums are added, which waits for every load before it)
  int mc[PF ? EPT : 1][8];
  double mv[PF ? EPT : 1][8];
  if constexpr (PF) {
#pragma unroll
    for (int e = 0; e < EPT; ++e)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = q < sw[e] ? q : (sw[e] > 0 ? sw[e] - 1 : 0);
        mc[e][q] = G(g.lcol)[sb[e] + 64 * kk];
        mv[e][q] = (double)val[sb[e] + 64 * kk];
      }
  }
  // keep the loads above in flight here: the scheduler would otherwise sink
  // them below the waits for the halo row and the partial sums
  __builtin_amdgcn_sched_barrier(0);
  const double hr = r0[c0], hs = s0v[c0], hw = w0[c0], hd = dv[c0];
  double t[3];
  partials_rest<1, 3>(part_in, g.nparts, px, t);
  block_sum_t<KBS, 3>(t, sh);
  if (status != KS_RUN) return;
  const gptr<KState> stw = G(g.st);
  const bool lead = lb == 0 && threadIdx.x == 0;
  const double gam = t[0], rr = t[1], del = t[2];
  if (!(finite(gam) && finite(rr) && finite(del))) {
    if (lead) stw->status = KS_NONFINITE;
    return;
  }
  if (rr <= lim) {
    if (lead) {
      stw->status = KS_PENDING;
      stw->rr = rr;
    }
    return;
  }
  const double beta = gam / g_old;
  const double den = del - beta * gam / a_old;
  if (!(den > 0.0)) {
    if (lead) stw->status = KS_BREAKDOWN;
    return;
  }
  const double alpha = gam / den;
  if (lead) {
    stw->sc[par] = gam;
    stw->alpha[par] = alpha;
    stw->rr = rr;
    stw->it += 1;
  }
  const gptr<double> r1 = G(par ? g.r[0] : g.r[1]), s1v = G(par ? g.s[0] : g.s[1]);
  double rn[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    rn[e] = 0.0;
    if (l >= own) continue;
    const int i = p0 + l;
    const double p = fma(beta, pi[e], di[e] * ri[e]);
    const double s = fma(beta, si[e], wi[e]);
    const double r = fma(-alpha, s, ri[e]);
    G(g.xp)[i] = fma(alpha, p, xi[e]);
    G(g.p)[i] = p;
    s1v[i] = s;
    r1[i] = r;
    rn[e] = r;
    loc[l] = di[e] * r;
  }
  // halo rows: the same r and u their owners compute in this launch
  if (h_in) {
    const double s = fma(beta, hs, hw);
    const double r = fma(-alpha, s, hr);
    loc[own + threadIdx.x] = hd * r;
  }
  for (int q = threadIdx.x + KBS; q < nh; q += KBS) {
    const int c = G(g.halo)[h0 + q];
    const double s = fma(beta, s0v[c], w0[c]);
    const double r = fma(-alpha, s, r0[c]);
    loc[own + q] = dv[c] * r;
  }
  __syncthreads();
  double y[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    y[e] = 0.0;
    const int w = sw[e];
    int k0 = 0;
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < 8; ++q) y[e] += q < w ? mv[e][q] * loc[mc[e][q]] : 0.0;
      k0 = 8;
    }
    for (int k = k0; k < w; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
        c[q] = G(g.lcol)[sb[e] + 64 * kk];
        a[q] = (double)val[sb[e] + 64 * kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) y[e] += k + q < w ? a[q] * loc[c[q]] : 0.0;
    }
  }
  const gptr<double> w1 = G(par ? g.w[0] : g.w[1]);
  double acc[3] = {};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    if (l >= own) continue;
    const double u = loc[l];
    w1[p0 + l] = y[e];
    acc[0] += rn[e] * u;
    acc[1] += rn[e] * rn[e];
    acc[2] += y[e] * u;
  }
  store_partials<1, 3>(acc, par ? g.part[0] : g.part[1], g.nparts, lb, sh);
}

// Groups and parts through the block map (any number of groups).
template <int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_fcg_iter(const FGroup* groups, const int2* bmap,
                                                  int par) {
  FGROUP_HEAD(bmap)
  extern __shared__ double loc[];
  __shared__ double sh[(KBS / 64) * 3];
  const int s0 = g.slice_ptr[lb], s1 = g.slice_ptr[lb + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // index words: this wave's slices (waves past a part's last slice re-read
  // it and discard the result) and the first halo row
  int sb[EPT], sw[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int sl0 = s0 + (KBS / 64) * e + wv;
    const int sl = sl0 < s1 ? sl0 : s1 - 1;
    const int a = G(g.sptr)[sl], z = G(g.sptr)[sl + 1];
    sb[e] = a + lane;
    sw[e] = sl0 < s1 ? (z - a) >> 6 : 0;
  }
  // (the halo array always holds at least one word; threads past the halo
  // use row 0 and discard what they read)
  const bool h_in = (int)threadIdx.x < nh;
  const int c0r = G(g.halo)[h_in ? h0 + (int)threadIdx.x : 0];
  fcg_iter_body<EPT, VT>(g, lb, p0, own, h0, nh, sb, sw, h_in ? c0r : 0, par, loc, sh);
}

// One group, passed by value, and one FBlk per block: the slice offsets and
// the first halo row come one dependent load after the block starts, where
// the block map, the group and the part tables take three.
template <int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_fcg_iter1(const FGroup g, const FBlk* blk,
                                                   const int32_t* hfirst, int par) {
  extern __shared__ double loc[];
  __shared__ double sh[(KBS / 64) * 3];
  const FBlk& B = blk[blockIdx.x];
  const int lb = B.lb, p0 = B.p0, own = B.own, h0 = B.h0, nh = B.nh;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  static_assert((KBS / 64) * EPT <= FBLK_SL, "slice slots of an FBlk");
  int sb[EPT], sw[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int2 d = B.sl[(KBS / 64) * e + wv];
    sb[e] = d.x + lane;
    sw[e] = d.y;
  }
  const int c0 = G(hfirst)[(size_t)blockIdx.x * KBS + threadIdx.x];
  fcg_iter_body<EPT, VT>(g, lb, p0, own, h0, nh, sb, sw, c0, par, loc, sh);
}

// x (original order) := part-order iterate; b == 0 systems: x := 0
__global__ void __launch_bounds__(KBS) k_fcg_finish(const FGroup* groups, const int2* bmap) {
  FGROUP_HEAD(bmap)
  (void)h0;
  (void)nh;
  const bool zero = g.st->status == KS_ZERO;
  for (int l = threadIdx.x; l < own; l += KBS) {
    const int i = p0 + l;
    g.x[g.perm[i]] = zero ? 0.0 : g.xp[i];
  }
}

template <class VT>
__global__ void k_fcg_gather_values(int64_t nent, const int32_t* src, const VT* val, VT* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nent) out[e] = src[e] >= 0 ? val[src[e]] : VT(0);
}

__global__ void k_fcg_gather_dinv(int64_t n, const int32_t* perm, const double* dinv,
                                  double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = dinv[perm[i]];
}

// ------------------------------------------------------------------ two iterations per launch
// s-step CG with s = 2 (Chronopoulos and Gear 1989; Carson and Demmel's
// communication-avoiding CG, monomial basis) with the Jacobi preconditioner
// D^{-1}, B = D^{-1} A. An outer step starts from (x, p, z = D^{-1} r) and the
// basis Y = [p, B p, B^2 p, z, B z] (all in the block's own rows); with the
// D-weighted Gram matrix Gm = Y^T D Y (one global reduction) two CG iterations
// run in the coordinates of Y: r.z = z^T D z and p.A p = p^T D (B p), and B
// maps the coordinates of p, B p and z to those of B p, B^2 p and B z. In exact
// arithmetic the iterates are those of textbook Jacobi-PCG, two per launch.
//
// One launch is one outer step. A block owns one part: it reduces the previous
// launch's Gram partials, forms the coefficients, and updates x on its own rows
// and p, z on its own rows, its halo and its second halo ring from the
// previous basis (written by their owners in the previous launch; the basis is
// double-buffered by launch parity). It then forms B p on its own and halo
// rows (the halo rows' matrix slices read p on the second ring), B^2 p and B z
// on its own rows, all out of LDS, and writes the new basis and the partials
// of the next Gram matrix and of ||D z||^2 = ||r||^2 (the residual of the x
// this launch starts from: the stop test lags by one outer step, and a system
// whose residual meets the tolerance keeps that x).

// index of Gram entry (a, b), a <= b, in the upper triangle, row by row
__host__ __device__ constexpr int g2i(int a, int b) { return a * 5 - a * (a - 1) / 2 + (b - a); }

__device__ __forceinline__ double g2quad(const double (&G)[5][5], const double (&u)[5],
                                         const double (&v)[5]) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < 5; ++b) t += G[a][b] * v[b];
    s += u[a] * t;
  }
  return s;
}

// Two CG iterations in the coordinates of Y (p, Bp, B^2 p, z, Bz). Returns
// false on a breakdown of the first iteration; the second is skipped (the
// step keeps the first iteration's x, p and z) when its residual or curvature
// is not positive, which only rounding at convergence produces.
__device__ __forceinline__ bool s2_coeffs(const double (&t)[16], double (&cx)[5],
                                          double (&cz)[5], double (&cp)[5]) {
  double G[5][5];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) G[a][b] = t[a <= b ? g2i(a, b) : g2i(b, a)];
#pragma unroll
  for (int k = 0; k < 5; ++k) cx[k] = cz[k] = cp[k] = 0.0;
  cp[0] = 1.0;
  cz[3] = 1.0;
  double zz = G[3][3];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double w[5] = {0.0, cp[0], cp[1], 0.0, cp[3]};   // B p in coordinates
    const double den = g2quad(G, cp, w);
    if (!(zz > 0.0 && den > 0.0)) return j > 0;
    const double al = zz / den;
    double czn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) czn[k] = cz[k] - al * w[k];
    const double zzn = g2quad(G, czn, czn);
    // rounding level reached within the step: keep the first iteration
    if (j > 0 && !(zzn > 0.0)) return true;
    const double be = zzn / zz;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      cx[k] += al * cp[k];
      cz[k] = czn[k];
      cp[k] = czn[k] + be * cp[k];
    }
    zz = zzn;
  }
  return true;
}

// The rows of a part's local numbering: own, halo, second ring.
struct F2Rows {
  int p0, own, h0, nh, g0, nh2;
  __device__ __forceinline__ int row(const FGroup& g, int l) const {
    if (l < own) return p0 + l;
    if (l < own + nh) return G(g.halo)[h0 + l - own];
    return G(g.halo2)[g0 + l - own - nh];
  }
};

// y[e] = (A loc)(own row KBS e + tid) for NV LDS vectors at once (locs[v] at
// offsets vo[v] in loc), from the part's own slices; rows past the part give 0.
template <int EPT, int NV, class VT>
__device__ __forceinline__ void own_spmv(const FGroup& g, int lb, const double* loc,
                                         const int (&vo)[NV], double (&y)[NV][EPT]) {
  const gptr<const VT> val = G(static_cast<const VT*>(g.val));
  const int s0 = G(g.slice_ptr)[lb], s1 = G(g.slice_ptr)[lb + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
#pragma unroll
    for (int v = 0; v < NV; ++v) y[v][e] = 0.0;
    const int sl = s0 + (KBS / 64) * e + wv;
    if (sl >= s1) continue;
    const int b0 = G(g.sptr)[sl];
    const int w = (G(g.sptr)[sl + 1] - b0) >> 6;
    const int base = b0 + lane;
    for (int k = 0; k < w; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
        c[q] = G(g.lcol)[base + 64 * kk];
        a[q] = (double)val[base + 64 * kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int v = 0; v < NV; ++v) y[v][e] += k + q < w ? a[q] * loc[vo[v] + c[q]] : 0.0;
    }
  }
}

// out[own + q] = D^{-1} (A loc)(halo row q) for the part's halo rows (their
// slices read own, halo and second-ring entries of loc).
template <class VT>
__device__ __forceinline__ void halo_spmv(const FGroup& g, int lb, const F2Rows& R,
                                          const double* loc, double* out) {
  const gptr<const VT> hval = G(static_cast<const VT*>(g.hval));
  const int s0 = G(g.hslice_ptr)[lb], s1 = G(g.hslice_ptr)[lb + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int sl = s0 + wv; sl < s1; sl += KBS / 64) {
    const int q = 64 * (sl - s0) + lane;
    const int b0 = G(g.hsptr)[sl];
    const int w = (G(g.hsptr)[sl + 1] - b0) >> 6;
    const int base = b0 + lane;
    double y = 0.0;
    for (int k = 0; k < w; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) {
        const int kk = k + qq < w ? k + qq : w - 1;
        c[qq] = G(g.hlcol)[base + 64 * kk];
        a[qq] = (double)hval[base + 64 * kk];
      }
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) y += k + qq < w ? a[qq] * loc[c[qq]] : 0.0;
    }
    if (q < R.nh) out[R.own + q] = G(g.dinv)[G(g.halo)[R.h0 + q]] * y;
  }
}

// The matrix powers and the partials of an outer step, with p and z of the
// step in LDS (lp, lz over own, halo and second ring): B p on own and halo
// rows, B^2 p and B z on own rows; the new basis goes to Yn (own rows) and the
// Gram partials and ||D z||^2 to part.
template <int EPT, class VT>
__device__ __forceinline__ void s2_powers(const FGroup& g, int lb, const F2Rows& R,
                                          double* lds, int L2, double* Yn, double* part,
                                          double* sh) {
  double* lp = lds;
  double* lz = lds + L2;
  double* lbp = lds + 2 * L2;   // B p on own and halo rows
  double ap[2][EPT];
  {
    const int vo[2] = {0, L2};
    own_spmv<EPT, 2, VT>(g, lb, lds, vo, ap);   // A p, A z on own rows
  }
  double bz[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    bz[e] = 0.0;
    if (l >= R.own) continue;
    const double di = G(g.dinv)[R.p0 + l];
    lbp[l] = di * ap[0][e];
    bz[e] = di * ap[1][e];
  }
  halo_spmv<VT>(g, lb, R, lp, lbp);
  __syncthreads();
  double a2[1][EPT];
  {
    const int vo[1] = {0};
    own_spmv<EPT, 1, VT>(g, lb, lbp, vo, a2);   // A (B p) on own rows
  }
  const int n = g.n;
  double acc[16] = {};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + (int)threadIdx.x;
    if (l >= R.own) continue;
    const int i = R.p0 + l;
    const double di = G(g.dinv)[i];
    const double v[5] = {lp[l], lbp[l], di * a2[0][e], lz[l], bz[e]};
#pragma unroll
    for (int j = 0; j < 5; ++j) G(Yn)[(size_t)j * n + i] = v[j];
    const double d = 1.0 / di;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const double da = d * v[a];
#pragma unroll
      for (int b = a; b < 5; ++b) acc[g2i(a, b)] += da * v[b];
    }
    const double r = d * v[3];
    acc[15] += r * r;
  }
  store_partials<2, 8>(acc, part, g.nparts, lb, sh);
}

// The 16 Gram partials of the previous launch, this thread's share (blocks
// tid, tid + KBS, ... in order, two records in flight): fewer registers than
// load_partials' four records of 16 values.
__device__ __forceinline__ void load_partials16(const double* part, int nb, double (&v)[16]) {
  constexpr int QC = 2;
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = 0.0;
  const gptr<const double> P = G(part);
  for (int q0 = 0; q0 * KBS < nb; q0 += QC) {
    double x[QC][16];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int b = (int)threadIdx.x + (q0 + q) * KBS;
      const int bc = b < nb ? b : nb - 1;
#pragma unroll
      for (int k = 0; k < 16; ++k) x[q][k] = P[part_index(k >> 3, k & 7, nb, bc)];
    }
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const bool ok = (int)threadIdx.x + (q0 + q) * KBS < nb;
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] += ok ? x[q][k] : 0.0;
    }
  }
}

// a value that is the same in every lane, kept in scalar registers
__device__ __forceinline__ double uniform(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

#define FGROUP2_HEAD(BMAP)                                                     \
  FGROUP_HEAD(BMAP)                                                            \
  const int g0_ = G(g.halo2_ptr)[lb];                                          \
  const F2Rows R{p0, own, h0, nh, g0_, G(g.halo2_ptr)[lb + 1] - g0_};          \
  const int L2 = own + nh + R.nh2;

// First outer step of a (re)start: p = z = D^{-1} r (r of the start, all
// rows), its basis and partials into y[par], part[par].
template <int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_fcg2_first(const FGroup* groups, const int2* bmap,
                                                    int mode, int par) {
  FGROUP2_HEAD(bmap)
  extern __shared__ double lds[];
  __shared__ double sh[(KBS / 64) * 16];
  if (!fcg_active(g, mode)) return;
  const gptr<const double> r = G((const double*)(par ? g.r[1] : g.r[0]));
  for (int l = threadIdx.x; l < L2; l += KBS) {
    const int i = R.row(g, l);
    const double z = G(g.dinv)[i] * r[i];
    lds[l] = z;
    lds[L2 + l] = z;
  }
  __syncthreads();
  s2_powers<EPT, VT>(g, lb, R, lds, L2, par ? g.y[1] : g.y[0], par ? g.part[1] : g.part[0],
                     sh);
}

// One outer step (two CG iterations). Loads are issued in dependency order:
// the index words (own slice offsets, this thread's halo slice and its halo or
// second-ring row), then, before the reduction, D^{-1} of the own rows, the
// basis of this thread's halo or ring row and the first partial sums; after
// the coefficients, the own rows' basis and x, and the first chunk of eight
// matrix entries of every own row and of this thread's halo row. Thread q
// takes halo row q (and ring row q - nhalo); parts with more halo and ring
// rows than threads take the rest in a loop.
template <int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_fcg2_iter(const FGroup* groups, const int2* bmap,
                                                   int par) {
  FGROUP2_HEAD(bmap)
  extern __shared__ double lds[];
  __shared__ double sh[(KBS / 64) * 16];
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int n = g.n;
  const int nr = nh + R.nh2;            // halo and second-ring rows
  const gptr<const VT> val = G(static_cast<const VT*>(g.val));
  const gptr<const VT> hval = G(static_cast<const VT*>(g.hval));
  const gptr<const double> Y = G((const double*)(par ? g.y[1] : g.y[0])), dv = G(g.dinv);
  // ---- index words
  const int s0 = G(g.slice_ptr)[lb], s1 = G(g.slice_ptr)[lb + 1];
  int sb[EPT], sw[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int sl0 = s0 + (KBS / 64) * e + wv;
    const int sl = sl0 < s1 ? sl0 : s1 - 1;
    const int a = G(g.sptr)[sl], z = G(g.sptr)[sl + 1];
    sb[e] = a + lane;
    sw[e] = sl0 < s1 ? (z - a) >> 6 : 0;
  }
  const int hs0 = G(g.hslice_ptr)[lb], hs1 = G(g.hslice_ptr)[lb + 1];
  const bool h_in = tid < nh, r_in = tid < nr;
  int hb = 0, hw = 0;
  if (hs1 > hs0) {   // the part has halo rows (uniform)
    const int hsl0 = hs0 + (tid >> 6);
    const int hsl = hsl0 < hs1 ? hsl0 : hs1 - 1;
    const int a = G(g.hsptr)[hsl], z = G(g.hsptr)[hsl + 1];
    hb = a + lane;
    hw = h_in ? (z - a) >> 6 : 0;
  }
  const int rrow = h_in ? G(g.halo)[h0 + tid]
                        : (r_in ? G(g.halo2)[R.g0 + tid - nh] : p0);
  // ---- data
  const gptr<const KState> st = G((const KState*)g.st);
  const int status = st->status;
  const double lim = st->tol2 * st->bb;
  double di[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + tid;
    di[e] = dv[p0 + (l < own ? l : 0)];
  }
  double yr[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) yr[j] = Y[(size_t)j * n + rrow];
  const double dr = dv[rrow];
  const double* part_in = par ? g.part[1] : g.part[0];
  double px[16];
  {
    const gptr<const double> P = G(part_in);
    const int bc = tid < g.nparts ? tid : g.nparts - 1;
#pragma unroll
    for (int k = 0; k < 16; ++k) px[k] = P[part_index(k >> 3, k & 7, g.nparts, bc)];
  }
  __builtin_amdgcn_sched_barrier(0);
  // ---- reduction and coefficients
  double t[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = 0.0;
  {
    const bool ok = tid < g.nparts;
#pragma unroll
    for (int k = 0; k < 16; ++k) t[k] += ok ? px[k] : 0.0;
  }
  {
    const gptr<const double> P = G(part_in);
    for (int q0 = 1; q0 * KBS < g.nparts; q0 += 2) {
      double x[2][16];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int b = tid + (q0 + q) * KBS;
        const int bc = b < g.nparts ? b : g.nparts - 1;
#pragma unroll
        for (int k = 0; k < 16; ++k) x[q][k] = P[part_index(k >> 3, k & 7, g.nparts, bc)];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const bool ok = tid + (q0 + q) * KBS < g.nparts;
#pragma unroll
        for (int k = 0; k < 16; ++k) t[k] += ok ? x[q][k] : 0.0;
      }
    }
  }
  block_sum_t<KBS, 16>(t, sh);
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = uniform(t[k]);
  if (status != KS_RUN) return;
  const gptr<KState> stw = G(g.st);
  const bool lead = lb == 0 && tid == 0;
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) fin &= finite(t[k]);
  if (!fin) {
    if (lead) stw->status = KS_NONFINITE;
    return;
  }
  const double rr = t[15];
  if (rr <= lim) {
    if (lead) {
      stw->status = KS_PENDING;
      stw->rr = rr;
    }
    return;
  }
  double cx[5], cz[5], cp[5];
  if (!s2_coeffs(t, cx, cz, cp)) {
    if (lead) stw->status = KS_BREAKDOWN;
    return;
  }
  if (lead) {
    stw->rr = rr;
    stw->it += 2;
  }
  // ---- p and z of this step; x
  auto comb = [](const double (&c)[5], const double* y) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) s = fma(c[j], y[j], s);
    return s;
  };
  double po[EPT], zo[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + tid;
    const int i = p0 + (l < own ? l : 0);
    double yo[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) yo[j] = Y[(size_t)j * n + i];
    const double xo = G(g.xp)[i];
    po[e] = comb(cp, yo);
    zo[e] = comb(cz, yo);
    if (l >= own) continue;
    lds[l] = po[e];
    lds[L2 + l] = zo[e];
    double xv = xo;
#pragma unroll
    for (int j = 0; j < 5; ++j) xv = fma(cx[j], yo[j], xv);
    G(g.xp)[i] = xv;
  }
  if (r_in) {
    lds[own + tid] = comb(cp, yr);
    lds[L2 + own + tid] = comb(cz, yr);
  }
  for (int q = tid + KBS; q < nr; q += KBS) {   // rows past the threads
    const int i = R.row(g, own + q);
    double y[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) y[j] = Y[(size_t)j * n + i];
    lds[own + q] = comb(cp, y);
    lds[L2 + own + q] = comb(cz, y);
  }
  // the first chunk of eight matrix entries of the own rows and of this
  // thread's halo row: issued here, not with the loads before the reduction,
  // where they would hold 48 more registers per thread through it and cost a
  // wave per SIMD
  int mc[EPT][8];
  double mv[EPT][8];
#pragma unroll
  for (int e = 0; e < EPT; ++e)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kk = q < sw[e] ? q : (sw[e] > 0 ? sw[e] - 1 : 0);
      mc[e][q] = G(g.lcol)[sb[e] + 64 * kk];
      mv[e][q] = (double)val[sb[e] + 64 * kk];
    }
  int hc[8];
  double hv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kk = q < hw ? q : (hw > 0 ? hw - 1 : 0);
    hc[q] = hs1 > hs0 ? G(g.hlcol)[hb + 64 * kk] : 0;
    hv[q] = hs1 > hs0 ? (double)hval[hb + 64 * kk] : 0.0;
  }
  __syncthreads();
  // ---- B p on own and halo rows, B z on own rows
  double* lbp = lds + 2 * L2;
  double bz[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + tid;
    double ap = 0.0, az = 0.0;
    const int w = sw[e];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      ap += q < w ? mv[e][q] * lds[mc[e][q]] : 0.0;
      az += q < w ? mv[e][q] * lds[L2 + mc[e][q]] : 0.0;
    }
    for (int k = 8; k < w; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
        c[q] = G(g.lcol)[sb[e] + 64 * kk];
        a[q] = (double)val[sb[e] + 64 * kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ap += k + q < w ? a[q] * lds[c[q]] : 0.0;
        az += k + q < w ? a[q] * lds[L2 + c[q]] : 0.0;
      }
    }
    bz[e] = di[e] * az;
    if (l < own) lbp[l] = di[e] * ap;
  }
  if (h_in) {
    double hp = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) hp += q < hw ? hv[q] * lds[hc[q]] : 0.0;
    for (int k = 8; k < hw; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < hw ? k + q : hw - 1;
        c[q] = G(g.hlcol)[hb + 64 * kk];
        a[q] = (double)hval[hb + 64 * kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) hp += k + q < hw ? a[q] * lds[c[q]] : 0.0;
    }
    lbp[own + tid] = dr * hp;
  }
  if (nh > KBS) {   // halo rows past the threads (uniform)
    const int hs = G(g.hslice_ptr)[lb];
    for (int q = tid + KBS; q < nh; q += KBS) {
      const int sl = hs + (q >> 6);
      const int b0 = G(g.hsptr)[sl] + (q & 63);
      const int w = (G(g.hsptr)[sl + 1] - G(g.hsptr)[sl]) >> 6;
      double hp = 0.0;
      for (int k = 0; k < w; ++k) hp += (double)hval[b0 + 64 * k] * lds[G(g.hlcol)[b0 + 64 * k]];
      lbp[own + q] = dv[G(g.halo)[h0 + q]] * hp;
    }
  }
  __syncthreads();
  // ---- B^2 p on own rows; the new basis and its partials
  const gptr<double> Yn = G(par ? g.y[0] : g.y[1]);
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int l = KBS * e + tid;
    const int w = sw[e];
    double a2 = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) a2 += q < w ? mv[e][q] * lbp[mc[e][q]] : 0.0;
    for (int k = 8; k < w; k += 8) {
      int c[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
        c[q] = G(g.lcol)[sb[e] + 64 * kk];
        a[q] = (double)val[sb[e] + 64 * kk];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) a2 += k + q < w ? a[q] * lbp[c[q]] : 0.0;
    }
    if (l >= own) continue;
    const int i = p0 + l;
    const double v[5] = {po[e], lbp[l], di[e] * a2, zo[e], bz[e]};
#pragma unroll
    for (int j = 0; j < 5; ++j) Yn[(size_t)j * n + i] = v[j];
    const double d = 1.0 / di[e];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const double da = d * v[a];
#pragma unroll
      for (int b = a; b < 5; ++b) acc[g2i(a, b)] += da * v[b];
    }
    const double r = d * v[3];
    acc[15] += r * r;
  }
  store_partials<2, 8>(acc, par ? g.part[0] : g.part[1], g.nparts, lb, sh);
}

// ------------------------------------------------------------------ launchers
template <int V>
using fic = std::integral_constant<int, V>;

template <class F>
static void with_ept_vt(const FLaunch& L, F f) {
  auto vt = [&](auto E) {
    if (L.fp32) f(E, float{});
    else f(E, double{});
  };
  switch (L.ept) {
    case 1: vt(fic<1>{}); break;
    case 2: vt(fic<2>{}); break;
    case 4: vt(fic<4>{}); break;
    case 8: vt(fic<8>{}); break;
    default: fail(IPCS_E_INVALID, "fused CG takes 1, 2, 4 or 8 rows per thread");
  }
}

#define FEPT decltype(E)::value
#define FVT decltype(V)

void fcg_start(hipStream_t s, const FLaunch& L, int mode, int par, int launched) {
  with_ept_vt(L, [&](auto E, auto V) {
    launch(k_fcg_resid<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.groups,
           L.bmap, mode, par);
    HIP_LAUNCH_OK();
    if (L.ipl == 2)
      launch(k_fcg2_first<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.groups,
             L.bmap, mode, par);
    else
      launch(k_fcg_first<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.groups,
             L.bmap, mode, par);
    HIP_LAUNCH_OK();
  });
  launch(k_fcg_decide, dim3(L.ngroups), dim3(KBS), 0, s, L.groups, mode, par, launched);
  HIP_LAUNCH_OK();
}

void fcg_iter(hipStream_t s, const FLaunch& L, int par) {
  with_ept_vt(L, [&](auto E, auto V) {
    if (L.ipl == 2)
      launch(k_fcg2_iter<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.groups,
             L.bmap, par);
    else if (L.blk)
      launch(k_fcg_iter1<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.one,
             L.blk, L.hfirst, par);
    else
      launch(k_fcg_iter<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.groups,
             L.bmap, par);
  });
  HIP_LAUNCH_OK();
}

void fcg_finish(hipStream_t s, const FLaunch& L) {
  launch(k_fcg_finish, dim3(L.nblocks), dim3(KBS), 0, s, L.groups, L.bmap);
  HIP_LAUNCH_OK();
}

void fcg_gather_values(hipStream_t s, bool fp32, int64_t nent, const int32_t* src,
                       const void* val, void* out) {
  const dim3 grid((unsigned)div_up(nent, BLOCK));
  if (fp32)
    launch(k_fcg_gather_values<float>, grid, dim3(BLOCK), 0, s, nent, src,
           static_cast<const float*>(val), static_cast<float*>(out));
  else
    launch(k_fcg_gather_values<double>, grid, dim3(BLOCK), 0, s, nent, src,
           static_cast<const double*>(val), static_cast<double*>(out));
  HIP_LAUNCH_OK();
}

void fcg_gather_dinv(hipStream_t s, int64_t n, const int32_t* perm, const double* dinv,
                     double* out) {
  launch(k_fcg_gather_dinv, dim3((unsigned)div_up(n, BLOCK)), dim3(BLOCK), 0, s, n, perm, dinv,
         out);
  HIP_LAUNCH_OK();
}

}  // namespace ipcs
