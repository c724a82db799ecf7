// Jacobi-preconditioned CG and BiCGStab for gfx950 on SELL-64 matrices.
//
// Parallel shape. Every kernel runs blocks of KBS = 256 threads (4 waves).
// Matrix kernels give each thread ept_m rows; a wavefront owns 64 consecutive
// rows, one per lane, and reads column k of its SELL slice as one coalesced
// 64-wide load of values and of column indices. The loads of a row are batched
// eight columns at a time: eight (column, value) loads, then the eight gathers
// of every system, then the FMAs, so that eight gathers per system are in flight
// per lane. Vector kernels give each thread kept_v(NS) entries. The systems of a
// group share the matrix (the velocity components of a run): each matrix entry
// is loaded once and applied to every system's vector. A launch serves many
// groups through a (group, block) map, e.g. all runs of a serving batch.
//
// Reductions are fence-free and deterministic (dev_util.hpp): a kernel writes
// one set of partial sums per block, and every block of the next kernel
// re-reduces all of them in a fixed order. Keeping blocks at 256 threads with several
// entries per thread keeps the number of records small (at most KNB_MAX).
// Each kernel issues its independent loads (state words, vector entries, then
// partial records) before its first wait: every load goes through a global
// (not flat) pointer, from an always-valid address (rows past the end read row
// 0 and are discarded), so no branch or wait separates them; scalars that
// depend on the reduction are applied last. Scalars never leave the device; the host polls status
// words only.
//
// PCG in the Chronopoulos-Gear form (one global reduction per iteration; the
// iterates are those of Jacobi-PCG, Saad 2003 Alg. 9.1, in exact arithmetic),
// with u = D^{-1} r, w = A u, s = A p:
//   spmv  : w = A u, partial u.w                           (no prologue)
//   update: [gamma = r.u, ||r||^2, delta = u.w] -> stop test;
//           beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old);
//           p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//           u = D^{-1} r, partials r.u, r.r
// BiCGStab (van der Vorst 1992, right preconditioning D^{-1}), four kernels:
//   b2 v = A phat, partial rhat.v                          (no prologue)
//   b3 [rhat.v, ||r||^2] stop test, alpha = rho / rhat.v; s = r - alpha v,
//      shat = D^{-1} s
//   b4 t = A shat, partials t.s, t.t, rhat.s, rhat.t       (no prologue)
//   b5 [t.s, t.t, rhat.s, rhat.t] omega = t.s / t.t; x += D^{-1}(alpha p + omega s)
//      (= alpha phat + omega shat, from vectors this kernel reads anyway),
//      r = s - omega t; rho' = rhat.r = rhat.s - omega rhat.t, beta =
//      (rho' / rho)(alpha / omega); p = r + beta (p - omega v), phat = D^{-1} p;
//      partial r.r
// Stopping rule: ||r||_2 <= tol ||b||_2 on the recursive residual, then
// confirmed with b - A x (restart from x if it fails), up to maxit iterations.
// A right-hand side whose norm is at the rounding level of the terms it was
// formed from (the pressure Poisson b is a difference of terms that cancel
// exactly at a discrete steady state) is treated as zero.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"
#include "launch.hpp"

namespace ipcs {

#define GROUP_HEAD(BMAP)                  \
  const int2 m_ = (BMAP)[blockIdx.x];     \
  const KGroup& g = groups[m_.x];         \
  const int lb = m_.y;

// Row i of the group's SELL-64 matrix applied to NS gathered vectors:
// acc[j] = sum_k A(i, col_k) * gath(j, col_k), in FP64 whatever the stored
// value type VT. The slice width is uniform in the wavefront; the last chunk
// of eight re-reads entry w-1 and discards it.
template <int NS, class VT, class GF>
__device__ __forceinline__ void sell_row(const KGroup& g, int i, GF gath, double (&acc)[NS]) {
  const gptr<const VT> val = G(static_cast<const VT*>(g.val));
  const gptr<const int32_t> col = G(g.col);
  const int s = i >> 6;
  const int b0 = G(g.sptr)[s];
  const int w = (G(g.sptr)[s + 1] - b0) >> 6;
  const int base = b0 + (i & 63);
#pragma unroll
  for (int j = 0; j < NS; ++j) acc[j] = 0.0;
  for (int k = 0; k < w; k += 8) {
    int c[8];
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kk = k + q < w ? k + q : w - 1;
      c[q] = col[base + 64 * kk];
      a[q] = (double)val[base + 64 * kk];
    }
    double xv[NS][8];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int q = 0; q < 8; ++q) xv[j][q] = gath(j, c[q]);
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[j] += k + q < w ? a[q] * xv[j][q] : 0.0;
  }
}

template <int EPT>
__device__ __forceinline__ int row_of(int lb, int e) {
  return (lb * EPT + e) * KBS + (int)threadIdx.x;
}

// Rows past the end of the last block load row 0 (always valid) and discard
// the result, so loads need no branch around them.
__device__ __forceinline__ int row_clamp(int i, int n) { return i < n ? i : 0; }

// ------------------------------------------------------------------ start / confirm
// r = b - A x for the systems that start (mode 0: all) or are confirmed
// (mode 1: PENDING or RESTART). PCG: u = D^{-1} r, p = s = 0. BiCGStab:
// rhat = p = r, phat = D^{-1} r. Partials r.r, r.u, b.b.
template <bool PCG, int NS, int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_start(const KGroup* groups, const int2* bmap, int mode) {
  GROUP_HEAD(bmap)
  __shared__ double sh[(KBS / 64) * NS * 3];
  bool act[NS];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int st = G(g.v[j].st)->status;
    act[j] = mode == 0 || st == KS_PENDING || st == KS_RESTART;
    any |= act[j];
  }
  double acc[NS * 3] = {};
  if (any) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = row_of<EPT>(lb, e);
      if (i >= g.n) continue;
      double ax[NS];
      sell_row<NS, VT>(g, i, [&](int j, int c) { return G(g.v[j].x)[c]; }, ax);
      const double di = G(g.dinv)[i];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        if (!act[j]) continue;
        const KVecs& V = g.v[j];
        const double bi = V.b[i], r = bi - ax[j];
        V.r[i] = r;
        if (PCG) {
          const double u = di * r;
          V.u[(size_t)i * NS] = u;
          V.p[i] = 0.0;
          V.s[i] = 0.0;
          acc[j * 3 + 1] += r * u;
        } else {
          V.u[(size_t)i * NS] = r;
          V.p[i] = r;
          V.phat[(size_t)i * NS] = di * r;
          acc[j * 3 + 1] += r * r;
        }
        acc[j * 3 + 0] += r * r;
        acc[j * 3 + 2] += bi * bi;
      }
    }
  }
  store_partials<NS, 3>(acc, g.part_m, g.nblk_m, lb, sh);
}

// One block per group: decide the status of the systems that were started or
// confirmed, initialize their scalars for an iteration of launch parity par,
// and seed the partials that iteration's first vector kernel reduces.
template <bool PCG, int NS>
__global__ void __launch_bounds__(KBS) k_decide(const KGroup* groups, int mode, int par,
                                                int launched) {
  const KGroup& g = groups[blockIdx.x];
  __shared__ double sh[(KBS / 64) * NS * 3];
  __shared__ int run_s[NS];
  double tot[NS * 3];
  load_partials<NS, 3>(g.part_m, g.nblk_m, tot);
  block_sum_t<KBS, NS * 3>(tot, sh);
  if (threadIdx.x == 0) {
    for (int j = 0; j < NS; ++j) {
      run_s[j] = 0;
      KState* st = g.v[j].st;
      const int s0 = st->status;
      const bool part = mode == 0 || s0 == KS_PENDING || s0 == KS_RESTART;
      if (!part) continue;
      if (mode == 0) {
        st->bb = tot[j * 3 + 2];
        st->it = 0;
        st->nchecks = 0;
      } else {
        st->nchecks += 1;
      }
      const double bb = st->bb, rr = tot[j * 3];
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
      st->status = nst;
      if (nst != KS_RUN) continue;
      if (PCG) {
        st->sc[par ^ 1] = INFINITY;   // beta = gamma / inf = 0 on the first iteration
        st->alpha[par ^ 1] = 1.0;
      } else {
        st->sc[par] = rr;             // rho_0 = rhat.r = r.r
        st->omega = 1.0;
      }
      run_s[j] = 1;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < g.nblk_v; b += KBS)
    for (int j = 0; j < NS; ++j) {
      if (!run_s[j]) continue;
      double* p = g.part_v[par];
      p[part_index(j, 0, g.nblk_v, b)] = b == 0 ? (PCG ? tot[j * 3 + 1] : tot[j * 3]) : 0.0;
      p[part_index(j, 1, g.nblk_v, b)] = b == 0 ? tot[j * 3] : 0.0;
    }
}

// ------------------------------------------------------------------ reduction totals
// This thread's share of the totals a vector kernel needs (block_sum_t then
// completes them): the same loads and order in a vector kernel's blocks and in
// the fold kernel, so folded totals are bitwise those a block would form.
// PCG update: [r.u, r.r] of the last update (part_v[par]), u.w of the SpMV
template <int NS>
__device__ __forceinline__ void cg_update_totals(const KGroup& g, int par, double (&t)[NS * 3]) {
  double a[NS * 2], b[NS];
  load_partials<NS, 2>(g.part_v[par], g.nblk_v, a);
  load_partials<NS, 1>(g.part_m, g.nblk_m, b);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    t[j * 3 + 0] = a[j * 2];
    t[j * 3 + 1] = a[j * 2 + 1];
    t[j * 3 + 2] = b[j];
  }
}
// BiCGStab s-update: [rhat.v (SpMV), r.r (last x-update)]
template <int NS>
__device__ __forceinline__ void bicg3_totals(const KGroup& g, int par, double (&t)[NS * 2]) {
  double a[NS], b[NS];
  load_partials<NS, 1>(g.part_m, g.nblk_m, a);
  load_partials<NS, 1>(g.part_v[par], g.nblk_v, b);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    t[j * 2] = a[j];
    t[j * 2 + 1] = b[j];
  }
}
// BiCGStab x-update: [t.s, t.t, rhat.s, rhat.t] (SpMV)
template <int NS>
__device__ __forceinline__ void bicg5_totals(const KGroup& g, double (&t)[NS * 4]) {
  load_partials<NS, 4>(g.part_m, g.nblk_m, t);
}

// One block per group: the totals of kernel KIND (0 PCG update, 1 BiCGStab
// s-update, 2 BiCGStab x-update) into g.fold, read by every block of that
// kernel in its folding form.
template <int KIND, int NS>
__global__ void __launch_bounds__(KBS) k_fold(const KGroup* groups, int par) {
  const KGroup& g = groups[blockIdx.x];
  constexpr int K = KIND == 0 ? 3 : KIND == 1 ? 2 : 4;
  __shared__ double sh[(KBS / 64) * NS * K];
  double t[NS * K];
  if constexpr (KIND == 0) cg_update_totals<NS>(g, par, t);
  else if constexpr (KIND == 1) bicg3_totals<NS>(g, par, t);
  else bicg5_totals<NS>(g, t);
  block_sum_t<KBS, NS * K>(t, sh);
  if ((int)threadIdx.x < NS * K) {
    double v = 0.0;
#pragma unroll
    for (int n = 0; n < NS * K; ++n) v = n == (int)threadIdx.x ? t[n] : v;
    G(g.fold)[threadIdx.x] = v;
  }
}

// ------------------------------------------------------------------ PCG (Chronopoulos-Gear)
template <int NS, int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_cg_spmv(const KGroup* groups, const int2* bmap) {
  GROUP_HEAD(bmap)
  __shared__ double sh[(KBS / 64) * NS];
  bool run[NS];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    run[j] = G(g.v[j].st)->status == KS_RUN;
    any |= run[j];
  }
  double y[EPT][NS], ui[EPT][NS];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = row_clamp(row_of<EPT>(lb, e), g.n);
    sell_row<NS, VT>(g, i, [&](int j, int c) { return G(g.v[j].u)[(size_t)c * NS]; }, y[e]);
#pragma unroll
    for (int j = 0; j < NS; ++j) ui[e][j] = G(g.v[j].u)[(size_t)i * NS];
  }
  if (!any) return;   // uniform: the states were written by an earlier kernel
  double acc[NS] = {};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = row_of<EPT>(lb, e);
    if (i >= g.n) continue;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (!run[j]) continue;
      G(g.v[j].w)[i] = y[e][j];
      acc[j] += y[e][j] * ui[e][j];
    }
  }
  store_partials<NS, 1>(acc, g.part_m, g.nblk_m, lb, sh);
}

template <int NS, bool FOLD>
__global__ void __launch_bounds__(KBS) k_cg_update(const KGroup* groups, const int2* bmap,
                                                   int par) {
  GROUP_HEAD(bmap)
  constexpr int EV = kept_v(NS);
  __shared__ double sh[(KBS / 64) * NS * 3];
  int status[NS];
  double g_old[NS], a_old[NS], lim[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const gptr<const KState> st = G((const KState*)g.v[j].st);
    status[j] = st->status;
    g_old[j] = st->sc[par ^ 1];
    a_old[j] = st->alpha[par ^ 1];
    lim[j] = st->tol2 * st->bb;
  }
  double di[EV], xi[EV][NS], ri[EV][NS], pi[EV][NS], si[EV][NS],
      wi[EV][NS];
#pragma unroll
  for (int e = 0; e < EV; ++e) {
    const int i = row_clamp(row_of<EV>(lb, e), g.n);
    di[e] = G(g.dinv)[i];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const KVecs& V = g.v[j];
      xi[e][j] = G(V.x)[i];
      ri[e][j] = G(V.r)[i];
      pi[e][j] = G(V.p)[i];
      si[e][j] = G(V.s)[i];
      wi[e][j] = G(V.w)[i];
    }
  }
  double t[NS * 3];
  if constexpr (FOLD) {
#pragma unroll
    for (int n = 0; n < NS * 3; ++n) t[n] = G((const double*)g.fold)[n];
  } else {
    cg_update_totals<NS>(g, par, t);
    block_sum_t<KBS, NS * 3>(t, sh);
  }
  const bool lead = lb == 0 && threadIdx.x == 0;
  bool go[NS];
  double al[NS], be[NS];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    go[j] = false;
    al[j] = be[j] = 0.0;
    if (status[j] != KS_RUN) continue;
    KState* st = g.v[j].st;
    const double gam = t[j * 3], rr = t[j * 3 + 1], del = t[j * 3 + 2];
    if (!(finite(gam) && finite(rr) && finite(del))) {
      if (lead) st->status = KS_NONFINITE;
      continue;
    }
    if (rr <= lim[j]) {
      if (lead) {
        st->status = KS_PENDING;
        st->rr = rr;
      }
      continue;
    }
    const double beta = gam / g_old[j];
    const double den = del - beta * gam / a_old[j];
    if (!(den > 0.0)) {
      if (lead) st->status = KS_BREAKDOWN;
      continue;
    }
    const double alpha = gam / den;
    if (lead) {
      st->sc[par] = gam;
      st->alpha[par] = alpha;
      st->rr = rr;
      st->it += 1;
    }
    go[j] = true;
    al[j] = alpha;
    be[j] = beta;
    any = true;
  }
  if (!any) return;   // uniform: every thread took the same decisions
  double acc[NS * 2] = {};
#pragma unroll
  for (int e = 0; e < EV; ++e) {
    const int i = row_of<EV>(lb, e);
    if (i >= g.n) continue;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (!go[j]) continue;
      const KVecs& V = g.v[j];
      const double p = di[e] * ri[e][j] + be[j] * pi[e][j];
      const double s = wi[e][j] + be[j] * si[e][j];
      const double x = xi[e][j] + al[j] * p;
      const double r = ri[e][j] - al[j] * s;
      const double u = di[e] * r;
      G(V.x)[i] = x;
      G(V.r)[i] = r;
      G(V.p)[i] = p;
      G(V.s)[i] = s;
      G(V.u)[(size_t)i * NS] = u;
      acc[j * 2] += r * u;
      acc[j * 2 + 1] += r * r;
    }
  }
  store_partials<NS, 2>(acc, g.part_v[par ^ 1], g.nblk_v, lb, sh);
}

// ------------------------------------------------------------------ BiCGStab
// b2 (WHICH = 0): v = A phat, partial rhat.v
// b4 (WHICH = 1): t = A shat, partials t.s, t.t, rhat.s, rhat.t
template <int WHICH, int NS, int EPT, class VT>
__global__ void __launch_bounds__(KBS) k_bicg_spmv(const KGroup* groups, const int2* bmap) {
  GROUP_HEAD(bmap)
  constexpr int K = WHICH == 0 ? 1 : 4;
  __shared__ double sh[(KBS / 64) * NS * K];
  bool run[NS];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    run[j] = G(g.v[j].st)->status == KS_RUN;
    any |= run[j];
  }
  // b4 follows the s-update of the same iteration, which has already ended
  // the systems whose residual met the tolerance: when none is left the
  // block skips its loads (the iteration launched past convergence would
  // otherwise read the whole matrix); b2 issues its loads first, as the
  // systems' status is decided after it
  if (WHICH == 1 && !any) return;
  double y[EPT][NS], rh[EPT][NS], si[EPT][NS];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = row_clamp(row_of<EPT>(lb, e), g.n);
    if (WHICH == 0)
      sell_row<NS, VT>(g, i, [&](int j, int c) { return G(g.v[j].phat)[(size_t)c * NS]; }, y[e]);
    else
      sell_row<NS, VT>(g, i, [&](int j, int c) { return G(g.v[j].shat)[(size_t)c * NS]; }, y[e]);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      rh[e][j] = G(g.v[j].u)[(size_t)i * NS];
      si[e][j] = WHICH == 1 ? G(g.v[j].s)[i] : 0.0;
    }
  }
  if (!any) return;
  double acc[NS * K] = {};
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int i = row_of<EPT>(lb, e);
    if (i >= g.n) continue;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (!run[j]) continue;
      const double yv = y[e][j];
      if (WHICH == 0) {
        G(g.v[j].w)[i] = yv;
        acc[j * K] += rh[e][j] * yv;
      } else {
        G(g.v[j].t)[i] = yv;
        acc[j * K + 0] += yv * si[e][j];
        acc[j * K + 1] += yv * yv;
        acc[j * K + 2] += rh[e][j] * si[e][j];
        acc[j * K + 3] += rh[e][j] * yv;
      }
    }
  }
  store_partials<NS, K>(acc, g.part_m, g.nblk_m, lb, sh);
}

template <int NS, bool FOLD>
__global__ void __launch_bounds__(KBS) k_bicg_3(const KGroup* groups, const int2* bmap, int par) {
  GROUP_HEAD(bmap)
  constexpr int EV = kept_v(NS);
  __shared__ double sh[(KBS / 64) * NS * 2];
  int status[NS];
  double rho[NS], lim[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const gptr<const KState> st = G((const KState*)g.v[j].st);
    status[j] = st->status;
    rho[j] = st->sc[par];
    lim[j] = st->tol2 * st->bb;
  }
  double di[EV], ri[EV][NS], vi[EV][NS];
#pragma unroll
  for (int e = 0; e < EV; ++e) {
    const int i = row_clamp(row_of<EV>(lb, e), g.n);
    di[e] = G(g.dinv)[i];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      ri[e][j] = G(g.v[j].r)[i];
      vi[e][j] = G(g.v[j].w)[i];
    }
  }
  double t[NS * 2];   // rhat.v, r.r
  if constexpr (FOLD) {
#pragma unroll
    for (int n = 0; n < NS * 2; ++n) t[n] = G((const double*)g.fold)[n];
  } else {
    bicg3_totals<NS>(g, par, t);
    block_sum_t<KBS, NS * 2>(t, sh);
  }
  const bool lead = lb == 0 && threadIdx.x == 0;
  bool go[NS];
  double al[NS];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    go[j] = false;
    al[j] = 0.0;
    if (status[j] != KS_RUN) continue;
    KState* st = g.v[j].st;
    const double rv = t[j * 2], rr = t[j * 2 + 1];
    if (!(finite(rv) && finite(rr))) {
      if (lead) st->status = KS_NONFINITE;
      continue;
    }
    if (rr <= lim[j]) {
      if (lead) {
        st->status = KS_PENDING;
        st->rr = rr;
      }
      continue;
    }
    const double alpha = rho[j] / rv;
    if (!(std::fabs(rv) >= 1e-300) || !finite(alpha)) {
      if (lead) {
        st->status = KS_RESTART;
        st->rr = rr;
      }
      continue;
    }
    if (lead) {
      st->alpha[0] = alpha;
      st->rr = rr;
    }
    go[j] = true;
    al[j] = alpha;
    any = true;
  }
  if (!any) return;
#pragma unroll
  for (int e = 0; e < EV; ++e) {
    const int i = row_of<EV>(lb, e);
    if (i >= g.n) continue;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (!go[j]) continue;
      const double s = ri[e][j] - al[j] * vi[e][j];
      G(g.v[j].s)[i] = s;
      G(g.v[j].shat)[(size_t)i * NS] = di[e] * s;
    }
  }
}

template <int NS, bool FOLD>
__global__ void __launch_bounds__(KBS) k_bicg_5(const KGroup* groups, const int2* bmap, int par) {
  GROUP_HEAD(bmap)
  constexpr int EV = kept_v(NS);
  __shared__ double sh[(KBS / 64) * NS * 4];
  int status[NS];
  double rho[NS], alpha[NS];
  bool live = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const gptr<const KState> st = G((const KState*)g.v[j].st);
    status[j] = st->status;
    rho[j] = st->sc[par];
    alpha[j] = st->alpha[0];
    live |= status[j] == KS_RUN;
  }
  if (!live) return;   // as in b4: nothing to update, skip the loads
  double di[EV], xi[EV][NS], si[EV][NS], ti[EV][NS], pi[EV][NS], vi[EV][NS];
#pragma unroll
  for (int e = 0; e < EV; ++e) {
    const int i = row_clamp(row_of<EV>(lb, e), g.n);
    di[e] = G(g.dinv)[i];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const KVecs& V = g.v[j];
      xi[e][j] = G(V.x)[i];
      si[e][j] = G(V.s)[i];
      ti[e][j] = G(V.t)[i];
      pi[e][j] = G(V.p)[i];
      vi[e][j] = G(V.w)[i];
    }
  }
  double t[NS * 4];   // t.s, t.t, rhat.s, rhat.t
  if constexpr (FOLD) {
#pragma unroll
    for (int n = 0; n < NS * 4; ++n) t[n] = G((const double*)g.fold)[n];
  } else {
    bicg5_totals<NS>(g, t);
    block_sum_t<KBS, NS * 4>(t, sh);
  }
  const bool lead = lb == 0 && threadIdx.x == 0;
  bool go[NS], full[NS];
  double om[NS], be[NS];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    go[j] = full[j] = false;
    om[j] = be[j] = 0.0;
    if (status[j] != KS_RUN) continue;
    KState* st = g.v[j].st;
    const double ts = t[j * 4], tt = t[j * 4 + 1], rs = t[j * 4 + 2], rt = t[j * 4 + 3];
    if (!(finite(ts) && finite(tt) && finite(rs) && finite(rt))) {
      if (lead) st->status = KS_NONFINITE;
      continue;
    }
    // t.t == 0 means A shat = 0, so s = 0: x + alpha phat solves the system
    const double omega = tt == 0.0 ? 0.0 : ts / tt;
    const double rho_n = rs - omega * rt;
    const double beta = (rho_n / rho[j]) * (alpha[j] / omega);
    int nst = KS_RUN;
    if (tt == 0.0) nst = KS_PENDING;
    else if (!(std::fabs(omega) >= 1e-300) || !(std::fabs(rho_n) >= 1e-300) || !finite(beta))
      nst = KS_RESTART;
    if (lead) {
      st->sc[par ^ 1] = rho_n;
      st->omega = omega;
      st->it += 1;
      if (nst != KS_RUN) st->status = nst;
    }
    go[j] = true;
    full[j] = nst == KS_RUN;
    om[j] = omega;
    be[j] = beta;
    any = true;
  }
  if (!any) return;
  double acc[NS] = {};
#pragma unroll
  for (int e = 0; e < EV; ++e) {
    const int i = row_of<EV>(lb, e);
    if (i >= g.n) continue;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      if (!go[j]) continue;
      const KVecs& V = g.v[j];
      G(V.x)[i] = xi[e][j] + di[e] * (alpha[j] * pi[e][j] + om[j] * si[e][j]);
      const double r = si[e][j] - om[j] * ti[e][j];
      G(V.r)[i] = r;
      acc[j] += r * r;
      if (full[j]) {
        const double p = r + be[j] * (pi[e][j] - om[j] * vi[e][j]);
        G(V.p)[i] = p;
        G(V.phat)[(size_t)i * NS] = di[e] * p;
      }
    }
  }
  store_partials<NS, 1>(acc, g.part_v[par ^ 1], g.nblk_v, lb, sh);
}

// ------------------------------------------------------------------ finish / poll
template <int NS>
__global__ void __launch_bounds__(KBS) k_finish(const KGroup* groups, const int2* bmap) {
  GROUP_HEAD(bmap)
  constexpr int EV = kept_v(NS);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    if (g.v[j].st->status != KS_ZERO) continue;
#pragma unroll
    for (int e = 0; e < EV; ++e) {
      const int i = row_of<EV>(lb, e);
      if (i < g.n) g.v[j].x[i] = 0.0;
    }
  }
}

__global__ void k_set_tol2(const KGroup* groups, int ngroups, double tol2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = t / GMAX, j = t % GMAX;
  if (gi < ngroups && j < groups[gi].nsys) groups[gi].v[j].st->tol2 = tol2;
}

__global__ void k_gather_states(const KGroup* groups, int ngroups, KState* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = t / GMAX, j = t % GMAX;
  if (gi < ngroups && j < groups[gi].nsys) out[t] = *groups[gi].v[j].st;
}

// ------------------------------------------------------------------ launchers
template <int V>
using ic = std::integral_constant<int, V>;

template <class F>
static void with_ns(int ns, F f) {
  switch (ns) {
    case 1: f(ic<1>{}); break;
    case 2: f(ic<2>{}); break;
    case 3: f(ic<3>{}); break;
    default: fail(IPCS_E_INVALID, "Krylov groups hold 1 to 3 systems");
  }
}

// matrix kernels: systems per group, rows per thread, stored value type
template <class F>
static void with_ns_ept(const KLaunch& L, F f) {
  with_ns(L.ns, [&](auto N) {
    auto vt = [&](auto E) {
      if (L.fp32) f(N, E, float{});
      else f(N, E, double{});
    };
    switch (L.ept_m) {
      case 1: vt(ic<1>{}); break;
      case 2: vt(ic<2>{}); break;
      case 4: vt(ic<4>{}); break;
      default: fail(IPCS_E_INVALID, "matrix kernels take 1, 2 or 4 rows per thread");
    }
  });
}

#define NSV decltype(N)::value
#define EPTV decltype(E)::value
#define VTV decltype(V)

template <bool PCG>
static void start_impl(hipStream_t s, const KLaunch& L, int mode, int par, int launched) {
  with_ns_ept(L, [&](auto N, auto E, auto V) {
    launch(k_start<PCG, NSV, EPTV, VTV>, dim3(L.nblocks_m), dim3(KBS), 0, s, L.groups,
                       L.bmap_m, mode);
  });
  HIP_LAUNCH_OK();
  with_ns(L.ns, [&](auto N) {
    launch(k_decide<PCG, NSV>, dim3(L.ngroups), dim3(KBS), 0, s, L.groups, mode,
                       par, launched);
  });
  HIP_LAUNCH_OK();
}

void pcg_start(hipStream_t s, const KLaunch& L, int mode, int par, int launched) {
  start_impl<true>(s, L, mode, par, launched);
}

void bicg_start(hipStream_t s, const KLaunch& L, int mode, int par, int launched) {
  start_impl<false>(s, L, mode, par, launched);
}

__global__ void k_stop_group(const KGroup* groups, int g) {
  const int j = threadIdx.x;
  if (j < groups[g].nsys && groups[g].v[j].st->status == KS_RUN)
    groups[g].v[j].st->status = KS_MAXIT;
}

void stop_group(hipStream_t s, const KLaunch& L, int g) {
  hipLaunchKernelGGL(k_stop_group, dim3(1), dim3(64), 0, s, L.groups, g);
  HIP_LAUNCH_OK();
}

void pcg_spmv_only(hipStream_t s, const KLaunch& L) {
  with_ns_ept(L, [&](auto N, auto E, auto V) {
    launch(k_cg_spmv<NSV, EPTV, VTV>, dim3(L.nblocks_m), dim3(KBS), 0, s, L.groups,
                       L.bmap_m);
  });
  HIP_LAUNCH_OK();
}

// The fold kernel is launched directly (not through launch()), so that a
// timing hook around the update times the update itself.
void pcg_update_only(hipStream_t s, const KLaunch& L, int par) {
  with_ns(L.ns, [&](auto N) {
    if (L.fold) {
      hipLaunchKernelGGL((k_fold<0, NSV>), dim3(L.ngroups), dim3(KBS), 0, s, L.groups, par);
      HIP_LAUNCH_OK();
      launch(k_cg_update<NSV, true>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v,
             par);
    } else {
      launch(k_cg_update<NSV, false>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v,
             par);
    }
  });
  HIP_LAUNCH_OK();
}

void pcg_iter(hipStream_t s, const KLaunch& L, int par) {
  pcg_spmv_only(s, L);
  pcg_update_only(s, L, par);
}

void bicg_spmv_only(hipStream_t s, const KLaunch& L) {
  with_ns_ept(L, [&](auto N, auto E, auto V) {
    launch(k_bicg_spmv<0, NSV, EPTV, VTV>, dim3(L.nblocks_m), dim3(KBS), 0, s, L.groups,
                       L.bmap_m);
  });
  HIP_LAUNCH_OK();
}

void bicg_update_s_only(hipStream_t s, const KLaunch& L, int par) {
  with_ns(L.ns, [&](auto N) {
    if (L.fold) {
      hipLaunchKernelGGL((k_fold<1, NSV>), dim3(L.ngroups), dim3(KBS), 0, s, L.groups, par);
      HIP_LAUNCH_OK();
      launch(k_bicg_3<NSV, true>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v, par);
    } else {
      launch(k_bicg_3<NSV, false>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v,
             par);
    }
  });
  HIP_LAUNCH_OK();
}

void bicg_spmv_t_only(hipStream_t s, const KLaunch& L) {
  with_ns_ept(L, [&](auto N, auto E, auto V) {
    launch(k_bicg_spmv<1, NSV, EPTV, VTV>, dim3(L.nblocks_m), dim3(KBS), 0, s, L.groups,
                       L.bmap_m);
  });
  HIP_LAUNCH_OK();
}

void bicg_update_x_only(hipStream_t s, const KLaunch& L, int par) {
  with_ns(L.ns, [&](auto N) {
    if (L.fold) {
      hipLaunchKernelGGL((k_fold<2, NSV>), dim3(L.ngroups), dim3(KBS), 0, s, L.groups, par);
      HIP_LAUNCH_OK();
      launch(k_bicg_5<NSV, true>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v, par);
    } else {
      launch(k_bicg_5<NSV, false>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v,
             par);
    }
  });
  HIP_LAUNCH_OK();
}

void bicg_iter(hipStream_t s, const KLaunch& L, int par) {
  bicg_spmv_only(s, L);
  bicg_update_s_only(s, L, par);
  bicg_spmv_t_only(s, L);
  bicg_update_x_only(s, L, par);
}

void ksys_finish(hipStream_t s, const KLaunch& L) {
  with_ns(L.ns, [&](auto N) {
    launch(k_finish<NSV>, dim3(L.nblocks_v), dim3(KBS), 0, s, L.groups, L.bmap_v);
  });
  HIP_LAUNCH_OK();
}

void set_tolerance(hipStream_t s, const KLaunch& L, double tol2) {
  const int n = L.ngroups * GMAX;
  hipLaunchKernelGGL(k_set_tol2, dim3((unsigned)div_up(n, 64)), dim3(64), 0, s, L.groups,
                     L.ngroups, tol2);
  HIP_LAUNCH_OK();
}

void gather_states(hipStream_t s, const KLaunch& L, KState* out) {
  const int n = L.ngroups * GMAX;
  hipLaunchKernelGGL(k_gather_states, dim3((unsigned)div_up(n, 64)), dim3(64), 0, s, L.groups,
                     L.ngroups, out);
  HIP_LAUNCH_OK();
}

}  // namespace ipcs
