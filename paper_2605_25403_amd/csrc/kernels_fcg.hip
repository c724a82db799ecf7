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
    launch(k_fcg_first<FEPT, FVT>, dim3(L.nblocks), dim3(KBS), (uint32_t)L.lds, s, L.groups,
           L.bmap, mode, par);
    HIP_LAUNCH_OK();
  });
  launch(k_fcg_decide, dim3(L.ngroups), dim3(KBS), 0, s, L.groups, mode, par, launched);
  HIP_LAUNCH_OK();
}

void fcg_iter(hipStream_t s, const FLaunch& L, int par) {
  with_ept_vt(L, [&](auto E, auto V) {
    if (L.blk)
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
