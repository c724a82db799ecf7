// Jacobi-preconditioned CG and BiCGStab for gfx950 on SELL-64 matrices.
//
// Layout and parallel shape. Matrices are stored in SELL-64 (see mesh.hpp):
// a wavefront owns 64 consecutive rows, one row per lane, and reads column k
// of its slice as one coalesced 64-wide load of values and of column indices;
// only the gathers x[col] are irregular. The systems of a group share the
// matrix (the velocity components of a run), so each matrix entry is loaded
// once and applied to every active system's vector. Every kernel runs one row
// or vector entry per thread in blocks of BS threads; a launch serves many
// groups through a (group, block) map, e.g. all runs of a serving batch.
//
// Reductions are fence-free and deterministic (dev_util.hpp): a kernel writes
// per-block partials, the next kernel re-reduces them in every block. Each
// kernel issues its independent loads (matrix entries, vector entries, the
// producer's partials, the state words) before it first waits, so their
// latencies overlap; scalars that depend on the reduction are applied last.
// Scalars never leave the device; the host only polls status words.
//
// PCG (Saad 2003, Alg. 9.1), two kernels per iteration:
//   spmv  : [r.z, r.r of the last update] -> convergence test, beta;
//           q = A z + beta A p_{k-1} (= A p_k), p_k = z + beta p_{k-1}
//           (double-buffered by iteration parity), partial p_k.q
//   update: [p.q] -> alpha = rho/p.q; x += alpha p, r -= alpha q,
//           z = D^{-1} r, partials r.z, r.r
// BiCGStab (van der Vorst 1992, right preconditioning D^{-1}), five kernels:
//   b1 [r.r, rhat.r] test, beta; p = r + beta (p - omega v), phat = D^{-1} p
//   b2 v = A phat, partial rhat.v
//   b3 [rhat.v] alpha; s = r - alpha v, shat = D^{-1} s
//   b4 t = A shat, partials t.s, t.t
//   b5 [t.s, t.t] omega; x += alpha phat + omega shat, r = s - omega t,
//      partials r.r, rhat.r
// Stopping rule: ||r||_2 <= tol ||b||_2 on the recursive residual, then
// confirmed with b - A x (restart from x if it fails), up to maxit iterations.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"

namespace ipcs {

#define GROUP_PROLOGUE                   \
  const int2 m_ = bmap[blockIdx.x];      \
  const KGroup& g = groups[m_.x];        \
  const int lb = m_.y;                   \
  const int ns = g.nsys;                 \
  const int i = lb * BS + (int)threadIdx.x; \
  const bool in = i < g.n;

// SELL-64 row i: slice base and width
struct SellRow {
  int base, w;
  __device__ __forceinline__ SellRow(const int32_t* sptr, int i) {
    const int s = i >> 6;
    const int b0 = sptr[s];
    base = b0 + (i & 63);
    w = (sptr[s + 1] - b0) >> 6;
  }
};

__device__ __forceinline__ bool is_run(const KGroup& g, int j) {
  return j < g.nsys && g.v[j].st->status == KS_RUN;
}

// ------------------------------------------------------------------ start / confirm
// r = b - A x and partials r.r, r.z (PCG; rhat.r = r.r for BiCGStab), b.b for
// systems that start (mode 0: all) or are confirmed (mode 1: status PENDING
// or RESTART).
template <bool PCG, int BS>
__global__ void __launch_bounds__(BS) k_start(const KGroup* groups, const int2* bmap,
                                                  int mode) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  bool act[GMAX];
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    act[j] = false;
    if (j < ns) {
      const int st = g.v[j].st->status;
      act[j] = mode == 0 || st == KS_PENDING || st == KS_RESTART;
    }
  }
  double acc[GMAX][3] = {};
  if (in) {
    const SellRow R(g.sptr, i);
    double ax[GMAX] = {};
    for (int k = 0; k < R.w; ++k) {
      const int idx = R.base + 64 * k;
      const double a = g.val[idx];
      const int c = g.col[idx];
#pragma unroll
      for (int j = 0; j < GMAX; ++j)
        if (act[j]) ax[j] += a * g.v[j].x[c];
    }
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!act[j]) continue;
      const KVecs& V = g.v[j];
      const double bi = V.b[i], r = bi - ax[j];
      V.r[i] = r;
      double z = r;
      if (PCG) z = g.dinv[i] * r;
      V.z[i] = z;   // PCG: z = D^{-1} r; BiCGStab: rhat = r
      acc[j][0] = r * r;
      acc[j][1] = r * z;
      acc[j][2] = bi * bi;
    }
  }
  store_partials<3>(acc, ns, g.part_m, lb, sh);
}

// One block per group: decide the status of the systems that were started or
// confirmed, and seed the partials the first iteration reduces.
template <bool PCG>
__global__ void __launch_bounds__(1024) k_decide(const KGroup* groups, int mode) {
  const KGroup& g = groups[blockIdx.x];
  const int ns = g.nsys;
  __shared__ double sh[16 * GMAX * 3];
  Partials<3> P;
  P.load(g.part_m, g.nblk, ns);
  double tot[GMAX][3];
  P.reduce(ns, tot, sh);
  __shared__ int act_s[GMAX];
  if (threadIdx.x == 0) {
    for (int j = 0; j < GMAX; ++j) {
      act_s[j] = 0;
      if (j >= ns) continue;
      KState* st = g.v[j].st;
      const bool part = mode == 0 || st->status == KS_PENDING || st->status == KS_RESTART;
      if (!part) continue;
      if (mode == 0) {
        st->bb = tot[j][2];
        st->it = 0;
        st->nchecks = 0;
      } else {
        st->nchecks += 1;
      }
      const double bb = st->bb, rr = tot[j][0];
      st->rr = rr;
      int nst = KS_RUN;
      if (bb == 0.0) nst = KS_ZERO;
      else if (!finite(rr)) nst = KS_NONFINITE;
      else if (rr <= st->tol2 * bb) nst = KS_DONE;
      else if (mode != 0 && st->it >= st->maxit) nst = KS_MAXIT;
      st->status = nst;
      if (nst == KS_RUN) {
        st->it0 = st->it;
        st->alpha = 1.0;
        st->omega = 1.0;
        st->tt_zero = 0;
        act_s[j] = 1;
      }
    }
  }
  __syncthreads();
  // the first iteration reduces part_v and must find (r.z, r.r) for PCG or
  // (r.r, rhat.r) for BiCGStab; only block 0's slot is non-zero
  for (int b = threadIdx.x; b < g.nblk; b += blockDim.x)
    for (int j = 0; j < ns; ++j) {
      if (!act_s[j]) continue;
      double* p = g.part_v + ((size_t)b * GMAX + j) * KP;
      p[0] = b == 0 ? (PCG ? tot[j][1] : tot[j][0]) : 0.0;
      p[1] = b == 0 ? tot[j][0] : 0.0;
    }
}

// ------------------------------------------------------------------ PCG
template <int BS>
__global__ void __launch_bounds__(BS) k_pcg_spmv(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  // state words (uniform loads), issued first
  bool run[GMAX];
  int par[GMAX];
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    run[j] = is_run(g, j);
    par[j] = j < ns ? (g.v[j].st->it & 1) : 0;
  }
  // A z and A p_{k-1}, independent of beta: their loads overlap the reduction
  double az[GMAX] = {}, ap[GMAX] = {}, zi[GMAX] = {}, poi[GMAX] = {};
  if (in) {
    const SellRow R(g.sptr, i);
    for (int k = 0; k < R.w; ++k) {
      const int idx = R.base + 64 * k;
      const double a = g.val[idx];
      const int c = g.col[idx];
#pragma unroll
      for (int j = 0; j < GMAX; ++j) {
        if (!run[j]) continue;
        const KVecs& V = g.v[j];
        az[j] += a * V.z[c];
        ap[j] += a * V.p[par[j] ^ 1][c];
      }
    }
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!run[j]) continue;
      zi[j] = g.v[j].z[i];
      poi[j] = g.v[j].p[par[j] ^ 1][i];
    }
  }
  Partials<2> Pv;
  Pv.load(g.part_v, g.nblk, ns);   // (r.z, r.r) of the last update
  double tot[GMAX][2];
  Pv.reduce(ns, tot, sh);
  double acc[GMAX][1] = {};
  bool any = false;
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    if (!run[j]) continue;
    KState* st = g.v[j].st;
    const int it = st->it;
    const bool first = it == st->it0;
    const double rz = tot[j][0], rr = tot[j][1];
    bool a = true;
    double beta = 0.0;
    if (!first) {
      if (!finite(rr)) {
        a = false;
        if (lb == 0 && threadIdx.x == 0) st->status = KS_NONFINITE;
      } else if (rr <= st->tol2 * st->bb || it >= st->maxit) {
        a = false;
        if (lb == 0 && threadIdx.x == 0) {
          st->status = KS_PENDING;
          st->rr = rr;
        }
      } else {
        beta = rz / st->rho[par[j] ^ 1];
      }
    }
    if (!a) continue;
    any = true;
    if (lb == 0 && threadIdx.x == 0) {
      st->rho[par[j]] = rz;
      st->par = par[j];
      st->rr = rr;
    }
    if (in) {
      const KVecs& V = g.v[j];
      const double q = first ? az[j] : az[j] + beta * ap[j];
      const double pi = first ? zi[j] : zi[j] + beta * poi[j];
      V.p[par[j]][i] = pi;
      V.q[i] = q;
      acc[j][0] = pi * q;
    }
  }
  // every thread took the same decisions; the block-wide OR makes the exit
  // provably uniform before the barriers in store_partials
  if (!__syncthreads_or(any)) return;
  store_partials<1>(acc, ns, g.part_m, lb, sh);
}

template <int BS>
__global__ void __launch_bounds__(BS) k_pcg_update(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  bool run[GMAX];
  int par[GMAX];
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    run[j] = is_run(g, j);
    par[j] = j < ns ? g.v[j].st->par : 0;
  }
  double xi[GMAX] = {}, pi[GMAX] = {}, ri[GMAX] = {}, qi[GMAX] = {};
  double di = 0.0;
  if (in) {
    di = g.dinv[i];
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!run[j]) continue;
      const KVecs& V = g.v[j];
      xi[j] = V.x[i];
      pi[j] = V.p[par[j]][i];
      ri[j] = V.r[i];
      qi[j] = V.q[i];
    }
  }
  Partials<1> Pm;
  Pm.load(g.part_m, g.nblk, ns);   // p.q
  double tot[GMAX][1];
  Pm.reduce(ns, tot, sh);
  double acc[GMAX][2] = {};
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    if (!run[j]) continue;
    KState* st = g.v[j].st;
    const double pq = tot[j][0];
    if (!finite(pq)) {
      if (lb == 0 && threadIdx.x == 0) st->status = KS_NONFINITE;
      continue;
    }
    if (!(pq > 0.0)) {
      if (lb == 0 && threadIdx.x == 0) st->status = KS_BREAKDOWN;
      continue;
    }
    const double alpha = st->rho[par[j]] / pq;
    if (lb == 0 && threadIdx.x == 0) st->it += 1;
    if (in) {
      const KVecs& V = g.v[j];
      V.x[i] = xi[j] + alpha * pi[j];
      const double r = ri[j] - alpha * qi[j];
      const double z = di * r;
      V.r[i] = r;
      V.z[i] = z;
      acc[j][0] = r * z;
      acc[j][1] = r * r;
    }
  }
  store_partials<2>(acc, ns, g.part_v, lb, sh);
}

// ------------------------------------------------------------------ BiCGStab
template <int BS>
__global__ void __launch_bounds__(BS) k_bicg_1(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  bool run[GMAX];
#pragma unroll
  for (int j = 0; j < GMAX; ++j) run[j] = is_run(g, j);
  double ri[GMAX] = {}, pi[GMAX] = {}, vi[GMAX] = {};
  double di = 0.0;
  if (in) {
    di = g.dinv[i];
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!run[j]) continue;
      ri[j] = g.v[j].r[i];
      pi[j] = g.v[j].p[0][i];
      vi[j] = g.v[j].q[i];
    }
  }
  Partials<2> Pv;
  Pv.load(g.part_v, g.nblk, ns);   // (r.r, rhat.r)
  double tot[GMAX][2];
  Pv.reduce(ns, tot, sh);
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    if (!run[j]) continue;
    KState* st = g.v[j].st;
    const int it = st->it, par = it & 1;
    const bool first = it == st->it0;
    const double rr = tot[j][0], rhr = tot[j][1], omega = st->omega;
    double beta = 0.0;
    if (!first) {
      const bool lead = lb == 0 && threadIdx.x == 0;
      if (!finite(rr)) {
        if (lead) st->status = KS_NONFINITE;
        continue;
      }
      if (rr <= st->tol2 * st->bb || st->tt_zero || it >= st->maxit) {
        if (lead) {
          st->status = KS_PENDING;
          st->rr = rr;
        }
        continue;
      }
      if (fabs(omega) < 1e-300 || fabs(rhr) < 1e-300) {
        if (lead) {
          st->status = KS_RESTART;
          st->rr = rr;
        }
        continue;
      }
      beta = (rhr / st->rho[par ^ 1]) * (st->alpha / omega);
    }
    if (lb == 0 && threadIdx.x == 0) {
      st->rho[par] = rhr;
      st->par = par;
      st->rr = rr;
    }
    if (in) {
      const double p = first ? ri[j] : ri[j] + beta * (pi[j] - omega * vi[j]);
      g.v[j].p[0][i] = p;
      g.v[j].phat[i] = di * p;
    }
  }
}

// WHICH = 0: v = A phat, partial rhat.v;  WHICH = 1: t = A shat, partials t.s, t.t
template <int WHICH, int BS>
__global__ void __launch_bounds__(BS) k_bicg_spmv(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  bool run[GMAX];
  bool any = false;
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    run[j] = is_run(g, j);
    any |= run[j];
  }
  if (!__syncthreads_or(any)) return;
  double acc[GMAX][2] = {};
  if (in) {
    const SellRow R(g.sptr, i);
    double y[GMAX] = {};
    for (int k = 0; k < R.w; ++k) {
      const int idx = R.base + 64 * k;
      const double a = g.val[idx];
      const int c = g.col[idx];
#pragma unroll
      for (int j = 0; j < GMAX; ++j)
        if (run[j]) y[j] += a * (WHICH == 0 ? g.v[j].phat[c] : g.v[j].shat[c]);
    }
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!run[j]) continue;
      const KVecs& V = g.v[j];
      if (WHICH == 0) {
        V.q[i] = y[j];
        acc[j][0] = V.z[i] * y[j];
      } else {
        V.t[i] = y[j];
        acc[j][0] = y[j] * V.s[i];
        acc[j][1] = y[j] * y[j];
      }
    }
  }
  store_partials<2>(acc, ns, g.part_m, lb, sh);
}

template <int BS>
__global__ void __launch_bounds__(BS) k_bicg_3(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  bool run[GMAX];
#pragma unroll
  for (int j = 0; j < GMAX; ++j) run[j] = is_run(g, j);
  double ri[GMAX] = {}, vi[GMAX] = {};
  double di = 0.0;
  if (in) {
    di = g.dinv[i];
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!run[j]) continue;
      ri[j] = g.v[j].r[i];
      vi[j] = g.v[j].q[i];
    }
  }
  Partials<1> Pm;
  Pm.load(g.part_m, g.nblk, ns);   // rhat.v
  double tot[GMAX][1];
  Pm.reduce(ns, tot, sh);
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    if (!run[j]) continue;
    KState* st = g.v[j].st;
    const double alpha = st->rho[st->par] / tot[j][0];
    if (!finite(alpha)) {
      if (lb == 0 && threadIdx.x == 0) st->status = KS_NONFINITE;
      continue;
    }
    if (lb == 0 && threadIdx.x == 0) st->alpha = alpha;
    if (in) {
      const double s = ri[j] - alpha * vi[j];
      g.v[j].s[i] = s;
      g.v[j].shat[i] = di * s;
    }
  }
}

template <int BS>
__global__ void __launch_bounds__(BS) k_bicg_5(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  __shared__ double sh[16 * GMAX * 3];
  bool run[GMAX];
#pragma unroll
  for (int j = 0; j < GMAX; ++j) run[j] = is_run(g, j);
  double xi[GMAX] = {}, phi[GMAX] = {}, shi[GMAX] = {}, si[GMAX] = {}, ti[GMAX] = {},
         rhi[GMAX] = {};
  if (in) {
#pragma unroll
    for (int j = 0; j < GMAX; ++j) {
      if (!run[j]) continue;
      const KVecs& V = g.v[j];
      xi[j] = V.x[i];
      phi[j] = V.phat[i];
      shi[j] = V.shat[i];
      si[j] = V.s[i];
      ti[j] = V.t[i];
      rhi[j] = V.z[i];
    }
  }
  Partials<2> Pm;
  Pm.load(g.part_m, g.nblk, ns);   // (t.s, t.t)
  double tot[GMAX][2];
  Pm.reduce(ns, tot, sh);
  double acc[GMAX][2] = {};
#pragma unroll
  for (int j = 0; j < GMAX; ++j) {
    if (!run[j]) continue;
    KState* st = g.v[j].st;
    const double alpha = st->alpha;
    const bool zero = tot[j][1] == 0.0;
    const double omega = zero ? 0.0 : tot[j][0] / tot[j][1];
    if (lb == 0 && threadIdx.x == 0) {
      st->omega = omega;
      st->tt_zero = zero;
      st->it += 1;
    }
    if (in) {
      const KVecs& V = g.v[j];
      V.x[i] = xi[j] + alpha * phi[j] + omega * shi[j];
      const double r = si[j] - omega * ti[j];
      V.r[i] = r;
      acc[j][0] = r * r;
      acc[j][1] = rhi[j] * r;
    }
  }
  store_partials<2>(acc, ns, g.part_v, lb, sh);
}

// ------------------------------------------------------------------ finish / poll
template <int BS>
__global__ void __launch_bounds__(BS) k_finish(const KGroup* groups, const int2* bmap) {
  GROUP_PROLOGUE
  if (!in) return;
  for (int j = 0; j < ns; ++j)
    if (g.v[j].st->status == KS_ZERO) g.v[j].x[i] = 0.0;
}

__global__ void k_gather_states(const KGroup* groups, int ngroups, KState* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = t / GMAX, j = t % GMAX;
  if (gi < ngroups && j < groups[gi].nsys) out[t] = *groups[gi].v[j].st;
}

// ------------------------------------------------------------------ launchers
#define LK(KER, L, s, ...)                                                                     \
  do {                                                                                         \
    switch ((L).bs) {                                                                          \
      case 256: hipLaunchKernelGGL(KER<256>, dim3((L).nblocks), dim3(256), 0, s, (L).groups,  \
                                   (L).bmap, ##__VA_ARGS__); break;                            \
      case 512: hipLaunchKernelGGL(KER<512>, dim3((L).nblocks), dim3(512), 0, s, (L).groups,  \
                                   (L).bmap, ##__VA_ARGS__); break;                            \
      case 1024: hipLaunchKernelGGL(KER<1024>, dim3((L).nblocks), dim3(1024), 0, s,           \
                                    (L).groups, (L).bmap, ##__VA_ARGS__); break;               \
      default: fail(IPCS_E_INVALID, "unsupported Krylov block size");                         \
    }                                                                                          \
    HIP_LAUNCH_OK();                                                                           \
  } while (0)

#define K_START_PCG(B) k_start<true, B>
#define K_START_BICG(B) k_start<false, B>
#define K_SPMV0(B) k_bicg_spmv<0, B>
#define K_SPMV1(B) k_bicg_spmv<1, B>

#define LK2(KMAC, L, s, ...)                                                                   \
  do {                                                                                         \
    switch ((L).bs) {                                                                          \
      case 256: hipLaunchKernelGGL(KMAC(256), dim3((L).nblocks), dim3(256), 0, s, (L).groups, \
                                   (L).bmap, ##__VA_ARGS__); break;                            \
      case 512: hipLaunchKernelGGL(KMAC(512), dim3((L).nblocks), dim3(512), 0, s, (L).groups, \
                                   (L).bmap, ##__VA_ARGS__); break;                            \
      case 1024: hipLaunchKernelGGL(KMAC(1024), dim3((L).nblocks), dim3(1024), 0, s,          \
                                    (L).groups, (L).bmap, ##__VA_ARGS__); break;               \
      default: fail(IPCS_E_INVALID, "unsupported Krylov block size");                         \
    }                                                                                          \
    HIP_LAUNCH_OK();                                                                           \
  } while (0)

void pcg_start(hipStream_t s, const KLaunch& L, int mode) {
  LK2(K_START_PCG, L, s, mode);
  hipLaunchKernelGGL(k_decide<true>, dim3(L.ngroups), dim3(1024), 0, s, L.groups, mode);
  HIP_LAUNCH_OK();
}

void pcg_iter(hipStream_t s, const KLaunch& L) {
  LK(k_pcg_spmv, L, s);
  LK(k_pcg_update, L, s);
}

void bicg_start(hipStream_t s, const KLaunch& L, int mode) {
  LK2(K_START_BICG, L, s, mode);
  hipLaunchKernelGGL(k_decide<false>, dim3(L.ngroups), dim3(1024), 0, s, L.groups, mode);
  HIP_LAUNCH_OK();
}

void bicg_iter(hipStream_t s, const KLaunch& L) {
  LK(k_bicg_1, L, s);
  LK2(K_SPMV0, L, s);
  LK(k_bicg_3, L, s);
  LK2(K_SPMV1, L, s);
  LK(k_bicg_5, L, s);
}

void ksys_finish(hipStream_t s, const KLaunch& L) { LK(k_finish, L, s); }

void gather_states(hipStream_t s, const KLaunch& L, KState* out) {
  const int n = L.ngroups * GMAX;
  hipLaunchKernelGGL(k_gather_states, dim3((unsigned)div_up(n, 64)), dim3(64), 0, s, L.groups,
                     L.ngroups, out);
  HIP_LAUNCH_OK();
}

void pcg_spmv_only(hipStream_t s, const KLaunch& L) { LK(k_pcg_spmv, L, s); }
void pcg_update_only(hipStream_t s, const KLaunch& L) { LK(k_pcg_update, L, s); }
void bicg_spmv_only(hipStream_t s, const KLaunch& L) { LK2(K_SPMV0, L, s); }

}  // namespace ipcs
