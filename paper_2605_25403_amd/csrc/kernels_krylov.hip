// Jacobi-preconditioned CG and BiCGStab on CSR matrices for gfx950.
//
// A launch serves any number of independent systems (velocity components,
// or the systems of several runs in the serving form): block b works on system
// bmap[b].x as its block bmap[b].y of sys.nblk. Rows are spread over lane
// groups of G lanes (a power of two <= 64, chosen near the mean row length)
// so one row's column indices and values are read by adjacent lanes with
// coalesced loads; the group sums its products with cross-lane shuffles.
// Dot products use per-block partials finished by the last block to arrive, in
// block order, so results are deterministic and identical whether a system is
// solved alone or together with others. All scalars (alpha, beta, omega, rho,
// norms, status) stay in device memory; the host only polls the status words.
//
// PCG (Saad 2003, Alg. 9.1), two kernels per iteration:
//   A: p_k = z + beta p_{k-1} (formed on the fly, double-buffered), q = A p_k,
//      p_k.q  -> alpha = rho / p_k.q
//   B: x += alpha p_k, r -= alpha q, z = D^{-1} r, r.z, r.r -> beta, test
// BiCGStab (van der Vorst 1992, right-preconditioned with D^{-1}), five kernels:
//   p = r + beta (p - omega v), phat = D^{-1} p | v = A phat, rhat.v -> alpha |
//   s = r - alpha v, shat = D^{-1} s | t = A shat, t.s, t.t -> omega |
//   x += alpha phat + omega shat, r = s - omega t, r.r, rhat.r -> test
// Stopping rule: ||r||_2 <= tol ||b||_2 on the recursive residual, then
// confirmed on b - A x (restart from x if it fails), up to maxit iterations.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"

namespace ipcs {

#define SYS_PROLOGUE                  \
  const int2 m_ = bmap[blockIdx.x];   \
  const KSys& S = sys[m_.x];          \
  const int lb = m_.y;                \
  KState* st = S.st;

template <int G>
__device__ __forceinline__ double row_dot(const KSys& S, int i, int lane, const double* x) {
  double s = 0.0;
  const int e = S.rowptr[i + 1];
  for (int k = S.rowptr[i] + lane; k < e; k += G) s += S.val[k] * x[S.col[k]];
  return group_sum<G>(s);
}

// ---------------------------------------------------------------- PCG
// mode 0: start (all systems); mode 1: confirm systems in KS_PENDING with the
// true residual and restart those that fail.
template <int G>
__global__ void __launch_bounds__(BLOCK) k_pcg_init(const KSys* sys, const int2* bmap, int mode) {
  SYS_PROLOGUE
  if (mode != 0 && st->status != KS_PENDING) return;
  const int lane = threadIdx.x % G;
  const int grp = lb * (BLOCK / G) + threadIdx.x / G, ngrp = S.nblk * (BLOCK / G);
  double* p0 = S.p[st->pc];
  double arr = 0.0, arz = 0.0, abb = 0.0;
  for (int i = grp; i < S.n; i += ngrp) {
    const double ax = row_dot<G>(S, i, lane, S.x);
    if (lane == 0) {
      const double bi = S.b[i], r = bi - ax, z = S.dinv[i] * r;
      S.r[i] = r;
      S.z[i] = z;
      p0[i] = 0.0;
      arr += r * r;
      arz += r * z;
      abb += bi * bi;
    }
  }
  const double v[3] = {arr, arz, abb};
  double tot[3];
  if (!reduce_last<3>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    if (mode == 0) {
      st->bb = tot[2];
      st->it = 0;
      st->nchecks = 0;
    } else {
      st->nchecks += 1;
    }
    const double bb = st->bb, rr = tot[0];
    st->rr = rr;
    int ns;
    if (bb == 0.0) ns = KS_ZERO;
    else if (!finite(rr)) ns = KS_NONFINITE;
    else if (rr <= st->tol2 * bb) ns = KS_DONE;
    else if (mode != 0 && st->it >= st->maxit) ns = KS_MAXIT;
    else {
      ns = KS_RUN;
      st->rho = tot[1];
      st->beta = 0.0;
    }
    st->status = ns;
  }
}

template <int G>
__global__ void __launch_bounds__(BLOCK) k_pcg_a(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const int lane = threadIdx.x % G;
  const int grp = lb * (BLOCK / G) + threadIdx.x / G, ngrp = S.nblk * (BLOCK / G);
  const double beta = st->beta;
  const int pc = st->pc;
  const double* po = S.p[pc];
  double* pn = S.p[pc ^ 1];
  const double* z = S.z;
  double acc = 0.0;
  for (int i = grp; i < S.n; i += ngrp) {
    double s = 0.0;
    const int e = S.rowptr[i + 1];
    for (int k = S.rowptr[i] + lane; k < e; k += G) {
      const int j = S.col[k];
      s += S.val[k] * (z[j] + beta * po[j]);
    }
    s = group_sum<G>(s);
    if (lane == 0) {
      const double pi = z[i] + beta * po[i];
      pn[i] = pi;
      S.q[i] = s;
      acc += pi * s;
    }
  }
  const double v[1] = {acc};
  double tot[1];
  if (!reduce_last<1>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    const double pq = tot[0];
    st->pc = pc ^ 1;
    if (!finite(pq)) st->status = KS_NONFINITE;
    else if (!(pq > 0.0)) st->status = KS_BREAKDOWN;
    else st->alpha = st->rho / pq;
  }
}

__global__ void __launch_bounds__(BLOCK) k_pcg_b(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const double alpha = st->alpha;
  const double* p = S.p[st->pc];
  double arz = 0.0, arr = 0.0;
  for (int i = lb * BLOCK + threadIdx.x; i < S.n; i += S.nblk * BLOCK) {
    S.x[i] += alpha * p[i];
    const double r = S.r[i] - alpha * S.q[i];
    const double z = S.dinv[i] * r;
    S.r[i] = r;
    S.z[i] = z;
    arz += r * z;
    arr += r * r;
  }
  const double v[2] = {arz, arr};
  double tot[2];
  if (!reduce_last<2>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    st->it += 1;
    const double rr = tot[1];
    st->rr = rr;
    if (!finite(rr)) st->status = KS_NONFINITE;
    else if (rr <= st->tol2 * st->bb || st->it >= st->maxit) st->status = KS_PENDING;
    else {
      st->beta = tot[0] / st->rho;
      st->rho = tot[0];
    }
  }
}

// ---------------------------------------------------------------- BiCGStab
// mode 0: start; mode 1: confirm KS_PENDING / restart KS_RESTART systems.
// Vectors: z = rhat, p[0] = p, q = v.
template <int G>
__global__ void __launch_bounds__(BLOCK) k_bicg_init(const KSys* sys, const int2* bmap, int mode) {
  SYS_PROLOGUE
  if (mode != 0 && st->status != KS_PENDING && st->status != KS_RESTART) return;
  const int lane = threadIdx.x % G;
  const int grp = lb * (BLOCK / G) + threadIdx.x / G, ngrp = S.nblk * (BLOCK / G);
  double arr = 0.0, abb = 0.0;
  for (int i = grp; i < S.n; i += ngrp) {
    const double ax = row_dot<G>(S, i, lane, S.x);
    if (lane == 0) {
      const double bi = S.b[i], r = bi - ax;
      S.r[i] = r;
      S.z[i] = r;
      S.p[0][i] = 0.0;
      S.q[i] = 0.0;
      arr += r * r;
      abb += bi * bi;
    }
  }
  const double v[2] = {arr, abb};
  double tot[2];
  if (!reduce_last<2>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    if (mode == 0) {
      st->bb = tot[1];
      st->it = 0;
      st->nchecks = 0;
    } else {
      st->nchecks += 1;
    }
    const double bb = st->bb, rr = tot[0];
    st->rr = rr;
    int ns;
    if (bb == 0.0) ns = KS_ZERO;
    else if (!finite(rr)) ns = KS_NONFINITE;
    else if (rr <= st->tol2 * bb) ns = KS_DONE;
    else if (mode != 0 && st->it >= st->maxit) ns = KS_MAXIT;
    else {
      ns = KS_RUN;
      st->rho = rr;   // rhat . r with rhat = r
      st->rho_old = 1.0;
      st->alpha = 1.0;
      st->omega = 1.0;
      st->tt_zero = 0;
    }
    st->status = ns;
  }
}

__global__ void __launch_bounds__(BLOCK) k_bicg_1(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const double omega = st->omega;
  const double beta = (st->rho / st->rho_old) * (st->alpha / omega);
  double* p = S.p[0];
  for (int i = lb * BLOCK + threadIdx.x; i < S.n; i += S.nblk * BLOCK) {
    const double pi = S.r[i] + beta * (p[i] - omega * S.q[i]);
    p[i] = pi;
    S.phat[i] = S.dinv[i] * pi;
  }
}

template <int G>
__global__ void __launch_bounds__(BLOCK) k_bicg_2(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const int lane = threadIdx.x % G;
  const int grp = lb * (BLOCK / G) + threadIdx.x / G, ngrp = S.nblk * (BLOCK / G);
  double acc = 0.0;
  for (int i = grp; i < S.n; i += ngrp) {
    const double s = row_dot<G>(S, i, lane, S.phat);
    if (lane == 0) {
      S.q[i] = s;
      acc += S.z[i] * s;
    }
  }
  const double v[1] = {acc};
  double tot[1];
  if (!reduce_last<1>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    const double alpha = st->rho / tot[0];
    if (!finite(alpha)) st->status = KS_NONFINITE;
    else st->alpha = alpha;
  }
}

__global__ void __launch_bounds__(BLOCK) k_bicg_3(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const double alpha = st->alpha;
  for (int i = lb * BLOCK + threadIdx.x; i < S.n; i += S.nblk * BLOCK) {
    const double s = S.r[i] - alpha * S.q[i];
    S.s[i] = s;
    S.shat[i] = S.dinv[i] * s;
  }
}

template <int G>
__global__ void __launch_bounds__(BLOCK) k_bicg_4(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const int lane = threadIdx.x % G;
  const int grp = lb * (BLOCK / G) + threadIdx.x / G, ngrp = S.nblk * (BLOCK / G);
  double ats = 0.0, att = 0.0;
  for (int i = grp; i < S.n; i += ngrp) {
    const double t = row_dot<G>(S, i, lane, S.shat);
    if (lane == 0) {
      S.t[i] = t;
      ats += t * S.s[i];
      att += t * t;
    }
  }
  const double v[2] = {ats, att};
  double tot[2];
  if (!reduce_last<2>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    if (tot[1] == 0.0) {
      st->omega = 0.0;
      st->tt_zero = 1;
    } else {
      st->omega = tot[0] / tot[1];
    }
  }
}

__global__ void __launch_bounds__(BLOCK) k_bicg_5(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_RUN) return;
  const double alpha = st->alpha, omega = st->omega;
  double arr = 0.0, arh = 0.0;
  for (int i = lb * BLOCK + threadIdx.x; i < S.n; i += S.nblk * BLOCK) {
    S.x[i] += alpha * S.phat[i] + omega * S.shat[i];
    const double r = S.s[i] - omega * S.t[i];
    S.r[i] = r;
    arr += r * r;
    arh += S.z[i] * r;
  }
  const double v[2] = {arr, arh};
  double tot[2];
  if (!reduce_last<2>(v, S.part, S.cnt, S.nblk, lb, tot)) return;
  if (threadIdx.x == 0) {
    st->it += 1;
    const double rr = tot[0];
    st->rr = rr;
    st->rho_old = st->rho;
    st->rho = tot[1];
    if (!finite(rr)) st->status = KS_NONFINITE;
    else if (rr <= st->tol2 * st->bb || st->tt_zero || st->it >= st->maxit)
      st->status = KS_PENDING;
    else if (fabs(omega) < 1e-300 || fabs(tot[1]) < 1e-300)
      st->status = KS_RESTART;
  }
}

// b == 0: x := 0 (the solution), then mark done.
__global__ void __launch_bounds__(BLOCK) k_ksys_zero(const KSys* sys, const int2* bmap) {
  SYS_PROLOGUE
  if (st->status != KS_ZERO) return;
  for (int i = lb * BLOCK + threadIdx.x; i < S.n; i += S.nblk * BLOCK) S.x[i] = 0.0;
}

__global__ void k_gather_states(const KSys* sys, int n, KState* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *sys[i].st;
}

// ---------------------------------------------------------------- launchers
#define LAUNCH_G(KER, G, nb, s, ...)                                                       \
  do {                                                                                     \
    switch (G) {                                                                           \
      case 4: hipLaunchKernelGGL(KER<4>, dim3(nb), dim3(BLOCK), 0, s, __VA_ARGS__); break;   \
      case 8: hipLaunchKernelGGL(KER<8>, dim3(nb), dim3(BLOCK), 0, s, __VA_ARGS__); break;   \
      case 16: hipLaunchKernelGGL(KER<16>, dim3(nb), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
      case 32: hipLaunchKernelGGL(KER<32>, dim3(nb), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
      case 64: hipLaunchKernelGGL(KER<64>, dim3(nb), dim3(BLOCK), 0, s, __VA_ARGS__); break; \
      default: fail(IPCS_E_INVALID, "unsupported lane group");                              \
    }                                                                                      \
    HIP_LAUNCH_OK();                                                                       \
  } while (0)

void pcg_init(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks, int mode) {
  LAUNCH_G(k_pcg_init, G, nblocks, s, sys, bmap, mode);
}

void pcg_iter(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks) {
  LAUNCH_G(k_pcg_a, G, nblocks, s, sys, bmap);
  hipLaunchKernelGGL(k_pcg_b, dim3(nblocks), dim3(BLOCK), 0, s, sys, bmap);
  HIP_LAUNCH_OK();
}

void bicg_init(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks, int mode) {
  LAUNCH_G(k_bicg_init, G, nblocks, s, sys, bmap, mode);
}

void bicg_iter(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks) {
  hipLaunchKernelGGL(k_bicg_1, dim3(nblocks), dim3(BLOCK), 0, s, sys, bmap);
  HIP_LAUNCH_OK();
  LAUNCH_G(k_bicg_2, G, nblocks, s, sys, bmap);
  hipLaunchKernelGGL(k_bicg_3, dim3(nblocks), dim3(BLOCK), 0, s, sys, bmap);
  HIP_LAUNCH_OK();
  LAUNCH_G(k_bicg_4, G, nblocks, s, sys, bmap);
  hipLaunchKernelGGL(k_bicg_5, dim3(nblocks), dim3(BLOCK), 0, s, sys, bmap);
  HIP_LAUNCH_OK();
}

void gather_states(hipStream_t s, const KSys* sys, int n, KState* out) {
  hipLaunchKernelGGL(k_gather_states, dim3((unsigned)div_up(n, 64)), dim3(64), 0, s, sys, n, out);
  HIP_LAUNCH_OK();
}

void ksys_zero(hipStream_t s, const KSys* sys, const int2* bmap, int nblocks) {
  hipLaunchKernelGGL(k_ksys_zero, dim3(nblocks), dim3(BLOCK), 0, s, sys, bmap);
  HIP_LAUNCH_OK();
}

}  // namespace ipcs
