// Right-hand sides of the three IPCS sub-steps (Section 2.2.1, eq. (9)),
// Dirichlet data, closed-form fields and small vector kernels for gfx950.
//
// Momentum  : b_c = (M/dt - C(U^n)) U^n_c - G_c P^n + F_c(t)        (interior rows)
// Pressure  : r   = -(rho/dt) sum_c D_c U*_c, then r -= mean(r)
// Correction: b_c = M U*_c - (dt/rho) G_c dP                          (interior rows)
// Interior rows next to the boundary subtract A_IB g (symmetric elimination);
// boundary rows carry g itself.
#include <hip/hip_runtime.h>

#include "builtin.hpp"
#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"

namespace ipcs {

static int grid_for(int64_t rows, int rows_per_block) {
  return (int)std::min<int64_t>(div_up(rows, rows_per_block), 8192);
}

// ---------------------------------------------------------------- fields
template <int D>
__global__ void k_eval_velocity(Builtin bi, const double* x, int64_t n, double t, double* U,
                                int64_t ldu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xi[D], u[D];
#pragma unroll
  for (int r = 0; r < D; ++r) xi[r] = x[i * D + r];
  builtin_velocity<D>(bi, xi, t, u);
#pragma unroll
  for (int c = 0; c < D; ++c) U[c * ldu + i] = u[c];
}

void eval_velocity(hipStream_t s, int dim, const Builtin& bi, const double* x, int64_t n,
                   double t, double* U, int64_t ldu) {
  const unsigned nb = (unsigned)div_up(n, 256);
  if (dim == 2) hipLaunchKernelGGL(k_eval_velocity<2>, dim3(nb), dim3(256), 0, s, bi, x, n, t, U, ldu);
  else hipLaunchKernelGGL(k_eval_velocity<3>, dim3(nb), dim3(256), 0, s, bi, x, n, t, U, ldu);
  HIP_LAUNCH_OK();
}

template <int D>
__global__ void k_eval_pressure(Builtin bi, const double* x, int64_t n, double t, double* P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xi[D];
#pragma unroll
  for (int r = 0; r < D; ++r) xi[r] = x[i * D + r];
  P[i] = builtin_pressure<D>(bi, xi, t);
}

void eval_pressure(hipStream_t s, int dim, const Builtin& bi, const double* x, int64_t n,
                   double t, double* P) {
  const unsigned nb = (unsigned)div_up(n, 256);
  if (dim == 2) hipLaunchKernelGGL(k_eval_pressure<2>, dim3(nb), dim3(256), 0, s, bi, x, n, t, P);
  else hipLaunchKernelGGL(k_eval_pressure<3>, dim3(nb), dim3(256), 0, s, bi, x, n, t, P);
  HIP_LAUNCH_OK();
}

template <int D>
__global__ void k_dirichlet_builtin(Builtin bi, const double* x2, const int32_t* bidx, int64_t nb,
                                    double t, double* g, int64_t n2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  const int64_t i = bidx[k];
  double xi[D], u[D];
#pragma unroll
  for (int r = 0; r < D; ++r) xi[r] = x2[i * D + r];
  builtin_velocity<D>(bi, xi, t, u);
#pragma unroll
  for (int c = 0; c < D; ++c) g[c * n2 + i] = u[c];
}

void dirichlet_builtin(hipStream_t s, int dim, const Builtin& bi, const double* x2,
                       const int32_t* bidx, int64_t nb, double t, double* gfull, int64_t n2) {
  if (nb <= 0) return;
  const unsigned g = (unsigned)div_up(nb, 256);
  if (dim == 2)
    hipLaunchKernelGGL(k_dirichlet_builtin<2>, dim3(g), dim3(256), 0, s, bi, x2, bidx, nb, t, gfull, n2);
  else
    hipLaunchKernelGGL(k_dirichlet_builtin<3>, dim3(g), dim3(256), 0, s, bi, x2, bidx, nb, t, gfull, n2);
  HIP_LAUNCH_OK();
}

__global__ void k_dirichlet_scatter(int dim, const double* gb, const int32_t* bidx, int64_t nb,
                                    double* g, int64_t n2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  for (int c = 0; c < dim; ++c) g[c * n2 + bidx[k]] = gb[k * dim + c];
}

void dirichlet_scatter(hipStream_t s, int dim, const double* gb, const int32_t* bidx, int64_t nb,
                       double* gfull, int64_t n2) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_dirichlet_scatter, dim3((unsigned)div_up(nb, 256)), dim3(256), 0, s, dim,
                     gb, bidx, nb, gfull, n2);
  HIP_LAUNCH_OK();
}

__global__ void k_copy_bc(int dim, const double* U, const uint8_t* bmask, const double* g,
                          double* out, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const bool b = bmask[i];
  for (int c = 0; c < dim; ++c) out[c * n2 + i] = b ? g[c * n2 + i] : U[c * n2 + i];
}

void copy_with_bc(hipStream_t s, int dim, const double* U, const uint8_t* bmask,
                  const double* gfull, double* out, int64_t n2) {
  hipLaunchKernelGGL(k_copy_bc, dim3((unsigned)div_up(n2, 256)), dim3(256), 0, s, dim, U, bmask,
                     gfull, out, n2);
  HIP_LAUNCH_OK();
}

// ---------------------------------------------------------------- right-hand sides
struct Ptrs3 {
  const double* p[3];
};

// b_c[i] = sum_j A[ij] X_c[j] - sc * sum_k Gc[ik] Y[k] + F_c[i] - sum lift[i] g_c
// on interior rows; g_c[i] on boundary rows. One lane group per row.
template <int D, int G>
__global__ void __launch_bounds__(256) k_rhs_p2(int64_t n2, const int32_t* rp22,
                                                const int32_t* col22, const double* A,
                                                const double* X, const int32_t* rp21,
                                                const int32_t* col21, Ptrs3 Gc, const double* Y,
                                                double sc, const double* F,
                                                const int32_t* lift_ptr, const int32_t* lift_col,
                                                const double* lift, const uint8_t* bmask,
                                                const double* g, double* b) {
  const int lane = threadIdx.x % G;
  const int64_t grp0 = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int64_t ngrp = (int64_t)gridDim.x * (256 / G);
  for (int64_t i = grp0; i < n2; i += ngrp) {
    if (bmask[i]) {
      if (lane == 0)
#pragma unroll
        for (int c = 0; c < D; ++c) b[c * n2 + i] = g[c * n2 + i];
      continue;
    }
    double s[D];
#pragma unroll
    for (int c = 0; c < D; ++c) s[c] = 0.0;
    for (int k = rp22[i] + lane; k < rp22[i + 1]; k += G) {
      const double a = A[k];
      const int j = col22[k];
#pragma unroll
      for (int c = 0; c < D; ++c) s[c] += a * X[c * n2 + j];
    }
    for (int k = rp21[i] + lane; k < rp21[i + 1]; k += G) {
      const double y = Y[col21[k]];
#pragma unroll
      for (int c = 0; c < D; ++c) s[c] -= sc * (Gc.p[c][k] * y);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) s[c] = group_sum<G>(s[c]);
    if (lane == 0) {
      for (int e = lift_ptr[i]; e < lift_ptr[i + 1]; ++e) {
        const double l = lift[e];
        const int j = lift_col[e];
#pragma unroll
        for (int c = 0; c < D; ++c) s[c] -= l * g[c * n2 + j];
      }
#pragma unroll
      for (int c = 0; c < D; ++c) b[c * n2 + i] = s[c] + (F ? F[c * n2 + i] : 0.0);
    }
  }
}

template <int D>
static void launch_rhs_p2(hipStream_t s, int G, int64_t n2, const int32_t* rp22,
                          const int32_t* col22, const double* A, const double* X,
                          const int32_t* rp21, const int32_t* col21, Ptrs3 Gc, const double* Y,
                          double sc, const double* F, const int32_t* lp, const int32_t* lc,
                          const double* lv, const uint8_t* bm, const double* g, double* b) {
  const int nb = grid_for(n2, 256 / G);
#define RHS_CASE(GG)                                                                            \
  case GG:                                                                                      \
    hipLaunchKernelGGL((k_rhs_p2<D, GG>), dim3(nb), dim3(256), 0, s, n2, rp22, col22, A, X, rp21, \
                       col21, Gc, Y, sc, F, lp, lc, lv, bm, g, b);                              \
    break;
  switch (G) {
    RHS_CASE(4)
    RHS_CASE(8)
    RHS_CASE(16)
    RHS_CASE(32)
    RHS_CASE(64)
    default: fail(IPCS_E_INVALID, "unsupported lane group");
  }
#undef RHS_CASE
  HIP_LAUNCH_OK();
}

void rhs_momentum(hipStream_t s, int dim, int G, int64_t n2, const int32_t* rp22,
                  const int32_t* col22, const double* E, const double* U, const int32_t* rp21,
                  const int32_t* col21, double* const* Gc, const double* P, const double* F,
                  const int32_t* lift_ptr, const int32_t* lift_col, const double* liftA,
                  const uint8_t* bmask, const double* gfull, double* b) {
  Ptrs3 gp{{Gc[0], Gc[1], dim == 3 ? Gc[2] : nullptr}};
  if (dim == 2)
    launch_rhs_p2<2>(s, G, n2, rp22, col22, E, U, rp21, col21, gp, P, 1.0, F, lift_ptr, lift_col,
                     liftA, bmask, gfull, b);
  else
    launch_rhs_p2<3>(s, G, n2, rp22, col22, E, U, rp21, col21, gp, P, 1.0, F, lift_ptr, lift_col,
                     liftA, bmask, gfull, b);
}

void rhs_correction(hipStream_t s, int dim, int G, int64_t n2, const int32_t* rp22,
                    const int32_t* col22, const double* M, const double* Us,
                    const int32_t* rp21, const int32_t* col21, double* const* Gc,
                    const double* dP, double scale, const int32_t* lift_ptr,
                    const int32_t* lift_col, const double* liftM, const uint8_t* bmask,
                    const double* gfull, double* b) {
  Ptrs3 gp{{Gc[0], Gc[1], dim == 3 ? Gc[2] : nullptr}};
  if (dim == 2)
    launch_rhs_p2<2>(s, G, n2, rp22, col22, M, Us, rp21, col21, gp, dP, scale, nullptr, lift_ptr,
                     lift_col, liftM, bmask, gfull, b);
  else
    launch_rhs_p2<3>(s, G, n2, rp22, col22, M, Us, rp21, col21, gp, dP, scale, nullptr, lift_ptr,
                     lift_col, liftM, bmask, gfull, b);
}

// r[k] = scale * sum_c sum_j D_c[kj] Us_c[j]; mean_out = sum(r)/n1 (deterministic)
template <int D, int G>
__global__ void __launch_bounds__(256) k_rhs_pressure(int64_t n1, const int32_t* rp,
                                                      const int32_t* col, Ptrs3 Dc,
                                                      const double* Us, int64_t n2, double scale,
                                                      double* r, double* part, uint32_t* cnt,
                                                      double* mean_out) {
  const int lane = threadIdx.x % G;
  const int64_t grp0 = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const int64_t ngrp = (int64_t)gridDim.x * (256 / G);
  double acc = 0.0;
  for (int64_t k = grp0; k < n1; k += ngrp) {
    double s = 0.0;
    for (int e = rp[k] + lane; e < rp[k + 1]; e += G) {
      const int j = col[e];
#pragma unroll
      for (int c = 0; c < D; ++c) s += Dc.p[c][e] * Us[c * n2 + j];
    }
    s = group_sum<G>(s);
    if (lane == 0) {
      const double v = scale * s;
      r[k] = v;
      acc += v;
    }
  }
  const double v[1] = {acc};
  double tot[1];
  if (reduce_last<1>(v, part, cnt, gridDim.x, blockIdx.x, tot) && threadIdx.x == 0)
    *mean_out = tot[0] / (double)n1;
}

void rhs_pressure(hipStream_t s, int dim, int G, int64_t n1, const int32_t* rp12,
                  const int32_t* col12, double* const* Dc, const double* Us, int64_t n2,
                  double scale, double* r, double* part, uint32_t* cnt, double* mean_out) {
  Ptrs3 dp{{Dc[0], Dc[1], dim == 3 ? Dc[2] : nullptr}};
  const int nb = (int)std::min<int64_t>(div_up(n1, 256 / G), 1024);
#define RP_CASE(DD, GG)                                                                      \
  hipLaunchKernelGGL((k_rhs_pressure<DD, GG>), dim3(nb), dim3(256), 0, s, n1, rp12, col12, dp, \
                     Us, n2, scale, r, part, cnt, mean_out)
  if (dim == 2) {
    switch (G) {
      case 8: RP_CASE(2, 8); break;
      case 16: RP_CASE(2, 16); break;
      case 32: RP_CASE(2, 32); break;
      default: RP_CASE(2, 64); break;
    }
  } else {
    switch (G) {
      case 8: RP_CASE(3, 8); break;
      case 16: RP_CASE(3, 16); break;
      case 32: RP_CASE(3, 32); break;
      default: RP_CASE(3, 64); break;
    }
  }
#undef RP_CASE
  HIP_LAUNCH_OK();
}

__global__ void k_sub_scalar(int64_t n, const double* scal, double* v) {
  const double a = *scal;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] -= a;
}

void sub_scalar(hipStream_t s, int64_t n, const double* scal, double* v) {
  hipLaunchKernelGGL(k_sub_scalar, dim3(grid_for(n, 256)), dim3(256), 0, s, n, scal, v);
  HIP_LAUNCH_OK();
}

// out = (w . v) / (sum w), deterministic
__global__ void __launch_bounds__(256) k_weighted_mean(int64_t n, const double* w,
                                                       const double* v, double* part,
                                                       uint32_t* cnt, double* out) {
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    a += w[i] * v[i];
    b += w[i];
  }
  const double x[2] = {a, b};
  double tot[2];
  if (reduce_last<2>(x, part, cnt, gridDim.x, blockIdx.x, tot) && threadIdx.x == 0)
    *out = tot[0] / tot[1];
}

void weighted_mean(hipStream_t s, int64_t n, const double* w, const double* v, double* part,
                   uint32_t* cnt, double* out) {
  const int nb = (int)std::min<int64_t>(div_up(n, 256), 1024);
  hipLaunchKernelGGL(k_weighted_mean, dim3(nb), dim3(256), 0, s, n, w, v, part, cnt, out);
  HIP_LAUNCH_OK();
}

__global__ void k_axpy(int64_t n, double a, const double* x, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

void axpy_inplace(hipStream_t s, int64_t n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, s, n, a, x, y);
  HIP_LAUNCH_OK();
}

}  // namespace ipcs
