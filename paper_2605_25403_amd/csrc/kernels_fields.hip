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

// out = the polynomial extrapolation to the next time level of the last NH
// values at equal steps (NH = 2: 2 h0 - h1; NH = 3: 3 h0 - 3 h1 + h2; h0 the
// newest) on interior rows, the Dirichlet data on boundary rows.
template <int NH>
__global__ void k_extrap_bc(int dim, const double* h0, const double* h1, const double* h2,
                            const uint8_t* bmask, const double* g, double* out, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  const bool b = bmask[i];
  for (int c = 0; c < dim; ++c) {
    const int64_t k = c * n2 + i;
    double v;
    if constexpr (NH == 2) v = 2.0 * h0[k] - h1[k];
    else v = 3.0 * (h0[k] - h1[k]) + h2[k];
    out[k] = b ? g[k] : v;
  }
}

void extrapolate_with_bc(hipStream_t s, int dim, int nh, const double* h0, const double* h1,
                         const double* h2, const uint8_t* bmask, const double* gfull,
                         double* out, int64_t n2) {
  const dim3 grid((unsigned)div_up(n2, 256));
  if (nh == 2)
    hipLaunchKernelGGL(k_extrap_bc<2>, grid, dim3(256), 0, s, dim, h0, h1, h2, bmask, gfull, out,
                       n2);
  else if (nh == 3)
    hipLaunchKernelGGL(k_extrap_bc<3>, grid, dim3(256), 0, s, dim, h0, h1, h2, bmask, gfull, out,
                       n2);
  else
    fail(IPCS_E_INVALID, "extrapolation takes 2 or 3 values");
  HIP_LAUNCH_OK();
}

// ---------------------------------------------------------------- right-hand sides
// Matrices are FP64, or FP32 in the mixed form (VT); vectors and sums are FP64.
template <class VT>
struct Ptrs3 {
  const VT* p[3];
};

// b_c[i] = sum_j A[ij] X_c[j] - sc * sum_k Gc[ik] Y[k] + F_c[i] - sum lift[i] g_c
// on interior rows; g_c[i] on boundary rows. One thread per row, both matrices
// in SELL-64 layout (coalesced value and column loads across the wavefront).
// Entries are taken eight at a time: their values and columns are loaded,
// then all their gathers, before any is added (the last chunk re-reads entry
// w-1 and adds zero for it), so that a lane keeps 8 D gathers in flight; the
// additions keep the entry order. Rows past n2 compute row 0 and discard it.
template <int D, class VT>
__global__ void __launch_bounds__(256) k_rhs_p2(int64_t n2, const int32_t* sp22,
                                                const int32_t* col22, const VT* A,
                                                const double* X, double sa,
                                                const int32_t* sp21,
                                                const int32_t* col21, Ptrs3<VT> Gc,
                                                const double* Y, double sc, const double* F,
                                                const int32_t* lift_ptr, const int32_t* lift_col,
                                                const double* lift, const uint8_t* bmask,
                                                const double* g, double* b) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i0 < n2;
  const int64_t i = live ? i0 : 0;
  const gptr<const double> Xg = G(X), Yg = G(Y), gg = G(g);
  double s[D];
#pragma unroll
  for (int c = 0; c < D; ++c) s[c] = 0.0;
  {
    const gptr<const VT> Ag = G(A);
    const gptr<const int32_t> cg = G(col22);
    const int sl = (int)(i >> 6), b0 = G(sp22)[sl], w = (G(sp22)[sl + 1] - b0) >> 6;
    const int base = b0 + (int)(i & 63);
    for (int k = 0; k < w; k += 8) {
      int jj[8];
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
        jj[q] = cg[base + 64 * kk];
        a[q] = (double)Ag[base + 64 * kk];
      }
      double xv[D][8];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int q = 0; q < 8; ++q) xv[c][q] = Xg[c * n2 + jj[q]];
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int c = 0; c < D; ++c) s[c] += k + q < w ? a[q] * xv[c][q] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) s[c] *= sa;
  }
  {
    const gptr<const int32_t> cg = G(col21);
    const int sl = (int)(i >> 6), b0 = G(sp21)[sl], w = (G(sp21)[sl + 1] - b0) >> 6;
    const int base = b0 + (int)(i & 63);
    for (int k = 0; k < w; k += 8) {
      double y[8], gv[D][8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kk = k + q < w ? k + q : w - 1;
#pragma unroll
        for (int c = 0; c < D; ++c) gv[c][q] = (double)G(Gc.p[c])[base + 64 * kk];
        y[q] = Yg[cg[base + 64 * kk]];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int c = 0; c < D; ++c) s[c] -= k + q < w ? sc * (gv[c][q] * y[q]) : 0.0;
    }
  }
  for (int e = G(lift_ptr)[i]; e < G(lift_ptr)[i + 1]; ++e) {
    const double l = G(lift)[e];
    const int j = G(lift_col)[e];
#pragma unroll
    for (int c = 0; c < D; ++c) s[c] -= l * gg[c * n2 + j];
  }
  if (!live) return;
  const gptr<double> bg = G(b);
  if (G(bmask)[i]) {
#pragma unroll
    for (int c = 0; c < D; ++c) bg[c * n2 + i] = gg[c * n2 + i];
    return;
  }
#pragma unroll
  for (int c = 0; c < D; ++c) bg[c * n2 + i] = s[c] + (F ? G(F)[c * n2 + i] : 0.0);
}

template <class VT>
static void rhs_p2_launch(hipStream_t s, int dim, int64_t n2, const int32_t* sp22,
                          const int32_t* col22, const void* A, const double* X, double sa,
                          const int32_t* sp21, const int32_t* col21, void* const* Gc,
                          const double* Y, double sc, const double* F, const int32_t* lift_ptr,
                          const int32_t* lift_col, const double* lift, const uint8_t* bmask,
                          const double* g, double* b) {
  Ptrs3<VT> gp{{(const VT*)Gc[0], (const VT*)Gc[1], dim == 3 ? (const VT*)Gc[2] : nullptr}};
  const unsigned nb = (unsigned)div_up(n2, 256);
  if (dim == 2)
    hipLaunchKernelGGL((k_rhs_p2<2, VT>), dim3(nb), dim3(256), 0, s, n2, sp22, col22,
                       (const VT*)A, X, sa, sp21, col21, gp, Y, sc, F, lift_ptr, lift_col, lift,
                       bmask, g, b);
  else
    hipLaunchKernelGGL((k_rhs_p2<3, VT>), dim3(nb), dim3(256), 0, s, n2, sp22, col22,
                       (const VT*)A, X, sa, sp21, col21, gp, Y, sc, F, lift_ptr, lift_col, lift,
                       bmask, g, b);
  HIP_LAUNCH_OK();
}

void rhs_momentum(hipStream_t s, int dim, bool fp32, int64_t n2, const int32_t* sp22,
                  const int32_t* col22, const void* E, double sa, double sg, const double* U,
                  const int32_t* sp21,
                  const int32_t* col21, void* const* Gc, const double* P, const double* F,
                  const int32_t* lift_ptr, const int32_t* lift_col, const double* liftA,
                  const uint8_t* bmask, const double* gfull, double* b) {
  if (fp32)
    rhs_p2_launch<float>(s, dim, n2, sp22, col22, E, U, sa, sp21, col21, Gc, P, sg, F,
                         lift_ptr, lift_col, liftA, bmask, gfull, b);
  else
    rhs_p2_launch<double>(s, dim, n2, sp22, col22, E, U, sa, sp21, col21, Gc, P, sg, F,
                          lift_ptr, lift_col, liftA, bmask, gfull, b);
}

void rhs_correction(hipStream_t s, int dim, bool fp32, int64_t n2, const int32_t* sp22,
                    const int32_t* col22, const void* M, const double* Us,
                    const int32_t* sp21, const int32_t* col21, void* const* Gc,
                    const double* dP, double scale, const int32_t* lift_ptr,
                    const int32_t* lift_col, const double* liftM, const uint8_t* bmask,
                    const double* gfull, double* b) {
  if (fp32)
    rhs_p2_launch<float>(s, dim, n2, sp22, col22, M, Us, 1.0, sp21, col21, Gc, dP, scale,
                         nullptr, lift_ptr, lift_col, liftM, bmask, gfull, b);
  else
    rhs_p2_launch<double>(s, dim, n2, sp22, col22, M, Us, 1.0, sp21, col21, Gc, dP, scale,
                          nullptr, lift_ptr, lift_col, liftM, bmask, gfull, b);
}

// r[k] = scale * sum_c sum_j D_c[kj] Us_c[j] (SELL-64, one thread per row) and
// per-block partial sums of r; k_sub_mean finishes the mean and subtracts it.
// Also the rounding level of each r_k: mag_k = |scale| sum |D_c[kj]| |Us_c[j]|,
// with per-block partial sums of r (part) and of mag^2 (part + 8192).
template <int D, class VT>
__global__ void __launch_bounds__(256) k_rhs_pressure(int64_t n1, const int32_t* sp,
                                                      const int32_t* col, Ptrs3<VT> Dc,
                                                      const double* Us, int64_t n2, double scale,
                                                      double* r, double* part) {
  __shared__ double sh[16];
  const int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k0 < n1;
  const int64_t k = live ? k0 : 0;
  double v = 0.0, mag = 0.0;
  {
    // eight entries at a time, loads before additions, entry order kept (as in k_rhs_p2)
    const gptr<const int32_t> cg = G(col);
    const gptr<const double> ug = G(Us);
    const int sl = (int)(k >> 6), b0 = G(sp)[sl], w = (G(sp)[sl + 1] - b0) >> 6;
    const int base = b0 + (int)(k & 63);
    double s = 0.0, a = 0.0;
    for (int e = 0; e < w; e += 8) {
      double dv[D][8], uv[D][8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int ee = e + q < w ? e + q : w - 1;
        const int j = cg[base + 64 * ee];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          dv[c][q] = (double)G(Dc.p[c])[base + 64 * ee];
          uv[c][q] = ug[c * n2 + j];
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double t = e + q < w ? dv[c][q] * uv[c][q] : 0.0;
          s += t;
          a += fabs(t);
        }
    }
    if (live) {
      v = scale * s;
      mag = fabs(scale) * a;
      G(r)[k] = v;
    }
  }
  const double t = block_sum(v, sh);
  const double q = block_sum(mag * mag, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t;
    part[8192 + blockIdx.x] = q;
  }
}

// floor = (64 eps)^2 * (sum of nb partials of mag^2), written to two places
__global__ void __launch_bounds__(256) k_noise_floor(int nb, const double* part, double* out0,
                                                     double* out1) {
  __shared__ double sh[16];
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) a += part[b];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) {
    const double c = 64.0 * 2.220446049250313e-16;
    if (out0) *out0 = c * c * a;
    if (out1) *out1 = c * c * a;
  }
}

// res = b - A x for an FP64 matrix A (SELL-64), with per-block partial sums of
// res (part_s) and res^2 (part_q)
__global__ void __launch_bounds__(256) k_resid(int64_t n, const int32_t* sp, const int32_t* col,
                                               const double* A, const double* x,
                                               const double* b, double* res, double* part_s,
                                               double* part_q) {
  __shared__ double sh[16];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const int sl = (int)(i >> 6), b0 = sp[sl], w = (sp[sl + 1] - b0) >> 6;
    const int base = b0 + (int)(i & 63);
    double s = 0.0;
    for (int e = 0; e < w; ++e) s += A[base + 64 * e] * x[col[base + 64 * e]];
    v = b[i] - s;
    res[i] = v;
  }
  const double t = block_sum(v, sh);
  const double q = block_sum(v * v, sh);
  if (threadIdx.x == 0) {
    part_s[blockIdx.x] = t;
    part_q[blockIdx.x] = q;
  }
}

// out[0] = sum of part_s, out[1] = sum of part_q (one block, fixed order)
__global__ void __launch_bounds__(256) k_total2(int nb, const double* part_s,
                                                const double* part_q, double* out) {
  __shared__ double sh[16];
  double a = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    a += part_s[b];
    c += part_q[b];
  }
  a = block_sum(a, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = c;
  }
}

// v -= (sum of nb partials) / n, every block reducing the partials itself
__global__ void __launch_bounds__(256) k_sub_mean(int64_t n, int nb, const double* part,
                                                  double* v, double* mean_out) {
  __shared__ double sh[16];
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) a += part[b];
  const double mean = block_sum(a, sh) / (double)n;
  if (blockIdx.x == 0 && threadIdx.x == 0) *mean_out = mean;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] -= mean;
}

void rhs_pressure(hipStream_t s, int dim, bool fp32, int64_t n1, const int32_t* sp12,
                  const int32_t* col12, void* const* Dc, const double* Us, int64_t n2,
                  double scale, double* r, double* part, double* mean_out, double* floor_out0,
                  double* floor_out1) {
  const int nb = (int)div_up(n1, 256);
  if (nb > 8192) fail(IPCS_E_INVALID, "pressure space too large for the partial buffer");
  auto go = [&](auto vt) {
    using VT = decltype(vt);
    Ptrs3<VT> dp{{(const VT*)Dc[0], (const VT*)Dc[1], dim == 3 ? (const VT*)Dc[2] : nullptr}};
    if (dim == 2)
      hipLaunchKernelGGL((k_rhs_pressure<2, VT>), dim3(nb), dim3(256), 0, s, n1, sp12, col12, dp,
                         Us, n2, scale, r, part);
    else
      hipLaunchKernelGGL((k_rhs_pressure<3, VT>), dim3(nb), dim3(256), 0, s, n1, sp12, col12, dp,
                         Us, n2, scale, r, part);
  };
  if (fp32) go(0.0f);
  else go(0.0);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(n1, 256)), dim3(256), 0, s, n1, nb, part, r,
                     mean_out);
  HIP_LAUNCH_OK();
  if (floor_out0 || floor_out1) {
    hipLaunchKernelGGL(k_noise_floor, dim3(1), dim3(256), 0, s, nb, part + 8192, floor_out0,
                       floor_out1);
    HIP_LAUNCH_OK();
  }
}

void residual_projected(hipStream_t s, int64_t n, const int32_t* sp, const int32_t* col,
                        const double* A, const double* x, const double* b, double* res,
                        double* part_s, double* part_q, double* totals, double* mean_out) {
  const int nb = (int)div_up(n, 256);
  if (nb > 8192) fail(IPCS_E_INVALID, "pressure space too large for the partial buffer");
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(256), 0, s, n, sp, col, A, x, b, res, part_s,
                     part_q);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_total2, dim3(1), dim3(256), 0, s, nb, part_s, part_q, totals);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(n, 256)), dim3(256), 0, s, n, nb, part_s, res,
                     mean_out);
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

// (w . v) / (sum w): per-block partials, then every block of the consumer
// re-reduces them; the consumer subtracts the mean from v.
__global__ void __launch_bounds__(256) k_wdot_part(int64_t n, const double* w, const double* v,
                                                   double* part) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    a += w[i] * v[i];
    b += w[i];
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

__global__ void __launch_bounds__(256) k_sub_wmean(int64_t n, int nb, const double* part,
                                                   double* v, double* out) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  const double mean = block_sum(a, sh) / block_sum(b, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = mean;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] -= mean;
}

void sub_weighted_mean(hipStream_t s, int64_t n, const double* w, double* v, double* part,
                       double* out) {
  const int nb = (int)std::min<int64_t>(div_up(n, 256), 1024);
  hipLaunchKernelGGL(k_wdot_part, dim3(nb), dim3(256), 0, s, n, w, v, part);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(k_sub_wmean, dim3(grid_for(n, 256)), dim3(256), 0, s, n, nb, part, v, out);
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
