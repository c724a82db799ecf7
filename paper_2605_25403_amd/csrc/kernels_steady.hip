// Kernels of the steady Navier-Stokes solver (Newton's method on the
// monolithic P2-P1 system; Section 2.2.1, Newton linearization, with the
// time-derivative term dropped for the steady equations of Section 2.1).
//
// The Newton matrix over x = (U_0, .., U_{d-1}, P) is kept in one SELL-64
// layout ("monolithic"); its values are composed from the blocks the
// row-owner assembly forms on their own patterns (nu K, C(U), N_ce(U), G_c,
// D_c), through a per-entry map (source entry, kind, components). The
// preconditioner's velocity block has a SELL layout of its own. The Krylov
// solver around them (flexible GMRES) uses the generic vector kernels below:
// a SELL product with an axpby, multi-dot products with deterministic
// two-pass reductions, multi-axpys and scalings by device scalars.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"
#include "steady.hpp"

namespace ipcs {

namespace {

constexpr int SBS = 256;                    // threads per block
constexpr int SCHUNK = SBS * 8;             // rows per block of the reductions

__global__ void __launch_bounds__(SBS)
k_compose(MonoCompose m) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m.nrows) return;
  const int64_t nu_rows = (int64_t)m.dim * m.n2;
  const bool vrow = r < nu_rows;
  const bool brow = vrow && m.bmask[r % m.n2];
  const int sl = (int)(r >> 6), w = (m.sptr[sl + 1] - m.sptr[sl]) >> 6;
  const int base = m.sptr[sl] + (int)(r & 63);
  for (int k = 0; k < w; ++k) {
    const int e = base + 64 * k;
    const int32_t src = m.src[e];
    const int code = m.code[e];
    const int kind = code & 7, c = (code >> 3) & 3, d = (code >> 5) & 3;
    const int64_t col = m.col[e];
    double pic = 0.0, nwt = 0.0;
    switch (kind) {
      case MONO_UU_DIAG:
        pic = m.nu * m.K[src] + m.C[src];
        nwt = pic + m.N[c * m.dim + d][src];
        break;
      case MONO_UU_OFF: nwt = m.N[c * m.dim + d][src]; break;
      case MONO_G: pic = nwt = m.Gc[c][src]; break;
      case MONO_D: pic = nwt = m.Dc[d][src]; break;
      default: break;   // padding
    }
    const bool bcol = col < nu_rows && m.bmask[col % m.n2];
    if (brow) {
      // boundary velocity row: the increment is zero there (identity row of
      // the Newton matrix); the residual row is zero
      nwt = (col == r && kind != MONO_PAD) ? 1.0 : 0.0;
      pic = 0.0;
    } else if (bcol) {
      nwt = 0.0;   // boundary columns eliminated; the residual keeps them
    }
    if (m.J) m.J[e] = nwt;
    if (m.Pic) m.Pic[e] = pic;
  }
}

// y = beta b + alpha A x over rows [0, nrows) of a SELL-64 FP64 matrix.
__global__ void __launch_bounds__(SBS)
k_sell_axpby(int64_t nrows, const int32_t* sp, const int32_t* col, const double* A,
             const double* x, double alpha, double beta, const double* b, double* y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int sl = (int)(r >> 6), w = (sp[sl + 1] - sp[sl]) >> 6;
  const int base = sp[sl] + (int)(r & 63);
  double s = 0.0;
  for (int k = 0; k < w; k += 4) {
    double a[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = k + q < w ? k + q : w - 1;
      const int e = base + 64 * kk;
      a[q] = k + q < w ? A[e] : 0.0;
      v[q] = x[col[e]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s += a[q] * v[q];
  }
  y[r] = (beta != 0.0 ? beta * b[r] : 0.0) + alpha * s;
}

// part[j * nblk + blk] = sum over the block's rows of V[j][i] * w[i], j < k
__global__ void __launch_bounds__(SBS)
k_mdot(int64_t n, const double* V, int64_t ldv, const double* w, int k, double* part, int nblk) {
  __shared__ double sh[SBS / 64];
  const int j = blockIdx.y;
  const double* v = V + (int64_t)j * ldv;
  const int64_t i0 = (int64_t)blockIdx.x * SCHUNK;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < min<int64_t>(n, i0 + SCHUNK); i += SBS) s += v[i] * w[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(int64_t)j * nblk + blockIdx.x] = s;
}

// out[j] = sum over blocks of part[j][.] in block order (one block per j);
// acc != 0 adds the result to out[j] instead of storing it
__global__ void __launch_bounds__(SBS)
k_mdot_fin(const double* part, int nblk, double* out, int acc) {
  __shared__ double sh[SBS / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += SBS) s += part[(int64_t)j * nblk + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = acc ? out[j] + s : s;
}

// y[i] += sign * sum_{j<k} h[j] V[j][i]
__global__ void __launch_bounds__(SBS)
k_maxpy(int64_t n, const double* V, int64_t ldv, const double* h, int k, double sign, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s += h[j] * V[(int64_t)j * ldv + i];
  y[i] += sign * s;
}

// y = x / sqrt(*nrm2)
__global__ void __launch_bounds__(SBS)
k_scale_inv_norm(int64_t n, const double* x, const double* nrm2, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = *nrm2;
  y[i] = q > 0.0 ? x[i] / sqrt(q) : 0.0;
}

// pressure part of the block-triangular preconditioner: zp = -nu vp / w
// (the lumped pressure mass scaled by 1/nu stands for the Schur complement)
__global__ void __launch_bounds__(SBS)
k_prec_p(int64_t n1, const double* vp, const double* w, double nu, double* zp) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n1) zp[k] = -nu * vp[k] / w[k];
}

// v -= f * (*scal)
__global__ void __launch_bounds__(SBS)
k_sub_scaled(int64_t n, const double* scal, double f, double* v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] -= f * *scal;
}

__global__ void __launch_bounds__(SBS) k_fill(int64_t n, double v, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

__global__ void __launch_bounds__(SBS) k_copy(int64_t n, const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// Jacobi diagonal of a SELL-64 FP64 matrix (1 where the diagonal is zero)
__global__ void __launch_bounds__(SBS)
k_inv_diag(int64_t n, const int32_t* sp, const int32_t* col, const double* A, double* dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int sl = (int)(r >> 6), w = (sp[sl + 1] - sp[sl]) >> 6;
  const int base = sp[sl] + (int)(r & 63);
  double d = 0.0;
  for (int k = 0; k < w; ++k)
    if (col[base + 64 * k] == r) d += A[base + 64 * k];
  dinv[r] = d != 0.0 ? 1.0 / d : 1.0;
}

inline int grid(int64_t n) { return (int)div_up(n, SBS); }

}  // namespace

void mono_compose(hipStream_t s, const MonoCompose& m) {
  if (m.nrows <= 0) return;
  launch(k_compose, dim3(grid(m.nrows)), dim3(SBS), 0, s, m);
}

void sell_axpby(hipStream_t s, int64_t nrows, const int32_t* sp, const int32_t* col,
                const double* A, const double* x, double alpha, double beta, const double* b,
                double* y) {
  if (nrows <= 0) return;
  launch(k_sell_axpby, dim3(grid(nrows)), dim3(SBS), 0, s, nrows, sp, col, A, x, alpha, beta,
         b, y);
}

int mdot_blocks(int64_t n) { return (int)std::max<int64_t>(1, div_up(n, SCHUNK)); }

void mdot(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* w, int k,
          double* part, double* out, int acc) {
  if (k <= 0) return;
  const int nb = mdot_blocks(n);
  launch(k_mdot, dim3(nb, k), dim3(SBS), 0, s, n, V, ldv, w, k, part, nb);
  launch(k_mdot_fin, dim3(k), dim3(SBS), 0, s, (const double*)part, nb, out, acc);
}

void maxpy(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* h, int k,
           double sign, double* y) {
  if (k <= 0 || n <= 0) return;
  launch(k_maxpy, dim3(grid(n)), dim3(SBS), 0, s, n, V, ldv, h, k, sign, y);
}

void scale_inv_norm(hipStream_t s, int64_t n, const double* x, const double* nrm2, double* y) {
  launch(k_scale_inv_norm, dim3(grid(n)), dim3(SBS), 0, s, n, x, nrm2, y);
}

void prec_pressure(hipStream_t s, int64_t n1, const double* vp, const double* w, double nu,
                   double* zp) {
  launch(k_prec_p, dim3(grid(n1)), dim3(SBS), 0, s, n1, vp, w, nu, zp);
}

void sub_scaled(hipStream_t s, int64_t n, const double* scal, double f, double* v) {
  if (n > 0) launch(k_sub_scaled, dim3(grid(n)), dim3(SBS), 0, s, n, scal, f, v);
}

void fill(hipStream_t s, int64_t n, double v, double* y) {
  if (n > 0) launch(k_fill, dim3(grid(n)), dim3(SBS), 0, s, n, v, y);
}

void copy_vec(hipStream_t s, int64_t n, const double* x, double* y) {
  if (n > 0) launch(k_copy, dim3(grid(n)), dim3(SBS), 0, s, n, x, y);
}

void sell_inv_diag(hipStream_t s, int64_t n, const int32_t* sp, const int32_t* col,
                   const double* A, double* dinv) {
  if (n > 0) launch(k_inv_diag, dim3(grid(n)), dim3(SBS), 0, s, n, sp, col, A, dinv);
}

}  // namespace ipcs
