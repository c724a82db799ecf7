// Plain structs passed to the kernels (device pointers only) and the launcher
// declarations implemented in the .hip files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ipcs {

constexpr int BLOCK = 256;        // threads per block of the Krylov/vector kernels
constexpr int KPART = 4;          // partial sums per block per Krylov system

// Krylov system status (device-resident, read by the host every few iterations)
enum KStatus : int32_t {
  KS_RUN = 0,        // iterating
  KS_PENDING = 1,    // recursive residual converged (or maxit): confirm with b - A x
  KS_DONE = 2,       // converged, true residual confirmed
  KS_ZERO = 3,       // b == 0: x := 0
  KS_RESTART = 4,    // BiCGStab breakdown: restart from the current x
  KS_MAXIT = -4,
  KS_BREAKDOWN = -5,
  KS_NONFINITE = -6
};

struct KState {
  double bb, rr;              // ||b||^2, ||r||^2 (recursive, or true after a check)
  double rho, rho_old;        // PCG: r.z; BiCGStab: rhat.r (new) and previous
  double alpha, beta, omega;
  double tol2;                // tol^2
  int32_t status, it, maxit, pc;   // pc: current PCG direction buffer (0/1)
  int32_t tt_zero, nchecks, pad0, pad1;
};

// One linear system A x = b with its Krylov work vectors. A is CSR with
// int32 indices and FP64 values; vectors are FP64.
struct KSys {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const double* dinv;         // Jacobi: 1 / diag(A)
  const double* b;
  double* x;
  double* r;
  double* z;                  // PCG z; BiCGStab rhat
  double* p[2];               // PCG direction (double buffered); BiCGStab p = p[0]
  double* q;                  // PCG A p; BiCGStab v
  double* s;                  // BiCGStab
  double* t;
  double* phat;
  double* shat;
  KState* st;
  double* part;               // [nblk][KPART]
  uint32_t* cnt;              // last-block arrival counter (left at 0)
  int32_t n;
  int32_t nblk;
};

// Row-owner assembly inputs (see mesh.hpp)
struct RowAsm {
  int32_t nrows;
  const int32_t* rowptr;      // CSR pattern of the output matrices
  const int32_t* inc_ptr;
  const int32_t* inc;         // cell << 4 | local row index
  const uint8_t* slot;
  int32_t stride;
  const int32_t* c2d;         // [nc][nloc2]
  int32_t nloc2;
  const double* X;            // vertex coordinates [nv][dim]
  double* out[3];
};

// Manufactured solution on the device
struct Builtin {
  int32_t kind;               // IPCS_SOL_* or 0
  double prm[4];
  double nu;
};

// ------------------------------------------------------------ launchers
// Assembly (kernels_asm.hip). bs = rows per block, lds = dynamic LDS bytes.
void asm_mass_stiff(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds);
void asm_conv_explicit(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds,
                       const double* U, int64_t n2, double inv_dt);
void asm_grad(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds);
void asm_div(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds);
void asm_kp(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds);
void asm_lumped_p1(int dim, hipStream_t s, const RowAsm& a, double* w);
void asm_forcing(int dim, hipStream_t s, const RowAsm& a, const Builtin& bi, const double* fq,
                 int64_t nc, double t, double* F, int64_t n2);
void form_eliminated(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* col,
                     const uint8_t* bmask, const double* M, const double* K, double cm,
                     double ck, double* out, double* dinv);
void inv_diagonal(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* col,
                  const double* val, double* dinv);
void lift_values(hipStream_t s, int64_t nlift, const int32_t* slot, const double* M,
                 const double* K, double cm, double ck, double* out);

// Krylov (kernels_krylov.hip). G = lanes per CSR row.
void pcg_init(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks, int mode);
void pcg_iter(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks);
void bicg_init(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks, int mode);
void bicg_iter(hipStream_t s, int G, const KSys* sys, const int2* bmap, int nblocks);
void ksys_zero(hipStream_t s, const KSys* sys, const int2* bmap, int nblocks);
// out[i] = *sys[i].st for i < n (one contiguous copy the host can fetch at once)
void gather_states(hipStream_t s, const KSys* sys, int n, KState* out);

// Fields and right-hand sides (kernels_fields.hip)
void eval_velocity(hipStream_t s, int dim, const Builtin& bi, const double* x, int64_t n,
                   double t, double* U, int64_t ldu);
void eval_pressure(hipStream_t s, int dim, const Builtin& bi, const double* x, int64_t n,
                   double t, double* P);
void dirichlet_builtin(hipStream_t s, int dim, const Builtin& bi, const double* x2,
                       const int32_t* bidx, int64_t nb, double t, double* gfull, int64_t n2);
void dirichlet_scatter(hipStream_t s, int dim, const double* gb, const int32_t* bidx,
                       int64_t nb, double* gfull, int64_t n2);
void copy_with_bc(hipStream_t s, int dim, const double* U, const uint8_t* bmask,
                  const double* gfull, double* out, int64_t n2);
void rhs_momentum(hipStream_t s, int dim, int G, int64_t n2, const int32_t* rp22,
                  const int32_t* col22, const double* E, const double* U, const int32_t* rp21,
                  const int32_t* col21, double* const* Gc, const double* P, const double* F,
                  const int32_t* lift_ptr, const int32_t* lift_col, const double* liftA,
                  const uint8_t* bmask, const double* gfull, double* b);
void rhs_pressure(hipStream_t s, int dim, int G, int64_t n1, const int32_t* rp12,
                  const int32_t* col12, double* const* Dc, const double* Us, int64_t n2,
                  double scale, double* r, double* part, uint32_t* cnt, double* mean_out);
void sub_scalar(hipStream_t s, int64_t n, const double* scal, double* v);
void rhs_correction(hipStream_t s, int dim, int G, int64_t n2, const int32_t* rp22,
                    const int32_t* col22, const double* M, const double* Us,
                    const int32_t* rp21, const int32_t* col21, double* const* Gc,
                    const double* dP, double scale, const int32_t* lift_ptr,
                    const int32_t* lift_col, const double* liftM, const uint8_t* bmask,
                    const double* gfull, double* b);
void weighted_mean(hipStream_t s, int64_t n, const double* w, const double* v, double* part,
                   uint32_t* cnt, double* out);   // out = (w.v)/(sum w)
void axpy_inplace(hipStream_t s, int64_t n, double a, const double* x, double* y);

}  // namespace ipcs
