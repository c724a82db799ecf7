// Steady incompressible Navier-Stokes by Newton's method on the monolithic
// Taylor-Hood P2-P1 system (the steady equations of Section 2.1; the Newton
// linearization of Section 2.2.1 without its time-derivative term; the
// workflow of Section 4.2: Newton steps to a relative tolerance).
//
// Each Newton step solves J(u^k) (dU, dP) = R(u^k, p^k) with
//   R_c = F_c - (nu K + C(U)) U_c - G_c P   (velocity rows off the boundary)
//   R_p = -sum_c D_c U_c                     (projected to zero sum)
//   J   = [[nu K + C(U) + N(U), G], [D, 0]], N_ce = (phi_j d_e u_c, phi_i),
// boundary velocity rows and columns eliminated (the iterates carry the
// Dirichlet data, the increments vanish there), by flexible GMRES with the
// block upper-triangular preconditioner [[A, G], [0, -S]]^{-1}: A the
// velocity block of J, applied by a loose inner Jacobi-BiCGStab solve, and
// S = (1/nu) diag(Mp 1) for the pressure Schur complement. The pressure is
// shifted to zero integral mean after every step.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "run.hpp"

namespace ipcs {

// entry kinds of the monolithic Newton matrix (code & 7); bits 3-4: the
// equation's velocity component c, bits 5-6: the unknown's component e
enum : int { MONO_PAD = 0, MONO_UU_DIAG = 1, MONO_UU_OFF = 2, MONO_G = 3, MONO_D = 4 };

// Inputs of the compose kernel: one thread per row of a monolithic SELL-64
// matrix (rows: U_0 .. U_{dim-1} of n2 each, then P); src indexes the entry's
// value in its block's own SELL array.
struct MonoCompose {
  int64_t nrows, n2;
  int dim;
  const int32_t* sptr;
  const int32_t* col;
  const int32_t* src;
  const uint8_t* code;
  const uint8_t* bmask;       // [n2]
  double nu;
  const double* K;            // P2P2 SELL values
  const double* C;            // P2P2 SELL values: C(U)
  const double* N[9];         // P2P2 SELL values: N_ce at [c * dim + e]
  const double* Gc[3];        // P2P1 SELL values
  const double* Dc[3];        // P1P2 SELL values
  double* J;                  // Newton matrix values (null: not formed)
  double* Pic;                // values of the residual's operator (null: not formed)
};

void mono_compose(hipStream_t s, const MonoCompose& m);
void sell_axpby(hipStream_t s, int64_t nrows, const int32_t* sp, const int32_t* col,
                const double* A, const double* x, double alpha, double beta, const double* b,
                double* y);
int mdot_blocks(int64_t n);
// out[j] (+)= V[j] . w for j < k (deterministic; part holds k * mdot_blocks(n))
void mdot(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* w, int k,
          double* part, double* out, int acc);
void maxpy(hipStream_t s, int64_t n, const double* V, int64_t ldv, const double* h, int k,
           double sign, double* y);
void scale_inv_norm(hipStream_t s, int64_t n, const double* x, const double* nrm2, double* y);
void prec_pressure(hipStream_t s, int64_t n1, const double* vp, const double* w, double nu,
                   double* zp);
void sub_scaled(hipStream_t s, int64_t n, const double* scal, double f, double* v);
void fill(hipStream_t s, int64_t n, double v, double* y);
void copy_vec(hipStream_t s, int64_t n, const double* x, double* y);
void sell_inv_diag(hipStream_t s, int64_t n, const int32_t* sp, const int32_t* col,
                   const double* A, double* dinv);

// A monolithic pattern over several blocks: its SELL-64 layout and, per
// entry, the source entry in its block's SELL array and the code above.
struct MonoPattern {
  Sell sell;
  std::vector<int32_t> src;
  std::vector<uint8_t> code;
};
// velocity_only: the preconditioner's velocity block (dim * n2 rows and
// columns); otherwise the Newton matrix over (U, P).
MonoPattern build_mono(const Mesh& m, bool velocity_only);

struct Steady {
  Run run;                    // mesh data, K, D_c, G_c, w, forcing, Dirichlet data, U, P
  ipcs_steady_params sp{};
  int dim = 2;
  int64_t n2 = 0, n1 = 0, nu_rows = 0, n = 0;
  MonoPattern mj, ma;
  // device arrays (in the workspace after the run's own)
  int32_t *j_sp = nullptr, *j_col = nullptr, *j_src = nullptr;
  uint8_t* j_code = nullptr;
  int32_t *a_sp = nullptr, *a_col = nullptr, *a_src = nullptr;
  uint8_t* a_code = nullptr;
  double *Jv = nullptr, *Pv = nullptr, *Av = nullptr, *dinvA = nullptr;
  double *Cv = nullptr, *Nv = nullptr;     // P2P2 values: C(U), N_ce (dim*dim arrays)
  double *x = nullptr, *bvec = nullptr, *R = nullptr, *dx = nullptr, *tmp = nullptr;
  double *V = nullptr, *Z = nullptr;       // FGMRES bases [(m+1)][n], [m][n]
  double *h = nullptr, *part = nullptr, *scal = nullptr;
  double* kva = nullptr;                   // inner BiCGStab vectors [8][nu_rows]
  double *ib = nullptr, *ix = nullptr;     // inner right-hand side and solution
  KState* kst = nullptr;
  KGroup* kgroup = nullptr;
  double *pm = nullptr, *pv0 = nullptr, *pv1 = nullptr, *pfold = nullptr;
  int2 *bm = nullptr, *bv = nullptr;
  KState* poll = nullptr;
  KSet setA;
  KState* pinned = nullptr;
  hipEvent_t ev[2] = {};
  int64_t ws_run = 0;
  // statistics of the last solve
  std::vector<double> history;             // ||dx|| / ||x|| per Newton step
  int lin_it = 0, inner_it = 0;

  ~Steady();
  // sizes, patterns and the workspace this mesh and these parameters need
  int64_t measure(std::shared_ptr<const Mesh> m, const ipcs_steady_params& p);
  void layout(Carver& c);
  void create(std::shared_ptr<const Mesh> m, const ipcs_steady_params& p, void* ws,
              int64_t bytes, hipStream_t s);
  void set_builtin(int kind, const double* prm, int nprm);
  void set_state(const double* u, const double* p);
  // one Newton step; returns ||dx|| / ||x|| (x after the update)
  double newton_step(ipcs_steady_stats* st);
  int solve(ipcs_steady_stats* st);
  void to_run();     // x -> the run's U, P (for read-back)
};

}  // namespace ipcs
