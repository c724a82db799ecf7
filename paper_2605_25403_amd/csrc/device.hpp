// Plain structs passed to the kernels (device pointers only) and the launcher
// declarations implemented in the .hip files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ipcs {

constexpr int BLOCK = 256;        // threads per block of small utility kernels
constexpr int KBS = 256;          // threads per block of every Krylov kernel
// vector entries per thread of Krylov vector kernels, by systems per group
// (more systems hold more vectors in registers per entry)
constexpr int kept_v(int ns) { return ns == 3 ? 2 : 4; }
constexpr int KPART_Q = 32;       // partial records per thread a consumer block loads
constexpr int KNB_MAX = KBS * KPART_Q;   // most producer blocks per group and kernel
constexpr int KP = 8;             // partial sums per system per block
constexpr int GMAX = 3;           // systems per group (velocity components)

// Krylov system status (device-resident, polled by the host every few iterations)
enum KStatus : int32_t {
  KS_RUN = 0,        // iterating
  KS_PENDING = 1,    // recursive residual converged: confirm with b - A x
  KS_DONE = 2,       // converged, true residual confirmed
  KS_ZERO = 3,       // b == 0: x := 0
  KS_RESTART = 4,    // BiCGStab breakdown: restart from the current x
  KS_MAXIT = -4,
  KS_BREAKDOWN = -5,
  KS_NONFINITE = -6,
  KS_STALL = -7      // restarts stopped lowering the true residual: tol out of reach
};
// Restarts in a row whose true residual is not 10% below the best one so far
// after which a solve stops as out of reach (KS_STALL).
constexpr int KSTALL_CHECKS = 3;

// Scalars of one Krylov system. Iteration scalars are double-buffered by the
// launch parity par the host passes: a kernel of parity par reads slot par^1
// (PCG) or par (BiCGStab) and block 0 writes the other slot, so no block reads
// a slot that another block of the same kernel writes. status is the one field
// a kernel may both read and write: block 0 only ever writes a status that
// every block derives from the same reduced values, so either value sends a
// block down the same branch.
struct KState {
  double bb, rr;              // ||b||^2, last ||r||^2
  double sc[2];               // PCG gamma = r.u, BiCGStab rho = rhat.r, by parity
  double alpha[2];            // PCG alpha by parity; BiCGStab alpha in [0]
  double omega;               // BiCGStab
  double tol2;                // tol^2
  double zero2;               // ||b||^2 at or below this is treated as b = 0 (0: none)
  double rr_best;             // least ||b - A x||^2 at a start or check
  int32_t status, it, nchecks;
  int32_t nstall;             // checks in a row without a 10% gain on rr_best
};

// Vectors of one system (FP64).
//   PCG (Chronopoulos-Gear form): r, u = D^{-1} r, p, s = A p, w = A u
//   BiCGStab: r, u = rhat, p, s, w = v = A phat, t = A shat, phat, shat
// The vectors the SpMVs gather (u, phat, shat) are interleaved over the
// group's nsys systems: entry i of system j is at u[i * nsys] with system j's
// pointer at base + j, so one gathered row serves every system of the group
// from one cache line. The others are contiguous per system.
struct KVecs {
  const double* b;
  double* x;
  double* r;
  double* u;
  double* p;
  double* s;
  double* w;
  double* t;
  double* phat;
  double* shat;
  KState* st;
};

// Up to GMAX systems that share one matrix (SELL-64 layout, FP64 values), so
// the matrix is read once per row for all of them. Matrix kernels run
// nblk_m = ceil(n / (KBS * ept_m)) blocks, vector kernels
// nblk_v = ceil(n / (KBS * kept_v(nsys))); both are at most KNB_MAX. Partial sums:
// part_m is written by matrix kernels, part_v[q] by vector kernels of launch
// parity q^1; records are [block][GMAX][KP].
struct KGroup {
  int32_t nsys, n;
  const int32_t* sptr;        // SELL slice offsets
  const int32_t* col;
  const void* val;            // FP64 values, or FP32 (KLaunch::fp32)
  const double* dinv;         // Jacobi: 1 / diag(A)
  int32_t nblk_m, nblk_v;
  int32_t maxit, pad;         // iteration cap of the group's systems
  double* part_m;
  double* part_v[2];
  double* fold;               // [GMAX * KP] totals folded once from the records
  KVecs v[GMAX];
};

// One pressure Poisson system for the one-kernel-per-iteration CG
// (kernels_fcg.hip): the matrix in the part-local SELL-64 layout of a row
// partition (mesh.hpp, PartSell), Krylov vectors in part order. r, s and w are
// double-buffered by launch parity (parts read their halo rows of the buffer
// that no block writes in that launch); x and p are only touched by their
// owning part. part[q] holds the partials [gamma = r.u, r.r, delta = w.u]
// written by launches of parity q^1 (and by the start with parity q).
struct FGroup {
  int32_t n, nparts;
  const int32_t* perm;        // part-order row -> original row
  const int32_t* part_ptr;    // [nparts+1]
  const int32_t* halo_ptr;    // [nparts+1]
  const int32_t* halo;        // part-order rows
  const int32_t* slice_ptr;   // [nparts+1]
  const int32_t* sptr;        // slice entry offsets
  const uint16_t* lcol;       // local column indices
  const void* val;            // FP64, or FP32 (FLaunch::fp32)
  const double* dinv;         // part order
  const double* b;            // right-hand side, original order
  double* x;                  // initial guess in, solution out; original order
  double* bp;                 // b in part order
  double* xp;                 // x in part order
  double* p;
  double* r[2];
  double* s[2];
  double* w[2];
  double* part[2];            // [KP][nparts] SoA partials by parity
  double* part_s;             // start partials [r.r, b.b]
  KState* st;
  int32_t maxit;
  int32_t ipl;                // CG iterations per launch (1 or 2)
  // two iterations per launch: the second halo ring, the halo rows' slices
  // (local columns over own, halo and second ring) and values, and the
  // basis p, B p, B^2 p, z, B z ([5][n], part order) by launch parity; the
  // Gram partials take 16 values per part in part[]
  const int32_t* halo2_ptr;   // [nparts+1]
  const int32_t* halo2;
  const int32_t* hslice_ptr;  // [nparts+1]
  const int32_t* hsptr;
  const uint16_t* hlcol;
  const void* hval;
  double* y[2];
};

// Row-owner assembly inputs (see mesh.hpp)
struct RowAsm {
  int32_t nrows;
  const int32_t* sptr;        // SELL-64 slice offsets of the output matrices
  const int32_t* inc_ptr;
  const int32_t* inc;         // cell << 5 | local row index
  const uint8_t* slot;
  int32_t stride;
  const int32_t* c2d;         // [nc][nloc2] velocity DOFs
  int32_t nloc2;
  const double* X;            // vertex coordinates [nv][dim]
  void* out[3];               // FP64 values, or FP32 in the mixed form
  int32_t pair;               // IPCS_PAIR_P2P1 (0) or IPCS_PAIR_P3P2 (2D)
  const int32_t* c2v;         // [nc][nv_stride]; first dim+1 entries: the vertices
  int32_t nv_stride;          //   (the pressure cell table; its vertices come first)
  // row-owner kernels: runs of xcd_chunk consecutive row blocks are dealt to
  // the 8 XCDs in turn (0: blocks in order), so that rows that share cells
  // are assembled through one XCD's L2
  int32_t xcd_chunk;
};

// Row block of a row-owner launch for hardware block b of nb: with chunk c > 0,
// XCD x (= b mod 8) runs blocks x c .. x c + c - 1, then 8 c + x c .. and so
// on; the tail past the last full round of 8 c blocks stays in order.
__device__ __forceinline__ int xcd_block(int b, int nb, int c) {
  if (c <= 0) return b;
  const int round = 8 * c;
  if (b >= nb / round * round) return b;
  return b / round * round + (b & 7) * c + (b >> 3) % c;
}

// Manufactured solution on the device
struct Builtin {
  int32_t kind;               // IPCS_SOL_* or 0
  double prm[4];
  double nu;
};

// ------------------------------------------------------------ launchers
// Assembly (kernels_asm.hip). bs = rows per block, lds = dynamic LDS bytes;
// fp32 selects FP32 arithmetic and FP32 outputs (mixed form).
void asm_mass_stiff(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds);
// E = M/dt + cs C(U) (cs = -1: the explicit form's E = M/dt - C(U^n); cs = +1:
// the semi-implicit form's M/dt + C(U^n)), row-owner in one pass (asm_conv),
// or in two passes: asm_conv_cells forms
// the local matrices of all nc cells into buf ([nc][n_loc][n_loc] values of the
// working type, cell-batched), asm_local_sum adds them into the rows of
// a.out[0] (row-owner, conflict-free).
void asm_conv(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds,
              const double* U, int64_t n2, double inv_dt, double cs);
void asm_conv_cells(int dim, bool fp32, hipStream_t s, const RowAsm& a, int64_t nc,
                    const double* U, int64_t n2, double inv_dt, double cs, void* buf);
void asm_local_sum(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds,
                   const void* buf);
void asm_grad(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds);
// a.out[0] <- N_ce(U): sum_q w |J| phi_i phi_j d_e u_c (FP64, P2-P1)
void asm_newton(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds, const double* U,
                int64_t n2, int c, int e);
void asm_div(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds);
void asm_kp(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds);
void asm_lumped_p1(int dim, hipStream_t s, const RowAsm& a, double* w);
void asm_forcing(int dim, hipStream_t s, const RowAsm& a, const Builtin& bi, const double* fq,
                 int64_t nc, double t, double* F, int64_t n2);
// SELL-64 matrices: sptr/col layout, rowptr gives the true row lengths.
// Values are FP32 when fp32 is set, else FP64; dinv and lift values are FP64.
void form_eliminated(hipStream_t s, bool fp32, int64_t n, const int32_t* sptr,
                     const int32_t* rowptr, const int32_t* col, const uint8_t* bmask,
                     const void* M, const void* K, double cm, double ck, void* out, double* dinv);
void inv_diagonal(hipStream_t s, bool fp32, int64_t n, const int32_t* sptr,
                  const int32_t* rowptr, const int32_t* col, const void* val, double* dinv);
void lift_values(hipStream_t s, bool fp32, int64_t nlift, const int32_t* slot, const void* M,
                 const void* K, double cm, double ck, double* out);
void round_to_f32(hipStream_t s, int64_t n, const double* src, float* dst);

// Krylov (kernels_krylov.hip). A launch covers ngroups groups with the same
// number of systems ns and matrix-kernel rows per thread ept_m; bmap_m/bmap_v
// map blocks to (group, block in group) for matrix/vector kernels.
struct KLaunch {
  const KGroup* groups;
  int ngroups;
  int ns;            // systems per group: 1..GMAX
  int ept_m;         // rows per thread of matrix kernels: 1, 2 or 4
  int fp32;          // matrix values are FP32 (vectors and sums stay FP64)
  const int2* bmap_m;
  int nblocks_m;
  const int2* bmap_v;
  int nblocks_v;
  // 1: after each matrix kernel, one block per group folds the partial-sum
  // records its vector kernel needs into KGroup::fold, and every block of the
  // vector kernel reads those totals instead of re-reducing all records
  // (bitwise the same totals); 0: every block re-reduces the records
  int fold;
};
// Start (mode 0) or confirm/restart (mode 1, systems PENDING or RESTART):
// r = b - A x, then the status decision. par is the parity of the next
// iteration launch; a restart of a group whose maxit iterations have been
// launched (launched >= maxit) becomes MAXIT instead.
void pcg_start(hipStream_t s, const KLaunch& L, int mode, int par, int launched);
void pcg_iter(hipStream_t s, const KLaunch& L, int par);
void bicg_start(hipStream_t s, const KLaunch& L, int mode, int par, int launched);
// Systems of group g still iterating become MAXIT (their cap was reached).
void stop_group(hipStream_t s, const KLaunch& L, int g);
void bicg_iter(hipStream_t s, const KLaunch& L, int par);
void ksys_finish(hipStream_t s, const KLaunch& L);            // b == 0 systems: x := 0
void gather_states(hipStream_t s, const KLaunch& L, KState* out);   // out[g*GMAX + j]
void set_tolerance(hipStream_t s, const KLaunch& L, double tol2);   // every system's tol^2
// single kernels of an iteration, for timing
void pcg_spmv_only(hipStream_t s, const KLaunch& L);
void pcg_update_only(hipStream_t s, const KLaunch& L, int par);
void bicg_spmv_only(hipStream_t s, const KLaunch& L);                 // v = A phat
void bicg_update_s_only(hipStream_t s, const KLaunch& L, int par);    // s, shat
void bicg_spmv_t_only(hipStream_t s, const KLaunch& L);               // t = A shat
void bicg_update_x_only(hipStream_t s, const KLaunch& L, int par);    // x, r, p, phat

// One block of a one-group fused CG launch, addressed by the block index
// alone: the part's row and halo ranges and, for each of its slices k, the
// first entry sl[k].x and the width sl[k].y (slots k >= ns repeat the last
// slice's start with width 0, so every address is valid without a test), so
// that a block reaches its matrix entries one dependent load after it starts.
constexpr int FBLK_SL = 32;   // parts of up to FBLK_SL * 64 rows
struct FBlk {
  int32_t lb, p0, own, h0, nh, ns, pad[2];
  int2 sl[FBLK_SL];
};

// One-kernel-per-iteration Jacobi-CG (kernels_fcg.hip) over ngroups FGroups
// with the same rows per thread ept (parts have at most KBS * ept rows);
// bmap maps blocks to (group, part); lds = dynamic LDS bytes (8 per local
// row of the largest part, own + halo). A one-group launch may also carry
// blk (one FBlk per block, in bmap's order), hfirst (per block, the first KBS
// halo rows, 0 past the halo) and a host copy of its group: its iterations
// then take the group by value and the per-block data by block index.
struct FLaunch {
  const FGroup* groups;
  int ngroups;
  int ept;           // 1, 2, 4 or 8
  int fp32;
  const int2* bmap;
  int nblocks;
  size_t lds;
  const FBlk* blk;
  const int32_t* hfirst;
  FGroup one;
  int ipl = 1;       // CG iterations per launch of every group
};
// Mode 0: x and b to part order, r = b - A x, w = A D^{-1} r, status decision.
// Mode 1 (systems PENDING or RESTART): the same from the current iterate.
void fcg_start(hipStream_t s, const FLaunch& F, int mode, int par, int launched);
void fcg_iter(hipStream_t s, const FLaunch& F, int par);
// x (original order) := the part-order iterate, or 0 for b == 0 systems
void fcg_finish(hipStream_t s, const FLaunch& F);
// part-order copies of a matrix's values and of its Jacobi diagonal
void fcg_gather_values(hipStream_t s, bool fp32, int64_t nent, const int32_t* src,
                       const void* val, void* out);
void fcg_gather_dinv(hipStream_t s, int64_t n, const int32_t* perm, const double* dinv,
                     double* out);

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
// out = the extrapolation to the next time level of the newest nh (2 or 3)
// values h0, h1, h2 at equal steps on interior rows, the Dirichlet data on
// boundary rows
void extrapolate_with_bc(hipStream_t s, int dim, int nh, const double* h0, const double* h1,
                         const double* h2, const uint8_t* bmask, const double* gfull,
                         double* out, int64_t n2);
// b_c = sa E U_c - sg G_c P + F_c with Dirichlet lifting (explicit: E = M/dt -
// C(U^n), sa = 1; semi-implicit: E = M, sa = 1/dt; sg = 1 for IPCS, 0 for the
// Chorin projection, whose momentum step has no pressure term)
void rhs_momentum(hipStream_t s, int dim, bool fp32, int64_t n2, const int32_t* sp22,
                  const int32_t* col22, const void* E, double sa, double sg, const double* U,
                  const int32_t* sp21,
                  const int32_t* col21, void* const* Gc, const double* P, const double* F,
                  const int32_t* lift_ptr, const int32_t* lift_col, const double* liftA,
                  const uint8_t* bmask, const double* gfull, double* b);
// r = scale * sum_c D_c Us_c, then r -= mean(r) (mean_out receives it)
// r = scale * sum_c D_c Us_c projected to zero sum (mean_out receives the mean).
// floor_out0/1 (if not null) receive (64 eps)^2 * sum_k (scale sum_c |D_c||Us_c|)_k^2,
// a generous bound on ||rounding error of r||^2: part needs 2 * 8192 doubles.
void rhs_pressure(hipStream_t s, int dim, bool fp32, int64_t n1, const int32_t* sp12,
                  const int32_t* col12, void* const* Dc, const double* Us, int64_t n2,
                  double scale, double* r, double* part, double* mean_out, double* floor_out0,
                  double* floor_out1);
// res = b - A x (FP64 A), then res -= mean(res); totals[0..1] = sum(res), sum(res^2)
// before the projection; mean_out receives the mean
void residual_projected(hipStream_t s, int64_t n, const int32_t* sp, const int32_t* col,
                        const double* A, const double* x, const double* b, double* res,
                        double* part_s, double* part_q, double* totals, double* mean_out);
void sub_scalar(hipStream_t s, int64_t n, const double* scal, double* v);
void rhs_correction(hipStream_t s, int dim, bool fp32, int64_t n2, const int32_t* sp22,
                    const int32_t* col22, const void* M, const double* Us,
                    const int32_t* sp21, const int32_t* col21, void* const* Gc,
                    const double* dP, double scale, const int32_t* lift_ptr,
                    const int32_t* lift_col, const double* liftM, const uint8_t* bmask,
                    const double* gfull, double* b);
// v -= (w.v)/(sum w); out receives the subtracted mean
void sub_weighted_mean(hipStream_t s, int64_t n, const double* w, double* v, double* part,
                       double* out);
void axpy_inplace(hipStream_t s, int64_t n, double a, const double* x, double* y);

}  // namespace ipcs
