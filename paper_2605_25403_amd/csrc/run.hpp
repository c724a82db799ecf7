// One IPCS run: its device workspace layout, constant matrices, state and the
// three sub-steps of eq. (9) (Section 2.2.1), plus the Krylov driver shared by
// single runs and batches.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "device.hpp"
#include "ipcs.h"
#include "mesh.hpp"

namespace ipcs {

// Carves a caller-provided device workspace; with base == nullptr it only
// measures.
struct Carver {
  char* base = nullptr;
  int64_t off = 0;
  template <class T>
  T* take(int64_t n) {
    off = (off + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * (int64_t)sizeof(T);
    return p;
  }
};

// A group of Krylov systems solved together (one launch per kernel).
struct SolveSet {
  int nsys = 0;
  int G = 16;                  // lanes per row
  int nblocks = 0;             // total blocks of a launch
  KSys* d_sys = nullptr;       // [nsys]
  int2* d_bmap = nullptr;      // [nblocks]
  std::vector<KSys> h_sys;
  std::vector<int2> h_bmap;
  KState* d_poll = nullptr;    // [nsys] contiguous copy of the states for polling
};

enum class KMethod { PCG, BICG };

// Runs a solve set to completion; h_states receives the final states.
// Returns IPCS_OK or the status of the first failed system.
int krylov_solve(hipStream_t s, const SolveSet& S, KMethod m, int check_every,
                 std::vector<KState>& h_states, KState* pinned);

// Build the interleaved block map for systems with the given block counts.
void build_bmap(const std::vector<int>& nblk, std::vector<int2>& bmap);

int lanes_for(double avg_row);
int nblk_for(int64_t n, int G);

struct AsmCfg {
  int bs = 256;
  size_t lds = 0;
};

struct Run {
  std::shared_ptr<const Mesh> mesh;
  ipcs_params prm{};
  hipStream_t stream = nullptr;
  int dim = 2;
  int64_t n1 = 0, n2 = 0, nc = 0, nv = 0, nb = 0, nlift = 0;
  int G22 = 16, G11 = 8, G12 = 16;
  AsmCfg cfg_mk, cfg_e, cfg_g, cfg_d, cfg_kp;

  // ---- device arrays (all inside the workspace)
  double* X = nullptr;
  int32_t* c2d = nullptr;
  double* x2 = nullptr;
  uint8_t* bmask = nullptr;
  int32_t* bidx = nullptr;
  int32_t *rp22 = nullptr, *col22 = nullptr, *rp21 = nullptr, *col21 = nullptr;
  int32_t *rp11 = nullptr, *col11 = nullptr, *rp12 = nullptr, *col12 = nullptr;
  int32_t *inc2p = nullptr, *inc2 = nullptr, *inc1p = nullptr, *inc1 = nullptr;
  uint8_t *s22 = nullptr, *s21 = nullptr, *s11 = nullptr, *s12 = nullptr;
  int32_t *lift_ptr = nullptr, *lift_slot = nullptr, *lift_col = nullptr;
  double *M = nullptr, *K = nullptr, *E = nullptr, *Ael = nullptr, *Mel = nullptr;
  double *Kp = nullptr, *Dc[3] = {}, *Gc[3] = {};
  double *liftA = nullptr, *liftM = nullptr;
  double *dinvA = nullptr, *dinvM = nullptr, *dinvKp = nullptr, *w = nullptr;
  double *U = nullptr, *Unew = nullptr, *Ustar = nullptr, *bU = nullptr, *F = nullptr,
         *gfull = nullptr;
  double *P = nullptr, *dP = nullptr, *rP = nullptr;
  double* kv2 = nullptr;      // Krylov work for the velocity systems [9][dim][n2]
  double* kv1 = nullptr;      // Krylov work for the Poisson system [5][n1]
  KState* kst = nullptr;      // [2*dim+1]
  double* kpart = nullptr;    // [(2*dim+1)][nblkmax][KPART]
  uint32_t* kcnt = nullptr;   // [2*dim+1]
  KSys* ksys = nullptr;       // [2*dim+1]
  int2* bmap_mom = nullptr;
  int2* bmap_p = nullptr;
  int2* bmap_corr = nullptr;
  double* spart = nullptr;    // scratch partials for one-off reductions [8192][KPART]
  uint32_t* scnt = nullptr;   // [4]
  double* scal = nullptr;     // [8] device scalars: 0 mean(r), 1 shift(dP), 2 mean(P)
  KState* poll = nullptr;     // [2*dim+1] polling copies of the Krylov states
  double* gb = nullptr;       // Dirichlet callback staging [nb][dim]
  double* fq = nullptr;       // forcing callback staging [dim][nc][nq]
  int64_t ws_bytes = 0;

  SolveSet set_mom, set_p, set_corr;
  KState* pinned = nullptr;   // host mirror for status polling

  // ---- problem data
  Builtin bi{};
  ipcs_field_fn f_cb = nullptr, g_cb = nullptr;
  void *f_ctx = nullptr, *g_ctx = nullptr;
  std::vector<double> h_xq;   // quadrature points for the forcing callback
  std::vector<double> h_xb;   // boundary node coordinates for the Dirichlet callback

  double t = 0.0, t1 = 0.0;
  bool A_dirty = false;
  int phase_next = IPCS_PHASE_ASM;
  bool has_F = false;
  hipEvent_t ev[5] = {};

  ~Run();
  void layout(Carver& c);
  void create(std::shared_ptr<const Mesh> m, const ipcs_params& p, void* ws, int64_t bytes,
              hipStream_t s);
  void upload_mesh();
  void assemble_constant();
  void reform_A();
  void setup_solvers();
  void set_builtin(int kind, const double* prm, int nprm);
  void set_state(const double* u, const double* p, double t);
  int phase(int which, ipcs_step_stats* st);
  int step(ipcs_step_stats* st);
  void normalize_pressure(double* Pdev);
};

void fill_stats_solve(const std::vector<KState>& hs, int which, ipcs_step_stats* st);

}  // namespace ipcs
