// One IPCS run: its device workspace layout, constant matrices, state and the
// three sub-steps of eq. (9) (Section 2.2.1), plus the host side of the Krylov
// solves shared by single runs and batches.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "launch.hpp"
#include "ipcs.h"
#include "mesh.hpp"
#include "rules.hpp"

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

// Per-launch event timing of selected kernels in the normal launch sequence
// (measurement hook). Pairs are read back after the stream has synchronized.
struct KTimer {
  uint32_t mask = 0;
  std::vector<hipEvent_t> ev;   // [2k], [2k+1] bracket the k-th timed launch
  std::vector<int> which;       // kernel id of the k-th timed launch
  double ms[IPCS_NKERNEL] = {};
  int64_t cnt[IPCS_NKERNEL] = {};
  ~KTimer();
  void reset(uint32_t m);
  template <class F>
  void run(hipStream_t s, int kid, F f) {
    if (kid < 0 || !((mask >> kid) & 1u)) {
      f();
      return;
    }
    const size_t k = which.size();
    while (ev.size() < 2 * (k + 1)) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      ev.push_back(e);
    }
    LaunchEvents le{ev[2 * k], ev[2 * k + 1]};
    launch_events() = &le;
    f();   // one kernel launch, which takes the events
    const bool taken = launch_events() == nullptr;
    launch_events() = nullptr;
    if (!taken) fail(IPCS_E_STATE, "timed launcher did not launch a kernel");
    which.push_back(kid);
  }
  void drain();   // the stream must have synchronized
};

// Host view of a set of Krylov groups solved by the same launches.
struct KSet {
  KLaunch L{};
  // pressure Poisson CG in one kernel per iteration (kernels_fcg.hip): the
  // launch uses F; L still serves status polling, caps and tolerances
  bool fused = false;
  FLaunch F{};
  std::vector<FGroup> h_fgroups;
  std::vector<KGroup> h_groups;
  KState* d_poll = nullptr;    // [ngroups * GMAX] polling copies of the states
  int last_iters = 0;          // iterations the previous solve took (poll schedule)
  double us_per_launch = 0.0;  // device time per iteration launch in the previous solve (0: none)
  double us_per_poll = 0.0;    // device idle time per status poll in the previous solve
  // kernel ids for timing: PCG {spmv, update} (fused: {iteration}),
  // BiCGStab {v, s, t, x}; -1: none
  int kid[4] = {-1, -1, -1, -1};
  // sets of several groups: device room for block maps over the groups that
  // are still unfinished (matrix, vector and fused maps back to back), so that
  // finished groups stop taking blocks; null: no compaction
  int2* d_compact = nullptr;
  int compact_cap = 0;
};

enum class KMethod { PCG, BICG };

// Runs a set to completion (each group at most its maxit iterations). h_states[g*GMAX + j]
// receives the final states. Returns IPCS_OK or the status of the first
// failed system.
// With time_bursts false the solve records no chunk-timing events and keeps
// the set's measured costs (us_per_launch, us_per_poll) as they are.
int krylov_solve(hipStream_t s, KSet& S, KMethod m, int check_every,
                 std::vector<KState>& h_states, KState* pinned, KTimer& T,
                 bool time_bursts = true);
int status_to_code(int kstatus);

// Pinned host staging for status polls (kPinnedStates states each), from a
// process-wide pool: freeing pinned memory waits for every stream of the
// device, so a run that ends (a served request) would otherwise stall the
// other runs' streams until the device drains. Buffers taken are given back
// when their run ends and are reused; the pool is freed with the process.
constexpr int kPinnedStates = 3 * GMAX;
KState* pinned_take();
void pinned_give(KState* p);

// Rows per thread of matrix kernels for a group of n rows, and the block
// counts of matrix / vector kernels (each at most KNB_MAX).
int kept_m_for(int64_t n, int ns);
int nblk_m_for(int64_t n, int ns);
int nblk_v_for(int64_t n, int ns);
int fold_for(int64_t n, int ns);   // KLaunch::fold for a group of n rows, ns systems
// (group, block) map interleaving the groups block by block
void build_bmap(const std::vector<int>& nblk, std::vector<int2>& bmap);
// The blocks of a launch are dealt to the 8 XCDs in turn (block b runs on XCD
// b % 8, each XCD with its own L2). Reorders a block map so that each XCD runs
// one contiguous range of its entries: neighbouring parts of a row partition
// (which share halo rows) then share an L2.
void xcd_order(std::vector<int2>& bmap);
// Deals runs of `chunk` consecutive entries to the XCDs in turn: XCD x takes
// runs x, x + 8, ... (the tail past the last full round stays in order).
void xcd_chunks(std::vector<int2>& bmap, int chunk);

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
  int64_t ne22 = 0, ne21 = 0, ne11 = 0, ne12 = 0;   // SELL entries per pattern
  AsmCfg cfg_mk, cfg_e, cfg_g, cfg_d, cfg_kp;

  // ---- device arrays (all inside the workspace)
  double* X = nullptr;
  int32_t* c2d = nullptr;
  int32_t* c2v = nullptr;      // pressure cell table: its first dim+1 entries are the vertices
  double* x2 = nullptr;
  double* xp = nullptr;        // pressure node coordinates (X itself for P2-P1)
  uint8_t* bmask = nullptr;
  int32_t* bidx = nullptr;
  // per pattern: SELL slice offsets, SELL columns, CSR row pointer (row lengths)
  int32_t *sp22 = nullptr, *col22 = nullptr, *rp22 = nullptr;
  int32_t *sp21 = nullptr, *col21 = nullptr, *rp21 = nullptr;
  int32_t *sp11 = nullptr, *col11 = nullptr, *rp11 = nullptr;
  int32_t *sp12 = nullptr, *col12 = nullptr, *rp12 = nullptr;
  int32_t *inc2p = nullptr, *inc2 = nullptr, *inc1p = nullptr, *inc1 = nullptr;
  uint8_t *s22 = nullptr, *s21 = nullptr, *s11 = nullptr, *s12 = nullptr;
  int32_t *lift_ptr = nullptr, *lift_slot = nullptr, *lift_col = nullptr;
  // matrix values: FP64, or FP32 in the mixed form (vsz bytes per value)
  bool mixed = false;
  int vsz = 8;
  void *M = nullptr, *K = nullptr, *E = nullptr, *Ael = nullptr, *Mel = nullptr;
  void *Kp = nullptr, *Dc[3] = {}, *Gc[3] = {};
  void* Eloc = nullptr;       // local matrices of the convection operator [nc][nloc][nloc]
  double* Kp64 = nullptr;     // FP64 Kp (the same array as Kp in the FP64 form)
  double *rIR = nullptr, *dIR = nullptr;   // mixed form: refinement residual, correction
  double ir_c = 0.0;          // mixed form: reduction per refinement pass seen last step
  // mixed form: iterations of each refinement pass of the last step; pass k's
  // inner solve sizes its polls from entry k (passes differ widely in length)
  static constexpr int kIrHist = 4;
  int ir_last[kIrHist] = {};
  double *liftA = nullptr, *liftM = nullptr;
  double *dinvA = nullptr, *dinvM = nullptr, *dinvKp = nullptr, *w = nullptr;
  double *U = nullptr, *Unew = nullptr, *Ustar = nullptr, *bU = nullptr, *F = nullptr,
         *gfull = nullptr;
  double *P = nullptr, *dP = nullptr, *rP = nullptr;
  // the three previous steps' tentative velocities (newest first), kept for
  // the extrapolated momentum start; mhist counts the steps completed since
  // the history was last cleared (kept up to kMhistFull)
  static constexpr int kMhistFull = 4;
  double* Ush[3] = {};
  int mhist = 0;
  double* kv2 = nullptr;      // Krylov work of the velocity systems [dim][8][n2]
  double* kv1 = nullptr;      // Krylov work of the Poisson system [5][n1]
  KState* kst = nullptr;      // [2*dim+1]
  KGroup* kgroups = nullptr;  // [3]: momentum, pressure, correction
  double* part_m[3] = {};     // per group (momentum, pressure, correction)
  double* part_v[3][2] = {};
  double* fold[3] = {};       // folded totals per group
  int2* bmap_m[3] = {};
  int2* bmap_v[3] = {};
  KState* poll = nullptr;     // [3 * GMAX]
  // pressure Poisson CG in one kernel per iteration on a row partition of Kp
  // (null pp: the two-kernel CG of the velocity solves)
  std::shared_ptr<const PartSell> pp;
  int fcg_ept = 0;
  int32_t *f_perm = nullptr, *f_part_ptr = nullptr, *f_halo_ptr = nullptr, *f_halo = nullptr,
          *f_slice_ptr = nullptr, *f_sptr = nullptr, *f_src = nullptr;
  uint16_t* f_lcol = nullptr;
  void* f_val = nullptr;      // Kp (inner CG values) in the partition's layout
  double *f_dinv = nullptr, *f_bp = nullptr, *f_xp = nullptr, *f_p = nullptr;
  double* f_vec = nullptr;    // r[2], s[2], w[2]
  double *f_part[2] = {}, *f_part_s = nullptr;
  int2* f_bmap = nullptr;
  FBlk* f_blk = nullptr;
  int32_t* f_hfirst = nullptr;
  bool f_blk_ok = false;       // every part's slice offsets fit an FBlk
  int fcg_s = 1;               // CG iterations per launch
  // two iterations per launch: second ring, halo rows' slices and values, basis
  int32_t *f_h2ptr = nullptr, *f_h2 = nullptr, *f_hsl = nullptr, *f_hsptr = nullptr,
          *f_hsrc = nullptr;
  uint16_t* f_hlcol = nullptr;
  void* f_hval = nullptr;
  double* f_y = nullptr;       // [2][5][n1]
  FGroup* fgroup = nullptr;
  double* spart = nullptr;    // scratch partials for one-off reductions [8192*2]
  uint32_t* scnt = nullptr;
  double* scal = nullptr;     // [8] device scalars: 0 mean(r), 1 mean(dP), 2 mean(P)
  double* gb = nullptr;       // Dirichlet callback staging [nb][dim]
  double* fq = nullptr;       // forcing callback staging [dim][nc][nq]
  int64_t ws_bytes = 0;

  KSet set_mom, set_p, set_corr;
  KState* pinned = nullptr;   // host mirror for status polling
  KTimer timer;

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
  void set_precision();   // mixed and vsz from prm.precision
  void sizes_from_mesh();
  void choose_poisson_form();
  void layout(Carver& c);
  // convection in two passes (cell-batched local matrices, then their
  // row-owner sum): 3D, and the P3-P2 pair in 2D
  bool two_pass_conv() const { return dim == 3 || mesh->pair == IPCS_PAIR_P3P2; }
  // points per cell of the pair's cell rule (the forcing quadrature)
  int cell_nq() const {
    if (mesh->pair == IPCS_PAIR_P3P2) return dim == 2 ? RuleT9::NQ : RuleTet9::NQ;
    return dim == 2 ? Rule<2>::NQ : Rule<3>::NQ;
  }
  void create(std::shared_ptr<const Mesh> m, const ipcs_params& p, void* ws, int64_t bytes,
              hipStream_t s);
  void upload_mesh();
  void assemble_constant();
  void reform_A();
  void setup_solvers();
  void set_builtin(int kind, const double* prm, int nprm);
  void set_state(const double* u, const double* p, double t);
  int phase(int which, ipcs_step_stats* st);
  void asm_phase();
  void pressure_rhs();
  void pressure_end();
  void clear_pressure_start();
  bool warm_p() const { return prm.poisson_start == IPCS_START_PREVIOUS; }
  bool extrap_m() const { return prm.momentum_start == IPCS_MSTART_EXTRAPOLATED; }
  // the next steps start their solves as the first after a new state would
  void clear_history() {
    mhist = 0;
    clear_pressure_start();
  }
  void correction_rhs();
  void correction_commit();
  void finish_step(ipcs_step_stats* st);
  int step(ipcs_step_stats* st);
  double profile_kernel(int kernel, int nlaunch);
  // host-side CSR values (FP64) of a device SELL matrix of value size vbytes
  void export_values(int pattern, const void* dev, int vbytes, double* out);
  int pressure_solve(std::vector<KState>& hs, ipcs_step_stats* st);
};

// Where a batch step keeps its shared-launch descriptors and status staging.
// Default (dev == nullptr): one stream-ordered device allocation per solve and
// pinned host staging. Fixed: a device array of dev_cap bytes and a host
// array of host_cap states, both reused solve after solve (the step waits for
// each solve before the next one writes its descriptors); nothing is
// allocated.
struct BatchMem {
  char* dev = nullptr;
  size_t dev_cap = 0;
  KState* host = nullptr;
  int host_cap = 0;
};

// One step of every run with shared Krylov launches on stream s (serving form).
int batch_step(Run* const* runs, int nruns, hipStream_t s, ipcs_step_stats* stats,
               const BatchMem& mem = BatchMem{});
// Largest descriptor space any one shared solve of a batch step of these runs
// takes (host computation only).
size_t batch_descriptor_bytes(Run* const* runs, int nruns);
// The fixed device array of ipcs_batch_step_noalloc on the current device
// (scratch.hip); *cap receives its size in bytes.
char* batch_scratch(size_t* cap);
// The fixed host array of status states for that device; *cap receives its
// length in states.
KState* batch_host_staging(int* cap);

void fill_stats_solve(const std::vector<KState>& hs, int nsys, int which, ipcs_step_stats* st);

}  // namespace ipcs
