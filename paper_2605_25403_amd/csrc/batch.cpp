// Serving form: one IPCS step (eq. (9), Section 2.2.1) for many runs at once.
//
// Assembly and right-hand sides are launched run by run on the batch stream
// (each is a handful of launches). The Krylov solves, where a step spends its
// time, are shared: the groups of every run (its momentum, Poisson and
// correction systems) go into one launch set, so each iteration of every run
// costs one launch per kernel for the whole batch. Each group keeps its own
// partial sums, scalars, status and stopping decision, and the block
// decomposition of a group does not depend on what else shares the launch, so
// a run's result in a batch is bitwise the one it gets alone.
//
// Launch sets are split by (systems per group, rows per thread of matrix
// kernels, matrix value type), which the kernels take as template arguments;
// Poisson systems in the one-kernel-per-iteration form (kernels_fcg.hip) form
// sets of their own by (rows per thread, value type), with the largest LDS
// size of their members.
// Their device descriptors (group table, block maps, polling slots) come from
// one stream-ordered allocation per solve, released stream-ordered, or, for
// callers that cannot allocate, from a fixed device array (BatchMem).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>

#include "common.hpp"
#include "device.hpp"
#include "run.hpp"

namespace ipcs {

namespace {

// pinned host staging for status polling, grown as needed
KState* pinned_states(int n) {
  thread_local KState* p = nullptr;
  thread_local int cap = 0;
  if (n > cap) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    HIP_OK(hipHostMalloc((void**)&p, sizeof(KState) * (size_t)n, hipHostMallocDefault));
    cap = n;
  }
  return p;
}

struct DevBuf {
  char* base = nullptr;
  hipStream_t s = nullptr;
  explicit DevBuf(hipStream_t st, size_t bytes) : s(st) {
    HIP_OK(hipMallocAsync((void**)&base, std::max<size_t>(bytes, 256), s));
  }
  ~DevBuf() {
    if (base) (void)hipFreeAsync(base, s);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// One shared launch set over the groups of several runs.
struct Shared {
  KSet S;
  std::vector<Run*> owner;   // run of each group
};

KSet& set_of(Run& r, int which) {
  return which == 0 ? r.set_mom : which == 1 ? r.set_p : r.set_corr;
}

// Plan of one shared launch set: its runs, block maps and the offsets of its
// descriptors in the solve's descriptor space.
struct Plan {
  bool fused = false;
  std::vector<Run*> rs;
  std::vector<int2> bm, bv, bf;
  size_t o_groups = 0, o_bm = 0, o_bv = 0, o_poll = 0, o_fgroups = 0, o_bf = 0, o_compact = 0;
};

// Plans the shared sets for system set `which` (0 momentum, 1 Poisson,
// 2 correction) of the given runs; returns the bytes their descriptors take.
size_t plan_shared(const std::vector<Run*>& runs, int which, std::vector<Plan>& plans) {
  // fused Poisson sets: (1, iterations per launch, rows per thread, value type);
  // others: (0, ns, ept_m, value type)
  std::map<std::tuple<int, int, int, int>, std::vector<Run*>> cls;
  for (Run* r : runs) {
    const KSet& K = set_of(*r, which);
    if (K.fused) cls[{1, K.F.ipl, K.F.ept, K.F.fp32}].push_back(r);
    else cls[{0, K.L.ns, K.L.ept_m, K.L.fp32}].push_back(r);
  }
  // sizes
  size_t bytes = 0;
  auto take = [&](size_t n) {
    bytes = (bytes + 255) / 256 * 256;
    const size_t off = bytes;
    bytes += n;
    return off;
  };
  plans.clear();
  for (auto& kv : cls) {
    Plan p;
    p.fused = std::get<0>(kv.first) == 1;
    p.rs = kv.second;
    std::vector<int> nm, nv, nf;
    for (Run* r : p.rs) {
      const KSet& K = set_of(*r, which);
      nm.push_back(K.h_groups[0].nblk_m);
      nv.push_back(K.h_groups[0].nblk_v);
      if (p.fused) nf.push_back(K.h_fgroups[0].nparts);
    }
    build_bmap(nm, p.bm);
    build_bmap(nv, p.bv);
    p.o_groups = take(sizeof(KGroup) * p.rs.size());
    p.o_bm = take(sizeof(int2) * p.bm.size());
    p.o_bv = take(sizeof(int2) * p.bv.size());
    p.o_poll = take(sizeof(KState) * GMAX * p.rs.size());
    if (p.fused) {
      // group by group, each XCD taking a contiguous range (neighbouring parts)
      for (size_t gi = 0; gi < nf.size(); ++gi)
        for (int b = 0; b < nf[gi]; ++b) p.bf.push_back(make_int2((int)gi, b));
      xcd_order(p.bf);
      p.o_fgroups = take(sizeof(FGroup) * p.rs.size());
      p.o_bf = take(sizeof(int2) * p.bf.size());
    }
    // room for the block maps over unfinished groups (krylov_solve)
    p.o_compact = take(sizeof(int2) * (p.bm.size() + p.bv.size() + p.bf.size()));
    plans.push_back(std::move(p));
  }
  return std::max<size_t>(bytes, 256);
}

// Builds the shared sets for system set `which` of the given runs. The
// descriptors live in mem's fixed array when it has one, else in buf, which
// the caller keeps alive until the solves have been enqueued.
std::vector<Shared> make_shared(const std::vector<Run*>& runs, int which, hipStream_t s,
                                std::unique_ptr<DevBuf>& buf, const BatchMem& mem) {
  std::vector<Plan> plans;
  const size_t bytes = plan_shared(runs, which, plans);
  char* base = nullptr;
  if (mem.dev) {
    // checked for the whole batch before its step began (batch_mem_check)
    if (bytes > mem.dev_cap) fail(IPCS_E_CAPACITY, "batch descriptors exceed the fixed array");
    base = mem.dev;
  } else {
    buf.reset(new DevBuf(s, bytes));
    base = buf->base;
  }
  std::vector<char> host(bytes, 0);
  std::vector<Shared> out;
  for (Plan& p : plans) {
    Shared sh;
    sh.owner = p.rs;
    KSet& S = sh.S;
    int last = 0;
    double us = 0.0, up = 0.0;
    for (Run* r : p.rs) {
      const KSet& own = set_of(*r, which);
      S.h_groups.push_back(own.h_groups[0]);
      last = std::max(last, own.last_iters);
      us = std::max(us, own.us_per_launch);
      up = std::max(up, own.us_per_poll);
    }
    std::memcpy(host.data() + p.o_groups, S.h_groups.data(), sizeof(KGroup) * p.rs.size());
    std::memcpy(host.data() + p.o_bm, p.bm.data(), sizeof(int2) * p.bm.size());
    std::memcpy(host.data() + p.o_bv, p.bv.data(), sizeof(int2) * p.bv.size());
    const KLaunch& L0 = set_of(*p.rs[0], which).L;
    // folded totals are bitwise the re-reduced ones: fold if any member would
    int fold = 0;
    for (Run* r : p.rs) fold |= set_of(*r, which).L.fold;
    S.L = KLaunch{reinterpret_cast<const KGroup*>(base + p.o_groups),
                  (int)p.rs.size(),
                  L0.ns,
                  L0.ept_m,
                  L0.fp32,
                  reinterpret_cast<const int2*>(base + p.o_bm),
                  (int)p.bm.size(),
                  reinterpret_cast<const int2*>(base + p.o_bv),
                  (int)p.bv.size(),
                  fold};
    S.d_poll = reinterpret_cast<KState*>(base + p.o_poll);
    S.d_compact = reinterpret_cast<int2*>(base + p.o_compact);
    S.compact_cap = (int)(p.bm.size() + p.bv.size() + p.bf.size());
    if (p.fused) {
      size_t lds = 0;
      for (Run* r : p.rs) {
        const KSet& own = set_of(*r, which);
        S.h_fgroups.push_back(own.h_fgroups[0]);
        lds = std::max(lds, own.F.lds);
      }
      std::memcpy(host.data() + p.o_fgroups, S.h_fgroups.data(), sizeof(FGroup) * p.rs.size());
      std::memcpy(host.data() + p.o_bf, p.bf.data(), sizeof(int2) * p.bf.size());
      const FLaunch& F0 = set_of(*p.rs[0], which).F;
      S.fused = true;
      S.F = FLaunch{reinterpret_cast<const FGroup*>(base + p.o_fgroups), (int)p.rs.size(),
                    F0.ept, F0.fp32, reinterpret_cast<const int2*>(base + p.o_bf),
                    (int)p.bf.size(), lds};
      S.F.ipl = F0.ipl;
    }
    S.last_iters = last;
    S.us_per_launch = us;
    S.us_per_poll = up;
    std::copy(std::begin(set_of(*p.rs[0], which).kid), std::end(set_of(*p.rs[0], which).kid),
              std::begin(S.kid));
    out.push_back(std::move(sh));
  }
  HIP_OK(hipMemcpyAsync(base, host.data(), bytes, hipMemcpyHostToDevice, s));
  // host is a pageable stack copy: finish the transfer before it goes away
  HIP_OK(hipStreamSynchronize(s));
  return out;
}

// Solves system set `which` of the runs together. rc[run] receives each run's
// status; stats are filled per run.
void solve_shared(const std::vector<Run*>& runs, int which, KMethod m, hipStream_t s,
                  std::map<Run*, int>& rc, std::map<Run*, ipcs_step_stats*>& st,
                  const BatchMem& mem) {
  if (runs.empty()) return;
  std::unique_ptr<DevBuf> buf;
  std::vector<Shared> sets = make_shared(runs, which, s, buf, mem);
  KTimer none;
  for (Shared& sh : sets) {
    int check_every = 1 << 30;
    for (Run* r : sh.owner) check_every = std::min(check_every, r->prm.check_every);
    std::vector<KState> hs;
    const int nslot = GMAX * (int)sh.owner.size();
    KState* pin = nullptr;
    if (mem.dev) {
      if (nslot > mem.host_cap) fail(IPCS_E_CAPACITY, "batch has more runs than the fixed staging");
      pin = mem.host;
    } else {
      pin = pinned_states(nslot);
    }
    // with a fixed array, solves take no chunk-timing events (the poll
    // schedule keeps the costs measured by earlier solves)
    krylov_solve(s, sh.S, m, check_every, hs, pin, none, mem.dev == nullptr);
    for (size_t g = 0; g < sh.owner.size(); ++g) {
      Run* r = sh.owner[g];
      set_of(*r, which).last_iters = sh.S.last_iters;
      set_of(*r, which).us_per_launch = sh.S.us_per_launch;
      set_of(*r, which).us_per_poll = sh.S.us_per_poll;
      const int ns = sh.S.h_groups[g].nsys;
      std::vector<KState> mine(hs.begin() + g * GMAX, hs.begin() + g * GMAX + ns);
      int code = IPCS_OK;
      for (const KState& k : mine) {
        const int c = status_to_code(k.status);
        if (code == IPCS_OK && c != IPCS_OK) code = c;
      }
      rc[r] = code;
      if (which != 1 || !r->mixed) fill_stats_solve(mine, ns, which + 1, st[r]);
      else if (st[r]) {
        st[r]->it_p += mine[0].it;
        st[r]->checks_p += mine[0].nchecks;
      }
    }
  }
}

}  // namespace

// Mixed-form refinement for several runs (Run::pressure_solve, shared
// inner solves): every pass checks each run's FP64 residual, then solves the
// correction systems of the runs that still need one together.
static void refine_shared(const std::vector<Run*>& runs, hipStream_t s, std::map<Run*, int>& rc,
                          std::map<Run*, ipcs_step_stats*>& st, const BatchMem& mem) {
  struct IR {
    double bb = -1.0, rel = 0.0, prev = 0.0, contraction = 0.0, floor_in = 0.0;
    double last_tol = 1.0, op_limit = 0.0;
    int outer = 0;
    double host[4] = {0.0, 0.0, 0.0, 0.0};
  };
  std::map<Run*, IR> ir;
  std::vector<Run*> active = runs;
  while (!active.empty()) {
    for (Run* r : active) {
      residual_projected(s, r->n1, r->sp11, r->col11, r->Kp64, r->dP, r->rP, r->rIR, r->spart,
                         r->spart + 8192, r->scal + 3, r->scal + 5);
      HIP_OK(hipMemcpyAsync(ir[r].host, r->scal + 3, 4 * sizeof(double), hipMemcpyDeviceToHost,
                            s));
    }
    HIP_OK(hipStreamSynchronize(s));
    std::vector<Run*> inner;
    for (Run* r : active) {
      IR& q = ir[r];
      const double rr = std::max(0.0, q.host[1] - q.host[0] * q.host[0] / (double)r->n1);
      if (q.bb < 0.0) q.bb = rr;
      q.rel = q.bb > 0.0 ? std::sqrt(rr / q.bb) : 0.0;
      if (!std::isfinite(rr)) {
        rc[r] = IPCS_E_NONFINITE;
        continue;
      }
      // done; an r at its own rounding level on the first pass is zero
      if (rr <= r->prm.tol_ir * r->prm.tol_ir * q.bb || (q.outer == 0 && rr <= q.host[3]))
        continue;
      if (q.outer >= 30) {
        rc[r] = IPCS_E_NOT_CONVERGED;
        continue;
      }
      if (q.outer > 0) {   // as in Run::pressure_solve
        q.contraction = q.rel / q.prev;
        if (q.contraction > 2.0 * q.last_tol) q.op_limit = std::max(q.op_limit, q.contraction);
      } else {
        q.contraction = r->ir_c;
      }
      q.prev = q.rel;
      const double need = r->prm.tol_ir / q.rel;
      const double tol_in =
          std::min(0.5, std::max({need, 0.5 * q.contraction, q.floor_in, r->prm.tol_p}));
      q.last_tol = tol_in;
      set_tolerance(s, r->set_p.L, tol_in * tol_in);
      if (q.outer > 0 || !r->warm_p())   // as in Run::pressure_solve
        HIP_OK(hipMemsetAsync(r->dIR, 0, sizeof(double) * r->n1, s));
      q.outer += 1;
      inner.push_back(r);
    }
    if (inner.empty()) break;
    // each pass sizes its polls from the same pass of the run's last step
    for (Run* r : inner) {
      const int k = ir[r].outer - 1;
      r->set_p.last_iters = k < Run::kIrHist ? r->ir_last[k] : 0;
    }
    std::map<Run*, int> rin;
    solve_shared(inner, 1, KMethod::PCG, s, rin, st, mem);
    for (Run* r : inner) {
      const int k = ir[r].outer - 1;
      if (k < Run::kIrHist) r->ir_last[k] = r->set_p.last_iters;
    }
    active.clear();
    for (Run* r : inner) {
      int c = rin[r];
      if (c == IPCS_E_BREAKDOWN) {   // as in Run::pressure_solve
        ir[r].floor_in = ir[r].floor_in == 0.0 ? 1e-6 : std::min(1e-2, ir[r].floor_in * 100.0);
        c = IPCS_OK;
      }
      if (c != IPCS_OK) {
        rc[r] = c;
        continue;
      }
      axpy_inplace(s, r->n1, 1.0, r->dIR, r->dP);
      active.push_back(r);
    }
  }
  for (Run* r : runs) {
    const IR& q = ir[r];
    if (q.op_limit > 0.0) r->ir_c = q.op_limit;   // as in Run::pressure_solve
    if (st[r]) {
      st[r]->res_p = q.rel;
      st[r]->ir_outer = q.outer;
    }
  }
}

size_t batch_descriptor_bytes(Run* const* runs, int nruns) {
  std::vector<Run*> all(runs, runs + nruns);
  std::vector<Plan> plans;
  size_t most = 0;
  // a subset's descriptors (the plain or mixed Poisson runs, the runs still
  // refining) never take more room than the whole batch's
  for (int which = 0; which < 3; ++which) most = std::max(most, plan_shared(all, which, plans));
  return most;
}

int batch_step(Run* const* runs, int nruns, hipStream_t s, ipcs_step_stats* stats,
               const BatchMem& mem) {
  std::vector<Run*> all(runs, runs + nruns);
  for (Run* r : all) {
    if (r->phase_next != IPCS_PHASE_ASM) fail(IPCS_E_STATE, "a run is in the middle of a step");
    if (r->dim != all[0]->dim) fail(IPCS_E_INVALID, "all runs of a batch have one dimension");
  }
  // every launch of the step goes on the batch stream
  std::vector<hipStream_t> saved;
  for (Run* r : all) {
    saved.push_back(r->stream);
    r->stream = s;
  }
  struct Restore {
    std::vector<Run*>& rs;
    std::vector<hipStream_t>& ss;
    ~Restore() {
      for (size_t i = 0; i < rs.size(); ++i) rs[i]->stream = ss[i];
    }
  } restore{all, saved};

  std::map<Run*, ipcs_step_stats*> st;
  std::map<Run*, int> rc;
  for (int i = 0; i < nruns; ++i) {
    st[all[i]] = stats ? &stats[i] : nullptr;
    if (stats) std::memset(&stats[i], 0, sizeof(ipcs_step_stats));
    rc[all[i]] = IPCS_OK;
  }
  auto alive = [&]() {
    std::vector<Run*> v;
    for (Run* r : all)
      if (rc[r] == IPCS_OK) v.push_back(r);
    return v;
  };
  auto mark = [&](int which) {
    for (Run* r : all)
      if (rc[r] != IPCS_OK && st[r] && st[r]->failed_solve == 0) st[r]->failed_solve = which;
  };
  // phase events: the batch's own, or (fixed memory) the first run's, which no
  // other work of that run uses during the batch
  hipEvent_t own[5] = {};
  hipEvent_t* e = mem.dev ? all[0]->ev : own;
  if (!mem.dev)
    for (auto& x : own) HIP_OK(hipEventCreate(&x));
  struct Ev {
    hipEvent_t* e;
    ~Ev() {
      for (int k = 0; k < 5; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    }
  } evguard{own};

  HIP_OK(hipEventRecord(e[0], s));
  for (Run* r : all) r->asm_phase();
  HIP_OK(hipEventRecord(e[1], s));
  solve_shared(alive(), 0, KMethod::BICG, s, rc, st, mem);
  mark(1);
  HIP_OK(hipEventRecord(e[2], s));
  std::vector<Run*> live = alive();
  std::vector<Run*> plain, mixed;
  for (Run* r : live) {
    r->pressure_rhs();
    (r->mixed ? mixed : plain).push_back(r);
  }
  solve_shared(plain, 1, KMethod::PCG, s, rc, st, mem);
  refine_shared(mixed, s, rc, st, mem);
  mark(2);
  for (Run* r : alive()) r->pressure_end();
  HIP_OK(hipEventRecord(e[3], s));
  live = alive();
  for (Run* r : live) r->correction_rhs();
  solve_shared(live, 2, KMethod::PCG, s, rc, st, mem);
  mark(3);
  live = alive();
  for (Run* r : live) r->correction_commit();
  HIP_OK(hipEventRecord(e[4], s));
  HIP_OK(hipEventSynchronize(e[4]));
  for (Run* r : live) r->finish_step(nullptr);
  float ms[4] = {};
  for (int k = 0; k < 4; ++k) HIP_OK(hipEventElapsedTime(&ms[k], e[k], e[k + 1]));
  int first = IPCS_OK;
  for (int i = 0; i < nruns; ++i) {
    Run* r = all[i];
    if (st[r]) {
      st[r]->status = rc[r];
      st[r]->t = r->t;
      st[r]->ms_asm = ms[0];
      st[r]->ms_mom = ms[1];
      st[r]->ms_p = ms[2];
      st[r]->ms_corr = ms[3];
    }
    if (first == IPCS_OK && rc[r] != IPCS_OK) first = rc[r];
  }
  return first;
}

}  // namespace ipcs
