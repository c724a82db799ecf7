// IPCS run: workspace layout, constant-matrix assembly, the three sub-steps of
// eq. (9) (Section 2.2.1) and the host side of the Krylov solves.
#include "run.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "builtin.hpp"
#include "common.hpp"
#include "rules.hpp"

namespace ipcs {

// Rows per thread of the matrix kernels: the fewest that keep a launch within
// KNB_MAX blocks (the partial-sum capacity). Where the vector kernels' blocks
// would re-read many records, the records are folded once (fold_for), so a
// larger matrix-kernel grid costs them nothing.
int kept_m_for(int64_t n, int ns) {
  const int64_t cap = KNB_MAX;
  for (int e : {1, 2, 4})
    if (div_up(n, (int64_t)KBS * e) <= cap) return e;
  if (div_up(n, (int64_t)KBS * 4) <= KNB_MAX) return 4;
  fail(IPCS_E_CAPACITY, "a Krylov system has more rows than one group supports");
}
int nblk_m_for(int64_t n, int ns) {
  return (int)std::max<int64_t>(1, div_up(n, (int64_t)KBS * kept_m_for(n, ns)));
}
constexpr int kMaxRefine = 30;   // mixed form: refinement passes

// Fold the partial-sum records once per group (KLaunch::fold) when the vector
// kernels' blocks would otherwise re-read more than kFoldBytes of records from
// L2 per launch (each block reads every record of the kernels before it).
constexpr double kFoldBytes = 16.0 * (1 << 20);
int fold_for(int64_t n, int ns) {
  const double nm = nblk_m_for(n, ns), nv = nblk_v_for(n, ns);
  return ns * (4.0 * nm + 2.0 * nv) * nv * 8.0 >= kFoldBytes ? 1 : 0;
}

int nblk_v_for(int64_t n, int ns) {
  const int64_t b = std::max<int64_t>(1, div_up(n, (int64_t)KBS * kept_v(ns)));
  if (b > KNB_MAX) fail(IPCS_E_CAPACITY, "a Krylov system has more rows than one group supports");
  return (int)b;
}

void build_bmap(const std::vector<int>& nblk, std::vector<int2>& bmap) {
  bmap.clear();
  int mx = 0;
  for (int b : nblk) mx = std::max(mx, b);
  for (int b = 0; b < mx; ++b)
    for (size_t g = 0; g < nblk.size(); ++g)
      if (b < nblk[g]) bmap.push_back(make_int2((int)g, b));
}

void xcd_order(std::vector<int2>& bmap) {
  constexpr int kXcd = 8;
  const int n = (int)bmap.size(), q = n / kXcd, rem = n % kXcd;
  std::vector<int2> out(n);
  for (int b = 0; b < n; ++b) {
    const int x = b % kXcd;
    out[b] = bmap[x * q + std::min(x, rem) + b / kXcd];
  }
  bmap.swap(out);
}

void xcd_chunks(std::vector<int2>& bmap, int chunk) {
  constexpr int kXcd = 8;
  const int n = (int)bmap.size();
  const int span = kXcd * chunk;
  std::vector<int2> out;
  out.reserve(n);
  // full spans: the k-th block of XCD x in span s is logical block
  // s*span + x*chunk + k
  const int full = n / span;
  for (int sp = 0; sp < full; ++sp)
    for (int k = 0; k < chunk; ++k)
      for (int x = 0; x < kXcd; ++x) out.push_back(bmap[sp * span + x * chunk + k]);
  for (int b = full * span; b < n; ++b) out.push_back(bmap[b]);   // tail in order
  bmap.swap(out);
}

// LDS a block may use on the current device (160 KiB on gfx950).
static size_t lds_limit() {
  int dev = 0, v = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  return v > 0 ? (size_t)v : 65536;
}

// LDS needed by the assembly kernel with bs rows per block: the largest
// number of SELL entries of the bs/64 slices a block owns, times the value size.
// The largest block that fits in 64 KiB (several blocks per CU); failing that,
// one 64-row block up to the device's limit (P3 rows on tetrahedra: 175
// entries, 89.6 KB of FP64 values per slice); failing that, lds 0: the row
// kernels accumulate in global memory.
static AsmCfg asm_cfg(const Sell& S, int vbytes) {
  auto need = [&](int bs) {
    int64_t mx = 0;
    const int per = bs / 64;
    for (int64_t s0 = 0; s0 < S.nslices; s0 += per) {
      const int64_t s1 = std::min<int64_t>(s0 + per, S.nslices);
      mx = std::max<int64_t>(mx, S.sptr[s1] - S.sptr[s0]);
    }
    return (size_t)mx * vbytes;
  };
  for (int bs : {256, 128, 64}) {
    const size_t lds = need(bs);
    if (lds <= 65536) return AsmCfg{bs, std::max<size_t>(lds, 8)};
  }
  const size_t lds = need(64);
  if (lds <= lds_limit()) return AsmCfg{64, lds};
  return AsmCfg{256, 0};
}

int status_to_code(int s) {
  switch (s) {
    case KS_MAXIT: return IPCS_E_NOT_CONVERGED;
    case KS_STALL: return IPCS_E_NOT_CONVERGED;
    case KS_BREAKDOWN: return IPCS_E_BREAKDOWN;
    case KS_NONFINITE: return IPCS_E_NONFINITE;
  }
  return IPCS_OK;
}

// Host side of a solve: start, then launch iterations in chunks and poll the
// status words between chunks. Chunks are sized from the previous solve of the
// same set: for one run the first one all of its length but a margin (a
// sixteenth, and at least the least chunk below), then half of the expected remaining
// iterations, but at least as many
// launches as take the device time one poll leaves idle (both measured with
// events in the previous solve; check_every before the first one, and never
// more than check_every). A solve
// that takes as long as the last one polls about 1 + log2 of the margin (in
// least chunks) times, and overshoots its convergence by about the cost of one
// poll. Past the expected
// length, or after a restart, chunks double from the least one. Launches past
// convergence are not free: kernels issue their loads before they read the
// status. Parity par alternates with every iteration launch.
static std::mutex g_pinned_mu;
static std::vector<KState*> g_pinned_free;

KState* pinned_take() {
  {
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      KState* p = g_pinned_free.back();
      g_pinned_free.pop_back();
      return p;
    }
  }
  KState* p = nullptr;
  HIP_OK(hipHostMalloc((void**)&p, sizeof(KState) * kPinnedStates, hipHostMallocDefault));
  return p;
}

void pinned_give(KState* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_pinned_mu);
  g_pinned_free.push_back(p);
}

LaunchEvents*& launch_events() {
  thread_local LaunchEvents* slot = nullptr;
  return slot;
}

KTimer::~KTimer() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

void KTimer::reset(uint32_t m) {
  mask = m;
  which.clear();
  for (int k = 0; k < IPCS_NKERNEL; ++k) {
    ms[k] = 0.0;
    cnt[k] = 0;
  }
}

void KTimer::drain() {
  for (size_t k = 0; k < which.size(); ++k) {
    float t = 0.f;
    HIP_OK(hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]));
    ms[which[k]] += t;
    cnt[which[k]] += 1;
  }
  which.clear();
}

// Timing events that bracket the chunks of a solve (per host thread, reused).
// From them a solve measures the device time per iteration launch and the gap
// a poll leaves on the device (the status read-back, the host's turn and the
// next launch), against which the least chunk of the next solve is sized.
static hipEvent_t* chunk_events(int n) {
  thread_local std::vector<hipEvent_t> pool;
  while ((int)pool.size() < n) {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool.data();
}
constexpr int kChunkEvents = 128;   // chunks timed per solve (the rest are not)

int krylov_solve(hipStream_t s, KSet& S, KMethod m, int check_every, std::vector<KState>& hs,
                 KState* pinned, KTimer& T, bool time_bursts) {
  // bursts of device work (the start, each chunk of iterations, each
  // confirmation) are bracketed by events while any are left: the gap between
  // the end of one burst and the start of the next is the cost of a poll
  hipEvent_t* ev = time_bursts ? chunk_events(2 * kChunkEvents) : nullptr;
  int nburst = 0, timed_launches = 0;
  double busy_ms = 0.0;
  std::vector<int> iter_burst;   // bursts that are chunks of iterations
  auto burst = [&](bool iters, auto work) {
    const bool timed = ev != nullptr && nburst < kChunkEvents;
    if (timed) HIP_OK(hipEventRecord(ev[2 * nburst], s));
    work();
    if (timed) {
      HIP_OK(hipEventRecord(ev[2 * nburst + 1], s));
      if (iters) iter_burst.push_back(nburst);
      ++nburst;
    }
    return timed;
  };
  const int nslot = S.L.ngroups * GMAX;
  hs.assign(nslot, KState{});
  auto fetch = [&]() {
    gather_states(s, S.L, S.d_poll);
    HIP_OK(hipMemcpyAsync(pinned, S.d_poll, sizeof(KState) * nslot, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    T.drain();
    for (int g = 0; g < S.L.ngroups; ++g)
      for (int j = 0; j < S.h_groups[g].nsys; ++j) hs[g * GMAX + j] = pinned[g * GMAX + j];
  };
  auto each = [&](auto f) {
    for (int g = 0; g < S.L.ngroups; ++g)
      for (int j = 0; j < S.h_groups[g].nsys; ++j) f(hs[g * GMAX + j]);
  };
  const bool fused = m == KMethod::PCG && S.fused;
  int ipl = fused ? S.F.ipl : 1;   // iterations per launch
  auto iterate = [&](int par) {
    if (fused) {
      T.run(s, S.kid[0], [&] { fcg_iter(s, S.F, par); });
    } else if (m == KMethod::PCG) {
      T.run(s, S.kid[0], [&] { pcg_spmv_only(s, S.L); });
      T.run(s, S.kid[1], [&] { pcg_update_only(s, S.L, par); });
    } else {
      T.run(s, S.kid[0], [&] { bicg_spmv_only(s, S.L); });
      T.run(s, S.kid[1], [&] { bicg_update_s_only(s, S.L, par); });
      T.run(s, S.kid[2], [&] { bicg_spmv_t_only(s, S.L); });
      T.run(s, S.kid[3], [&] { bicg_update_x_only(s, S.L, par); });
    }
  };
  int par = 0, launched = 0;
  auto start = [&](int mode) {
    if (fused) fcg_start(s, S.F, mode, par, launched);
    else if (m == KMethod::PCG) pcg_start(s, S.L, mode, par, launched);
    else bicg_start(s, S.L, mode, par, launched);
  };
  // groups with systems still iterating: the least remaining cap among them
  auto remaining = [&]() {
    int rem = -1;
    for (int g = 0; g < S.L.ngroups; ++g) {
      bool run = false;
      for (int j = 0; j < S.h_groups[g].nsys; ++j) run |= hs[g * GMAX + j].status == KS_RUN;
      if (run) rem = rem < 0 ? S.h_groups[g].maxit - launched
                             : std::min(rem, S.h_groups[g].maxit - launched);
    }
    return rem;
  };
  // block maps over the unfinished groups (sets of several groups): rebuilt
  // when finished groups hold at least a sixth of the launch's blocks.
  // A group's own blocks and partial sums are the same in every map, so
  // results do not depend on the compaction.
  std::vector<int2> cm, cv, cf;   // host copies, alive until the next sync
  const KLaunch L_full = S.L;
  const FLaunch F_full = S.F;
  auto compact = [&]() {
    if (!S.d_compact || S.L.ngroups < 2) return;
    std::vector<int> nm(S.L.ngroups, 0), nv(S.L.ngroups, 0), nf(S.L.ngroups, 0);
    int tm = 0;
    for (int g = 0; g < S.L.ngroups; ++g) {
      bool open = false;
      for (int j = 0; j < S.h_groups[g].nsys; ++j) {
        const int st = hs[g * GMAX + j].status;
        open |= st == KS_RUN || st == KS_PENDING || st == KS_RESTART;
      }
      if (!open) continue;
      nm[g] = S.h_groups[g].nblk_m;
      nv[g] = S.h_groups[g].nblk_v;
      if (fused) nf[g] = S.h_fgroups[g].nparts;
      tm += fused ? nf[g] : nm[g];
    }
    const int now = fused ? S.F.nblocks : S.L.nblocks_m;
    if (tm == 0 || 6 * (now - tm) < now) return;
    build_bmap(nm, cm);
    build_bmap(nv, cv);
    cf.clear();
    if (fused) {
      for (int g = 0; g < S.L.ngroups; ++g)
        for (int b = 0; b < nf[g]; ++b) cf.push_back(make_int2(g, b));
      xcd_order(cf);
    }
    const size_t need = cm.size() + cv.size() + cf.size();
    if ((int)need > S.compact_cap) return;
    int2* d = S.d_compact;
    HIP_OK(hipMemcpyAsync(d, cm.data(), sizeof(int2) * cm.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(d + cm.size(), cv.data(), sizeof(int2) * cv.size(),
                          hipMemcpyHostToDevice, s));
    if (!cf.empty())
      HIP_OK(hipMemcpyAsync(d + cm.size() + cv.size(), cf.data(), sizeof(int2) * cf.size(),
                            hipMemcpyHostToDevice, s));
    S.L.bmap_m = d;
    S.L.nblocks_m = (int)cm.size();
    S.L.bmap_v = d + cm.size();
    S.L.nblocks_v = (int)cv.size();
    if (fused) {
      S.F.bmap = d + cm.size() + cv.size();
      S.F.nblocks = (int)cf.size();
    }
  };
  burst(false, [&] { start(0); });
  fetch();
  const int every = std::max(1, check_every);
  const int least =
      S.us_per_launch > 0.0 && S.us_per_poll > 0.0
          ? std::max(1, std::min(every, (int)std::ceil(S.us_per_poll / S.us_per_launch)))
          : every;
  bool restarted = false;
  int tail = 0;   // polls made in the unknown tail of the solve
  auto iterations = [&]() {
    for (;;) {
      bool run = false;
      each([&](const KState& k) { run |= (k.status == KS_RUN); });
      if (!run) break;
      // groups whose cap is reached stop (on the device too), the others go on
      bool stopped = false;
      for (int g = 0; g < S.L.ngroups; ++g) {
        if (launched < S.h_groups[g].maxit) continue;
        bool here = false;
        for (int j = 0; j < S.h_groups[g].nsys; ++j) {
          KState& k = hs[g * GMAX + j];
          if (k.status == KS_RUN) {
            k.status = KS_MAXIT;
            here = true;
          }
        }
        if (here) stop_group(s, S.L, g);
        stopped |= here;
      }
      if (stopped) continue;
      const int rem = remaining();
      // after a restart, or past the previous solve's length, the remaining
      // iterations are unknown: chunks (of launches) grow geometrically from
      // the least one
      int chunk;
      if (restarted || launched >= S.last_iters) {
        chunk = least << std::min(tail, 10);
        ++tail;
      } else if (launched == 0 && S.L.ngroups == 1) {
        // (sets of several runs halve from the start: their runs end at
        // different counts, and a poll is where finished ones leave the launches)
        chunk = std::max(least, (S.last_iters - std::max(least * ipl, S.last_iters / 16)) / ipl);
      } else {
        chunk = std::max(least, (S.last_iters - launched) / 2 / ipl);
      }
      chunk = std::max(1, std::min(chunk, (rem + ipl - 1) / ipl));
      if (burst(true, [&] {
            for (int k = 0; k < chunk; ++k) {
              iterate(par);
              par ^= 1;
            }
          }))
        timed_launches += chunk;
      launched += chunk * ipl;
      fetch();
      compact();
      bool pend = false;
      each([&](const KState& k) { pend |= (k.status == KS_PENDING || k.status == KS_RESTART); });
      if (pend) {
        burst(false, [&] { start(1); });
        fetch();
        bool again = false;
        each([&](const KState& k) { again |= k.status == KS_RUN; });
        if (again && !restarted) tail = 0;
        restarted |= again;
      }
    }
  };
  iterations();
  // Two iterations per launch (s-step CG) reach a less accurate true residual
  // than one: where its checks stall above the tolerance, the system restarts
  // from its iterate with one iteration per launch, which takes it the rest
  // of the way. (A system alone and in a batch stalls at the same point, so
  // the switch keeps their results equal.)
  if (fused && ipl == 2) {
    bool any = false;
    for (int g = 0; g < S.L.ngroups; ++g)
      for (int j = 0; j < S.h_groups[g].nsys; ++j) {
        const int idx = g * GMAX + j;
        if (hs[idx].status != KS_STALL) continue;
        KState k = hs[idx];
        k.status = KS_RESTART;
        k.nstall = 0;
        pinned[idx] = k;
        hs[idx] = k;
        HIP_OK(hipMemcpyAsync(S.h_groups[g].v[j].st, &pinned[idx], sizeof(KState),
                              hipMemcpyHostToDevice, s));
        any = true;
      }
    if (any) {
      S.F.ipl = ipl = 1;
      burst(false, [&] { start(1); });
      fetch();
      if (!restarted) tail = 0;
      restarted = true;
      iterations();
    }
  }
  int iters = 0;
  each([&](const KState& k) { iters = std::max(iters, k.it); });
  S.last_iters = iters;   // the poll schedule of the next solve of this set
  S.L = L_full;           // the finish covers every group
  S.F = F_full;
  // the stream has synchronized (last fetch): every recorded event is done
  for (int k : iter_burst) {
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
    busy_ms += ms;
  }
  if (timed_launches > 0) S.us_per_launch = 1000.0 * busy_ms / timed_launches;
  if (nburst > 1) {
    double gaps = 0.0;
    for (int k = 1; k < nburst; ++k) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, ev[2 * k - 1], ev[2 * k]));
      gaps += ms;
    }
    S.us_per_poll = 1000.0 * gaps / (nburst - 1);
  }
  if (fused) fcg_finish(s, S.F);
  else ksys_finish(s, S.L);
  int rc = IPCS_OK;
  each([&](const KState& k) {
    const int c = status_to_code(k.status);
    if (rc == IPCS_OK && c != IPCS_OK) rc = c;
  });
  return rc;
}

// ------------------------------------------------------------------ layout
void Run::set_precision() {
  mixed = prm.precision == IPCS_MIXED;
  vsz = mixed ? 4 : 8;
}

void Run::sizes_from_mesh() {
  const Mesh& m = *mesh;
  dim = m.dim;
  n1 = m.n1;
  n2 = m.n2;
  nc = m.nc;
  nv = m.nv;
  nb = (int64_t)m.bidx.size();
  nlift = (int64_t)m.lift_slot.size();
  ne22 = m.e22.nent;
  ne21 = m.e21.nent;
  ne11 = m.e11.nent;
  ne12 = m.e12.nent;
  choose_poisson_form();
}

// Row blocks of the convection assembly (row-owner and local-sum passes) are
// dealt to the XCDs in runs of this many: consecutive rows share cells and
// velocity values, which one XCD's L2 then serves
constexpr int kAsmXcdChunk = 8;

// Largest own + halo row count of a part the fused Poisson CG keeps in LDS
// (8 bytes each, under 64 KiB with the kernel's static reduction space).
constexpr int kFcgLocalMax = 8000;
// Default part size: about 2-3 parts per CU on the 2D and 3D workloads; the
// block streams its own rows once and gathers its halo from neighbours that
// the block map places on the same XCD.
constexpr int kFcgRows = 384;

// The pressure Poisson CG runs one kernel per iteration on a row partition of
// Kp when its parts fit (LDS, partial-sum capacity); otherwise two kernels.
void Run::choose_poisson_form() {
  pp.reset();
  fcg_ept = 0;
  fcg_s = 1;
  f_blk_ok = false;
  const int req = prm.poisson_part_rows;
  if (req < 0) return;
  const int s = prm.poisson_s == 2 ? 2 : 1;
  auto q = mesh->parts11(req > 0 ? req : kFcgRows, s);
  int biggest = 0;
  for (int p = 0; p < q->nparts; ++p)
    biggest = std::max(biggest, q->part_ptr[p + 1] - q->part_ptr[p]);
  // LDS of a block (8 bytes per local value): one iteration per launch, u
  // over own and halo rows; two, p and z over own, halo and second ring and
  // B p over own and halo rows
  const int64_t local = s == 2 ? 2 * (int64_t)q->lds2_max + q->lds_max : q->lds_max;
  const bool fits = local <= kFcgLocalMax && q->nparts <= KNB_MAX;
  if (!fits) {
    if (req > 0 || s == 2)
      fail(IPCS_E_CAPACITY, "the Poisson partition's parts reference more rows than fit in LDS");
    return;
  }
  fcg_s = s;
  pp = q;
  for (int e : {1, 2, 4, 8})
    if (KBS * e >= biggest) {
      fcg_ept = e;
      break;
    }
  int most_slices = 0;
  for (int p = 0; p < q->nparts; ++p)
    most_slices = std::max(most_slices, q->slice_ptr[p + 1] - q->slice_ptr[p]);
  f_blk_ok = most_slices <= FBLK_SL;
}

void Run::layout(Carver& c) {
  const Mesh& m = *mesh;
  const int nsys = 2 * dim + 1;
  X = c.take<double>(nv * dim);
  c2d = c.take<int32_t>(nc * m.nloc2);
  c2v = c.take<int32_t>(nc * m.nloc1);
  x2 = c.take<double>(n2 * dim);
  xp = m.pair == IPCS_PAIR_P2P1 ? X : c.take<double>(n1 * dim);
  bmask = c.take<uint8_t>(n2);
  bidx = c.take<int32_t>(std::max<int64_t>(nb, 1));
  sp22 = c.take<int32_t>(m.e22.nslices + 1);
  col22 = c.take<int32_t>(ne22);
  rp22 = c.take<int32_t>(n2 + 1);
  sp21 = c.take<int32_t>(m.e21.nslices + 1);
  col21 = c.take<int32_t>(ne21);
  rp21 = c.take<int32_t>(n2 + 1);
  sp11 = c.take<int32_t>(m.e11.nslices + 1);
  col11 = c.take<int32_t>(ne11);
  rp11 = c.take<int32_t>(n1 + 1);
  sp12 = c.take<int32_t>(m.e12.nslices + 1);
  col12 = c.take<int32_t>(ne12);
  rp12 = c.take<int32_t>(n1 + 1);
  inc2p = c.take<int32_t>(n2 + 1);
  inc2 = c.take<int32_t>((int64_t)m.inc2.code.size());
  inc1p = c.take<int32_t>(n1 + 1);
  inc1 = c.take<int32_t>((int64_t)m.inc1.code.size());
  s22 = c.take<uint8_t>((int64_t)m.s22.slot.size());
  s21 = c.take<uint8_t>((int64_t)m.s21.slot.size());
  s11 = c.take<uint8_t>((int64_t)m.s11.slot.size());
  s12 = c.take<uint8_t>((int64_t)m.s12.slot.size());
  lift_ptr = c.take<int32_t>(n2 + 1);
  lift_slot = c.take<int32_t>(std::max<int64_t>(nlift, 1));
  lift_col = c.take<int32_t>(std::max<int64_t>(nlift, 1));
  auto vals = [&](int64_t n) -> void* { return c.take<char>(n * vsz); };
  M = vals(ne22);
  K = vals(ne22);
  E = vals(ne22);
  Eloc = two_pass_conv() ? c.take<char>(nc * (int64_t)m.nloc2 * m.nloc2 * vsz) : nullptr;
  Ael = vals(ne22);
  Mel = vals(ne22);
  Kp = vals(ne11);
  Kp64 = mixed ? c.take<double>(ne11) : static_cast<double*>(Kp);
  for (int k = 0; k < 3; ++k) {
    // the divergence matrices stay FP64 in both forms (Run::assemble_constant)
    Dc[k] = k < dim ? c.take<double>(ne12) : nullptr;
    Gc[k] = k < dim ? vals(ne21) : nullptr;
  }
  liftA = c.take<double>(std::max<int64_t>(nlift, 1));
  liftM = c.take<double>(std::max<int64_t>(nlift, 1));
  dinvA = c.take<double>(n2);
  dinvM = c.take<double>(n2);
  dinvKp = c.take<double>(n1);
  w = c.take<double>(n1);
  U = c.take<double>(dim * n2);
  Unew = c.take<double>(dim * n2);
  Ustar = c.take<double>(dim * n2);
  bU = c.take<double>(dim * n2);
  F = c.take<double>(dim * n2);
  gfull = c.take<double>(dim * n2);
  for (auto& h : Ush) h = extrap_m() ? c.take<double>(dim * n2) : nullptr;
  P = c.take<double>(n1);
  dP = c.take<double>(n1);
  rP = c.take<double>(n1);
  kv2 = c.take<double>(8 * dim * n2);
  kv1 = c.take<double>(5 * n1);
  rIR = mixed ? c.take<double>(n1) : nullptr;
  dIR = mixed ? c.take<double>(n1) : nullptr;
  kst = c.take<KState>(nsys);
  kgroups = c.take<KGroup>(3);
  for (int gi = 0; gi < 3; ++gi) {
    const int64_t n = gi == 1 ? n1 : n2;
    const int ns = gi == 1 ? 1 : dim;
    const int bm = nblk_m_for(n, ns), bv = nblk_v_for(n, ns);
    part_m[gi] = c.take<double>((int64_t)bm * GMAX * KP);
    part_v[gi][0] = c.take<double>((int64_t)bv * GMAX * KP);
    part_v[gi][1] = c.take<double>((int64_t)bv * GMAX * KP);
    fold[gi] = c.take<double>((int64_t)GMAX * KP);
    bmap_m[gi] = c.take<int2>(bm);
    bmap_v[gi] = c.take<int2>(bv);
  }
  poll = c.take<KState>(3 * GMAX);
  if (pp) {
    const PartSell& q = *pp;
    f_perm = c.take<int32_t>(n1);
    f_part_ptr = c.take<int32_t>(q.nparts + 1);
    f_halo_ptr = c.take<int32_t>(q.nparts + 1);
    f_halo = c.take<int32_t>(std::max<int64_t>((int64_t)q.halo.size(), 1));
    f_slice_ptr = c.take<int32_t>(q.nparts + 1);
    f_sptr = c.take<int32_t>((int64_t)q.sptr.size());
    f_src = c.take<int32_t>(std::max<int64_t>(q.nent, 1));
    f_lcol = c.take<uint16_t>(std::max<int64_t>(q.nent, 1));
    f_val = c.take<char>(std::max<int64_t>(q.nent, 1) * vsz);
    f_dinv = c.take<double>(n1);
    f_bp = c.take<double>(n1);
    f_xp = c.take<double>(n1);
    f_p = c.take<double>(n1);
    f_vec = c.take<double>(6 * n1);
    // partials: 3 values per part (one iteration per launch), or the 16 of the
    // Gram matrix and ||r||^2 (two)
    const int kp = fcg_s == 2 ? 2 * KP : KP;
    for (int k = 0; k < 2; ++k) f_part[k] = c.take<double>((int64_t)kp * q.nparts);
    f_part_s = c.take<double>((int64_t)KP * q.nparts);
    f_bmap = c.take<int2>(q.nparts);
    f_blk = c.take<FBlk>(q.nparts);
    f_hfirst = c.take<int32_t>((int64_t)KBS * q.nparts);
    if (fcg_s == 2) {
      f_h2ptr = c.take<int32_t>(q.nparts + 1);
      f_h2 = c.take<int32_t>(std::max<int64_t>((int64_t)q.halo2.size(), 1));
      f_hsl = c.take<int32_t>(q.nparts + 1);
      f_hsptr = c.take<int32_t>((int64_t)q.hsptr.size());
      f_hsrc = c.take<int32_t>(std::max<int64_t>(q.hnent, 1));
      f_hlcol = c.take<uint16_t>(std::max<int64_t>(q.hnent, 1));
      f_hval = c.take<char>(std::max<int64_t>(q.hnent, 1) * vsz);
      f_y = c.take<double>(10 * n1);
    }
    fgroup = c.take<FGroup>(1);
  }
  spart = c.take<double>(8192 * 2);
  scnt = c.take<uint32_t>(4);
  scal = c.take<double>(8);
  gb = c.take<double>(std::max<int64_t>(nb, 1) * dim);
  fq = c.take<double>(prm.callbacks ? (int64_t)dim * nc * cell_nq() : 1);
}

Run::~Run() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  pinned_give(pinned);
}

template <class T>
static void up(hipStream_t s, T* dst, const std::vector<T>& src) {
  if (!src.empty())
    HIP_OK(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s));
}

void Run::upload_mesh() {
  const Mesh& m = *mesh;
  up(stream, X, m.X);
  up(stream, c2d, m.c2d);
  up(stream, c2v, m.c2dp);
  up(stream, x2, m.x2);
  if (xp != X) up(stream, xp, m.xp);
  up(stream, bmask, m.bmask);
  up(stream, bidx, m.bidx);
  up(stream, sp22, m.e22.sptr);
  up(stream, col22, m.e22.col);
  up(stream, rp22, m.p22.rowptr);
  up(stream, sp21, m.e21.sptr);
  up(stream, col21, m.e21.col);
  up(stream, rp21, m.p21.rowptr);
  up(stream, sp11, m.e11.sptr);
  up(stream, col11, m.e11.col);
  up(stream, rp11, m.p11.rowptr);
  up(stream, sp12, m.e12.sptr);
  up(stream, col12, m.e12.col);
  up(stream, rp12, m.p12.rowptr);
  up(stream, inc2p, m.inc2.ptr);
  up(stream, inc2, m.inc2.code);
  up(stream, inc1p, m.inc1.ptr);
  up(stream, inc1, m.inc1.code);
  up(stream, s22, m.s22.slot);
  up(stream, s21, m.s21.slot);
  up(stream, s11, m.s11.slot);
  up(stream, s12, m.s12.slot);
  up(stream, lift_ptr, m.lift_ptr);
  up(stream, lift_slot, m.lift_slot);
  up(stream, lift_col, m.lift_col);
  if (pp) {
    const PartSell& q = *pp;
    up(stream, f_perm, q.perm);
    up(stream, f_part_ptr, q.part_ptr);
    up(stream, f_halo_ptr, q.halo_ptr);
    up(stream, f_halo, q.halo);
    up(stream, f_slice_ptr, q.slice_ptr);
    up(stream, f_sptr, q.sptr);
    up(stream, f_src, q.src);
    up(stream, f_lcol, q.lcol);
    if (fcg_s == 2) {
      up(stream, f_h2ptr, q.halo2_ptr);
      up(stream, f_h2, q.halo2);
      up(stream, f_hsl, q.hslice_ptr);
      up(stream, f_hsptr, q.hsptr);
      up(stream, f_hsrc, q.hsrc);
      up(stream, f_hlcol, q.hlcol);
    }
    std::vector<int2> bm(q.nparts);
    for (int p = 0; p < q.nparts; ++p) bm[p] = make_int2(0, p);
    xcd_order(bm);
    up(stream, f_bmap, bm);
    // per-block descriptors and first halo rows, in the block map's order
    std::vector<FBlk> blk(q.nparts);
    std::vector<int32_t> hf((size_t)KBS * q.nparts, 0);
    for (int b = 0; b < q.nparts; ++b) {
      const int lb = bm[b].y;
      FBlk& d = blk[b];
      std::memset(&d, 0, sizeof(d));
      d.lb = lb;
      d.p0 = q.part_ptr[lb];
      d.own = q.part_ptr[lb + 1] - d.p0;
      d.h0 = q.halo_ptr[lb];
      d.nh = q.halo_ptr[lb + 1] - d.h0;
      const int s0 = q.slice_ptr[lb];
      d.ns = q.slice_ptr[lb + 1] - s0;
      for (int k = 0; k < FBLK_SL; ++k) {
        const int sl = s0 + std::min(k, d.ns - 1);
        d.sl[k] = make_int2(q.sptr[sl], k < d.ns ? (q.sptr[sl + 1] - q.sptr[sl]) / 64 : 0);
      }
      for (int t = 0; t < std::min(d.nh, KBS); ++t) hf[(size_t)b * KBS + t] = q.halo[d.h0 + t];
    }
    up(stream, f_blk, blk);
    up(stream, f_hfirst, hf);
    // bm, blk, hf are stack copies: the transfers must end before they go away
    HIP_OK(hipStreamSynchronize(stream));
  }
}

void Run::assemble_constant() {
  const Mesh& m = *mesh;
  RowAsm a22{(int32_t)n2, sp22, inc2p, inc2, s22, m.s22.stride, c2d, m.nloc2, X, {M, K, nullptr},
             m.pair, c2v, m.nloc1};
  asm_mass_stiff(dim, mixed, stream, a22, cfg_mk.bs, cfg_mk.lds);
  RowAsm a21{(int32_t)n2, sp21, inc2p, inc2, s21, m.s21.stride, c2d, m.nloc2, X,
             {Gc[0], Gc[1], Gc[2]}, m.pair, c2v, m.nloc1};
  asm_grad(dim, mixed, stream, a21, cfg_g.bs, cfg_g.lds);
  // D_c is assembled and stored in FP64 in both forms. The pressure
  // right-hand side -(rho/dt) sum_c D_c U*_c is a sum of terms that cancel to
  // within a factor ~1e7 of their magnitudes at 512^2 (U* is nearly
  // divergence-free), so FP32 values would leave it with rounding noise of
  // the order of the result itself. One FP64 product per step costs little.
  RowAsm a12{(int32_t)n1, sp12, inc1p, inc1, s12, m.s12.stride, c2d, m.nloc2, X,
             {Dc[0], Dc[1], Dc[2]}, m.pair, c2v, m.nloc1};
  asm_div(dim, false, stream, a12, cfg_d.bs, cfg_d.lds);
  // Kp is assembled in FP64 in both forms. The mixed form keeps that FP64
  // copy for the refinement residual and gives the inner CG the same matrix
  // rounded to FP32, the FP32 operator closest to it, so that a refinement
  // pass is limited by the inner tolerance rather than by the operator.
  RowAsm a11{(int32_t)n1, sp11, inc1p, inc1, s11, m.s11.stride, c2d, m.nloc2, X,
             {Kp64, nullptr, nullptr}, m.pair, c2v, m.nloc1};
  const AsmCfg kp64 = asm_cfg(mesh->e11, 8);   // FP64 values in both forms
  asm_kp(dim, false, stream, a11, kp64.bs, kp64.lds);
  if (mixed) round_to_f32(stream, ne11, Kp64, static_cast<float*>(Kp));
  asm_lumped_p1(dim, stream, a11, w);
  inv_diagonal(stream, mixed, n1, sp11, rp11, col11, Kp, dinvKp);
  if (pp) {
    fcg_gather_values(stream, mixed, pp->nent, f_src, Kp, f_val);
    if (fcg_s == 2 && pp->hnent > 0) fcg_gather_values(stream, mixed, pp->hnent, f_hsrc, Kp, f_hval);
    fcg_gather_dinv(stream, n1, f_perm, dinvKp, f_dinv);
  }
  form_eliminated(stream, mixed, n2, sp22, rp22, col22, bmask, M, nullptr, 1.0, 0.0, Mel, dinvM);
  lift_values(stream, mixed, nlift, lift_slot, M, nullptr, 1.0, 0.0, liftM);
}

void Run::reform_A() {
  form_eliminated(stream, mixed, n2, sp22, rp22, col22, bmask, M, K, 1.0 / prm.dt, prm.nu, Ael,
                  dinvA);
  lift_values(stream, mixed, nlift, lift_slot, M, K, 1.0 / prm.dt, prm.nu, liftA);
  bi.nu = prm.nu;
  A_dirty = false;
}

static KState fresh_state(double tol, int /*maxit*/) {
  KState k;
  std::memset(&k, 0, sizeof(k));
  k.tol2 = tol * tol;
  k.status = KS_DONE;
  return k;
}

void Run::setup_solvers() {
  const int nsys = 2 * dim + 1;
  std::vector<KState> st(nsys);
  std::vector<KGroup> grp(3);
  for (int gi = 0; gi < 3; ++gi) {
    KGroup& g = grp[gi];
    std::memset(&g, 0, sizeof(g));
    const int64_t n = gi == 1 ? n1 : n2;
    g.n = (int32_t)n;
    g.nblk_m = nblk_m_for(n, gi == 1 ? 1 : dim);
    g.nblk_v = nblk_v_for(n, gi == 1 ? 1 : dim);
    g.maxit = prm.maxit;
    g.part_m = part_m[gi];
    g.part_v[0] = part_v[gi][0];
    g.part_v[1] = part_v[gi][1];
    g.fold = fold[gi];
    if (gi == 1) {   // pressure Poisson: Kp dP = r (mixed: Kp d = refinement residual)
      g.nsys = 1;
      g.sptr = sp11;
      g.col = col11;
      g.val = Kp;
      g.dinv = dinvKp;
      KVecs& V = g.v[0];
      V.b = mixed ? rIR : rP;
      V.x = mixed ? dIR : dP;
      V.r = kv1;
      V.u = kv1 + n1;
      V.p = kv1 + 2 * n1;
      V.s = kv1 + 3 * n1;
      V.w = kv1 + 4 * n1;
      V.st = kst + dim;
      st[dim] = fresh_state(prm.tol_p, prm.maxit);
      continue;
    }
    const bool mom = gi == 0;
    g.nsys = dim;
    g.sptr = sp22;
    g.col = col22;
    g.val = mom ? Ael : Mel;
    g.dinv = mom ? dinvA : dinvM;
    // r, p, s, w, t per component; u, phat, shat interleaved over the
    // components (the vectors the SpMVs gather)
    double* il = kv2 + (size_t)5 * dim * n2;
    for (int c = 0; c < dim; ++c) {
      double* base = kv2 + (size_t)c * 5 * n2;
      KVecs& V = g.v[c];
      V.b = bU + (size_t)c * n2;
      V.x = (mom ? Ustar : Unew) + (size_t)c * n2;
      V.r = base;
      V.p = base + n2;
      V.s = base + 2 * n2;
      V.w = base + 3 * n2;
      V.t = base + 4 * n2;
      V.u = il + c;
      V.phat = il + (size_t)dim * n2 + c;
      V.shat = il + (size_t)2 * dim * n2 + c;
      const int sidx = mom ? c : dim + 1 + c;
      V.st = kst + sidx;
      st[sidx] = fresh_state(mom ? prm.tol_mom : prm.tol_corr, prm.maxit);
    }
  }
  HIP_OK(hipMemcpyAsync(kgroups, grp.data(), sizeof(KGroup) * 3, hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(kst, st.data(), sizeof(KState) * nsys, hipMemcpyHostToDevice, stream));
  std::vector<std::vector<int2>> maps_m(3), maps_v(3);
  auto mk = [&](KSet& S, int gi) {
    S.h_groups = {grp[gi]};
    build_bmap({grp[gi].nblk_m}, maps_m[gi]);
    build_bmap({grp[gi].nblk_v}, maps_v[gi]);
    // matrix kernels gather from a band of rows around their own: runs of 8
    // consecutive row blocks per XCD share those gathers in its L2 (one
    // contiguous range per XCD instead is slower: the 8 streams at a stride
    // of 1/8 of the matrix contend for the same memory channels)
    xcd_chunks(maps_m[gi], 8);
    HIP_OK(hipMemcpyAsync(bmap_m[gi], maps_m[gi].data(), sizeof(int2) * maps_m[gi].size(),
                          hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(bmap_v[gi], maps_v[gi].data(), sizeof(int2) * maps_v[gi].size(),
                          hipMemcpyHostToDevice, stream));
    S.L = KLaunch{kgroups + gi,      1, grp[gi].nsys, kept_m_for(grp[gi].n, grp[gi].nsys), mixed ? 1 : 0,
                  bmap_m[gi],        (int)maps_m[gi].size(),
                  bmap_v[gi],        (int)maps_v[gi].size(),
                  fold_for(grp[gi].n, grp[gi].nsys)};
    S.d_poll = poll + gi * GMAX;
    S.last_iters = 0;
  };
  mk(set_mom, 0);
  mk(set_p, 1);
  mk(set_corr, 2);
  set_p.fused = pp != nullptr;
  if (pp) {
    const KVecs& V = grp[1].v[0];
    FGroup f;
    std::memset(&f, 0, sizeof(f));
    f.n = (int32_t)n1;
    f.nparts = pp->nparts;
    f.perm = f_perm;
    f.part_ptr = f_part_ptr;
    f.halo_ptr = f_halo_ptr;
    f.halo = f_halo;
    f.slice_ptr = f_slice_ptr;
    f.sptr = f_sptr;
    f.lcol = f_lcol;
    f.val = f_val;
    f.dinv = f_dinv;
    f.b = V.b;
    f.x = V.x;
    f.bp = f_bp;
    f.xp = f_xp;
    f.p = f_p;
    for (int k = 0; k < 2; ++k) {
      f.r[k] = f_vec + (size_t)k * n1;
      f.s[k] = f_vec + (size_t)(2 + k) * n1;
      f.w[k] = f_vec + (size_t)(4 + k) * n1;
      f.part[k] = f_part[k];
    }
    f.part_s = f_part_s;
    f.st = V.st;
    f.maxit = prm.maxit;
    f.ipl = fcg_s;
    if (fcg_s == 2) {
      f.halo2_ptr = f_h2ptr;
      f.halo2 = f_h2;
      f.hslice_ptr = f_hsl;
      f.hsptr = f_hsptr;
      f.hlcol = f_hlcol;
      f.hval = f_hval;
      f.y[0] = f_y;
      f.y[1] = f_y + 5 * (size_t)n1;
    }
    set_p.h_fgroups = {f};
    HIP_OK(hipMemcpyAsync(fgroup, set_p.h_fgroups.data(), sizeof(f), hipMemcpyHostToDevice,
                          stream));
    set_p.F = FLaunch{fgroup, 1, fcg_ept, mixed ? 1 : 0, f_bmap, pp->nparts,
                      sizeof(double) * (size_t)pp->lds_max};
    set_p.F.ipl = fcg_s;
    // two iterations per launch: p and z over own, halo and second ring, B p
    // over own and halo rows
    if (fcg_s == 2) set_p.F.lds = sizeof(double) * (size_t)(2 * pp->lds2_max + pp->lds_max);
    if (f_blk_ok && fcg_s == 1) {
      set_p.F.blk = f_blk;
      set_p.F.hfirst = f_hfirst;
      set_p.F.one = f;
    }
  }
  const int kid_mom[4] = {IPCS_KERNEL_BICG_SPMV, IPCS_KERNEL_BICG_UPDATE_S,
                          IPCS_KERNEL_BICG_SPMV_T, IPCS_KERNEL_BICG_UPDATE_X};
  for (int k = 0; k < 4; ++k) set_mom.kid[k] = kid_mom[k];
  set_p.kid[0] = pp ? IPCS_KERNEL_PCG_FUSED_P : IPCS_KERNEL_PCG_SPMV_P;
  set_p.kid[1] = pp ? -1 : IPCS_KERNEL_PCG_UPDATE_P;
  set_corr.kid[0] = IPCS_KERNEL_PCG_SPMV_M;
  set_corr.kid[1] = IPCS_KERNEL_PCG_UPDATE_M;
  HIP_OK(hipStreamSynchronize(stream));
}

void Run::create(std::shared_ptr<const Mesh> m, const ipcs_params& p, void* ws, int64_t bytes,
                 hipStream_t s) {
  mesh = std::move(m);
  prm = p;
  stream = s;
  set_precision();
  sizes_from_mesh();
  const Mesh& mm = *mesh;
  cfg_mk = asm_cfg(mm.e22, vsz);
  cfg_e = asm_cfg(mm.e22, vsz);
  cfg_g = asm_cfg(mm.e21, vsz);
  cfg_d = asm_cfg(mm.e12, 8);
  cfg_kp = asm_cfg(mm.e11, vsz);
  Carver meas;
  layout(meas);
  if (!ws || bytes < meas.off)
    fail(IPCS_E_NOMEM, "workspace too small: need " + std::to_string(meas.off) + " bytes");
  Carver c;
  c.base = static_cast<char*>(ws);
  layout(c);
  ws_bytes = bytes;
  pinned = pinned_take();
  for (auto& e : ev) HIP_OK(hipEventCreate(&e));
  upload_mesh();
  // value arrays: SELL padding entries must read as zero
  for (void* v : {M, K, E, Ael, Mel}) HIP_OK(hipMemsetAsync(v, 0, (size_t)vsz * ne22, stream));
  HIP_OK(hipMemsetAsync(Kp, 0, (size_t)vsz * ne11, stream));
  if (mixed) {
    HIP_OK(hipMemsetAsync(Kp64, 0, sizeof(double) * ne11, stream));
    HIP_OK(hipMemsetAsync(rIR, 0, sizeof(double) * n1, stream));
    HIP_OK(hipMemsetAsync(dIR, 0, sizeof(double) * n1, stream));
  }
  for (int k = 0; k < dim; ++k) {
    HIP_OK(hipMemsetAsync(Dc[k], 0, sizeof(double) * ne12, stream));
    HIP_OK(hipMemsetAsync(Gc[k], 0, (size_t)vsz * ne21, stream));
  }
  const size_t vbytes = sizeof(double) * dim * n2;
  for (double* v : {U, Unew, Ustar, bU, F, gfull}) HIP_OK(hipMemsetAsync(v, 0, vbytes, stream));
  for (double* v : {P, dP, rP}) HIP_OK(hipMemsetAsync(v, 0, sizeof(double) * n1, stream));
  // Krylov vectors start finite (gathers of padding columns read them)
  HIP_OK(hipMemsetAsync(kv2, 0, sizeof(double) * 8 * dim * n2, stream));
  HIP_OK(hipMemsetAsync(kv1, 0, sizeof(double) * 5 * n1, stream));
  HIP_OK(hipMemsetAsync(scal, 0, sizeof(double) * 8, stream));
  assemble_constant();
  reform_A();
  setup_solvers();
  t = prm.t0;
  if (prm.callbacks) {
    const int nq = cell_nq();
    std::vector<double> lam((size_t)nq * (dim + 1)), wq(nq);
    if (mm.pair == IPCS_PAIR_P3P2 && dim == 3) tet_rule9(lam.data(), wq.data());
    else
      for (int q = 0; q < nq; ++q)
        for (int k = 0; k <= dim; ++k)
          lam[(size_t)q * (dim + 1) + k] = mm.pair == IPCS_PAIR_P3P2 ? RuleT9::lam(q, k)
                                           : dim == 2               ? Rule<2>::lam(q, k)
                                                                    : Rule<3>::lam(q, k);
    h_xq.resize((size_t)nc * nq * dim);
    for (int64_t cc = 0; cc < nc; ++cc)
      for (int q = 0; q < nq; ++q)
        for (int r = 0; r < dim; ++r) {
          double x = 0.0;
          for (int k = 0; k <= dim; ++k)
            x += lam[(size_t)q * (dim + 1) + k] * mm.X[(size_t)mm.c2dp[cc * mm.nloc1 + k] * dim + r];
          h_xq[((size_t)cc * nq + q) * dim + r] = x;
        }
  }
  h_xb.resize((size_t)nb * dim);
  for (int64_t k = 0; k < nb; ++k)
    for (int r = 0; r < dim; ++r) h_xb[k * dim + r] = mm.x2[(size_t)mm.bidx[k] * dim + r];
  HIP_OK(hipStreamSynchronize(stream));
}

void Run::set_builtin(int kind, const double* p, int np) {
  const bool ok2 = kind == IPCS_SOL_TAYLOR_GREEN_2D || kind == IPCS_SOL_JOHN_2D ||
                   kind == IPCS_SOL_POLY_STEADY_2D || kind == IPCS_SOL_POLY_CUBIC_2D;
  const bool ok3 = kind == IPCS_SOL_BELTRAMI_3D || kind == IPCS_SOL_POLY_STEADY_3D ||
                   kind == IPCS_SOL_POLY_CUBIC_3D;
  if (!((dim == 2 && ok2) || (dim == 3 && ok3)))
    fail(IPCS_E_INVALID, "built-in solution kind does not match the mesh dimension");
  Builtin b{};
  b.kind = kind;
  b.nu = prm.nu;
  if (kind == IPCS_SOL_TAYLOR_GREEN_2D) b.prm[0] = M_PI;
  if (kind == IPCS_SOL_BELTRAMI_3D) {
    b.prm[0] = M_PI / 4;
    b.prm[1] = M_PI / 2;
  }
  for (int i = 0; i < std::min(np, 4); ++i) b.prm[i] = p[i];
  bi = b;
  f_cb = g_cb = nullptr;
  eval_velocity(stream, dim, bi, x2, n2, t, U, n2);
  eval_pressure(stream, dim, bi, xp, n1, t, P);
  sub_weighted_mean(stream, n1, w, P, spart, scal + 2);
  clear_history();
  phase_next = IPCS_PHASE_ASM;
  HIP_OK(hipStreamSynchronize(stream));
}

void Run::set_state(const double* u, const double* p, double tt) {
  HIP_OK(hipMemcpyAsync(U, u, sizeof(double) * dim * n2, hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(P, p, sizeof(double) * n1, hipMemcpyHostToDevice, stream));
  clear_history();
  HIP_OK(hipStreamSynchronize(stream));
  t = tt;
  phase_next = IPCS_PHASE_ASM;
}

void fill_stats_solve(const std::vector<KState>& hs, int nsys, int which, ipcs_step_stats* st) {
  if (!st) return;
  for (int c = 0; c < nsys; ++c) {
    const KState& k = hs[c];
    const double res = k.bb > 0 ? std::sqrt(k.rr / k.bb) : 0.0;
    if (which == 1) {
      st->it_mom[c] = k.it;
      st->res_mom[c] = res;
    } else if (which == 2) {
      st->it_p = k.it;
      st->res_p = res;
      st->checks_p = k.nchecks;
    } else {
      st->it_corr[c] = k.it;
      st->res_corr[c] = res;
    }
  }
}

// Step pieces shared by single runs and batches (all on the run's stream).

// Dirichlet data and forcing at t^{n+1}, the convection term, momentum RHS, U* start.
// Explicit (eq. (9) as printed): E = M/dt - C(U^n) and b = E U^n - G P^n + F;
// A = M/dt + nu K is constant. Semi-implicit: E = M/dt + C(U^n), A = E + nu K
// with its Dirichlet elimination and lifting re-formed every step, and
// b = M U^n / dt - G P^n + F.
void Run::asm_phase() {
  const bool semi = prm.convection == IPCS_CONV_SEMI_IMPLICIT;
  if (A_dirty && !semi) reform_A();
  bi.nu = prm.nu;
  t1 = t + prm.dt;
  HIP_OK(hipEventRecord(ev[0], stream));
  if (g_cb) {
    std::vector<double> vals((size_t)nb * dim);
    g_cb(g_ctx, dim, nb, h_xb.data(), t1, vals.data());
    HIP_OK(hipMemcpyAsync(gb, vals.data(), sizeof(double) * vals.size(), hipMemcpyHostToDevice,
                          stream));
    dirichlet_scatter(stream, dim, gb, bidx, nb, gfull, n2);
    HIP_OK(hipStreamSynchronize(stream));
  } else if (bi.kind) {
    dirichlet_builtin(stream, dim, bi, x2, bidx, nb, t1, gfull, n2);
  }
  const Mesh& m = *mesh;
  RowAsm a22{(int32_t)n2, sp22, inc2p, inc2, s22, m.s22.stride, c2d, m.nloc2, X,
             {E, nullptr, nullptr}, m.pair, c2v, m.nloc1, kAsmXcdChunk};
  has_F = false;
  if (f_cb) {
    const int nq = cell_nq();
    std::vector<double> vals((size_t)nc * nq * dim), tr(vals.size());
    f_cb(f_ctx, dim, nc * nq, h_xq.data(), t1, vals.data());
    for (int64_t i = 0; i < nc * nq; ++i)
      for (int c = 0; c < dim; ++c) tr[(size_t)c * nc * nq + i] = vals[i * dim + c];
    HIP_OK(hipMemcpyAsync(fq, tr.data(), sizeof(double) * tr.size(), hipMemcpyHostToDevice,
                          stream));
    asm_forcing(dim, stream, a22, bi, fq, nc, t1, F, n2);
    HIP_OK(hipStreamSynchronize(stream));
    has_F = true;
  } else if (builtin_has_force(bi.kind)) {
    asm_forcing(dim, stream, a22, bi, nullptr, nc, t1, F, n2);
    has_F = true;
  }
  // 3D and the P3-P2 pair: cell-batched local matrices, then their row-owner
  // sum; P2-P1 in 2D: one row-owner pass (cheaper where a cell has 6 rows and
  // 7 quadrature points)
  const double cs = semi ? 1.0 : -1.0;
  if (two_pass_conv()) {
    timer.run(stream, IPCS_KERNEL_ASM_CONV,
              [&] { asm_conv_cells(dim, mixed, stream, a22, nc, U, n2, 1.0 / prm.dt, cs, Eloc); });
    timer.run(stream, IPCS_KERNEL_ASM_SUM,
              [&] { asm_local_sum(dim, mixed, stream, a22, cfg_e.bs, cfg_e.lds, Eloc); });
  } else {
    timer.run(stream, IPCS_KERNEL_ASM_CONV, [&] {
      asm_conv(dim, mixed, stream, a22, cfg_e.bs, cfg_e.lds, U, n2, 1.0 / prm.dt, cs);
    });
  }
  if (semi) {
    form_eliminated(stream, mixed, n2, sp22, rp22, col22, bmask, E, K, 1.0, prm.nu, Ael, dinvA);
    lift_values(stream, mixed, nlift, lift_slot, E, K, 1.0, prm.nu, liftA);
    A_dirty = false;
  }
  const double sg = prm.scheme == IPCS_SCHEME_CHORIN ? 0.0 : 1.0;
  rhs_momentum(stream, dim, mixed, n2, sp22, col22, semi ? M : E, semi ? 1.0 / prm.dt : 1.0, sg,
               U, sp21, col21, Gc, P, has_F ? F : nullptr, lift_ptr, lift_col, liftA, bmask,
               gfull, bU);
  // the momentum solve's start: the extrapolation of the last tentative
  // velocities, quadratic once its three values leave out the first step of
  // the history (the scheme's initial layer makes that one rough in time),
  // linear from two; U^n before
  if (extrap_m() && mhist >= 2)
    extrapolate_with_bc(stream, dim, mhist >= kMhistFull ? 3 : 2, Ush[0], Ush[1], Ush[2], bmask,
                        gfull, Ustar, n2);
  else
    copy_with_bc(stream, dim, U, bmask, gfull, Ustar, n2);
  HIP_OK(hipEventRecord(ev[1], stream));
}

// r = -(rho/dt) sum_c D_c U*_c projected to zero sum; the start of the
// solve: dP = 0, or the previous step's dP (FP64 form: dP keeps it; mixed
// form: the first refinement pass's correction d starts there, dP = 0).
void Run::pressure_rhs() {
  // r is a difference of terms that cancel exactly at a discrete steady
  // state; an r no larger than a bound on its own rounding error is treated
  // as zero (dP = 0): on the solve's state in the FP64 form, in the
  // refinement test (scal[6]) in the mixed form
  rhs_pressure(stream, dim, false, n1, sp12, col12, Dc, Ustar, n2, -prm.rho / prm.dt, rP, spart,
               scal + 0, mixed ? nullptr : &(kst + dim)->zero2, scal + 6);
  if (warm_p() && mixed)
    HIP_OK(hipMemcpyAsync(dIR, dP, sizeof(double) * n1, hipMemcpyDeviceToDevice, stream));
  if (!warm_p() || mixed) HIP_OK(hipMemsetAsync(dP, 0, sizeof(double) * n1, stream));
}

// The next solve starts from dP = 0 (a new state or trajectory).
void Run::clear_pressure_start() {
  HIP_OK(hipMemsetAsync(dP, 0, sizeof(double) * n1, stream));
}

// dP shifted to zero integral mean.
void Run::pressure_end() {
  sub_weighted_mean(stream, n1, w, dP, spart, scal + 1);
  HIP_OK(hipEventRecord(ev[3], stream));
}

// b_c = M U*_c - (dt/rho) G_c dP with Dirichlet data; U^{n+1} starts at U*.
void Run::correction_rhs() {
  rhs_correction(stream, dim, mixed, n2, sp22, col22, M, Ustar, sp21, col21, Gc, dP,
                 prm.dt / prm.rho, lift_ptr, lift_col, liftM, bmask, gfull, bU);
  HIP_OK(hipMemcpyAsync(Unew, Ustar, sizeof(double) * dim * n2, hipMemcpyDeviceToDevice,
                        stream));
}

// P^{n+1} = P^n + dP (IPCS) or dP (Chorin), U^{n+1} (enqueued).
void Run::correction_commit() {
  if (prm.scheme == IPCS_SCHEME_CHORIN)
    HIP_OK(hipMemcpyAsync(P, dP, sizeof(double) * n1, hipMemcpyDeviceToDevice, stream));
  else
    axpy_inplace(stream, n1, 1.0, dP, P);
  HIP_OK(hipMemcpyAsync(U, Unew, sizeof(double) * dim * n2, hipMemcpyDeviceToDevice, stream));
  if (extrap_m()) {   // U*^(n+1) becomes the newest of the three kept
    HIP_OK(hipMemcpyAsync(Ush[2], Ustar, sizeof(double) * dim * n2, hipMemcpyDeviceToDevice,
                          stream));
    std::rotate(Ush, Ush + 2, Ush + 3);
    mhist = std::min(mhist + 1, kMhistFull);
  }
  HIP_OK(hipEventRecord(ev[4], stream));
}

// Waits for the step to finish, then t^{n+1} and the phase timings.
void Run::finish_step(ipcs_step_stats* st) {
  HIP_OK(hipEventSynchronize(ev[4]));
  timer.drain();
  t = t1;
  if (st) {
    st->t = t;
    HIP_OK(hipEventElapsedTime(&st->ms_asm, ev[0], ev[1]));
    HIP_OK(hipEventElapsedTime(&st->ms_mom, ev[1], ev[2]));
    HIP_OK(hipEventElapsedTime(&st->ms_p, ev[2], ev[3]));
    HIP_OK(hipEventElapsedTime(&st->ms_corr, ev[3], ev[4]));
  }
}

int Run::phase(int which, ipcs_step_stats* st) {
  if (which != phase_next)
    fail(IPCS_E_STATE, "IPCS phases must run in order; expected phase " +
                           std::to_string(phase_next) + ", got " + std::to_string(which));
  std::vector<KState> hs;
  int rc = IPCS_OK;
  switch (which) {
    case IPCS_PHASE_ASM:
      asm_phase();
      phase_next = IPCS_PHASE_MOMENTUM;
      return IPCS_OK;
    case IPCS_PHASE_MOMENTUM:
      rc = krylov_solve(stream, set_mom, KMethod::BICG, prm.check_every, hs, pinned,
                        timer);
      fill_stats_solve(hs, dim, 1, st);
      HIP_OK(hipEventRecord(ev[2], stream));
      if (rc != IPCS_OK) {
        if (st) st->failed_solve = 1;
        phase_next = IPCS_PHASE_ASM;
        return rc;
      }
      phase_next = IPCS_PHASE_PRESSURE;
      return IPCS_OK;
    case IPCS_PHASE_PRESSURE:
      pressure_rhs();
      rc = pressure_solve(hs, st);
      if (rc != IPCS_OK) {
        if (st) st->failed_solve = 2;
        phase_next = IPCS_PHASE_ASM;
        return rc;
      }
      pressure_end();
      phase_next = IPCS_PHASE_CORRECTION;
      return IPCS_OK;
    case IPCS_PHASE_CORRECTION:
      correction_rhs();
      rc = krylov_solve(stream, set_corr, KMethod::PCG, prm.check_every, hs, pinned,
                        timer);
      fill_stats_solve(hs, dim, 3, st);
      phase_next = IPCS_PHASE_ASM;
      if (rc != IPCS_OK) {
        if (st) st->failed_solve = 3;
        return rc;
      }
      correction_commit();
      finish_step(st);
      return IPCS_OK;
  }
  fail(IPCS_E_INVALID, "unknown phase " + std::to_string(which));
}

int Run::step(ipcs_step_stats* st) {
  if (phase_next != IPCS_PHASE_ASM) fail(IPCS_E_STATE, "a step is in progress (phase API)");
  if (st) std::memset(st, 0, sizeof(*st));
  for (int ph = IPCS_PHASE_ASM; ph <= IPCS_PHASE_CORRECTION; ++ph) {
    const int rc = phase(ph, st);
    if (rc != IPCS_OK) {
      if (st) {
        st->status = rc;
        st->t = t;
      }
      return rc;
    }
  }
  return IPCS_OK;
}

// Times nlaunch back-to-back launches of one kernel of the step on this run's
// data. The solver states are forced to "iterating" first and checked after:
// every timed launch must have done its full work.
double Run::profile_kernel(int kernel, int nlaunch) {
  if (phase_next != IPCS_PHASE_ASM) fail(IPCS_E_STATE, "profile only between steps");
  if (kernel < 0 || kernel >= IPCS_NKERNEL) fail(IPCS_E_INVALID, "unknown kernel id");
  const bool mom = kernel == IPCS_KERNEL_BICG_SPMV || kernel == IPCS_KERNEL_BICG_SPMV_T ||
                   kernel == IPCS_KERNEL_BICG_UPDATE_S || kernel == IPCS_KERNEL_BICG_UPDATE_X;
  const bool corr = kernel == IPCS_KERNEL_PCG_SPMV_M || kernel == IPCS_KERNEL_PCG_UPDATE_M;
  const bool assembly = kernel == IPCS_KERNEL_ASM_CONV || kernel == IPCS_KERNEL_ASM_SUM;
  const KSet* S = mom ? &set_mom : corr ? &set_corr : assembly ? nullptr : &set_p;
  const bool fused = kernel == IPCS_KERNEL_PCG_FUSED_P;
  if (fused != (S == &set_p && set_p.fused) && S == &set_p)
    fail(IPCS_E_INVALID, fused ? "this run's Poisson CG is not the fused form"
                               : "this run's Poisson CG is the fused form");
  // the solver states (tolerances, zero level) are restored after timing
  std::vector<KState> saved;
  if (S) {
    const KGroup& g = S->h_groups[0];
    saved.resize(g.nsys);
    for (int j = 0; j < g.nsys; ++j)
      HIP_OK(hipMemcpyAsync(&saved[j], g.v[j].st, sizeof(KState), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    for (int j = 0; j < g.nsys; ++j) {
      KState& k = pinned[j];
      std::memset(&k, 0, sizeof(k));
      k.status = KS_RUN;
      k.sc[0] = k.sc[1] = 1.0;
      k.alpha[0] = k.alpha[1] = 1.0;
      k.omega = 1.0;
      k.bb = 1.0;
      k.tol2 = 0.0;
      HIP_OK(hipMemcpyAsync(g.v[j].st, &k, sizeof(KState), hipMemcpyHostToDevice, stream));
    }
    // partials the kernels reduce in their prologue, in block 0 (zeros
    // elsewhere), chosen so that every timed launch takes the full iteration
    // path: CG gamma = r.r = 1, delta = 2 (alpha = beta = 1); BiCGStab
    // rhat.v = 2, r.r = 1, t.s = t.t = rhat.s = 2, rhat.t = 1 (omega = 1, rho' = 1)
    if (fused) {
      // fused CG partials [gamma, r.r, delta] = [1, 1, 2] in part 0
      std::vector<double> pf((size_t)KP * set_p.F.nblocks, 0.0);
      for (int k = 0; k < 3; ++k) pf[(size_t)k * set_p.F.nblocks] = k == 2 ? 2.0 : 1.0;
      HIP_OK(hipMemcpyAsync(f_part[0], pf.data(), sizeof(double) * pf.size(),
                            hipMemcpyHostToDevice, stream));
      HIP_OK(hipStreamSynchronize(stream));
    }
    std::vector<double> pm((size_t)g.nblk_m * GMAX * KP, 0.0), pv((size_t)g.nblk_v * GMAX * KP, 0.0);
    for (int j = 0; j < g.nsys; ++j)
      for (int k = 0; k < KP; ++k) {
        pm[(size_t)(j * KP + k) * g.nblk_m] = k == 3 ? 1.0 : 2.0;   // block 0, SoA layout
        pv[(size_t)(j * KP + k) * g.nblk_v] = 1.0;
      }
    HIP_OK(hipMemcpyAsync(g.part_m, pm.data(), sizeof(double) * pm.size(), hipMemcpyHostToDevice,
                          stream));
    for (int q = 0; q < 2; ++q)
      HIP_OK(hipMemcpyAsync(g.part_v[q], pv.data(), sizeof(double) * pv.size(),
                            hipMemcpyHostToDevice, stream));
    HIP_OK(hipStreamSynchronize(stream));
  }
  const Mesh& m = *mesh;
  RowAsm a22{(int32_t)n2, sp22, inc2p, inc2, s22, m.s22.stride, c2d, m.nloc2, X,
             {E, nullptr, nullptr}, m.pair, c2v, m.nloc1, kAsmXcdChunk};
  auto launch = [&]() {
    switch (kernel) {
      case IPCS_KERNEL_PCG_SPMV_P: pcg_spmv_only(stream, set_p.L); break;
      case IPCS_KERNEL_PCG_UPDATE_P: pcg_update_only(stream, set_p.L, 0); break;
      case IPCS_KERNEL_ASM_CONV: {
        const double cs = prm.convection == IPCS_CONV_SEMI_IMPLICIT ? 1.0 : -1.0;
        if (two_pass_conv())
          asm_conv_cells(dim, mixed, stream, a22, nc, U, n2, 1.0 / prm.dt, cs, Eloc);
        else asm_conv(dim, mixed, stream, a22, cfg_e.bs, cfg_e.lds, U, n2, 1.0 / prm.dt, cs);
        break;
      }
      case IPCS_KERNEL_ASM_SUM:
        if (!two_pass_conv())
          fail(IPCS_E_INVALID, "this run's convection assembly takes one pass");
        asm_local_sum(dim, mixed, stream, a22, cfg_e.bs, cfg_e.lds, Eloc);
        break;
      case IPCS_KERNEL_BICG_SPMV: bicg_spmv_only(stream, set_mom.L); break;
      case IPCS_KERNEL_PCG_SPMV_M: pcg_spmv_only(stream, set_corr.L); break;
      case IPCS_KERNEL_BICG_SPMV_T: bicg_spmv_t_only(stream, set_mom.L); break;
      case IPCS_KERNEL_BICG_UPDATE_S: bicg_update_s_only(stream, set_mom.L, 0); break;
      case IPCS_KERNEL_BICG_UPDATE_X: bicg_update_x_only(stream, set_mom.L, 0); break;
      case IPCS_KERNEL_PCG_UPDATE_M: pcg_update_only(stream, set_corr.L, 0); break;
      case IPCS_KERNEL_PCG_FUSED_P: fcg_iter(stream, set_p.F, 0); break;
      default: fail(IPCS_E_INVALID, "unknown kernel id");
    }
  };
  launch();   // warm
  HIP_OK(hipEventRecord(ev[0], stream));
  for (int i = 0; i < nlaunch; ++i) launch();
  HIP_OK(hipEventRecord(ev[1], stream));
  HIP_OK(hipEventSynchronize(ev[1]));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
  if (S) {
    gather_states(stream, S->L, S->d_poll);
    HIP_OK(hipMemcpyAsync(pinned, S->d_poll, sizeof(KState) * GMAX, hipMemcpyDeviceToHost,
                          stream));
    HIP_OK(hipStreamSynchronize(stream));
    const KGroup& g = S->h_groups[0];
    std::vector<KState> after(pinned, pinned + g.nsys);
    for (int j = 0; j < g.nsys; ++j)
      HIP_OK(hipMemcpyAsync(g.v[j].st, &saved[j], sizeof(KState), hipMemcpyHostToDevice, stream));
    HIP_OK(hipStreamSynchronize(stream));
    for (int j = 0; j < g.nsys; ++j)
      if (after[j].status != KS_RUN)
      {
        char msg[512];
        const KState& k = after[j];
        std::snprintf(msg, sizeof msg,
                      "profiled kernel %d left system %d in status %d (rr %.3e bb %.3e tol2 %.3e "
                      "it %d); timing discarded",
                      kernel, j, k.status, k.rr, k.bb, k.tol2, k.it);
        fail(IPCS_E_STATE, msg);
      }
  }
  return 1000.0 * ms / nlaunch;
}

void Run::export_values(int pattern, const void* dev, int vbytes, double* out) {
  const Sell& S = mesh->sell(pattern);
  const Pattern& P = mesh->pattern(pattern);
  std::vector<double> h(S.nent);
  if (vbytes == 4) {
    std::vector<float> hf(S.nent);
    HIP_OK(hipMemcpyAsync(hf.data(), dev, sizeof(float) * S.nent, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    for (int64_t k = 0; k < S.nent; ++k) h[k] = hf[k];
  } else {
    HIP_OK(hipMemcpyAsync(h.data(), dev, sizeof(double) * S.nent, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
  }
  for (int64_t i = 0; i < P.nrows; ++i)
    for (int k = 0; k < P.rowptr[i + 1] - P.rowptr[i]; ++k)
      out[P.rowptr[i] + k] = h[S.index(i, k)];
}

// Pressure Poisson solve (eq. (9), second line). FP64 form: one Jacobi-CG
// solve of Kp dP = r to tol_p. Mixed form: iterative refinement in FP64 on
// the FP64 Kp: res = r - Kp dP (projected to zero sum), stop when
// ||res|| <= tol_ir ||r||, else solve Kp32 d = res with Jacobi-CG on the FP32
// matrix (FP64 vectors and sums) to a loose relative tolerance and add d.
int Run::pressure_solve(std::vector<KState>& hs, ipcs_step_stats* st) {
  if (!mixed) {
    const int rc = krylov_solve(stream, set_p, KMethod::PCG, prm.check_every, hs,
                                pinned, timer);
    fill_stats_solve(hs, 1, 2, st);
    return rc;
  }
  double* tot = scal + 3;   // [3] sum(res), [4] sum(res^2); [5] mean; [6] noise floor
  double host[4];
  double bb = -1.0, rel = 0.0, prev = 0.0, contraction = 0.0, last_tol = 1.0, op_limit = 0.0;
  double floor_in = 0.0;   // raised after an inner breakdown
  int inner_total = 0, checks_total = 0, outer = 0, rc = IPCS_OK;
  for (;; ++outer) {
    residual_projected(stream, n1, sp11, col11, Kp64, dP, rP, rIR, spart, spart + 8192, tot,
                       scal + 5);
    HIP_OK(hipMemcpyAsync(host, tot, sizeof(host), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    const double rr = std::max(0.0, host[1] - host[0] * host[0] / (double)n1);
    const double floor2 = host[3];
    if (bb < 0.0) bb = rr;   // dP = 0 on the first pass: res = r
    rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    if (!std::isfinite(rr)) {
      rc = IPCS_E_NONFINITE;
      break;
    }
    if (rr <= prm.tol_ir * prm.tol_ir * bb || (outer == 0 && rr <= floor2)) break;
    if (outer >= kMaxRefine) {
      rc = IPCS_E_NOT_CONVERGED;
      break;
    }
    // inner tolerance: the reduction still needed, but not below half of the
    // reduction a pass achieves (the FP32 operator's limit: seen on the
    // previous pass, or on the previous step for the first pass)
    if (outer > 0) {
      contraction = rel / prev;
      // a pass that stopped well short of its inner tolerance was limited by
      // the FP32 operator: remember that reduction for the next step
      if (contraction > 2.0 * last_tol) op_limit = std::max(op_limit, contraction);
    } else {
      contraction = ir_c;
    }
    prev = rel;
    const double need = prm.tol_ir / rel;
    const double tol_in =
        std::min(0.5, std::max({need, 0.5 * contraction, floor_in, prm.tol_p}));
    last_tol = tol_in;
    set_tolerance(stream, set_p.L, tol_in * tol_in);
    if (outer > 0 || !warm_p()) HIP_OK(hipMemsetAsync(dIR, 0, sizeof(double) * n1, stream));
    set_p.last_iters = outer < kIrHist ? ir_last[outer] : 0;
    rc = krylov_solve(stream, set_p, KMethod::PCG, prm.check_every, hs, pinned, timer);
    if (outer < kIrHist) ir_last[outer] = set_p.last_iters;
    inner_total += hs[0].it;
    checks_total += hs[0].nchecks;
    if (rc == IPCS_E_BREAKDOWN) {
      // Kp rounded to FP32 is singular only up to rounding and can be
      // marginally indefinite: the pass ends at its last iterate (x is not
      // updated by the breaking iteration) and later passes stop earlier
      floor_in = floor_in == 0.0 ? 1e-6 : std::min(1e-2, floor_in * 100.0);
      rc = IPCS_OK;
    }
    if (rc != IPCS_OK) break;
    axpy_inplace(stream, n1, 1.0, dIR, dP);
  }
  if (op_limit > 0.0) ir_c = op_limit;   // kept while the operator keeps limiting passes
  if (st) {
    st->it_p = inner_total;
    st->checks_p = checks_total;
    st->res_p = rel;
    st->ir_outer = outer;
  }
  return rc;
}

}  // namespace ipcs
