// Cell-quadrature assembly kernels for gfx950 (row-owner, conflict-free).
//
// Each thread owns one matrix row (a velocity or pressure DOF). It walks the
// cells incident to its DOF, evaluates that cell's local matrix row by the
// cell rule (degree 5 for P2-P1, degree 8 for P3-P2; reference tables in
// constant memory) and adds it into the row's slots,
// which live in LDS in the same SELL-64 layout as the value array. After a
// barrier the block writes its slices back with coalesced stores. No value is
// written by two threads, so there are no atomics and the result is
// deterministic.
//
// Local matrices (Section 2.2.1, weak forms of eq. (9)), on a cell K with affine
// map x = x0 + J xi, gradients grad phi = J^{-T} grad_ref phi:
//   M_ij = sum_q w_q |J| phi_i phi_j              K_ij = sum_q w_q |J| grad phi_i . grad phi_j
//   C_ij = sum_q w_q |J| phi_i (u_h . grad phi_j) with u_h = sum_m U_m phi_m
//   (G_c)_ik = sum_q w_q |J| phi_i d_c psi_k      (D_c)_kj = sum_q w_q |J| psi_k d_c phi_j
//   Kp_kl = |K| grad psi_k . grad psi_l           w_k = int_K psi_k = |K|/(d+1)
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "dev_util.hpp"
#include "device.hpp"
#include "launch.hpp"
#include "builtin.hpp"
#include "rules.hpp"

namespace ipcs {

// Geometry of a cell: formed in FP64 from the vertex coordinates (the
// differences x_k - x_0 cancel digits on fine meshes), then rounded to the
// working type R of the quadrature loop.
template <int D, class R = double>
struct Geo {
  R Ji[D][D];   // J^{-1}
  R det;        // |det J|
};

// From the vertex coordinates xc[k] of the cell's vertices k = 0..D.
template <int D, class R = double>
__device__ __forceinline__ Geo<D, R> cell_geo_x(const double (&xc)[D + 1][D]) {
  double J[D][D], Ji[D][D], det;
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int r = 0; r < D; ++r) J[r][k] = xc[k + 1][r] - xc[0][r];
  if constexpr (D == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double id = 1.0 / det;
    Ji[0][0] = J[1][1] * id;
    Ji[0][1] = -J[0][1] * id;
    Ji[1][0] = -J[1][0] * id;
    Ji[1][1] = J[0][0] * id;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
  Geo<D, R> g;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) g.Ji[a][b] = (R)Ji[a][b];
  g.det = (R)fabs(det);
  return g;
}

template <int D>
__device__ __forceinline__ void load_coords(const double* X, const int32_t* v,
                                            double (&xc)[D + 1][D]) {
#pragma unroll
  for (int k = 0; k <= D; ++k)
#pragma unroll
    for (int r = 0; r < D; ++r) xc[k][r] = X[(size_t)v[k] * D + r];
}

template <int D, class R = double>
__device__ __forceinline__ Geo<D, R> cell_geo(const double* X, const int32_t* dofs) {
  double xc[D + 1][D];
  load_coords<D>(X, dofs, xc);
  return cell_geo_x<D, R>(xc);
}

// The vertex ids of a cell (for its geometry), from the cell-vertex table.
template <int D>
__device__ __forceinline__ void cell_vertices(const RowAsm& a, int64_t cell, int32_t (&v)[D + 1]) {
#pragma unroll
  for (int k = 0; k <= D; ++k) v[k] = a.c2v[cell * a.nv_stride + k];
}

// Reference-element tables at the quadrature points, built at compile time
// (in FP64, then rounded to R) and kept in constant memory: indices that are
// uniform across a wavefront (q, j) are served by the scalar cache, the
// row-dependent entries (the row's local index li) by ordinary cached loads.
template <int D, class R = double>
struct Tab {
  static constexpr int NQ = Rule<D>::NQ, NL = P2<D>::NLOC;
  R w[NQ];
  R lam[NQ][D + 1];
  R phi[NQ][NL];
  R dphi[NQ][NL][D];
  constexpr Tab() : w(), lam(), phi(), dphi() {
    for (int q = 0; q < NQ; ++q) {
      double l[D + 1] = {};
      for (int k = 0; k <= D; ++k) l[k] = Rule<D>::lam(q, k);
      w[q] = (R)Rule<D>::w(q);
      for (int k = 0; k <= D; ++k) lam[q][k] = (R)l[k];
      for (int j = 0; j < NL; ++j) {
        phi[q][j] = (R)P2<D>::phi(j, l);
        for (int r = 0; r < D; ++r) dphi[q][j][r] = (R)P2<D>::dphi(j, r, l);
      }
    }
  }
};

__constant__ Tab<2, double> c_tab2 = Tab<2, double>();
__constant__ Tab<3, double> c_tab3 = Tab<3, double>();
__constant__ Tab<2, float> c_tab2f = Tab<2, float>();
__constant__ Tab<3, float> c_tab3f = Tab<3, float>();

template <int D, class R>
__device__ __forceinline__ const Tab<D, R>& tab() {
  if constexpr (D == 2 && std::is_same_v<R, double>) return c_tab2;
  else if constexpr (D == 3 && std::is_same_v<R, double>) return c_tab3;
  else if constexpr (D == 2) return c_tab2f;
  else return c_tab3f;
}

// physical gradient components of reference gradient gr: g_b = sum_a Ji[a][b] gr_a
template <int D, class R>
__device__ __forceinline__ void phys(const Geo<D, R>& g, const R* gr, R* out) {
#pragma unroll
  for (int b = 0; b < D; ++b) {
    R s = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) s += g.Ji[a][b] * gr[a];
    out[b] = s;
  }
}

// ------------------------------------------------------------------ ops
// Each op fills v[NOUT][NCOL] = the local row li of NOUT matrices, computed and
// accumulated in its working type R (double, or float in the mixed form).
template <int D, int WHICH, class R>
struct OpMassStiff {   // P2 x P2: M (WHICH 0) or K (WHICH 1)
  using real = R;
  static constexpr int NOUT = 1, NCOL = P2<D>::NLOC, NDOF = 0;   // geometry only
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const Tab<D, R>& T = tab<D, R>();
#pragma unroll 1
    for (int q = 0; q < Rule<D>::NQ; ++q) {
      const R wq = T.w[q] * g.det;
      if (WHICH == 0) {
        const R ci = wq * T.phi[q][li];
#pragma unroll
        for (int j = 0; j < NCOL; ++j) v[0][j] += ci * T.phi[q][j];
      } else {
        R gi[D];
        phys<D, R>(g, T.dphi[q][li], gi);
#pragma unroll
        for (int j = 0; j < NCOL; ++j) {
          R gj[D];
          phys<D, R>(g, T.dphi[q][j], gj);
          R s = 0;
#pragma unroll
          for (int b = 0; b < D; ++b) s += gi[b] * gj[b];
          v[0][j] += wq * s;
        }
      }
    }
  }
};


template <int D, class R>
struct OpConv {   // P2 x P2: E = M/dt + cs C(U), cs = -1 (explicit) or +1 (semi-implicit)
  using real = R;
  static constexpr int NOUT = 1, NCOL = P2<D>::NLOC, NDOF = P2<D>::NLOC;
  const double* U;        // [D][n2]
  int64_t n2;
  double inv_dt;
  double cs;
  // the cell's nodal velocities, loaded apart from the evaluation so that a
  // row can fetch its next cell's while it evaluates this one
  struct Nodal {
    R Uc[D][NCOL];
  };
  __device__ void load(const int32_t* dofs, Nodal& nd) const {
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int m = 0; m < NCOL; ++m) nd.Uc[c][m] = (R)U[(size_t)c * n2 + dofs[m]];
  }
  __device__ void operator()(const Geo<D, R>& g, const int32_t* dofs, int li,
                             R (&v)[NOUT][NCOL]) const {
    Nodal nd;
    load(dofs, nd);
    (*this)(g, nd, li, v);
  }
  __device__ void operator()(const Geo<D, R>& g, const Nodal& nd, int li,
                             R (&v)[NOUT][NCOL]) const {
    const Tab<D, R>& T = tab<D, R>();
    const auto& Uc = nd.Uc;
    const R idt = (R)inv_dt, csr = (R)cs;
#pragma unroll 1
    for (int q = 0; q < Rule<D>::NQ; ++q) {
      R uq[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        R s = 0;
#pragma unroll
        for (int m = 0; m < NCOL; ++m) s += Uc[c][m] * T.phi[q][m];
        uq[c] = s;
      }
      R beta[D];   // J^{-1} u_h: reference-frame velocity
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R s = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) s += g.Ji[a][c] * uq[c];
        beta[a] = s;
      }
      const R ci = T.w[q] * g.det * T.phi[q][li];
#pragma unroll
      for (int j = 0; j < NCOL; ++j) {
        R adv = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) adv += beta[a] * T.dphi[q][j][a];
        v[0][j] += ci * (T.phi[q][j] * idt + csr * adv);
      }
    }
  }
};
// P2 x P2: N_ce = sum_q w |J| phi_i phi_j d_e u_c(x_q), the matrix of the
// Newton term ((du . grad) u, v) coupling component e of the increment to
// component c of the equation (steady solver, Newton linearization of
// Section 2.2.1)
template <int D, class R>
struct OpNewton {
  using real = R;
  static constexpr int NOUT = 1, NCOL = P2<D>::NLOC, NDOF = P2<D>::NLOC;
  const double* U;        // [D][n2]
  int64_t n2;
  int c, e;
  struct Nodal {   // component c of the cell's nodal velocities
    R Uc[NCOL];
  };
  __device__ void load(const int32_t* dofs, Nodal& nd) const {
#pragma unroll
    for (int m = 0; m < NCOL; ++m) nd.Uc[m] = (R)U[(size_t)c * n2 + dofs[m]];
  }
  __device__ void operator()(const Geo<D, R>& g, const int32_t* dofs, int li,
                             R (&v)[NOUT][NCOL]) const {
    Nodal nd;
    load(dofs, nd);
    (*this)(g, nd, li, v);
  }
  __device__ void operator()(const Geo<D, R>& g, const Nodal& nd, int li,
                             R (&v)[NOUT][NCOL]) const {
    const Tab<D, R>& T = tab<D, R>();
    const auto& Uc = nd.Uc;
#pragma unroll 1
    for (int q = 0; q < Rule<D>::NQ; ++q) {
      R gr[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R s = 0;
#pragma unroll
        for (int m = 0; m < NCOL; ++m) s += Uc[m] * T.dphi[q][m][a];
        gr[a] = s;
      }
      R gp[D];
      phys<D, R>(g, gr, gp);
      R due = gp[0];
#pragma unroll
      for (int b = 1; b < D; ++b) due = (e == b) ? gp[b] : due;
      const R ci = T.w[q] * g.det * T.phi[q][li] * due;
#pragma unroll
      for (int j = 0; j < NCOL; ++j) v[0][j] += ci * T.phi[q][j];
    }
  }
};

template <int D, class R>
struct OpGrad {   // P2 rows x P1 cols: G_c for one component c
  using real = R;
  static constexpr int NOUT = 1, NCOL = D + 1, NDOF = 0;   // geometry only
  int c;
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const Tab<D, R>& T = tab<D, R>();
    R int_phi = 0;
#pragma unroll 1
    for (int q = 0; q < Rule<D>::NQ; ++q) int_phi += T.w[q] * T.phi[q][li];
    int_phi *= g.det;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
      R gr[D], gp[D];
#pragma unroll
      for (int a = 0; a < D; ++a) gr[a] = (R)P2<D>::template dlam<double>(k, a);
      phys<D, R>(g, gr, gp);
      R gc = gp[0];
#pragma unroll
      for (int cc = 1; cc < D; ++cc) gc = (c == cc) ? gp[cc] : gc;
      v[0][k] += int_phi * gc;
    }
  }
};

template <int D, class R>
struct OpDiv {   // P1 rows x P2 cols: D_c for one component c
  using real = R;
  static constexpr int NOUT = 1, NCOL = P2<D>::NLOC, NDOF = 0;   // geometry only
  int c;
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const Tab<D, R>& T = tab<D, R>();
#pragma unroll 1
    for (int q = 0; q < Rule<D>::NQ; ++q) {
      const R ci = T.w[q] * g.det * T.lam[q][li];
#pragma unroll
      for (int j = 0; j < NCOL; ++j) {
        R gp[D];
        phys<D, R>(g, T.dphi[q][j], gp);
        R gc = gp[0];
#pragma unroll
        for (int cc = 1; cc < D; ++cc) gc = (c == cc) ? gp[cc] : gc;
        v[0][j] += ci * gc;
      }
    }
  }
};

template <int D, class R>
struct OpKp {   // P1 x P1 stiffness
  using real = R;
  static constexpr int NOUT = 1, NCOL = D + 1, NDOF = 0;   // geometry only
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    R gl[D + 1][D];
#pragma unroll
    for (int k = 0; k <= D; ++k) {
      R gr[D];
#pragma unroll
      for (int a = 0; a < D; ++a) gr[a] = (R)P2<D>::template dlam<double>(k, a);
      phys<D, R>(g, gr, gl[k]);
    }
    R gi[D];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      R s = gl[0][b];
#pragma unroll
      for (int m = 1; m <= D; ++m) s = (li == m) ? gl[m][b] : s;
      gi[b] = s;
    }
    const R vol = g.det * (R)ref_measure<D>();
#pragma unroll
    for (int k = 0; k <= D; ++k) {
      R s = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) s += gi[b] * gl[k][b];
      v[0][k] += vol * s;
    }
  }
};

// ------------------------------------------------------------------ P3-P2 pair
// Tables of the P3-P2 pair at the points of its cell rule: P3 velocity basis
// phi and P2 pressure basis psi, values and reference gradients.
// Triangles: the 25-point degree-8 rule, tables built at compile time and kept
// in constant memory (10.4 KB in FP64).
template <class R>
struct Tab3 {
  static constexpr int NQ = RuleT9::NQ, NL = P3T::NLOC, NP = P2<2>::NLOC;
  R w[NQ];
  R lam[NQ][3];
  R phi[NQ][NL];
  R dphi[NQ][NL][2];
  R psi[NQ][NP];
  R dpsi[NQ][NP][2];
  constexpr Tab3() : w(), lam(), phi(), dphi(), psi(), dpsi() {
    for (int q = 0; q < NQ; ++q) {
      double l[3] = {};
      for (int k = 0; k < 3; ++k) l[k] = RuleT9::lam(q, k);
      w[q] = (R)RuleT9::w(q);
      for (int k = 0; k < 3; ++k) lam[q][k] = (R)l[k];
      for (int j = 0; j < NL; ++j) {
        phi[q][j] = (R)P3T::phi(j, l);
        for (int r = 0; r < 2; ++r) dphi[q][j][r] = (R)P3T::dphi(j, r, l);
      }
      for (int j = 0; j < NP; ++j) {
        psi[q][j] = (R)P2<2>::phi(j, l);
        for (int r = 0; r < 2; ++r) dpsi[q][j][r] = (R)P2<2>::dphi(j, r, l);
      }
    }
  }
};

// Tetrahedra: the 125-point conical rule (degree 9), whose nodes come from a
// host-side root finder; 125 KB in FP64, so the tables live in global device
// memory (filled once per device before the first launch that reads them).
// Loads at wavefront-uniform indices still go through the scalar cache.
template <class R>
struct Tab3Tet {
  static constexpr int NQ = RuleTet9::NQ, NL = P3Tet::NLOC, NP = P2<3>::NLOC;
  R w[NQ];
  R lam[NQ][4];
  R phi[NQ][NL];
  R dphi[NQ][NL][3];
  R psi[NQ][NP];
  R dpsi[NQ][NP][3];
};

__constant__ Tab3<double> c_tab3p = Tab3<double>();
__constant__ Tab3<float> c_tab3pf = Tab3<float>();
__device__ Tab3Tet<double> g_tab3t;
__device__ Tab3Tet<float> g_tab3tf;

template <int D>
struct P3Of;
template <>
struct P3Of<2> {
  using B = P3T;
  template <class R>
  using Tab = Tab3<R>;
};
template <>
struct P3Of<3> {
  using B = P3Tet;
  template <class R>
  using Tab = Tab3Tet<R>;
};

template <int D, class R>
__device__ __forceinline__ const typename P3Of<D>::template Tab<R>& tab3() {
  if constexpr (D == 2 && std::is_same_v<R, double>) return c_tab3p;
  else if constexpr (D == 2) return c_tab3pf;
  else if constexpr (std::is_same_v<R, double>) return g_tab3t;
  else return g_tab3tf;
}

template <class R>
static void fill_tet_tables(Tab3Tet<R>& T, const double* lam, const double* w) {
  constexpr int NQ = Tab3Tet<R>::NQ;
  for (int q = 0; q < NQ; ++q) {
    const double* l = lam + 4 * q;
    T.w[q] = (R)w[q];
    for (int k = 0; k < 4; ++k) T.lam[q][k] = (R)l[k];
    for (int j = 0; j < P3Tet::NLOC; ++j) {
      T.phi[q][j] = (R)P3Tet::phi(j, l);
      for (int r = 0; r < 3; ++r) T.dphi[q][j][r] = (R)P3Tet::dphi(j, r, l);
    }
    for (int j = 0; j < P2<3>::NLOC; ++j) {
      T.psi[q][j] = (R)P2<3>::phi(j, l);
      for (int r = 0; r < 3; ++r) T.dpsi[q][j][r] = (R)P2<3>::dphi(j, r, l);
    }
  }
}

// Fill the tetrahedral tables on the current device (once per device).
static void ensure_tet_tables() {
  static std::mutex mu;
  static std::vector<char> done;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, 0);
  if (done[dev]) return;
  std::vector<double> lam(4 * RuleTet9::NQ), w(RuleTet9::NQ);
  tet_rule9(lam.data(), w.data());
  auto t64 = std::make_unique<Tab3Tet<double>>();
  auto t32 = std::make_unique<Tab3Tet<float>>();
  fill_tet_tables(*t64, lam.data(), w.data());
  fill_tet_tables(*t32, lam.data(), w.data());
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(g_tab3t), t64.get(), sizeof(Tab3Tet<double>)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(g_tab3tf), t32.get(), sizeof(Tab3Tet<float>)));
  HIP_OK(hipDeviceSynchronize());
  done[dev] = 1;
}

static void need_tables(int dim, const RowAsm& a) {
  if (dim == 3 && a.pair == IPCS_PAIR_P3P2) ensure_tet_tables();
}

// the c-th physical gradient component of a reference gradient
template <int D, class R>
__device__ __forceinline__ R phys_c(const Geo<D, R>& g, const R* gr, int c) {
  R p[D];
  phys<D, R>(g, gr, p);
  R s = p[0];
#pragma unroll
  for (int b = 1; b < D; ++b) s = (c == b) ? p[b] : s;
  return s;
}

template <int D, int WHICH, class R>
struct Op3MassStiff {   // P3 x P3: M (WHICH 0) or K (WHICH 1)
  using real = R;
  static constexpr int NOUT = 1, NCOL = P3Of<D>::B::NLOC, NDOF = 0;   // geometry only
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const auto& T = tab3<D, R>();
#pragma unroll 1
    for (int q = 0; q < T.NQ; ++q) {
      const R wq = T.w[q] * g.det;
      if (WHICH == 0) {
        const R ci = wq * T.phi[q][li];
#pragma unroll
        for (int j = 0; j < NCOL; ++j) v[0][j] += ci * T.phi[q][j];
      } else {
        R gi[D];
        phys<D, R>(g, T.dphi[q][li], gi);
#pragma unroll
        for (int j = 0; j < NCOL; ++j) {
          R gj[D];
          phys<D, R>(g, T.dphi[q][j], gj);
          R s = 0;
#pragma unroll
          for (int b = 0; b < D; ++b) s += gi[b] * gj[b];
          v[0][j] += wq * s;
        }
      }
    }
  }
};

template <int D, class R>
struct Op3Conv {   // P3 x P3: E = M/dt + cs C(U)
  using real = R;
  static constexpr int NOUT = 1, NCOL = P3Of<D>::B::NLOC, NDOF = NCOL;
  const double* U;        // [D][n2]
  int64_t n2;
  double inv_dt;
  double cs;
  __device__ void operator()(const Geo<D, R>& g, const int32_t* dofs, int li,
                             R (&v)[NOUT][NCOL]) const {
    const auto& T = tab3<D, R>();
    R Uc[D][NCOL];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int m = 0; m < NCOL; ++m) Uc[c][m] = (R)U[(size_t)c * n2 + dofs[m]];
    const R idt = (R)inv_dt, csr = (R)cs;
#pragma unroll 1
    for (int q = 0; q < T.NQ; ++q) {
      R uq[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        R s = 0;
#pragma unroll
        for (int m = 0; m < NCOL; ++m) s += Uc[c][m] * T.phi[q][m];
        uq[c] = s;
      }
      R beta[D];   // J^{-1} u_h
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R s = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) s += g.Ji[a][c] * uq[c];
        beta[a] = s;
      }
      const R ci = T.w[q] * g.det * T.phi[q][li];
#pragma unroll
      for (int j = 0; j < NCOL; ++j) {
        R adv = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) adv += beta[a] * T.dphi[q][j][a];
        v[0][j] += ci * (T.phi[q][j] * idt + csr * adv);
      }
    }
  }
};

template <int D, class R>
struct Op3Grad {   // P3 rows x P2 cols: (G_c)_ik = sum_q w |J| phi_i d_c psi_k
  using real = R;
  static constexpr int NOUT = 1, NCOL = P2<D>::NLOC, NDOF = 0;
  int c;
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const auto& T = tab3<D, R>();
#pragma unroll 1
    for (int q = 0; q < T.NQ; ++q) {
      const R ci = T.w[q] * g.det * T.phi[q][li];
#pragma unroll
      for (int k = 0; k < NCOL; ++k) v[0][k] += ci * phys_c<D, R>(g, T.dpsi[q][k], c);
    }
  }
};

template <int D, class R>
struct Op3Div {   // P2 rows x P3 cols: (D_c)_kj = sum_q w |J| psi_k d_c phi_j
  using real = R;
  static constexpr int NOUT = 1, NCOL = P3Of<D>::B::NLOC, NDOF = 0;
  int c;
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const auto& T = tab3<D, R>();
#pragma unroll 1
    for (int q = 0; q < T.NQ; ++q) {
      const R ci = T.w[q] * g.det * T.psi[q][li];
#pragma unroll
      for (int j = 0; j < NCOL; ++j) v[0][j] += ci * phys_c<D, R>(g, T.dphi[q][j], c);
    }
  }
};

template <int D, class R>
struct Op3Kp {   // P2 x P2 stiffness of the pressure space
  using real = R;
  static constexpr int NOUT = 1, NCOL = P2<D>::NLOC, NDOF = 0;
  __device__ void operator()(const Geo<D, R>& g, const int32_t*, int li,
                             R (&v)[NOUT][NCOL]) const {
    const auto& T = tab3<D, R>();
#pragma unroll 1
    for (int q = 0; q < T.NQ; ++q) {
      const R wq = T.w[q] * g.det;
      R gi[D];
      phys<D, R>(g, T.dpsi[q][li], gi);
#pragma unroll
      for (int k = 0; k < NCOL; ++k) {
        R gk[D];
        phys<D, R>(g, T.dpsi[q][k], gk);
        R s = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) s += gi[b] * gk[b];
        v[0][k] += wq * s;
      }
    }
  }
};

// ------------------------------------------------------------------ kernel
// What a row's walk over its incident cells loads per cell, in dependency
// order: the incidence code; the cell's vertex ids and (ops that read U) its
// velocity DOFs; the vertex coordinates and the op's nodal values (ops with a
// Nodal type load them apart from the evaluation).
template <class Op, class = void>
struct NodalOf {
  static constexpr bool on = false;
  struct type {};
};
template <class Op>
struct NodalOf<Op, std::void_t<typename Op::Nodal>> {
  static constexpr bool on = true;
  using type = typename Op::Nodal;
};

template <int D, class Op>
struct CellIdx {
  int32_t dl[Op::NDOF > 0 ? Op::NDOF : 1];
  int32_t vx[D + 1];
};

template <int D, class Op>
struct CellVals {
  double xc[D + 1][D];
  typename NodalOf<Op>::type nd;
};

template <int D, class Op>
__device__ __forceinline__ void load_idx(const RowAsm& a, int code, CellIdx<D, Op>& ix) {
  const int cell = code >> 5;
  if constexpr (Op::NDOF > 0) {
    const int32_t* dofs = a.c2d + (size_t)cell * a.nloc2;
#pragma unroll
    for (int m = 0; m < Op::NDOF; ++m) ix.dl[m] = dofs[m];
  }
  cell_vertices<D>(a, cell, ix.vx);
}

template <int D, class Op>
__device__ __forceinline__ void load_vals(const RowAsm& a, const Op& op, const CellIdx<D, Op>& ix,
                                          CellVals<D, Op>& cv) {
  load_coords<D>(a.X, ix.vx, cv.xc);
  if constexpr (NodalOf<Op>::on) op.load(ix.dl, cv.nd);
}

// One thread per output row; the block owns whole SELL-64 slices (blockDim a
// multiple of 64), accumulates their values in LDS in the SELL layout and
// writes them back as one contiguous, coalesced range. Values are of the op's
// working type (double, or float in the mixed form).
//
// The walk over a row's incident cells is software-pipelined: while cell p is
// evaluated, the coordinates and nodal values of cell p+1, the indices of cell
// p+2 and the incidence code of cell p+3 are in flight, so each cell costs
// about one memory latency overlapped with the previous cell's arithmetic
// instead of three in a row. Prefetches past the row's last cell re-read its
// last incidence entry and are discarded. The cells are evaluated and added in
// incidence order, as without the pipeline.
template <int D, class Op>
__global__ void __launch_bounds__(256) k_asm_rows(RowAsm a, Op op) {
  using R = typename Op::real;
  extern __shared__ double lds_raw[];
  R* lds = reinterpret_cast<R*>(lds_raw);
  constexpr int NOUT = Op::NOUT, NCOL = Op::NCOL;
  const int r0 = xcd_block(blockIdx.x, gridDim.x, a.xcd_chunk) * blockDim.x;
  const int s0 = r0 >> 6;
  const int s1 = min((r0 + (int)blockDim.x + 63) >> 6, (a.nrows + 63) >> 6);
  const int base = a.sptr[s0];
  const int bent = a.sptr[s1] - base;
  for (int k = threadIdx.x; k < NOUT * bent; k += blockDim.x) lds[k] = R(0);
  __syncthreads();
  const int row = r0 + threadIdx.x;
  if (row < a.nrows) {
    const int off = a.sptr[row >> 6] - base + (row & 63);
    const int pb = a.inc_ptr[row], pe = a.inc_ptr[row + 1];
    if (pb < pe) {
      const int last = pe - 1;
      // prologue: codes of cells pb, pb+1, pb+2; indices of pb, pb+1; values of pb
      int code = a.inc[pb];
      int code1 = a.inc[min(pb + 1, last)];
      int code2 = a.inc[min(pb + 2, last)];
      CellIdx<D, Op> ix;
      load_idx<D, Op>(a, code, ix);
      CellIdx<D, Op> ix1;
      load_idx<D, Op>(a, code1, ix1);
      CellVals<D, Op> cv;
      load_vals<D, Op>(a, op, ix, cv);
      for (int p = pb; p < pe; ++p) {
        // in flight during this cell's evaluation
        CellVals<D, Op> cv1;
        load_vals<D, Op>(a, op, ix1, cv1);
        CellIdx<D, Op> ix2;
        load_idx<D, Op>(a, code2, ix2);
        const int code3 = a.inc[min(p + 3, last)];
        const uint8_t* sl = a.slot + (size_t)p * a.stride;
        int sj[NCOL];
#pragma unroll
        for (int j = 0; j < NCOL; ++j) sj[j] = sl[j];
        // keep the loads above ahead of this cell's arithmetic
        __builtin_amdgcn_sched_barrier(0);
        const Geo<D, R> g = cell_geo_x<D, R>(cv.xc);
        R v[NOUT][NCOL];
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
          for (int j = 0; j < NCOL; ++j) v[o][j] = R(0);
        if constexpr (NodalOf<Op>::on) op(g, cv.nd, code & 31, v);
        else op(g, ix.dl, code & 31, v);
#pragma unroll
        for (int j = 0; j < NCOL; ++j) {
          const int s = off + 64 * sj[j];
#pragma unroll
          for (int o = 0; o < NOUT; ++o) lds[o * bent + s] += v[o][j];
        }
        code = code1;
        code1 = code2;
        code2 = code3;
        ix = ix1;
        ix1 = ix2;
        cv = cv1;
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < bent; k += blockDim.x)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) static_cast<R*>(a.out[o])[base + k] = lds[o * bent + k];
}

// The same for row blocks whose slices exceed the LDS of a block (P3 rows on
// tetrahedra reach 175 entries): each thread clears its own row in the output
// and accumulates into it there. Rows are still owned by one thread, so there
// are no atomics and the sums are formed in the same order as above.
template <int D, class Op>
__global__ void __launch_bounds__(256) k_asm_rows_g(RowAsm a, Op op) {
  using R = typename Op::real;
  constexpr int NOUT = Op::NOUT, NCOL = Op::NCOL;
  const int row = xcd_block(blockIdx.x, gridDim.x, a.xcd_chunk) * blockDim.x + threadIdx.x;
  if (row >= a.nrows) return;
  const int sl0 = row >> 6;
  const int w = (a.sptr[sl0 + 1] - a.sptr[sl0]) >> 6;
  const int off = a.sptr[sl0] + (row & 63);
  for (int k = 0; k < w; ++k)
#pragma unroll
    for (int o = 0; o < NOUT; ++o) static_cast<R*>(a.out[o])[off + 64 * k] = R(0);
  for (int p = a.inc_ptr[row]; p < a.inc_ptr[row + 1]; ++p) {
    const int code = a.inc[p];
    const int cell = code >> 5, li = code & 31;
    int32_t dl[Op::NDOF > 0 ? Op::NDOF : 1];
    if constexpr (Op::NDOF > 0) {
      const int32_t* dofs = a.c2d + (size_t)cell * a.nloc2;
#pragma unroll
      for (int m = 0; m < Op::NDOF; ++m) dl[m] = dofs[m];
    }
    int32_t vx[D + 1];
    cell_vertices<D>(a, cell, vx);
    const Geo<D, R> g = cell_geo<D, R>(a.X, vx);
    R v[NOUT][NCOL];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
      for (int j = 0; j < NCOL; ++j) v[o][j] = R(0);
    op(g, dl, li, v);
    const uint8_t* slp = a.slot + (size_t)p * a.stride;
#pragma unroll
    for (int j = 0; j < NCOL; ++j) {
      const int e = off + 64 * slp[j];
#pragma unroll
      for (int o = 0; o < NOUT; ++o) static_cast<R*>(a.out[o])[e] += v[o][j];
    }
  }
}

// lds == 0: the block's slices do not fit in LDS (global accumulation)
template <int D, class Op>
static void launch_rows(hipStream_t s, const RowAsm& a, const Op& op, int bs, size_t lds) {
  if (a.nrows <= 0) return;
  const int nb = (int)div_up(a.nrows, bs);
  if (lds == 0) launch(k_asm_rows_g<D, Op>, dim3(nb), dim3(bs), 0, s, a, op);
  else launch(k_asm_rows<D, Op>, dim3(nb), dim3(bs), (uint32_t)lds, s, a, op);
}

// Dispatch over dimension and working type.
template <template <int, class> class OpT, class... P>
static void rows_dr(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds,
                    P... prm) {
  if (dim == 2 && !fp32) launch_rows<2>(s, a, OpT<2, double>{prm...}, bs, lds);
  else if (dim == 2) launch_rows<2>(s, a, OpT<2, float>{prm...}, bs, lds);
  else if (!fp32) launch_rows<3>(s, a, OpT<3, double>{prm...}, bs, lds);
  else launch_rows<3>(s, a, OpT<3, float>{prm...}, bs, lds);
}

template <int D, class R>
using OpMass = OpMassStiff<D, 0, R>;
template <int D, class R>
using OpStiff = OpMassStiff<D, 1, R>;

template <int D, class R>
using Op3Mass = Op3MassStiff<D, 0, R>;
template <int D, class R>
using Op3Stiff = Op3MassStiff<D, 1, R>;

// a.out[0] <- M, a.out[1] <- K
void asm_mass_stiff(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds) {
  RowAsm am = a, ak = a;
  ak.out[0] = a.out[1];
  if (a.pair == IPCS_PAIR_P3P2) {
    need_tables(dim, a);
    rows_dr<Op3Mass>(dim, fp32, s, am, bs, lds);
    rows_dr<Op3Stiff>(dim, fp32, s, ak, bs, lds);
    return;
  }
  rows_dr<OpMass>(dim, fp32, s, am, bs, lds);
  rows_dr<OpStiff>(dim, fp32, s, ak, bs, lds);
}
void asm_conv(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds,
              const double* U, int64_t n2, double inv_dt, double cs) {
  if (a.pair == IPCS_PAIR_P3P2) {
    need_tables(dim, a);
    return rows_dr<Op3Conv>(dim, fp32, s, a, bs, lds, U, n2, inv_dt, cs);
  }
  rows_dr<OpConv>(dim, fp32, s, a, bs, lds, U, n2, inv_dt, cs);
}
// a.out[0] <- N_ce(U) (P2-P1, FP64; steady solver)
void asm_newton(int dim, hipStream_t s, const RowAsm& a, int bs, size_t lds, const double* U,
                int64_t n2, int c, int e) {
  if (a.pair == IPCS_PAIR_P3P2) fail(IPCS_E_INVALID, "the steady solver uses the P2-P1 pair");
  rows_dr<OpNewton>(dim, false, s, a, bs, lds, U, n2, c, e);
}
// a.out[c] <- G_c (one launch per component)
void asm_grad(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds) {
  need_tables(dim, a);
  for (int c = 0; c < dim; ++c) {
    RowAsm ac = a;
    ac.out[0] = a.out[c];
    if (a.pair == IPCS_PAIR_P3P2) rows_dr<Op3Grad>(dim, fp32, s, ac, bs, lds, c);
    else rows_dr<OpGrad>(dim, fp32, s, ac, bs, lds, c);
  }
}
// a.out[c] <- D_c
void asm_div(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds) {
  need_tables(dim, a);
  for (int c = 0; c < dim; ++c) {
    RowAsm ac = a;
    ac.out[0] = a.out[c];
    if (a.pair == IPCS_PAIR_P3P2) rows_dr<Op3Div>(dim, fp32, s, ac, bs, lds, c);
    else rows_dr<OpDiv>(dim, fp32, s, ac, bs, lds, c);
  }
}
void asm_kp(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds) {
  if (a.pair == IPCS_PAIR_P3P2) {
    need_tables(dim, a);
    return rows_dr<Op3Kp>(dim, fp32, s, a, bs, lds);
  }
  rows_dr<OpKp>(dim, fp32, s, a, bs, lds);
}

// ------------------------------------------------------------------ cell-batched convection
// E = M/dt + cs C(U) in two passes (used in 3D, both pairs). The row-owner
// kernel above (OpConv, Op3Conv) recomputes a cell's geometry and u_h at every
// quadrature point for each of the cell's rows (n_loc times): 10 times in 3D
// with P2 and 14 points, 20 times with P3 and 125 points, while in 2D (6 rows,
// 7 points) that recomputation costs less than storing and re-reading the
// local matrices; in 3D the rows of a slice also differ widely in their number
// of incident cells (a P3 vertex row has 24, a face row 2), which leaves lanes
// idle. Here a block first forms the local matrices of 256 / n_loc cells
// once, one thread per (cell, local row): the cell's threads share U at its
// DOFs, its geometry and the reference-frame velocity
// beta_q = J^{-1} u_h(x_q) at every quadrature point through LDS, and each
// thread forms its local row: for every quadrature point q,
//   v_j += w_q |det J| phi_li(x_q) (phi_j(x_q) / dt + cs beta_q . grad_ref phi_j(x_q)),
// the same operations in the same order as the row-owner ops. The local rows
// go to a buffer [cell][local row][local column]; k_asm_local then adds them
// into the matrix rows with the conflict-free row-owner scatter.

// The velocity element of a pair: local rows, rule points, tables.
template <int D, int P3, class R>
struct VelElem;
template <int D, class R>
struct VelElem<D, 0, R> {
  static constexpr int NL = P2<D>::NLOC, NQ = Rule<D>::NQ;
  __device__ static const Tab<D, R>& table() { return tab<D, R>(); }
};
template <int D, class R>
struct VelElem<D, 1, R> {
  static constexpr int NL = P3Of<D>::B::NLOC, NQ = P3Of<D>::template Tab<R>::NQ;
  __device__ static const typename P3Of<D>::template Tab<R>& table() { return tab3<D, R>(); }
};

template <int D, class R, int P3>
__global__ void __launch_bounds__(256) k_conv_cells(RowAsm a, int64_t nc, const double* U,
                                                    int64_t n2, double inv_dt, double cs, R* out) {
  using E = VelElem<D, P3, R>;
  const int32_t* c2d = a.c2d;
  const int nloc2 = a.nloc2;
  constexpr int NL = E::NL, NQ = E::NQ, CPB = 256 / NL;
  __shared__ R s_u[CPB][D][NL];          // U_c at the cell's DOFs
  __shared__ R s_beta[CPB][NQ][D];       // J^{-1} u_h(x_q)
  __shared__ R s_det[CPB];
  __shared__ R s_ji[CPB][D][D];
  const int cl = threadIdx.x / NL, li = threadIdx.x % NL;
  const int64_t cell = (int64_t)blockIdx.x * CPB + cl;
  const bool act = cl < CPB && cell < nc;
  const auto& T = E::table();
  int32_t dl[NL];
  if (act) {
#pragma unroll
    for (int m = 0; m < NL; ++m) dl[m] = c2d[cell * nloc2 + m];
#pragma unroll
    for (int c = 0; c < D; ++c) s_u[cl][c][li] = (R)U[(size_t)c * n2 + dl[li]];
    if (li == 0) {
      int32_t vx[D + 1];
      cell_vertices<D>(a, cell, vx);
      const Geo<D, R> g = cell_geo<D, R>(a.X, vx);
      s_det[cl] = g.det;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) s_ji[cl][a][c] = g.Ji[a][c];
    }
  }
  __syncthreads();
  if (act) {
    for (int q = li; q < NQ; q += NL) {
      R uq[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        R sum = 0;
#pragma unroll
        for (int m = 0; m < NL; ++m) sum += s_u[cl][c][m] * T.phi[q][m];
        uq[c] = sum;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        R sum = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) sum += s_ji[cl][a][c] * uq[c];
        s_beta[cl][q][a] = sum;
      }
    }
  }
  __syncthreads();
  const R idt = (R)inv_dt, csr = (R)cs, det = act ? s_det[cl] : R(0);
  R v[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) v[j] = R(0);
  // the factor d_qj = phi_j(x_q) / dt + cs beta_q . grad_ref phi_j(x_q) is the
  // same for every row of a cell: the cell's threads form it for a chunk of QC
  // points in LDS, then each row adds w_q |J| phi_li(x_q) d_qj over the chunk
  constexpr int QC = 5;
  __shared__ R s_d[CPB][QC][NL];
  for (int q0 = 0; q0 < NQ; q0 += QC) {
    if (act) {
      for (int e = li; e < QC * NL; e += NL) {
        const int q = q0 + e / NL, j = e % NL;
        if (q < NQ) {
          R adv = 0;
#pragma unroll
          for (int a = 0; a < D; ++a) adv += s_beta[cl][q][a] * T.dphi[q][j][a];
          s_d[cl][e / NL][j] = T.phi[q][j] * idt + csr * adv;
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int qq = 0; qq < QC; ++qq) {
        const int q = q0 + qq;
        if (q >= NQ) break;
        const R ci = T.w[q] * det * T.phi[q][li];
#pragma unroll
        for (int j = 0; j < NL; ++j) v[j] += ci * s_d[cl][qq][j];
      }
    }
    __syncthreads();
  }
  if (!act) return;
  R* o = out + ((size_t)cell * NL + li) * NL;
#pragma unroll
  for (int j = 0; j < NL; ++j) o[j] = v[j];
}

// Row-owner sum of stored local rows: row r adds local row li of each incident
// cell into its slots (the scatter of k_asm_rows, without recomputation).
template <int D, class R, int P3>
__global__ void __launch_bounds__(256) k_asm_local(RowAsm a, const R* loc) {
  constexpr int NL = VelElem<D, P3, R>::NL;
  extern __shared__ double lds_raw[];
  R* lds = reinterpret_cast<R*>(lds_raw);
  const int r0 = xcd_block(blockIdx.x, gridDim.x, a.xcd_chunk) * blockDim.x;
  const int s0 = r0 >> 6;
  const int s1 = min((r0 + (int)blockDim.x + 63) >> 6, (a.nrows + 63) >> 6);
  const int base = a.sptr[s0];
  const int bent = a.sptr[s1] - base;
  for (int k = threadIdx.x; k < bent; k += blockDim.x) lds[k] = R(0);
  __syncthreads();
  const int row = r0 + threadIdx.x;
  if (row < a.nrows) {
    const int off = a.sptr[row >> 6] - base + (row & 63);
    const int pb = a.inc_ptr[row], pe = a.inc_ptr[row + 1];
    // incident cells in batches of NB: the batch's codes, then its local rows
    // and slot indices, then the additions in incidence order (entries past
    // the row's last cell re-read it and are not added)
    constexpr int NB = NL <= 10 ? 4 : 2;
    for (int p = pb; p < pe; p += NB) {
      int code[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) code[k] = a.inc[min(p + k, pe - 1)];
      R v[NB][NL];
      int sj[NB][NL];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int cell = code[k] >> 5, li = code[k] & 31;
        const R* lr = loc + ((size_t)cell * NL + li) * NL;
        const uint8_t* sl = a.slot + (size_t)min(p + k, pe - 1) * a.stride;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          v[k][j] = lr[j];
          sj[k][j] = sl[j];
        }
      }
      // all of the batch's loads in flight before the first addition
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (p + k >= pe) break;
#pragma unroll
        for (int j = 0; j < NL; ++j) lds[off + 64 * sj[k][j]] += v[k][j];
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < bent; k += blockDim.x) static_cast<R*>(a.out[0])[base + k] = lds[k];
}

// The same where a block's slices exceed LDS: each thread clears its row in
// the output and accumulates there (same owner, same order of additions).
template <int D, class R, int P3>
__global__ void __launch_bounds__(256) k_asm_local_g(RowAsm a, const R* loc) {
  constexpr int NL = VelElem<D, P3, R>::NL;
  const int row = xcd_block(blockIdx.x, gridDim.x, a.xcd_chunk) * blockDim.x + threadIdx.x;
  if (row >= a.nrows) return;
  R* out = static_cast<R*>(a.out[0]);
  const int sl0 = row >> 6;
  const int w = (a.sptr[sl0 + 1] - a.sptr[sl0]) >> 6;
  const int off = a.sptr[sl0] + (row & 63);
  for (int k = 0; k < w; ++k) out[off + 64 * k] = R(0);
  for (int p = a.inc_ptr[row]; p < a.inc_ptr[row + 1]; ++p) {
    const int code = a.inc[p];
    const int cell = code >> 5, li = code & 31;
    const R* lr = loc + ((size_t)cell * NL + li) * NL;
    const uint8_t* sl = a.slot + (size_t)p * a.stride;
#pragma unroll
    for (int j = 0; j < NL; ++j) out[off + 64 * sl[j]] += lr[j];
  }
}

// ------------------------------------------------------------------ cell pass on matrix cores
// For the velocity elements with ten local rows (P2 on tetrahedra, P3 on
// triangles) the local matrices of a batch of cells are one dense product.
// With b_q = J^{-1} u_h(x_q) the reference-frame velocity (as above),
//   E_ij = (|J| / dt) Mref_ij + sum_{q, a} (cs |J| b_q[a]) (w_q phi_i(x_q) dref_a phi_j(x_q)),
// Mref_ij = sum_q w_q phi_i(x_q) phi_j(x_q): the row of a cell's K = D NQ + 1
// coefficients [cs |J| b_q[a] for every (q, a), |J| / dt] times the fixed
// table T[k][i NL + j] (K padded to a multiple of 4, the 100 columns to 112).
// A wavefront takes 16 cells as the M dimension of the 16x16x4 MFMA (FP32
// in the mixed form, FP64 otherwise), the table in 7 column tiles of 16 from
// LDS (each block builds it once from the FP64 reference tables), and writes
// the cells' local matrices to the buffer the local-sum pass reads. Lane l
// feeds row l mod 16 (its cell) and K slot l / 16 of each group of four; the
// slots are dealt to the four lane groups so that a lane forms b_q at as few
// quadrature points as possible.
template <int D, int NQ>
struct MfmaSlots {
  static constexpr int MASS = -1, PAD = -2;
  static constexpr int K = (D * NQ + 1 + 3) / 4 * 4, S = K / 4;
  // slot 4 s + g: q * 4 + a, MASS or PAD; point q's D items go to group
  // q mod 4 while it has room, else to the next group with room
  int item[K];
  constexpr MfmaSlots() : item() {
    int fill[4] = {0, 0, 0, 0};
    for (int k = 0; k < K; ++k) item[k] = PAD;
    for (int v = 0; v <= D * NQ; ++v) {
      const int q = v / D;
      int g = v < D * NQ ? q & 3 : 0;
      while (fill[g] >= S) g = (g + 1) & 3;
      item[4 * fill[g] + g] = v < D * NQ ? q * 4 + v % D : MASS;
      fill[g] += 1;
    }
  }
};
// the tables of the two elements the matrix-core pass serves, built at compile time
__constant__ MfmaSlots<3, Rule<3>::NQ> c_slots_tet_p2 = MfmaSlots<3, Rule<3>::NQ>();
__constant__ MfmaSlots<2, RuleT9::NQ> c_slots_tri_p3 = MfmaSlots<2, RuleT9::NQ>();

template <int D, int NQ>
__device__ __forceinline__ const MfmaSlots<D, NQ>& mfma_slots() {
  if constexpr (D == 3) return c_slots_tet_p2;
  else return c_slots_tri_p3;
}

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

template <class R>
__device__ __forceinline__ auto mfma16(R a, R b, typename std::conditional<std::is_same_v<R, float>, mf4, md4>::type c) {
  if constexpr (std::is_same_v<R, float>) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int D, class R, int P3>
__global__ void __launch_bounds__(256, 3) k_conv_cells_mfma(RowAsm a, int64_t nc, const double* U,
                                                         int64_t n2, double inv_dt, double cs,
                                                         R* out) {
  using E = VelElem<D, P3, double>;
  constexpr int NL = E::NL, NQ = E::NQ, NN = NL * NL, NT = (NN + 15) / 16, NC = 16 * NT;
  static_assert(NL == 10, "matrix-core cell pass: elements with ten local rows");
  using SL = MfmaSlots<D, NQ>;
  constexpr int K = SL::K, S = SL::S;
  using acc_t = typename std::conditional<std::is_same_v<R, float>, mf4, md4>::type;
  __shared__ R sT[K][NC];
  __shared__ R sPhi[NQ][NL];
  __shared__ int sItem[K];
  const auto& T = E::table();
  {
    static_assert(std::is_same_v<SL, std::remove_cv_t<std::remove_reference_t<decltype(mfma_slots<D, NQ>())>>>,
                  "slot table of this element");
    for (int k = threadIdx.x; k < K; k += blockDim.x) sItem[k] = mfma_slots<D, NQ>().item[k];
    for (int e = threadIdx.x; e < NQ * NL; e += blockDim.x)
      sPhi[e / NL][e % NL] = (R)T.phi[e / NL][e % NL];
    __syncthreads();
    for (int e = threadIdx.x; e < K * NC; e += blockDim.x) {
      const int k = e / NC, n = e % NC, it = sItem[k];
      double v = 0.0;
      if (n < NN && it != SL::PAD) {
        const int i = n / NL, j = n % NL;
        if (it == SL::MASS) {
          for (int q = 0; q < NQ; ++q) v += T.w[q] * T.phi[q][i] * T.phi[q][j];
        } else {
          const int q = it >> 2, c = it & 3;
          v = T.w[q] * T.phi[q][i] * T.dphi[q][j][c];
        }
      }
      sT[k][n] = (R)v;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
  const int64_t ntile = (nc + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntile;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t c0 = tile * 16;
    const int64_t cell = c0 + m < nc ? c0 + m : nc - 1;
    int32_t vx[D + 1];
    cell_vertices<D>(a, cell, vx);
    const Geo<D, R> geo = cell_geo<D, R>(a.X, vx);
    const int32_t* dofs = a.c2d + (size_t)cell * a.nloc2;
    R u[D][NL];
#pragma unroll
    for (int mm = 0; mm < NL; ++mm) {
      const int32_t dm = dofs[mm];
#pragma unroll
      for (int c = 0; c < D; ++c) u[c][mm] = (R)U[(size_t)c * n2 + dm];
    }
    const R idt = (R)inv_dt, csd = (R)cs * geo.det;
    R av[S];
    int qprev = -1;
    R uh[D] = {};
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      const int it = sItem[4 * sl + g];
      R v = R(0);
      if (it == SL::MASS) {
        v = geo.det * idt;
      } else if (it >= 0) {
        const int q = it >> 2, c = it & 3;
        if (q != qprev) {
#pragma unroll
          for (int cc = 0; cc < D; ++cc) {
            R sum = R(0);
#pragma unroll
            for (int mm = 0; mm < NL; ++mm) sum += u[cc][mm] * sPhi[q][mm];
            uh[cc] = sum;
          }
          qprev = q;
        }
        R b = R(0);   // (J^{-1} u_h)[c], the row chosen without an indexed array
#pragma unroll
        for (int r = 0; r < D; ++r) {
          R br = R(0);
#pragma unroll
          for (int cc = 0; cc < D; ++cc) br += geo.Ji[r][cc] * uh[cc];
          b = c == r ? br : b;
        }
        v = csd * b;
      }
      av[sl] = v;
    }
    acc_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
    // each slot's column tiles are read from LDS one slot ahead of its MFMAs
    R bt[2][NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bt[0][t] = sT[g][16 * t + m];
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      if (sl + 1 < S) {
#pragma unroll
        for (int t = 0; t < NT; ++t) bt[(sl + 1) & 1][t] = sT[4 * (sl + 1) + g][16 * t + m];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        // FP32: the transposed product (table as the first operand), so that a
        // lane ends with four consecutive entries of one cell
        if constexpr (std::is_same_v<R, float>) acc[t] = mfma16<R>(bt[sl & 1][t], av[sl], acc[t]);
        else acc[t] = mfma16<R>(av[sl], bt[sl & 1][t], acc[t]);
      }
    }
    if constexpr (std::is_same_v<R, float>) {
      // lane l: entries 16 t + 4 (l / 16) + r, r = 0..3, of cell c0 + l mod 16
      // (NN = 100 is a multiple of 4: a group of four is in range or not at all)
      const int64_t oc = c0 + m;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = 16 * t + 4 * g;
        if (n < NN && oc < nc) *reinterpret_cast<mf4*>(out + (size_t)oc * NN + n) = acc[t];
      }
    } else {
      // lane l: rows l / 16 + 4 r (cells) of column l mod 16 (entries)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = 16 * t + m;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t oc = c0 + g + 4 * r;
          if (n < NN && oc < nc) out[(size_t)oc * NN + n] = acc[t][r];
        }
      }
    }
  }
}

template <int D, class R, int P3>
static void conv_cells(hipStream_t s, const RowAsm& a, int64_t nc, const double* U, int64_t n2,
                       double inv_dt, double cs, void* buf) {
  constexpr int NL = VelElem<D, P3, R>::NL, CPB = 256 / NL;
  if (nc <= 0) return;
  if constexpr (NL == 10) {
    // matrix cores: one tile of 16 cells per wavefront, at most 8 blocks per CU
    const int64_t tiles = div_up(nc, 16);
    const unsigned nb = (unsigned)std::min<int64_t>(div_up(tiles, 4), 2048);
    launch(k_conv_cells_mfma<D, R, P3>, dim3(nb), dim3(256), 0, s, a, nc, U, n2, inv_dt, cs,
           static_cast<R*>(buf));
  } else {
    launch(k_conv_cells<D, R, P3>, dim3((unsigned)div_up(nc, CPB)), dim3(256), 0, s, a, nc, U, n2,
           inv_dt, cs, static_cast<R*>(buf));
  }
}

template <int D, class R, int P3>
static void local_sum(hipStream_t s, const RowAsm& a, int bs, size_t lds, const void* buf) {
  if (a.nrows <= 0) return;
  const dim3 grid((unsigned)div_up(a.nrows, bs));
  if (lds == 0)
    launch(k_asm_local_g<D, R, P3>, grid, dim3(bs), 0, s, a, static_cast<const R*>(buf));
  else
    launch(k_asm_local<D, R, P3>, grid, dim3(bs), (uint32_t)lds, s, a,
           static_cast<const R*>(buf));
}

// dispatch over dimension, working type and pair
template <class F>
static void with_dr_pair(int dim, bool fp32, int pair, F f) {
  auto d3 = [&](auto R) {
    if (pair == IPCS_PAIR_P3P2) f(std::integral_constant<int, 3>{}, R, std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 3>{}, R, std::integral_constant<int, 0>{});
  };
  auto d2 = [&](auto R) {
    if (pair == IPCS_PAIR_P3P2) f(std::integral_constant<int, 2>{}, R, std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 2>{}, R, std::integral_constant<int, 0>{});
  };
  if (dim == 2) {
    if (fp32) d2(float{});
    else d2(double{});
  } else {
    if (fp32) d3(float{});
    else d3(double{});
  }
}

void asm_conv_cells(int dim, bool fp32, hipStream_t s, const RowAsm& a, int64_t nc,
                    const double* U, int64_t n2, double inv_dt, double cs, void* buf) {
  need_tables(dim, a);
  with_dr_pair(dim, fp32, a.pair, [&](auto D, auto R, auto P) {
    conv_cells<decltype(D)::value, decltype(R), decltype(P)::value>(s, a, nc, U, n2, inv_dt, cs,
                                                                     buf);
  });
}

void asm_local_sum(int dim, bool fp32, hipStream_t s, const RowAsm& a, int bs, size_t lds,
                   const void* buf) {
  with_dr_pair(dim, fp32, a.pair, [&](auto D, auto R, auto P) {
    local_sum<decltype(D)::value, decltype(R), decltype(P)::value>(s, a, bs, lds, buf);
  });
}

// ------------------------------------------------------------------ vectors
// Lumped P1 mass w_k = sum over incident cells of |K|/(d+1).
template <int D>
__global__ void __launch_bounds__(256) k_lumped_p1(RowAsm a, double* w) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.nrows) return;
  double s = 0.0;
  for (int p = a.inc_ptr[row]; p < a.inc_ptr[row + 1]; ++p) {
    const int cell = a.inc[p] >> 5;
    int32_t dl[D + 1];
    cell_vertices<D>(a, cell, dl);
    s += cell_geo<D>(a.X, dl).det * (ref_measure<D>() / (D + 1));
  }
  w[row] = s;
}

// P2 pressure (P3-P2 pair): w_k = sum over incident cells of sum_q w_q |J| psi_k(x_q)
template <int D>
__global__ void __launch_bounds__(256) k_lumped_p2(RowAsm a, double* w) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.nrows) return;
  const auto& T = tab3<D, double>();
  double s = 0.0;
  for (int p = a.inc_ptr[row]; p < a.inc_ptr[row + 1]; ++p) {
    const int cell = a.inc[p] >> 5, li = a.inc[p] & 31;
    int32_t dl[D + 1];
    cell_vertices<D>(a, cell, dl);
    double iq = 0.0;
    for (int q = 0; q < T.NQ; ++q) iq += T.w[q] * T.psi[q][li];
    s += cell_geo<D>(a.X, dl).det * iq;
  }
  w[row] = s;
}

void asm_lumped_p1(int dim, hipStream_t s, const RowAsm& a, double* w) {
  const int nb = (int)div_up(a.nrows, 256);
  need_tables(dim, a);
  if (a.pair == IPCS_PAIR_P3P2 && dim == 2)
    hipLaunchKernelGGL((k_lumped_p2<2>), dim3(nb), dim3(256), 0, s, a, w);
  else if (a.pair == IPCS_PAIR_P3P2)
    hipLaunchKernelGGL((k_lumped_p2<3>), dim3(nb), dim3(256), 0, s, a, w);
  else if (dim == 2) hipLaunchKernelGGL((k_lumped_p1<2>), dim3(nb), dim3(256), 0, s, a, w);
  else hipLaunchKernelGGL((k_lumped_p1<3>), dim3(nb), dim3(256), 0, s, a, w);
  HIP_LAUNCH_OK();
}

// Forcing vector F_{c,i} = sum_q w_q |J| f_c(x_q, t) phi_i(x_q); f from a
// built-in closed form or from values fq[c][cell][q] supplied by the host.
template <int D>
__global__ void __launch_bounds__(256) k_forcing(RowAsm a, Builtin bi, const double* fq,
                                                 int64_t nc, double t, double* F, int64_t n2) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.nrows) return;
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int p = a.inc_ptr[row]; p < a.inc_ptr[row + 1]; ++p) {
    const int code = a.inc[p];
    const int cell = code >> 5, li = code & 31;
    int32_t dl[D + 1];
    cell_vertices<D>(a, cell, dl);
    const Geo<D> g = cell_geo<D>(a.X, dl);
    const Tab<D, double>& T = tab<D, double>();
#pragma unroll 1
    for (int q = 0; q < Rule<D>::NQ; ++q) {
      const double ci = T.w[q] * g.det * T.phi[q][li];
      double f[D];
      if (fq) {
#pragma unroll
        for (int c = 0; c < D; ++c)
          f[c] = fq[((size_t)c * nc + cell) * Rule<D>::NQ + q];
      } else {
        double x[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k <= D; ++k) s += T.lam[q][k] * a.X[(size_t)dl[k] * D + r];
          x[r] = s;
        }
        builtin_force<D>(bi, x, t, f);
      }
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += ci * f[c];
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) F[(size_t)c * n2 + row] = acc[c];
}

// The same for P3 velocity rows (P3-P2 pair) on its cell rule; fq holds f at
// the rule's NQ points per cell.
template <int D>
__global__ void __launch_bounds__(256) k_forcing_p3(RowAsm a, Builtin bi, const double* fq,
                                                    int64_t nc, double t, double* F, int64_t n2) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= a.nrows) return;
  const auto& T = tab3<D, double>();
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  for (int p = a.inc_ptr[row]; p < a.inc_ptr[row + 1]; ++p) {
    const int code = a.inc[p];
    const int cell = code >> 5, li = code & 31;
    int32_t dl[D + 1];
    cell_vertices<D>(a, cell, dl);
    const Geo<D> g = cell_geo<D>(a.X, dl);
#pragma unroll 1
    for (int q = 0; q < T.NQ; ++q) {
      const double ci = T.w[q] * g.det * T.phi[q][li];
      double f[D];
      if (fq) {
#pragma unroll
        for (int c = 0; c < D; ++c) f[c] = fq[((size_t)c * nc + cell) * T.NQ + q];
      } else {
        double x[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
          double sx = 0.0;
#pragma unroll
          for (int k = 0; k <= D; ++k) sx += T.lam[q][k] * a.X[(size_t)dl[k] * D + r];
          x[r] = sx;
        }
        builtin_force<D>(bi, x, t, f);
      }
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += ci * f[c];
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) F[(size_t)c * n2 + row] = acc[c];
}

void asm_forcing(int dim, hipStream_t s, const RowAsm& a, const Builtin& bi, const double* fq,
                 int64_t nc, double t, double* F, int64_t n2) {
  const int nb = (int)div_up(a.nrows, 256);
  need_tables(dim, a);
  if (a.pair == IPCS_PAIR_P3P2 && dim == 2)
    hipLaunchKernelGGL((k_forcing_p3<2>), dim3(nb), dim3(256), 0, s, a, bi, fq, nc, t, F, n2);
  else if (a.pair == IPCS_PAIR_P3P2)
    hipLaunchKernelGGL((k_forcing_p3<3>), dim3(nb), dim3(256), 0, s, a, bi, fq, nc, t, F, n2);
  else if (dim == 2)
    hipLaunchKernelGGL((k_forcing<2>), dim3(nb), dim3(256), 0, s, a, bi, fq, nc, t, F, n2);
  else
    hipLaunchKernelGGL((k_forcing<3>), dim3(nb), dim3(256), 0, s, a, bi, fq, nc, t, F, n2);
  HIP_LAUNCH_OK();
}

// ------------------------------------------------------------------ elimination
// out = cm*M + ck*K with Dirichlet rows and columns eliminated (zero, unit
// diagonal on boundary rows); dinv = 1/diag(out) in FP64. One thread per row,
// SELL-64 layout; padding entries are left untouched (zero). VT is the value
// type of M, K and out.
template <class VT>
__global__ void __launch_bounds__(256) k_form_elim(int64_t n, const int32_t* sptr,
                                                   const int32_t* rowptr, const int32_t* col,
                                                   const uint8_t* bmask, const VT* M,
                                                   const VT* K, double cm, double ck,
                                                   VT* out, double* dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool bi = bmask[i];
  const int len = rowptr[i + 1] - rowptr[i];
  const int base = sptr[i >> 6] + (int)(i & 63);
  double diag = 1.0;
  for (int k = 0; k < len; ++k) {
    const int idx = base + 64 * k;
    const int j = col[idx];
    VT v;
    if (bi || bmask[j]) v = (j == i) ? VT(1) : VT(0);
    else v = (VT)(cm * (double)M[idx] + (K ? ck * (double)K[idx] : 0.0));
    out[idx] = v;
    if (j == i) diag = (double)v;
  }
  dinv[i] = 1.0 / diag;
}

void form_eliminated(hipStream_t s, bool fp32, int64_t n, const int32_t* sptr,
                     const int32_t* rowptr, const int32_t* col, const uint8_t* bmask,
                     const void* M, const void* K, double cm, double ck, void* out,
                     double* dinv) {
  const dim3 g((unsigned)div_up(n, 256));
  if (fp32)
    hipLaunchKernelGGL(k_form_elim<float>, g, dim3(256), 0, s, n, sptr, rowptr, col, bmask,
                       (const float*)M, (const float*)K, cm, ck, (float*)out, dinv);
  else
    hipLaunchKernelGGL(k_form_elim<double>, g, dim3(256), 0, s, n, sptr, rowptr, col, bmask,
                       (const double*)M, (const double*)K, cm, ck, (double*)out, dinv);
  HIP_LAUNCH_OK();
}

template <class VT>
__global__ void k_inv_diag(int64_t n, const int32_t* sptr, const int32_t* rowptr,
                           const int32_t* col, const VT* val, double* dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int len = rowptr[i + 1] - rowptr[i];
  const int base = sptr[i >> 6] + (int)(i & 63);
  double d = 0.0;
  for (int k = 0; k < len; ++k)
    if (col[base + 64 * k] == i) d = (double)val[base + 64 * k];
  dinv[i] = 1.0 / d;
}

void inv_diagonal(hipStream_t s, bool fp32, int64_t n, const int32_t* sptr,
                  const int32_t* rowptr, const int32_t* col, const void* val, double* dinv) {
  const dim3 g((unsigned)div_up(n, 256));
  if (fp32)
    hipLaunchKernelGGL(k_inv_diag<float>, g, dim3(256), 0, s, n, sptr, rowptr, col,
                       (const float*)val, dinv);
  else
    hipLaunchKernelGGL(k_inv_diag<double>, g, dim3(256), 0, s, n, sptr, rowptr, col,
                       (const double*)val, dinv);
  HIP_LAUNCH_OK();
}

// Lifting values (FP64) of the boundary columns: out[e] = cm*M[slot] + ck*K[slot]
template <class VT>
__global__ void k_lift_vals(int64_t n, const int32_t* slot, const VT* M, const VT* K, double cm,
                            double ck, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int k = slot[e];
  out[e] = (double)(VT)(cm * (double)M[k] + (K ? ck * (double)K[k] : 0.0));
}

void lift_values(hipStream_t s, bool fp32, int64_t nlift, const int32_t* slot, const void* M,
                 const void* K, double cm, double ck, double* out) {
  if (nlift <= 0) return;
  const dim3 g((unsigned)div_up(nlift, 256));
  if (fp32)
    hipLaunchKernelGGL(k_lift_vals<float>, g, dim3(256), 0, s, nlift, slot, (const float*)M,
                       (const float*)K, cm, ck, out);
  else
    hipLaunchKernelGGL(k_lift_vals<double>, g, dim3(256), 0, s, nlift, slot, (const double*)M,
                       (const double*)K, cm, ck, out);
  HIP_LAUNCH_OK();
}

__global__ void k_round_f32(int64_t n, const double* src, float* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

void round_to_f32(hipStream_t s, int64_t n, const double* src, float* dst) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_round_f32, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, n, src, dst);
  HIP_LAUNCH_OK();
}

}  // namespace ipcs
