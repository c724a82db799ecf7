// Degree-5 cell quadrature rules and P1/P2 Lagrange bases on the reference
// simplex, usable from host and device code.
//
// Every integrand of the IPCS step with P2-P1 elements (Section 2.2.1, eq. (9))
// is a polynomial of degree <= 5 on each cell (mass 4, convection 5, the rest
// <= 2), so a rule exact to degree 5 gives the matrices up to rounding.
//   triangle   : Radon's 7-point rule (Stroud T2:5-1), points (1/3,1/3,1/3),
//                (a,a,1-2a), (b,b,1-2b) with a,b = (6 -+ sqrt 15)/21 and weights
//                9/80, (155 -+ sqrt 15)/2400 (reference area 1/2).
//   tetrahedron: the symmetric 14-point degree-5 rule with orbits
//                (a,a,a,1-3a), (b,b,b,1-3b) and (c,c,1/2-c,1/2-c) (Walkington),
//                weights summing to the reference volume 1/6.
// Points are barycentric; lam_0 = 1 - sum xi.
#pragma once
#include <hip/hip_runtime.h>

namespace ipcs {

template <int D>
struct Rule;

template <>
struct Rule<2> {
  static constexpr int NQ = 7;
  // q = 0: centroid; q = 1..3: orbit a (1-2a at k = q-1); q = 4..6: orbit b
  __host__ __device__ static constexpr double lam(int q, int k) {
    constexpr double a = 0.1012865073234563388, a2 = 0.7974269853530873224;
    constexpr double b = 0.4701420641051150898, b2 = 0.05971587178976982046;
    return q == 0 ? 1.0 / 3.0 : (q <= 3 ? (k == q - 1 ? a2 : a) : (k == q - 4 ? b2 : b));
  }
  __host__ __device__ static constexpr double w(int q) {
    return q == 0 ? 0.1125 : (q <= 3 ? 0.06296959027241357630 : 0.06619707639425309037);
  }
};

template <>
struct Rule<3> {
  static constexpr int NQ = 14;
  // q = 0..3: orbit a (1-3a at k = q); q = 4..7: orbit b; q = 8..13: orbit c
  // with c on the two vertices of local edge q-8 (order 01,02,03,12,13,23)
  __host__ __device__ static constexpr double lam(int q, int k) {
    constexpr double a = 0.0927352503108912, a3 = 1.0 - 3.0 * 0.0927352503108912;
    constexpr double b = 0.3108859192633006, b3 = 1.0 - 3.0 * 0.3108859192633006;
    constexpr double c = 0.4544962958743504, ch = 0.5 - 0.4544962958743504;
    if (q < 4) return k == q ? a3 : a;
    if (q < 8) return k == q - 4 ? b3 : b;
    const int e = q - 8;
    const int ea = e < 3 ? 0 : (e < 5 ? 1 : 2);
    const int eb = e < 3 ? e + 1 : (e == 3 ? 2 : 3);
    return (k == ea || k == eb) ? c : ch;
  }
  __host__ __device__ static constexpr double w(int q) {
    return q < 4 ? 0.01224884051939366 : (q < 8 ? 0.01878132095300264 : 0.007091003462846911);
  }
};

// Local P2 node order: vertices, then edges. 2D: v1v2, v2v0, v0v1.
// 3D: 01, 02, 03, 12, 13, 23.
template <int D>
struct Edges;
template <>
struct Edges<2> {
  static constexpr int NE = 3;
  __host__ __device__ static constexpr int a(int e) { return e == 0 ? 1 : (e == 1 ? 2 : 0); }
  __host__ __device__ static constexpr int b(int e) { return e == 0 ? 2 : (e == 1 ? 0 : 1); }
};
template <>
struct Edges<3> {
  static constexpr int NE = 6;
  __host__ __device__ static constexpr int a(int e) { return e < 3 ? 0 : (e < 5 ? 1 : 2); }
  __host__ __device__ static constexpr int b(int e) {
    return e < 3 ? e + 1 : (e == 3 ? 2 : 3);
  }
};

template <int D>
struct P2 {
  static constexpr int NV = D + 1;
  static constexpr int NLOC = D + 1 + Edges<D>::NE;
  // value of basis function j at barycentric point lam
  template <class T>
  __host__ __device__ static constexpr T phi(int j, const T* lam) {
    if (j < NV) return lam[j] * (T(2) * lam[j] - T(1));
    const int e = j - NV;
    return T(4) * lam[Edges<D>::a(e)] * lam[Edges<D>::b(e)];
  }
  // derivative of basis function j with respect to reference coordinate x_r
  // (d lam_0/dx_r = -1, d lam_k/dx_r = delta_{k-1,r})
  template <class T>
  __host__ __device__ static constexpr T dlam(int k, int r) {
    return k == 0 ? T(-1) : (k - 1 == r ? T(1) : T(0));
  }
  template <class T>
  __host__ __device__ static constexpr T dphi(int j, int r, const T* lam) {
    if (j < NV) return (T(4) * lam[j] - T(1)) * dlam<T>(j, r);
    const int e = j - NV;
    const int ka = Edges<D>::a(e), kb = Edges<D>::b(e);
    return T(4) * (lam[kb] * dlam<T>(ka, r) + lam[ka] * dlam<T>(kb, r));
  }
};

// Integral of lam_k over the reference simplex is 1/(d!(d+1)).
template <int D>
__host__ __device__ constexpr double ref_measure() {
  return D == 2 ? 0.5 : 1.0 / 6.0;
}

}  // namespace ipcs
