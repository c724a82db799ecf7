// Cell quadrature rules and P1/P2/P3 Lagrange bases on the reference simplex,
// usable from host and device code.
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

// ------------------------------------------------------------------ P3-P2 (triangles)
// Cell rule for the P3-P2 pair, whose convection integrand P3 (P3 . grad P3)
// has degree 8: the collapsed (Duffy) product of 5-point Gauss-Legendre rules.
// With x = u, y = v (1 - u) the triangle integral is the integral over the unit
// square of f(u, v (1 - u)) (1 - u); for f of degree <= 8 that integrand has
// degree <= 9 in u and <= 8 in v, which the 5-point rule integrates exactly
// (the rule is exact to degree 8, not 9: the factor 1 - u costs one degree).
// Gauss-Legendre on [-1, 1], 5 points: 0 and +-(1/3) sqrt(5 -+ 2 sqrt(10/7)),
// weights 128/225 and (322 +- 13 sqrt 70)/900; mapped to [0, 1] by t -> (1+t)/2
// with weights halved. Point q = 5 i + j takes u from node i and v from node j.
struct GL5 {
  __host__ __device__ static constexpr double t(int i) {
    constexpr double a = 0.5384693101056830910, b = 0.9061798459386639928;
    return i == 0 ? -b : i == 1 ? -a : i == 2 ? 0.0 : i == 3 ? a : b;
  }
  __host__ __device__ static constexpr double w(int i) {
    constexpr double wa = 0.4786286704993664680, wb = 0.2369268850561890875;
    return (i == 0 || i == 4) ? wb : (i == 1 || i == 3) ? wa : 128.0 / 225.0;
  }
};

struct RuleT9 {
  static constexpr int NQ = 25;
  __host__ __device__ static constexpr double u(int q) { return 0.5 * (1.0 + GL5::t(q / 5)); }
  __host__ __device__ static constexpr double v(int q) { return 0.5 * (1.0 + GL5::t(q % 5)); }
  // barycentric coordinates of x = u, y = v (1 - u): lam = (1 - x - y, x, y)
  __host__ __device__ static constexpr double lam(int q, int k) {
    const double x = u(q), y = v(q) * (1.0 - u(q));
    return k == 0 ? 1.0 - x - y : (k == 1 ? x : y);
  }
  __host__ __device__ static constexpr double w(int q) {
    return 0.25 * GL5::w(q / 5) * GL5::w(q % 5) * (1.0 - u(q));
  }
};

// P3 on triangles. Local order: v0, v1, v2; for each local edge (a, b) of
// (v1v2, v2v0, v0v1) the node at lam_a = 2/3, then the node at lam_b = 2/3; the
// centroid. Basis: vertex lam_i (3 lam_i - 1)(3 lam_i - 2) / 2; edge node p
// of edge (p, q) 9/2 lam_p lam_q (3 lam_p - 1); centroid 27 lam_0 lam_1 lam_2.
struct P3T {
  static constexpr int NV = 3;
  static constexpr int NLOC = 10;
  // for local node j = 3 + 2e + k: the nearer vertex p and the other q
  __host__ __device__ static constexpr int ep(int j) {
    return ((j - 3) & 1) ? Edges<2>::b((j - 3) >> 1) : Edges<2>::a((j - 3) >> 1);
  }
  __host__ __device__ static constexpr int eq(int j) {
    return ((j - 3) & 1) ? Edges<2>::a((j - 3) >> 1) : Edges<2>::b((j - 3) >> 1);
  }
  template <class T>
  __host__ __device__ static constexpr T phi(int j, const T* lam) {
    if (j < 3) return T(0.5) * lam[j] * (T(3) * lam[j] - T(1)) * (T(3) * lam[j] - T(2));
    if (j < 9) {
      const T lp = lam[ep(j)], lq = lam[eq(j)];
      return T(4.5) * lp * lq * (T(3) * lp - T(1));
    }
    return T(27) * lam[0] * lam[1] * lam[2];
  }
  template <class T>
  __host__ __device__ static constexpr T dphi(int j, int r, const T* lam) {
    if (j < 3)
      return T(0.5) * (T(27) * lam[j] * lam[j] - T(18) * lam[j] + T(2)) * P2<2>::dlam<T>(j, r);
    if (j < 9) {
      const int p = ep(j), q = eq(j);
      const T lp = lam[p], lq = lam[q];
      return T(4.5) * lq * (T(6) * lp - T(1)) * P2<2>::dlam<T>(p, r) +
             T(4.5) * lp * (T(3) * lp - T(1)) * P2<2>::dlam<T>(q, r);
    }
    return T(27) * (lam[1] * lam[2] * P2<2>::dlam<T>(0, r) + lam[0] * lam[2] * P2<2>::dlam<T>(1, r) +
                    lam[0] * lam[1] * P2<2>::dlam<T>(2, r));
  }
};

// ------------------------------------------------------------------ P3-P2 (tetrahedra)
// P3 on tetrahedra: 20 nodes. Local order: v0..v3; for each local edge (a, b)
// of (01, 02, 03, 12, 13, 23) the node at lam_a = 2/3, then the node at
// lam_b = 2/3; the centroids of the faces opposite v0, v1, v2, v3. Basis as
// on triangles; face node 27 lam_a lam_b lam_c.
struct P3Tet {
  static constexpr int NV = 4;
  static constexpr int NLOC = 20;
  __host__ __device__ static constexpr int ep(int j) {
    return ((j - 4) & 1) ? Edges<3>::b((j - 4) >> 1) : Edges<3>::a((j - 4) >> 1);
  }
  __host__ __device__ static constexpr int eq(int j) {
    return ((j - 4) & 1) ? Edges<3>::a((j - 4) >> 1) : Edges<3>::b((j - 4) >> 1);
  }
  // the m-th vertex (m = 0, 1, 2) of the face opposite vertex f
  __host__ __device__ static constexpr int fv(int f, int m) { return m < f ? m : m + 1; }
  template <class T>
  __host__ __device__ static constexpr T phi(int j, const T* lam) {
    if (j < 4) return T(0.5) * lam[j] * (T(3) * lam[j] - T(1)) * (T(3) * lam[j] - T(2));
    if (j < 16) {
      const T lp = lam[ep(j)], lq = lam[eq(j)];
      return T(4.5) * lp * lq * (T(3) * lp - T(1));
    }
    const int f = j - 16;
    return T(27) * lam[fv(f, 0)] * lam[fv(f, 1)] * lam[fv(f, 2)];
  }
  template <class T>
  __host__ __device__ static constexpr T dphi(int j, int r, const T* lam) {
    if (j < 4)
      return T(0.5) * (T(27) * lam[j] * lam[j] - T(18) * lam[j] + T(2)) * P2<3>::dlam<T>(j, r);
    if (j < 16) {
      const int p = ep(j), q = eq(j);
      const T lp = lam[p], lq = lam[q];
      return T(4.5) * lq * (T(6) * lp - T(1)) * P2<3>::dlam<T>(p, r) +
             T(4.5) * lp * (T(3) * lp - T(1)) * P2<3>::dlam<T>(q, r);
    }
    const int f = j - 16, a = fv(f, 0), b = fv(f, 1), c = fv(f, 2);
    return T(27) * (lam[b] * lam[c] * P2<3>::dlam<T>(a, r) + lam[a] * lam[c] * P2<3>::dlam<T>(b, r) +
                    lam[a] * lam[b] * P2<3>::dlam<T>(c, r));
  }
};

// Cell rule of the P3-P2 pair on tetrahedra: Stroud's conical product of
// 5-point Gauss-Jacobi rules (weights (1-u)^2, (1-v), 1 on [0, 1]), 125 points,
// exact to degree 9 (the convection integrand has degree 8). With
// x = u, y = v (1 - u), z = s (1 - u)(1 - v) the Jacobian (1-u)^2 (1-v) is the
// Jacobi weight. Nodes are the roots of the Jacobi polynomials P_5^(a,0) on
// [-1, 1] (Newton's method from a sign-change bracket), weights from the
// Gauss-Jacobi formula 2^(a+1) / ((1 - t^2) P_5'(t)^2) scaled to [0, 1]; built
// on the host (tet_rule9) and kept with the kernels' tables in device memory.
struct RuleTet9 {
  static constexpr int N1 = 5;
  static constexpr int NQ = N1 * N1 * N1;
};
// lam[NQ][4], w[NQ] (weights sum to 1/6)
void tet_rule9(double* lam, double* w);

// Integral of lam_k over the reference simplex is 1/(d!(d+1)).
template <int D>
__host__ __device__ constexpr double ref_measure() {
  return D == 2 ? 0.5 : 1.0 / 6.0;
}

}  // namespace ipcs
