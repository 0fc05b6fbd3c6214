// Metric terms of curved hexahedra from their geometry nodes, for the fused stage.
//
// Every 3D element carries its map x(xi) as the 27 nodes of a triquadratic Lagrange
// interpolant (equispaced nodes -1, 0, 1 per axis; straight elements are stored with
// their trilinear map evaluated at these nodes, which the triquadratic interpolant
// reproduces exactly).  From them a workgroup forms, in FP64:
//   * at every solution point, J = dx/dxi, S = |J| J^-1 (rows S_k = a_{k+1} x a_{k+2}
//     with a_k the columns of J) and 1/|J|;
//   * at every flux point on face (k, s), the face row S_k (which needs only the two
//     tangential columns, i.e. the face's nine nodes), the area factor A = |S_k| and the
//     outward unit normal (2s - 1) S_k / A.
// The volume columns are sum-factorised across the workgroup in LDS, axis by axis:
//   pass A   VA  = sum over a0 of l_a0(xi_i0) X and of l'_a0(xi_i0) X     (3 -> n along xi)
//            FA0 = on the faces xi = -1, +1 (a0 = 0, 2): sum over a1 of l, l' (along eta)
//            FA1 = on the faces eta = -1, +1 (a1 = 0, 2): sum over a0 of l, l' (along xi)
//   pass B   VB  = sum over a1 of l_a1(xi_i1) VA (both kinds) and of l'_a1(xi_i1) VA
//   point    J columns: sums over a2 of VB; the faces zeta = -1, +1 (a2 = 0, 2) read VB
//            directly, the xi and eta faces finish their sums over a2 from FA0, FA1.
// The functions below are the per-thread work of each pass; the caller separates the
// passes with workgroup barriers.  They are plain C++ so the same index arithmetic can be
// run on the host.
#pragma once

#include <cmath>
#include <cstdint>

#ifndef FR_HD
#define FR_HD __host__ __device__
#endif

// Keeps the device scheduler from hoisting the LDS reads of all three coordinates at once
// (their registers would add to the stage's prefetched loads); nothing on the host.
#if defined(__HIP_DEVICE_COMPILE__)
#define FR_GEOM_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define FR_GEOM_FENCE() ((void)0)
#endif

namespace fr {
namespace geom {

constexpr int NODES = 27;  // triquadratic geometry nodes a0 + 3 a1 + 9 a2

// LDS sizes and offsets, in doubles, for EW elements of N solution points per axis
template <int N, int EW> struct Lay {
  static constexpr int NVA = 54 * N;         // [c 3][i0 N][a1 3][a2 3][kind 2]
  static constexpr int NF0 = 36 * N;         // [s 2][c 3][i1 N][a2 3][kind 2]
  static constexpr int NF1 = 36 * N;         // [s 2][c 3][i0 N][a2 3][kind 2]
  static constexpr int NA = NVA + NF0 + NF1; // pass A outputs per element
  static constexpr int NB = 27 * N * N;      // [c 3][i0 N][i1 N][a2 3][kind 3]
  static constexpr int NX = NODES * 3;       // [a 27][c 3]
};

// Quadratic Lagrange basis (nodes -1, 0, 1) and its derivative at the N Gauss-Legendre
// points: gq[(kind * 3 + a) * N + i], kind 0 = l_a(xi_i), kind 1 = l_a'(xi_i).  The
// host fills the table from the FP64 Gauss-Legendre nodes.
template <int N> FR_HD inline double gw(const double *gq, int kind, int a, int i) { return gq[(kind * 3 + a) * N + i]; }

// X in LDS: node a, coordinate c of element slot e at Xl[(a * 3 + c) * EW + e]
template <int EW> FR_HD inline double xnode(const double *Xl, int e, int a, int c) { return Xl[(a * 3 + c) * EW + e]; }

// pass A, output t of NA * EW (element fastest): VA, FA0, FA1 back to back
template <int N, int EW>
FR_HD inline double pass_a(const double *Xl, const double *gq, int t) {
  using L = Lay<N, EW>;
  const int e = t % EW;
  int r = t / EW;
  double s = 0.0;
  if (r < L::NVA) {
    const int k = r % 2, a2 = (r / 2) % 3, a1 = (r / 6) % 3, i0 = (r / 18) % N, c = r / (18 * N);
    for (int a0 = 0; a0 < 3; ++a0) s += gw<N>(gq, k, a0, i0) * xnode<EW>(Xl, e, a0 + 3 * a1 + 9 * a2, c);
    return s;
  }
  r -= L::NVA;
  if (r < L::NF0) {  // face xi = -1 (sd 0) or +1 (sd 1): sum along eta
    const int k = r % 2, a2 = (r / 2) % 3, i1 = (r / 6) % N, c = (r / (6 * N)) % 3, sd = r / (18 * N);
    for (int a1 = 0; a1 < 3; ++a1) s += gw<N>(gq, k, a1, i1) * xnode<EW>(Xl, e, 2 * sd + 3 * a1 + 9 * a2, c);
    return s;
  }
  r -= L::NF0;
  {  // face eta = -1 or +1: sum along xi
    const int k = r % 2, a2 = (r / 2) % 3, i0 = (r / 6) % N, c = (r / (6 * N)) % 3, sd = r / (18 * N);
    for (int a0 = 0; a0 < 3; ++a0) s += gw<N>(gq, k, a0, i0) * xnode<EW>(Xl, e, a0 + 3 * (2 * sd) + 9 * a2, c);
    return s;
  }
}

template <int N, int EW> FR_HD inline int va(int e, int c, int i0, int a1, int a2, int k) {
  return ((((c * N + i0) * 3 + a1) * 3 + a2) * 2 + k) * EW + e;
}
template <int N, int EW> FR_HD inline int fa(int e, int sd, int c, int i, int a2, int k) {
  return (((((sd * 3 + c) * N + i) * 3 + a2) * 2 + k) * EW + e);
}
template <int N, int EW> FR_HD inline int vb(int e, int c, int i0, int i1, int a2, int k3) {
  return ((((c * N + i0) * N + i1) * 3 + a2) * 3 + k3) * EW + e;
}

// pass B, output t of NB * EW: kind 0 = (l, l), 1 = (l', l), 2 = (l, l') in (xi, eta)
template <int N, int EW>
FR_HD inline double pass_b(const double *A, const double *gq, int t) {
  const int e = t % EW, r = t / EW;
  const int k3 = r % 3, a2 = (r / 3) % 3, i1 = (r / 9) % N, i0 = (r / (9 * N)) % N, c = r / (9 * N * N);
  const int kin = k3 == 1 ? 1 : 0, kw = k3 == 2 ? 1 : 0;
  double s = 0.0;
  for (int a1 = 0; a1 < 3; ++a1) s += gw<N>(gq, kw, a1, i1) * A[va<N, EW>(e, c, i0, a1, a2, kin)];
  return s;
}

FR_HD inline void cross(const double u[3], const double v[3], double w[3]) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

// S = |J| J^-1 (S[k][c]) and |J| at solution point i = i0 + N i1 + N^2 i2 of slot e
template <int N, int EW>
FR_HD inline double point_metrics(const double *B, const double *gq, int e, int i, double S[3][3]) {
  const int i0 = i % N, i1 = (i / N) % N, i2 = i / (N * N);
  double l[3], d[3], a[3][3];  // a[k][c]: column k of J
  for (int a2 = 0; a2 < 3; ++a2) {
    l[a2] = gw<N>(gq, 0, a2, i2);
    d[a2] = gw<N>(gq, 1, a2, i2);
  }
  for (int c = 0; c < 3; ++c) {
    FR_GEOM_FENCE();
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int a2 = 0; a2 < 3; ++a2) {
      s0 += l[a2] * B[vb<N, EW>(e, c, i0, i1, a2, 1)];
      s1 += l[a2] * B[vb<N, EW>(e, c, i0, i1, a2, 2)];
      s2 += d[a2] * B[vb<N, EW>(e, c, i0, i1, a2, 0)];
    }
    a[0][c] = s0;
    a[1][c] = s1;
    a[2][c] = s2;
  }
  FR_GEOM_FENCE();
  cross(a[1], a[2], S[0]);
  cross(a[2], a[0], S[1]);
  cross(a[0], a[1], S[2]);
  return a[0][0] * S[0][0] + a[0][1] * S[0][1] + a[0][2] * S[0][2];
}

// face row S_k at flux point q = f * N^2 + m of slot e (f = 2k + s); returns A = |S_k|
// and writes the outward unit normal
template <int N, int EW>
FR_HD inline double face_metrics(const double *A, const double *B, const double *gq, int e, int q, double nrm[3]) {
  const int f = q / (N * N), m = q % (N * N), k = f / 2, sd = f % 2;
  const int p0 = m % N, p1 = m / N;  // face axes in increasing order, the lower fastest
  double u[3], v[3], Sk[3];
  if (k == 2) {  // zeta face: the xi and eta columns at a2 = 2 sd straight from pass B
    for (int c = 0; c < 3; ++c) {
      u[c] = B[vb<N, EW>(e, c, p0, p1, 2 * sd, 1)];
      v[c] = B[vb<N, EW>(e, c, p0, p1, 2 * sd, 2)];
    }
  } else {
    // xi face: (eta, zeta) = (p0, p1), columns a_1 = sum l'(eta) l(zeta) X, a_2 = l(eta) l'(zeta) X
    // eta face: (xi, zeta) = (p0, p1), columns a_2 = l(xi) l'(zeta) X, a_0 = l'(xi) l(zeta) X
    const double *F = A + Lay<N, EW>::NVA * EW + (k == 1 ? Lay<N, EW>::NF0 * EW : 0);
    double l[3], d[3];
    for (int a2 = 0; a2 < 3; ++a2) {
      l[a2] = gw<N>(gq, 0, a2, p1);
      d[a2] = gw<N>(gq, 1, a2, p1);
    }
    for (int c = 0; c < 3; ++c) {
      FR_GEOM_FENCE();
      double su = 0.0, sv = 0.0;
      for (int a2 = 0; a2 < 3; ++a2) {
        if (k == 0) {
          su += l[a2] * F[fa<N, EW>(e, sd, c, p0, a2, 1)];  // a_1
          sv += d[a2] * F[fa<N, EW>(e, sd, c, p0, a2, 0)];  // a_2
        } else {
          su += d[a2] * F[fa<N, EW>(e, sd, c, p0, a2, 0)];  // a_2
          sv += l[a2] * F[fa<N, EW>(e, sd, c, p0, a2, 1)];  // a_0
        }
      }
      u[c] = su;
      v[c] = sv;
    }
    FR_GEOM_FENCE();
  }
  cross(u, v, Sk);
  const double area = std::sqrt(Sk[0] * Sk[0] + Sk[1] * Sk[1] + Sk[2] * Sk[2]);
  const double sg = sd ? 1.0 : -1.0;
  for (int c = 0; c < 3; ++c) nrm[c] = sg * Sk[c] / area;
  return area;
}

}  // namespace geom
}  // namespace fr
