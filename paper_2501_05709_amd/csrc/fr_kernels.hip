// gfx950 kernels of the FR residual and RK4 update.
//
// Data layout (all per-element arrays): element blocks of EB = 16 elements,
// [block][point][channel][16], element fastest.  A wavefront reads the same
// point and channel of 16 consecutive elements, which is both the MFMA B
// operand (K = points, N = elements) and a coalesced 64/128-byte segment.
//
// The FR operators (interpolation to flux points, gradient, gradient
// correction, divergence with the interpolated normal-flux correction folded
// in, flux correction) are dense matrices applied to all elements of a block
// with v_mfma_*_16x16x4 (f32 or f64): one wave owns a 16-row tile of an
// operator's output for 16 elements and all variables, so the pointwise
// physics that follows runs in the epilogue on the accumulator registers:
// lane l holds four rows (MF<T>::row) of element l%16 for every variable.
//
// Stage sequence (Huynh's FR with BR1, classic RK4):
//   K_INTERP  u_f = M_int u                                  (MFMA)
//   K_FACE    u_c - u_f (BR1 mean or boundary value), Rusanov F_I*.n
//   K_GRAD    G = M_grad u + M_gcorr (u_c - u_f); grad u = S^T G/|J|;
//             F~ = S (F_inv - F_vis)                          (MFMA + epilogue)
//   K_VISC    grad u_f = M_int grad u; P = F_vis.n/2 (interior) or the full
//             boundary common flux; wall force terms           (MFMA + epilogue)
//   K_DIVRK   R = -(M_divS F~ + M_corr A(F_I* - P + P_nbr))/|J|; RK4 stage
//                                                              (MFMA + epilogue)
// Metric terms are FP64 in both precisions; the metric products are formed
// in FP64 and rounded to the working precision.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fr_internal.hpp"
#include "fr_geom.hpp"

namespace fr {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
// Accumulator rows held by lane group g = lane/16 in register j (column =
// lane % 16): f32 16x16x4 keeps four consecutive rows per group, f64 16x16x4
// interleaves them (measured on gfx950).
template <> struct MF<float> {
  using C = floatx4;
  __device__ static inline int row(int g, int j) { return 4 * g + j; }
  __device__ static inline C mac(float a, float b, C c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MF<double> {
  using C = doublex4;
  __device__ static inline int row(int g, int j) { return g + 4 * j; }
  __device__ static inline C mac(double a, double b, C c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <int DIM, int ORDER> struct Shape {
  static constexpr int N = ORDER + 1;
  static constexpr int NU = DIM == 2 ? N * N : N * N * N;
  static constexpr int NFP = DIM == 2 ? N : N * N;
  static constexpr int NF = 2 * DIM * NFP;
  static constexpr int NV = DIM + 2;
  static constexpr int NUP = (NU + 15) / 16 * 16;
  static constexpr int NFPAD = (NF + 15) / 16 * 16;
  static constexpr int KU = (NU + 3) / 4 * 4;
  static constexpr int KF = (NF + 3) / 4 * 4;
  static constexpr int RTU = NUP / 16, RTF = NFPAD / 16;
  static constexpr int KTU = KU / 4, KTF = KF / 4;
  static constexpr int NG = DIM * NV;  // gradient / transformed-flux channels
};

template <typename T> struct KArgs {
  T *U, *US, *ACC, *UF, *DU, *FI, *GU, *FT, *PV, *RES;
  const T *opInt, *opGrad, *opGcorr, *opDivS, *opCorr, *basis;
  const double *SM, *IJ, *FN, *FA, *bdt, *fsd, *wface;
  const double *XN, *GQ;
  const double *XC, *ZZ, *FCX;
  const double *IJC, *IZ;
  double *FC, *fsum, *stage64;
  const int *NB, *NBF, *bcount, *bdesign;
  const int64_t *bcanon, *wall_first;
  int *flag;
  const int *MO, *MG, *MC;
  const double *MW;
  const T *const *GUF, *const *GPV;
  T *MT;
  const int *PO, *PC;
  const double *PW;
  int64_t nblk, n_canon;
  int ndesign;
  int xcd;      // fused stage: map consecutive tiles to one XCD
  int scatter;  // trace interpolation: write each trace into its partner's slot
  T gam, mu, kappa, igm1;  // igm1 = 1/(gamma - 1)
};

// ---------------------------------------------------------------------------
// gas physics (paper Eqs. (1)-(7))
// ---------------------------------------------------------------------------

// reciprocal and square root: hardware rcp and sqrt (1 ulp) in the FP32 form,
// correctly rounded in FP64
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float sqrtv(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double sqrtv(double x) { return sqrt(x); }

template <typename T, int D> struct Gas {
  static constexpr int NV = D + 2;
  T gam, mu, kappa, igm1;  // igm1 = 1/(gamma - 1), formed on the host

  // pressure from the conserved state and 1/rho
  __device__ inline T pressure(const T *u, T ir) const {
    T ke = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) ke += u[1 + i] * u[1 + i];
    return (gam - T(1)) * (u[D + 1] - T(0.5) * ke * ir);
  }
  __device__ inline T pressure(const T *u) const { return pressure(u, recip(u[0])); }

  __device__ inline void flux_inv(const T *u, T F[D][NV]) const {
    const T ir = recip(u[0]);
    T v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = u[1 + i] * ir;
    const T p = pressure(u, ir);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      F[j][0] = u[1 + j];
#pragma unroll
      for (int i = 0; i < D; ++i) F[j][1 + i] = u[1 + i] * v[j] + (i == j ? p : T(0));
      F[j][D + 1] = v[j] * (u[D + 1] + p);
    }
  }

  // F_vis,j = (0, tau_ij, v_i tau_ij - q_j), q_j = -(mu gamma/Pr) de/dx_j;
  // g[j][var] = d(var)/dx_j.  adiabatic drops q.
  __device__ inline void flux_vis(const T *u, const T g[D][NV], T F[D][NV], bool adiabatic) const {
    const T ir = recip(u[0]);
    T v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = u[1 + i] * ir;
    const T E = u[D + 1] * ir;
    T dv[D][D], de[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T vdv = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        dv[i][j] = (g[j][1 + i] - v[i] * g[j][0]) * ir;
        vdv += v[i] * dv[i][j];
      }
      de[j] = (g[j][D + 1] - E * g[j][0]) * ir - vdv;
    }
    T div = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) div += dv[i][i];
    const T kap = adiabatic ? T(0) : kappa;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      F[j][0] = 0;
      T work = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const T tau = mu * (dv[i][j] + dv[j][i] - (i == j ? T(2.0 / 3.0) * div : T(0)));
        F[j][1 + i] = tau;
        work += v[i] * tau;
      }
      F[j][D + 1] = work + kap * de[j];
    }
  }

  // F_vis . n for a unit normal n, formed directly: (0, tau n, v . tau n - q . n)
  __device__ inline void flux_vis_n(const T *u, const T g[D][NV], const T *n, T *Fn, bool adiabatic) const {
    const T ir = recip(u[0]);
    T v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = u[1 + i] * ir;
    const T E = u[D + 1] * ir;
    T dv[D][D], qn = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T vdv = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        dv[i][j] = (g[j][1 + i] - v[i] * g[j][0]) * ir;
        vdv += v[i] * dv[i][j];
      }
      qn += ((g[j][D + 1] - E * g[j][0]) * ir - vdv) * n[j];
    }
    T div = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) div += dv[i][i];
    const T d23 = T(2.0 / 3.0) * div;
    T work = 0;
    Fn[0] = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T s = -d23 * n[i];
#pragma unroll
      for (int j = 0; j < D; ++j) s += (dv[i][j] + dv[j][i]) * n[j];
      Fn[1 + i] = mu * s;
      work += v[i] * Fn[1 + i];
    }
    Fn[D + 1] = adiabatic ? work : work + kappa * qn;
  }

  // Rusanov common flux for the outward unit normal n of the own side:
  // normal fluxes of both sides, wave speed max(|v.n| + c) of the two sides
  __device__ inline void rusanov(const T *uL, const T *uR, const T *n, T *Fn) const {
    const T irL = recip(uL[0]), irR = recip(uR[0]);
    T vnL = 0, vnR = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      vnL += uL[1 + j] * n[j];
      vnR += uR[1 + j] * n[j];
    }
    vnL *= irL;
    vnR *= irR;
    const T pL = pressure(uL, irL), pR = pressure(uR, irR);
    const T lamL = fabs(vnL) + sqrtv(gam * pL * irL);
    const T lamR = fabs(vnR) + sqrtv(gam * pR * irR);
    const T lam = lamL > lamR ? lamL : lamR;
    // F(u).n = (rho vn, rho v vn + p n, vn (rho E + p))
    Fn[0] = T(0.5) * (uL[0] * vnL + uR[0] * vnR) - T(0.5) * lam * (uR[0] - uL[0]);
#pragma unroll
    for (int i = 0; i < D; ++i)
      Fn[1 + i] = T(0.5) * (uL[1 + i] * vnL + pL * n[i] + uR[1 + i] * vnR + pR * n[i]) -
                  T(0.5) * lam * (uR[1 + i] - uL[1 + i]);
    Fn[D + 1] = T(0.5) * (vnL * (uL[D + 1] + pL) + vnR * (uR[D + 1] + pR)) - T(0.5) * lam * (uR[D + 1] - uL[D + 1]);
  }

  // Riemann-invariant far field: outgoing invariant from the interior,
  // incoming from the free stream; entropy and tangential velocity from the
  // upwind side.
  __device__ inline void farfield(const T *uL, const T *n, const double *fs, T *ub) const {
    const T rhoL = uL[0], irL = recip(rhoL);
    T vL[D], vI[D];
    T vnL = 0, vnI = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      vL[j] = uL[1 + j] * irL;
      vI[j] = T(fs[1 + j]);
      vnL += vL[j] * n[j];
      vnI += vI[j] * n[j];
    }
    const T pL = pressure(uL, irL);
    const T rhoI = T(fs[0]), pI = T(fs[4]);
    const T cL = sqrtv(gam * pL * irL), cI = sqrtv(gam * pI / rhoI);
    const T Rp = vnL + T(2) * cL * igm1;
    const T Rm = vnI - T(2) * cI * igm1;
    const T vnb = T(0.5) * (Rp + Rm);
    const T cb = T(0.25) * (gam - T(1)) * (Rp - Rm);
    T s, vt[D];
    if (vnb < T(0)) {
      s = pI / pow(rhoI, gam);
#pragma unroll
      for (int j = 0; j < D; ++j) vt[j] = vI[j] - vnI * n[j];
    } else {
      s = pL / pow(rhoL, gam);
#pragma unroll
      for (int j = 0; j < D; ++j) vt[j] = vL[j] - vnL * n[j];
    }
    const T rhob = pow(cb * cb / (gam * s), igm1);
    const T pb = rhob * cb * cb / gam;
    T ke = 0;
    ub[0] = rhob;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const T vb = vt[j] + vnb * n[j];
      ub[1 + j] = rhob * vb;
      ke += vb * vb;
    }
    ub[D + 1] = pb * igm1 + T(0.5) * rhob * ke;
  }

  // no-slip adiabatic wall: common solution with zero velocity
  __device__ inline void wall_common(const T *uL, T *uc) const {
    T ke = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) ke += uL[1 + i] * uL[1 + i];
    uc[0] = uL[0];
#pragma unroll
    for (int i = 0; i < D; ++i) uc[1 + i] = 0;
    uc[D + 1] = uL[D + 1] - T(0.5) * ke * recip(uL[0]);
  }
};

__device__ inline size_t at(int64_t blk, int pt, int ch, int e, int NPT, int NCH) {
  return lay(blk, pt, ch, e, NPT, NCH);
}

// The same arrays addressed as the block's base (wave-uniform: scalar registers) plus a
// 32-bit byte offset per lane within the block, so that loads and stores take the
// global "scalar base + vector offset" form instead of 64-bit address arithmetic in
// every lane. One block of any per-element array spans far less than 4 GiB.
template <typename T> __device__ inline T *blk_base(T *p, int64_t blk, int NPT, int NCH) {
  return p + size_t(blk) * size_t(NSB * NPT * NCH * SB);
}
__device__ inline unsigned lay_in(int pt, int ch, int e, int NPT, int NCH) {
  return ((unsigned(e) / SB * unsigned(NPT) + unsigned(pt)) * unsigned(NCH) + unsigned(ch)) * SB + unsigned(e) % SB;
}
template <typename T> __device__ inline T &in_blk(T *base, unsigned off) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return *reinterpret_cast<T *>(reinterpret_cast<C *>(base) + off * unsigned(sizeof(T)));
}

// ---------------------------------------------------------------------------
// reference-element index maps (conventions of include/fr.h)
// ---------------------------------------------------------------------------
template <int DIM, int N> struct Ref {
  // the line through face point m of a face on axis k: solution point base + j * stride
  // at position j.  Written with selects, not branches, because k is a run-time value
  // in the flux-point passes.
  __device__ static inline void line_of(int k, int m, int &base, int &stride) {
    if (DIM == 2) {
      base = k == 0 ? N * m : m;
      stride = k == 0 ? 1 : N;
      return;
    }
    const int a = m % N, b = m / N;
    const int sa = k == 0 ? N : 1, sb = k == 2 ? N : N * N;
    base = a * sa + b * sb;
    stride = k == 0 ? 1 : (k == 1 ? N : N * N);
  }
  __device__ static inline int line(int k, int m, int j) {
    int base, stride;
    line_of(k, m, base, stride);
    return base + j * stride;
  }
  // position along axis k and face-point index of solution point i
  __device__ static inline void locate(int i, int k, int &ik, int &m) {
    const int c0 = i % N, c1 = (i / N) % N, c2 = i / (N * N);
    if (DIM == 2) {
      ik = k == 0 ? c0 : c1;
      m = k == 0 ? c1 : c0;
      return;
    }
    if (k == 0) { ik = c0; m = c1 + N * c2; }
    else if (k == 1) { ik = c1; m = c0 + N * c2; }
    else { ik = c2; m = c0 + N * c1; }
  }
};

// ---------------------------------------------------------------------------
// epilogues shared by the dense-MFMA and the sum-factorised kernels
// ---------------------------------------------------------------------------

// physical gradient grad u = S^T G / |J| and transformed flux F~ = S (F_inv - F_vis)
// at solution point i of element slot e; G is the corrected reference gradient
template <typename T, int DIM, int ORDER>
__device__ inline void grad_epilogue(const KArgs<T> &a, const Gas<T, DIM> &gas, int64_t blk, int i, int e,
                                     const T *u, const T G[DIM][DIM + 2]) {
  using S = Shape<DIM, ORDER>;
  double Sm[DIM][DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int c = 0; c < DIM; ++c) Sm[k][c] = a.SM[at(blk, i, k * DIM + c, e, S::NUP, DIM * DIM)];
  const double ij = a.IJ[lay(blk, i, 0, e, S::NUP, 1)];
  T gu[DIM][S::NV];
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) s += Sm[k][c] * double(G[k][v]);
      gu[c][v] = T(s * ij);
    }
  T Fi[DIM][S::NV], Fv[DIM][S::NV];
  gas.flux_inv(u, Fi);
  gas.flux_vis(u, gu, Fv, false);
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int v = 0; v < S::NV; ++v) a.GU[at(blk, i, c * S::NV + v, e, S::NUP, S::NG)] = gu[c][v];
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < DIM; ++c) s += Sm[k][c] * double(Fi[c][v] - Fv[c][v]);
      a.FT[at(blk, i, k * S::NV + v, e, S::NUP, S::NG)] = T(s);
    }
}

// viscous part of the common flux at flux point q from the gradient trace gf:
// interior -> half the own viscous normal flux; boundary -> the full common flux
template <typename T, int DIM, int ORDER>
__device__ inline void visc_epilogue(const KArgs<T> &a, const Gas<T, DIM> &gas, int64_t blk, int q, int e,
                                     const T gf[DIM][DIM + 2], int forces) {
  using S = Shape<DIM, ORDER>;
  T uf[S::NV], n[DIM], pv[S::NV];
#pragma unroll
  for (int v = 0; v < S::NV; ++v) uf[v] = a.UF[at(blk, q, v, e, S::NFPAD, S::NV)];
  double nd[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    nd[c] = a.FN[at(blk, q, c, e, S::NFPAD, DIM)];
    n[c] = T(nd[c]);
  }
  const int nb = a.NB[lay(blk, q, 0, e, S::NFPAD, 1)];
  T fn[S::NV];
  if (nb >= 0) {
    gas.flux_vis_n(uf, gf, n, fn, false);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) pv[v] = T(0.5) * fn[v];
  } else {
    const int code = -nb;
    T ub[S::NV];
    if ((code & 3) == BC_FARFIELD) {
      gas.farfield(uf, n, a.fsd + 5 * a.bdesign[blk], ub);
      gas.flux_vis_n(ub, gf, n, fn, false);
    } else {
      gas.wall_common(uf, ub);
      gas.flux_vis_n(ub, gf, n, fn, true);
    }
#pragma unroll
    for (int v = 0; v < S::NV; ++v) pv[v] = a.FI[at(blk, q, v, e, S::NFPAD, S::NV)] - fn[v];
    if (forces && (code & 3) == BC_WALL) {
      // traction of the fluid on the body: W A (p n - tau . n), interior trace
      T Fw[DIM][S::NV];
      gas.flux_vis(uf, gf, Fw, false);
      const double p = double(gas.pressure(uf));
      const double wA = a.wface[q] * a.FA[lay(blk, q, 0, e, S::NFPAD, 1)];
      const int64_t w = code >> 2;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        double tn = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) tn += double(Fw[c][1 + i]) * nd[c];
        a.FC[w * 3 + i] = wA * (p * nd[i] - tn);
      }
      if (DIM == 2) a.FC[w * 3 + 2] = 0.0;
    }
  }
#pragma unroll
  for (int v = 0; v < S::NV; ++v) a.PV[at(blk, q, v, e, S::NFPAD, S::NV)] = pv[v];
}

// transformed outward common normal flux at flux point q: A (F_I* - P + P_nbr), or A P at a boundary
template <typename T, int DIM, int ORDER>
__device__ inline void common_flux(const KArgs<T> &a, int64_t blk, int q, int e, T *b) {
  using S = Shape<DIM, ORDER>;
  const size_t fq = lay(blk, q, 0, e, S::NFPAD, 1);
  const int nb = a.NB[fq];
  const double A = a.FA[fq];
  if (nb >= 0) {
    const size_t base = size_t(nb / SB) * S::NV * SB + (nb % SB);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      const T f = a.FI[at(blk, q, v, e, S::NFPAD, S::NV)] - a.PV[at(blk, q, v, e, S::NFPAD, S::NV)] +
                  a.PV[base + v * SB];
      b[v] = T(A * double(f));
    }
  } else {
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = T(A * double(a.PV[at(blk, q, v, e, S::NFPAD, S::NV)]));
  }
}

// R = -div / |J| and the RK4 stage update at solution point i
template <typename T, int DIM, int ORDER>
__device__ inline void rk_epilogue(const KArgs<T> &a, int64_t blk, int i, int e, const T *div, int mode, int &bad) {
  using S = Shape<DIM, ORDER>;
  const double ij = a.IJ[lay(blk, i, 0, e, S::NUP, 1)];
  const T dt = T(a.bdt[blk]);
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    const size_t x = at(blk, i, v, e, S::NUP, S::NV);
    const T r = T(-double(div[v]) * ij);
    if (mode == MODE_RESID) {
      a.RES[x] = r;
    } else if (mode == MODE_RK0) {
      a.ACC[x] = r;
      a.US[x] = a.U[x] + T(0.5) * dt * r;
    } else if (mode == MODE_RK1) {
      a.ACC[x] += T(2) * r;
      a.US[x] = a.U[x] + T(0.5) * dt * r;
    } else if (mode == MODE_RK2) {
      a.ACC[x] += T(2) * r;
      a.US[x] = a.U[x] + dt * r;
    } else {
      const T un = a.U[x] + dt / T(6) * (a.ACC[x] + r);
      a.U[x] = un;
      bad |= !isfinite(un);
    }
  }
}

// ---------------------------------------------------------------------------
// K_FACE: common solution and Rusanov flux, one thread per element flux point
// ---------------------------------------------------------------------------
// u_c - u_f (BR1 mean, far-field ghost or wall value) and the Rusanov flux at
// flux point q, from the element's own trace uf and its partner's trace
template <typename T, int DIM, int ORDER>
__device__ inline void face_common(const KArgs<T> &a, const Gas<T, DIM> &gas, int64_t blk, int q, int e,
                                   const T *uf, T *du, T *fi) {
  using S = Shape<DIM, ORDER>;
  T ur[S::NV], n[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) n[j] = T(a.FN[at(blk, q, j, e, S::NFPAD, DIM)]);
  const int nb = a.NB[lay(blk, q, 0, e, S::NFPAD, 1)];
  if (nb >= 0) {
    const size_t base = size_t(nb / SB) * S::NV * SB + (nb % SB);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      ur[v] = a.UF[base + v * SB];
      du[v] = T(0.5) * (ur[v] - uf[v]);
    }
  } else if (((-nb) & 3) == BC_FARFIELD) {
    gas.farfield(uf, n, a.fsd + 5 * a.bdesign[blk], ur);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) du[v] = ur[v] - uf[v];
  } else {
    T uc[S::NV];
    gas.wall_common(uf, uc);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) du[v] = uc[v] - uf[v];
    ur[0] = uf[0];
#pragma unroll
    for (int i = 0; i < DIM; ++i) ur[1 + i] = -uf[1 + i];
    ur[DIM + 1] = uf[DIM + 1];
  }
  gas.rusanov(uf, ur, n, fi);
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_face(KArgs<T> a) {
  using S = Shape<DIM, ORDER>;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int e = int(t & 15);
  const int q = int((t >> 4) % S::NFPAD);
  const int64_t blk = (t >> 4) / S::NFPAD;
  if (blk >= a.nblk || q >= S::NF || e >= a.bcount[blk]) return;
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa, a.igm1};
  T uf[S::NV], du[S::NV], fi[S::NV];
#pragma unroll
  for (int v = 0; v < S::NV; ++v) uf[v] = a.UF[at(blk, q, v, e, S::NFPAD, S::NV)];
  face_common<T, DIM, ORDER>(a, gas, blk, q, e, uf, du, fi);
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    a.DU[at(blk, q, v, e, S::NFPAD, S::NV)] = du[v];
    a.FI[at(blk, q, v, e, S::NFPAD, S::NV)] = fi[v];
  }
}

// ---------------------------------------------------------------------------
// dense-MFMA kernels: one wave = one 16-row tile of an operator x 16 elements
// ---------------------------------------------------------------------------
template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_interp(KArgs<T> a, const T *__restrict__ X) {
  using S = Shape<DIM, ORDER>;
  using M = MF<T>;
  const int lane = threadIdx.x & 63;
  const int64_t gw = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (gw >= a.nblk * S::RTF) return;
  const int64_t blk = gw / S::RTF;
  const int rt = int(gw % S::RTF);
  const int g = lane >> 4, e = lane & 15;
  typename M::C acc[S::NV];
#pragma unroll
  for (int v = 0; v < S::NV; ++v) acc[v] = typename M::C{0, 0, 0, 0};
  const T *Xb = X + lay(blk, 0, 0, e, S::NUP, S::NV);
#pragma unroll 4
  for (int kt = 0; kt < S::KTU; ++kt) {
    const T av = a.opInt[(size_t(rt) * S::KTU + kt) * 64 + lane];
    const int pt = kt * 4 + g;
#pragma unroll
    for (int v = 0; v < S::NV; ++v) acc[v] = M::mac(av, Xb[(pt * S::NV + v) * SB], acc[v]);
  }
  if (e >= a.bcount[blk]) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int q = rt * 16 + M::row(g, j);
    if (q < S::NF) {
#pragma unroll
      for (int v = 0; v < S::NV; ++v) a.UF[at(blk, q, v, e, S::NFPAD, S::NV)] = acc[v][j];
    }
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_grad(KArgs<T> a, const T *__restrict__ X) {
  using S = Shape<DIM, ORDER>;
  using M = MF<T>;
  const int lane = threadIdx.x & 63;
  const int64_t gw = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (gw >= a.nblk * S::RTU) return;
  const int64_t blk = gw / S::RTU;
  const int rt = int(gw % S::RTU);
  const int g = lane >> 4, e = lane & 15;
  typename M::C acc[DIM][S::NV];
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int v = 0; v < S::NV; ++v) acc[k][v] = typename M::C{0, 0, 0, 0};
  const T *Xb = X + lay(blk, 0, 0, e, S::NUP, S::NV);
#pragma unroll 2
  for (int kt = 0; kt < S::KTU; ++kt) {
    const int pt = kt * 4 + g;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = Xb[(pt * S::NV + v) * SB];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const T av = a.opGrad[((size_t(k) * S::RTU + rt) * S::KTU + kt) * 64 + lane];
#pragma unroll
      for (int v = 0; v < S::NV; ++v) acc[k][v] = M::mac(av, b[v], acc[k][v]);
    }
  }
  const T *Db = a.DU + lay(blk, 0, 0, e, S::NFPAD, S::NV);
#pragma unroll 2
  for (int kt = 0; kt < S::KTF; ++kt) {
    const int pt = kt * 4 + g;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = Db[(pt * S::NV + v) * SB];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const T av = a.opGcorr[((size_t(k) * S::RTU + rt) * S::KTF + kt) * 64 + lane];
#pragma unroll
      for (int v = 0; v < S::NV; ++v) acc[k][v] = M::mac(av, b[v], acc[k][v]);
    }
  }
  if (e >= a.bcount[blk]) return;
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa, a.igm1};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = rt * 16 + M::row(g, j);
    if (i >= S::NU) break;
    T u[S::NV], G[DIM][S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) u[v] = Xb[(i * S::NV + v) * SB];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int v = 0; v < S::NV; ++v) G[k][v] = acc[k][v][j];
    grad_epilogue<T, DIM, ORDER>(a, gas, blk, i, e, u, G);
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_visc(KArgs<T> a, int forces) {
  using S = Shape<DIM, ORDER>;
  using M = MF<T>;
  const int lane = threadIdx.x & 63;
  const int64_t gw = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (gw >= a.nblk * S::RTF) return;
  const int64_t blk = gw / S::RTF;
  const int rt = int(gw % S::RTF);
  const int g = lane >> 4, e = lane & 15;
  typename M::C acc[DIM][S::NV];
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int v = 0; v < S::NV; ++v) acc[k][v] = typename M::C{0, 0, 0, 0};
  const T *Gb = a.GU + lay(blk, 0, 0, e, S::NUP, S::NG);
#pragma unroll 2
  for (int kt = 0; kt < S::KTU; ++kt) {
    const T av = a.opInt[(size_t(rt) * S::KTU + kt) * 64 + lane];
    const int pt = kt * 4 + g;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int v = 0; v < S::NV; ++v)
        acc[k][v] = M::mac(av, Gb[(pt * S::NG + k * S::NV + v) * SB], acc[k][v]);
  }
  if (e >= a.bcount[blk]) return;
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa, a.igm1};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int q = rt * 16 + M::row(g, j);
    if (q >= S::NF) break;
    T gf[DIM][S::NV];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int v = 0; v < S::NV; ++v) gf[c][v] = acc[c][v][j];
    visc_epilogue<T, DIM, ORDER>(a, gas, blk, q, e, gf, forces);
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_divrk(KArgs<T> a, int mode) {
  using S = Shape<DIM, ORDER>;
  using M = MF<T>;
  const int lane = threadIdx.x & 63;
  const int64_t gw = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (gw >= a.nblk * S::RTU) return;
  const int64_t blk = gw / S::RTU;
  const int rt = int(gw % S::RTU);
  const int g = lane >> 4, e = lane & 15;
  const int nvalid = a.bcount[blk];
  typename M::C acc[S::NV];
#pragma unroll
  for (int v = 0; v < S::NV; ++v) acc[v] = typename M::C{0, 0, 0, 0};
  const T *Fb = a.FT + lay(blk, 0, 0, e, S::NUP, S::NG);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
#pragma unroll 2
    for (int kt = 0; kt < S::KTU; ++kt) {
      const T av = a.opDivS[((size_t(rt) * DIM + k) * S::KTU + kt) * 64 + lane];
      const int pt = kt * 4 + g;
#pragma unroll
      for (int v = 0; v < S::NV; ++v) acc[v] = M::mac(av, Fb[(pt * S::NG + k * S::NV + v) * SB], acc[v]);
    }
  }
#pragma unroll 2
  for (int kt = 0; kt < S::KTF; ++kt) {
    const T av = a.opCorr[(size_t(rt) * S::KTF + kt) * 64 + lane];
    const int q = kt * 4 + g;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = 0;
    if (q < S::NF && e < nvalid) common_flux<T, DIM, ORDER>(a, blk, q, e, b);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) acc[v] = M::mac(av, b[v], acc[v]);
  }
  if (e >= nvalid) return;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = rt * 16 + M::row(g, j);
    if (i >= S::NU) break;
    T div[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) div[v] = acc[v][j];
    rk_epilogue<T, DIM, ORDER>(a, blk, i, e, div, mode, bad);
  }
  if (bad) atomicOr(a.flag, 1);
}

// ---------------------------------------------------------------------------
// sum-factorised kernels: a workgroup stages the inputs of EW elements in LDS
// ([point][channel][EW], element fastest) and applies the 1D operators along
// the solution-point lines; outputs and epilogues are those of the dense kernels
// ---------------------------------------------------------------------------
template <typename T, int DIM, int ORDER> struct TS {
  using S = Shape<DIM, ORDER>;
  static constexpr int ew(int bytes) {
    return bytes * 16 <= 65536 ? 16 : bytes * 8 <= 65536 ? 8 : bytes * 4 <= 65536 ? 4 : 2;
  }
  static constexpr int EW_INTERP = ew(S::NU * S::NV * int(sizeof(T)));
  static constexpr int EW_GRAD = ew((S::NU + S::NF) * S::NV * int(sizeof(T)));
  static constexpr int EW_VISC = ew(S::NU * S::NG * int(sizeof(T)));
  static constexpr int EW_DIV = ew((S::NU * S::NG + S::NF * S::NV) * int(sizeof(T)));
};

// 1D basis in LDS: D[N][N], l(-1)[N], l(+1)[N], gL'[N], gR'[N], and the
// strong-form divergence operator Dv = D - gR' l(+1)^T - gL' l(-1)^T (the
// derivative of the flux polynomial minus its interpolated face corrections)
template <typename T, int N> struct Basis {
  static constexpr int COUNT = 2 * N * N + 4 * N;
  T D[N][N], lm[N], lp[N], gl[N], gr[N], Dv[N][N];
  // entry t of the members taken in order, the order of the source array
  __device__ inline void put(int t, T v) { reinterpret_cast<T *>(this)[t] = v; }
  __device__ inline void load(const T *src) {
    for (int t = threadIdx.x; t < 2 * N * N + 4 * N; t += blockDim.x) {
      if (t < N * N) D[t / N][t % N] = src[t];
      else if (t < N * N + N) lm[t - N * N] = src[t];
      else if (t < N * N + 2 * N) lp[t - N * N - N] = src[t];
      else if (t < N * N + 3 * N) gl[t - N * N - 2 * N] = src[t];
      else if (t < N * N + 4 * N) gr[t - N * N - 3 * N] = src[t];
      else Dv[(t - N * N - 4 * N) / N][(t - N * N - 4 * N) % N] = src[t];
    }
  }
};

// The basis of a WG-thread workgroup in registers: issued with the other prefetches
// (no loop, so the wait before it goes to LDS counts only the loads issued before it)
template <typename T, int N, int WG> struct BasisRegs {
  static constexpr int C = Basis<T, N>::COUNT, R = (C + WG - 1) / WG;
  T v[R];
  __device__ inline void issue(const T *src, int tid) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[min(tid + r * WG, C - 1)];
    // keep these loads ahead of every later one: the scheduler would otherwise sink
    // them to their use, where the in-order wait for them drains all the others
    __builtin_amdgcn_sched_barrier(0);
  }
  __device__ inline void store(Basis<T, N> &B, int tid) const {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (tid + r * WG < C) B.put(tid + r * WG, v[r]);
  }
};

// copy channels [0, NCH) of points [0, NPT) of EW elements starting at slot e0 into LDS
template <typename T, int NPT, int NPTG, int NCH, int EW>
__device__ inline void stage_in(T *dst, const T *src_blk, int e0) {
  for (int t = threadIdx.x; t < NPT * NCH * EW; t += blockDim.x) {
    const int e = e0 + t % EW, pc = t / EW;
    dst[t] = src_blk[(size_t(e / SB) * NPTG * NCH + pc) * SB + e % SB];
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void t_interp(KArgs<T> a, const T *__restrict__ X) {
  using S = Shape<DIM, ORDER>;
  constexpr int EW = TS<T, DIM, ORDER>::EW_INTERP, NS = EB / EW, N = S::N;
  __shared__ T Us[S::NU * S::NV * EW];
  __shared__ Basis<T, N> B;
  const int64_t blk = blockIdx.x / NS;
  const int e0 = int(blockIdx.x % NS) * EW;
  const int nvalid = a.bcount[blk];
  if (e0 >= nvalid) return;
  B.load(a.basis);
  stage_in<T, S::NU, S::NUP, S::NV, EW>(Us, X + size_t(blk) * S::NUP * S::NV * EB, e0);
  __syncthreads();
  for (int t = threadIdx.x; t < S::NF * EW; t += blockDim.x) {
    const int e = t % EW, q = t / EW;
    if (e0 + e >= nvalid) continue;
    const int f = q / S::NFP, m = q % S::NFP, k = f / 2;
    const T *l = (f & 1) ? B.lp : B.lm;
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) s += l[j] * Us[(Ref<DIM, N>::line(k, m, j) * S::NV + v) * EW + e];
      if (a.scatter) {
        // exchange by scatter: into the partner's slot (a boundary point has none)
        const int nb = a.NB[lay(blk, q, 0, e0 + e, S::NFPAD, 1)];
        if (nb >= 0) a.UF[size_t(nb / SB) * S::NV * SB + (nb % SB) + v * SB] = s;
      } else {
        a.UF[at(blk, q, v, e0 + e, S::NFPAD, S::NV)] = s;
      }
    }
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void t_grad(KArgs<T> a, const T *__restrict__ X) {
  using S = Shape<DIM, ORDER>;
  constexpr int EW = TS<T, DIM, ORDER>::EW_GRAD, NS = EB / EW, N = S::N;
  __shared__ T Us[S::NU * S::NV * EW];
  __shared__ T Ds[S::NF * S::NV * EW];
  __shared__ Basis<T, N> B;
  const int64_t blk = blockIdx.x / NS;
  const int e0 = int(blockIdx.x % NS) * EW;
  const int nvalid = a.bcount[blk];
  if (e0 >= nvalid) return;
  B.load(a.basis);
  stage_in<T, S::NU, S::NUP, S::NV, EW>(Us, X + size_t(blk) * S::NUP * S::NV * EB, e0);
  stage_in<T, S::NF, S::NFPAD, S::NV, EW>(Ds, a.DU + size_t(blk) * S::NFPAD * S::NV * EB, e0);
  __syncthreads();
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa, a.igm1};
  for (int t = threadIdx.x; t < S::NU * EW; t += blockDim.x) {
    const int e = t % EW, i = t / EW;
    if (e0 + e >= nvalid) continue;
    T G[DIM][S::NV], u[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) u[v] = Us[(i * S::NV + v) * EW + e];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ik, m;
      Ref<DIM, N>::locate(i, k, ik, m);
      const int qp = (2 * k + 1) * S::NFP + m, qm = 2 * k * S::NFP + m;
#pragma unroll
      for (int v = 0; v < S::NV; ++v) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) s += B.D[ik][j] * Us[(Ref<DIM, N>::line(k, m, j) * S::NV + v) * EW + e];
        s += B.gr[ik] * Ds[(qp * S::NV + v) * EW + e] + B.gl[ik] * Ds[(qm * S::NV + v) * EW + e];
        G[k][v] = s;
      }
    }
    grad_epilogue<T, DIM, ORDER>(a, gas, blk, i, e0 + e, u, G);
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void t_visc(KArgs<T> a, int forces) {
  using S = Shape<DIM, ORDER>;
  constexpr int EW = TS<T, DIM, ORDER>::EW_VISC, NS = EB / EW, N = S::N;
  __shared__ T Gs[S::NU * S::NG * EW];
  __shared__ Basis<T, N> B;
  const int64_t blk = blockIdx.x / NS;
  const int e0 = int(blockIdx.x % NS) * EW;
  const int nvalid = a.bcount[blk];
  if (e0 >= nvalid) return;
  B.load(a.basis);
  stage_in<T, S::NU, S::NUP, S::NG, EW>(Gs, a.GU + size_t(blk) * S::NUP * S::NG * EB, e0);
  __syncthreads();
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa, a.igm1};
  for (int t = threadIdx.x; t < S::NF * EW; t += blockDim.x) {
    const int e = t % EW, q = t / EW;
    if (e0 + e >= nvalid) continue;
    const int f = q / S::NFP, m = q % S::NFP, k = f / 2;
    const T *l = (f & 1) ? B.lp : B.lm;
    T gf[DIM][S::NV];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int v = 0; v < S::NV; ++v) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) s += l[j] * Gs[(Ref<DIM, N>::line(k, m, j) * S::NG + c * S::NV + v) * EW + e];
        gf[c][v] = s;
      }
    visc_epilogue<T, DIM, ORDER>(a, gas, blk, q, e0 + e, gf, forces);
  }
}

template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void t_divrk(KArgs<T> a, int mode) {
  using S = Shape<DIM, ORDER>;
  constexpr int EW = TS<T, DIM, ORDER>::EW_DIV, NS = EB / EW, N = S::N;
  __shared__ T Fs[S::NU * S::NG * EW];
  __shared__ T Cs[S::NF * S::NV * EW];
  __shared__ Basis<T, N> B;
  const int64_t blk = blockIdx.x / NS;
  const int e0 = int(blockIdx.x % NS) * EW;
  const int nvalid = a.bcount[blk];
  if (e0 >= nvalid) return;
  B.load(a.basis);
  stage_in<T, S::NU, S::NUP, S::NG, EW>(Fs, a.FT + size_t(blk) * S::NUP * S::NG * EB, e0);
  for (int t = threadIdx.x; t < S::NF * EW; t += blockDim.x) {
    const int e = t % EW, q = t / EW;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = 0;
    if (e0 + e < nvalid) common_flux<T, DIM, ORDER>(a, blk, q, e0 + e, b);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) Cs[(q * S::NV + v) * EW + e] = b[v];
  }
  __syncthreads();
  int bad = 0;
  for (int t = threadIdx.x; t < S::NU * EW; t += blockDim.x) {
    const int e = t % EW, i = t / EW;
    if (e0 + e >= nvalid) continue;
    T div[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) div[v] = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ik, m;
      Ref<DIM, N>::locate(i, k, ik, m);
      const int qp = (2 * k + 1) * S::NFP + m, qm = 2 * k * S::NFP + m;
#pragma unroll
      for (int v = 0; v < S::NV; ++v) {
        T d = 0, fp = 0, fm = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const T f = Fs[(Ref<DIM, N>::line(k, m, j) * S::NG + k * S::NV + v) * EW + e];
          d += B.D[ik][j] * f;
          fp += B.lp[j] * f;
          fm += B.lm[j] * f;
        }
        // outward discontinuous normal flux: +F~_k at xi_k = +1, -F~_k at xi_k = -1
        div[v] += d + B.gr[ik] * (Cs[(qp * S::NV + v) * EW + e] - fp) -
                  B.gl[ik] * (Cs[(qm * S::NV + v) * EW + e] + fm);
      }
    }
    rk_epilogue<T, DIM, ORDER>(a, blk, i, e0 + e, div, mode, bad);
  }
  if (bad) atomicOr(a.flag, 1);
}

// the other side's face data at mortar point pt: sum over its entries of weight x the
// value of group MG[j] at partner code MC[j] in the face layout, in FP64, entry order
template <typename T, int NV>
__device__ inline void mortar_sum(const KArgs<T> &a, const T *const *grp, int64_t pt, T out[NV]) {
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int j = a.MO[pt]; j < a.MO[pt + 1]; ++j) {
    const T *src = grp[a.MG[j]];
    const int c = a.MC[j];
    const double wj = a.MW[j];
    const size_t base = size_t(c / SB) * NV * SB + (c % SB);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += wj * double(src[base + v * SB]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = T(acc[v]);
}

// ---------------------------------------------------------------------------
// fused stage: two launches per RK stage, sum-factorised, LDS-staged
//
//   k_stage_a: trace and common solution, Rusanov flux, corrected gradient,
//              transformed flux, gradient trace and viscous half-flux, volume
//              divergence (interpolated normal-flux correction included);
//              writes Q = F_I* - P (or the whole boundary common flux), P, RV
//   k_stage_b: transformed common flux A (Q + P_partner), flux correction,
//              R = -(RV + corr)/|J|, RK4 stage, trace of the next stage state
//
// Workgroups are mapped so that the EB/EW sub-blocks of one element block,
// and neighbouring blocks, run on the same XCD (dispatch is round-robin over
// the 8 XCDs), keeping partner traces and shared segments in one L2.
// ---------------------------------------------------------------------------
// Face of flux point q in a fused-stage flux-point pass (slot t = tid + it * WG, q = t / EW,
// WG a multiple of 64). When a wavefront's 64 slots are exactly the NFP points of one face
// for EW elements (NFP * EW = 64: FP32 at p = 3 with 4 elements per workgroup), the face is
// the same in every lane and is read as a scalar, so the face-axis selects that follow run
// on the scalar unit instead of the vector ALUs.
template <int NFP, int EW> __device__ inline int face_of(int q) {
  if constexpr (NFP * EW == 64) return __builtin_amdgcn_readfirstlane(q / NFP);
  return q / NFP;
}

__device__ inline int64_t xcd_remap(int64_t wg, int64_t nwg) {
  const int64_t full = nwg / 8 * 8;
  return wg < full ? (wg % 8) * (nwg / 8) + wg / 8 : wg;
}

enum { FV_NODE = 0, FV_STORED = 1, FV_MORTAR = 2, FV_EXTR = 3, FV_MORTAR_EXTR = 4 };
// an order group of a variable-order mesh (mortar points), with stored or column metrics
template <int FV> constexpr bool mortar_fv() { return FV == FV_MORTAR || FV == FV_MORTAR_EXTR; }

// Tile shapes of the fused stage, one per launch (picked by the autotuner): TILE_DEFAULT
// sizes the workgroup from the LDS budgets below; TILE_HALF and TILE_QUARTER give it a
// half or a quarter of those elements (at least one): smaller workgroups, more of them
// per compute unit, each waiting at its barriers for fewer waves. TILE_MFMA (first launch
// only) is the default workgroup with the reference gradient and the volume divergence
// on the matrix cores (FP32 at order 3) instead of the vector ALUs; the same fused
// multiply-adds in the same order, so the same results bit for bit.
enum { TILE_DEFAULT = 0, TILE_HALF = 1, TILE_QUARTER = 2, TILE_MFMA = 3 };

template <typename T, int DIM, int ORDER, int TILE = TILE_DEFAULT> struct FS {
  using S = Shape<DIM, ORDER>;
  static constexpr int ew0(int bytes, int budget) {
    return bytes * 16 <= budget ? 16 : bytes * 8 <= budget ? 8 : bytes * 4 <= budget ? 4 : bytes * 2 <= budget ? 2 : 1;
  }
  static constexpr int ew(int bytes, int budget) {
    return TILE == TILE_DEFAULT || TILE == TILE_MFMA ? ew0(bytes, budget)
           : (ew0(bytes, budget) >> TILE) > 0        ? ew0(bytes, budget) >> TILE
                                                     : 1;
  }
  // stage a: max(state + jumps, gradient + transformed flux) per element (aliased)
  static constexpr int LDS_A_ELEM = (S::NU * S::NV + S::NF * S::NV) > 2 * S::NU * S::NG
                                        ? (S::NU * S::NV + S::NF * S::NV) : 2 * S::NU * S::NG;
  // threads per element: one per solution point from p = 3 up; below, the flux points
  // outnumber the solution points (P1: 24 against 8) and one thread per flux point
  // gives the low orders' small grids more waves to hide latency with
  static constexpr int TPE = ORDER >= 3 ? S::NU : (S::NF > S::NU ? S::NF : S::NU);
  static constexpr int ewt(int e) { return ORDER >= 3 || TPE * e <= 256 || e == 1 ? e : ewt(e / 2); }
  static constexpr int EW_A = ewt(ew(LDS_A_ELEM * int(sizeof(T)), 40960));
  static constexpr int WG_A = TPE * EW_A >= 256 ? 256 : (TPE * EW_A + 63) / 64 * 64;
  // stage b: common flux at faces and the new state
  static constexpr int EW_B = ewt(ew((S::NF * S::NV + S::NU * S::NV) * int(sizeof(T)), 32768));
  static constexpr int WG_B = TPE * EW_B >= 256 ? 256 : (TPE * EW_B + 63) / 64 * 64;
};

// MORTAR: the mesh is one order group of a variable-order mesh, whose neighbour codes
// may name mortar points (compiled out otherwise)
// Fused-stage variants (FV): FV_NODE, a 3D one-order mesh forms its metrics from the
// geometry nodes (fr_geom.hpp) instead of reading them: S and 1/|J| at the solution
// points, the unit normal and area factor at the flux points.  The area factor is folded
// into the half fluxes the first launch writes (Q and P are stored as A Q and A P), so
// the second launch reads no face metrics.  FV_STORED reads the stored metrics (2D
// meshes, and the 3D alternative the autotuner times); FV_MORTAR is an order group of a
// variable-order mesh with mortar points (stored metrics); FV_EXTR, a mesh of z-extruded
// elements, forms S, 1/|J|, normals and area factors from its column metrics (the 2D
// Jacobian at the n^2 solution-point columns, z_zeta at the n layers, the face columns)
// with a few FP64 products, and scales the half fluxes as FV_NODE does. FV_MORTAR_EXTR is an
// order group on z-extruded elements: the first launch forms its metrics from the column
// data as FV_EXTR does but stores Q and P unscaled, as the mortar interpolation and
// projection take them; the second launch scales them by the stored face areas and takes
// 1/|J| from the column factors.
template <typename T, int DIM, int ORDER, int FV, int TILE = TILE_DEFAULT> struct NodeMetrics {
  using S = Shape<DIM, ORDER>;
  using F = FS<T, DIM, ORDER, TILE>;
  static constexpr bool ON = DIM == 3 && FV == FV_NODE;
  static constexpr int EW = F::EW_A;
  using G = geom::Lay<S::N, EW>;
  static constexpr int cmax(int x, int y) { return x > y ? x : y; }
  // bytes: the stage's own LDS; with node metrics, pass A outputs from 0 (the state and
  // jumps later reuse them) and the nodes, then pass B outputs, past both
  static constexpr int STATE_B = (S::NU + S::NF) * S::NV * int(sizeof(T)) * EW;
  static constexpr int OWN_B = F::LDS_A_ELEM * int(sizeof(T)) * EW;
  static constexpr int VB_OFF = ON ? (cmax(G::NA * 8 * EW, STATE_B) + 15) / 16 * 16 : 0;
  static constexpr int BYTES = ON ? cmax(OWN_B, VB_OFF + cmax(G::NB, G::NX) * 8 * EW) : OWN_B;
};

// register budget: 4 waves per SIMD in FP32 (3 with node metrics, whose FP64 metric
// products need more registers), 2 in FP64
// SCAT: the neighbour exchange by scatter. The previous launch (or the trace
// interpolation) wrote each partner's trace into this element's slot of UF, so the
// partner traces load from the own slots; the viscous half flux P goes to the partner's
// slot of PV, where the second launch reads it from its own. Without SCAT both are
// gathered through the neighbour codes. Not with mortar faces.
template <typename T, int DIM, int ORDER, int FV, int TILE, bool SCAT>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (NodeMetrics<T, DIM, ORDER, FV>::ON ? 3 : 4) : 2, 8)))
void k_stage_a(KArgs<T> a, const T *__restrict__ X, int forces) {
  constexpr bool MORTAR = mortar_fv<FV>();
  static_assert(!(SCAT && MORTAR), "mortar faces exchange by gather");
  using S = Shape<DIM, ORDER>;
  using F = FS<T, DIM, ORDER, TILE>;
  using NM = NodeMetrics<T, DIM, ORDER, FV, TILE>;
  constexpr bool NODEM = NM::ON;
  constexpr bool EXTR = DIM == 3 && (FV == FV_EXTR || FV == FV_MORTAR_EXTR);
  constexpr bool SCALED = NODEM || (EXTR && !MORTAR);  // Q and P stored times the area factor
  // FP32 form: metric factors (formed in FP64) rounded to FP32 once per point or flux
  // point, products in FP32
  constexpr bool MP32 = sizeof(T) == 4;
  // the matrix-core tile: FP32 at p = 3 with 4 elements per workgroup of 4 waves (node
  // metrics keep their geometry passes in the LDS the gradient pass reuses)
  constexpr bool MFG =
      sizeof(T) == 4 && DIM == 3 && ORDER == 3 && !NODEM && TILE == TILE_MFMA && F::EW_A == 4 && F::WG_A == 256;
  constexpr int NCOL = S::N * S::N, NFC = 4 * S::N + S::N * S::N;
  constexpr int EW = F::EW_A, WG = F::WG_A, NS = EB / EW, N = S::N, NV = S::NV, NG = S::NG;
  constexpr int FI = (S::NF * EW + WG - 1) / WG, PI = (S::NU * EW + WG - 1) / WG;
  // LDS: [state | jumps] while the gradient is formed, then [gradient | flux]; before
  // both, with node metrics, the geometry passes
  __shared__ __align__(16) unsigned char Lraw[NM::BYTES];
  T *L = reinterpret_cast<T *>(Lraw);
  T *Us = L, *Ds = L + S::NU * NV * EW;
  T *Gs = L, *Fs = L + S::NU * NG * EW;
  __shared__ Basis<T, N> B;
  // FP32: the Rusanov fluxes of the face pass wait in LDS through the gradient and flux
  // passes (each lane reads back only what it wrote); held in registers they spill
  constexpr bool FQL = sizeof(T) == 4;
  __shared__ T Lq[FQL ? S::NF * NV * EW : 1];
  // node metrics: the quadratic basis table
  __shared__ double GQs[NODEM ? 6 * N : 1];
  const int64_t wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);
  const int64_t blk = wg / NS;
  const int e0 = int(wg % NS) * EW;
  const int nvalid = a.bcount[blk];
  if (e0 >= nvalid) return;
  const int tid = threadIdx.x;
  // this block's part of the per-element arrays (uniform); lanes add 32-bit offsets
  const int *NBb = blk_base(a.NB, blk, S::NFPAD, 1);
  const T *UFb = blk_base<const T>(a.UF, blk, S::NFPAD, NV);
  const double *FCXb = blk_base(a.FCX, blk, NFC, 2), *XCb = blk_base(a.XC, blk, NCOL, 4);
  const double *ZZb = blk_base(a.ZZ, blk, N, 1);
  T *PVb = blk_base(a.PV, blk, S::NFPAD, NV), *FIb = blk_base(a.FI, blk, S::NFPAD, NV);
  T *FTb = blk_base(a.FT, blk, S::NUP, NV);

  // ---- prefetch in the order of first use: basis, neighbour codes, stage state,
  // normals, partner traces (once the codes are back); the metrics of the solution
  // points go last, so that they stay in flight through the flux-point pass and the
  // gradient. Every load is unconditional, with indices clamped into the block (idle
  // lanes and empty slots load values that are never used): the wait before a use
  // then counts exactly the loads issued before it, instead of draining them all.
  constexpr int SI = (S::NU * NV * EW + WG - 1) / WG;
  BasisRegs<T, N, WG> bas;
  bas.issue(a.basis, tid);
  // geometry nodes and the quadratic basis table first: the geometry passes run while the
  // other prefetches are in flight
  constexpr int XI = NODEM ? (geom::NODES * 3 * EW + WG - 1) / WG : 1;
  double xr[XI], gqv = 0.0;
  if constexpr (NODEM) {
#pragma unroll
    for (int r = 0; r < XI; ++r) {
      const int t = min(tid + r * WG, geom::NODES * 3 * EW - 1);
      const int eg = e0 + t % EW;
      xr[r] = a.XN[(size_t(blk * NSB + eg / SB) * (geom::NODES * 3) + t / EW) * SB + eg % SB];
    }
    gqv = a.GQ[min(tid, 6 * N - 1)];
  }
  int nbv[FI];
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
    nbv[it] = in_blk(NBb, lay_in(q, 0, eg, S::NFPAD, 1));
  }
  T ust[SI];
  const T *Xb = X + size_t(blk) * S::NUP * NV * EB;
#pragma unroll
  for (int r = 0; r < SI; ++r) {
    const int t = min(tid + r * WG, S::NU * NV * EW - 1);
    const int e = e0 + t % EW;
    ust[r] = in_blk(Xb, (unsigned(e) / SB * (S::NUP * NV) + unsigned(t) / EW) * SB + unsigned(e) % SB);
  }
  double nrd[FI][DIM], Av[FI];
  double fcv[EXTR ? FI : 1][2], fzv[EXTR ? FI : 1];  // column metrics of the flux point's face
  if constexpr (EXTR) {
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
      const int f = face_of<S::NFP, EW>(q), m = q % S::NFP, k = f / 2, sd = f & 1;
      const int col = k == 0 ? sd * N + m % N : (k == 1 ? 2 * N + sd * N + m % N : 4 * N + m);
      fcv[it][0] = in_blk(FCXb, lay_in(col, 0, eg, NFC, 2));
      fcv[it][1] = in_blk(FCXb, lay_in(col, 1, eg, NFC, 2));
      fzv[it] = in_blk(ZZb, lay_in(m / N, 0, eg, N, 1));
    }
  } else if constexpr (!NODEM) {
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
#pragma unroll
      for (int c = 0; c < DIM; ++c) nrd[it][c] = a.FN[at(blk, q, c, eg, S::NFPAD, DIM)];
      Av[it] = 1.0;
    }
  }
  T ur[FI][NV];
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int nb = nbv[it];
    if constexpr (SCAT) {
      // the partner's trace, written into this slot (never used at a boundary point)
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
#pragma unroll
      for (int v = 0; v < NV; ++v) ur[it][v] = in_blk(UFb, lay_in(q, v, eg, S::NFPAD, NV));
    } else if (MORTAR && nb < 0 && ((-nb) & 3) == BC_MORTAR) {
      // the other side's trace at this point: its face points' traces interpolated
      // (higher-order side) or projected (lower-order side)
      mortar_sum<T, NV>(a, a.GUF, (-nb) >> 3, ur[it]);
    } else {
      // a boundary code loads slot 0 and never uses it
      const int p = nb > 0 ? nb : 0;
      const size_t base = size_t(p / SB) * NV * SB + (p % SB);
#pragma unroll
      for (int v = 0; v < NV; ++v) ur[it][v] = a.UF[base + v * SB];
    }
  }
  double Sm[PI][DIM][DIM], ijv[PI];
  double xcv[EXTR ? PI : 1][4], zzv[EXTR ? PI : 1];  // column metrics of the solution point
  if constexpr (EXTR) {
#pragma unroll
    for (int it = 0; it < PI; ++it) {
      const int t = tid + it * WG, i = min(t / EW, S::NU - 1), eg = e0 + t % EW;
#pragma unroll
      for (int c = 0; c < 4; ++c) xcv[it][c] = in_blk(XCb, lay_in(i % NCOL, c, eg, NCOL, 4));
      zzv[it] = in_blk(ZZb, lay_in(i / NCOL, 0, eg, N, 1));
    }
  } else if constexpr (!NODEM) {
#pragma unroll
    for (int it = 0; it < PI; ++it) {
      const int t = tid + it * WG, i = min(t / EW, S::NU - 1), eg = e0 + t % EW;
#pragma unroll
      for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int c = 0; c < DIM; ++c) Sm[it][k][c] = a.SM[at(blk, i, k * DIM + c, eg, S::NUP, DIM * DIM)];
      ijv[it] = a.IJ[lay(blk, i, 0, eg, S::NUP, 1)];
    }
  } else {
    // ---- metrics from the nodes, in FP64: pass A (VA, FA0, FA1 from offset 0), pass B
    // (VB over the nodes, past the state and jumps, so that it lasts until the gradient
    // pass), then per thread its flux points' normals and area factors (the xi and eta
    // faces before the barrier that frees pass A's outputs for the state, the zeta faces
    // after it); S and 1/|J| of the solution points follow in the gradient pass
    double *GA = reinterpret_cast<double *>(Lraw);
    double *GB = reinterpret_cast<double *>(Lraw + NM::VB_OFF);
#pragma unroll
    for (int r = 0; r < XI; ++r) {
      const int t = tid + r * WG;
      if (t < geom::NODES * 3 * EW) GB[t] = xr[r];
    }
    if (tid < 6 * N) GQs[tid] = gqv;
    __syncthreads();
#pragma unroll 2
    for (int t = tid; t < NM::G::NA * EW; t += WG) GA[t] = geom::pass_a<N, EW>(GB, GQs, t);
    __syncthreads();
#pragma unroll 2
    for (int t = tid; t < NM::G::NB * EW; t += WG) GB[t] = geom::pass_b<N, EW>(GA, GQs, t);
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1);
      if (q / S::NFP < 4) Av[it] = geom::face_metrics<N, EW>(GA, GB, GQs, t % EW, q, nrd[it]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1);
      if (q / S::NFP >= 4) Av[it] = geom::face_metrics<N, EW>(GA, GB, GQs, t % EW, q, nrd[it]);
    }
  }
  bas.store(B, tid);
#pragma unroll
  for (int r = 0; r < SI; ++r) {
    const int t = tid + r * WG;
    if (t < S::NU * NV * EW) Us[t] = ust[r];
  }
  __syncthreads();
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa, a.igm1};

  // ---- faces: own trace, common solution jump (LDS), Rusanov flux (registers)
  T ufv[FI][NV], fiv[FI][NV], nrm[FI][DIM];
  if constexpr (EXTR) {
    // face row S_k of J = [[x_xi, x_eta, 0], [y_xi, y_eta, 0], [0, 0, z_zeta]]: on a xi face
    // (y_eta z, -x_eta z, 0), on an eta face (-z y_xi, z x_xi, 0), on a zeta face
    // (0, 0, x_xi y_eta - y_xi x_eta); area factor |S_k|, outward normal (2s - 1) S_k / |S_k|
#pragma unroll
    for (int it = 0; it < FI; ++it) {
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1);
      const int f = face_of<S::NFP, EW>(q), k = f / 2;
      const double z = fzv[it], u = fcv[it][0], w = fcv[it][1];
      double sk[3];
      sk[0] = k == 0 ? w * z : (k == 1 ? -(z * w) : 0.0);
      sk[1] = k == 0 ? -(u * z) : (k == 1 ? z * u : 0.0);
      sk[2] = k == 2 ? u : 0.0;
      const double a2 = sk[0] * sk[0] + sk[1] * sk[1] + sk[2] * sk[2];
      if constexpr (MP32) {
        // FP32 form: |S_k|^2 in FP64, rounded once; the area and the unit normal in FP32
        const float area = sqrtv(float(a2)), ia = (f & 1) ? recip(area) : -recip(area);
        Av[it] = area;
#pragma unroll
        for (int c = 0; c < DIM; ++c) nrd[it][c] = float(sk[c]) * ia;
      } else {
        const double area = sqrt(a2);
        const double ia = ((f & 1) ? 1.0 : -1.0) / area;
        Av[it] = area;
#pragma unroll
        for (int c = 0; c < DIM; ++c) nrd[it][c] = sk[c] * ia;
      }
    }
  }
#pragma unroll
  for (int it = 0; it < FI; ++it)
#pragma unroll
    for (int c = 0; c < DIM; ++c) nrm[it][c] = T(nrd[it][c]);
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, e = t % EW, q = t / EW, eg = e0 + e;
    if (t >= S::NF * EW) break;
    T du[NV];
    if (eg < nvalid) {
      const int f = face_of<S::NFP, EW>(q), m = q % S::NFP, k = f / 2;
      const T *l = (f & 1) ? B.lp : B.lm;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T sv = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) sv += l[j] * Us[(Ref<DIM, N>::line(k, m, j) * NV + v) * EW + e];
        ufv[it][v] = sv;
      }
      const int nb = nbv[it];
      T ub[NV];
      if (nb >= 0 || (MORTAR && ((-nb) & 3) == BC_MORTAR)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          ub[v] = ur[it][v];
          du[v] = T(0.5) * (ub[v] - ufv[it][v]);
        }
      } else if (((-nb) & 3) == BC_FARFIELD) {
        gas.farfield(ufv[it], nrm[it], a.fsd + 5 * a.bdesign[blk], ub);
#pragma unroll
        for (int v = 0; v < NV; ++v) du[v] = ub[v] - ufv[it][v];
      } else {
        T uc[NV];
        gas.wall_common(ufv[it], uc);
#pragma unroll
        for (int v = 0; v < NV; ++v) du[v] = uc[v] - ufv[it][v];
        ub[0] = ufv[it][0];
#pragma unroll
        for (int c = 0; c < DIM; ++c) ub[1 + c] = -ufv[it][1 + c];
        ub[DIM + 1] = ufv[it][DIM + 1];
      }
      gas.rusanov(ufv[it], ub, nrm[it], fiv[it]);
      if constexpr (FQL) {
#pragma unroll
        for (int v = 0; v < NV; ++v) Lq[(q * NV + v) * EW + e] = fiv[it][v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) du[v] = 0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Ds[(q * NV + v) * EW + e] = du[v];
  }
  __syncthreads();

  // ---- solution points: corrected reference gradient (registers), then LDS is reused;
  // with node metrics also S and 1/|J| from pass B's outputs, still intact above the
  // state and jumps
  T Gr[PI][DIM][NV], ui[PI][NV];
  if constexpr (MFG) {
    // On the matrix cores: for axis k and variable v, the 16 solution-point lines along k
    // of the 4 elements are the 16 blocks of one v_mfma_f32_4x4x1 chain (block = line,
    // its 4 columns = the elements, its 4 rows = the points of the line). Six rank-1 steps
    // accumulate G = D u + g_R' (u_c - u_f)_+ + g_L' (u_c - u_f)_-; the A operand is the
    // basis column (lane = 4 line + row), the B operand the line's value of each element
    // (lane = 4 line + element). Lane 4 m + e then holds G_k at the 4 points of line m of
    // element e, which it writes to the flux region of LDS (free until the transformed
    // flux overwrites it point by point); each thread reads back its own point's 15
    // channels after the barrier. Waves take the 15 (k, v) pairs in turn.
    const int lane = tid & 63, wave = tid >> 6, ml = lane >> 2, el = lane & 3;
    T ad[N], agr = B.gr[el], agl = B.gl[el];
#pragma unroll
    for (int j = 0; j < N; ++j) ad[j] = B.D[el][j];
    T *Gref = L + S::NU * NG * EW;
#pragma unroll
    for (int sk = 0; sk < (NG + 3) / 4; ++sk) {
      const int tk = wave + 4 * sk;
      if (tk >= NG) break;  // wave-uniform: every lane of the wave runs the chain
      const int k = tk / NV, v = tk % NV;
      int base, stride;
      Ref<DIM, N>::line_of(k, ml, base, stride);
      const T *ul = Us + (base * NV + v) * EW + el;
      floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < N; ++j) c = __builtin_amdgcn_mfma_f32_4x4x1f32(ad[j], ul[j * stride * NV * EW], c, 0, 0, 0);
      const int qp = (2 * k + 1) * S::NFP + ml, qm = 2 * k * S::NFP + ml;
      c = __builtin_amdgcn_mfma_f32_4x4x1f32(agr, Ds[(qp * NV + v) * EW + el], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_4x4x1f32(agl, Ds[(qm * NV + v) * EW + el], c, 0, 0, 0);
      T *gl = Gref + (base * NG + tk) * EW + el;
#pragma unroll
      for (int r = 0; r < N; ++r) gl[r * stride * NG * EW] = c[r];
    }
#pragma unroll
    for (int it = 0; it < PI; ++it) {
      const int t = tid + it * WG, e = t % EW, i = t / EW;
      if (t >= S::NU * EW) break;
#pragma unroll
      for (int v = 0; v < NV; ++v) ui[it][v] = Us[(i * NV + v) * EW + e];
    }
  } else {
#pragma unroll
  for (int it = 0; it < PI; ++it) {
    const int t = tid + it * WG, e = t % EW, i = t / EW;
    if constexpr (NODEM) {
      double Sg[3][3];
      ijv[it] = 1.0 / geom::point_metrics<N, EW>(reinterpret_cast<const double *>(Lraw + NM::VB_OFF), GQs, e,
                                                  min(i, S::NU - 1), Sg);
#pragma unroll
      for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int c = 0; c < DIM; ++c) Sm[it][k][c] = Sg[k][c];
    }
    if (t >= S::NU * EW) break;
#pragma unroll
    for (int v = 0; v < NV; ++v) ui[it][v] = Us[(i * NV + v) * EW + e];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ik, m;
      Ref<DIM, N>::locate(i, k, ik, m);
      const int qp = (2 * k + 1) * S::NFP + m, qm = 2 * k * S::NFP + m;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // one fused multiply-add per term, in the order of the matrix-core chain
        T sv = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) sv = fma(B.D[ik][j], Us[(Ref<DIM, N>::line(k, m, j) * NV + v) * EW + e], sv);
        sv = fma(B.gr[ik], Ds[(qp * NV + v) * EW + e], sv);
        sv = fma(B.gl[ik], Ds[(qm * NV + v) * EW + e], sv);
        Gr[it][k][v] = sv;
      }
    }
  }
  }
  __syncthreads();
  // physical gradient and transformed flux into the aliased LDS
#pragma unroll
  for (int it = 0; it < PI; ++it) {
    const int t = tid + it * WG, e = t % EW, i = t / EW, eg = e0 + e;
    if (t >= S::NU * EW) break;
    if constexpr (MFG) {
      // this point's reference gradient from the matrix-core pass (before this thread's
      // transformed flux overwrites the same words)
#pragma unroll
      for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) Gr[it][k][v] = L[S::NU * NG * EW + (i * NG + k * NV + v) * EW + e];
    }
    if constexpr (EXTR) {
      // S = |J| J^-1 by rows (a_{k+1} x a_{k+2}) and |J| = a_0 . S_0 for
      // a_0 = (x_xi, y_xi, 0), a_1 = (x_eta, y_eta, 0), a_2 = (0, 0, z_zeta)
      const double xx = xcv[it][0], xe = xcv[it][1], yx = xcv[it][2], ye = xcv[it][3], z = zzv[it];
      Sm[it][0][0] = ye * z;
      Sm[it][0][1] = -(xe * z);
      Sm[it][0][2] = 0.0;
      Sm[it][1][0] = -(z * yx);
      Sm[it][1][1] = z * xx;
      Sm[it][1][2] = 0.0;
      Sm[it][2][0] = 0.0;
      Sm[it][2][1] = 0.0;
      Sm[it][2][2] = xx * ye - yx * xe;
      // FP32 form: |J| rounded once, its reciprocal in FP32
      const double jac = xx * Sm[it][0][0] + yx * Sm[it][0][1];
      ijv[it] = MP32 ? double(recip(float(jac))) : 1.0 / jac;
    }
    if (eg >= nvalid) {
#pragma unroll
      for (int c = 0; c < NG; ++c) Gs[(i * NG + c) * EW + e] = Fs[(i * NG + c) * EW + e] = 0;
      continue;
    }
    // physical gradient S^T G / |J| and transformed flux S (F_inv - F_vis). The metric
    // factors of the point are formed in FP64. The FP64 form multiplies in FP64; the FP32
    // form rounds the point's factors S/|J| and S to FP32 once and multiplies in FP32, as
    // its operators and fluxes. Zeros of the block form of S are skipped on column metrics.
    T gu[DIM][NV];
    double Mj[DIM][DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int c = 0; c < DIM; ++c) Mj[k][c] = (EXTR || MP32) ? Sm[it][k][c] * ijv[it] : Sm[it][k][c];
    T Mt[DIM][DIM], St[DIM][DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        St[k][c] = T(Sm[it][k][c]);
        // column metrics in the FP32 form: S/|J| from the rounded S and 1/|J|
        Mt[k][c] = (MP32 && EXTR) ? St[k][c] * T(ijv[it]) : T(Mj[k][c]);
      }
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (MP32) {
          T sg = 0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            if (EXTR && (k == 2) != (c == 2)) continue;
            sg = fma(Mt[k][c], Gr[it][k][v], sg);
          }
          gu[c][v] = sg;
        } else {
          double sg = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            if (EXTR && (k == 2) != (c == 2)) continue;  // zero in the block form of S
            sg += Mj[k][c] * double(Gr[it][k][v]);
          }
          gu[c][v] = T(EXTR ? sg : sg * ijv[it]);
        }
        Gs[(i * NG + c * NV + v) * EW + e] = gu[c][v];
      }
    T Fi[DIM][NV], Fv[DIM][NV];
    gas.flux_inv(ui[it], Fi);
    gas.flux_vis(ui[it], gu, Fv, false);
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (MP32) {
          T sf = 0;
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            if (EXTR && (k == 2) != (c == 2)) continue;
            sf = fma(St[k][c], Fi[c][v] - Fv[c][v], sf);
          }
          Fs[(i * NG + k * NV + v) * EW + e] = sf;
        } else {
          double sf = 0.0;
#pragma unroll
          for (int c = 0; c < DIM; ++c) {
            if (EXTR && (k == 2) != (c == 2)) continue;
            sf += Sm[it][k][c] * double(Fi[c][v] - Fv[c][v]);
          }
          Fs[(i * NG + k * NV + v) * EW + e] = T(sf);
        }
      }
  }
  __syncthreads();

  // ---- flux points: gradient trace, viscous half-flux P, Q = F_I* - P (boundary: full flux)
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, e = t % EW, q = t / EW, eg = e0 + e;
    if (t >= S::NF * EW) break;
    if (eg >= nvalid) continue;
    const int f = face_of<S::NFP, EW>(q), m = q % S::NFP, k = f / 2;
    const T *l = (f & 1) ? B.lp : B.lm;
    T gf[DIM][NV];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T sv = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) sv += l[j] * Gs[(Ref<DIM, N>::line(k, m, j) * NG + c * NV + v) * EW + e];
        gf[c][v] = sv;
      }
    const int nb = nbv[it];
    T fn[NV];
    if (nb >= 0 || (MORTAR && ((-nb) & 3) == BC_MORTAR)) {
      gas.flux_vis_n(ufv[it], gf, nrm[it], fn, false);
      // P to the partner's slot (exchange by scatter) or to this one
      T *pdst = SCAT ? a.PV + (size_t(nb / SB) * NV * SB + (nb % SB)) : nullptr;
      const unsigned own = lay_in(q, 0, eg, S::NFPAD, NV);
      const T Af = T(Av[it]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T pv = T(0.5) * fn[v];
        const T qv = (FQL ? Lq[(q * NV + v) * EW + e] : fiv[it][v]) - pv;
        const T ps = SCALED ? (MP32 ? Af * pv : T(Av[it] * double(pv))) : pv;
        if constexpr (SCAT)
          pdst[v * SB] = ps;
        else
          in_blk(PVb, own + v * SB) = ps;
        in_blk(FIb, own + v * SB) = SCALED ? (MP32 ? Af * qv : T(Av[it] * double(qv))) : qv;
      }
    } else {
      const int code = -nb;
      T ub[NV];
      if ((code & 3) == BC_FARFIELD) {
        gas.farfield(ufv[it], nrm[it], a.fsd + 5 * a.bdesign[blk], ub);
        gas.flux_vis_n(ub, gf, nrm[it], fn, false);
      } else {
        gas.wall_common(ufv[it], ub);
        gas.flux_vis_n(ub, gf, nrm[it], fn, true);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T qv = (FQL ? Lq[(q * NV + v) * EW + e] : fiv[it][v]) - fn[v];
        in_blk(FIb, lay_in(q, v, eg, S::NFPAD, NV)) = SCALED ? (MP32 ? T(Av[it]) * qv : T(Av[it] * double(qv))) : qv;
      }
      if (forces && (code & 3) == BC_WALL) {
        // traction of the fluid on the body: W A (p n - tau . n), interior trace
        T Fw[DIM][NV];
        gas.flux_vis(ufv[it], gf, Fw, false);
        double nd[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) nd[c] = a.FN[at(blk, q, c, eg, S::NFPAD, DIM)];
        const double p = double(gas.pressure(ufv[it]));
        const double wA = a.wface[q] * a.FA[lay(blk, q, 0, eg, S::NFPAD, 1)];
        const int64_t w = code >> 2;
#pragma unroll
        for (int ii = 0; ii < DIM; ++ii) {
          double tn = 0.0;
#pragma unroll
          for (int c = 0; c < DIM; ++c) tn += double(Fw[c][1 + ii]) * nd[c];
          a.FC[w * 3 + ii] = wA * (p * nd[ii] - tn);
        }
        if (DIM == 2) a.FC[w * 3 + 2] = 0.0;
      }
    }
  }

  // ---- solution points: volume divergence with the interpolated normal-flux correction
  if constexpr (MFG) {
    // On the matrix cores, as the gradient: for axis k and variable v, the lines along k
    // of the 4 elements are the 16 blocks of a v_mfma_f32_4x4x1 chain over the 4 points
    // of each line, A = the rows of Dv. The per-axis parts wait in registers until every
    // wave has read its last gradient trace, then go to the gradient's LDS; each thread
    // sums its own point's three in axis order after the second barrier.
    const int lane = tid & 63, wave = tid >> 6, ml = lane >> 2, el = lane & 3;
    T av[N];
#pragma unroll
    for (int j = 0; j < N; ++j) av[j] = B.Dv[el][j];
    constexpr int NT = (NG + 3) / 4;
    floatx4 cd[NT];
#pragma unroll
    for (int sk = 0; sk < NT; ++sk) {
      const int tk = wave + 4 * sk;
      cd[sk] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (tk >= NG) break;  // wave-uniform
      int base, stride;
      Ref<DIM, N>::line_of(tk / NV, ml, base, stride);
      const T *fl = Fs + (base * NG + tk) * EW + el;
#pragma unroll
      for (int j = 0; j < N; ++j) cd[sk] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[j], fl[j * stride * NG * EW], cd[sk], 0, 0, 0);
    }
    __syncthreads();
    // per-axis parts [axis][point][variable][element] over the gradient's LDS
    T *Pk = Gs;
#pragma unroll
    for (int sk = 0; sk < NT; ++sk) {
      const int tk = wave + 4 * sk;
      if (tk >= NG) break;
      const int k = tk / NV, v = tk % NV;
      int base, stride;
      Ref<DIM, N>::line_of(k, ml, base, stride);
      T *pl = Pk + ((k * S::NU + base) * NV + v) * EW + el;
#pragma unroll
      for (int r = 0; r < N; ++r) pl[r * stride * NV * EW] = cd[sk][r];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PI; ++it) {
      const int t = tid + it * WG, e = t % EW, i = t / EW, eg = e0 + e;
      if (t >= S::NU * EW) break;
      if (eg >= nvalid) continue;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T div = 0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) div += Pk[((k * S::NU + i) * NV + v) * EW + e];
        in_blk(FTb, lay_in(i, v, eg, S::NUP, NV)) = div;
      }
    }
    return;
  }
#pragma unroll
  for (int it = 0; it < PI; ++it) {
    const int t = tid + it * WG, e = t % EW, i = t / EW, eg = e0 + e;
    if (t >= S::NU * EW) break;
    if (eg >= nvalid) continue;
    T div[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) div[v] = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ik, m;
      Ref<DIM, N>::locate(i, k, ik, m);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // one fused multiply-add per term, in the order of the matrix-core chain
        T d = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) d = fma(B.Dv[ik][j], Fs[(Ref<DIM, N>::line(k, m, j) * NG + k * NV + v) * EW + e], d);
        div[v] += d;
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) in_blk(FTb, lay_in(i, v, eg, S::NUP, NV)) = div[v];
  }
}

// register budget: 5 waves per SIMD in FP32 (the occupancy its default LDS sizing is made
// for), 2 in FP64
// SCAT: the partner's half flux P loads from the own slot of PV (the first launch put it
// there), and the next stage's trace goes to the partner's slot of UF
template <typename T, int DIM, int ORDER, int MODE, int FV, int TILE, bool SCAT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 2, 8)))
void k_stage_b(KArgs<T> a) {
  constexpr int mode = MODE;  // RK stage or residual: fixes what is read and written
  constexpr bool MORTAR = mortar_fv<FV>();
  static_assert(!(SCAT && MORTAR), "mortar faces exchange by gather");
  using S = Shape<DIM, ORDER>;
  using F = FS<T, DIM, ORDER, TILE>;
  // the first launch stored the half fluxes times the area factor (metrics from the
  // geometry nodes or the extruded columns); with the columns, 1/|J| is the product of
  // the column's and the layer's reciprocal factors (FP64)
  constexpr bool COLJ = DIM == 3 && (FV == FV_EXTR || FV == FV_MORTAR_EXTR);
  // NODEM: the first launch stored Q and P times the area factor
  constexpr bool NODEM = NodeMetrics<T, DIM, ORDER, FV>::ON || (COLJ && !MORTAR);
  constexpr int EW = F::EW_B, WG = F::WG_B, NS = EB / EW, N = S::N, NV = S::NV;
  constexpr int FI = (S::NF * EW + WG - 1) / WG, PI = (S::NU * EW + WG - 1) / WG;
  __shared__ T Cs[S::NF * NV * EW];
  __shared__ T Un[S::NU * NV * EW];
  __shared__ Basis<T, N> B;
  const int64_t wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);
  const int64_t blk = wg / NS;
  const int e0 = int(wg % NS) * EW;
  const int nvalid = a.bcount[blk];
  if (e0 >= nvalid) return;
  const int tid = threadIdx.x;
  // this block's part of the per-element arrays (uniform); lanes add 32-bit offsets
  const int *NBb = blk_base(a.NB, blk, S::NFPAD, 1), *NBFb = blk_base(a.NBF, blk, 2 * DIM, 1);
  const double *FAb = blk_base(a.FA, blk, S::NFPAD, 1);
  const T *FIb = blk_base<const T>(a.FI, blk, S::NFPAD, NV), *PVb = blk_base<const T>(a.PV, blk, S::NFPAD, NV);
  const T *FTb = blk_base<const T>(a.FT, blk, S::NUP, NV);
  T *Ub = blk_base(a.U, blk, S::NUP, NV), *USb = blk_base(a.US, blk, S::NUP, NV);
  T *ACCb = blk_base(a.ACC, blk, S::NUP, NV), *RESb = blk_base(a.RES, blk, S::NUP, NV);
  T *UFb = blk_base(a.UF, blk, S::NFPAD, NV);
  const double *IJCb = blk_base(a.IJC, blk, S::N * S::N, 1), *IZb = blk_base(a.IZ, blk, S::N, 1);
  const double *IJb = blk_base(a.IJ, blk, S::NUP, 1);
  const T dt = T(a.bdt[blk]);

  // ---- prefetch in the order of first use: basis, face inputs (codes first, so that
  // the partner gather issues early), then the point inputs, which stay in flight
  // through the flux pass. In FP32 the face loop has no idle lanes, and loads are
  // unconditional with indices clamped into the block, as in k_stage_a. In FP64 half
  // the waves are idle in the last face iteration; there the lanes that hold no flux
  // point, and the slots past the last element, skip their loads (faster as measured).
  constexpr bool SKIP = sizeof(T) == 8;
  BasisRegs<T, N, WG> bas;
  bas.issue(a.basis, tid);
  int nbv[FI];
  double Av[FI];
  T qv[FI][NV], pn[FI][NV];
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
    nbv[it] = -BC_FARFIELD;
    if (!SKIP || (t < S::NF * EW && eg < nvalid)) {
      // per-face codes where the mesh has them (24 B per element in 3D instead of 384)
      if (!MORTAR && a.NBF)
        nbv[it] = point_code(in_blk(NBFb, lay_in(q / S::NFP, 0, eg, 2 * DIM, 1)), q % S::NFP, N, S::NFP, S::NFPAD, DIM);
      else
        nbv[it] = in_blk(NBb, lay_in(q, 0, eg, S::NFPAD, 1));
    }
  }
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
    if (!SKIP || (t < S::NF * EW && eg < nvalid)) {
      Av[it] = NODEM ? 1.0 : in_blk(FAb, lay_in(q, 0, eg, S::NFPAD, 1));
#pragma unroll
      for (int v = 0; v < NV; ++v) qv[it][v] = in_blk(FIb, lay_in(q, v, eg, S::NFPAD, NV));
    }
  }
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int nb = nbv[it];
    if constexpr (SCAT) {
      const int t = tid + it * WG, q = min(t / EW, S::NF - 1), eg = e0 + t % EW;
      if (!SKIP || (t < S::NF * EW && eg < nvalid)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) pn[it][v] = in_blk(PVb, lay_in(q, v, eg, S::NFPAD, NV));
      }
    } else if (MORTAR && nb < 0 && ((-nb) & 3) == BC_MORTAR) {
      const int64_t pt = (-nb) >> 3;
      if (((-nb) >> 2) & 1) {
        // lower-order side: the complete transformed common flux, the L2 projection of
        // the higher-order side's (MT, written by that group's second launch, which runs
        // before this one), with the outward sign of this side; FP64 sums in entry order
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        for (int j = a.PO[pt]; j < a.PO[pt + 1]; ++j) {
          const double wj = a.PW[j];
          const size_t src = size_t(a.PC[j]) * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] += wj * double(a.MT[src + v]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) pn[it][v] = T(-1.0 * acc[v]);
      } else {
        // higher-order side: the other side's half viscous flux, interpolated to this
        // point (that group's first launch wrote it)
        mortar_sum<T, NV>(a, a.GPV, pt, pn[it]);
      }
    } else if (!SKIP || nb >= 0) {
      // unconditional form: a boundary code loads slot 0 and never uses it
      const int p = nb > 0 ? nb : 0;
      const size_t base = size_t(p / SB) * NV * SB + (p % SB);
#pragma unroll
      for (int v = 0; v < NV; ++v) pn[it][v] = a.PV[base + v * SB];
    }
  }
  T rv[PI][NV], un[PI][NV], ac[PI][NV];
  double ijv[PI];
#pragma unroll
  for (int it = 0; it < PI; ++it) {
    const int t = tid + it * WG, i = min(t / EW, S::NU - 1), eg = e0 + t % EW;
    if (!SKIP || (t < S::NU * EW && eg < nvalid)) {
      ijv[it] = COLJ ? in_blk(IJCb, lay_in(i % (S::N * S::N), 0, eg, S::N * S::N, 1)) *
                           in_blk(IZb, lay_in(i / (S::N * S::N), 0, eg, S::N, 1))
                     : in_blk(IJb, lay_in(i, 0, eg, S::NUP, 1));
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const unsigned x = lay_in(i, v, eg, S::NUP, NV);
        rv[it][v] = in_blk(FTb, x);
        un[it][v] = mode == MODE_RESID ? T(0) : in_blk(Ub, x);
        ac[it][v] = (mode == MODE_RK1 || mode == MODE_RK2 || mode == MODE_RK3) ? in_blk(ACCb, x) : T(0);
      }
    }
  }
  bas.store(B, tid);

  // ---- transformed outward common flux A (Q + P_partner), boundary: A Q
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, e = t % EW, q = t / EW, eg = e0 + e;
    if (t >= S::NF * EW) break;
    T b[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) b[v] = 0;
    if (eg < nvalid) {
      const int code = -nbv[it];
      if (nbv[it] >= 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) b[v] = NODEM ? qv[it][v] + pn[it][v] : T(Av[it] * double(qv[it][v] + pn[it][v]));
      } else if (MORTAR && (code & 3) == BC_MORTAR) {
        const size_t base = size_t(code >> 3) * NV;
        if ((code >> 2) & 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) b[v] = pn[it][v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            b[v] = T(Av[it] * double(qv[it][v] + pn[it][v]));
            a.MT[base + v] = b[v];
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) b[v] = NODEM ? qv[it][v] : T(Av[it] * double(qv[it][v]));
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Cs[(q * NV + v) * EW + e] = b[v];
  }
  __syncthreads();

  // ---- R = -(RV + corrections)/|J| and the RK4 stage
  int bad = 0;
#pragma unroll
  for (int it = 0; it < PI; ++it) {
    const int t = tid + it * WG, e = t % EW, i = t / EW, eg = e0 + e;
    if (t >= S::NU * EW) break;
    if (eg >= nvalid) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Un[(i * NV + v) * EW + e] = 0;
      continue;
    }
    T div[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) div[v] = rv[it][v];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ik, m;
      Ref<DIM, N>::locate(i, k, ik, m);
      const int qp = (2 * k + 1) * S::NFP + m, qm = 2 * k * S::NFP + m;
#pragma unroll
      for (int v = 0; v < NV; ++v) div[v] += B.gr[ik] * Cs[(qp * NV + v) * EW + e] - B.gl[ik] * Cs[(qm * NV + v) * EW + e];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const unsigned x = lay_in(i, v, eg, S::NUP, NV);
      // FP32 form: 1/|J| rounded once, the product in FP32
      const T r = sizeof(T) == 4 ? -div[v] * T(ijv[it]) : T(-double(div[v]) * ijv[it]);
      T next = 0;
      if (mode == MODE_RESID) {
        in_blk(RESb, x) = r;
      } else if (mode == MODE_RK0) {
        in_blk(ACCb, x) = r;
        next = un[it][v] + T(0.5) * dt * r;
        in_blk(USb, x) = next;
      } else if (mode == MODE_RK1) {
        in_blk(ACCb, x) = ac[it][v] + T(2) * r;
        next = un[it][v] + T(0.5) * dt * r;
        in_blk(USb, x) = next;
      } else if (mode == MODE_RK2) {
        in_blk(ACCb, x) = ac[it][v] + T(2) * r;
        next = un[it][v] + dt * r;
        in_blk(USb, x) = next;
      } else {
        next = un[it][v] + dt / T(6) * (ac[it][v] + r);
        in_blk(Ub, x) = next;
        bad |= !isfinite(next);
      }
      Un[(i * NV + v) * EW + e] = next;
    }
  }
  if (bad) atomicOr(a.flag, 1);
  if (mode == MODE_RESID) return;
  __syncthreads();

  // ---- trace of the next stage input at the flux points
#pragma unroll
  for (int it = 0; it < FI; ++it) {
    const int t = tid + it * WG, e = t % EW, q = t / EW, eg = e0 + e;
    if (t >= S::NF * EW) break;
    if (eg >= nvalid) continue;
    if (SCAT && nbv[it] < 0) continue;  // a boundary point has no partner to receive it
    const int f = q / S::NFP, m = q % S::NFP, k = f / 2;
    const T *l = (f & 1) ? B.lp : B.lm;
    T *pdst = SCAT ? a.UF + (size_t(nbv[it] / SB) * NV * SB + (nbv[it] % SB)) : nullptr;
    const unsigned own = lay_in(q, 0, eg, S::NFPAD, NV);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T sv = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) sv += l[j] * Un[(Ref<DIM, N>::line(k, m, j) * NV + v) * EW + e];
      if constexpr (SCAT)
        pdst[v * SB] = sv;
      else
        in_blk(UFb, own + v * SB) = sv;
    }
  }

}

// ---------------------------------------------------------------------------
// pack / unpack between canonical FP64 [E][nu][nv] and the block layout
// ---------------------------------------------------------------------------
template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_pack(KArgs<T> a, T *dst, int to_device) {
  using S = Shape<DIM, ORDER>;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int e = int(t & 15);
  const int64_t r = t >> 4;
  const int v = int(r % S::NV);
  const int i = int((r / S::NV) % S::NUP);
  const int64_t blk = r / (S::NV * S::NUP);
  if (blk >= a.nblk || i >= S::NU || e >= a.bcount[blk]) return;
  const size_t c = (size_t(a.bcanon[blk] + e) * S::NU + i) * S::NV + v;
  const size_t x = at(blk, i, v, e, S::NUP, S::NV);
  if (to_device)
    dst[x] = T(a.stage64[c]);
  else
    a.stage64[c] = double(dst[x]);
}

// ---------------------------------------------------------------------------
// wall force reduction: one workgroup per design, fixed summation order
// ---------------------------------------------------------------------------
#if FR_PART == 4
__global__ __launch_bounds__(256) void k_force_reduce(const double *FC, const int64_t *wall_first,
                                                       double *fsum) {
  const int d = blockIdx.x;
  const int64_t w0 = wall_first[d], w1 = wall_first[d + 1];
  __shared__ double red[3][256];
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t w = w0 + threadIdx.x; w < w1; w += 256)
    for (int c = 0; c < 3; ++c) s[c] += FC[w * 3 + c];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = fsum + 8 * d;
    for (int c = 0; c < 3; ++c) {
      o[c] += red[c][0];
      o[4 + c] = red[c][0];
    }
    o[3] += 1.0;
  }
}

__global__ void k_clear_flag(int *flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}
#endif

// ---------------------------------------------------------------------------
// sampling: the FR interpolant of the stage-0 state at points (one thread each)
// ---------------------------------------------------------------------------
// slot[p] = block * EB + element slot; w[p][DIM][N] are the 1D Lagrange weights of the
// Gauss-Legendre solution points at the point's reference coordinates
template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_probe(KArgs<T> a, int64_t n, const int64_t *__restrict__ slot,
                                               const double *__restrict__ w, const int64_t *__restrict__ dst,
                                               double *__restrict__ out) {
  using S = Shape<DIM, ORDER>;
  constexpr int N = S::N, NV = S::NV;
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t blk = slot[p] / EB;
  const int e = int(slot[p] % EB);
  const double *wp = w + p * DIM * N;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int c2 = 0; c2 < (DIM == 3 ? N : 1); ++c2)
    for (int c1 = 0; c1 < N; ++c1)
      for (int c0 = 0; c0 < N; ++c0) {
        const double wt = wp[c0] * wp[N + c1] * (DIM == 3 ? wp[2 * N + c2] : 1.0);
        const int i = c0 + N * c1 + N * N * c2;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += wt * double(a.U[at(blk, i, v, e, S::NUP, NV)]);
      }
  const int64_t o = dst ? dst[p] : p;  // row of the output (points of several order groups)
#pragma unroll
  for (int v = 0; v < NV; ++v) out[o * NV + v] = acc[v];
}

template <typename T, int DIM, int ORDER>
static hipError_t probe_t(const LaunchCfg &c, const DevArrays &d, int64_t n, const int64_t *slot, const double *w,
                          const int64_t *dst, double *out) {
  KArgs<T> a = make_args<T>(c, d);
  hipLaunchKernelGGL((k_probe<T, DIM, ORDER>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, c.stream, a, n, slot,
                     w, dst, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T> static KArgs<T> make_args(const LaunchCfg &c, const DevArrays &d) {
  KArgs<T> a;
  a.U = (T *)d.U; a.US = (T *)d.US; a.ACC = (T *)d.ACC; a.UF = (T *)d.UF; a.DU = (T *)d.DU;
  a.FI = (T *)d.FI; a.GU = (T *)d.GU; a.FT = (T *)d.FT; a.PV = (T *)d.PV; a.RES = (T *)d.RES;
  a.opInt = (const T *)d.opInt; a.opGrad = (const T *)d.opGrad; a.opGcorr = (const T *)d.opGcorr;
  a.opDivS = (const T *)d.opDivS; a.opCorr = (const T *)d.opCorr; a.basis = (const T *)d.basis;
  a.SM = d.SM; a.IJ = d.IJ; a.FN = d.FN; a.FA = d.FA; a.bdt = d.bdt; a.fsd = d.fsd; a.wface = d.wface;
  a.XN = d.XN; a.GQ = d.GQ;
  a.XC = d.XC; a.ZZ = d.ZZ; a.FCX = d.FCX;
  a.IJC = d.IJC; a.IZ = d.IZ;
  a.FC = d.FC; a.fsum = d.fsum; a.stage64 = d.stage64;
  a.NB = d.NB; a.NBF = d.NBF; a.bcount = d.bcount; a.bdesign = d.bdesign; a.bcanon = d.bcanon; a.wall_first = d.wall_first;
  a.flag = d.flag;
  a.MO = d.MO; a.MG = d.MG; a.MC = d.MC; a.MW = d.MW;
  a.GUF = (const T *const *)d.GUF; a.GPV = (const T *const *)d.GPV; a.MT = (T *)d.MT;
  a.PO = d.PO; a.PC = d.PC; a.PW = d.PW;
  a.nblk = c.nblk; a.n_canon = c.n_canon; a.ndesign = c.ndesign;
  a.xcd = (c.variant_mask & NO_XCD_REMAP) ? 0 : 1;
  a.scatter = 0;
  a.gam = T(c.gamma); a.mu = T(c.mu); a.kappa = T(c.mu * c.gamma / c.prandtl);
  a.igm1 = T(1.0 / (c.gamma - 1.0));
  return a;
}

template <typename T, int DIM, int ORDER, int FV, int TILE, bool SCAT>
static void go_stage_a(const LaunchCfg &c, const KArgs<T> &a, const T *X, bool forces) {
  using F = FS<T, DIM, ORDER, TILE>;
  const dim3 grid(static_cast<unsigned>(c.nblk * (EB / F::EW_A)));
  hipLaunchKernelGGL((k_stage_a<T, DIM, ORDER, FV, TILE, SCAT>), grid, dim3(F::WG_A), 0, c.stream, a, X,
                     int(forces));
}

// tile shapes other than the default are compiled for 3D one-order meshes of order 1 up
template <int DIM, int ORDER, int FV> constexpr bool tiled() { return DIM == 3 && ORDER >= 1 && !mortar_fv<FV>(); }

template <typename T, int DIM, int ORDER, int FV, bool SCAT>
static void launch_stage_a_tiles(const LaunchCfg &c, const KArgs<T> &a, const T *X, bool forces) {
  if constexpr (tiled<DIM, ORDER, FV>()) {
    switch (tile_a(c.variant_mask)) {
      case TILE_HALF: return go_stage_a<T, DIM, ORDER, FV, TILE_HALF, SCAT>(c, a, X, forces);
      case TILE_QUARTER: return go_stage_a<T, DIM, ORDER, FV, TILE_QUARTER, SCAT>(c, a, X, forces);
      case TILE_MFMA:
        if constexpr (sizeof(T) == 4 && ORDER == 3)
          return go_stage_a<T, DIM, ORDER, FV, TILE_MFMA, SCAT>(c, a, X, forces);
        break;
      default: break;
    }
  }
  go_stage_a<T, DIM, ORDER, FV, TILE_DEFAULT, SCAT>(c, a, X, forces);
}

// the exchange by scatter exists for one-order meshes (no mortar faces)
template <typename T, int DIM, int ORDER, int FV>
static void launch_stage_a(const LaunchCfg &c, const KArgs<T> &a, const T *X, bool forces) {
  if constexpr (!mortar_fv<FV>())
    if (c.variant_mask & SCATTER_EXCHANGE) return launch_stage_a_tiles<T, DIM, ORDER, FV, true>(c, a, X, forces);
  launch_stage_a_tiles<T, DIM, ORDER, FV, false>(c, a, X, forces);
}

template <typename T, int DIM, int ORDER, int FV, int TILE, bool SCAT>
static hipError_t go_stage_b(const LaunchCfg &c, int mode, const KArgs<T> &a) {
  using F = FS<T, DIM, ORDER, TILE>;
  const dim3 grid(static_cast<unsigned>(c.nblk * (EB / F::EW_B))), wgs(F::WG_B);
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, wgs, 0, c.stream, a); };
  switch (mode) {
    case MODE_RK0: go(k_stage_b<T, DIM, ORDER, MODE_RK0, FV, TILE, SCAT>); break;
    case MODE_RK1: go(k_stage_b<T, DIM, ORDER, MODE_RK1, FV, TILE, SCAT>); break;
    case MODE_RK2: go(k_stage_b<T, DIM, ORDER, MODE_RK2, FV, TILE, SCAT>); break;
    case MODE_RK3: go(k_stage_b<T, DIM, ORDER, MODE_RK3, FV, TILE, SCAT>); break;
    case MODE_RESID: go(k_stage_b<T, DIM, ORDER, MODE_RESID, FV, TILE, SCAT>); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int DIM, int ORDER, int FV, bool SCAT>
static hipError_t launch_stage_b_tiles(const LaunchCfg &c, int mode, const KArgs<T> &a) {
  if constexpr (tiled<DIM, ORDER, FV>()) {
    switch (tile_b(c.variant_mask)) {
      case TILE_HALF: return go_stage_b<T, DIM, ORDER, FV, TILE_HALF, SCAT>(c, mode, a);
      case TILE_QUARTER: return go_stage_b<T, DIM, ORDER, FV, TILE_QUARTER, SCAT>(c, mode, a);
      default: break;
    }
  }
  return go_stage_b<T, DIM, ORDER, FV, TILE_DEFAULT, SCAT>(c, mode, a);
}

template <typename T, int DIM, int ORDER, int FV>
static hipError_t launch_stage_b(const LaunchCfg &c, int mode, const KArgs<T> &a) {
  if constexpr (!mortar_fv<FV>())
    if (c.variant_mask & SCATTER_EXCHANGE) return launch_stage_b_tiles<T, DIM, ORDER, FV, true>(c, mode, a);
  return launch_stage_b_tiles<T, DIM, ORDER, FV, false>(c, mode, a);
}

template <typename T, int DIM, int ORDER>
static hipError_t launch_t(int kernel, const LaunchCfg &c, const DevArrays &d, int stage, int mode,
                           bool forces) {
  using S = Shape<DIM, ORDER>;
  using TT = TS<T, DIM, ORDER>;
  KArgs<T> a = make_args<T>(c, d);
  const T *X = stage == 0 ? a.U : a.US;
  const dim3 blk(256);
  const bool tensor = (c.variant_mask >> kernel) & 1;
  switch (kernel) {
    case K_INTERP:
      // the exchange by scatter wants the initial trace in the partners' slots: the
      // sum-factorised trace kernel writes it there (a.scatter)
      a.scatter = (c.variant_mask & SCATTER_EXCHANGE) && !d.MO ? 1 : 0;
      if (tensor || a.scatter)
        hipLaunchKernelGGL((t_interp<T, DIM, ORDER>), dim3(c.nblk * (EB / TT::EW_INTERP)), blk, 0, c.stream, a, X);
      else
        hipLaunchKernelGGL((k_interp<T, DIM, ORDER>), dim3((c.nblk * S::RTF + 3) / 4), blk, 0, c.stream, a, X);
      break;
    case K_FACE: {
      const int64_t thr = c.nblk * S::NFPAD * EB;
      hipLaunchKernelGGL((k_face<T, DIM, ORDER>), dim3((thr + 255) / 256), blk, 0, c.stream, a);
      break;
    }
    case K_GRAD:
      if (tensor)
        hipLaunchKernelGGL((t_grad<T, DIM, ORDER>), dim3(c.nblk * (EB / TT::EW_GRAD)), blk, 0, c.stream, a, X);
      else
        hipLaunchKernelGGL((k_grad<T, DIM, ORDER>), dim3((c.nblk * S::RTU + 3) / 4), blk, 0, c.stream, a, X);
      break;
    case K_VISC:
      if (tensor)
        hipLaunchKernelGGL((t_visc<T, DIM, ORDER>), dim3(c.nblk * (EB / TT::EW_VISC)), blk, 0, c.stream, a,
                           int(forces));
      else
        hipLaunchKernelGGL((k_visc<T, DIM, ORDER>), dim3((c.nblk * S::RTF + 3) / 4), blk, 0, c.stream, a,
                           int(forces));
      break;
    case K_STAGE_A:
      if (d.MO && DIM == 3 && (c.variant_mask & EXTRUDED_METRICS) && d.XC && d.IJC)
        launch_stage_a<T, DIM, ORDER, DIM == 3 ? FV_MORTAR_EXTR : FV_MORTAR>(c, a, X, forces);
      else if (d.MO)
        launch_stage_a<T, DIM, ORDER, FV_MORTAR>(c, a, X, forces);
      else if (DIM == 3 && (c.variant_mask & EXTRUDED_METRICS) && d.XC)
        launch_stage_a<T, DIM, ORDER, DIM == 3 ? FV_EXTR : FV_STORED>(c, a, X, forces);
      else if (DIM == 3 && !(c.variant_mask & STORED_METRICS))
        launch_stage_a<T, DIM, ORDER, DIM == 3 ? FV_NODE : FV_STORED>(c, a, X, forces);
      else
        launch_stage_a<T, DIM, ORDER, FV_STORED>(c, a, X, forces);
      break;
    case K_STAGE_B:
      if (d.MO && DIM == 3 && (c.variant_mask & EXTRUDED_METRICS) && d.XC && d.IJC)
        return launch_stage_b<T, DIM, ORDER, DIM == 3 ? FV_MORTAR_EXTR : FV_MORTAR>(c, mode, a);
      if (d.MO) return launch_stage_b<T, DIM, ORDER, FV_MORTAR>(c, mode, a);
      // the extruded first launch scales the half fluxes by the area factor like FV_NODE,
      // and the second takes 1/|J| from the column factors
      if (DIM == 3 && (c.variant_mask & EXTRUDED_METRICS) && d.XC && d.IJC)
        return launch_stage_b<T, DIM, ORDER, DIM == 3 ? FV_EXTR : FV_STORED>(c, mode, a);
      if (DIM == 3 && !(c.variant_mask & STORED_METRICS))
        return launch_stage_b<T, DIM, ORDER, DIM == 3 ? FV_NODE : FV_STORED>(c, mode, a);
      return launch_stage_b<T, DIM, ORDER, FV_STORED>(c, mode, a);
    case K_DIVRK:
      if (tensor)
        hipLaunchKernelGGL((t_divrk<T, DIM, ORDER>), dim3(c.nblk * (EB / TT::EW_DIV)), blk, 0, c.stream, a, mode);
      else
        hipLaunchKernelGGL((k_divrk<T, DIM, ORDER>), dim3((c.nblk * S::RTU + 3) / 4), blk, 0, c.stream, a, mode);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int DIM, int ORDER>
static hipError_t pack_t(const LaunchCfg &c, const DevArrays &d, bool to_dev, void *dst) {
  using S = Shape<DIM, ORDER>;
  KArgs<T> a = make_args<T>(c, d);
  const int64_t thr = c.nblk * S::NUP * S::NV * EB;
  hipLaunchKernelGGL((k_pack<T, DIM, ORDER>), dim3((thr + 255) / 256), dim3(256), 0, c.stream, a, (T *)dst,
                     int(to_dev));
  return hipGetLastError();
}

// The launchers are compiled in five parts, one object each, built in parallel: parts
// 0-3 hold the kernels of one precision and dimension (0 FP64 2D, 1 FP64 3D, 2 FP32 2D,
// 3 FP32 3D) for every order, part 4 the dispatch over them and the small kernels.
#ifndef FR_PART
#error "compile with -DFR_PART=0..4"
#endif
#define FR_CAT2(a, b) a##b
#define FR_CAT(a, b) FR_CAT2(a, b)

#if FR_PART < 4
using PartT = typename std::conditional<(FR_PART >= 2), float, double>::type;
constexpr int PART_DIM = (FR_PART & 1) ? 3 : 2;

#define FR_ORDERS(FN, ...)                                \
  do {                                                    \
    switch (c.order) {                                    \
      case 0: return FN<PartT, PART_DIM, 0>(__VA_ARGS__); \
      case 1: return FN<PartT, PART_DIM, 1>(__VA_ARGS__); \
      case 2: return FN<PartT, PART_DIM, 2>(__VA_ARGS__); \
      case 3: return FN<PartT, PART_DIM, 3>(__VA_ARGS__); \
      case 4: return FN<PartT, PART_DIM, 4>(__VA_ARGS__); \
      default: return hipErrorInvalidValue;               \
    }                                                     \
  } while (0)

hipError_t FR_CAT(launch_kernel_part, FR_PART)(int kernel, const LaunchCfg &c, const DevArrays &a, int stage,
                                               int mode, bool forces) {
  FR_ORDERS(launch_t, kernel, c, a, stage, mode, forces);
}
hipError_t FR_CAT(launch_pack_part, FR_PART)(const LaunchCfg &c, const DevArrays &a, bool to_dev, void *dst) {
  FR_ORDERS(pack_t, c, a, to_dev, dst);
}
hipError_t FR_CAT(launch_probe_part, FR_PART)(const LaunchCfg &c, const DevArrays &a, int64_t n, const int64_t *slot,
                                              const double *w, const int64_t *dst, double *out) {
  FR_ORDERS(probe_t, c, a, n, slot, w, dst, out);
}
#else
#define FR_PART_DECL(k)                                                                                         \
  hipError_t launch_kernel_part##k(int, const LaunchCfg &, const DevArrays &, int, int, bool);                   \
  hipError_t launch_pack_part##k(const LaunchCfg &, const DevArrays &, bool, void *);                           \
  hipError_t launch_probe_part##k(const LaunchCfg &, const DevArrays &, int64_t, const int64_t *, const double *, \
                                  const int64_t *, double *);
FR_PART_DECL(0)
FR_PART_DECL(1)
FR_PART_DECL(2)
FR_PART_DECL(3)

// part holding the kernels of a launch configuration (precision 0 = FP64, 1 = FP32)
static int part_of(const LaunchCfg &c) {
  if ((c.prec != 0 && c.prec != 1) || (c.dim != 2 && c.dim != 3)) return -1;
  return 2 * c.prec + (c.dim == 3 ? 1 : 0);
}

#define FR_PARTS(FN, ...)                       \
  do {                                          \
    switch (part_of(c)) {                       \
      case 0: return FN##_part0(__VA_ARGS__);   \
      case 1: return FN##_part1(__VA_ARGS__);   \
      case 2: return FN##_part2(__VA_ARGS__);   \
      case 3: return FN##_part3(__VA_ARGS__);   \
      default: return hipErrorInvalidValue;     \
    }                                           \
  } while (0)

bool kernels_available(int prec, int dim, int order) {
  return (prec == 0 || prec == 1) && (dim == 2 || dim == 3) && order >= 0 && order <= 4;
}

hipError_t launch_kernel(int kernel, const LaunchCfg &c, const DevArrays &a, int stage, int mode, bool forces) {
  FR_PARTS(launch_kernel, kernel, c, a, stage, mode, forces);
}

hipError_t launch_pack(const LaunchCfg &c, const DevArrays &a, bool to_dev, void *dst) {
  FR_PARTS(launch_pack, c, a, to_dev, dst);
}

hipError_t launch_probe(const LaunchCfg &c, const DevArrays &a, int64_t n, const int64_t *slot, const double *w,
                        const int64_t *dst, double *out) {
  FR_PARTS(launch_probe, c, a, n, slot, w, dst, out);
}

hipError_t launch_force_reduce(const LaunchCfg &c, const DevArrays &a) {
  hipLaunchKernelGGL(k_force_reduce, dim3(c.ndesign), dim3(256), 0, c.stream, a.FC, a.wall_first, a.fsum);
  return hipGetLastError();
}

hipError_t launch_clear_flag(const LaunchCfg &c, const DevArrays &a) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, c.stream, a.flag);
  return hipGetLastError();
}
#endif

}  // namespace fr
