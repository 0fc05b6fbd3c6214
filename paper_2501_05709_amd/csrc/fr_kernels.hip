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

#include "fr_internal.hpp"

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
  const T *opInt, *opGrad, *opGcorr, *opDivS, *opCorr;
  const double *SM, *IJ, *FN, *FA, *bdt, *fsd, *wface;
  double *FC, *fsum, *stage64;
  const int *NB, *bcount, *bdesign;
  const int64_t *bcanon, *wall_first;
  int *flag;
  int64_t nblk, n_canon;
  int ndesign;
  T gam, mu, kappa;
};

// ---------------------------------------------------------------------------
// gas physics (paper Eqs. (1)-(7))
// ---------------------------------------------------------------------------

template <typename T, int D> struct Gas {
  static constexpr int NV = D + 2;
  T gam, mu, kappa;

  __device__ inline T pressure(const T *u) const {
    T ke = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) ke += u[1 + i] * u[1 + i];
    return (gam - T(1)) * (u[D + 1] - T(0.5) * ke / u[0]);
  }

  __device__ inline void flux_inv(const T *u, T F[D][NV]) const {
    const T ir = T(1) / u[0];
    T v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = u[1 + i] * ir;
    const T p = pressure(u);
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
    const T ir = T(1) / u[0];
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

  __device__ inline void rusanov(const T *uL, const T *uR, const T *n, T *Fn) const {
    T FL[D][NV], FR[D][NV];
    flux_inv(uL, FL);
    flux_inv(uR, FR);
    T vnL = 0, vnR = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      vnL += uL[1 + j] * n[j];
      vnR += uR[1 + j] * n[j];
    }
    vnL /= uL[0];
    vnR /= uR[0];
    const T lamL = fabs(vnL) + sqrt(gam * pressure(uL) / uL[0]);
    const T lamR = fabs(vnR) + sqrt(gam * pressure(uR) / uR[0]);
    const T lam = lamL > lamR ? lamL : lamR;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T fl = 0, fr = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        fl += FL[j][v] * n[j];
        fr += FR[j][v] * n[j];
      }
      Fn[v] = T(0.5) * (fl + fr) - T(0.5) * lam * (uR[v] - uL[v]);
    }
  }

  // Riemann-invariant far field: outgoing invariant from the interior,
  // incoming from the free stream; entropy and tangential velocity from the
  // upwind side.
  __device__ inline void farfield(const T *uL, const T *n, const double *fs, T *ub) const {
    const T rhoL = uL[0];
    T vL[D], vI[D];
    T vnL = 0, vnI = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      vL[j] = uL[1 + j] / rhoL;
      vI[j] = T(fs[1 + j]);
      vnL += vL[j] * n[j];
      vnI += vI[j] * n[j];
    }
    const T pL = pressure(uL);
    const T rhoI = T(fs[0]), pI = T(fs[4]);
    const T cL = sqrt(gam * pL / rhoL), cI = sqrt(gam * pI / rhoI);
    const T Rp = vnL + T(2) * cL / (gam - T(1));
    const T Rm = vnI - T(2) * cI / (gam - T(1));
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
    const T rhob = pow(cb * cb / (gam * s), T(1) / (gam - T(1)));
    const T pb = rhob * cb * cb / gam;
    T ke = 0;
    ub[0] = rhob;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const T vb = vt[j] + vnb * n[j];
      ub[1 + j] = rhob * vb;
      ke += vb * vb;
    }
    ub[D + 1] = pb / (gam - T(1)) + T(0.5) * rhob * ke;
  }

  // no-slip adiabatic wall: common solution with zero velocity
  __device__ inline void wall_common(const T *uL, T *uc) const {
    T ke = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) ke += uL[1 + i] * uL[1 + i];
    uc[0] = uL[0];
#pragma unroll
    for (int i = 0; i < D; ++i) uc[1 + i] = 0;
    uc[D + 1] = uL[D + 1] - T(0.5) * ke / uL[0];
  }
};

__device__ inline size_t at(int64_t blk, int pt, int ch, int e, int NPT, int NCH) {
  return ((size_t(blk) * NPT + pt) * NCH + ch) * EB + e;
}

// ---------------------------------------------------------------------------
// K_INTERP: u_f = M_int u
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
  const T *Xb = X + size_t(blk) * S::NUP * S::NV * EB;
#pragma unroll 4
  for (int kt = 0; kt < S::KTU; ++kt) {
    const T av = a.opInt[(size_t(rt) * S::KTU + kt) * 64 + lane];
    const int pt = kt * 4 + g;
#pragma unroll
    for (int v = 0; v < S::NV; ++v) acc[v] = M::mac(av, Xb[(pt * S::NV + v) * EB + e], acc[v]);
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

// ---------------------------------------------------------------------------
// K_FACE: common solution and Rusanov flux, one thread per element flux point
// ---------------------------------------------------------------------------
template <typename T, int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_face(KArgs<T> a) {
  using S = Shape<DIM, ORDER>;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int e = int(t & 15);
  const int q = int((t >> 4) % S::NFPAD);
  const int64_t blk = (t >> 4) / S::NFPAD;
  if (blk >= a.nblk || q >= S::NF || e >= a.bcount[blk]) return;
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa};
  T uf[S::NV], ur[S::NV], du[S::NV], fi[S::NV], n[DIM];
#pragma unroll
  for (int v = 0; v < S::NV; ++v) uf[v] = a.UF[at(blk, q, v, e, S::NFPAD, S::NV)];
#pragma unroll
  for (int j = 0; j < DIM; ++j) n[j] = T(a.FN[at(blk, q, j, e, S::NFPAD, DIM)]);
  const int nb = a.NB[(size_t(blk) * S::NFPAD + q) * EB + e];
  if (nb >= 0) {
    const size_t base = size_t(nb / EB) * S::NV * EB + (nb % EB);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      ur[v] = a.UF[base + v * EB];
      du[v] = T(0.5) * (ur[v] - uf[v]);
    }
    gas.rusanov(uf, ur, n, fi);
  } else if (((-nb) & 3) == BC_FARFIELD) {
    gas.farfield(uf, n, a.fsd + 5 * a.bdesign[blk], ur);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) du[v] = ur[v] - uf[v];
    gas.rusanov(uf, ur, n, fi);
  } else {
    T uc[S::NV];
    gas.wall_common(uf, uc);
#pragma unroll
    for (int v = 0; v < S::NV; ++v) du[v] = uc[v] - uf[v];
    ur[0] = uf[0];
#pragma unroll
    for (int i = 0; i < DIM; ++i) ur[1 + i] = -uf[1 + i];
    ur[DIM + 1] = uf[DIM + 1];
    gas.rusanov(uf, ur, n, fi);
  }
#pragma unroll
  for (int v = 0; v < S::NV; ++v) {
    a.DU[at(blk, q, v, e, S::NFPAD, S::NV)] = du[v];
    a.FI[at(blk, q, v, e, S::NFPAD, S::NV)] = fi[v];
  }
}

// ---------------------------------------------------------------------------
// K_GRAD: corrected gradient -> physical gradient -> transformed flux
// ---------------------------------------------------------------------------
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
  const T *Xb = X + size_t(blk) * S::NUP * S::NV * EB;
#pragma unroll 2
  for (int kt = 0; kt < S::KTU; ++kt) {
    const int pt = kt * 4 + g;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = Xb[(pt * S::NV + v) * EB + e];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const T av = a.opGrad[((size_t(k) * S::RTU + rt) * S::KTU + kt) * 64 + lane];
#pragma unroll
      for (int v = 0; v < S::NV; ++v) acc[k][v] = M::mac(av, b[v], acc[k][v]);
    }
  }
  const T *Db = a.DU + size_t(blk) * S::NFPAD * S::NV * EB;
#pragma unroll 2
  for (int kt = 0; kt < S::KTF; ++kt) {
    const int pt = kt * 4 + g;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = Db[(pt * S::NV + v) * EB + e];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const T av = a.opGcorr[((size_t(k) * S::RTU + rt) * S::KTF + kt) * 64 + lane];
#pragma unroll
      for (int v = 0; v < S::NV; ++v) acc[k][v] = M::mac(av, b[v], acc[k][v]);
    }
  }
  if (e >= a.bcount[blk]) return;
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = rt * 16 + M::row(g, j);
    if (i >= S::NU) break;
    T u[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) u[v] = Xb[(i * S::NV + v) * EB + e];
    double Sm[DIM][DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int c = 0; c < DIM; ++c) Sm[k][c] = a.SM[at(blk, i, k * DIM + c, e, S::NUP, DIM * DIM)];
    const double ij = a.IJ[(size_t(blk) * S::NUP + i) * EB + e];
    T gu[DIM][S::NV];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int v = 0; v < S::NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) s += Sm[k][c] * double(acc[k][v][j]);
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
}

// ---------------------------------------------------------------------------
// K_VISC: gradient trace and viscous common-flux parts at flux points
// ---------------------------------------------------------------------------
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
  const T *Gb = a.GU + size_t(blk) * S::NUP * S::NG * EB;
#pragma unroll 2
  for (int kt = 0; kt < S::KTU; ++kt) {
    const T av = a.opInt[(size_t(rt) * S::KTU + kt) * 64 + lane];
    const int pt = kt * 4 + g;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int v = 0; v < S::NV; ++v)
        acc[k][v] = M::mac(av, Gb[(pt * S::NG + k * S::NV + v) * EB + e], acc[k][v]);
  }
  if (e >= a.bcount[blk]) return;
  const Gas<T, DIM> gas{a.gam, a.mu, a.kappa};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int q = rt * 16 + M::row(g, j);
    if (q >= S::NF) break;
    T uf[S::NV], gf[DIM][S::NV], n[DIM], Fv[DIM][S::NV], pv[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) uf[v] = a.UF[at(blk, q, v, e, S::NFPAD, S::NV)];
    double nd[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      nd[c] = a.FN[at(blk, q, c, e, S::NFPAD, DIM)];
      n[c] = T(nd[c]);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int v = 0; v < S::NV; ++v) gf[c][v] = acc[c][v][j];
    const int nb = a.NB[(size_t(blk) * S::NFPAD + q) * EB + e];
    if (nb >= 0) {
      gas.flux_vis(uf, gf, Fv, false);
#pragma unroll
      for (int v = 0; v < S::NV; ++v) {
        T s = 0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) s += Fv[c][v] * n[c];
        pv[v] = T(0.5) * s;
      }
    } else {
      const int code = -nb;
      T ub[S::NV];
      if ((code & 3) == BC_FARFIELD) {
        gas.farfield(uf, n, a.fsd + 5 * a.bdesign[blk], ub);
        gas.flux_vis(ub, gf, Fv, false);
      } else {
        gas.wall_common(uf, ub);
        gas.flux_vis(ub, gf, Fv, true);
      }
#pragma unroll
      for (int v = 0; v < S::NV; ++v) {
        T s = 0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) s += Fv[c][v] * n[c];
        pv[v] = a.FI[at(blk, q, v, e, S::NFPAD, S::NV)] - s;
      }
      if (forces && (code & 3) == BC_WALL) {
        // traction of the fluid on the body: W A (p n - tau . n), interior trace
        T Fw[DIM][S::NV];
        gas.flux_vis(uf, gf, Fw, false);
        const double p = double(gas.pressure(uf));
        const double wA = a.wface[q] * a.FA[(size_t(blk) * S::NFPAD + q) * EB + e];
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
}

// ---------------------------------------------------------------------------
// K_DIVRK: corrected divergence, residual, fused RK4 stage
// ---------------------------------------------------------------------------
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
  const T *Fb = a.FT + size_t(blk) * S::NUP * S::NG * EB;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
#pragma unroll 2
    for (int kt = 0; kt < S::KTU; ++kt) {
      const T av = a.opDivS[((size_t(rt) * DIM + k) * S::KTU + kt) * 64 + lane];
      const int pt = kt * 4 + g;
#pragma unroll
      for (int v = 0; v < S::NV; ++v) acc[v] = M::mac(av, Fb[(pt * S::NG + k * S::NV + v) * EB + e], acc[v]);
    }
  }
#pragma unroll 2
  for (int kt = 0; kt < S::KTF; ++kt) {
    const T av = a.opCorr[(size_t(rt) * S::KTF + kt) * 64 + lane];
    const int q = kt * 4 + g;
    T b[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) b[v] = 0;
    if (q < S::NF && e < nvalid) {
      const size_t fq = (size_t(blk) * S::NFPAD + q) * EB + e;
      const int nb = a.NB[fq];
      const double A = a.FA[fq];
      if (nb >= 0) {
        const size_t base = size_t(nb / EB) * S::NV * EB + (nb % EB);
#pragma unroll
        for (int v = 0; v < S::NV; ++v) {
          const T f = a.FI[at(blk, q, v, e, S::NFPAD, S::NV)] - a.PV[at(blk, q, v, e, S::NFPAD, S::NV)] +
                      a.PV[base + v * EB];
          b[v] = T(A * double(f));
        }
      } else {
#pragma unroll
        for (int v = 0; v < S::NV; ++v) b[v] = T(A * double(a.PV[at(blk, q, v, e, S::NFPAD, S::NV)]));
      }
    }
#pragma unroll
    for (int v = 0; v < S::NV; ++v) acc[v] = M::mac(av, b[v], acc[v]);
  }
  if (e >= nvalid) return;
  const T dt = T(a.bdt[blk]);
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = rt * 16 + M::row(g, j);
    if (i >= S::NU) break;
    const double ij = a.IJ[(size_t(blk) * S::NUP + i) * EB + e];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
      const size_t x = at(blk, i, v, e, S::NUP, S::NV);
      const T r = T(-double(acc[v][j]) * ij);
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
  if (bad) atomicOr(a.flag, 1);
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

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T> static KArgs<T> make_args(const LaunchCfg &c, const DevArrays &d) {
  KArgs<T> a;
  a.U = (T *)d.U; a.US = (T *)d.US; a.ACC = (T *)d.ACC; a.UF = (T *)d.UF; a.DU = (T *)d.DU;
  a.FI = (T *)d.FI; a.GU = (T *)d.GU; a.FT = (T *)d.FT; a.PV = (T *)d.PV; a.RES = (T *)d.RES;
  a.opInt = (const T *)d.opInt; a.opGrad = (const T *)d.opGrad; a.opGcorr = (const T *)d.opGcorr;
  a.opDivS = (const T *)d.opDivS; a.opCorr = (const T *)d.opCorr;
  a.SM = d.SM; a.IJ = d.IJ; a.FN = d.FN; a.FA = d.FA; a.bdt = d.bdt; a.fsd = d.fsd; a.wface = d.wface;
  a.FC = d.FC; a.fsum = d.fsum; a.stage64 = d.stage64;
  a.NB = d.NB; a.bcount = d.bcount; a.bdesign = d.bdesign; a.bcanon = d.bcanon; a.wall_first = d.wall_first;
  a.flag = d.flag;
  a.nblk = c.nblk; a.n_canon = c.n_canon; a.ndesign = c.ndesign;
  a.gam = T(c.gamma); a.mu = T(c.mu); a.kappa = T(c.mu * c.gamma / c.prandtl);
  return a;
}

template <typename T, int DIM, int ORDER>
static hipError_t launch_t(int kernel, const LaunchCfg &c, const DevArrays &d, int stage, int mode,
                           bool forces) {
  using S = Shape<DIM, ORDER>;
  KArgs<T> a = make_args<T>(c, d);
  const T *X = stage == 0 ? a.U : a.US;
  const dim3 blk(256);
  switch (kernel) {
    case K_INTERP: {
      const int64_t waves = c.nblk * S::RTF;
      hipLaunchKernelGGL((k_interp<T, DIM, ORDER>), dim3((waves + 3) / 4), blk, 0, c.stream, a, X);
      break;
    }
    case K_FACE: {
      const int64_t thr = c.nblk * S::NFPAD * EB;
      hipLaunchKernelGGL((k_face<T, DIM, ORDER>), dim3((thr + 255) / 256), blk, 0, c.stream, a);
      break;
    }
    case K_GRAD: {
      const int64_t waves = c.nblk * S::RTU;
      hipLaunchKernelGGL((k_grad<T, DIM, ORDER>), dim3((waves + 3) / 4), blk, 0, c.stream, a, X);
      break;
    }
    case K_VISC: {
      const int64_t waves = c.nblk * S::RTF;
      hipLaunchKernelGGL((k_visc<T, DIM, ORDER>), dim3((waves + 3) / 4), blk, 0, c.stream, a, int(forces));
      break;
    }
    case K_DIVRK: {
      const int64_t waves = c.nblk * S::RTU;
      hipLaunchKernelGGL((k_divrk<T, DIM, ORDER>), dim3((waves + 3) / 4), blk, 0, c.stream, a, mode);
      break;
    }
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

#define FR_DISPATCH(FN, ...)                                                              \
  do {                                                                                    \
    const int key = c.prec * 100 + c.dim * 10 + c.order;                                  \
    switch (key) {                                                                        \
      case 21: return FN<double, 2, 1>(__VA_ARGS__);                                      \
      case 22: return FN<double, 2, 2>(__VA_ARGS__);                                      \
      case 23: return FN<double, 2, 3>(__VA_ARGS__);                                      \
      case 24: return FN<double, 2, 4>(__VA_ARGS__);                                      \
      case 31: return FN<double, 3, 1>(__VA_ARGS__);                                      \
      case 32: return FN<double, 3, 2>(__VA_ARGS__);                                      \
      case 33: return FN<double, 3, 3>(__VA_ARGS__);                                      \
      case 34: return FN<double, 3, 4>(__VA_ARGS__);                                      \
      case 121: return FN<float, 2, 1>(__VA_ARGS__);                                      \
      case 122: return FN<float, 2, 2>(__VA_ARGS__);                                      \
      case 123: return FN<float, 2, 3>(__VA_ARGS__);                                      \
      case 124: return FN<float, 2, 4>(__VA_ARGS__);                                      \
      case 131: return FN<float, 3, 1>(__VA_ARGS__);                                      \
      case 132: return FN<float, 3, 2>(__VA_ARGS__);                                      \
      case 133: return FN<float, 3, 3>(__VA_ARGS__);                                      \
      case 134: return FN<float, 3, 4>(__VA_ARGS__);                                      \
      default: return hipErrorInvalidValue;                                               \
    }                                                                                     \
  } while (0)

bool kernels_available(int prec, int dim, int order) {
  return (prec == 0 || prec == 1) && (dim == 2 || dim == 3) && order >= 1 && order <= 4;
}

hipError_t launch_kernel(int kernel, const LaunchCfg &c, const DevArrays &a, int stage, int mode, bool forces) {
  FR_DISPATCH(launch_t, kernel, c, a, stage, mode, forces);
}

hipError_t launch_pack(const LaunchCfg &c, const DevArrays &a, bool to_dev, void *dst) {
  FR_DISPATCH(pack_t, c, a, to_dev, dst);
}

hipError_t launch_force_reduce(const LaunchCfg &c, const DevArrays &a) {
  hipLaunchKernelGGL(k_force_reduce, dim3(c.ndesign), dim3(256), 0, c.stream, a.FC, a.wall_first, a.fsum);
  return hipGetLastError();
}

hipError_t launch_clear_flag(const LaunchCfg &c, const DevArrays &a) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, c.stream, a.flag);
  return hipGetLastError();
}

}  // namespace fr
