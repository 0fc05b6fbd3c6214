// Far-field acoustic pressure from samples on a stationary permeable data surface in a
// uniform stream: the moving-medium time-domain solution of the FW-H equation without
// the quadrupole term (the paper's Appendices A and B), summed by the advanced-time
// approach, with spanwise copies of the surface.  FP64 throughout.
//
// Device layout: the source strengths of every sample are formed when the sample is
// appended and kept as four time series per panel, [Q, L1, L2, L3][panel][time], time
// contiguous.  For one observer:
//   k_fwh_delay   per (copy, panel): arrival delay R / c0; per-block min and max
//   (host)        the common observer-time window from the extreme delays
//   k_fwh_filter  per panel: every copy's integrands at the window's observer times are
//                 one 8-tap stencil over the panel's series (cubic interpolation in source
//                 time composed with the fourth-order time derivative), weighted by the
//                 panel's geometric factors; the copies share the panel's series, so their
//                 stencils add up to one filter per series, formed once per evaluation
//   k_fwh_sum     per (panel chunk, time chunk): each panel's filters applied to its
//                 series at the chunk's observer times; partial sums per panel chunk
//   k_fwh_reduce_groups, k_fwh_reduce
//                 per observer time: the partial sums in fixed chunk order, in two levels
// Because the surface and the observer are stationary and the observer times are spaced
// by the sampling interval, each panel's fractional delay and hence its stencil weights
// are the same for every observer time: the sum is a delay-and-sum over the series.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "fr_internal.hpp"

namespace {

constexpr int NQ = 4;          // Q, L1, L2, L3
constexpr int SUM_WG = 256;    // threads of k_fwh_sum
constexpr int SUM_OUT = 8;     // consecutive observer times per thread
constexpr int SUM_PANELS = 8;  // panels per chunk
constexpr int SUM_PAIRS = 64;  // copies of one panel whose weights share the LDS
constexpr int SUM_SPAN = SUM_WG * SUM_OUT + 7 + 256;  // staged samples per series (delay spread up to 256)

struct Err {
  fr_status code;
  std::string msg;
};
[[noreturn]] void fail(fr_status c, const std::string &m) { throw Err{c, m}; }
void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(FR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
template <class F> fr_status guarded(F &&f) {
  try {
    f();
    return FR_OK;
  } catch (const Err &e) {
    fr::set_last_error(e.msg.c_str());
    return e.code;
  } catch (const std::bad_alloc &) {
    fr::set_last_error("host allocation failed");
    return FR_E_NOMEM;
  }
}

struct Stream {
  double mach[3], U[3], c0, rho0, p0, g2;
};

// amplitude radius R*, phase radius R and their gradients for r = x - y (Appendix B)
struct Radii {
  double Rs, R, gRs[3], gR[3];
};
__device__ inline Radii radii(const double *x, const double *y, const Stream &s) {
  Radii o;
  double r[3], rr = 0.0, Mr = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    r[i] = x[i] - y[i];
    rr += r[i] * r[i];
    Mr += s.mach[i] * r[i];
  }
  o.Rs = sqrt(rr + s.g2 * Mr * Mr) / sqrt(s.g2);
  o.R = s.g2 * (o.Rs - Mr);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.gRs[i] = (r[i] + s.g2 * Mr * s.mach[i]) / (s.g2 * o.Rs);
    o.gR[i] = s.g2 * (o.gRs[i] - s.mach[i]);
  }
  return o;
}

__device__ inline void panel_position(const double *geo, int64_t j, int c, int ncopy, const double *shift,
                                      double *y) {
  const double k = double(c) - 0.5 * double(ncopy - 1);
#pragma unroll
  for (int i = 0; i < 3; ++i) y[i] = geo[j * 7 + i] + k * shift[i];
}

// source strengths of appended snapshots (Appendix A, stationary surface):
// Q = rho (u_n + U_n) - rho0 U_n, L_i = (p - p0) n_i + rho u_i (u_n + U_n)
__global__ __launch_bounds__(256) void k_fwh_append(const double *__restrict__ samples, const double *__restrict__ geo,
                                                    int64_t np, int64_t nsnap, int64_t k0, int64_t cap, Stream s,
                                                    double *__restrict__ src) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np * nsnap) return;
  const int64_t j = t % np, k = t / np;
  const double *x = samples + (k * np + j) * 5;
  const double *n = geo + j * 7 + 3;
  const double rho = x[0], p = x[4];
  const double un = x[1] * n[0] + x[2] * n[1] + x[3] * n[2];
  const double Un = s.U[0] * n[0] + s.U[1] * n[1] + s.U[2] * n[2];
  const double flux = rho * (un + Un);
  const int64_t col = j * cap + k0 + k;
  src[0 * np * cap + col] = flux - s.rho0 * Un;
#pragma unroll
  for (int i = 0; i < 3; ++i) src[(1 + i) * np * cap + col] = (p - s.p0) * n[i] + flux * x[1 + i];
}

// samples from sampled conserved variables [n][nv]: rho, u - U (disturbance velocity), p
__global__ __launch_bounds__(256) void k_fwh_cons(const double *__restrict__ cons, int64_t n, int nv, int dim,
                                                  double gamma, Stream s, double *__restrict__ stage) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double *c = cons + j * nv;
  const double rho = c[0], ir = 1.0 / rho;
  double u[3] = {0.0, 0.0, 0.0}, ke = 0.0;
  for (int i = 0; i < dim; ++i) {
    u[i] = c[1 + i] * ir;
    ke += u[i] * u[i];
  }
  stage[j * 5 + 0] = rho;
#pragma unroll
  for (int i = 0; i < 3; ++i) stage[j * 5 + 1 + i] = u[i] - s.U[i];
  stage[j * 5 + 4] = (gamma - 1.0) * (c[dim + 1] - 0.5 * rho * ke);
}

__device__ inline double arrival_delay(const double *geo, int64_t cj, int64_t np, int ncopy, const double *shift,
                                       const double *xo, const Stream &s) {
  double y[3];
  panel_position(geo, cj % np, int(cj / np), ncopy, shift, y);
  return radii(xo, y, s).R / s.c0;
}

struct Geo3 {
  double shift[3], xo[3];
};

// arrival delay of every (copy, panel); per-block minimum and maximum
__global__ __launch_bounds__(256) void k_fwh_delay(const double *__restrict__ geo, int64_t np, int ncopy, Geo3 g,
                                                   Stream s, double *__restrict__ mm) {
  __shared__ double lo[256], hi[256];
  const int64_t n = np * ncopy;
  double a = INFINITY, b = -INFINITY;
  for (int64_t cj = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; cj < n; cj += int64_t(gridDim.x) * blockDim.x) {
    const double d = arrival_delay(geo, cj, np, ncopy, g.shift, g.xo, s);
    a = fmin(a, d);
    b = fmax(b, d);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mm[2 * blockIdx.x] = lo[0];
    mm[2 * blockIdx.x + 1] = hi[0];
  }
}

struct Window {
  double t_start, dt, tau0;
  int64_t n_out, nt;
  double t_end;  // end of the common window (the grid's last time is at most this)
};

// Stencil of copy c of panel j: the 8 weights per source series (cubic interpolation in
// source time composed with the fourth-order derivative, times the geometric factors of
// the thickness and loading integrands and the panel area, Appendix B) applied to the
// samples from the returned index (relative to observer time 0) on.
__device__ inline int64_t copy_stencil(const double *geo, int64_t j, int c, int ncopy, const Geo3 &g, const Stream &s,
                                       const Window &w, double area, double *wt) {
  const int64_t nv = w.nt - 4;  // samples with a time derivative
  double y[3];
  panel_position(geo, j, c, ncopy, g.shift, y);
  const Radii r = radii(g.xo, y, s);
  // position of observer time 0 among the panel's derivative-bearing samples; the clamp
  // keeps every stencil inside the record (it only absorbs rounding)
  const double pos0 = (w.t_start - w.tau0 - r.R / s.c0) / w.dt - 2.0;
  int64_t i0 = int64_t(floor(pos0));
  const int64_t i0max = nv - 3 - (w.n_out - 1);
  i0 = i0 > i0max ? i0max : i0;
  i0 = i0 < 1 ? 1 : i0;
  if (wt) {
    const double MR = s.mach[0] * r.gR[0] + s.mach[1] * r.gR[1] + s.mach[2] * r.gR[2];
    const double MRs = s.mach[0] * r.gRs[0] + s.mach[1] * r.gRs[1] + s.mach[2] * r.gRs[2];
    double a[NQ], b[NQ];
    a[0] = area * (1.0 - MR) / r.Rs;            // x Qdot
    b[0] = -area * s.c0 * MRs / (r.Rs * r.Rs);  // x Q
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      a[1 + i] = area * r.gR[i] / (s.c0 * r.Rs);   // x Ldot_i
      b[1 + i] = area * r.gRs[i] / (r.Rs * r.Rs);  // x L_i
    }
    const double sf = pos0 - double(i0);
    // cubic Lagrange weights (nodes -1..2) and their composition with the fourth-order
    // derivative (1, -8, 0, 8, -1) / 12 dt: 8 taps from sample i0 - 1
    const double l[4] = {-sf * (sf - 1.0) * (sf - 2.0) / 6.0, (sf + 1.0) * (sf - 1.0) * (sf - 2.0) / 2.0,
                         -(sf + 1.0) * sf * (sf - 2.0) / 2.0, (sf + 1.0) * sf * (sf - 1.0) / 6.0};
    double wv[8], wd[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) wv[d] = wd[d] = 0.0;
    const double fd[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
    const double idt = 1.0 / (12.0 * w.dt);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      wv[u + 2] += l[u];
#pragma unroll
      for (int v = 0; v < 5; ++v) wd[u + v] += l[u] * fd[v] * idt;
    }
#pragma unroll
    for (int x = 0; x < NQ; ++x)
#pragma unroll
      for (int d = 0; d < 8; ++d) wt[x * 8 + d] = a[x] * wd[d] + b[x] * wv[d];
  }
  return i0 - 1;
}

// All copies of a panel carry the same sample series, so their stencils add up to one
// filter per series over the copies' delay spread: H[x][k] = sum over copies c and taps d
// with b_c - b_min + d = k of the copy's weight (b_c its first sample).  k_fwh_filter forms
// H once per panel and evaluation: (1) the copies' first samples and their extremes,
// (2) H in LDS, the copies' weights going through LDS in batches of SUM_PAIRS and each
// thread owning filter taps (summed in copy order).  k_fwh_sum then, per panel of its
// chunk, (3) stages the stretch of the four series that its time chunk needs and applies
// H to each thread's SUM_OUT consecutive observer times.  This does (spread + 8) instead
// of 8 x copies multiply-adds per output; a panel whose copies' delays spread over more
// than HMAX - 8 samples is summed copy by copy instead.
constexpr int HMAX = 256 + 8;
// filter rows padded to whole blocks of SUM_OUT taps (the taps past nh stay zero)
constexpr int HROW = (HMAX + SUM_OUT - 1) / SUM_OUT * SUM_OUT + 4;

// Per panel, once per evaluation (the same for every time chunk): the first sample of
// each copy, their minimum b_min, and the combined filter of the copies, filt[j][x][k]
// for x < NQ, k < HROW (zero past nh); meta[j] = {b_min, nh}, nh = -1 when the copies'
// delays spread over more than HMAX - 8 samples (that panel is summed copy by copy).
__global__ __launch_bounds__(SUM_WG) void k_fwh_filter(const double *__restrict__ geo, int64_t np, int ncopy, Geo3 g,
                                                       Stream s, Window w, double *__restrict__ filt,
                                                       int64_t *__restrict__ meta) {
  __shared__ double Wt[SUM_PAIRS][NQ * 8];
  __shared__ int64_t Wb[SUM_PAIRS];
  __shared__ double H[NQ][HROW];
  __shared__ int64_t red_lo[SUM_WG], red_hi[SUM_WG];
  const int64_t j = blockIdx.x;
  const int tid = threadIdx.x;
  const double area = geo[j * 7 + 6];
  // (1) first samples of all copies: their minimum and maximum
  int64_t blo = INT64_MAX, bhi = INT64_MIN;
  for (int c = tid; c < ncopy; c += SUM_WG) {
    const int64_t b = copy_stencil(geo, j, c, ncopy, g, s, w, area, nullptr);
    blo = b < blo ? b : blo;
    bhi = b > bhi ? b : bhi;
  }
  red_lo[tid] = blo;
  red_hi[tid] = bhi;
  __syncthreads();
  for (int h = SUM_WG / 2; h > 0; h >>= 1) {
    if (tid < h) {
      red_lo[tid] = red_lo[tid + h] < red_lo[tid] ? red_lo[tid + h] : red_lo[tid];
      red_hi[tid] = red_hi[tid + h] > red_hi[tid] ? red_hi[tid + h] : red_hi[tid];
    }
    __syncthreads();
  }
  const int64_t bmin = red_lo[0], bmax = red_hi[0];
  const int nh = int(bmax - bmin) + 8;  // taps of the combined filter
  if (tid == 0) {
    meta[2 * j] = bmin;
    meta[2 * j + 1] = nh <= HMAX ? nh : -1;
  }
  if (nh > HMAX) return;
  // (2) combined filter, copies in batches of SUM_PAIRS, each thread owning taps
  for (int t = tid; t < NQ * HROW; t += SUM_WG) H[t / HROW][t % HROW] = 0.0;
  for (int c0 = 0; c0 < ncopy; c0 += SUM_PAIRS) {
    const int nb = ncopy - c0 < SUM_PAIRS ? ncopy - c0 : SUM_PAIRS;
    if (tid < nb) Wb[tid] = copy_stencil(geo, j, c0 + tid, ncopy, g, s, w, area, Wt[tid]) - bmin;
    __syncthreads();
    for (int k = tid; k < nh; k += SUM_WG) {
      double hx[NQ];
#pragma unroll
      for (int x = 0; x < NQ; ++x) hx[x] = H[x][k];
      for (int p = 0; p < nb; ++p) {
        const int64_t d = int64_t(k) - Wb[p];
        if (d >= 0 && d < 8) {
#pragma unroll
          for (int x = 0; x < NQ; ++x) hx[x] += Wt[p][x * 8 + d];
        }
      }
#pragma unroll
      for (int x = 0; x < NQ; ++x) H[x][k] = hx[x];
    }
    __syncthreads();
  }
  for (int t = tid; t < NQ * HROW; t += SUM_WG) filt[j * NQ * HROW + t] = H[t / HROW][t % HROW];
}

// Thickness and loading integrands of the panels of one chunk at the observer times of
// one time chunk, summed; partial sums per chunk: part[chunk][2][n_out].
__global__ __launch_bounds__(SUM_WG) void k_fwh_sum(const double *__restrict__ src, const double *__restrict__ geo,
                                                    int64_t np, int64_t cap, int ncopy, Geo3 g, Stream s, Window w,
                                                    const double *__restrict__ filt, const int64_t *__restrict__ meta,
                                                    double *__restrict__ part) {
  __shared__ double Wt[SUM_PAIRS][NQ * 8];
  __shared__ int64_t Wb[SUM_PAIRS];
  // one source series at a time; the combined-filter path stores sample e at
  // (e % SUM_OUT) * XQ + e / SUM_OUT, so that the lanes of a wave, SUM_OUT samples apart,
  // read consecutive words; 2 SUM_OUT zero samples past the staged stretch (the filter
  // loop runs whole blocks of SUM_OUT taps)
  constexpr int XQ = SUM_SPAN / SUM_OUT + 4;
  __shared__ double Xs[1][SUM_OUT * XQ];
  __shared__ double H[NQ][HROW];
  __shared__ int64_t lo_s, hi_s;
  const int64_t chunk = blockIdx.y;
  const int tid = threadIdx.x;
  const int64_t mt0 = int64_t(blockIdx.x) * SUM_WG * SUM_OUT;  // first observer time of the chunk
  const int64_t m0 = mt0 + int64_t(tid) * SUM_OUT;
  const int64_t mlast = (mt0 + SUM_WG * SUM_OUT < w.n_out ? mt0 + SUM_WG * SUM_OUT : w.n_out) - 1;
  double accT[SUM_OUT], accL[SUM_OUT];
#pragma unroll
  for (int o = 0; o < SUM_OUT; ++o) accT[o] = accL[o] = 0.0;
  const int64_t j0 = chunk * SUM_PANELS, j1 = j0 + SUM_PANELS < np ? j0 + SUM_PANELS : np;
  for (int64_t j = j0; j < j1; ++j) {
    const double area = geo[j * 7 + 6];
    const int64_t bmin = meta[2 * j];
    const int nh = int(meta[2 * j + 1]);
    if (nh > 0) {
      // the panel's combined filter (the previous panel's last barrier has passed)
      for (int t = tid; t < NQ * HROW; t += SUM_WG) H[t / HROW][t % HROW] = filt[j * NQ * HROW + t];
      // (3) each series over [bmin + mt0, bmax + mlast + 8) in turn, then the filter
      const int64_t lo = bmin + mt0, span = int64_t(nh - 8) + (mlast - mt0) + 8;
      for (int x = 0; x < NQ; ++x) {
        for (int64_t k = tid; k < span + 2 * SUM_OUT; k += SUM_WG)
          Xs[0][int(k % SUM_OUT) * XQ + int(k / SUM_OUT)] = k < span ? src[(x * np + j) * cap + lo + k] : 0.0;
        __syncthreads();
        if (m0 <= mlast) {
          // this thread's samples start at tid * SUM_OUT. Taps go in blocks of SUM_OUT
          // over a window of 2 SUM_OUT samples, w[r] = sample tid * SUM_OUT + SUM_OUT b + r,
          // in tap order for each output (the zero taps past nh add nothing):
          // SUM_OUT^2 multiply-adds per SUM_OUT samples read, the taps read as a broadcast
          const double *X0 = &Xs[0][tid];
          double w[2 * SUM_OUT], acc[SUM_OUT];
#pragma unroll
          for (int r = 0; r < SUM_OUT; ++r) {
            w[r] = X0[r * XQ];
            acc[r] = 0.0;
          }
          const int nblk = (nh + SUM_OUT - 1) / SUM_OUT;
          for (int b = 0; b < nblk; ++b) {
#pragma unroll
            for (int r = 0; r < SUM_OUT; ++r) w[SUM_OUT + r] = X0[r * XQ + b + 1];
#pragma unroll
            for (int kk = 0; kk < SUM_OUT; ++kk) {
              const double hk = H[x][SUM_OUT * b + kk];
#pragma unroll
              for (int o = 0; o < SUM_OUT; ++o) acc[o] += hk * w[o + kk];
            }
#pragma unroll
            for (int r = 0; r < SUM_OUT; ++r) w[r] = w[SUM_OUT + r];
          }
#pragma unroll
          for (int o = 0; o < SUM_OUT; ++o) {
            if (x == 0) accT[o] += acc[o];
            else accL[o] += acc[o];
          }
        }
        __syncthreads();
      }
      continue;
    }
    // copy by copy (delay spread beyond the combined filter)
    for (int c0 = 0; c0 < ncopy; c0 += SUM_PAIRS) {
      const int nb = ncopy - c0 < SUM_PAIRS ? ncopy - c0 : SUM_PAIRS;
      if (tid < nb) Wb[tid] = copy_stencil(geo, j, c0 + tid, ncopy, g, s, w, area, Wt[tid]);
      __syncthreads();
      // stretch of samples the batch touches over this time chunk
      if (tid == 0) {
        int64_t lo = Wb[0], hi = Wb[0];
        for (int p = 1; p < nb; ++p) {
          lo = Wb[p] < lo ? Wb[p] : lo;
          hi = Wb[p] > hi ? Wb[p] : hi;
        }
        lo_s = lo + mt0;
        hi_s = hi + mlast + 8;  // one past the last sample
      }
      __syncthreads();
      const int64_t lo = lo_s, span = hi_s - lo_s;
      // copies whose stretch does not fit are applied straight from global memory
      const bool staged = span <= SUM_SPAN;
      for (int x = 0; x < NQ; ++x) {
        if (staged)
          for (int64_t k = tid; k < span; k += SUM_WG) Xs[0][k] = src[(x * np + j) * cap + lo + k];
        __syncthreads();
        if (m0 < w.n_out) {
          const bool full = m0 + SUM_OUT <= w.n_out;
          for (int p = 0; p < nb; ++p) {
            const int64_t base = Wb[p] + m0;  // sample of tap 0 for observer time m0
            double xs[SUM_OUT + 7];
            const int nvalid = full ? SUM_OUT + 7 : int(w.n_out - m0) + 7;
            if (staged) {
              const double *X = &Xs[0][base - lo];
#pragma unroll
              for (int d = 0; d < SUM_OUT + 7; ++d) xs[d] = d < nvalid ? X[d] : 0.0;
            } else {
              const double *X = src + (x * np + j) * cap + base;
#pragma unroll
              for (int d = 0; d < SUM_OUT + 7; ++d) xs[d] = d < nvalid ? X[d] : 0.0;
            }
#pragma unroll
            for (int o = 0; o < SUM_OUT; ++o) {
              double sv = 0.0;
#pragma unroll
              for (int d = 0; d < 8; ++d) sv += Wt[p][x * 8 + d] * xs[o + d];
              if (x == 0) accT[o] += sv;
              else accL[o] += sv;
            }
          }
        }
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int o = 0; o < SUM_OUT; ++o) {
    const int64_t m = m0 + o;
    if (m >= w.n_out) break;
    part[(chunk * 2 + 0) * w.n_out + m] = accT[o];
    part[(chunk * 2 + 1) * w.n_out + m] = accL[o];
  }
}

// first level of the chunk reduction: group g of RED_GROUPS sums its contiguous range of
// panel chunks, in chunk order, for every observer time: part2[g][2][n_out]
constexpr int RED_GROUPS = 64;
__global__ __launch_bounds__(256) void k_fwh_reduce_groups(const double *__restrict__ part, int64_t nchunk,
                                                           int64_t n_out, double *__restrict__ part2) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (m >= n_out) return;
  const int64_t c0 = g * nchunk / RED_GROUPS, c1 = (g + 1) * nchunk / RED_GROUPS;
  double t = 0.0, l = 0.0;
  for (int64_t c = c0; c < c1; ++c) {
    t += part[(c * 2 + 0) * n_out + m];
    l += part[(c * 2 + 1) * n_out + m];
  }
  part2[(g * 2 + 0) * n_out + m] = t;
  part2[(g * 2 + 1) * n_out + m] = l;
}

// p'_T, p'_L and p' at each observer time: partial sums in chunk order, over 4 pi
__global__ __launch_bounds__(256) void k_fwh_reduce(const double *__restrict__ part, int64_t nchunk, int64_t n_out,
                                                    double *__restrict__ out) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= n_out) return;
  double t = 0.0, l = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) {
    t += part[(c * 2 + 0) * n_out + m];
    l += part[(c * 2 + 1) * n_out + m];
  }
  const double f = 1.0 / (4.0 * M_PI);
  out[m] = (t + l) * f;
  out[n_out + m] = t * f;
  out[2 * n_out + m] = l * f;
}

}  // namespace

struct fr_fwh {
  int device = 0;
  hipStream_t stream = nullptr;
  fr_alloc_fn alloc = nullptr;
  fr_free_fn free = nullptr;
  void *ctx = nullptr;
  int64_t np = 0, cap = 0, nt = 0;
  int ncopy = 1;
  double shift[3] = {0, 0, 0}, dt = 0, tau0 = 0;
  Stream s{};
  double *geo = nullptr, *src = nullptr, *stage = nullptr, *mm = nullptr, *part = nullptr, *part2 = nullptr,
         *out = nullptr, *filt = nullptr, *meta = nullptr;
  size_t stage_bytes = 0, part_bytes = 0, part2_bytes = 0, out_bytes = 0, filt_bytes = 0, meta_bytes = 0;
  std::vector<void *> owned;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;

  void *dalloc(size_t n) {
    void *p = nullptr;
    if (alloc) {
      p = alloc(n, ctx, stream);
      if (!p) fail(FR_E_NOMEM, "device allocation callback failed");
    } else if (hipMalloc(&p, n) != hipSuccess) {
      fail(FR_E_NOMEM, "hipMalloc failed");
    }
    owned.push_back(p);
    return p;
  }
  void dfree(void *p) {
    if (!p) return;
    owned.erase(std::remove(owned.begin(), owned.end(), p), owned.end());
    if (free) free(p, ctx, stream);
    else (void)hipFree(p);
  }
  ~fr_fwh() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void *p : owned) {
      if (free) free(p, ctx, stream);
      else (void)hipFree(p);
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
  // device scratch that grows on demand: partial sums and outputs
  double *grow(double *&p, size_t &have, size_t need) {
    if (need > have) {
      dfree(p);
      p = (double *)dalloc(need);
      have = need;
    }
    return p;
  }
  // enqueue the source strengths of one probed snapshot (device [np][nv] conserved
  // variables) at the end of the record, on the record's stream
  void append_sample(const fr::ProbeRun &r) {
    if (r.n != np) fail(FR_E_ARG, "probe and record have different point counts");
    if (nt + 1 > cap) fail(FR_E_ARG, "record capacity exceeded");
    hip_check(hipSetDevice(device), "hipSetDevice");
    grow(stage, stage_bytes, size_t(np) * 5 * sizeof(double));
    const unsigned blocks = unsigned((np + 255) / 256);
    hipLaunchKernelGGL(k_fwh_cons, dim3(blocks), dim3(256), 0, stream, r.out, np, r.nv, r.dim, r.gamma, s, stage);
    hip_check(hipGetLastError(), "sample kernel");
    hipLaunchKernelGGL(k_fwh_append, dim3(blocks), dim3(256), 0, stream, stage, geo, np, int64_t(1), nt, cap, s, src);
    hip_check(hipGetLastError(), "append kernel");
    nt += 1;
  }
  // observer-time window of the common record (the oracle's rule, same arithmetic)
  Window window(const double *xo) {
    if (nt < 8) fail(FR_E_STATE, "fewer than 8 samples recorded");
    Geo3 g;
    for (int i = 0; i < 3; ++i) {
      g.shift[i] = shift[i];
      g.xo[i] = xo[i];
    }
    constexpr int blocks = 64;
    hipLaunchKernelGGL(k_fwh_delay, dim3(blocks), dim3(256), 0, stream, geo, np, ncopy, g, s, mm);
    hip_check(hipGetLastError(), "delay kernel");
    double h[2 * blocks];
    hip_check(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, stream), "delay copy");
    hip_check(hipStreamSynchronize(stream), "delay sync");
    double dmin = INFINITY, dmax = -INFINITY;
    for (int b = 0; b < blocks; ++b) {
      dmin = std::min(dmin, h[2 * b]);
      dmax = std::max(dmax, h[2 * b + 1]);
    }
    Window w;
    w.dt = dt;
    w.tau0 = tau0;
    w.nt = nt;
    w.t_start = (tau0 + 2 * dt + dmax) + dt;
    const double t_end = (tau0 + double(nt - 3) * dt + dmin) - 2.0 * dt;
    w.t_end = t_end;
    w.n_out = int64_t(std::floor((t_end - w.t_start) / dt + 1e-9)) + 1;
    if (w.n_out <= 0) fail(FR_E_STATE, "record too short for the spread of arrival times");
    if (w.n_out > nt - 7) fail(FR_E_STATE, "observer window longer than the record");
    return w;
  }
};

extern "C" {

fr_status fr_fwh_create(const fr_fwh_desc *d, fr_fwh **out) {
  return guarded([&] {
    if (!out) fail(FR_E_ARG, "null output");
    *out = nullptr;
    if (!d || d->n_points <= 0 || !d->points || !d->normals || !d->areas || d->n_copies < 1 || d->capacity < 8 ||
        !(d->dt > 0.0) || !(d->c0 > 0.0))
      fail(FR_E_ARG, "invalid FW-H descriptor");
    const double m2 = d->mach[0] * d->mach[0] + d->mach[1] * d->mach[1] + d->mach[2] * d->mach[2];
    if (!(m2 < 1.0)) fail(FR_E_ARG, "free-stream Mach number must be below 1");
    hip_check(hipSetDevice(d->device), "hipSetDevice");
    auto *h = new fr_fwh();
    try {
      h->device = d->device;
      h->stream = (hipStream_t)d->stream;
      h->alloc = d->alloc;
      h->free = d->free;
      h->ctx = d->alloc_ctx;
      h->np = d->n_points;
      h->cap = d->capacity;
      h->ncopy = d->n_copies;
      h->dt = d->dt;
      h->tau0 = d->tau0;
      for (int i = 0; i < 3; ++i) {
        h->shift[i] = d->copy_shift[i];
        h->s.mach[i] = d->mach[i];
        h->s.U[i] = d->c0 * d->mach[i];
      }
      h->s.c0 = d->c0;
      h->s.rho0 = d->rho0;
      h->s.p0 = d->p0;
      h->s.g2 = 1.0 / (1.0 - m2);
      std::vector<double> g(size_t(h->np) * 7);
      for (int64_t j = 0; j < h->np; ++j) {
        for (int i = 0; i < 3; ++i) {
          g[j * 7 + i] = d->points[j * 3 + i];
          g[j * 7 + 3 + i] = d->normals[j * 3 + i];
        }
        g[j * 7 + 6] = d->areas[j];
      }
      h->geo = (double *)h->dalloc(g.size() * sizeof(double));
      hip_check(hipMemcpyAsync(h->geo, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice, h->stream),
                "geometry upload");
      h->src = (double *)h->dalloc(size_t(NQ) * h->np * h->cap * sizeof(double));
      h->mm = (double *)h->dalloc(2 * 64 * sizeof(double));
      hip_check(hipEventCreate(&h->ev0), "event");
      hip_check(hipEventCreate(&h->ev1), "event");
      hip_check(hipStreamSynchronize(h->stream), "create sync");
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

void fr_fwh_destroy(fr_fwh *h) { delete h; }

fr_status fr_fwh_append(fr_fwh *h, int64_t n, const double *samples) {
  return guarded([&] {
    if (!h || n < 0 || (n > 0 && !samples)) fail(FR_E_ARG, "bad argument");
    if (h->nt + n > h->cap) fail(FR_E_ARG, "record capacity exceeded");
    if (n == 0) return;
    hip_check(hipSetDevice(h->device), "hipSetDevice");
    const size_t bytes = size_t(n) * h->np * 5 * sizeof(double);
    h->grow(h->stage, h->stage_bytes, bytes);
    hip_check(hipMemcpyAsync(h->stage, samples, bytes, hipMemcpyHostToDevice, h->stream), "sample upload");
    const int64_t thr = n * h->np;
    hipLaunchKernelGGL(k_fwh_append, dim3((thr + 255) / 256), dim3(256), 0, h->stream, h->stage, h->geo, h->np, n,
                       h->nt, h->cap, h->s, h->src);
    hip_check(hipGetLastError(), "append kernel");
    hip_check(hipStreamSynchronize(h->stream), "append sync");
    h->nt += n;
  });
}

fr_status fr_fwh_append_probe(fr_fwh *h, fr_probe *p) {
  return guarded([&] {
    if (!h || !p) fail(FR_E_ARG, "bad argument");
    fr::ProbeRun r{};
    const fr_status st = fr::probe_run(p, true, &r);  // complete on return
    if (st != FR_OK) fail(st, fr_last_error());
    h->append_sample(r);
    hip_check(hipStreamSynchronize(h->stream), "append sync");
  });
}

fr_status fr_fwh_samples(const fr_fwh *h, int64_t *n) {
  return guarded([&] {
    if (!h || !n) fail(FR_E_ARG, "bad argument");
    *n = h->nt;
  });
}

fr_status fr_fwh_window(fr_fwh *h, const double *observer, double *t_start, int64_t *n_out) {
  return guarded([&] {
    if (!h || !observer || !t_start || !n_out) fail(FR_E_ARG, "bad argument");
    hip_check(hipSetDevice(h->device), "hipSetDevice");
    const Window w = h->window(observer);
    *t_start = w.t_start;
    *n_out = w.n_out;
  });
}

}  // extern "C"

// Allocation-free evaluation (fr_fwh_pressure_at_noalloc): the evaluation's
// intermediate arrays live in one static device array per GPU instead of buffers the
// record grows.  In host code `scratch` names a host-side stand-in; its device address
// on the current GPU comes from hipGetSymbolAddress and is the only way host code
// refers to it.
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
// device buffers of one pressure evaluation
struct Scratch {
  double *part, *part2, *out, *filt;
  int64_t *meta;
};

// p' on the grid w (inside the common window) into host p, p_thickness, p_loading, with
// the evaluation's intermediate arrays in sc
void fwh_launch(fr_fwh *h, const double *observer, const Window &w, const Scratch &sc, double *p,
                double *p_thickness, double *p_loading) {
  const int64_t nchunk = (h->np + SUM_PANELS - 1) / SUM_PANELS;
  Geo3 g;
  for (int i = 0; i < 3; ++i) {
    g.shift[i] = h->shift[i];
    g.xo[i] = observer[i];
  }
  const int64_t per_block = int64_t(SUM_WG) * SUM_OUT;
  const dim3 grid(unsigned((w.n_out + per_block - 1) / per_block), unsigned(nchunk));
  hip_check(hipEventRecord(h->ev0, h->stream), "event");
  hipLaunchKernelGGL(k_fwh_filter, dim3(unsigned(h->np)), dim3(SUM_WG), 0, h->stream, h->geo, h->np, h->ncopy, g, h->s,
                     w, sc.filt, sc.meta);
  hip_check(hipGetLastError(), "filter kernel");
  hipLaunchKernelGGL(k_fwh_sum, grid, dim3(SUM_WG), 0, h->stream, h->src, h->geo, h->np, h->cap, h->ncopy, g, h->s, w,
                     sc.filt, static_cast<const int64_t *>(sc.meta), sc.part);
  hip_check(hipGetLastError(), "sum kernel");
  hipLaunchKernelGGL(k_fwh_reduce_groups, dim3(unsigned((w.n_out + 255) / 256), RED_GROUPS), dim3(256), 0, h->stream,
                     sc.part, nchunk, w.n_out, sc.part2);
  hip_check(hipGetLastError(), "reduce kernel");
  hipLaunchKernelGGL(k_fwh_reduce, dim3(unsigned((w.n_out + 255) / 256)), dim3(256), 0, h->stream, sc.part2,
                     int64_t(RED_GROUPS), w.n_out, sc.out);
  hip_check(hipGetLastError(), "reduce kernel");
  hip_check(hipEventRecord(h->ev1, h->stream), "event");
  const size_t nb = size_t(w.n_out) * sizeof(double);
  hip_check(hipMemcpyAsync(p, sc.out, nb, hipMemcpyDeviceToHost, h->stream), "copy p");
  if (p_thickness)
    hip_check(hipMemcpyAsync(p_thickness, sc.out + w.n_out, nb, hipMemcpyDeviceToHost, h->stream), "copy pT");
  if (p_loading)
    hip_check(hipMemcpyAsync(p_loading, sc.out + 2 * w.n_out, nb, hipMemcpyDeviceToHost, h->stream), "copy pL");
  hip_check(hipStreamSynchronize(h->stream), "pressure sync");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, h->ev0, h->ev1), "elapsed");
  h->last_ms = ms;
}

void check_chunks(int64_t np) {
  if ((np + SUM_PANELS - 1) / SUM_PANELS > 65535)
    fail(FR_E_UNSUPPORTED, "too many panels for one launch");  // also bounds the filter grid
}

// the record's own buffers, grown on demand
void fwh_compute(fr_fwh *h, const double *observer, const Window &w, double *p, double *p_thickness,
                 double *p_loading) {
  check_chunks(h->np);
  const int64_t nchunk = (h->np + SUM_PANELS - 1) / SUM_PANELS;
  Scratch sc;
  sc.part = h->grow(h->part, h->part_bytes, size_t(nchunk) * 2 * w.n_out * sizeof(double));
  sc.part2 = h->grow(h->part2, h->part2_bytes, size_t(RED_GROUPS) * 2 * w.n_out * sizeof(double));
  sc.out = h->grow(h->out, h->out_bytes, size_t(3) * w.n_out * sizeof(double));
  sc.filt = h->grow(h->filt, h->filt_bytes, size_t(h->np) * NQ * HROW * sizeof(double));
  sc.meta = reinterpret_cast<int64_t *>(h->grow(h->meta, h->meta_bytes, size_t(h->np) * 2 * sizeof(int64_t)));
  fwh_launch(h, observer, w, sc, p, p_thickness, p_loading);
}

// bytes of each intermediate array of an evaluation of np panels at n_out observer
// times, each rounded up to 256; the total is what the static array must hold
struct NoallocLayout {
  size_t filt, meta, part, part2, out, total;
};
size_t up256(size_t b) { return (b + 255) / 256 * 256; }
NoallocLayout noalloc_layout(int64_t np, int64_t n_out) {
  NoallocLayout L;
  const size_t nchunk = size_t((np + SUM_PANELS - 1) / SUM_PANELS);
  L.filt = up256(size_t(np) * NQ * HROW * sizeof(double));
  L.meta = up256(size_t(np) * 2 * sizeof(int64_t));
  L.part = up256(nchunk * 2 * size_t(n_out) * sizeof(double));
  L.part2 = up256(size_t(RED_GROUPS) * 2 * size_t(n_out) * sizeof(double));
  L.out = up256(size_t(3) * size_t(n_out) * sizeof(double));
  L.total = L.filt + L.meta + L.part + L.part2 + L.out;
  return L;
}

// device address of `scratch` on each GPU, looked up once per device with that device
// current (each GPU holds its own copy of the array)
constexpr int NOALLOC_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[NOALLOC_DEVICES] = {};

unsigned char *scratch_on(int device) {
  if (device < 0 || device >= NOALLOC_DEVICES) fail(FR_E_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static scratch address");
    if (!ptr) fail(FR_E_DEVICE, "static scratch has no device address");
    g_scratch_ptr[device] = static_cast<unsigned char *>(ptr);
  }
  return g_scratch_ptr[device];
}
}  // namespace

extern "C" {

fr_status fr_fwh_pressure(fr_fwh *h, const double *observer, int64_t capacity, double *t_start, int64_t *n_out,
                          double *p, double *p_thickness, double *p_loading) {
  return guarded([&] {
    if (!h || !observer || !t_start || !n_out || !p) fail(FR_E_ARG, "bad argument");
    hip_check(hipSetDevice(h->device), "hipSetDevice");
    const Window w = h->window(observer);
    *t_start = w.t_start;
    *n_out = w.n_out;
    if (capacity < w.n_out) fail(FR_E_ARG, "output capacity below the window length");
    fwh_compute(h, observer, w, p, p_thickness, p_loading);
  });
}

fr_status fr_fwh_pressure_at(fr_fwh *h, const double *observer, double t_start, int64_t n, double *p,
                             double *p_thickness, double *p_loading) {
  return guarded([&] {
    if (!h || !observer || !p || n <= 0) fail(FR_E_ARG, "bad argument");
    hip_check(hipSetDevice(h->device), "hipSetDevice");
    Window w = h->window(observer);
    const double tol = 1e-9 * w.dt;
    if (t_start < w.t_start - tol || t_start + double(n - 1) * w.dt > w.t_end + tol)
      fail(FR_E_ARG, "observer times outside the common window");
    w.t_start = t_start;
    w.n_out = n;
    fwh_compute(h, observer, w, p, p_thickness, p_loading);
  });
}

fr_status fr_fwh_pressure_at_noalloc(fr_fwh *h, const double *observer, double t_start, int64_t n, double *p,
                                     double *p_thickness, double *p_loading) {
  return guarded([&] {
    if (!h || !observer || !p || n <= 0) fail(FR_E_ARG, "bad argument");
    check_chunks(h->np);
    // sizes first: a request beyond the static array launches nothing
    const NoallocLayout L = noalloc_layout(h->np, n);
    if (L.total > NOALLOC_BYTES)
      fail(FR_E_ARG, "panels x observer times need " + std::to_string(L.total) + " bytes of scratch, more than the " +
                         std::to_string(NOALLOC_BYTES) + " of the allocation-free path");
    hip_check(hipSetDevice(h->device), "hipSetDevice");
    unsigned char *base = scratch_on(h->device);
    Window w = h->window(observer);
    const double tol = 1e-9 * w.dt;
    if (t_start < w.t_start - tol || t_start + double(n - 1) * w.dt > w.t_end + tol)
      fail(FR_E_ARG, "observer times outside the common window");
    w.t_start = t_start;
    w.n_out = n;
    // every element of these arrays that a kernel reads is written earlier in the same
    // evaluation, so the previous call's contents need no clearing
    Scratch sc;
    size_t off = 0;
    sc.filt = reinterpret_cast<double *>(base + off);
    off += L.filt;
    sc.meta = reinterpret_cast<int64_t *>(base + off);
    off += L.meta;
    sc.part = reinterpret_cast<double *>(base + off);
    off += L.part;
    sc.part2 = reinterpret_cast<double *>(base + off);
    off += L.part2;
    sc.out = reinterpret_cast<double *>(base + off);
    fwh_launch(h, observer, w, sc, p, p_thickness, p_loading);
  });
}

fr_status fr_fwh_time_ms(const fr_fwh *h, double *ms) {
  return guarded([&] {
    if (!h || !ms) fail(FR_E_ARG, "bad argument");
    *ms = h->last_ms;
  });
}

}  // extern "C"

fr_status fr::fwh_append_probe_async(::fr_fwh *h, ::fr_probe *p) {
  return guarded([&] {
    if (!h || !p) fail(FR_E_ARG, "bad argument");
    fr::ProbeRun r{};
    const fr_status st = fr::probe_run(p, false, &r);
    if (st != FR_OK) fail(st, fr_last_error());
    if (r.stream != h->stream) fail(FR_E_ARG, "record and probe mesh run on different streams");
    h->append_sample(r);
  });
}

size_t fr::fwh_footprint(int64_t n_points, int64_t capacity) {
  const size_t np = size_t(n_points), cap = size_t(capacity);
  const size_t nchunk = (np + SUM_PANELS - 1) / SUM_PANELS;
  // geometry, source series, one staged snapshot, delay extremes, the panels' combined
  // filters and their first samples, and at most a window of capacity observer times of
  // partial sums and outputs
  return (np * 7 + size_t(NQ) * np * cap + np * 5 + 2 * 64 + np * (size_t(NQ) * HROW + 2) + nchunk * 2 * cap +
          size_t(RED_GROUPS) * 2 * cap + 3 * cap) * sizeof(double);
}
