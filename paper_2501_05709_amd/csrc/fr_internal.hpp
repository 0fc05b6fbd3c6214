// Internal interface between the host library (fr_host.cpp) and the gfx950
// kernels (fr_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/fr.h"

struct fr_probe;
struct fr_mesh;
struct fr_fwh;

namespace fr {

constexpr int EB = 16;  // elements per block: the N extent of one MFMA tile
constexpr int SB = 4;   // elements per sub-block: contiguous run of one point and channel
constexpr int NSB = EB / SB;

// Index of (point pt, channel ch) of element slot e in block blk of a per-element
// array with NPT points and NCH channels.  Layout [block][sub-block][point][channel][SB]:
// the SB elements of a sub-block are contiguous for each point and channel, and the
// whole sub-block is one contiguous run, so a workgroup that owns a sub-block reads
// and writes it in full segments.
__host__ __device__ inline size_t lay(int64_t blk, int pt, int ch, int e, int NPT, int NCH) {
  return ((size_t(blk * NSB + e / SB) * NPT + pt) * NCH + ch) * SB + size_t(e % SB);
}

// Packed boundary code stored in the neighbour table: -(kind | index << 2),
// index = position of a wall flux point in the compact wall list.
constexpr int BC_WALL = 1;
constexpr int BC_FARFIELD = 2;
// A flux point on a face shared with an element of another order: index =
// (mortar point << 1) | side, side 1 on the lower-order element.  Its partner data
// are formed in the fused kernels from the mortar tables (DevArrays::MO, MG, MC, MW).
constexpr int BC_MORTAR = 3;

enum Kernel {
  K_FACE = 1,    // common solution and Rusanov flux at every flux point
  K_GRAD = 2,    // corrected gradient, physical gradient, transformed flux
  K_VISC = 3,    // gradient trace, viscous normal flux (and wall force terms)
  K_DIVRK = 4,   // corrected divergence, residual, fused RK4 stage update
  K_INTERP = 5,  // solution trace at flux points
  K_STAGE_A = 6, // fused: faces, gradient, fluxes, viscous half-flux, volume divergence
  K_STAGE_B = 7, // fused: flux correction, RK4 stage update, next trace
};

// Variant-mask bit of the fused stage on 3D one-order meshes: read the stored FP64
// metrics instead of forming them from the geometry nodes
constexpr unsigned STORED_METRICS = 1u << 6;
// Launch shape of the fused stage: no remap of consecutive tiles onto one XCD
constexpr unsigned NO_XCD_REMAP = 1u << 7;
// Fused stage on a mesh of z-extruded elements: metrics from the column data (XC, ZZ, FCX)
constexpr unsigned EXTRUDED_METRICS = 1u << 8;
// Tile shape of the fused stage's first launch (bits 9-10) and second launch (bits 11-12):
// 0 the default workgroup, 1 half its elements, 2 a quarter (at least one); for the first
// launch also 3, the default workgroup with the reference gradient and the volume
// divergence on the matrix cores (FP32 at order 3; elsewhere it runs the default).
// Compiled for 3D one-order meshes of order 1 up; other meshes run the default.
constexpr int TILE_A_SHIFT = 9, TILE_B_SHIFT = 11;
constexpr unsigned TILE_BITS = (3u << TILE_A_SHIFT) | (3u << TILE_B_SHIFT);
constexpr int N_TILES = 3, N_TILES_A = 4;
// Neighbour exchange of the fused stage by scatter: each trace and viscous half flux is
// written into the partner's slot and read from the own slot (one-order meshes; mortar
// faces keep the gather through the neighbour codes)
constexpr unsigned SCATTER_EXCHANGE = 1u << 13;
inline int tile_a(unsigned mask) { return int((mask >> TILE_A_SHIFT) & 3u); }
inline int tile_b(unsigned mask) { return int((mask >> TILE_B_SHIFT) & 3u); }
inline unsigned tile_bits(int ta, int tb) { return (unsigned(ta) << TILE_A_SHIFT) | (unsigned(tb) << TILE_B_SHIFT); }
inline bool tiles_compiled(int dim, int order, bool mixed) { return dim == 3 && order >= 1 && !mixed; }
// Face-point map of a per-face neighbour code (host and device): point m of a face with n
// points per line goes to the partner face's point face_map(m); in 3D m = a + n b, the map
// bits are 4 swap (a, b), 1 reverse a, 2 reverse b; on the lines of 2D faces only bit 1.
__host__ __device__ inline int face_map(int m, int map, int n, int dim) {
  if (dim == 2) return (map & 1) ? n - 1 - m : m;
  int a = m % n, b = m / n;
  if (map & 4) {
    const int t = a;
    a = b;
    b = t;
  }
  if (map & 1) a = n - 1 - a;
  if (map & 2) b = n - 1 - b;
  return a + n * b;
}
// Per-point neighbour code (NB's form) of point m of a face from the face's per-face code
// (NBF's form); n points per line, nfp per face, nfpad per element in the NB layout.
__host__ __device__ inline int point_code(int fc, int m, int n, int nfp, int nfpad, int dim) {
  if (fc < 0) {
    const int kind = (-fc) & 3;
    return kind == BC_WALL ? -(kind | ((((-fc) >> 2) + m) << 2)) : fc;
  }
  const int ps = fc >> 6, pf = (fc >> 3) & 7;
  return int(lay(ps / EB, pf * nfp + face_map(m, fc & 7, n, dim), 0, ps % EB, nfpad, 1));
}

// Modes of K_DIVRK
enum { MODE_RK0 = 0, MODE_RK1 = 1, MODE_RK2 = 2, MODE_RK3 = 3, MODE_RESID = 4 };

struct DevArrays {
  // state and stage arrays, element type = real of the form (float or double)
  void *U = nullptr, *US = nullptr, *ACC = nullptr, *UF = nullptr, *DU = nullptr, *FI = nullptr;
  void *GU = nullptr, *FT = nullptr, *PV = nullptr, *RES = nullptr;
  // operators (real), swizzled into MFMA A-operand order
  void *opInt = nullptr, *opGrad = nullptr, *opGcorr = nullptr, *opDivS = nullptr, *opCorr = nullptr;
  // 1D basis (real): D[n][n], l(-1)[n], l(+1)[n], g_L'[n], g_R'[n]
  void *basis = nullptr;
  // FP64 geometry, all in the sub-blocked layout of lay()
  double *SM = nullptr;  // NUP points, dim*dim channels: S = |J| J^-1
  double *IJ = nullptr;  // NUP points, 1 channel: 1/|J|
  double *FN = nullptr;  // NFPAD points, dim channels: outward unit normal
  double *FA = nullptr;  // NFPAD points, 1 channel: |S^T n_hat|
  int *NB = nullptr;     // NFPAD points, 1 channel: partner lay(blk, q, 0, slot, NFPAD, 1), or boundary code
  // the same per face (2 dim faces, 1 channel), for one-order meshes whose matched faces
  // all map their points by one of the 8 symmetries of the square (null otherwise): an
  // interior face holds ((partner block * EB + slot) << 6) | (partner face << 3) | map, a
  // boundary face the per-point code of its first point (wall points number on from it)
  int *NBF = nullptr;
  // 3D: the element map as 27 triquadratic nodes (lay: 27 points, 3 channels), from which
  // the fused stage forms its metrics, and the quadratic basis and its derivative at the
  // Gauss-Legendre points, GQ[(kind * 3 + a) * n + i] (kind 0: l_a, 1: l_a')
  double *XN = nullptr;
  double *GQ = nullptr;
  // 3D meshes whose elements are all z-extruded: per element the 2D Jacobian columns
  // (x_xi, x_eta, y_xi, y_eta) at the n^2 solution-point columns (lay: n^2 points, 4
  // channels), z_zeta at the n solution-point layers (n points, 1 channel), and per face
  // column (4n + n^2 points, 2 channels): (x_eta, y_eta) on the xi faces (side s, eta
  // point m: s n + m), (x_xi, y_xi) on the eta faces (2n + s n + m), the 2D Jacobian
  // determinant of the zeta faces' columns (4n + column)
  double *XC = nullptr, *ZZ = nullptr, *FCX = nullptr;
  // extruded meshes: 1/|J| = IJC[column] IZ[layer], the reciprocal 2D Jacobian determinant
  // of the n^2 solution-point columns and the reciprocal z_zeta of the n layers
  double *IJC = nullptr, *IZ = nullptr;
  int *bcount = nullptr;   // [blk] valid elements in the block
  int *bdesign = nullptr;  // [blk]
  int64_t *bcanon = nullptr;  // [blk] canonical element index of slot 0
  double *bdt = nullptr;   // [blk]
  double *fsd = nullptr;   // [design][5] free stream
  double *wface = nullptr; // [NFPAD] face quadrature weight per flux point
  double *FC = nullptr;    // [n_wall][3] wall force contributions
  int64_t *wall_first = nullptr;  // [design + 1] compact wall ranges
  double *fsum = nullptr;  // [design][8]: sum Fx,Fy,Fz, count, last Fx,Fy,Fz, spare
  int *flag = nullptr;     // non-finite flag
  double *stage64 = nullptr;  // canonical FP64 staging [E][nu][nv]
  // mortar data of a variable-order mesh, shared by its order groups. Per mortar point s
  // (a flux point on a face shared with an element of another order), entries
  // [MO[s], MO[s + 1]) read partner code MC[] of order group MG[] with weight MW[]: the
  // other side's face points interpolated to s (higher-order side) or projected onto
  // it (lower-order side). The first launch applies them to the groups' traces GUF[g]
  // (the other side's trace at s), the second launch of a higher-order side to their
  // half viscous fluxes GPV[g]. MT, [mortar point][nv] (real): the transformed common
  // flux of a higher-order side, projected onto the lower-order points by entries
  // [PO[s], PO[s + 1]) (MT points PC[], weights PW[]; empty for higher-order points).
  const int *MO = nullptr, *MG = nullptr, *MC = nullptr;
  const double *MW = nullptr;
  const void *const *GUF = nullptr, *const *GPV = nullptr;  // device arrays of group pointers
  void *MT = nullptr;
  const int *PO = nullptr, *PC = nullptr;
  const double *PW = nullptr;
};

struct LaunchCfg {
  int prec = 0, dim = 3, order = 3;
  int64_t nblk = 0;
  int ndesign = 1;
  int64_t n_canon = 0;  // canonical elements
  double gamma = 1.4, mu = 0.0, prandtl = 0.72;
  hipStream_t stream = nullptr;
  // bit k set: kernel k (enum Kernel) runs its sum-factorised variant, else dense MFMA
  unsigned variant_mask = 0;
};

// Shape constants for a (dim, order) pair
struct Dims {
  int n, nu, nfp, nf, nv, nup, nfpad, ku, kf;
  Dims(int dim, int order) {
    n = order + 1;
    nu = dim == 2 ? n * n : n * n * n;
    nfp = dim == 2 ? n : n * n;
    nf = 2 * dim * nfp;
    nv = dim + 2;
    nup = (nu + 15) / 16 * 16;
    nfpad = (nf + 15) / 16 * 16;
    ku = (nu + 3) / 4 * 4;
    kf = (nf + 3) / 4 * 4;
  }
};

// Launchers (fr_kernels.hip).  Return hipSuccess or the launch error.
bool kernels_available(int prec, int dim, int order);
hipError_t launch_kernel(int kernel, const LaunchCfg &c, const DevArrays &a, int stage, int mode,
                         bool forces);
hipError_t launch_pack(const LaunchCfg &c, const DevArrays &a, bool to_device_layout, void *dst_res);
hipError_t launch_force_reduce(const LaunchCfg &c, const DevArrays &a);
hipError_t launch_clear_flag(const LaunchCfg &c, const DevArrays &a);

// dst (may be null): output row of each point, else the point's own index
hipError_t launch_probe(const LaunchCfg &c, const DevArrays &a, int64_t n, const int64_t *slot, const double *w,
                        const int64_t *dst, double *out);

// Message returned by fr_last_error() for the calling thread (fr_host.cpp).
void set_last_error(const char *msg);

// Sample the state of a probe's mesh at its points into a device buffer [n][nv] (FP64
// conserved variables) on the mesh's stream; complete on return when wait is set.  Also
// reports the mesh's dim and gamma.  Errors come back as a status with the message set
// for fr_last_error(), never as an exception (fr_host.cpp).
struct ProbeRun {
  const double *out;
  int64_t n;
  int nv, dim;
  double gamma;
  hipStream_t stream;
};
fr_status probe_run(::fr_probe *p, bool wait, ProbeRun *out);

// Enqueue n RK4 steps of m on its stream without waiting.  clear_flag false keeps the
// non-finite flag raised by steps enqueued before, so one later fr_sync covers them all.
fr_status step_enqueue(::fr_mesh *m, int64_t n, bool clear_flag);

// Enqueue the reset of the running lift and drag means of every design of m.
fr_status means_clear(::fr_mesh *m);

// Enqueue one snapshot of probe p and its append to record h (fr_fwh.hip), without
// waiting.  The record must run on the probe mesh's stream.
fr_status fwh_append_probe_async(::fr_fwh *h, ::fr_probe *p);

// Upper bounds of the device bytes held by a probe of n points and by an FW-H record
// of n_points panels and capacity samples, including what its pressure calls grow.
size_t probe_footprint(int64_t n, int dim, int order);

// Whether every element of a 3D mesh is z-extruded (x and y the same in every node layer,
// z the same across each layer): such meshes also carry column metrics (DevArrays::XC..)
bool desc_extruded(const fr_mesh_desc &d);
size_t fwh_footprint(int64_t n_points, int64_t capacity);

}  // namespace fr
