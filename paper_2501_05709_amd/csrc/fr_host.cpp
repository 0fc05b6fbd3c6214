// Host side of the FR library: basis and operator construction, mesh
// connectivity, FP64 geometry, block packing, HIP graphs and the C ABI of
// include/fr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fr.h"
#include "fr_internal.hpp"

using namespace fr;

namespace {

thread_local std::string g_err;

struct FrError {
  fr_status code;
  std::string msg;
};

[[noreturn]] void fail(fr_status c, const std::string &m) { throw FrError{c, m}; }

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(FR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// static-partition parallel loop over [0, n) on the host's hardware threads
template <class F> void parallel_for(int64_t n, F &&f) {
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(std::thread::hardware_concurrency(), (n + 1023) / 1024));
  if (nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  for (int64_t t = 0; t < nt; ++t)
    pool.emplace_back([&, t] {
      const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
      for (int64_t i = lo; i < hi; ++i) f(i);
    });
  for (auto &th : pool) th.join();
}

template <class F> fr_status guarded(F &&f) {
  try {
    f();
    return FR_OK;
  } catch (const FrError &e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return FR_E_NOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return FR_E_ARG;
  }
}

// ---------------------------------------------------------------------------
// 1D basis: Gauss-Legendre points, barycentric Lagrange algebra, Radau g'
// ---------------------------------------------------------------------------
struct Basis1D {
  int n;
  std::vector<double> x, w, bw;   // nodes, weights, barycentric weights
  std::vector<double> D;          // D[i*n+j] = l_j'(x_i)
  std::vector<double> lm, lp;     // l_j(-1), l_j(+1)
  std::vector<double> gLd, gRd;   // g_L'(x_i), g_R'(x_i)

  static void legendre_pair(int k, double t, double &P, double &Pm1) {
    // P_k(t) and P_{k-1}(t) by Bonnet's recursion
    double a = 1.0, b = t;
    if (k == 0) { P = 1.0; Pm1 = 0.0; return; }
    for (int m = 1; m < k; ++m) {
      const double c = ((2 * m + 1) * t * b - m * a) / (m + 1);
      a = b;
      b = c;
    }
    P = b;
    Pm1 = a;
  }
  // derivative of P_k from (t^2 - 1) P_k' = k (t P_k - P_{k-1}); interior t only
  static double legendre_d(int k, double t) {
    if (k == 0) return 0.0;
    double P, Pm1;
    legendre_pair(k, t, P, Pm1);
    return k * (t * P - Pm1) / (t * t - 1.0);
  }

  explicit Basis1D(int order) : n(order + 1) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
      // Newton on P_n from the Chebyshev-Gauss guess, ascending order
      double t = -std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
      for (int it = 0; it < 60; ++it) {
        double P, Pm1;
        legendre_pair(n, t, P, Pm1);
        const double dP = n * (t * P - Pm1) / (t * t - 1.0);
        const double step = P / dP;
        t -= step;
        if (std::fabs(step) < 4e-17) break;
      }
      x[i] = t;
      const double dP = legendre_d(n, t);
      w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
    bw.assign(n, 1.0);
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k)
        if (k != j) bw[j] /= (x[j] - x[k]);
    D.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) {
      double diag = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        D[i * n + j] = (bw[j] / bw[i]) / (x[i] - x[j]);
        diag -= D[i * n + j];
      }
      D[i * n + i] = diag;
    }
    lm = eval_all(-1.0);
    lp = eval_all(1.0);
    gRd.resize(n);
    gLd.resize(n);
    for (int i = 0; i < n; ++i) {
      gRd[i] = 0.5 * (legendre_d(order, x[i]) + legendre_d(order + 1, x[i]));
      gLd[i] = -0.5 * (legendre_d(order, -x[i]) + legendre_d(order + 1, -x[i]));
    }
  }
  // l_j(t) for all j, barycentric form of the second kind
  std::vector<double> eval_all(double t) const {
    std::vector<double> out(n, 0.0);
    for (int j = 0; j < n; ++j)
      if (t == x[j]) { out[j] = 1.0; return out; }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += bw[j] / (t - x[j]);
    for (int j = 0; j < n; ++j) out[j] = bw[j] / (t - x[j]) / den;
    return out;
  }
};

// ---------------------------------------------------------------------------
// reference-element index maps (conventions of include/fr.h)
// ---------------------------------------------------------------------------
struct RefElem {
  int dim, n, nu, nfp, nf;
  RefElem(int d, int order) : dim(d), n(order + 1) {
    nu = d == 2 ? n * n : n * n * n;
    nfp = d == 2 ? n : n * n;
    nf = 2 * d * nfp;
  }
  // the two axes spanning face axis k, lower first
  std::array<int, 2> face_axes(int k) const {
    if (dim == 2) return {1 - k, -1};
    if (k == 0) return {1, 2};
    if (k == 1) return {0, 2};
    return {0, 1};
  }
  std::array<int, 3> upt_idx(int i) const { return {i % n, (i / n) % n, dim == 3 ? i / (n * n) : 0}; }
  int upt(const std::array<int, 3> &c) const { return c[0] + n * c[1] + (dim == 3 ? n * n * c[2] : 0); }
  // solution point on the line through face point m of a face on axis k, at position j
  int line_point(int k, int m, int j) const {
    std::array<int, 3> c{0, 0, 0};
    auto ax = face_axes(k);
    c[k] = j;
    c[ax[0]] = m % n;
    if (dim == 3) c[ax[1]] = m / n;
    return upt(c);
  }
  int face_index(int i, int k) const {  // face point m of solution point i for axis k
    auto c = upt_idx(i);
    auto ax = face_axes(k);
    return dim == 2 ? c[ax[0]] : c[ax[0]] + n * c[ax[1]];
  }
  std::array<double, 3> fpt_ref(const Basis1D &b, int f, int m) const {
    const int k = f / 2;
    std::array<double, 3> r{0, 0, 0};
    r[k] = (f & 1) ? 1.0 : -1.0;
    auto ax = face_axes(k);
    r[ax[0]] = b.x[m % n];
    if (dim == 3) r[ax[1]] = b.x[m / n];
    return r;
  }
};

// ---------------------------------------------------------------------------
// dense operators
// ---------------------------------------------------------------------------
struct Operators {
  Dims dm;
  std::vector<double> Mint, Mgrad, Mgcorr, MdivS, Mcorr;  // row-major
  int nu, nf, dim;
  Operators(int d, int order) : dm(d, order) {
    Basis1D b(order);
    RefElem R(d, order);
    nu = R.nu;
    nf = R.nf;
    dim = d;
    const int n = R.n, nfp = R.nfp;
    Mint.assign(size_t(nf) * nu, 0.0);
    Mgrad.assign(size_t(d) * nu * nu, 0.0);
    Mgcorr.assign(size_t(d) * nu * nf, 0.0);
    std::vector<double> Mdiv(size_t(nu) * d * nu, 0.0), Mnint(size_t(nf) * d * nu, 0.0);
    Mcorr.assign(size_t(nu) * nf, 0.0);
    for (int f = 0; f < 2 * d; ++f) {
      const int k = f / 2;
      const double sg = (f & 1) ? 1.0 : -1.0;
      const auto &l = (f & 1) ? b.lp : b.lm;
      for (int m = 0; m < nfp; ++m) {
        const int q = f * nfp + m;
        for (int j = 0; j < n; ++j) {
          const int i = R.line_point(k, m, j);
          Mint[size_t(q) * nu + i] = l[j];
          Mnint[size_t(q) * d * nu + k * nu + i] = sg * l[j];
        }
      }
    }
    for (int i = 0; i < nu; ++i) {
      const auto c = R.upt_idx(i);
      for (int k = 0; k < d; ++k) {
        const int m = R.face_index(i, k), ik = c[k];
        for (int j = 0; j < n; ++j) {
          const int jj = R.line_point(k, m, j);
          Mgrad[(size_t(k) * nu + i) * nu + jj] += b.D[ik * n + j];
          Mdiv[size_t(i) * d * nu + k * nu + jj] += b.D[ik * n + j];
        }
        const int qp = (2 * k + 1) * nfp + m, qm = 2 * k * nfp + m;
        Mgcorr[(size_t(k) * nu + i) * nf + qp] = b.gRd[ik];
        Mgcorr[(size_t(k) * nu + i) * nf + qm] = b.gLd[ik];
        Mcorr[size_t(i) * nf + qp] = b.gRd[ik];
        Mcorr[size_t(i) * nf + qm] = -b.gLd[ik];
      }
    }
    // strong-form divergence: the interpolated normal flux correction folded in
    MdivS = Mdiv;
    for (int i = 0; i < nu; ++i)
      for (int q = 0; q < nf; ++q) {
        const double c = Mcorr[size_t(i) * nf + q];
        if (c == 0.0) continue;
        for (int col = 0; col < d * nu; ++col) MdivS[size_t(i) * d * nu + col] -= c * Mnint[size_t(q) * d * nu + col];
      }
  }
};

// MFMA A-operand order: tile (rt, kt), lane l -> M[rt*16 + l%16][kt*4 + l/16]
template <class Get>
void swizzle(std::vector<double> &out, int rtiles, int ktiles, Get get) {
  for (int rt = 0; rt < rtiles; ++rt)
    for (int kt = 0; kt < ktiles; ++kt)
      for (int l = 0; l < 64; ++l) out.push_back(get(rt * 16 + l % 16, kt * 4 + l / 16));
}

// ---------------------------------------------------------------------------
// per-design host geometry and connectivity
// ---------------------------------------------------------------------------
struct HostMesh {
  int dim, order, q;
  int64_t E;
  std::vector<double> S, detJ, xu;      // [E][nu][dim*dim], [E][nu], [E][nu][3]
  std::vector<double> fn, fA, fx;       // [E][nf][dim], [E][nf], [E][nf][3]
  std::vector<int64_t> nbr;             // [E][nf]: e'*nf + q' or -kind
};

void shape_q(int q, double t, double *N, double *dN) {
  if (q == 1) {
    N[0] = 0.5 * (1.0 - t); N[1] = 0.5 * (1.0 + t);
    dN[0] = -0.5; dN[1] = 0.5;
  } else {
    N[0] = 0.5 * t * (t - 1.0); N[1] = 1.0 - t * t; N[2] = 0.5 * t * (t + 1.0);
    dN[0] = t - 0.5; dN[1] = -2.0 * t; dN[2] = t + 0.5;
  }
}

// x(r) and the columns a_k = dx/dr_k
void geom_map(const fr_mesh_desc &d, int64_t e, const std::array<double, 3> &r, double x[3], double a[3][3]) {
  const int dim = d.dim, q = d.geom_order, na = q + 1;
  double N[3][3], dN[3][3];
  for (int k = 0; k < dim; ++k) shape_q(q, r[k], N[k], dN[k]);
  for (int i = 0; i < 3; ++i) {
    x[i] = 0.0;
    for (int k = 0; k < 3; ++k) a[k][i] = 0.0;
  }
  const int nn = dim == 2 ? na * na : na * na * na;
  const int64_t *en = d.elem_nodes + e * nn;
  for (int c2 = 0; c2 < (dim == 3 ? na : 1); ++c2)
    for (int c1 = 0; c1 < na; ++c1)
      for (int c0 = 0; c0 < na; ++c0) {
        const int aidx = c0 + na * c1 + na * na * c2;
        const double *X = d.nodes + en[aidx] * dim;
        const int cc[3] = {c0, c1, c2};
        double val = 1.0;
        for (int k = 0; k < dim; ++k) val *= N[k][cc[k]];
        for (int i = 0; i < dim; ++i) x[i] += val * X[i];
        for (int k = 0; k < dim; ++k) {
          double dv = 1.0;
          for (int kk = 0; kk < dim; ++kk) dv *= (kk == k) ? dN[kk][cc[kk]] : N[kk][cc[kk]];
          for (int i = 0; i < dim; ++i) a[k][i] += dv * X[i];
        }
      }
}

// S rows: S_k = a_{k+1} x a_{k+2} (3D) so that S = |J| J^-1; returns |J|
double metric_rows(int dim, double a[3][3], double S[3][3]) {
  if (dim == 2) {
    S[0][0] = a[1][1]; S[0][1] = -a[1][0];
    S[1][0] = -a[0][1]; S[1][1] = a[0][0];
    return a[0][0] * a[1][1] - a[0][1] * a[1][0];
  }
  for (int k = 0; k < 3; ++k) {
    const double *u = a[(k + 1) % 3], *v = a[(k + 2) % 3];
    S[k][0] = u[1] * v[2] - u[2] * v[1];
    S[k][1] = u[2] * v[0] - u[0] * v[2];
    S[k][2] = u[0] * v[1] - u[1] * v[0];
  }
  return a[0][0] * S[0][0] + a[0][1] * S[0][1] + a[0][2] * S[0][2];
}

// A z-extruded element: x and y the same in every node layer and z a function of
// zeta alone (equal across each layer), so J = [[x_xi, x_eta, 0], [y_xi, y_eta, 0],
// [0, 0, z_zeta]] with the 2D part independent of zeta and z_zeta of zeta alone.
bool elem_extruded(const fr_mesh_desc &d, int64_t e) {
  if (d.dim != 3) return false;
  const int na = d.geom_order + 1;
  const int64_t *en = d.elem_nodes + e * na * na * na;
  for (int a2 = 0; a2 < na; ++a2)
    for (int a1 = 0; a1 < na; ++a1)
      for (int a0 = 0; a0 < na; ++a0) {
        const double *X = d.nodes + en[a0 + na * a1 + na * na * a2] * 3;
        const double *X0 = d.nodes + en[a0 + na * a1] * 3;
        const double *Z = d.nodes + en[na * na * a2] * 3;
        if (X[0] != X0[0] || X[1] != X0[1] || X[2] != Z[2]) return false;
      }
  return true;
}

// Column metrics of an extruded element at the order's Gauss-Legendre points x[]: the 2D
// Jacobian (x_xi, x_eta, y_xi, y_eta) at (x[i0], x[i1]), from the node layer a2 = 0, and
// z_zeta at x[i2], from the nodes of column (0, 0)
void extruded_jacobian(const fr_mesh_desc &d, int64_t e, double xi, double eta, double jac[4]) {
  const int q = d.geom_order, na = q + 1;
  const int64_t *en = d.elem_nodes + e * na * na * na;
  double N0[3], dN0[3], N1[3], dN1[3];
  shape_q(q, xi, N0, dN0);
  shape_q(q, eta, N1, dN1);
  for (int c = 0; c < 4; ++c) jac[c] = 0.0;
  for (int a1 = 0; a1 < na; ++a1)
    for (int a0 = 0; a0 < na; ++a0) {
      const double *X = d.nodes + en[a0 + na * a1] * 3;
      const double w0 = dN0[a0] * N1[a1], w1 = N0[a0] * dN1[a1];
      jac[0] += w0 * X[0];
      jac[1] += w1 * X[0];
      jac[2] += w0 * X[1];
      jac[3] += w1 * X[1];
    }
}
double extruded_zzeta(const fr_mesh_desc &d, int64_t e, double zeta) {
  const int q = d.geom_order, na = q + 1;
  const int64_t *en = d.elem_nodes + e * na * na * na;
  double N[3], dN[3];
  shape_q(q, zeta, N, dN);
  double z = 0.0;
  for (int a2 = 0; a2 < na; ++a2) z += dN[a2] * d.nodes[en[na * na * a2] * 3 + 2];
  return z;
}

struct KeyHash {
  size_t operator()(const std::array<int64_t, 4> &k) const {
    size_t h = 1469598103934665603ull;
    for (auto v : k) h = (h ^ size_t(v)) * 1099511628211ull;
    return h;
  }
};

// boundary-list kind of a face shared with an element of another order, as the
// order groups of a variable-order mesh list them (never in a caller's descriptor)
constexpr int64_t KIND_MORTAR = BC_MORTAR;

HostMesh build_host_mesh(const fr_mesh_desc &d, bool allow_mortar = false) {
  const int dim = d.dim, order = d.order, q = d.geom_order;
  RefElem R(dim, order);
  Basis1D b(order);
  HostMesh H;
  H.dim = dim; H.order = order; H.q = q; H.E = d.n_elems;
  const int64_t E = d.n_elems;
  const int nu = R.nu, nf = R.nf, nfp = R.nfp, na = q + 1;
  const int nn = dim == 2 ? na * na : na * na * na;
  for (int64_t i = 0; i < E * nn; ++i)
    if (d.elem_nodes[i] < 0 || d.elem_nodes[i] >= d.n_nodes) fail(FR_E_ARG, "element node id out of range");
  H.S.resize(size_t(E) * nu * dim * dim);
  H.detJ.resize(size_t(E) * nu);
  H.xu.assign(size_t(E) * nu * 3, 0.0);
  H.fn.resize(size_t(E) * nf * dim);
  H.fA.resize(size_t(E) * nf);
  H.fx.assign(size_t(E) * nf * 3, 0.0);
  std::vector<char> bad_e(size_t(E), 0);
  parallel_for(E, [&](int64_t e) {
    bool &bad = reinterpret_cast<bool &>(bad_e[size_t(e)]);
    for (int i = 0; i < nu; ++i) {
      auto c = R.upt_idx(i);
      std::array<double, 3> r{b.x[c[0]], b.x[c[1]], dim == 3 ? b.x[c[2]] : 0.0};
      double x[3], a[3][3], S[3][3];
      geom_map(d, e, r, x, a);
      const double det = metric_rows(dim, a, S);
      if (!(det > 0.0)) bad = true;
      H.detJ[e * nu + i] = det;
      for (int k = 0; k < dim; ++k)
        for (int j = 0; j < dim; ++j) H.S[(size_t(e) * nu + i) * dim * dim + k * dim + j] = S[k][j];
      for (int j = 0; j < dim; ++j) H.xu[(size_t(e) * nu + i) * 3 + j] = x[j];
    }
    for (int f = 0; f < 2 * dim; ++f)
      for (int m = 0; m < nfp; ++m) {
        const int qq = f * nfp + m, k = f / 2;
        auto r = R.fpt_ref(b, f, m);
        double x[3], a[3][3], S[3][3];
        geom_map(d, e, r, x, a);
        const double det = metric_rows(dim, a, S);
        if (!(det > 0.0)) bad = true;
        double nrm = 0.0;
        for (int j = 0; j < dim; ++j) nrm += S[k][j] * S[k][j];
        nrm = std::sqrt(nrm);
        const double sg = (f & 1) ? 1.0 : -1.0;
        H.fA[size_t(e) * nf + qq] = nrm;
        for (int j = 0; j < dim; ++j) {
          H.fn[(size_t(e) * nf + qq) * dim + j] = sg * S[k][j] / nrm;
          H.fx[(size_t(e) * nf + qq) * 3 + j] = x[j];
        }
      }
  });
  for (char b : bad_e)
    if (b) fail(FR_E_MESH, "non-positive Jacobian");

  // ---- connectivity: faces by corner node ids, then by periodic translation
  const int nfe = 2 * dim, nc = dim == 2 ? 2 : 4;
  auto corner_local = [&](int f, int c) {
    const int k = f / 2;
    std::array<int, 3> a{0, 0, 0};
    a[k] = (f & 1) * q;
    auto ax = R.face_axes(k);
    a[ax[0]] = (c & 1) * q;
    if (dim == 3) a[ax[1]] = ((c >> 1) & 1) * q;
    return a[0] + na * a[1] + na * na * a[2];
  };
  H.nbr.assign(size_t(E) * nf, INT64_MIN);
  std::vector<char> done(size_t(E) * nfe, 0);
  struct Pair { int64_t a, b; double shift[3]; };
  std::vector<Pair> pairs;
  {
    std::unordered_map<std::array<int64_t, 4>, int64_t, KeyHash> seen;
    seen.reserve(size_t(E) * nfe);
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < nfe; ++f) {
        std::array<int64_t, 4> key{-1, -1, -1, -1};
        for (int c = 0; c < nc; ++c) key[c] = d.elem_nodes[e * nn + corner_local(f, c)];
        std::sort(key.begin(), key.begin() + nc);
        auto it = seen.find(key);
        if (it == seen.end()) {
          seen.emplace(key, e * nfe + f);
        } else {
          if (it->second < 0) fail(FR_E_MESH, "face shared by more than two elements");
          pairs.push_back({it->second, e * nfe + f, {0, 0, 0}});
          done[it->second] = done[e * nfe + f] = 1;
          it->second = -1;
        }
      }
  }
  for (int64_t i = 0; i < d.n_bfaces; ++i) {
    const int64_t e = d.bfaces[3 * i], f = d.bfaces[3 * i + 1], kind = d.bfaces[3 * i + 2];
    if (e < 0 || e >= E || f < 0 || f >= nfe ||
        (kind != FR_BC_WALL && kind != FR_BC_FARFIELD && !(allow_mortar && kind == KIND_MORTAR)))
      fail(FR_E_ARG, "invalid boundary face entry");
    if (done[e * nfe + f]) fail(FR_E_MESH, "boundary face is also an interior face");
    done[e * nfe + f] = 2;
    for (int m = 0; m < nfp; ++m) H.nbr[size_t(e) * nf + f * nfp + m] = -kind;
  }
  // periodic: hash face centroids on a fine grid; look the translated centroid up
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < d.n_nodes; ++i)
      for (int k = 0; k < dim; ++k) {
        lo[k] = std::min(lo[k], d.nodes[i * dim + k]);
        hi[k] = std::max(hi[k], d.nodes[i * dim + k]);
      }
    double ext = 0.0;
    for (int k = 0; k < dim; ++k) ext = std::max(ext, hi[k] - lo[k]);
    const double tol = 1e-9 * ext, cell = 1e-6 * ext;
    std::vector<int64_t> open;
    for (int64_t fi = 0; fi < E * nfe; ++fi)
      if (!done[fi]) open.push_back(fi);
    auto centroid = [&](int64_t fi, double c[3]) {
      const int64_t e = fi / nfe;
      const int f = int(fi % nfe);
      c[0] = c[1] = c[2] = 0.0;
      for (int cc = 0; cc < nc; ++cc) {
        const double *X = d.nodes + d.elem_nodes[e * nn + corner_local(f, cc)] * dim;
        for (int k = 0; k < dim; ++k) c[k] += X[k] / nc;
      }
    };
    std::map<std::array<int64_t, 3>, std::vector<int64_t>> grid;
    auto cellkey = [&](const double c[3]) {
      return std::array<int64_t, 3>{int64_t(std::floor(c[0] / cell)), int64_t(std::floor(c[1] / cell)),
                                    int64_t(std::floor(c[2] / cell))};
    };
    for (auto fi : open) {
      double c[3];
      centroid(fi, c);
      grid[cellkey(c)].push_back(fi);
    }
    for (auto fi : open) {
      if (done[fi]) continue;
      double c[3];
      centroid(fi, c);
      bool found = false;
      for (int p = 0; p < d.n_periodic && !found; ++p)
        for (int sg = -1; sg <= 1 && !found; sg += 2) {
          double t[3] = {0, 0, 0}, ct[3];
          for (int k = 0; k < dim; ++k) t[k] = sg * d.periodic_shift[p * dim + k];
          for (int k = 0; k < 3; ++k) ct[k] = c[k] + t[k];
          auto base = cellkey(ct);
          for (int dz = -1; dz <= 1 && !found; ++dz)
            for (int dy = -1; dy <= 1 && !found; ++dy)
              for (int dx = -1; dx <= 1 && !found; ++dx) {
                auto it = grid.find({base[0] + dx, base[1] + dy, base[2] + dz});
                if (it == grid.end()) continue;
                for (auto fj : it->second) {
                  if (fj == fi || done[fj]) continue;
                  double c2[3];
                  centroid(fj, c2);
                  bool same = true;
                  for (int k = 0; k < dim; ++k)
                    if (std::fabs(c2[k] - ct[k]) > tol) same = false;
                  if (!same) continue;
                  pairs.push_back({fi, fj, {t[0], t[1], t[2]}});
                  done[fi] = done[fj] = 1;
                  found = true;
                  break;
                }
              }
        }
      if (!found) fail(FR_E_MESH, "face is neither matched, periodic nor a listed boundary");
    }
  }
  // flux points of a matched face pair: nearest partner point by position
  for (const auto &P : pairs) {
    const int64_t eA = P.a / nfe, eB = P.b / nfe;
    const int fA = int(P.a % nfe), fB = int(P.b % nfe);
    // length scale of the face: the spread of its flux points, or (one flux point,
    // order 0) the distance from the element's solution point to it
    double hA = 0.0;
    for (int m = 0; m < nfp; ++m)
      for (int k = 0; k < dim; ++k)
        hA = std::max(hA, std::fabs(H.fx[(size_t(eA) * nf + fA * nfp + m) * 3 + k] -
                                    (nfp > 1 ? H.fx[(size_t(eA) * nf + fA * nfp) * 3 + k]
                                             : H.xu[size_t(eA) * nu * 3 + k])));
    const double ptol = 1e-7 * std::max(hA, 1e-300);
    for (int m = 0; m < nfp; ++m) {
      const double *xa = &H.fx[(size_t(eA) * nf + fA * nfp + m) * 3];
      int best = -1;
      double bd = 1e300;
      for (int m2 = 0; m2 < nfp; ++m2) {
        const double *xb = &H.fx[(size_t(eB) * nf + fB * nfp + m2) * 3];
        double dd = 0.0;
        for (int k = 0; k < dim; ++k) dd = std::max(dd, std::fabs(xa[k] + P.shift[k] - xb[k]));
        if (dd < bd) { bd = dd; best = m2; }
      }
      if (bd > ptol) fail(FR_E_MESH, "flux points of a matched face do not coincide");
      const int64_t ga = eA * nf + fA * nfp + m, gb = eB * nf + fB * nfp + best;
      if (H.nbr[ga] != INT64_MIN || H.nbr[gb] != INT64_MIN) fail(FR_E_MESH, "flux point matched twice");
      H.nbr[ga] = gb;
      H.nbr[gb] = ga;
    }
  }
  for (auto v : H.nbr)
    if (v == INT64_MIN) fail(FR_E_MESH, "unmatched flux point");
  return H;
}

}  // namespace

// ---------------------------------------------------------------------------
// the solver handle
// ---------------------------------------------------------------------------
struct DesignInfo {
  int64_t e0 = 0, E = 0, blk0 = 0, nblk = 0, wall0 = 0, nwall = 0;
  double dt = 0, fs[5] = {0, 0, 0, 0, 0}, ref_area = 1, lift[3] = {0, 0, 0}, drag[3] = {0, 0, 0};
};

struct fr_mesh {
  int dim = 3, order = 3, prec = 0, device = 0;
  Dims dm{3, 3};
  int64_t E = 0, nblk = 0, nwall = 0;
  std::vector<DesignInfo> designs;
  std::vector<int64_t> nbr_canon;   // [E][nf]
  std::vector<double> xu;           // [E][nu][3]
  double gamma = 1.4, prandtl = 0.72, mu = 0.0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  fr_alloc_fn alloc = nullptr;
  fr_free_fn dfree = nullptr;
  void *alloc_ctx = nullptr;
  std::vector<void *> allocations;
  size_t bytes = 0;
  DevArrays a;
  LaunchCfg cfg;
  bool state_set = false;
  // UF holds the trace of the current state (the last stage of a step writes it), so
  // the next step need not interpolate it again
  bool trace_valid = false;
  // the wall forces of the state the last step left are not yet in the sums: the next
  // step's first stage adds them (its force pass reads that state), or flush_forces does
  // when they are read first
  bool forces_pending = false;
  hipGraphExec_t graph_first = nullptr, graph_rest = nullptr, graph_multi = nullptr;
  bool extruded = false;  // 3D, every element z-extruded: column metrics present

  // variable order: one uniform-order solver per order present (ascending order),
  // all on this handle's stream and sharing its mortar tables (DevArrays MO.., MT, PO..)
  std::vector<std::unique_ptr<fr_mesh>> groups;
  std::vector<int> eorder;              // [E] element order
  std::vector<int> egroup;              // [E] group of the element
  std::vector<int64_t> elocal;          // [E] canonical index of the element within its group
  std::vector<int64_t> eslot;           // [E] block * EB + slot of the element in its group
  std::vector<std::vector<int>> gdesign;  // [group][design]: the design's index in the group, or -1
  std::vector<int64_t> uoff;            // [E + 1] first solution point of the element
  int64_t n_mortar = 0;                 // mortar points
  std::vector<const void *> group_uf, group_pv;  // the groups' UF and PV arrays
  bool mixed() const { return !groups.empty(); }

  size_t real_size() const { return prec == FR_FP32 ? 4 : 8; }

  void *dalloc(size_t n) {
    if (n == 0) n = 256;
    void *p = nullptr;
    if (alloc) {
      p = alloc(n, alloc_ctx, stream);
      if (!p) fail(FR_E_NOMEM, "device allocation callback failed");
    } else {
      if (hipMalloc(&p, n) != hipSuccess) fail(FR_E_NOMEM, "hipMalloc failed");
    }
    allocations.push_back(p);
    bytes += n;
    if (hipMemsetAsync(p, 0, n, stream) != hipSuccess) fail(FR_E_DEVICE, "hipMemsetAsync failed");
    return p;
  }
  template <class T> T *upload(const std::vector<T> &v) {
    T *p = (T *)dalloc(v.size() * sizeof(T));
    hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream), "upload");
    return p;
  }
  // teardown: errors are not reported from a destructor
  ~fr_mesh() {
    if (graph_first) (void)hipGraphExecDestroy(graph_first);
    if (graph_rest) (void)hipGraphExecDestroy(graph_rest);
    if (graph_multi) (void)hipGraphExecDestroy(graph_multi);
    groups.clear();  // they run on this handle's stream
    if (stream) (void)hipStreamSynchronize(stream);
    for (void *p : allocations) {
      if (dfree)
        dfree(p, alloc_ctx, stream);
      else
        (void)hipFree(p);
    }
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

void validate_desc(const fr_mesh_desc *d) {
  if (!d) fail(FR_E_ARG, "null descriptor");
  if (d->dim != 2 && d->dim != 3) fail(FR_E_ARG, "dim must be 2 or 3");
  if (d->geom_order != 1 && d->geom_order != 2) fail(FR_E_ARG, "geom_order must be 1 or 2");
  if (d->precision != FR_FP64 && d->precision != FR_FP32) fail(FR_E_ARG, "unknown precision");
  if (!kernels_available(d->precision, d->dim, d->order)) fail(FR_E_UNSUPPORTED, "order not compiled in (0..4)");
  if (d->n_elems <= 0 || !d->elem_nodes || d->n_nodes <= 0 || !d->nodes) fail(FR_E_ARG, "empty mesh");
  if (d->n_periodic < 0 || (d->n_periodic > 0 && !d->periodic_shift)) fail(FR_E_ARG, "bad periodic list");
  if (d->n_bfaces < 0 || (d->n_bfaces > 0 && !d->bfaces)) fail(FR_E_ARG, "bad boundary list");
  if (!(d->gamma > 1.0) || !(d->prandtl > 0.0) || !(d->mu >= 0.0)) fail(FR_E_ARG, "bad gas constants");
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) fail(FR_E_ARG, "dt must be positive");
}

// kernels (bit = enum Kernel) that run the sum-factorised variant unless tuned otherwise
// keyed by (precision, dim, order, size class): the size class is the bit length of the
// block count, so a choice timed on a small mesh is not carried over to a large batch
std::map<int, unsigned> g_tuned;
std::mutex g_tuned_mu;
int tune_key(int prec, int dim, int order, int64_t nblk) {
  int bits = 0;
  while (nblk > 0) {
    ++bits;
    nblk >>= 1;
  }
  return ((prec * 10 + dim) * 10 + order) * 64 + bits;
}
unsigned default_variants(int prec, int dim, int order, int64_t nblk, bool extruded) {
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  auto it = g_tuned.find(tune_key(prec, dim, order, nblk));
  if (it != g_tuned.end()) {
    // a choice timed on an extruded mesh: other meshes of its class take the stored metrics
    if ((it->second & EXTRUDED_METRICS) && !extruded) return (it->second & ~EXTRUDED_METRICS) | STORED_METRICS;
    return it->second;
  }
  // fused stage, sum-factorised trace; column metrics on an extruded mesh, else the stored
  // ones (faster than forming them from the geometry nodes on every mesh timed)
  return 1u | (1u << K_INTERP) | (extruded ? EXTRUDED_METRICS : dim == 3 ? STORED_METRICS : 0u);
}

constexpr unsigned FUSED = 1u;  // variant-mask bit 0: two fused launches per stage

void drop_graphs(fr_mesh *M);

// Mortar points of one order group: for (element, face) of the group, the first
// mortar point of the face and the side (1: the lower-order element)
struct MortarMap {
  // key: the element's canonical index in the group (its designs concatenated) * 2 dim + face
  std::unordered_map<int64_t, std::pair<int64_t, int>> face;
};

void build_solver(fr_mesh *M, const fr_mesh_desc *descs, int nd, const MortarMap *mm = nullptr) {
  const fr_mesh_desc &d0 = descs[0];
  M->dim = d0.dim;
  M->order = d0.order;
  M->prec = d0.precision;
  M->device = d0.device;
  M->dm = Dims(d0.dim, d0.order);
  M->gamma = d0.gamma;
  M->prandtl = d0.prandtl;
  M->mu = d0.mu;
  M->alloc = d0.alloc;
  M->dfree = d0.free;
  M->alloc_ctx = d0.alloc_ctx;
  hip_check(hipSetDevice(d0.device), "hipSetDevice");
  if (d0.stream) {
    M->stream = (hipStream_t)d0.stream;
  } else {
    hip_check(hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking), "hipStreamCreate");
    M->own_stream = true;
  }
  const Dims &D = M->dm;
  const int dim = M->dim, nu = D.nu, nf = D.nf, nv = D.nv, NUP = D.nup, NFPAD = D.nfpad;
  // per-design host meshes
  std::vector<HostMesh> hm;
  hm.reserve(nd);
  int64_t e0 = 0, blk0 = 0, w0 = 0;
  for (int i = 0; i < nd; ++i) {
    hm.push_back(build_host_mesh(descs[i], mm != nullptr));
    DesignInfo di;
    di.e0 = e0;
    di.E = descs[i].n_elems;
    di.blk0 = blk0;
    di.nblk = (di.E + EB - 1) / EB;
    di.dt = descs[i].dt;
    for (int k = 0; k < 5; ++k) di.fs[k] = descs[i].freestream[k];
    di.ref_area = descs[i].ref_area;
    for (int k = 0; k < 3; ++k) {
      di.lift[k] = descs[i].lift_dir[k];
      di.drag[k] = descs[i].drag_dir[k];
    }
    di.wall0 = w0;
    for (auto v : hm.back().nbr)
      if (v == -FR_BC_WALL) ++di.nwall;
    w0 += di.nwall;
    e0 += di.E;
    blk0 += di.nblk;
    M->designs.push_back(di);
  }
  M->E = e0;
  M->nblk = blk0;
  M->nwall = w0;
  const int64_t NB = M->nblk;
  // canonical neighbour table and solution points (concatenated)
  M->nbr_canon.resize(size_t(M->E) * nf);
  M->xu.resize(size_t(M->E) * nu * 3);
  // block-layout geometry and tables
  std::vector<double> SM(size_t(NB) * NUP * dim * dim * EB, 0.0), IJ(size_t(NB) * NUP * EB, 0.0);
  std::vector<double> FN(size_t(NB) * NFPAD * dim * EB, 0.0), FA(size_t(NB) * NFPAD * EB, 0.0);
  std::vector<int> NBt(size_t(NB) * NFPAD * EB, 0);
  // 3D meshes of z-extruded elements: column metrics; empty slots hold the unit cube
  bool extruded = dim == 3;
  for (int di = 0; di < nd && extruded; ++di)
    for (int64_t e = 0; e < descs[di].n_elems && extruded; ++e) extruded = elem_extruded(descs[di], e);
  M->extruded = extruded;
  const int ncol = D.n * D.n, nfc = 4 * D.n + D.n * D.n;
  std::vector<double> XC(extruded ? size_t(NB) * ncol * 4 * EB : 0, 0.0), ZZ(extruded ? size_t(NB) * D.n * EB : 0, 1.0),
      FCX(extruded ? size_t(NB) * nfc * 2 * EB : 0, 0.0), IJC(extruded ? size_t(NB) * ncol * EB : 0, 1.0),
      IZ(extruded ? size_t(NB) * D.n * EB : 0, 1.0);
  if (extruded)
    for (int64_t blk = 0; blk < NB; ++blk)
      for (int sl = 0; sl < EB; ++sl) {
        for (int c = 0; c < ncol; ++c) {
          XC[lay(blk, c, 0, sl, ncol, 4)] = 1.0;
          XC[lay(blk, c, 3, sl, ncol, 4)] = 1.0;
          FCX[lay(blk, 4 * D.n + c, 0, sl, nfc, 2)] = 1.0;
        }
        for (int m = 0; m < D.n; ++m)
          for (int sd = 0; sd < 2; ++sd) {
            FCX[lay(blk, sd * D.n + m, 1, sl, nfc, 2)] = 1.0;      // xi faces: y_eta
            FCX[lay(blk, 2 * D.n + sd * D.n + m, 0, sl, nfc, 2)] = 1.0;  // eta faces: x_xi
          }
      }
  // 3D: triquadratic geometry nodes per element; empty slots hold the reference cube
  constexpr int NX = 27;
  std::vector<double> XN(dim == 3 ? size_t(NB) * NX * 3 * EB : 0, 0.0);
  if (dim == 3)
    for (int64_t blk = 0; blk < NB; ++blk)
      for (int sl = 0; sl < EB; ++sl)
        for (int a = 0; a < NX; ++a)
          for (int c = 0; c < 3; ++c)
            XN[lay(blk, a, c, sl, NX, 3)] = double((c == 0 ? a % 3 : c == 1 ? (a / 3) % 3 : a / 9) - 1);
  std::vector<int> bcount(NB), bdesign(NB);
  std::vector<int64_t> bcanon(NB), wall_first(nd + 1);
  std::vector<double> bdt(NB), fsd(size_t(nd) * 5);
  auto dev_slot = [&](int64_t g) {  // canonical element -> (block, slot)
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (M->designs[mid].e0 <= g) lo = mid; else hi = mid - 1;
    }
    const auto &di = M->designs[lo];
    const int64_t le = g - di.e0;
    return std::pair<int64_t, int>(di.blk0 + le / EB, int(le % EB));
  };
  if (int64_t(NB) * NFPAD * EB >= (int64_t(1) << 31)) fail(FR_E_UNSUPPORTED, "mesh too large for 32-bit tables");
  const Basis1D basis_n(M->order);
  for (int di = 0; di < nd; ++di) {
    const auto &H = hm[di];
    const auto &ds = M->designs[di];
    wall_first[di] = ds.wall0;
    for (int k = 0; k < 5; ++k) fsd[di * 5 + k] = ds.fs[k];
    for (int64_t b = 0; b < ds.nblk; ++b) {
      const int64_t blk = ds.blk0 + b;
      bcount[blk] = int(std::min<int64_t>(EB, ds.E - b * EB));
      bdesign[blk] = di;
      bcanon[blk] = ds.e0 + b * EB;
      bdt[blk] = ds.dt;
    }
    // wall flux points are numbered in canonical (element, flux point) order
    std::vector<int64_t> wall_base(size_t(ds.E) + 1, 0);
    for (int64_t e = 0; e < ds.E; ++e) {
      int64_t c = 0;
      for (int qq = 0; qq < nf; ++qq) c += H.nbr[size_t(e) * nf + qq] == -FR_BC_WALL;
      wall_base[e + 1] = wall_base[e] + c;
    }
    parallel_for(ds.E, [&](int64_t e) {
      int64_t widx = ds.wall0 + wall_base[e];
      const int64_t g = ds.e0 + e;
      const int64_t blk = ds.blk0 + e / EB;
      const int s = int(e % EB);
      if (dim == 3)
        for (int a = 0; a < NX; ++a) {
          const std::array<double, 3> r{double(a % 3 - 1), double((a / 3) % 3 - 1), double(a / 9 - 1)};
          double x[3], jac[3][3];
          geom_map(descs[di], e, r, x, jac);
          for (int c = 0; c < 3; ++c) XN[lay(blk, a, c, s, NX, 3)] = x[c];
        }
      if (extruded) {
        const Basis1D &gl = basis_n;
        for (int i1 = 0; i1 < D.n; ++i1)
          for (int i0 = 0; i0 < D.n; ++i0) {
            double jc[4];
            extruded_jacobian(descs[di], e, gl.x[size_t(i0)], gl.x[size_t(i1)], jc);
            for (int c = 0; c < 4; ++c) XC[lay(blk, i0 + D.n * i1, c, s, ncol, 4)] = jc[c];
            FCX[lay(blk, 4 * D.n + i0 + D.n * i1, 0, s, nfc, 2)] = jc[0] * jc[3] - jc[2] * jc[1];
            IJC[lay(blk, i0 + D.n * i1, 0, s, ncol, 1)] = 1.0 / FCX[lay(blk, 4 * D.n + i0 + D.n * i1, 0, s, nfc, 2)];
            FCX[lay(blk, 4 * D.n + i0 + D.n * i1, 1, s, nfc, 2)] = 0.0;
          }
        for (int i2 = 0; i2 < D.n; ++i2) {
          ZZ[lay(blk, i2, 0, s, D.n, 1)] = extruded_zzeta(descs[di], e, gl.x[size_t(i2)]);
          IZ[lay(blk, i2, 0, s, D.n, 1)] = 1.0 / ZZ[lay(blk, i2, 0, s, D.n, 1)];
        }
        for (int sd = 0; sd < 2; ++sd)
          for (int m = 0; m < D.n; ++m) {
            double jc[4];
            extruded_jacobian(descs[di], e, sd ? 1.0 : -1.0, gl.x[size_t(m)], jc);  // xi face: x_eta, y_eta
            FCX[lay(blk, sd * D.n + m, 0, s, nfc, 2)] = jc[1];
            FCX[lay(blk, sd * D.n + m, 1, s, nfc, 2)] = jc[3];
            extruded_jacobian(descs[di], e, gl.x[size_t(m)], sd ? 1.0 : -1.0, jc);  // eta face: x_xi, y_xi
            FCX[lay(blk, 2 * D.n + sd * D.n + m, 0, s, nfc, 2)] = jc[0];
            FCX[lay(blk, 2 * D.n + sd * D.n + m, 1, s, nfc, 2)] = jc[2];
          }
      }
      for (int i = 0; i < nu; ++i) {
        for (int c = 0; c < dim * dim; ++c)
          SM[lay(blk, i, c, s, NUP, dim * dim)] = H.S[(size_t(e) * nu + i) * dim * dim + c];
        IJ[lay(blk, i, 0, s, NUP, 1)] = 1.0 / H.detJ[size_t(e) * nu + i];
        for (int c = 0; c < 3; ++c) M->xu[(size_t(g) * nu + i) * 3 + c] = H.xu[(size_t(e) * nu + i) * 3 + c];
      }
      for (int qq = 0; qq < nf; ++qq) {
        const size_t hq = size_t(e) * nf + qq;
        for (int c = 0; c < dim; ++c) FN[lay(blk, qq, c, s, NFPAD, dim)] = H.fn[hq * dim + c];
        FA[lay(blk, qq, 0, s, NFPAD, 1)] = H.fA[hq];
        const int64_t p = H.nbr[hq];
        int code;
        if (p >= 0) {
          const int64_t gp = ds.e0 + p / nf;
          const int qp = int(p % nf);
          auto bs = dev_slot(gp);
          code = int(lay(bs.first, qp, 0, bs.second, NFPAD, 1));
          M->nbr_canon[size_t(g) * nf + qq] = gp * nf + qp;
        } else if (-p == KIND_MORTAR) {
          const auto &fs = mm->face.at(g * 2 * dim + qq / D.nfp);
          const int64_t idx = ((fs.first + qq % D.nfp) << 1) | fs.second;
          code = -int(BC_MORTAR | (idx << 2));
          M->nbr_canon[size_t(g) * nf + qq] = p;
        } else {
          const int kind = int(-p);
          code = kind == FR_BC_WALL ? -int(kind | (widx++ << 2)) : -kind;
          M->nbr_canon[size_t(g) * nf + qq] = p;
        }
        NBt[lay(blk, qq, 0, s, NFPAD, 1)] = code;
      }
    });
  }
  wall_first[nd] = M->nwall;
  // per-face neighbour codes from the per-point ones (one-order meshes): every point of a
  // matched face must name the same partner element and face, through one symmetry of the
  // square; a boundary face one kind, its wall points numbered on from the first. Any
  // other face leaves the mesh on the per-point codes.
  std::vector<int> NBFt;
  if (!mm) {
    const int nfc = 2 * dim, nfp = D.nfp;
    NBFt.assign(size_t(NB) * nfc * EB, 0);
    bool ok = true;
    for (int64_t blk = 0; blk < NB && ok; ++blk)
      for (int sl = 0; sl < bcount[size_t(blk)] && ok; ++sl)
        for (int f = 0; f < nfc && ok; ++f) {
          const int c0 = NBt[lay(blk, f * nfp, 0, sl, NFPAD, 1)];
          int code = c0;
          if (c0 < 0) {
            for (int m = 1; m < nfp && ok; ++m) {
              const int c = NBt[lay(blk, f * nfp + m, 0, sl, NFPAD, 1)];
              const int want = ((-c0) & 3) == FR_BC_WALL ? -(((-c0) & 3) | ((((-c0) >> 2) + m) << 2)) : c0;
              ok = c == want;
            }
          } else {
            // decode the partner of point 0: c0 = lay(pblk, q', 0, pslot, NFPAD, 1)
            const int64_t cs = c0 / SB, ps_blk = cs / (int64_t(NSB) * NFPAD);
            const int pq = int(cs % NFPAD);
            const int psl = int(((cs / NFPAD) % NSB) * SB + c0 % SB);
            const int pf = pq / nfp;
            int map = -1;
            for (int o = 0; o < (dim == 2 ? 2 : 8) && map < 0; ++o) {
              bool all = true;
              for (int m = 0; m < nfp && all; ++m)
                all = NBt[lay(blk, f * nfp + m, 0, sl, NFPAD, 1)] ==
                      int(lay(ps_blk, pf * nfp + face_map(m, o, D.n, dim), 0, psl, NFPAD, 1));
              if (all) map = o;
            }
            ok = map >= 0 && (ps_blk * EB + psl) < (int64_t(1) << 25);
            code = int((((ps_blk * EB + psl) << 3) | pf) << 3 | map);
          }
          NBFt[lay(blk, f, 0, sl, nfc, 1)] = code;
        }
    // the decoding the kernels apply must give back every per-point code
    for (int64_t blk = 0; blk < NB && ok; ++blk)
      for (int sl = 0; sl < bcount[size_t(blk)] && ok; ++sl)
        for (int q = 0; q < nf && ok; ++q) {
          const int fc = NBFt[lay(blk, q / nfp, 0, sl, nfc, 1)];
          ok = point_code(fc, q % nfp, D.n, nfp, NFPAD, dim) == NBt[lay(blk, q, 0, sl, NFPAD, 1)];
        }
    if (!ok) NBFt.clear();
  }
  // operators
  Operators op(dim, M->order);
  const int RTU = NUP / 16, RTF = NFPAD / 16, KTU = D.ku / 4, KTF = D.kf / 4;
  std::vector<double> sInt, sGrad, sGcorr, sDivS, sCorr;
  swizzle(sInt, RTF, KTU, [&](int r, int c) { return (r < nf && c < nu) ? op.Mint[size_t(r) * nu + c] : 0.0; });
  for (int k = 0; k < dim; ++k) {
    swizzle(sGrad, RTU, KTU, [&](int r, int c) {
      return (r < nu && c < nu) ? op.Mgrad[(size_t(k) * nu + r) * nu + c] : 0.0;
    });
    swizzle(sGcorr, RTU, KTF, [&](int r, int c) {
      return (r < nu && c < nf) ? op.Mgcorr[(size_t(k) * nu + r) * nf + c] : 0.0;
    });
  }
  for (int rt = 0; rt < RTU; ++rt)
    for (int k = 0; k < dim; ++k)
      for (int kt = 0; kt < KTU; ++kt)
        for (int l = 0; l < 64; ++l) {
          const int r = rt * 16 + l % 16, c = kt * 4 + l / 16;
          sDivS.push_back((r < nu && c < nu) ? op.MdivS[size_t(r) * dim * nu + k * nu + c] : 0.0);
        }
  swizzle(sCorr, RTU, KTF, [&](int r, int c) { return (r < nu && c < nf) ? op.Mcorr[size_t(r) * nf + c] : 0.0; });
  auto upload_real = [&](const std::vector<double> &v) -> void * {
    if (M->prec == FR_FP64) return M->upload(v);
    std::vector<float> f(v.begin(), v.end());
    return M->upload(f);
  };
  DevArrays &a = M->a;
  a.opInt = upload_real(sInt);
  a.opGrad = upload_real(sGrad);
  a.opGcorr = upload_real(sGcorr);
  a.opDivS = upload_real(sDivS);
  a.opCorr = upload_real(sCorr);
  {
    Basis1D b(M->order);
    std::vector<double> bv(b.D);
    bv.insert(bv.end(), b.lm.begin(), b.lm.end());
    bv.insert(bv.end(), b.lp.begin(), b.lp.end());
    bv.insert(bv.end(), b.gLd.begin(), b.gLd.end());
    bv.insert(bv.end(), b.gRd.begin(), b.gRd.end());
    // strong-form 1D divergence: Dv = D - gR' l(+1)^T - gL' l(-1)^T
    for (int i = 0; i < b.n; ++i)
      for (int j = 0; j < b.n; ++j) bv.push_back(b.D[i * b.n + j] - b.gRd[i] * b.lp[j] - b.gLd[i] * b.lm[j]);
    a.basis = upload_real(bv);
  }
  a.SM = M->upload(SM);
  a.IJ = M->upload(IJ);
  a.FN = M->upload(FN);
  a.FA = M->upload(FA);
  a.NB = M->upload(NBt);
  if (!NBFt.empty()) a.NBF = M->upload(NBFt);
  if (extruded) {
    a.XC = M->upload(XC);
    a.ZZ = M->upload(ZZ);
    a.FCX = M->upload(FCX);
    a.IJC = M->upload(IJC);
    a.IZ = M->upload(IZ);
  }
  if (dim == 3) {
    a.XN = M->upload(XN);
    Basis1D b(M->order);
    std::vector<double> gq(size_t(6) * b.n);
    for (int i = 0; i < b.n; ++i) {
      double l[3], d[3];
      shape_q(2, b.x[size_t(i)], l, d);
      for (int k = 0; k < 3; ++k) {
        gq[size_t(k * b.n + i)] = l[k];
        gq[size_t((3 + k) * b.n + i)] = d[k];
      }
    }
    a.GQ = M->upload(gq);
  }
  a.bcount = M->upload(bcount);
  a.bdesign = M->upload(bdesign);
  a.bcanon = M->upload(bcanon);
  a.bdt = M->upload(bdt);
  a.fsd = M->upload(fsd);
  a.wall_first = M->upload(wall_first);
  {
    Basis1D b(M->order);
    RefElem R(dim, M->order);
    std::vector<double> wf(NFPAD, 0.0);
    for (int f = 0; f < 2 * dim; ++f)
      for (int m = 0; m < R.nfp; ++m) wf[f * R.nfp + m] = dim == 2 ? b.w[m] : b.w[m % R.n] * b.w[m / R.n];
    a.wface = M->upload(wf);
  }
  const size_t rs = M->real_size();
  const size_t nU = size_t(NB) * NUP * nv * EB, nF = size_t(NB) * NFPAD * nv * EB, nG = size_t(NB) * NUP * dim * nv * EB;
  a.U = M->dalloc(nU * rs);
  a.US = M->dalloc(nU * rs);
  a.ACC = M->dalloc(nU * rs);
  a.RES = M->dalloc(nU * rs);
  a.UF = M->dalloc(nF * rs);
  a.DU = M->dalloc(nF * rs);
  a.FI = M->dalloc(nF * rs);
  a.PV = M->dalloc(nF * rs);
  a.GU = M->dalloc(nG * rs);
  a.FT = M->dalloc(nG * rs);
  a.FC = (double *)M->dalloc(std::max<int64_t>(M->nwall, 1) * 3 * sizeof(double));
  a.fsum = (double *)M->dalloc(size_t(nd) * 8 * sizeof(double));
  a.flag = (int *)M->dalloc(sizeof(int));
  a.stage64 = (double *)M->dalloc(size_t(M->E) * nu * nv * sizeof(double));
  LaunchCfg &c = M->cfg;
  c.prec = M->prec;
  c.dim = dim;
  c.order = M->order;
  c.nblk = NB;
  c.ndesign = nd;
  c.n_canon = M->E;
  c.gamma = M->gamma;
  c.mu = M->mu;
  c.prandtl = M->prandtl;
  c.stream = M->stream;
  c.variant_mask = default_variants(c.prec, dim, M->order, NB, M->extruded);
  hip_check(hipStreamSynchronize(M->stream), "mesh upload");
}

// ---------------------------------------------------------------------------
// variable order: order groups coupled by mortar faces
// ---------------------------------------------------------------------------

// Legendre polynomial P_k(t)
double legendre(int k, double t) {
  double P, Pm1;
  Basis1D::legendre_pair(k, t, P, Pm1);
  return P;
}

// A face shared by elements of different orders, seen from its higher-order
// element H: the orientation O maps H's face coordinates to L's, t = O s
struct MortarFace {
  int64_t eH, eL;  // canonical elements
  int fH, fL;
  int O[2][2];
  int64_t baseH = 0, baseL = 0;  // first mortar point of each side
};

void build_mixed(fr_mesh *M, const fr_mesh_desc *descs, int nd) {
  const fr_mesh_desc &d = descs[0];
  const int dim = d.dim, nfe = 2 * dim;
  M->dim = dim;
  M->prec = d.precision;
  M->device = d.device;
  M->gamma = d.gamma;
  M->prandtl = d.prandtl;
  M->mu = d.mu;
  M->alloc = d.alloc;
  M->dfree = d.free;
  M->alloc_ctx = d.alloc_ctx;
  hip_check(hipSetDevice(d.device), "hipSetDevice");
  if (d.stream) {
    M->stream = (hipStream_t)d.stream;
  } else {
    hip_check(hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking), "hipStreamCreate");
    M->own_stream = true;
  }
  // element orders of all designs, concatenated (a design without elem_order has its
  // `order` everywhere), and the orders present
  std::vector<int64_t> de0(size_t(nd) + 1, 0);
  for (int i = 0; i < nd; ++i) {
    de0[size_t(i) + 1] = de0[size_t(i)] + descs[i].n_elems;
    for (int64_t e = 0; e < descs[i].n_elems; ++e)
      M->eorder.push_back(descs[i].elem_order ? descs[i].elem_order[e] : descs[i].order);
  }
  const int64_t E = de0[size_t(nd)];
  M->E = E;
  std::vector<int> edes(static_cast<size_t>(E));
  for (int i = 0; i < nd; ++i)
    for (int64_t e = de0[size_t(i)]; e < de0[size_t(i) + 1]; ++e) edes[size_t(e)] = i;
  std::vector<int> present;
  for (int p : M->eorder) {
    if (!kernels_available(d.precision, dim, p)) fail(FR_E_UNSUPPORTED, "element order not compiled in (0..4)");
    if (std::find(present.begin(), present.end(), p) == present.end()) present.push_back(p);
  }
  std::sort(present.begin(), present.end());
  const size_t ng = present.size();
  M->order = present.back();
  M->dm = Dims(dim, M->order);
  // groups: the designs with elements of each order, in design order; per element its
  // group, its index within its design's part of the group and its canonical index in
  // the group (the group's designs concatenated)
  M->gdesign.assign(ng, std::vector<int>(size_t(nd), -1));
  std::vector<std::vector<int64_t>> gcount(ng, std::vector<int64_t>(size_t(nd), 0));
  M->egroup.resize(size_t(E));
  M->elocal.resize(size_t(E));
  M->eslot.resize(size_t(E));
  M->uoff.assign(size_t(E) + 1, 0);
  std::vector<int64_t> eli(static_cast<size_t>(E));  // index within the design's part of the group
  for (int64_t e = 0; e < E; ++e) {
    const int g = int(std::find(present.begin(), present.end(), M->eorder[size_t(e)]) - present.begin());
    M->egroup[size_t(e)] = g;
    eli[size_t(e)] = gcount[size_t(g)][size_t(edes[size_t(e)])]++;
    const int n = M->eorder[size_t(e)] + 1;
    M->uoff[size_t(e) + 1] = M->uoff[size_t(e)] + (dim == 2 ? n * n : n * n * n);
  }
  std::vector<std::vector<int64_t>> gde0(ng), gdblk0(ng);  // per group, per design in it
  for (size_t g = 0; g < ng; ++g) {
    int64_t c = 0, blk = 0;
    for (int i = 0; i < nd; ++i) {
      if (!gcount[g][size_t(i)]) continue;
      M->gdesign[g][size_t(i)] = int(gde0[g].size());
      gde0[g].push_back(c);
      gdblk0[g].push_back(blk);
      c += gcount[g][size_t(i)];
      blk += (gcount[g][size_t(i)] + EB - 1) / EB;
    }
  }
  for (int64_t e = 0; e < E; ++e) {
    const size_t g = size_t(M->egroup[size_t(e)]);
    const int gi = M->gdesign[g][size_t(edes[size_t(e)])];
    M->elocal[size_t(e)] = gde0[g][size_t(gi)] + eli[size_t(e)];
    M->eslot[size_t(e)] = (gdblk0[g][size_t(gi)] + eli[size_t(e)] / EB) * EB + eli[size_t(e)] % EB;
  }
  // faces and their orientation from each design at order 1 (2 or 2 x 2 face points at
  // +-1/sqrt(3) along each face axis, matched by position); element indices global
  const int nfp1 = dim == 2 ? 2 : 4, nf1 = nfe * nfp1;
  const double x1 = 1.0 / std::sqrt(3.0);
  auto coords1 = [&](int m, double s[2]) {
    s[0] = (m & 1) ? x1 : -x1;
    s[1] = dim == 3 ? (((m >> 1) & 1) ? x1 : -x1) : 0.0;
  };
  std::vector<MortarFace> faces;
  for (int i = 0; i < nd; ++i) {
    fr_mesh_desc d1 = descs[i];
    d1.order = 1;
    d1.elem_order = nullptr;
    const HostMesh H1 = build_host_mesh(d1);
    const int64_t base = de0[size_t(i)];
    for (int64_t le = 0; le < descs[i].n_elems; ++le)
      for (int f = 0; f < nfe; ++f) {
        const int64_t p = H1.nbr[size_t(le) * nf1 + f * nfp1];
        if (p < 0) continue;
        const int64_t e = base + le, ep = base + p / nf1;
        const int fp = int((p % nf1) / nfp1);
        const int oe = M->eorder[size_t(e)], op = M->eorder[size_t(ep)];
        if (oe <= op) continue;  // each mortar face once, from its higher-order side
        MortarFace mf;
        mf.eH = e; mf.fH = f; mf.eL = ep; mf.fL = fp;
        // O from the images of face points 1 and 2 (steps along each face axis) of point 0
        double t[3][2];
        for (int m = 0; m < (dim == 2 ? 2 : 3); ++m) {
          const int64_t q = H1.nbr[size_t(le) * nf1 + f * nfp1 + m];
          coords1(int(q % nf1) % nfp1, t[m]);
        }
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) mf.O[r][c] = 0;
        for (int r = 0; r < (dim == 2 ? 1 : 2); ++r) {
          mf.O[r][0] = int(std::lround((t[1][r] - t[0][r]) / (2.0 * x1)));
          if (dim == 3) mf.O[r][1] = int(std::lround((t[2][r] - t[0][r]) / (2.0 * x1)));
        }
        faces.push_back(mf);
      }
  }
  // mortar points: each face's higher-order points, then its lower-order points
  std::vector<MortarMap> maps(ng);
  int64_t np = 0;
  auto nfp_of = [&](int p) { return dim == 2 ? p + 1 : (p + 1) * (p + 1); };
  for (auto &mf : faces) {
    mf.baseH = np;
    np += nfp_of(M->eorder[size_t(mf.eH)]);
    mf.baseL = np;
    np += nfp_of(M->eorder[size_t(mf.eL)]);
    maps[size_t(M->egroup[size_t(mf.eH)])].face[M->elocal[size_t(mf.eH)] * nfe + mf.fH] = {mf.baseH, 0};
    maps[size_t(M->egroup[size_t(mf.eL)])].face[M->elocal[size_t(mf.eL)] * nfe + mf.fL] = {mf.baseL, 1};
  }
  M->n_mortar = np;
  if ((np << 3) >= (int64_t(1) << 31)) fail(FR_E_UNSUPPORTED, "too many mortar points for 32-bit codes");
  // the order groups: per design present, the sub-mesh of its elements of that order,
  // whose faces to other orders are listed as mortar faces
  for (size_t g = 0; g < ng; ++g) {
    std::vector<std::vector<int64_t>> en(static_cast<size_t>(nd)), bf(static_cast<size_t>(nd));
    for (int i = 0; i < nd; ++i) {
      if (M->gdesign[g][size_t(i)] < 0) continue;
      const fr_mesh_desc &di = descs[i];
      const int na = di.geom_order + 1, nn = dim == 2 ? na * na : na * na * na;
      const int64_t base = de0[size_t(i)];
      for (int64_t le = 0; le < di.n_elems; ++le)
        if (M->egroup[size_t(base + le)] == int(g))
          en[size_t(i)].insert(en[size_t(i)].end(), di.elem_nodes + le * nn, di.elem_nodes + (le + 1) * nn);
      for (int64_t k = 0; k < di.n_bfaces; ++k) {
        const int64_t le = di.bfaces[3 * k];
        if (le < 0 || le >= di.n_elems) fail(FR_E_ARG, "invalid boundary face entry");
        if (M->egroup[size_t(base + le)] != int(g)) continue;
        bf[size_t(i)].insert(bf[size_t(i)].end(), {eli[size_t(base + le)], di.bfaces[3 * k + 1], di.bfaces[3 * k + 2]});
      }
    }
    for (const auto &kv : maps[g].face) {
      // group-canonical element -> its design and its index within the design's part
      const int64_t ge = kv.first / nfe;
      int gi = int(std::upper_bound(gde0[g].begin(), gde0[g].end(), ge) - gde0[g].begin()) - 1;
      int i = 0;
      while (M->gdesign[g][size_t(i)] != gi) ++i;
      bf[size_t(i)].insert(bf[size_t(i)].end(), {ge - gde0[g][size_t(gi)], kv.first % nfe, KIND_MORTAR});
    }
    std::vector<fr_mesh_desc> dgs;
    for (int i = 0; i < nd; ++i) {
      if (M->gdesign[g][size_t(i)] < 0) continue;
      fr_mesh_desc dg = descs[i];
      dg.order = present[g];
      dg.elem_order = nullptr;
      dg.n_elems = gcount[g][size_t(i)];
      dg.elem_nodes = en[size_t(i)].data();
      dg.n_bfaces = int64_t(bf[size_t(i)].size() / 3);
      dg.bfaces = bf[size_t(i)].empty() ? nullptr : bf[size_t(i)].data();
      dg.stream = M->stream;
      dgs.push_back(dg);
    }
    std::unique_ptr<fr_mesh> G(new fr_mesh());
    build_solver(G.get(), dgs.data(), int(dgs.size()), &maps[g]);
    G->cfg.variant_mask = FUSED | (1u << K_INTERP) | (G->extruded ? EXTRUDED_METRICS : 0u);
    M->groups.push_back(std::move(G));
  }
  for (auto &G : M->groups) {
    M->nblk += G->nblk;
    M->nwall += G->nwall;
  }
  for (int i = 0; i < nd; ++i) {
    DesignInfo di;
    di.e0 = de0[size_t(i)];
    di.E = descs[i].n_elems;
    di.dt = descs[i].dt;
    for (int k = 0; k < 5; ++k) di.fs[k] = descs[i].freestream[k];
    di.ref_area = descs[i].ref_area;
    for (int k = 0; k < 3; ++k) {
      di.lift[k] = descs[i].lift_dir[k];
      di.drag[k] = descs[i].drag_dir[k];
    }
    M->designs.push_back(di);
  }
  // gather tables
  auto code_of = [&](int64_t e, int f, int m) {  // partner code of a face point in its group
    const fr_mesh &G = *M->groups[size_t(M->egroup[size_t(e)])];
    const int64_t sl = M->eslot[size_t(e)];
    const int q = f * G.dm.nfp + m;
    return int(lay(sl / EB, q, 0, int(sl % EB), G.dm.nfpad, 1));
  };
  std::vector<int> row_out, row_off{0}, ent_grp, ent_code;
  std::vector<double> ent_w;
  struct LowRow { int out; std::vector<int> code; std::vector<double> w; };
  std::vector<LowRow> low;
  std::vector<std::vector<int>> rowsB_code(0);
  // face geometry helpers on each side
  for (int pass = 0; pass < 2; ++pass) {
    for (const auto &mf : faces) {
      const int pH = M->eorder[size_t(mf.eH)], pL = M->eorder[size_t(mf.eL)];
      const Basis1D bH(pH), bL(pL);
      const int nH = pH + 1, nL = pL + 1, nfpH = nfp_of(pH), nfpL = nfp_of(pL);
      const int gH = M->egroup[size_t(mf.eH)], gL = M->egroup[size_t(mf.eL)];
      // L-face coordinates of every H point
      std::vector<std::array<double, 2>> tH(static_cast<size_t>(nfpH));
      for (int j = 0; j < nfpH; ++j) {
        const double sj[2] = {bH.x[j % nH], dim == 3 ? bH.x[j / nH] : 0.0};
        for (int r = 0; r < 2; ++r) tH[size_t(j)][size_t(r)] = mf.O[r][0] * sj[0] + mf.O[r][1] * sj[1];
      }
      if (pass == 0) {
        // higher-order points: interpolants of the lower-order side's face data
        for (int j = 0; j < nfpH; ++j) {
          row_out.push_back(int(mf.baseH + j));
          const auto l0 = bL.eval_all(tH[size_t(j)][0]);
          const auto l1 = dim == 3 ? bL.eval_all(tH[size_t(j)][1]) : std::vector<double>(1, 1.0);
          for (int i = 0; i < nfpL; ++i) {
            ent_grp.push_back(gL);
            ent_code.push_back(code_of(mf.eL, mf.fL, i));
            ent_w.push_back(l0[size_t(i % nL)] * (dim == 3 ? l1[size_t(i / nL)] : 1.0));
          }
          row_off.push_back(int(ent_w.size()));
        }
        continue;
      }
      // lower-order points: L2 projection onto the lower order's face polynomials of
      // the higher-order side's face data, integrated by the higher-order face quadrature
      std::vector<double> P(size_t(nfpL) * nfpH, 0.0);
      for (int i = 0; i < nfpL; ++i) {
        const double ti[2] = {bL.x[i % nL], dim == 3 ? bL.x[i / nL] : 0.0};
        for (int j = 0; j < nfpH; ++j) {
          const double W = dim == 2 ? bH.w[j] : bH.w[j % nH] * bH.w[j / nH];
          double acc = 0.0;
          for (int k1 = 0; k1 <= (dim == 3 ? pL : 0); ++k1)
            for (int k0 = 0; k0 <= pL; ++k0) {
              double c = 0.5 * (2 * k0 + 1) * legendre(k0, ti[0]) * legendre(k0, tH[size_t(j)][0]);
              if (dim == 3) c *= 0.5 * (2 * k1 + 1) * legendre(k1, ti[1]) * legendre(k1, tH[size_t(j)][1]);
              acc += c;
            }
          P[size_t(i) * nfpH + j] = W * acc;
        }
      }
      for (int i = 0; i < nfpL; ++i) {
        row_out.push_back(int(mf.baseL + i));
        LowRow lr{int(mf.baseL + i), {}, {}};
        for (int j = 0; j < nfpH; ++j) {
          ent_grp.push_back(gH);
          ent_code.push_back(code_of(mf.eH, mf.fH, j));
          ent_w.push_back(P[size_t(i) * nfpH + j]);
          lr.code.push_back(int(mf.baseH + j));
          lr.w.push_back(P[size_t(i) * nfpH + j]);
        }
        row_off.push_back(int(ent_w.size()));
        low.push_back(std::move(lr));
      }
    }
  }
  // projection onto the lower-order sides, per mortar point: MT points and weights
  std::vector<int> po(size_t(std::max<int64_t>(np, 1)) + 1, 0), pc;
  std::vector<double> pw;
  {
    std::vector<const LowRow *> at_point(size_t(std::max<int64_t>(np, 1)), nullptr);
    for (const auto &lr : low) at_point[size_t(lr.out)] = &lr;
    for (size_t q = 0; q < at_point.size(); ++q) {
      if (at_point[q]) {
        pc.insert(pc.end(), at_point[q]->code.begin(), at_point[q]->code.end());
        pw.insert(pw.end(), at_point[q]->w.begin(), at_point[q]->w.end());
      }
      po[q + 1] = int(pw.size());
    }
  }
  if (pw.empty()) {  // keep the tables valid
    pc.push_back(0);
    pw.push_back(0.0);
  }
  // the rows again, per mortar point: each point is the output of exactly one row
  std::vector<int> mo(size_t(std::max<int64_t>(np, 1)) + 1, 0), mg, mc;
  std::vector<double> mw;
  {
    std::vector<int64_t> row_of(size_t(std::max<int64_t>(np, 1)), -1);
    for (size_t r = 0; r < row_out.size(); ++r) row_of[size_t(row_out[r])] = int64_t(r);
    for (size_t q = 0; q < row_of.size(); ++q) {
      const int64_t r = row_of[q];
      if (r >= 0)
        for (int j = row_off[size_t(r)]; j < row_off[size_t(r) + 1]; ++j) {
          mg.push_back(ent_grp[size_t(j)]);
          mc.push_back(ent_code[size_t(j)]);
          mw.push_back(ent_w[size_t(j)]);
        }
      mo[q + 1] = int(mw.size());
    }
  }
  if (mw.empty()) {  // no mortar face: keep the tables valid
    mg.push_back(0);
    mc.push_back(0);
    mw.push_back(0.0);
  }
  M->a.MO = M->upload(mo);
  M->a.MG = M->upload(mg);
  M->a.MC = M->upload(mc);
  M->a.MW = M->upload(mw);
  for (auto &G : M->groups) {
    M->group_uf.push_back(G->a.UF);
    M->group_pv.push_back(G->a.PV);
  }
  M->a.GUF = M->upload(M->group_uf);
  M->a.GPV = M->upload(M->group_pv);
  M->a.PO = M->upload(po);
  M->a.PC = M->upload(pc);
  M->a.PW = M->upload(pw);
  M->a.MT = M->dalloc(size_t(std::max<int64_t>(np, 1)) * (dim + 2) * M->real_size());
  // the groups run the mortar build of the fused kernels (DevArrays::MO set) only when
  // the mesh has mortar points; with one order present they run the one-order build
  if (np == 0) M->a.MO = nullptr;
  for (auto &G : M->groups) {
    G->a.MO = M->a.MO;
    G->a.MG = M->a.MG;
    G->a.MC = M->a.MC;
    G->a.MW = M->a.MW;
    G->a.GUF = M->a.GUF;
    G->a.GPV = M->a.GPV;
    G->a.MT = M->a.MT;
    G->a.PO = M->a.PO;
    G->a.PC = M->a.PC;
    G->a.PW = M->a.PW;
  }
  M->a.flag = (int *)M->dalloc(sizeof(int));
  M->cfg = M->groups[0]->cfg;  // reports the kernel structure of the (first) order group
  hip_check(hipStreamSynchronize(M->stream), "mesh upload");
}


void profile_steps(fr_mesh *m, int64_t steps, double *ms, int64_t *launches);

void drop_graphs(fr_mesh *M) {
  if (M->graph_first) (void)hipGraphExecDestroy(M->graph_first);
  if (M->graph_rest) (void)hipGraphExecDestroy(M->graph_rest);
  if (M->graph_multi) (void)hipGraphExecDestroy(M->graph_multi);
  M->graph_first = M->graph_rest = M->graph_multi = nullptr;
}

void lk(fr_mesh *M, int kernel, int stage, int mode, bool forces) {
  hip_check(launch_kernel(kernel, M->cfg, M->a, stage, mode, forces), "kernel launch");
}

// one RK4 stage (or the residual, mode MODE_RESID) of a variable-order mesh: the
// first fused launch of every group (each forms the other sides' traces at its mortar
// points from the groups' traces), then the second launch group by group from the
// highest order down. A higher-order side interpolates the lower side's half viscous
// fluxes (written by the first launches) to its mortar points and writes its
// transformed common flux there; a lower-order side projects that flux, written by the
// higher group's second launch before its own, onto its points.
void enqueue_stage_mixed(fr_mesh *M, int stage, int mode, bool forces) {
  for (auto &G : M->groups) {
    const bool f = forces && G->nwall > 0;
    lk(G.get(), K_STAGE_A, stage, 0, f);
    if (f) hip_check(launch_force_reduce(G->cfg, G->a), "force reduce");
  }
  for (size_t g = M->groups.size(); g-- > 0;) lk(M->groups[g].get(), K_STAGE_B, stage, mode, false);
}

// one RK4 step; force terms of the step's input state are reduced if `forces`
void enqueue_step(fr_mesh *M, bool forces) {
  if (M->mixed()) {
    for (int s = 0; s < 4; ++s) enqueue_stage_mixed(M, s, s, forces && s == 0);
    return;
  }
  if (M->cfg.variant_mask & FUSED) {
    for (int s = 0; s < 4; ++s) {
      const bool f = forces && s == 0 && M->nwall > 0;
      lk(M, K_STAGE_A, s, 0, f);
      if (f) hip_check(launch_force_reduce(M->cfg, M->a), "force reduce");
      lk(M, K_STAGE_B, s, s, false);
    }
    return;
  }
  for (int s = 0; s < 4; ++s) {
    const bool f = forces && s == 0 && M->nwall > 0;
    lk(M, K_FACE, s, 0, false);
    lk(M, K_GRAD, s, 0, false);
    lk(M, K_VISC, s, 0, f);
    if (f) hip_check(launch_force_reduce(M->cfg, M->a), "force reduce");
    lk(M, K_DIVRK, s, s, false);
    // trace of the next stage input: US for stages 1..3, U after the update
    lk(M, K_INTERP, s < 3 ? 1 : 0, 0, false);
  }
}

// steps captured in one graph: the whole batch advances GRAPH_STEPS RK4 steps per launch
constexpr int64_t GRAPH_STEPS = 8;

hipGraphExec_t capture_step(fr_mesh *M, bool forces, int64_t steps = 1) {
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(M->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    for (int64_t s = 0; s < steps; ++s) enqueue_step(M, forces);
  } catch (...) {
    (void)hipStreamEndCapture(M->stream, &g);  // the launch error is the one reported
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_check(hipStreamEndCapture(M->stream, &g), "end capture");
  hipGraphExec_t ex = nullptr;
  hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  return ex;
}

// The wall forces of the state the last steps left, added to the sums if they are not
// there yet: one force pass over that state (its trace is current) and the reduction.
void flush_forces(fr_mesh *M) {
  if (!M->forces_pending) return;
  hip_check(hipSetDevice(M->device), "hipSetDevice");
  if (M->mixed()) {
    for (auto &G : M->groups)
      if (G->nwall > 0) {
        lk(G.get(), K_STAGE_A, 0, 0, true);
        hip_check(launch_force_reduce(G->cfg, G->a), "force reduce");
      }
  } else if (M->cfg.variant_mask & FUSED) {
    lk(M, K_STAGE_A, 0, 0, true);
    hip_check(launch_force_reduce(M->cfg, M->a), "force reduce");
  } else {
    lk(M, K_FACE, 0, 0, false);
    lk(M, K_GRAD, 0, 0, false);
    lk(M, K_VISC, 0, 0, true);
    hip_check(launch_force_reduce(M->cfg, M->a), "force reduce");
  }
  M->forces_pending = false;
}

// Before anything overwrites the trace or the state outside a step: the pending forces
// are taken while their state and trace are still there, and the next step interpolates
// the trace again.
void release_trace(fr_mesh *M) {
  flush_forces(M);
  M->trace_valid = false;
}

// n steps. The state's trace is interpolated only if no step left it; the first step
// adds the wall forces of its input state to the sums only if the previous steps left
// them pending (the input state of the first step after the state was set is not
// averaged), every later step does. The forces of the last state stay pending.
void step_async(fr_mesh *M, int64_t n, bool clear_flag = true) {
  if (!M->state_set) fail(FR_E_STATE, "no state set");
  if (n < 0) fail(FR_E_ARG, "negative step count");
  if (n == 0) return;
  hip_check(hipSetDevice(M->device), "hipSetDevice");
  if (!M->graph_first) M->graph_first = capture_step(M, false);
  if (!M->graph_rest) M->graph_rest = capture_step(M, true);
  if (!M->graph_multi && n > GRAPH_STEPS) M->graph_multi = capture_step(M, true, GRAPH_STEPS);
  const bool pending = M->forces_pending;
  auto launch_steps = [&] {
    hip_check(hipGraphLaunch(pending ? M->graph_rest : M->graph_first, M->stream), "graph launch");
    int64_t left = n - 1;
    for (; left >= GRAPH_STEPS && M->graph_multi; left -= GRAPH_STEPS)
      hip_check(hipGraphLaunch(M->graph_multi, M->stream), "graph launch");
    for (; left > 0; --left) hip_check(hipGraphLaunch(M->graph_rest, M->stream), "graph launch");
  };
  if (M->mixed()) {
    for (auto &G : M->groups) {
      if (clear_flag) hip_check(launch_clear_flag(G->cfg, G->a), "clear flag");
      if (!M->trace_valid) lk(G.get(), K_INTERP, 0, 0, false);
    }
  } else {
    if (clear_flag) hip_check(launch_clear_flag(M->cfg, M->a), "clear flag");
    if (!M->trace_valid) lk(M, K_INTERP, 0, 0, false);
  }
  launch_steps();
  M->trace_valid = true;
  M->forces_pending = M->nwall > 0;
}

void sync_check(fr_mesh *M) {
  std::vector<int> flags(std::max<size_t>(M->groups.size(), 1), 0);
  if (M->mixed()) {
    for (size_t g = 0; g < M->groups.size(); ++g)
      hip_check(hipMemcpyAsync(&flags[g], M->groups[g]->a.flag, sizeof(int), hipMemcpyDeviceToHost, M->stream),
                "flag copy");
  } else {
    hip_check(hipMemcpyAsync(&flags[0], M->a.flag, sizeof(int), hipMemcpyDeviceToHost, M->stream), "flag copy");
  }
  hip_check(hipStreamSynchronize(M->stream), "stream sync");
  for (int f : flags)
    if (f) fail(FR_E_NONFINITE, "non-finite state after a step");
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fr_last_error(void) { return g_err.c_str(); }

fr_status fr_batch_create(const fr_mesh_desc *descs, int32_t n, fr_mesh **out) {
  return guarded([&] {
    if (!out) fail(FR_E_ARG, "null output");
    *out = nullptr;
    if (!descs || n <= 0) fail(FR_E_ARG, "no descriptors");
    bool mixed = false;
    for (int i = 0; i < n; ++i) mixed = mixed || descs[i].elem_order != nullptr;
    if (mixed) {
      // variable order: designs with and without per-element orders together; each order
      // group covers every design that has elements of its order
      for (int i = 0; i < n; ++i) {
        fr_mesh_desc d = descs[i];
        if (d.elem_order) d.order = 1;  // each element's own order is checked with the groups
        validate_desc(&d);
        const auto &a = descs[0], &b = descs[i];
        if (a.dim != b.dim || a.precision != b.precision || a.gamma != b.gamma || a.prandtl != b.prandtl ||
            a.mu != b.mu || a.device != b.device || a.stream != b.stream)
          fail(FR_E_ARG, "batched designs must share dim, precision, gas constants, device and stream");
      }
      std::unique_ptr<fr_mesh> M(new fr_mesh());
      build_mixed(M.get(), descs, n);
      *out = M.release();
      return;
    }
    for (int i = 0; i < n; ++i) {
      validate_desc(&descs[i]);
      const auto &a = descs[0], &b = descs[i];
      if (a.dim != b.dim || a.order != b.order || a.precision != b.precision || a.gamma != b.gamma ||
          a.prandtl != b.prandtl || a.mu != b.mu || a.device != b.device || a.stream != b.stream)
        fail(FR_E_ARG, "batched designs must share dim, order, precision, gas constants, device and stream");
    }
    std::unique_ptr<fr_mesh> M(new fr_mesh());
    build_solver(M.get(), descs, n);
    *out = M.release();
  });
}

fr_status fr_mesh_create(const fr_mesh_desc *desc, fr_mesh **out) { return fr_batch_create(desc, 1, out); }

void fr_mesh_destroy(fr_mesh *m) { delete m; }

fr_status fr_mesh_info(const fr_mesh *m, int64_t *info) {
  return guarded([&] {
    if (!m || !info) fail(FR_E_ARG, "null argument");
    info[0] = m->dim; info[1] = m->order; info[2] = int64_t(m->designs.size()); info[3] = m->E;
    info[4] = m->dm.nu; info[5] = m->dm.nf; info[6] = m->dm.nv; info[7] = m->prec; info[8] = m->nblk;
    info[9] = int64_t(m->bytes);
    if (m->mixed()) {  // ragged: no single point count per element
      info[4] = info[5] = 0;
      for (auto &G : m->groups) info[9] += int64_t(G->bytes);
    }
  });
}

fr_status fr_design_range(const fr_mesh *m, int32_t design, int64_t *first, int64_t *count) {
  return guarded([&] {
    if (!m || !first || !count || design < 0 || design >= int(m->designs.size())) fail(FR_E_ARG, "bad design");
    *first = m->designs[design].e0;
    *count = m->designs[design].E;
  });
}

fr_status fr_solution_points(const fr_mesh *m, double *xyz) {
  return guarded([&] {
    if (!m || !xyz) fail(FR_E_ARG, "null argument");
    if (m->mixed()) {
      for (int64_t e = 0; e < m->E; ++e) {
        const fr_mesh &G = *m->groups[size_t(m->egroup[size_t(e)])];
        const size_t nu = size_t(G.dm.nu);
        std::memcpy(xyz + m->uoff[size_t(e)] * 3, G.xu.data() + size_t(m->elocal[size_t(e)]) * nu * 3,
                    nu * 3 * sizeof(double));
      }
      return;
    }
    std::memcpy(xyz, m->xu.data(), m->xu.size() * sizeof(double));
  });
}

fr_status fr_mesh_points(const fr_mesh *m, int64_t *n_points) {
  return guarded([&] {
    if (!m || !n_points) fail(FR_E_ARG, "null argument");
    *n_points = m->mixed() ? m->uoff.back() : m->E * m->dm.nu;
  });
}

fr_status fr_neighbours(const fr_mesh *m, int64_t *nbr) {
  return guarded([&] {
    if (!m || !nbr) fail(FR_E_ARG, "null argument");
    if (m->mixed()) fail(FR_E_UNSUPPORTED, "neighbour table of a variable-order mesh");
    std::memcpy(nbr, m->nbr_canon.data(), m->nbr_canon.size() * sizeof(int64_t));
  });
}

fr_status fr_connectivity(const fr_mesh_desc *desc, int64_t *nbr, double *xyz) {
  return guarded([&] {
    if (!nbr) fail(FR_E_ARG, "null argument");
    if (desc && desc->elem_order) fail(FR_E_UNSUPPORTED, "neighbour table of a variable-order mesh");
    validate_desc(desc);
    HostMesh H = build_host_mesh(*desc);
    std::memcpy(nbr, H.nbr.data(), H.nbr.size() * sizeof(int64_t));
    if (xyz) std::memcpy(xyz, H.xu.data(), H.xu.size() * sizeof(double));
  });
}

// the part of a ragged canonical state held by group g, or back
static void split_state(const fr_mesh *m, size_t g, const double *u, double *ug, bool to_group) {
  const int nv = m->dim + 2;
  const fr_mesh &G = *m->groups[g];
  const size_t per = size_t(G.dm.nu) * nv;
  for (int64_t e = 0; e < m->E; ++e) {
    if (m->egroup[size_t(e)] != int(g)) continue;
    double *a = ug + size_t(m->elocal[size_t(e)]) * per;
    const double *b = u + size_t(m->uoff[size_t(e)]) * nv;
    if (to_group)
      std::memcpy(a, b, per * sizeof(double));
    else
      std::memcpy(const_cast<double *>(b), a, per * sizeof(double));
  }
}

fr_status fr_set_state(fr_mesh *m, const double *u) {
  return guarded([&] {
    if (!m || !u) fail(FR_E_ARG, "null argument");
    if (m->mixed()) {
      for (size_t g = 0; g < m->groups.size(); ++g) {
        fr_mesh &G = *m->groups[g];
        std::vector<double> ug(size_t(G.E) * G.dm.nu * G.dm.nv);
        split_state(m, g, u, ug.data(), true);
        const fr_status st = fr_set_state(&G, ug.data());
        if (st != FR_OK) fail(st, g_err);
      }
      m->state_set = true;
      m->trace_valid = m->forces_pending = false;
      return;
    }
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    const size_t n = size_t(m->E) * m->dm.nu * m->dm.nv;
    hip_check(hipMemcpyAsync(m->a.stage64, u, n * sizeof(double), hipMemcpyHostToDevice, m->stream), "state upload");
    hip_check(launch_pack(m->cfg, m->a, true, m->a.U), "pack");
    hip_check(hipMemsetAsync(m->a.fsum, 0, m->designs.size() * 8 * sizeof(double), m->stream), "clear sums");
    hip_check(hipStreamSynchronize(m->stream), "set state");
    m->state_set = true;
    m->trace_valid = m->forces_pending = false;
  });
}

fr_status fr_get_state(const fr_mesh *m, double *u) {
  return guarded([&] {
    if (!m || !u) fail(FR_E_ARG, "null argument");
    if (!m->state_set) fail(FR_E_STATE, "no state set");
    if (m->mixed()) {
      for (size_t g = 0; g < m->groups.size(); ++g) {
        const fr_mesh &G = *m->groups[g];
        std::vector<double> ug(size_t(G.E) * G.dm.nu * G.dm.nv);
        const fr_status st = fr_get_state(&G, ug.data());
        if (st != FR_OK) fail(st, g_err);
        split_state(m, g, u, ug.data(), false);
      }
      return;
    }
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    const size_t n = size_t(m->E) * m->dm.nu * m->dm.nv;
    hip_check(launch_pack(m->cfg, m->a, false, m->a.U), "unpack");
    hip_check(hipMemcpyAsync(u, m->a.stage64, n * sizeof(double), hipMemcpyDeviceToHost, m->stream), "state download");
    hip_check(hipStreamSynchronize(m->stream), "get state");
  });
}

fr_status fr_step_async(fr_mesh *m, int64_t n) {
  return guarded([&] {
    if (!m) fail(FR_E_ARG, "null mesh");
    step_async(m, n);
  });
}

fr_status fr_sync(fr_mesh *m) {
  return guarded([&] {
    if (!m) fail(FR_E_ARG, "null mesh");
    sync_check(m);
  });
}

fr_status fr_step(fr_mesh *m, int64_t n) {
  return guarded([&] {
    if (!m) fail(FR_E_ARG, "null mesh");
    step_async(m, n);
    sync_check(m);
  });
}

fr_status fr_forces(const fr_mesh *m, int32_t design, double *out) {
  return guarded([&] {
    if (!m || !out || design < 0 || design >= int(m->designs.size())) fail(FR_E_ARG, "bad argument");
    flush_forces(const_cast<fr_mesh *>(m));  // the sums are read on the same stream
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (m->mixed()) {  // the design's wall sums in every group add up; their step counts agree
      for (size_t g = 0; g < m->groups.size(); ++g) {
        const fr_mesh &G = *m->groups[g];
        const int gi = m->gdesign[g][size_t(design)];
        if (gi < 0 || G.designs[size_t(gi)].nwall == 0) continue;
        double sg[8];
        hip_check(hipMemcpyAsync(sg, G.a.fsum + 8 * gi, sizeof(sg), hipMemcpyDeviceToHost, m->stream), "forces");
        hip_check(hipStreamSynchronize(m->stream), "forces");
        for (int k : {0, 1, 2, 4, 5, 6}) s[k] += sg[k];
        s[3] = sg[3];
      }
    } else {
      hip_check(hipMemcpyAsync(s, m->a.fsum + 8 * design, sizeof(s), hipMemcpyDeviceToHost, m->stream), "forces");
      hip_check(hipStreamSynchronize(m->stream), "forces");
    }
    const auto &d = m->designs[design];
    double U2 = 0.0;
    for (int k = 1; k <= 3; ++k) U2 += d.fs[k] * d.fs[k];
    const double qref = 0.5 * d.fs[0] * U2 * d.ref_area;
    auto proj = [&](const double *F, const double *dir) {
      return (F[0] * dir[0] + F[1] * dir[1] + F[2] * dir[2]) / qref;
    };
    const double cnt = s[3];
    out[0] = proj(s + 4, d.lift);
    out[1] = proj(s + 4, d.drag);
    out[2] = s[4]; out[3] = s[5]; out[4] = s[6];
    double mean[3] = {0, 0, 0};
    if (cnt > 0)
      for (int k = 0; k < 3; ++k) mean[k] = s[k] / cnt;
    out[5] = cnt > 0 ? proj(mean, d.lift) : 0.0;
    out[6] = cnt > 0 ? proj(mean, d.drag) : 0.0;
    out[7] = cnt;
  });
}

fr_status fr_residual(fr_mesh *m, const double *u, double *r) {
  return guarded([&] {
    if (!m || !u || !r) fail(FR_E_ARG, "null argument");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    release_trace(m);  // the residual's input takes the trace arrays
    if (m->mixed()) {
      std::vector<std::vector<double>> ug(m->groups.size());
      for (size_t g = 0; g < m->groups.size(); ++g) {
        fr_mesh &G = *m->groups[g];
        ug[g].resize(size_t(G.E) * G.dm.nu * G.dm.nv);
        split_state(m, g, u, ug[g].data(), true);
        hip_check(hipMemcpyAsync(G.a.stage64, ug[g].data(), ug[g].size() * sizeof(double), hipMemcpyHostToDevice,
                                 m->stream), "upload");
        hip_check(launch_pack(G.cfg, G.a, true, G.a.US), "pack");
        lk(&G, K_INTERP, 1, 0, false);
      }
      enqueue_stage_mixed(m, 1, MODE_RESID, false);
      for (size_t g = 0; g < m->groups.size(); ++g) {
        fr_mesh &G = *m->groups[g];
        hip_check(launch_pack(G.cfg, G.a, false, G.a.RES), "unpack");
        hip_check(hipMemcpyAsync(ug[g].data(), G.a.stage64, ug[g].size() * sizeof(double), hipMemcpyDeviceToHost,
                                 m->stream), "download");
      }
      hip_check(hipStreamSynchronize(m->stream), "residual");
      for (size_t g = 0; g < m->groups.size(); ++g) split_state(m, g, r, ug[g].data(), false);
      return;
    }
    const size_t n = size_t(m->E) * m->dm.nu * m->dm.nv;
    hip_check(hipMemcpyAsync(m->a.stage64, u, n * sizeof(double), hipMemcpyHostToDevice, m->stream), "upload");
    hip_check(launch_pack(m->cfg, m->a, true, m->a.US), "pack");
    lk(m, K_INTERP, 1, 0, false);
    if (m->cfg.variant_mask & FUSED) {
      lk(m, K_STAGE_A, 1, 0, false);
      lk(m, K_STAGE_B, 1, MODE_RESID, false);
    } else {
      lk(m, K_FACE, 1, 0, false);
      lk(m, K_GRAD, 1, 0, false);
      lk(m, K_VISC, 1, 0, false);
      lk(m, K_DIVRK, 1, MODE_RESID, false);
    }
    hip_check(launch_pack(m->cfg, m->a, false, m->a.RES), "unpack");
    hip_check(hipMemcpyAsync(r, m->a.stage64, n * sizeof(double), hipMemcpyDeviceToHost, m->stream), "download");
    hip_check(hipStreamSynchronize(m->stream), "residual");
  });
}

fr_status fr_state_device(const fr_mesh *m, void **ptr, int64_t *bytes) {
  return guarded([&] {
    if (!m || !ptr || !bytes) fail(FR_E_ARG, "null argument");
    if (m->mixed()) fail(FR_E_UNSUPPORTED, "a variable-order state lives in several arrays");
    release_trace(const_cast<fr_mesh *>(m));  // the caller may write the state through it
    *ptr = m->a.U;
    *bytes = int64_t(m->nblk) * m->dm.nup * m->dm.nv * EB * int64_t(m->real_size());
  });
}

fr_status fr_select_kernels(fr_mesh *m, int32_t mask) {
  return guarded([&] {
    if (!m) fail(FR_E_ARG, "null mesh");
    if (m->mixed()) {
      if (!(unsigned(mask) & FUSED)) fail(FR_E_UNSUPPORTED, "variable-order meshes run the fused stage only");
      return;
    }
    if ((unsigned(mask) & EXTRUDED_METRICS) && !m->extruded)
      fail(FR_E_UNSUPPORTED, "column metrics need a mesh of z-extruded elements");
    if ((unsigned(mask) & TILE_BITS) &&
        (!tiles_compiled(m->dim, m->order, false) || tile_a(unsigned(mask)) >= N_TILES_A ||
         tile_b(unsigned(mask)) >= N_TILES))
      fail(FR_E_UNSUPPORTED, "tile shapes other than the default exist for 3D meshes of order 1 to 4 only");
    if ((unsigned(mask) & SCATTER_EXCHANGE) && !(unsigned(mask) & FUSED))
      fail(FR_E_UNSUPPORTED, "the exchange by scatter belongs to the fused stage");
    release_trace(m);  // the trace layout may change with the structure (exchange by scatter)
    m->cfg.variant_mask = unsigned(mask) & (FUSED | (1u << K_INTERP) | (1u << K_GRAD) | (1u << K_VISC) |
                                            (1u << K_DIVRK) | STORED_METRICS | NO_XCD_REMAP | EXTRUDED_METRICS |
                                            TILE_BITS | SCATTER_EXCHANGE);
    drop_graphs(m);
  });
}

fr_status fr_selected_kernels(const fr_mesh *m, int32_t *mask) {
  return guarded([&] {
    if (!m || !mask) fail(FR_E_ARG, "null argument");
    *mask = int32_t(m->cfg.variant_mask);
  });
}

fr_status fr_autotune(fr_mesh *m, int64_t steps, int32_t *mask_out) {
  return guarded([&] {
    if (!m || steps <= 0) fail(FR_E_ARG, "bad argument");
    if (!m->state_set) fail(FR_E_STATE, "no state set");
    if (m->mixed()) {  // one structure only
      if (mask_out) *mask_out = int32_t(m->cfg.variant_mask);
      return;
    }
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    release_trace(m);  // the timed steps run on a copy of the state and leave their own trace
    const size_t nb = size_t(m->nblk) * m->dm.nup * m->dm.nv * EB * m->real_size();
    // keep the state: time on a copy, restore it afterwards
    hip_check(hipMemcpyAsync(m->a.RES, m->a.U, nb, hipMemcpyDeviceToDevice, m->stream), "save state");
    const unsigned all = (1u << K_INTERP) | (1u << K_GRAD) | (1u << K_VISC) | (1u << K_DIVRK);
    double ms_dense[8], ms_tensor[8], ms_fused[8];
    int64_t n[8];
    m->cfg.variant_mask = 0;
    profile_steps(m, steps, ms_dense, n);
    hip_check(hipMemcpyAsync(m->a.U, m->a.RES, nb, hipMemcpyDeviceToDevice, m->stream), "restore state");
    m->cfg.variant_mask = all;
    profile_steps(m, steps, ms_tensor, n);
    hip_check(hipMemcpyAsync(m->a.U, m->a.RES, nb, hipMemcpyDeviceToDevice, m->stream), "restore state");
    // the fused stage: in 3D with each metric source the mesh allows, each with the tiles
    // of consecutive blocks remapped onto one XCD or not, and the neighbour exchange by
    // gather or by scatter
    double fused = 1e300;
    unsigned fused_mask = FUSED | (1u << K_INTERP);
    for (unsigned metrics : {0u, STORED_METRICS, EXTRUDED_METRICS}) {
      if (metrics && m->dim != 3) continue;
      if (metrics == EXTRUDED_METRICS && !m->extruded) continue;
      for (unsigned shape : {0u, NO_XCD_REMAP, SCATTER_EXCHANGE, NO_XCD_REMAP | SCATTER_EXCHANGE}) {
        m->cfg.variant_mask = FUSED | (1u << K_INTERP) | metrics | shape;
        profile_steps(m, steps, ms_fused, n);
        hip_check(hipMemcpyAsync(m->a.U, m->a.RES, nb, hipMemcpyDeviceToDevice, m->stream), "restore state");
        const double t = ms_fused[K_STAGE_A] + ms_fused[K_STAGE_B];
        if (t < fused) {
          fused = t;
          fused_mask = m->cfg.variant_mask;
        }
      }
    }
    // tile shapes of the two fused launches, each timed on its own kernel with the other
    // launch at the shape chosen so far
    if (tiles_compiled(m->dim, m->order, false)) {
      double best_a = 1e300, best_b = 1e300;
      int ta_best = 0, tb_best = 0;
      for (int ta = 0; ta < N_TILES_A; ++ta) {
        m->cfg.variant_mask = (fused_mask & ~TILE_BITS) | tile_bits(ta, 0);
        profile_steps(m, steps, ms_fused, n);
        hip_check(hipMemcpyAsync(m->a.U, m->a.RES, nb, hipMemcpyDeviceToDevice, m->stream), "restore state");
        if (ms_fused[K_STAGE_A] < best_a) {
          best_a = ms_fused[K_STAGE_A];
          ta_best = ta;
        }
        if (ta == 0) best_b = ms_fused[K_STAGE_B];
      }
      for (int tb = 1; tb < N_TILES; ++tb) {
        m->cfg.variant_mask = (fused_mask & ~TILE_BITS) | tile_bits(ta_best, tb);
        profile_steps(m, steps, ms_fused, n);
        hip_check(hipMemcpyAsync(m->a.U, m->a.RES, nb, hipMemcpyDeviceToDevice, m->stream), "restore state");
        if (ms_fused[K_STAGE_B] < best_b) {
          best_b = ms_fused[K_STAGE_B];
          tb_best = tb;
        }
      }
      fused_mask = (fused_mask & ~TILE_BITS) | tile_bits(ta_best, tb_best);
      fused = std::min(fused, best_a + best_b);
    }
    unsigned mask = 0;
    double split = ms_dense[K_FACE];
    for (int k : {int(K_INTERP), int(K_GRAD), int(K_VISC), int(K_DIVRK)}) {
      if (ms_tensor[k] < ms_dense[k]) mask |= 1u << k;
      split += std::min(ms_tensor[k], ms_dense[k]);
    }
    if (fused < split) mask = fused_mask;
    m->cfg.variant_mask = mask;
    {
      std::lock_guard<std::mutex> lock(g_tuned_mu);
      g_tuned[tune_key(m->prec, m->dim, m->order, m->nblk)] = mask;
    }
    drop_graphs(m);
    hip_check(hipStreamSynchronize(m->stream), "autotune");
    if (mask_out) *mask_out = int32_t(mask);
  });
}

fr_status fr_profile_kernels(fr_mesh *m, int64_t steps, double *ms, int64_t *launches) {
  return guarded([&] {
    if (!m || !ms || !launches || steps <= 0) fail(FR_E_ARG, "bad argument");
    if (m->mixed()) fail(FR_E_UNSUPPORTED, "per-kernel profile of a variable-order mesh");
    if (!m->state_set) fail(FR_E_STATE, "no state set");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    release_trace(m);  // the profiled steps advance the state and leave no force sums
    profile_steps(m, steps, ms, launches);
  });
}

}  // extern "C"

namespace {
void profile_steps(fr_mesh *m, int64_t steps, double *ms, int64_t *launches) {
  {
    for (int k = 0; k < 8; ++k) { ms[k] = 0.0; launches[k] = 0; }
    std::vector<hipEvent_t> ev;
    std::vector<int> kid;
    auto timed = [&](int kernel, int stage, int mode, bool forces) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "event");
      hip_check(hipEventCreate(&b), "event");
      hip_check(hipEventRecord(a, m->stream), "event");
      lk(m, kernel, stage, mode, forces);
      hip_check(hipEventRecord(b, m->stream), "event");
      ev.push_back(a);
      ev.push_back(b);
      kid.push_back(kernel);
    };
    hip_check(launch_clear_flag(m->cfg, m->a), "clear flag");
    lk(m, K_INTERP, 0, 0, false);
    for (int64_t s = 0; s < steps; ++s)
      for (int st = 0; st < 4; ++st) {
        if (m->cfg.variant_mask & FUSED) {
          timed(K_STAGE_A, st, 0, false);
          timed(K_STAGE_B, st, st, false);
          continue;
        }
        timed(K_FACE, st, 0, false);
        timed(K_GRAD, st, 0, false);
        timed(K_VISC, st, 0, false);
        timed(K_DIVRK, st, st, false);
        timed(K_INTERP, st < 3 ? 1 : 0, 0, false);
      }
    sync_check(m);
    for (size_t i = 0; i < kid.size(); ++i) {
      float t = 0.f;
      hip_check(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]), "elapsed");
      ms[kid[i]] += t;
      ms[0] += t;
      launches[kid[i]] += 1;
      launches[0] += 1;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
  }
}
}  // namespace

void fr::set_last_error(const char *msg) { g_err = msg ? msg : ""; }

bool fr::desc_extruded(const fr_mesh_desc &d) {
  if (d.dim != 3) return false;
  for (int64_t e = 0; e < d.n_elems; ++e)
    if (!elem_extruded(d, e)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// sampling the solution at points
// ---------------------------------------------------------------------------
struct fr_probe {
  fr_mesh *m = nullptr;
  int64_t n = 0;
  std::vector<int64_t> elem;  // canonical element within the design
  std::vector<double> xi;     // [n][3]
  int64_t *slot = nullptr;    // device [n]: block * EB + element slot
  double *w = nullptr;        // device [n][dim][order + 1]
  double *out = nullptr;      // device [n][nv]
  // variable-order mesh: the points in each order group, evaluated by that group's
  // kernel into their rows of `out`
  struct Part {
    int group = 0;
    int64_t n = 0;
    int64_t *slot = nullptr, *dst = nullptr;
    double *w = nullptr;
  };
  std::vector<Part> parts;
  ~fr_probe() {
    (void)hipFree(slot);
    (void)hipFree(w);
    (void)hipFree(out);
    for (auto &q : parts) {
      (void)hipFree(q.slot);
      (void)hipFree(q.dst);
      (void)hipFree(q.w);
    }
  }
};

namespace {

// x(r) = p by Newton's method from the element centre; true with r when the
// iteration converges inside the reference cube (tolerance 1e-10). Converged: a step
// below 1e-14, or below 1e-10 and no smaller than the one before (the round-off floor,
// which in thin curved elements lies above 1e-14)
bool locate_in(const fr_mesh_desc &d, int64_t e, const double *p, std::array<double, 3> &r) {
  const int dim = d.dim;
  r = {0.0, 0.0, 0.0};
  double prev = INFINITY;
  for (int it = 0; it < 50; ++it) {
    double x[3], a[3][3];
    geom_map(d, e, r, x, a);
    double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, b[3] = {0, 0, 0};  // J[i][k] = dx_i / dr_k
    for (int i = 0; i < dim; ++i) {
      b[i] = p[i] - x[i];
      for (int k = 0; k < dim; ++k) J[i][k] = a[k][i];
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(std::fabs(det) > 0.0)) return false;
    double dr[3];
    for (int k = 0; k < 3; ++k) {  // Cramer's rule
      double M[3][3];
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) M[i][c] = c == k ? b[i] : J[i][c];
      dr[k] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
               M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
    }
    double step = 0.0, big = 0.0;
    for (int k = 0; k < dim; ++k) {
      r[k] += dr[k];
      step = std::max(step, std::fabs(dr[k]));
      big = std::max(big, std::fabs(r[k]));
    }
    if (step < 1e-14 || (step < 1e-10 && step >= prev)) {
      for (int k = 0; k < dim; ++k)
        if (std::fabs(r[k]) > 1.0 + 1e-10) return false;
      return true;
    }
    if (big > 3.0) return false;
    prev = step;
  }
  return false;
}

}  // namespace

extern "C" {

fr_status fr_probe_create(fr_mesh *m, const fr_mesh_desc *desc, int32_t design, int64_t n, const double *points,
                          fr_probe **out) {
  return guarded([&] {
    if (!out) fail(FR_E_ARG, "null output");
    *out = nullptr;
    if (!m || !desc || n <= 0 || !points || design < 0 || design >= int(m->designs.size()))
      fail(FR_E_ARG, "bad argument");
    if (!m->mixed() && desc->elem_order) fail(FR_E_ARG, "descriptor does not match the mesh design");
    if (m->mixed()) {
      fr_mesh_desc d1 = *desc;
      d1.order = 1;
      validate_desc(&d1);
    } else {
      validate_desc(desc);
    }
    const auto &ds = m->designs[design];
    if (desc->n_elems != ds.E || desc->dim != m->dim || (!m->mixed() && desc->order != m->order))
      fail(FR_E_ARG, "descriptor does not match the mesh design");
    const int dim = desc->dim, na = desc->geom_order + 1;
    const int nn = dim == 2 ? na * na : na * na * na;
    const int64_t E = desc->n_elems;
    // padded node bounding boxes and a uniform grid of about E cells over them
    std::vector<double> lo(size_t(E) * 3, 0.0), hi(size_t(E) * 3, 0.0);
    double glo[3] = {INFINITY, INFINITY, INFINITY}, ghi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t e = 0; e < E; ++e) {
      double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int a = 0; a < nn; ++a) {
        const double *X = desc->nodes + desc->elem_nodes[e * nn + a] * dim;
        for (int i = 0; i < dim; ++i) {
          l[i] = std::min(l[i], X[i]);
          h[i] = std::max(h[i], X[i]);
        }
      }
      double ext = 0.0;
      for (int i = 0; i < dim; ++i) ext = std::max(ext, h[i] - l[i]);
      for (int i = 0; i < dim; ++i) {
        lo[e * 3 + i] = l[i] - 0.1 * ext;
        hi[e * 3 + i] = h[i] + 0.1 * ext;
        glo[i] = std::min(glo[i], lo[e * 3 + i]);
        ghi[i] = std::max(ghi[i], hi[e * 3 + i]);
      }
    }
    const int cells = std::max(1, int(std::pow(double(E), 1.0 / dim)));
    auto cell = [&](int i, double x) {
      const int c = int((x - glo[i]) / (ghi[i] - glo[i]) * cells);
      return std::min(std::max(c, 0), cells - 1);
    };
    const int64_t ncell = dim == 2 ? int64_t(cells) * cells : int64_t(cells) * cells * cells;
    std::vector<std::vector<int64_t>> grid(static_cast<size_t>(ncell));
    for (int64_t e = 0; e < E; ++e) {
      int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
      for (int i = 0; i < dim; ++i) {
        c0[i] = cell(i, lo[e * 3 + i]);
        c1[i] = cell(i, hi[e * 3 + i]);
      }
      for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
          for (int x = c0[0]; x <= c1[0]; ++x) grid[size_t(x + cells * (y + int64_t(cells) * z))].push_back(e);
    }
    auto *p = new fr_probe();
    try {
      p->m = m;
      p->n = n;
      p->elem.assign(size_t(n), -1);
      p->xi.assign(size_t(n) * 3, 0.0);
      std::vector<int> bad(size_t(n), 0);
      parallel_for(n, [&](int64_t i) {
        const double *x = points + i * 3;
        int c[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) c[k] = cell(k, x[k]);
        const auto &cand = grid[size_t(c[0] + cells * (c[1] + int64_t(cells) * c[2]))];  // ascending
        for (int64_t e : cand) {
          bool in = true;
          for (int k = 0; k < dim; ++k) in = in && x[k] >= lo[e * 3 + k] && x[k] <= hi[e * 3 + k];
          std::array<double, 3> r;
          if (in && locate_in(*desc, e, x, r)) {
            p->elem[size_t(i)] = e;
            for (int k = 0; k < 3; ++k) p->xi[size_t(i) * 3 + k] = r[k];
            return;
          }
        }
        bad[size_t(i)] = 1;
      });
      for (int64_t i = 0; i < n; ++i)
        if (bad[size_t(i)]) fail(FR_E_ARG, "point " + std::to_string(i) + " lies in no element");
      hip_check(hipSetDevice(m->device), "hipSetDevice");
      if (m->mixed()) {
        hip_check(hipMalloc(&p->out, size_t(n) * (dim + 2) * sizeof(double)), "probe alloc");
        for (size_t g = 0; g < m->groups.size(); ++g) {
          const fr_mesh &G = *m->groups[g];
          Basis1D B(G.order);
          std::vector<int64_t> slot, dst;
          std::vector<double> w;
          for (int64_t i = 0; i < n; ++i) {
            const int64_t e = ds.e0 + p->elem[size_t(i)];
            if (m->egroup[size_t(e)] != int(g)) continue;
            slot.push_back(m->eslot[size_t(e)]);
            dst.push_back(i);
            for (int k = 0; k < dim; ++k) {
              const auto l = B.eval_all(p->xi[size_t(i) * 3 + k]);
              w.insert(w.end(), l.begin(), l.end());
            }
          }
          if (slot.empty()) continue;
          fr_probe::Part q;
          q.group = int(g);
          q.n = int64_t(slot.size());
          p->parts.push_back(q);
          auto &pq = p->parts.back();
          hip_check(hipMalloc(&pq.slot, slot.size() * sizeof(int64_t)), "probe alloc");
          hip_check(hipMalloc(&pq.dst, dst.size() * sizeof(int64_t)), "probe alloc");
          hip_check(hipMalloc(&pq.w, w.size() * sizeof(double)), "probe alloc");
          hip_check(hipMemcpyAsync(pq.slot, slot.data(), slot.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                                   m->stream), "probe upload");
          hip_check(hipMemcpyAsync(pq.dst, dst.data(), dst.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                                   m->stream), "probe upload");
          hip_check(hipMemcpyAsync(pq.w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, m->stream),
                    "probe upload");
          hip_check(hipStreamSynchronize(m->stream), "probe sync");
        }
        *out = p;
        return;
      }
      const int N = m->order + 1;
      Basis1D B(m->order);
      std::vector<int64_t> slot(static_cast<size_t>(n));
      std::vector<double> w(size_t(n) * dim * N);
      for (int64_t i = 0; i < n; ++i) {
        const int64_t le = p->elem[size_t(i)];
        slot[size_t(i)] = (ds.blk0 + le / EB) * EB + le % EB;
        for (int k = 0; k < dim; ++k) {
          const auto l = B.eval_all(p->xi[size_t(i) * 3 + k]);
          for (int j = 0; j < N; ++j) w[(size_t(i) * dim + k) * N + j] = l[j];
        }
      }
      hip_check(hipMalloc(&p->slot, slot.size() * sizeof(int64_t)), "probe alloc");
      hip_check(hipMalloc(&p->w, w.size() * sizeof(double)), "probe alloc");
      hip_check(hipMalloc(&p->out, size_t(n) * m->dm.nv * sizeof(double)), "probe alloc");
      hip_check(hipMemcpyAsync(p->slot, slot.data(), slot.size() * sizeof(int64_t), hipMemcpyHostToDevice, m->stream),
                "probe upload");
      hip_check(hipMemcpyAsync(p->w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, m->stream),
                "probe upload");
      hip_check(hipStreamSynchronize(m->stream), "probe sync");
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

void fr_probe_destroy(fr_probe *p) { delete p; }

fr_status fr_probe_locate(const fr_probe *p, int64_t *elem, double *xi) {
  return guarded([&] {
    if (!p || !elem || !xi) fail(FR_E_ARG, "null argument");
    std::memcpy(elem, p->elem.data(), p->elem.size() * sizeof(int64_t));
    std::memcpy(xi, p->xi.data(), p->xi.size() * sizeof(double));
  });
}

fr_status fr_probe_sample(fr_probe *p, double *out) {
  return guarded([&] {
    if (!p || !out) fail(FR_E_ARG, "null argument");
    fr::ProbeRun r{};
    const fr_status st = fr::probe_run(p, true, &r);
    if (st != FR_OK) fail(st, g_err);
    hip_check(hipMemcpy(out, r.out, size_t(r.n) * r.nv * sizeof(double), hipMemcpyDeviceToHost), "probe copy");
  });
}

}  // extern "C"

fr_status fr::probe_run(::fr_probe *p, bool wait, ProbeRun *out) {
  return guarded([&] {
    if (!p || !out) fail(FR_E_ARG, "null argument");
    fr_mesh *m = p->m;
    if (!m->state_set) fail(FR_E_STATE, "no state set");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    if (m->mixed()) {
      for (const auto &q : p->parts) {
        const fr_mesh &G = *m->groups[size_t(q.group)];
        hip_check(launch_probe(G.cfg, G.a, q.n, q.slot, q.w, q.dst, p->out), "probe kernel");
      }
    } else {
      hip_check(launch_probe(m->cfg, m->a, p->n, p->slot, p->w, nullptr, p->out), "probe kernel");
    }
    if (wait) hip_check(hipStreamSynchronize(m->stream), "probe sync");
    *out = ProbeRun{p->out, p->n, m->dim + 2, m->dim, m->gamma, m->stream};
  });
}

fr_status fr::step_enqueue(::fr_mesh *m, int64_t n, bool clear_flag) {
  return guarded([&] {
    if (!m) fail(FR_E_ARG, "null mesh");
    step_async(m, n, clear_flag);
  });
}

fr_status fr::means_clear(::fr_mesh *m) {
  return guarded([&] {
    if (!m) fail(FR_E_ARG, "null mesh");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    m->forces_pending = false;  // the current state is not part of the new means
    if (m->mixed()) {  // every order group keeps its own wall sums
      for (auto &G : m->groups)
        hip_check(hipMemsetAsync(G->a.fsum, 0, G->designs.size() * 8 * sizeof(double), m->stream), "clear sums");
      return;
    }
    hip_check(hipMemsetAsync(m->a.fsum, 0, m->designs.size() * 8 * sizeof(double), m->stream), "clear sums");
  });
}

size_t fr::probe_footprint(int64_t n, int dim, int order) {
  // slot, interpolation weights and output buffer of fr_probe_create
  return size_t(n) * (sizeof(int64_t) + size_t(dim) * (order + 1) * sizeof(double) + (dim + 2) * sizeof(double));
}
