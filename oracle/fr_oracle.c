/*
 * fr_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the flux reconstruction (FR)
 * residual of the compressible Navier-Stokes equations, its classic RK4
 * update and the wall force integral.  Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this file; the product path never
 * does.  It shares no source with the GPU library.
 *
 * What it follows
 *   - Governing equations: the paper's Section 2.1, Eqs. (1)-(7): conserved
 *     variables (rho, rho u_i, rho E), inviscid flux, viscous flux, ideal-gas
 *     pressure, Stokes stress and the enthalpy-gradient heat flux with
 *     gamma = 1.4.  The printed energy entry of the viscous flux carries a
 *     sign that is inconsistent with dU/dt + div F = 0 and with the momentum
 *     entry; the reading used is F = F_inv - F_vis with
 *     F_vis,j = (0, tau_ij, u_i tau_ij - q_j).
 *   - Spatial scheme: FR in the Huynh (2007) form that the paper cites for
 *     its solver (Section 1).  The paper gives no FR details, so the standard
 *     choices are taken: Gauss-Legendre solution points in a tensor product,
 *     flux points on the faces where the solution-point lines meet them,
 *     g_DG (Radau) correction functions, Rusanov inviscid common flux with
 *     the larger of the two one-sided wave speeds, BR1 common solution and
 *     common viscous flux (arithmetic means, no penalty), and the
 *     discontinuous normal flux taken from the interpolant of the
 *     transformed flux.
 *   - Time scheme: classic four-stage RK4 with a fixed step.  (The paper
 *     uses a second-order optimal RK scheme with adaptive steps, Section
 *     3.1; its coefficients are not given.)
 *   - Boundaries: periodic pairs by translation; Riemann-invariant far field
 *     (the paper names it for its Appendix D box); no-slip adiabatic wall.
 *   - Wall force: integral of (p n - tau . n) over wall faces with n the
 *     element's outward normal (pointing from the fluid into the body); the
 *     time-averaged lift and drag of Section 3.2 are means of its
 *     projections.
 *
 * Everything is written as plain loops over elements, lines and points in
 * the order the method defines them; there is no blocking or fusion.
 * Compile with -O2 -ffp-contract=off (no fused multiply-adds).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 8       /* up to order 7 */
#define BC_WALL 1
#define BC_FARFIELD 2

/* 1D basis of one order on [-1,1] */
typedef struct {
  int n;
  double xi[MAXN], w[MAXN];
  double D[MAXN][MAXN];      /* D[i][j] = l_j'(xi_i) */
  double lm[MAXN], lp[MAXN]; /* l_j(-1), l_j(+1) */
  double gLd[MAXN], gRd[MAXN];
} orc_basis1d;

/* a face shared by elements of different orders: A has the higher order;
 * corner c of A's face sits at corner pi[c] of B's face */
typedef struct {
  long eA, eB;
  int fA, fB;
  int pi[4];
} orc_mortar;

typedef struct {
  int dim, order, q, nv;     /* order: the largest element order */
  long E, nnodes;
  double gamma, pr, mu;
  double fs[5];              /* free stream: rho, vx, vy, vz, p */
  orc_basis1d bas[MAXN];     /* by order */
  int *ord;                  /* [E] element order */
  long *uo, *fo;             /* [E+1] first solution / flux point of each element */
  long NU, NF;               /* solution and flux points of the mesh */
  /* geometry; element e owns points uo[e] .. uo[e+1]-1 and fo[e] .. fo[e+1]-1 */
  double *S;    /* [NU][3][3]  S[k][j] = |J| dxi_k/dx_j */
  double *detJ; /* [NU] */
  double *xu;   /* [NU][3] */
  double *fnv;  /* [NF][3] outward unit normal */
  double *fA;   /* [NF] |S^T n_hat| */
  double *fxyz; /* [NF][3] */
  long *nbr;    /* [NF] partner flux point, -BC kind, or -(MORTAR0 + mortar index) */
  long nmortar;
  orc_mortar *mortar;
  /* scratch */
  double *uf, *gu, *guf;
  int mock;
  double mock_lambda;
} orc_mesh;

#define MORTAR0 4

/* per-element sizes */
static int el_n(const orc_mesh *M, long e) { return M->ord[e] + 1; }
static int el_nu(const orc_mesh *M, long e) { return (int)(M->uo[e + 1] - M->uo[e]); }
static int el_nfp(const orc_mesh *M, long e) { int n = el_n(M, e); return M->dim == 2 ? n : n * n; }
static int el_nf(const orc_mesh *M, long e) { return (int)(M->fo[e + 1] - M->fo[e]); }

/* ------------------------------------------------------------------ */
/* 1D basis                                                           */
/* ------------------------------------------------------------------ */

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence */
static void legendre(int n, double x, double *P, double *dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1; /* P'_k = P'_{k-2} + (2k-1) P_{k-1} */
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

static double lagrange(int n, const double *x, int j, double t) {
  double v = 1.0;
  for (int m = 0; m < n; ++m)
    if (m != j) v *= (t - x[m]) / (x[j] - x[m]);
  return v;
}

/* derivative of the product form: sum over the dropped factor */
static double lagrange_d(int n, const double *x, int j, double t) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    if (k == j) continue;
    double v = 1.0 / (x[j] - x[k]);
    for (int m = 0; m < n; ++m)
      if (m != j && m != k) v *= (t - x[m]) / (x[j] - x[m]);
    s += v;
  }
  return s;
}

int orc_basis(int order, double *xi, double *w, double *D, double *lm, double *lp,
              double *gLd, double *gRd) {
  int n = order + 1;
  if (order < 0 || n > MAXN) return -1;
  /* Gauss-Legendre nodes: roots of P_n by Newton from the cosine guess */
  double x[MAXN], ww[MAXN];
  for (int i = 0; i < n; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, &P, &dP);
      double dt = P / dP;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(n, t, &P, &dP);
    x[n - 1 - i] = t;
    ww[n - 1 - i] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
  for (int i = 0; i < n; ++i) { xi[i] = x[i]; w[i] = ww[i]; }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) D[i * n + j] = lagrange_d(n, x, j, x[i]);
  for (int j = 0; j < n; ++j) {
    lm[j] = lagrange(n, x, j, -1.0);
    lp[j] = lagrange(n, x, j, 1.0);
  }
  /* g_R = (P_p + P_{p+1})/2 (right Radau correction), g_L(x) = g_R(-x) */
  for (int i = 0; i < n; ++i) {
    double P, dPa, dPb;
    legendre(order, x[i], &P, &dPa);
    legendre(order + 1, x[i], &P, &dPb);
    gRd[i] = 0.5 * (dPa + dPb);
    legendre(order, -x[i], &P, &dPa);
    legendre(order + 1, -x[i], &P, &dPb);
    gLd[i] = -0.5 * (dPa + dPb);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* index helpers                                                      */
/* ------------------------------------------------------------------ */

/* solution point index of the point on face-line (k, m) with i_k = j, n points per line */
static int line_pt(const orc_mesh *M, int n, int k, int m, int j) {
  if (M->dim == 2) {
    if (k == 0) return j + n * m;
    return m + n * j;
  }
  int a = m % n, b = m / n;
  if (k == 0) return j + n * a + n * n * b;
  if (k == 1) return a + n * j + n * n * b;
  return a + n * b + n * n * j;
}

/* position of solution point i along axis k, and its face-line index m */
static void pt_line(const orc_mesh *M, int n, int i, int k, int *ik, int *m) {
  int c[3] = {i % n, (i / n) % n, i / (n * n)};
  *ik = c[k];
  if (M->dim == 2) { *m = (k == 0) ? c[1] : c[0]; return; }
  if (k == 0) *m = c[1] + n * c[2];
  else if (k == 1) *m = c[0] + n * c[2];
  else *m = c[0] + n * c[1];
}

/* reference coordinates of flux point (face f, face point m) of an element with basis B */
static void fpt_ref(const orc_mesh *M, const orc_basis1d *B, int f, int m, double r[3]) {
  int k = f / 2, s = f % 2, n = B->n;
  r[0] = r[1] = r[2] = 0.0;
  r[k] = s ? 1.0 : -1.0;
  if (M->dim == 2) { r[1 - k] = B->xi[m]; return; }
  int a = m % n, b = m / n;
  int ax0 = (k == 0) ? 1 : 0, ax1 = (k == 2) ? 1 : 2;
  r[ax0] = B->xi[a];
  r[ax1] = B->xi[b];
}

/* face coordinates of face point m (along the face's first and second axis) */
static void face_coords(const orc_mesh *M, const orc_basis1d *B, int m, double s[2]) {
  if (M->dim == 2) { s[0] = B->xi[m]; s[1] = 0.0; return; }
  s[0] = B->xi[m % B->n];
  s[1] = B->xi[m / B->n];
}

/* face coordinates of face corner c */
static void corner_coords(int dim, int c, double t[2]) {
  if (dim == 2) { t[0] = c ? 1.0 : -1.0; t[1] = 0.0; return; }
  t[0] = (c & 1) ? 1.0 : -1.0;
  t[1] = ((c >> 1) & 1) ? 1.0 : -1.0;
}

/* coordinates on B's face of the point at s on A's face, when corner c of A's
 * face sits at corner pi[c] of B's: the affine map through corners 0, 1 (and 2) */
static void map_face(int dim, const int *pi, const double s[2], double t[2]) {
  double T0[2], T1[2], T2[2];
  corner_coords(dim, pi[0], T0);
  corner_coords(dim, pi[1], T1);
  if (dim == 2) {
    t[0] = T0[0] + 0.5 * (s[0] + 1.0) * (T1[0] - T0[0]);
    t[1] = 0.0;
    return;
  }
  corner_coords(dim, pi[2], T2);
  for (int i = 0; i < 2; ++i)
    t[i] = T0[i] + 0.5 * (s[0] + 1.0) * (T1[i] - T0[i]) + 0.5 * (s[1] + 1.0) * (T2[i] - T0[i]);
}

/* ------------------------------------------------------------------ */
/* geometry                                                           */
/* ------------------------------------------------------------------ */

static void shape1d(int q, double t, double *N, double *dN) {
  double nodes[3];
  for (int a = 0; a <= q; ++a) nodes[a] = -1.0 + 2.0 * a / q;
  for (int a = 0; a <= q; ++a) {
    N[a] = lagrange(q + 1, nodes, a, t);
    dN[a] = lagrange_d(q + 1, nodes, a, t);
  }
}

/* x(r) and J = dx/dr for element e at reference point r */
static void map_point(const orc_mesh *M, const double *nodes, const long *en, long e,
                      const double r[3], double x[3], double J[3][3]) {
  int q = M->q, d = M->dim, na = q + 1;
  double N[3][3], dN[3][3];
  for (int k = 0; k < d; ++k) shape1d(q, r[k], N[k], dN[k]);
  for (int i = 0; i < 3; ++i) {
    x[i] = 0.0;
    for (int j = 0; j < 3; ++j) J[i][j] = (i == j && i >= d) ? 1.0 : 0.0;
  }
  int nn = (d == 2) ? na * na : na * na * na;
  for (int a = 0; a < nn; ++a) {
    int ac[3] = {a % na, (a / na) % na, a / (na * na)};
    long id = en[e * nn + a];
    double val = 1.0, der[3];
    for (int k = 0; k < d; ++k) val *= N[k][ac[k]];
    for (int j = 0; j < d; ++j) {
      der[j] = 1.0;
      for (int k = 0; k < d; ++k) der[j] *= (k == j) ? dN[k][ac[k]] : N[k][ac[k]];
    }
    for (int i = 0; i < d; ++i) {
      double xa = nodes[id * d + i];
      x[i] += val * xa;
      for (int j = 0; j < d; ++j) J[i][j] += der[j] * xa;
    }
  }
}

/* S = adj(J) = |J| J^{-1}, returns |J| */
static double adjugate(int d, double J[3][3], double S[3][3]) {
  memset(S, 0, 9 * sizeof(double));
  if (d == 2) {
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    S[0][0] = J[1][1];
    S[0][1] = -J[0][1];
    S[1][0] = -J[1][0];
    S[1][1] = J[0][0];
    return det;
  }
  S[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  S[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  S[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  S[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  S[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  S[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  S[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  S[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  S[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * S[0][0] + J[0][1] * S[1][0] + J[0][2] * S[2][0];
}

/* ------------------------------------------------------------------ */
/* face matching                                                      */
/* ------------------------------------------------------------------ */

/* element-local node index of face corner c of face f */
static int corner_node(const orc_mesh *M, int f, int c) {
  int k = f / 2, s = f % 2, q = M->q, na = q + 1;
  int a[3] = {0, 0, 0};
  a[k] = s * q;
  if (M->dim == 2) {
    a[1 - k] = c * q;
    return a[0] + na * a[1];
  }
  int ax0 = (k == 0) ? 1 : 0, ax1 = (k == 2) ? 1 : 2;
  a[ax0] = (c & 1) * q;
  a[ax1] = ((c >> 1) & 1) * q;
  return a[0] + na * a[1] + na * na * a[2];
}

typedef struct { long key[4]; long e; int f; } face_rec;

static int cmp_face(const void *pa, const void *pb) {
  const face_rec *a = pa, *b = pb;
  for (int i = 0; i < 4; ++i) {
    if (a->key[i] < b->key[i]) return -1;
    if (a->key[i] > b->key[i]) return 1;
  }
  if (a->e != b->e) return a->e < b->e ? -1 : 1;
  return a->f - b->f;
}

static void sort4(long *v, int n) {
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && v[j - 1] > v[j]; --j) { long t = v[j]; v[j] = v[j - 1]; v[j - 1] = t; }
}

/* corner c of A sits at corner pi[c] of B; write the face-point map (n points per line) */
static int face_perm(const orc_mesh *M, int n, const int *pi, int *mp) {
  int d = M->dim;
  if (d == 2) {
    /* corners 0,1 are the ends of the line; pi[0] is where A's start lands */
    for (int a = 0; a < n; ++a) mp[a] = pi[0] == 0 ? a : n - 1 - a;
    return 0;
  }
  int o[2] = {pi[0] & 1, (pi[0] >> 1) & 1};
  int u[2] = {(pi[1] & 1) - o[0], ((pi[1] >> 1) & 1) - o[1]};
  int v[2] = {(pi[2] & 1) - o[0], ((pi[2] >> 1) & 1) - o[1]};
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      int c0 = o[0] * (n - 1) + a * u[0] + b * v[0];
      int c1 = o[1] * (n - 1) + a * u[1] + b * v[1];
      if (c0 < 0 || c0 >= n || c1 < 0 || c1 >= n) return -1;
      mp[a + n * b] = c0 + n * c1;
    }
  return 0;
}

/* growable list of mortar faces (filled while faces are matched) */
static int add_mortar(orc_mesh *M, long eA, int fA, long eB, int fB, const int *pi) {
  int nc = M->dim == 2 ? 2 : 4;
  orc_mortar r;
  if (M->ord[eA] > M->ord[eB]) {
    r.eA = eA; r.fA = fA; r.eB = eB; r.fB = fB;
    for (int c = 0; c < 4; ++c) r.pi[c] = c < nc ? pi[c] : 0;
  } else { /* B is the higher order: invert the corner map */
    r.eA = eB; r.fA = fB; r.eB = eA; r.fB = fA;
    for (int c = 0; c < 4; ++c) r.pi[c] = 0;
    for (int c = 0; c < nc; ++c) r.pi[pi[c]] = c;
  }
  if ((M->nmortar & (M->nmortar - 1)) == 0) {
    long cap = M->nmortar ? 2 * M->nmortar : 1;
    orc_mortar *nm = realloc(M->mortar, cap * sizeof(orc_mortar));
    if (!nm) return -1;
    M->mortar = nm;
  }
  long k = M->nmortar++;
  M->mortar[k] = r;
  for (int side = 0; side < 2; ++side) {
    long e = side ? r.eB : r.eA;
    int f = side ? r.fB : r.fA, nfp = el_nfp(M, e);
    for (int m = 0; m < nfp; ++m) M->nbr[M->fo[e] + f * nfp + m] = -(MORTAR0 + k);
  }
  return 0;
}

static int link_faces(orc_mesh *M, long eA, int fA, long eB, int fB, const int *pi) {
  if (M->ord[eA] != M->ord[eB]) return add_mortar(M, eA, fA, eB, fB, pi);
  int mp[MAXN * MAXN];
  int n = el_n(M, eA), nfp = el_nfp(M, eA);
  if (face_perm(M, n, pi, mp)) return -1;
  for (int m = 0; m < nfp; ++m) {
    long qa = M->fo[eA] + fA * nfp + m, qb = M->fo[eB] + fB * nfp + mp[m];
    M->nbr[qa] = qb;
    M->nbr[qb] = qa;
  }
  return 0;
}

typedef struct { double c[3]; long id; } cent_rec;

static int cmp_cent(const void *pa, const void *pb) {
  const cent_rec *a = pa, *b = pb;
  if (a->c[0] < b->c[0]) return -1;
  if (a->c[0] > b->c[0]) return 1;
  return a->id < b->id ? -1 : (a->id > b->id);
}

static int build_connectivity(orc_mesh *M, const double *nodes, const long *en,
                              int nper, const double *shift, long nbf, const long *bf) {
  long E = M->E;
  int d = M->dim, nfe = 2 * d, nc = (d == 2) ? 2 : 4, na = M->q + 1;
  int nn = (d == 2) ? na * na : na * na * na;
  long F = E * nfe;
  for (long i = 0; i < M->NF; ++i) M->nbr[i] = 0x7fffffffffffL;
  face_rec *rec = malloc(F * sizeof(face_rec));
  for (long e = 0; e < E; ++e)
    for (int f = 0; f < nfe; ++f) {
      face_rec *r = &rec[e * nfe + f];
      r->e = e; r->f = f;
      for (int c = 0; c < 4; ++c) r->key[c] = -1;
      for (int c = 0; c < nc; ++c) r->key[c] = en[e * nn + corner_node(M, f, c)];
      sort4(r->key, nc);
    }
  qsort(rec, F, sizeof(face_rec), cmp_face);
  char *done = calloc(F, 1);
  int err = 0;
  for (long i = 0; i < F; ++i) {
    long j = i + 1;
    while (j < F && memcmp(rec[j].key, rec[i].key, sizeof(rec[i].key)) == 0) ++j;
    if (j - i == 2) {
      long eA = rec[i].e, eB = rec[i + 1].e;
      int fA = rec[i].f, fB = rec[i + 1].f;
      int pi[4];
      for (int c = 0; c < nc; ++c) {
        long id = en[eA * nn + corner_node(M, fA, c)];
        pi[c] = -1;
        for (int c2 = 0; c2 < nc; ++c2)
          if (en[eB * nn + corner_node(M, fB, c2)] == id) pi[c] = c2;
      }
      if (link_faces(M, eA, fA, eB, fB, pi)) err = -1;
      done[eA * nfe + fA] = done[eB * nfe + fB] = 1;
    } else if (j - i > 2) {
      err = -2;
    }
    i = j - 1;
  }
  free(rec);
  /* boundary faces */
  for (long b = 0; b < nbf; ++b) {
    long e = bf[3 * b], f = bf[3 * b + 1], kind = bf[3 * b + 2];
    if (e < 0 || e >= E || f < 0 || f >= nfe || done[e * nfe + f]) { err = -3; continue; }
    for (int m = 0; m < el_nfp(M, e); ++m) M->nbr[M->fo[e] + f * el_nfp(M, e) + m] = -kind;
    done[e * nfe + f] = 1;
  }
  /* periodic faces: corners coincide after a listed translation.  Unmatched
   * faces are sorted by the x of their corner centroid so that the partner
   * of a translated face is found by bisection. */
  if (nper > 0) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (long i = 0; i < M->nnodes; ++i)
      for (int k = 0; k < d; ++k) {
        double v = nodes[i * d + k];
        if (v < lo[k]) lo[k] = v;
        if (v > hi[k]) hi[k] = v;
      }
    double ext = 0.0;
    for (int k = 0; k < d; ++k) ext = fmax(ext, hi[k] - lo[k]);
    double tol = 1e-9 * ext;
    long nfree = 0;
    for (long a = 0; a < F; ++a) nfree += !done[a];
    cent_rec *cr = malloc((nfree + 1) * sizeof(cent_rec));
    long t = 0;
    for (long a = 0; a < F; ++a) {
      if (done[a]) continue;
      long e = a / nfe; int f = a % nfe;
      cr[t].id = a;
      for (int k = 0; k < 3; ++k) cr[t].c[k] = 0.0;
      for (int c = 0; c < nc; ++c)
        for (int k = 0; k < d; ++k) cr[t].c[k] += nodes[en[e * nn + corner_node(M, f, c)] * d + k] / nc;
      ++t;
    }
    qsort(cr, nfree, sizeof(cent_rec), cmp_cent);
    for (long ia = 0; ia < nfree; ++ia) {
      long a = cr[ia].id;
      if (done[a]) continue;
      long eA = a / nfe; int fA = a % nfe;
      int found = 0;
      for (int p = 0; p < nper && !found; ++p)
        for (int sg = -1; sg <= 1 && !found; sg += 2) {
          double tx = cr[ia].c[0] + sg * shift[p * d];
          long lo_i = 0, hi_i = nfree;
          while (lo_i < hi_i) { /* first entry with x >= tx - tol */
            long mid = (lo_i + hi_i) / 2;
            if (cr[mid].c[0] < tx - tol) lo_i = mid + 1; else hi_i = mid;
          }
          for (long ib = lo_i; ib < nfree && cr[ib].c[0] <= tx + tol && !found; ++ib) {
            long b = cr[ib].id;
            if (done[b] || b == a) continue;
            long eB = b / nfe; int fB = b % nfe;
            int pi[4], ok = 1;
            for (int c = 0; c < nc && ok; ++c) {
              const double *xa = &nodes[en[eA * nn + corner_node(M, fA, c)] * d];
              pi[c] = -1;
              for (int c2 = 0; c2 < nc; ++c2) {
                const double *xb = &nodes[en[eB * nn + corner_node(M, fB, c2)] * d];
                int same = 1;
                for (int k = 0; k < d; ++k)
                  if (fabs(xa[k] + sg * shift[p * d + k] - xb[k]) > tol) same = 0;
                if (same) pi[c] = c2;
              }
              if (pi[c] < 0) ok = 0;
            }
            if (ok) {
              if (link_faces(M, eA, fA, eB, fB, pi)) err = -1;
              done[a] = done[b] = 1;
              found = 1;
            }
          }
        }
      if (!found) err = -4;
    }
    free(cr);
  }
  for (long a = 0; a < F; ++a)
    if (!done[a]) err = -4;
  free(done);
  return err;
}

/* ------------------------------------------------------------------ */
/* physics                                                            */
/* ------------------------------------------------------------------ */

static void primitives(const orc_mesh *M, const double *u, double *rho, double v[3], double *p) {
  int d = M->dim;
  *rho = u[0];
  double ke = 0.0;
  v[0] = v[1] = v[2] = 0.0;
  for (int i = 0; i < d; ++i) { v[i] = u[1 + i] / u[0]; ke += v[i] * u[1 + i]; }
  *p = (M->gamma - 1.0) * (u[d + 1] - 0.5 * ke);
}

/* inviscid flux in physical direction j */
static void flux_inv(const orc_mesh *M, const double *u, double F[3][5]) {
  int d = M->dim;
  double rho, v[3], p;
  primitives(M, u, &rho, v, &p);
  for (int j = 0; j < d; ++j) {
    F[j][0] = u[1 + j];
    for (int i = 0; i < d; ++i) F[j][1 + i] = u[1 + i] * v[j] + (i == j ? p : 0.0);
    F[j][d + 1] = v[j] * (u[d + 1] + p);
  }
}

/* viscous flux F_vis,j = (0, tau_ij, v_i tau_ij - q_j); g[j][var] = d u_var / d x_j.
 * adiabatic != 0 drops the heat flux. */
static void flux_vis(const orc_mesh *M, const double *u, double g[3][5], double F[3][5],
                     int adiabatic) {
  int d = M->dim;
  double rho = u[0], v[3] = {0, 0, 0}, E = u[d + 1] / rho;
  for (int i = 0; i < d; ++i) v[i] = u[1 + i] / rho;
  double dv[3][3] = {{0}}, de[3] = {0, 0, 0};
  for (int j = 0; j < d; ++j) {
    for (int i = 0; i < d; ++i) dv[i][j] = (g[j][1 + i] - v[i] * g[j][0]) / rho;
    double dE = (g[j][d + 1] - E * g[j][0]) / rho;
    double vdv = 0.0;
    for (int i = 0; i < d; ++i) vdv += v[i] * dv[i][j];
    de[j] = dE - vdv;
  }
  double div = 0.0;
  for (int i = 0; i < d; ++i) div += dv[i][i];
  double mu = M->mu;
  double kappa = adiabatic ? 0.0 : mu * M->gamma / M->pr;
  for (int j = 0; j < d; ++j) {
    F[j][0] = 0.0;
    double work = 0.0;
    for (int i = 0; i < d; ++i) {
      double tau = mu * (dv[i][j] + dv[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));
      F[j][1 + i] = tau;
      work += v[i] * tau;
    }
    /* q_j = -kappa de/dx_j  ->  v_i tau_ij - q_j = work + kappa de_j */
    F[j][d + 1] = work + kappa * de[j];
  }
}

static double sound_speed(const orc_mesh *M, const double *u) {
  double rho, v[3], p;
  primitives(M, u, &rho, v, &p);
  return sqrt(M->gamma * p / rho);
}

/* Rusanov common normal flux for outward unit normal n of the L side */
static void rusanov(const orc_mesh *M, const double *uL, const double *uR, const double *n,
                    double *Fn) {
  int d = M->dim, nv = M->nv;
  double FL[3][5], FR[3][5];
  flux_inv(M, uL, FL);
  flux_inv(M, uR, FR);
  double vnL = 0.0, vnR = 0.0;
  for (int j = 0; j < d; ++j) { vnL += uL[1 + j] / uL[0] * n[j]; vnR += uR[1 + j] / uR[0] * n[j]; }
  double lamL = fabs(vnL) + sound_speed(M, uL), lamR = fabs(vnR) + sound_speed(M, uR);
  double lam = lamL > lamR ? lamL : lamR;
  for (int v = 0; v < nv; ++v) {
    double fl = 0.0, fr = 0.0;
    for (int j = 0; j < d; ++j) { fl += FL[j][v] * n[j]; fr += FR[j][v] * n[j]; }
    Fn[v] = 0.5 * (fl + fr) - 0.5 * lam * (uR[v] - uL[v]);
  }
}

static void vis_normal(const orc_mesh *M, const double *u, double g[3][5], const double *n,
                       double *Fn, int adiabatic) {
  double F[3][5];
  flux_vis(M, u, g, F, adiabatic);
  for (int v = 0; v < M->nv; ++v) {
    Fn[v] = 0.0;
    for (int j = 0; j < M->dim; ++j) Fn[v] += F[j][v] * n[j];
  }
}

/* Riemann-invariant far-field ghost state */
static void farfield_ghost(const orc_mesh *M, const double *uL, const double *n, double *ub) {
  int d = M->dim;
  double g = M->gamma;
  double rhoL, vL[3], pL;
  primitives(M, uL, &rhoL, vL, &pL);
  double cL = sqrt(g * pL / rhoL);
  double rhoI = M->fs[0], pI = M->fs[4], vI[3] = {M->fs[1], M->fs[2], M->fs[3]};
  double cI = sqrt(g * pI / rhoI);
  double vnL = 0.0, vnI = 0.0;
  for (int j = 0; j < d; ++j) { vnL += vL[j] * n[j]; vnI += vI[j] * n[j]; }
  double Rp = vnL + 2.0 * cL / (g - 1.0);
  double Rm = vnI - 2.0 * cI / (g - 1.0);
  double vnb = 0.5 * (Rp + Rm);
  double cb = 0.25 * (g - 1.0) * (Rp - Rm);
  double s, vt[3];
  if (vnb < 0.0) { /* inflow: entropy and tangential velocity from the free stream */
    s = pI / pow(rhoI, g);
    for (int j = 0; j < d; ++j) vt[j] = vI[j] - vnI * n[j];
  } else {
    s = pL / pow(rhoL, g);
    for (int j = 0; j < d; ++j) vt[j] = vL[j] - vnL * n[j];
  }
  double rhob = pow(cb * cb / (g * s), 1.0 / (g - 1.0));
  double pb = rhob * cb * cb / g;
  double ke = 0.0;
  ub[0] = rhob;
  for (int j = 0; j < d; ++j) {
    double vb = vt[j] + vnb * n[j];
    ub[1 + j] = rhob * vb;
    ke += vb * vb;
  }
  ub[d + 1] = pb / (g - 1.0) + 0.5 * rhob * ke;
}

/* ------------------------------------------------------------------ */
/* mesh creation                                                      */
/* ------------------------------------------------------------------ */

void orc_destroy(orc_mesh *M) {
  if (!M) return;
  free(M->S); free(M->detJ); free(M->xu); free(M->fnv); free(M->fA); free(M->fxyz);
  free(M->nbr); free(M->uf); free(M->gu); free(M->guf);
  free(M->ord); free(M->uo); free(M->fo); free(M->mortar);
  free(M);
}

/* Mesh with order orders[e] in element e (orders == NULL: every element has
 * `order`).  Returns 0, or <0 on a bad mesh (-5: non-positive Jacobian). */
int orc_create_mixed(int dim, int order, const int *orders, int q, long nnodes, const double *nodes,
                     long E, const long *elem_nodes, int nper, const double *shift, long nbf,
                     const long *bfaces, double gamma, double pr, double mu, const double *fs,
                     orc_mesh **out) {
  *out = NULL;
  if ((dim != 2 && dim != 3) || (q != 1 && q != 2)) return -1;
  orc_mesh *M = calloc(1, sizeof(orc_mesh));
  M->dim = dim; M->q = q;
  M->nv = dim + 2;
  M->E = E; M->nnodes = nnodes;
  M->gamma = gamma; M->pr = pr; M->mu = mu;
  for (int i = 0; i < 5; ++i) M->fs[i] = fs ? fs[i] : 0.0;
  M->ord = malloc((E > 0 ? E : 1) * sizeof(int));
  M->uo = malloc((E + 1) * sizeof(long));
  M->fo = malloc((E + 1) * sizeof(long));
  M->order = 0;
  M->uo[0] = M->fo[0] = 0;
  for (long e = 0; e < E; ++e) {
    int p = orders ? orders[e] : order;
    if (p < 0 || p + 1 > MAXN) { orc_destroy(M); return -1; }
    M->ord[e] = p;
    if (p > M->order) M->order = p;
    int n = p + 1;
    M->uo[e + 1] = M->uo[e] + (dim == 2 ? n * n : n * n * n);
    M->fo[e + 1] = M->fo[e] + 2 * dim * (dim == 2 ? n : n * n);
  }
  if (E == 0) M->order = order;
  for (int p = 0; p + 1 <= MAXN; ++p) {
    orc_basis1d *B = &M->bas[p];
    double Dflat[MAXN * MAXN];
    B->n = p + 1;
    orc_basis(p, B->xi, B->w, Dflat, B->lm, B->lp, B->gLd, B->gRd);
    for (int i = 0; i < B->n; ++i)
      for (int j = 0; j < B->n; ++j) B->D[i][j] = Dflat[i * B->n + j];
  }
  long NU = M->NU = M->uo[E], NF = M->NF = M->fo[E];
  int nv = M->nv;
  M->S = malloc((NU + 1) * 9 * sizeof(double));
  M->detJ = malloc((NU + 1) * sizeof(double));
  M->xu = malloc((NU + 1) * 3 * sizeof(double));
  M->fnv = malloc((NF + 1) * 3 * sizeof(double));
  M->fA = malloc((NF + 1) * sizeof(double));
  M->fxyz = malloc((NF + 1) * 3 * sizeof(double));
  M->nbr = malloc((NF + 1) * sizeof(long));
  M->uf = malloc((NF + 1) * nv * sizeof(double));
  M->gu = malloc((NU + 1) * 3 * nv * sizeof(double));
  M->guf = malloc((NF + 1) * 3 * nv * sizeof(double));
  int bad = 0;
#pragma omp parallel for reduction(| : bad)
  for (long e = 0; e < E; ++e) {
    const orc_basis1d *B = &M->bas[M->ord[e]];
    int n = B->n, nu = el_nu(M, e), nfp = el_nfp(M, e);
    for (int i = 0; i < nu; ++i) {
      int c[3] = {i % n, (i / n) % n, i / (n * n)};
      double r[3] = {B->xi[c[0]], B->xi[c[1]], dim == 3 ? B->xi[c[2]] : 0.0};
      double x[3], J[3][3], S[3][3];
      long a = M->uo[e] + i;
      map_point(M, nodes, elem_nodes, e, r, x, J);
      double det = adjugate(dim, J, S);
      if (!(det > 0.0)) bad = 1;
      M->detJ[a] = det;
      memcpy(&M->S[a * 9], S, sizeof(S));
      for (int k = 0; k < 3; ++k) M->xu[a * 3 + k] = x[k];
    }
    for (int f = 0; f < 2 * dim; ++f)
      for (int m = 0; m < nfp; ++m) {
        int k = f / 2;
        long a = M->fo[e] + f * nfp + m;
        double sg = (f % 2) ? 1.0 : -1.0;
        double r[3], x[3], J[3][3], S[3][3];
        fpt_ref(M, B, f, m, r);
        map_point(M, nodes, elem_nodes, e, r, x, J);
        double det = adjugate(dim, J, S);
        if (!(det > 0.0)) bad = 1;
        double aa = 0.0;
        for (int j = 0; j < dim; ++j) aa += S[k][j] * S[k][j];
        aa = sqrt(aa);
        M->fA[a] = aa;
        for (int j = 0; j < 3; ++j) M->fnv[a * 3 + j] = j < dim ? sg * S[k][j] / aa : 0.0;
        for (int j = 0; j < 3; ++j) M->fxyz[a * 3 + j] = x[j];
      }
  }
  if (bad) { orc_destroy(M); return -5; }
  int err = build_connectivity(M, nodes, elem_nodes, nper, shift, nbf, bfaces);
  if (err) { orc_destroy(M); return err; }
  *out = M;
  return 0;
}

int orc_create(int dim, int order, int q, long nnodes, const double *nodes, long E,
               const long *elem_nodes, int nper, const double *shift, long nbf,
               const long *bfaces, double gamma, double pr, double mu, const double *fs,
               orc_mesh **out) {
  return orc_create_mixed(dim, order, NULL, q, nnodes, nodes, E, elem_nodes, nper, shift, nbf, bfaces,
                          gamma, pr, mu, fs, out);
}

/* face quadrature weight of face point m of an element with basis B */
static double face_weight(const orc_mesh *M, const orc_basis1d *B, int m) {
  return M->dim == 2 ? B->w[m] : B->w[m % B->n] * B->w[m / B->n];
}

/* Data on a face shared by elements of different orders (a mortar face).  The
 * low-order element's face data is its polynomial interpolant through its face
 * points; the high-order element samples it at its own face points.  Data of
 * the high-order element reaches the low-order one as its L2 projection onto the
 * low order's face polynomials, evaluated at the low-order face points; the
 * projection integral is taken by the high-order face quadrature. */

/* interpolant of the low side's face data g (point m at g[m * stride]) at the
 * high-side face point mA */
static double mortar_up(const orc_mesh *M, const orc_mortar *R, int mA, const double *g, int stride) {
  const orc_basis1d *BA = &M->bas[M->ord[R->eA]], *BB = &M->bas[M->ord[R->eB]];
  double sA[2], t[2];
  face_coords(M, BA, mA, sA);
  map_face(M->dim, R->pi, sA, t);
  int nB = BB->n, nfpB = el_nfp(M, R->eB);
  double s = 0.0;
  for (int m = 0; m < nfpB; ++m) {
    double l = lagrange(nB, BB->xi, m % nB, t[0]);
    if (M->dim == 3) l *= lagrange(nB, BB->xi, m / nB, t[1]);
    s += l * g[m * stride];
  }
  return s;
}

/* L2 projection of the high side's face data h (point j at h[j * stride]) onto
 * the low order's face polynomials, at the low-side face point mB */
static double mortar_down(const orc_mesh *M, const orc_mortar *R, int mB, const double *h, int stride) {
  const orc_basis1d *BA = &M->bas[M->ord[R->eA]], *BB = &M->bas[M->ord[R->eB]];
  int pB = M->ord[R->eB], nfpA = el_nfp(M, R->eA), d = M->dim;
  double tB[2];
  face_coords(M, BB, mB, tB);
  double out = 0.0;
  for (int k1 = 0; k1 <= (d == 3 ? pB : 0); ++k1)
    for (int k0 = 0; k0 <= pB; ++k0) {
      /* coefficient of L_k0(t0) L_k1(t1): (2k+1)/2 per axis times the integral */
      double c = 0.0;
      for (int j = 0; j < nfpA; ++j) {
        double sA[2], t[2], P0, P1 = 1.0, dP;
        face_coords(M, BA, j, sA);
        map_face(d, R->pi, sA, t);
        legendre(k0, t[0], &P0, &dP);
        if (d == 3) legendre(k1, t[1], &P1, &dP);
        c += face_weight(M, BA, j) * h[j * stride] * P0 * P1;
      }
      c *= 0.5 * (2 * k0 + 1);
      if (d == 3) c *= 0.5 * (2 * k1 + 1);
      double L0, L1 = 1.0, dP;
      legendre(k0, tB[0], &L0, &dP);
      if (d == 3) legendre(k1, tB[1], &L1, &dP);
      out += c * L0 * L1;
    }
  return out;
}

/* ------------------------------------------------------------------ */
/* residual                                                           */
/* ------------------------------------------------------------------ */

/* interior trace of u at every flux point */
static void pass_interp(orc_mesh *M, const double *u) {
  int nv = M->nv;
#pragma omp parallel for
  for (long e = 0; e < M->E; ++e) {
    const orc_basis1d *B = &M->bas[M->ord[e]];
    int n = B->n, nfp = el_nfp(M, e);
    for (int f = 0; f < 2 * M->dim; ++f) {
      const double *l = (f % 2) ? B->lp : B->lm;
      for (int m = 0; m < nfp; ++m)
        for (int v = 0; v < nv; ++v) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += l[j] * u[(M->uo[e] + line_pt(M, n, f / 2, m, j)) * nv + v];
          M->uf[(M->fo[e] + f * nfp + m) * nv + v] = s;
        }
    }
  }
}

/* face point m of face f of element e on a mortar face: which side it is on */
static const orc_mortar *mortar_of(const orc_mesh *M, long code) { return &M->mortar[-code - MORTAR0]; }

/* common solution at flux point qq of element e (BR1 mean, or boundary value) */
static void common_solution(const orc_mesh *M, long e, int qq, double *uc) {
  int nv = M->nv, d = M->dim;
  long a = M->fo[e] + qq;
  const double *uL = &M->uf[a * nv];
  long nb = M->nbr[a];
  if (nb >= 0) {
    const double *uR = &M->uf[nb * nv];
    for (int v = 0; v < nv; ++v) uc[v] = 0.5 * (uL[v] + uR[v]);
  } else if (nb <= -MORTAR0) {
    /* mean of the own trace and the other side's trace brought to this point:
     * interpolated up on the high side, projected down on the low side */
    const orc_mortar *R = mortar_of(M, nb);
    int nfp = el_nfp(M, e), m = qq % nfp;
    for (int v = 0; v < nv; ++v) {
      double uo;
      if (e == R->eA && qq / nfp == R->fA)
        uo = mortar_up(M, R, m, &M->uf[(M->fo[R->eB] + R->fB * el_nfp(M, R->eB)) * nv + v], nv);
      else
        uo = mortar_down(M, R, m, &M->uf[(M->fo[R->eA] + R->fA * el_nfp(M, R->eA)) * nv + v], nv);
      uc[v] = 0.5 * (uL[v] + uo);
    }
  } else if (nb == -BC_FARFIELD) {
    farfield_ghost(M, uL, &M->fnv[a * 3], uc);
  } else { /* wall: zero velocity, same density and internal energy */
    double ke = 0.0;
    for (int i = 0; i < d; ++i) ke += uL[1 + i] * uL[1 + i] / uL[0];
    uc[0] = uL[0];
    for (int i = 0; i < d; ++i) uc[1 + i] = 0.0;
    uc[d + 1] = uL[d + 1] - 0.5 * ke;
  }
}

/* corrected physical gradient at solution points and its trace at flux points */
static void pass_gradient(orc_mesh *M, const double *u) {
  int nv = M->nv, d = M->dim;
#pragma omp parallel for
  for (long e = 0; e < M->E; ++e) {
    const orc_basis1d *B = &M->bas[M->ord[e]];
    int n = B->n, nu = el_nu(M, e), nf = el_nf(M, e), nfp = el_nfp(M, e);
    long uo = M->uo[e], fo = M->fo[e];
    double du[6 * MAXN * MAXN][5];
    for (int qq = 0; qq < nf; ++qq) {
      double uc[5];
      common_solution(M, e, qq, uc);
      for (int v = 0; v < nv; ++v) du[qq][v] = uc[v] - M->uf[(fo + qq) * nv + v];
    }
    for (int i = 0; i < nu; ++i) {
      double G[3][5];
      for (int k = 0; k < d; ++k) {
        int ik, m;
        pt_line(M, n, i, k, &ik, &m);
        int qm = (2 * k) * nfp + m, qp = (2 * k + 1) * nfp + m;
        for (int v = 0; v < nv; ++v) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += B->D[ik][j] * u[(uo + line_pt(M, n, k, m, j)) * nv + v];
          s += du[qp][v] * B->gRd[ik] + du[qm][v] * B->gLd[ik];
          G[k][v] = s;
        }
      }
      const double *S = &M->S[(uo + i) * 9];
      double J = M->detJ[uo + i];
      for (int j = 0; j < d; ++j)
        for (int v = 0; v < nv; ++v) {
          double s = 0.0;
          for (int k = 0; k < d; ++k) s += S[k * 3 + j] * G[k][v];
          M->gu[((uo + i) * 3 + j) * nv + v] = s / J;
        }
    }
    for (int f = 0; f < 2 * d; ++f) {
      const double *l = (f % 2) ? B->lp : B->lm;
      for (int m = 0; m < nfp; ++m)
        for (int j = 0; j < d; ++j)
          for (int v = 0; v < nv; ++v) {
            double s = 0.0;
            for (int jj = 0; jj < n; ++jj)
              s += l[jj] * M->gu[((uo + line_pt(M, n, f / 2, m, jj)) * 3 + j) * nv + v];
            M->guf[((fo + f * nfp + m) * 3 + j) * nv + v] = s;
          }
    }
  }
}

/* common normal flux (physical, per unit area) for L-side flux point aL */
static void interior_flux(const orc_mesh *M, long aL, long aR, double *Fn) {
  int nv = M->nv;
  const double *uL = &M->uf[aL * nv], *uR = &M->uf[aR * nv];
  const double *n = &M->fnv[aL * 3];
  double gL[3][5], gR[3][5], FI[5], FvL[5], FvR[5];
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < nv; ++v) {
      gL[j][v] = M->guf[(aL * 3 + j) * nv + v];
      gR[j][v] = M->guf[(aR * 3 + j) * nv + v];
    }
  rusanov(M, uL, uR, n, FI);
  vis_normal(M, uL, gL, n, FvL, 0);
  vis_normal(M, uR, gR, n, FvR, 0);
  for (int v = 0; v < nv; ++v) Fn[v] = FI[v] - 0.5 * (FvL[v] + FvR[v]);
}

/* Transformed common normal flux A F*.n at the high-side point mA of a mortar
 * face.  The low side enters through the interpolants of its trace and of its
 * half viscous normal flux F_v(u, grad u).n / 2 (with its own normal). */
static void mortar_flux_high(const orc_mesh *M, const orc_mortar *R, int mA, double *T) {
  int nv = M->nv;
  long a = M->fo[R->eA] + R->fA * el_nfp(M, R->eA) + mA;
  int nfpB = el_nfp(M, R->eB);
  long b0 = M->fo[R->eB] + R->fB * nfpB;
  const double *uL = &M->uf[a * nv];
  const double *n = &M->fnv[a * 3];
  double uR[5], gL[3][5], FI[5], FvL[5], PB[MAXN * MAXN][5];
  for (int v = 0; v < nv; ++v) uR[v] = mortar_up(M, R, mA, &M->uf[b0 * nv + v], nv);
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < nv; ++v) gL[j][v] = M->guf[(a * 3 + j) * nv + v];
  for (int m = 0; m < nfpB; ++m) {
    double gB[3][5], Fv[5];
    for (int j = 0; j < 3; ++j)
      for (int v = 0; v < nv; ++v) gB[j][v] = M->guf[((b0 + m) * 3 + j) * nv + v];
    vis_normal(M, &M->uf[(b0 + m) * nv], gB, &M->fnv[(b0 + m) * 3], Fv, 0);
    for (int v = 0; v < nv; ++v) PB[m][v] = 0.5 * Fv[v];
  }
  rusanov(M, uL, uR, n, FI);
  vis_normal(M, uL, gL, n, FvL, 0);
  for (int v = 0; v < nv; ++v) {
    double pb = mortar_up(M, R, mA, &PB[0][v], 5);
    T[v] = M->fA[a] * (FI[v] - 0.5 * FvL[v] + pb);
  }
}

static void boundary_flux(const orc_mesh *M, long a, long kind, double *Fn) {
  int nv = M->nv, d = M->dim;
  const double *uL = &M->uf[a * nv];
  const double *n = &M->fnv[a * 3];
  double g[3][5], FI[5], FV[5], ub[5];
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < nv; ++v) g[j][v] = M->guf[(a * 3 + j) * nv + v];
  if (kind == BC_FARFIELD) {
    farfield_ghost(M, uL, n, ub);
    rusanov(M, uL, ub, n, FI);
    vis_normal(M, ub, g, n, FV, 0);
  } else {
    double ug[5], uc[5], ke = 0.0;
    ug[0] = uL[0];
    for (int i = 0; i < d; ++i) { ug[1 + i] = -uL[1 + i]; ke += uL[1 + i] * uL[1 + i] / uL[0]; }
    ug[d + 1] = uL[d + 1];
    rusanov(M, uL, ug, n, FI);
    uc[0] = uL[0];
    for (int i = 0; i < d; ++i) uc[1 + i] = 0.0;
    uc[d + 1] = uL[d + 1] - 0.5 * ke;
    vis_normal(M, uc, g, n, FV, 1);
  }
  for (int v = 0; v < nv; ++v) Fn[v] = FI[v] - FV[v];
}

/* transformed flux at solution points, corrected divergence, R = -div/|J| */
static void pass_divergence(orc_mesh *M, const double *u, double *R) {
  int nv = M->nv, d = M->dim;
#pragma omp parallel for
  for (long e = 0; e < M->E; ++e) {
    const orc_basis1d *B = &M->bas[M->ord[e]];
    int n = B->n, nu = el_nu(M, e), nfp = el_nfp(M, e);
    long uo = M->uo[e], fo = M->fo[e];
    double Ft[MAXN * MAXN * MAXN][3][5];
    double dlt[6 * MAXN * MAXN][5];
    for (int i = 0; i < nu; ++i) {
      const double *ui = &u[(uo + i) * nv];
      double g[3][5], FI[3][5], FV[3][5];
      for (int j = 0; j < 3; ++j)
        for (int v = 0; v < nv; ++v) g[j][v] = j < d ? M->gu[((uo + i) * 3 + j) * nv + v] : 0.0;
      flux_inv(M, ui, FI);
      flux_vis(M, ui, g, FV, 0);
      const double *S = &M->S[(uo + i) * 9];
      for (int k = 0; k < d; ++k)
        for (int v = 0; v < nv; ++v) {
          double s = 0.0;
          for (int j = 0; j < d; ++j) s += S[k * 3 + j] * (FI[j][v] - FV[j][v]);
          Ft[i][k][v] = s;
        }
    }
    for (int f = 0; f < 2 * d; ++f) {
      int k = f / 2;
      double sg = (f % 2) ? 1.0 : -1.0;
      const double *l = (f % 2) ? B->lp : B->lm;
      for (int m = 0; m < nfp; ++m) {
        int qq = f * nfp + m;
        long a = fo + qq, b = M->nbr[a];
        double T[5];
        if (b >= 0) {
          double Fn[5];
          if (a < b) {
            interior_flux(M, a, b, Fn);
          } else { /* the partner is the L side; its normal is opposite */
            interior_flux(M, b, a, Fn);
            for (int v = 0; v < nv; ++v) Fn[v] = -Fn[v];
          }
          for (int v = 0; v < nv; ++v) T[v] = M->fA[a] * Fn[v];
        } else if (b <= -MORTAR0) {
          const orc_mortar *Rm = mortar_of(M, b);
          if (e == Rm->eA && f == Rm->fA) {
            mortar_flux_high(M, Rm, m, T);
          } else {
            /* the low side takes minus the projection of the high side's flux */
            double TH[MAXN * MAXN][5];
            int nfpA = el_nfp(M, Rm->eA);
            for (int j = 0; j < nfpA; ++j) mortar_flux_high(M, Rm, j, TH[j]);
            for (int v = 0; v < nv; ++v) T[v] = -mortar_down(M, Rm, m, &TH[0][v], 5);
          }
        } else {
          double Fn[5];
          boundary_flux(M, a, -b, Fn);
          for (int v = 0; v < nv; ++v) T[v] = M->fA[a] * Fn[v];
        }
        for (int v = 0; v < nv; ++v) {
          double fd = 0.0;
          for (int j = 0; j < n; ++j) fd += l[j] * Ft[line_pt(M, n, k, m, j)][k][v];
          dlt[qq][v] = T[v] - sg * fd;
        }
      }
    }
    for (int i = 0; i < nu; ++i) {
      double J = M->detJ[uo + i];
      for (int v = 0; v < nv; ++v) {
        double div = 0.0;
        for (int k = 0; k < d; ++k) {
          int ik, m;
          pt_line(M, n, i, k, &ik, &m);
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += B->D[ik][j] * Ft[line_pt(M, n, k, m, j)][k][v];
          s += dlt[(2 * k + 1) * nfp + m][v] * B->gRd[ik] - dlt[(2 * k) * nfp + m][v] * B->gLd[ik];
          div += s;
        }
        R[(uo + i) * nv + v] = -div / J;
      }
    }
  }
}

int orc_residual(orc_mesh *M, const double *u, double *R) {
  long N = M->NU * M->nv;
  if (M->mock) {
    for (long i = 0; i < N; ++i) R[i] = M->mock_lambda * u[i];
    return 0;
  }
  pass_interp(M, u);
  pass_gradient(M, u);
  pass_divergence(M, u, R);
  return 0;
}

/* corrected physical gradient of u at the solution points, [NU][3][nv] */
int orc_gradient(orc_mesh *M, const double *u, double *g) {
  pass_interp(M, u);
  pass_gradient(M, u);
  memcpy(g, M->gu, M->NU * 3 * M->nv * sizeof(double));
  return 0;
}

/* wall force F = sum over wall flux points of W A (p n - tau . n) */
int orc_forces(orc_mesh *M, const double *u, double *F) {
  pass_interp(M, u);
  pass_gradient(M, u);
  int nv = M->nv, d = M->dim;
  F[0] = F[1] = F[2] = 0.0;
  for (long e = 0; e < M->E; ++e) {
    const orc_basis1d *B = &M->bas[M->ord[e]];
    int nf = el_nf(M, e), nfp = el_nfp(M, e);
    for (int qq = 0; qq < nf; ++qq) {
      long a = M->fo[e] + qq;
      if (M->nbr[a] != -BC_WALL) continue;
      const double *uL = &M->uf[a * nv];
      const double *nn = &M->fnv[a * 3];
      double rho, v[3], p, g[3][5], Fv[3][5];
      primitives(M, uL, &rho, v, &p);
      for (int j = 0; j < 3; ++j)
        for (int vv = 0; vv < nv; ++vv) g[j][vv] = M->guf[(a * 3 + j) * nv + vv];
      flux_vis(M, uL, g, Fv, 0);
      double wA = face_weight(M, B, qq % nfp) * M->fA[a];
      for (int i = 0; i < d; ++i) {
        double tn = 0.0;
        for (int j = 0; j < d; ++j) tn += Fv[j][1 + i] * nn[j]; /* tau_ij n_j */
        F[i] += wA * (p * nn[i] - tn);
      }
    }
  }
  return 0;
}

/* classic RK4 steps; if Fhist is non-NULL the wall force after each step is
 * stored in Fhist[step*3 .. step*3+2] */
int orc_rk4(orc_mesh *M, double *u, double dt, long nsteps, double *Fhist) {
  long N = M->NU * M->nv;
  double *k = malloc(N * sizeof(double)), *acc = malloc(N * sizeof(double)),
         *us = malloc(N * sizeof(double));
  const double c[4] = {0.0, 0.5, 0.5, 1.0}, b[4] = {1.0, 2.0, 2.0, 1.0};
  for (long s = 0; s < nsteps; ++s) {
    for (int st = 0; st < 4; ++st) {
      if (st == 0) {
        memcpy(us, u, N * sizeof(double));
      } else {
        for (long i = 0; i < N; ++i) us[i] = u[i] + c[st] * dt * k[i];
      }
      orc_residual(M, us, k);
      for (long i = 0; i < N; ++i) acc[i] = (st == 0 ? 0.0 : acc[i]) + b[st] * k[i];
    }
    for (long i = 0; i < N; ++i) u[i] = u[i] + dt / 6.0 * acc[i];
    if (Fhist) orc_forces(M, u, &Fhist[s * 3]);
  }
  free(k); free(acc); free(us);
  return 0;
}

/* ------------------------------------------------------------------ */
/* accessors for tests                                                */
/* ------------------------------------------------------------------ */

void orc_sizes(const orc_mesh *M, long *out) {
  int n = M->order + 1;
  out[0] = M->dim; out[1] = M->order; out[2] = M->dim == 2 ? n * n : n * n * n;
  out[3] = 2 * M->dim * (M->dim == 2 ? n : n * n); out[4] = M->nv; out[5] = M->E;
  out[6] = M->dim == 2 ? n : n * n; out[7] = M->NU; out[8] = M->NF; out[9] = M->nmortar;
}
void orc_neighbours(const orc_mesh *M, long *out) { memcpy(out, M->nbr, M->NF * sizeof(long)); }
void orc_solution_points(const orc_mesh *M, double *xyz) { memcpy(xyz, M->xu, M->NU * 3 * sizeof(double)); }
void orc_flux_points(const orc_mesh *M, double *xyz) { memcpy(xyz, M->fxyz, M->NF * 3 * sizeof(double)); }
void orc_metrics(const orc_mesh *M, double *detJ, double *fA, double *fn) {
  if (detJ) memcpy(detJ, M->detJ, M->NU * sizeof(double));
  if (fA) memcpy(fA, M->fA, M->NF * sizeof(double));
  if (fn) memcpy(fn, M->fnv, M->NF * 3 * sizeof(double));
}
void orc_set_mock(orc_mesh *M, int on, double lambda) { M->mock = on; M->mock_lambda = lambda; }
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
/* far-field ghost state for an interior state and outward unit normal */
void orc_farfield_state(const orc_mesh *M, const double *uL, const double *n, double *ub) {
  farfield_ghost(M, uL, n, ub);
}
