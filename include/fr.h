/*
 * fr.h -- C ABI of the MI355X flux reconstruction (FR) solver library.
 *
 * The library advances the compressible Navier-Stokes equations of the
 * paper's Section 2.1 (Eqs. (1)-(7): conserved variables rho, rho u_i,
 * rho E; F = F_inv - F_vis with F_vis,j = (0, tau_ij, u_i tau_ij - q_j);
 * ideal gas; Stokes stress; heat flux from the enthalpy gradient) on
 * quadrilateral (2D) or hexahedral (3D) elements with an FR discretisation
 * (Huynh 2007, named in the paper's Section 1 for its solver) and classic
 * RK4 in time.  The design evaluation of the paper's Algorithm 1 needs the
 * flow advanced on one candidate mesh and the time-averaged lift and drag
 * (Section 3.4, objective function); these calls are exactly that.
 *
 * Scheme (fixed): Gauss-Legendre solution points (tensor product), flux
 * points where the solution-point lines meet the faces, g_DG (Radau)
 * correction functions, Rusanov inviscid common flux, BR1 common solution
 * and viscous flux, periodic faces by translation, Riemann-invariant far
 * field, no-slip adiabatic wall.
 *
 * Conventions shared by every array below
 *   - Reference element [-1,1]^dim.  Geometry nodes of an element are the
 *     (q+1)^dim equispaced Lagrange nodes, lexicographic with xi fastest:
 *     node a = a0 + (q+1) a1 + (q+1)^2 a2 at xi_k = -1 + 2 a_k / q.
 *   - Solution point i = i0 + n i1 + n^2 i2 (n = order + 1), xi fastest.
 *   - Local face f = 2k + s lies on axis k at xi_k = -1 (s = 0) or +1
 *     (s = 1).  Flux point q = f * nfp + m, nfp = n^(dim-1); m runs over the
 *     remaining axes in increasing axis order, the lower axis fastest.
 *   - States are conserved variables in FP64, canonical layout
 *     [element][solution point][variable], variables (rho, rho u, rho v,
 *     [rho w,] rho E).
 *
 * Errors: every call returns an fr_status; FR_OK is 0 and errors are
 * negative.  fr_last_error() returns a thread-local message for the last
 * failing call of the calling thread.  No C++ exception crosses the ABI.
 *
 * Ownership: input arrays are caller-owned, read during the call and never
 * retained.  A handle owns its device memory (allocated through the
 * optional alloc/free callbacks, else hipMalloc/hipFree) until destroyed.
 *
 * Threading: a handle is not thread-safe; distinct handles may be used
 * from distinct threads.  Work is ordered on the handle's stream.
 */
#ifndef FR_H
#define FR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_mesh fr_mesh;
typedef struct fr_pool fr_pool;
typedef struct fr_probe fr_probe;

typedef enum {
  FR_OK = 0,
  FR_E_ARG = -1,         /* invalid argument or descriptor */
  FR_E_MESH = -2,        /* unmatched face, bad connectivity or non-positive Jacobian */
  FR_E_NOMEM = -3,       /* allocation failed, or a pool request does not fit its budget */
  FR_E_DEVICE = -4,      /* HIP runtime error */
  FR_E_NONFINITE = -5,   /* a step produced a non-finite state (left in place) */
  FR_E_STATE = -6,       /* call not valid in the current state (e.g. no state set) */
  FR_E_UNSUPPORTED = -7  /* order, dimension or precision not compiled in */
} fr_status;

enum { FR_FP64 = 0, FR_FP32 = 1 };        /* state, operator and flux precision */
enum { FR_BC_WALL = 1, FR_BC_FARFIELD = 2 };

typedef void *(*fr_alloc_fn)(size_t bytes, void *ctx, void *stream);
typedef void (*fr_free_fn)(void *ptr, void *ctx, void *stream);

/* One mesh and its flow constants.  All pointers are host pointers. */
typedef struct {
  int32_t dim;             /* 2 or 3 */
  int32_t order;           /* polynomial order p, 0..4 (0: one solution point, a finite volume) */
  int32_t geom_order;      /* q = 1 (straight) or 2 (quadratic, curved) */
  int32_t precision;       /* FR_FP64 or FR_FP32 (metrics and force sums are FP64 in both) */
  int64_t n_nodes;
  const double *nodes;     /* [n_nodes][dim] */
  int64_t n_elems;
  const int64_t *elem_nodes; /* [n_elems][(q+1)^dim] node ids */
  int32_t n_periodic;
  const double *periodic_shift; /* [n_periodic][dim] translations pairing periodic faces */
  int64_t n_bfaces;
  const int64_t *bfaces;   /* [n_bfaces][3] = {element, local face, FR_BC_*} */
  double gamma, prandtl, mu; /* ratio of specific heats, Prandtl number, constant viscosity */
  double freestream[5];    /* rho, u, v, w, p: far-field state and force normalisation */
  double ref_area;         /* C = F . dir / (0.5 rho |U|^2 ref_area) */
  double lift_dir[3], drag_dir[3];
  double dt;               /* fixed RK4 step */
  int32_t device;          /* HIP device ordinal */
  void *stream;            /* hipStream_t to order work on, or NULL for the default stream */
  fr_alloc_fn alloc;       /* optional device allocator (e.g. a framework's caching allocator) */
  fr_free_fn free;
  void *alloc_ctx;
  const int32_t *elem_order; /* [n_elems] per-element order 0..4, or NULL: `order` everywhere.
                              * See "Variable order" below. */
} fr_mesh_desc;

/* Variable order (Section 3.1: the paper lowers the solution order toward the
 * far-field boundaries so that acoustic waves leave without reflecting).
 * With elem_order set, element e carries order elem_order[e] and `order`
 * is ignored.  A face shared by elements of different orders carries a
 * mortar: the lower-order element's trace and half viscous normal flux
 * enter the higher-order side as their interpolants at its flux points,
 * where the common flux is formed; the lower-order side takes the L2
 * projection of the higher-order side's transformed common flux onto its
 * own face polynomials (exact in the higher order's face quadrature), so
 * the face integrals of both sides agree and the scheme stays
 * conservative.  The state of such a mesh is ragged: [sum of n_u(e)][nv],
 * element e's solution points contiguous, in element order (fr_set_state,
 * fr_get_state, fr_residual, fr_solution_points).  Variable-order meshes run
 * the fused two-launch stage only, and fr_neighbours, fr_state_device and
 * fr_profile_kernels report FR_E_UNSUPPORTED for them.  They batch like
 * one-order meshes (fr_batch_create): designs with and without elem_order
 * together, each order group of the batch covering the elements of that order
 * of every design, the batch state the designs' ragged states concatenated.
 * Probes and served requests with a data surface work on them (each point is
 * evaluated with its element's order). */

/* Build a solver for one mesh: connectivity (faces matched by node ids,
 * periodic faces by the listed translations, flux points by position),
 * FP64 metrics, operators, device arrays.  FR_E_MESH if a face is neither
 * matched nor listed as a boundary, or a Jacobian is not positive.
 * Follows Algorithm 1 (each candidate design gets its own mesh before its
 * flow solve) and the set-up of Section 3.1 (spanwise-periodic airfoil grid,
 * curved elements); the FR discretisation is the one named in Section 1. */
fr_status fr_mesh_create(const fr_mesh_desc *desc, fr_mesh **out);

/* Several meshes (candidate designs) advanced together by every kernel
 * launch: the layer of parallelism that runs the 2n poll designs of the
 * paper's Algorithm 1 concurrently.  All descriptors must share dim,
 * precision, gamma, prandtl, mu, device and stream, and, unless some
 * descriptor sets elem_order (variable order, above), order; dt, free stream
 * and force normalisation are per design.  State arrays of the batch are
 * the designs' canonical arrays concatenated in descriptor order.  FR_E_ARG
 * if the descriptors do not share those fields. */
fr_status fr_batch_create(const fr_mesh_desc *descs, int32_t n_designs, fr_mesh **out);

void fr_mesh_destroy(fr_mesh *m);

/* info[0..9] = dim, order, n_designs, total elements, solution points per
 * element, flux points per element, variables, precision, element blocks,
 * device bytes held. */
fr_status fr_mesh_info(const fr_mesh *m, int64_t *info);

/* Elements of design d and their offset in the concatenated arrays. */
fr_status fr_design_range(const fr_mesh *m, int32_t design, int64_t *first, int64_t *count);

/* Physical coordinates of the solution points, [elements][n_u][3] (z = 0 in 2D),
 * into caller-owned host memory: where initial conditions are evaluated. */
fr_status fr_solution_points(const fr_mesh *m, double *xyz);

/* Partner of every flux point, [elements][n_f]: e' * n_f + q' for an
 * interior or periodic face, -kind for a boundary face (element indices
 * are positions in the concatenated arrays). */
fr_status fr_neighbours(const fr_mesh *m, int64_t *nbr);

/* Solution points of the mesh: n_elems * n_u, or the sum of n_u(e) over the
 * elements of a variable-order mesh (the length of its ragged state). */
fr_status fr_mesh_points(const fr_mesh *m, int64_t *n_points);

/* Host-only variant of the neighbour table for a single descriptor: runs
 * the connectivity and geometry checks without touching a device.  nbr is
 * [n_elems][n_f] as for fr_neighbours; xyz (may be NULL) receives the
 * solution points [n_elems][n_u][3]. */
fr_status fr_connectivity(const fr_mesh_desc *desc, int64_t *nbr, double *xyz);

/* Set / get the conserved state (host, FP64, canonical layout): the
 * variables of Eq. (2) of Section 2.1, rho, rho u_i, rho E, at every
 * solution point.  Setting the state also clears the running lift and drag
 * means (Section 3.4 averages them over the solve).  u is read (set) or
 * written (get) during the call only.  FR_E_STATE from fr_get_state before
 * any state was set. */
fr_status fr_set_state(fr_mesh *m, const double *u);
fr_status fr_get_state(const fr_mesh *m, double *u);

/* Advance n RK4 steps of dt on the device and wait for them: the time
 * integration of Eq. (1) of Section 2.1, du/dt = -div F, with classic
 * four-stage Runge-Kutta and a fixed step in place of the paper's
 * second-order scheme with adaptive steps (Section 3.1, whose coefficients
 * are not given).  After each step the wall force of the new state is added
 * to the running means: in the next step's first stage, which reads that
 * state anyway, or, for the last state, when fr_forces reads the sums (or
 * a call that overwrites the trace, such as fr_residual, comes first); the
 * sums are those of adding it at once.
 * FR_E_NONFINITE if any step produced a non-finite
 * value (the state is left as computed); FR_E_STATE if no state was set;
 * FR_E_ARG for n < 0. */
fr_status fr_step(fr_mesh *m, int64_t n);

/* Enqueue n steps (as fr_step) without waiting; the state stays in device
 * memory.  This is what lets the poll designs of Algorithm 1 run side by
 * side on one device. */
fr_status fr_step_async(fr_mesh *m, int64_t n);
/* Wait for enqueued work; reports FR_E_NONFINITE like fr_step. */
fr_status fr_sync(fr_mesh *m);

/* out[0..7] = C_L, C_D, F_x, F_y, F_z of the last step; mean C_L, mean C_D
 * over the steps since the state was set; number of steps averaged.
 * Lift and drag come from the wall traction integral of (p n - tau . n),
 * with p and the stress tau of Eqs. (5)-(6) of Section 2.1; the means are
 * the time-averaged lift and drag coefficients of the objective of Section
 * 3.4 (summed in FP64).  If the wall forces of the last step's state are
 * not yet in the sums (fr_step adds them in the next step), this call first
 * runs their force pass on the mesh's stream.  out is host memory of 8
 * doubles; FR_E_ARG for a design index outside the batch. */
fr_status fr_forces(const fr_mesh *m, int32_t design, double *out);

/* Test hook: R(u) = du/dt of the semi-discretisation, i.e. -div F of Eq. (1)
 * of Section 2.1 with F = F_inv - F_vis of Eqs. (3)-(4), host FP64 canonical
 * arrays in and out ([points][variables], caller-owned).  Leaves the current
 * state untouched. */
fr_status fr_residual(fr_mesh *m, const double *u, double *r);

/* Device pointer and layout of the state, for callers that keep data on
 * the device: blocks of 16 elements, each split into 4 sub-blocks of 4;
 * layout [block][sub-block][n_u padded to 16][variables][4 elements]. */
fr_status fr_state_device(const fr_mesh *m, void **ptr, int64_t *bytes);

/* Kernel-timing hook for benchmarks: runs `steps` RK4 steps with HIP events
 * around every launch on the handle's stream and returns, per kernel id, the
 * summed milliseconds and the launch count in ms_per_kernel[0..7] and
 * launches[0..7] (index 0 = all kernels).  Kernel ids: 1 face, 2 gradient
 * and flux, 3 viscous trace, 4 divergence and RK update, 5 interpolation,
 * 6 fused stage part a, 7 fused stage part b. */
fr_status fr_profile_kernels(fr_mesh *m, int64_t steps, double *ms_per_kernel, int64_t *launches);

/* Kernel structure and operator back-end.  Bit 0 set: each RK stage is two
 * fused launches (faces, gradient, fluxes and volume divergence; then the
 * flux correction, RK update and next trace), with the operators applied by
 * sum factorisation along the solution-point lines.  Bit 0 clear: five
 * launches per stage (face, gradient/flux, viscous trace, divergence/RK
 * update, interpolation); bit k (k = 2, 3, 4, 5 for those four operator
 * kernels) set selects sum factorisation (VALU, LDS-staged inputs), clear
 * the dense element-batched MFMA contraction.  Bit 6 (3D, fused stage): read
 * the stored FP64 metrics instead of forming S, |J|, the face normals and
 * areas in FP64 from each element's 27 geometry nodes.  Bit 8 (meshes whose
 * elements are all z-extruded, x and y the same in every node layer and z a
 * function of zeta alone, as spanwise-extruded airfoil grids and boxes are):
 * form them from per-element column metrics instead, the 2D Jacobian at the
 * solution-point columns, z_zeta per layer and the face columns (FP64; the
 * default on such meshes; FR_E_UNSUPPORTED on others).  Bit 7 set turns off
 * the remap that sends the workgroups of consecutive element blocks to one
 * XCD (and so into one L2).  Every choice gives the same result
 * to round-off (bit 7 bit for bit).  The default is the last
 * autotuned choice for this (precision, dim, order, size class) in the
 * process, else the fused stage with metrics from the nodes (column metrics
 * on an extruded mesh). */
fr_status fr_select_kernels(fr_mesh *m, int32_t mask);
fr_status fr_selected_kernels(const fr_mesh *m, int32_t *mask);

/* Autotuner: times the fused stage (in 3D with metrics from the nodes and
 * with stored metrics, and with column metrics on an extruded mesh, each with
 * and without the XCD remap of bit 7) and
 * both variants of every split operator kernel for
 * `steps` steps on this mesh with HIP events (the state is saved and
 * restored), keeps the fastest configuration, records it for later meshes of
 * the same precision, dimension, order and size class (the bit length of the
 * count of 16-element blocks), and returns the mask. */
fr_status fr_autotune(fr_mesh *m, int64_t steps, int32_t *mask_out);

/* ---- served requests: continuous batching under an HBM budget ---------- */

/* A pool admits solve requests while their device footprint fits in
 * hbm_budget bytes; admitted requests run concurrently on the device.  Pool
 * calls are thread-safe: one host thread may admit requests (building their
 * meshes) while another launches and collects steps. */
fr_status fr_pool_create(size_t hbm_budget, int32_t device, fr_pool **out);
void fr_pool_destroy(fr_pool *p);

/* Bytes of device memory a request with this descriptor would hold. */
fr_status fr_footprint(const fr_mesh_desc *desc, size_t *bytes);

/* Admit a request that runs `steps` RK4 steps from state u0 (canonical
 * FP64, may be NULL for the uniform free stream).  FR_E_NOMEM if it does
 * not fit now; nothing is allocated then.  *slot identifies it. */
fr_status fr_pool_admit(fr_pool *p, const fr_mesh_desc *desc, const double *u0, int64_t steps,
                        int64_t *slot);

/* Enqueue up to k further steps for every running request and wait for
 * them.  Slots that have finished are written to done[0..*n_done-1]
 * (capacity max_done). */
fr_status fr_pool_tick(fr_pool *p, int64_t k, int64_t *done, int32_t max_done, int32_t *n_done);

/* The two halves of fr_pool_tick: enqueue up to k steps for every running
 * request without waiting (the host is then free, e.g. to admit requests),
 * and wait for the enqueued steps and report the requests that finished
 * (or failed: their fr_pool_result returns the error). */
fr_status fr_pool_launch(fr_pool *p, int64_t k);
fr_status fr_pool_collect(fr_pool *p, int64_t *done, int32_t max_done, int32_t *n_done);

/* Result of a finished request (fr_forces layout) and its state if u is
 * not NULL; frees the slot and its device memory. */
fr_status fr_pool_result(fr_pool *p, int64_t slot, double *out, double *u);

/* used[0] = bytes held, used[1] = running requests. */
fr_status fr_pool_usage(const fr_pool *p, int64_t *used);

/* ---- Sampling the solution at points ---------------------------------
 *
 * The discrete FR solution inside an element is the tensor-product Lagrange
 * interpolant through its Gauss-Legendre solution points.  A probe locates
 * each point in the mesh (Newton's method on the element geometry map; the
 * lowest-index element whose reference cube holds the point, among those
 * whose node bounding box, padded by a tenth of its largest extent, holds
 * it) and evaluates that interpolant of the current state: the flow samples
 * on the permeable data surface of the paper's Section 3.1.
 */

/* Locate n points ([n][3]; dim 2 ignores z) in design `design` of mesh m,
 * whose descriptor is desc (the one m was built from).  The probe refers to
 * m, which must outlive it.  FR_E_ARG if a point lies in no element. */
fr_status fr_probe_create(fr_mesh *m, const fr_mesh_desc *desc, int32_t design, int64_t n,
                          const double *points, fr_probe **out);
void fr_probe_destroy(fr_probe *p);

/* Host copies of the located elements (canonical index within the design,
 * [n]) and reference coordinates ([n][3]). */
fr_status fr_probe_locate(const fr_probe *p, int64_t *elem, double *xi);

/* The current state at the points: host [n][variables], conserved, FP64.
 * FR_E_STATE if the mesh has no state. */
fr_status fr_probe_sample(fr_probe *p, double *out);

/* ---- Far-field acoustics: FW-H from a permeable data surface ----------
 *
 * The acoustic pressure at an observer from flow samples on a stationary
 * permeable data surface in a uniform stream (the paper's Appendix A source
 * terms and Appendix B solution of the FW-H equation with a moving medium,
 * quadrupole term dropped), summed by the advanced-time approach of
 * Appendix B, with spanwise copies of the surface (Section 3.3: the data
 * surface of a spanwise-periodic flow is repeated along the span).
 *
 *   Q   = rho (u_n + U_n) - rho0 U_n,  L_i = (p - p0) n_i + rho u_i (u_n + U_n)
 *   4 pi p'_T = sum_S [(1 - M_R) Qdot / R* - c0 Q M_R* / R*^2] dS
 *   4 pi p'_L = sum_S [Ldot_R / (c0 R*) + L_R* / R*^2] dS
 *
 * with u the flow velocity relative to the stream (disturbance velocity),
 * R*, R the amplitude and phase radii of the stream, and every panel's
 * samples arriving at t = tau + R / c0.  Time derivatives are fourth-order
 * central differences (the two samples at each end of the record have
 * none); panel series are interpolated to the observer times by cubic
 * Lagrange interpolation.  The observer times are spaced by the sampling
 * interval dt and run from the latest first arrival plus dt to the earliest
 * last arrival less 2 dt, so that every stencil lies inside every panel's
 * record.  FP64 throughout; results do not depend on launch shapes (fixed
 * summation order).
 */
typedef struct fr_fwh fr_fwh;

typedef struct {
  int64_t n_points;        /* panels of one copy of the data surface */
  const double *points;    /* [n_points][3] panel centres (copied) */
  const double *normals;   /* [n_points][3] outward unit normals (copied) */
  const double *areas;     /* [n_points] panel areas (copied) */
  int32_t n_copies;        /* >= 1; copy k sits at (k - (n_copies - 1) / 2) copy_shift */
  double copy_shift[3];
  double mach[3];          /* free-stream Mach vector, |M| < 1 */
  double c0, rho0, p0;     /* free-stream sound speed, density, pressure */
  double dt, tau0;         /* sampling interval, time of the first sample */
  int64_t capacity;        /* samples per panel the record holds, >= 8 */
  int32_t device;
  void *stream;            /* hipStream_t, or NULL */
  fr_alloc_fn alloc;       /* optional device allocator, as in fr_mesh_desc */
  fr_free_fn free;
  void *alloc_ctx;
} fr_fwh_desc;

/* Create a record of capacity * n_points samples on the device
 * (4 * 8 bytes per sample).  FR_E_ARG for an invalid descriptor. */
fr_status fr_fwh_create(const fr_fwh_desc *desc, fr_fwh **out);
void fr_fwh_destroy(fr_fwh *h);

/* Append n snapshots: host [n][n_points][5] = rho, u1, u2, u3, p with u the
 * disturbance velocity; their source strengths are formed on the device.
 * FR_E_ARG when the record would exceed its capacity. */
fr_status fr_fwh_append(fr_fwh *h, int64_t n, const double *samples);

/* Append one snapshot sampled by probe p (its points are the record's
 * panels, in order): the mesh state at the points, as rho, u - U, p with U
 * the record's stream velocity c0 M, straight from the device.  FR_E_ARG if
 * the probe's point count differs from the record's. */
fr_status fr_fwh_append_probe(fr_fwh *h, fr_probe *p);

/* Snapshots recorded so far. */
fr_status fr_fwh_samples(const fr_fwh *h, int64_t *n);

/* Observer-time window for observer[3]: first time and number of times.
 * FR_E_STATE if the record is shorter than the spread of arrival times. */
fr_status fr_fwh_window(fr_fwh *h, const double *observer, double *t_start, int64_t *n_out);

/* p'(t) at observer[3] on the window's times, into host p[capacity]; its
 * thickness and loading parts into p_thickness and p_loading when those are
 * not NULL.  FR_E_ARG if capacity is below the window length. */
fr_status fr_fwh_pressure(fr_fwh *h, const double *observer, int64_t capacity, double *t_start,
                          int64_t *n_out, double *p, double *p_thickness, double *p_loading);

/* p'(t) at observer[3] on the caller's grid t_start + m dt, m < n, which must
 * lie inside the window of fr_fwh_window (FR_E_ARG otherwise): to align
 * several observers or runs on one time grid. */
fr_status fr_fwh_pressure_at(fr_fwh *h, const double *observer, double t_start, int64_t n, double *p,
                             double *p_thickness, double *p_loading);

/* Allocation-free variant of fr_fwh_pressure_at, for callers that cannot
 * allocate device memory while they run: work under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, kernels and
 * results (bit for bit) as fr_fwh_pressure_at; the evaluation's intermediate
 * arrays (per-panel combined filters and first samples, partial sums, outputs)
 * live in one static device array of 64 MiB instead of buffers the record
 * grows, and the call allocates nothing.  The library holds that array on every
 * GPU it runs on until the process ends.  Limit: n_points panels at n observer
 * times need, in bytes, each term rounded up to 256,
 *   8576 n_points + 16 n_points + 16 n ceil(n_points / 8) + 1024 n + 24 n
 * (e.g. 3,000 panels at 4,000 observer times); a larger request returns
 * FR_E_ARG before anything runs.  Every call on one GPU uses the same array and
 * leaves its contents behind (each evaluation writes every element it reads
 * first): calls that overlap on one GPU, from different threads or streams,
 * race, and the caller must serialise them. */
fr_status fr_fwh_pressure_at_noalloc(fr_fwh *h, const double *observer, double t_start, int64_t n, double *p,
                                     double *p_thickness, double *p_loading);

/* Device time (ms) of the last fr_fwh_pressure or fr_fwh_pressure_at (HIP
 * events on its stream around the per-panel filter, summation and reduction
 * kernels). */
fr_status fr_fwh_time_ms(const fr_fwh *h, double *ms);

/* ---- Served requests with a data surface -------------------------------
 *
 * One candidate design of the optimisation loop (Algorithm 1): its flow is
 * advanced, sampled on a permeable data surface and propagated to the far
 * field by the FW-H solver above, while other candidates run beside it in
 * the same pool.  After `warmup` steps the state is sampled at the surface
 * points (as fr_probe_sample, design 0) every `every` steps, n_samples
 * times, the first sample at source time 0, and each snapshot is appended to
 * an FW-H record (as fr_fwh_append_probe) without a host round trip.  The
 * record's medium is the request's free stream (desc->freestream = rho, u,
 * v, w, p): c0 = sqrt(gamma p / rho), Mach vector (u, v, w) / c0, rho0 =
 * rho, p0 = p; its sampling interval is every * desc->dt.  The running lift
 * and drag means restart at the first sample, so the request's result
 * (fr_pool_result) holds the means over the sampled period: the mean
 * coefficients of the objective of Section 3.4.
 */
typedef struct {
  int64_t n_points;        /* panels of one copy of the data surface */
  const double *points;    /* [n_points][3] panel centres (copied) */
  const double *normals;   /* [n_points][3] outward unit normals (copied) */
  const double *areas;     /* [n_points] panel areas (copied) */
  int32_t n_copies;        /* spanwise copies, as fr_fwh_desc */
  double copy_shift[3];
  int64_t warmup;          /* steps before the first sample, >= 0 */
  int64_t every;           /* steps between samples, >= 1 */
  int64_t n_samples;       /* snapshots, >= 8 */
} fr_pool_surface;

/* Admit a request that runs warmup + (n_samples - 1) * every steps from u0
 * (as fr_pool_admit) and samples the surface s.  Its footprint includes the
 * probe and the record.  FR_E_NOMEM if it does not fit now (nothing is
 * allocated then); FR_E_ARG for an invalid surface or a point that lies in
 * no element. */
fr_status fr_pool_admit_sampled(fr_pool *p, const fr_mesh_desc *desc, const double *u0,
                                const fr_pool_surface *s, int64_t *slot);

/* Acoustic pressure at observer[3] of a finished sampled request, with the
 * arguments and results of fr_fwh_pressure (no thickness and loading
 * parts).  Call it before fr_pool_result, which frees the request.
 * FR_E_STATE if the request has not finished, failed, or has no surface. */
fr_status fr_pool_pressure(fr_pool *p, int64_t slot, const double *observer, int64_t capacity,
                           double *t_start, int64_t *n_out, double *pressure);

const char *fr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FR_H */
