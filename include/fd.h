/*
 * fd.h -- C ABI of libfd, the MI355X (gfx950) Fast-Diagonalization library.
 *
 * The library applies the inverse of Kronecker-sum preconditioner blocks
 *
 *     P = sum_i w_i (M_d (x) ... (x) K_i (x) ... (x) M_1)          (1)
 *
 * (Montardini, Sangalli, Tani 2018, Sec. 5 eq. prec3D_TH for the velocity
 * blocks P_V,k, eq. precQ for the pressure block P_Q = M_d (x) .. (x) M_1,
 * and the Appendix for the coefficient-aware blocks) by the Fast
 * Diagonalization method of Sec. 5.2, Algorithm 1:
 *
 *     K_i U_i = M_i U_i D_i,  U_i^T M_i U_i = I                     (eq. eig_dec)
 *     z = (U_d (x) .. (x) U_1) Lambda^{-1} (U_d (x) .. (x) U_1)^T r,
 *     Lambda = sum_i w_i (I (x) .. (x) D_i (x) .. (x) I).
 *
 * Optionally with the diagonal scaling of Sec. 6: P^G = D^{1/2} P D^{1/2},
 * [D]_ii = [target]_ii / [P]_ii, so z = D^{-1/2} P^{-1} D^{-1/2} r.
 *
 * Vector layout (Sec. 2.3, definition of vec): a block of sizes
 * (n_1, .., n_d) is a vector of prod(n_i) elements with i_1 fastest.
 *
 * Conventions for every call:
 *  - Host pointers are read during the call only; the caller keeps ownership
 *    and may free them on return.
 *  - Device pointers are caller-owned device memory (e.g. from torch); the
 *    library never frees them.
 *  - Every call returns an fd_status. On failure a thread-local message is
 *    available from fd_last_error(); no exception crosses the ABI.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream). Work
 *    is enqueued asynchronously; execution errors surface at the caller's
 *    synchronisation.
 */
#ifndef FD_H_
#define FD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FD_OK = 0,
  FD_E_ARG = 1,          /* invalid argument: sizes, NULL pointers, asymmetric input */
  FD_E_NOTSPD = 2,       /* M not positive definite, or an eigenvalue sum <= 0 */
  FD_E_NOMEM = 3,        /* host or device allocation failed */
  FD_E_HIP = 4,          /* a HIP runtime call failed (message names it) */
  FD_E_UNSUPPORTED = 5   /* valid request the library does not implement */
} fd_status;

/* Arithmetic of the mode products. FD_F64 plans take FP64 vectors; all other
 * plans take FP32 vectors and keep FP32 intermediates. The 1D eigensolve and
 * the Lambda^{-1} values are FP64 for every precision.
 *  FD_BF16 / FD_F16: operands rounded to bf16 / fp16, FP32 MFMA accumulation.
 *  FD_BF16_SPLIT / FD_F16_SPLIT: both operands split as hi + lo in the
 *  16-bit type; the products hi*hi + hi*lo + lo*hi are accumulated in FP32.
 *  FD_FP8_SPLIT: the same split with FP8 E4M3 operands (FP32 accumulation);
 *  each pass scales its data and each factor image by powers of two so that
 *  the 448 range limit is not reached (undone exactly on output). Only for
 *  plans without diag_target and with every n[i] <= 224, and not in
 *  persistent batches (FD_E_UNSUPPORTED otherwise). */
typedef enum {
  FD_F64 = 0,
  FD_F32 = 1,
  FD_BF16 = 2,
  FD_F16 = 3,
  FD_BF16_SPLIT = 4,
  FD_F16_SPLIT = 5,
  FD_FP8_SPLIT = 6
} fd_precision;

typedef struct fd_plan_s* fd_plan;

/* One unit of work for fd_apply / fd_apply_batched: apply `plan` to `nrhs`
 * vectors. Vector j starts at r + j*ld (elements) and its result is written
 * at z + j*ld. ld >= N of the plan. z may alias r exactly (in-place apply);
 * partially overlapping r and z are not allowed. r and z are FP64 for FD_F64
 * plans and FP32 otherwise. Between the passes of Algorithm 1 the library
 * keeps its intermediate tensors in z, so z must not be read by others before
 * the apply completes. */
typedef struct {
  fd_plan plan;
  const void* r;
  void* z;
  int32_t nrhs;
  int64_t ld;
} fd_work;

/* ---------------------------------------------------------------- host-only */

/* Univariate factors on a uniform mesh of [0,1] (Sec. 5, the matrices below
 * eq. prec3D_TH and eq. precQ; weighted pairs of the Appendix):
 *   [K]_ls = int tau b'_l b'_s,  [M]_ls = int mu b_l b_s,
 * over the B-splines of `degree` on the open uniform knot vector with n_el
 * elements and interior knot multiplicity degree - regularity (Sec. 2.1).
 * dirichlet != 0 drops the first and last function. Quadrature: `npts`
 * Gauss-Legendre points per element (npts <= 0 selects degree + 1).
 * tau_q / mu_q: NULL (weight 1) or n_el*npts weights at the quadrature points,
 * element-major, points in increasing order inside each element.
 * *n_out receives the matrix order m; K and M (host, caller-allocated, may be
 * NULL to query m only) receive m*m column-major entries.
 * Errors: FD_E_ARG for n_el < 1, degree < 1 or > 12, regularity outside
 * [-1, degree-1], npts > 16, or m < 1 after the boundary condition. */
fd_status fd_assemble_1d(int32_t n_el, int32_t degree, int32_t regularity, int32_t dirichlet,
                         int32_t npts, const double* tau_q, const double* mu_q,
                         int32_t* n_out, double* K, double* M);

/* The Nitsche-modified stiffness factor K~ of the Raviart-Thomas velocity
 * blocks (Sec. 5, the factors below eq. prec3D_RT), over all m B-splines of
 * the degree/regularity space on the uniform mesh (no function dropped):
 *   [K~]_ls = int b'_l b'_s - ( b'_l(1) b_s(1) - b'_l(0) b_s(0)
 *             + b'_s(1) b_l(1) - b'_s(0) b_l(0) )
 *             + 2 (c_pen / h) ( b_l(1) b_s(1) + b_l(0) b_s(0) ),   h = 1 / n_el,
 * the one-direction face terms of the parametric Nitsche form. The matching
 * mass factor is fd_assemble_1d's M with dirichlet = 0; the experiments use
 * c_pen = 5 (regularity + 1). *n_out receives m; K (host, m*m column-major,
 * caller-allocated) may be NULL to query m only. Errors: FD_E_ARG as
 * fd_assemble_1d, or c_pen < 0. */
fd_status fd_nitsche_stiffness_1d(int32_t n_el, int32_t degree, int32_t regularity, double c_pen, int32_t* n_out,
                                  double* K);

/* Mixed univariate integrals over all functions of two spline spaces on the
 * uniform mesh of fd_assemble_1d: X[l][m] = int b_{a,l}^(da) b_{b,m}^(db),
 * da, db in {0, 1} (value or first derivative), space a of (deg_a, reg_a),
 * space b of (deg_b, reg_b), no function dropped. These are the factors of
 * the Stokes blocks that the preconditioner does not hold (Sec. 3: the
 * off-diagonal velocity blocks A_rs and the divergence blocks B_r of the
 * cube). Quadrature: npts Gauss points per element (npts <= 0 selects
 * max(deg_a, deg_b) + 2, exact for these products). *ma, *mb receive the
 * space dimensions; X (host, ma*mb column-major) may be NULL to query them.
 * Errors: FD_E_ARG. Host computation only. */
fd_status fd_mixed_1d(int32_t n_el, int32_t deg_a, int32_t reg_a, int32_t da, int32_t deg_b, int32_t reg_b,
                      int32_t db, int32_t npts, int32_t* ma, int32_t* mb, double* X);

/* Gauss-Legendre points and weights on the element mesh used by
 * fd_assemble_1d: x, w host arrays of n_el*npts (element-major). */
fd_status fd_quadrature_1d(int32_t n_el, int32_t npts, double* x, double* w);

/* Step 1 of Algorithm 1 for one direction (eq. eig_dec): U (n*n column-major,
 * columns are eigenvectors) and d (n, ascending) with K U = M U diag(d),
 * U^T M U = I. K, M: host, n*n column-major, symmetric to 1e-12 relative.
 * K may be NULL (mass-only: d = 0, U = M^{-1/2} in the Cholesky sense).
 * Errors: FD_E_ARG (n < 1, NULL M, asymmetry), FD_E_NOTSPD (Cholesky of M
 * fails). Host computation only; needs no GPU. */
fd_status fd_factor_1d(int32_t n, const double* K, const double* M, double* U, double* d);

/* ------------------------------------------- coefficient-aware blocks */

/* Coefficient matrices of the TH velocity blocks (Sec. 3, eq. Q_TH):
 * C_k = nu (J^{-1} J^{-T} + D_k D_k^T) |det J|, D_k = J^{-1} e_k, and the
 * TH pressure-mass weight nu^{-1} |det J| (eq. weighted-pressure-mass), at
 * npts points.
 *  jac : host, npts * ndim * ndim, point-major, row-major per point:
 *        jac[(p*ndim + a)*ndim + b] = dG_a / deta_b.
 *  nu  : host, npts viscosity values at the physical points G(eta_p).
 *  component: -1 for every C_k, or one k in [0, ndim) (then C holds only
 *        that matrix, as if k were 0 below).
 *  C   : host output or NULL, ndim^3 * npts (ndim^2 * npts for one
 *        component), field-major:
 *        C[((k*ndim + a)*ndim + b)*npts + p] = (C_k)_{ab} at point p.
 *  q_weight: host output or NULL, npts.
 * Errors: FD_E_ARG (ndim not 2 or 3, npts < 1, NULL inputs, a singular
 * Jacobian or nu <= 0 at some point). Host computation only. */
fd_status fd_geometry_coefficients(int32_t ndim, int64_t npts, const double* jac, const double* nu,
                                   int32_t component, double* C, double* q_weight);

/* Separable approximation of the diagonal of one C_k (Appendix):
 * c_jj(eta) ~ tau_j(eta_j) prod_{i != j} mu_i(eta_i) on a tensor grid of
 * nq[0] x .. x nq[ndim-1] quadrature points (direction 1 fastest).
 *  c     : host, entry j's field starts at c + j*stride (stride >= prod nq);
 *          for C_k as laid out by fd_geometry_coefficients, c = C +
 *          k*ndim*ndim*npts and stride = (ndim + 1)*npts. Entries must be > 0.
 *  sweeps, tol: at most `sweeps` sweeps of the alternating midrange
 *          (Diliberto-Straus) fit of log c_jj, stopping early once no
 *          factor value moves by more than tol (in log scale).
 *  tau, mu: host outputs, sum(nq) values, direction 1's points first.
 * The non-tau factors of each fit are normalised to geometric mean 1 (the
 * constant goes into tau_j) and mu_i is the geometric mean of the estimates
 * from the entries j != i. Errors: FD_E_ARG. Host computation only. */
fd_status fd_separable_factors(int32_t ndim, const int32_t* nq, const double* c, int64_t stride,
                               int32_t sweeps, double tol, double* tau, double* mu);

/* Diagonal of a Galerkin operator with pointwise coefficients on the
 * tensor-product spline space of fd_assemble_1d's (n_el[i], degree,
 * regularity, dirichlet) in every direction, with the quadrature grid of
 * npts Gauss points per element (npts <= 0: degree + 1):
 *  order 1: [A]_ii = int sum_{a,b} c_ab d_a B_i d_b B_i, coef holds ndim^2
 *           fields, field (a, b) at coef + (a*ndim + b)*P (the layout of one
 *           C_k from fd_geometry_coefficients), P = prod(n_el[i]*npts);
 *  order 0: [Q]_ii = int c B_i^2, coef holds one field of P values.
 * Fields are on the grid with direction 1 fastest, element-major points per
 * direction. diag: host output, prod(n_i) values, i_1 fastest. This is
 * diag(A_kk) for D_V and diag(Q) for D_Q (Sec. 6): pass it to fd_setup as
 * diag_target. Errors: FD_E_ARG. Host computation only. */
fd_status fd_operator_diagonal(int32_t ndim, const int32_t* n_el, int32_t degree, int32_t regularity,
                               int32_t dirichlet, int32_t npts, int32_t order, const double* coef,
                               double* diag);

/* ---------------------------------------------------------------- plans */

/* Build a plan for one block (1) with ndim in {2, 3} directions.
 *  n[i]      : order of the direction-i factors (2 <= n[i] <= 256), with
 *              N = prod(n) < 2^28.
 *  K[i], M[i]: host FP64, n[i]*n[i] column-major, symmetric; M[i] SPD.
 *              K == NULL makes a mass-only plan (P = M_d (x) .. (x) M_1,
 *              Lambda = I, eq. precQ).
 *  w         : ndim direction weights (NULL = all ones); eq. prec3D_TH uses
 *              weight 2 on the direction of the velocity component.
 *  diag_target: NULL, or N = prod(n) host FP64 values, the diagonal of the
 *              matrix the block stands for (A_kk or Q of Sec. 6); the plan then
 *              applies z = D^{-1/2} P^{-1} D^{-1/2} r with
 *              D = diag_target / diag(P). Entries must be > 0.
 * The factors are computed in FP64 on the host, then packed in the precision
 * of `prec` and copied to the current HIP device (one copy per plan).
 * Errors: FD_E_ARG, FD_E_NOTSPD (M not SPD, or Lambda has an entry <= 0, or
 * a diag_target/diag(P) ratio <= 0), FD_E_NOMEM, FD_E_HIP. */
fd_status fd_setup(int32_t ndim, const int32_t* n, const double* const* K,
                   const double* const* M, const double* w, const double* diag_target,
                   fd_precision prec, fd_plan* out);

/* Release the plan and its device memory. The caller must make sure no apply
 * using it is still executing. NULL is accepted. */
fd_status fd_destroy(fd_plan plan);

/* A mass-only plan (P_Q = M_d (x) .. (x) M_1, eq. precQ) applied by the
 * banded route of Sec. 5.2: each M_i (host FP64, n[i]*n[i] column-major,
 * symmetric positive definite, bandwidth b_i <= 16, e.g. b_i = degree for
 * B-spline mass matrices) is factored M_i = L_i L_i^T on the host in FP64,
 * and an apply runs one launch per direction that solves L_i L_i^T along
 * that mode for every pencil (O(b_i n_i) per pencil instead of the FD
 * form's O(n_i^2)); arithmetic in FP64 for FD_F64 plans, FP32 otherwise
 * (vectors as for fd_setup). The plan works with fd_apply and
 * fd_apply_batched (alone or beside FD plans of the same I/O type); the
 * persistent batch and fd_plan_factors refuse it (FD_E_UNSUPPORTED).
 * Errors: FD_E_ARG (sizes as fd_setup, asymmetry, bandwidth above 16),
 * FD_E_NOTSPD, FD_E_NOMEM, FD_E_HIP. */
fd_status fd_setup_mass_banded(int32_t ndim, const int32_t* n, const double* const* M, fd_precision prec,
                               fd_plan* out);

/* Plan queries: N = prod(n); device bytes held by the plan. */
int64_t fd_plan_size(fd_plan plan);
size_t fd_plan_device_bytes(fd_plan plan);

/* Device-memory cap, for callers that budget HBM (a plan cache under a
 * budget, a service sharing the GPU): the device bytes the library holds at
 * once (plans, fixed-batch tables, setup temporaries; never the caller's r
 * and z) stay at or below `bytes`; 0 removes the cap (the default). An
 * fd_setup, fd_setup_mass_banded or fd_batch_create whose allocation would
 * pass the cap fails with FD_E_NOMEM, exactly as on an exhausted device, and
 * holds nothing afterwards. Lowering the cap below what is held frees
 * nothing; it refuses later allocations. Process-wide (all devices,
 * all threads). Always FD_OK. */
fd_status fd_set_device_limit(size_t bytes);
/* Device bytes the library holds now, the quantity the cap bounds. */
size_t fd_device_bytes_held(void);
/* Device workspace an apply of `nrhs` vectors needs beyond the plan and the
 * caller's r and z: 0. The first pass reads r and writes z, every later pass
 * of Algorithm 1 runs in place on z (a tile reads all of its pencils before
 * it stores them, and tiles own disjoint pencils), so callers that budget
 * device memory count only the plan bytes and their vectors. */
size_t fd_workspace_bytes(fd_plan plan, int32_t nrhs);

/* Copy the FP64 factors of direction `dir` back to host arrays (U: n*n
 * column-major, d: n; either may be NULL). For tests and diagnostics. */
fd_status fd_plan_factors(fd_plan plan, int32_t dir, double* U, double* d);

/* ---------------------------------------------------------------- apply */

/* z = P^{-1} r (Algorithm 1, steps 2-4) for nrhs vectors of one plan, on
 * `stream`. Launch errors are returned; there is no host synchronisation. */
fd_status fd_apply(fd_plan plan, const void* r, void* z, int32_t nrhs, int64_t ld, void* stream);

/* Apply a heterogeneous list of work units (different plans, sizes and
 * dimensions; all plans of one precision class: FD_F64, or FP32-I/O) as one
 * set of launches on `stream`: each pass of Algorithm 1 is one launch over the
 * tiles of every unit. Equivalent to calling fd_apply on each unit. */
fd_status fd_apply_batched(int32_t count, const fd_work* work, void* stream);

/* ------------------------------------------------------ persistent batch */

/* A prepared batched apply that runs as ONE persistent kernel launch.
 *
 * fd_batch_create takes a fixed list of works (as for fd_apply_batched; all
 * plans of one precision class, every factor order n <= 128) and lays out
 * the passes of Algorithm 1 of every work stage by stage on the device. Each
 * fd_batch_apply is then a single launch of a persistent grid (every
 * workgroup resident) that walks the tiles of each stage and meets at a
 * grid-wide barrier between stages; a tile runs the pass body of its unit
 * (factor staged in LDS), so patches of different sizes, degrees and
 * precisions of one class share the launch. The r and z buffers named in the
 * works are fixed at creation; their contents may change between applies.
 *
 * The grid is one 8-wavefront workgroup per CU. A stage runs each of its
 * passes with one of three bodies: 0 wide (factor resident in LDS, the
 * register-budget tile width), 1 narrow (factor resident in LDS, one 16-pencil
 * tile per wavefront), 2 pipelined (factor and pencil blocks streamed through
 * an LDS ring by direct loads; FP64/FP32/BF16/FP16 passes that scale neither
 * input nor output, the other passes of the stage run wide). The
 * configuration word holds the choice of stage s in bits 2s and 2s + 1.
 * fd_batch_tune chooses greedily stage by stage: it times the whole apply
 * (`reps` launches on `stream`, after one warm-up) with each choice that
 * changes the stage and keeps the fastest; later applies use the result
 * (*choice = the configuration word). An untuned batch runs every stage
 * wide. Tuning synchronizes the device.
 *
 * Staged route (configuration word 1 << 10): when every work of the batch is
 * a 3D BF16/FP16 plan on the slab route (Sec. 5.2, Algorithm 1 steps 2-4 as
 * a slab pass over the two in-plane modes, the fused last-mode pass and a
 * slab pass back, the tensor kept in 16 bits inside z in between), an apply
 * is instead one launch per stage and row-tile group (at most 3 x 9), each
 * reading its units from a table built at creation; no grid barrier, so it
 * needs no co-resident grid. fd_batch_tune times it after the greedy search
 * and keeps it if faster; fd_batch_set_config(1 << 10) on a batch without
 * it is FD_E_UNSUPPORTED. Results agree with the persistent route within the
 * precision's rounding (the routes round intermediates differently).
 *
 * Applies of one batch must be ordered (one stream, or synchronized): they
 * share the barrier counter. A barrier wait is bounded: if the grid cannot be
 * fully resident (other kernels occupy the device), the waits give up after
 * seconds, the results are undefined and fd_batch_check reports FD_E_HIP.
 * fd_batch_check waits for the device and reports that flag (and then
 * restarts the counter, so the batch can run again). Errors of
 * create: FD_E_ARG (as fd_apply_batched), FD_E_UNSUPPORTED (mixed precision
 * classes, n > 128, factor image above LDS), FD_E_NOMEM, FD_E_HIP. */
typedef struct fd_batch_s* fd_batch;
fd_status fd_batch_create(int32_t count, const fd_work* work, fd_batch* out);
fd_status fd_batch_apply(fd_batch batch, void* stream);
fd_status fd_batch_tune(fd_batch batch, void* stream, int32_t reps, int32_t* choice);
/* Sets the body choices directly (a configuration word, e.g. from an earlier
 * tune; a choice of 3 is FD_E_ARG; 1 << 10 selects the staged route; bit 11
 * with body choices selects the segment route: every segment of the
 * persistent layout as a launch of its own with its own LDS size, in stage
 * order on the stream, bit-identical results, no grid barrier and hence no
 * co-residency requirement); synchronizes the device. fd_batch_tune also
 * times the segment route with the chosen bodies and keeps it if faster. */
fd_status fd_batch_set_config(fd_batch batch, int32_t config);
/* Tiles per apply, grid size and configuration word. */
fd_status fd_batch_info(fd_batch batch, int64_t* tiles, int32_t* grid, int32_t* config);
/* A 64-bit signature of what the batch's layout and tuned configuration
 * depend on (the device's CU count, the precision class and, per work, the
 * plan's sizes, route and scaling and nrhs; not the buffers): batches with
 * equal signatures may share a configuration word, so a caller can keep
 * tuning results across processes (fd_batch_set_config). FD_E_ARG on NULL. */
fd_status fd_batch_signature(fd_batch batch, uint64_t* sig);
fd_status fd_batch_check(fd_batch batch);
fd_status fd_batch_destroy(fd_batch batch);

/* The persistent batched apply without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): runs `count` works (the same
 * rules as fd_batch_create: one precision class, every n <= 128, no
 * FD_FP8_SPLIT) as ONE persistent launch with the body choices of the
 * configuration word `config` (as fd_batch_set_config; 0 = every stage wide),
 * computing the same results as an fd_batch with that configuration.
 * Per call it enqueues on `stream` a one-wavefront fill kernel that zeroes the
 * barrier counter and the status word, an asynchronous host-to-device copy of
 * the pass tables, and the batch kernel; it calls no hipMalloc, hipFree or
 * other allocating routine. The barrier counter, error flag and pass tables
 * live in a static device array of 2 MiB per GPU (allocated with the code
 * object, held until the process ends; set up on the first call on a device,
 * with that device current). Lists whose pass tables exceed it (about 9,000
 * passes, e.g. more than 400 3D patches of 4 blocks) are FD_E_ARG with a
 * message. Every call on one GPU shares that array: calls on different
 * streams that overlap on the device race and give undefined results; calls
 * ordered on one stream are safe. The host part is serialized internally.
 * `status`: NULL or a caller-owned device int32 set to 0 by this call and to
 * 1 if a grid-barrier wait gave up (the grid could not be fully resident;
 * the results are then undefined); read it after synchronizing. Errors:
 * FD_E_ARG (as fd_batch_create, a bad configuration word, tables above the
 * limit), FD_E_UNSUPPORTED (as fd_batch_create), FD_E_HIP. */
fd_status fd_apply_persistent_static(int32_t count, const fd_work* work, int32_t config, int32_t* status,
                                     void* stream);

/* ---------------------------------------------------------------- diagnostics */

/* Per-stage kernel timing. While enabled, the launches of each stage of
 * fd_apply / fd_apply_batched are bracketed by two HIP events recorded on the
 * stream the kernels run on. Stages: 0 mode-1 forward, 1 mode-2 forward,
 * 2 last-mode forward + Lambda^{-1} + last-mode backward, 3 mode-2 backward,
 * 4 mode-1 backward (2D plans use stages 0, 2, 4). fd_timing_read waits for
 * the recorded events, adds the milliseconds of each stage into ms[0..4] and
 * the number of bracketed stage executions into count[0..4] (both host arrays
 * of 5, overwritten), and clears the record. Not for concurrent use from
 * several host threads. */
fd_status fd_timing_enable(int32_t enable);
fd_status fd_timing_read(double* ms, int32_t* count);

/* Per-launch times of the last fd_timing_read: while timing is enabled every
 * kernel launch is also bracketed by two events, and fd_timing_read sums them
 * per launch class (stage, kernel family, largest factor order n of the
 * launch, precision). fd_timing_launches copies up to `capacity` classes into
 * `out` (host array) and stores the number of classes in *n_out. */
typedef struct fd_launch_time {
  int32_t stage;   /* 0..4 as above */
  int32_t family;  /* 3 pipelined LDS GEMM, 2 LDS-resident factor, 1 global factor */
  int32_t n;       /* largest factor order of the units in the launch */
  int32_t prec;    /* fd_precision */
  double ms;       /* summed milliseconds */
  int32_t count;   /* launches summed */
} fd_launch_time;
fd_status fd_timing_launches(int32_t capacity, fd_launch_time* out, int32_t* n_out);

/* Message of the last failed call on this thread ("" if none). */
const char* fd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FD_H_ */
