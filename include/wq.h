/*
 * wq.h -- C ABI of the MI355X (gfx950) weighted-quadrature matrix-formation
 * library.
 *
 * Method: Calabro, Sangalli, Tani, "Fast formation of isogeometric Galerkin
 * matrices by weighted quadrature" (arXiv:1605.01238).  The library forms,
 * row by row, the isogeometric Galerkin mass matrix M~ and stiffness matrix
 * S~ of the scalar model problem of Section 3 on one 3D tensor-product spline
 * patch of degree p with maximal continuity C^{p-1}:
 *   - univariate weighted-quadrature (WQ) rules, four per basis function and
 *     direction (Section 4, eqs. quadrule/exact/support; Algorithm 2),
 *   - the integrand coefficients at the global quadrature points (Section 3,
 *     eqs. mass2, stiff, coef_stiff; Algorithm 1),
 *   - every row by sum factorization (Section 6, eq. sumfactorization,
 *     Algorithm 3, and its stiffness analogue), written straight into a CSR
 *     slot.
 *
 * Conventions (all indices 0-based):
 *   - Direction 1 is fastest: the linear index of (i1, i2, i3) is
 *     i1 + n1*(i2 + n2*i3) (Section 3).  Row = test function i, column =
 *     trial function j.  Columns of a row are strictly increasing.  Every
 *     structurally nonzero pair (supports overlapping, Section 3) is stored,
 *     even if its value is 0.  No symmetrisation, no boundary conditions.
 *   - Quadrature points (Remark 4.1): all interior knots, midpoints of the
 *     internal knot-spans, and in each of the two boundary knot-spans [a,b]
 *     the p+1 points a + k(b-a)/(p+2), k = 1..p+1 (strictly inside).
 *     n_qp = 2*n_el + 2*p - 1 per direction.
 *   - Weight pairing (alpha, beta): beta = derivative order on the test
 *     function (inside the weight), alpha = derivative order on the trial
 *     function (the integrand).  The rule is exact:
 *       sum_q w^(alpha,beta)_{i,q} B_j^(alpha)(x_q) = int B_i^(beta) B_j^(alpha)
 *     for all j overlapping i, with minimum Euclidean norm (Algorithm 2).
 *   - Stiffness coefficient at a point: K = a * det(J) * J^{-1} J^{-T}
 *     (eq. coef_stiff, times the scalar diffusion coefficient a); the mass
 *     coefficient is det(J) (eq. mass2).
 *
 * Memory and streams: the library never allocates device memory.  The
 * caller allocates one workspace (size from wq_sizes) and all outputs, and
 * owns them.  A bound plan owns one HIP stream and two events of its own
 * (see wq_setup), released by wq_plan_destroy.  Device calls are
 * asynchronous on the given HIP stream (0 = the legacy default stream).
 * Host pointers are read before the call returns.  A plan is a host object;
 * it is not thread-safe; distinct plans are independent.
 * Ordering: the device calls of one plan share its workspace (tables, the
 * coefficient field and the first-contraction buffer), so they must be
 * ordered, e.g. issued on one stream; wq_assemble calls of one plan on
 * different streams without such ordering race on that buffer.  Calls on
 * distinct plans (distinct workspaces) may overlap freely.
 *
 * Errors: every call returns a wq_status; nothing is thrown across the ABI.
 * Host-detectable errors are returned immediately and leave the plan
 * unchanged.  Device-detected conditions (det J <= 0 at a quadrature point,
 * a breakdown of a weight solve) are latched in the workspace and reported
 * by wq_sync.  wq_last_error gives a human-readable message.
 */
#ifndef WQ_H
#define WQ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wq_plan wq_plan;

typedef enum {
  WQ_OK = 0,
  WQ_EINVAL = -1,     /* bad argument (null pointer, d, p, precision, flags) */
  WQ_EKNOTS = -2,     /* knot vector not open / not non-decreasing / repeated interior knot / too few spans */
  WQ_ESINGULAR = -3,  /* a weight system broke down on the device */
  WQ_EGEOM = -4,      /* det J <= 0 (or not finite) at some quadrature point */
  WQ_ENOSPACE = -5,   /* workspace smaller than wq_sizes requires, or misaligned */
  WQ_EDEVICE = -6,    /* a HIP runtime call failed */
  WQ_ESTATE = -7      /* call order violated (e.g. assemble before setup) */
} wq_status;

enum { WQ_MASS = 1, WQ_STIFF = 2 };
enum { WQ_FP64 = 0, WQ_FP32 = 1 };

/* Degrees the library is compiled for (kernels are instantiated per degree). */
#define WQ_MIN_P 2
#define WQ_MAX_P 6

typedef struct {
  int64_t n[3];          /* basis functions per direction, n_l = n_el,l + p */
  int64_t n_qp[3];       /* quadrature points per direction */
  int64_t n_rows;        /* N_DOF = n1 n2 n3 */
  int64_t nnz;           /* exact nonzeros per matrix (same pattern for M~ and S~) */
  int64_t n_qp_total;    /* N_QP = n_qp1 n_qp2 n_qp3 */
  size_t workspace_bytes;/* device workspace the caller must provide */
  size_t value_bytes;    /* bytes of one value array (nnz * 8 or nnz * 4) */
} wq_sizes_t;

/*
 * Create a plan (host only; no device work).
 *   d          3; 2 for a plane patch, 1 for a curve (Section 3 with two
 *              or one direction; Section 7.1 for d = 1).  A plan of d < 3
 *              reports n[k] = n_qp[k] = 1 for the absent directions and
 *              forms the rows of the lower-dimensional problem, of length
 *              #I_i1 #I_i2 (d = 2) or #I_i1 (d = 1), with the same calls.
 *              For d = 1 the stiffness matrix is that of (a u')' with
 *              K = a / J, the mass matrix that of u with weight J.
 *   p          degree, WQ_MIN_P..WQ_MAX_P; the same in every direction.
 *   n_knots[d] length of each knot vector (n_l + p + 1).
 *   knots[d]   host pointers to FP64 knot vectors: open (first and last
 *              p+1 knots equal), non-decreasing, interior knots simple
 *              (C^{p-1}); at least p+2 knot-spans per direction.  Non-uniform
 *              spacing is allowed (Section 2).  Copied into the plan.
 *   precision  WQ_FP64: coefficient field, operators, accumulation and
 *              values in FP64.  WQ_FP32: the same in FP32 ("FP32 bulk"),
 *              while weights, det J and J^{-1} are still computed in FP64.
 *   out        receives the plan (NULL on error).
 * Errors: WQ_EINVAL (also for a patch beyond the kernels' 32-bit index
 * limits: N_DOF or N_QP of 2^31 or more, or, for d = 3, n_qp1 * n_qp2 *
 * (2p+1) * 8 of 2^32 or more), WQ_EKNOTS.
 */
wq_status wq_plan_create(int d, int p, const int64_t* n_knots, const double* const* knots,
                         int precision, wq_plan** out);

/* Sizes of the problem and of the workspace (host only). */
wq_status wq_sizes(const wq_plan* plan, wq_sizes_t* out);

/* Parametric quadrature-point coordinates of direction dir (0..d-1) into the
 * host array x_host[n_qp[dir]] (host only; Remark 4.1). */
wq_status wq_qpoints(const wq_plan* plan, int dir, double* x_host);

/*
 * Bind the caller's device workspace (>= workspace_bytes, 256-byte aligned)
 * to the plan and upload the knot vectors into it (small host-to-device
 * copy, asynchronous on stream).  Must precede every call below.  Binding a
 * new workspace invalidates earlier setup.
 * Errors: WQ_EINVAL, WQ_ENOSPACE, WQ_EDEVICE.
 */
wq_status wq_bind(wq_plan* plan, void* workspace, size_t bytes, hipStream_t stream);

/*
 * Device setup (asynchronous on stream; reads only device memory):
 *   1. univariate stage for every direction and basis function: B-spline
 *      values and derivatives at the quadrature points (Algorithm 1), exact
 *      1D integrals by (p+1)-point Gauss per knot-span (Algorithm 1), and the
 *      four minimum-norm weight solves (Algorithm 2) in FP64;
 *   2. geometry stage at every quadrature point: J = dF/dzeta of the spline
 *      map F(zeta) = sum_i C_i B_i(zeta), det J, and the coefficient field
 *      (det J; K = a det J J^{-1} J^{-T}) stored in the plan's precision.
 *   ctrl_dev  device FP64 control points, [n3][n2][n1][3] (i1 fastest,
 *             physical x,y,z innermost; [n2][n1][2] for d = 2, [n1] for
 *             d = 1, which must increase strictly so that J > 0); copied
 *             into the workspace, so the
 *             caller may free it after the call has completed on stream.
 *   coef_dev  device FP64 array of the diffusion coefficient a at the
 *             quadrature points, [n_qp3][n_qp2][n_qp1] (q1 fastest), or NULL
 *             for a = 1.  Read during this call only.
 * Ordering: stage 1 runs on a stream owned by the plan, after all work
 * already queued on `stream`; wq_assemble, wq_weights and wq_sync wait for
 * it (on their own stream), so results are as if everything ran on
 * `stream`, while wq_pattern, wq_field and wq_set_coefficient, which do not
 * read its tables, may overlap it.
 * Errors: WQ_EINVAL, WQ_ESTATE, WQ_EDEVICE; det J <= 0 and solve breakdowns
 * are latched for wq_sync.
 */
wq_status wq_setup(wq_plan* plan, const double* ctrl_dev, const double* coef_dev, hipStream_t stream);

/*
 * NURBS (Section 3: a rational denominator enters through the factor c).
 * As wq_setup, for the rational map F = sum_i w_i C_i B_i / sum_i w_i B_i:
 *   weights_dev  device FP64 weights of the control points, [n3][n2][n1]
 *                (as ctrl_dev without its last axis), all > 0; copied into
 *                the workspace.  W <= 0 or det J <= 0 at a point is latched
 *                like a bad geometry (WQ_EGEOM at wq_sync).
 *   basis        WQ_BASIS_BSPLINE: test and trial functions are the
 *                B-splines (both matrices; only J is rational).
 *                WQ_BASIS_NURBS: they are the rational functions
 *                R_i = w_i B_i / W of the same net; the mass is formed with
 *                c = det J / W^2 and every entry (i, j) is then scaled by
 *                w_i w_j (one extra pass over the values).  The stiffness
 *                of rational functions is not formed: assembly calls with
 *                WQ_STIFF return WQ_EINVAL.
 * wq_set_coefficient and wq_qp_physical keep the rational map; a later
 * wq_setup returns the plan to a polynomial map.  Batches (wq_batch_create)
 * refuse plans set up with WQ_BASIS_NURBS.
 * Errors: as wq_setup; WQ_EINVAL for a null weights pointer or another basis.
 */
#define WQ_BASIS_BSPLINE 0
#define WQ_BASIS_NURBS 1
wq_status wq_setup_nurbs(wq_plan* plan, const double* ctrl_dev, const double* weights_dev, const double* coef_dev,
                         int basis, hipStream_t stream);

/* New control net on the same knots (a polynomial map; e.g. a shape
 * update, or the next geometry of a serving loop that shares knots and
 * degree): the geometry stage of wq_setup only — copies the net and
 * re-forms the coefficient field; the univariate rules of the last
 * wq_setup are kept (they depend only on the knots and p, Algorithm 2).
 * ctrl_dev and coef_dev as in wq_setup.  Requires a prior wq_setup; ordered
 * like every other call of the plan.
 * Errors: WQ_EINVAL (null net), WQ_ESTATE (no wq_setup yet), WQ_EDEVICE. */
wq_status wq_set_geometry(wq_plan* plan, const double* ctrl_dev, const double* coef_dev, hipStream_t stream);

/* New diffusion coefficient a on the same geometry: recomputes the
 * coefficient field (the geometry stage of wq_setup; the univariate rules
 * are kept); coef_dev as in wq_setup.  Requires a prior wq_setup.  Ordered
 * like every other call of the plan (see Ordering above): an assembly
 * still in flight on another stream must be waited for first, as the 3D
 * geometry passes also use the plan's first-contraction buffer as scratch.
 * Requests on a resident geometry (wq_assemble_request) avoid both: they
 * bring their own field and buffer. */
wq_status wq_set_coefficient(wq_plan* plan, const double* coef_dev, hipStream_t stream);

/* Physical quadrature points F(x_q) into x_dev[n_qp3][n_qp2][n_qp1][3]
 * (x_dev[n_qp2][n_qp1][2] for d = 2, [n_qp1] for d = 1; device FP64), e.g. to sample a
 * coefficient a(x).  Requires wq_setup. */
wq_status wq_qp_physical(const wq_plan* plan, double* x_dev, hipStream_t stream);

/*
 * CSR pattern (Section 3, sets I_i): row_ptr_dev[n_rows + 1] (int64) and
 * col_idx_dev[nnz] (int32), both device, caller-owned.  Rows have length
 * prod_l #I_{l,i_l} with #I = min(n-1, i+p) - max(0, i-p) + 1.  Requires
 * wq_bind (not wq_setup).
 */
wq_status wq_pattern(const wq_plan* plan, int64_t* row_ptr_dev, int32_t* col_idx_dev,
                     hipStream_t stream);

/*
 * Form the matrix values into CSR slots (Algorithm 3 and its stiffness
 * analogue), asynchronous on stream.
 *   which           WQ_MASS, WQ_STIFF or WQ_MASS|WQ_STIFF.
 *   mass_vals_dev   device array [nnz] of double (WQ_FP64) or float
 *                   (WQ_FP32); required iff which has WQ_MASS, else ignored.
 *   stiff_vals_dev  likewise for WQ_STIFF.
 * Values are in the order of wq_pattern's col_idx.  Requires wq_setup.
 * With both matrices the mass is formed on the plan's own stream (with a
 * first-contraction buffer of its own) beside the stiffness on `stream`,
 * which waits for it before any later work: the call is ordered on
 * `stream` as a whole.
 * Errors: WQ_EINVAL, WQ_ESTATE, WQ_EDEVICE.
 */
wq_status wq_assemble(wq_plan* plan, int which, void* mass_vals_dev, void* stiff_vals_dev,
                      hipStream_t stream);

/*
 * Requests: the matrices of a plan for a new diffusion coefficient a(x) on
 * its resident geometry (weights, operators, det J and J^{-1} of the last
 * wq_setup), formed into a caller-owned request context instead of the
 * plan's workspace, so that requests on one plan may run concurrently on
 * different streams (each with its own context and outputs; they only read
 * the plan).  Same method as wq_set_coefficient + wq_assemble (Section 3,
 * eq. coef_stiff times a; Section 6, Algorithm 3): the coefficients are the
 * plan's a = 1 field with K multiplied by a(x_q).
 *   wq_request_bytes     bytes of one request context.
 *   wq_assemble_request  ctx: device, >= wq_request_bytes, 256-byte aligned,
 *                        caller-owned, contents overwritten; coef_dev as in
 *                        wq_setup (NULL: a = 1); which, mass_vals_dev,
 *                        stiff_vals_dev as in wq_assemble.  Asynchronous on
 *                        stream.  The plan's field must be that of a = 1
 *                        (its last wq_setup or wq_set_coefficient had a NULL
 *                        coefficient), else WQ_ESTATE.
 * Errors: WQ_EINVAL, WQ_ESTATE, WQ_ENOSPACE, WQ_EDEVICE.
 */
wq_status wq_request_bytes(const wq_plan* plan, size_t* bytes);
wq_status wq_assemble_request(wq_plan* plan, void* ctx, size_t ctx_bytes, const double* coef_dev, int which,
                              void* mass_vals_dev, void* stiff_vals_dev, hipStream_t stream);

/*
 * Batches: many independent patches formed together (rows of different
 * patches are independent like the rows of one patch, Section 1; each patch
 * is Section 6, Algorithm 3 as in wq_assemble).  The patches are plans of
 * their own (created, bound and set up as usual; distinct plans; any mix of
 * degree, size, d and precision).  Per class of equal (p, d, precision) one
 * launch forms the first contraction of all its patches and one persistent
 * launch forms all their rows from a device work queue, or (a schedule the
 * autotuner may pick) the single-patch kernels run patch after patch on
 * the class's stream.  Classes run concurrently.  Values equal
 * wq_assemble's bit for bit.
 *   wq_batch_create  host only; n plans, copied as pointers (the plans must
 *                    outlive the batch and keep their workspaces while the
 *                    batch is used).  WQ_EINVAL on a null or repeated plan.
 *   wq_batch_sizes   bytes of the batch workspace (descriptors and work-queue
 *                    counters) and the number of classes.
 *   wq_batch_bind    device workspace (>= wq_batch_sizes, 256-byte aligned,
 *                    caller-owned) and the output arrays of every patch:
 *                    mass_vals[n] / stiff_vals[n] (device pointers, either
 *                    array may be NULL, entries NULL where not formed).
 *                    Uploads the descriptors on stream.  Every plan must be
 *                    bound; binding a plan again requires binding the batch
 *                    again.
 *   wq_batch_tune    autotuner: per class, times the candidate schedules
 *                    (runs of rows per pencil, persistent workgroups per
 *                    compute unit; or one launch per patch) on the bound
 *                    patches and keeps the fastest
 *                    for `which`; synchronizes stream.  Requires wq_setup of
 *                    every plan; overwrites the outputs.
 *   wq_batch_assemble  forms `which` for every patch, asynchronously on
 *                    stream.  use_graph != 0: the launch sequence is captured
 *                    once into a HIP graph (per which and stream; re-captured
 *                    after bind or tune) and replayed; needs a stream other
 *                    than the legacy default stream.
 *   wq_batch_schedule  class k: info[6] = {p, d, precision, patches,
 *                    work-item target, workgroups per compute unit (0: one
 *                    launch per patch)}.
 * Errors: WQ_EINVAL, WQ_ENOSPACE, WQ_ESTATE (unbound batch or plan, plan not
 * set up), WQ_EDEVICE; wq_batch_last_error gives the message.  Like plans, a
 * batch is a host object, not thread-safe; a batch and the plans it holds
 * must not be used concurrently on different streams.
 */
typedef struct wq_batch wq_batch;
wq_status wq_batch_create(int n, wq_plan* const* plans, wq_batch** out);
wq_status wq_batch_sizes(const wq_batch* batch, size_t* workspace_bytes, int* n_classes);
wq_status wq_batch_bind(wq_batch* batch, void* workspace, size_t bytes, void* const* mass_vals,
                        void* const* stiff_vals, hipStream_t stream);
wq_status wq_batch_tune(wq_batch* batch, int which, hipStream_t stream);
wq_status wq_batch_assemble(wq_batch* batch, int which, int use_graph, hipStream_t stream);
wq_status wq_batch_schedule(const wq_batch* batch, int k, int* info);
const char* wq_batch_last_error(const wq_batch* batch);
void wq_batch_destroy(wq_batch* batch);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * values as wq_assemble (same arguments, same results bit for bit) with the
 * first-contraction buffer taken from a static scratch array of the library
 * instead of the workspace.  The array is WQ_STATIC_SCRATCH_BYTES per GPU,
 * held from the loading of the library until the process ends; the patch is
 * formed in slabs of i3 planes that fit in it.  The call allocates nothing
 * (no hipMalloc, no allocating library routine).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams,
 * different plans) race and must be ordered by the caller.
 * A plane patch or curve (d < 3) has no first contraction and uses no
 * scratch: any size is accepted.
 * Errors: as wq_assemble; WQ_ENOSPACE (d = 3) if one plane of the buffer,
 * n_qp1 * n_qp2 * (2p+1) * (8 channels with WQ_STIFF, else 1) * value
 * size, exceeds the array.
 */
#define WQ_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
wq_status wq_assemble_static(wq_plan* plan, int which, void* mass_vals_dev, void* stiff_vals_dev,
                             hipStream_t stream);

/*
 * Export intermediate products for inspection/testing (device, asynchronous):
 *   wq_weights: the FP64 weights of direction dir and pairing index
 *     pair = 2*beta + alpha for (alpha, beta) in {(0,0),(1,0),(0,1),(1,1)},
 *     as w_dev[n][qcap] with w_dev[i][k] the weight at quadrature point
 *     q_start(i) + k (zero beyond #Q_i); q_start_dev[n], q_count_dev[n]
 *     (int32) give Q_i.  qcap = 3p+1.
 *   wq_field: the coefficient field in the plan's precision, as
 *     field_dev[7][n_qp3][n_qp2][n_qp1] with channels
 *     (det J, K11, K22, K33, K12, K13, K23).
 */
wq_status wq_weights(const wq_plan* plan, int dir, int pair, double* w_dev, int32_t* q_start_dev,
                     int32_t* q_count_dev, hipStream_t stream);
wq_status wq_field(const wq_plan* plan, void* field_dev, hipStream_t stream);

/*
 * Wait for all work of the plan on stream, then report latched device
 * conditions (and clear them): WQ_EGEOM if det J <= 0 somewhere,
 * WQ_ESINGULAR if a weight solve broke down, WQ_EDEVICE on a runtime error.
 */
wq_status wq_sync(wq_plan* plan, hipStream_t stream);

/* Message for the last error of this plan (never NULL; "" if none).  With
 * plan == NULL: the message of the last failed wq_plan_create on the calling
 * thread (which knot vector failed which check). */
const char* wq_last_error(const wq_plan* plan);

/* Free the plan (host memory only; the caller frees its device buffers). */
void wq_plan_destroy(wq_plan* plan);

/* Library version string. */
const char* wq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WQ_H */
