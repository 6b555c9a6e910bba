/*
 * qpmi.h -- C ABI of libqpmi.so, a batched, differentiable dense QP solver
 * for AMD MI355X (gfx950), after the OptNet layer of Amos & Kolter (2017).
 *
 * Every problem is the quadratic program of Section 3, eq. qp2:
 *
 *     minimize_z   1/2 z^T Q z + q^T z
 *     subject to   A z = b,   G z <= h
 *
 * with z in R^nz, Q in R^{nz x nz} (only its symmetric part (Q + Q^T)/2 is
 * used; it must be positive definite on the null space of A, and the method
 * as built needs Q + G^T D G positive definite, which holds for Q > 0),
 * A in R^{neq x nz} of full row rank, G in R^{nineq x nz}.
 *
 * Naming.  The paper calls the equality count m and the inequality count p
 * (A in R^{m x n}, G in R^{p x n}); this header uses nz (variables),
 * nineq (rows of G, h, lambda, s) and neq (rows of A, b, nu) instead.
 *
 * Memory.  Every pointer argument named as "device" is a HIP device pointer
 * on the current device; arrays are row-major and batch-major.  The caller
 * owns every buffer (inputs, outputs, state and workspace); the library never
 * allocates device memory and keeps no per-call global state.  Calls are
 * asynchronous on the given stream (a hipStream_t passed as void*, NULL =
 * the default stream) and are thread-safe for distinct buffers.
 *
 * Errors.  Call-level errors are negative return codes detected on the host
 * before any launch, with outputs untouched.  Per-problem outcomes are written
 * asynchronously into status[] (QP_STATUS_*) and iters[].
 */
#ifndef QPMI_H
#define QPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- types -------------------------------------------------------------- */

typedef enum { QP_F32 = 0, QP_F64 = 1 } qp_dtype;

/* Call-level return codes. */
enum {
    QP_OK = 0,
    QP_EARG = -1,    /* bad dims, batch, stride or a NULL required pointer    */
    QP_EWS = -2,     /* workspace smaller than qp_workspace_query() requires  */
    QP_EDTYPE = -3,  /* unknown dtype                                         */
    QP_EHIP = -4,    /* a HIP launch failed; qp_last_hip_error() has the code */
    QP_ENODEV = -5,  /* no usable gfx950 device / code object                 */
    QP_ETOOBIG = -6  /* a problem exceeds the library's size limits           */
};

/* Per-problem outcomes written to status[]. */
enum {
    QP_STATUS_OPTIMAL = 0,   /* stopping test met (see qp_opts.tol)                     */
    QP_STATUS_MAX_ITER = 1,  /* max_iter Newton steps taken; last iterate returned      */
    QP_STATUS_BREAKDOWN = 2, /* non-positive or non-finite pivot in the factorization of
                                the initial point or the first iterate; no factor is
                                stored and the backward writes zero gradients            */
    QP_STATUS_NONFINITE = 3, /* non-finite input or iterate; no factor is stored and the
                                backward writes zero gradients                           */
    QP_STATUS_STALLED = 4    /* the factorization of the next iterate lost positive
                                definiteness in working precision before the tolerance was
                                met (QP_VARIANT_ELIM: that of H, which the backward reads,
                                at the iterate the steps ended on); the last iterate whose
                                factorization succeeded is returned (iters counts its
                                steps) with its factor stored                            */
};

typedef struct {
    int32_t nz;    /* variables, >= 1             */
    int32_t nineq; /* inequality rows, >= 0       */
    int32_t neq;   /* equality rows, 0 <= neq < nz */
} qp_dims;

/* Solver options (qp_default_opts fills them per dtype). */
typedef struct {
    int32_t max_iter;     /* Newton steps after the initial point (default 20)          */
    int32_t refine_steps; /* backward solve: F64, at most this many steps of iterative
                             refinement on the unreduced K_sym residual, ending once the
                             error left (estimated from the corrections) is below 1e-8
                             of the solution or a correction no longer halves
                             (default 8); F32, the FP64 projected CG
                             preconditioned by the FP32 factor runs at most
                             10 * refine_steps iterations (default 3, so 30)              */
    double tol;           /* stop when max(mu, |r_x|inf, |r_s|inf, |r_y|inf) <= tol,
                             mu = s^T lambda / nineq (default 1e-8 F64, 1e-3 F32)        */
    int32_t variant;      /* kernel variant: 0 = pick automatically, else a QP_VARIANT_* */
    uint32_t flags;       /* QP_FLAG_* bits (others must be 0)                           */
} qp_opts;

/* Flags of qp_opts.flags.
 * QP_FLAG_G_UNIT_ROWS: every row of G is a signed unit vector (one entry +1 or
 *   -1, the rest 0), as for bounds z_j <= h_k or -z_j <= h_k (the box and
 *   non-negativity constraints of the Sudoku layer, Section 4.4, and of
 *   the ReLU layer in the proof of Theorem 2).  G is still passed densely.  The
 *   register-tile and streamed-tile policies then form G^T D G as a diagonal and apply G by
 *   gathers instead of products; a problem whose G does not have the structure
 *   (checked in the kernel) is solved by the dense path.  Results equal the
 *   dense path's up to rounding.  Used by the register-tile and streamed-tile
 *   policies, in uniform and uneven batches (an uneven batch with a problem on
 *   QP_VARIANT_ELIM runs the dense path for all); the generic and elimination-
 *   order policies accept the flag and run the dense path.  The backward is
 *   unchanged. */
/* QP_FLAG_BWD_FP32: the FP32 backward computes in FP32 only: the reduced
 *   solve with the stored FP32 factor and iterative refinement on the
 *   unreduced K_sym residual in FP32 (at most refine_steps steps, ending once
 *   the error left, estimated from the corrections, is below 1e-4 of the
 *   solution or a correction no longer halves).  Without the flag the FP32
 *   backward runs a projected conjugate gradient in FP64 preconditioned by the
 *   FP32 factor, which stays accurate at the ill-conditioned iterates that end
 *   FP32 solves.  Ignored for FP64. */
enum { QP_FLAG_G_UNIT_ROWS = 1u, QP_FLAG_BWD_FP32 = 2u };

enum {
    QP_VARIANT_AUTO = 0,
    QP_VARIANT_GENERIC = 1, /* one workgroup per problem, factor in global memory        */
    QP_VARIANT_LDS = 2,     /* one workgroup per problem, factor resident in LDS          */
    QP_VARIANT_TILED = 3,   /* register-resident 16x16 MFMA tiles (nz <= 128; FP32 <= 256) */
    QP_VARIANT_STREAM = 4,  /* factor in the state buffer, 16x16 MFMA tiles streamed       */
    QP_VARIANT_ELIM = 5     /* the paper's elimination order (Section 3.1.1, the footnote on
                               the LU of K_sym): Qs (nz x nz) and the Schur complement on A
                               (neq x neq) factored once per solve, only an nineq x nineq
                               matrix C + D(s / lambda), C = G M G^T with M the inverse of
                               [Qs A^T; A 0] restricted to z, factored per Newton step.
                               Where Qs is not positive definite the problem is solved
                               by the tiled (or, above nz = 128, streamed) policy.
                               Applies for nineq <= 128 and <= nz rounded up to a
                               multiple of 16, with its LDS regions (G U_Q among them)
                               fitting; the nz x nz factorizations run on register tiles
                               up to nz = 128 and on streamed tiles above; elsewhere the
                               automatic plan runs.  Cheaper per step than forming H where
                               nineq < nz.  The forward ends by factoring H at the returned
                               iterate, so the state and the backward are those of the
                               other variants.  Results equal theirs up to rounding.      */
};

/* Problem data of a uniform batch: device pointers plus per-problem strides in
 * elements between consecutive problems (0 = the array is shared by the whole
 * batch).  Within a problem: Q [nz*nz], q [nz], A [neq*nz], b [neq],
 * G [nineq*nz], h [nineq], all contiguous row-major.  A/b (G/h) may be NULL
 * when neq (nineq) is 0. */
typedef struct {
    const void *Q, *q, *A, *b, *G, *h;
    int64_t sQ, sq, sA, sb, sG, sh;
} qp_data;

/* ---- queries -------------------------------------------------------------- */

/* Fill *opts with the defaults for dtype.  Returns QP_OK or QP_EDTYPE. */
int32_t qp_default_opts(qp_dtype dtype, qp_opts *opts);

/* Bytes of the opaque per-problem factor `state` written by the forward and
 * read by the backward (the factor of the symmetrised KKT matrix of
 * Section 3.1.1 at the returned iterate).  The state of a batch is
 * batch * (*state_bytes), problem i at offset i * (*state_bytes). */
int32_t qp_state_bytes(qp_dtype dtype, qp_dims dims, size_t *state_bytes);

/* Bytes of device workspace a forward / backward call over `batch` problems
 * of `dims` needs (may be 0).  The workspace is scratch: contents are not
 * preserved across calls and it may be reused once the call has completed
 * on its stream. */
int32_t qp_workspace_query(qp_dtype dtype, int32_t batch, qp_dims dims, const qp_opts *opts,
                           size_t *fwd_ws_bytes, size_t *bwd_ws_bytes);

/* ---- forward ---------------------------------------------------------------- */

/* Solve `batch` QPs by the primal-dual interior point method of Section 3.1
 * (affine direction, eq. cvxgen:affine; centering-plus-corrector direction,
 * eq. cvxgen:cc; symmetrised KKT system reduced to (Q + G^T D G) with a Schur
 * complement on A, factored by Cholesky once per iterate).
 * Outputs (device, written for every problem):
 *   z [batch*nz], lam [batch*nineq], nu [batch*neq], s [batch*nineq] (slacks),
 *   state [batch*state_bytes] (opaque factor for qp_backward_batched),
 *   status [batch] (QP_STATUS_*), iters [batch] (Newton steps taken).
 * lam/s may be NULL iff nineq == 0, nu iff neq == 0.
 * ws: device workspace of at least fwd_ws_bytes (NULL when that is 0). */
int32_t qp_forward_batched(qp_dtype dtype, int32_t batch, qp_dims dims, const qp_data *data,
                           const qp_opts *opts, void *z, void *lam, void *nu, void *s, void *state,
                           int32_t *status, int32_t *iters, void *ws, size_t ws_bytes,
                           void *stream);

/* ---- backward ----------------------------------------------------------------- */

/* Gradients of a loss l through the QP solution (Section 3.1.1): solve
 * eq. grads-system with the stored factor (no new factorization).  F64: the
 * factor's solve plus at most opts->refine_steps steps of iterative refinement
 * on the unreduced symmetrised KKT residual (see qp_opts.refine_steps).  F32:
 * projected preconditioned conjugate gradients on the reduced system with FP64
 * vectors and products, the FP32 factor as preconditioner (accurate where
 * cond(H) eps32 exceeds 1); with QP_FLAG_BWD_FP32, the F64 scheme in FP32.  Then
 * eq. grads:
 *   dQ = 1/2 (d_z z^T + z d_z^T), dq = d_z, dA = d_nu z^T + nu d_z^T,
 *   db = -d_nu, dG = D(lam) d_lam z^T + lam d_z^T, dh = -D(lam) d_lam.
 * Inputs (device): data (the same problem data as the forward), z, lam, nu, s,
 * state (as written by the forward), dl_dz [batch*nz].
 * Outputs (device, nullable = not requested), per problem and contiguous:
 *   dQ [batch*nz*nz], dq [batch*nz], dA [batch*neq*nz], db [batch*neq],
 *   dG [batch*nineq*nz], dh [batch*nineq].
 * Gradients of batch-shared inputs (stride 0) are still written per problem;
 * summing them over the batch is the caller's choice.  A problem whose forward
 * ended BREAKDOWN or NONFINITE has no stored factor: its gradients are written
 * as zeros. */
int32_t qp_backward_batched(qp_dtype dtype, int32_t batch, qp_dims dims, const qp_data *data,
                            const qp_opts *opts, const void *z, const void *lam, const void *nu,
                            const void *s, const void *state, const void *dl_dz, void *dQ,
                            void *dq, void *dA, void *db, void *dG, void *dh, void *ws,
                            size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): qp_backward_batched
 * without a workspace argument, computing the same results with the same
 * kernels.  The adjoint vectors live in a library-owned static device array of
 * QP_NOALLOC_SCRATCH_BYTES on each GPU, present from the time the library's
 * code object is loaded on that GPU until the process ends; the call allocates
 * and frees nothing.  Returns QP_EWS when the backward's workspace
 * (qp_workspace_query) exceeds that size (e.g. more than 4096 FP64 problems with
 * nz + nineq + neq <= 512), QP_EHIP when the array's device address cannot be
 * obtained.  Every call on one GPU uses the same array, and its contents are
 * the last call's: calls that overlap in time on one GPU (from several streams
 * or threads) race and must be serialised by the caller. */
#define QP_NOALLOC_SCRATCH_BYTES (16u << 20)
int32_t qp_backward_batched_noalloc(qp_dtype dtype, int32_t batch, qp_dims dims,
                                    const qp_data *data, const qp_opts *opts, const void *z,
                                    const void *lam, const void *nu, const void *s,
                                    const void *state, const void *dl_dz, void *dQ, void *dq,
                                    void *dA, void *db, void *dG, void *dh, void *stream);

/* ---- uneven batches ------------------------------------------------------------ */

/* One problem of an uneven batch.  All offsets are in elements of the dtype
 * (state: in bytes) into the base pointers of the call; arrays of one problem
 * are contiguous row-major as in qp_data. */
typedef struct {
    int32_t nz, nineq, neq, variant; /* variant: as qp_opts.variant, 0 = auto     */
    int64_t Q, q, A, b, G, h;        /* input offsets (element)                   */
    int64_t z, lam, nu;              /* output offsets: z/dq, lam/s/dh, nu/db     */
    int64_t state;                   /* byte offset into state (qp_state_bytes)   */
} qp_problem_desc;

/* Solve `count` problems of different sizes in one persistent launch.
 * desc_dev: device array of `count` descriptors; desc_host: the same array in
 * host memory (used to size the launch; never retained).  `order_dev`
 * (device, `count` int32, may be NULL = identity) gives the order in which
 * workgroups pick problems (largest first balances the launch).
 * base_in: element base pointer of the packed inputs (Q..h of every problem);
 * z, lam, nu, s: element base pointers of the packed outputs (s uses the lam
 * offsets); state: byte base pointer; status/iters: [count] device.
 * ws must hold fwd bytes from qp_varlen_workspace_query. */
int32_t qp_varlen_workspace_query(qp_dtype dtype, int32_t count, const qp_problem_desc *desc_host,
                                  const qp_opts *opts, size_t *fwd_ws_bytes, size_t *bwd_ws_bytes,
                                  size_t *state_bytes_total);

int32_t qp_forward_varlen(qp_dtype dtype, int32_t count, const qp_problem_desc *desc_dev,
                          const qp_problem_desc *desc_host, const int32_t *order_dev,
                          const void *base_in, const qp_opts *opts, void *z, void *lam, void *nu,
                          void *s, void *state, int32_t *status, int32_t *iters, void *ws,
                          size_t ws_bytes, void *stream);

/* Backward of an uneven batch.  Gradient outputs use the input offsets of the
 * descriptors (dQ at desc.Q, dq at desc.q, ... in packed buffers shaped like the
 * inputs); need_dev (device, `count` int32, NULL = all) selects the problems
 * whose gradients are computed; others are skipped (their gradient entries are
 * left untouched). dl_dz uses the z offsets.  ws holds the adjoint vectors of
 * problem i at element offset desc.z + desc.lam + desc.nu (nz + nineq + neq
 * entries): with z, lam, nu offsets packed in descriptor order these are the
 * prefix sums of nz + nineq + neq; overlapping adjoint ranges are rejected
 * (QP_EARG).  Problems whose forward ended BREAKDOWN or NONFINITE get zero
 * gradients. */
int32_t qp_backward_varlen(qp_dtype dtype, int32_t count, const qp_problem_desc *desc_dev,
                           const qp_problem_desc *desc_host, const int32_t *need_dev,
                           const void *base_in, const qp_opts *opts, const void *z,
                           const void *lam, const void *nu, const void *s, const void *state,
                           const void *dl_dz, void *grad_base, void *ws, size_t ws_bytes,
                           void *stream);

/* ---- diagnostics ---------------------------------------------------------------- */

/* The hipError_t of the last QP_EHIP return on this thread (0 if none). */
int32_t qp_last_hip_error(void);

/* The factorization policy the forward runs for one problem of `dims` when
 * `variant` (a QP_VARIANT_*, 0 = automatic) is requested, on the current
 * device: *policy receives QP_VARIANT_GENERIC (factor in global memory),
 * QP_VARIANT_LDS, QP_VARIANT_TILED, QP_VARIANT_STREAM or QP_VARIANT_ELIM, and *lds_bytes (may
 * be NULL) the dynamic LDS of its workgroup.  The plan depends on the problem's
 * own dims, the variant and the device's LDS size only.  Host-side; launches
 * nothing.  Returns QP_OK, QP_EDTYPE, QP_EARG or QP_ETOOBIG (no policy fits). */
int32_t qp_plan(qp_dtype dtype, qp_dims dims, int32_t variant, int32_t *policy, int32_t *lds_bytes);

/* Library version as 10000*major + 100*minor + patch. */
int32_t qp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QPMI_H */
