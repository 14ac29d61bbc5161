/*
 * spin.h -- C ABI of the MI355X (gfx950) Strassen block-recursive inverter.
 *
 * The library inverts dense square matrices with Strassen's inversion scheme
 * (Alg. 1, Sec. 3.1 of "SPIN: A Fast and Scalable Matrix Inversion Method in
 * Apache Spark"; the recursive block form is Alg. 2, Sec. 3.3):
 *
 *     [A11 A12]^-1   [C11 C12]      I = A11^-1, II = A21 I, III = I A12,
 *     [A21 A22]    = [C21 C22]      V = A21 III - A22, VI = V^-1,
 *                                   C12 = III VI, C21 = VI II,
 *                                   C11 = I - III C21, C22 = -VI,
 *
 * recursing on A11 and on the Schur complement until a block has order at most
 * `leaf`, which is inverted directly (the paper allows any method there; this
 * library uses Gauss-Jordan elimination with partial pivoting in FP64).
 *
 * Conventions shared by every entry point
 *   Layout     column-major with a leading dimension, as the paper stores its
 *              matrix blocks (Sec. 3.2).  `Ainv` uses its own leading dimension
 *              `ldx` (>= n).  A row-major caller may pass its buffers unchanged:
 *              the transpose of the inverse is the inverse of the transpose, so
 *              a row-major A yields the row-major inverse.
 *   Memory     A, Ainv: device pointers owned by the caller.  A is never
 *              written; A and Ainv must not overlap (SPIN_E_ALIAS).  The
 *              library owns a per-stream workspace, allocated on first use,
 *              kept for reuse and freed by spin_release().
 *   Streams    every compute call is enqueued on `stream` (0 = the null
 *              stream) and returns before the GPU finishes.  Calls on one
 *              stream are ordered; calls from several host threads must use
 *              different streams.
 *   Graphs     the first inversion with a given entry point, mode, order,
 *              leading dimensions, buffers and stream workspace records its
 *              launch sequence as a HIP graph; later identical calls replay it.  At
 *              most 64 graphs are kept (the cache is emptied when full, after
 *              waiting for the device).  The environment variable
 *              SPIN_NO_GRAPH=1 makes every call launch its kernels directly.
 *   Leaves     two further environment variables change how a leaf is
 *              eliminated but never its result: SPIN_NO_SPEC=1 runs the pivot
 *              search at every step instead of first trying the diagonal
 *              pivots and verifying them; SPIN_DUO_SPIN=<count> lowers the
 *              bound on each wait of a panel eliminated by two workgroups
 *              (a wait that runs out sends the panel to the one-workgroup
 *              search).  Both are read when a call is enqueued, and a graph
 *              recorded earlier keeps the setting it was recorded with, so
 *              set them before the first call or with SPIN_NO_GRAPH=1.
 *   Errors     the return value is an argument or resource status known at
 *              enqueue time: 0 = enqueued, negative = SPIN_E_* (nothing was
 *              enqueued).  The numerical status (a zero or non-finite leaf
 *              pivot, refinement divergence) is written by the GPU and read by
 *              spin_info() after the work completes.
 */
#ifndef SPIN_H
#define SPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *spin_stream_t; /* same object as hipStream_t */

/* ---- status codes --------------------------------------------------------- */
#define SPIN_OK 0
#define SPIN_E_NULL (-1)      /* a required pointer is NULL                    */
#define SPIN_E_N (-2)         /* n < 1 (or n beyond SPIN_MAX_N)                */
#define SPIN_E_LD (-3)        /* a leading dimension is smaller than n         */
#define SPIN_E_LEAF (-4)      /* leaf < 1 or leaf > SPIN_MAX_LEAF              */
#define SPIN_E_ALIAS (-5)     /* A and Ainv overlap                            */
#define SPIN_E_MODE (-6)      /* unknown precision mode or refinement count    */
#define SPIN_E_COUNT (-7)     /* batch count < 0 or above SPIN_MAX_BATCH       */
#define SPIN_E_SCRATCH (-8)   /* spin_invert_noalloc: the order needs more
                                 workspace than its fixed scratch holds        */
#define SPIN_E_NOMEM (-10)    /* device allocation of the workspace failed     */
#define SPIN_E_HIP (-11)      /* a HIP runtime call or kernel launch failed    */
/* numerical status (positive values come from spin_info / info arrays):      */
/*   k > 0  : the pivot search for global column k (1-based) found only zero  */
/*            or non-finite candidates; the inverse is unspecified.           */
#define SPIN_NS_DIVERGED (-100) /* refinement failed: |I - A X_k|_F did not
                                   decrease from one Newton step to the next,
                                   or rho = |A X - I|_F / (|A|_F |X|_F) of the
                                   refined result is above 1e-12 (or NaN)     */

#define SPIN_MAX_LEAF 2048
#define SPIN_MAX_N (1 << 20)
#define SPIN_MAX_BATCH 65536

/* precision modes */
#define SPIN_FP64 0        /* every product and every leaf in FP64            */
#define SPIN_MIXED_FP32 1  /* block products in FP32 (FP32 MFMA, FP32 accumulation),
                              FP64 leaves, FP64 Newton refinement              */
#define SPIN_MIXED_BF16 2  /* block products on BF16 matrix cores: FP32 operands
                              rounded to BF16 (nearest even), FP32 accumulation;
                              FP64 leaves and refinement.  Too coarse for
                              kappa ~ 1e4 (refinement diverges, flagged)       */
#define SPIN_MIXED_BF16X3 3 /* as SPIN_MIXED_BF16 with each operand split into
                              hi = bf16(x), lo = bf16(x - hi) and the products
                              hi*hi + lo*hi + hi*lo accumulated in FP32
                              (about 16 significant bits per operand); needs
                              one refinement step more than SPIN_MIXED_FP32   */
/* Schedule flag, OR-ed into a mode (A must then be exactly symmetric): the
 * recursion runs the symmetric schedule of spin_invert_spd.  Accepted by
 * spin_invert_mixed (mixed modes: the FP32-storage recursion with the mode's
 * product flavour, then the same FP64 refinement) and by the batched and
 * serving entry points (SPIN_FP64 | SPIN_SYMMETRIC gives spin_invert_spd's
 * result bit for bit, a mixed mode spin_invert_mixed's with the flag).
 * Anywhere else, or with an unknown mode, it is SPIN_E_MODE. */
#define SPIN_SYMMETRIC 16
/* Refinement flag, OR-ed into a mixed mode of spin_invert_mixed only: the
 * Newton residual R = I - A X, the update X + X R and the acceptance
 * residual are formed by spin_gemm_int8's emulation (14 moduli, operands
 * rounded to 47 bits per row / column at order 16384, more below) instead of
 * FP64 matrix cores; n <= 131071 (spin_gemm_int8's limit on k), else
 * SPIN_E_N.  The batched and serving entry points reject it. */
#define SPIN_REFINE_INT8 32

/* ---- FP64 inversion ------------------------------------------------------- */
/* Ainv (n x n, ldx) := A^-1 for A (n x n, lda), FP64 throughout.
 * Alg. 1 / Alg. 2; blocks of order <= leaf are inverted by Gauss-Jordan with
 * partial pivoting.  Leading blocks and Schur complements must be
 * nonsingular (true for SPD and strictly diagonally dominant A); otherwise the
 * leaf that meets a zero pivot column reports it through spin_info(). */
int spin_invert(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                int64_t leaf, spin_stream_t stream);

/* ---- FP64 inversion without allocation ------------------------------------ */
/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops that forbid allocation): the inversion of spin_invert, with
 * the same arguments, kernels, schedule and result bit for bit, whose
 * workspace is a fixed device array of SPIN_NOALLOC_SCRATCH_MB MiB that the
 * library holds on each GPU it runs on until the process ends.  The call
 * makes no device allocation, captures no graph and launches its kernels
 * directly on `stream`.
 *   Limit      the order and leaf must fit the array: spin_workspace_bytes(n,
 *              leaf, SPIN_FP64) <= SPIN_NOALLOC_SCRATCH_MB MiB (about n <= 2800);
 *              larger requests return SPIN_E_SCRATCH and enqueue nothing.
 *   Status     written by the GPU to the device int *info (0, or the 1-based
 *              column of a failing leaf pivot) after the work completes, in
 *              stream order; info may be NULL.  spin_info() does not cover
 *              this call.
 *   Sharing    every call on one GPU uses that GPU's one array, whatever the
 *              stream: calls that overlap in time on one GPU race and give
 *              unspecified results; order them (one stream, or events).
 * Other arguments and errors as for spin_invert. */
#define SPIN_NOALLOC_SCRATCH_MB 64
int spin_invert_noalloc(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                        int64_t leaf, int *info, spin_stream_t stream);

/* ---- FP64 inversion through a block LU factorisation ---------------------- */
/* Ainv := A^-1 by the method the paper compares SPIN with (Sec. 5, after Liu
 * et al.): A = L U without pivoting (as Alg. 1 assumes every leading block
 * and Schur complement nonsingular), L^-1 and U^-1 by block recursion on the
 * product kernels, then Ainv = U^-1 L^-1.  Per node: {U12 = Li11 A12,
 * L21 = A21 Ui11}, S = A22 - L21 U12, {T1 = L21 Li11, T2 = Ui11 U12}, the
 * recursion on S, {Li21 = -Li22 T1, Ui12 = -T2 Ui22}.  Leaves (order <= leaf
 * <= 128, else SPIN_E_LEAF) factor and invert in one workgroup.  Arguments,
 * layout, ownership and status reporting as for spin_invert; the workspace
 * holds L^-1 and U^-1 (2 n^2 words) besides the recursion's
 * (spin_plan_ws_elems_lu). */
int spin_invert_lu(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                   int64_t leaf, spin_stream_t stream);

/* ---- FP64 inversion of a symmetric matrix --------------------------------- */
/* Ainv := A^-1 for an exactly symmetric A (the positive-definite matrices the
 * paper targets, Sec. 2.1), Alg. 1 specialised: every block the recursion
 * inverts is then symmetric, so III = I A12 = II^T, and a node needs
 *   II = A21 I,  S = A22 - II A12,  C22 = S^-1,  C21 = -C22 II,
 *   C12 = C21^T,  C11 = I - C12 II,
 * where S and C11, being symmetric, are formed on and below the diagonal only
 * and mirrored: about 6 h^3 flops per node against 12 h^3.  Every block a
 * node passes on is thereby exactly symmetric outside the leaves, which keeps
 * the residual at the level of spin_invert's.
 * Arguments, layout, ownership, workspace (spin_workspace_bytes with
 * SPIN_FP64 covers it) and status reporting are those of spin_invert.  Both
 * triangles of A are read; for a matrix that is not exactly symmetric the
 * result is unspecified.  Ainv is exactly symmetric outside the diagonal
 * leaf blocks. */
int spin_invert_spd(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                    int64_t leaf, spin_stream_t stream);

/* ---- mixed-precision inversion with Newton refinement --------------------- */
typedef struct spin_report {
    double rho_before;   /* |A X0 - I|_F / (|A|_F |X0|_F) of the unrefined inverse */
    double rho_after;    /* same after the refinement steps                         */
    double r0_fro;       /* |I - A X0|_F                                            */
    double r_fro[8];     /* |I - A X_k|_F before step k (k < steps)                 */
    int steps;           /* refinement steps performed                              */
    int status;          /* 0, k > 0 (pivot failure) or SPIN_NS_DIVERGED            */
} spin_report;

/* Ainv := A^-1 computed with the recursion's block products in the precision
 * of `mode` (FP32 working copies of A and of the recursion's outputs) and FP64
 * leaves, followed by `ns_steps` (0..8) FP64 Newton steps
 *     R = I - A X,  X <- X + X R
 * (Newton iteration as the stabiliser of Strassen inversion, Sec. 2.1).
 * When ns_steps > 0 the call also accepts or rejects the refined result on
 * the device: one more FP64 product forms R = I - A X, and unless
 * rho = |R|_F / (|A|_F |X|_F) <= 1e-12 the status (spin_info) becomes
 * SPIN_NS_DIVERGED; the result stays in Ainv either way.
 * mode | SPIN_SYMMETRIC (exactly symmetric A) runs the recursion on the
 * symmetric schedule of spin_invert_spd, about half the block-product work;
 * the refinement is unchanged.  If `rep` is non-NULL the call waits for the stream, evaluates both residuals
 * on the GPU and fills *rep; with rep == NULL the call is asynchronous and
 * no residual is computed. */
int spin_invert_mixed(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                      int64_t leaf, int mode, int ns_steps, spin_report *rep,
                      spin_stream_t stream);

/* ---- block product -------------------------------------------------------- */
/* D (m x n, ldd) := alpha * A (m x k, lda) * B (k x n, ldb) + beta * C0 (m x n, ldc)
 * plus the identity on the diagonal when add_identity != 0.  This is the
 * paper's `multiply` (Sec. 3.3) with its `subtract` (Alg. 2) and the sign of
 * `scalarMul` (Alg. 5) folded into the epilogue.  dtype SPIN_FP64: double
 * operands and result, FP64 MFMA.  dtype SPIN_MIXED_FP32: float operands and
 * result, FP32 MFMA with FP32 accumulation.  dtype SPIN_MIXED_BF16 /
 * SPIN_MIXED_BF16X3: float operands and result, the operands rounded (split)
 * to BF16 as described for those modes, FP32 accumulation; alpha, beta and
 * the identity are applied in FP64 before the FP32 store.  C0 may be NULL when beta == 0 and
 * may equal D (each element is read before it is written); A and B must not
 * overlap D.  Asynchronous on `stream`. */
int spin_gemm(int dtype, int64_t m, int64_t n, int64_t k, double alpha,
              const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
              const void *C0, int64_t ldc, void *D, int64_t ldd, int add_identity,
              spin_stream_t stream);

/* ---- FP64-accurate product on INT8 matrix cores --------------------------- */
/* D (m x n, ldd) := epilogue(A (m x k, lda) * B (k x n, ldb)), FP64 operands
 * and result, column-major, computed on INT8 matrix cores by the integer
 * modular scheme of Ozaki, Uchino and Imamura (Ozaki scheme II, 2025): row i
 * of A is scaled by a power of two and rounded to an integer of at most
 * beta_a bits (nearest, ties to even; the row's largest magnitude sets the
 * scale), column j of B likewise to beta_b bits; the integer product is
 * formed exactly from `moduli` INT8 residue products (2 <= moduli <= 15,
 * pairwise coprime moduli 256, 255, 253, 251, 247, 241, 239, 233, ...) and
 * Chinese remaindering, rounded once to FP64 and scaled back.  This is the
 * product the Newton refinement needs in FP64 (Newton iteration as the
 * stabiliser of Strassen inversion, Sec. 2.1).
 *   epilogue 0: D = A B;  1: D = I - A B (m == n);  2: D = C0 + A B (C0 may
 *               equal D, each element is read before it is written).
 *   beta_a, beta_b <= 0: the largest equal pair the moduli allow at this k
 *   (at most 53).  Otherwise 1 + log2(k) + beta_a + beta_b must stay below
 *   log2 of the product of the moduli (SPIN_E_MODE).
 *   k <= 131071: the matrix cores sum k residue products (|r| <= 128) in
 *   int32, exact while k 128^2 < 2^31 (SPIN_E_N above).
 * Error against the exact product: |D - A B| <= 2^-beta (m_i sum_k |b_kj| +
 * n_j sum_k |a_ik|) + k 2^-2beta m_i n_j + 2^-53 |D| before the epilogue
 * (m_i, n_j: the largest magnitudes of row i of A and column j of B).  A row
 * of A or a column of B holding Inf or NaN gives NaN in its row / column.
 * Uses the stream's workspace (about 3 moduli m n bytes); asynchronous. */
int spin_gemm_int8(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                   int64_t ldb, int epilogue, const double *C0, int64_t ldc, double *D, int64_t ldd,
                   int moduli, int beta_a, int beta_b, spin_stream_t stream);

/* ---- status and residual -------------------------------------------------- */
/* Waits for `stream` and returns the numerical status of the last inversion
 * enqueued on it: 0, k > 0 (1-based failing pivot column) or SPIN_NS_DIVERGED. */
int spin_info(spin_stream_t stream);

/* rho = |A X - I|_F / (|A|_F |X|_F) in FP64 on the GPU (the residual measure
 * used to accept an inverse).  Waits for `stream`; writes *rho. */
int spin_residual(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx,
                  double *rho, spin_stream_t stream);

/* Bytes of library workspace one inversion of order n needs in `mode`. */
size_t spin_workspace_bytes(int64_t n, int64_t leaf, int mode);

/* Short static description of a status code. */
const char *spin_strerror(int code);

/* Frees every cached workspace and captured graph (waits for the device). */
void spin_release(void);

/* ---- batched inversion and continuous batching ---------------------------- */
/* Inverts `count` independent matrices (each column-major, its own order n[i]
 * and leading dimensions; mode[i] = SPIN_FP64 or one of the mixed modes with
 * `ns_steps` refinement steps, either optionally | SPIN_SYMMETRIC) with cross-request
 * batching: at each step the block products of all requests run in grouped
 * matrix-core launches and their leaves in one batched leaf launch.  Every
 * request's result is bit for bit the one spin_invert / spin_invert_spd /
 * spin_invert_mixed would give it alone.  Waits for the stream; info[i]
 * (optional) receives request i's numerical status. */
int spin_invert_batch(int64_t count, const double *const *A, const int64_t *n,
                      const int64_t *lda, double *const *Ainv, const int64_t *ldx,
                      const int *mode, int64_t leaf, int ns_steps, int *info,
                      spin_stream_t stream);

/* Continuous-batching server (one host thread drives it).  The server owns a
 * device workspace pool of pool_bytes (allocated at the first tick); requests
 * wait in a FIFO queue and are admitted when one of max_active slots is free
 * and their workspace (spin_server_request_bytes) fits in the pool.  Each
 * tick launches the next step of every admitted request on `stream`, grouped
 * across requests as in spin_invert_batch; requests finish independently and
 * their pool space is reused by the queue.  A and Ainv of a submitted request
 * must stay valid until spin_server_poll reports it. */
typedef struct spin_server spin_server;
spin_server *spin_server_create(size_t pool_bytes, int max_active, int64_t leaf, int ns_steps);
void spin_server_destroy(spin_server *srv);
/* Queues one request, mode as for spin_invert_batch (returns 0, or SPIN_E_*
 * when the arguments are invalid or the request could never fit in the pool). */
int spin_server_submit(spin_server *srv, const double *A, int64_t n, int64_t lda, double *Ainv,
                       int64_t ldx, int mode, int64_t tag);
/* Host only: admits queued requests that fit (returns how many). */
int spin_server_admit(spin_server *srv);
/* Admits, then enqueues one step of every admitted request; returns the
 * number of admitted, unfinished requests or a negative SPIN_E_* code. */
int spin_server_tick(spin_server *srv, spin_stream_t stream);
/* Does not wait for queued work: writes up to cap (tag, status) pairs of
 * requests whose work has completed since the last poll and frees their pool
 * space; returns the count, or a negative SPIN_E_* code.  A finished
 * request's status words are read on the server's own non-blocking stream.
 * A status of SPIN_E_HIP means they could not be read. */
int64_t spin_server_poll(spin_server *srv, int64_t *tags, int *info, int64_t cap);
int spin_server_stats(spin_server *srv, int64_t *queued, int64_t *active, size_t *pool_used);
/* Pool bytes one request of order n and mode `mode` (SPIN_SYMMETRIC allowed
 * as above) needs (0 for invalid arguments). */
size_t spin_server_request_bytes(int64_t n, int64_t leaf, int mode);

/* ---- schedule introspection (host only, no GPU needed) -------------------- */
/* One step of the recursion schedule as the executor runs it (S-form: the
 * Schur complement S = A22 - A21 A11^-1 A12 = -V is formed and inverted
 * directly, so C22 = S^-1 and C12 = -III C22, C21 = -C22 II). */
typedef struct spin_plan_op {
    int kind;        /* 0 = group of block products, 1 = leaf inversion,
                        2 = transpose, 3 = mirror (spin_plan_describe_spd only),
                        4 = LU leaf, 5 = zero fill (spin_plan_describe_lu only) */
    int count;       /* products in the group (1 or 2); 1 for a leaf          */
    int level;       /* recursion depth of the node that issues it            */
    int flags;       /* bit q: product q (m == n) forms only its lower triangle;
                        a mirror step fills the strict upper one.  Bit 2: the
                        executor does the next step (a mirror of this result,
                        or its transpose into a block no operand occupies) in
                        this product's epilogue, with the same result          */
    /* products: D = alpha * op_a * op_b + beta * C0 (+ I if add_identity)    */
    int64_t m[2], n[2], k[2];
    int a_buf[2], b_buf[2], c_buf[2], d_buf[2];  /* 0 = A, 1 = Ainv, 2 = workspace */
    int64_t a_off[2], b_off[2], c_off[2], d_off[2]; /* element offsets           */
    int64_t a_ld[2], b_ld[2], c_ld[2], d_ld[2];
    double alpha[2], beta[2];
    /* leaf: out (order L, at d_*[0]) := in^-1 (at a_*[0]); col0 = global column */
    /* transpose: d (n[0] x m[0], at d_*[0]) := a (m[0] x n[0], at a_*[0])^T      */
    /* mirror: the order-m[0] block at d_*[0] gets d[i][j] = d[j][i] for j > i    */
    /* LU leaf: L^-1 at d_*[0] and U^-1 at c_*[0] of the order-L block at a_*[0]  */
    /* zero fill: the m[0] x n[0] block at d_*[0]                                  */
    int64_t leaf_order, col0;
} spin_plan_op;

/* Writes up to `cap` steps of the schedule for (n, leaf) into ops[] (ops may
 * be NULL with cap 0) and returns the total number of steps, or a negative
 * SPIN_E_* code.  Element offsets refer to A (lda), Ainv (ldx) and a workspace
 * of spin_plan_ws_elems(n, leaf) elements.  *flops (optional) receives the
 * schedule's arithmetic count: 2 m n k per product, 2 L^3 per leaf. */
int64_t spin_plan_describe(int64_t n, int64_t lda, int64_t ldx, int64_t leaf,
                           spin_plan_op *ops, int64_t cap, double *flops);
/* The same for the schedule of spin_invert_spd (kinds 0, 1 and 2); its
 * workspace is at most spin_plan_ws_elems(n, leaf) elements. */
int64_t spin_plan_describe_spd(int64_t n, int64_t lda, int64_t ldx, int64_t leaf,
                               spin_plan_op *ops, int64_t cap, double *flops);
/* The same for spin_invert_lu (kinds 0, 4 and 5; leaf <= 128), with its
 * workspace size in elements. */
int64_t spin_plan_describe_lu(int64_t n, int64_t lda, int64_t ldx, int64_t leaf,
                              spin_plan_op *ops, int64_t cap, double *flops);
int64_t spin_plan_ws_elems_lu(int64_t n, int64_t leaf);
int64_t spin_plan_ws_elems(int64_t n, int64_t leaf);

/* ---- per-kernel timing (for profiling; forces eager launches) ------------- */
typedef struct spin_trace_rec {
    char kernel[48];  /* kernel family and tile shape                           */
    double ms;        /* HIP-event time of the launch on its stream             */
    double flops;     /* algorithmic flops of the launch                        */
    double bytes;     /* algorithmic HBM bytes of the launch (operands + result) */
    int level;        /* recursion level (-1 outside the recursion)             */
} spin_trace_rec;

/* While enabled, inversions run eagerly (no graph replay) and every kernel
 * launch is bracketed by HIP events on its stream. */
int spin_trace_enable(int on);
/* Waits for the traced work, copies up to `cap` records (returns the count
 * available) and clears the trace buffer. */
int64_t spin_trace_collect(spin_trace_rec *recs, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif /* SPIN_H */
