/*
 * phylograd -- log-likelihood and all branch-length gradients of a
 * phylogenetic CTMC model on one AMD Instinct MI355X (gfx950).
 *
 * Method: Ji et al., "Gradients do grow on trees: a linear-time
 * O(N)-dimensional gradient for statistical phylogenetics".
 *   - post-order pruning pass, Section 2.3, Eqs. (postOrderPartialUpdate)
 *     and (rootInnerProduct);
 *   - pre-order pass, Section 2.4, Eq. (preOrderUpdate);
 *   - per-branch derivative, Section 2.5, Eq. (singleRateCaseGradient), with
 *     rate categories, Section 2.6, Eqs. (discreteRateLikelihood) and
 *     (GradientWithGamma);
 *   - diagonal of the Hessian, Section 2.7, Eq. (Hessian).
 *
 * Conventions (Section 2.1, made 0-based):
 *   - N tips are nodes 0..N-1, internal nodes N..2N-2, the root is 2N-2;
 *   - a branch is named by its child node: branch b (0 <= b < 2N-2) joins
 *     node b to parent[b]; t[b] is its length;
 *   - Q[x*m + y] is the rate from parent state x to child state y
 *     (row-major, off-diagonals >= 0, rows sum to 0); the transition matrix
 *     of branch b in rate category l is exp(Q * rate[l] * t[b]);
 *   - the root distribution need not be the stationary one and Q need not be
 *     reversible;
 *   - tip observations are bit masks, bit x set = state x allowed (a
 *     one-hot mask is an observed state, all bits set is missing data,
 *     Section 2.1's modified tip vector for partial observation);
 *   - logL = sum_s w_s log L_s over site patterns s with weights w_s >= 0.
 *
 * Every function returns PG_OK (0) or a negative PG_E_* code, never
 * throws and never aborts; pg_last_error() describes the last failure.
 * All inputs are copied: the caller may free them when a call returns.
 * Outputs are caller-allocated.  A context is not thread-safe; distinct
 * contexts are independent.  All device work of a context runs in order on
 * one HIP stream (its own, or the one given by pg_set_stream).
 */
#ifndef PHYLOGRAD_H
#define PHYLOGRAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define PG_OK             0
#define PG_E_INVALID     -1  /* bad argument: NULL pointer, bad size, t not finite or < 0 */
#define PG_E_TREE        -2  /* not a rooted binary tree in the numbering above        */
#define PG_E_MODEL       -3  /* Q, root frequencies or rate categories malformed       */
#define PG_E_PATTERNS    -4  /* empty mask, state beyond m, weight < 0 or not finite   */
#define PG_E_STATE       -5  /* call order: tree, patterns and model not all set       */
#define PG_E_OOM         -6  /* device allocation failed                               */
#define PG_E_DEVICE      -7  /* HIP runtime error or no usable gfx950 device           */
#define PG_E_ZERO_LIK    -8  /* some pattern with w_s > 0 has likelihood 0: logL=-inf  */
#define PG_E_UNSUPPORTED -9  /* state count or precision without a compiled kernel     */

/* ---- precisions ------------------------------------------------------ */
/* PG_FP64: partial vectors, transition matrices and arithmetic in FP64.
 * PG_FP32: partial vectors and their arithmetic in FP32; the transition
 *          matrices are computed in FP64 and rounded once; the per-pattern
 *          scale exponents, the site-weighted sums of logL and of the
 *          gradient stay in FP64.
 * PG_SPLIT_BF16: partial vectors in FP32; every matrix-vector product with
 *          a transition matrix (or with Q) runs on the BF16 matrix cores
 *          with FP32 accumulation, each FP32 operand carried as three BF16
 *          parts (hi + mid + lo) and the six part products of order >=
 *          2^-16 summed; transition matrices enter as P - I.  They are
 *          formed in FP64 from an eigen-decomposition of Q computed by
 *          pg_set_model (scaling and squaring when Q is not usably
 *          diagonalisable; see pg_eigensystem).  Any 2 <= n_states <= 64
 *          (padded to 64); meant for large state spaces such as 61 codons.
 *          The Hessian's Q^2 products are split the same way. */
#define PG_FP64 0
#define PG_FP32 1
#define PG_SPLIT_BF16 2

/* ---- kernels reported by pg_get_timing ------------------------------- */
#define PG_K_PMAT  0  /* transition matrices exp(Q rate t)                     */
#define PG_K_POST  1  /* post-order pass, rescaling, root values               */
#define PG_K_ROOT  2  /* logL reduction of calls without a gradient            */
#define PG_K_PRE   3  /* pre-order pass fused with the gradient                */
#define PG_K_GSUM  4  /* fixed-order per-branch gradient reduction, with logL  */
#define PG_K_COUNT 5

typedef struct pg_ctx pg_ctx;

/* Create a context on HIP device `device` with precision PG_FP64, PG_FP32
 * or PG_SPLIT_BF16 (any other value: PG_E_UNSUPPORTED).  No device memory is
 * allocated until the first evaluation.  Fails with PG_E_DEVICE when the
 * device does not exist or is not gfx950.  *out is NULL on failure; the
 * caller owns the context and frees it with pg_destroy. */
int pg_create(int device, int precision, pg_ctx** out);

/* Release the context and all its device memory (waits for its stream). */
void pg_destroy(pg_ctx* ctx);

/* Message for the last failing call on ctx (never NULL; "" if none).
 * With ctx == NULL, the message of the last failed pg_create. */
const char* pg_last_error(const pg_ctx* ctx);

/* Run all later device work on `hip_stream` (a hipStream_t, e.g. torch's
 * current stream); NULL restores the context's own stream.  The caller
 * keeps ownership of the stream and must keep it alive. */
int pg_set_stream(pg_ctx* ctx, void* hip_stream);

/* Tree topology (Section 2.1).  parent[2N-1]: parent[v] for every node,
 * parent[2N-2] == -1 for the root; every internal node has exactly two
 * children and every node reaches the root.  N >= 2.  Changing N drops the
 * patterns. Errors: PG_E_INVALID (NULL, N < 2), PG_E_TREE. */
int pg_set_tree(pg_ctx* ctx, int32_t n_tips, const int32_t* parent);

/* Site patterns (Section 2.1: sites are independent, a tip's partial
 * vector is the indicator of its observed state, or of the allowed states
 * when it is partly observed or missing).  tip_masks[N*S], row-major: row v
 * (tip v), column s, bit x = state x allowed, 2 <= m <= 64; weights[S]
 * finite and >= 0 (a pattern's multiplicity in logL = sum_s w_s log L_s).
 * Both arrays are copied.  Needs the tree.
 * Errors: PG_E_STATE (no tree), PG_E_INVALID, PG_E_PATTERNS (empty mask,
 * a bit >= m, more than 255 - m distinct partial-ambiguity masks). */
int pg_set_patterns(pg_ctx* ctx, int32_t n_patterns, int32_t n_states,
                    const uint64_t* tip_masks, const double* weights);

/* Substitution model (Sections 2.1 and 2.6).  Q[m*m] row-major generator,
 * root_freqs[m] a probability vector, cat_rates[K] >= 0 and
 * cat_weights[K] a probability vector (the discrete rate categories
 * gamma_l and Pr(gamma_l)), 1 <= K <= 64.  All arrays are copied.  Compiled
 * state counts: m = 4 and m = 20 for PG_FP64 and PG_FP32; any
 * 2 <= m <= 64 for PG_SPLIT_BF16.  Errors: PG_E_INVALID (NULL), PG_E_MODEL
 * (negative off-diagonal, a row not summing to 0, a frequency or weight
 * vector not summing to 1, a negative rate), PG_E_UNSUPPORTED (m without a
 * kernel for the context's precision). */
int pg_set_model(pg_ctx* ctx, int32_t n_states, const double* Q,
                 const double* root_freqs, int32_t n_cats,
                 const double* cat_rates, const double* cat_weights);

/* Non-homogeneous model (Section 2.1: the process may differ between
 * branches): branch b (the branch above node b) evolves under rate matrix
 * Q[model_of_branch[b]], Q[n_models*m*m] row-major generators checked as by
 * pg_set_model; root_freqs and the rate categories stay those of
 * pg_set_model.  The gradient and Hessian use each branch's own matrix.
 * Both arrays are copied.  n_models = 0 returns to the homogeneous model.
 * Cleared by pg_set_tree with a different N or pg_set_model with a
 * different m.  Every precision; the transition matrices of a
 * non-homogeneous model come from scaling and squaring of each branch's
 * matrix.  Errors: PG_E_STATE (no tree or model), PG_E_INVALID (NULL, index
 * out of range), PG_E_MODEL. */
int pg_set_branch_models(pg_ctx* ctx, int32_t n_models, const double* Q, const int32_t* model_of_branch);

/* Partial re-evaluation: logL after changing the lengths of the n branches
 * branches[i] to t_new[i] (i < n), the other lengths staying those of the
 * resident partials, which must come from a host-pointer pg_logL,
 * pg_logL_and_grad or pg_logL_update.  Recomputes only the changed
 * transition matrices and the post-order nodes that depend on them (each
 * changed internal node and the ancestors of every changed branch), so a
 * single-branch change costs O(depth) nodes.  The first call on a context
 * switches on per-node scale-exponent storage and runs one full forward
 * pass; later full evaluations keep the exponents (2 bytes per node,
 * pattern and category).  The result, and the partials it leaves for
 * pg_grad, are bitwise those of a full evaluation at the new lengths.
 * Every precision, split-BF16 included.
 * Errors: PG_E_STATE (no such partials), PG_E_INVALID, PG_E_ZERO_LIK. */
int pg_logL_update(pg_ctx* ctx, int32_t n, const int32_t* branches, const double* t_new, double* logL);

/* One evaluation from host memory: t[2N-2] branch lengths in, *logL and,
 * unless grad == NULL, grad[2N-2] = dlogL/dt_b out.  logL is the post-order
 * pass (Section 2.3, Eqs. postOrderPartialUpdate and rootInnerProduct, with
 * categories Eq. discreteRateLikelihood); the gradient is the pre-order pass
 * (Section 2.4, Eq. preOrderUpdate) with every branch's derivative formed in
 * the same traversal (Section 2.5 Eq. singleRateCaseGradient, Section 2.6
 * Eq. GradientWithGamma).  Blocks until done.
 * Errors: PG_E_STATE, PG_E_INVALID (t), PG_E_ZERO_LIK (*logL = -inf, grad
 * left unspecified), PG_E_DEVICE, PG_E_OOM. */
int pg_logL_and_grad(pg_ctx* ctx, const double* t, double* logL, double* grad);

/* Post-order pass only (transition matrices, pruning, root; Section 2.3,
 * Eqs. postOrderPartialUpdate and rootInnerProduct): *logL out.  Blocks.
 * The partial vectors stay resident on the device for a later pg_grad.
 * Errors as pg_logL_and_grad. */
int pg_logL(pg_ctx* ctx, const double* t, double* logL);

/* Pre-order pass fused with the gradient (Section 2.4 Eq. preOrderUpdate,
 * Sections 2.5-2.6 Eqs. singleRateCaseGradient and GradientWithGamma) on
 * the partials left by the last successful pg_logL (or pg_logL_and_grad):
 * grad[2N-2] (host, caller-allocated) out.  Blocks.  PG_E_STATE if there are
 * none or the tree, patterns or model changed since. */
int pg_grad(pg_ctx* ctx, double* grad);

/* Diagonal of the Hessian, d2 logL / dt_b^2, Section 2.7 Eq. (Hessian),
 * on the partials left by the last pg_logL or pg_logL_and_grad.  Also
 * returns the gradient in grad[2N-2] unless grad == NULL.  Blocks.  Every
 * precision; the second-derivative numerators use Q^2 of each branch's
 * rate matrix (split-BF16: Q^2 carried in three BF16 parts). */
int pg_hessian_diag(pg_ctx* ctx, double* grad, double* hess);

/* Device-pointer variant of pg_logL_and_grad (same passes and sections):
 * d_t[2N-2] (FP64, device), d_logL[1] and
 * d_grad[2N-2] (device, d_grad may be NULL) are read and written
 * asynchronously on the context's stream; pointers must stay valid until
 * that stream reaches this work.  No host synchronisation.  Branch lengths
 * are checked on the device: a non-finite or negative t_b, or a zero
 * likelihood, makes *d_logL NaN or -inf and is reported by the next
 * pg_status() call. */
int pg_logL_and_grad_device(pg_ctx* ctx, const double* d_t, double* d_logL,
                            double* d_grad);

/* Device-pointer pre-order pass (as pg_grad, Sections 2.4-2.6): the
 * gradient of the partials left by the
 * last evaluation (pg_logL_and_grad_device with d_grad == NULL, pg_logL,
 * ...) is written to d_grad[2N-2] (device) asynchronously on the context's
 * stream; no host synchronisation.  This is the backward of an autograd
 * function whose forward was the logL-only evaluation.  PG_E_STATE if there
 * are no resident partials. */
int pg_grad_device(pg_ctx* ctx, double* d_grad);

/* Allocation-free variant of pg_logL_and_grad_device, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, passes
 * and results (bit for bit) as pg_logL_and_grad_device; d_grad == NULL
 * computes logL only.  It never calls hipMalloc, hipFree or any other
 * allocating routine for device memory: every device buffer of the
 * evaluation (tip codes, schedule, model tables, transition matrices,
 * messages, pre-order vectors, root values, tile partials, status) lives in
 * one library-owned array per device of PG_NOALLOC_MAX_BYTES bytes, which
 * each GPU the library runs on holds until the process ends.  The inputs
 * are copied into it from the context's host copies (set by pg_set_tree,
 * pg_set_patterns, pg_set_model, pg_set_branch_models) on the context's
 * stream at every call; host-side planning runs on the first call after
 * one of those changes.  Problems needing more than PG_NOALLOC_MAX_BYTES
 * (see pg_footprint_bytes for the scale) fail with PG_E_INVALID.
 * Asynchronous like the device variant; errors of the evaluation itself (a
 * bad branch length, a zero likelihood) show only as NaN or -inf in
 * *d_logL (pg_status does not see them).  The context's own device buffers
 * and resident partials are neither used nor changed (pg_grad and
 * pg_grad_device keep referring to the last other evaluation).  Every call
 * on one GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (on different streams, from different
 * threads or contexts) race and give undefined results; calls in order on
 * one stream are safe.  PG_E_DEVICE if the array's device address could not
 * be found when the context was created. */
#define PG_NOALLOC_MAX_BYTES (64ll << 20)
int pg_logL_and_grad_noalloc(pg_ctx* ctx, const double* d_t, double* d_logL, double* d_grad);

/* Device-side status of the last device-pointer evaluation (waits for the
 * stream): PG_OK, PG_E_INVALID (bad t) or PG_E_ZERO_LIK. */
int pg_status(pg_ctx* ctx);

/* Kernel timing.  While enabled, each evaluation records a pair of HIP
 * events around every kernel on the context's stream (no synchronisation
 * between kernels).  pg_get_timing waits for the recorded events, writes,
 * for each PG_K_* kernel, the summed milliseconds into ms[k] and the number
 * of launches into launches[k] (arrays of PG_K_COUNT entries; either may be
 * NULL), then resets the sums. */
int pg_set_timing(pg_ctx* ctx, int enable);
int pg_get_timing(pg_ctx* ctx, double* ms, int64_t* launches);

/* Device bytes the context holds now (for admission by HBM footprint), and
 * the bytes it would hold for a problem of the given size. */
int64_t pg_device_bytes(const pg_ctx* ctx);
int64_t pg_footprint_bytes(int32_t n_tips, int32_t n_patterns, int32_t n_states,
                           int32_t n_cats, int precision);

/* The eigen-decomposition pg_set_model computes for a PG_SPLIT_BF16 or a
 * 20-state context (host only, no device needed): Q = V B V^-1 with B block
 * diagonal, 1x1 blocks re[j] for real eigenvalues (kind[j] = 0) and, for a conjugate
 * pair re +- i im, the 2x2 block [[re, im], [-im, re]] on columns j, j+1
 * (kind 1, 2) that hold the real and imaginary parts of the eigenvector of
 * re + i im.  V, Vinv: m x m row-major (caller-allocated, like re, im,
 * kind[m]); cond = ||V||_1 ||V^-1||_1; resid = max|V B V^-1 - Q| / max|Q|.
 * The split-BF16 kernels use it when cond <= 1e6 and resid <= 1e-11, the
 * 20-state FP64 kernels when cond <= 1e4 and resid <= 1e-13 (FP32: as
 * split-BF16), each with a homogeneous model, and scaling and squaring
 * otherwise.  PG_E_MODEL when no decomposition was
 * found (e.g. the QR iteration did not converge). */
int pg_eigensystem(int32_t m, const double* Q, double* V, double* Vinv, double* re, double* im,
                   int32_t* kind, double* cond, double* resid);

/* ---- serving: many gradient sessions with continuous batching --------
 *
 * A server owns a worker thread, an upload thread and an HBM budget.
 * pg_server_open creates a session (its own tree, patterns and model,
 * checked as by pg_set_*, and planned on the caller's thread), which waits
 * in arrival order until the device bytes it may take (its buffers rounded
 * to the session memory pool's 64 KiB granule, plus 1/8 for the pool's
 * reuse of larger blocks) fit next to the admitted sessions and fewer than
 * max_sessions are admitted.  An admitted session's buffers are allocated
 * and its inputs copied by the upload thread on a stream of its own while
 * batches keep running; it is then charged what the pool handed out.  The
 * pool's blocks in use plus cached never exceed the budget.
 * pg_server_submit queues one evaluation (logL and, if want_grad, the
 * gradient) with host branch lengths t[2N-2]; the worker runs the oldest
 * queued call of every admitted session together as one batch (one launch
 * per kernel for all of them), and calls that arrive meanwhile join the next
 * batch.  A call gives the same result, bit for bit, whether it runs alone or
 * in a batch.  pg_server_wait blocks until a call is done, copies logL and
 * grad (caller-allocated, 2N-2), and reports the time from submit to
 * completion.  pg_server_close lets the session's queued calls finish, then
 * frees its device memory, which admits waiting sessions.  If a session's
 * upload fails, its queued calls complete with that error and the server
 * closes the session (pg_server_close then returns PG_E_STATE).  Server
 * functions are thread-safe. */
typedef struct pg_server pg_server;

/* precision: PG_FP64, PG_FP32 or PG_SPLIT_BF16 (every session of a server
 * uses it).  Errors: PG_E_INVALID (NULL, budget <= 0, max_sessions < 1),
 * PG_E_DEVICE, PG_E_UNSUPPORTED (an unknown precision). */
int pg_server_create(int device, int precision, int64_t hbm_budget_bytes, int32_t max_sessions,
                     pg_server** out);
/* Stops the worker (queued calls of admitted sessions finish first) and
 * frees everything. */
void pg_server_destroy(pg_server* srv);
const char* pg_server_last_error(const pg_server* srv);

/* Arguments as pg_set_tree, pg_set_patterns and pg_set_model.  Errors: those
 * of the pg_set_* calls, PG_E_OOM if the session alone exceeds the budget. */
int pg_server_open(pg_server* srv, int32_t n_tips, const int32_t* parent, int32_t n_patterns,
                   int32_t n_states, const uint64_t* tip_masks, const double* weights,
                   const double* Q, const double* root_freqs, int32_t n_cats,
                   const double* cat_rates, const double* cat_weights, int64_t* session);

/* t is copied.  Errors: PG_E_STATE (unknown or closing session),
 * PG_E_INVALID (t not finite or < 0). */
int pg_server_submit(pg_server* srv, int64_t session, const double* t, int32_t want_grad,
                     int64_t* ticket);

/* Returns the call's status (PG_OK, PG_E_ZERO_LIK, PG_E_DEVICE, ...); logL,
 * grad and latency_ns may be NULL.  A ticket can be waited for once. */
int pg_server_wait(pg_server* srv, int64_t ticket, double* logL, double* grad, int64_t* latency_ns);

int pg_server_close(pg_server* srv, int64_t session);

/* Counters, written to out[0..min(n, PG_SRV_STAT_COUNT)-1]: */
#define PG_SRV_STEPS          0  /* batches run                          */
#define PG_SRV_CALLS          1  /* calls completed                      */
#define PG_SRV_MAX_BATCH      2  /* largest batch                        */
#define PG_SRV_ADMITTED_TOTAL 3  /* sessions ever admitted               */
#define PG_SRV_ADMITTED_NOW   4  /* sessions admitted now                */
#define PG_SRV_WAITING_NOW    5  /* sessions waiting for admission now   */
#define PG_SRV_IN_USE_BYTES   6  /* device bytes of admitted sessions    */
#define PG_SRV_PEAK_BYTES     7  /* largest in-use bytes so far          */
#define PG_SRV_MAX_WAITING    8  /* longest admission queue so far       */
#define PG_SRV_PEAK_HELD      9  /* largest device bytes held by the session
                                    memory pool (in use plus cached), never
                                    above the budget                      */
#define PG_SRV_STAT_COUNT     10
int pg_server_stats(pg_server* srv, int64_t* out, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* PHYLOGRAD_H */
