/*
 * hqr.h -- C-ABI of libhqr.so: Hessenberg -> real Schur form on one MI355X (gfx950).
 *
 * The operation is the multishift QR algorithm with aggressive early deflation
 * (AED) of Myllykoski, "Algorithm 1019: A Task-based Multi-shift QR/QZ Algorithm
 * with Aggressive Early Deflation", ACM TOMS 48(1), 2021:
 *   - problem statement: Sec. 2, eqs. (hessenberg_form), (schur_form), (2by2_blocks):
 *     H = Q T Q^T with T upper quasi-triangular, 1x1 blocks for real eigenvalues
 *     and 2x2 blocks for complex conjugate pairs;
 *   - the iteration H <- Qhat^T H Qhat, Q <- Q Qhat: Sec. 2.1;
 *   - tightly coupled bulge chains chased in diagonal windows whose accumulated
 *     transformations are applied off-diagonal by matrix products: Sec. 2.3;
 *   - AED (window Schur form, spike test with eigenvalue reordering, Hessenberg
 *     restoration): Sec. 2.5 "Aggressive early deflation"; deflation
 *     conditions: Sec. 5.6 "Comment regarding the deflation conditions and
 *     the accuracy" (LAPACK-style by default, norm-stable and fixed on request).
 *
 * Conventions shared by every entry point
 *   - Matrices are FP64, column major.  All matrix/vector pointers are DEVICE
 *     pointers unless stated otherwise; the caller owns every buffer.
 *   - Return value: 0 ok; -k argument k invalid (non-finite H entries count as
 *     argument 1); +i failed to converge within the iteration limit (the
 *     1-based rows i+1..n hold converged eigenvalues); -1000-e a HIP runtime
 *     error e.
 *   - Streams: work is ordered after prior work on `stream` (0 = the legacy
 *     default stream).  The library keeps per-device workspace and helper
 *     streams, created on first use and released by hqr_finalize().
 */
#ifndef HQR_H
#define HQR_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm parameters; a zero field means "automatic".
 *   ns      shifts per sweep (even)                         (Sec. 2.3)
 *   nw      AED window size, at most 1024                    (Sec. 2.5)
 *   nmin    blocks of order <= nmin go to the small solver   (task 'small Schur', Sec. 3.2)
 *   nibble  skip the sweep when 100*nd > nibble*nw           (Sec. 2.5, repeated AED;
 *           0 = 60 for active blocks above 256 rows, 14 for smaller ones) 
 *   kexsh   exceptional shifts after kexsh steps without deflation
 *   itmax   iteration limit (AED steps + sweeps)             (Sec. 2.1)
 *   window  bulge-chasing window order (<= 96)              (Sec. 3.2, 'push bulges')
 *   bulges_per_window  bulges in one window chain
 *   defl_mode  deflation conditions of Sec. 5.6: 0 = LAPACK-style (item 1:
 *              Ahues-Tisseur subdiagonal test, spike entries against u|t_kk|
 *              or u*h^, floor nu*n/u); 1 = norm-stable (item 2: subdiagonal
 *              and spike entries against u*||H||_F, the Frobenius norm of the
 *              input's Hessenberg part); 2 = fixed (item 3: against
 *              defl_thold, finite and >= 0).  Other values are rejected.
 *   streams    1 = everything on the caller's stream; 2 = updates outside the
 *              active block and to Q on a second stream (Sec. 3.4, ordering,
 *              prioritization and lowest-priority tasks)
 *   small_shifts  shifts per sweep of the one-workgroup solver (2 = Francis
 *              double shift; 4..16 = chains of bulges shifted by the
 *              eigenvalues of the trailing block, Sec. 2.3)
 *   aed_ns, aed_nw, aed_nmin  ns, nw and nmin of the recursive solve that
 *              reduces an AED window larger than the one-workgroup solver
 *              (the AED reduce state of Sec. 3.3); nw is capped at 96
 *   aed_mode   how AED windows larger than 96 run (Sec. 3.5, "Adaptive
 *              approach"): 0 = adaptive, 1 = sequential whenever the window
 *              is at most aed_seq_max, 2 = always parallel.  Sequential: one
 *              workgroup reduces the window, tests every candidate and
 *              reorders the failures.  Parallel: the recursive solve on many
 *              kernels, then chains of deflation and reordering windows.
 *              Adaptive: sequential when the predicted time of the sequential
 *              AED (a w^3, a refined from the measured sequential AEDs) is
 *              below the predicted time of the update work still queued on
 *              the deferred stream, which it would overlap; windows above
 *              aed_seq_max always run in parallel.  Other values are rejected.
 *   aed_seq_max  largest window the sequential AED takes (0 = 512; at most 1024)
 *   aed_nibble   nibble of the recursive solve of AED windows larger than 96
 *              (0 = automatic) */
typedef struct hqr_params {
    int ns, nw, nmin, nibble, kexsh;
    int64_t itmax;
    int window, bulges_per_window;
    int defl_mode;
    double defl_thold;
    int streams;
    int small_shifts;
    int aed_ns, aed_nw, aed_nmin;
    int aed_mode, aed_seq_max;
    int aed_nibble;
} hqr_params;

/* Process-wide defaults used by later calls.  Returns 0 or -1 (NULL / invalid). */
int hqr_set_params(const hqr_params *p);
/* Current defaults (zeros mean automatic). */
int hqr_get_params(hqr_params *p);

/* Reduce the upper Hessenberg H (n x n, leading dimension ld >= max(1,n)) to
 * real Schur form.  In: H upper Hessenberg (entries below the first
 * subdiagonal are ignored); Q = Q0 (identity or a Hessenberg-reduction
 * factor), or NULL to skip accumulation (Q then uses the same ld).
 * Out: H = T (standardized 2x2 blocks, exact zeros below the subdiagonal;
 * padding rows n..ld-1 untouched), Q = Q0 * Qhat, wr/wi (device, n entries)
 * = eigenvalues in diagonal order, conjugate pairs adjacent with wi > 0 first.
 * Blocks the host until done: the driver reads back one small status record
 * per iteration (the deflation count and the shifts of each AED step). */
int hqr_schur(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi, void *stream);

/* Reduction of a dense square matrix to upper Hessenberg form, the phase
 * before the Schur reduction (Sec. 1: dense -> Hessenberg -> Schur form;
 * Sec. 5.5 "Comment regarding the Hessenberg reduction phase"):
 * A (n x n, leading dimension ld >= max(1,n), column major, device) is
 * overwritten by H = Q_h^T A Q_h with exact zeros below the subdiagonal;
 * Q (device, same ld; may be NULL) is overwritten by Q Q_h (pass the identity
 * to obtain Q_h).  Q_h e_1 = e_1 and the reflectors follow the convention
 * beta = -sign(alpha) ||x||, so H and Q_h are those of LAPACK's dgehrd/dorghr
 * up to rounding.  Blocked Householder reduction: per panel of 32 columns a
 * one-workgroup column kernel and a many-workgroup matrix-vector product,
 * then FP64-MFMA updates of the rest.  Blocks the host until done.
 * Returns 0, -k for a bad argument k (non-finite entries of A count as
 * argument 1), or -1000-e for a HIP error e. */
int hqr_hessenberg(double *A, double *Q, int64_t n, int64_t ld, void *stream);

/* Same as hqr_schur with explicit parameters for this call only (p may be NULL). */
int hqr_schur_ex(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi, void *stream,
                 const hqr_params *p);

/* Batched form for many small independent problems (the paper's
 * small-block double-shift Francis solver of Sec. 3.2, `small Schur'), one
 * workgroup per matrix.  Matrix i has order n[i], stored packed column major at
 * H + offsets[i] with leading dimension n[i]; Q likewise (Q may be NULL;
 * otherwise it must hold Q0, e.g. identity, on entry, and receives Q0*Qhat).
 * Orders <= 96 are solved with matrix and factor in LDS, larger ones in place
 * in global memory (the L2-resident path).  A counting sort on the device
 * orders the batch by decreasing order; two persistent grids (global tier,
 * then LDS tier) take matrices from that queue one at a time, longest first;
 * orders above a threshold go to half of the global grid only (cache
 * footprint; see hqr_set_batched_launch).
 * Orders <= 96 run double-shift steps; larger orders follow the per-bucket
 * table of hqr_set_batched_table (AED window and shifts, default double
 * shifts); hqr_params does not apply here.  Matrices of order 0 get info 0
 * and are not touched.
 * Eigenvalues of matrix i go to wr/wi + eig_offsets[i]; info[i] receives the
 * per-matrix code (0 or +i).  offsets, n, eig_offsets, info are device
 * arrays.  Asynchronous on `stream`.  The queue lives in a buffer the library
 * keeps per (device, stream): a call with a larger batch than any before on
 * that stream allocates it (4*(batch+8) bytes), so capture a call into a HIP
 * graph only after an uncaptured call of at least that batch on that stream.
 * Calls that overlap on one stream cannot happen; calls on different streams
 * use different queues.  Returns 0, or -k for a bad argument k. */
int hqr_schur_batched(double *H, double *Q, const int64_t *offsets, const int32_t *n, int32_t batch,
                      double *wr, double *wi, const int64_t *eig_offsets, int32_t *info, void *stream);

/* hqr_schur_batched for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the work queue in a fixed
 * device array of the library (4 * (8 + 2^20) bytes, held on each GPU the
 * library runs on until the process ends) instead of a buffer allocated on
 * first use.  batch must not exceed 2^20 (1048576); larger batches return -5
 * without doing any work.  The call allocates nothing, neither device nor
 * host memory.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (on different streams, or from several threads) race
 * and must not be issued; calls ordered on one stream are fine.  Arguments,
 * layout, ownership and return codes as for hqr_schur_batched. */
int hqr_schur_batched_noalloc(double *H, double *Q, const int64_t *offsets, const int32_t *n, int32_t batch,
                              double *wr, double *wi, const int64_t *eig_offsets, int32_t *info, void *stream);

/* Launch shape of the batched form's global-memory grid (orders > 96):
 * wg_per_cu workgroups per CU (1..8, default 2), and orders above wide_n
 * (96..4095, default 320) taken by half of that grid only, so that the
 * cache footprint of the matrices in flight (about 176*n bytes per bulge
 * position each) stays within L2.  Chosen by timing (the package's
 * autotuner); applies to later hqr_schur_batched calls.  Returns 0, -1 bad
 * wg_per_cu, -2 bad wide_n. */
int hqr_set_batched_launch(int32_t wg_per_cu, int32_t wide_n);
/* Current values (host pointers); returns 0, or -1 for a NULL pointer. */
int hqr_get_batched_launch(int32_t *wg_per_cu, int32_t *wide_n);

/* Per-size-bucket parameters of the batched form for orders above 96 (AED,
 * Sec. 2.5; shifts per step, Sec. 2.3): bucket i (0 <= i < nb <= 8) holds the
 * orders up to upper[i] (strictly increasing; the last bucket also takes
 * every larger order).  nw[i] = 0 runs double-shift Francis for the bucket;
 * otherwise nw[i] (8..64) is the AED window, held in LDS with its factor
 * while H and Q stay in global memory, and ns[i] (even, 2..64) the number of
 * undeflated candidates nearest the bottom used as shifts after each AED
 * step, in ns[i]/2 double-shift sweeps (in exact arithmetic one sweep with a
 * chain of ns[i]/2 bulges).  Active blocks of order <= 75, or after three AED
 * steps without a deflation, finish with double shifts.  nb = 0 (default)
 * restores double shifts for every order.  The package's autotuner picks the
 * table by timing candidates per bucket; applies to later hqr_schur_batched
 * calls.  Returns 0, -1 bad nb, -2 bad upper, -3 bad nw, -4 bad ns. */
int hqr_set_batched_table(int32_t nb, const int32_t *upper, const int32_t *nw, const int32_t *ns);
/* Current table (host arrays of 8 entries); returns 0, or -1 for a NULL pointer. */
int hqr_get_batched_table(int32_t *nb, int32_t *upper, int32_t *nw, int32_t *ns);

/* Right eigenvectors of H = Q T Q^T from its real Schur form, the phase after
 * the Schur reduction (Sec. 1: the eigenvectors of H are Q times those of
 * the Schur form).  T (quasi-triangular with standardized 2x2 blocks, as
 * hqr_schur returns it), Q: n x n, leading dimension ld, device; wr/wi: the
 * eigenvalues as hqr_schur returns them (diagonal order, pairs adjacent
 * with wi > 0 first).  X (n x n, leading dimension ldx, device) receives the
 * vectors in LAPACK's dgeev layout: column j holds the real vector of a real
 * eigenvalue; for a pair (j, j+1) columns j and j+1 hold the real and
 * imaginary parts of the vector of wr[j] + i wi[j].  Each vector has unit
 * 2-norm and its largest component real.  Vectors of T come from
 * quasi-triangular back substitution (one lane per eigenvalue, 2x2 blocks
 * solved exactly, pivots floored at u max|T|), then X = Q Y on FP64 MFMA.
 * n <= 8192.  Workspace (12 n^2 doubles) is kept per (device, stream);
 * blocks the host until done.  Returns 0, -k for a bad argument k, or
 * -1000-e for a HIP error e. */
int hqr_eigenvectors(const double *T, const double *Q, int64_t n, int64_t ld, const double *wr, const double *wi,
                     double *X, int64_t ldx, void *stream);

/* Backward pass of the eigenvalues (the differentiated form beside the
 * solver) for a batch of Schur forms H_i = Q_i T_i Q_i^T, packed like the
 * batched form: matrix i has order n[i] and T_i, Q_i and dH_i sit column major
 * at T + offsets[i], Q + offsets[i], dH + offsets[i] with leading dimension
 * n[i]; its eigenvalues (wr/wi, as returned by the solver: diagonal order,
 * pairs adjacent with wi > 0 first) and cotangents g = dL/dRe(lambda) +
 * i dL/dIm(lambda) (gwr/gwi) sit at offset e_i = n[0] + ... + n[i-1].
 * Writes dH_i = Re(conj(Y) diag(conj(g)/(y^H x)) X^T), X and Y holding the
 * right and left eigenvectors, obtained from T_i by quasi-triangular
 * substitution and back-transformed by Q_i (the eigenvector relation of
 * Sec. 2 "Modern QR algorithm and related work": the eigenvectors of H are
 * Q times those of the Schur form).  hess_mask != 0 zeroes entries below the
 * first subdiagonal (the forward reads only the Hessenberg part).
 * All arrays are device arrays; 0 <= n[i] <= 8192; eigenvalues must be
 * simple.  The call reads n and offsets back to the host (it synchronizes
 * `stream` once at its start), then enqueues the kernels asynchronously.
 * Workspace (10 n_i^2 + 1 doubles per matrix, in chunks of at most 2 GiB
 * unless one matrix needs more) is kept per (device, stream) and grows only;
 * calls on one stream are serialized.  Returns 0, -k for a bad argument k
 * (a negative or too large order counts as argument 4, a negative offset as
 * 3), or -1000-e for a HIP error e. */
int hqr_eig_backward_batched(const double *T, const double *Q, const int64_t *offsets, const int32_t *n,
                             int32_t batch, const double *wr, const double *wi, const double *gwr,
                             const double *gwi, double *dH, int32_t hess_mask, void *stream);

/* Generalized real Schur form of many small Hessenberg-triangular pairs (the
 * QZ variant: Sec. 2, remarks on the generalized case; Sec. 3.2 'push
 * infinities').  Pair b has order n[b] >= 0, H_b upper Hessenberg and T_b
 * upper triangular (entries below are ignored), each stored column major
 * with leading dimension n[b] at H + offsets[b] and T + offsets[b] (device).
 * Out: H_b = S_b = Q_b^T H_b Z_b quasi upper triangular (2x2 blocks only for
 * complex conjugate pairs, exact zeros below), T_b = Q_b^T T_b Z_b upper
 * triangular; Q and Z (device, same layout, may be NULL) are multiplied from
 * the right (pass identities to obtain Q_b and Z_b).  The generalized
 * eigenvalues (alphar + i alphai) / beta of pair b are written in diagonal
 * order at eig_offsets[b] (beta >= 0; beta = 0 marks an infinite eigenvalue,
 * decided by |t_kk| <= u ||T_b||_F as in the paper; such an eigenvalue is
 * chased to the top of its block by rotations and deflated there).  Double
 * implicit shift QZ, one workgroup per pair: pairs of order <= 64 are held in
 * LDS with Q and Z, larger ones are reduced in place in global memory (below
 * the subdiagonal of H and the diagonal of T the arrays are overwritten with
 * zeros).  info[b] = 0, k > 0 when the iteration limit 30 max(10, n) was
 * reached with row k-1 unconverged, -1 for a negative order.  Asynchronous on
 * `stream`.  Returns 0, -k for a bad argument k (NULL pointer, batch < 0), or
 * -1000-e for a HIP error. */
int hqr_qz_batched(double *H, double *T, double *Q, double *Z, const int64_t *offsets, const int32_t *n,
                   int32_t batch, double *alphar, double *alphai, double *beta, const int64_t *eig_offsets,
                   int32_t *info, void *stream);

/* Timing and counters of the last hqr_schur call on this thread:
 * stats[0] AED steps, [1] sweeps, [2] shifts used, [3] eigenvalues deflated by
 * AED, [4] small-solver calls, [5] host synchronizations, [6] kernel launches,
 * [7] chase windows, [8] deflation windows and [9] reordering windows of the
 * deflation checks of large AED windows, [10] sequential and [11] parallel
 * AEDs of windows larger than 96.  Returns the number of entries written
 * (<= len, at most 12). */
int hqr_last_stats(int64_t *stats, int len);

/* Kernel-class timing for measurement tools.  When enabled, the driver
 * brackets its launches with HIP events on the launching stream and sums the
 * elapsed times per class: 0 one-workgroup LDS iteration (small solver / AED),
 * 1 bulge-chasing windows, 2 FP64-MFMA update products, 3 large-window AED
 * kernels, 4 other.  hqr_profile_read returns, per class, milliseconds,
 * launches, and the algorithmic flops and bytes the driver counted for those
 * launches (update products: 2 K^2 per panel row/column; bytes: panel read
 * and write plus the factor).  Reading synchronizes with the recorded events.
 * Returns the number of classes written, or -1 on NULL arguments. */
int hqr_profile_enable(int on);
int hqr_profile_reset(void);
int hqr_profile_read(double *ms, int64_t *launches, double *flops, double *bytes, int nclass);
/* Counters of the one-workgroup LDS iteration kernel summed over the profiled
 * launches: [0..3] device wall-clock ticks (100 MHz) of the Schur solve, the
 * reordering (spike test and swaps), the Hessenberg restoration and the whole
 * kernel; [4] barrier-separated bulge-chase phases; [5] single-bulge steps;
 * [6] adjacent-block swaps; [7] launches that solved a small block; [8]
 * launches that performed an AED step; [9] phases of the pipelined
 * reordering.  Writes min(len, 10) entries and returns that count, or -1 on
 * NULL / len <= 0. */
int hqr_profile_ticks(int64_t *ticks, int len);

/* Free per-device workspace and helper streams. */
int hqr_finalize(void);

#ifdef __cplusplus
}
#endif
#endif
