// Internal declarations shared by the kernels and the host driver of libhqr.
// Not part of the public ABI (see include/hqr.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hqr {

// Largest matrix order the one-workgroup solver keeps in LDS together with its
// accumulated orthogonal factor (2 * 96 * 97 * 8 B = 149 KB of the 160 KB LDS).
constexpr int MMAX = 96;
constexpr int LDM = MMAX + 1;      // odd leading dimension: spreads LDS banks
constexpr int NT = 256;            // threads of the LDS kernels (4 waves)
constexpr int WMAX = 96;           // largest bulge-chasing window
constexpr int GMAX = 16;           // most bulges chased in one window
constexpr int MAXWIN = 16;         // most windows in one chase round
constexpr int MAXCAND = 1024;      // candidate eigenvalues returned by one AED step
constexpr int MAX_UPDATE_K = 1024; // largest AED window (window copies and factor workspaces are sized for it)

// Deflation conditions of the solver (Sec. 5.6, "Comment regarding the
// deflation conditions and the accuracy").  thr < 0: LAPACK-style conditions
// (item 1): the Ahues-Tisseur subdiagonal test and the u|t_kk| / u h^ spike
// tests, floor smlnum = nu n / u.  thr >= 0: every subdiagonal entry and every
// spike entry of a candidate block is compared with thr -- the norm-stable
// conditions (item 2) with thr = u ||H||_F, or the fixed conditions (item 3)
// with thr = the caller's threshold.  smlnum also floors the Bai-Demmel
// acceptance test in every mode.
struct Defl {
    double smlnum;
    double thr;
};

// Status record of one iteration, written by the device and read back by the
// host (the only host synchronization per iteration).
struct IterStatus {
    int kind;    // 0: the block was small and is now in Schur form; 1: AED step
    int ktop;    // top row of the active block
    int kwtop;   // top row of the AED window (kind 1) / of the block (kind 0)
    int nw;      // order of the window / block that was transformed
    int nd;      // eigenvalues deflated (kind 1)
    int ns;      // undeflated candidates (kind 1)
    int ncand;   // number of candidate eigenvalues in cr/ci
    int info;    // 0, or >0 when the small solver did not converge
    int changed; // 1 when H was modified and the factor must be propagated
    int pad;     // scratch word for small device-to-host reads
    int nphase;  // LDS iteration kernel: barrier-separated bulge-chase phases
    int nbstep;  // LDS iteration kernel: single-bulge steps (a phase moves one or more bulges)
    int nswap;   // LDS iteration kernel: adjacent-block swaps attempted
    int nrphase; // LDS iteration kernel: phases of the pipelined reordering
    double beta; // new subdiagonal entry left of a large AED window after restoration;
                 // for the LDS iteration kernel: its algorithmic flop count
    long long tick[4]; // LDS iteration kernel: wall-clock ticks of Schur solve, reordering, restoration, total
    double cr[MAXCAND];
    double ci[MAXCAND];
};

// One bulge-chasing window of a chase round.  Global row/column indices.
struct ChaseWin {
    int a, wa;        // window rows/cols a .. a+wa-1
    int p0;           // position of the group's lowest bulge at step 0
    int nsteps;       // chase steps in this window
    int kend;         // last reflector position allowed in this window
    int nb;           // bulges of the group
    int shift_off;    // index of the group's first shift in the shift array
    int slot;         // index of the U buffer written by this window
    int vig_lo, vig_hi; // positions whose subdiagonal is final after the top bulge passes
};

struct ChaseRound {
    int nwin;
    int ktop, kbot;
    ChaseWin w[MAXWIN];
};

// One in-place update X <- X*U (side 0) or X <- U^T*X (side 1) with U of order
// K (stored transposed, padded to K16 = round_up(K,16): Ut[j + k*K16] = U[k][j]).
//   side 0: X is a (rows x K) panel: element (r, k) at X[r + k*ldx]
//   side 1: X is a (K x cols) panel: element (k, c) at X[k + c*ldx]
struct UpdJob {
    double *X;
    const double *Ut;
    int64_t ldx;
    int count;   // rows (side 0) or columns (side 1) of the panel
    int K, K16;
    int side;
    int tile;    // panel rows/cols per workgroup
    int tiles;   // ceil(count / tile)
    int pad;
};
constexpr int MAXJOBS = 48;
struct UpdBatch {
    int njobs;
    int pad;
    int first_tile[MAXJOBS + 1];
    UpdJob job[MAXJOBS];
};

// ---- launchers (hqr_lds.hip) ----
// One driver iteration on the active block that ends at kbot: locate ktop,
// then either reduce a small block to Schur form or perform an AED step with
// window nw (<= MMAX).  Writes the factor (transposed, padded) to Ut.
hipError_t launch_iter(double *H, int64_t ld, int n, int ilo, int kbot, int nw, int nmin,
                       Defl dfl, int64_t itmax, double *Ut, IterStatus *st, hipStream_t s, int nsmall);
// Locate the top of the active block only (st->ktop).
hipError_t launch_find_block(double *H, int64_t ld, int ilo, int kbot, Defl dfl, IterStatus *st,
                             hipStream_t s);
// Chase round: one workgroup per window; U factors written transposed to Ubuf.
hipError_t launch_chase(double *H, int64_t ld, const ChaseRound &r, const double *sr, const double *si,
                        Defl dfl, double *Ubuf, int64_t ustride, hipStream_t s);
// Window [nw - wd, nw) of a large AED window (T in global memory; wd <=
// MMAX, one row less if the top boundary would split a 2x2 block), its
// spike taken from row 0 of V: a deflation window tests its candidates
// bottom-up with the nforced bottom ones counted as failed, and moves the
// failures to its top; a reordering window (reorder != 0) moves the nforced
// bottom candidates to its top without testing the others.
hipError_t launch_corner_deflate(double *T, int64_t ldt, int nw, int wd, const double *V, int64_t ldv,
                                 double s, Defl dfl, double *Ut, IterStatus *st, int nforced, int reorder,
                                 hipStream_t stream);
// Hessenberg restoration of T(0:ns,0:ns) in global memory with the spike,
// applied to T(0:ns, ns:nw) and to V (rows 0..nv-1).
hipError_t launch_restore(double *T, int64_t ldt, int nw, int ns, double *V, int64_t ldv, int nv,
                          double s, double *work, IterStatus *st, hipStream_t stream);
// Copy a window out of H (zeroing below the subdiagonal), set V = I.
hipError_t launch_window_copy(const double *H, int64_t ld, int kwtop, int nw, double *T, int64_t ldt,
                              double *V, int64_t ldv, hipStream_t s);
// Eigenvalues of the diagonal blocks of a quasi-triangular T(0:m, 0:m).
hipError_t launch_block_eigs(const double *T, int64_t ldt, int m, double *wr, double *wi,
                             hipStream_t s);
// Standardize the 2x2 blocks of T (n x n) in rows lo..n-1 and extract
// eigenvalues, applying the rotations to T and Q (may be NULL).
hipError_t launch_finalize_ws(double *H, int64_t ld, int n, int lo, double *Q, double *wr, double *wi, double *ws,
                              hipStream_t s);
hipError_t launch_check_finite(const double *H, int64_t ld, int n, int *flag, hipStream_t s);
hipError_t launch_check_finite_full(const double *A, int64_t ld, int n, int *flag, hipStream_t s);
// Frobenius norm of the Hessenberg part of H (n x n) into *out (device), for
// the norm-stable deflation threshold; ws holds n doubles of scratch.
hipError_t launch_hess_fro(const double *H, int64_t ld, int n, double *ws, double *out, hipStream_t s);
hipError_t launch_zero_lower(double *H, int64_t ld, int n, hipStream_t s);
hipError_t launch_transpose_pad(const double *V, int64_t ldv, int K, double *Ut, int K16,
                                hipStream_t s);
// Work queue of the batched form: QHDR header ints, then the matrix indices
// in order of decreasing order n (longest first).
constexpr int QHDR = 8;
// Per-size-bucket parameters of the batched form: bucket i holds the orders
// up to upper[i] (ascending; the last bucket takes every larger order); nw[i]
// is its AED window (0: double-shift Francis only; at most BWIN) and ns[i] the
// shifts per AED step.  Buckets apply to the orders above the LDS limit.
constexpr int BWIN = 64;
constexpr int MAXBUCKET = 8;
struct BatchedTable {
    int nb;
    int upper[MAXBUCKET], nw[MAXBUCKET], ns[MAXBUCKET];
};
hipError_t launch_batched(double *H, double *Q, const int64_t *offsets, const int32_t *n, int batch,
                          double *wr, double *wi, const int64_t *eoff, int32_t *info, int32_t *queue,
                          int wg_per_cu, int wide_n, const BatchedTable &tab, hipStream_t s);
// Backward pass of the eigenvalues (hqr_grad.hip): one descriptor per matrix
// (offsets in doubles of T_b/Q_b/dH_b, of its eigenvalue slots, of its
// workspace from the chunk's base -- 10 n^2 + 1 doubles -- and its order).
struct BwdDesc {
    int64_t toff, eoff, woff;
    int n, pad;
};
// Right eigenvectors of H = Q T Q^T (T, Q packed with leading dimension n, one
// descriptor with woff 0) into X (dgeev layout, leading dimension ldx).
hipError_t launch_eigenvectors(const double *T, const double *Q, const BwdDesc *D, int n, const double *wr,
                               const double *wi, double *ws, double *X, int64_t ldx, hipStream_t s);
// One chunk of nb matrices (descriptors D, device), largest order nmax.
hipError_t launch_eig_backward_chunk(const double *T, const double *Q, const BwdDesc *D, int nb, int nmax,
                                     const double *wr, const double *wi, const double *gwr, const double *gwi,
                                     double *dH, int hess_mask, double *ws, hipStream_t s);

// ---- blocked Householder Hessenberg reduction (hqr_hess.hip) ----
constexpr int NBH = 32; // panel width
// Doubles of workspace hess_reduce / restore_blocked need for order m, nr
// extra columns and nz rows of Z.
size_t hess_ws_doubles(int m, int nr, int nz);
// A (m x m, lda) <- Q^T A Q upper Hessenberg; the nr columns stored right of A
// (A + m*lda ...) <- Q^T (them); Z (nz x m, ldz; may be NULL) <- Z Q.
hipError_t hess_reduce(double *A, int64_t lda, int m, int nr, double *Z, int64_t ldz, int nz, double *ws,
                       hipStream_t s);
// Hessenberg restoration of a large AED window: spike reflector from s * V(0, 0:ns),
// applied to T rows/columns 0..ns-1 and V columns, then hess_reduce of
// T(0:ns, 0:ns) with the window columns ns..nw-1 and V (nv rows); the new
// subdiagonal entry left of the window (beta) goes to *beta_dev.
hipError_t restore_blocked(double *T, int64_t ldt, int nw, int ns, double *Vw, int64_t ldv, int nv, double s,
                           double *ws, double *beta_dev, hipStream_t st);

// ---- launchers (hqr_gemm.hip) ----
// Sequential AED of a window copy (one workgroup): Schur form, spike test and
// reordering of all candidates; the result in st (ns, nd, info).
hipError_t launch_seq_aed(double *T, int w, double *V, double s, Defl dfl, int nwb, int nsb, IterStatus *st,
                          hipStream_t strm);
hipError_t launch_updates(const UpdBatch &b, hipStream_t s);
void free_update_ws();
// QZ variant: one workgroup per Hessenberg-triangular pair of order <= 64 (hqr_qz.hip).
hipError_t launch_qz_batched(double *H, double *T, double *Q, double *Z, const int64_t *offsets, const int32_t *n,
                             int batch, double *alphar, double *alphai, double *beta, const int64_t *eoff,
                             int32_t *info, hipStream_t s);
// C = beta C + alpha op(A) op(B) (column major; op 1 = transposed), FP64 MFMA,
// 64 x 64 tiles; tag 0 / 1 only selects the kernel name shown in profiles.
hipError_t gemm_mfma(int tag, int mm, int nn, int kk, double alpha, const double *A, int64_t lda, int opA,
                     const double *B, int64_t ldb, int opB, double beta, double *C, int64_t ldc, hipStream_t s);
int update_tile(int K16, int side);

} // namespace hqr
