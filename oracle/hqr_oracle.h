/*
 * hqr_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded CPU reference for the multishift QR algorithm
 * with aggressive early deflation (Myllykoski, "Algorithm 1019: A Task-based
 * Multi-shift QR/QZ Algorithm with Aggressive Early Deflation", ACM TOMS 48(1),
 * 2021).  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header or constant with the GPU library.
 *
 * All matrices are column major FP64 with leading dimension ld >= n.
 * Q may be NULL (transformations not accumulated).
 * Return codes: 0 ok, -k argument k invalid, +i failed to converge (rows
 * i+1..n hold converged eigenvalues, in the 1-based LAPACK sense).
 */
#ifndef HQR_ORACLE_H
#define HQR_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Real Schur form of an upper Hessenberg H (Sec. 2, eqs. schur_form / 2by2_blocks).
   H is overwritten by T; Q (if non-NULL) by Q*Qhat.  wr/wi receive eigenvalues
   in diagonal order, conjugate pairs adjacent with positive imaginary part first. */
int hqr_oracle_schur(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi);

/* Same, with explicit algorithm parameters (0 = automatic) and run statistics:
   stats[0] = AED steps, stats[1] = sweeps, stats[2] = shifts used,
   stats[3] = eigenvalues deflated by AED, stats[4] = small-solver calls,
   stats[5] = reflectors applied.  stats may be NULL. */
int hqr_oracle_schur_ex(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi,
                        int ns, int nw, int nmin, int64_t itmax, int64_t *stats);

/* Same as hqr_oracle_schur_ex with the deflation conditions of Sec. 5.6
   ("Comment regarding the deflation conditions and the accuracy"):
   defl_mode 0 = LAPACK-style (item 1), 1 = norm-stable (item 2: subdiagonal
   and spike entries <= u ||H||_F, the norm of the input's Hessenberg part),
   2 = fixed (item 3: <= defl_thold).  Returns -12 for a bad mode/threshold. */
int hqr_oracle_schur_defl(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi,
                          int ns, int nw, int nmin, int64_t itmax, int64_t *stats, int defl_mode,
                          double defl_thold);

/* One multishift sweep (Sec. 2.3, tightly coupled chain) on the active block
   [ktop, kbot] (0-based, inclusive) with nshifts shifts (even; conjugate pairs
   adjacent, bulge j uses shifts 2j, 2j+1).  vigilant != 0 enables the
   vigilant deflation check of each subdiagonal entry once the topmost
   bulge of the chain has passed it (LAPACK-style conditions). */
int hqr_oracle_sweep(double *H, double *Q, int64_t n, int64_t ld, int64_t ktop, int64_t kbot,
                     int nshifts, const double *sr, const double *si, int vigilant);

/* Swap the adjacent diagonal blocks of sizes p and q that start at row j of the
   quasi-triangular T (Sec. 2.5, eigenvalue reordering).  Returns 0 on success,
   1 if the swap was rejected as too ill-conditioned (T and Q untouched). */
int hqr_oracle_swap(double *T, double *Q, int64_t n, int64_t ld, int64_t j, int p, int q);

/* Standardize a real 2x2 block [[a,b],[c,d]] in place (eq. 2by2_blocks):
   returns the rotation (cs, sn) with G = [[cs,-sn],[sn,cs]], block <- G^T B G,
   and 1 for a complex pair, 0 for real eigenvalues. */
int hqr_oracle_std2x2(double *a, double *b, double *c, double *d, double *cs, double *sn);

/* One aggressive-early-deflation step (Sec. 2.5) on the active block [ktop,kbot]
   with window nw.  Returns nd >= 0 (eigenvalues deflated); writes the
   undeflated candidates to cr/ci (count in *ncand). */
int hqr_oracle_aed(double *H, double *Q, int64_t n, int64_t ld, int64_t ktop, int64_t kbot,
                   int nw, double *cr, double *ci, int *ncand);
/* Same with the deflation conditions of Sec. 5.6 (defl_mode as for
   hqr_oracle_schur_defl; the norm-stable threshold uses ||H||_F of the H
   passed here).  Returns -11 for a bad mode/threshold. */
int hqr_oracle_aed_ex(double *H, double *Q, int64_t n, int64_t ld, int64_t ktop, int64_t kbot,
                      int nw, double *cr, double *ci, int *ncand, int defl_mode, double defl_thold);

/* Gradient of a real loss of the eigenvalues: given the Schur form (T, Q) of H
   and g_i = dL/dRe(l_i) + i dL/dIm(l_i), writes dL/dH (n x n, leading dim ld).
   hess_mask != 0 zeroes entries below the first subdiagonal. */
int hqr_oracle_eig_backward(const double *T, const double *Q, int64_t n, int64_t ld,
                            const double *wr, const double *wi, const double *gwr,
                            const double *gwi, double *dH, int hess_mask);

/* Generalized real Schur form of a Hessenberg-triangular pair (the QZ
   variant: Sec. 2 remarks on the generalized case; Sec. 3.2 'push
   infinities'): H (upper Hessenberg) and T (upper triangular), n x n,
   leading dimension ld, column major, are overwritten by S = Q^T H Z (quasi
   upper triangular, 2x2 blocks only for complex pairs) and Q^T T Z (upper
   triangular); Q and Z (may be NULL) are multiplied from the right.  The
   generalized eigenvalues (alphar + i alphai) / beta go to the three arrays
   in diagonal order (beta >= 0; beta = 0 is an infinite eigenvalue).  Double
   implicit shift QZ with 3x3 reflectors from the left and right reflectors
   restoring T; diagonal entries of T with |t_kk| <= u ||T||_F are set to
   zero and the infinite eigenvalue is chased to the top of its block by
   rotations and deflated there.  itmax <= 0: 30 max(10, n) iterations.
   Returns 0, or 1 + the bottom row of the block that did not converge. */
int hqr_oracle_qz(double *H, double *T, double *Q, double *Z, int64_t n, int64_t ld, double *alphar,
                  double *alphai, double *beta, int64_t itmax);

/* Test hook: plants one deliberate mistake (see the mutation list in the
   source) so that tests can show the pins catch it.  0 = none. */
void hqr_oracle_set_mutation(int m);

/* Test hook: on != 0 makes every block swap report rejection (failure forcing). */
void hqr_oracle_force_swap_failure(int on);

/* Test hook: swaps rejected by the Bai-Demmel stability test since the last
   reset (forced rejections not counted); reset != 0 clears the count. */
int64_t hqr_oracle_swap_rejections(int reset);

#ifdef __cplusplus
}
#endif
#endif
