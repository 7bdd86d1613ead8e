/*
 * hqr_oracle.c -- TEST INFRASTRUCTURE ONLY (see hqr_oracle.h).
 *
 * A plain CPU statement of the multishift QR algorithm with aggressive early
 * deflation described by Myllykoski (ACM TOMS 48(1), 2021), written for
 * readability, not speed:
 *   - every orthogonal transformation is applied directly to the full rows and
 *     columns of H (and to Q); there is no accumulation into windows and no
 *     blocking, so nothing here resembles the GPU implementation;
 *   - the small-block solver is the textbook double-implicit-shift Francis
 *     iteration (Sec. 2.2 and Fig. double_shift of the paper; Golub & Van Loan
 *     Algs. 7.5.1-7.5.2);
 *   - the sweep introduces a tightly coupled chain of bulges one by one and
 *     chases them as a unit (Sec. 2.3, Fig. multi_shift);
 *   - AED follows the three sub-steps of Sec. 2.5 (Fig. multi_shift_aed):
 *     Schur-reduce the window, test candidates bottom-up with the deflation
 *     conditions of Sec. 5.6 "Comment regarding the deflation conditions and
 *     the accuracy" (LAPACK-style by default; norm-stable and fixed on
 *     request) and move failures to the top with Bai-Demmel swaps, then
 *     remove the spike by a Householder reflector and a Householder
 *     Hessenberg reduction;
 *   - failed candidates become the next shifts; the AED step is repeated when
 *     it deflated many eigenvalues (Sec. 2.5, last paragraph).
 * Readings of points the paper leaves open are marked "Reading:".
 */
#include "hqr_oracle.h"
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* Unit roundoff as fixed by the accuracy-metrics section (u = 2^-52). */
static const double U = DBL_EPSILON;

static int g_mut = 0;
void hqr_oracle_set_mutation(int m) { g_mut = m; }

/* Failure forcing (test hook): every swap is reported as rejected, which
   exercises the halting rule of the reordering. */
static int g_force_reject = 0;
void hqr_oracle_force_swap_failure(int on) { g_force_reject = on; }
/* Mutation list (test hook only):
 *  1  shift polynomial first column drops the h12*h21 term
 *  2  reflectors are not applied to Q
 *  3  AED propagates V^T instead of V to the rows above the window
 *  4  1x1 swap applies the rotation from the left only
 *  5  complex 2x2 eigenvalue imaginary part drops the |c| factor
 *  6  AED deflation threshold loosened by 1e8
 *  7  gradient uses g instead of conj(g)
 *  8  spike reflector is not applied to the columns right of the undeflated part
 *  9  the 2x2 AED threshold h^ drops both square roots
 * 10  the 2x2 AED threshold h^ uses |t(k-1,k)| in place of sqrt|t(k-1,k) t(k,k-1)|
 * 11  the swap acceptance threshold drops the factor ||D||_max (10 u only)
 * 12  the norm-stable / fixed 2x2 AED test looks at the bottom spike entry only
 * 13  the norm-stable threshold uses max |h_ij| in place of ||H||_F
 */

/* Swaps rejected by the stability test since the last reset (test hook). */
static long g_rejects = 0;
int64_t hqr_oracle_swap_rejections(int reset)
{
    long r = g_rejects;
    if (reset) g_rejects = 0;
    return (int64_t)r;
}

typedef struct {
    int ns, nw, nmin, nibble, kexsh;
    long itmax;
    double smlnum; /* nu * n / u with n the order of the full problem */
    /* Deflation conditions (Sec. 5.6): 0 = LAPACK-style; 1 = norm-stable and
       2 = fixed, both an absolute threshold dthr on subdiagonal and spike
       entries (u ||H||_F resp. the caller's epsilon_thold). */
    int defl_mode;
    double dthr;
    int64_t *stats;
} oparams;

/* ------------------------------------------------------------------------- */
/* Elementary pieces                                                           */
/* ------------------------------------------------------------------------- */

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* Overflow-safe Euclidean norm of x[0..m-1]. */
static double norm2(int m, const double *x)
{
    double scale = 0, ssq = 1;
    for (int i = 0; i < m; ++i) {
        double a = fabs(x[i]);
        if (a == 0) continue;
        if (a > scale) {
            ssq = 1 + ssq * (scale / a) * (scale / a);
            scale = a;
        } else {
            ssq += (a / scale) * (a / scale);
        }
    }
    return scale * sqrt(ssq);
}

/* Householder reflector P = I - tau v v^T, v[0] = 1, with P x = beta e_0.
   Reading (sign convention): beta = -sign(x0) ||x||, sign(0) = +1; when
   x[1..] is zero the reflector is the identity (tau = 0, beta = x0). */
static void house(int m, const double *x, double *v, double *tau, double *beta)
{
    v[0] = 1.0;
    double tail = (m > 1) ? norm2(m - 1, x + 1) : 0.0;
    if (tail == 0.0) {
        *tau = 0.0;
        *beta = x[0];
        for (int i = 1; i < m; ++i) v[i] = 0.0;
        return;
    }
    double nrm = hypot(x[0], tail);
    double b = (x[0] >= 0.0) ? -nrm : nrm;
    *tau = (b - x[0]) / b;
    double scal = 1.0 / (x[0] - b);
    for (int i = 1; i < m; ++i) v[i] = x[i] * scal;
    *beta = b;
}

/* rows r0..r0+m-1 of A, columns c0..c1:  A <- P A */
static void refl_left(double *A, long ld, int r0, int m, const double *v, double tau, int c0, int c1)
{
    if (tau == 0.0) return;
    for (int j = c0; j <= c1; ++j) {
        double s = 0;
        for (int i = 0; i < m; ++i) s += v[i] * A[IX(r0 + i, j, ld)];
        s *= tau;
        for (int i = 0; i < m; ++i) A[IX(r0 + i, j, ld)] -= s * v[i];
    }
}

/* columns c0..c0+m-1 of A, rows r0..r1:  A <- A P */
static void refl_right(double *A, long ld, int c0, int m, const double *v, double tau, int r0, int r1)
{
    if (tau == 0.0 || A == NULL) return;
    for (int i = r0; i <= r1; ++i) {
        double s = 0;
        for (int j = 0; j < m; ++j) s += A[IX(i, c0 + j, ld)] * v[j];
        s *= tau;
        for (int j = 0; j < m; ++j) A[IX(i, c0 + j, ld)] -= s * v[j];
    }
}

/* Rotation G = [[cs,-sn],[sn,cs]] on indices (k,k+1):
   rows k,k+1 (columns c0..c1) <- G^T rows;  columns (rows r0..r1) <- columns G. */
static void rot_left(double *A, long ld, int k, double cs, double sn, int c0, int c1)
{
    for (int j = c0; j <= c1; ++j) {
        double x = A[IX(k, j, ld)], y = A[IX(k + 1, j, ld)];
        A[IX(k, j, ld)] = cs * x + sn * y;
        A[IX(k + 1, j, ld)] = -sn * x + cs * y;
    }
}
static void rot_right(double *A, long ld, int k, double cs, double sn, int r0, int r1)
{
    if (A == NULL) return;
    for (int i = r0; i <= r1; ++i) {
        double x = A[IX(i, k, ld)], y = A[IX(i, k + 1, ld)];
        A[IX(i, k, ld)] = cs * x + sn * y;
        A[IX(i, k + 1, ld)] = -sn * x + cs * y;
    }
}

/* Dense m x m orthogonal G (column major, m <= 4) on indices k..k+m-1. */
static void small_left(double *A, long ld, int k, int m, const double *G, int c0, int c1)
{
    double t[4];
    for (int j = c0; j <= c1; ++j) {
        for (int r = 0; r < m; ++r) {
            double s = 0;
            for (int i = 0; i < m; ++i) s += G[i + r * m] * A[IX(k + i, j, ld)];
            t[r] = s;
        }
        for (int r = 0; r < m; ++r) A[IX(k + r, j, ld)] = t[r];
    }
}
static void small_right(double *A, long ld, int k, int m, const double *G, int r0, int r1)
{
    if (A == NULL) return;
    double t[4];
    for (int i = r0; i <= r1; ++i) {
        for (int c = 0; c < m; ++c) {
            double s = 0;
            for (int l = 0; l < m; ++l) s += A[IX(i, k + l, ld)] * G[l + c * m];
            t[c] = s;
        }
        for (int c = 0; c < m; ++c) A[IX(i, k + c, ld)] = t[c];
    }
}

/* ------------------------------------------------------------------------- */
/* 2x2 standardization (eq. 2by2_blocks: complex pairs only in 2x2 blocks)    */
/* ------------------------------------------------------------------------- */

/* Rotation that standardizes B = [[a,b],[c,d]].  Reading of "standardized":
   real eigenvalues -> upper triangular; complex -> equal diagonal, b'c' < 0.
   mode: 0 = already standard, 1 = rotate to triangular, 2 = rotate to equal diagonal. */
static int std_rotation(double a, double b, double c, double d, double *cs, double *sn)
{
    *cs = 1.0;
    *sn = 0.0;
    if (c == 0.0) return 0;
    if (b == 0.0) { /* swap the two diagonal entries: G = [[0,-1],[1,0]] */
        *cs = 0.0;
        *sn = 1.0;
        return 1;
    }
    double p = 0.5 * (a - d);
    double sc = dmax(fabs(p), dmax(fabs(b), fabs(c)));
    double disc = (p / sc) * (p / sc) + (b / sc) * (c / sc);
    if (disc >= 0.0) {
        /* first column of G along the eigenvector (z, c), z = lambda1 - d with
           lambda1 = (a+d)/2 + sign(p) sqrt(p^2 + bc) (no cancellation). */
        double z = p + copysign(sc * sqrt(disc), p);
        double r = hypot(z, c);
        *cs = z / r;
        *sn = c / r;
        return 1;
    }
    if (a == d) return 0; /* disc < 0 with p = 0 means b c < 0: already standard */
    /* choose theta with (a-d) cos 2theta + (b+c) sin 2theta = 0, cos 2theta >= 0 */
    double al = b + c, be = a - d;
    double r = hypot(al, be);
    double sg = (al >= 0.0) ? 1.0 : -1.0;
    double c2 = sg * al / r, s2 = -sg * be / r;
    *cs = sqrt(0.5 * (1.0 + c2));
    *sn = s2 / (2.0 * *cs);
    return 2;
}

int hqr_oracle_std2x2(double *a, double *b, double *c, double *d, double *cs, double *sn)
{
    double B[4] = {*a, *c, *b, *d};
    double ccs = 1, ssn = 0;
    int cplx = 0;
    for (int pass = 0; pass < 3; ++pass) {
        double x, y;
        int mode = std_rotation(B[0], B[2], B[1], B[3], &x, &y);
        if (mode == 0) {
            cplx = (B[1] != 0.0);
            break;
        }
        rot_left(B, 2, 0, x, y, 0, 1);
        rot_right(B, 2, 0, x, y, 0, 1);
        double t = ccs * x - ssn * y; /* compose G_total = G_total * G */
        ssn = ssn * x + ccs * y;
        ccs = t;
        if (mode == 1) {
            B[1] = 0.0;
            cplx = 0;
            break;
        }
        double avg = 0.5 * (B[0] + B[3]);
        B[0] = B[3] = avg;
        if (B[2] * B[1] < 0.0) {
            cplx = 1;
            break;
        }
    }
    *a = B[0];
    *c = B[1];
    *b = B[2];
    *d = B[3];
    *cs = ccs;
    *sn = ssn;
    return cplx;
}

/* Standardize the 2x2 block at (k,k+1) of the n x n matrix H in place,
   transforming full rows (columns k..n-1), columns (rows 0..k+1) and Q.
   Returns 1 for a complex pair, 0 if the block is (now) triangular. */
static int standardize_at(double *H, long ld, int n, double *Q, long ldq, int nq, int k)
{
    for (int pass = 0; pass < 3; ++pass) {
        double a = H[IX(k, k, ld)], b = H[IX(k, k + 1, ld)];
        double c = H[IX(k + 1, k, ld)], d = H[IX(k + 1, k + 1, ld)];
        double cs, sn;
        int mode = std_rotation(a, b, c, d, &cs, &sn);
        if (mode == 0) return c != 0.0;
        rot_left(H, ld, k, cs, sn, k, n - 1);
        rot_right(H, ld, k, cs, sn, 0, k + 1);
        if (g_mut != 2) rot_right(Q, ldq, k, cs, sn, 0, nq - 1);
        if (mode == 1) {
            H[IX(k + 1, k, ld)] = 0.0;
            return 0;
        }
        double avg = 0.5 * (H[IX(k, k, ld)] + H[IX(k + 1, k + 1, ld)]);
        H[IX(k, k, ld)] = H[IX(k + 1, k + 1, ld)] = avg;
        if (H[IX(k, k + 1, ld)] * H[IX(k + 1, k, ld)] < 0.0) return 1;
    }
    return H[IX(k + 1, k, ld)] != 0.0;
}

/* Eigenvalues of a standardized block at k of size 1 or 2. */
static void block_eigs(const double *H, long ld, int k, int sz, double *re, double *im)
{
    if (sz == 1) {
        re[0] = H[IX(k, k, ld)];
        im[0] = 0.0;
        return;
    }
    double a = H[IX(k, k, ld)], b = H[IX(k, k + 1, ld)];
    double c = H[IX(k + 1, k, ld)], d = H[IX(k + 1, k + 1, ld)];
    if (c == 0.0) {
        re[0] = a; im[0] = 0; re[1] = d; im[1] = 0;
        return;
    }
    double w = (g_mut == 5) ? sqrt(fabs(b)) : sqrt(fabs(b)) * sqrt(fabs(c));
    re[0] = re[1] = 0.5 * (a + d);
    im[0] = w;
    im[1] = -w;
}

/* Eigenvalues of an arbitrary real 2x2 (used for shifts). */
static void eig2(double a, double b, double c, double d, double *r1, double *i1, double *r2, double *i2)
{
    double p = 0.5 * (a - d);
    double sc = dmax(fabs(p), dmax(fabs(b), fabs(c)));
    if (sc == 0.0) {
        *r1 = a; *r2 = d; *i1 = *i2 = 0;
        return;
    }
    double disc = (p / sc) * (p / sc) + (b / sc) * (c / sc);
    double mid = 0.5 * (a + d);
    if (disc >= 0.0) {
        double r = sc * sqrt(disc);
        *r1 = mid + r;
        *r2 = mid - r;
        *i1 = *i2 = 0.0;
    } else {
        double w = sc * sqrt(-disc);
        *r1 = *r2 = mid;
        *i1 = w;
        *i2 = -w;
    }
}

/* ------------------------------------------------------------------------- */
/* Deflation tests (Sec. 5.6, item 1)                                          */
/* ------------------------------------------------------------------------- */

/* Vigilant test of the subdiagonal entry H[k,k-1] inside the block [lo,hi].
   LAPACK-style (Sec. 5.6, item 1; reading): the paper only says the vigilant
   check mirrors LAPACK 3.9.0, whose documented test is the Ahues-Tisseur
   criterion (LAWN 122): first |h21| <= u(|h11|+|h22|) (neighbours if that
   sum is 0), then |h21||h12| <= u |h22| |h11-h22| in an overflow-safe form,
   floor smlnum.  Norm-stable and fixed conditions (items 2 and 3): the entry
   itself against the absolute threshold. */
static int negligible(const double *H, long ld, int k, int lo, int hi, const oparams *P)
{
    double h21 = fabs(H[IX(k, k - 1, ld)]);
    if (P->defl_mode != 0) return h21 <= P->dthr;
    double smlnum = P->smlnum;
    if (h21 <= smlnum) return 1;
    double h11 = H[IX(k - 1, k - 1, ld)], h22 = H[IX(k, k, ld)];
    double tst = fabs(h11) + fabs(h22);
    if (tst == 0.0) {
        if (k - 2 >= lo) tst += fabs(H[IX(k - 1, k - 2, ld)]);
        if (k + 1 <= hi) tst += fabs(H[IX(k + 1, k, ld)]);
    }
    if (h21 > U * tst) return 0;
    double h12 = fabs(H[IX(k - 1, k, ld)]);
    double ab = dmax(h21, h12), ba = dmin(h21, h12);
    double aa = dmax(fabs(h22), fabs(h11 - h22)), bb = dmin(fabs(h22), fabs(h11 - h22));
    double s = aa + ab;
    return ba * (ab / s) <= dmax(smlnum, U * (bb * (aa / s)));
}

/* ------------------------------------------------------------------------- */
/* Multishift sweep: tightly coupled bulge chain (Sec. 2.3)                    */
/* ------------------------------------------------------------------------- */

/* First column of (H - s1 I)(H - s2 I) restricted to rows ktop..ktop+2,
   divided by a positive scale; s1, s2 are a conjugate pair or two reals. */
static void shift_column(const double *H, long ld, int ktop, int kbot, double re1, double im1,
                         double re2, double im2, double *x)
{
    double h11 = H[IX(ktop, ktop, ld)], h21 = H[IX(ktop + 1, ktop, ld)];
    double h12 = H[IX(ktop, ktop + 1, ld)], h22 = H[IX(ktop + 1, ktop + 1, ld)];
    double h32 = (ktop + 2 <= kbot) ? H[IX(ktop + 2, ktop + 1, ld)] : 0.0;
    double s = fabs(h11 - re2) + fabs(im2) + fabs(h21);
    if (s == 0.0) {
        x[0] = x[1] = x[2] = 0.0;
        return;
    }
    double h21s = h21 / s;
    x[0] = (h11 - re1) * ((h11 - re2) / s) - im1 * (im2 / s) + (g_mut == 1 ? 0.0 : h12 * h21s);
    x[1] = h21s * (h11 + h22 - re1 - re2);
    x[2] = h21s * h32;
}

/* Chase nb = nshifts/2 bulges through [ktop,kbot] of the n x n matrix H.
   Bulge j enters at step 3j (when bulge j-1 has moved three rows) and every
   step moves each bulge one row, the lowest bulge first.  Each reflector is
   applied at once to the full rows and columns of H and to Q.
   Vigilant deflation (Sec. 3.2, 'push bulges': the tasks of the last set of
   tightly coupled bulges scan the subdiagonal): a subdiagonal entry is tested
   right after the topmost bulge -- the last one of the chain -- has passed
   it, when no later reflector of the sweep reads or changes it; this equals
   one scan after the sweep. */
static long sweep(double *H, long ld, int n, double *Q, long ldq, int nq, int ktop, int kbot,
                  int nshifts, const double *sr, const double *si, int vigilant, const oparams *P)
{
    int nb = nshifts / 2;
    long nrefl = 0;
    if (nb <= 0 || kbot - ktop < 1) return 0;
    int tmax = (kbot - 2) - (ktop - 1) + 3 * (nb - 1);
    for (int t = 0; t <= tmax; ++t) {
        for (int j = 0; j < nb; ++j) {
            int k = ktop - 1 + t - 3 * j;
            if (k < ktop - 1 || k > kbot - 2) continue;
            int m = (kbot - k < 3) ? kbot - k : 3;
            double x[3], v[3], tau, beta;
            if (k == ktop - 1) {
                shift_column(H, ld, ktop, kbot, sr[2 * j], si[2 * j], sr[2 * j + 1], si[2 * j + 1], x);
            } else {
                for (int i = 0; i < m; ++i) x[i] = H[IX(k + 1 + i, k, ld)];
            }
            house(m, x, v, &tau, &beta);
            int c0;
            if (k >= ktop) {
                H[IX(k + 1, k, ld)] = beta;
                for (int i = 1; i < m; ++i) H[IX(k + 1 + i, k, ld)] = 0.0;
                c0 = k + 1;
            } else {
                c0 = ktop;
            }
            refl_left(H, ld, k + 1, m, v, tau, c0, n - 1);
            int r1 = (k + 4 < kbot) ? k + 4 : kbot;
            refl_right(H, ld, k + 1, m, v, tau, 0, r1);
            if (g_mut != 2) refl_right(Q, ldq, k + 1, m, v, tau, 0, nq - 1);
            ++nrefl;
            if (vigilant && j == nb - 1 && k >= ktop && H[IX(k + 1, k, ld)] != 0.0 &&
                negligible(H, ld, k + 1, ktop, kbot, P))
                H[IX(k + 1, k, ld)] = 0.0;
        }
    }
    return nrefl;
}

int hqr_oracle_sweep(double *H, double *Q, int64_t n, int64_t ld, int64_t ktop, int64_t kbot,
                     int nshifts, const double *sr, const double *si, int vigilant)
{
    if (n < 0) return -3;
    if (ld < (n > 1 ? n : 1)) return -4;
    if (ktop < 0 || kbot >= n || ktop > kbot) return -5;
    if (nshifts < 0 || (nshifts & 1)) return -7;
    oparams P;
    memset(&P, 0, sizeof P);
    P.smlnum = DBL_MIN * ((double)n / U);
    sweep(H, ld, (int)n, Q, ld, (int)n, (int)ktop, (int)kbot, nshifts, sr, si, vigilant, &P);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Small-block solver: double-implicit-shift Francis QR (Sec. 2.2)            */
/* ------------------------------------------------------------------------- */

/* Reduces the active block [ilo,ihi] of H (n x n) to standardized real Schur
   form.  Rows/columns outside the block are updated as well (full T).
   Returns 0, or 1 + (row index) of the block that failed to converge. */
static int qr_small(double *H, long ld, int n, double *Q, long ldq, int nq, int ilo, int ihi,
                    const oparams *P)
{
    long itmax = 30L * (long)((ihi - ilo + 1) > 10 ? (ihi - ilo + 1) : 10);
    long total = 0;
    int i = ihi;
    if (P->stats) P->stats[4]++;
    while (i >= ilo) {
        int its = 0, l = ilo;
        for (;;) {
            for (l = i; l > ilo; --l) {
                if (H[IX(l, l - 1, ld)] == 0.0) break;
                if (negligible(H, ld, l, ilo, i, P)) {
                    H[IX(l, l - 1, ld)] = 0.0;
                    break;
                }
            }
            if (l >= i - 1) break;
            if (total >= itmax) return i + 1;
            double a, b, c, d;
            if (its == 10) { /* Reading: EISPACK-style exceptional shifts */
                double ss = fabs(H[IX(l + 1, l, ld)]) + fabs(H[IX(l + 2, l + 1, ld)]);
                a = 0.75 * ss + H[IX(l, l, ld)];
                b = -0.4375 * ss;
                c = ss;
                d = a;
            } else if (its == 20) {
                double ss = fabs(H[IX(i, i - 1, ld)]) + fabs(H[IX(i - 1, i - 2, ld)]);
                a = 0.75 * ss + H[IX(i, i, ld)];
                b = -0.4375 * ss;
                c = ss;
                d = a;
            } else {
                a = H[IX(i - 1, i - 1, ld)];
                b = H[IX(i - 1, i, ld)];
                c = H[IX(i, i - 1, ld)];
                d = H[IX(i, i, ld)];
            }
            double sr[2], si[2];
            eig2(a, b, c, d, &sr[0], &si[0], &sr[1], &si[1]);
            if (si[0] == 0.0) { /* two real shifts: use the one nearer h_ii twice */
                double hii = H[IX(i, i, ld)];
                double pick = (fabs(sr[0] - hii) <= fabs(sr[1] - hii)) ? sr[0] : sr[1];
                sr[0] = sr[1] = pick;
            }
            long nr = sweep(H, ld, n, Q, ldq, nq, l, i, 2, sr, si, 0, P);
            if (P->stats) P->stats[5] += nr;
            ++its;
            ++total;
        }
        if (l == i) {
            i -= 1;
        } else { /* l == i-1 : 2x2 block */
            standardize_at(H, ld, n, Q, ldq, nq, i - 1);
            i -= 2;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Bai-Demmel swap of adjacent diagonal blocks (Sec. 2.5, step 2)             */
/* ------------------------------------------------------------------------- */

/* Solve K y = r (m <= 4) by Gaussian elimination with complete pivoting;
   tiny pivots are replaced by smin. */
static void solve_cp(int m, double *K, double *r, double *y, double smin)
{
    int perm_c[4];
    for (int i = 0; i < m; ++i) perm_c[i] = i;
    for (int k = 0; k < m; ++k) {
        int pr = k, pc = k;
        double best = -1;
        for (int i = k; i < m; ++i)
            for (int j = k; j < m; ++j)
                if (fabs(K[i + 4 * j]) > best) {
                    best = fabs(K[i + 4 * j]);
                    pr = i;
                    pc = j;
                }
        if (pr != k) {
            for (int j = 0; j < m; ++j) {
                double t = K[k + 4 * j];
                K[k + 4 * j] = K[pr + 4 * j];
                K[pr + 4 * j] = t;
            }
            double t = r[k];
            r[k] = r[pr];
            r[pr] = t;
        }
        if (pc != k) {
            for (int i = 0; i < m; ++i) {
                double t = K[i + 4 * k];
                K[i + 4 * k] = K[i + 4 * pc];
                K[i + 4 * pc] = t;
            }
            int t = perm_c[k];
            perm_c[k] = perm_c[pc];
            perm_c[pc] = t;
        }
        if (fabs(K[k + 4 * k]) < smin) K[k + 4 * k] = (K[k + 4 * k] >= 0) ? smin : -smin;
        for (int i = k + 1; i < m; ++i) {
            double f = K[i + 4 * k] / K[k + 4 * k];
            for (int j = k; j < m; ++j) K[i + 4 * j] -= f * K[k + 4 * j];
            r[i] -= f * r[k];
        }
    }
    double z[4];
    for (int k = m - 1; k >= 0; --k) {
        double s = r[k];
        for (int j = k + 1; j < m; ++j) s -= K[k + 4 * j] * z[j];
        z[k] = s / K[k + 4 * k];
    }
    for (int k = 0; k < m; ++k) y[perm_c[k]] = z[k];
}

/* Swap block A11 (p x p at row j) with the following block A22 (q x q).
   T is nt x nt quasi-triangular; V (nv rows) accumulates.  Returns 0 or 1 (rejected). */
static int swap_blocks(double *T, long ld, int nt, double *V, long ldv, int nv, int j, int p, int q,
                       double smlnum)
{
    int m = p + q;
    if (g_force_reject) return 1;
    if (p == 1 && q == 1) {
        double t11 = T[IX(j, j, ld)], t12 = T[IX(j, j + 1, ld)], t22 = T[IX(j + 1, j + 1, ld)];
        double r = hypot(t12, t22 - t11);
        if (r == 0.0) return 0; /* equal eigenvalues, nothing to move */
        double cs = t12 / r, sn = (t22 - t11) / r; /* G e1 is the eigenvector of t22 */
        rot_left(T, ld, j, cs, sn, j, nt - 1);
        if (g_mut != 4) rot_right(T, ld, j, cs, sn, 0, j + 1);
        if (g_mut != 2) rot_right(V, ldv, j, cs, sn, 0, nv - 1);
        T[IX(j + 1, j, ld)] = 0.0;
        T[IX(j, j, ld)] = t22;
        T[IX(j + 1, j + 1, ld)] = t11;
        return 0;
    }
    double D[16], dnorm = 0;
    for (int c = 0; c < m; ++c)
        for (int r = 0; r < m; ++r) {
            D[r + 4 * c] = T[IX(j + r, j + c, ld)];
            dnorm = dmax(dnorm, fabs(D[r + 4 * c]));
        }
    double thresh = dmax(10.0 * U * ((g_mut == 11) ? 1.0 : dnorm), smlnum);
    /* Sylvester equation A11 X - X A22 = A12 (p x q) through its Kronecker form */
    int pq = p * q;
    double K[16] = {0}, rhs[4], X[4];
    double kmax = 0;
    for (int c = 0; c < q; ++c)
        for (int r = 0; r < p; ++r) {
            int row = r + p * c;
            rhs[row] = D[r + 4 * (p + c)];
            for (int c2 = 0; c2 < q; ++c2)
                for (int r2 = 0; r2 < p; ++r2) {
                    int col = r2 + p * c2;
                    double v = 0;
                    if (c == c2) v += D[r + 4 * r2];
                    if (r == r2) v -= D[(p + c2) + 4 * (p + c)];
                    K[row + 4 * col] = v;
                    kmax = dmax(kmax, fabs(v));
                }
        }
    solve_cp(pq, K, rhs, X, dmax(U * kmax, smlnum));
    /* M = [-X ; I_q] (m x q);  QR by q Householder reflectors -> Qs (m x m) */
    double M[16] = {0}, Qs[16] = {0};
    for (int c = 0; c < q; ++c) {
        for (int r = 0; r < p; ++r) M[r + 4 * c] = -X[r + p * c];
        M[(p + c) + 4 * c] = 1.0;
    }
    for (int i = 0; i < m; ++i) Qs[i + 4 * i] = 1.0;
    for (int c = 0; c < q; ++c) {
        double x[4], v[4], tau, beta;
        int len = m - c;
        for (int r = 0; r < len; ++r) x[r] = M[(c + r) + 4 * c];
        house(len, x, v, &tau, &beta);
        refl_left(M, 4, c, len, v, tau, c, q - 1);
        refl_right(Qs, 4, c, len, v, tau, 0, m - 1); /* Qs <- Qs P_c */
    }
    /* D' = Qs^T D Qs */
    double T1[16], Dn[16];
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
            double s = 0;
            for (int l = 0; l < m; ++l) s += D[r + 4 * l] * Qs[l + 4 * c];
            T1[r + 4 * c] = s;
        }
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
            double s = 0;
            for (int l = 0; l < m; ++l) s += Qs[l + 4 * r] * T1[l + 4 * c];
            Dn[r + 4 * c] = s;
        }
    double err1 = 0;
    for (int c = 0; c < q; ++c)
        for (int r = q; r < m; ++r) {
            err1 = dmax(err1, fabs(Dn[r + 4 * c]));
            Dn[r + 4 * c] = 0.0;
        }
    /* reconstruction test: Qs Dn Qs^T must equal D */
    double err2 = 0;
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
            double s = 0;
            for (int l = 0; l < m; ++l)
                for (int l2 = 0; l2 < m; ++l2) s += Qs[r + 4 * l] * Dn[l + 4 * l2] * Qs[c + 4 * l2];
            err2 = dmax(err2, fabs(s - D[r + 4 * c]));
        }
    if (err1 > thresh || err2 > thresh) {
        ++g_rejects;
        return 1;
    }
    double G[16];
    for (int c = 0; c < m; ++c)
        for (int r = 0; r < m; ++r) G[r + m * c] = Qs[r + 4 * c];
    if (j + m <= nt - 1) small_left(T, ld, j, m, G, j + m, nt - 1);
    if (j > 0) small_right(T, ld, j, m, G, 0, j - 1);
    if (g_mut != 2) small_right(V, ldv, j, m, G, 0, nv - 1);
    for (int c = 0; c < m; ++c)
        for (int r = 0; r < m; ++r) T[IX(j + r, j + c, ld)] = Dn[r + 4 * c];
    if (q == 2) standardize_at(T, ld, nt, V, ldv, nv, j);
    if (p == 2) standardize_at(T, ld, nt, V, ldv, nv, j + q);
    return 0;
}

int hqr_oracle_swap(double *T, double *Q, int64_t n, int64_t ld, int64_t j, int p, int q)
{
    if (n < 0) return -3;
    if (ld < (n > 1 ? n : 1)) return -4;
    if (p < 1 || p > 2) return -6;
    if (q < 1 || q > 2) return -7;
    if (j < 0 || j + p + q > n) return -5;
    double smlnum = DBL_MIN * ((double)n / U);
    return swap_blocks(T, ld, (int)n, Q, ld, (int)n, (int)j, p, q, smlnum);
}

/* size of the diagonal block that starts at k (T quasi-triangular, order nt) */
static int block_size_at(const double *T, long ld, int nt, int k)
{
    return (k + 1 < nt && T[IX(k + 1, k, ld)] != 0.0) ? 2 : 1;
}

/* Move the block starting at ifst up to row ilst by adjacent swaps.
   Returns 0, or 1 if a swap was rejected or a 2x2 block split on the way
   (the reordering then halts; T stays in valid Schur form). */
static int move_up(double *T, long ld, int nt, double *V, long ldv, int nv, int ifst, int ilst,
                   double smlnum)
{
    int here = ifst;
    int sz = block_size_at(T, ld, nt, here);
    while (here > ilst) {
        int above = (here - 2 >= 0 && T[IX(here - 1, here - 2, ld)] != 0.0) ? 2 : 1;
        int j = here - above;
        if (j < ilst) return 1; /* would split a block at the boundary */
        /* V carries the spike as its last row, so the spike moves with V */
        if (swap_blocks(T, ld, nt, V, ldv, nv, j, above, sz, smlnum)) return 1;
        here = j;
        if (sz == 2 && T[IX(here + 1, here, ld)] == 0.0) return 1; /* split */
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Driver with aggressive early deflation                                      */
/* ------------------------------------------------------------------------- */

static int schur_driver(double *H, long ld, int n, double *Q, long ldq, int nq, int ilo, int ihi,
                        const oparams *P);

/* Reading of the automatic parameters: a shift count that grows with the
   block (LAPACK's documented table) and an AED window equal to ns for
   blocks up to 500, 3ns/2 above. */
static void auto_params(int nh, int *ns, int *nw)
{
    int s;
    if (nh < 30) s = 2;
    else if (nh < 60) s = 4;
    else if (nh < 150) s = 10;
    else if (nh < 590) {
        int lg = (int)lround(log((double)nh) / log(2.0));
        s = nh / (lg > 0 ? lg : 1);
        if (s < 10) s = 10;
    } else if (nh < 3000) s = 64;
    else if (nh < 6000) s = 128;
    else s = 256;
    s -= s & 1;
    *ns = s;
    *nw = (nh <= 500) ? s : 3 * s / 2;
}

/* One AED step on [ktop,kbot]: returns nd and the undeflated candidates. */
static int aed_step(double *H, long ld, int n, double *Q, long ldq, int nq, int ktop, int kbot,
                    int nw, double *cr, double *ci, int *ncand, const oparams *P)
{
    int kwtop = kbot - nw + 1;
    double s = (kwtop > ktop) ? H[IX(kwtop, kwtop - 1, ld)] : 0.0;
    /* copy the window; V = I.  V carries one extra row (row nw) holding the
       spike so that every transformation keeps it current. */
    long ldt = nw, ldv = nw + 1;
    double *T = calloc((size_t)nw * nw, sizeof(double));
    double *V = calloc((size_t)(nw + 1) * nw, sizeof(double));
    for (int j = 0; j < nw; ++j) {
        for (int i = 0; i <= j + 1 && i < nw; ++i) T[IX(i, j, ldt)] = H[IX(kwtop + i, kwtop + j, ld)];
        V[IX(j, j, ldv)] = 1.0;
    }
    /* sub-step 1: Schur form of the window (recursively for large windows) */
    int info;
    oparams Pin = *P;
    Pin.stats = NULL;
    if (nw <= P->nmin) {
        info = qr_small(T, ldt, nw, V, ldv, nw, 0, nw - 1, &Pin);
    } else {
        auto_params(nw, &Pin.ns, &Pin.nw);
        if (Pin.nw >= nw) Pin.nw = nw / 2;
        info = schur_driver(T, ldt, nw, V, ldv, nw, 0, nw - 1, &Pin);
    }
    /* spike = s * V(1,:) -- kept in the extra row of V */
    for (int j = 0; j < nw; ++j) V[IX(nw, j, ldv)] = s * V[IX(0, j, ldv)];
    /* Standardize every 2x2 block of the window (the recursive solver leaves
       AED-deflated blocks standardized as well; this pass is idempotent). */
    for (int k = 0; k < nw - 1;) {
        if (T[IX(k + 1, k, ldt)] != 0.0) {
            standardize_at(T, ldt, nw, V, ldv, nw + 1, k);
            k += 2;
        } else {
            k += 1;
        }
    }
    /* sub-step 2: bottom-up deflation test; failures move to the top */
    int ns = nw;
    int ilst = (info > 0) ? info : 0; /* unconverged leading part is never evaluated */
    int halted = 0;
    double thr_scale = (g_mut == 6) ? 1e8 : 1.0;
    while (ilst < ns && !halted) {
        int two = (ns >= 2 && T[IX(ns - 1, ns - 2, ldt)] != 0.0);
        if (two && ns - 2 < ilst) break; /* a 2x2 block straddling the boundary */
        int k = ns - 1;
        int defl;
        if (P->defl_mode != 0) {
            /* norm-stable / fixed conditions: every spike entry of the block
               against the absolute threshold */
            defl = fabs(V[IX(nw, k, ldv)]) <= P->dthr;
            if (two && g_mut != 12) defl = defl && fabs(V[IX(nw, k - 1, ldv)]) <= P->dthr;
        } else if (!two) {
            double foo = fabs(T[IX(k, k, ldt)]);
            defl = fabs(V[IX(nw, k, ldv)]) <= dmax(P->smlnum, thr_scale * U * foo);
        } else {
            /* h^ of the 2x2 block as printed in Sec. 5.6, item 1 */
            double d1 = fabs(T[IX(k, k, ldt)] * T[IX(k - 1, k - 1, ldt)]);
            double d2 = fabs(T[IX(k - 1, k, ldt)] * T[IX(k, k - 1, ldt)]);
            double hh;
            if (g_mut == 9) hh = d1 + d2;
            else if (g_mut == 10) hh = sqrt(d1) + fabs(T[IX(k - 1, k, ldt)]);
            else hh = sqrt(d1) + sqrt(d2);
            double sp = dmax(fabs(V[IX(nw, k, ldv)]), fabs(V[IX(nw, k - 1, ldv)]));
            defl = sp <= dmax(P->smlnum, thr_scale * U * hh);
        }
        int sz = two ? 2 : 1;
        if (defl) {
            ns -= sz;
        } else {
            int ifst = ns - sz;
            if (ifst > ilst) {
                if (move_up(T, ldt, nw, V, ldv, nw + 1, ifst, ilst, P->smlnum) != 0) halted = 1;
            }
            ilst += sz;
        }
    }
    int nd = nw - ns;
    /* candidates: eigenvalues of the undeflated blocks, in diagonal order */
    int nc = 0;
    for (int k = 0; k < ns;) {
        int sz = (k + 1 < ns && T[IX(k + 1, k, ldt)] != 0.0) ? 2 : 1;
        block_eigs(T, ldt, k, sz, cr + nc, ci + nc);
        nc += sz;
        k += sz;
    }
    *ncand = nc;
    if (nd > 0) {
        double beta = 0.0;
        if (ns >= 1) beta = V[IX(nw, 0, ldv)];
        /* sub-step 3: remove the spike and restore Hessenberg form */
        if (ns > 1 && s != 0.0) {
            double *x = malloc(sizeof(double) * ns), *v = malloc(sizeof(double) * ns), tau;
            for (int i = 0; i < ns; ++i) x[i] = V[IX(nw, i, ldv)];
            house(ns, x, v, &tau, &beta);
            refl_left(T, ldt, 0, ns, v, tau, 0, (g_mut == 8) ? ns - 1 : nw - 1);
            refl_right(T, ldt, 0, ns, v, tau, 0, ns - 1);
            refl_right(V, ldv, 0, ns, v, tau, 0, nw - 1);
            for (int c = 0; c + 2 < ns; ++c) { /* Householder Hessenberg reduction */
                int len = ns - c - 1;
                for (int i = 0; i < len; ++i) x[i] = T[IX(c + 1 + i, c, ldt)];
                double b2;
                house(len, x, v, &tau, &b2);
                T[IX(c + 1, c, ldt)] = b2;
                for (int i = 1; i < len; ++i) T[IX(c + 1 + i, c, ldt)] = 0.0;
                refl_left(T, ldt, c + 1, len, v, tau, c + 1, nw - 1);
                refl_right(T, ldt, c + 1, len, v, tau, 0, ns - 1);
                refl_right(V, ldv, c + 1, len, v, tau, 0, nw - 1);
            }
            free(x);
            free(v);
        }
        /* copy back; new subdiagonal entry from the reduced spike */
        for (int j = 0; j < nw; ++j)
            for (int i = 0; i < nw; ++i)
                H[IX(kwtop + i, kwtop + j, ld)] = (i <= j + 1) ? T[IX(i, j, ldt)] : 0.0;
        if (kwtop > ktop) H[IX(kwtop, kwtop - 1, ld)] = (ns >= 1) ? beta : 0.0;
        /* propagate V to the rest of H and to Q (plain triple loops) */
        double *row = malloc(sizeof(double) * nw);
        for (int i = 0; i < kwtop; ++i) {
            for (int c = 0; c < nw; ++c) {
                double acc = 0;
                for (int l = 0; l < nw; ++l)
                    acc += H[IX(i, kwtop + l, ld)] *
                           ((g_mut == 3) ? V[IX(c, l, ldv)] : V[IX(l, c, ldv)]);
                row[c] = acc;
            }
            for (int c = 0; c < nw; ++c) H[IX(i, kwtop + c, ld)] = row[c];
        }
        for (int jc = kbot + 1; jc < n; ++jc) {
            for (int r = 0; r < nw; ++r) {
                double acc = 0;
                for (int l = 0; l < nw; ++l) acc += V[IX(l, r, ldv)] * H[IX(kwtop + l, jc, ld)];
                row[r] = acc;
            }
            for (int r = 0; r < nw; ++r) H[IX(kwtop + r, jc, ld)] = row[r];
        }
        if (Q && g_mut != 2) {
            for (int i = 0; i < nq; ++i) {
                for (int c = 0; c < nw; ++c) {
                    double acc = 0;
                    for (int l = 0; l < nw; ++l) acc += Q[IX(i, kwtop + l, ldq)] * V[IX(l, c, ldv)];
                    row[c] = acc;
                }
                for (int c = 0; c < nw; ++c) Q[IX(i, kwtop + c, ldq)] = row[c];
            }
        }
        free(row);
    }
    free(T);
    free(V);
    return nd;
}

/* Frobenius norm of the Hessenberg part of H (overflow-safe), for the
   norm-stable deflation conditions. */
static double hess_fro(const double *H, long ld, int n)
{
    double scale = 0, ssq = 1, amax = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n && i <= j + 1; ++i) {
            double a = fabs(H[IX(i, j, ld)]);
            if (a == 0) continue;
            amax = dmax(amax, a);
            if (a > scale) {
                ssq = 1 + ssq * (scale / a) * (scale / a);
                scale = a;
            } else {
                ssq += (a / scale) * (a / scale);
            }
        }
    return (g_mut == 13) ? amax : scale * sqrt(ssq);
}

/* Deflation threshold of the conditions of Sec. 5.6: mode 1 (norm-stable)
   u ||H||_F of the whole input, computed once (an orthogonal similarity keeps
   the norm, and the recursive window solve inherits the absolute value);
   mode 2 (fixed) the caller's threshold. */
static int set_defl(oparams *P, const double *H, long ld, int n, int mode, double thold)
{
    P->defl_mode = mode;
    P->dthr = 0.0;
    if (mode == 1) P->dthr = U * hess_fro(H, ld, n);
    else if (mode == 2) {
        if (!(thold >= 0.0) || !isfinite(thold)) return -1;
        P->dthr = thold;
    } else if (mode != 0) return -1;
    return 0;
}

int hqr_oracle_aed_ex(double *H, double *Q, int64_t n, int64_t ld, int64_t ktop, int64_t kbot,
                      int nw, double *cr, double *ci, int *ncand, int defl_mode, double defl_thold)
{
    if (n < 0) return -3;
    if (ld < (n > 1 ? n : 1)) return -4;
    if (ktop < 0 || kbot >= n || ktop > kbot) return -5;
    if (nw < 1 || nw > kbot - ktop + 1) return -7;
    oparams P;
    memset(&P, 0, sizeof P);
    P.nmin = 75;
    P.nibble = 14;
    P.kexsh = 6;
    P.smlnum = DBL_MIN * ((double)n / U);
    if (set_defl(&P, H, ld, (int)n, defl_mode, defl_thold)) return -11;
    return aed_step(H, ld, (int)n, Q, ld, Q ? (int)n : 0, (int)ktop, (int)kbot, nw, cr, ci, ncand, &P);
}

int hqr_oracle_aed(double *H, double *Q, int64_t n, int64_t ld, int64_t ktop, int64_t kbot,
                   int nw, double *cr, double *ci, int *ncand)
{
    return hqr_oracle_aed_ex(H, Q, n, ld, ktop, kbot, nw, cr, ci, ncand, 0, 0.0);
}

/* Main loop over the bottom unreduced block (Sec. 2.1 outline, Sec. 2.5). */
static int schur_driver(double *H, long ld, int n, double *Q, long ldq, int nq, int ilo, int ihi,
                        const oparams *P)
{
    int kbot = ihi;
    long it = 0;
    int ndfl = 1;
    double *cr = malloc(sizeof(double) * (n + 1)), *ci = malloc(sizeof(double) * (n + 1));
    double *sr = malloc(sizeof(double) * (n + 1)), *si = malloc(sizeof(double) * (n + 1));
    int info = 0;
    while (kbot >= ilo) {
        int ktop = ilo;
        for (int k = kbot; k > ilo; --k) {
            if (H[IX(k, k - 1, ld)] == 0.0 || negligible(H, ld, k, ilo, kbot, P)) {
                H[IX(k, k - 1, ld)] = 0.0;
                ktop = k;
                break;
            }
        }
        int nh = kbot - ktop + 1;
        if (nh <= P->nmin) {
            int r = qr_small(H, ld, n, Q, ldq, nq, ktop, kbot, P);
            if (r) {
                info = r;
                break;
            }
            kbot = ktop - 1;
            ndfl = 1;
            continue;
        }
        if (++it > P->itmax) {
            info = kbot + 1;
            break;
        }
        int nw = P->nw < nh ? P->nw : nh;
        int nc = 0;
        int nd = aed_step(H, ld, n, Q, ldq, nq, ktop, kbot, nw, cr, ci, &nc, P);
        if (P->stats) {
            P->stats[0]++;
            P->stats[3] += nd;
        }
        kbot -= nd;
        ndfl = (nd > 0) ? 1 : ndfl + 1;
        if (nd > 0 && 100 * nd > P->nibble * nw) continue; /* AED again, no sweep */
        if (kbot - ktop + 1 <= P->nmin) continue;
        int nsh = 0;
        if (ndfl % P->kexsh == 0) {
            /* Reading: exceptional shifts from the trailing subdiagonal */
            int want = P->ns;
            if (want > kbot - ktop - 1) want = (kbot - ktop - 1) & ~1;
            for (int i = kbot; i >= ktop + 2 && nsh + 2 <= want; i -= 2) {
                double ss = fabs(H[IX(i, i - 1, ld)]) + fabs(H[IX(i - 1, i - 2, ld)]);
                double a = 0.75 * ss + H[IX(i, i, ld)];
                eig2(a, ss, -0.4375 * ss, a, &sr[nsh], &si[nsh], &sr[nsh + 1], &si[nsh + 1]);
                nsh += 2;
            }
        } else {
            /* Reading: the bottommost candidates, conjugate pairs kept together,
               real shifts paired in order; an odd real left over is dropped. */
            int want = P->ns < nc ? P->ns : nc;
            int start = nc - want;
            if (start > 0 && start < nc && ci[start] < 0.0) start++; /* do not split a pair */
            double rr[2];
            int nr = 0;
            for (int i = nc - 1; i >= start; --i) {
                if (ci[i] != 0.0) {
                    if (ci[i] < 0.0 && i - 1 >= start) {
                        sr[nsh] = cr[i - 1];
                        si[nsh] = ci[i - 1];
                        sr[nsh + 1] = cr[i];
                        si[nsh + 1] = ci[i];
                        nsh += 2;
                        --i;
                    }
                } else {
                    rr[nr++] = cr[i];
                    if (nr == 2) {
                        sr[nsh] = rr[0];
                        si[nsh] = 0;
                        sr[nsh + 1] = rr[1];
                        si[nsh + 1] = 0;
                        nsh += 2;
                        nr = 0;
                    }
                }
            }
            if (nsh < 2 || (nd > 0 && nsh < P->ns / 2)) continue; /* too few: AED again */
        }
        if (nsh < 2) continue;
        long nrf = sweep(H, ld, n, Q, ldq, nq, ktop, kbot, nsh, sr, si, 1, P);
        if (P->stats) {
            P->stats[1]++;
            P->stats[2] += nsh;
            P->stats[5] += nrf;
        }
    }
    free(cr);
    free(ci);
    free(sr);
    free(si);
    return info;
}

int hqr_oracle_schur_defl(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi,
                          int ns, int nw, int nmin, int64_t itmax, int64_t *stats, int defl_mode,
                          double defl_thold)
{
    if (n < 0) return -3;
    if (n == 0) return 0;
    if (H == NULL) return -1;
    if (ld < n) return -4;
    if (wr == NULL) return -5;
    if (wi == NULL) return -6;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n && i <= j + 1; ++i)
            if (!isfinite(H[IX(i, j, ld)])) return -1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j + 2; i < n; ++i) H[IX(i, j, ld)] = 0.0;
    oparams P;
    memset(&P, 0, sizeof P);
    auto_params((int)n, &P.ns, &P.nw);
    if (ns > 0) P.ns = ns & ~1;
    if (nw > 0) P.nw = nw;
    P.nmin = nmin > 0 ? nmin : 75;
    if (P.nmin < 12) P.nmin = 12;
    P.nibble = 14;
    P.kexsh = 6;
    P.itmax = itmax > 0 ? (long)itmax : 30L * (n > 10 ? (long)n : 10L);
    P.smlnum = DBL_MIN * ((double)n / U);
    if (set_defl(&P, H, ld, (int)n, defl_mode, defl_thold)) return -12;
    if (stats) memset(stats, 0, 6 * sizeof(int64_t));
    P.stats = stats;
    int info = schur_driver(H, ld, (int)n, Q, ld, Q ? (int)n : 0, 0, (int)n - 1, &P);
    /* finalize: standardize every 2x2 block, eigenvalues in diagonal order */
    int lim = info > 0 ? info : 0;
    for (int k = 0; k < n;) {
        if (k + 1 < n && H[IX(k + 1, k, ld)] != 0.0 && k >= lim) {
            standardize_at(H, ld, (int)n, Q, ld, Q ? (int)n : 0, k);
            int sz = (H[IX(k + 1, k, ld)] != 0.0) ? 2 : 1;
            block_eigs(H, ld, k, sz, wr + k, wi + k);
            k += sz;
        } else if (k + 1 < n && H[IX(k + 1, k, ld)] != 0.0) {
            wr[k] = wi[k] = 0.0; /* unconverged part */
            k += 1;
        } else {
            wr[k] = H[IX(k, k, ld)];
            wi[k] = 0.0;
            k += 1;
        }
    }
    return info;
}

int hqr_oracle_schur_ex(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi,
                        int ns, int nw, int nmin, int64_t itmax, int64_t *stats)
{
    return hqr_oracle_schur_defl(H, Q, n, ld, wr, wi, ns, nw, nmin, itmax, stats, 0, 0.0);
}

int hqr_oracle_schur(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi)
{
    return hqr_oracle_schur_ex(H, Q, n, ld, wr, wi, 0, 0, 0, 0, NULL);
}

/* ------------------------------------------------------------------------- */
/* Eigenvectors from the Schur form and the eigenvalue gradient               */
/* ------------------------------------------------------------------------- */

/* Solve (B - lam I) z = r for a 1x1 or 2x2 real block B (complex lam). */
static void blk_solve(int sz, const double *B, double complex lam, double complex *r, double smin)
{
    if (sz == 1) {
        double complex d = B[0] - lam;
        if (cabs(d) < smin) d = smin;
        r[0] = r[0] / d;
        return;
    }
    double complex a = B[0] - lam, b = B[2], c = B[1], d = B[3] - lam;
    double complex det = a * d - b * c;
    if (cabs(det) < smin) det = smin;
    double complex x0 = (d * r[0] - b * r[1]) / det;
    double complex x1 = (a * r[1] - c * r[0]) / det;
    r[0] = x0;
    r[1] = x1;
}

int hqr_oracle_eig_backward(const double *T, const double *Q, int64_t n64, int64_t ld,
                            const double *wr, const double *wi, const double *gwr,
                            const double *gwi, double *dH, int hess_mask)
{
    int n = (int)n64;
    if (n < 0) return -3;
    if (ld < n) return -4;
    double tnorm = 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) tnorm = dmax(tnorm, fabs(T[IX(i, j, ld)]));
    double smin = dmax(U * tnorm, DBL_MIN);
    /* block starts */
    int *bs = malloc(sizeof(int) * (n + 1)), *bsz = malloc(sizeof(int) * (n + 1));
    int nb = 0;
    for (int k = 0; k < n;) {
        int sz = (k + 1 < n && T[IX(k + 1, k, ld)] != 0.0) ? 2 : 1;
        bs[nb] = k;
        bsz[nb] = sz;
        ++nb;
        k += sz;
    }
    double complex *y = malloc(sizeof(double complex) * n), *z = malloc(sizeof(double complex) * n);
    double complex *X = malloc(sizeof(double complex) * (size_t)n * n);
    double complex *Y = malloc(sizeof(double complex) * (size_t)n * n);
    double complex *cf = malloc(sizeof(double complex) * n);
    for (int b = 0; b < nb; ++b) {
        int k = bs[b], sz = bsz[b];
        for (int e = 0; e < sz; ++e) {
            int idx = k + e;
            double complex lam = wr[idx] + I * wi[idx];
            for (int i = 0; i < n; ++i) y[i] = z[i] = 0;
            if (sz == 1) {
                y[k] = 1;
                z[k] = 1;
            } else {
                double bb = T[IX(k, k + 1, ld)], cc = T[IX(k + 1, k, ld)];
                double w = wi[idx];
                /* right: (B - lam) y = 0  ->  y = (1, i w / b); left: z = (1, -i w / c)
                   for the eigenvalue a + i w (w of either sign) */
                y[k] = 1;
                y[k + 1] = I * w / bb;
                z[k] = 1;
                z[k + 1] = -I * w / cc;
            }
            /* right vector: back substitution upward */
            for (int bb2 = b - 1; bb2 >= 0; --bb2) {
                int j = bs[bb2], s2 = bsz[bb2];
                double complex r[2];
                for (int e2 = 0; e2 < s2; ++e2) {
                    double complex acc = 0;
                    for (int l = j + s2; l < k + sz; ++l) acc += T[IX(j + e2, l, ld)] * y[l];
                    r[e2] = -acc;
                }
                double B[4] = {T[IX(j, j, ld)], 0, 0, 0};
                if (s2 == 2) {
                    B[1] = T[IX(j + 1, j, ld)];
                    B[2] = T[IX(j, j + 1, ld)];
                    B[3] = T[IX(j + 1, j + 1, ld)];
                }
                blk_solve(s2, B, lam, r, smin);
                for (int e2 = 0; e2 < s2; ++e2) y[j + e2] = r[e2];
            }
            /* left vector: z^H (T - lam I) = 0  <=>  (T^T - conj(lam)) z = 0, forward */
            for (int bb2 = b + 1; bb2 < nb; ++bb2) {
                int j = bs[bb2], s2 = bsz[bb2];
                double complex r[2];
                for (int e2 = 0; e2 < s2; ++e2) {
                    double complex acc = 0;
                    for (int l = k; l < j; ++l) acc += T[IX(l, j + e2, ld)] * z[l];
                    r[e2] = -acc;
                }
                double B[4] = {T[IX(j, j, ld)], 0, 0, 0}; /* transpose of the block */
                if (s2 == 2) {
                    B[1] = T[IX(j, j + 1, ld)];
                    B[2] = T[IX(j + 1, j, ld)];
                    B[3] = T[IX(j + 1, j + 1, ld)];
                }
                blk_solve(s2, B, conj(lam), r, smin);
                for (int e2 = 0; e2 < s2; ++e2) z[j + e2] = r[e2];
            }
            /* back-transform x = Q y, yl = Q z */
            for (int a = 0; a < n; ++a) {
                double complex sx = 0, sy = 0;
                for (int l = 0; l < n; ++l) {
                    double q = Q ? Q[IX(a, l, ld)] : (a == l ? 1.0 : 0.0);
                    sx += q * y[l];
                    sy += q * z[l];
                }
                X[(size_t)idx * n + a] = sx;
                Y[(size_t)idx * n + a] = sy;
            }
            double complex d = 0;
            for (int a = 0; a < n; ++a) d += conj(Y[(size_t)idx * n + a]) * X[(size_t)idx * n + a];
            double complex g = gwr[idx] + I * gwi[idx];
            cf[idx] = ((g_mut == 7) ? g : conj(g)) / d;
        }
    }
    /* dL/dH = Re( conj(Y) diag(conj(g)/(y^H x)) X^T ) */
    for (int bcol = 0; bcol < n; ++bcol)
        for (int a = 0; a < n; ++a) {
            double complex acc = 0;
            for (int i = 0; i < n; ++i)
                acc += conj(Y[(size_t)i * n + a]) * cf[i] * X[(size_t)i * n + bcol];
            dH[IX(a, bcol, ld)] = (hess_mask && a > bcol + 1) ? 0.0 : creal(acc);
        }
    free(bs);
    free(bsz);
    free(y);
    free(z);
    free(X);
    free(Y);
    free(cf);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The QZ variant (Sec. 2, remarks on the generalized case; Sec. 3.2 'push    */
/* infinities'): double implicit shift QZ on a Hessenberg-triangular pair.    */
/* Every transformation is applied to the full rows and columns of H and T.   */
/* ------------------------------------------------------------------------- */

/* Reflector P = I - tau v v^T, v[m-1] = 1, with x^T P = beta e_{m-1}^T: the
   Householder reflector of the reversed vector, reversed. */
static void house_last(int m, const double *x, double *v, double *tau, double *beta)
{
    double xr[3], vr[3];
    for (int i = 0; i < m; ++i) xr[i] = x[m - 1 - i];
    house(m, xr, vr, tau, beta);
    for (int i = 0; i < m; ++i) v[i] = vr[m - 1 - i];
}

/* Rotation zeroing the second entry of (a, b): c = a/r, s = b/r. */
static void qz_rot(double a, double b, double *c, double *s)
{
    double r = hypot(a, b);
    if (r == 0.0) {
        *c = 1.0;
        *s = 0.0;
    } else {
        *c = a / r;
        *s = b / r;
    }
}

/* rows p, p+1 of A (all columns) <- G rows, G = [[c, s], [-s, c]] */
static void qz_rows(double *A, long ld, int n, int p, double c, double s)
{
    for (int j = 0; j < n; ++j) {
        double x = A[IX(p, j, ld)], y = A[IX(p + 1, j, ld)];
        A[IX(p, j, ld)] = c * x + s * y;
        A[IX(p + 1, j, ld)] = -s * x + c * y;
    }
}

/* columns a, b of A (all rows): col a <- c col a + s col b, col b <- -s col a + c col b */
static void qz_cols(double *A, long ld, int n, int a, int b, double c, double s)
{
    if (A == NULL) return;
    for (int i = 0; i < n; ++i) {
        double x = A[IX(i, a, ld)], y = A[IX(i, b, ld)];
        A[IX(i, a, ld)] = c * x + s * y;
        A[IX(i, b, ld)] = -s * x + c * y;
    }
}

/* Left rotation on rows p, p+1 of H and T, accumulated into Q (Q <- Q G^T). */
static void qz_left(double *H, double *T, double *Q, long ld, int n, int p, double c, double s)
{
    qz_rows(H, ld, n, p, c, s);
    if (g_mut != 22) qz_rows(T, ld, n, p, c, s);
    qz_cols(Q, ld, n, p, p + 1, c, s);
}

/* Right rotation on columns a, b of H, T and Z. */
static void qz_right(double *H, double *T, double *Z, long ld, int n, int a, int b, double c, double s)
{
    qz_cols(H, ld, n, a, b, c, s);
    qz_cols(T, ld, n, a, b, c, s);
    qz_cols(Z, ld, n, a, b, c, s);
}

/* An infinite eigenvalue at T[j,j] = 0 inside the block [l, i] is chased to
   the top of the block and deflated there (the 'push infinities' task chases
   them up the diagonal with rotations).  Each step moves the zero from j to
   j-1 with a right rotation on columns (j-1, j) that zeroes T[j-1,j-1], and
   removes the fill H[j+1,j-1] this leaves with a left rotation on rows
   (j, j+1).  At the top, a left rotation on rows (l, l+1) zeroes H[l+1,l]:
   the 1x1 block l (with T[l,l] = 0) decouples. */
static void qz_push_up(double *H, double *T, double *Q, double *Z, long ld, int n, int l, int i, int j)
{
    double c, s;
    for (int jc = j; jc > l; --jc) {
        qz_rot(T[IX(jc - 1, jc, ld)], T[IX(jc - 1, jc - 1, ld)], &c, &s);
        qz_right(H, T, Z, ld, n, jc, jc - 1, c, s);
        T[IX(jc - 1, jc - 1, ld)] = 0.0;
        if (jc + 1 <= i) {
            qz_rot(H[IX(jc, jc - 1, ld)], H[IX(jc + 1, jc - 1, ld)], &c, &s);
            qz_left(H, T, Q, ld, n, jc, c, s);
            H[IX(jc + 1, jc - 1, ld)] = 0.0;
        }
    }
    qz_rot(H[IX(l, l, ld)], H[IX(l + 1, l, ld)], &c, &s);
    qz_left(H, T, Q, ld, n, l, c, s);
    H[IX(l + 1, l, ld)] = 0.0;
}

/* Generalized eigenvalues of the 2x2 pair (A, B) at rows/columns k, k+1
   (B upper triangular, nonsingular): the eigenvalues of A B^{-1}. */
static void qz_eig2(const double *H, const double *T, long ld, int k, double *r1, double *i1, double *r2,
                    double *i2)
{
    double a11 = H[IX(k, k, ld)], a12 = H[IX(k, k + 1, ld)], a21 = H[IX(k + 1, k, ld)], a22 = H[IX(k + 1, k + 1, ld)];
    double b11 = T[IX(k, k, ld)], b12 = T[IX(k, k + 1, ld)], b22 = T[IX(k + 1, k + 1, ld)];
    /* B^{-1} = [[1/b11, -b12/(b11 b22)], [0, 1/b22]] */
    double m11 = a11 / b11, m21 = a21 / b11;
    double m12 = (a12 - m11 * b12) / b22, m22 = (a22 - m21 * b12) / b22;
    eig2(m11, m12, m21, m22, r1, i1, r2, i2);
}

/* A 2x2 block at k, k+1 whose pair has real eigenvalues is split: a right
   rotation whose first column spans the null space of A - lambda B, then a
   left rotation making the first column of B Z triangular; both pairs'
   (k+1, k) entries become zero. */
static void qz_split2(double *H, double *T, double *Q, double *Z, long ld, int n, int k, double lam)
{
    double m11 = H[IX(k, k, ld)] - lam * T[IX(k, k, ld)], m12 = H[IX(k, k + 1, ld)] - lam * T[IX(k, k + 1, ld)];
    double m21 = H[IX(k + 1, k, ld)], m22 = H[IX(k + 1, k + 1, ld)] - lam * T[IX(k + 1, k + 1, ld)];
    /* null vector (z1, z2) of M from its larger row */
    double z1, z2;
    if (hypot(m11, m12) >= hypot(m21, m22)) {
        z1 = -m12;
        z2 = m11;
    } else {
        z1 = -m22;
        z2 = m21;
    }
    double c, s;
    qz_rot(z1, z2, &c, &s);
    if (c == 1.0 && s == 0.0 && z1 == 0.0 && z2 == 0.0) return;
    /* columns (k, k+1): new col k = c col k + s col k+1 (first column = (c, s) ~ (z1, z2)) */
    qz_right(H, T, Z, ld, n, k, k + 1, c, s);
    qz_rot(T[IX(k, k, ld)], T[IX(k + 1, k, ld)], &c, &s);
    qz_left(H, T, Q, ld, n, k, c, s);
    H[IX(k + 1, k, ld)] = 0.0;
    T[IX(k + 1, k, ld)] = 0.0;
}

/* One double-shift QZ sweep over the block [l, i] (i - l >= 2) with the
   shifts (re1 + i im1, re2 + i im2) (a conjugate pair or two reals).  The
   first column of (H T^{-1} - s1)(H T^{-1} - s2) on rows l..l+2 gives the
   reflector that introduces the bulge; at each position k a 3x3 reflector
   from the left (rows k+1..k+3) moves the bulge of H down, and two
   reflectors from the right restore T: one from row k+3 of T (columns
   k+1..k+3 mapped to the last column) and one from row k+2 (columns k+1..k+2). */
static void qz_sweep(double *H, double *T, double *Q, double *Z, long ld, int n, int l, int i, double re1,
                     double im1, double re2, double im2)
{
    const double sum = re1 + re2, prod = (g_mut == 23) ? -(re1 * re2 - im1 * im2) : re1 * re2 - im1 * im2;
    const double t11 = T[IX(l, l, ld)], t12 = T[IX(l, l + 1, ld)], t22 = T[IX(l + 1, l + 1, ld)];
    const double h11 = H[IX(l, l, ld)], h21 = H[IX(l + 1, l, ld)], h12 = H[IX(l, l + 1, ld)];
    const double h22 = H[IX(l + 1, l + 1, ld)], h32 = H[IX(l + 2, l + 1, ld)];
    /* N e1 with N = H T^{-1}, then y = T^{-1} N e1 and N^2 e1 = H y */
    const double ne0 = h11 / t11, ne1 = h21 / t11;
    const double y2 = ne1 / t22, y1 = (ne0 - t12 * y2) / t11;
    double x[3];
    x[0] = h11 * y1 + h12 * y2 - sum * ne0 + prod;
    x[1] = h21 * y1 + h22 * y2 - sum * ne1;
    x[2] = h32 * y2;
    for (int k = l - 1; k <= i - 2; ++k) {
        const int m = (i - k < 3) ? i - k : 3;
        double v[3], tau, beta;
        if (k >= l) {
            for (int r = 0; r < m; ++r) x[r] = H[IX(k + 1 + r, k, ld)];
        }
        house(m, x, v, &tau, &beta);
        refl_left(H, ld, k + 1, m, v, tau, 0, n - 1);
        refl_left(T, ld, k + 1, m, v, tau, 0, n - 1);
        if (Q) refl_right(Q, ld, k + 1, m, v, tau, 0, n - 1);
        if (k >= l) {
            H[IX(k + 1, k, ld)] = beta;
            for (int r = 1; r < m; ++r) H[IX(k + 1 + r, k, ld)] = 0.0;
        }
        /* restore T: row k+m first (columns k+1..k+m onto the last), then row k+m-1 */
        double w[3], tw, bw;
        for (int r = 0; r < m; ++r) w[r] = T[IX(k + m, k + 1 + r, ld)];
        house_last(m, w, v, &tw, &bw);
        refl_right(H, ld, k + 1, m, v, tw, 0, n - 1);
        refl_right(T, ld, k + 1, m, v, tw, 0, n - 1);
        if (Z) refl_right(Z, ld, k + 1, m, v, tw, 0, n - 1);
        for (int r = 0; r < m - 1; ++r) T[IX(k + m, k + 1 + r, ld)] = 0.0;
        if (m == 3) {
            for (int r = 0; r < 2; ++r) w[r] = T[IX(k + 2, k + 1 + r, ld)];
            house_last(2, w, v, &tw, &bw);
            refl_right(H, ld, k + 1, 2, v, tw, 0, n - 1);
            refl_right(T, ld, k + 1, 2, v, tw, 0, n - 1);
            if (Z && g_mut != 21) refl_right(Z, ld, k + 1, 2, v, tw, 0, n - 1);
            T[IX(k + 2, k + 1, ld)] = 0.0;
        }
    }
}

int hqr_oracle_qz(double *H, double *T, double *Q, double *Z, int64_t n64, int64_t ld64, double *alphar,
                  double *alphai, double *beta, int64_t itmax)
{
    const int n = (int)n64;
    const long ld = (long)ld64;
    if (n < 0 || ld < (n > 1 ? n : 1) || !H || !T) return -1;
    if (n == 0) return 0;
    if (itmax <= 0) itmax = 30 * (int64_t)(n > 10 ? n : 10);
    double tn = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) tn = hypot(tn, T[IX(i, j, ld)]);
    /* Reading: the paper adopts LAPACK's convention |t_kk| <= u ||T||_F for
       an infinite eigenvalue; the subdiagonal test of H is the conventional
       |h_{k,k-1}| <= u (|h_{k-1,k-1}| + |h_kk|) with floor nu n / u. */
    const double btol = U * tn, smlnum = DBL_MIN * ((double)n / U);
    for (int k = 0; k < n; ++k)
        if (fabs(T[IX(k, k, ld)]) <= btol) T[IX(k, k, ld)] = 0.0;
    int i = n - 1, its = 0;
    int64_t it = 0;
    while (i >= 0) {
        int l = i;
        while (l > 0) {
            double h = fabs(H[IX(l, l - 1, ld)]);
            double tst = fabs(H[IX(l - 1, l - 1, ld)]) + fabs(H[IX(l, l, ld)]);
            if (h <= dmax(smlnum, U * tst)) {
                H[IX(l, l - 1, ld)] = 0.0;
                break;
            }
            --l;
        }
        int kz = -1;
        for (int k = l; k <= i; ++k)
            if (T[IX(k, k, ld)] == 0.0) {
                kz = k;
                break;
            }
        if (kz >= 0 && l < i) {
            qz_push_up(H, T, Q, Z, ld, n, l, i, kz);
            /* the rotations change diagonal entries of T: re-apply the threshold below l */
            for (int k = l + 1; k <= i; ++k)
                if (fabs(T[IX(k, k, ld)]) <= btol) T[IX(k, k, ld)] = 0.0;
            its = 0;
            continue;
        }
        if (l == i) {
            double a = H[IX(i, i, ld)], b = T[IX(i, i, ld)];
            if (b < 0.0) {
                a = -a;
                b = -b;
            }
            alphar[i] = a;
            alphai[i] = 0.0;
            beta[i] = b;
            --i;
            its = 0;
            continue;
        }
        if (l == i - 1) {
            double r1, i1, r2, i2;
            qz_eig2(H, T, ld, i - 1, &r1, &i1, &r2, &i2);
            if (i1 == 0.0) {
                qz_split2(H, T, Q, Z, ld, n, i - 1, r1);
                continue; /* two 1x1 blocks now */
            }
            alphar[i - 1] = r1;
            alphai[i - 1] = fabs(i1);
            beta[i - 1] = 1.0;
            alphar[i] = r2;
            alphai[i] = -fabs(i1);
            beta[i] = 1.0;
            i -= 2;
            its = 0;
            continue;
        }
        if (it >= itmax) return i + 1;
        double r1, i1, r2, i2;
        if (its == 10 || its == 20) {
            /* exceptional shifts: a real double shift off the bottom entries */
            double ss = fabs(H[IX(i, i - 1, ld)] / T[IX(i - 1, i - 1, ld)]) +
                        fabs(H[IX(i - 1, i - 2, ld)] / T[IX(i - 2, i - 2, ld)]);
            r1 = r2 = H[IX(i, i, ld)] / T[IX(i, i, ld)] + 0.75 * ss;
            i1 = i2 = 0.0;
        } else {
            qz_eig2(H, T, ld, i - 1, &r1, &i1, &r2, &i2);
            if (i1 == 0.0) {
                /* two real shifts: both at the one closer to the bottom ratio */
                double tb = H[IX(i, i, ld)] / T[IX(i, i, ld)];
                double pick = (fabs(r1 - tb) <= fabs(r2 - tb)) ? r1 : r2;
                r1 = r2 = pick;
            }
        }
        qz_sweep(H, T, Q, Z, ld, n, l, i, r1, i1, r2, i2);
        for (int k = l; k <= i; ++k)
            if (fabs(T[IX(k, k, ld)]) <= btol) T[IX(k, k, ld)] = 0.0;
        ++it;
        ++its;
    }
    return 0;
}
