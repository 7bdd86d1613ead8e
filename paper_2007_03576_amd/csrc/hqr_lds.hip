// LDS-resident one-workgroup kernels of libhqr (gfx950).
//
// A workgroup of 256 threads keeps a matrix of order <= 96 and its accumulated
// orthogonal factor in LDS and performs the sequential parts of the multishift
// QR algorithm with AED (Myllykoski, ACM TOMS 48(1), 2021):
//   * the small-block solver (task 'small Schur', Sec. 3.2 "Task types"): Francis double-shift
//     iterations (Sec. 2.2), each sweep a bulge chased through the block;
//   * the AED step for windows that fit LDS (task 'small AED', Sec. 3.2 and
//     Sec. 2.5): Schur form of the window, bottom-up spike test with the
//     conditions of Sec. 5.6 ("Comment regarding the deflation conditions and
//     the accuracy"), reordering of failed candidates by
//     Bai-Demmel swaps, spike removal and Hessenberg restoration;
//   * the bulge-chasing windows of a multishift sweep (task 'push bulges',
//     Sec. 3.2 and Sec. 2.3): a chain of tightly coupled bulges chased inside
//     a diagonal window while the reflectors accumulate into U.
// Every step of a chain moves all bulges by one row in three barrier-separated
// phases: generate the reflectors (one thread per bulge), apply them from the
// left (threads over columns), then from the right and into the accumulated
// factor (threads over rows).  Reflectors of one step act on disjoint index
// triples, so the phases are race free.
#include "hqr_common.h"
#include <algorithm>
#include <cfloat>
#include <climits>
#include <mutex>
#include <utility>
#include <vector>

namespace hqr {

constexpr double kU = 2.220446049250313080847e-16; // unit roundoff 2^-52

// Small per-workgroup state used by every solver piece.
// State of the pipelined deflation check and reordering of an AED window.
constexpr int MV = 32; // most block moves in flight
struct ReorderState {
    double G[MV * 16];               // exchange of each lane of the current phase (order m, column major)
    int pos[2][MV], sz[MV], dst[MV]; // moves in flight (ring indexed by move id), position double buffered
    int sj[MV], sm[MV];              // exchange of each lane: first row and order (0: none)
    int roff[MV + 1], coff[MV + 1];  // prefix sums of the row and column work items per lane
    int xj[MV], xk[MV], xr[MV];      // exchange of each lane: first row, kind, outcome
    int head, tail, ns, ilst, halt, chk_done, done, rtot, ctot;
};

struct SmemCore {
    double bv1[GMAX], bv2[GMAX], btau[GMAX];
    int bk[GMAX], bm[GMAX], bc0[GMAX];
    double sr[2 * GMAX], si[2 * GMAX];
    double red[NT / 64];
    double sc[8];
    int ic[8];
    double shb[16 * 16]; // trailing block whose eigenvalues become the shifts of a multishift sweep
    double flops;        // algorithmic flops of the reflector applications (thread 0 counts)
    int nphase, nbstep, nswap, nrphase; // event counters (thread 0 counts)
    ReorderState ro;
};

// LDS-resident matrix and accumulated factor for orders <= MMAX.
struct Smem : SmemCore {
    double A[MMAX * LDM];
    double Z[LDM * LDM];          // one spare row for a carried spike
    double vec[LDM];
    unsigned char vflag[WMAX];
};

// ---------------------------------------------------------------------------
// scalar helpers (one thread)

__device__ inline void house3(int m, double x0, double x1, double x2, double &v1, double &v2,
                              double &tau, double &beta)
{
    double t1 = (m > 1) ? x1 : 0.0, t2 = (m > 2) ? x2 : 0.0;
    double tail = hypot(t1, t2);
    if (tail == 0.0) {
        tau = 0.0;
        beta = x0;
        v1 = v2 = 0.0;
        return;
    }
    double nrm = hypot(x0, tail);
    double b = (x0 >= 0.0) ? -nrm : nrm;
    tau = (b - x0) / b;
    double r = 1.0 / (x0 - b);
    v1 = t1 * r;
    v2 = t2 * r;
    beta = b;
}

// house3 with one square root and no scaling when every entry lies well
// inside the range where squaring neither overflows nor underflows (the
// usual case); otherwise the scaled form above.
__device__ inline void house3f(int m, double x0, double x1, double x2, double &v1, double &v2, double &tau,
                               double &beta)
{
    const double t1 = (m > 1) ? x1 : 0.0, t2 = (m > 2) ? x2 : 0.0;
    if (t1 == 0.0 && t2 == 0.0) {
        tau = 0.0;
        beta = x0;
        v1 = v2 = 0.0;
        return;
    }
    const double amax = fmax(fabs(x0), fmax(fabs(t1), fabs(t2)));
    if (!(amax > 0x1p-450 && amax < 0x1p+450)) {
        house3(m, x0, x1, x2, v1, v2, tau, beta);
        return;
    }
    const double nrm = sqrt(fma(x0, x0, fma(t1, t1, t2 * t2)));
    const double b = (x0 >= 0.0) ? -nrm : nrm;
    const double d = x0 - b; // |d| = |x0| + nrm
    const double rd = 1.0 / d;
    tau = -d / b;
    v1 = t1 * rd;
    v2 = t2 * rd;
    beta = b;
}

// Vigilant (subdiagonal) deflation test of A[k,k-1] inside [lo,hi].
// LAPACK-style conditions: the Ahues-Tisseur criterion; norm-stable and fixed
// conditions: |A[k,k-1]| <= thr (Sec. 5.6, items 2 and 3).  LD is int for LDS
// and int64_t for global memory.
template <typename LD>
__device__ inline bool small_sub(const double *A, LD lda, int k, int lo, int hi, const Defl &dfl)
{
    double h21 = fabs(A[k + (k - 1) * lda]);
    if (dfl.thr >= 0.0) return h21 <= dfl.thr;
    if (h21 <= dfl.smlnum) return true;
    double h11 = A[(k - 1) + (k - 1) * lda], h22 = A[k + k * lda];
    double tst = fabs(h11) + fabs(h22);
    if (tst == 0.0) {
        if (k - 2 >= lo) tst += fabs(A[(k - 1) + (k - 2) * lda]);
        if (k + 1 <= hi) tst += fabs(A[(k + 1) + k * lda]);
    }
    if (h21 > kU * tst) return false;
    double h12 = fabs(A[(k - 1) + k * lda]);
    double ab = fmax(h21, h12), ba = fmin(h21, h12);
    double d = fabs(h11 - h22);
    double aa = fmax(fabs(h22), d), bb = fmin(fabs(h22), d);
    double s = aa + ab;
    return ba * (ab / s) <= fmax(dfl.smlnum, kU * (bb * (aa / s)));
}

// Rotation G = [[cs,-sn],[sn,cs]] that standardizes [[a,b],[c,d]] (G^T B G):
// real eigenvalues -> upper triangular (mode 1); complex -> equal diagonal (mode 2).
__device__ inline int std_rot(double a, double b, double c, double d, double &cs, double &sn)
{
    cs = 1.0;
    sn = 0.0;
    if (c == 0.0) return 0;
    if (b == 0.0) {
        cs = 0.0;
        sn = 1.0;
        return 1;
    }
    double p = 0.5 * (a - d);
    double scl = fmax(fabs(p), fmax(fabs(b), fabs(c)));
    double ps = p / scl;
    double disc = ps * ps + (b / scl) * (c / scl);
    if (disc >= 0.0) {
        double z = p + copysign(scl * sqrt(disc), p);
        double r = hypot(z, c);
        cs = z / r;
        sn = c / r;
        return 1;
    }
    if (a == d) return 0;
    double al = b + c, be = a - d;
    double r = hypot(al, be);
    double sg = (al >= 0.0) ? 1.0 : -1.0;
    double c2 = sg * al / r, s2 = -sg * be / r;
    cs = sqrt(0.5 * (1.0 + c2));
    sn = s2 / (2.0 * cs);
    return 2;
}

__device__ inline void eig2x2(double a, double b, double c, double d, double &r1, double &i1, double &r2,
                              double &i2)
{
    double p = 0.5 * (a - d);
    double scl = fmax(fabs(p), fmax(fabs(b), fabs(c)));
    if (scl == 0.0) {
        r1 = a; r2 = d; i1 = i2 = 0.0;
        return;
    }
    double ps = p / scl;
    double disc = ps * ps + (b / scl) * (c / scl);
    double mid = 0.5 * (a + d);
    if (disc >= 0.0) {
        double r = scl * sqrt(disc);
        r1 = mid + r;
        r2 = mid - r;
        i1 = i2 = 0.0;
    } else {
        double w = scl * sqrt(-disc);
        r1 = r2 = mid;
        i1 = w;
        i2 = -w;
    }
}

// (H - s1)(H - s2) e_kt restricted to rows kt..kt+2, divided by a positive scale.
__device__ inline void shift_column(const double *A, int lda, int kt, int kb, double re1, double im1,
                                    double re2, double im2, double &x0, double &x1, double &x2)
{
    double h11 = A[kt + kt * lda], h21 = A[(kt + 1) + kt * lda];
    double h12 = A[kt + (kt + 1) * lda], h22 = A[(kt + 1) + (kt + 1) * lda];
    double h32 = (kt + 2 <= kb) ? A[(kt + 2) + (kt + 1) * lda] : 0.0;
    double s = fabs(h11 - re2) + fabs(im2) + fabs(h21);
    if (s == 0.0) {
        x0 = x1 = x2 = 0.0;
        return;
    }
    double f = h21 / s;
    x0 = f * h12 + (h11 - re1) * ((h11 - re2) / s) - im1 * (im2 / s);
    x1 = f * (h11 + h22 - re1 - re2);
    x2 = f * h32;
}

// ---------------------------------------------------------------------------
// block-level helpers (all threads call them)

__device__ inline double block_sum(SmemCore &S, double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) S.red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t += S.red[i];
    return t;
}

__device__ inline double block_max(SmemCore &S, double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) S.red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t = fmax(t, S.red[i]);
    return t;
}

// Reflector of one bulge at position k (acting on k+1..k+m, local kl = k - off):
// from the shift polynomial when the bulge is introduced (k = ktop-1), else
// from the bulge column.
__device__ inline void bulge_reflector(const SmemCore &S, const double *A, int lda, int off, int ktop, int kbot,
                                       int b, int k, int &m, double &v1, double &v2, double &tau, double &beta)
{
    m = min(3, kbot - k);
    const int kl = k - off;
    double x0, x1, x2;
    if (k == ktop - 1) {
        shift_column(A, lda, kl + 1, kbot - off, S.sr[2 * b], S.si[2 * b], S.sr[2 * b + 1], S.si[2 * b + 1], x0, x1,
                     x2);
    } else {
        x0 = A[(kl + 1) + kl * lda];
        x1 = A[(kl + 2) + kl * lda];
        x2 = (m == 3) ? A[(kl + 3) + kl * lda] : 0.0;
    }
    house3(m, x0, x1, x2, v1, v2, tau, beta);
    if (m < 3) v2 = 0.0;
}

// y <- P y for an m-vector (m = 2 or 3), P = I - tau v v^T, v = (1, v1, v2).
__device__ inline void refl3(int m, double tau, double v1, double v2, double &y0, double &y1, double &y2)
{
    double s = tau * (y0 + v1 * y1 + (m == 3 ? v2 * y2 : 0.0));
    y0 -= s;
    y1 -= s * v1;
    if (m == 3) y2 -= s * v2;
}

// 1/d from the hardware reciprocal (about 28 correct bits) and two Newton
// steps (within an ulp; measured 0.5 ulp over binades 2^-100..2^100).
__device__ inline double rcp_nr(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

// house3f for the chase: the two quotients from reciprocals (shorter
// dependency chains than correctly rounded division, same accuracy class).
__device__ inline void house3c(int m, double x0, double x1, double x2, double &v1, double &v2, double &tau,
                               double &beta)
{
    const double t1 = (m > 1) ? x1 : 0.0, t2 = (m > 2) ? x2 : 0.0;
    // fast path: squares neither overflow nor underflow (checked alongside,
    // on ss, and redone with the scaled form when they might)
    const double q = fma(t1, t1, t2 * t2);
    const double ss = fma(x0, x0, q);
    const double nrm = sqrt(ss);
    const double b = (x0 >= 0.0) ? -nrm : nrm;
    const double d = x0 - b; // |d| = |x0| + nrm
    const double rd = rcp_nr(d);
    tau = -d * rcp_nr(b);
    v1 = t1 * rd;
    v2 = t2 * rd;
    beta = b;
    if (!(ss > 0x1p-900 && ss < 0x1p+900 && q > 0x1p-900)) {
        if (t1 == 0.0 && t2 == 0.0) {
            tau = 0.0;
            beta = x0;
            v1 = v2 = 0.0;
        } else {
            house3(m, x0, x1, x2, v1, v2, tau, beta);
        }
    }
}

// 1/sqrt(s) from the hardware estimate and two Newton steps, for s well
// inside the normal range (within a few ulps).
__device__ inline double rsq_nr(double s)
{
    double r = __builtin_amdgcn_rsq(s);
    double t = s * r;
    double e = fma(-t, r, 1.0);
    r = fma(r * 0.5, e, r);
    t = s * r;
    e = fma(-t, r, 1.0);
    return fma(r * 0.5, e, r);
}

// house3c with the norm from a reciprocal square root: tau = 1 + |x0|/||x||
// needs no quotient, and the one reciprocal (of x0 - beta) gives v.  Shorter
// dependency chain than a rounded square root followed by a reciprocal.
__device__ inline void house3r(int m, double x0, double x1, double x2, double &v1, double &v2, double &tau,
                               double &beta)
{
    const double t1 = (m > 1) ? x1 : 0.0, t2 = (m > 2) ? x2 : 0.0;
    const double q = fma(t1, t1, t2 * t2);
    const double ss = fma(x0, x0, q);
    if (ss > 0x1p-900 && ss < 0x1p+900 && q > 0x1p-900) {
        const double r = rsq_nr(ss);
        const double nrm = ss * r;
        const double b = (x0 >= 0.0) ? -nrm : nrm;
        const double rd = rcp_nr(x0 - b);
        tau = fma(fabs(x0), r, 1.0);
        v1 = t1 * rd;
        v2 = t2 * rd;
        beta = b;
    } else if (t1 == 0.0 && t2 == 0.0) {
        tau = 0.0;
        beta = x0;
        v1 = v2 = 0.0;
    } else {
        house3(m, x0, x1, x2, v1, v2, tau, beta);
    }
}

// Chase nb bulges through the matrix held in LDS (or global memory).  Indices
// are global; local index = global - off.  Active block [ktop,kbot].  Bulge b
// is at position p0 + t - 3b at step t and acts when ktop-1 <= k <= kend (a
// reflector at k acts on rows/columns k+1..k+3).  Left application: local
// columns up to colhi; right application: local rows 0..min(k+4,kbot); Z (nz
// rows) accumulates.
//
// One step applies the reflectors of all active bulges in a single barrier
// phase.  The regions they touch are split so that no element is written by
// two threads: each bulge's own m x m block (P^T B P), the cross blocks between
// the rows of a higher bulge and the columns of a lower one (P_hi^T X P_lo),
// the left products right of the lowest active block, the right products
// above the highest active block plus each bulge's row k+4, and Z.  The
// geometry of a step (active bulges, positions, orders) follows from t alone
// and is computed by every thread; only the reflectors pass through LDS, one
// thread per bulge forming them before the products.  For a single bulge
// every thread computes the reflector itself (no barrier before the products)
// and the bulge column is written one step later, when no thread reads it
// any more.
template <int NTH = NT>
__device__ __forceinline__ void chain_chase(SmemCore &S, double *A, int lda, int off, int ktop, int kbot, int p0, int nsteps,
                            int kend, int nb, int colhi, double *Z, int ldz, int nz)
{
    const int tid = threadIdx.x;
    const int kbl = kbot - off;
    double fl = 0.0;
    if (nb == 1) {
        // pending bulge-column write (thread 0)
        int pend_kl = -1, pend_m = 0;
        double pend_beta = 0.0;
        for (int t = 0; t < nsteps; ++t) {
            const int k = p0 + t;
            if (k < ktop - 1 || k > kend) continue;
            int m;
            double v1, v2, tau, beta;
            bulge_reflector(S, A, lda, off, ktop, kbot, 0, k, m, v1, v2, tau, beta);
            const int kl = k - off;
            // the introduction reads the leading block, which the products overwrite
            if (k == ktop - 1) __syncthreads();
            if (tid == 0) {
                S.nphase += 1;
                S.nbstep += 1;
            }
            const int c0L = kl + m + 1;
            const int ncL = max(0, colhi - c0L + 1);
            const int nrR = max(0, kl + 1);
            const int perR = nrR + nz + 1;
            const int total = ncL + perR + 1;
            if (tid == 0) fl += 4.0 * 3.0 * (double)(ncL + perR) + 40.0;
            if (tau != 0.0)
                for (int it = tid; it < total; it += NTH) {
                    if (it < ncL) {
                        double *col = A + (c0L + it) * lda + kl + 1;
                        double y0 = col[0], y1 = col[1], y2 = (m == 3) ? col[2] : 0.0;
                        refl3(m, tau, v1, v2, y0, y1, y2);
                        col[0] = y0;
                        col[1] = y1;
                        if (m == 3) col[2] = y2;
                    } else if (it < ncL + perR) {
                        const int r = it - ncL;
                        double *Mx;
                        int ld;
                        if (r < nrR) {
                            Mx = A + r;
                            ld = lda;
                        } else if (r < nrR + nz) {
                            Mx = Z + (r - nrR);
                            ld = ldz;
                        } else {
                            if (m != 3 || kl + 4 > kbl) continue;
                            Mx = A + (kl + 4);
                            ld = lda;
                        }
                        double y0 = Mx[(kl + 1) * ld], y1 = Mx[(kl + 2) * ld], y2 = (m == 3) ? Mx[(kl + 3) * ld] : 0.0;
                        refl3(m, tau, v1, v2, y0, y1, y2);
                        Mx[(kl + 1) * ld] = y0;
                        Mx[(kl + 2) * ld] = y1;
                        if (m == 3) Mx[(kl + 3) * ld] = y2;
                    } else {
                        double *a = A + (kl + 1) + (kl + 1) * lda;
                        double B00 = a[0], B10 = a[1], B01 = a[lda], B11 = a[1 + lda];
                        double B02 = (m == 3) ? a[2 * lda] : 0.0, B12 = (m == 3) ? a[1 + 2 * lda] : 0.0;
                        double B20 = (m == 3) ? a[2] : 0.0, B21 = (m == 3) ? a[2 + lda] : 0.0;
                        double B22 = (m == 3) ? a[2 + 2 * lda] : 0.0;
                        refl3(3, tau, v1, v2, B00, B10, B20);
                        refl3(3, tau, v1, v2, B01, B11, B21);
                        refl3(3, tau, v1, v2, B02, B12, B22);
                        refl3(3, tau, v1, v2, B00, B01, B02);
                        refl3(3, tau, v1, v2, B10, B11, B12);
                        refl3(3, tau, v1, v2, B20, B21, B22);
                        a[0] = B00;
                        a[1] = B10;
                        a[lda] = B01;
                        a[1 + lda] = B11;
                        if (m == 3) {
                            a[2] = B20;
                            a[2 + lda] = B21;
                            a[2 * lda] = B02;
                            a[1 + 2 * lda] = B12;
                            a[2 + 2 * lda] = B22;
                        }
                    }
                }
            if (tid == 0) {
                // write the previous step's bulge column (nobody reads it now)
                if (pend_m > 0) {
                    A[(pend_kl + 1) + pend_kl * lda] = pend_beta;
                    A[(pend_kl + 2) + pend_kl * lda] = 0.0;
                    if (pend_m == 3) A[(pend_kl + 3) + pend_kl * lda] = 0.0;
                }
                pend_m = (k >= ktop) ? m : 0;
                pend_kl = kl;
                pend_beta = beta;
            }
            __syncthreads();
        }
        if (tid == 0 && pend_m > 0) {
            A[(pend_kl + 1) + pend_kl * lda] = pend_beta;
            A[(pend_kl + 2) + pend_kl * lda] = 0.0;
            if (pend_m == 3) A[(pend_kl + 3) + pend_kl * lda] = 0.0;
        }
        if (tid == 0) S.flops += fl;
        __syncthreads();
        return;
    }
    for (int t = 0; t < nsteps; ++t) {
        // active bulges b: ktop - 1 <= p0 + t - 3b <= kend
        const int k0 = p0 + t;
        const int blo = max(0, (k0 - kend + 2 + 3 * NTH) / 3 - NTH);            // ceil((k0 - kend) / 3)
        const int bhi = min(nb - 1, (k0 - (ktop - 1) + 3 * NTH) / 3 - NTH);     // floor((k0 - ktop + 1) / 3)
        if (blo > bhi) continue;
        if (tid >= blo && tid <= bhi) {
            const int b = tid, k = k0 - 3 * b;
            const int m = min(3, kbot - k);
            const int kl = k - off;
            double x0, x1, x2;
            if (k == ktop - 1) {
                shift_column(A, lda, kl + 1, kbl, S.sr[2 * b], S.si[2 * b], S.sr[2 * b + 1], S.si[2 * b + 1], x0, x1,
                             x2);
            } else {
                x0 = A[(kl + 1) + kl * lda];
                x1 = A[(kl + 2) + kl * lda];
                x2 = (m == 3) ? A[(kl + 3) + kl * lda] : 0.0;
            }
            double v1, v2, tau, beta;
            house3r(m, x0, x1, x2, v1, v2, tau, beta);
            if (m < 3) v2 = 0.0;
            if (k >= ktop) {
                A[(kl + 1) + kl * lda] = beta;
                A[(kl + 2) + kl * lda] = 0.0;
                if (m == 3) A[(kl + 3) + kl * lda] = 0.0;
            }
            S.bv1[b] = v1;
            S.bv2[b] = v2;
            S.btau[b] = tau;
        }
        __syncthreads();
        const int nact = bhi - blo + 1;
        if (tid == 0) {
            S.nphase += 1;
            S.nbstep += nact;
        }
        // bulge b: local position k0 - 3b - off, order min(3, kbot - (k0 - 3b))
        auto KL = [&](int b) { return k0 - 3 * b - off; };
        auto M = [&](int b) { return min(3, kbot - (k0 - 3 * b)); };
        const int klo = KL(blo), mlo = M(blo);
        const int khi = KL(bhi);
        const int c0L = klo + mlo + 1;             // free left columns: c0L..colhi
        const int ncL = max(0, colhi - c0L + 1);
        const int nrR = max(0, khi + 1);           // free right rows: 0..khi
        const int perR = nrR + nz + 1;             // + Z rows + row k+4
        const int npairs = nact * (nact - 1) / 2;
        const int nL = nact * ncL, nR = nact * perR;
        const int total = nL + nR + nact + npairs;
        // it / ncL and q / perR through single-precision reciprocals: exact,
        // since the quotients are at least 1/(2 n) from an integer and the
        // counts are far below 2^20
        const float rL = 1.0f / (float)max(ncL, 1), rR = 1.0f / (float)perR;
        if (tid == 0) fl += 4.0 * 3.0 * (double)(nL + nR) + 40.0 * (nact + npairs);
        for (int it = tid; it < total; it += NTH) {
            if (it < nL) {
                const int bi = (int)(((float)it + 0.5f) * rL);
                const int b = blo + bi, c = c0L + (it - bi * ncL);
                const double tau = S.btau[b], v1 = S.bv1[b], v2 = S.bv2[b];
                const int m = M(b), r = KL(b) + 1;
                double *col = A + c * lda + r;
                double y0 = col[0], y1 = col[1], y2 = (m == 3) ? col[2] : 0.0;
                if (tau == 0.0) continue;
                refl3(m, tau, v1, v2, y0, y1, y2);
                col[0] = y0;
                col[1] = y1;
                if (m == 3) col[2] = y2;
            } else if (it < nL + nR) {
                const int q = it - nL;
                const int bi = (int)(((float)q + 0.5f) * rR);
                const int b = blo + bi, r = q - bi * perR;
                const int m = M(b), kl = KL(b);
                double *Mx;
                int ld;
                if (r < nrR) {
                    Mx = A + r;
                    ld = lda;
                } else if (r < nrR + nz) {
                    Mx = Z + (r - nrR);
                    ld = ldz;
                } else {
                    if (m != 3 || kl + 4 > kbl) continue;
                    Mx = A + (kl + 4);
                    ld = lda;
                }
                const double tau = S.btau[b], v1 = S.bv1[b], v2 = S.bv2[b];
                double y0 = Mx[(kl + 1) * ld], y1 = Mx[(kl + 2) * ld], y2 = (m == 3) ? Mx[(kl + 3) * ld] : 0.0;
                if (tau == 0.0) continue;
                refl3(m, tau, v1, v2, y0, y1, y2);
                Mx[(kl + 1) * ld] = y0;
                Mx[(kl + 2) * ld] = y1;
                if (m == 3) Mx[(kl + 3) * ld] = y2;
            } else if (it < nL + nR + nact) {
                // own block: B <- P^T B P on rows/columns kl+1..kl+m (m = 2 is the 3x3
                // case with v2 = 0 and the third row/column left out)
                const int b = blo + (it - nL - nR);
                const int m = M(b), kl = KL(b);
                const double tau = S.btau[b], v1 = S.bv1[b], v2 = S.bv2[b];
                if (tau == 0.0) continue;
                double B00, B01, B02, B10, B11, B12, B20 = 0.0, B21 = 0.0, B22 = 0.0;
                double *a = A + (kl + 1) + (kl + 1) * lda;
                B00 = a[0];
                B10 = a[1];
                B01 = a[lda];
                B11 = a[1 + lda];
                B02 = (m == 3) ? a[2 * lda] : 0.0;
                B12 = (m == 3) ? a[1 + 2 * lda] : 0.0;
                if (m == 3) {
                    B20 = a[2];
                    B21 = a[2 + lda];
                    B22 = a[2 + 2 * lda];
                }
                refl3(3, tau, v1, v2, B00, B10, B20);
                refl3(3, tau, v1, v2, B01, B11, B21);
                refl3(3, tau, v1, v2, B02, B12, B22);
                refl3(3, tau, v1, v2, B00, B01, B02);
                refl3(3, tau, v1, v2, B10, B11, B12);
                refl3(3, tau, v1, v2, B20, B21, B22);
                a[0] = B00;
                a[1] = B10;
                a[lda] = B01;
                a[1 + lda] = B11;
                if (m == 3) {
                    a[2] = B20;
                    a[2 + lda] = B21;
                    a[2 * lda] = B02;
                    a[1 + 2 * lda] = B12;
                    a[2 + 2 * lda] = B22;
                }
            } else {
                // cross block: rows of bulge bu (higher) x columns of bulge bd (lower)
                int pp = it - nL - nR - nact;
                int i = 0;
                while (pp >= nact - 1 - i) {
                    pp -= nact - 1 - i;
                    ++i;
                }
                const int bd = blo + i, bu = blo + i + 1 + pp;
                const int mu = M(bu), md = M(bd), ku = KL(bu), kd = KL(bd);
                const double tu = S.btau[bu], td = S.btau[bd];
                const double u1 = S.bv1[bu], u2 = S.bv2[bu], d1 = S.bv1[bd], d2 = S.bv2[bd];
                double *x = A + (ku + 1) + (kd + 1) * lda;
                double X00 = x[0], X10 = x[1], X20 = (mu == 3) ? x[2] : 0.0;
                double X01 = x[lda], X11 = x[1 + lda], X21 = (mu == 3) ? x[2 + lda] : 0.0;
                double X02 = 0.0, X12 = 0.0, X22 = 0.0;
                if (md == 3) {
                    X02 = x[2 * lda];
                    X12 = x[1 + 2 * lda];
                    X22 = (mu == 3) ? x[2 + 2 * lda] : 0.0;
                }
                if (tu != 0.0) {
                    refl3(3, tu, u1, u2, X00, X10, X20);
                    refl3(3, tu, u1, u2, X01, X11, X21);
                    refl3(3, tu, u1, u2, X02, X12, X22);
                }
                if (td != 0.0) {
                    refl3(3, td, d1, d2, X00, X01, X02);
                    refl3(3, td, d1, d2, X10, X11, X12);
                    refl3(3, td, d1, d2, X20, X21, X22);
                }
                x[0] = X00;
                x[1] = X10;
                x[lda] = X01;
                x[1 + lda] = X11;
                if (mu == 3) {
                    x[2] = X20;
                    x[2 + lda] = X21;
                }
                if (md == 3) {
                    x[2 * lda] = X02;
                    x[1 + 2 * lda] = X12;
                    if (mu == 3) x[2 + 2 * lda] = X22;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) S.flops += fl;
}

// Single-bulge chase (one double-shift sweep) through the matrix held in LDS:
// the reflector at k acts on rows/columns k+1..k+m of the active block
// [ktop,kbot] (indices global, local = global - off), left products on local
// columns up to colhi, right products on local rows 0..k+4 and on the nz rows
// of Z.  One barrier per step.  Every thread computes the reflector itself;
// the entries a thread updates are loaded before the reflector is formed, so
// their latency hides behind it.  Items: row and column segments of three
// entries (one product each) on threads 0..NT-11 and round-robin beyond; the
// nine entries of the diagonal block B (both products, B <- P B P entry by
// entry from u = B v, w = B^T v and v^T B v) on the last nine threads, and
// the bulge column on thread NT-10, written one step later when nobody reads
// it.  The last wave has no segments while the block has at most 246 of
// them, so its longer chains do not hold up the others.
__device__ __forceinline__ void chase1(SmemCore &S, double *A, int lda, int off, int ktop, int kbot, int p0,
                                       int nsteps, int kend, int colhi, double *Z, int ldz, int nz)
{
    const int tid = threadIdx.x;
    const int kbl = kbot - off;
    int pend_kl = -1, pend_m = 0, nph = 0;
    double pend_beta = 0.0;
    double fl = 0.0;
    constexpr int OWN0 = NT - 9, PEND = NT - 10, NSEG1 = NT - 10;
    const int er = (tid - OWN0) % 3, ec = (tid - OWN0) / 3; // entry of the diagonal block (tid >= OWN0)
    for (int t = 0; t < nsteps; ++t) {
        const int k = p0 + t;
        if (k < ktop - 1 || k > kend) continue;
        const int kl = k - off;
        const int m = min(3, kbot - k);
        const bool intro = (k == ktop - 1);
        const int c0L = kl + m + 1;
        const int ncL = max(0, colhi - c0L + 1);
        const int nrR = kl + 1;
        const bool extra = (m == 3 && kl + 4 <= kbl);
        const int perR = nrR + nz + (extra ? 1 : 0);
        const int nseg = ncL + perR; // row/column segments
        const bool own = tid >= OWN0;
        const bool mine = own && er < m && ec < m;
        const int it = tid;
        const bool seg = tid < NSEG1 && it < nseg;
        double sx0 = 0.0, sx1 = 0.0, sx2 = 0.0;
        if (intro) {
            shift_column(A, lda, kl + 1, kbl, S.sr[0], S.si[0], S.sr[1], S.si[1], sx0, sx1, sx2);
            __syncthreads(); // the leading block is read before anyone overwrites it
        }
        // Loads in the order the data is needed: the diagonal block (last
        // nine threads), the bulge column, then this thread's segment.  The column
        // and segment loads are unconditional (a harmless in-bounds address
        // where there is nothing to load) so that waiting for the column does
        // not wait for the segment, whose latency then hides behind the
        // reflector.
        double B00 = 0.0, B01 = 0.0, B02 = 0.0, B10 = 0.0, B11 = 0.0, B12 = 0.0, B20 = 0.0, B21 = 0.0, B22 = 0.0;
        double *a = A + (kl + 1) + (kl + 1) * lda;
        if (own) {
            B00 = a[0];
            B10 = a[1];
            B01 = a[lda];
            B11 = a[1 + lda];
            if (m == 3) {
                B02 = a[2 * lda];
                B12 = a[1 + 2 * lda];
                B20 = a[2];
                B21 = a[2 + lda];
                B22 = a[2 + 2 * lda];
            }
        }
        const double *xc = A + (kl + 1) + max(kl, 0) * lda;
        double x0 = xc[0], x1 = xc[1], x2 = xc[(m == 3) ? 2 : 1];
        // segment geometry without branches: column segment (left product),
        // row of A above the block, row of Z, or row kl+4 (right product)
        const int r = it - ncL;
        const bool isL = it < ncL, isA = !isL && r < nrR, isZ = !isL && !isA && r < nrR + nz;
        double *base = isZ ? Z : A;
        const int ldb = isZ ? ldz : lda;
        const int prow = !seg ? 0 : (isL ? (kl + 1) : (isA ? r : (isZ ? r - nrR : kl + 4)));
        const int pcol = !seg ? 0 : (isL ? (c0L + it) : (kl + 1));
        const int st = (!seg || isL) ? 1 : ldb;
        double *p = base + prow + pcol * ldb;
        double y0 = p[0], y1 = p[st], y2 = p[((m == 3) ? 2 : 1) * st];
        if (intro) {
            x0 = sx0;
            x1 = sx1;
            x2 = sx2;
        }
        if (m < 3) {
            x2 = 0.0;
            y2 = 0.0;
        }
        // the last nine threads (one wave) all read B before any of them writes its entry
        __builtin_amdgcn_wave_barrier();
        double v1, v2, tau, beta;
        house3c(m, x0, x1, x2, v1, v2, tau, beta);
        if (m < 3) v2 = 0.0;
        if (tau != 0.0) {
            if (seg) {
                refl3(m, tau, v1, v2, y0, y1, y2);
                p[0] = y0;
                p[st] = y1;
                if (m == 3) p[2 * st] = y2;
            } else if (mine) {
                // B' = B - tau v w^T - tau u v^T + tau^2 (v^T u) v v^T
                const double u0 = B00 + v1 * B01 + v2 * B02;
                const double u1 = B10 + v1 * B11 + v2 * B12;
                const double u2 = B20 + v1 * B21 + v2 * B22;
                const double gam = u0 + v1 * u1 + v2 * u2;
                const double vr = (er == 0) ? 1.0 : (er == 1 ? v1 : v2);
                const double vc = (ec == 0) ? 1.0 : (ec == 1 ? v1 : v2);
                const double ur = (er == 0) ? u0 : (er == 1 ? u1 : u2);
                const double b0c = (ec == 0) ? B00 : (ec == 1 ? B01 : B02);
                const double b1c = (ec == 0) ? B10 : (ec == 1 ? B11 : B12);
                const double b2c = (ec == 0) ? B20 : (ec == 1 ? B21 : B22);
                const double wc = b0c + v1 * b1c + v2 * b2c;
                const double brc = (er == 0) ? b0c : (er == 1 ? b1c : b2c);
                a[er + ec * lda] = brc - tau * (vr * wc + ur * vc) + tau * tau * gam * vr * vc;
            }
            // further segments (matrices with more rows than threads)
            for (int it2 = tid + NSEG1; it2 < nseg; it2 += NT) {
                double *q;
                int sq;
                if (it2 < ncL) {
                    q = A + (c0L + it2) * lda + (kl + 1);
                    sq = 1;
                } else {
                    const int r2 = it2 - ncL;
                    if (r2 < nrR) {
                        q = A + r2 + (kl + 1) * lda;
                        sq = lda;
                    } else if (r2 < nrR + nz) {
                        q = Z + (r2 - nrR) + (kl + 1) * ldz;
                        sq = ldz;
                    } else {
                        q = A + (kl + 4) + (kl + 1) * lda;
                        sq = lda;
                    }
                }
                double z0 = q[0], z1 = q[sq], z2 = (m == 3) ? q[2 * sq] : 0.0;
                refl3(m, tau, v1, v2, z0, z1, z2);
                q[0] = z0;
                q[sq] = z1;
                if (m == 3) q[2 * sq] = z2;
            }
        }
        if (tid == PEND) {
            if (pend_m > 0) {
                A[(pend_kl + 1) + pend_kl * lda] = pend_beta;
                A[(pend_kl + 2) + pend_kl * lda] = 0.0;
                if (pend_m == 3) A[(pend_kl + 3) + pend_kl * lda] = 0.0;
            }
            pend_m = intro ? 0 : m;
            pend_kl = kl;
            pend_beta = beta;
            fl += 4.0 * 3.0 * (double)nseg + 40.0;
            ++nph;
        }
        __syncthreads();
    }
    if (tid == PEND) {
        if (pend_m > 0) {
            A[(pend_kl + 1) + pend_kl * lda] = pend_beta;
            A[(pend_kl + 2) + pend_kl * lda] = 0.0;
            if (pend_m == 3) A[(pend_kl + 3) + pend_kl * lda] = 0.0;
        }
        S.flops += fl;
        S.nphase += nph;
        S.nbstep += nph;
    }
    __syncthreads();
}

// Broadcast of a double held by one lane of the wave (scalar read of the lane).
__device__ inline double lane_bcast(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Single-bulge sweep (one double-shift step) over the active block [kt,kb]
// of the matrix in LDS (local indices), left products on columns up to colhi,
// right products on rows 0..k+4 and on the nz rows of Z, with a one-step
// lookahead on the reflectors.  The last wave (the core) owns the 3x3
// diagonal block B (rows/columns k+1..k+3): at position k its lanes 0..8 load
// B and form one entry each of P B P (from u = B v, w = B^T v and v^T B v),
// lanes 9..11 write the bulge column (beta, 0, 0); the two entries of P B P in
// the next bulge column reach every lane by a scalar lane read, and with the
// fill-in of row k+4 (-tau v2 h, h the untouched subdiagonal entry below the
// block) the core forms the reflector of position k+1 and passes it on
// through LDS.  The other waves read the reflector of position k from LDS and
// apply it to the row and column segments of three entries outside the
// block.  Nothing the core reads at position k is written by another wave at
// position k, so one barrier per position suffices, and the reflector is
// formed once per position, off the segment waves' path.
__device__ __forceinline__ void chase_la(SmemCore &S, double *A, int lda, int kt, int kb, int colhi, double *Z,
                                         int ldz, int nz)
{
    constexpr int NSEGT = NT - 64; // threads of the segment waves
    const int tid = threadIdx.x;
    const bool core = tid >= NSEGT;
    const int lane = tid - NSEGT;
    const int er = lane % 3, ec = lane / 3; // this lane's entry of the block (lanes 0..8)
    const int kfirst = kt - 1, klast = kb - 2;
    double fl = 0.0;
    double cv1 = 0.0, cv2 = 0.0, ctau = 0.0, cbeta = 0.0, ch = 0.0;
    if (core) {
        const double *a = A + kt + kt * lda;
        const double h11 = a[0], h21 = a[1], h12 = a[lda], h22 = a[1 + lda];
        const double h32 = (kt + 2 <= kb) ? a[2 + lda] : 0.0;
        ch = (kt + 3 <= kb) ? A[(kt + 3) + (kt + 2) * lda] : 0.0;
        const double sr0 = S.sr[0], si0 = S.si[0], sr1 = S.sr[1], si1 = S.si[1];
        const double sc = fabs(h11 - sr1) + fabs(si1) + fabs(h21);
        double x0 = 0.0, x1 = 0.0, x2 = 0.0;
        if (sc != 0.0) {
            const double f = h21 / sc;
            x0 = f * h12 + (h11 - sr0) * ((h11 - sr1) / sc) - si0 * (si1 / sc);
            x1 = f * (h11 + h22 - sr0 - sr1);
            x2 = f * h32;
        }
        const int m0 = min(3, kb - kfirst);
        house3r(m0, x0, x1, x2, cv1, cv2, ctau, cbeta);
        if (m0 < 3) cv2 = 0.0;
        if (lane == 0) {
            S.bv1[0] = cv1;
            S.bv2[0] = cv2;
            S.btau[0] = ctau;
        }
    }
    __syncthreads();
    for (int k = kfirst; k <= klast; ++k) {
        const int par = (k - kfirst) & 1;
        const int m = min(3, kb - k);
        const bool extra = (m == 3 && k + 4 <= kb);
        if (!core) {
            const double v1 = S.bv1[par], v2 = S.bv2[par], tau = S.btau[par];
            const int c0L = k + m + 1;
            const int ncL = max(0, colhi - c0L + 1), nrR = k + 1;
            const int nseg = ncL + nrR + nz + (extra ? 1 : 0);
            // Matrix in LDS: one segment per thread and step.  In global
            // memory: SG segments per thread and pass with all loads issued
            // before the first store (the segments of one position are
            // disjoint), so a pass waits for one memory latency instead of
            // one per segment (measured: 17 % faster batched solves of orders
            // 97..256; the same grouping costs 4 % per position in LDS).
            constexpr int SG = 8;
            if (__builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void *)A)) {
                // stored back unconditionally (tau = 0 leaves the segment
                // unchanged), so the segment's loads go out with the reflector's
                for (int it = tid; it < nseg; it += NSEGT) {
                    const int r = it - ncL;
                    const bool isL = it < ncL, isA = !isL && r < nrR, isZ = !isL && !isA && r < nrR + nz;
                    double *base = isZ ? Z : A;
                    const int ldb = isZ ? ldz : lda;
                    const int prow = isL ? (k + 1) : (isA ? r : (isZ ? r - nrR : k + 4));
                    const int pcol = isL ? (c0L + it) : (k + 1);
                    const int st = isL ? 1 : ldb;
                    double *p = base + prow + pcol * ldb;
                    double y0 = p[0], y1 = p[st], y2 = (m == 3) ? p[2 * st] : 0.0;
                    refl3(m, tau, v1, v2, y0, y1, y2);
                    p[0] = y0;
                    p[st] = y1;
                    if (m == 3) p[2 * st] = y2;
                }
            } else
            for (int it0 = tid; it0 < nseg; it0 += SG * NSEGT) {
                double *pp[SG];
                int stp[SG];
                double y[SG][3];
#pragma unroll
                for (int g = 0; g < SG; ++g) {
                    const int it = it0 + g * NSEGT;
                    pp[g] = nullptr;
                    stp[g] = 0;
                    y[g][0] = y[g][1] = y[g][2] = 0.0;
                    if (it < nseg) {
                        const int r = it - ncL;
                        const bool isL = it < ncL, isA = !isL && r < nrR, isZ = !isL && !isA && r < nrR + nz;
                        double *base = isZ ? Z : A;
                        const int ldb = isZ ? ldz : lda;
                        const int prow = isL ? (k + 1) : (isA ? r : (isZ ? r - nrR : k + 4));
                        const int pcol = isL ? (c0L + it) : (k + 1);
                        const int st = isL ? 1 : ldb;
                        double *p = base + prow + pcol * ldb;
                        pp[g] = p;
                        stp[g] = st;
                        y[g][0] = p[0];
                        y[g][1] = p[st];
                        y[g][2] = (m == 3) ? p[2 * st] : 0.0;
                    }
                }
                if (tau != 0.0) {
#pragma unroll
                    for (int g = 0; g < SG; ++g) {
                        if (!pp[g]) continue;
                        double y0 = y[g][0], y1 = y[g][1], y2 = y[g][2];
                        refl3(m, tau, v1, v2, y0, y1, y2);
                        double *p = pp[g];
                        const int st = stp[g];
                        p[0] = y0;
                        p[st] = y1;
                        if (m == 3) p[2 * st] = y2;
                    }
                }
            }
            if (tid == 0) fl += 12.0 * (double)nseg + 40.0;
        } else {
            // the block, final since the last barrier and written below only by the core
            const double *a = A + (k + 1) + (k + 1) * lda;
            const double B00 = a[0], B10 = a[1], B01 = a[lda], B11 = a[1 + lda];
            const double B20 = (m == 3) ? a[2] : 0.0, B21 = (m == 3) ? a[2 + lda] : 0.0;
            const double B02 = (m == 3) ? a[2 * lda] : 0.0, B12 = (m == 3) ? a[1 + 2 * lda] : 0.0;
            const double B22 = (m == 3) ? a[2 + 2 * lda] : 0.0;
            const double hn = (k + 5 <= kb) ? A[(k + 5) + (k + 4) * lda] : 0.0;
            __builtin_amdgcn_wave_barrier(); // every core lane has read B before any writes it
            // this lane's entry of P B P = B - tau v w^T - tau u v^T + tau^2 (v^T u) v v^T
            const double v1 = cv1, v2 = cv2, tau = ctau;
            const double b0c = (ec == 0) ? B00 : (ec == 1 ? B01 : B02);
            const double b1c = (ec == 0) ? B10 : (ec == 1 ? B11 : B12);
            const double b2c = (ec == 0) ? B20 : (ec == 1 ? B21 : B22);
            double val = (er == 0) ? b0c : (er == 1 ? b1c : b2c);
            if (tau != 0.0) {
                const double u0 = B00 + v1 * B01 + v2 * B02;
                const double u1 = B10 + v1 * B11 + v2 * B12;
                const double u2 = B20 + v1 * B21 + v2 * B22;
                const double gam = u0 + v1 * u1 + v2 * u2;
                const double wc = b0c + v1 * b1c + v2 * b2c;
                const double vr = (er == 0) ? 1.0 : (er == 1 ? v1 : v2);
                const double vc = (ec == 0) ? 1.0 : (ec == 1 ? v1 : v2);
                const double ur = (er == 0) ? u0 : (er == 1 ? u1 : u2);
                val = val - tau * (vr * wc + ur * vc) + tau * tau * gam * vr * vc;
            }
            // the block and the bulge column first: their stores overlap the reflector below
            if (lane < 9 && er < m && ec < m) A[(k + 1 + er) + (k + 1 + ec) * lda] = val;
            if (lane >= 9 && lane < 12 && k > kfirst && lane - 9 < m)
                A[(k + lane - 8) + k * lda] = (lane == 9) ? cbeta : 0.0;
            if (k < klast) {
                // reflector of position k+1 from rows k+2..k+4 of column k+1:
                // entries (1,0) and (2,0) of P B P (lanes 1 and 2) and the fill-in of row k+4
                const double x0 = lane_bcast(val, 1), x1 = lane_bcast(val, 2);
                const int m1 = min(3, kb - (k + 1));
                const double r0 = (extra && tau != 0.0) ? -(tau * (v2 * ch)) : 0.0; // as the row segment computes it
                double nv1, nv2, ntau, nbeta;
                house3r(m1, x0, x1, (m1 == 3) ? r0 : 0.0, nv1, nv2, ntau, nbeta);
                if (m1 < 3) nv2 = 0.0;
                if (lane == 0) {
                    S.bv1[par ^ 1] = nv1;
                    S.bv2[par ^ 1] = nv2;
                    S.btau[par ^ 1] = ntau;
                }
                cv1 = nv1;
                cv2 = nv2;
                ctau = ntau;
                cbeta = nbeta;
                ch = hn;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        S.flops += fl;
        S.nphase += klast - kfirst + 1;
        S.nbstep += klast - kfirst + 1;
    }
    __syncthreads();
}

// Largest l in (lo,hi] whose subdiagonal A[l,l-1] is zero or negligible
// (then set to zero); lo if there is none.
__device__ __forceinline__ int find_split(SmemCore &S, double *A, int lda, int lo, int hi, const Defl &dfl)
{
    if (threadIdx.x == 0) S.ic[0] = lo;
    __syncthreads();
    for (int l = hi - (int)threadIdx.x; l > lo; l -= NT) {
        if (A[l + (l - 1) * lda] == 0.0 || small_sub(A, lda, l, lo, hi, dfl)) {
            atomicMax(&S.ic[0], l);
            break;
        }
    }
    __syncthreads();
    int l = S.ic[0];
    __syncthreads();
    if (threadIdx.x == 0 && l > lo) A[l + (l - 1) * lda] = 0.0;
    __syncthreads();
    return l;
}

// Standardize the 2x2 block at (k,k+1): rows k,k+1 over columns k..ncol-1,
// columns over rows 0..k+1, Z columns over nz rows.  Returns 1 for a complex pair.
__device__ __forceinline__ int std_block(SmemCore &S, double *A, int lda, int ncol, double *Z, int ldz, int nz, int k)
{
    for (int pass = 0; pass < 3; ++pass) {
        if (threadIdx.x == 0) {
            double cs, sn;
            int mode = std_rot(A[k + k * lda], A[k + (k + 1) * lda], A[(k + 1) + k * lda],
                               A[(k + 1) + (k + 1) * lda], cs, sn);
            S.ic[1] = mode;
            S.sc[0] = cs;
            S.sc[1] = sn;
        }
        __syncthreads();
        int mode = S.ic[1];
        double cs = S.sc[0], sn = S.sc[1];
        if (mode == 0) {
            int res = A[(k + 1) + k * lda] != 0.0;
            __syncthreads();
            return res;
        }
        for (int j = k + (int)threadIdx.x; j < ncol; j += NT) {
            double x = A[k + j * lda], y = A[(k + 1) + j * lda];
            A[k + j * lda] = cs * x + sn * y;
            A[(k + 1) + j * lda] = -sn * x + cs * y;
        }
        __syncthreads();
        for (int it = threadIdx.x; it < (k + 2) + nz; it += NT) {
            double *M;
            int ld;
            if (it < k + 2) {
                M = A + it;
                ld = lda;
            } else {
                M = Z + (it - (k + 2));
                ld = ldz;
            }
            double x = M[k * ld], y = M[(k + 1) * ld];
            M[k * ld] = cs * x + sn * y;
            M[(k + 1) * ld] = -sn * x + cs * y;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (mode == 1) {
                A[(k + 1) + k * lda] = 0.0;
            } else {
                double avg = 0.5 * (A[k + k * lda] + A[(k + 1) + (k + 1) * lda]);
                A[k + k * lda] = avg;
                A[(k + 1) + (k + 1) * lda] = avg;
            }
        }
        __syncthreads();
        if (mode == 1) return 0;
        if (A[k + (k + 1) * lda] * A[(k + 1) + k * lda] < 0.0) return 1;
    }
    return A[(k + 1) + k * lda] != 0.0;
}

// One Francis double-shift iteration on the active block [l,i] (full T and Z):
// shifts from the trailing 2x2 (exceptional shifts at iterations 10 and 20).
__device__ __forceinline__ void ds_step(SmemCore &S, double *A, int lda, int m, double *Z, int ldz, int nz, int l, int i, int its)
{
    if (threadIdx.x == 0) {
        double a, b, c, d;
        if (its == 10) {
            double ss = fabs(A[(l + 1) + l * lda]) + fabs(A[(l + 2) + (l + 1) * lda]);
            a = 0.75 * ss + A[l + l * lda];
            b = -0.4375 * ss;
            c = ss;
            d = a;
        } else if (its == 20) {
            double ss = fabs(A[i + (i - 1) * lda]) + fabs(A[(i - 1) + (i - 2) * lda]);
            a = 0.75 * ss + A[i + i * lda];
            b = -0.4375 * ss;
            c = ss;
            d = a;
        } else {
            a = A[(i - 1) + (i - 1) * lda];
            b = A[(i - 1) + i * lda];
            c = A[i + (i - 1) * lda];
            d = A[i + i * lda];
        }
        double r1, i1, r2, i2;
        eig2x2(a, b, c, d, r1, i1, r2, i2);
        if (i1 == 0.0) {
            double hii = A[i + i * lda];
            double pick = (fabs(r1 - hii) <= fabs(r2 - hii)) ? r1 : r2;
            r1 = r2 = pick;
        }
        S.sr[0] = r1;
        S.si[0] = i1;
        S.sr[1] = r2;
        S.si[1] = i2;
    }
    __syncthreads();
    chase_la(S, A, lda, l, i, m - 1, Z, ldz, nz);
}

// Francis double-shift QR on the whole matrix A (order m, full T), Z accumulates.
// Returns 0 or 1 + the bottom row of the block that did not converge.
// Rows ilo..ihi only when given (ihi < 0: the whole matrix); the updates
// still cover the full rows and columns of the order-m matrix.
__device__ __forceinline__ int qr_ds(SmemCore &S, double *A, int lda, int m, double *Z, int ldz, int nz, const Defl &dfl,
                     int64_t itmax_in, int ilo = 0, int ihi = -1)
{
    int64_t itmax = 30 * (int64_t)max(10, m);
    if (itmax_in > 0 && itmax_in < itmax) itmax = itmax_in;
    int64_t total = 0;
    int i = (ihi < 0) ? m - 1 : ihi;
    while (i >= ilo) {
        int its = 0, l;
        for (;;) {
            l = find_split(S, A, lda, ilo, i, dfl);
            if (l >= i - 1) break;
            if (total >= itmax) return i + 1;
            ds_step(S, A, lda, m, Z, ldz, nz, l, i, its);
            ++its;
            ++total;
        }
        if (l == i) {
            i -= 1;
        } else {
            std_block(S, A, lda, m, Z, ldz, nz, i - 1);
            i -= 2;
        }
    }
    return 0;
}

// Small-block QR with multishift sweeps: when the active block is large
// enough, the eigenvalues of its trailing ns x ns block (ns <= nsmax <= 16)
// become the shifts of a chain of ns/2 tightly coupled bulges chased through
// the block in one pass (Sec. 2.3); otherwise, and at the exceptional-shift
// iterations, a double-shift step.  nsmax <= 2 gives the plain Francis QR.
__device__ __forceinline__ int qr_small(SmemCore &S, double *A, int lda, int m, double *Z, int ldz, int nz, const Defl &dfl,
                        int64_t itmax_in, int nsmax = 2)
{
    if (nsmax <= 2) return qr_ds(S, A, lda, m, Z, ldz, nz, dfl, itmax_in);
    nsmax = min(nsmax, 16) & ~1;
    int64_t itmax = 30 * (int64_t)max(10, m);
    if (itmax_in > 0 && itmax_in < itmax) itmax = itmax_in;
    int64_t total = 0;
    int i = m - 1;
    while (i >= 0) {
        int its = 0, l;
        for (;;) {
            l = find_split(S, A, lda, 0, i, dfl);
            if (l >= i - 1) break;
            if (total >= itmax) return i + 1;
            const int nh = i - l + 1;
            int ns = min(nsmax, (nh / 4) & ~1);
            int nsh = 0;
            if (ns >= 4 && its != 10 && its != 20) {
                const int j0 = i - ns + 1;
                for (int it = threadIdx.x; it < ns * ns; it += NT) {
                    int r = it % ns, c = it / ns;
                    S.shb[r + c * ns] = (r <= c + 1) ? A[(j0 + r) + (j0 + c) * lda] : 0.0;
                }
                __syncthreads();
                int inf = qr_ds(S, S.shb, ns, ns, S.shb, ns, 0, dfl, 0); // no Z rows (nz = 0)
                if (threadIdx.x == 0) {
                    // pair the eigenvalues of the converged part, bottom first
                    int cnt = 0;
                    double rr = 0.0;
                    bool have = false;
                    int k = ns - 1;
                    while (k >= inf && cnt + 2 <= 2 * GMAX) {
                        bool two = (k >= 1 && k - 1 >= inf && S.shb[k + (k - 1) * ns] != 0.0);
                        if (two) {
                            double r1, i1, r2, i2;
                            eig2x2(S.shb[(k - 1) + (k - 1) * ns], S.shb[(k - 1) + k * ns], S.shb[k + (k - 1) * ns],
                                   S.shb[k + k * ns], r1, i1, r2, i2);
                            S.sr[cnt] = r1;
                            S.si[cnt] = i1;
                            S.sr[cnt + 1] = r2;
                            S.si[cnt + 1] = i2;
                            cnt += 2;
                            k -= 2;
                        } else {
                            double v = S.shb[k + k * ns];
                            if (have) {
                                S.sr[cnt] = rr;
                                S.si[cnt] = 0.0;
                                S.sr[cnt + 1] = v;
                                S.si[cnt + 1] = 0.0;
                                cnt += 2;
                                have = false;
                            } else {
                                rr = v;
                                have = true;
                            }
                            k -= 1;
                        }
                    }
                    S.ic[4] = cnt;
                }
                __syncthreads();
                nsh = S.ic[4];
                __syncthreads();
            }
            if (nsh >= 4) {
                const int nb = nsh / 2;
                chain_chase(S, A, lda, 0, l, i, l - 1, (i - 2) - (l - 1) + 1 + 3 * (nb - 1), i - 2, nb, m - 1, Z,
                            ldz, nz);
            } else {
                ds_step(S, A, lda, m, Z, ldz, nz, l, i, its);
            }
            ++its;
            ++total;
        }
        if (l == i) {
            i -= 1;
        } else {
            std_block(S, A, lda, m, Z, ldz, nz, i - 1);
            i -= 2;
        }
    }
    return 0;
}

// Standardizing rotation of a 2x2 block held in registers: returns the total
// rotation (cs, sn) and leaves the standardized values in (a, b, c, d).
__device__ inline void std2_regs(double &a, double &b, double &c, double &d, double &cst, double &snt)
{
    cst = 1.0;
    snt = 0.0;
    for (int pass = 0; pass < 3; ++pass) {
        double cs, sn;
        int mode = std_rot(a, b, c, d, cs, sn);
        if (mode == 0) break;
        double m00 = a * cs + b * sn, m01 = -a * sn + b * cs;
        double m10 = c * cs + d * sn, m11 = -c * sn + d * cs;
        a = cs * m00 + sn * m10;
        b = cs * m01 + sn * m11;
        c = -sn * m00 + cs * m10;
        d = -sn * m01 + cs * m11;
        double t = cst * cs - snt * sn;
        snt = snt * cs + cst * sn;
        cst = t;
        if (mode == 1) {
            c = 0.0;
            break;
        }
        double avg = 0.5 * (a + d);
        a = d = avg;
        if (b * c < 0.0) break;
    }
}

// One thread: orthogonal G exchanging the blocks of D = T(j:j+M, j:j+M)
// (top block P x P, bottom block Q x Q; at least one of them 2x2), with the
// two new diagonal blocks standardized.  On success Dn = G^T D G, with its
// (2,1) block exactly zero, replaces D in T and G goes to Gout (column
// major, order M); on rejection nothing is written.  Bai-Demmel: solve A11 X - X A22 = A12, QR of [-X; I_Q],
// weak (new (2,1) block) and strong (reconstruction) stability tests.
// Sizes are compile-time so every array stays in registers; pivot choices
// are applied through unrolled selects.
template <int P, int Q>
__device__ bool swap_xform(double *Tw, int ldt, int j, double smlnum, double *Gout)
{
    const double *T = Tw;
    constexpr int M = P + Q, PQ = P * Q;
    double D[M][M];
    double dnorm = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int r = 0; r < M; ++r) {
            D[r][c] = T[(j + r) + (j + c) * ldt];
            dnorm = fmax(dnorm, fabs(D[r][c]));
        }
    const double thresh = fmax(10.0 * kU * dnorm, smlnum);
    // Kronecker form of the Sylvester equation: unknown x[r + P c] = X[r][c]
    double K[PQ][PQ], rhs[PQ];
    double kmax = 0.0;
#pragma unroll
    for (int c = 0; c < Q; ++c)
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int row = r + P * c;
            rhs[row] = D[r][P + c];
#pragma unroll
            for (int c2 = 0; c2 < Q; ++c2)
#pragma unroll
                for (int r2 = 0; r2 < P; ++r2) {
                    double v = 0.0;
                    if (c == c2) v += D[r][r2];
                    if (r == r2) v -= D[P + c2][P + c];
                    K[row][r2 + P * c2] = v;
                    kmax = fmax(kmax, fabs(v));
                }
        }
    const double smin = fmax(kU * kmax, smlnum);
    int perm[PQ];
#pragma unroll
    for (int i = 0; i < PQ; ++i) perm[i] = i;
#pragma unroll
    for (int k = 0; k < PQ; ++k) {
        int br = k, bc = k;
        double best = -1.0;
#pragma unroll
        for (int i = k; i < PQ; ++i)
#pragma unroll
            for (int c2 = k; c2 < PQ; ++c2)
                if (fabs(K[i][c2]) > best) {
                    best = fabs(K[i][c2]);
                    br = i;
                    bc = c2;
                }
#pragma unroll
        for (int i = k + 1; i < PQ; ++i)
            if (br == i) {
#pragma unroll
                for (int c2 = 0; c2 < PQ; ++c2) {
                    double t = K[k][c2];
                    K[k][c2] = K[i][c2];
                    K[i][c2] = t;
                }
                double t = rhs[k];
                rhs[k] = rhs[i];
                rhs[i] = t;
            }
#pragma unroll
        for (int c2 = k + 1; c2 < PQ; ++c2)
            if (bc == c2) {
#pragma unroll
                for (int i = 0; i < PQ; ++i) {
                    double t = K[i][k];
                    K[i][k] = K[i][c2];
                    K[i][c2] = t;
                }
                int t = perm[k];
                perm[k] = perm[c2];
                perm[c2] = t;
            }
        if (fabs(K[k][k]) < smin) K[k][k] = (K[k][k] >= 0.0) ? smin : -smin;
#pragma unroll
        for (int i = k + 1; i < PQ; ++i) {
            const double f = K[i][k] / K[k][k];
#pragma unroll
            for (int c2 = k; c2 < PQ; ++c2) K[i][c2] -= f * K[k][c2];
            rhs[i] -= f * rhs[k];
        }
    }
    double z[PQ], x[PQ];
#pragma unroll
    for (int k = PQ - 1; k >= 0; --k) {
        double acc = rhs[k];
#pragma unroll
        for (int c2 = k + 1; c2 < PQ; ++c2) acc -= K[k][c2] * z[c2];
        z[k] = acc / K[k][k];
    }
#pragma unroll
    for (int t = 0; t < PQ; ++t) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < PQ; ++k)
            if (perm[k] == t) v = z[k];
        x[t] = v;
    }
    // QR of [-X; I_Q] (M x Q) by Q Householder reflectors accumulated into G
    double Mm[M][Q], G[M][M];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
#pragma unroll
        for (int r = 0; r < P; ++r) Mm[r][c] = -x[r + P * c];
#pragma unroll
        for (int r = 0; r < Q; ++r) Mm[P + r][c] = (r == c) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) G[r][c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        double nrm2 = 0.0;
#pragma unroll
        for (int r = c + 1; r < M; ++r) nrm2 += Mm[r][c] * Mm[r][c];
        const double x0 = Mm[c][c];
        double v[M];
#pragma unroll
        for (int r = 0; r < M; ++r) v[r] = 0.0;
        v[c] = 1.0;
        double tau = 0.0;
        if (nrm2 > 0.0) {
            const double nrm = sqrt(x0 * x0 + nrm2);
            const double bb = (x0 >= 0.0) ? -nrm : nrm;
            tau = (bb - x0) / bb;
            const double sc = 1.0 / (x0 - bb);
#pragma unroll
            for (int r = c + 1; r < M; ++r) v[r] = Mm[r][c] * sc;
        }
        if (tau != 0.0) {
#pragma unroll
            for (int cc = c; cc < Q; ++cc) {
                double acc = 0.0;
#pragma unroll
                for (int r = c; r < M; ++r) acc += v[r] * Mm[r][cc];
                acc *= tau;
#pragma unroll
                for (int r = c; r < M; ++r) Mm[r][cc] -= acc * v[r];
            }
#pragma unroll
            for (int rr = 0; rr < M; ++rr) {
                double acc = 0.0;
#pragma unroll
                for (int r = c; r < M; ++r) acc += G[rr][r] * v[r];
                acc *= tau;
#pragma unroll
                for (int r = c; r < M; ++r) G[rr][r] -= acc * v[r];
            }
        }
    }
    double DG[M][M], Dn[M][M];
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < M; ++l) acc += D[r][l] * G[l][c];
            DG[r][c] = acc;
        }
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < M; ++l) acc += G[l][r] * DG[l][c];
            Dn[r][c] = acc;
        }
    double e1 = 0.0;
#pragma unroll
    for (int c = 0; c < Q; ++c)
#pragma unroll
        for (int r = Q; r < M; ++r) {
            e1 = fmax(e1, fabs(Dn[r][c]));
            Dn[r][c] = 0.0;
        }
    double e2 = 0.0;
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < M; ++l) {
                double tt = 0.0;
#pragma unroll
                for (int l2 = 0; l2 < M; ++l2) tt += Dn[l][l2] * G[c][l2];
                acc += G[r][l] * tt;
            }
            e2 = fmax(e2, fabs(acc - D[r][c]));
        }
    if (e1 > thresh || e2 > thresh) return false;
    // standardize the new diagonal blocks; the rotations join G
    if (Q == 2) {
        double a = Dn[0][0], b = Dn[0][1], c = Dn[1][0], d = Dn[1][1], cs, sn;
        std2_regs(a, b, c, d, cs, sn);
#pragma unroll
        for (int cc = 2; cc < M; ++cc) { // rows 0,1 right of the block
            double y0 = Dn[0][cc], y1 = Dn[1][cc];
            Dn[0][cc] = cs * y0 + sn * y1;
            Dn[1][cc] = -sn * y0 + cs * y1;
        }
#pragma unroll
        for (int rr = 0; rr < M; ++rr) {
            double y0 = G[rr][0], y1 = G[rr][1];
            G[rr][0] = cs * y0 + sn * y1;
            G[rr][1] = -sn * y0 + cs * y1;
        }
        Dn[0][0] = a;
        Dn[0][1] = b;
        Dn[1][0] = c;
        Dn[1][1] = d;
    }
    if (P == 2) {
        const int q0 = Q;
        double a = Dn[q0][q0], b = Dn[q0][q0 + 1], c = Dn[q0 + 1][q0], d = Dn[q0 + 1][q0 + 1], cs, sn;
        std2_regs(a, b, c, d, cs, sn);
#pragma unroll
        for (int rr = 0; rr < Q; ++rr) { // rows above the block, its two columns
            double y0 = Dn[rr][q0], y1 = Dn[rr][q0 + 1];
            Dn[rr][q0] = cs * y0 + sn * y1;
            Dn[rr][q0 + 1] = -sn * y0 + cs * y1;
        }
#pragma unroll
        for (int rr = 0; rr < M; ++rr) {
            double y0 = G[rr][q0], y1 = G[rr][q0 + 1];
            G[rr][q0] = cs * y0 + sn * y1;
            G[rr][q0 + 1] = -sn * y0 + cs * y1;
        }
        Dn[q0][q0] = a;
        Dn[q0][q0 + 1] = b;
        Dn[q0 + 1][q0] = c;
        Dn[q0 + 1][q0 + 1] = d;
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int r = 0; r < M; ++r) {
            Gout[r + M * c] = G[r][c];
            Tw[(j + r) + (j + c) * ldt] = Dn[r][c];
        }
    return true;
}

// Bottom-up deflation test of the candidates of the quasi-triangular T (order
// nt) with spike entries sp_k = spscale * Z[sprow + k*ldz]; each failed
// candidate moves up to the first free position of the undeflated region,
// the remaining candidates shift down (Sec. 2.5, and the concurrent deflate
// and reordering windows of Sec. 3.5 "Parallel aggressive early deflation").
//
// The moves are pipelined: a failed candidate starts to move as soon as it is
// examined, and the next candidate (the block now below it) is examined as
// soon as its own entries are final, i.e. after the first exchange of the move
// above it.  Every phase performs, for all moves at once, one exchange of
// adjacent blocks per move whose block above is free, so a move trails the one
// ahead of it by one block.  Exchanges of one phase touch disjoint diagonal
// ranges: their left products (rows) are applied first, then their right
// products (columns of T above the range and of Z), so every entry sees the
// same products as in the one-move-at-a-time order; only the rounding order
// of the entries shared by two exchanges differs.  Wave 0 schedules: lane i
// owns the i-th active move, the lane after the last one examines candidates;
// each lane also forms its exchange (rotation, or Bai-Demmel with standardized
// blocks).  A rejected exchange, or a moving 2x2 block that splits, halts the
// reordering after its phase; T stays quasi-triangular and everything above
// the deflated bottom counts as undeflated.  Returns the number of undeflated
// leading rows.
__device__ __forceinline__ int aed_deflate(SmemCore &S, double *T, int ldt, int nt, double *Z, int ldz, int nz, int sprow,
                           double spscale, int ilst0, const Defl &dfl, int nforced = 0, bool reorder_only = false)
{
    const double smlnum = dfl.smlnum;
    ReorderState &R = S.ro;
    const int tid = threadIdx.x;
    if (tid == 0) {
        R.head = R.tail = 0;
        R.ns = nt;
        R.ilst = ilst0;
        R.halt = 0;
        R.chk_done = (ilst0 >= nt) ? 1 : 0;
        R.done = 0;
    }
    __syncthreads();
    int par = 0, nphase = 0;
    while (!R.done) {
        // wave 0's scheduling state, carried across the exchange step
        const int lane = tid;
        int head = 0, tail = 0, nact = 0;
        bool halt0 = false, chk_done = false;
        int ns = 0, ilst = 0;
        int slot = -1, pos = 0, sz = 0, dst = 0;
        int sj = -1, sp = 0;
        bool fin = false, bad = false, created = false;
        if (tid < 64) {
            // (a) scheduling from the state left by the previous phase; no LDS
            // writes until every lane has read what it needs
            head = R.head;
            tail = R.tail;
            nact = tail - head;
            halt0 = R.halt != 0;
            chk_done = R.chk_done != 0;
            ns = R.ns;
            ilst = R.ilst;
            if (!halt0 && lane < nact) {
                const int id = head + lane;
                slot = id % MV;
                pos = R.pos[par][slot];
                sz = R.sz[slot];
                dst = R.dst[slot];
                if (pos == dst) {
                    fin = true;
                } else {
                    const int lim = (lane == 0) ? 0 : R.pos[par][(id - 1) % MV] + R.sz[(id - 1) % MV];
                    const int above = (pos >= 2 && T[(pos - 1) + (pos - 2) * ldt] != 0.0) ? 2 : 1;
                    const int j = pos - above;
                    if (j < dst) {
                        bad = true;
                    } else if (j >= lim) {
                        sj = j;
                        sp = above;
                    }
                }
            }
            if (!halt0 && !chk_done && lane == nact && nact < MV) {
                const int lim2 = (nact > 0) ? R.pos[par][(tail - 1) % MV] + R.sz[(tail - 1) % MV] : 0;
                for (;;) {
                    if (ilst >= ns) {
                        chk_done = true;
                        break;
                    }
                    const bool two = (ns >= 2 && T[(ns - 1) + (ns - 2) * ldt] != 0.0);
                    if (two && ns - 2 < ilst) {
                        chk_done = true;
                        break;
                    }
                    const int csz = two ? 2 : 1, k = ns - 1, cand = ns - csz;
                    if (cand < lim2) break; // still touched by the move above it
                    bool defl;
                    if (dfl.thr >= 0.0) {
                        // norm-stable / fixed conditions: each spike entry of the block
                        defl = fabs(spscale * Z[sprow + k * ldz]) <= dfl.thr;
                        if (two) defl = defl && fabs(spscale * Z[sprow + (k - 1) * ldz]) <= dfl.thr;
                    } else if (!two) {
                        const double foo = fabs(T[k + k * ldt]);
                        defl = fabs(spscale * Z[sprow + k * ldz]) <= fmax(smlnum, kU * foo);
                    } else {
                        const double hh = sqrt(fabs(T[k + k * ldt] * T[(k - 1) + (k - 1) * ldt])) +
                                          sqrt(fabs(T[(k - 1) + k * ldt] * T[k + (k - 1) * ldt]));
                        const double spk = fmax(fabs(spscale * Z[sprow + k * ldz]),
                                                fabs(spscale * Z[sprow + (k - 1) * ldz]));
                        defl = spk <= fmax(smlnum, kU * hh);
                    }
                    if (cand >= nt - nforced) defl = false; // failed in an earlier deflation window
                    // reordering window: the forced failures move to the top,
                    // every other candidate stays below them untested
                    else if (reorder_only) defl = true;
                    if (defl) {
                        ns -= csz;
                        continue;
                    }
                    if (cand == ilst) { // already in place
                        ilst += csz;
                        continue;
                    }
                    created = true;
                    slot = tail % MV;
                    pos = cand;
                    sz = csz;
                    dst = ilst;
                    const int above = (cand >= 2 && T[(cand - 1) + (cand - 2) * ldt] != 0.0) ? 2 : 1;
                    const int j = cand - above;
                    if (j < ilst) bad = true;
                    else if (j >= lim2) {
                        sj = j;
                        sp = above;
                    }
                    ilst += csz;
                    break;
                }
            }
            // publish the lane's exchange: kind 0 (1x1 past 1x1), 1 (1x1
            // past 2x2), 2 (2x2 past 1x1) or 3 (2x2 past 2x2)
            if (lane < MV) {
                R.xj[lane] = sj;
                R.xk[lane] = (sj >= 0) ? 2 * (sz - 1) + (sp - 1) : -1;
            }
        }
        __syncthreads();
        // (b) the exchanges: wave w forms those of kind w (the kinds run on
        // different SIMDs instead of one after another in divergent lanes of
        // one wave), writes the new diagonal block into T, G into the lane's
        // slot and the outcome (1 done, 2 done with a 2x2 block split, 0
        // rejected) into xr
        {
            const int w = tid >> 6, l = tid & 63;
            if (l < MV && R.xk[l] == w) {
                const int j = R.xj[l];
                double *G = R.G + l * 16;
                bool ok = true;
                int szl = 1;
                if (w == 0) {
                    const double t11 = T[j + j * ldt], t12 = T[j + (j + 1) * ldt];
                    const double t22 = T[(j + 1) + (j + 1) * ldt];
                    const double rr = hypot(t12, t22 - t11);
                    double cs = 1.0, sn = 0.0;
                    if (rr != 0.0) {
                        cs = t12 / rr;
                        sn = (t22 - t11) / rr;
                    }
                    G[0] = cs;
                    G[1] = sn;
                    G[2] = -sn;
                    G[3] = cs;
                    T[j + j * ldt] = t22;
                    T[j + (j + 1) * ldt] = cs * (-t11 * sn + t12 * cs) + sn * (t22 * cs);
                    T[(j + 1) + j * ldt] = 0.0;
                    T[(j + 1) + (j + 1) * ldt] = t11;
                } else if (w == 1) {
                    ok = swap_xform<2, 1>(T, ldt, j, smlnum, G);
                } else if (w == 2) {
                    ok = swap_xform<1, 2>(T, ldt, j, smlnum, G);
                    szl = 2;
                } else {
                    ok = swap_xform<2, 2>(T, ldt, j, smlnum, G);
                    szl = 2;
                }
                R.xr[l] = !ok ? 0 : ((szl == 2 && T[(j + 1) + j * ldt] == 0.0) ? 2 : 1);
            }
        }
        __syncthreads();
        if (tid < 64) {
            const int res = (sj >= 0) ? R.xr[lane] : 1;
            const bool ok = res != 0, split = res == 2;
            const bool moved = (sj >= 0) && ok;
            if (slot >= 0) {
                R.pos[par ^ 1][slot] = moved ? sj : pos;
                if (created) {
                    R.sz[slot] = sz;
                    R.dst[slot] = dst;
                }
            }
            // finished moves leave the head of the queue in order
            const unsigned long long finm = __ballot(fin || (moved && sj == dst));
            const unsigned long long stop = __ballot(bad || !ok || split);
            const unsigned long long tried = __ballot(sj >= 0);
            // prefix sums of the row and column work items of this phase
            const int m = sp + sz;
            int rc = moved ? (nt - (sj + m)) : 0, cc = moved ? (sj + nz) : 0;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int r2 = __shfl_up(rc, d), c2 = __shfl_up(cc, d);
                if (lane >= d) {
                    rc += r2;
                    cc += c2;
                }
            }
            if (lane < MV) {
                R.sj[lane] = moved ? sj : 0;
                R.sm[lane] = moved ? m : 0;
                R.roff[lane + 1] = rc;
                R.coff[lane + 1] = cc;
            }
            if (lane == 63) {
                R.rtot = rc;
                R.ctot = cc;
            }
            if (lane == 0) {
                R.roff[0] = 0;
                R.coff[0] = 0;
                const int nfin = __ffsll((long long)~finm) - 1;
                R.head = head + min(nfin, nact);
                if (stop) R.halt = 1;
                S.nswap += __popcll(tried);
            }
            if (lane == nact && nact < MV && !halt0) {
                R.ns = ns;
                R.ilst = ilst;
                R.chk_done = chk_done ? 1 : 0;
                if (created) R.tail = tail + 1;
            }
        }
        __syncthreads();
        const int rtot = R.rtot, ctot = R.ctot;
        // left products: rows sj..sj+m-1 over the columns right of the range
        {
            int s = 0;
            for (int it = tid; it < rtot; it += NT) {
                while (it >= R.roff[s + 1]) ++s;
                const int j = R.sj[s], m = R.sm[s];
                const double *G = R.G + s * 16;
                const int c = j + m + (it - R.roff[s]);
                double x[4], y[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = (r < m) ? T[(j + r) + c * ldt] : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (i < m && r < m) acc += G[i + m * r] * x[i];
                    y[r] = acc;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r < m) T[(j + r) + c * ldt] = y[r];
            }
        }
        __syncthreads();
        // right products: columns sj..sj+m-1 over the rows of T above the range and all rows of Z
        {
            int s = 0;
            for (int it = tid; it < ctot; it += NT) {
                while (it >= R.coff[s + 1]) ++s;
                const int j = R.sj[s], m = R.sm[s];
                const double *G = R.G + s * 16;
                const int rr = it - R.coff[s];
                double *Mx;
                int ld;
                if (rr < j) {
                    Mx = T + rr;
                    ld = ldt;
                } else {
                    Mx = Z + (rr - j);
                    ld = ldz;
                }
                double x[4], y[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) x[c] = (c < m) ? Mx[(j + c) * ld] : 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < 4; ++l)
                        if (l < m && c < m) acc += x[l] * G[l + m * c];
                    y[c] = acc;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < m) Mx[(j + c) * ld] = y[c];
            }
        }
        ++nphase;
        if (tid == 0) {
            S.nrphase += 1;
            // every phase moves the oldest block or examines a candidate, so
            // nt * nt phases bound the loop; the cap only guards that argument
            if (R.halt || (R.chk_done && R.head == R.tail) || nphase >= nt * nt + 64) R.done = 1;
        }
        par ^= 1;
        __syncthreads();
    }
    const int ns = R.ns;
    __syncthreads();
    return ns;
}

// v^T x over len entries of x (stride st) with four partial sums, so the
// multiply-adds form four short dependency chains instead of one long one.
__device__ __forceinline__ double dot_v(const double *v, const double *x, int64_t st, int len)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = 0;
    for (; i + 3 < len; i += 4) {
        s0 = fma(v[i], x[i * st], s0);
        s1 = fma(v[i + 1], x[(i + 1) * st], s1);
        s2 = fma(v[i + 2], x[(i + 2) * st], s2);
        s3 = fma(v[i + 3], x[(i + 3) * st], s3);
    }
    for (; i < len; ++i) s0 = fma(v[i], x[i * st], s0);
    return (s0 + s1) + (s2 + s3);
}

// x <- x - a v over len entries of x (stride st).
__device__ __forceinline__ void axpy_v(double a, const double *v, double *x, int64_t st, int len)
{
    int i = 0;
    for (; i + 3 < len; i += 4) {
        x[i * st] -= a * v[i];
        x[(i + 1) * st] -= a * v[i + 1];
        x[(i + 2) * st] -= a * v[i + 2];
        x[(i + 3) * st] -= a * v[i + 3];
    }
    for (; i < len; ++i) x[i * st] -= a * v[i];
}

// Householder vector of x = vec[0..len-1] (in LDS): overwrites vec with v
// (v[0] = 1) and returns tau; beta in S.sc[2].
template <class SM>
__device__ __forceinline__ double house_vec(SM &S, double *vec, int len)
{
    double amax = 0.0;
    for (int i = 1 + (int)threadIdx.x; i < len; i += NT) amax = fmax(amax, fabs(vec[i]));
    amax = block_max(S, amax);
    double ss = 0.0;
    if (amax > 0.0)
        for (int i = 1 + (int)threadIdx.x; i < len; i += NT) {
            double t = vec[i] / amax;
            ss += t * t;
        }
    ss = block_sum(S, ss);
    double tau = 0.0, beta = vec[0], scal = 0.0;
    if (amax > 0.0) {
        double tail = amax * sqrt(ss);
        double x0 = vec[0];
        double nrm = hypot(x0, tail);
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tau = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
    }
    __syncthreads();
    for (int i = 1 + (int)threadIdx.x; i < len; i += NT) vec[i] = (tau != 0.0) ? vec[i] * scal : 0.0;
    if (threadIdx.x == 0) {
        vec[0] = 1.0;
        S.sc[2] = beta;
    }
    __syncthreads();
    return tau;
}

// Spike removal and Householder Hessenberg reduction of T(0:ns,0:ns) in LDS;
// the reflectors also update T(0:ns, ns:nt) and Z (nz rows).  The spike is
// spscale * Z[sprow, 0:ns] on entry.  Returns the new subdiagonal entry.
template <class SM>
__device__ __forceinline__ double restore_lds(SM &S, double *T, int ldt, int nt, int ns, double *Z, int ldz, int nz,
                              int sprow, double spscale)
{
    double *v = S.vec;
    for (int i = threadIdx.x; i < ns; i += NT) v[i] = spscale * Z[sprow + i * ldz];
    __syncthreads();
    double tau = house_vec(S, v, ns);
    double beta = S.sc[2];
    for (int step = -1; step < ns - 2; ++step) {
        int r0, len, c0;
        if (step >= 0) {
            r0 = step + 1;
            len = ns - r0;
            for (int i = threadIdx.x; i < len; i += NT) v[i] = T[(r0 + i) + step * ldt];
            __syncthreads();
            tau = house_vec(S, v, len);
            if (threadIdx.x == 0) {
                T[r0 + step * ldt] = S.sc[2];
            }
            for (int i = 1 + (int)threadIdx.x; i < len; i += NT) T[(r0 + i) + step * ldt] = 0.0;
            c0 = step + 1;
        } else {
            r0 = 0;
            len = ns;
            c0 = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) S.flops += 4.0 * len * (double)((nt - c0) + ns + nz);
        if (tau != 0.0) {
            // left: rows r0..r0+len-1, columns c0..nt-1
            for (int c = c0 + (int)threadIdx.x; c < nt; c += NT) {
                double *col = T + r0 + c * ldt;
                axpy_v(tau * dot_v(v, col, 1, len), v, col, 1, len);
            }
            __syncthreads();
            // right: columns r0..r0+len-1 over rows 0..ns-1 of T and all rows of Z
            for (int it = threadIdx.x; it < ns + nz; it += NT) {
                double *M;
                int ld;
                if (it < ns) {
                    M = T + it;
                    ld = ldt;
                } else {
                    M = Z + (it - ns);
                    ld = ldz;
                }
                double *row = M + r0 * ld;
                axpy_v(tau * dot_v(v, row, ld, len), v, row, ld, len);
            }
        }
        __syncthreads();
    }
    return beta;
}

// Store Z^T (order m) zero padded to order K16 into Ut (column major, ld K16).
template <int NTH = NT>
__device__ __forceinline__ void store_factor_t(const double *Z, int ldz, int m, double *Ut)
{
    int K16 = (m + 15) & ~15;
    for (int it = threadIdx.x; it < K16 * K16; it += NTH) {
        int j = it % K16, k = it / K16; // Ut[j + k*K16] = Z[k][j]
        Ut[it] = (j < m && k < m) ? Z[k + j * ldz] : 0.0;
    }
}

template <int NTH = NT>
__device__ __forceinline__ void identity_lds(double *Z, int ldz, int m, int rows)
{
    for (int it = threadIdx.x; it < rows * m; it += NTH) {
        int r = it % rows, c = it / rows;
        Z[r + c * ldz] = (r == c) ? 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------------------
// kernels

__global__ void __launch_bounds__(NT) k_find_block(double *H, int64_t ld, int ilo, int kbot, Defl dfl,
                                                   IterStatus *st)
{
    __shared__ int best;
    if (threadIdx.x == 0) best = ilo;
    __syncthreads();
    for (int l = kbot - (int)threadIdx.x; l > ilo; l -= NT) {
        if (H[l + (int64_t)(l - 1) * ld] == 0.0 || small_sub(H, ld, l, ilo, kbot, dfl)) {
            atomicMax(&best, l);
            break;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int l = best;
        if (l > ilo) H[l + (int64_t)(l - 1) * ld] = 0.0;
        st->ktop = l;
    }
}

__global__ void __launch_bounds__(NT) k_iter(double *H, int64_t ld, int n, int ilo, int kbot, int nw, int nmin,
                                             Defl dfl, int64_t itmax, double *Ut, IterStatus *st, int nsmall)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const int tid = threadIdx.x;
    const long long t_start = wall_clock64();
    // locate the active block
    if (tid == 0) {
        S.ic[3] = ilo;
        S.flops = 0.0;
        S.nphase = S.nbstep = S.nswap = S.nrphase = 0;
    }
    __syncthreads();
    for (int l = kbot - tid; l > ilo; l -= NT) {
        if (H[l + (int64_t)(l - 1) * ld] == 0.0 || small_sub(H, ld, l, ilo, kbot, dfl)) {
            atomicMax(&S.ic[3], l);
            break;
        }
    }
    __syncthreads();
    const int ktop = S.ic[3];
    __syncthreads();
    if (tid == 0 && ktop > ilo) H[ktop + (int64_t)(ktop - 1) * ld] = 0.0;
    const int nh = kbot - ktop + 1;
    const bool small = (nh <= nmin) || (nh <= MMAX && nh <= nw);
    const int m = small ? nh : min(nw, nh);
    const int kw = kbot - m + 1;
    double s = 0.0;
    if (!small && kw > ktop) s = H[kw + (int64_t)(kw - 1) * ld];
    // load the block / window, zero below the subdiagonal; Z = I
    for (int it = tid; it < m * m; it += NT) {
        int r = it % m, c = it / m;
        S.A[r + c * LDM] = (r <= c + 1) ? H[(kw + r) + (int64_t)(kw + c) * ld] : 0.0;
    }
    identity_lds(S.Z, LDM, m, m);
    __syncthreads();
    int info = qr_small(S, S.A, LDM, m, S.Z, LDM, m, dfl, itmax, nsmall);
    const long long t_schur = wall_clock64();
    long long t_defl = t_schur, t_rest = t_schur;
    int ns = 0, nd = m;
    double beta = 0.0;
    if (!small) {
        // spike = s * Z(0,:); bottom-up test; failures move to the top
        ns = aed_deflate(S, S.A, LDM, m, S.Z, LDM, m, 0, s, info > 0 ? info : 0, dfl);
        t_defl = wall_clock64();
        nd = m - ns;
        if (tid == 0) {
            // candidates: eigenvalues of the undeflated blocks, diagonal order
            int k = 0;
            while (k < ns) {
                int sz = (k + 1 < ns && S.A[(k + 1) + k * LDM] != 0.0) ? 2 : 1;
                if (sz == 1) {
                    st->cr[k] = S.A[k + k * LDM];
                    st->ci[k] = 0.0;
                } else {
                    double r1, i1, r2, i2;
                    eig2x2(S.A[k + k * LDM], S.A[k + (k + 1) * LDM], S.A[(k + 1) + k * LDM],
                           S.A[(k + 1) + (k + 1) * LDM], r1, i1, r2, i2);
                    if (i1 < 0.0) {
                        double t = i1;
                        i1 = i2;
                        i2 = t;
                    }
                    st->cr[k] = r1;
                    st->ci[k] = i1;
                    st->cr[k + 1] = r2;
                    st->ci[k + 1] = i2;
                }
                k += sz;
            }
        }
        if (nd > 0) {
            if (ns >= 1) beta = s * S.Z[0];
            if (ns > 1 && s != 0.0) beta = restore_lds(S, S.A, LDM, m, ns, S.Z, LDM, m, 0, s);
        }
        t_rest = wall_clock64();
    }
    __syncthreads();
    const bool changed = small || nd > 0;
    if (changed) {
        for (int it = tid; it < m * m; it += NT) {
            int r = it % m, c = it / m;
            H[(kw + r) + (int64_t)(kw + c) * ld] = (r <= c + 1) ? S.A[r + c * LDM] : 0.0;
        }
        if (!small && kw > ktop && tid == 0) H[kw + (int64_t)(kw - 1) * ld] = (ns >= 1) ? beta : 0.0;
        store_factor_t(S.Z, LDM, m, Ut);
    }
    if (tid == 0) {
        st->kind = small ? 0 : 1;
        st->ktop = ktop;
        st->kwtop = kw;
        st->nw = m;
        st->nd = small ? m : nd;
        st->ns = small ? 0 : ns;
        st->ncand = small ? 0 : ns;
        st->info = small ? (info > 0 ? kw + info : 0) : 0;
        st->changed = changed ? 1 : 0;
        st->beta = S.flops;
        st->nphase = S.nphase;
        st->nbstep = S.nbstep;
        st->nswap = S.nswap;
        st->nrphase = S.nrphase;
        st->tick[0] = t_schur - t_start;
        st->tick[1] = t_defl - t_schur;
        st->tick[2] = t_rest - t_defl;
        st->tick[3] = wall_clock64() - t_start;
    }
}

// One workgroup per window of a chase round.  The window owns all of the
// CU's LDS, so the workgroup takes 16 waves: each chase step is a few
// thousand independent LDS-latency-bound reflector applications.
constexpr int CHASE_NT = 1024;
__global__ void __launch_bounds__(CHASE_NT) k_chase(double *H, int64_t ld, ChaseRound R, const double *sr,
                                                    const double *si, Defl dfl, double *Ubuf, int64_t ustride)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const ChaseWin W = R.w[blockIdx.x];
    const int tid = threadIdx.x;
    const int a = W.a, wa = W.wa;
    for (int it = tid; it < wa * wa; it += CHASE_NT) {
        int r = it % wa, c = it / wa;
        S.A[r + c * LDM] = H[(a + r) + (int64_t)(a + c) * ld];
    }
    identity_lds<CHASE_NT>(S.Z, LDM, wa, wa);
    if (tid < 2 * W.nb) {
        S.sr[tid] = sr[W.shift_off + tid];
        S.si[tid] = si[W.shift_off + tid];
    }
    if (tid == 0) {
        S.flops = 0.0;
        S.nphase = S.nbstep = 0;
    }
    __syncthreads();
    chain_chase<CHASE_NT>(S, S.A, LDM, a, R.ktop, R.kbot, W.p0, W.nsteps, W.kend, W.nb, wa - 1, S.Z, LDM, wa);
    // vigilant deflation behind the top bulge (entries final for this sweep)
    int nv = W.vig_hi - W.vig_lo + 1;
    for (int i = tid; i < nv; i += CHASE_NT) {
        int k = W.vig_lo + i; // test subdiagonal (k+1, k)
        int kl = k - a;
        bool z = false;
        if (kl >= 0 && kl + 1 < wa && S.A[(kl + 1) + kl * LDM] != 0.0)
            z = small_sub(S.A, LDM, kl + 1, max(R.ktop - a, 0), min(R.kbot - a, wa - 1), dfl);
        S.vflag[i] = z ? 1 : 0;
    }
    __syncthreads();
    for (int i = tid; i < nv; i += CHASE_NT)
        if (S.vflag[i]) {
            int kl = W.vig_lo + i - a;
            S.A[(kl + 1) + kl * LDM] = 0.0;
        }
    __syncthreads();
    for (int it = tid; it < wa * wa; it += CHASE_NT) {
        int r = it % wa, c = it / wa;
        H[(a + r) + (int64_t)(a + c) * ld] = S.A[r + c * LDM];
    }
    store_factor_t<CHASE_NT>(S.Z, LDM, wa, Ubuf + (int64_t)W.slot * ustride);
}

// Corner deflation of a large AED window held in global memory.
__global__ void __launch_bounds__(NT) k_corner_deflate(double *T, int64_t ldt, int nw, int wd, const double *V,
                                                       int64_t ldv, double s, Defl dfl, double *Ut,
                                                       IterStatus *st, int nforced, int reorder)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const int tid = threadIdx.x;
    int c0 = nw - wd;
    if (c0 > 0 && T[c0 + (int64_t)(c0 - 1) * ldt] != 0.0) { // do not split a 2x2 block
        c0 += 1;
        wd -= 1;
    }
    for (int it = tid; it < wd * wd; it += NT) {
        int r = it % wd, c = it / wd;
        S.A[r + c * LDM] = T[(c0 + r) + (int64_t)(c0 + c) * ldt];
    }
    identity_lds(S.Z, LDM, wd, wd);
    for (int c = tid; c < wd; c += NT) S.Z[wd + c * LDM] = s * V[(int64_t)(c0 + c) * ldv];
    if (tid == 0) S.nswap = S.nrphase = 0;
    __syncthreads();
    int nsc = aed_deflate(S, S.A, LDM, wd, S.Z, LDM, wd + 1, wd, 1.0, 0, dfl, min(nforced, wd), reorder != 0);
    const int halted = S.ro.halt;
    __syncthreads();
    for (int it = tid; it < wd * wd; it += NT) {
        int r = it % wd, c = it / wd;
        T[(c0 + r) + (int64_t)(c0 + c) * ldt] = S.A[r + c * LDM];
    }
    store_factor_t(S.Z, LDM, wd, Ut);
    if (tid == 0) {
        st->ns = c0 + nsc;
        st->nd = nw - (c0 + nsc);
        st->kwtop = c0; // corner offset
        st->nw = wd;
        st->info = halted;
    }
}

// Hessenberg restoration of a large window in global memory (one workgroup).
__global__ void __launch_bounds__(1024) k_restore_global(double *T, int64_t ldt, int nw, int ns, double *V,
                                                         int64_t ldv, int nv, double s, double *vbuf,
                                                         IterStatus *st)
{
    __shared__ double red[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    auto bsum = [&](double x) {
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = x;
        __syncthreads();
        double t = 0.0;
        for (int i = 0; i < (nt >> 6); ++i) t += red[i];
        return t;
    };
    auto bmax = [&](double x) {
        for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = x;
        __syncthreads();
        double t = 0.0;
        for (int i = 0; i < (nt >> 6); ++i) t = fmax(t, red[i]);
        return t;
    };
    double *v = vbuf;
    double beta_spike = 0.0;
    for (int step = -1; step < ns - 2; ++step) {
        int r0, len, c0;
        if (step < 0) {
            r0 = 0;
            len = ns;
            c0 = 0;
            for (int i = tid; i < len; i += nt) v[i] = s * V[(int64_t)i * ldv];
        } else {
            r0 = step + 1;
            len = ns - r0;
            c0 = step + 1;
            for (int i = tid; i < len; i += nt) v[i] = T[(r0 + i) + (int64_t)step * ldt];
        }
        __syncthreads();
        double amax = 0.0;
        for (int i = 1 + tid; i < len; i += nt) amax = fmax(amax, fabs(v[i]));
        amax = bmax(amax);
        double ss = 0.0;
        if (amax > 0.0)
            for (int i = 1 + tid; i < len; i += nt) {
                double t = v[i] / amax;
                ss += t * t;
            }
        ss = bsum(ss);
        double x0 = v[0], tau = 0.0, beta = x0, scal = 0.0;
        if (amax > 0.0) {
            double nrm = hypot(x0, amax * sqrt(ss));
            beta = (x0 >= 0.0) ? -nrm : nrm;
            tau = (beta - x0) / beta;
            scal = 1.0 / (x0 - beta);
        }
        __syncthreads();
        for (int i = 1 + tid; i < len; i += nt) v[i] = (tau != 0.0) ? v[i] * scal : 0.0;
        if (tid == 0) v[0] = 1.0;
        if (step < 0) {
            beta_spike = beta;
        } else {
            if (tid == 0) T[r0 + (int64_t)step * ldt] = beta;
            for (int i = 1 + tid; i < len; i += nt) T[(r0 + i) + (int64_t)step * ldt] = 0.0;
        }
        __syncthreads();
        if (tau != 0.0) {
            for (int c = c0 + tid; c < nw; c += nt) {
                double *col = T + (int64_t)c * ldt + r0;
                axpy_v(tau * dot_v(v, col, 1, len), v, col, 1, len);
            }
            __syncthreads();
            for (int it = tid; it < ns + nv; it += nt) {
                double *M;
                int64_t l2;
                if (it < ns) {
                    M = T + it;
                    l2 = ldt;
                } else {
                    M = V + (it - ns);
                    l2 = ldv;
                }
                double *row = M + (int64_t)r0 * l2;
                axpy_v(tau * dot_v(v, row, l2, len), v, row, l2, len);
            }
        }
        __syncthreads();
    }
    if (tid == 0) st->beta = beta_spike;
}

__global__ void k_window_copy(const double *H, int64_t ld, int kwtop, int nw, double *T, int64_t ldt, double *V,
                              int64_t ldv)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tot = (int64_t)nw * nw;
    if (idx >= tot) return;
    int r = (int)(idx % nw), c = (int)(idx / nw);
    T[r + c * ldt] = (r <= c + 1) ? H[(kwtop + r) + (int64_t)(kwtop + c) * ld] : 0.0;
    V[r + c * ldv] = (r == c) ? 1.0 : 0.0;
}

__global__ void k_block_eigs(const double *T, int64_t ldt, int m, double *wr, double *wi)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    // block start: k is the second row of a 2x2 block if T[k,k-1] != 0
    bool second = (k > 0 && T[k + (int64_t)(k - 1) * ldt] != 0.0);
    bool first = (k + 1 < m && T[(k + 1) + (int64_t)k * ldt] != 0.0);
    if (!first && !second) {
        wr[k] = T[k + (int64_t)k * ldt];
        wi[k] = 0.0;
        return;
    }
    int k0 = first ? k : k - 1;
    double r1, i1, r2, i2;
    eig2x2(T[k0 + (int64_t)k0 * ldt], T[k0 + (int64_t)(k0 + 1) * ldt], T[(k0 + 1) + (int64_t)k0 * ldt],
           T[(k0 + 1) + (int64_t)(k0 + 1) * ldt], r1, i1, r2, i2);
    if (i1 < 0.0) {
        double t = i1;
        i1 = i2;
        i2 = t;
    }
    wr[k] = first ? r1 : r2;
    wi[k] = first ? i1 : i2;
}

// Final pass, stage 1: standardizing rotation for every 2x2 block (computed on
// a register copy of the block); blocks that need one are appended to a list.
__global__ void k_fin_rot(const double *H, int64_t ld, int n, int lo, double *rc, double *rs, int *list,
                          int *count, double *blk)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < lo || k >= n) return; // rows above lo did not converge: no blocks there
    bool first = (k + 1 < n && H[(k + 1) + (int64_t)k * ld] != 0.0);
    bool second = (k > 0 && H[k + (int64_t)(k - 1) * ld] != 0.0);
    if (!first || second) return; // blocks never overlap in quasi-triangular T
    double a = H[k + (int64_t)k * ld], b = H[k + (int64_t)(k + 1) * ld];
    double c = H[(k + 1) + (int64_t)k * ld], d = H[(k + 1) + (int64_t)(k + 1) * ld];
    double cst = 1.0, snt = 0.0;
    int any = 0;
    for (int pass = 0; pass < 3; ++pass) {
        double cs, sn;
        int mode = std_rot(a, b, c, d, cs, sn);
        if (mode == 0) break;
        any = 1;
        double m00 = a * cs + b * sn, m01 = -a * sn + b * cs;
        double m10 = c * cs + d * sn, m11 = -c * sn + d * cs;
        a = cs * m00 + sn * m10;
        b = cs * m01 + sn * m11;
        c = -sn * m00 + cs * m10;
        d = -sn * m01 + cs * m11;
        double t = cst * cs - snt * sn;
        snt = snt * cs + cst * sn;
        cst = t;
        if (mode == 1) {
            c = 0.0;
            break;
        }
        double avg = 0.5 * (a + d);
        a = d = avg;
        if (b * c < 0.0) break;
    }
    if (any) {
        int slot = atomicAdd(count, 1);
        list[slot] = k;
        rc[k] = cst;
        rs[k] = snt;
        blk[4 * k + 0] = a;
        blk[4 * k + 1] = c;
        blk[4 * k + 2] = b;
        blk[4 * k + 3] = d;
    }
}

// stage 2: rows k,k+1 over columns k+2..n-1 (G^T from the left)
__global__ void k_fin_rows(double *H, int64_t ld, int n, const double *rc, const double *rs, const int *list,
                           const int *count)
{
    int cnt = *count;
    for (int e = blockIdx.y; e < cnt; e += gridDim.y) {
        int k = list[e];
        double cs = rc[k], sn = rs[k];
        for (int j = k + 2 + blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
            double x = H[k + (int64_t)j * ld], y = H[(k + 1) + (int64_t)j * ld];
            H[k + (int64_t)j * ld] = cs * x + sn * y;
            H[(k + 1) + (int64_t)j * ld] = -sn * x + cs * y;
        }
    }
}

// stage 3: columns k,k+1 over rows 0..k-1 of H and all rows of Q; block values
__global__ void k_fin_cols(double *H, int64_t ld, int n, double *Q, const double *rc, const double *rs,
                           const int *list, const int *count, const double *blk)
{
    int cnt = *count;
    for (int e = blockIdx.y; e < cnt; e += gridDim.y) {
        int k = list[e];
        double cs = rc[k], sn = rs[k];
        int rows = k + (Q ? n : 0);
        for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < rows; it += gridDim.x * blockDim.x) {
            double *M = (it < k) ? H + it : Q + (it - k);
            double x = M[(int64_t)k * ld], y = M[(int64_t)(k + 1) * ld];
            M[(int64_t)k * ld] = cs * x + sn * y;
            M[(int64_t)(k + 1) * ld] = -sn * x + cs * y;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            H[k + (int64_t)k * ld] = blk[4 * k + 0];
            H[(k + 1) + (int64_t)k * ld] = blk[4 * k + 1];
            H[k + (int64_t)(k + 1) * ld] = blk[4 * k + 2];
            H[(k + 1) + (int64_t)(k + 1) * ld] = blk[4 * k + 3];
        }
    }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

__global__ void k_zero_lower(double *H, int64_t ld, int n)
{
    int c = blockIdx.x;
    for (int r = c + 2 + threadIdx.x; r < n; r += blockDim.x) H[r + (int64_t)c * ld] = 0.0;
}

// non-finite entries anywhere in the n x n matrix (column per workgroup)
__global__ void k_check_finite_full(const double *A, int64_t ld, int n, int *flag)
{
    const int c = blockIdx.x;
    for (int r = threadIdx.x; r < n; r += blockDim.x)
        if (!isfinite(A[r + (int64_t)c * ld])) atomicOr(flag, 1);
}

__global__ void k_check_finite(const double *H, int64_t ld, int n, int *flag)
{
    int c = blockIdx.x;
    int rmax = min(c + 1, n - 1);
    for (int r = threadIdx.x; r <= rmax; r += blockDim.x) {
        double x = H[r + (int64_t)c * ld];
        if (!isfinite(x)) atomicOr(flag, 1);
    }
}

// Frobenius norm of the Hessenberg part: one workgroup per column writes the
// column's scaled sum of squares (scale = column max), then one workgroup
// combines them.  Exact zeros are skipped; no overflow for finite input.
__global__ void k_hess_fro_cols(const double *H, int64_t ld, int n, double *ws)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    const int rmax = min(c + 1, n - 1);
    double mx = 0.0;
    for (int r = threadIdx.x; r <= rmax; r += blockDim.x) mx = fmax(mx, fabs(H[r + (int64_t)c * ld]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    double ss = 0.0;
    if (mx > 0.0)
        for (int r = threadIdx.x; r <= rmax; r += blockDim.x) {
            const double x = H[r + (int64_t)c * ld] / mx;
            ss += x * x;
        }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ws[2 * c] = mx;
        ws[2 * c + 1] = red[0];
    }
}

__global__ void k_hess_fro_sum(const double *ws, int n, double *out)
{
    __shared__ double red[256];
    double mx = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) mx = fmax(mx, ws[2 * c]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    double ss = 0.0;
    if (mx > 0.0)
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            const double r = ws[2 * c] / mx;
            ss += ws[2 * c + 1] * r * r;
        }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = mx * sqrt(red[0]);
}

__global__ void k_transpose_pad(const double *V, int64_t ldv, int K, double *Ut, int K16)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)K16 * K16) return;
    int j = (int)(idx % K16), k = (int)(idx / K16);
    Ut[idx] = (j < K && k < K) ? V[k + (int64_t)j * ldv] : 0.0;
}

// ---------------------------------------------------------------------------
// launchers

static_assert(sizeof(Smem) <= 160 * 1024, "the LDS kernels need one workgroup's 160 KB of LDS at most");
static size_t smem_bytes() { return sizeof(Smem); }

// Dynamic-LDS limit of an LDS kernel, set once per (kernel, device) so that
// later launches (also under stream capture) make no attribute call.
static hipError_t prep(const void *fn)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &d : done)
        if (d.first == fn && d.second == dev) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_bytes());
    if (e == hipSuccess) done.emplace_back(fn, dev);
    return e;
}

hipError_t launch_iter(double *H, int64_t ld, int n, int ilo, int kbot, int nw, int nmin, Defl dfl,
                       int64_t itmax, double *Ut, IterStatus *st, hipStream_t s, int nsmall)
{
    hipError_t e = prep((const void *)k_iter);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_iter, dim3(1), dim3(NT), smem_bytes(), s, H, ld, n, ilo, kbot, nw, nmin, dfl,
                       itmax, Ut, st, nsmall);
    return hipGetLastError();
}

hipError_t launch_find_block(double *H, int64_t ld, int ilo, int kbot, Defl dfl, IterStatus *st,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_find_block, dim3(1), dim3(NT), 0, s, H, ld, ilo, kbot, dfl, st);
    return hipGetLastError();
}

hipError_t launch_chase(double *H, int64_t ld, const ChaseRound &r, const double *sr, const double *si,
                        Defl dfl, double *Ubuf, int64_t ustride, hipStream_t s)
{
    hipError_t e = prep((const void *)k_chase);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chase, dim3(r.nwin), dim3(CHASE_NT), smem_bytes(), s, H, ld, r, sr, si, dfl, Ubuf,
                       ustride);
    return hipGetLastError();
}

hipError_t launch_corner_deflate(double *T, int64_t ldt, int nw, int wd, const double *V, int64_t ldv,
                                 double s, Defl dfl, double *Ut, IterStatus *st, int nforced, int reorder,
                                 hipStream_t stream)
{
    hipError_t e = prep((const void *)k_corner_deflate);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_corner_deflate, dim3(1), dim3(NT), smem_bytes(), stream, T, ldt, nw, wd, V, ldv, s,
                       dfl, Ut, st, nforced, reorder);
    return hipGetLastError();
}

hipError_t launch_restore(double *T, int64_t ldt, int nw, int ns, double *V, int64_t ldv, int nv, double s,
                          double *work, IterStatus *st, hipStream_t stream)
{
    hipLaunchKernelGGL(k_restore_global, dim3(1), dim3(1024), 0, stream, T, ldt, nw, ns, V, ldv, nv, s, work,
                       st);
    return hipGetLastError();
}

hipError_t launch_window_copy(const double *H, int64_t ld, int kwtop, int nw, double *T, int64_t ldt,
                              double *V, int64_t ldv, hipStream_t s)
{
    int64_t tot = (int64_t)nw * nw;
    int blocks = (int)((tot + 255) / 256);
    hipLaunchKernelGGL(k_window_copy, dim3(blocks), dim3(256), 0, s, H, ld, kwtop, nw, T, ldt, V, ldv);
    return hipGetLastError();
}

hipError_t launch_block_eigs(const double *T, int64_t ldt, int m, double *wr, double *wi, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_eigs, dim3((m + 255) / 256), dim3(256), 0, s, T, ldt, m, wr, wi);
    return hipGetLastError();
}

hipError_t launch_check_finite_full(const double *A, int64_t ld, int n, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_finite_full, dim3(n), dim3(256), 0, s, A, ld, n, flag);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double *H, int64_t ld, int n, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_finite, dim3(n), dim3(256), 0, s, H, ld, n, flag);
    return hipGetLastError();
}

hipError_t launch_zero_lower(double *H, int64_t ld, int n, hipStream_t s)
{
    if (n < 3) return hipSuccess;
    hipLaunchKernelGGL(k_zero_lower, dim3(n), dim3(256), 0, s, H, ld, n);
    return hipGetLastError();
}

hipError_t launch_hess_fro(const double *H, int64_t ld, int n, double *ws, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_hess_fro_cols, dim3(n), dim3(256), 0, s, H, ld, n, ws);
    hipLaunchKernelGGL(k_hess_fro_sum, dim3(1), dim3(256), 0, s, ws, n, out);
    return hipGetLastError();
}

hipError_t launch_transpose_pad(const double *V, int64_t ldv, int K, double *Ut, int K16, hipStream_t s)
{
    int64_t tot = (int64_t)K16 * K16;
    hipLaunchKernelGGL(k_transpose_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, ldv, K, Ut,
                       K16);
    return hipGetLastError();
}

// Final standardization pass over the 2x2 blocks in rows lo..n-1 (lo > 0 when
// the rows above did not converge); ws holds 8n doubles of scratch.
hipError_t launch_finalize_ws(double *H, int64_t ld, int n, int lo, double *Q, double *wr, double *wi, double *ws,
                              hipStream_t s)
{
    double *rc = ws, *rs = ws + n, *blk = ws + 2 * (int64_t)n;
    int *list = reinterpret_cast<int *>(ws + 6 * (int64_t)n);
    int *count = reinterpret_cast<int *>(ws + 7 * (int64_t)n);
    int nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, count, 0);
    hipLaunchKernelGGL(k_fin_rot, dim3(nb), dim3(256), 0, s, H, ld, n, lo, rc, rs, list, count, blk);
    hipLaunchKernelGGL(k_fin_rows, dim3(nb, 64), dim3(256), 0, s, H, ld, n, rc, rs, list, count);
    hipLaunchKernelGGL(k_fin_cols, dim3((2 * n + 255) / 256, 64), dim3(256), 0, s, H, ld, n, Q, rc, rs, list,
                       count, blk);
    hipLaunchKernelGGL(k_block_eigs, dim3(nb), dim3(256), 0, s, H, ld, n, wr, wi);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched form: persistent grids fed from a work queue, one workgroup per matrix

// Eigenvalues of a finished quasi-triangular matrix (2x2 blocks standardized):
// one thread walks the diagonal.
__device__ void batched_eigs(const double *A, int lda, int n, double *er, double *ei)
{
    int k = 0;
    while (k < n) {
        bool two = (k + 1 < n && A[(k + 1) + (int64_t)k * lda] != 0.0);
        if (!two) {
            er[k] = A[k + (int64_t)k * lda];
            ei[k] = 0.0;
            k += 1;
        } else {
            double r1, i1, r2, i2;
            eig2x2(A[k + (int64_t)k * lda], A[k + (int64_t)(k + 1) * lda], A[(k + 1) + (int64_t)k * lda],
                   A[(k + 1) + (int64_t)(k + 1) * lda], r1, i1, r2, i2);
            if (i1 < 0.0) {
                double t = i1;
                i1 = i2;
                i2 = t;
            }
            er[k] = r1;
            ei[k] = i1;
            er[k + 1] = r2;
            ei[k + 1] = i2;
            k += 2;
        }
    }
}

// Next queue position for this workgroup (one atomic per matrix, broadcast
// through LDS).
__device__ __forceinline__ int queue_next(SmemCore &S, int32_t *head)
{
    if (threadIdx.x == 0) S.ic[7] = atomicAdd(head, 1);
    __syncthreads();
    const int k = S.ic[7];
    __syncthreads();
    return k;
}

constexpr int QBINS = 4096;
constexpr int QNT = 1024;
__device__ __forceinline__ int order_bin(int n) { return n <= 0 ? 0 : min(n, QBINS - 1); }

// Longest-first order of the batch: counting sort of the orders (one
// workgroup, bins in LDS), then the queue heads: q[0] = 0 for the orders
// above wide_n (positions [0, q[5])), q[4] = q[5] for the other orders of
// the global tier (positions [q[5], q[2])), q[1] = q[2] = number of orders
// above the LDS limit for the LDS tier (positions [q[2], q[3])), q[3] =
// number of positive orders.  Empty matrices (order <= 0, sorted last) are
// finished here.
__global__ void __launch_bounds__(QNT) k_batched_order(const int32_t *nn, int batch, int wide_n, int32_t *q,
                                                       int32_t *info)
{
    __shared__ int cnt[QBINS];
    __shared__ int part[QNT];
    const int tid = threadIdx.x;
    for (int b = tid; b < QBINS; b += QNT) cnt[b] = 0;
    __syncthreads();
    for (int i = tid; i < batch; i += QNT) atomicAdd(&cnt[order_bin(nn[i])], 1);
    __syncthreads();
    // thread t owns the four bins QBINS-1-4t .. QBINS-4-4t (counted from the top)
    int own = 0;
    for (int k = 0; k < 4; ++k) own += cnt[QBINS - 1 - (4 * tid + k)];
    part[tid] = own;
    __syncthreads();
    for (int off = 1; off < QNT; off <<= 1) {
        int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int base = part[tid] - own; // items in higher bins
    for (int k = 0; k < 4; ++k) {
        const int b = QBINS - 1 - (4 * tid + k);
        const int c = cnt[b];
        cnt[b] = base;
        base += c;
    }
    __syncthreads();
    const int nbig = cnt[MMAX];   // start of bin MMAX = number of orders above MMAX
    const int nwide = cnt[wide_n]; // number of orders above wide_n (MMAX <= wide_n < QBINS)
    const int npos = cnt[0];      // start of bin 0 = number of positive orders
    __syncthreads();
    int32_t *order = q + QHDR;
    for (int i = tid; i < batch; i += QNT) {
        const int pos = atomicAdd(&cnt[order_bin(nn[i])], 1);
        order[pos] = i;
        if (nn[i] <= 0) info[i] = 0;
    }
    if (tid == 0) {
        q[0] = 0;
        q[1] = nbig;
        q[2] = nbig;
        q[3] = npos;
        q[4] = nwide;
        q[5] = nwide;
    }
}

// Orders up to the LDS limit: double-shift solver with matrix and factor in
// LDS.  Bulge chains (more than 2 shifts) are switched off in the batched
// kernels: runs with them did not finish and the cause is not yet known.
__global__ void __launch_bounds__(NT) k_batched(double *H, double *Q, const int64_t *offs, const int32_t *nn,
                                                int batch, double *wr, double *wi, const int64_t *eoff,
                                                int32_t *info, int32_t *q)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const int tid = threadIdx.x;
    const int32_t *order = q + QHDR;
    const int npos = q[3];
    for (;;) {
        const int k = queue_next(S, &q[1]);
        if (k >= npos) break;
        const int b = order[k];
        const int n = nn[b];
        double *A = H + offs[b];
        for (int it = tid; it < n * n; it += NT) {
            int r = it % n, c = it / n;
            S.A[r + c * LDM] = (r <= c + 1) ? A[it] : 0.0;
        }
        identity_lds(S.Z, LDM, n, n);
        __syncthreads();
        const Defl dfl{DBL_MIN * ((double)n / kU), -1.0};
        int inf = qr_small(S, S.A, LDM, n, S.Z, LDM, n, dfl, 0, 2);
        __syncthreads();
        for (int it = tid; it < n * n; it += NT) {
            int r = it % n, c = it / n;
            A[it] = (r <= c + 1) ? S.A[r + c * LDM] : 0.0;
        }
        if (tid == 0) {
            batched_eigs(S.A, LDM, n, wr + eoff[b], wi + eoff[b]);
            info[b] = inf;
        }
        __syncthreads();
        if (Q) {
            // Q <- Q0 * Z: stage Q0 in the (now free) A buffer
            double *Qb = Q + offs[b];
            for (int it = tid; it < n * n; it += NT) {
                int r = it % n, c = it / n;
                S.A[r + c * LDM] = Qb[it];
            }
            __syncthreads();
            for (int it = tid; it < n * n; it += NT) {
                int r = it % n, c = it / n;
                double acc = 0.0;
                for (int kk = 0; kk < n; ++kk) acc += S.A[r + kk * LDM] * S.Z[kk + c * LDM];
                Qb[it] = acc;
            }
        }
        __syncthreads();
    }
}

// Orders above the LDS limit: the double-shift solver with the matrix and Q
// in global memory (L2 resident); small LDS footprint, two workgroups per CU.
__global__ void __launch_bounds__(NT) k_batched_global(double *H, double *Q, const int64_t *offs,
                                                       const int32_t *nn, int batch, double *wr, double *wi,
                                                       const int64_t *eoff, int32_t *info, int32_t *q)
{
    __shared__ SmemCore S;
    const int tid = threadIdx.x;
    const int32_t *order = q + QHDR;
    const int nbig = q[2], nwide = q[5];
    // the lower half of the grid takes the orders above wide_n first, then
    // joins the upper half on the rest
    bool wide = blockIdx.x < (gridDim.x + 1) / 2 && nwide > 0;
    for (;;) {
        int k;
        if (wide) {
            k = queue_next(S, &q[0]);
            if (k >= nwide) {
                wide = false;
                continue;
            }
        } else {
            k = queue_next(S, &q[4]);
            if (k >= nbig) break;
        }
        const int b = order[k];
        const int n = nn[b];
        double *A = H + offs[b];
        for (int it = tid; it < n * n; it += NT) {
            int r = it % n, c = it / n;
            if (r > c + 1) A[it] = 0.0;
        }
        double *Z = Q ? Q + offs[b] : A; // without Q: no Z rows (nz = 0)
        __syncthreads();
        const Defl dfl{DBL_MIN * ((double)n / kU), -1.0};
        int inf = qr_small(S, A, n, n, Z, n, Q ? n : 0, dfl, 0, 2);
        __syncthreads();
        if (tid == 0) {
            batched_eigs(A, n, n, wr + eoff[b], wi + eoff[b]);
            info[b] = inf;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// batched form with aggressive early deflation (orders above the LDS limit):
// H and Q stay in global memory, an LDS window of order <= BWIN holds the AED
// window and its factor.  Per matrix and size bucket: AED window nw and
// shifts per step ns (Sec. 2.5); the ns undeflated candidates nearest the
// bottom are used as ns/2 successive double-shift sweeps, which in exact
// arithmetic equal one sweep with a chain of ns/2 bulges (Sec. 2.3, implicit
// Q theorem).

constexpr int LDB = BWIN + 1;
constexpr int BNMIN = 75; // active blocks of at most this order finish with double shifts
struct SmemB : SmemCore {
    double A[BWIN * LDB];
    double Z[LDB * LDB];
    double vec[LDB];
    double cr[BWIN], ci[BWIN]; // candidate eigenvalues of the AED window
    double pr[BWIN], pi[BWIN]; // the shifts of the next sweeps, paired
};
static_assert(2 * sizeof(SmemB) <= 160 * 1024, "two AED workgroups per CU");

// X(0:rows, 0:nw) <- X Z for a panel in global memory (leading dimension ldx),
// row chunks staged through the LDS buffer buf (BWIN x LDB).
__device__ void bw_right(double *X, int64_t ldx, int rows, int nw, const double *Z, double *buf)
{
    for (int r0 = 0; r0 < rows; r0 += BWIN) {
        const int rc = min(BWIN, rows - r0);
        for (int it = threadIdx.x; it < rc * nw; it += NT) {
            const int r = it % rc, k = it / rc;
            buf[r + k * LDB] = X[(r0 + r) + (int64_t)k * ldx];
        }
        __syncthreads();
        for (int it = threadIdx.x; it < rc * nw; it += NT) {
            const int r = it % rc, j = it / rc;
            double a0 = 0.0, a1 = 0.0;
            int k = 0;
            for (; k + 1 < nw; k += 2) {
                a0 += buf[r + k * LDB] * Z[k + j * LDB];
                a1 += buf[r + (k + 1) * LDB] * Z[(k + 1) + j * LDB];
            }
            if (k < nw) a0 += buf[r + k * LDB] * Z[k + j * LDB];
            X[(r0 + r) + (int64_t)j * ldx] = a0 + a1;
        }
        __syncthreads();
    }
}

// X(0:nw, 0:cols) <- Z^T X for a panel in global memory.
__device__ void bw_left(double *X, int64_t ldx, int cols, int nw, const double *Z, double *buf)
{
    for (int c0 = 0; c0 < cols; c0 += BWIN) {
        const int cc = min(BWIN, cols - c0);
        for (int it = threadIdx.x; it < cc * nw; it += NT) {
            const int k = it % nw, c = it / nw;
            buf[k + c * LDB] = X[k + (int64_t)(c0 + c) * ldx];
        }
        __syncthreads();
        for (int it = threadIdx.x; it < cc * nw; it += NT) {
            const int j = it % nw, c = it / nw;
            double a0 = 0.0, a1 = 0.0;
            int k = 0;
            for (; k + 1 < nw; k += 2) {
                a0 += Z[k + j * LDB] * buf[k + c * LDB];
                a1 += Z[(k + 1) + j * LDB] * buf[(k + 1) + c * LDB];
            }
            if (k < nw) a0 += Z[k + j * LDB] * buf[k + c * LDB];
            X[j + (int64_t)(c0 + c) * ldx] = a0 + a1;
        }
        __syncthreads();
    }
}

// One matrix of order n (leading dimension n) in global memory, Q (may be
// NULL) accumulated: AED steps with window nwb and up to nsb shifts, double
// shifts once the active block is small (or after three AED steps without a
// deflation).  Returns 0 or the failure code of the small solver / the
// iteration limit (1-based row).
__device__ __forceinline__ int batched_aed_solve(SmemB &S, double *A, int n, double *Q, int nwb, int nsb, const Defl &dfl)
{
    const int nz = Q ? n : 0;
    double *Z = Q ? Q : A; // without Q: no Z rows (nz = 0)
    const int64_t itmax = 30 * (int64_t)max(10, n);
    int64_t iters = 0;
    int kbot = n - 1, nodefl = 0;
    while (kbot >= 0) {
        const int ktop = find_split(S, A, n, 0, kbot, dfl);
        const int nh = kbot - ktop + 1;
        if (nh <= BNMIN || nodefl >= 3) {
            const int inf = qr_ds(S, A, n, n, Z, n, nz, dfl, 0, ktop, kbot);
            if (inf > 0) return inf;
            kbot = ktop - 1;
            nodefl = 0;
            continue;
        }
        if (++iters > itmax) return kbot + 1;
        const int nw = min(nwb, nh);
        const int kw = kbot - nw + 1;
        const double s = (kw > ktop) ? A[kw + (int64_t)(kw - 1) * n] : 0.0;
        for (int it = threadIdx.x; it < nw * nw; it += NT) {
            const int r = it % nw, c = it / nw;
            S.A[r + c * LDB] = (r <= c + 1) ? A[(kw + r) + (int64_t)(kw + c) * n] : 0.0;
        }
        identity_lds(S.Z, LDB, nw, nw);
        __syncthreads();
        const int winf = qr_ds(S, S.A, LDB, nw, S.Z, LDB, nw, dfl, 0);
        const int ns = aed_deflate(S, S.A, LDB, nw, S.Z, LDB, nw, 0, s, winf > 0 ? winf : 0, dfl);
        const int nd = nw - ns;
        if (threadIdx.x == 0) {
            // candidates: eigenvalues of the undeflated blocks in diagonal order
            int k = 0;
            while (k < ns) {
                const int sz = (k + 1 < ns && S.A[(k + 1) + k * LDB] != 0.0) ? 2 : 1;
                if (sz == 1) {
                    S.cr[k] = S.A[k + k * LDB];
                    S.ci[k] = 0.0;
                } else {
                    double r1, i1, r2, i2;
                    eig2x2(S.A[k + k * LDB], S.A[k + (k + 1) * LDB], S.A[(k + 1) + k * LDB],
                           S.A[(k + 1) + (k + 1) * LDB], r1, i1, r2, i2);
                    if (i1 < 0.0) {
                        const double t = i1;
                        i1 = i2;
                        i2 = t;
                    }
                    S.cr[k] = r1;
                    S.ci[k] = i1;
                    S.cr[k + 1] = r2;
                    S.ci[k + 1] = i2;
                }
                k += sz;
            }
            // the bottommost min(nsb, ns) candidates, conjugate pairs together,
            // real ones paired in order, an odd real one left over dropped
            const int want = min(nsb, ns);
            int start = ns - want;
            if (start > 0 && start < ns && S.ci[start] < 0.0) start++;
            int nsh = 0, nr = 0;
            double rr = 0.0;
            for (int i = ns - 1; i >= start; --i) {
                if (S.ci[i] != 0.0) {
                    if (S.ci[i] < 0.0 && i - 1 >= start) {
                        S.pr[nsh] = S.cr[i - 1];
                        S.pi[nsh] = S.ci[i - 1];
                        S.pr[nsh + 1] = S.cr[i];
                        S.pi[nsh + 1] = S.ci[i];
                        nsh += 2;
                        --i;
                    }
                } else if (nr == 0) {
                    rr = S.cr[i];
                    nr = 1;
                } else {
                    S.pr[nsh] = rr;
                    S.pi[nsh] = 0.0;
                    S.pr[nsh + 1] = S.cr[i];
                    S.pi[nsh + 1] = 0.0;
                    nsh += 2;
                    nr = 0;
                }
            }
            S.ic[5] = nsh;
        }
        __syncthreads();
        const int nsh = S.ic[5];
        if (nd > 0) {
            double beta = 0.0;
            if (ns >= 1) beta = s * S.Z[0];
            if (ns > 1 && s != 0.0) beta = restore_lds(S, S.A, LDB, nw, ns, S.Z, LDB, nw, 0, s);
            for (int it = threadIdx.x; it < nw * nw; it += NT) {
                const int r = it % nw, c = it / nw;
                A[(kw + r) + (int64_t)(kw + c) * n] = (r <= c + 1) ? S.A[r + c * LDB] : 0.0;
            }
            if (kw > ktop && threadIdx.x == 0) A[kw + (int64_t)(kw - 1) * n] = (ns >= 1) ? beta : 0.0;
            __syncthreads();
            // the window's factor on the rows above it, the columns right of
            // the active block and Q (S.A is free now and stages the panels)
            bw_right(A + (int64_t)kw * n, n, kw, nw, S.Z, S.A);
            bw_left(A + kw + (int64_t)(kbot + 1) * n, n, n - kbot - 1, nw, S.Z, S.A);
            if (Q) bw_right(Q + (int64_t)kw * n, n, n, nw, S.Z, S.A);
            kbot -= nd;
            nodefl = 0;
            if (100 * nd > 14 * nw) continue; // many deflations: AED again
        } else {
            ++nodefl;
        }
        if (kbot - ktop + 1 <= BNMIN) continue;
        for (int p = 0; p + 1 < nsh; p += 2) {
            if (threadIdx.x == 0) {
                S.sr[0] = S.pr[p];
                S.si[0] = S.pi[p];
                S.sr[1] = S.pr[p + 1];
                S.si[1] = S.pi[p + 1];
            }
            __syncthreads();
            chase_la(S, A, n, ktop, kbot, n - 1, Z, n, nz);
        }
    }
    return 0;
}

// Orders above the LDS limit with a per-bucket (nw, ns) table: matrices of
// buckets with an AED window solve with batched_aed_solve, the others with
// double shifts as in k_batched_global.  Same work queue as k_batched_global.
__global__ void __launch_bounds__(NT) k_batched_aed(double *H, double *Q, const int64_t *offs, const int32_t *nn,
                                                    int batch, double *wr, double *wi, const int64_t *eoff,
                                                    int32_t *info, int32_t *q, BatchedTable tab)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SmemB &S = *reinterpret_cast<SmemB *>(smem_raw);
    const int tid = threadIdx.x;
    const int32_t *order = q + QHDR;
    const int nbig = q[2], nwide = q[5];
    bool wide = blockIdx.x < (gridDim.x + 1) / 2 && nwide > 0;
    for (;;) {
        int k;
        if (wide) {
            k = queue_next(S, &q[0]);
            if (k >= nwide) {
                wide = false;
                continue;
            }
        } else {
            k = queue_next(S, &q[4]);
            if (k >= nbig) break;
        }
        const int b = order[k];
        const int n = nn[b];
        double *A = H + offs[b];
        for (int it = tid; it < n * n; it += NT) {
            int r = it % n, c = it / n;
            if (r > c + 1) A[it] = 0.0;
        }
        int bk = 0;
        while (bk + 1 < tab.nb && n > tab.upper[bk]) ++bk;
        const int nwb = min(tab.nw[bk], BWIN), nsb = tab.ns[bk] & ~1;
        double *Qb = Q ? Q + offs[b] : nullptr;
        __syncthreads();
        const Defl dfl{DBL_MIN * ((double)n / kU), -1.0};
        int inf;
        if (nwb >= 8 && nsb >= 2)
            inf = batched_aed_solve(S, A, n, Qb, nwb, nsb, dfl);
        else
            inf = qr_small(S, A, n, n, Qb ? Qb : A, n, Qb ? n : 0, dfl, 0, 2);
        __syncthreads();
        if (tid == 0) {
            batched_eigs(A, n, n, wr + eoff[b], wi + eoff[b]);
            info[b] = inf;
        }
        __syncthreads();
    }
}

// Sequential AED of a window too large for the LDS solver (Sec. 3.5,
// "Adaptive approach": the variant one worker runs alone): one workgroup
// reduces the window copy T (order w, leading dimension w, zeros below the
// subdiagonal) to Schur form with V (= I on entry) accumulating, by the
// batched form's per-matrix solver (its own small AED windows in LDS, nwb and
// nsb), then examines every candidate bottom-up against the spike s V(0, :)
// and moves the failures to the top (the pipelined reordering, here in global
// memory).  st->ns = undeflated leading rows, st->nd = w - ns, st->info > 0
// when the Schur reduction stopped at its iteration limit (the rows above it
// then count as undeflated).
__global__ void __launch_bounds__(NT) k_seq_aed(double *T, int w, double *V, double s, Defl dfl, int nwb, int nsb,
                                                IterStatus *st)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SmemB &S = *reinterpret_cast<SmemB *>(smem_raw);
    if (threadIdx.x == 0) {
        S.flops = 0.0;
        S.nphase = S.nbstep = S.nswap = S.nrphase = 0;
    }
    __syncthreads();
    const int info = batched_aed_solve(S, T, w, V, nwb, nsb, dfl);
    __syncthreads();
    const int ns = aed_deflate(S, T, w, w, V, w, w, 0, s, info > 0 ? info : 0, dfl);
    if (threadIdx.x == 0) {
        st->ns = ns;
        st->nd = w - ns;
        st->info = info;
        st->kwtop = 0;
        st->nw = w;
        st->nswap = S.nswap;
        st->nrphase = S.nrphase;
    }
}

hipError_t launch_seq_aed(double *T, int w, double *V, double s, Defl dfl, int nwb, int nsb, IterStatus *st,
                          hipStream_t strm)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_seq_aed, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sizeof(SmemB));
        if (e != hipSuccess) return e;
        attr = true;
    }
    nwb = std::min(std::max(nwb, 8), BWIN);
    nsb = std::max(2, nsb & ~1);
    hipLaunchKernelGGL(k_seq_aed, dim3(1), dim3(NT), sizeof(SmemB), strm, T, w, V, s, dfl, nwb, nsb, st);
    return hipGetLastError();
}

hipError_t launch_batched(double *H, double *Q, const int64_t *offsets, const int32_t *n, int batch, double *wr,
                          double *wi, const int64_t *eoff, int32_t *info, int32_t *queue, int wg_per_cu, int wide_n,
                          const BatchedTable &tab, hipStream_t s)
{
    hipError_t e = prep((const void *)k_batched);
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    ncu = std::max(ncu, 1);
    wide_n = std::min(std::max(wide_n, MMAX), QBINS - 1);
    wg_per_cu = std::min(std::max(wg_per_cu, 1), 8);
    hipLaunchKernelGGL(k_batched_order, dim3(1), dim3(QNT), 0, s, n, batch, wide_n, queue, info);
    // orders > MMAX first (they dominate the time), then the LDS tier; each
    // grid drains its queue longest-first
    bool aed = false;
    for (int i = 0; i < tab.nb; ++i) aed = aed || (tab.upper[i] > MMAX && tab.nw[i] >= 8 && tab.ns[i] >= 2);
    if (aed) {
        static bool attr = false;
        if (!attr) {
            e = hipFuncSetAttribute((const void *)k_batched_aed, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)sizeof(SmemB));
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL(k_batched_aed, dim3(std::min(batch, wg_per_cu * ncu)), dim3(NT), sizeof(SmemB), s, H, Q,
                           offsets, n, batch, wr, wi, eoff, info, queue, tab);
    } else {
        hipLaunchKernelGGL(k_batched_global, dim3(std::min(batch, wg_per_cu * ncu)), dim3(NT), 0, s, H, Q, offsets,
                           n, batch, wr, wi, eoff, info, queue);
    }
    hipLaunchKernelGGL(k_batched, dim3(std::min(batch, ncu)), dim3(NT), smem_bytes(), s, H, Q, offsets, n, batch,
                       wr, wi, eoff, info, queue);
    return hipGetLastError();
}

} // namespace hqr
