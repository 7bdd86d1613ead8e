// QZ variant of libhqr for small Hessenberg-triangular pairs (gfx950).
//
// The generalized problem (Sec. 2, remarks on the generalized case): a pair
// (H, T), H upper Hessenberg and T upper triangular, is reduced to the
// generalized real Schur form (S, T') = Q^T (H, T) Z, S quasi upper
// triangular (2x2 blocks only for complex conjugate pairs), T' upper
// triangular; the generalized eigenvalues are (alphar + i alphai) / beta,
// beta = 0 for an infinite eigenvalue.  Double implicit shift QZ: the first
// column of (H T^{-1} - s1)(H T^{-1} - s2) introduces the bulge; a 3x3
// reflector from the left moves the 2x2 bulge of H down while reflectors from
// the right restore the triangularity of T (its 1x1 bulge moves along).
// Diagonal entries of T with |t_kk| <= u ||T||_F count as zero (the paper's
// convention); such an infinite eigenvalue is chased up to the top of its
// block with rotations and deflated there (the 'push infinities' task of
// Sec. 3.2).
//
// One workgroup per pair, the pair and its Q and Z held in LDS (order <= 64,
// four 64 x 65 arrays, 133 KB).  Thread 0 forms each transformation (a 2x2 or
// 3x3 orthogonal matrix) in LDS; all threads then apply it to the rows of H
// and T and the columns of Q (left) or to the columns of H, T and Z (right),
// one row or column per thread.
#include "hqr_common.h"
#include <algorithm>
#include <cfloat>
#include <climits>

namespace hqr {

constexpr int QZMAX = 64;
constexpr int LDQZ = QZMAX + 1;
constexpr double kUq = 2.220446049250313080847e-16; // unit roundoff 2^-52

// Control block of a workgroup: the transformation thread 0 formed and its
// decisions.
struct QZCtl {
    double G[9];  // the transformation to apply (row major, m x m)
    double x[3];  // vector that defines the next reflector
    int ic[8];    // decisions of thread 0: action, l, kz, i, its
    double sc[8]; // scalars of thread 0: shifts, thresholds
    int lsplit, kzero;  // top of the active block, first zero diagonal entry of T in it
    double red[NT];     // per-thread partial norms
};

// Pairs of order <= QZMAX: H, T, Q and Z in LDS.
struct SmemQZ : QZCtl {
    double H[QZMAX * LDQZ], T[QZMAX * LDQZ], Q[QZMAX * LDQZ], Z[QZMAX * LDQZ];
};

// Where the pair and its factors live: LDS (leading dimension LDQZ) or the
// caller's global arrays (leading dimension n); Q or Z may be null in global
// memory (not accumulated).
struct QZV {
    double *H, *T, *Q, *Z;
    int ld;
};

// ---- thread-0 scalar helpers ----------------------------------------------

// Reflector P = I - tau v v^T, v[0] = 1, P x = beta e_0 (beta = -sign(x0)||x||;
// identity when the tail is zero).
__device__ __forceinline__ void qz_house(int m, const double *x, double *v, double &tau, double &beta)
{
    double amax = 0.0;
    for (int i = 1; i < m; ++i) amax = fmax(amax, fabs(x[i]));
    v[0] = 1.0;
    for (int i = 1; i < m; ++i) v[i] = 0.0;
    if (amax == 0.0) {
        tau = 0.0;
        beta = x[0];
        return;
    }
    double s = 0.0;
    for (int i = 1; i < m; ++i) s += (x[i] / amax) * (x[i] / amax);
    const double nrm = hypot(x[0], amax * sqrt(s));
    const double b = (x[0] >= 0.0) ? -nrm : nrm;
    tau = (b - x[0]) / b;
    const double sc = 1.0 / (x[0] - b);
    for (int i = 1; i < m; ++i) v[i] = x[i] * sc;
    beta = b;
}

// G = I - tau v v^T (m x m) into S.G.
__device__ __forceinline__ void qz_set_house(QZCtl &S, int m, const double *v, double tau)
{
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            S.G[i * 3 + k] = (i < m && k < m) ? ((i == k ? 1.0 : 0.0) - tau * v[i] * v[k]) : 0.0;
}

// Reflector acting from the right on a row vector w (length m): w P = gamma e_{m-1}.
__device__ __forceinline__ void qz_set_house_last(QZCtl &S, int m, const double *w)
{
    double wr[3], vr[3], v[3], tau, beta;
    for (int i = 0; i < m; ++i) wr[i] = w[m - 1 - i];
    qz_house(m, wr, vr, tau, beta);
    for (int i = 0; i < m; ++i) v[i] = vr[m - 1 - i];
    qz_set_house(S, m, v, tau);
}

// 2x2 matrix [[a, b], [c, d]] into S.G.
__device__ __forceinline__ void qz_set2(QZCtl &S, double a, double b, double c, double d)
{
    for (int q = 0; q < 9; ++q) S.G[q] = 0.0;
    S.G[0] = a;
    S.G[1] = b;
    S.G[3] = c;
    S.G[4] = d;
}

// (c, s) with c = a / r, s = b / r (identity for a zero vector).
__device__ __forceinline__ void qz_cs(double a, double b, double &c, double &s)
{
    const double r = hypot(a, b);
    if (r == 0.0) {
        c = 1.0;
        s = 0.0;
    } else {
        c = a / r;
        s = b / r;
    }
}

// Eigenvalues of the 2x2 pair at (k, k+1): those of A B^{-1}.
__device__ __forceinline__ void qz_eig2(const QZV &M, int k, double &r1, double &i1, double &r2, double &i2)
{
    const double *H = M.H, *T = M.T;
    const double a11 = H[k + k * M.ld], a12 = H[k + (k + 1) * M.ld];
    const double a21 = H[(k + 1) + k * M.ld], a22 = H[(k + 1) + (k + 1) * M.ld];
    const double b11 = T[k + k * M.ld], b12 = T[k + (k + 1) * M.ld], b22 = T[(k + 1) + (k + 1) * M.ld];
    const double m11 = a11 / b11, m21 = a21 / b11;
    const double m12 = (a12 - m11 * b12) / b22, m22 = (a22 - m21 * b12) / b22;
    const double p = 0.5 * (m11 - m22);
    const double sc = fmax(fabs(p), fmax(fabs(m12), fabs(m21)));
    const double mid = 0.5 * (m11 + m22);
    if (sc == 0.0) {
        r1 = m11;
        r2 = m22;
        i1 = i2 = 0.0;
        return;
    }
    const double disc = (p / sc) * (p / sc) + (m12 / sc) * (m21 / sc);
    if (disc >= 0.0) {
        const double r = sc * sqrt(disc);
        r1 = mid + r;
        r2 = mid - r;
        i1 = i2 = 0.0;
    } else {
        const double w = sc * sqrt(-disc);
        r1 = r2 = mid;
        i1 = w;
        i2 = -w;
    }
}

// ---- block-level application --------------------------------------------

// Applies S.G (formed by thread 0 before the call) from the left to rows
// p..p+m-1 of H and T (side 0, Q <- Q G^T) or from the right to columns
// p..p+m-1 of H, T and Z (side 1).
__device__ __forceinline__ void qz_apply(QZCtl &S, const QZV &M, int n, int side, int p, int m)
{
    __syncthreads();
    double g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = S.G[q];
    for (int it = threadIdx.x; it < 3 * n; it += NT) {
        const int which = it / n, r = it - which * n;
        double x[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
        if (side == 0 && which < 2) {
            double *A = which == 0 ? M.H : M.T; // column r of A, rows p..p+m-1
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < m) x[k] = A[(p + k) + r * M.ld];
#pragma unroll
            for (int i = 0; i < 3; ++i) y[i] = g[i * 3] * x[0] + g[i * 3 + 1] * x[1] + g[i * 3 + 2] * x[2];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < m) A[(p + i) + r * M.ld] = y[i];
        } else {
            double *A = side == 0 ? M.Q : (which == 0 ? M.H : (which == 1 ? M.T : M.Z)); // row r
            if (A == nullptr) continue; // factor not accumulated
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < m) x[k] = A[r + (p + k) * M.ld];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                y[j] = (side == 0) ? (x[0] * g[j * 3] + x[1] * g[j * 3 + 1] + x[2] * g[j * 3 + 2])
                                   : (x[0] * g[j] + x[1] * g[3 + j] + x[2] * g[6 + j]);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (j < m) A[r + (p + j) * M.ld] = y[j];
        }
    }
    __syncthreads();
}

// Zero diagonal entries of T below the threshold in [lo, hi].
__device__ __forceinline__ void qz_threshold(const QZV &M, int lo, int hi, double btol)
{
    for (int k = lo + (int)threadIdx.x; k <= hi; k += NT)
        if (fabs(M.T[k + k * M.ld]) <= btol) M.T[k + k * M.ld] = 0.0;
    __syncthreads();
}

// Chase the zero at T[kz,kz] to T[l,l] and deflate it there (H[l+1,l] = 0).
__device__ __forceinline__ void qz_push_up(QZCtl &S, const QZV &M, int n, int l, int i, int kz)
{
    const int tid = threadIdx.x;
    for (int jc = kz; jc > l; --jc) {
        if (tid == 0) {
            double c, s;
            qz_cs(M.T[(jc - 1) + jc * M.ld], M.T[(jc - 1) + (jc - 1) * M.ld], c, s);
            qz_set2(S, c, s, -s, c); // columns (jc-1, jc)
        }
        qz_apply(S, M, n, 1, jc - 1, 2);
        if (tid == 0) M.T[(jc - 1) + (jc - 1) * M.ld] = 0.0;
        if (jc + 1 <= i) {
            if (tid == 0) {
                double c, s;
                qz_cs(M.H[jc + (jc - 1) * M.ld], M.H[(jc + 1) + (jc - 1) * M.ld], c, s);
                qz_set2(S, c, s, -s, c); // rows (jc, jc+1)
            }
            qz_apply(S, M, n, 0, jc, 2);
            if (tid == 0) M.H[(jc + 1) + (jc - 1) * M.ld] = 0.0;
        }
    }
    if (tid == 0) {
        double c, s;
        qz_cs(M.H[l + l * M.ld], M.H[(l + 1) + l * M.ld], c, s);
        qz_set2(S, c, s, -s, c);
    }
    qz_apply(S, M, n, 0, l, 2);
    if (tid == 0) M.H[(l + 1) + l * M.ld] = 0.0;
    __syncthreads();
}

// Split a 2x2 block at (k, k+1) with the real eigenvalue lam.
__device__ __forceinline__ void qz_split2(QZCtl &S, const QZV &M, int n, int k, double lam)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        const double *H = M.H, *T = M.T;
        const double m11 = H[k + k * M.ld] - lam * T[k + k * M.ld];
        const double m12 = H[k + (k + 1) * M.ld] - lam * T[k + (k + 1) * M.ld];
        const double m21 = H[(k + 1) + k * M.ld];
        const double m22 = H[(k + 1) + (k + 1) * M.ld] - lam * T[(k + 1) + (k + 1) * M.ld];
        double z1, z2;
        if (hypot(m11, m12) >= hypot(m21, m22)) {
            z1 = -m12;
            z2 = m11;
        } else {
            z1 = -m22;
            z2 = m21;
        }
        double c, s;
        qz_cs(z1, z2, c, s);
        qz_set2(S, c, -s, s, c); // first column (c, s) spans the null vector
    }
    qz_apply(S, M, n, 1, k, 2);
    if (tid == 0) {
        double c, s;
        qz_cs(M.T[k + k * M.ld], M.T[(k + 1) + k * M.ld], c, s);
        qz_set2(S, c, s, -s, c);
    }
    qz_apply(S, M, n, 0, k, 2);
    if (tid == 0) {
        M.H[(k + 1) + k * M.ld] = 0.0;
        M.T[(k + 1) + k * M.ld] = 0.0;
    }
    __syncthreads();
}

// One double-shift sweep over [l, i] (i - l >= 2), shifts in S.sc[0..3].
__device__ __forceinline__ void qz_sweep(QZCtl &S, const QZV &M, int n, int l, int i)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        const double re1 = S.sc[0], im1 = S.sc[1], re2 = S.sc[2], im2 = S.sc[3];
        const double sum = re1 + re2, prod = re1 * re2 - im1 * im2;
        const double *H = M.H, *T = M.T;
        const double t11 = T[l + l * M.ld], t12 = T[l + (l + 1) * M.ld], t22 = T[(l + 1) + (l + 1) * M.ld];
        const double h11 = H[l + l * M.ld], h21 = H[(l + 1) + l * M.ld], h12 = H[l + (l + 1) * M.ld];
        const double h22 = H[(l + 1) + (l + 1) * M.ld], h32 = H[(l + 2) + (l + 1) * M.ld];
        const double ne0 = h11 / t11, ne1 = h21 / t11;
        const double y2 = ne1 / t22, y1 = (ne0 - t12 * y2) / t11;
        S.x[0] = h11 * y1 + h12 * y2 - sum * ne0 + prod;
        S.x[1] = h21 * y1 + h22 * y2 - sum * ne1;
        S.x[2] = h32 * y2;
    }
    for (int k = l - 1; k <= i - 2; ++k) {
        const int m = min(3, i - k);
        if (tid == 0) {
            double x[3], v[3], tau, beta;
            for (int r = 0; r < m; ++r) x[r] = (k >= l) ? M.H[(k + 1 + r) + k * M.ld] : S.x[r];
            qz_house(m, x, v, tau, beta);
            qz_set_house(S, m, v, tau);
            S.sc[4] = beta;
        }
        qz_apply(S, M, n, 0, k + 1, m);
        if (tid == 0) {
            if (k >= l) {
                M.H[(k + 1) + k * M.ld] = S.sc[4];
                for (int r = 1; r < m; ++r) M.H[(k + 1 + r) + k * M.ld] = 0.0;
            }
            double w[3];
            for (int r = 0; r < m; ++r) w[r] = M.T[(k + m) + (k + 1 + r) * M.ld];
            qz_set_house_last(S, m, w);
        }
        qz_apply(S, M, n, 1, k + 1, m);
        if (tid == 0) {
            for (int r = 0; r < m - 1; ++r) M.T[(k + m) + (k + 1 + r) * M.ld] = 0.0;
            if (m == 3) {
                double w[2] = {M.T[(k + 2) + (k + 1) * M.ld], M.T[(k + 2) + (k + 2) * M.ld]};
                qz_set_house_last(S, 2, w);
            }
        }
        if (m == 3) {
            qz_apply(S, M, n, 1, k + 1, 2);
            if (tid == 0) M.T[(k + 2) + (k + 1) * M.ld] = 0.0;
        }
        __syncthreads();
    }
}

// Actions decided by thread 0 each round.
enum { QZ_DONE = 0, QZ_PUSH = 1, QZ_ONE = 2, QZ_TWO = 3, QZ_SWEEP = 4, QZ_FAIL = 5 };

// One pair of order n in the view M, reduced in place; the eigenvalues go to
// ar, ai, be.  Returns 0, or 1 + the row at which the iteration limit
// stopped the reduction.
__device__ __forceinline__ int qz_solve(QZCtl &S, const QZV &M, int n, double *ar, double *ai, double *be)
{
    const int tid = threadIdx.x;
    // ||T||_F of the input's triangle (Sec. 2: |t_kk| <= u ||T||_F is
    // infinite): per-thread partial norms, combined by thread 0
    double tp = 0.0;
    for (int it = tid; it < n * n; it += NT) {
        const int r = it % n, c = it / n;
        if (r <= c) tp = hypot(tp, M.T[r + c * M.ld]);
    }
    S.red[tid] = tp;
    __syncthreads();
    if (tid == 0) {
        double tn = 0.0;
        for (int t = 0; t < NT; ++t) tn = hypot(tn, S.red[t]);
        S.sc[5] = kUq * tn;
        S.sc[6] = DBL_MIN * ((double)n / kUq);
        S.ic[3] = n - 1; // i
        S.ic[4] = 0;     // iterations since the last deflation
        S.ic[5] = 0;     // iterations
    }
    __syncthreads();
    const double btol = S.sc[5], smlnum = S.sc[6];
    const int64_t itmax = 30 * (int64_t)max(10, n);
    qz_threshold(M, 0, n - 1, btol);
    int result = 0;
    for (;;) {
        // the top l of the active block ending at row i (its last negligible
        // subdiagonal entry, 0 if none) and the first zero diagonal entry of
        // T in [l, i], both searched by all threads
        const int i0 = S.ic[3];
        if (tid == 0) {
            S.lsplit = 0;
            S.kzero = INT_MAX;
        }
        __syncthreads();
        for (int l = i0 - tid; l > 0; l -= NT) {
            const double h = fabs(M.H[l + (l - 1) * M.ld]);
            const double tst = fabs(M.H[(l - 1) + (l - 1) * M.ld]) + fabs(M.H[l + l * M.ld]);
            if (h <= fmax(smlnum, kUq * tst)) {
                atomicMax(&S.lsplit, l);
                break;
            }
        }
        __syncthreads();
        for (int k = S.lsplit + tid; k <= i0; k += NT)
            if (M.T[k + k * M.ld] == 0.0) {
                atomicMin(&S.kzero, k);
                break;
            }
        __syncthreads();
        if (tid == 0) {
            const int i = __builtin_amdgcn_readfirstlane(S.ic[3]);
            int act = QZ_DONE, l = 0, kz = -1;
            if (i >= 0) {
                l = S.lsplit;
                if (l > 0) M.H[l + (l - 1) * M.ld] = 0.0;
                kz = (S.kzero == INT_MAX) ? -1 : S.kzero;
                // The decision inputs are moved to scalar registers first:
                // this compiler lowered the select of the action below to
                // a scalar select on a stale condition code while the
                // comparison itself was a vector compare (measured: every
                // sweep was reported as the iteration limit).
                l = __builtin_amdgcn_readfirstlane(l);
                kz = __builtin_amdgcn_readfirstlane(kz);
                const int cnt = __builtin_amdgcn_readfirstlane(S.ic[5]);
                if (kz >= 0 && l < i) act = QZ_PUSH;
                else if (l == i) act = QZ_ONE;
                else if (l == i - 1) act = QZ_TWO;
                else if (cnt >= itmax) act = QZ_FAIL;
                else act = QZ_SWEEP;
            }
            S.ic[0] = act;
            S.ic[1] = l;
            S.ic[2] = kz;
            if (act == QZ_ONE) {
                double a = M.H[i + i * M.ld], bt = M.T[i + i * M.ld];
                if (bt < 0.0) {
                    a = -a;
                    bt = -bt;
                }
                ar[i] = a;
                ai[i] = 0.0;
                be[i] = bt;
                S.ic[3] = i - 1;
                S.ic[4] = 0;
            } else if (act == QZ_TWO) {
                double r1, i1, r2, i2;
                qz_eig2(M, i - 1, r1, i1, r2, i2);
                S.sc[0] = r1;
                S.ic[7] = (i1 == 0.0) ? 1 : 0; // real pair: split the block
                if (i1 != 0.0) {
                    ar[i - 1] = r1;
                    ai[i - 1] = fabs(i1);
                    be[i - 1] = 1.0;
                    ar[i] = r2;
                    ai[i] = -fabs(i1);
                    be[i] = 1.0;
                    S.ic[3] = i - 2;
                    S.ic[4] = 0;
                }
            } else if (act == QZ_SWEEP) {
                double r1, i1, r2, i2;
                const int its = S.ic[4];
                if (its == 10 || its == 20) {
                    const double ss = fabs(M.H[i + (i - 1) * M.ld] / M.T[(i - 1) + (i - 1) * M.ld]) +
                                      fabs(M.H[(i - 1) + (i - 2) * M.ld] / M.T[(i - 2) + (i - 2) * M.ld]);
                    r1 = r2 = M.H[i + i * M.ld] / M.T[i + i * M.ld] + 0.75 * ss;
                    i1 = i2 = 0.0;
                } else {
                    qz_eig2(M, i - 1, r1, i1, r2, i2);
                    if (i1 == 0.0) {
                        const double tb = M.H[i + i * M.ld] / M.T[i + i * M.ld];
                        const double pick = (fabs(r1 - tb) <= fabs(r2 - tb)) ? r1 : r2;
                        r1 = r2 = pick;
                    }
                }
                S.sc[0] = r1;
                S.sc[1] = i1;
                S.sc[2] = r2;
                S.sc[3] = i2;
                S.ic[4] = its + 1;
                S.ic[5] += 1;
            }
        }
        __syncthreads();
        const int act = S.ic[0], l = S.ic[1], kz = S.ic[2];
        const int i = (act == QZ_SWEEP || act == QZ_PUSH || act == QZ_TWO) ? S.ic[3] : -1;
        const int split = S.ic[7];
        const double lam = S.sc[0];
        __syncthreads();
        if (act == QZ_DONE) break;
        if (act == QZ_FAIL) {
            result = S.ic[3] + 1;
            break;
        }
        if (act == QZ_PUSH) {
            qz_push_up(S, M, n, l, i, kz);
            qz_threshold(M, l + 1, i, btol);
            if (tid == 0) S.ic[4] = 0;
        } else if (act == QZ_TWO && split) {
            qz_split2(S, M, n, i - 1, lam);
        } else if (act == QZ_SWEEP) {
            qz_sweep(S, M, n, l, i);
            qz_threshold(M, l, i, btol);
        }
        __syncthreads();
    }
    __syncthreads();
    return result;
}

// Pairs of order 1..QZMAX, held in LDS with Q and Z (identity when not
// accumulated); other orders are left to k_qz_global.
__global__ void __launch_bounds__(NT) k_qz_batched(double *H, double *T, double *Q, double *Z,
                                                   const int64_t *offs, const int32_t *nn, int batch,
                                                   double *alphar, double *alphai, double *beta,
                                                   const int64_t *eoff, int32_t *info)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SmemQZ &S = *reinterpret_cast<SmemQZ *>(smem_raw);
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < batch; b += gridDim.x) {
        const int n = nn[b];
        if (n < 0 || n > QZMAX) continue;
        if (n == 0) {
            if (tid == 0) info[b] = 0;
            continue;
        }
        const int64_t o = offs[b];
        const QZV M{S.H, S.T, S.Q, S.Z, LDQZ};
        for (int it = tid; it < n * n; it += NT) {
            const int r = it % n, c = it / n;
            M.H[r + c * M.ld] = (r <= c + 1) ? H[o + it] : 0.0;
            M.T[r + c * M.ld] = (r <= c) ? T[o + it] : 0.0;
            M.Q[r + c * M.ld] = Q ? Q[o + it] : (r == c ? 1.0 : 0.0);
            M.Z[r + c * M.ld] = Z ? Z[o + it] : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        const int result = qz_solve(S, M, n, alphar + eoff[b], alphai + eoff[b], beta + eoff[b]);
        for (int it = tid; it < n * n; it += NT) {
            const int r = it % n, c = it / n;
            H[o + it] = M.H[r + c * M.ld];
            T[o + it] = M.T[r + c * M.ld];
            if (Q) Q[o + it] = M.Q[r + c * M.ld];
            if (Z) Z[o + it] = M.Z[r + c * M.ld];
        }
        if (tid == 0) info[b] = result;
        __syncthreads();
    }
}

// Pairs of order above QZMAX, reduced in place in the caller's arrays (the
// same steps as k_qz_batched, every access a global-memory one); negative
// orders are argument errors.
__global__ void __launch_bounds__(NT) k_qz_global(double *H, double *T, double *Q, double *Z,
                                                  const int64_t *offs, const int32_t *nn, int batch,
                                                  double *alphar, double *alphai, double *beta,
                                                  const int64_t *eoff, int32_t *info)
{
    __shared__ QZCtl S;
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < batch; b += gridDim.x) {
        const int n = nn[b];
        if (n < 0) {
            if (tid == 0) info[b] = -1;
            continue;
        }
        if (n <= QZMAX) continue;
        const int64_t o = offs[b];
        const QZV M{H + o, T + o, Q ? Q + o : nullptr, Z ? Z + o : nullptr, n};
        // zeros below the subdiagonal of H and below the diagonal of T
        for (int it = tid; it < n * n; it += NT) {
            const int r = it % n, c = it / n;
            if (r > c + 1) M.H[it] = 0.0;
            if (r > c) M.T[it] = 0.0;
        }
        __syncthreads();
        const int result = qz_solve(S, M, n, alphar + eoff[b], alphai + eoff[b], beta + eoff[b]);
        if (tid == 0) info[b] = result;
        __syncthreads();
    }
}

hipError_t launch_qz_batched(double *H, double *T, double *Q, double *Z, const int64_t *offsets, const int32_t *n,
                             int batch, double *alphar, double *alphai, double *beta, const int64_t *eoff,
                             int32_t *info, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_qz_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sizeof(SmemQZ));
        if (e != hipSuccess) return e;
        attr = true;
    }
    int dev = 0, ncu = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = std::max(1, std::min(batch, std::max(ncu, 1)));
    hipLaunchKernelGGL(k_qz_batched, dim3(grid), dim3(NT), sizeof(SmemQZ), s, H, T, Q, Z, offsets, n, batch, alphar,
                       alphai, beta, eoff, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // orders above the LDS limit: two workgroups per CU, each pair in place
    const int grid2 = std::max(1, std::min(batch, 2 * std::max(ncu, 1)));
    hipLaunchKernelGGL(k_qz_global, dim3(grid2), dim3(NT), 0, s, H, T, Q, Z, offsets, n, batch, alphar, alphai, beta,
                       eoff, info);
    return hipGetLastError();
}

} // namespace hqr
