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

namespace hqr {

constexpr int QZMAX = 64;
constexpr int LDQZ = QZMAX + 1;
constexpr double kUq = 2.220446049250313080847e-16; // unit roundoff 2^-52

struct SmemQZ {
    double H[QZMAX * LDQZ], T[QZMAX * LDQZ], Q[QZMAX * LDQZ], Z[QZMAX * LDQZ];
    double G[9];  // the transformation to apply (row major, m x m)
    double x[3];  // vector that defines the next reflector
    int ic[8];    // decisions of thread 0: action, l, kz, i, its
    double sc[8]; // scalars of thread 0: shifts, thresholds
};

// ---- thread-0 scalar helpers ----------------------------------------------

// Reflector P = I - tau v v^T, v[0] = 1, P x = beta e_0 (beta = -sign(x0)||x||;
// identity when the tail is zero).
__device__ void qz_house(int m, const double *x, double *v, double &tau, double &beta)
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
__device__ void qz_set_house(SmemQZ &S, int m, const double *v, double tau)
{
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            S.G[i * 3 + k] = (i < m && k < m) ? ((i == k ? 1.0 : 0.0) - tau * v[i] * v[k]) : 0.0;
}

// Reflector acting from the right on a row vector w (length m): w P = gamma e_{m-1}.
__device__ void qz_set_house_last(SmemQZ &S, int m, const double *w)
{
    double wr[3], vr[3], v[3], tau, beta;
    for (int i = 0; i < m; ++i) wr[i] = w[m - 1 - i];
    qz_house(m, wr, vr, tau, beta);
    for (int i = 0; i < m; ++i) v[i] = vr[m - 1 - i];
    qz_set_house(S, m, v, tau);
}

// 2x2 matrix [[a, b], [c, d]] into S.G.
__device__ void qz_set2(SmemQZ &S, double a, double b, double c, double d)
{
    for (int q = 0; q < 9; ++q) S.G[q] = 0.0;
    S.G[0] = a;
    S.G[1] = b;
    S.G[3] = c;
    S.G[4] = d;
}

// (c, s) with c = a / r, s = b / r (identity for a zero vector).
__device__ void qz_cs(double a, double b, double &c, double &s)
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
__device__ void qz_eig2(const SmemQZ &S, int k, double &r1, double &i1, double &r2, double &i2)
{
    const double *H = S.H, *T = S.T;
    const double a11 = H[k + k * LDQZ], a12 = H[k + (k + 1) * LDQZ];
    const double a21 = H[(k + 1) + k * LDQZ], a22 = H[(k + 1) + (k + 1) * LDQZ];
    const double b11 = T[k + k * LDQZ], b12 = T[k + (k + 1) * LDQZ], b22 = T[(k + 1) + (k + 1) * LDQZ];
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
__device__ void qz_apply(SmemQZ &S, int n, int side, int p, int m)
{
    __syncthreads();
    double g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = S.G[q];
    for (int it = threadIdx.x; it < 3 * n; it += NT) {
        const int which = it / n, r = it - which * n;
        double x[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
        if (side == 0 && which < 2) {
            double *A = which == 0 ? S.H : S.T; // column r of A, rows p..p+m-1
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < m) x[k] = A[(p + k) + r * LDQZ];
#pragma unroll
            for (int i = 0; i < 3; ++i) y[i] = g[i * 3] * x[0] + g[i * 3 + 1] * x[1] + g[i * 3 + 2] * x[2];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < m) A[(p + i) + r * LDQZ] = y[i];
        } else {
            double *A = side == 0 ? S.Q : (which == 0 ? S.H : (which == 1 ? S.T : S.Z)); // row r
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < m) x[k] = A[r + (p + k) * LDQZ];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                y[j] = (side == 0) ? (x[0] * g[j * 3] + x[1] * g[j * 3 + 1] + x[2] * g[j * 3 + 2])
                                   : (x[0] * g[j] + x[1] * g[3 + j] + x[2] * g[6 + j]);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (j < m) A[r + (p + j) * LDQZ] = y[j];
        }
    }
    __syncthreads();
}

// Zero diagonal entries of T below the threshold in [lo, hi].
__device__ void qz_threshold(SmemQZ &S, int lo, int hi, double btol)
{
    for (int k = lo + (int)threadIdx.x; k <= hi; k += NT)
        if (fabs(S.T[k + k * LDQZ]) <= btol) S.T[k + k * LDQZ] = 0.0;
    __syncthreads();
}

// Chase the zero at T[kz,kz] to T[l,l] and deflate it there (H[l+1,l] = 0).
__device__ void qz_push_up(SmemQZ &S, int n, int l, int i, int kz)
{
    const int tid = threadIdx.x;
    for (int jc = kz; jc > l; --jc) {
        if (tid == 0) {
            double c, s;
            qz_cs(S.T[(jc - 1) + jc * LDQZ], S.T[(jc - 1) + (jc - 1) * LDQZ], c, s);
            qz_set2(S, c, s, -s, c); // columns (jc-1, jc)
        }
        qz_apply(S, n, 1, jc - 1, 2);
        if (tid == 0) S.T[(jc - 1) + (jc - 1) * LDQZ] = 0.0;
        if (jc + 1 <= i) {
            if (tid == 0) {
                double c, s;
                qz_cs(S.H[jc + (jc - 1) * LDQZ], S.H[(jc + 1) + (jc - 1) * LDQZ], c, s);
                qz_set2(S, c, s, -s, c); // rows (jc, jc+1)
            }
            qz_apply(S, n, 0, jc, 2);
            if (tid == 0) S.H[(jc + 1) + (jc - 1) * LDQZ] = 0.0;
        }
    }
    if (tid == 0) {
        double c, s;
        qz_cs(S.H[l + l * LDQZ], S.H[(l + 1) + l * LDQZ], c, s);
        qz_set2(S, c, s, -s, c);
    }
    qz_apply(S, n, 0, l, 2);
    if (tid == 0) S.H[(l + 1) + l * LDQZ] = 0.0;
    __syncthreads();
}

// Split a 2x2 block at (k, k+1) with the real eigenvalue lam.
__device__ void qz_split2(SmemQZ &S, int n, int k, double lam)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        const double *H = S.H, *T = S.T;
        const double m11 = H[k + k * LDQZ] - lam * T[k + k * LDQZ];
        const double m12 = H[k + (k + 1) * LDQZ] - lam * T[k + (k + 1) * LDQZ];
        const double m21 = H[(k + 1) + k * LDQZ];
        const double m22 = H[(k + 1) + (k + 1) * LDQZ] - lam * T[(k + 1) + (k + 1) * LDQZ];
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
    qz_apply(S, n, 1, k, 2);
    if (tid == 0) {
        double c, s;
        qz_cs(S.T[k + k * LDQZ], S.T[(k + 1) + k * LDQZ], c, s);
        qz_set2(S, c, s, -s, c);
    }
    qz_apply(S, n, 0, k, 2);
    if (tid == 0) {
        S.H[(k + 1) + k * LDQZ] = 0.0;
        S.T[(k + 1) + k * LDQZ] = 0.0;
    }
    __syncthreads();
}

// One double-shift sweep over [l, i] (i - l >= 2), shifts in S.sc[0..3].
__device__ void qz_sweep(SmemQZ &S, int n, int l, int i)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        const double re1 = S.sc[0], im1 = S.sc[1], re2 = S.sc[2], im2 = S.sc[3];
        const double sum = re1 + re2, prod = re1 * re2 - im1 * im2;
        const double *H = S.H, *T = S.T;
        const double t11 = T[l + l * LDQZ], t12 = T[l + (l + 1) * LDQZ], t22 = T[(l + 1) + (l + 1) * LDQZ];
        const double h11 = H[l + l * LDQZ], h21 = H[(l + 1) + l * LDQZ], h12 = H[l + (l + 1) * LDQZ];
        const double h22 = H[(l + 1) + (l + 1) * LDQZ], h32 = H[(l + 2) + (l + 1) * LDQZ];
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
            for (int r = 0; r < m; ++r) x[r] = (k >= l) ? S.H[(k + 1 + r) + k * LDQZ] : S.x[r];
            qz_house(m, x, v, tau, beta);
            qz_set_house(S, m, v, tau);
            S.sc[4] = beta;
        }
        qz_apply(S, n, 0, k + 1, m);
        if (tid == 0) {
            if (k >= l) {
                S.H[(k + 1) + k * LDQZ] = S.sc[4];
                for (int r = 1; r < m; ++r) S.H[(k + 1 + r) + k * LDQZ] = 0.0;
            }
            double w[3];
            for (int r = 0; r < m; ++r) w[r] = S.T[(k + m) + (k + 1 + r) * LDQZ];
            qz_set_house_last(S, m, w);
        }
        qz_apply(S, n, 1, k + 1, m);
        if (tid == 0) {
            for (int r = 0; r < m - 1; ++r) S.T[(k + m) + (k + 1 + r) * LDQZ] = 0.0;
            if (m == 3) {
                double w[2] = {S.T[(k + 2) + (k + 1) * LDQZ], S.T[(k + 2) + (k + 2) * LDQZ]};
                qz_set_house_last(S, 2, w);
            }
        }
        if (m == 3) {
            qz_apply(S, n, 1, k + 1, 2);
            if (tid == 0) S.T[(k + 2) + (k + 1) * LDQZ] = 0.0;
        }
        __syncthreads();
    }
}

// Actions decided by thread 0 each round.
enum { QZ_DONE = 0, QZ_PUSH = 1, QZ_ONE = 2, QZ_TWO = 3, QZ_SWEEP = 4, QZ_FAIL = 5 };

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
        if (n < 0 || n > QZMAX) {
            if (tid == 0) info[b] = -1;
            continue;
        }
        if (n == 0) {
            if (tid == 0) info[b] = 0;
            continue;
        }
        const int64_t o = offs[b];
        for (int it = tid; it < n * n; it += NT) {
            const int r = it % n, c = it / n;
            S.H[r + c * LDQZ] = (r <= c + 1) ? H[o + it] : 0.0;
            S.T[r + c * LDQZ] = (r <= c) ? T[o + it] : 0.0;
            S.Q[r + c * LDQZ] = Q ? Q[o + it] : (r == c ? 1.0 : 0.0);
            S.Z[r + c * LDQZ] = Z ? Z[o + it] : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        if (tid == 0) {
            // ||T||_F of the input's triangle (Sec. 2: |t_kk| <= u ||T||_F is infinite)
            double tn = 0.0;
            for (int c = 0; c < n; ++c)
                for (int r = 0; r <= c; ++r) tn = hypot(tn, S.T[r + c * LDQZ]);
            S.sc[5] = kUq * tn;
            S.sc[6] = DBL_MIN * ((double)n / kUq);
            S.ic[3] = n - 1; // i
            S.ic[4] = 0;     // iterations since the last deflation
            S.ic[5] = 0;     // iterations
        }
        __syncthreads();
        const double btol = S.sc[5], smlnum = S.sc[6];
        const int64_t itmax = 30 * (int64_t)max(10, n);
        qz_threshold(S, 0, n - 1, btol);
        double *ar = alphar + eoff[b], *ai = alphai + eoff[b], *be = beta + eoff[b];
        int result = 0;
        for (;;) {
            if (tid == 0) {
                const int i = __builtin_amdgcn_readfirstlane(S.ic[3]);
                int act = QZ_DONE, l = 0, kz = -1;
                if (i >= 0) {
                    l = i;
                    while (l > 0) {
                        const double h = fabs(S.H[l + (l - 1) * LDQZ]);
                        const double tst = fabs(S.H[(l - 1) + (l - 1) * LDQZ]) + fabs(S.H[l + l * LDQZ]);
                        if (h <= fmax(smlnum, kUq * tst)) {
                            S.H[l + (l - 1) * LDQZ] = 0.0;
                            break;
                        }
                        --l;
                    }
                    for (int k = l; k <= i; ++k)
                        if (S.T[k + k * LDQZ] == 0.0) {
                            kz = k;
                            break;
                        }
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
                    double a = S.H[i + i * LDQZ], bt = S.T[i + i * LDQZ];
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
                    qz_eig2(S, i - 1, r1, i1, r2, i2);
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
                        const double ss = fabs(S.H[i + (i - 1) * LDQZ] / S.T[(i - 1) + (i - 1) * LDQZ]) +
                                          fabs(S.H[(i - 1) + (i - 2) * LDQZ] / S.T[(i - 2) + (i - 2) * LDQZ]);
                        r1 = r2 = S.H[i + i * LDQZ] / S.T[i + i * LDQZ] + 0.75 * ss;
                        i1 = i2 = 0.0;
                    } else {
                        qz_eig2(S, i - 1, r1, i1, r2, i2);
                        if (i1 == 0.0) {
                            const double tb = S.H[i + i * LDQZ] / S.T[i + i * LDQZ];
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
                qz_push_up(S, n, l, i, kz);
                qz_threshold(S, l + 1, i, btol);
                if (tid == 0) S.ic[4] = 0;
            } else if (act == QZ_TWO && split) {
                qz_split2(S, n, i - 1, lam);
            } else if (act == QZ_SWEEP) {
                qz_sweep(S, n, l, i);
                qz_threshold(S, l, i, btol);
            }
            __syncthreads();
        }
        __syncthreads();
        for (int it = tid; it < n * n; it += NT) {
            const int r = it % n, c = it / n;
            H[o + it] = S.H[r + c * LDQZ];
            T[o + it] = S.T[r + c * LDQZ];
            if (Q) Q[o + it] = S.Q[r + c * LDQZ];
            if (Z) Z[o + it] = S.Z[r + c * LDQZ];
        }
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
    return hipGetLastError();
}

} // namespace hqr
