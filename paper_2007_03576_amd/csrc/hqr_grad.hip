// Backward pass of the eigenvalues of a real Schur form (gfx950).
//
// For a simple eigenvalue lambda_i of H with right and left eigenvectors
// x_i, y_i (H x = lambda x, y^H H = lambda y^H), d lambda_i = y_i^H dH x_i /
// (y_i^H x_i).  For a real loss L with cotangents g_i = dL/dRe + i dL/dIm,
//     dL/dH = Re( conj(Y) diag(conj(g_i) / (y_i^H x_i)) X^T ).
// The eigenvectors come from the Schur form (Sec. 2 of the paper: solve
// (S - lambda I) y = 0 and back-transform x = Q y):
//   1. batched quasi-triangular back substitution for the right vectors of T
//      and forward substitution for the left vectors (one lane per
//      eigenvalue, complex arithmetic, 2x2 diagonal blocks solved exactly);
//   2. X = Q Yr, Y = Q Zl and dL/dH = W X^T with batched FP64-MFMA products;
//   3. the coefficients c_i and the columns of W by per-eigenvalue reductions.
#include "hqr_common.h"
#include <algorithm>
#include <cfloat>

namespace hqr {

typedef double dbl4g __attribute__((ext_vector_type(4)));
constexpr double kUg = 2.220446049250313080847e-16;

// max |T| per matrix (for the pivot floor of the substitutions)
__global__ void k_tnorm(const double *T, int n, double *tn)
{
    __shared__ double red[256];
    const double *Tb = T + (int64_t)blockIdx.x * n * n;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)n * n; i += blockDim.x) m = fmax(m, fabs(Tb[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) tn[blockIdx.x] = red[0];
}

__device__ inline void cdiv(double ar, double ai, double br, double bi, double &qr, double &qi)
{
    // (ar + i ai) / (br + i bi), scaled
    if (fabs(br) >= fabs(bi)) {
        double r = bi / br, d = br + bi * r;
        qr = (ar + ai * r) / d;
        qi = (ai - ar * r) / d;
    } else {
        double r = br / bi, d = bi + br * r;
        qr = (ar * r + ai) / d;
        qi = (ai * r - ar) / d;
    }
}

// Solve the complex 2x2 system (B - mu I) x = r for a real 2x2 block B.
__device__ inline void solve2(double b00, double b01, double b10, double b11, double mur, double mui, double r0r,
                              double r0i, double r1r, double r1i, double smin, double &x0r, double &x0i,
                              double &x1r, double &x1i)
{
    double a_r = b00 - mur, a_i = -mui, d_r = b11 - mur, d_i = -mui;
    // det = a d - b01 b10
    double det_r = a_r * d_r - a_i * d_i - b01 * b10;
    double det_i = a_r * d_i + a_i * d_r;
    if (hypot(det_r, det_i) < smin) {
        det_r = smin;
        det_i = 0.0;
    }
    // x0 = (d r0 - b01 r1)/det ; x1 = (a r1 - b10 r0)/det
    double n0r = d_r * r0r - d_i * r0i - b01 * r1r, n0i = d_r * r0i + d_i * r0r - b01 * r1i;
    double n1r = a_r * r1r - a_i * r1i - b10 * r0r, n1i = a_r * r1i + a_i * r1r - b10 * r0i;
    cdiv(n0r, n0i, det_r, det_i, x0r, x0i);
    cdiv(n1r, n1i, det_r, det_i, x1r, x1i);
}

// Right (Y) and left (Z) eigenvectors of the quasi-triangular T_b, one lane
// per eigenvalue.  Storage: per matrix a 2n x n column-major array with the
// real part of vector e, entry l at [e + l*2n] and the imaginary part at
// [n + e + l*2n] (lanes of a wave touch consecutive addresses).
__global__ void __launch_bounds__(64) k_eigvec(const double *T, int n, const double *wr, const double *wi,
                                               const double *tn, double *Ys, double *Zs)
{
    const int b = blockIdx.y;
    const double *Tb = T + (int64_t)b * n * n;
    const int e = blockIdx.x * 64 + threadIdx.x;
    const bool act = e < n;
    const int64_t ld2 = 2 * (int64_t)n;
    double *Y = Ys + (int64_t)b * ld2 * n;
    double *Z = Zs + (int64_t)b * ld2 * n;
    const double smin = fmax(kUg * tn[b], DBL_MIN);
    int k = 0, sz = 1;
    double lr = 0.0, li = 0.0;
    if (act) {
        bool second = (e > 0 && Tb[e + (int64_t)(e - 1) * n] != 0.0);
        bool first = (e + 1 < n && Tb[(e + 1) + (int64_t)e * n] != 0.0);
        k = second ? e - 1 : e;
        sz = (first || second) ? 2 : 1;
        lr = wr[(int64_t)b * n + e];
        li = wi[(int64_t)b * n + e];
        for (int l = 0; l < n; ++l) {
            Y[e + l * ld2] = 0.0;
            Y[n + e + l * ld2] = 0.0;
            Z[e + l * ld2] = 0.0;
            Z[n + e + l * ld2] = 0.0;
        }
        // the eigenvalue's own block
        Y[e + k * ld2] = 1.0;
        Z[e + k * ld2] = 1.0;
        if (sz == 2) {
            double bb = Tb[k + (int64_t)(k + 1) * n], cc = Tb[(k + 1) + (int64_t)k * n];
            Y[n + e + (k + 1) * ld2] = li / bb;   // y1 = i w / b
            Z[n + e + (k + 1) * ld2] = -li / cc;  // z1 = -i w / c
        }
    }
    // wave-uniform ranges
    int kmax = act ? k : 0, kmin = act ? k + sz : n;
    for (int off = 32; off > 0; off >>= 1) {
        kmax = max(kmax, __shfl_xor(kmax, off, 64));
        kmin = min(kmin, __shfl_xor(kmin, off, 64));
    }
    int lmax = min(n, kmax + 2);
    // right vectors: rows j < k, bottom up
    int j = kmax - 1;
    while (j >= 0) {
        bool two = (j > 0 && Tb[j + (int64_t)(j - 1) * n] != 0.0);
        int j0 = two ? j - 1 : j;
        bool on = act && j < k;
        double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
        for (int l = j + 1; l < lmax; ++l) {
            double yr = Y[e * act + l * ld2], yi = Y[n + e * act + l * ld2];
            double t1 = Tb[j + (int64_t)l * n];
            s1r += t1 * yr;
            s1i += t1 * yi;
            if (two) {
                double t0 = Tb[j0 + (int64_t)l * n];
                s0r += t0 * yr;
                s0i += t0 * yi;
            }
        }
        if (on) {
            if (!two) {
                double dr = Tb[j + (int64_t)j * n] - lr, di = -li;
                if (hypot(dr, di) < smin) {
                    dr = smin;
                    di = 0.0;
                }
                double qr, qi;
                cdiv(-s1r, -s1i, dr, di, qr, qi);
                Y[e + j * ld2] = qr;
                Y[n + e + j * ld2] = qi;
            } else {
                // the l = j term of row j0 was excluded above: solve the block
                double x0r, x0i, x1r, x1i;
                solve2(Tb[j0 + (int64_t)j0 * n], Tb[j0 + (int64_t)j * n], Tb[j + (int64_t)j0 * n],
                       Tb[j + (int64_t)j * n], lr, li, -s0r, -s0i, -s1r, -s1i, smin, x0r, x0i, x1r, x1i);
                Y[e + j0 * ld2] = x0r;
                Y[n + e + j0 * ld2] = x0i;
                Y[e + j * ld2] = x1r;
                Y[n + e + j * ld2] = x1i;
            }
        }
        j = j0 - 1;
    }
    // left vectors: (T^T - conj(lambda)) z = 0, rows j >= k+sz, top down
    j = kmin;
    while (j < n) {
        bool two = (j + 1 < n && Tb[(j + 1) + (int64_t)j * n] != 0.0);
        bool on = act && j >= k + sz;
        int lo = act ? k : kmin;
        (void)lo;
        double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
        int lstart = max(0, kmin - 2);
        for (int l = lstart; l < j; ++l) {
            double zr = Z[e * act + l * ld2], zi = Z[n + e * act + l * ld2];
            double t0 = Tb[l + (int64_t)j * n];
            s0r += t0 * zr;
            s0i += t0 * zi;
            if (two) {
                double t1 = Tb[l + (int64_t)(j + 1) * n];
                s1r += t1 * zr;
                s1i += t1 * zi;
            }
        }
        if (on) {
            if (!two) {
                double dr = Tb[j + (int64_t)j * n] - lr, di = li; // conj(lambda)
                if (hypot(dr, di) < smin) {
                    dr = smin;
                    di = 0.0;
                }
                double qr, qi;
                cdiv(-s0r, -s0i, dr, di, qr, qi);
                Z[e + j * ld2] = qr;
                Z[n + e + j * ld2] = qi;
            } else {
                // transpose of the block, shifted by conj(lambda)
                double x0r, x0i, x1r, x1i;
                solve2(Tb[j + (int64_t)j * n], Tb[(j + 1) + (int64_t)j * n], Tb[j + (int64_t)(j + 1) * n],
                       Tb[(j + 1) + (int64_t)(j + 1) * n], lr, -li, -s0r, -s0i, -s1r, -s1i, smin, x0r, x0i, x1r,
                       x1i);
                Z[e + j * ld2] = x0r;
                Z[n + e + j * ld2] = x0i;
                Z[e + (j + 1) * ld2] = x1r;
                Z[n + e + (j + 1) * ld2] = x1i;
            }
        }
        j += two ? 2 : 1;
    }
}

// Batched C = op(A) op(B) (m x nn, inner dimension kk), FP64 MFMA.
// opA/opB: 0 = as stored (column major), 1 = transposed.
constexpr int GT = 64, GK = 16, GPAD = 4;
__global__ void __launch_bounds__(256) k_gemm_batched(int m, int nn, int kk, const double *A, int64_t lda,
                                                      int64_t sA, int opA, const double *B, int64_t ldb,
                                                      int64_t sB, int opB, double *C, int64_t ldc, int64_t sC)
{
    __shared__ double As[GK][GT + GPAD];
    __shared__ double Bs[GK][GT + GPAD];
    const int bz = blockIdx.z;
    A += (int64_t)bz * sA;
    B += (int64_t)bz * sB;
    C += (int64_t)bz * sC;
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int l16 = lane & 15, lq = lane >> 4;
    dbl4g acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = (dbl4g){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < kk; k0 += GK) {
        for (int it = tid; it < GT * GK; it += 256) {
            int mi, ki;
            if (opA == 0) {
                mi = it % GT;
                ki = it / GT;
            } else {
                ki = it % GK;
                mi = it / GK;
            }
            int gm = m0 + mi, gk = k0 + ki;
            double v = 0.0;
            if (gm < m && gk < kk) v = (opA == 0) ? A[gm + (int64_t)gk * lda] : A[gk + (int64_t)gm * lda];
            As[ki][mi] = v;
            int nj, kj;
            if (opB == 0) {
                kj = it % GK;
                nj = it / GK;
            } else {
                nj = it % GT;
                kj = it / GT;
            }
            int gn = n0 + nj, gk2 = k0 + kj;
            double w = 0.0;
            if (gn < nn && gk2 < kk) w = (opB == 0) ? B[gk2 + (int64_t)gn * ldb] : B[gn + (int64_t)gk2 * ldb];
            Bs[kj][nj] = w;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            double af[2], bf[2];
            for (int a = 0; a < 2; ++a) af[a] = As[ks + lq][wm + a * 16 + l16];
            for (int c = 0; c < 2; ++c) bf[c] = Bs[ks + lq][wn + c * 16 + l16];
            for (int a = 0; a < 2; ++a)
                for (int c = 0; c < 2; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[c], acc[a][c], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane holds D[lq + 4r][l16]
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm + a * 16 + lq + 4 * r;
                int gn = n0 + wn + c * 16 + l16;
                if (gm < m && gn < nn) C[gm + (int64_t)gn * ldc] = acc[a][c][r];
            }
}

// c_i = conj(g_i) / (y_i^H x_i) and the columns of W = [A1, -A2]:
//   A1 = Yr diag(cr) + Yi diag(ci),  A2 = Yr diag(ci) - Yi diag(cr)
// X = [Xr | Xi], Yl = [Yr | Yi] are n x 2n (ld n).  One block per (i, b).
__global__ void k_coef(int n, const double *X, const double *Yl, const double *gwr, const double *gwi, double *W)
{
    __shared__ double red[2][256];
    const int i = blockIdx.x, b = blockIdx.y;
    const int64_t nn2 = 2 * (int64_t)n * n;
    const double *Xb = X + b * nn2, *Yb = Yl + b * nn2;
    double *Wb = W + b * nn2;
    double dr = 0.0, di = 0.0;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        double yr = Yb[a + (int64_t)i * n], yi = Yb[a + (int64_t)(n + i) * n];
        double xr = Xb[a + (int64_t)i * n], xi = Xb[a + (int64_t)(n + i) * n];
        dr += yr * xr + yi * xi; // conj(y) x
        di += yr * xi - yi * xr;
    }
    red[0][threadIdx.x] = dr;
    red[1][threadIdx.x] = di;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    dr = red[0][0];
    di = red[1][0];
    double gr = gwr[(int64_t)b * n + i], gi = -gwi[(int64_t)b * n + i]; // conj(g)
    double cr, ci;
    cdiv(gr, gi, dr, di, cr, ci);
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        double yr = Yb[a + (int64_t)i * n], yi = Yb[a + (int64_t)(n + i) * n];
        Wb[a + (int64_t)i * n] = yr * cr + yi * ci;
        Wb[a + (int64_t)(n + i) * n] = -(yr * ci - yi * cr);
    }
}

__global__ void k_hess_mask(int n, double *dH)
{
    const int c = blockIdx.x, b = blockIdx.y;
    double *D = dH + (int64_t)b * n * n;
    for (int r = c + 2 + threadIdx.x; r < n; r += blockDim.x) D[r + (int64_t)c * n] = 0.0;
}

static hipError_t gemm(int m, int nn, int kk, const double *A, int64_t lda, int64_t sA, int opA, const double *B,
                       int64_t ldb, int64_t sB, int opB, double *C, int64_t ldc, int64_t sC, int batch,
                       hipStream_t s)
{
    dim3 grid((m + GT - 1) / GT, (nn + GT - 1) / GT, batch);
    hipLaunchKernelGGL(k_gemm_batched, grid, dim3(256), 0, s, m, nn, kk, A, lda, sA, opA, B, ldb, sB, opB, C, ldc,
                       sC);
    return hipGetLastError();
}

namespace {
double *g_gws = nullptr;
size_t g_gws_bytes = 0;
}

hipError_t launch_eig_backward(const double *T, const double *Q, int n, int batch, const double *wr,
                               const double *wi, const double *gwr, const double *gwi, double *dH, int hess_mask,
                               hipStream_t s)
{
    const int64_t nn = (int64_t)n * n;
    // per matrix: Ys, Zs (2n x n), X, Yl, W (n x 2n) and the norm
    const size_t per = (size_t)(10 * nn + 1) * sizeof(double);
    int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)batch, ((size_t)1 << 31) / per));
    size_t need = per * chunk;
    if (need > g_gws_bytes) {
        if (g_gws) {
            hipError_t e = hipFree(g_gws);
            if (e != hipSuccess) return e;
        }
        g_gws = nullptr;
        hipError_t e = hipMalloc(&g_gws, need);
        if (e != hipSuccess) return e;
        g_gws_bytes = need;
    }
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        int nb = std::min(chunk, batch - b0);
        double *Ys = g_gws, *Zs = Ys + 2 * nn * chunk, *X = Zs + 2 * nn * chunk, *Yl = X + 2 * nn * chunk;
        double *W = Yl + 2 * nn * chunk, *tn = W + 2 * nn * chunk;
        const double *Tb = T + b0 * nn, *Qb = Q + b0 * nn;
        hipLaunchKernelGGL(k_tnorm, dim3(nb), dim3(256), 0, s, Tb, n, tn);
        hipLaunchKernelGGL(k_eigvec, dim3((n + 63) / 64, nb), dim3(64), 0, s, Tb, n, wr + (int64_t)b0 * n,
                           wi + (int64_t)b0 * n, tn, Ys, Zs);
        hipError_t e;
        // X = Q Ys^T, Yl = Q Zs^T   (Ys is 2n x n, ld 2n)
        if ((e = gemm(n, 2 * n, n, Qb, n, nn, 0, Ys, 2 * n, 2 * nn, 1, X, n, 2 * nn, nb, s)) != hipSuccess) return e;
        if ((e = gemm(n, 2 * n, n, Qb, n, nn, 0, Zs, 2 * n, 2 * nn, 1, Yl, n, 2 * nn, nb, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_coef, dim3(n, nb), dim3(256), 0, s, n, X, Yl, gwr + (int64_t)b0 * n,
                           gwi + (int64_t)b0 * n, W);
        // dH = W X^T (K = 2n)
        if ((e = gemm(n, n, 2 * n, W, n, 2 * nn, 0, X, n, 2 * nn, 1, dH + b0 * nn, n, nn, nb, s)) != hipSuccess)
            return e;
        if (hess_mask) hipLaunchKernelGGL(k_hess_mask, dim3(n, nb), dim3(64), 0, s, n, dH + b0 * nn);
    }
    return hipGetLastError();
}

} // namespace hqr
