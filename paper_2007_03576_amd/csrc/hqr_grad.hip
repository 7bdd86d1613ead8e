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

// Per-matrix descriptor of a backward call: offsets of T_b / Q_b / dH_b
// (doubles), of its eigenvalues and cotangents, of its workspace (doubles from
// the chunk's base), and its order.
//   workspace of matrix b (n = n_b): Ys, Zs (2n x n each: right / left
//   eigenvectors of T, real parts in rows 0..n-1, imaginary in n..2n-1),
//   X, Yl, W (n x 2n each), then max|T_b|; 10 n^2 + 1 doubles.

// max |T| per matrix (for the pivot floor of the substitutions)
__global__ void k_tnorm(const double *T, const BwdDesc *D, double *ws)
{
    __shared__ double red[256];
    const BwdDesc d = D[blockIdx.x];
    const int n = d.n;
    const double *Tb = T + d.toff;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)n * n; i += blockDim.x) m = fmax(m, fabs(Tb[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) ws[d.woff + 10 * (int64_t)n * n] = red[0];
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
// [n + e + l*2n] (lanes of a wave touch consecutive addresses).  Grid:
// (ceil(max n / 64), matrices); blocks past a matrix's order return at once.
__global__ void __launch_bounds__(64) k_eigvec(const double *T, const BwdDesc *D, const double *wr,
                                               const double *wi, double *ws)
{
    const BwdDesc d = D[blockIdx.y];
    const int n = d.n;
    if ((int)blockIdx.x * 64 >= n) return; // whole block past the order (uniform)
    const double *Tb = T + d.toff;
    const int e = blockIdx.x * 64 + threadIdx.x;
    const bool act = e < n;
    const int64_t ld2 = 2 * (int64_t)n;
    double *Y = ws + d.woff;
    double *Z = Y + 2 * (int64_t)n * n;
    const double smin = fmax(kUg * ws[d.woff + 10 * (int64_t)n * n], DBL_MIN);
    int k = 0, sz = 1;
    double lr = 0.0, li = 0.0;
    if (act) {
        bool second = (e > 0 && Tb[e + (int64_t)(e - 1) * n] != 0.0);
        bool first = (e + 1 < n && Tb[(e + 1) + (int64_t)e * n] != 0.0);
        k = second ? e - 1 : e;
        sz = (first || second) ? 2 : 1;
        lr = wr[d.eoff + e];
        li = wi[d.eoff + e];
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

// Batched products of the backward pass on FP64 MFMA, 64 x 64 output tiles
// per workgroup, per-matrix shapes from the descriptors:
//   which 0: X  = Q Ys^T   (n x 2n, inner n)
//   which 1: Yl = Q Zs^T   (n x 2n, inner n)
//   which 2: dH = W X^T    (n x n, inner 2n)
// Grid: (ceil(max rows / 64), ceil(max cols / 64), matrices); tiles past a
// matrix's shape return before the first barrier.
constexpr int GT = 64, GK = 16, GPAD = 4;
__global__ void __launch_bounds__(256) k_gemm_bwd(int which, const double *Qg, const BwdDesc *D, double *ws,
                                                  double *dH)
{
    __shared__ double As[GK][GT + GPAD];
    __shared__ double Bs[GK][GT + GPAD];
    const BwdDesc d = D[blockIdx.z];
    const int n = d.n;
    const int64_t nn = (int64_t)n * n;
    double *wb = ws + d.woff;
    const double *A, *B;
    double *C;
    int m, nc, kk;
    int64_t lda, ldb, ldc;
    if (which < 2) {
        A = Qg + d.toff;
        lda = n;
        B = wb + (which == 0 ? 0 : 2 * nn); // Ys or Zs, 2n x n, used transposed
        ldb = 2 * (int64_t)n;
        C = wb + (which == 0 ? 4 * nn : 6 * nn); // X or Yl
        ldc = n;
        m = n;
        nc = 2 * n;
        kk = n;
    } else {
        A = wb + 8 * nn; // W, n x 2n
        lda = n;
        B = wb + 4 * nn; // X, n x 2n, used transposed
        ldb = n;
        C = dH + d.toff;
        ldc = n;
        m = n;
        nc = n;
        kk = 2 * n;
    }
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    if (m0 >= m || n0 >= nc) return; // uniform per workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int l16 = lane & 15, lq = lane >> 4;
    dbl4g acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = (dbl4g){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < kk; k0 += GK) {
        for (int it = tid; it < GT * GK; it += 256) {
            // A as stored (column major): rows along the tile's first index
            const int mi = it % GT, ki = it / GT;
            const int gm = m0 + mi, gk = k0 + ki;
            As[ki][mi] = (gm < m && gk < kk) ? A[gm + (int64_t)gk * lda] : 0.0;
            // B used transposed: B^T(k, j) = B[j + k*ldb]
            const int nj = it % GT, kj = it / GT;
            const int gn = n0 + nj, gk2 = k0 + kj;
            Bs[kj][nj] = (gn < nc && gk2 < kk) ? B[gn + (int64_t)gk2 * ldb] : 0.0;
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
                if (gm < m && gn < nc) C[gm + (int64_t)gn * ldc] = acc[a][c][r];
            }
}

// c_i = conj(g_i) / (y_i^H x_i) and the columns of W = [A1, -A2]:
//   A1 = Yr diag(cr) + Yi diag(ci),  A2 = Yr diag(ci) - Yi diag(cr)
// X = [Xr | Xi], Yl = [Yr | Yi] are n x 2n (ld n).  One block per (i, b).
__global__ void k_coef(const BwdDesc *D, const double *gwr, const double *gwi, double *ws)
{
    __shared__ double red[2][256];
    const BwdDesc d = D[blockIdx.y];
    const int n = d.n;
    const int i = blockIdx.x;
    if (i >= n) return; // uniform per workgroup
    const int64_t nn = (int64_t)n * n;
    const double *Xb = ws + d.woff + 4 * nn, *Yb = ws + d.woff + 6 * nn;
    double *Wb = ws + d.woff + 8 * nn;
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
    double gr = gwr[d.eoff + i], gi = -gwi[d.eoff + i]; // conj(g)
    double cr, ci;
    cdiv(gr, gi, dr, di, cr, ci);
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        double yr = Yb[a + (int64_t)i * n], yi = Yb[a + (int64_t)(n + i) * n];
        Wb[a + (int64_t)i * n] = yr * cr + yi * ci;
        Wb[a + (int64_t)(n + i) * n] = -(yr * ci - yi * cr);
    }
}

__global__ void k_hess_mask(const BwdDesc *D, double *dH)
{
    const BwdDesc d = D[blockIdx.y];
    const int n = d.n, c = blockIdx.x;
    if (c >= n) return;
    double *Db = dH + d.toff;
    for (int r = c + 2 + threadIdx.x; r < n; r += blockDim.x) Db[r + (int64_t)c * n] = 0.0;
}

// Right eigenvectors of H in LAPACK's dgeev layout from X = [Re | Im] (n x 2n,
// column e = vector of eigenvalue e): a real eigenvalue gets one real column;
// the pair (e, e+1) with wi[e] > 0 gets Re(x) and Im(x) of the vector of
// wr[e] + i wi[e].  Each vector is scaled to unit 2-norm with its largest
// component real and positive.  One workgroup per eigenvalue.
__global__ void __launch_bounds__(256) k_evec_pack(int n, const double *Xw, const double *wi, double *Xo,
                                                   int64_t ldx)
{
    __shared__ double red[256];
    __shared__ int ired[256];
    const int e = blockIdx.x;
    if (wi[e] < 0.0) return; // written together with its partner
    const bool cplx = wi[e] > 0.0;
    const double *xr = Xw + (int64_t)e * n, *xi = Xw + (int64_t)(n + e) * n;
    double ss = 0.0, best = -1.0;
    int bi = 0;
    for (int r = threadIdx.x; r < n; r += 256) {
        const double a = xr[r], b = cplx ? xi[r] : 0.0;
        const double m2 = a * a + b * b;
        ss += m2;
        if (m2 > best) {
            best = m2;
            bi = r;
        }
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double nrm = sqrt(red[0]);
    __syncthreads();
    red[threadIdx.x] = best;
    ired[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && (red[threadIdx.x + w] > red[threadIdx.x] ||
                                    (red[threadIdx.x + w] == red[threadIdx.x] &&
                                     ired[threadIdx.x + w] < ired[threadIdx.x])))
        {
            red[threadIdx.x] = red[threadIdx.x + w];
            ired[threadIdx.x] = ired[threadIdx.x + w];
        }
        __syncthreads();
    }
    const int k = ired[0];
    // rotation c - i s that makes component k real and positive, with 1/||x||
    double c = 1.0, sn = 0.0;
    const double ak = xr[k], bk = cplx ? xi[k] : 0.0;
    const double mk = hypot(ak, bk);
    if (mk > 0.0) {
        c = ak / mk;
        sn = bk / mk;
    }
    const double sc = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    for (int r = threadIdx.x; r < n; r += 256) {
        const double a = xr[r], b = cplx ? xi[r] : 0.0;
        // (a + i b)(c - i sn) = (a c + b sn) + i (b c - a sn)
        Xo[r + (int64_t)e * ldx] = (a * c + b * sn) * sc;
        if (cplx) Xo[r + (int64_t)(e + 1) * ldx] = (b * c - a * sn) * sc;
    }
}

hipError_t launch_eigenvectors(const double *T, const double *Q, const BwdDesc *D, int n, const double *wr,
                               const double *wi, double *ws, double *X, int64_t ldx, hipStream_t s)
{
    const int tiles = (n + GT - 1) / GT, tiles2 = (2 * n + GT - 1) / GT;
    hipLaunchKernelGGL(k_tnorm, dim3(1), dim3(256), 0, s, T, D, ws);
    hipLaunchKernelGGL(k_eigvec, dim3((n + 63) / 64, 1), dim3(64), 0, s, T, D, wr, wi, ws);
    hipLaunchKernelGGL(k_gemm_bwd, dim3(tiles, tiles2, 1), dim3(256), 0, s, 0, Q, D, ws, (double *)nullptr);
    hipLaunchKernelGGL(k_evec_pack, dim3(n), dim3(256), 0, s, n, ws + 4 * (int64_t)n * n, wi, X, ldx);
    return hipGetLastError();
}

hipError_t launch_eig_backward_chunk(const double *T, const double *Q, const BwdDesc *D, int nb, int nmax,
                                     const double *wr, const double *wi, const double *gwr, const double *gwi,
                                     double *dH, int hess_mask, double *ws, hipStream_t s)
{
    if (nb <= 0 || nmax <= 0) return hipSuccess;
    const int tiles = (nmax + GT - 1) / GT, tiles2 = (2 * nmax + GT - 1) / GT;
    hipLaunchKernelGGL(k_tnorm, dim3(nb), dim3(256), 0, s, T, D, ws);
    hipLaunchKernelGGL(k_eigvec, dim3((nmax + 63) / 64, nb), dim3(64), 0, s, T, D, wr, wi, ws);
    // X = Q Ys^T, Yl = Q Zs^T
    hipLaunchKernelGGL(k_gemm_bwd, dim3(tiles, tiles2, nb), dim3(256), 0, s, 0, Q, D, ws, dH);
    hipLaunchKernelGGL(k_gemm_bwd, dim3(tiles, tiles2, nb), dim3(256), 0, s, 1, Q, D, ws, dH);
    hipLaunchKernelGGL(k_coef, dim3(nmax, nb), dim3(256), 0, s, D, gwr, gwi, ws);
    // dH = W X^T
    hipLaunchKernelGGL(k_gemm_bwd, dim3(tiles, tiles, nb), dim3(256), 0, s, 2, Q, D, ws, dH);
    if (hess_mask) hipLaunchKernelGGL(k_hess_mask, dim3(nmax, nb), dim3(64), 0, s, D, dH);
    return hipGetLastError();
}

} // namespace hqr
