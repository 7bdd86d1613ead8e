// Blocked Householder reduction to upper Hessenberg form on gfx950 (many CUs).
//
// Two users in libhqr:
//   * the phase before the Schur reduction (Sec. 1: dense matrix -> Hessenberg
//     form -> Schur form; Sec. 5.5 "Comment regarding the Hessenberg reduction
//     phase"): A <- Q_h^T A Q_h, Q <- Q Q_h (hqr_hessenberg);
//   * the Hessenberg restoration of a large AED window (Sec. 2.5, third
//     sub-step): after the spike has been reduced to beta e_1 by one
//     reflector, the undeflated leading block of the window's Schur form is
//     reduced back to Hessenberg form, its transformation also applied from
//     the left to the window columns right of the block and from the right
//     to the window's orthogonal factor.
//
// Panels of NBH columns.  With A0 the matrix at the start of a panel, Q_p =
// I - V T V^T the product of the panel's reflectors and Y = A0 V T:
//   * column c = k + j of the result is Q_j^T (A0 - Y_j V_j^T) e_c (only the
//     panel's first j reflectors act on it); its reflector extends V and T,
//     and y_j = A0 v_j is a matrix-vector product over all rows (k_hh_gemv,
//     many workgroups, partial sums per column chunk) that the next column's
//     kernel folds into Y (k_hh_col, one workgroup of 512 threads);
//   * after the panel: A <- Q_p^T (A0 - Y V^T) on the columns right of the
//     panel (extra columns R included in the left product) and Z <- Z Q_p,
//     as FP64-MFMA matrix products (k_gemm64).
// Everything stays on the device: no host synchronization inside.
#include "hqr_common.h"
#include <algorithm>
#include <cfloat>

namespace hqr {

typedef double dbl4h __attribute__((ext_vector_type(4)));

constexpr int HT = 512; // threads of the panel-column kernel (register budget 256)

// Sum of `cnt` per-thread partial values (cnt <= NBH = 32) over the
// workgroup; every thread receives all sums in out[] (LDS scratch red:
// 16 x NBH).  Within a wave the 32 values are reduced by halving exchanges:
// at the stage with partner lane ^ d (d = 32, 16, .., 2) each lane keeps the
// half of its values selected by its bit d and adds the partner's copy of
// that half, so 31 exchanges leave lanes 2i and 2i + 1 with the partial sums
// of value i over their 32-lane halves, and one more exchange completes them.
__device__ inline void hh_multi_sum(const double (&vals)[NBH], int cnt, double *red, double *out)
{
    static_assert(NBH == 32, "halving exchange assumes 32 values");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double v[NBH];
#pragma unroll
    for (int i = 0; i < NBH; ++i) v[i] = vals[i];
#pragma unroll
    for (int w = NBH, d = 32; w > 1; w >>= 1, d >>= 1) {
        const bool up = (lane & d) != 0;
        const int h = w >> 1;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const double send = up ? v[i] : v[i + h];
            const double keep = up ? v[i + h] : v[i];
            v[i] = keep + __shfl_xor(send, d, 64);
        }
    }
    const double tot = v[0] + __shfl_xor(v[0], 1, 64);
    __syncthreads(); // earlier readers of red are done
    if ((lane & 1) == 0) red[wave * NBH + (lane >> 1)] = tot;
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[w * NBH + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

__device__ inline double hh_sum(double v, double *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

__device__ inline double hh_max(double v, double *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t = fmax(t, red[w]);
    return t;
}

// Workgroup max of a and sum of b in one exchange (both returned in place).
__device__ inline void hh_max_sum(double &a, double &b, double *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        a = fmax(a, __shfl_xor(a, off, 64));
        b += __shfl_xor(b, off, 64);
    }
    __syncthreads();
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < nw; ++w) {
        ta = fmax(ta, red[2 * w]);
        tb += red[2 * w + 1];
    }
    a = ta;
    b = tb;
}

// Panel step j (column c = k + j) of a matrix of order m, leading dimension
// lda.  When j > 0 first completes Y(:, j-1) = tau_{j-1} (sum of the GEMV
// partials - Y(:, :j-1) w_{j-1}).  When form != 0 then forms column c,
// writes its final values and its reflector (V(:, j), tau_j, T(:, j),
// w_j = V(:, :j)^T v_j).  V, Y: m x NBH (ld m); T: NBH x NBH; W: NBH x NBH
// (column j = w_j); tau: NBH; part: nchunk x m.
__global__ void __launch_bounds__(HT) k_hh_col(double *A, int64_t lda, int m, int k, int j, int form,
                                               double *V, double *Y, double *Tm, double *W, double *tau,
                                               const double *part, int nchunk)
{
    __shared__ double red[16 * NBH];
    __shared__ double sv[NBH];
    __shared__ double sv2[NBH];
    __shared__ double sT[NBH * NBH]; // T(:, :j) of the panel, read by the small triangular products
    const int tid = threadIdx.x;
    const int64_t ldm = m;
    if (j > 0) {
        const int jp = j - 1;
        const double tp = tau[jp];
        // loops over static bounds with predicates, so the loads of a row
        // are all in flight at once instead of one latency per term
        for (int r = tid; r < m; r += HT) {
            double y0 = 0.0, y1 = 0.0;
#pragma unroll 8
            for (int q = 0; q < nchunk; q += 2) {
                y0 += part[(int64_t)q * m + r];
                if (q + 1 < nchunk) y1 += part[(int64_t)(q + 1) * m + r];
            }
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < jp) s += Y[r + i * ldm] * W[i + jp * NBH];
            Y[r + jp * ldm] = tp * ((y0 + y1) - s);
        }
        __syncthreads();
    }
    if (!form) return;
    const int c = k + j;
    // x = A0(:, c) - Y(:, :j) V(c, :j)^T ; kept in V(:, j) as scratch until the reflector is known
    if (tid < j) sv[tid] = V[c + tid * ldm];
    for (int it = tid; it < NBH * j; it += HT) sT[it] = Tm[it];
    __syncthreads();
    double *x = V + (int64_t)j * ldm;
    double loc[NBH];
#pragma unroll
    for (int i = 0; i < NBH; ++i) loc[i] = 0.0;
    for (int r = tid; r < m; r += HT) {
        double v = A[r + (int64_t)c * lda];
#pragma unroll
        for (int i = 0; i < NBH; ++i)
            if (i < j) v -= Y[r + i * ldm] * sv[i];
        x[r] = v;
        if (r >= k + 1) {
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < j) loc[i] += V[r + i * ldm] * v;
        }
    }
    // x(k+1:) <- Q_{j-1}^T x = x - V T^T (V^T x)
    hh_multi_sum(loc, j, red, sv);
    if (tid < j) { // (T^T s)_i = sum_{l <= i} T(l, i) s_l, one thread per i
        double t = 0.0;
        for (int l = 0; l <= tid; ++l) t += sT[l + tid * NBH] * sv[l];
        sv2[tid] = t;
    }
    __syncthreads();
    double amax = 0.0, ssr = 0.0;
    for (int r = tid; r < m; r += HT) {
        double v = x[r];
        if (r >= k + 1) {
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < j) v -= V[r + i * ldm] * sv2[i];
        }
        x[r] = v;
        if (r <= c) A[r + (int64_t)c * lda] = v; // final rows 0..c of column c
        if (r >= c + 2) {
            amax = fmax(amax, fabs(v));
            ssr = fma(v, v, ssr);
        }
    }
    // the tail's largest entry and unscaled sum of squares in one reduction;
    // the scaled pass runs only when the squares could over- or underflow
    hh_max_sum(amax, ssr, red);
    const double x0 = x[c + 1]; // read before any thread overwrites x below
    double tnorm = 0.0;
    if (amax >= 0x1p-480 && amax <= 0x1p+480) {
        tnorm = sqrt(ssr);
    } else if (amax > 0.0) {
        double ss = 0.0;
        for (int r = c + 2 + tid; r < m; r += HT) {
            const double t = x[r] / amax;
            ss += t * t;
        }
        ss = hh_sum(ss, red);
        tnorm = amax * sqrt(ss);
    }
    double tj = 0.0, beta = x0, scal = 0.0;
    if (amax > 0.0) {
        const double nrm = hypot(x0, tnorm);
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tj = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
    }
    // v_j (unit at c+1, zero above), the reduced column, w_j = V(:, :j)^T v_j
#pragma unroll
    for (int i = 0; i < NBH; ++i) loc[i] = 0.0;
    for (int r = tid; r < m; r += HT) {
        double v;
        if (r <= c) v = 0.0;
        else if (r == c + 1) v = 1.0;
        else v = (tj != 0.0) ? x[r] * scal : 0.0;
        x[r] = v;
        if (r == c + 1) A[r + (int64_t)c * lda] = beta;
        else if (r > c + 1) A[r + (int64_t)c * lda] = 0.0;
        if (r >= c + 1) {
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < j) loc[i] += V[r + i * ldm] * v;
        }
    }
    hh_multi_sum(loc, j, red, sv);
    if (tid < j) { // T(:j, j) = -tau_j T(:j, :j) w_j, one thread per row
        W[tid + j * NBH] = sv[tid];
        double t = 0.0;
        for (int l = tid; l < j; ++l) t += sT[tid + l * NBH] * sv[l];
        Tm[tid + j * NBH] = -tj * t;
    } else if (tid < NBH) {
        Tm[tid + j * NBH] = (tid == j) ? tj : 0.0;
    }
    if (tid == 0) tau[j] = tj;
}

// k_hh_col for m <= 2 HT: each thread owns rows tid and tid + HT and keeps
// their entries of the column in registers from its first load to the final
// reflector (no store and reload of the work column between the steps), loads
// its rows of V(:, :j) once for the update and the w_j product, and receives
// x(c+1) through LDS.  Every kernel starts with a cold L2 (the GEMV before it
// ran on all XCDs), so each avoided global round trip is a memory latency.
__global__ void __launch_bounds__(HT) k_hh_col2(double *A, int64_t lda, int m, int k, int j, int form,
                                                double *V, double *Y, double *Tm, double *W, double *tau,
                                                const double *part, int nchunk)
{
    __shared__ double red[16 * NBH];
    __shared__ double sv[NBH];
    __shared__ double sv2[NBH];
    __shared__ double sT[NBH * NBH];
    __shared__ double sx0;
    const int tid = threadIdx.x;
    const int64_t ldm = m;
    const int c = k + j;
    // the loads that do not depend on the step below go out first
    if (form) {
        if (tid < j) sv[tid] = V[c + tid * ldm];
        for (int it = tid; it < NBH * j; it += HT) sT[it] = Tm[it];
    }
    if (j > 0) {
        const int jp = j - 1;
        const double tp = tau[jp];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = tid + q * HT;
            if (r >= m) continue;
            double y0 = 0.0, y1 = 0.0;
#pragma unroll 8
            for (int qq = 0; qq < nchunk; qq += 2) {
                y0 += part[(int64_t)qq * m + r];
                if (qq + 1 < nchunk) y1 += part[(int64_t)(qq + 1) * m + r];
            }
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < jp) s += Y[r + i * ldm] * W[i + jp * NBH];
            Y[r + jp * ldm] = tp * ((y0 + y1) - s);
        }
    }
    if (!form) return;
    __syncthreads();
    // x = A0(:, c) - Y(:, :j) V(c, :j)^T, and the partial sums of V^T x
    double xr[2] = {0.0, 0.0};
    double loc[NBH];
#pragma unroll
    for (int i = 0; i < NBH; ++i) loc[i] = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = tid + q * HT;
        if (r >= m) continue;
        double v = A[r + (int64_t)c * lda];
#pragma unroll
        for (int i = 0; i < NBH; ++i)
            if (i < j) v -= Y[r + i * ldm] * sv[i];
        xr[q] = v;
        if (r >= k + 1) {
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < j) loc[i] += V[r + i * ldm] * v;
        }
    }
    // x(k+1:) <- Q_{j-1}^T x = x - V T^T (V^T x)
    hh_multi_sum(loc, j, red, sv);
    if (tid < j) {
        double t = 0.0;
        for (int l = 0; l <= tid; ++l) t += sT[l + tid * NBH] * sv[l];
        sv2[tid] = t;
    }
    __syncthreads();
    double vr[2][NBH]; // this thread's rows of V(:, :j), kept for the w_j product
    double amax = 0.0, ssr = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = tid + q * HT;
#pragma unroll
        for (int i = 0; i < NBH; ++i) vr[q][i] = 0.0;
        if (r >= m) continue;
        double v = xr[q];
        if (r >= k + 1) {
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < j) {
                    vr[q][i] = V[r + i * ldm];
                    v -= vr[q][i] * sv2[i];
                }
        }
        xr[q] = v;
        if (r <= c) A[r + (int64_t)c * lda] = v; // final rows 0..c of column c
        if (r == c + 1) sx0 = v;
        if (r >= c + 2) {
            amax = fmax(amax, fabs(v));
            ssr = fma(v, v, ssr);
        }
    }
    hh_max_sum(amax, ssr, red); // its barriers also publish sx0
    const double x0 = sx0;
    double tnorm = 0.0;
    if (amax >= 0x1p-480 && amax <= 0x1p+480) {
        tnorm = sqrt(ssr);
    } else if (amax > 0.0) {
        double ss = 0.0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = tid + q * HT;
            if (r >= c + 2 && r < m) {
                const double t = xr[q] / amax;
                ss += t * t;
            }
        }
        ss = hh_sum(ss, red);
        tnorm = amax * sqrt(ss);
    }
    double tj = 0.0, beta = x0, scal = 0.0;
    if (amax > 0.0) {
        const double nrm = hypot(x0, tnorm);
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tj = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
    }
    // v_j (unit at c+1, zero above) into V(:, j), the reduced column, w_j = V(:, :j)^T v_j
#pragma unroll
    for (int i = 0; i < NBH; ++i) loc[i] = 0.0;
    double *x = V + (int64_t)j * ldm;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = tid + q * HT;
        if (r >= m) continue;
        double v;
        if (r <= c) v = 0.0;
        else if (r == c + 1) v = 1.0;
        else v = (tj != 0.0) ? xr[q] * scal : 0.0;
        x[r] = v;
        if (r == c + 1) A[r + (int64_t)c * lda] = beta;
        else if (r > c + 1) A[r + (int64_t)c * lda] = 0.0;
        if (r >= c + 1) {
#pragma unroll
            for (int i = 0; i < NBH; ++i)
                if (i < j) loc[i] += vr[q][i] * v;
        }
    }
    hh_multi_sum(loc, j, red, sv);
    if (tid < j) { // T(:j, j) = -tau_j T(:j, :j) w_j, one thread per row
        W[tid + j * NBH] = sv[tid];
        double t = 0.0;
        for (int l = tid; l < j; ++l) t += sT[tid + l * NBH] * sv[l];
        Tm[tid + j * NBH] = -tj * t;
    } else if (tid < NBH) {
        Tm[tid + j * NBH] = (tid == j) ? tj : 0.0;
    }
    if (tid == 0) tau[j] = tj;
}

// Partial sums of y = A(:, c+1:m) v(c+1:m) for column chunks: grid (row
// blocks of 256, nchunk); part[q * m + r].
__global__ void __launch_bounds__(256) k_hh_gemv(const double *A, int64_t lda, int m, int c, const double *v,
                                                 double *part, int nchunk)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    const int c0 = c + 1, ncol = m - c0;
    const int per = (ncol + nchunk - 1) / nchunk;
    const int lo = c0 + q * per, hi = min(m, lo + per);
    if (r >= m) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int col = lo;
    for (; col + 3 < hi; col += 4) {
        s0 += A[r + (int64_t)col * lda] * v[col];
        s1 += A[r + (int64_t)(col + 1) * lda] * v[col + 1];
        s2 += A[r + (int64_t)(col + 2) * lda] * v[col + 2];
        s3 += A[r + (int64_t)(col + 3) * lda] * v[col + 3];
    }
    for (; col < hi; ++col) s0 += A[r + (int64_t)col * lda] * v[col];
    part[(int64_t)q * m + r] = (s0 + s1) + (s2 + s3);
}

// Spike reflector of a large AED window (Sec. 2.5): g = s * Z(0, 0:m) (row 0
// of the window's factor), reflector P = I - tau u u^T with P g = beta e_1;
// u, tau and beta go to hv (m + 2 doubles: u, tau, beta).  One workgroup.
__global__ void __launch_bounds__(HT) k_hh_spike(const double *Z, int64_t ldz, int m, double s, double *hv)
{
    __shared__ double red[16];
    const int tid = threadIdx.x;
    double amax = 0.0;
    for (int i = 1 + tid; i < m; i += HT) amax = fmax(amax, fabs(s * Z[(int64_t)i * ldz]));
    amax = hh_max(amax, red);
    double ss = 0.0;
    if (amax > 0.0)
        for (int i = 1 + tid; i < m; i += HT) {
            const double t = s * Z[(int64_t)i * ldz] / amax;
            ss += t * t;
        }
    ss = hh_sum(ss, red);
    const double x0 = s * Z[0];
    double tj = 0.0, beta = x0, scal = 0.0;
    if (amax > 0.0) {
        const double nrm = hypot(x0, amax * sqrt(ss));
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tj = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
    }
    for (int i = tid; i < m; i += HT) hv[i] = (i == 0) ? 1.0 : ((tj != 0.0) ? s * Z[(int64_t)i * ldz] * scal : 0.0);
    if (tid == 0) {
        hv[m] = tj;
        hv[m + 1] = beta;
    }
}

// One reflector u (length m, from hv) applied from the left to columns
// 0..ncol-1 of M (rows 0..m-1): one thread per column.
__global__ void k_hh_refl_left(double *M, int64_t ldm, int m, int ncol, const double *hv)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncol) return;
    const double t = hv[m];
    if (t == 0.0) return;
    double *x = M + (int64_t)col * ldm;
    double d = 0.0;
    for (int i = 0; i < m; ++i) d += hv[i] * x[i];
    d *= t;
    for (int i = 0; i < m; ++i) x[i] -= d * hv[i];
}

// The same reflector from the right to rows 0..nrow-1 of M (columns 0..m-1):
// one thread per row.
__global__ void k_hh_refl_right(double *M, int64_t ldm, int m, int nrow, const double *hv)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nrow) return;
    const double t = hv[m];
    if (t == 0.0) return;
    double d = 0.0;
    for (int i = 0; i < m; ++i) d += M[row + (int64_t)i * ldm] * hv[i];
    d *= t;
    for (int i = 0; i < m; ++i) M[row + (int64_t)i * ldm] -= d * hv[i];
}

size_t hess_ws_doubles(int m, int nr, int nz)
{
    const size_t mm = (size_t)std::max(m, 1);
    const size_t nchunk = 64;
    // V, Y, VT (m x NBH), T, W (NBH x NBH), tau (NBH), partials (nchunk x m),
    // WL (NBH x (m + nr)), ZW, ZT (nz x NBH), spike vector (m + 2)
    return 3 * mm * NBH + 2 * (size_t)NBH * NBH + NBH + nchunk * mm + (size_t)NBH * (mm + nr) +
           2 * (size_t)std::max(nz, 1) * NBH + mm + 2;
}

hipError_t hess_reduce(double *A, int64_t lda, int m, int nr, double *Z, int64_t ldz, int nz, double *ws,
                       hipStream_t s)
{
    if (m < 3) return hipSuccess;
    const size_t mm = (size_t)m;
    double *V = ws, *Y = V + mm * NBH, *VT = Y + mm * NBH;
    double *Tm = VT + mm * NBH, *W = Tm + NBH * NBH, *tau = W + NBH * NBH;
    double *part = tau + NBH;
    // chunks of columns for the GEMV partials: about 1024 workgroups in all
    const int rblk = (m + 255) / 256;
    const int nchunk_max = 64;
    double *WL = part + (size_t)nchunk_max * mm;
    double *ZW = WL + (size_t)NBH * (mm + nr);
    double *ZT = ZW + (size_t)std::max(nz, 1) * NBH;
    hipError_t e;
    for (int k = 0; k < m - 2; k += NBH) {
        const int nb = std::min(NBH, m - 2 - k);
        int nchunk = 1;
        // columns of at most 2 HT rows: the register-resident column kernel
        auto col = (m <= 2 * HT) ? k_hh_col2 : k_hh_col;
        for (int j = 0; j < nb; ++j) {
            const int c = k + j;
            hipLaunchKernelGGL(col, dim3(1), dim3(HT), 0, s, A, lda, m, k, j, 1, V, Y, Tm, W, tau, part, nchunk);
            const int ncol = m - (c + 1);
            nchunk = std::max(1, std::min(nchunk_max, std::min(ncol / 16, (1024 + rblk - 1) / rblk)));
            hipLaunchKernelGGL(k_hh_gemv, dim3(rblk, nchunk), dim3(256), 0, s, A, lda, m, c, V + (size_t)j * mm,
                               part, nchunk);
        }
        // complete Y(:, nb-1)
        hipLaunchKernelGGL(col, dim3(1), dim3(HT), 0, s, A, lda, m, k, nb, 0, V, Y, Tm, W, tau, part, nchunk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int c1 = k + nb; // first column right of the panel
        const int r0 = k + 1;  // first row the reflectors touch
        // right: A(0:m, c1:m) -= Y V(c1:m, :)^T
        if ((e = gemm_mfma(0, m, m - c1, nb, -1.0, Y, m, 0, V + c1, m, 1, 1.0, A + (int64_t)c1 * lda, lda, s)) !=
            hipSuccess)
            return e;
        // left: M = A(r0:m, c1:m+nr);  WL = V(r0:m, :)^T M;  M -= (V T^T)(r0:m, :) WL
        const int ncl = m + nr - c1;
        if ((e = gemm_mfma(0, nb, ncl, m - r0, 1.0, V + r0, m, 1, A + r0 + (int64_t)c1 * lda, lda, 0, 0.0, WL, NBH,
                         s)) != hipSuccess)
            return e;
        if ((e = gemm_mfma(0, m - r0, nb, nb, 1.0, V + r0, m, 0, Tm, NBH, 1, 0.0, VT + r0, m, s)) != hipSuccess)
            return e;
        if ((e = gemm_mfma(0, m - r0, ncl, nb, -1.0, VT + r0, m, 0, WL, NBH, 0, 1.0, A + r0 + (int64_t)c1 * lda, lda,
                         s)) != hipSuccess)
            return e;
        // Z(0:nz, r0:m) <- Z (I - V T V^T):  ZW = Z V;  ZT = ZW T;  Z -= ZT V^T
        if (Z && nz > 0) {
            if ((e = gemm_mfma(0, nz, nb, m - r0, 1.0, Z + (int64_t)r0 * ldz, ldz, 0, V + r0, m, 0, 0.0, ZW, nz, s)) !=
                hipSuccess)
                return e;
            if ((e = gemm_mfma(0, nz, nb, nb, 1.0, ZW, nz, 0, Tm, NBH, 0, 0.0, ZT, nz, s)) != hipSuccess) return e;
            if ((e = gemm_mfma(0, nz, m - r0, nb, -1.0, ZT, nz, 0, V + r0, m, 1, 1.0, Z + (int64_t)r0 * ldz, ldz, s)) !=
                hipSuccess)
                return e;
        }
    }
    return hipGetLastError();
}

hipError_t restore_blocked(double *T, int64_t ldt, int nw, int ns, double *Vw, int64_t ldv, int nv, double s,
                           double *ws, double *beta_dev, hipStream_t st)
{
    // the spike reflector on rows/columns 0..ns-1: T rows (all nw columns),
    // T columns (rows 0..ns-1; the rows below are zero there), V columns
    const size_t need = hess_ws_doubles(ns, nw - ns, nv);
    double *hv = ws + need - (ns + 2);
    hipLaunchKernelGGL(k_hh_spike, dim3(1), dim3(HT), 0, st, Vw, ldv, ns, s, hv);
    hipLaunchKernelGGL(k_hh_refl_left, dim3((nw + 255) / 256), dim3(256), 0, st, T, ldt, ns, nw, hv);
    hipLaunchKernelGGL(k_hh_refl_right, dim3((ns + 255) / 256), dim3(256), 0, st, T, ldt, ns, ns, hv);
    hipLaunchKernelGGL(k_hh_refl_right, dim3((nv + 255) / 256), dim3(256), 0, st, Vw, ldv, ns, nv, hv);
    hipError_t e = hipMemcpyAsync(beta_dev, hv + ns + 1, sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    return hess_reduce(T, ldt, ns, nw - ns, Vw, ldv, nv, ws, st);
}

} // namespace hqr
