// Off-diagonal update products of libhqr on the FP64 matrix cores of gfx950.
//
// After a diagonal window has been processed (bulge chasing, AED, small Schur
// solve) its accumulated orthogonal factor U (order K) must be applied to the
// rest of the matrix: from the left to the rows of the window right of it,
// from the right to the columns above it, and to Q (Sec. 2.3 and Sec. 3.2.1,
// 'left update' / 'right update' tasks).  Windows of order <= 96 (bulge
// chasing, AED and deflation windows) are applied in place by k_update_s: U
// in LDS, each wave's 16-row (or 16-column) strip of X in registers, read
// whole before it is overwritten.  Larger windows (large AED windows) are
// applied out of place by a tiled MFMA product into a workspace and copied
// back.  All products use V_MFMA_F64_16X16X4_F64.
#include "hqr_common.h"
#include <mutex>
#include <vector>

namespace hqr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int UPD_THREADS = 256;

// Panel rows/columns per workgroup of k_update_s (four waves of 16).
int update_tile(int K16, int side)
{
    (void)K16;
    (void)side;
    return 64;
}

// C(0:mm, 0:nn) = beta C + alpha op(A) op(B), inner dimension kk, FP64 MFMA,
// 64 x 64 tiles; opA/opB 0 = as stored (column major), 1 = transposed.  The
// tag only names the caller in profiles (0: Hessenberg reduction, 1: updates
// of windows larger than 96).
constexpr int HGT = 64, HGK = 16, HGP = 4;
template <int TAG>
__global__ void __launch_bounds__(256) k_gemm64(int mm, int nn, int kk, double alpha, const double *A, int64_t lda,
                                                 int opA, const double *B, int64_t ldb, int opB, double beta,
                                                 double *C, int64_t ldc)
{
    __shared__ double As[HGK][HGT + HGP];
    __shared__ double Bs[HGK][HGT + HGP];
    const int m0 = blockIdx.x * HGT, n0 = blockIdx.y * HGT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int l16 = lane & 15, lq = lane >> 4;
    dbl4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = (dbl4){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < kk; k0 += HGK) {
        for (int it = tid; it < HGT * HGK; it += 256) {
            int mi, ki;
            if (opA == 0) {
                mi = it % HGT;
                ki = it / HGT;
            } else {
                ki = it % HGK;
                mi = it / HGK;
            }
            const int gm = m0 + mi, gk = k0 + ki;
            double v = 0.0;
            if (gm < mm && gk < kk) v = (opA == 0) ? A[gm + (int64_t)gk * lda] : A[gk + (int64_t)gm * lda];
            As[ki][mi] = v;
            int nj, kj;
            if (opB == 0) {
                kj = it % HGK;
                nj = it / HGK;
            } else {
                nj = it % HGT;
                kj = it / HGT;
            }
            const int gn = n0 + nj, gk2 = k0 + kj;
            double w = 0.0;
            if (gn < nn && gk2 < kk) w = (opB == 0) ? B[gk2 + (int64_t)gn * ldb] : B[gn + (int64_t)gk2 * ldb];
            Bs[kj][nj] = w;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < HGK; ks += 4) {
            double af[2], bf[2];
            for (int a = 0; a < 2; ++a) af[a] = As[ks + lq][wm + a * 16 + l16];
            for (int b = 0; b < 2; ++b) bf[b] = Bs[ks + lq][wn + b * 16 + l16];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane holds D[lq + 4r][l16] of each 16 x 16 block
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + a * 16 + lq + 4 * r;
                const int gn = n0 + wn + b * 16 + l16;
                if (gm < mm && gn < nn) {
                    double *p = C + gm + (int64_t)gn * ldc;
                    *p = (beta == 0.0 ? 0.0 : beta * *p) + alpha * acc[a][b][r];
                }
            }
}

hipError_t gemm_mfma(int tag, int mm, int nn, int kk, double alpha, const double *A, int64_t lda, int opA,
                     const double *B, int64_t ldb, int opB, double beta, double *C, int64_t ldc, hipStream_t s)
{
    if (mm <= 0 || nn <= 0) return hipSuccess;
    dim3 grid((mm + HGT - 1) / HGT, (nn + HGT - 1) / HGT);
    if (tag == 0)
        hipLaunchKernelGGL(k_gemm64<0>, grid, dim3(256), 0, s, mm, nn, kk, alpha, A, lda, opA, B, ldb, opB, beta, C, ldc);
    else
        hipLaunchKernelGGL(k_gemm64<1>, grid, dim3(256), 0, s, mm, nn, kk, alpha, A, lda, opA, B, ldb, opB, beta, C, ldc);
    return hipGetLastError();
}

// Windows of order K <= 96 (chase, AED and deflation windows): U is staged
// in LDS once per workgroup (Us[k * ustr + j] = U(k, j), zero outside K), and
// each wave keeps the whole K-long strip of its 16 panel rows/columns in
// registers, read before anything is written, so the update stays in place
// and the LDS holds only U (two workgroups per CU).  Side 0 (X <- X U, rows of
// X): D[j][a] = sum_k U(k, j) X(a, k), U fragments as the A operand.  Side 1
// (X <- U^T X, columns of X): D[a][j] = sum_k X(k, a) U(k, j), U fragments as
// the B operand, so the 16 lanes of a result row write 16 consecutive rows j
// of a column.
constexpr int SK_MAX = 96;
constexpr int SK_STEPS = SK_MAX / 4;

__global__ void __launch_bounds__(UPD_THREADS) k_update_s(UpdBatch B)
{
    extern __shared__ __align__(16) double Us[];
    int bid = blockIdx.x;
    int j = 0;
    while (j + 1 < B.njobs && bid >= B.first_tile[j + 1]) ++j;
    const UpdJob J = B.job[j];
    const int t = bid - B.first_tile[j];
    const int a_base = t * J.tile;
    const int cnt = min(J.tile, J.count - a_base);
    const int K = J.K, K16 = J.K16, ustr = K16 + 2;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    double *X = J.X;
    const int64_t ldx = J.ldx;
    // this wave's panel strip: rows/columns a_base + 16 wave + l16, k = k0 + lq
    const int a = wave * 16 + l16;
    const bool arow = a < cnt;
    double pf[SK_STEPS];
#pragma unroll
    for (int s4 = 0; s4 < SK_STEPS; ++s4) {
        const int k = 4 * s4 + lq;
        double v = 0.0;
        if (4 * s4 < K16 && arow && k < K)
            v = (J.side == 0) ? X[(int64_t)(a_base + a) + (int64_t)k * ldx] : X[(int64_t)k + (int64_t)(a_base + a) * ldx];
        pf[s4] = v;
    }
    const double *Ut = J.Ut;
    for (int it = tid; it < K16 * K16; it += UPD_THREADS) {
        const int jj = it % K16, k = it / K16;
        Us[k * ustr + jj] = (k < K && jj < K) ? Ut[(int64_t)k * K16 + jj] : 0.0;
    }
    __syncthreads();
    if (wave * 16 >= cnt) return;
    const int ntj = K16 / 16;
    dbl4 acc[SK_MAX / 16];
#pragma unroll
    for (int q = 0; q < SK_MAX / 16; ++q) acc[q] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const double *ub = Us + lq * ustr + l16;
    if (J.side == 0) {
#pragma unroll
        for (int s4 = 0; s4 < SK_STEPS; ++s4) {
            if (4 * s4 >= K16) break;
            const double *uk = ub + 4 * s4 * ustr;
#pragma unroll
            for (int q = 0; q < SK_MAX / 16; ++q)
                if (q < ntj) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(uk[q * 16], pf[s4], acc[q], 0, 0, 0);
        }
        // D[j][a]: j = 16 q + lq + 4 r, a = l16
        if (!arow) return;
#pragma unroll
        for (int q = 0; q < SK_MAX / 16; ++q) {
            if (q >= ntj) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jj = q * 16 + lq + 4 * r;
                if (jj < K) X[(int64_t)(a_base + a) + (int64_t)jj * ldx] = acc[q][r];
            }
        }
    } else {
#pragma unroll
        for (int s4 = 0; s4 < SK_STEPS; ++s4) {
            if (4 * s4 >= K16) break;
            const double *uk = ub + 4 * s4 * ustr;
#pragma unroll
            for (int q = 0; q < SK_MAX / 16; ++q)
                if (q < ntj) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(pf[s4], uk[q * 16], acc[q], 0, 0, 0);
        }
        // D[a][j]: a = 16 wave + lq + 4 r, j = 16 q + l16
#pragma unroll
        for (int q = 0; q < SK_MAX / 16; ++q) {
            if (q >= ntj) continue;
            const int jj = q * 16 + l16;
            if (jj >= K) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ao = wave * 16 + lq + 4 * r;
                if (ao < cnt) X[(int64_t)jj + (int64_t)(a_base + ao) * ldx] = acc[q][r];
            }
        }
    }
}

// Workspace of the out-of-place products, one per (device, stream), grown on
// demand (the stream is synchronized before a smaller buffer is released).
struct BigWs {
    int dev;
    hipStream_t s;
    double *p;
    size_t n;
};
static std::mutex g_bigws_mu;
static std::vector<BigWs> g_bigws;

static double *big_ws(hipStream_t s, size_t need)
{
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_bigws_mu);
    for (auto &w : g_bigws)
        if (w.dev == dev && w.s == s) {
            if (w.n < need) {
                hipStreamSynchronize(s);
                hipFree(w.p);
                w.p = nullptr;
                w.n = 0;
                if (hipMalloc((void **)&w.p, need * sizeof(double)) != hipSuccess) return nullptr;
                w.n = need;
            }
            return w.p;
        }
    BigWs w{dev, s, nullptr, 0};
    if (hipMalloc((void **)&w.p, need * sizeof(double)) != hipSuccess) return nullptr;
    w.n = need;
    g_bigws.push_back(w);
    return w.p;
}

void free_update_ws()
{
    std::lock_guard<std::mutex> lk(g_bigws_mu);
    for (auto &w : g_bigws) {
        hipSetDevice(w.dev);
        hipStreamSynchronize(w.s);
        hipFree(w.p);
    }
    g_bigws.clear();
}

// Windows of order K <= 96 go to k_update_s in one launch.  A larger window's
// factor (large AED windows) is applied out of place: W = X U (rows) or
// W = U^T X (columns) by the tiled MFMA product, then W is copied back into X.
hipError_t launch_updates(const UpdBatch &b, hipStream_t s)
{
    if (b.njobs <= 0) return hipSuccess;
    UpdBatch sm;
    sm.njobs = 0;
    sm.first_tile[0] = 0;
    int kmax = 0;
    for (int j = 0; j < b.njobs; ++j) {
        const UpdJob &J = b.job[j];
        if (J.count <= 0) continue;
        if (J.K16 <= SK_MAX) {
            UpdJob Js = J;
            Js.tile = 4 * 16;
            Js.tiles = (J.count + Js.tile - 1) / Js.tile;
            sm.job[sm.njobs] = Js;
            sm.first_tile[sm.njobs + 1] = sm.first_tile[sm.njobs] + Js.tiles;
            sm.njobs++;
            kmax = kmax > J.K16 ? kmax : J.K16;
            continue;
        }
        const size_t need = (size_t)J.count * (size_t)J.K;
        double *W = big_ws(s, need);
        if (!W) return hipErrorOutOfMemory;
        hipError_t e;
        if (J.side == 0) {
            // rows: W (count x K) = X (count x K) U, U(k, j) = Ut[k K16 + j]
            e = gemm_mfma(1, J.count, J.K, J.K, 1.0, J.X, J.ldx, 0, J.Ut, J.K16, 1, 0.0, W, J.count, s);
            if (e != hipSuccess) return e;
            e = hipMemcpy2DAsync(J.X, J.ldx * sizeof(double), W, (size_t)J.count * sizeof(double),
                                 (size_t)J.count * sizeof(double), J.K, hipMemcpyDeviceToDevice, s);
        } else {
            // columns: W (K x count) = U^T X (K x count)
            e = gemm_mfma(1, J.K, J.count, J.K, 1.0, J.Ut, J.K16, 0, J.X, J.ldx, 0, 0.0, W, J.K, s);
            if (e != hipSuccess) return e;
            e = hipMemcpy2DAsync(J.X, J.ldx * sizeof(double), W, (size_t)J.K * sizeof(double),
                                 (size_t)J.K * sizeof(double), J.count, hipMemcpyDeviceToDevice, s);
        }
        if (e != hipSuccess) return e;
    }
    if (sm.njobs == 0 || sm.first_tile[sm.njobs] <= 0) return hipSuccess;
    static bool attr_s = false;
    if (!attr_s) {
        hipError_t e = hipFuncSetAttribute((const void *)k_update_s, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr_s = true;
    }
    const size_t lds_s = (size_t)kmax * (size_t)(kmax + 2) * sizeof(double);
    hipLaunchKernelGGL(k_update_s, dim3(sm.first_tile[sm.njobs]), dim3(UPD_THREADS), lds_s, s, sm);
    return hipGetLastError();
}

} // namespace hqr
