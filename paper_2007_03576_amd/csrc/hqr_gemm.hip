// Off-diagonal update products of libhqr on the FP64 matrix cores of gfx950.
//
// After a diagonal window has been processed (bulge chasing, AED, small Schur
// solve) its accumulated orthogonal factor U (order K) must be applied to the
// rest of the matrix: from the left to the rows of the window right of it,
// from the right to the columns above it, and to Q (Sec. 2.3 and Sec. 3.2.1,
// 'left update' / 'right update' tasks).  Each workgroup owns a panel of
// `tile` rows (right update) or columns (left update) of X, stages the whole
// K-long panel in LDS, and overwrites it with the product, so the update is
// in place without a second buffer.  Both sides compute D = U^T * P^T with
// V_MFMA_F64_16X16X4_F64: the A operand comes from U^T (stored transposed so
// that the 16 lanes of a fragment read 128 contiguous bytes), the B operand
// from the LDS panel.
#include "hqr_common.h"

namespace hqr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int UPD_THREADS = 256;

// Panel rows/columns per workgroup: 64, fewer when the K16 x (tile + 4) panel
// would not fit the 160 KB of LDS (K16 <= 1024, see MAX_UPDATE_K).
int update_tile(int K16, int side)
{
    (void)side;
    int t = 64;
    while (t > 16 && (size_t)K16 * (size_t)(t + 4) * 8 > 160 * 1024) t /= 2;
    return t;
}

// Output strips of 16 per wave item, and wave items per workgroup.
constexpr int SG = 6;
constexpr int UPD_WAVES = UPD_THREADS / 64;

__global__ void __launch_bounds__(UPD_THREADS) k_update(UpdBatch B)
{
    extern __shared__ __align__(16) double Pt[];
    int bid = blockIdx.x;
    int j = 0;
    while (j + 1 < B.njobs && bid >= B.first_tile[j + 1]) ++j;
    const UpdJob J = B.job[j];
    const int t = bid - B.first_tile[j];
    const int TA = J.tile;
    const int TAP = TA + 4;
    const int a_base = t * TA;
    const int cnt = min(TA, J.count - a_base);
    const int K = J.K, K16 = J.K16;
    const int tid = threadIdx.x;
    double *X = J.X;
    const int64_t ldx = J.ldx;
    // stage the panel: Pt[k*TAP + a]
    if (J.side == 0) {
        for (int it = tid; it < K16 * TA; it += UPD_THREADS) {
            int a = it % TA, k = it / TA;
            double v = 0.0;
            if (a < cnt && k < K) v = X[(int64_t)(a_base + a) + (int64_t)k * ldx];
            Pt[k * TAP + a] = v;
        }
    } else {
        for (int it = tid; it < K16 * TA; it += UPD_THREADS) {
            int k = it % K16, a = it / K16;
            double v = 0.0;
            if (a < cnt && k < K) v = X[(int64_t)k + (int64_t)(a_base + a) * ldx];
            Pt[k * TAP + a] = v;
        }
    }
    __syncthreads();
    // work items: (panel tile of 16 rows/columns, group of up to SG output
    // strips of 16); with K <= 96 the four waves take one panel tile each and
    // every strip, so they carry equal MFMA work.  The update is in place, so
    // the whole K-long panel of a tile belongs to one workgroup: it reads all
    // of it before it writes any output.
    const int lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int ntj = K16 / 16;
    const int nta = (cnt + 15) / 16;
    const int ngrp = (ntj + SG - 1) / SG;
    const double *Ut = J.Ut;
    for (int item = wave; item < nta * ngrp; item += UPD_WAVES) {
        const int at = item % nta, j0 = (item / nta) * SG;
        const int nj = min(SG, ntj - j0);
        dbl4 acc[SG];
#pragma unroll
        for (int q = 0; q < SG; ++q) acc[q] = (dbl4){0.0, 0.0, 0.0, 0.0};
        const double *ua = Ut + j0 * 16 + l16 + (int64_t)lq * K16;
        const double *pb = Pt + lq * TAP + at * 16 + l16;
#pragma unroll 2
        for (int k0 = 0; k0 < K16; k0 += 4) {
            const double bf = pb[k0 * TAP];
            const double *uk = ua + (int64_t)k0 * K16;
#pragma unroll
            for (int q = 0; q < SG; ++q)
                if (q < nj) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(uk[q * 16], bf, acc[q], 0, 0, 0);
        }
        // D[i][n]: i = lq + 4r (row of U^T, i.e. output index j), n = l16 (panel index a);
        // lane layout of the f64 16x16x4 result checked on gfx950
        const int a = at * 16 + l16;
        if (a >= cnt) continue;
#pragma unroll
        for (int q = 0; q < SG; ++q) {
            if (q >= nj) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jj = (j0 + q) * 16 + lq + 4 * r;
                if (jj >= K) continue;
                const double v = acc[q][r];
                if (J.side == 0)
                    X[(int64_t)(a_base + a) + (int64_t)jj * ldx] = v;
                else
                    X[(int64_t)jj + (int64_t)(a_base + a) * ldx] = v;
            }
        }
    }
}

hipError_t launch_updates(const UpdBatch &b, hipStream_t s)
{
    if (b.njobs <= 0) return hipSuccess;
    int total = b.first_tile[b.njobs];
    if (total <= 0) return hipSuccess;
    size_t lds = 0;
    for (int j = 0; j < b.njobs; ++j) {
        size_t need = (size_t)b.job[j].K16 * (size_t)(b.job[j].tile + 4) * sizeof(double);
        if (need > lds) lds = need;
    }
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_update, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_update, dim3(total), dim3(UPD_THREADS), lds, s, b);
    return hipGetLastError();
}

} // namespace hqr
