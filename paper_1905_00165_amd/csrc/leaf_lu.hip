// Diagonal-block kernel, general (LU) form; see leaf_common.h.
#include "leaf_common.h"

namespace dpp {
namespace {

using namespace leaf;

// ---------------------------------------------------------------------- LU
template <typename T, bool SPLIT>
__global__ __launch_bounds__(kRowsPerWG) void leaf_lu(const DevProb* __restrict__ probs, int64_t c0,
                                               int64_t j0, int ss)
{
    const DevProb P = probs[blockIdx.y];
    const int64_t n = P.n;
    if (c0 >= n) return;
    const int bs = (int)((n - c0) < L ? (n - c0) : L);
    const int64_t idx0 = c0 + bs + (int64_t)blockIdx.x * kRowsPerWG;
    if (blockIdx.x > 0 && idx0 >= n) return;

    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda;

    __shared__ double sL[L * L];  // sL[t*L + k] = L11[k][t]  (strict lower, column t)
    __shared__ double sU[L * L];  // sU[t*L + k] = U11[t][k]  (upper with diagonal, row t)
    __shared__ double sB[L];      // broadcast row of the current pivot

    const int tid = threadIdx.x;
    if (tid < L) {
        const int lane = tid;
        double a[L];  // row `lane` of the block
#pragma unroll
        for (int k = 0; k < L; ++k)
            a[k] = (lane < bs && k < bs) ? (double)A[(c0 + lane) + (c0 + k) * lda] : 0.0;
        const double ul = lane < bs ? P.u[c0 + lane] : 2.0;
        double mydp = 1.0;
        int mykeep = 0;

#pragma unroll
        for (int j = 0; j < L; ++j) {
            if (j < bs) {
                const double d = readlane_d(a[j], j);
                const double uj = readlane_d(ul, j);
                const bool keep = uj < d;
                const double dp = keep ? d : d - 1.0;
                if (lane == j) {
#pragma unroll
                    for (int k = 0; k < L; ++k)
                        if (k > j) sB[k] = a[k];  // row j of U
                }
                __builtin_amdgcn_wave_barrier();
                // Only rows below the pivot are updated: rows <= j already hold
                // final entries of U.
                const double l = (lane > j) ? a[j] / dp : 0.0;
#pragma unroll
                for (int k = 0; k < L; ++k)
                    if (k > j) a[k] -= l * sB[k];
                __builtin_amdgcn_wave_barrier();
                if (lane == j) {
                    a[j] = dp;
                    mydp = dp;
                    mykeep = keep ? 1 : 0;
                } else if (lane > j) {
                    a[j] = l;
                }
            }
        }

#pragma unroll
        for (int k = 0; k < L; ++k) {
            sL[k * L + lane] = (k < lane && lane < bs) ? a[k] : 0.0;
            sU[lane * L + k] = (k >= lane && lane < bs) ? a[k] : (k == lane ? 1.0 : 0.0);
        }

        // The factored block goes to the workspace strip, not to A: other
        // workgroups of this launch may still be loading the original block
        // from A for their own copy of the chain. A later launch copies the
        // strip into A (no kernel reads the diagonal blocks from A).
        if (blockIdx.x == 0 && lane < bs) {
            double* blk = P.diag + (c0 / L) * (L * L);
#pragma unroll
            for (int k = 0; k < L; ++k) blk[k * L + lane] = a[k];
            P.mask[c0 + lane] = (uint8_t)mykeep;
            P.piv[c0 + lane] = mydp;
        }
    }
    __syncthreads();

    // Rows below and columns right of a block exist only when the block is a
    // full 64 wide (a ragged block is the last one), so bs == L here.
    const int64_t r = idx0 + tid;
    if (r < n) {
        const int voff = tid * (int)sizeof(T);
        const int cstride = (int)(lda * (int64_t)sizeof(T));
        // Column panel: L21 = A21 U11^{-1}, row r: x U11 = a.
        {
            const __amdgpu_buffer_rsrc_t rs =
                strip_rsrc(A + idx0 + c0 * lda, (int64_t)L * lda * (int64_t)sizeof(T));
            double x[L];
#pragma unroll
            for (int k = 0; k < L; ++k) x[k] = buf_load<T>(rs, voff, k * cstride);
#pragma unroll
            for (int t = 0; t < L; ++t) {
                x[t] = x[t] / sU[t * L + t];
                const double xt = x[t];
#pragma unroll
                for (int k = 0; k < L; ++k)
                    if (k > t) x[k] -= xt * sU[t * L + k];
            }
#pragma unroll
            for (int k = 0; k < L; ++k) buf_store<T>(x[k], rs, voff, k * cstride);
            if constexpr (SPLIT) {
                const int64_t off = r * ss + (int)(c0 - j0);
                store_split_row(split_plane(P.split, n, ss, 0) + off,
                                split_plane(P.split, n, ss, 1) + off, x, L);
            }
        }
        // Row panel: U12 = L11^{-1} A12, column r: L11 y = a (64 contiguous
        // entries of column r).
        {
            T* col = A + c0 + r * lda;
            double y[L];
#pragma unroll
            for (int k = 0; k < L; ++k) y[k] = (double)col[k];
#pragma unroll
            for (int t = 0; t < L; ++t) {
                const double yt = y[t];
#pragma unroll
                for (int k = 0; k < L; ++k)
                    if (k > t) y[k] -= yt * sL[t * L + k];
            }
#pragma unroll
            for (int k = 0; k < L; ++k) col[k] = (T)y[k];
            if constexpr (SPLIT) {
                const int64_t off = r * ss + (int)(c0 - j0);
                store_split_row(split_plane(P.split, n, ss, 2) + off,
                                split_plane(P.split, n, ss, 3) + off, y, L);
            }
        }
    }
}

template <typename T>
hipError_t launch_t(bool split, const DevProb* probs, int nprob, int64_t nmax, int64_t c0,
                    int64_t j0, int ss, hipStream_t s)
{
    const int64_t below = nmax - c0 - L;
    const int gx = below > 0 ? (int)((below + kRowsPerWG - 1) / kRowsPerWG) : 1;
    dim3 grid(gx, nprob), block(kRowsPerWG);
    if (split) hipLaunchKernelGGL((leaf_lu<T, true>), grid, block, 0, s, probs, c0, j0, ss);
    else hipLaunchKernelGGL((leaf_lu<T, false>), grid, block, 0, s, probs, c0, j0, ss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_lu(int dtype, bool split, const DevProb* probs, int nprob, int64_t nmax,
                      int64_t c0, int64_t j0, int ss, hipStream_t s)
{
    if (dtype == 0) return launch_t<double>(split, probs, nprob, nmax, c0, j0, ss, s);
    return launch_t<float>(split, probs, nprob, nmax, c0, j0, ss, s);
}

}  // namespace dpp
