// Diagonal-block kernel, Hermitian (LDL^H) form; see leaf_common.h.
#include "leaf_common.h"

namespace dpp {
namespace {

using namespace leaf;

// ------------------------------------------------------------------- LDL^H
template <typename T, bool SPLIT>
__global__ __launch_bounds__(kRowsPerWG) void leaf_ldlh(const DevProb* __restrict__ probs, int64_t c0,
                                                 int64_t j0, int ss)
{
    const DevProb P = probs[blockIdx.y];
    const int64_t n = P.n;
    if (c0 >= n) return;
    const int bs = (int)((n - c0) < L ? (n - c0) : L);
    const int64_t row0 = c0 + bs + (int64_t)blockIdx.x * kRowsPerWG;
    if (blockIdx.x > 0 && row0 >= n) return;

    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda;

    __shared__ double sL[L * L];  // sL[t*L + k] = L11[k][t] (column t), zero elsewhere
    __shared__ double sD[L];      // D1 (modified pivots)
    __shared__ double sB[L];      // broadcast column of the current pivot

    const int tid = threadIdx.x;
    if (tid < L) {
        const int lane = tid;
        // Row `lane` of the block, lower part; the rest starts at 0 and only
        // ever receives finite garbage that no decision reads.
        double a[L];
#pragma unroll
        for (int k = 0; k < L; ++k)
            a[k] = (lane < bs && k <= lane) ? (double)A[(c0 + lane) + (c0 + k) * lda] : 0.0;
        const double ul = lane < bs ? P.u[c0 + lane] : 2.0;
        double mydp = 1.0;
        int mykeep = 0;

#pragma unroll
        for (int j = 0; j < L; ++j) {
            if (j < bs) {
                const double d = readlane_d(a[j], j);   // A[j][j]
                const double uj = readlane_d(ul, j);
                const bool keep = uj < d;                // Bernoulli(d) with stream u_j
                const double dp = keep ? d : d - 1.0;   // Prop. 4 on rejection
                const double c = a[j];                   // A[lane][j], unscaled
                sB[lane] = c;
                __builtin_amdgcn_wave_barrier();
                const double l = c / dp;
#pragma unroll
                for (int k = 0; k < L; ++k)
                    if (k > j) a[k] -= l * sB[k];  // A[lane][k] -= l_lane * A[k][j]
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
        for (int k = 0; k < L; ++k) sL[k * L + lane] = (k < lane && lane < bs) ? a[k] : 0.0;
        sD[lane] = (lane < bs) ? mydp : 1.0;

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

    // Panel solve: row r of A21 becomes W = A21 L11^{-T} (= L21 D1), then
    // L21 = W D1^{-1}. Rows below a block exist only when the block is a full
    // 64 wide (a ragged block is the last one), so bs == L here.
    const int64_t r = row0 + tid;
    if (r < n) {
        // Strip = columns [c0, c0+64) from row row0 on; lane offset tid rows,
        // column k at k * lda elements.
        const __amdgpu_buffer_rsrc_t rs =
            strip_rsrc(A + row0 + c0 * lda, (int64_t)L * lda * (int64_t)sizeof(T));
        const int voff = tid * (int)sizeof(T);
        const int cstride = (int)(lda * (int64_t)sizeof(T));
        double x[L];
#pragma unroll
        for (int k = 0; k < L; ++k) x[k] = buf_load<T>(rs, voff, k * cstride);
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const double wt = x[t];
#pragma unroll
            for (int k = 0; k < L; ++k)
                if (k > t) x[k] -= wt * sL[t * L + k];
        }
        if constexpr (SPLIT) {
            // W = L21 D1 first, then x becomes L21 in place.
            const int64_t off = r * ss + (int)(c0 - j0);
            store_split_row(split_plane(P.split, n, ss, 2) + off,
                            split_plane(P.split, n, ss, 3) + off, x, L);
        }
#pragma unroll
        for (int k = 0; k < L; ++k) {
            x[k] = x[k] / sD[k];
            buf_store<T>(x[k], rs, voff, k * cstride);
        }
        if constexpr (SPLIT) {
            const int64_t off = r * ss + (int)(c0 - j0);
            store_split_row(split_plane(P.split, n, ss, 0) + off,
                            split_plane(P.split, n, ss, 1) + off, x, L);
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
    if (split) hipLaunchKernelGGL((leaf_ldlh<T, true>), grid, block, 0, s, probs, c0, j0, ss);
    else hipLaunchKernelGGL((leaf_ldlh<T, false>), grid, block, 0, s, probs, c0, j0, ss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_ldlh(int dtype, bool split, const DevProb* probs, int nprob, int64_t nmax,
                      int64_t c0, int64_t j0, int ss, hipStream_t s)
{
    if (dtype == 0) return launch_t<double>(split, probs, nprob, nmax, c0, j0, ss, s);
    return launch_t<float>(split, probs, nprob, nmax, c0, j0, ss, s);
}

}  // namespace dpp
