// On-device conversion of a Hermitian L-ensemble kernel L into the marginal
// kernel K = I - (L + I)^{-1} (the conversion the paper's closing section
// names as the natural companion of the blocked sampler), by the sampler's own
// factorization engine:
//
//   With M = L + I (positive definite for positive semi-definite L) and n'
//   = n rounded up to a multiple of 64, the 2n' x 2n' symmetric matrix
//       G = [ M' I ]      M' = diag(M, I_{n'-n})
//           [ I  0 ]
//   factored through its first n' pivots has trailing Schur complement
//   0 - I M'^{-1} I = -M'^{-1} = diag(-M^{-1}, -I). The sampler's blocked
//   LDL^H with every pivot kept (u = 0 < d_j, since every pivot of a positive
//   definite M is positive) is exactly that partial factorization, so
//       K = I + G[n':n'+n, n':n'+n],
//   and ln det(L + I) = sum of the logs of the first n' pivots (the padding
//   pivots are 1). A pivot that is not positive (L not positive
//   semi-definite, or too ill-conditioned) shows as a rejected index.
//
// This file holds the three elementwise kernels around that factorization:
// building G (and u = 0) from L, reading K out of G (both triangles), and the
// per-problem status. All arithmetic is FP64 whatever the storage type of L and
// K.
#include "dpp_internal.h"

namespace dpp {
namespace {

constexpr int kTile = 64;
constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void lens_augment(const LensDesc* __restrict__ descs)
{
    const LensDesc D = descs[blockIdx.z];
    const int64_t m = 2 * D.np;
    const int64_t bi = blockIdx.y, bj = blockIdx.x;  // row and column tile
    if (bj > bi || bi * kTile >= m) return;          // lower tiles only
    const T* __restrict__ L = static_cast<const T*>(D.L);
    for (int e = threadIdx.x; e < kTile * kTile; e += kThreads) {
        const int64_t i = bi * kTile + e % kTile, j = bj * kTile + e / kTile;
        if (i >= m || j > i) continue;
        double v = 0.0;
        if (i < D.np) {                              // M' = diag(L + I, I)
            v = (i == j) ? 1.0 : 0.0;
            if (i < D.n) v += (double)L[i + j * D.ldl];
        } else if (j < D.np) {                       // the identity block below M'
            v = (i - D.np == j) ? 1.0 : 0.0;
        }
        D.aug[i + j * m] = v;
    }
    if (bi == 0 && bj == 0)
        for (int64_t j = threadIdx.x; j < m; j += kThreads) D.u[j] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void lens_extract(const LensDesc* __restrict__ descs)
{
    const LensDesc D = descs[blockIdx.z];
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bi * kTile >= D.n || bj * kTile >= D.n) return;
    const int64_t m = 2 * D.np;
    T* __restrict__ K = static_cast<T*>(D.K);
    for (int e = threadIdx.x; e < kTile * kTile; e += kThreads) {
        const int64_t i = bi * kTile + e % kTile, j = bj * kTile + e / kTile;
        if (i >= D.n || j >= D.n) continue;
        const int64_t r = D.np + (i > j ? i : j), c = D.np + (i > j ? j : i);  // lower triangle of G
        K[i + j * D.ldk] = (T)((i == j ? 1.0 : 0.0) + D.aug[r + c * m]);
    }
}

// info = 1 when a pivot of M' was not positive (a rejected index) or the
// factorization reported a zero or NaN pivot; logdet = ln det(L + I).
__global__ __launch_bounds__(kThreads) void lens_status(const LensDesc* __restrict__ descs)
{
    const LensDesc D = descs[blockIdx.x];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = *D.sinfo != 0;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < D.np; j += kThreads)
        if (D.mask[j] == 0) bad = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) {
        *D.info = bad;
        if (D.logdet) *D.logdet = *D.loglik;
    }
}

struct LensChunk {
    LensDesc d[kLensDescPerLaunch];
    int cnt;
};
static_assert(sizeof(LensChunk) <= 4096, "kernel arguments are limited to 4 KiB");

__global__ void store_lens_descs(LensChunk chunk, LensDesc* __restrict__ dst)
{
    const int i = threadIdx.x;
    if (i < chunk.cnt) dst[i] = chunk.d[i];
}

}  // namespace

hipError_t launch_store_lens_descs(const LensDesc* host, int cnt, LensDesc* dst, hipStream_t s)
{
    LensChunk chunk;
    for (int i = 0; i < cnt; ++i) chunk.d[i] = host[i];
    chunk.cnt = cnt;
    hipLaunchKernelGGL(store_lens_descs, dim3(1), dim3(64), 0, s, chunk, dst);
    return hipGetLastError();
}

hipError_t launch_lens_augment(int dtype, const LensDesc* descs, int count, int64_t mmax,
                               hipStream_t s)
{
    const unsigned t = (unsigned)((mmax + kTile - 1) / kTile);
    dim3 grid(t, t, (unsigned)count);
    if (dtype == 0) hipLaunchKernelGGL((lens_augment<double>), grid, dim3(kThreads), 0, s, descs);
    else hipLaunchKernelGGL((lens_augment<float>), grid, dim3(kThreads), 0, s, descs);
    return hipGetLastError();
}

hipError_t launch_lens_extract(int dtype, const LensDesc* descs, int count, int64_t nmax,
                               hipStream_t s)
{
    const unsigned t = (unsigned)((nmax + kTile - 1) / kTile);
    dim3 grid(t, t, (unsigned)count);
    if (dtype == 0) hipLaunchKernelGGL((lens_extract<double>), grid, dim3(kThreads), 0, s, descs);
    else hipLaunchKernelGGL((lens_extract<float>), grid, dim3(kThreads), 0, s, descs);
    return hipGetLastError();
}

hipError_t launch_lens_status(const LensDesc* descs, int count, hipStream_t s)
{
    hipLaunchKernelGGL(lens_status, dim3((unsigned)count), dim3(kThreads), 0, s, descs);
    return hipGetLastError();
}

}  // namespace dpp
