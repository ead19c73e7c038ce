// Small Hermitian (real symmetric) problems in one workgroup each, with the
// whole matrix in LDS: the unblocked sampler of Sec. 2 (Theorem 2) run as
// written, pivot by pivot, on the lower triangle held in FP64.
//
// At pivot j, with d the current diagonal entry: keep j iff u_j < d, else
// d' = d - 1 (Prop. 4); then for every row i > j and column j < k <= i the
// trailing entry loses A_ij A_kj / d'. LDS keeps the unscaled columns (the
// W = L D of the factorization) until the end, so an update never reads a
// value another thread is rescaling; A receives L = W D^{-1}, D and, past
// npiv, the conditional kernel (the Schur complement) in the storage type.
//
// Layout: rows packed lower-triangular, row i at offset i (i + 1) / 2, so
// thread i owns row i (n <= 256 threads). In a step every active lane reads
// the same A_kj at the same time (a broadcast) and updates its own row. The
// cost is about n^2 / 2 dependent LDS updates on the busiest thread and one
// barrier per pivot, against the blocked path's launches per 64 pivots: for
// small n the workgroup finishes before the blocked path's first launches do.
// The arithmetic is FP64 for every precision (no split products at this size).
#include <atomic>

#include "dpp_internal.h"

namespace dpp {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t tri(int64_t i) { return i * (i + 1) / 2; }

template <typename T>
__global__ __launch_bounds__(kThreads) void small_ldlh(const DevProb* __restrict__ probs)
{
    extern __shared__ __attribute__((aligned(16))) double smem[];
    const DevProb P = probs[blockIdx.x];
    const int n = (int)P.n;
    const int npiv = (int)P.npiv;
    const int tid = threadIdx.x;
    double* const S = smem;               // packed lower triangle, n (n + 1) / 2
    double* const su = smem + tri(n);     // the uniforms of the decided indices

    // Load the lower triangle by columns (coalesced): column k, rows k..n-1.
    int64_t ldk;
    const T* __restrict__ K = first_source<T>(P, true, ldk);
    for (int k = 0; k < n; ++k)
        for (int i = k + tid; i < n; i += kThreads) S[tri(i) + k] = (double)K[i + (int64_t)k * ldk];
    for (int j = tid; j < npiv; j += kThreads) su[j] = P.u[j];
    __syncthreads();

    const int i = tid;  // the row this thread updates
    double* const row = S + tri(i < n ? i : 0);
    for (int j = 0; j < npiv; ++j) {
        const double d = S[tri(j) + j];
        const bool keep = su[j] < d;          // Bernoulli(d) with stream u_j
        const double dp = keep ? d : d - 1.0;  // Prop. 4 on rejection
        if (i > j && i < n) {
            const double l = row[j] / dp;
            for (int k = j + 1; k <= i; ++k) row[k] -= l * S[tri(k) + j];
        }
        __syncthreads();  // every update of this step read column j unchanged
        if (i == j) {
            row[j] = dp;
            P.mask[j] = keep ? 1 : 0;
            P.piv[j] = dp;
        }
        __syncthreads();  // the next pivot's diagonal and column are final
    }

    // A: L = W D^{-1} in the decided columns, D on their diagonal, and the
    // conditional kernel in the trailing block (written by columns).
    T* __restrict__ A = static_cast<T*>(P.A);
    for (int k = 0; k < n; ++k) {
        const double inv = k < npiv ? 1.0 / S[tri(k) + k] : 1.0;
        for (int r = k + tid; r < n; r += kThreads) {
            const double v = S[tri(r) + k];
            A[r + (int64_t)k * P.lda] = (T)(r > k && k < npiv ? v * inv : v);
        }
    }
}

}  // namespace

size_t small_ldlh_lds_bytes(int64_t n)
{
    return (size_t)(n * (n + 1) / 2 + n) * sizeof(double);
}

hipError_t launch_small_ldlh(int dtype, const DevProb* probs, int nprob, int64_t nmax,
                             hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    if (nmax > kSmallMax || (dtype != 0 && dtype != 1)) return hipErrorInvalidValue;
    const auto kd = small_ldlh<double>;
    const auto kf = small_ldlh<float>;
    // The dynamic-LDS limit is a per-device function attribute: set both
    // instances to the largest size once on each device the kernel runs on.
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
    if (!bit || !(attr_set.load() & bit)) {
        const int most = (int)small_ldlh_lds_bytes(kSmallMax);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kd),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, most);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(kf),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, most);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit);
    }
    const size_t lds = small_ldlh_lds_bytes(nmax);
    if (dtype == 0) hipLaunchKernelGGL(kd, dim3(nprob), dim3(kThreads), lds, s, probs);
    else hipLaunchKernelGGL(kf, dim3(nprob), dim3(kThreads), lds, s, probs);
    return hipGetLastError();
}

}  // namespace dpp
