// Log-likelihood, info word and decision diagnostics of each problem (gfx950).
//
// The likelihood of the returned sample is the product of the absolute values
// of the modified pivots (Theorem 2), so loglik = sum_j ln|d'_j| over the
// decided indices j < npiv (the probability of those decisions). The sum runs
// in a fixed order (each thread sums a contiguous chunk in index order, then a
// fixed binary tree), so the result is bitwise reproducible. info is the
// 1-based index of the first pivot that is exactly zero or NaN (0 if none).
//
// Diagnostics (optional): with d_j the pre-decision probability (d'_j if kept,
// d'_j + 1 if rejected, since a rejection subtracts 1, Prop. 4), the smallest
// |u_j - d_j| (how near a decision came to a tie), the number of d_j outside
// [-1e-12, 1 + 1e-12] and the largest distance of a d_j from [0, 1].
#include "dpp_internal.h"

namespace dpp {
namespace {

constexpr int kThreads = 256;
constexpr double kRangeSlack = 1e-12;

__global__ __launch_bounds__(kThreads) void finalize(const DevProb* __restrict__ probs)
{
    const DevProb P = probs[blockIdx.x];
    const int64_t n = P.npiv;  // the decided indices
    const int tid = threadIdx.x;
    const int64_t chunk = (n + kThreads - 1) / kThreads;
    const int64_t lo = tid * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    const bool diag = P.stats != nullptr;
    double s = 0.0, gap = INFINITY, far = 0.0, outside = 0.0;
    int64_t first = INT64_MAX;
    for (int64_t j = lo; j < hi; ++j) {
        const double p = P.piv[j];
        s += log(fabs(p));
        if (first == INT64_MAX && (p == 0.0 || p != p)) first = j;
        if (diag) {
            const double d = P.mask[j] ? p : p + 1.0;
            gap = fmin(gap, fabs(P.u[j] - d));
            const double dist = d < 0.0 ? -d : (d > 1.0 ? d - 1.0 : 0.0);
            far = fmax(far, dist);
            outside += (d < -kRangeSlack || d > 1.0 + kRangeSlack) ? 1.0 : 0.0;
        }
    }
    __shared__ double ss[kThreads], sg[kThreads], sd[kThreads], so[kThreads];
    __shared__ int64_t sf[kThreads];
    ss[tid] = s;
    sf[tid] = first;
    sg[tid] = gap;
    sd[tid] = far;
    so[tid] = outside;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            ss[tid] = ss[tid] + ss[tid + w];
            sf[tid] = sf[tid] < sf[tid + w] ? sf[tid] : sf[tid + w];
            sg[tid] = fmin(sg[tid], sg[tid + w]);
            sd[tid] = fmax(sd[tid], sd[tid + w]);
            so[tid] = so[tid] + so[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        *P.loglik = ss[0];
        *P.info = sf[0] == INT64_MAX ? 0 : (int32_t)(sf[0] + 1);
        if (diag) {
            P.stats[0] = sg[0];
            P.stats[1] = so[0];
            P.stats[2] = sd[0];
        }
    }
}

template <typename T, bool HERM>
__global__ __launch_bounds__(256) void store_diag(const DevProb* __restrict__ probs)
{
    const DevProb P = probs[blockIdx.y];
    const int64_t c0 = (int64_t)blockIdx.x * kLeaf;
    if (c0 >= P.npiv) return;  // blocks past npiv hold the conditional kernel, not factors
    const int bs = (int)((P.n - c0) < kLeaf ? (P.n - c0) : kLeaf);
    const double* blk = P.diag + (int64_t)blockIdx.x * kLeaf * kLeaf;
    T* A = static_cast<T*>(P.A);
    for (int e = threadIdx.x; e < kLeaf * kLeaf; e += 256) {
        const int i = e % kLeaf, k = e / kLeaf;
        if (i < bs && k < bs && (!HERM || k <= i))
            A[(c0 + i) + (c0 + k) * P.lda] = (T)blk[e];
    }
}

// Complex kernels: blocks of kLeafC complex columns (16 bytes per entry).
template <bool HERM>
__global__ __launch_bounds__(256) void store_diag_c(const DevProb* __restrict__ probs)
{
    const DevProb P = probs[blockIdx.y];
    const int64_t c0 = (int64_t)blockIdx.x * kLeafC;
    if (c0 >= P.npiv) return;
    const int bs = (int)((P.n - c0) < kLeafC ? (P.n - c0) : kLeafC);
    const double2* blk = reinterpret_cast<const double2*>(P.diag) + (int64_t)blockIdx.x * kLeafC * kLeafC;
    double2* A = static_cast<double2*>(P.A);
    for (int e = threadIdx.x; e < kLeafC * kLeafC; e += 256) {
        const int i = e % kLeafC, k = e / kLeafC;
        if (i < bs && k < bs && (!HERM || k <= i)) A[(c0 + i) + (c0 + k) * P.lda] = blk[e];
    }
}

struct DescChunk {
    DevProb d[kDescPerLaunch];
    int cnt;
};
static_assert(sizeof(DescChunk) <= 4096, "kernel arguments are limited to 4 KiB");

__global__ void store_descs(DescChunk chunk, DevProb* __restrict__ dst)
{
    const int i = threadIdx.x;
    if (i < chunk.cnt) dst[i] = chunk.d[i];
}

}  // namespace

hipError_t launch_store_descs(const DevProb* host, int cnt, DevProb* dst, hipStream_t s)
{
    DescChunk chunk;
    for (int i = 0; i < cnt; ++i) chunk.d[i] = host[i];
    chunk.cnt = cnt;
    hipLaunchKernelGGL(store_descs, dim3(1), dim3(64), 0, s, chunk, dst);
    return hipGetLastError();
}

hipError_t launch_store_diag(bool herm, int dtype, const DevProb* probs, int nprob, int64_t nmax,
                             hipStream_t s)
{
    if (dtype == 2) {
        dim3 gridc((unsigned)((nmax + kLeafC - 1) / kLeafC), nprob);
        if (herm) hipLaunchKernelGGL((store_diag_c<true>), gridc, dim3(256), 0, s, probs);
        else hipLaunchKernelGGL((store_diag_c<false>), gridc, dim3(256), 0, s, probs);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((nmax + kLeaf - 1) / kLeaf), nprob);
    if (herm) {
        if (dtype == 0) hipLaunchKernelGGL((store_diag<double, true>), grid, dim3(256), 0, s, probs);
        else hipLaunchKernelGGL((store_diag<float, true>), grid, dim3(256), 0, s, probs);
    } else {
        if (dtype == 0) hipLaunchKernelGGL((store_diag<double, false>), grid, dim3(256), 0, s, probs);
        else hipLaunchKernelGGL((store_diag<float, false>), grid, dim3(256), 0, s, probs);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const DevProb* probs, int nprob, hipStream_t s)
{
    hipLaunchKernelGGL(finalize, dim3(nprob), dim3(kThreads), 0, s, probs);
    return hipGetLastError();
}

}  // namespace dpp
