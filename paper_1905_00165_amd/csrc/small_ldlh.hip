// Small Hermitian (real symmetric) problems in one workgroup each: the
// unblocked sampler of Sec. 2 (Theorem 2) run as written, pivot by pivot, on
// the lower triangle held in FP64 registers.
//
// At pivot j, with d the current diagonal entry: keep j iff u_j < d, else
// d' = d - 1 (Prop. 4); then every trailing entry (i, k), i, k > j, loses
// l_i w_k, with w column j and l_i = w_i / d'.
//
// Layout: the lower triangle is cut into 8 x 8 blocks, one per thread, which
// keeps its 64 entries in registers for the whole run (a diagonal block also
// holds the mirror of its lower half, updated alike and never stored).
// Threads enumerate the blocks column by column, so a wavefront mostly shares
// one block column. Per pivot the threads of block column j / 8 publish column
// j (their local column j % 8, a compile-time register index: the pivots of a
// block column are an unrolled loop) in LDS and the owner of the diagonal
// entry decides and publishes d'; after one barrier every thread reads 8 + 8
// column values and updates its block: 64 independent FMAs. Column buffers
// alternate between consecutive pivots, so the next pivot's writes never
// overtake a slow reader of this one (two pivots apart there is a barrier in
// between). Nothing inside the pivot loop touches global memory: a barrier
// waits for the wavefront's outstanding global stores, so the decisions stay
// in LDS until the end. The columns stay unscaled (W = L D) until the end; A
// then receives L = W D^{-1}, D and, past npiv, the conditional kernel (the
// Schur complement), in the storage type, and mask and pivots are written.
// The workgroup has as many threads as the launch's largest problem has
// blocks (rounded up to whole wavefronts), so small sizes leave room for
// more workgroups per CU.
//
// The arithmetic of an entry (its updates in pivot order, each one FMA with
// l_i = w_i * (1 / d')) does not depend on the block layout, so a problem's
// result does not depend on the other problems of its launch. The arithmetic
// is FP64 for every precision (no split products at this size).
#include "dpp_internal.h"

namespace dpp {
namespace {

constexpr int kNB = 8;                                             // block edge
constexpr int kMaxBlocks = (int)(kSmallMax / kNB) * (int)(kSmallMax / kNB + 1) / 2;
constexpr int kThreads = (kMaxBlocks + 63) / 64 * 64;              // 300 blocks -> 320 threads
static_assert(kSmallMax % kNB == 0, "whole blocks");

// Threads of a launch whose largest problem has n = nmax.
int threads_for(int64_t nmax)
{
    const int g = (int)((nmax + kNB - 1) / kNB);
    return (g * (g + 1) / 2 + 63) / 64 * 64;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void small_ldlh(const DevProb* __restrict__ probs)
{
    __shared__ double colb[2][kSmallMax];  // column j, alternating buffers
    __shared__ double dps[kSmallMax];      // d' of every decided pivot
    __shared__ double su[kSmallMax];       // the uniforms
    __shared__ uint8_t skeep[kSmallMax];   // the decisions
    const DevProb P = probs[blockIdx.x];
    const int n = (int)P.n;
    const int npiv = (int)P.npiv;
    const int G = (n + kNB - 1) / kNB;  // block rows of this problem

    // Block (tr, tc), tr >= tc, of thread t: column by column.
    int tr = -1, tc = -1;
    {
        int t = threadIdx.x;
        for (int c = 0; c < G; ++c) {
            if (t < G - c) {
                tc = c;
                tr = c + t;
                break;
            }
            t -= G - c;
        }
    }
    const bool active = tc >= 0;
    const int i0 = tr * kNB, k0 = tc * kNB;

    for (int j = threadIdx.x; j < npiv; j += blockDim.x) su[j] = P.u[j];

    // Load the block (entries past n are zero; above the diagonal, the mirror).
    int64_t ldk;
    const T* __restrict__ K = first_source<T>(P, true, ldk);
    double a[kNB][kNB];
#pragma unroll
    for (int r = 0; r < kNB; ++r)
#pragma unroll
        for (int c = 0; c < kNB; ++c) {
            const int i = i0 + r, k = k0 + c;
            a[r][c] = active && i < n && k < n
                          ? (double)(i >= k ? K[i + (int64_t)k * ldk] : K[k + (int64_t)i * ldk])
                          : 0.0;
        }
    __syncthreads();

    for (int jb = 0; jb < G; ++jb) {
#pragma unroll
        for (int c = 0; c < kNB; ++c) {
            const int j = jb * kNB + c;
            if (j < npiv) {  // uniform over the workgroup
                double* const col = colb[j & 1];
                if (active && tc == jb) {
#pragma unroll
                    for (int r = 0; r < kNB; ++r) col[i0 + r] = a[r][c];
                    if (tr == jb) {
                        const double d = a[c][c];
                        const bool keep = su[j] < d;           // Bernoulli(d) with stream u_j
                        const double dp = keep ? d : d - 1.0;  // Prop. 4 on rejection
                        dps[j] = dp;
                        skeep[j] = keep ? 1 : 0;
                    }
                }
                __syncthreads();
                if (active && i0 + kNB - 1 > j && k0 + kNB - 1 > j) {
                    const double rdp = 1.0 / dps[j];
                    double l[kNB], w[kNB];
#pragma unroll
                    for (int r = 0; r < kNB; ++r) l[r] = col[i0 + r] * rdp;
#pragma unroll
                    for (int q = 0; q < kNB; ++q) w[q] = col[k0 + q];
                    if (i0 > j && k0 > j) {  // every entry of the block is trailing
#pragma unroll
                        for (int r = 0; r < kNB; ++r)
#pragma unroll
                            for (int q = 0; q < kNB; ++q) a[r][q] = __builtin_fma(-l[r], w[q], a[r][q]);
                    } else {  // the block straddles row or column j
#pragma unroll
                        for (int r = 0; r < kNB; ++r)
#pragma unroll
                            for (int q = 0; q < kNB; ++q)
                                if (i0 + r > j && k0 + q > j) a[r][q] = __builtin_fma(-l[r], w[q], a[r][q]);
                    }
                }
            }
        }
    }
    __syncthreads();  // every d' is visible

    for (int j = threadIdx.x; j < npiv; j += blockDim.x) {
        P.mask[j] = skeep[j];
        P.piv[j] = dps[j];
    }
    // A: L = W D^{-1} in the decided columns, D on their diagonal, and the
    // conditional kernel in the trailing block; lower triangle only.
    T* __restrict__ A = static_cast<T*>(P.A);
    if (!active) return;
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
        const int k = k0 + c;
        const double inv = k < npiv ? 1.0 / dps[k < npiv ? k : 0] : 1.0;
#pragma unroll
        for (int r = 0; r < kNB; ++r) {
            const int i = i0 + r;
            if (i < n && k < n && i >= k) {
                const double v = k < npiv ? (i == k ? dps[k] : a[r][c] * inv) : a[r][c];
                A[i + (int64_t)k * P.lda] = (T)v;
            }
        }
    }
}

}  // namespace

hipError_t launch_small_ldlh(int dtype, const DevProb* probs, int nprob, int64_t nmax,
                             hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    if (nmax > kSmallMax || (dtype != 0 && dtype != 1)) return hipErrorInvalidValue;
    const int threads = threads_for(nmax);
    if (dtype == 0) hipLaunchKernelGGL(small_ldlh<double>, dim3(nprob), dim3(threads), 0, s, probs);
    else hipLaunchKernelGGL(small_ldlh<float>, dim3(nprob), dim3(threads), 0, s, probs);
    return hipGetLastError();
}

}  // namespace dpp
