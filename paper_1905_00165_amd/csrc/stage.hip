// Staging of a working copy for the in-place LDL^H sampler: the sampler
// reads and overwrites only the lower triangle of A (Sec. 3, the Hermitian
// specialization), so restoring a working copy from K needs only that
// triangle: half the bytes of a full copy.
#include "dpp_internal.h"

namespace dpp {
namespace {

constexpr int kTile = 64;

// One 64x64 tile of the lower triangle per workgroup (tiles (I, J), J <= I,
// numbered column by column); thread t copies row t % 64 of the tile for 16 of
// its columns, so each column's 64 rows move as one coalesced 512-byte run
// (FP64).
template <typename T>
__global__ __launch_bounds__(256) void copy_lower(T* __restrict__ dst, const T* __restrict__ src,
                                                  int64_t n, int64_t ldd, int64_t lds)
{
    const int64_t NT = (n + kTile - 1) / kTile;
    int64_t t = blockIdx.x, J = 0;
    while (J < NT && t >= NT - J) {  // tiles in tile column J: NT - J
        t -= NT - J;
        ++J;
    }
    if (J >= NT) return;
    const int64_t I = J + t;
    const int64_t r = I * kTile + (threadIdx.x & (kTile - 1));
    if (r >= n) return;
    const int64_t cbase = J * kTile + (threadIdx.x >> 6) * 16;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t c = cbase + k;
        if (c < n && c <= r) dst[r + c * ldd] = src[r + c * lds];
    }
}

}  // namespace

hipError_t launch_copy_lower(int dtype, void* dst, const void* src, int64_t n, int64_t ldd,
                             int64_t lds, hipStream_t s)
{
    const int64_t NT = (n + kTile - 1) / kTile;
    const int64_t tiles = NT * (NT + 1) / 2;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    if (dtype == 0)
        hipLaunchKernelGGL(copy_lower<double>, dim3((unsigned)tiles), dim3(256), 0, s,
                           static_cast<double*>(dst), static_cast<const double*>(src), n, ldd, lds);
    else
        hipLaunchKernelGGL(copy_lower<float>, dim3((unsigned)tiles), dim3(256), 0, s,
                           static_cast<float*>(dst), static_cast<const float*>(src), n, ldd, lds);
    return hipGetLastError();
}

}  // namespace dpp
