// Diagonal-block kernels of the blocked DPP sampler (gfx950).
//
// One launch handles the 64-wide diagonal block [c0, c0+64) of every problem in
// a batch. Following the blocked sampler of Sec. 3 (the blocked LU listing with
// its diagonal-block factorization replaced by the unblocked sampler), each
// workgroup
//   1. runs the unblocked sampler (Sec. 2, Theorem 2) on the diagonal block:
//      at pivot j, with d the current diagonal entry, keep j iff u_j < d, else
//      d <- d - 1; scale column j by the modified pivot and apply the rank-one
//      Schur update to the rest of the block. This chain runs on wavefront 0
//      with one row of the block per lane, held in registers; the column that
//      drives each rank-one update is broadcast through LDS.
//   2. solves its share of the panel below the block against the factored
//      block (and, for LU, of the row panel to its right), one row (column)
//      per thread with the factored block in LDS.
// Every workgroup of a launch makes the same decisions from the same data
// (the chain is deterministic), so the panel solves need no second launch;
// workgroup 0 alone writes the block, the mask and the pivots.
// All arithmetic is FP64 whatever the storage type T.
#pragma once
#include "dpp_internal.h"

namespace dpp {
namespace leaf {

constexpr int L = kLeaf;
constexpr int kRowsPerWG = 512;  // one panel row per thread; 8 wavefronts

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Round-to-nearest-even FP32 -> BF16 bit pattern (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h)
{
    return __builtin_bit_cast(float, h << 16);
}

// Raw buffer access to a column strip of A: base points at the strip's first
// element, `voff` is a per-lane byte offset and `soff` a per-column byte
// offset held in a scalar register, so a lane's 64 column loads share one
// address register and issue back to back.
constexpr int kBufFlags = 0x00020000;  // raw 32-bit data format, gfx9 resource word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t strip_rsrc(const void* base, int64_t bytes)
{
    const int nrec = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, nrec, kBufFlags);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void buf_store<float>(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)v), r, voff, soff, 0);
}

// hi/lo BF16 split of one value: hi = bf16(x), lo = bf16(x - hi), so that
// hi + lo carries about 16 significant bits of x.
__device__ __forceinline__ void split_bf16(double x, uint16_t& hi, uint16_t& lo)
{
    const uint32_t xh = bf16_bits((float)x);
    hi = (uint16_t)xh;
    lo = (uint16_t)bf16_bits((float)(x - (double)bf16_value(xh)));
}

// Write the hi/lo BF16 split of v[0..63] to two rows (64 bf16 each, 16-byte
// aligned), as 8 stores of 16 bytes per row.
__device__ __forceinline__ void store_split_row(uint16_t* hi_row, uint16_t* lo_row,
                                                const double (&v)[L], int bs)
{
#pragma unroll
    for (int g = 0; g < L / 8; ++g) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            uint32_t hh[2], ll[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int k = g * 8 + e * 2 + t;
                const double x = (k < bs) ? v[k] : 0.0;
                const uint32_t xh = bf16_bits((float)x);
                const double rem = x - (double)bf16_value(xh);
                hh[t] = xh;
                ll[t] = bf16_bits((float)rem);
            }
            h[e] = hh[0] | (hh[1] << 16);
            l[e] = ll[0] | (ll[1] << 16);
        }
        *reinterpret_cast<uint4*>(hi_row + g * 8) = make_uint4(h[0], h[1], h[2], h[3]);
        *reinterpret_cast<uint4*>(lo_row + g * 8) = make_uint4(l[0], l[1], l[2], l[3]);
    }
}

}  // namespace leaf
}  // namespace dpp
