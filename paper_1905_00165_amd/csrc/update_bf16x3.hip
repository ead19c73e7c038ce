// Split-BF16 Schur-complement update of the blocked DPP sampler on gfx950 MFMA.
//
// Same update as update_f64.hip (the outer-product update of the blocked
// factorization, Sec. 3), with each factor x split as hi + lo, hi = bf16(x),
// lo = bf16(x - hi), and the product formed as hi*hi' + hi*lo' + lo*hi' on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (the lo*lo' term, about
// 2^-16 of the product, is dropped). The FP32 sum is subtracted from the
// stored value in FP64 and rounded to the storage type.
//
// The split copies are written by the diagonal-block kernel while it solves the
// panel, in a row-major [row][k] layout (k contiguous), so a 16-byte load
// yields the 8 consecutive k values one lane of the MFMA operand holds:
//   A side (rows of C): hi/lo of L;  B side (cols of C): hi/lo of W = L D
//   (LDL^H) or of U^T (LU).
//
// Tiling: 256 threads own a 128x128 tile of C, each wavefront 64x64 as 2x2
// blocks of 32x32; K advances 32 at a time through LDS.
#include "dpp_internal.h"

namespace dpp {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TM = 128;
constexpr int TN = 128;
constexpr int KC = 32;
constexpr int RS = KC + 8;  // LDS row stride in bf16 (80 bytes)

struct TileCoord {
    int64_t i0, j0;
};

__device__ __forceinline__ bool tile_of(int64_t t, int64_t NR, int64_t NC, bool herm,
                                        TileCoord& tc)
{
    if (!herm) {
        if (t >= NR * NC) return false;
        tc.i0 = (t % NR) * TM;
        tc.j0 = (t / NR) * TN;
        return true;
    }
    int64_t J = 0, before = 0;
    for (; J < NC; ++J) {
        const int64_t here = NR - J;
        if (t < before + here) break;
        before += here;
    }
    if (J >= NC) return false;
    tc.i0 = (J + (t - before)) * TM;
    tc.j0 = J * TN;
    return true;
}

__device__ __forceinline__ bf8 as_bf8(uint4 v)
{
    return __builtin_bit_cast(bf8, v);
}

template <typename T, bool HERM>
__global__ __launch_bounds__(256) void update_bf16x3(const DevProb* __restrict__ probs,
                                                     int64_t base, int64_t ncols_req, int64_t k0,
                                                     int kw, int64_t j0, int ss)
{
    const DevProb P = probs[blockIdx.y];
    const int64_t n = P.n;
    const int64_t nrows = n - base;
    if (nrows <= 0 || k0 + kw > n) return;
    const int64_t ncols = ncols_req < nrows ? ncols_req : nrows;
    const int64_t NR = (nrows + TM - 1) / TM, NC = (ncols + TN - 1) / TN;
    TileCoord tc;
    if (!tile_of(blockIdx.x, NR, NC, HERM, tc)) return;

    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda;
    const uint16_t* __restrict__ Lh = split_plane(P.split, n, ss, 0);
    const uint16_t* __restrict__ Ll = split_plane(P.split, n, ss, 1);
    const uint16_t* __restrict__ Bh = split_plane(P.split, n, ss, 2);
    const uint16_t* __restrict__ Bl = split_plane(P.split, n, ss, 3);

    __shared__ __attribute__((aligned(16))) uint16_t sAh[TM * RS];
    __shared__ __attribute__((aligned(16))) uint16_t sAl[TM * RS];
    __shared__ __attribute__((aligned(16))) uint16_t sBh[TN * RS];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[TN * RS];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    f16v acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[bi][bj][e] = 0.0f;

    const int64_t rowA0 = base + tc.i0;
    const int64_t colB0 = base + tc.j0;
    const int64_t colEnd = base + ncols;
    const int kk0 = (int)(k0 - j0);

    for (int kc = 0; kc < kw; kc += KC) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = (tid >> 2) + 64 * q;
            const int seg = tid & 3;
            const int64_t ga = rowA0 + r;
            const int64_t gb = colB0 + r;
            const int64_t offa = ga * ss + kk0 + kc + seg * 8;
            const int64_t offb = gb * ss + kk0 + kc + seg * 8;
            const uint4 z = make_uint4(0, 0, 0, 0);
            const uint4 vah = ga < n ? *reinterpret_cast<const uint4*>(Lh + offa) : z;
            const uint4 val = ga < n ? *reinterpret_cast<const uint4*>(Ll + offa) : z;
            const uint4 vbh = gb < colEnd ? *reinterpret_cast<const uint4*>(Bh + offb) : z;
            const uint4 vbl = gb < colEnd ? *reinterpret_cast<const uint4*>(Bl + offb) : z;
            *reinterpret_cast<uint4*>(&sAh[r * RS + seg * 8]) = vah;
            *reinterpret_cast<uint4*>(&sAl[r * RS + seg * 8]) = val;
            *reinterpret_cast<uint4*>(&sBh[r * RS + seg * 8]) = vbh;
            *reinterpret_cast<uint4*>(&sBl[r * RS + seg * 8]) = vbl;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC / 16; ++ks) {
            const int kb = ks * 16 + 8 * (lane >> 5);
            bf8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int ra = wm * 64 + b * 32 + (lane & 31);
                const int rb = wn * 64 + b * 32 + (lane & 31);
                ah[b] = as_bf8(*reinterpret_cast<const uint4*>(&sAh[ra * RS + kb]));
                al[b] = as_bf8(*reinterpret_cast<const uint4*>(&sAl[ra * RS + kb]));
                bh[b] = as_bf8(*reinterpret_cast<const uint4*>(&sBh[rb * RS + kb]));
                bl[b] = as_bf8(*reinterpret_cast<const uint4*>(&sBl[rb * RS + kb]));
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);
                }
        }
        __syncthreads();
    }

    // D block layout of the 32x32 MFMA: element e of lane l is row
    // 8*(e/4) + 4*(l/32) + e%4, column l%32.
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int64_t gc = colB0 + wn * 64 + bj * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t gr =
                    rowA0 + wm * 64 + bi * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const bool ok = gr < n && gc < colEnd && (!HERM || gr >= gc);
                if (ok) {
                    T* p = &A[gr + gc * lda];
                    *p = (T)((double)*p - (double)acc[bi][bj][e]);
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_update_bf16x3(bool herm, int dtype, const DevProb* probs, int nprob,
                                int64_t nmax, int64_t base, int64_t ncols, int64_t k0, int kw,
                                int64_t j0, int ss, hipStream_t s)
{
    const int64_t nrows = nmax - base;
    if (nrows <= 0) return hipSuccess;
    const int64_t nc = ncols < nrows ? ncols : nrows;
    const int64_t NR = (nrows + TM - 1) / TM, NC = (nc + TN - 1) / TN;
    const int64_t tiles = herm ? NC * NR - NC * (NC - 1) / 2 : NR * NC;
    dim3 grid((unsigned)tiles, nprob), block(256);
    if (herm) {
        if (dtype == 0) hipLaunchKernelGGL((update_bf16x3<double, true>), grid, block, 0, s, probs, base, ncols, k0, kw, j0, ss);
        else hipLaunchKernelGGL((update_bf16x3<float, true>), grid, block, 0, s, probs, base, ncols, k0, kw, j0, ss);
    } else {
        if (dtype == 0) hipLaunchKernelGGL((update_bf16x3<double, false>), grid, block, 0, s, probs, base, ncols, k0, kw, j0, ss);
        else hipLaunchKernelGGL((update_bf16x3<float, false>), grid, block, 0, s, probs, base, ncols, k0, kw, j0, ss);
    }
    return hipGetLastError();
}

}  // namespace dpp
