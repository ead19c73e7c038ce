// Split-BF16 Schur-complement update of the blocked DPP sampler on gfx950 MFMA.
//
// Same update as update_f64.hip (the outer-product update of the blocked
// factorization, Sec. 3), with each factor x split as hi + lo, hi = bf16(x),
// lo = bf16(x - hi), and the product formed as hi*hi' + hi*lo' + lo*hi' on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (the lo*lo' term, about
// 2^-16 of the product, is dropped). The FP32 sum is subtracted from the
// stored value in FP64 and rounded to the storage type.
//
// Operands come from the split copies the diagonal-block kernel writes while it
// solves the panel, row-major [row][k] (k contiguous), so 16 bytes are the 8
// consecutive k one MFMA lane holds:
//   rows of C: hi/lo of L;  cols of C: hi/lo of W = L D (LDL^H) or of U^T (LU).
//
// Tiling: 256 threads (4 wavefronts) own a 256x256 tile of C; wavefront
// (wr, wc) owns 128x128 as 4x4 blocks of 32x32, so each 16-k step reads 16
// fragments from LDS and issues 48 MFMAs. K advances 32 at a time through two
// LDS buffers of 64 KiB (one 16 KiB plane per operand). Global -> LDS copies
// use the gfx950 direct-to-LDS loads (global_load_lds_dwordx4): wavefront w
// fills plane w, each instruction writing 1 KiB (16 rows x 64 bytes); stage
// s+1 is in flight while stage s is multiplied, one barrier per stage. LDS rows
// are 64 bytes with their four 16-byte segments XOR-swizzled by row, so the
// fragment reads of consecutive rows spread over the banks.
// The MFMA takes the column operand first, so each lane's accumulators map to
// one row of C and lanes 0-31 cover 32 consecutive rows of a column: the
// read-modify-write of column-major C is coalesced. Operand rows past the end
// of the region are read from the last valid row instead: they only feed
// accumulators that are never stored.
// Workgroup b runs tile (b % 8) * (G / 8) + b / 8 (G the grid size, a multiple
// of 8): the 8 XCDs each take a contiguous range of tiles, which share operand
// panels in that XCD's L2.
#include "dpp_internal.h"

namespace dpp {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TM = 256;                       // tile rows (== tile cols)
constexpr int KC = 32;                        // k per LDS stage
constexpr int kThreads = 256;
constexpr int kRowBytes = KC * 2;             // 64
constexpr int kPlaneBytes = TM * kRowBytes;   // 16 KiB
constexpr int kBufBytes = 4 * kPlaneBytes;    // Lh, Ll, Wh, Wl
constexpr int kLdsBytes = 2 * kBufBytes;      // double buffered

struct TileCoord {
    int64_t i0, j0;
};

__device__ __forceinline__ bool tile_of(int64_t t, int64_t NR, int64_t NC, bool herm,
                                        TileCoord& tc)
{
    if (!herm) {
        if (t >= NR * NC) return false;
        tc.i0 = (t % NR) * TM;
        tc.j0 = (t / NR) * TM;
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
    tc.j0 = J * TM;
    return true;
}

__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }

// Byte offset of logical 16-byte segment `seg` of row `r` inside a plane.
__device__ __forceinline__ int lds_off(int r, int seg)
{
    return r * kRowBytes + ((seg ^ swz(r)) << 4);
}

typedef const void __attribute__((address_space(1)))* gptr_t;
typedef void __attribute__((address_space(3)))* lptr_t;

template <typename T, bool HERM>
__global__ __launch_bounds__(kThreads, 1) void update_bf16x3(const DevProb* __restrict__ probs,
                                                             int64_t base, int64_t ncols_req,
                                                             int64_t k0, int kw, int64_t j0,
                                                             int ss)
{
    const DevProb P = probs[blockIdx.y];
    const int64_t n = P.n;
    const int64_t nrows = n - base;
    if (nrows <= 0 || k0 + kw > n) return;
    const int64_t ncols = ncols_req < nrows ? ncols_req : nrows;
    const int64_t NR = (nrows + TM - 1) / TM, NC = (ncols + TM - 1) / TM;
    const int64_t per_xcd = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    TileCoord tc;
    if (!tile_of(t, NR, NC, HERM, tc)) return;

    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda;

    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    const int64_t rowT0 = base + tc.i0;
    const int64_t colT0 = base + tc.j0;
    const int64_t colEnd = base + ncols;
    const int kk0 = (int)(k0 - j0);

    // Direct-to-LDS copies: wavefront `wave` fills plane `wave`. Instruction q
    // (0..15) writes rows 16q .. 16q+15 of the plane; lane l supplies row
    // 16q + l/4, physical segment l%4, i.e. logical segment (l%4) ^ swz(row);
    // swz(16q + l/4) does not depend on q.
    const int plane = wave;
    const uint16_t* src_plane = split_plane(P.split, n, ss, plane);
    const int64_t first = plane < 2 ? rowT0 : colT0;
    const int64_t last = (plane < 2 ? n : colEnd) - 1;  // rows past it: reuse it
    const int rl = lane >> 2;
    const int seg8 = ((lane & 3) ^ swz(rl)) * 8;
    auto issue_stage = [&](int kc, int buf) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            int64_t g = first + 16 * q + rl;
            g = g < last ? g : last;
            __builtin_amdgcn_global_load_lds(
                (gptr_t)(src_plane + g * ss + kk0 + kc + seg8),
                (lptr_t)(lds + buf * kBufBytes + plane * kPlaneBytes + q * 1024), 16, 0, 0);
        }
    };

    f16v acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[rb][cb][e] = 0.0f;

    const int nstages = kw / KC;
    issue_stage(0, 0);
    for (int s = 0; s < nstages; ++s) {
        const int buf = s & 1;
        // This wavefront's copies of stage s are in LDS; the barrier makes
        // everyone's visible and retires every read of the other buffer.
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        if (s + 1 < nstages) issue_stage((s + 1) * KC, buf ^ 1);
        const unsigned char* B0 = lds + buf * kBufBytes;
        bf8 lh[2][4], ll[2][4], wh[2][4], wl[2][4];
        auto read_frags = [&](int ks) {
            const int seg = ks * 2 + (lane >> 5);  // 8 k values per lane
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int ra = wr * 128 + b * 32 + (lane & 31);
                const int rc = wc * 128 + b * 32 + (lane & 31);
                lh[ks][b] = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4*>(B0 + 0 * kPlaneBytes + lds_off(ra, seg)));
                ll[ks][b] = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4*>(B0 + 1 * kPlaneBytes + lds_off(ra, seg)));
                wh[ks][b] = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4*>(B0 + 2 * kPlaneBytes + lds_off(rc, seg)));
                wl[ks][b] = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4*>(B0 + 3 * kPlaneBytes + lds_off(rc, seg)));
            }
        };
        auto mfmas = [&](int ks) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[ks][cb], lh[ks][rb], acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl[ks][cb], lh[ks][rb], acc[rb][cb], 0, 0, 0);
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[ks][cb], ll[ks][rb], acc[rb][cb], 0, 0, 0);
                }
        };
        read_frags(0);
        read_frags(1);
        mfmas(0);
        mfmas(1);
        // Schedule: k-step 0's 16 fragment reads, then its 48 MFMAs with
        // k-step 1's 16 reads interleaved one per 3 MFMAs, then k-step 1's MFMAs.
        __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);   // DS read
        for (int i = 0; i < 16; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 48, 0);
    }

    // Accumulator layout of the 32x32 MFMA with the column operand first:
    // element e of lane l is C row (l % 32), C column 8*(e/4) + 4*(l/32) + e%4
    // of the 32x32 block. For each pair of blocks all 32 C values of a lane are
    // loaded before any is stored: the stores could alias later loads, so
    // interleaving them would serialize one memory round trip per element.
    // Tile-relative indices: row i, column j of the tile; stored iff
    // i < rlim, j < clim and (lower part) i - j >= dd.
    const int rlim = (int)(n - rowT0);
    const int clim = (int)(colEnd - colT0);
    const int dd = (int)(colT0 - rowT0);
    const int jl = wc * 128 + 4 * (lane >> 5);  // lane part of the column
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int i = wr * 128 + rb * 32 + (lane & 31);
        T* const p0 = A + (rowT0 + i) + (colT0 + jl) * lda;
#pragma unroll
        for (int c2 = 0; c2 < 4; c2 += 2) {
            double cv[2][16];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int ju = (c2 + h) * 32 + 8 * (e >> 2) + (e & 3);  // uniform part
                    const int j = jl + ju;
                    const bool ok = i < rlim && j < clim && (!HERM || i - j >= dd);
                    cv[h][e] = ok ? (double)p0[ju * lda] : 0.0;
                }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int ju = (c2 + h) * 32 + 8 * (e >> 2) + (e & 3);
                    const int j = jl + ju;
                    const bool ok = i < rlim && j < clim && (!HERM || i - j >= dd);
                    if (ok) p0[ju * lda] = (T)(cv[h][e] - (double)acc[rb][c2 + h][e]);
                }
        }
    }
}

template <typename T, bool HERM>
hipError_t launch_t(const DevProb* probs, int nprob, unsigned grid_x, int64_t base, int64_t ncols,
                    int64_t k0, int kw, int64_t j0, int ss, hipStream_t s)
{
    auto k = update_bf16x3<T, HERM>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k, dim3(grid_x, nprob), dim3(kThreads), kLdsBytes, s, probs, base, ncols,
                       k0, kw, j0, ss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_update_bf16x3(bool herm, int dtype, const DevProb* probs, int nprob,
                                int64_t nmax, int64_t base, int64_t ncols, int64_t k0, int kw,
                                int64_t j0, int ss, hipStream_t s)
{
    const int64_t nrows = nmax - base;
    if (nrows <= 0) return hipSuccess;
    if (kw % KC != 0) return hipErrorInvalidValue;
    const int64_t nc = ncols < nrows ? ncols : nrows;
    const int64_t NR = (nrows + TM - 1) / TM, NC = (nc + TM - 1) / TM;
    const int64_t tiles = herm ? NC * NR - NC * (NC - 1) / 2 : NR * NC;
    const unsigned grid_x = (unsigned)((tiles + 7) / 8 * 8);  // XCD remap needs a multiple of 8
    if (herm) {
        if (dtype == 0) return launch_t<double, true>(probs, nprob, grid_x, base, ncols, k0, kw, j0, ss, s);
        return launch_t<float, true>(probs, nprob, grid_x, base, ncols, k0, kw, j0, ss, s);
    }
    if (dtype == 0) return launch_t<double, false>(probs, nprob, grid_x, base, ncols, k0, kw, j0, ss, s);
    return launch_t<float, false>(probs, nprob, grid_x, base, ncols, k0, kw, j0, ss, s);
}

}  // namespace dpp
