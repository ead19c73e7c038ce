// Split-BF16 Schur-complement update of the blocked DPP sampler on gfx950 MFMA.
//
// Same update as update_f64.hip (the outer-product update of the blocked
// factorization, Sec. 3), with each factor value x cut into NP BF16 pieces
// p_0 = bf16(x), p_i = bf16(x - p_0 - ... - p_{i-1}) (dpp_internal.h), and
// the product formed from the pairs of pieces whose orders sum to at most
// NP - 1 on v_mfma_f32_32x32x16_bf16 with FP32 accumulation:
//   NP = 2 (update_bf16x3): hi*hi' + hi*lo' + lo*hi'; the dropped lo*lo' and
//     the pieces' rounding leave about 2^-16 of each product;
//   NP = 3 (update_bf16x6): p0*p0' + p0*p1' + p1*p0' + p0*p2' + p2*p0' +
//     p1*p1'; about 2^-24 of each product is left. One FP32 sum over a long
//     k range would then dominate the error (each addition rounds to 2^-24
//     of a partial sum that can be much larger than the result), so the sum
//     is two-level: the MFMAs accumulate 64 k at a time (Shape::FL) from
//     zero, and each such chunk sum is added into a second FP32 total, so no
//     FP32 sum runs over more than max(64, kw / 64) terms. Both sets fit two
//     wavefronts per SIMD (64 x 64 per wavefront).
//   FP16 form (update_fp16x3, real LDL^H): hi*hi' + hi*lo' + lo*hi' on
//     v_mfma_f32_32x32x16_f16 over the FP16 pieces of balanced, row-scaled
//     values (dpp_internal.h). FP16's 11 bits make the pieces carry 22 bits
//     of each value, but only relative to its row's 64-column block: so the
//     MFMAs run 64 k at a time, and each chunk sum is multiplied by its row's
//     and its column's factors (powers of two: exact) and added into FP32
//     totals. The factors of a chunk are loaded into registers at its first
//     stage, before that stage's copies, so the stage waits below also cover
//     them one stage later.
// The sum is subtracted from the stored value in FP64 and rounded to the
// storage type.
//
// Operands come from the split copies the diagonal-block kernel writes while it
// solves the panel, tiled so that the rows one stage copies are contiguous
// (plane_off in dpp_internal.h); 16 bytes are the 8 consecutive k one MFMA
// lane holds:
//   rows of C: pieces of L;  cols of C: pieces of W = L D (LDL^H) or of U^T (LU).
//
// Tiling (template Shape): a workgroup owns a TM x TN tile of C split over
// WR x WC wavefronts, each owning RB x CB blocks of 32x32 (wide shape:
// 256x256 on 8 wavefronts of 128x64, so each 16-k step reads NP * 6
// fragments from LDS and issues 8 MFMAs per product term per wavefront;
// narrower shapes serve the narrow updates inside a panel). K advances KC (16
// or 32) at a time through NST LDS stages holding the 2 NP operand planes,
// NST - 1 of them in flight while one is multiplied, one barrier per stage.
// Global -> LDS copies use the gfx950 direct-to-LDS loads
// (global_load_lds_dwordx4), each instruction writing 1 KiB. LDS rows are
// KC * 2 bytes with their 16-byte segments XOR-swizzled by row (swz below).
// The MFMA takes the column operand first, so each lane's accumulators map to
// one row of C and lanes 0-31 cover 32 consecutive rows of a column: the
// read-modify-write of column-major C is coalesced. Operand rows past the end
// of the region are read from the last valid row instead: they only feed
// accumulators that are never stored.
// One launch covers the problems of several size groups (GroupMap): workgroup
// b takes slot (b % 8) * (G / 8) + b / 8 of the launch (G the grid size, a
// multiple of 8), so the 8 XCDs each take a contiguous range of tiles, and the
// slot names a problem and one of its tiles. In the wide shape
// tiles are ordered by groups of 4 tile columns, row by row within a group, so
// the ~32 tiles an XCD runs at once form an 8x4 block that shares 8 row panels
// and 4 column panels in that XCD's L2.
#include <atomic>
#include <type_traits>

#include "dpp_internal.h"

namespace dpp {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef const void __attribute__((address_space(1)))* gptr_t;
typedef void __attribute__((address_space(3)))* lptr_t;

constexpr int kKAlign = 32;        // every update's k range is a multiple of this
constexpr int kGroupCols = 4;      // tile columns per group of the wide order

// TM x TN tile on WR x WC wavefronts; K advances KC at a time through NST LDS
// stages (NST - 1 of them in flight while one is multiplied); NP BF16 pieces
// per operand value. FL > 0: the FP32 accumulators are added into FP32
// totals (and restart from zero) every FL stages, so no MFMA chain runs over
// more than FL * KC values of k. F16: the FP16 form (NP = 2, FL * KC = 64,
// one chunk per 64-column block of the row factors).
template <int TM_, int TN_, int WR_, int WC_, int MINB_, int EP_, int KC_, int NST_, int NP_,
          int FL_ = 0, bool F16_ = false>
struct Shape {
    static constexpr int TM = TM_, TN = TN_, WR = WR_, WC = WC_;
    static constexpr int MINB = MINB_;  // workgroups per CU the register budget allows
    static constexpr int EP = EP_;      // 32x32 blocks per epilogue round
    static constexpr int KC = KC_, NST = NST_;
    static constexpr int NP = NP_;                                 // pieces per value
    static constexpr int FL = FL_;                                 // stages per chunk (0: one chain)
    static constexpr bool F16 = F16_;
    static constexpr int NTERM = NP == 2 ? 3 : 6;                  // product terms
    static constexpr int ROWB = KC * 2;                            // bytes per operand row and stage
    static constexpr int KSTEPS = KC / 16;                         // MFMA k steps per stage
    static constexpr int NW = WR * WC, THREADS = 64 * NW;
    static constexpr int RB = TM / (32 * WR), CB = TN / (32 * WC);  // 32x32 blocks per wave
    static constexpr int A_PLANE = TM * ROWB, W_PLANE = TN * ROWB;
    static constexpr int BUF = NP * (A_PLANE + W_PLANE);           // pieces of L, then of W
    static constexpr int LDS = NST * BUF;
    static constexpr int COPIES = BUF / 1024;                       // 1 KiB copies per stage
    static constexpr int PER_WAVE = (COPIES + NW - 1) / NW;         // per wavefront
    static constexpr int LPR = ROWB / 16;                           // lanes per row in a copy
    static constexpr int READS = NP * (RB + CB);                    // fragments per k step
    static constexpr int MFMAS = NTERM * RB * CB;
    static_assert(NP == 2 || NP == 3, "two or three pieces");
    static_assert(KC == 16 || KC == 32, "rows of 32 or 64 bytes");
    static_assert(kKAlign % KC == 0, "stages must tile every k range");
    static_assert(BUF % 1024 == 0, "whole 1 KiB copies");
    static_assert(A_PLANE % 1024 == 0 && W_PLANE % 1024 == 0, "no copy straddles two planes");
    static_assert(LDS <= 160 * 1024 / MINB, "LDS of MINB workgroups per CU");
    static_assert(NST >= 2 && NST <= 4, "vmcnt bookkeeping covers 2..4 stages");
    static_assert(!F16 || (NP == 2 && FL * KC == 64), "FP16 form: chunks are the 64-column blocks");
};
// (L piece, W piece) of product term t: the pairs whose orders sum to at most
// NP - 1, larger terms first.
__device__ __forceinline__ constexpr int term_a(int t) { return t == 2 ? 1 : t == 4 ? 2 : t == 5 ? 1 : 0; }
__device__ __forceinline__ constexpr int term_b(int t) { return t == 1 ? 1 : t == 3 ? 2 : t == 5 ? 1 : 0; }

using Wide3 = Shape<256, 256, 2, 4, 1, 1, 16, 4, 2>;
using Medium3 = Shape<256, 128, 2, 2, 2, 1, 16, 3, 2>;
using Narrow3 = Shape<128, 64, 4, 1, 3, 1, 32, 2, 2>;
// Six products: MFMA chains of 64 k, summed into FP32 totals (64 x 64 per
// wavefront, so both sets fit two workgroups per CU; three LDS stages).
using Wide6 = Shape<128, 128, 2, 2, 2, 1, 16, 3, 3, 4>;
using Medium6 = Wide6;
using Narrow6 = Shape<128, 64, 4, 1, 2, 1, 32, 2, 3, 2>;
// FP16 form: chunks of 64 k scaled into FP32 totals, as the six products.
using Wide16 = Shape<128, 128, 2, 2, 2, 1, 16, 4, 2, 4, true>;
using Narrow16 = Shape<128, 64, 4, 1, 2, 1, 32, 2, 2, 2, true>;

// MFMAs spread evenly over the READS fragment reads that follow the first
// group: slot r gets floor((r+1) M / R) - floor(r M / R) MFMAs, then one read.
template <int M, int R, int r = 0>
__device__ __forceinline__ void interleave_mfma_reads()
{
    if constexpr (r < R) {
        constexpr int cnt = (r + 1) * M / R - r * M / R;
        if constexpr (cnt > 0) __builtin_amdgcn_sched_group_barrier(0x008, cnt, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                           // DS read
        interleave_mfma_reads<M, R, r + 1>();
    }
}

// XOR swizzle of the 16-byte segments of LDS row r. A fragment read (lane l:
// row l % 32, one segment) is served 16 lanes at a time, 256 bytes over the
// 64 banks, so the 16 consecutive rows of a group must land on 16 distinct
// 16-byte bank quads. With 64-byte rows (four segments, four rows per 256
// bytes) rows r, r+4, r+8, r+12 need four different segment flips: bits 2-3
// of the row. With 32-byte rows (two segments, eight rows per 256 bytes) rows
// r and r+8 need different flips: bit 2 xor bit 3. (A flip that spreads only
// 8 rows leaves half of the LDS cycles as bank conflicts.) The flip uses row
// bits below 4 only, so it is the same for a row of a plane and for that row
// inside the 16- or 32-row block one direct-to-LDS copy writes.
template <int ROWB>
__device__ __forceinline__ int swz(int r)
{
    return ROWB == 64 ? (r >> 2) & 3 : ((r >> 2) ^ (r >> 3)) & 1;
}

// s_waitcnt immediate that waits until at most N vector-memory loads of this
// wavefront are outstanding (expcnt and lgkmcnt left at their maxima, i.e.
// not waited on). gfx9 layout: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8.
template <int N>
constexpr int vmcnt_imm()
{
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit counter");
    return (N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8);
}
static_assert(vmcnt_imm<0>() == 0x0F70 && vmcnt_imm<6>() == 0x0F76 && vmcnt_imm<24>() == 0x4F78,
              "s_waitcnt encoding");

constexpr int kBufFlags = 0x00020000;  // raw 32-bit data format, gfx9 resource word 3
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ double buf_load_c(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load_c<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load_c<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store_c(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ void buf_store_c<double>(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void buf_store_c<float>(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)v), r, voff, soff, 0);
}

// Byte offset of logical 16-byte segment `seg` of row `r` inside a plane.
template <int ROWB>
__device__ __forceinline__ int lds_off(int r, int seg)
{
    return r * ROWB + ((seg ^ swz<ROWB>(r)) << 4);
}

struct TileCoord {
    int64_t i0, j0;  // tile indices (row tile, column tile)
};

// Grouped order over the tiles of the region (NR x NC tiles of equal size;
// Hermitian: only J <= I). Groups of kGroupCols tile columns, row by row.
__device__ __forceinline__ bool grouped_tile(int64_t t, int64_t NR, int64_t NC, bool herm,
                                             TileCoord& tc)
{
    for (int64_t J0 = 0; J0 < NC; J0 += kGroupCols) {
        const int64_t gw = NC - J0 < kGroupCols ? NC - J0 : kGroupCols;
        const int64_t tri = herm ? gw * (gw - 1) / 2 : 0;
        const int64_t rows = herm ? NR - (J0 + gw - 1) : NR;  // rows with all gw columns
        const int64_t count = tri + (rows > 0 ? rows : 0) * gw;
        if (t >= count) {
            t -= count;
            continue;
        }
        if (t < tri) {  // rows J0 .. J0+gw-2 hold 1 .. gw-1 tiles
            int64_t i = 0;
            while ((i + 1) * (i + 2) / 2 <= t) ++i;
            tc.i0 = J0 + i;
            tc.j0 = J0 + (t - i * (i + 1) / 2);
        } else {
            const int64_t p = t - tri;
            tc.i0 = (herm ? J0 + gw - 1 : 0) + p / gw;
            tc.j0 = J0 + p % gw;
        }
        return true;
    }
    return false;
}

// CPLX: complex kernels (T = double, the parts of complex entries). Region,
// k0, kw and j0 count complex rows and columns; the tile runs over the real
// rows of C' (two per complex row) and the real k of the planes (two per
// complex column), dpp_internal.h.
template <typename T, bool HERM, class S, bool CPLX>
__device__ __forceinline__ void update_body(const DevProb* __restrict__ probs, const GroupMap& M,
                                            Region rg, int64_t k0, int kw, int64_t j0, int ss,
                                            unsigned char* lds)
{
    constexpr int RS = CPLX ? 2 : 1;  // real rows (and real k) per complex one
    // XCD-contiguous order over the launch (grid size a multiple of 8), then
    // the problem and its tile.
    int pi, tw, unused;
    if (!group_slot(M, xcd_order(blockIdx.x, gridDim.x), pi, tw, unused)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    const int64_t rEndC = rg.r0 + rg.rlen < n ? rg.r0 + rg.rlen : n;
    const int64_t cEnd = rg.c0 + rg.clen < n ? rg.c0 + rg.clen : n;
    const int64_t nrows = rEndC - rg.r0, ncols = cEnd - rg.c0;
    if (nrows <= 0 || ncols <= 0 || k0 + kw > n || k0 >= P.npiv) return;
    // Only decided columns contribute: k in [k0, min(k0 + kw, npiv)).
    const int kwp = RS * (k0 + kw <= P.npiv ? kw : (int)(P.npiv - k0));
    const int64_t NR = (nrows * RS + S::TM - 1) / S::TM, NC = (ncols + S::TN - 1) / S::TN;
    const int64_t t = tw;
    TileCoord tc;
    if constexpr (S::TM == S::TN) {
        if (!grouped_tile(t, NR, NC, HERM && !CPLX, tc)) return;
    } else {
        if (t >= NR * NC) return;
        tc.i0 = t % NR;
        tc.j0 = t / NR;
        if (HERM && !CPLX && (tc.i0 + 1) * S::TM <= tc.j0 * S::TN) return;
    }
    // Hermitian: skip tiles entirely above the diagonal (complex: by the
    // complex row of the tile's last real row).
    if (CPLX && HERM && (tc.i0 * S::TM + S::TM - 1) / RS < tc.j0 * S::TN) return;

    // C as a real column-major matrix with RS real rows per row of the region.
    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda * RS;
    int64_t lds_;  // leading dimension of the source C is read from (K when k0 == 0)
    const T* __restrict__ Csrc = first_source<T>(P, k0 == 0, lds_);
    lds_ *= RS;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar arithmetic
    const int wr = wave / S::WC, wc = wave % S::WC;

    const int64_t rowT0 = rg.r0 * RS + tc.i0 * S::TM;  // real rows of C'
    const int64_t colT0 = rg.c0 + tc.j0 * S::TN;
    const int64_t colEnd = cEnd;
    const int64_t rEnd = rEndC * RS;
    const int kk0 = (int)(RS * (k0 - j0));

    // Direct-to-LDS copies. Copy i of a stage writes bytes [1024 i, 1024 i + 1024)
    // of the buffer (the pieces of L, then of W, back to back): 1024 / ROWB rows of
    // one plane. Lane l supplies row l / LPR of that block, physical segment
    // l % LPR, i.e. logical segment (l % LPR) ^ swz(row); the block starts at a
    // multiple of 16 rows, so swz depends on l only. A lane's source for a
    // stage at k offset kc is its pointer at kc = 0 plus kc * 32 elements:
    // plane_off is linear in k across steps of 16 (512 elements per step, the
    // rows' 32-k blocks being consecutive), so the pointers are formed once.
    const int rl = lane / S::LPR;
    const int seg8 = ((lane % S::LPR) ^ swz<S::ROWB>(rl)) * 8;
    const uint16_t* src[S::PER_WAVE];
    int dst_off[S::PER_WAVE];  // byte offset of each copy in a stage buffer
#pragma unroll
    for (int q = 0; q < S::PER_WAVE; ++q) {
        // Copy index, uniform. When the wavefronts do not divide the copies
        // evenly, the last one repeats the last copy (the same bytes to the
        // same place), so every wavefront issues PER_WAVE and stays
        // branch-free.
        int i = wave * S::PER_WAVE + q;
        i = i < S::COPIES ? i : S::COPIES - 1;
        const int off = i * 1024;
        int plane, row0;
        if (off < S::NP * S::A_PLANE) {
            plane = off / S::A_PLANE;
            row0 = (off % S::A_PLANE) / S::ROWB;
        } else {
            const int o2 = off - S::NP * S::A_PLANE;
            plane = S::NP + o2 / S::W_PLANE;
            row0 = (o2 % S::W_PLANE) / S::ROWB;
        }
        const int64_t first = plane < S::NP ? rowT0 : colT0;
        const int64_t last = (plane < S::NP ? rEnd : colEnd) - 1;  // rows past it: reuse it
        int64_t g = first + row0 + rl;
        g = g < last ? g : last;
        src[q] = split_plane(P.split, RS * n, n, ss, S::NP, plane) + plane_off(g, kk0 + seg8, ss);
        dst_off[q] = off;
    }
    const int nstages = kwp / S::KC;
    // Every stage issues its copies, also past the last one (they then reread
    // the last stage into the buffer freed next), so that the copies are
    // branch-free and can be interleaved with the matrix products, and the
    // wait below has one form. They are drained before the epilogue.
    auto issue_stage = [&](int st) {
        const int64_t kc = (int64_t)(st < nstages ? st : nstages - 1) * S::KC;
        unsigned char* const dst = lds + (st % S::NST) * S::BUF;
#pragma unroll
        for (int q = 0; q < S::PER_WAVE; ++q)
            __builtin_amdgcn_global_load_lds((gptr_t)(src[q] + kc * 32), (lptr_t)(dst + dst_off[q]), 16, 0,
                                             0);
    };

    f16v acc[S::RB][S::CB];
#pragma unroll
    for (int rb = 0; rb < S::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < S::CB; ++cb)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[rb][cb][e] = 0.0f;
    constexpr bool TWO_LEVEL = S::FL > 0;  // two-level sums (chunks, then FP32 totals)
    float acct[TWO_LEVEL ? S::RB : 1][TWO_LEVEL ? S::CB : 1][16];
    if constexpr (TWO_LEVEL) {
#pragma unroll
        for (int rb = 0; rb < S::RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < S::CB; ++cb)
#pragma unroll
                for (int e = 0; e < 16; ++e) acct[rb][cb][e] = 0.0f;
    }
    // FP16 form: the factors of the current chunk for this lane's rows (one
    // per row block) and columns (16 per column block, in four runs of 4
    // consecutive columns: the accumulator layout below). Rows and column
    // runs past the region read the last valid ones; they only scale
    // accumulators that are never stored.
    constexpr int NSCALE = S::F16 ? S::RB + 4 * S::CB : 0;  // loads per chunk
    float rsv[S::F16 ? S::RB : 1];
    f4v csv[S::F16 ? S::CB : 1][4];
    // Loads through the global address space: a generic (flat) load would
    // also count against the LDS wait counter, so the fragment waits of the
    // chunk's first stage would wait for these loads as well.
    typedef const __attribute__((address_space(1))) float* gfloat_t;
    typedef const __attribute__((address_space(1))) f4v* gf4v_t;
    auto load_scales = [&](int st) {
        if constexpr (S::F16) {
            const int c = (kk0 + st * S::KC) / 64;  // the chunk's 64-column block
#pragma unroll
            for (int rb = 0; rb < S::RB; ++rb) {
                int64_t g = rowT0 + wr * (S::TM / S::WR) + rb * 32 + (lane & 31);
                g = g < rEnd - 1 ? g : rEnd - 1;
                rsv[rb] = *(gfloat_t)(P.scale + scale_off(n, ss, 0, c, g));
            }
            const int64_t last4 = (colEnd - 1) & ~(int64_t)3;
#pragma unroll
            for (int cb = 0; cb < S::CB; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int64_t g = colT0 + wc * (S::TN / S::WC) + cb * 32 + 8 * q + 4 * (lane >> 5);
                    g = g < last4 ? g : last4;
                    csv[cb][q] = *(gf4v_t)(P.scale + scale_off(n, ss, 1, c, g));
                }
        }
    };

    // The value of the update at accumulator element e of block (rb, cb).
    auto acc_value = [&](int rb, int cb, int e) -> double {
        if constexpr (TWO_LEVEL) return (double)acct[rb][cb][e];
        return (double)acc[rb][cb][e];
    };

    // Epilogue geometry (see the accumulator layout below): tile-relative row
    // i, column j; stored iff i < rlim, j < clim and (lower part) i - j >= dd.
    // Rounds r = (rb, pair of column blocks); each round is 32 values per lane.
    const int rlim = (int)(rEnd - rowT0);
    const int clim = (int)(colEnd - colT0);
    const int dd = (int)(colT0 - rowT0 / RS);
    const int jl = wc * (S::TN / S::WC) + 4 * (lane >> 5);  // lane part of the column
    constexpr int CP = S::EP;                                // column blocks per round
    constexpr int ROUNDS = S::RB * (S::CB / CP);
    auto c_ptr = [&](int rb) {
        const int i = wr * (S::TM / S::WR) + rb * 32 + (lane & 31);
        return A + (rowT0 + i) + (colT0 + jl) * lda;
    };
    auto c_src = [&](int rb) {
        const int i = wr * (S::TM / S::WR) + rb * 32 + (lane & 31);
        return Csrc + (rowT0 + i) + (colT0 + jl) * lds_;
    };
    auto c_ok = [&](int rb, int ju) {
        const int i = wr * (S::TM / S::WR) + rb * 32 + (lane & 31);
        const int j = jl + ju;
        // Complex: the real row i of the tile is complex row (rowT0 + i) / 2
        // (rowT0 is even), i.e. i / 2 - j >= dd with dd = colT0 - rowT0 / 2.
        return i < rlim && j < clim && (!HERM || (CPLX ? (i >> 1) : i) - j >= dd);
    };
    // Interior tiles (fully inside the region and, for the lower part, fully
    // below the diagonal) take a branch-free path: raw buffer loads and stores
    // with one per-lane offset and a scalar per-column offset. Edge tiles use
    // per-element predicates.
    const bool interior = rlim >= S::TM && clim >= S::TN &&
                          (!HERM || (CPLX ? rowT0 / RS >= colT0 + S::TN - 1 : -dd >= S::TN - 1));
    const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
        A + rowT0 + colT0 * lda, 0,
        (int)(((int64_t)S::TN * lda) * (int64_t)sizeof(T) < 0x7fffffff
                  ? ((int64_t)S::TN * lda) * (int64_t)sizeof(T) : 0x7fffffff),
        kBufFlags);
    const __amdgpu_buffer_rsrc_t crs_in = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(Csrc) + rowT0 + colT0 * lds_, 0,
        (int)(((int64_t)S::TN * lds_) * (int64_t)sizeof(T) < 0x7fffffff
                  ? ((int64_t)S::TN * lds_) * (int64_t)sizeof(T) : 0x7fffffff),
        kBufFlags);
    auto c_voff = [&](int rb, int64_t ld) {
        const int i = wr * (S::TM / S::WR) + rb * 32 + (lane & 31);
        return (int)((i + (int64_t)jl * ld) * (int64_t)sizeof(T));
    };
    auto c_load = [&](int r, double (&cv)[CP][16]) {
        const int rb = r / (S::CB / CP), c2 = (r % (S::CB / CP)) * CP;
        if (interior) {
            const int vo = c_voff(rb, lds_);
#pragma unroll
            for (int h = 0; h < CP; ++h)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int ju = (c2 + h) * 32 + 8 * (e >> 2) + (e & 3);
                    cv[h][e] = buf_load_c<T>(crs_in, vo, (int)(ju * lds_ * (int64_t)sizeof(T)));
                }
            return;
        }
        const T* const p0 = c_src(rb);
#pragma unroll
        for (int h = 0; h < CP; ++h)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int ju = (c2 + h) * 32 + 8 * (e >> 2) + (e & 3);
                cv[h][e] = c_ok(rb, ju) ? (double)p0[ju * lds_] : 0.0;
            }
    };
    auto c_store = [&](int r, const double (&cv)[CP][16]) {
        const int rb = r / (S::CB / CP), c2 = (r % (S::CB / CP)) * CP;
        if (interior) {
            const int vo = c_voff(rb, lda);
#pragma unroll
            for (int h = 0; h < CP; ++h)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int ju = (c2 + h) * 32 + 8 * (e >> 2) + (e & 3);
                    buf_store_c<T>(cv[h][e] - acc_value(rb, c2 + h, e), crs, vo,
                                   (int)(ju * lda * (int64_t)sizeof(T)));
                }
            return;
        }
        T* const p0 = c_ptr(rb);
#pragma unroll
        for (int h = 0; h < CP; ++h)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int ju = (c2 + h) * 32 + 8 * (e >> 2) + (e & 3);
                if (c_ok(rb, ju)) p0[ju * lda] = (T)(cv[h][e] - acc_value(rb, c2 + h, e));
            }
    };

    double cva[CP][16], cvb[CP][16];
    // The single-chain form with two pieces has the registers to load the
    // first C round during its last stage; every other form loads it after
    // the loop.
    constexpr bool C_PREFETCH = S::NP == 2 && !TWO_LEVEL;
    for (int p = 0; p < S::NST - 1; ++p) issue_stage(p);
    // One stage: wait for its copies, refill the buffer freed last, then its
    // k steps on the matrix cores.
    // first_c (std::bool_constant): the first stage of a chunk of the
    // two-level forms. Its first product term starts the chunk sums from zero
    // (so the flush need not clear the accumulators), and in the FP16 form it
    // also loads the chunk's factors.
    const f16v zero16 = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f,
                         0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    auto stage = [&](int st, bool prefetch_c, auto first_c) {
        constexpr bool FRESH = TWO_LEVEL && decltype(first_c)::value;
        constexpr bool LOAD_SCALES = S::F16 && FRESH;
        const int buf = st % S::NST;
        // This wavefront's copies of stage st are in LDS (the NST - 2 later
        // stages already issued may still be in flight); the barrier makes
        // everyone's visible and retires every read of the buffer refilled
        // next.
        __builtin_amdgcn_s_waitcnt(vmcnt_imm<(S::NST - 2) * S::PER_WAVE>());
        // A bare s_barrier: __syncthreads() would add a release fence, i.e.
        // vmcnt(0), and drain the stages still in flight. Ordering needs no
        // fence here: each wavefront has waited for its own copies of this
        // stage, and its reads of the buffer refilled below returned before
        // the MFMAs that consumed them. The memory clobber keeps the compiler
        // from moving LDS accesses across the barrier.
        asm volatile("s_barrier" ::: "memory");
        // First C round in flight during the last stage (C_PREFETCH).
        if (C_PREFETCH && prefetch_c) c_load(0, cva);
        const unsigned char* B0 = lds + buf * S::BUF;
        using Frag = std::conditional_t<S::F16, h8, bf8>;
        Frag lp[S::NP][S::KSTEPS][S::RB], wp[S::NP][S::KSTEPS][S::CB];
        auto read_l = [&](int p, int ks) {
            const int seg = ks * 2 + (lane >> 5);  // 8 k values per lane
#pragma unroll
            for (int b = 0; b < S::RB; ++b) {
                const int ra = wr * (S::TM / S::WR) + b * 32 + (lane & 31);
                lp[p][ks][b] = __builtin_bit_cast(Frag, *reinterpret_cast<const uint4*>(B0 + p * S::A_PLANE + lds_off<S::ROWB>(ra, seg)));
            }
        };
        auto read_w = [&](int p, int ks) {
            const int seg = ks * 2 + (lane >> 5);
#pragma unroll
            for (int b = 0; b < S::CB; ++b) {
                const int rc = wc * (S::TN / S::WC) + b * 32 + (lane & 31);
                wp[p][ks][b] = __builtin_bit_cast(Frag, *reinterpret_cast<const uint4*>(B0 + S::NP * S::A_PLANE + p * S::W_PLANE + lds_off<S::ROWB>(rc, seg)));
            }
        };
        // Fragments in the order the MFMAs below consume them: L0, W0, W1, L1
        // (and W2, L2 with three pieces).
        auto read_frags = [&](int ks) {
            read_l(0, ks);
            read_w(0, ks);
            read_w(1, ks);
            read_l(1, ks);
            if constexpr (S::NP == 3) {
                read_w(2, ks);
                read_l(2, ks);
            }
        };
        // The products of one accumulator are RB*CB MFMAs apart, so
        // consecutive MFMAs never wait on each other's result.
        // fresh_c (std::bool_constant): the first k step of a chunk, whose
        // first term accumulates onto zero.
        auto mfmas = [&](int ks, auto fresh_c) {
#pragma unroll
            for (int term = 0; term < S::NTERM; ++term)
#pragma unroll
                for (int rb = 0; rb < S::RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < S::CB; ++cb) {
                        const f16v c = (decltype(fresh_c)::value && term == 0) ? zero16 : acc[rb][cb];
                        if constexpr (S::F16)
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                wp[term_b(term)][ks][cb], lp[term_a(term)][ks][rb], c, 0, 0, 0);
                        else
                            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                wp[term_b(term)][ks][cb], lp[term_a(term)][ks][rb], c, 0, 0, 0);
                    }
        };
        constexpr auto fresh0 = std::bool_constant<FRESH>{};
        constexpr auto later = std::false_type{};
        if constexpr (S::KSTEPS == 2) {
            if constexpr (LOAD_SCALES) load_scales(st);
            read_frags(0);
            read_frags(1);
            // The next stage's copies after this stage's fragment reads (they
            // write LDS, so they cannot move above reads of LDS; the buffer
            // they fill was last read before the barrier).
            issue_stage(st + S::NST - 1);
            mfmas(0, fresh0);
            mfmas(1, later);
            // Schedule: (a chunk's factors,) k step 0's fragment reads, then
            // its MFMAs with k step 1's reads interleaved evenly, then k step
            // 1's MFMAs with the next stage's copies in between.
            static_assert(S::MFMAS >= S::PER_WAVE, "a product per copy");
            if constexpr (LOAD_SCALES) __builtin_amdgcn_sched_group_barrier(0x020, NSCALE, 0);  // VMEM read
            __builtin_amdgcn_sched_group_barrier(0x100, S::READS, 0);  // DS read
            interleave_mfma_reads<S::MFMAS, S::READS>();
            for (int q = 0; q < S::PER_WAVE; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
            }
            __builtin_amdgcn_sched_group_barrier(0x008, S::MFMAS - S::PER_WAVE, 0);
        } else {
            if constexpr (LOAD_SCALES) load_scales(st);
            read_frags(0);
            issue_stage(st + S::NST - 1);  // after the fragment reads, as above
            mfmas(0, fresh0);
            // Schedule: (a chunk's factors,) the fragments of the first
            // product term (p0 x p0'), then its MFMAs with the remaining
            // fragment reads interleaved, then the next stage's copies between
            // further MFMAs.
            constexpr int first = S::RB + S::CB, rest = S::READS - first;
            static_assert(S::MFMAS - rest >= S::PER_WAVE, "a product per copy");
            if constexpr (LOAD_SCALES) __builtin_amdgcn_sched_group_barrier(0x020, NSCALE, 0);  // VMEM read
            __builtin_amdgcn_sched_group_barrier(0x100, first, 0);
            for (int r = 0; r < rest; ++r) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            for (int q = 0; q < S::PER_WAVE; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
            }
            __builtin_amdgcn_sched_group_barrier(0x008, S::MFMAS - rest - S::PER_WAVE, 0);
        }
    };
    if constexpr (TWO_LEVEL) {
        // Chunks of FL stages; after each the FP32 sums move into the FP32
        // totals, and the chunk's first stage (peeled) restarts them from
        // zero. The flush sits outside the stage loop, unconditionally: a
        // flush inside it (taken on some iterations) makes the accumulators a
        // merge of two values at the loop's back edge, which the compiler
        // then keeps in VGPRs and copies to and from the MFMA's accumulation
        // registers every stage.
        for (int s0 = 0; s0 < nstages; s0 += S::FL) {
            const int s1 = s0 + S::FL < nstages ? s0 + S::FL : nstages;
            stage(s0, false, std::true_type{});
            for (int st = s0 + 1; st < s1; ++st) stage(st, false, std::false_type{});
#pragma unroll
            for (int rb = 0; rb < S::RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < S::CB; ++cb)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        if constexpr (S::F16)  // the factors are powers of two: the product is exact
                            acct[rb][cb][e] = __builtin_fmaf(acc[rb][cb][e], rsv[rb] * csv[cb][e >> 2][e & 3],
                                                             acct[rb][cb][e]);
                        else
                            acct[rb][cb][e] += acc[rb][cb][e];
                    }
        }
    } else {
        // The last stage apart: it also starts the first C round's loads.
        for (int st = 0; st < nstages - 1; ++st) stage(st, false, std::false_type{});
        stage(nstages - 1, true, std::false_type{});
    }
    // The copies issued past the last stage still write LDS: drain them
    // before the workgroup can end.
    __builtin_amdgcn_s_waitcnt(vmcnt_imm<0>());

    // Accumulator layout of the 32x32 MFMA with the column operand first:
    // element e of lane l is C row (l % 32), C column 8*(e/4) + 4*(l/32) + e%4
    // of the 32x32 block. Each round's 32 C values of a lane are all loaded
    // before any is stored: the stores could alias later loads, so
    // interleaving them would serialize one memory round trip per element.
    // Round r + 1 is loaded before round r is stored, so one round's latency
    // overlaps the previous round's stores.
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        double (&cur)[CP][16] = (r & 1) ? cvb : cva;
        double (&nxt)[CP][16] = (r & 1) ? cva : cvb;
        if (!C_PREFETCH && r == 0) c_load(0, cur);
        if (r + 1 < ROUNDS) c_load(r + 1, nxt);
        c_store(r, cur);
    }
}

// The product forms as separate kernels, so that profiles tell them apart.
template <typename T, bool HERM, class S, bool CPLX>
__global__ __launch_bounds__(S::THREADS, S::MINB) void update_bf16x3(const DevProb* __restrict__ probs,
                                                                     GroupMap M, Region rg, int64_t k0,
                                                                     int kw, int64_t j0, int ss)
{
    static_assert(S::NP == 2 && !S::F16, "three products from two pieces");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    update_body<T, HERM, S, CPLX>(probs, M, rg, k0, kw, j0, ss, lds);
}
template <typename T, bool HERM, class S, bool CPLX>
__global__ __launch_bounds__(S::THREADS, S::MINB) void update_bf16x6(const DevProb* __restrict__ probs,
                                                                     GroupMap M, Region rg, int64_t k0,
                                                                     int kw, int64_t j0, int ss)
{
    static_assert(S::NP == 3, "six products from three pieces");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    update_body<T, HERM, S, CPLX>(probs, M, rg, k0, kw, j0, ss, lds);
}

template <typename T, bool HERM, class S, bool CPLX>
__global__ __launch_bounds__(S::THREADS, S::MINB) void update_fp16x3(const DevProb* __restrict__ probs,
                                                                     GroupMap M, Region rg, int64_t k0,
                                                                     int kw, int64_t j0, int ss)
{
    static_assert(S::F16 && HERM && !CPLX, "the FP16 form serves real Hermitian problems");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    update_body<T, HERM, S, CPLX>(probs, M, rg, k0, kw, j0, ss, lds);
}

template <typename T, bool HERM, class S, bool CPLX>
constexpr auto kernel_of()
{
    if constexpr (S::F16) return update_fp16x3<T, HERM, S, CPLX>;
    else if constexpr (S::NP == 2) return update_bf16x3<T, HERM, S, CPLX>;
    else return update_bf16x6<T, HERM, S, CPLX>;
}

template <typename T, bool HERM, class S, bool CPLX>
hipError_t launch_shape(const DevProb* probs, const GroupSpan* spans, int nspan, Region rg,
                        int64_t k0, int kw, int64_t j0, int ss, hipStream_t s)
{
    GroupMap M;
    M.ng = 0;
    M.off[0] = 0;
    int64_t total = 0;
    for (int i = 0; i < nspan; ++i) {
        const GroupSpan& g = spans[i];
        const int64_t nrows = (rg.r0 + rg.rlen < g.nmax ? rg.r0 + rg.rlen : g.nmax) - rg.r0;
        const int64_t nc = (rg.c0 + rg.clen < g.nmax ? rg.c0 + rg.clen : g.nmax) - rg.c0;
        const int64_t NR = (nrows * (CPLX ? 2 : 1) + S::TM - 1) / S::TM, NC = (nc + S::TN - 1) / S::TN;
        const int64_t tiles = (HERM && !CPLX && S::TM == S::TN) ? NC * NR - NC * (NC - 1) / 2 : NR * NC;
        M.p0[M.ng] = (int)g.p0;
        M.wpp[M.ng] = (int)tiles;
        M.aux[M.ng] = 0;
        total += tiles * g.count;
        M.off[++M.ng] = (int)total;
    }
    if (total == 0) return hipSuccess;
    const unsigned grid_x = (unsigned)((total + 7) / 8 * 8);  // XCD order needs a multiple of 8
    const auto k = kernel_of<T, HERM, S, CPLX>();
    // The dynamic-LDS limit is a per-device function attribute: set it once
    // on each device the kernel runs on.
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
    if (!bit || !(attr_set.load() & bit)) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit);
    }
    hipLaunchKernelGGL(k, dim3(grid_x), dim3(S::THREADS), S::LDS, s, probs, M, rg, k0, kw, j0, ss);
    return hipGetLastError();
}

// The tile shape follows the width of each group's updated column range;
// groups of one shape share a launch.
template <typename T, bool HERM, int NP, bool CPLX, bool F16 = false>
hipError_t launch_t(const DevProb* probs, const GroupSpan* spans, int nspan, Region rg, int64_t k0,
                    int kw, int64_t j0, int ss, hipStream_t s)
{
    using Narrow = std::conditional_t<F16, Narrow16, std::conditional_t<NP == 2, Narrow3, Narrow6>>;
    using Medium = std::conditional_t<F16, Wide16, std::conditional_t<NP == 2, Medium3, Medium6>>;
    using Wide = std::conditional_t<F16, Wide16, std::conditional_t<NP == 2, Wide3, Wide6>>;
    GroupSpan by[3][kMaxGroupsPerLaunch];
    int cnt[3] = {0, 0, 0};
    for (int i = 0; i < nspan; ++i) {
        const GroupSpan& g = spans[i];
        const int64_t nrows = (rg.r0 + rg.rlen < g.nmax ? rg.r0 + rg.rlen : g.nmax) - rg.r0;
        const int64_t nc = (rg.c0 + rg.clen < g.nmax ? rg.c0 + rg.clen : g.nmax) - rg.c0;
        if (nrows <= 0 || nc <= 0 || k0 + kw > g.nmax) continue;
        const int shape = nc <= 128 ? 0 : (nc <= 256 ? 1 : 2);
        by[shape][cnt[shape]++] = g;
    }
    hipError_t e = hipSuccess;
    if (cnt[0]) e = launch_shape<T, HERM, Narrow, CPLX>(probs, by[0], cnt[0], rg, k0, kw, j0, ss, s);
    if (e == hipSuccess && cnt[1])
        e = launch_shape<T, HERM, Medium, CPLX>(probs, by[1], cnt[1], rg, k0, kw, j0, ss, s);
    if (e == hipSuccess && cnt[2])
        e = launch_shape<T, HERM, Wide, CPLX>(probs, by[2], cnt[2], rg, k0, kw, j0, ss, s);
    return e;
}

template <int NP>
hipError_t launch_np(bool herm, int dtype, const DevProb* probs, const GroupSpan* spans, int nspan,
                     Region rg, int64_t k0, int kw, int64_t j0, int ss, hipStream_t s)
{
    if (dtype == 2) {
        if (herm) return launch_t<double, true, NP, true>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
        return launch_t<double, false, NP, true>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
    }
    if (herm) {
        if (dtype == 0) return launch_t<double, true, NP, false>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
        return launch_t<float, true, NP, false>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
    }
    if (dtype == 0) return launch_t<double, false, NP, false>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
    return launch_t<float, false, NP, false>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
}

}  // namespace

hipError_t launch_update_split(bool herm, int dtype, int pieces, bool f16, const DevProb* probs,
                               const GroupSpan* spans, int nspan, Region rg, int64_t k0, int kw,
                               int64_t j0, int ss, hipStream_t s)
{
    // Every stage covers kKAlign real k: 32 real or 16 complex columns.
    if ((kw * (dtype == 2 ? 2 : 1)) % kKAlign != 0 || (herm && rg.r0 != rg.c0) ||
        nspan > kMaxGroupsPerLaunch)
        return hipErrorInvalidValue;
    if (f16) {
        // Real Hermitian only; chunks start on the 64-column blocks of the factors.
        if (!herm || dtype == 2 || pieces != 2 || (k0 - j0) % 64 != 0) return hipErrorInvalidValue;
        if (dtype == 0) return launch_t<double, true, 2, false, true>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
        return launch_t<float, true, 2, false, true>(probs, spans, nspan, rg, k0, kw, j0, ss, s);
    }
    if (pieces == 2) return launch_np<2>(herm, dtype, probs, spans, nspan, rg, k0, kw, j0, ss, s);
    if (pieces == 3) return launch_np<3>(herm, dtype, probs, spans, nspan, rg, k0, kw, j0, ss, s);
    return hipErrorInvalidValue;
}

}  // namespace dpp
