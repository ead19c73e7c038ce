// FP64 Schur-complement update of the blocked DPP sampler on gfx950 MFMA.
//
// After a group of pivots [k0, k0+kw) has been decided and its panel solved,
// the trailing matrix receives the outer-product update of the blocked
// factorization (Sec. 3, the last line of the blocked LU loop; for Hermitian
// K the symmetric form the paper notes halves the work):
//   LDL^H: C[r][c] -= sum_k L[r][k] * d'_k * L[c][k]   (lower part only)
//   LU:    C[r][c] -= sum_k L[r][k] * U[k][c]
// for r in [r0, r0 + rlen), c in [c0, c0 + clen), both clipped to n (LDL^H:
// r0 = c0, rows to n). The modified pivots d'_k of
// rejected indices already include the -1 of Prop. 4, so this is a plain
// product: Prop. 5 is what makes the blocked update equal to the unblocked one.
//
// Tiling: a 256-thread workgroup owns a 128x128 tile of C; its four wavefronts
// each own 64x64 as 4x4 blocks of v_mfma_f64_16x16x4f64. K advances in chunks
// of 16 staged through two LDS buffers (k-major, so the column-major source is
// read with unit stride); the next chunk's loads are in flight while the
// current one is multiplied. For LDL^H only tiles on or below the diagonal are launched.
// One launch covers the problems of several size groups (GroupMap): workgroup
// b takes slot (b % 8) * (G / 8) + b / 8 of the launch (G, the grid size, is a
// multiple of 8), so each XCD takes a contiguous range of tiles, and the slot
// names a problem and one of its tiles.
//
// Complex kernels (CPLX) run the same product on the real forms of the
// factors (dpp_internal.h): a tile is 128 real rows of C' (64 complex rows)
// by 128 complex columns, and each staged chunk of 16 real k (8 complex
// columns) is built from the complex panel in A as it is stored to LDS: L'
// rows 2i and 2i + 1 from L_i, W' from W = L D' (LDL^H) or from the rows of U
// (LU). Hermitian tiles entirely above the diagonal exit at once.
#include "dpp_internal.h"

namespace dpp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 128;       // tile rows
constexpr int TN = 128;       // tile cols
constexpr int KC = 16;        // k per LDS stage
constexpr int PAD = 2;        // LDS row padding (doubles)

struct TileCoord {
    int64_t i0, j0;
};

// Map a linear tile index to (row tile, col tile) of the region. For the
// Hermitian case the region is the lower trapezoid {J <= I}; tiles are ordered
// by column tile, then row tile.
__device__ __forceinline__ bool tile_of(int64_t t, int64_t NR, int64_t NC, bool herm,
                                        TileCoord& tc)
{
    if (!herm) {
        if (t >= NR * NC) return false;
        tc.i0 = (t % NR) * TM;
        tc.j0 = (t / NR) * TN;
        return true;
    }
    // count of tiles in columns < J: J*NR - J*(J-1)/2
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

// Load through the global address space: a generic (flat) load also counts
// against the LDS wait counter, so every LDS fragment wait would then wait for
// the next chunk's operand loads as well.
template <typename T>
__device__ __forceinline__ double gload(const T* p)
{
    return (double)*(const __attribute__((address_space(1))) T*)(p);
}

template <typename T>
__device__ __forceinline__ void gstore(T* p, double v)
{
    *(__attribute__((address_space(1))) T*)(p) = (T)v;
}

template <typename T, bool HERM, bool CPLX>
__global__ __launch_bounds__(256, 2) void update_f64(const DevProb* __restrict__ probs, GroupMap M,
                                                  Region rg, int64_t k0, int kw)
{
    static_assert(!CPLX || sizeof(T) == 8, "complex storage: FP64 parts");
    constexpr int RS = CPLX ? 2 : 1;  // real rows of C per row of the region
    // XCD-contiguous order over the launch (grid size a multiple of 8), then
    // the problem and its tile.
    int pi, tw, unused;
    if (!group_slot(M, xcd_order(blockIdx.x, gridDim.x), pi, tw, unused)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    const int64_t rEnd = rg.r0 + rg.rlen < n ? rg.r0 + rg.rlen : n;
    const int64_t cEnd = rg.c0 + rg.clen < n ? rg.c0 + rg.clen : n;
    const int64_t nrows = rEnd - rg.r0, ncols = cEnd - rg.c0;
    if (nrows <= 0 || ncols <= 0 || k0 + kw > n || k0 >= P.npiv) return;
    // Only decided columns contribute: k in [k0, min(k0 + kw, npiv)).
    if (k0 + kw > P.npiv) kw = (int)(P.npiv - k0);
    const int64_t NR = (nrows * RS + TM - 1) / TM, NC = (ncols + TN - 1) / TN;
    const int64_t t = tw;
    TileCoord tc;
    if (!tile_of(t, NR, NC, HERM && !CPLX, tc)) return;
    // Complex Hermitian: skip tiles entirely above the diagonal.
    if (CPLX && HERM && rg.r0 + (tc.i0 + TM - 1) / RS < rg.c0 + tc.j0) return;

    // C as a real column-major matrix: RS real rows per row of the region.
    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda * RS;
    int64_t lds_;  // leading dimension of the source C is read from (K when k0 == 0)
    const T* __restrict__ Csrc = first_source<T>(P, k0 == 0, lds_);
    lds_ *= RS;
    const double* __restrict__ piv = P.piv;

    // Two LDS buffers: chunk c + 1 is loaded into registers while chunk c is
    // multiplied, then stored to the other buffer; one barrier per chunk.
    __shared__ double sA[2][KC][TM + PAD];
    __shared__ double sB[2][KC][TN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    d4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

    const int64_t rowA0 = rg.r0 * RS + tc.i0;  // real row of C at tile row 0
    const int64_t colB0 = rg.c0 + tc.j0;       // column of C at tile col 0
    const int64_t rEndR = rEnd * RS;

    // Register staging of one chunk. A: thread -> (i = tid % 128, kk = tid/128 + 2q).
    // B (LDL^H): (j = tid % 128, kk = tid/128 + 2q), B[k][c] = L[c][k] * d'_k.
    // B (LU): (kk = tid % 16, j = tid/16 + 16q), B[k][c] = U[k][c] = A[k][c].
    // The loads are unconditional (rows and columns past the region re-read
    // the last one; they only feed accumulators that are never stored) and
    // nothing uses their values before store_chunk, so they stay in flight
    // during the current chunk's products; the pivot scaling of B happens at
    // the store for the same reason.
    // Complex: A: (complex row i = tid % 64, complex k = tid/64 + 4q, q < 2);
    // B (LDL^H): (j = tid % 128, complex k = tid/128 + 2q, q < 4); B (LU):
    // (complex k = tid % 8, j = tid/8 + 32q, q < 4); each complex value fills
    // its entries of the real forms at the store.
    double ra[KC / 2], rb[KC / 2], rp[KC / 2];
    auto load_chunk = [&](int kc) {
        if constexpr (CPLX) {
            const int64_t kb = k0 + kc / 2;  // first complex column of the chunk
            const int64_t r0c = rowA0 / 2;
            const int64_t gr = r0c + (tid & 63) < rEnd ? r0c + (tid & 63) : rEnd - 1;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const T* p = A + 2 * (gr + (kb + (tid >> 6) + 4 * q) * P.lda);
                ra[2 * q] = gload(p);
                ra[2 * q + 1] = gload(p + 1);
            }
            if constexpr (HERM) {
                const int64_t gc = colB0 + (tid & (TN - 1)) < cEnd ? colB0 + (tid & (TN - 1)) : cEnd - 1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t gk = kb + (tid >> 7) + 2 * q;
                    const T* p = A + 2 * (gc + gk * P.lda);
                    rb[2 * q] = gload(p);
                    rb[2 * q + 1] = gload(p + 1);
                    rp[q] = gload(piv + gk);
                }
            } else {
                const int64_t gk = kb + (tid & 7);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t gc0 = colB0 + (tid >> 3) + 32 * q;
                    const int64_t gc = gc0 < cEnd ? gc0 : cEnd - 1;
                    const T* p = A + 2 * (gk + gc * P.lda);
                    rb[2 * q] = gload(p);
                    rb[2 * q + 1] = gload(p + 1);
                }
            }
            return;
        }
        {
            const int64_t gr = rowA0 + (tid & (TM - 1)) < rEnd ? rowA0 + (tid & (TM - 1)) : rEnd - 1;
#pragma unroll
            for (int q = 0; q < KC / 2; ++q) {
                const int64_t gk = k0 + kc + (tid >> 7) + 2 * q;
                ra[q] = gload(A + gr + gk * lda);
            }
        }
        if constexpr (HERM) {
            const int64_t gc = colB0 + (tid & (TN - 1)) < cEnd ? colB0 + (tid & (TN - 1)) : cEnd - 1;
#pragma unroll
            for (int q = 0; q < KC / 2; ++q) {
                const int64_t gk = k0 + kc + (tid >> 7) + 2 * q;
                rb[q] = gload(A + gc + gk * lda);
                rp[q] = gload(piv + gk);
            }
        } else {
            const int64_t gk = k0 + kc + (tid & (KC - 1));
#pragma unroll
            for (int q = 0; q < TN / 16; ++q) {
                const int64_t gc0 = colB0 + (tid >> 4) + 16 * q;
                const int64_t gc = gc0 < cEnd ? gc0 : cEnd - 1;
                rb[q] = gload(A + gk + gc * lda);
            }
        }
    };
    auto store_chunk = [&](int buf) {
        if constexpr (CPLX) {
            // L' rows 2i, 2i + 1 (HERM: (Re, Im), (Im, -Re); LU: (Re, -Im), (Im, Re)).
            const int i = tid & 63;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int kk = 2 * ((tid >> 6) + 4 * q);
                const double re = ra[2 * q], im = ra[2 * q + 1];
                sA[buf][kk][2 * i] = re;
                sA[buf][kk + 1][2 * i] = HERM ? im : -im;
                sA[buf][kk][2 * i + 1] = im;
                sA[buf][kk + 1][2 * i + 1] = HERM ? -re : re;
            }
            if constexpr (HERM) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = 2 * ((tid >> 7) + 2 * q);
                    sB[buf][kk][tid & (TN - 1)] = rb[2 * q] * rp[q];
                    sB[buf][kk + 1][tid & (TN - 1)] = rb[2 * q + 1] * rp[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = 2 * (tid & 7);
                    sB[buf][kk][(tid >> 3) + 32 * q] = rb[2 * q];
                    sB[buf][kk + 1][(tid >> 3) + 32 * q] = rb[2 * q + 1];
                }
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < KC / 2; ++q) sA[buf][(tid >> 7) + 2 * q][tid & (TM - 1)] = ra[q];
        if constexpr (HERM) {
#pragma unroll
            for (int q = 0; q < KC / 2; ++q) sB[buf][(tid >> 7) + 2 * q][tid & (TN - 1)] = rb[q] * rp[q];
        } else {
#pragma unroll
            for (int q = 0; q < TN / 16; ++q) sB[buf][tid & (KC - 1)][(tid >> 4) + 16 * q] = rb[q];
        }
    };
    static_assert(TN / 16 == KC / 2, "B staging uses KC/2 registers in both forms");

    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    const int nchunks = kw * RS / KC;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunks) load_chunk((ch + 1) * KC);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            double af[4], bf[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                af[b] = sA[buf][kk][wm * 64 + b * 16 + (lane & 15)];
                bf[b] = sB[buf][kk][wn * 64 + b * 16 + (lane & 15)];
            }
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[bj], af[bi], acc[bi][bj],
                                                                       0, 0, 0);
        }
        // The other buffer was last read in chunk ch - 1, before the barrier
        // that ended it.
        if (ch + 1 < nchunks) store_chunk(buf ^ 1);
        __syncthreads();
    }

    // D block layout of v_mfma_f64_16x16x4f64 (measured on gfx950): element e
    // of lane l is row l/16 + 4e, column l%16 of the product. The column
    // operand goes first, so lane l holds C row l%16 and C columns l/16 + 4e:
    // 16 lanes cover 16 consecutive rows of one column of column-major C.
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int64_t gr = rowA0 + wm * 64 + bi * 16 + (lane & 15);
        T* const rowp = A + gr;
        const T* const srcp = Csrc + gr;
        // All loads of this 16-row block before any store (see update_split.hip).
        double cv[4][4];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gc = colB0 + wn * 64 + bj * 16 + (lane >> 4) + 4 * e;
                const bool ok = gr < rEndR && gc < cEnd && (!HERM || gr / RS >= gc);
                cv[bj][e] = ok ? gload(srcp + gc * lds_) : 0.0;
            }
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gc = colB0 + wn * 64 + bj * 16 + (lane >> 4) + 4 * e;
                const bool ok = gr < rEndR && gc < cEnd && (!HERM || gr / RS >= gc);
                if (ok) gstore(rowp + gc * lda, cv[bj][e] - acc[bi][bj][e]);
            }
    }
}

// Real Hermitian kernels with FP64 storage: the same product with the operands
// copied straight from A into LDS by the direct-to-LDS loads
// (global_load_lds_dword), so no register staging and no LDS store phase at
// the end of a chunk. A stage holds 16 k of both operands: k-row kk of an
// operand is its 128 rows of column k (1 KiB), in four 256-byte blocks of 32
// rows. One copy instruction fills one block: lane j supplies word j % 2 of
// the double at slot j / 2, and the rows are clamped one by one (rows past
// the region re-read the last one; they only feed accumulators that are
// never stored). Within a block, odd k-rows hold row m at slot m ^ 16: the
// 16 lanes of a fragment read that take k-row kk + 1 then use the other 32
// banks from the 16 that take k-row kk. B is L unscaled; the pivots d'_k
// multiply its fragments as they are read (the product the register path
// forms before its LDS store, so the results are the same); they are copied
// with the operands (32 from the stage's first k, indices clamped to n - 1),
// so no register holds a load across stages. Two stages: the next one is
// copied while the current one is multiplied, one barrier each.
constexpr int kDmaOps = 2 * KC * TM * 8;   // bytes: A then B, 16 k-rows of 1 KiB each
constexpr int kDmaStage = kDmaOps + 256;   // then the pivots
static_assert(TM == TN, "both operands in 128-row k-rows");

__global__ __launch_bounds__(256, 2) void update_f64_dma(const DevProb* __restrict__ probs, GroupMap M,
                                                      Region rg, int64_t k0, int kw)
{
    typedef const void __attribute__((address_space(1)))* gptr_t;
    typedef void __attribute__((address_space(3)))* lptr_t;
    int pi, tw, unused;
    if (!group_slot(M, xcd_order(blockIdx.x, gridDim.x), pi, tw, unused)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    const int64_t rEnd = rg.r0 + rg.rlen < n ? rg.r0 + rg.rlen : n;
    const int64_t cEnd = rg.c0 + rg.clen < n ? rg.c0 + rg.clen : n;
    const int64_t nrows = rEnd - rg.r0, ncols = cEnd - rg.c0;
    if (nrows <= 0 || ncols <= 0 || k0 + kw > n || k0 >= P.npiv) return;
    if (k0 + kw > P.npiv) kw = (int)(P.npiv - k0);
    const int64_t NR = (nrows + TM - 1) / TM, NC = (ncols + TN - 1) / TN;
    TileCoord tc;
    if (!tile_of(tw, NR, NC, true, tc)) return;

    double* __restrict__ A = static_cast<double*>(P.A);
    const int64_t lda = P.lda;
    int64_t lds_;
    const double* __restrict__ Csrc = first_source<double>(P, k0 == 0, lds_);
    const double* __restrict__ piv = P.piv;

    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * kDmaStage];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t rowA0 = rg.r0 + tc.i0, colB0 = rg.c0 + tc.j0;

    // Copies: wavefront w fills k-rows 4w .. 4w + 3 of both operands, four
    // blocks each (32 copies per stage). Byte offsets in a column of A of
    // this lane's double in block q, for even and odd k-rows (A side, B side).
    int offA[4][2], offB[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const int m = (lane >> 1) ^ (par << 4);
            int64_t ga = rowA0 + 32 * q + m, gb = colB0 + 32 * q + m;
            ga = ga < rEnd - 1 ? ga : rEnd - 1;
            gb = gb < cEnd - 1 ? gb : cEnd - 1;
            offA[q][par] = (int)(ga * 8) + 4 * (lane & 1);
            offB[q][par] = (int)(gb * 8) + 4 * (lane & 1);
        }
    const int nstages = kw / KC;
    // Stage st's copies (past the last stage they re-read it into the buffer
    // that is free next, so the copies stay branch-free); wavefront 0 also
    // copies the stage's pivots.
    auto issue_stage = [&](int st) {
        const int64_t kc = k0 + (int64_t)(st < nstages ? st : nstages - 1) * KC;
        unsigned char* const dst = lds + (st & 1) * kDmaStage;
        if (wave == 0) {
            const int64_t ip = kc + (lane >> 1) < n - 1 ? kc + (lane >> 1) : n - 1;
            __builtin_amdgcn_global_load_lds((gptr_t)(reinterpret_cast<const char*>(piv + ip) + 4 * (lane & 1)),
                                             (lptr_t)(dst + kDmaOps), 4, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int kk = 4 * wave + r;
            const char* col = reinterpret_cast<const char*>(A + (kc + kk) * lda);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                __builtin_amdgcn_global_load_lds((gptr_t)(col + offA[q][kk & 1]),
                                                 (lptr_t)(dst + kk * 1024 + q * 256), 4, 0, 0);
                __builtin_amdgcn_global_load_lds((gptr_t)(col + offB[q][kk & 1]),
                                                 (lptr_t)(dst + KC * 1024 + kk * 1024 + q * 256), 4, 0, 0);
            }
        }
    };

    d4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};

    // Fragment slots: lane l reads row (16 b + l % 16) of its wavefront's 64
    // rows in k-row 4 ks + l / 16; the parity of that k-row is bit 4 of l.
    const int par = (lane >> 4) & 1;
    int fa[4], fb[4];  // byte offsets inside a k-row
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int ra = wm * 64 + b * 16 + (lane & 15), rb = wn * 64 + b * 16 + (lane & 15);
        fa[b] = (ra >> 5) * 256 + (((ra & 31) ^ (par << 4)) << 3) + (lane >> 4) * 1024;
        fb[b] = (rb >> 5) * 256 + (((rb & 31) ^ (par << 4)) << 3) + (lane >> 4) * 1024;
    }

    issue_stage(0);
    for (int st = 0; st < nstages; ++st) {
        // This wavefront's copies and pivot loads of stage st are complete
        // (nothing later has been issued); the barrier makes every
        // wavefront's copies visible and retires every read of the buffer
        // refilled next (last read in stage st - 1).
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        asm volatile("s_barrier" ::: "memory");
        const unsigned char* const B0 = lds + (st & 1) * kDmaStage;
        double dk[4];  // the pivot of k-row 4 ks + lane / 16
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            dk[ks] = *reinterpret_cast<const double*>(B0 + kDmaOps + (4 * ks + (lane >> 4)) * 8);
        double af[4][4], bf[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            af[0][b] = *reinterpret_cast<const double*>(B0 + fa[b]);
            bf[0][b] = *reinterpret_cast<const double*>(B0 + KC * 1024 + fb[b]) * dk[0];
        }
        issue_stage(st + 1);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            if (ks + 1 < 4) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    af[ks + 1][b] = *reinterpret_cast<const double*>(B0 + (ks + 1) * 4096 + fa[b]);
                    bf[ks + 1][b] =
                        *reinterpret_cast<const double*>(B0 + KC * 1024 + (ks + 1) * 4096 + fb[b]) * dk[ks + 1];
                }
            }
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[ks][bj], af[ks][bi], acc[bi][bj],
                                                                       0, 0, 0);
        }
    }
    // The copies issued past the last stage still write LDS.
    __builtin_amdgcn_s_waitcnt(0x0F70);

    // Epilogue as in update_f64 (D layout: lane l holds C row l % 16 and C
    // columns l / 16 + 4e of each 16 x 16 block).
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int64_t gr = rowA0 + wm * 64 + bi * 16 + (lane & 15);
        double* const rowp = A + gr;
        const double* const srcp = Csrc + gr;
        double cv[4][4];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gc = colB0 + wn * 64 + bj * 16 + (lane >> 4) + 4 * e;
                const bool ok = gr < rEnd && gc < cEnd && gr >= gc;
                cv[bj][e] = ok ? gload(srcp + gc * lds_) : 0.0;
            }
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gc = colB0 + wn * 64 + bj * 16 + (lane >> 4) + 4 * e;
                const bool ok = gr < rEnd && gc < cEnd && gr >= gc;
                if (ok) gstore(rowp + gc * lda, cv[bj][e] - acc[bi][bj][e]);
            }
    }
}

}  // namespace

hipError_t launch_update_f64(bool herm, int dtype, const DevProb* probs, const GroupSpan* spans,
                             int nspan, Region rg, int64_t k0, int kw, hipStream_t s)
{
    if (herm && rg.r0 != rg.c0) return hipErrorInvalidValue;
    const bool cplx = dtype == 2;
    if (kw % (cplx ? KC / 2 : KC) != 0 || nspan > kMaxGroupsPerLaunch) return hipErrorInvalidValue;
    GroupMap M;
    M.ng = 0;
    M.off[0] = 0;
    int64_t total = 0;
    for (int i = 0; i < nspan; ++i) {
        const GroupSpan& g = spans[i];
        const int64_t nrows = (rg.r0 + rg.rlen < g.nmax ? rg.r0 + rg.rlen : g.nmax) - rg.r0;
        const int64_t nc = (rg.c0 + rg.clen < g.nmax ? rg.c0 + rg.clen : g.nmax) - rg.c0;
        if (nrows <= 0 || nc <= 0 || k0 + kw > g.nmax) continue;
        const int64_t NR = (nrows * (cplx ? 2 : 1) + TM - 1) / TM, NC = (nc + TN - 1) / TN;
        const int64_t tiles = herm && !cplx ? NC * NR - NC * (NC - 1) / 2 : NR * NC;
        M.p0[M.ng] = (int)g.p0;
        M.wpp[M.ng] = (int)tiles;
        M.aux[M.ng] = 0;
        total += tiles * g.count;
        M.off[++M.ng] = (int)total;
    }
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)((total + 7) / 8 * 8)), block(256);
    if (cplx) {
        if (herm) hipLaunchKernelGGL((update_f64<double, true, true>), grid, block, 0, s, probs, M, rg, k0, kw);
        else hipLaunchKernelGGL((update_f64<double, false, true>), grid, block, 0, s, probs, M, rg, k0, kw);
    } else if (herm) {
        if (dtype == 0) hipLaunchKernelGGL(update_f64_dma, grid, block, 0, s, probs, M, rg, k0, kw);
        else hipLaunchKernelGGL((update_f64<float, true, false>), grid, block, 0, s, probs, M, rg, k0, kw);
    } else {
        if (dtype == 0) hipLaunchKernelGGL((update_f64<double, false, false>), grid, block, 0, s, probs, M, rg, k0, kw);
        else hipLaunchKernelGGL((update_f64<float, false, false>), grid, block, 0, s, probs, M, rg, k0, kw);
    }
    return hipGetLastError();
}

}  // namespace dpp
