// Diagonal-block kernel, general (LU) form; see leaf_common.h.
#include "leaf_common.h"

namespace dpp {
namespace {

using namespace leaf;

// ---------------------------------------------------------------------- LU
// Step 1 (wavefront 0, every workgroup): the unblocked sampler on the 64x64
// diagonal block, one block row per lane; at pivot j the row of U (lane j's
// registers) is broadcast by readlane and the rows below take the rank-one
// update.
//
// Step 2: both panels, with the factored block L11 (unit lower) and U11
// (upper, the modified pivots on its diagonal), each as solves X T^T = A of
// leaf_common.h's solve_group:
//   column panel, rows r below the block: L21 U11 = A21, i.e. X = A21 with
//     T = U11^T (lower, non-unit);
//   row panel, columns r right of the block: L11 U12 = A12, i.e. for each
//     column U12^T L11^T = A12^T: X = A12^T with T = L11 (unit lower).
// The row panel's columns are contiguous in memory; they pass through the
// wavefront's LDS tile so that loads and stores stay coalesced. A receives L21
// and U12; the split planes, the BF16 pieces of L21 by row and of U12^T by
// column.
// Each workgroup takes the same number of rows of the column panel and
// columns of the row panel (splitting them over separate workgroups measured
// slower: the chain, repeated per workgroup, dominates).
//
// LDS holds the factored block once, packed as the chain leaves it (strict
// lower part L11, upper part U11, by columns with pitch kLP: the row panel
// reads L11 by columns, the column panel U11^T, i.e. the same array by rows;
// the odd pitch keeps both access patterns free of bank conflicts), and one
// set of diagonal-block inverses, those of U11^T for the column panel, then
// those of L11 for the row panel: 75 KiB, so two workgroups fit on a CU when
// a launch needs more than one round.
constexpr int kLP = 70;  // three-way at worst for both read orders of solve_group

template <typename T, int NPC>
__global__ __launch_bounds__(kThreads, 2) void leaf_lu(const DevProb* __restrict__ probs, GroupMap M,
                                             int64_t c0, int64_t j0, int ss)
{
    int pi, bx, gpw;  // problem, workgroup within it, row groups per wavefront
    if (!group_slot(M, blockIdx.x, pi, bx, gpw)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    if (c0 >= P.npiv) return;  // npiv <= n: only the first npiv indices are decided
    const int bs = (int)((n - c0) < L ? (n - c0) : L);
    const int64_t idx0 = c0 + bs + (int64_t)bx * (kWaves * 16 * gpw);
    if (bx > 0 && idx0 >= n) return;

    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda;
    int64_t lds;  // leading dimension of the source the loads read (K at column 0)
    const T* __restrict__ S = first_source<T>(P, c0 == 0, lds);

    // sP[k + t*kLP] = entry (k, t) of the factored block: L11[k][t] for k > t,
    // U11[k][t] for k <= t.
    constexpr int kSmem = kWaves * 16 * kTilePitch + L * kLP + 4 * kInvBlock;
    static_assert(kSmem * sizeof(double) <= kLdsPerTwo, "two workgroups per CU");
    __shared__ double smem[kSmem];
    double* const sT = smem;
    double* const sP = smem + kWaves * 16 * kTilePitch;
    double* const sI = sP + L * kLP;                 // inverses of the diagonal blocks

    const int tid = threadIdx.x;
    if (tid < L) {
        const int lane = tid;
        double a[L];  // row `lane` of the block
        {
            // Buffer loads: the column offset is a scalar, so the 64 loads
            // share one address register; reads past the end of A return 0.
            const int64_t base = c0 + c0 * lds;
            const __amdgpu_buffer_rsrc_t rb =
                strip_rsrc(S + base, ((n - 1) * lds + n - base) * (int64_t)sizeof(T));
            const int cs = (int)(lds * (int64_t)sizeof(T));
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const double v = buf_load<T>(rb, lane * (int)sizeof(T), k * cs);
                a[k] = (lane < bs && k < bs) ? v : 0.0;
            }
#pragma unroll
            for (int k = 0; k < L; ++k) asm volatile("" : "+v"(a[k]));
        }
        const double ul = lane < bs ? P.u[c0 + lane] : 2.0;
        double mydp = 1.0;
        int mykeep = 0;
        int me = lane;

#pragma unroll
        for (int j = 0; j < L; ++j) {
            // Keeps the per-step lane masks from being hoisted out of the
            // unrolled loop into scalar registers (and spilled).
            asm volatile("" : "+v"(me));
            if (j < bs) {
                const double d = readlane_d(a[j], j);
                const double uj = readlane_d(ul, j);
                const bool keep = uj < d;                // Bernoulli(d) with stream u_j
                const double dp = keep ? d : d - 1.0;   // Prop. 4 on rejection
                const bool isj = me == j, below = me > j;
                // Rows at or above the pivot keep their entries (rows of U).
                const double l = below ? a[j] / dp : 0.0;
                // Row j of U lives in lane j's registers: it is read lane by
                // lane with readlane (into scalar registers), 16 entries ahead
                // of their FMAs. Writing it to LDS from the one lane and
                // reading it back took 35 instead of 21 us per chain.
#pragma unroll
                for (int kb = 0; kb < L; kb += 16) {
                    double v[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j) v[i] = readlane_d(a[kb + i], j);
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j) a[kb + i] -= l * v[i];
                }
                asm volatile("" ::: "memory");
                __builtin_amdgcn_wave_barrier();
                a[j] = isj ? dp : (below ? l : a[j]);
                mydp = isj ? dp : mydp;
                mykeep = isj ? (keep ? 1 : 0) : mykeep;
            }
        }

#pragma unroll
        for (int k = 0; k < L; ++k) sP[lane + k * kLP] = lane < bs ? a[k] : (k == lane ? 1.0 : 0.0);

        // The factored block goes to the workspace strip, not to A: other
        // workgroups of this launch may still be loading the original block
        // from A for their own copy of the chain. A later launch copies the
        // strip into A (no kernel reads the diagonal blocks from A).
        if (bx == 0 && lane < bs) {
            double* blk = P.diag + (c0 / L) * (L * L);
#pragma unroll
            for (int k = 0; k < L; ++k) blk[k * L + lane] = a[k];
            P.mask[c0 + lane] = (uint8_t)mykeep;
            P.piv[c0 + lane] = mydp;
        }
    }
    __syncthreads();
    // Rows below and columns right of a block exist only when the block is a
    // full 64 wide (a ragged block is the last one), so bs == L from here on.
    if (idx0 >= n) return;

    // U11^T is lower triangular with the pivots on its diagonal.
    if (tid < 64) invert_diag_blocks<false, kLP, true>(sP, sI, tid);
    __syncthreads();

    const int lane = tid & 63;
    const int q = lane >> 4, i16 = lane & 15;
    const int64_t w0 = idx0 + (int64_t)(tid >> 6) * (16 * gpw);
    // A wavefront without rows still takes part in the barriers below.
    const int ngroups = w0 >= n ? 0 : ((int)((n - w0 + 15) / 16) < gpw ? (int)((n - w0 + 15) / 16) : gpw);
    double* const tile = sT + (tid >> 6) * (16 * kTilePitch);
    const int cstride = (int)(lda * (int64_t)sizeof(T));
    const int istride = (int)(lds * (int64_t)sizeof(T));

    // Split planes from the tile: lane l writes row l/4 (of the group),
    // entries 8(l%4) + [0, 8) and 32 + 8(l%4) + [0, 8), 16-byte pieces.
    auto planes_from_tile = [&](int64_t gr0, int q0) {
        const int tr = lane >> 2, tc = 8 * (lane & 3);
        const int64_t rr = gr0 + tr;
        if (rr >= n) return;
        const int kk = (int)(c0 - j0) + tc;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            double v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = tile[tr * kTilePitch + 32 * half + tc + c];
            store_pieces8<NPC>(P.split, n, ss, q0, rr, kk + 32 * half, v);
        }
    };

    // ---- column panel: rows w0 + 16g + i16 of columns [c0, c0+64) ----------
    if (ngroups > 0) {
        const __amdgpu_buffer_rsrc_t rs =
            strip_rsrc(A + w0 + c0 * lda, (int64_t)L * lda * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rsi =
            strip_rsrc(S + w0 + c0 * lds, (int64_t)L * lds * (int64_t)sizeof(T));
        auto row_of = [&](int g) {
            const int64_t r = w0 + 16 * g + i16;
            return (int)((r < n ? r : n - 1) - w0) * (int)sizeof(T);  // tail rows re-read the last row
        };
        double nxt[16];
        {
            const int v = row_of(0) + q * istride;
#pragma unroll
            for (int k = 0; k < 16; ++k) nxt[k] = buf_load<T>(rsi, v, 4 * k * istride);
        }
        for (int g = 0; g < ngroups; ++g) {
            double cur[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) cur[k] = nxt[k];
            if (g + 1 < ngroups) {
                const int v = row_of(g + 1) + q * istride;
#pragma unroll
                for (int k = 0; k < 16; ++k) nxt[k] = buf_load<T>(rsi, v, 4 * k * istride);
            }
            d4 x[4];
            solve_group<kLP, true>(sP, sI, cur, x, q, i16);  // L21 = A21 U11^{-1}
            if (w0 + 16 * g + i16 < n) {
                const int v = row_of(g) + q * cstride;
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) buf_store<T>(x[b][e], rs, v, (16 * b + 4 * e) * cstride);
            }
            if constexpr (NPC > 0) {
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) tile[i16 * kTilePitch + 16 * b + 4 * e + q] = x[b][e];
                __builtin_amdgcn_wave_barrier();
                planes_from_tile(w0 + 16 * g, 0);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }

    // The inverses of L11's diagonal blocks replace those of U11^T once every
    // wavefront is done with the column panel.
    __syncthreads();
    if (tid < 64) invert_diag_blocks<true, kLP, false>(sP, sI, tid);  // L11: unit diagonal
    __syncthreads();

    // ---- row panel: columns w0 + 16g + i of rows [c0, c0+64) ---------------
    // Lane l moves column l/4, entries 16(l%4) + [0, 16), through the tile.
    // The next group's loads are issued before the current group's solve;
    // they are unconditional (columns past n re-read the last one, whose
    // results are not stored).
    if (ngroups > 0) {
        const int tcl = lane >> 2, tk = 16 * (lane & 3);
        auto load_cols = [&](int g, double (&dst)[16]) {
            const int64_t col = w0 + 16 * g + tcl;
            const T* src = S + c0 + (col < n ? col : n - 1) * lds + tk;
#pragma unroll
            for (int k = 0; k < 16; ++k) dst[k] = (double)src[k];
        };
        double nxt[16];
        load_cols(0, nxt);
        for (int g = 0; g < ngroups; ++g) {
            const int64_t col = w0 + 16 * g + tcl;
#pragma unroll
            for (int k = 0; k < 16; ++k) tile[tcl * kTilePitch + tk + k] = nxt[k];
            if (g + 1 < ngroups) load_cols(g + 1, nxt);
            __builtin_amdgcn_wave_barrier();
            double cur[16];
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) cur[4 * b + e] = tile[i16 * kTilePitch + 16 * b + 4 * e + q];
            __builtin_amdgcn_wave_barrier();
            d4 x[4];
            solve_group<kLP, false>(sP, sI, cur, x, q, i16);  // U12^T = A12^T L11^{-T}
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) tile[i16 * kTilePitch + 16 * b + 4 * e + q] = x[b][e];
            __builtin_amdgcn_wave_barrier();
            if (col < n) {
                T* dst = A + c0 + col * lda + tk;
#pragma unroll
                for (int k = 0; k < 16; ++k) dst[k] = (T)tile[tcl * kTilePitch + tk + k];
            }
            if constexpr (NPC > 0) planes_from_tile(w0 + 16 * g, NPC);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

template <typename T>
hipError_t launch_t(int pieces, const DevProb* probs, const GroupSpan* spans, int nspan, int64_t c0,
                    int64_t j0, int ss, hipStream_t s)
{
    // Sized for one workgroup per CU: sizing for two (half the row groups per
    // wavefront, twice the redundant chains) measured slower.
    GroupMap M;
    const int64_t total = leaf_map(spans, nspan, c0, L, 1, M);
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)total), block(kThreads);
    if (pieces == 3) hipLaunchKernelGGL((leaf_lu<T, 3>), grid, block, 0, s, probs, M, c0, j0, ss);
    else if (pieces == 2) hipLaunchKernelGGL((leaf_lu<T, 2>), grid, block, 0, s, probs, M, c0, j0, ss);
    else hipLaunchKernelGGL((leaf_lu<T, 0>), grid, block, 0, s, probs, M, c0, j0, ss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_lu(int dtype, int pieces, const DevProb* probs, const GroupSpan* spans,
                          int nspan, int64_t c0, int64_t j0, int ss, hipStream_t s)
{
    if (pieces != 0 && pieces != 2 && pieces != 3) return hipErrorInvalidValue;
    if (nspan > kMaxGroupsPerLaunch) return hipErrorInvalidValue;
    if (dtype == 0) return launch_t<double>(pieces, probs, spans, nspan, c0, j0, ss, s);
    return launch_t<float>(pieces, probs, spans, nspan, c0, j0, ss, s);
}

}  // namespace dpp
