// Diagonal-block kernel, Hermitian (LDL^H) form; see leaf_common.h for the
// chain. The panel solve below the block runs on the matrix cores.
#include "leaf_common.h"

namespace dpp {
namespace {

using namespace leaf;


// ------------------------------------------------------------------- LDL^H
// Step 1 (wavefront 0, every workgroup): the unblocked sampler on the 64x64
// diagonal block, one block row per lane; see leaf_common.h.
//
// Step 2: the panel rows below the block. With W = A21 L11^{-T} (the unscaled
// columns, W = L21 D1) and the 64 columns cut into four 16-column blocks,
//   W_b = (A_b - sum_{c<b} W_c L_bc^T) L_bb^{-T},    b = 0..3,
// or, transposed, W_b^T = L_bb^{-1} (A_b^T - sum_{c<b} L_bc W_c^T). Each
// product has a 16x16 block of L11 (or the inverse of a diagonal block) on the
// left and the 16 rows of a row group on the right. v_mfma_f64_16x16x4f64
// leaves output element e of lane l at row l/16 + 4e, column l%16, and takes
// its right-hand operand for 4-deep slab s as row l/16, column l%16 of that
// slab -- so output element e = s of one product is, lane for lane, slab s of
// the right-hand operand of the next, and a row group never leaves registers.
// The four inverses L_bb^{-1} (unit lower triangular) are formed once per
// workgroup by forward substitution, one column per lane.
// Then L21 = W D1^{-1}; A receives L21, the split planes W and L21 (F16:
// their FP16 form, dpp_internal.h: each column balanced by rho_k, each row's
// 64 values of this block normalised by 2^e, the factor 2^-e kept per row).
template <typename T, int NPC, bool F16>
__global__ __launch_bounds__(kThreads, 2) void leaf_ldlh(const DevProb* __restrict__ probs, GroupMap M,
                                               int64_t c0, int64_t j0, int ss)
{
    int pi, bx, gpw;  // problem, workgroup within it, row groups per wavefront
    if (!group_slot(M, blockIdx.x, pi, bx, gpw)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    if (c0 >= P.npiv) return;  // npiv <= n: only the first npiv indices are decided
    const int bs = (int)((n - c0) < L ? (n - c0) : L);
    const int64_t row0 = c0 + bs + (int64_t)bx * (kWaves * 16 * gpw);
    if (bx > 0 && row0 >= n) return;

    T* __restrict__ A = static_cast<T*>(P.A);
    const int64_t lda = P.lda;
    int64_t lds;  // leading dimension of the source the loads read (K at column 0)
    const T* __restrict__ S = first_source<T>(P, c0 == 0, lds);

    // One LDS array carved by hand so that sB sits at address 0: the chain's
    // 64-entry broadcast reads then all use one base register and immediate
    // offsets.
    constexpr int kSmem = 2 * L + L * kBP + 4 * kInvBlock + kWaves * 16 * kTilePitch;
    static_assert(kSmem * sizeof(double) <= kLdsPerTwo, "two workgroups per CU");
    __shared__ __attribute__((aligned(16))) double smem[kSmem];
    double* const sB = smem;               // chain: broadcast columns of the current two pivots
    double* const sR = smem + L;           // 1 / D1 (written after the chain, over sB's second half)
    int* const sRho = reinterpret_cast<int*>(smem);  // F16: column balance exponents (after the chain, over sB)
    double* const sL = smem + 2 * L;       // sL[t*kBP + k] = L11[k][t] for k > t, zero elsewhere
    double* const sI = sL + L * kBP;       // the inverses of L11's 16 x 16 diagonal blocks
    double* const sT = sI + 4 * kInvBlock;  // per wavefront: W of one row group, row-major

    const int tid = threadIdx.x;
    if (tid < L) {
        const int lane = tid;
        // Row `lane` of the block, lower part; the rest starts at 0 and only
        // ever receives finite garbage that no decision reads.
        double a[L];
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
                a[k] = (lane < bs && k <= lane) ? v : 0.0;
            }
        }
        const double ul = lane < bs ? P.u[c0 + lane] : 2.0;
        double mydp = 1.0;
        int mykeep = 0;
        int me = lane;

        // Two pivots per step: pivot j is decided, column j + 1 alone takes
        // its rank-1 update from pivot j, pivot j + 1 is decided, and the
        // columns after it take both rank-1 updates in the same order as two
        // one-pivot steps would (so every value is the same, bit for bit). The
        // two broadcast columns sit side by side in LDS, one 16-byte read per
        // entry. Past a ragged block's end (j + 1 >= bs) column j + 1 is all
        // zeros and u = 2 there, so that pivot rejects, l1 = -0 and its update
        // adds zeros.
        double2* const sB2 = reinterpret_cast<double2*>(sB);
#pragma unroll
        for (int j = 0; j < L; j += 2) {
            // Keeps the compiler from hoisting the per-step lane masks
            // (lane == j, lane > j) out of the unrolled loop, where they
            // would occupy 128 scalar registers and spill.
            asm volatile("" : "+v"(me));
            if (j < bs) {
                const double d = readlane_d(a[j], j);   // A[j][j]
                const double uj = readlane_d(ul, j);
                const bool keep = uj < d;                // Bernoulli(d) with stream u_j
                const double dp = keep ? d : d - 1.0;   // Prop. 4 on rejection
                const double c = a[j];                   // A[lane][j], unscaled
                const double l = c / dp;
                a[j + 1] -= l * readlane_d(c, j + 1);    // A[lane][j+1] -= l_lane * A[j+1][j]
                const double d1 = readlane_d(a[j + 1], j + 1);
                const double u1 = readlane_d(ul, j + 1);
                const bool keep1 = u1 < d1;
                const double dp1 = keep1 ? d1 : d1 - 1.0;
                const double c1 = a[j + 1];
                const double l1 = c1 / dp1;
                sB2[lane] = make_double2(c, c1);
                __builtin_amdgcn_wave_barrier();
                // Broadcast reads in batches of 16, all issued before their
                // FMAs, so up to 15 are in flight (left to itself the
                // compiler keeps two or three, and the chain waits on each).
#pragma unroll
                for (int kb = 0; kb < L; kb += 16) {
                    double2 v[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j + 1) v[i] = sB2[kb + i];  // A[k][j], A[k][j+1]
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j + 1) {
                            a[kb + i] -= l * v[i].x;
                            a[kb + i] -= l1 * v[i].y;
                        }
                }
                // No LDS access moves across this point: hoisting the next
                // step's reads would hold them in registers and spill.
                asm volatile("" ::: "memory");
                __builtin_amdgcn_wave_barrier();
                const bool isj = me == j;
                a[j] = isj ? dp : (me > j ? l : c);
                mydp = isj ? dp : mydp;
                mykeep = isj ? (keep ? 1 : 0) : mykeep;
                const bool isj1 = me == j + 1;
                a[j + 1] = isj1 ? dp1 : (me > j + 1 ? l1 : c1);
                mydp = isj1 ? dp1 : mydp;
                mykeep = isj1 ? (keep1 ? 1 : 0) : mykeep;
            }
        }

#pragma unroll
        for (int k = 0; k < L; ++k) sL[k * kBP + lane] = (k < lane && lane < bs) ? a[k] : 0.0;
        sR[lane] = (lane < bs) ? 1.0 / mydp : 1.0;
        if constexpr (F16) sRho[lane] = (lane < bs) ? f16_rho_exp(mydp) : 0;

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
    // Rows below a block exist only when the block is a full 64 wide (a
    // ragged block is the last one), so bs == L from here on.
    if (row0 >= n) return;

    if (tid < 64) invert_diag_blocks<true>(sL, sI, tid);  // L_bb^{-1}
    __syncthreads();

    const int lane = tid & 63;
    const int q = lane >> 4, i16 = lane & 15;
    const int64_t wrow0 = row0 + (int64_t)(tid >> 6) * (16 * gpw);
    if (wrow0 >= n) return;

    // Strip = columns [c0, c0+64) from row wrow0 on, read from S and written
    // to A; lane (q, i16) of group g reads row wrow0 + 16g + i16 of columns
    // q + 4e + 16b.
    const __amdgpu_buffer_rsrc_t rs =
        strip_rsrc(A + wrow0 + c0 * lda, (int64_t)L * lda * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rsi =
        strip_rsrc(S + wrow0 + c0 * lds, (int64_t)L * lds * (int64_t)sizeof(T));
    const int cstride = (int)(lda * (int64_t)sizeof(T));
    const int istride = (int)(lds * (int64_t)sizeof(T));
    const int ngroups = (int)((n - wrow0 + 15) / 16) < gpw ? (int)((n - wrow0 + 15) / 16) : gpw;

    auto row_of = [&](int g) {
        const int64_t r = wrow0 + 16 * g + i16;
        return (int)((r < n ? r : n - 1) - wrow0) * (int)sizeof(T);  // tail rows re-read the last row
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
        solve_group(sL, sI, cur, x, q, i16);  // W = A21 L11^{-T}
        // x[b][e] = W[row][16b + 4e + q], row = wrow0 + 16g + i16.
        const int64_t r = wrow0 + 16 * g + i16;
        if constexpr (NPC > 0) {
            // The split planes are row-major: stage W through LDS so that each
            // lane writes 16-byte pieces of one row (lane l: row l/4, columns
            // 8(l%4) + [0, 8) and 32 + 8(l%4) + [0, 8)).
            double* const tile = sT + (tid >> 6) * (16 * kTilePitch);
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) tile[i16 * kTilePitch + 16 * b + 4 * e + q] = x[b][e];
            __builtin_amdgcn_wave_barrier();
            const int tr = lane >> 2, tc = 8 * (lane & 3);
            const int64_t rr = wrow0 + 16 * g + tr;
            const int kk = (int)(c0 - j0) + tc;
            if constexpr (F16) {
                // Row rr's 64 values sit in lanes 4 tr .. 4 tr + 3 (16 each):
                // balance, then the block maximum of each side over those lanes.
                double wv[2][8], lv[2][8];
                double mw = 0.0, ml = 0.0;
#pragma unroll
                for (int half = 0; half < 2; ++half)
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int col = 32 * half + tc + c;
                        const double w = tile[tr * kTilePitch + col];
                        const int h = sRho[col];
                        wv[half][c] = __builtin_ldexp(w, -h);            // W / rho
                        lv[half][c] = __builtin_ldexp(w * sR[col], h);   // L rho
                        mw = __builtin_fmax(mw, __builtin_fabs(wv[half][c]));
                        ml = __builtin_fmax(ml, __builtin_fabs(lv[half][c]));
                    }
                mw = __builtin_fmax(mw, __shfl_xor(mw, 1));
                mw = __builtin_fmax(mw, __shfl_xor(mw, 2));
                ml = __builtin_fmax(ml, __shfl_xor(ml, 1));
                ml = __builtin_fmax(ml, __shfl_xor(ml, 2));
                const int ew = f16_row_exp(mw), el = f16_row_exp(ml);
                if (rr < n) {
                    const int64_t pst = plane_rows(n) * (int64_t)ss;
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            wv[half][c] = __builtin_ldexp(wv[half][c], ew);
                            lv[half][c] = __builtin_ldexp(lv[half][c], el);
                        }
                        store_f16_pieces8_at(split_plane(P.split, n, ss, 2), pst, ss, rr, kk + 32 * half,
                                             wv[half]);
                        store_f16_pieces8_at(split_plane(P.split, n, ss, 0), pst, ss, rr, kk + 32 * half,
                                             lv[half]);
                    }
                    if ((lane & 3) == 0) {
                        const int blk = (int)((c0 - j0) / L);
                        P.scale[scale_off(n, ss, 0, blk, rr)] = (float)__builtin_ldexp(1.0, -el);
                        P.scale[scale_off(n, ss, 1, blk, rr)] = (float)__builtin_ldexp(1.0, -ew);
                    }
                }
            } else if (rr < n) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    double wv[8], lv[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int col = 32 * half + tc + c;
                        wv[c] = tile[tr * kTilePitch + col];
                        lv[c] = wv[c] * sR[col];
                    }
                    store_pieces8<NPC>(P.split, n, ss, NPC, rr, kk + 32 * half, wv);  // W = L D
                    store_pieces8<NPC>(P.split, n, ss, 0, rr, kk + 32 * half, lv);    // L
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (r < n) {
            const int v = row_of(g) + q * cstride;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    buf_store<T>(x[b][e] * sR[16 * b + 4 * e + q], rs, v, (16 * b + 4 * e) * cstride);
        }
    }
}

template <typename T>
hipError_t launch_t(int pieces, bool f16, const DevProb* probs, const GroupSpan* spans, int nspan,
                    int64_t c0, int64_t j0, int ss, hipStream_t s)
{
    GroupMap M;
    const int64_t total = leaf_map(spans, nspan, c0, L, 2, M);  // two workgroups per CU
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)total), block(kThreads);
    if (f16) hipLaunchKernelGGL((leaf_ldlh<T, 2, true>), grid, block, 0, s, probs, M, c0, j0, ss);
    else if (pieces == 3) hipLaunchKernelGGL((leaf_ldlh<T, 3, false>), grid, block, 0, s, probs, M, c0, j0, ss);
    else if (pieces == 2) hipLaunchKernelGGL((leaf_ldlh<T, 2, false>), grid, block, 0, s, probs, M, c0, j0, ss);
    else hipLaunchKernelGGL((leaf_ldlh<T, 0, false>), grid, block, 0, s, probs, M, c0, j0, ss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_ldlh(int dtype, int pieces, bool f16, const DevProb* probs,
                            const GroupSpan* spans, int nspan, int64_t c0, int64_t j0, int ss,
                            hipStream_t s)
{
    if ((pieces != 0 && pieces != 2 && pieces != 3) || (f16 && pieces != 2)) return hipErrorInvalidValue;
    if (nspan > kMaxGroupsPerLaunch) return hipErrorInvalidValue;
    if (dtype == 0) return launch_t<double>(pieces, f16, probs, spans, nspan, c0, j0, ss, s);
    return launch_t<float>(pieces, f16, probs, spans, nspan, c0, j0, ss, s);
}

}  // namespace dpp
