// Diagonal-block kernels for complex kernels K (storage: interleaved real and
// imaginary FP64 parts, column-major), the complex forms of leaf_ldlh.hip and
// leaf_lu.hip (the paper's complex kernels: the domino-tiling examples of
// Sec. 1 and the dense complex LU experiment of Sec. 3).
//
// A conditional inclusion probability is real, so the decision at pivot j
// uses the real part d of the diagonal entry: keep j iff u_j < d, else the
// pivot loses 1 (Prop. 4); the returned pivot is the real d'. The Hermitian
// form keeps D real and subtracts l_i d' conj(l_k); the LU form scales the
// column by the whole complex pivot. Prop. 2 holds with unit-modulus
// similarities, so a complex similarity of a Hermitian kernel samples the
// same law.
//
// Layout: blocks of kLeafC = 32 complex columns. The chain runs on wavefront
// 0 with one complex block row per lane (lanes 0..31; 64 FP64 registers, as
// for a real row of 64). The panel solves then run on the real forms of the
// complex matrices (dpp_internal.h): a complex 32-column row is the 64 real
// values (Re, Im) of its entries, and a complex triangular solve X M = A is
// the real solve X' M'' = A' with M'' made of the 2x2 blocks [[a, b], [-b, a]]
// of the entries a + ib of M. Writing T for the transposed form, so that
// X' T^T = A', T has the 2x2 blocks R(z) = [[Re z, -Im z], [Im z, Re z]] of the
// entries of the complex lower triangular T_c = M^T, and R carries products
// and inverses of complex matrices to those of their real forms. Thus
// leaf_common.h's MFMA solve serves unchanged, with T in LDS as a 64 x 64 real
// matrix and the inverses of its 16 x 16 diagonal blocks, R of the inverses of
// T_c's 8 x 8 complex diagonal blocks.
#include "leaf_common.h"

namespace dpp {
namespace {

using namespace leaf;

constexpr int LC = kLeafC;  // complex columns per block (32)
constexpr int LR = 2 * LC;  // real columns of the block's real form (64)
static_assert(LR == L, "the real form of a complex block is one real block wide");

struct cd {
    double x, y;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * conj(b)
__device__ __forceinline__ cd cmulc(cd a, cd b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
__device__ __forceinline__ cd readlane_c(cd v, int lane) { return {readlane_d(v.x, lane), readlane_d(v.y, lane)}; }

// Loads one complex entry (16 bytes) of a column strip: voff per lane, soff
// per column (bytes).
__device__ __forceinline__ cd buf_load_c(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return {__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0)),
            __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff + 8, soff, 0))};
}

// Tt[t' * kBP + k'] = T[k'][t'] for the real form T = R(T_c) of a complex lower
// triangular 32 x 32 matrix T_c: lane k (< 32) holds row k of T_c in z[0..31]
// (z[t] = T_c[k][t] for t <= k) and writes real columns 2k, 2k + 1 of every
// real row pair; entries above the complex diagonal are written as zeros.
// (leaf_zldlh writes the same layout straight from its chain registers.)
__device__ __forceinline__ void store_real_form(double* Tt, const cd (&z)[LC], int k)
{
#pragma unroll
    for (int t = 0; t < LC; ++t) {
        const cd v = t <= k ? z[t] : cd{0.0, 0.0};
        // R(v) = [[Re, -Im], [Im, Re]] at rows 2k + s', columns 2t + s.
        Tt[(2 * t) * kBP + 2 * k] = v.x;
        Tt[(2 * t) * kBP + 2 * k + 1] = v.y;
        Tt[(2 * t + 1) * kBP + 2 * k] = -v.y;
        Tt[(2 * t + 1) * kBP + 2 * k + 1] = v.x;
    }
}

// Pieces of the real forms of 8 consecutive real k (4 complex columns) of
// one row x' = (Re, Im, ...) of a panel, for the split planes of the update:
// L' rows 2i and 2i + 1 from the row of L, W' row i from the row of W (or
// U^T). HERM: L'[2i] = x', L'[2i + 1] = (Im, -Re); LU: L'[2i] = (Re, -Im),
// L'[2i + 1] = (Im, Re).
template <bool HERM>
__device__ __forceinline__ void lprime_rows(const double (&x)[8], double (&r0)[8], double (&r1)[8])
{
#pragma unroll
    for (int c = 0; c < 8; c += 2) {
        r0[c] = x[c];
        r0[c + 1] = HERM ? x[c + 1] : -x[c + 1];
        r1[c] = x[c + 1];
        r1[c + 1] = HERM ? -x[c] : x[c];
    }
}

// ----------------------------------------------------------- Hermitian form
// Step 1 (wavefront 0): the unblocked sampler on the 32 x 32 complex block,
// lower triangle, row per lane: at pivot j, d = Re A_jj, keep iff u_j < d, d'
// = d or d - 1, and A_ik -= (A_ij / d') conj(A_kj) for j < k <= i, with the
// unscaled column broadcast through LDS.
// Step 2: W = A21 L11^{-H} (X M = A21 with M = L11^H, T_c = conj(L11), unit
// lower) on the matrix cores; L21 = W D1^{-1} to A; with NPC pieces the real
// forms L' and W' to the split planes.
template <int NPC>
__global__ __launch_bounds__(kThreads, 2) void leaf_zldlh(const DevProb* __restrict__ probs, GroupMap M,
                                                    int64_t c0, int64_t j0, int ss)
{
    int pi, bx, gpw;  // problem, workgroup within it, row groups per wavefront
    if (!group_slot(M, blockIdx.x, pi, bx, gpw)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    if (c0 >= P.npiv) return;
    const int bs = (int)((n - c0) < LC ? (n - c0) : LC);
    const int64_t row0 = c0 + bs + (int64_t)bx * (kWaves * 16 * gpw);
    if (bx > 0 && row0 >= n) return;

    cd* __restrict__ A = static_cast<cd*>(P.A);
    const int64_t lda = P.lda;
    int64_t lds;
    const cd* __restrict__ S = first_source<cd>(P, c0 == 0, lds);

    constexpr int kSmem = 2 * LC + LC + LR * kBP + 4 * kInvBlock + kWaves * 16 * kTilePitch;
    static_assert(kSmem * sizeof(double) <= kLdsPerTwo, "two workgroups per CU");
    __shared__ __attribute__((aligned(16))) double smem[kSmem];
    cd* const sB = reinterpret_cast<cd*>(smem);  // chain: the unscaled column of the pivot
    double* const sR = smem + 2 * LC;            // 1 / D1
    double* const sL = sR + LC;                  // real form of T_c = conj(L11), as Tt
    double* const sI = sL + LR * kBP;            // inverses of its 16 x 16 diagonal blocks
    double* const sT = sI + 4 * kInvBlock;       // per wavefront: one row group, row-major

    const int tid = threadIdx.x;
    if (tid < 64) {
        const int lane = tid;
        cd a[LC];
        {
            const int64_t base = c0 + c0 * lds;
            const __amdgpu_buffer_rsrc_t rb =
                strip_rsrc(S + base, ((n - 1) * lds + n - base) * (int64_t)sizeof(cd));
            const int cs = (int)(lds * (int64_t)sizeof(cd));
            const int lr = lane < LC ? lane : 0;
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const cd v = buf_load_c(rb, lr * (int)sizeof(cd), k * cs);
                a[k] = (lane < bs && k <= lane) ? v : cd{0.0, 0.0};
            }
        }
        const double ul = lane < bs ? P.u[c0 + lane] : 2.0;
        double mydp = 1.0;
        int mykeep = 0;
        int me = lane;
#pragma unroll
        for (int j = 0; j < LC; ++j) {
            asm volatile("" : "+v"(me));
            if (j < bs) {
                const double d = readlane_d(a[j].x, j);  // Re A[j][j]
                const double uj = readlane_d(ul, j);
                const bool keep = uj < d;
                const double dp = keep ? d : d - 1.0;   // Prop. 4 on rejection
                const cd c = a[j];                       // A[lane][j], unscaled
                const cd l = {c.x / dp, c.y / dp};
                if (lane < LC) sB[lane] = c;
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int kb = 0; kb < LC; kb += 16) {
                    cd v[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j) v[i] = sB[kb + i];
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j) {
                            const cd m = cmulc(l, v[i]);  // l_lane conj(A[k][j])
                            a[kb + i].x -= m.x;
                            a[kb + i].y -= m.y;
                        }
                }
                asm volatile("" ::: "memory");
                __builtin_amdgcn_wave_barrier();
                const bool isj = me == j;
                a[j] = isj ? cd{dp, 0.0} : (me > j ? l : c);
                mydp = isj ? dp : mydp;
                mykeep = isj ? (keep ? 1 : 0) : mykeep;
            }
        }
        if (lane < LC) {
            // Row `lane` of T_c = conj(L11) (unit diagonal; the identity past
            // a ragged block's end) in real form, straight from the registers.
#pragma unroll
            for (int t = 0; t < LC; ++t) {
                const cd v = (t < lane && lane < bs) ? cd{a[t].x, -a[t].y}
                                                     : (t == lane ? cd{1.0, 0.0} : cd{0.0, 0.0});
                sL[(2 * t) * kBP + 2 * lane] = v.x;
                sL[(2 * t) * kBP + 2 * lane + 1] = v.y;
                sL[(2 * t + 1) * kBP + 2 * lane] = -v.y;
                sL[(2 * t + 1) * kBP + 2 * lane + 1] = v.x;
            }
            sR[lane] = lane < bs ? 1.0 / mydp : 1.0;
            if (bx == 0 && lane < bs) {
                cd* blk = reinterpret_cast<cd*>(P.diag) + (c0 / LC) * (LC * LC);
#pragma unroll
                for (int k = 0; k < LC; ++k) blk[k * LC + lane] = a[k];
                P.mask[c0 + lane] = (uint8_t)mykeep;
                P.piv[c0 + lane] = mydp;
            }
        }
    }
    __syncthreads();
    if (row0 >= n) return;

    if (tid < 64) invert_diag_blocks<true>(sL, sI, tid);  // unit lower real form
    __syncthreads();

    const int lane = tid & 63;
    const int q = lane >> 4, i16 = lane & 15;
    const int64_t wrow0 = row0 + (int64_t)(tid >> 6) * (16 * gpw);
    if (wrow0 >= n) return;

    // Lane (q, i16) holds real column r' = 16b + 4e + q of its row: complex
    // column 8b + 2e + q/2, part q % 2.
    const __amdgpu_buffer_rsrc_t rs =
        strip_rsrc(A + wrow0 + c0 * lda, (int64_t)LC * lda * (int64_t)sizeof(cd));
    const __amdgpu_buffer_rsrc_t rsi =
        strip_rsrc(S + wrow0 + c0 * lds, (int64_t)LC * lds * (int64_t)sizeof(cd));
    const int cstride = (int)(lda * (int64_t)sizeof(cd));
    const int istride = (int)(lds * (int64_t)sizeof(cd));
    const int lane_a = (q & 1) * 8 + (q >> 1) * cstride;
    const int lane_s = (q & 1) * 8 + (q >> 1) * istride;
    const int ngroups = (int)((n - wrow0 + 15) / 16) < gpw ? (int)((n - wrow0 + 15) / 16) : gpw;

    auto row_of = [&](int g) {
        const int64_t r = wrow0 + 16 * g + i16;
        return (int)((r < n ? r : n - 1) - wrow0) * (int)sizeof(cd);
    };
    double nxt[16];
    {
        const int v = row_of(0) + lane_s;
#pragma unroll
        for (int k = 0; k < 16; ++k) nxt[k] = buf_load<double>(rsi, v, 2 * k * istride);
    }
    for (int g = 0; g < ngroups; ++g) {
        double cur[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) cur[k] = nxt[k];
        if (g + 1 < ngroups) {
            const int v = row_of(g + 1) + lane_s;
#pragma unroll
            for (int k = 0; k < 16; ++k) nxt[k] = buf_load<double>(rsi, v, 2 * k * istride);
        }
        d4 x[4];
        solve_group(sL, sI, cur, x, q, i16);  // W' = A21' T^{-T}
        const int64_t r = wrow0 + 16 * g + i16;
        if constexpr (NPC > 0) {
            double* const tile = sT + (tid >> 6) * (16 * kTilePitch);
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) tile[i16 * kTilePitch + 16 * b + 4 * e + q] = x[b][e];
            __builtin_amdgcn_wave_barrier();
            const int tr = lane >> 2, tc = 8 * (lane & 3);
            const int64_t rr = wrow0 + 16 * g + tr;
            if (rr < n) {
                const int kk = 2 * (int)(c0 - j0) + tc;
                uint16_t* const lp = split_plane(P.split, 2 * n, n, ss, NPC, 0);
                uint16_t* const wp = split_plane(P.split, 2 * n, n, ss, NPC, NPC);
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    double wv[8], lv[8], l0[8], l1[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int col = 32 * half + tc + c;
                        wv[c] = tile[tr * kTilePitch + col];
                        lv[c] = wv[c] * sR[col >> 1];
                    }
                    lprime_rows<true>(lv, l0, l1);
                    store_pieces8_at<NPC>(wp, plane_rows(n) * ss, ss, rr, kk + 32 * half, wv);
                    store_pieces8_at<NPC>(lp, plane_rows(2 * n) * ss, ss, 2 * rr, kk + 32 * half, l0);
                    store_pieces8_at<NPC>(lp, plane_rows(2 * n) * ss, ss, 2 * rr + 1, kk + 32 * half, l1);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (r < n) {
            const int v = row_of(g) + lane_a;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    buf_store<double>(x[b][e] * sR[8 * b + 2 * e + (q >> 1)], rs, v,
                                      (8 * b + 2 * e) * cstride);
        }
    }
}

// ------------------------------------------------------------------ LU form
// Step 1 (wavefront 0): the unblocked sampler on the 32 x 32 complex block,
// whole rows: pivot p = A_jj, d = Re p; keep iff u_j < d, else p <- p - 1;
// rows below scale by 1/p and take A_ik -= l_i A_jk, the row of U read from
// lane j's registers.
// Step 2: L21 = A21 U11^{-1} (T_c = U11^T, non-unit: complex inverses of its
// diagonal blocks) and U12 = L11^{-1} A12 (T_c = L11, unit), both on the
// matrix cores through the real forms; the row panel's columns pass through
// the wavefront's LDS tile (a complex column segment of 32 entries is the 64
// real values of its real form, contiguous in memory).
template <int NPC>
__global__ __launch_bounds__(kThreads, 1) void leaf_zlu(const DevProb* __restrict__ probs, GroupMap M,
                                                  int64_t c0, int64_t j0, int ss)
{
    int pi, bx, gpw;  // problem, workgroup within it, row groups per wavefront
    if (!group_slot(M, blockIdx.x, pi, bx, gpw)) return;
    const DevProb P = probs[pi];
    const int64_t n = P.n;
    if (c0 >= P.npiv) return;
    const int bs = (int)((n - c0) < LC ? (n - c0) : LC);
    const int64_t idx0 = c0 + bs + (int64_t)bx * (kWaves * 16 * gpw);
    if (bx > 0 && idx0 >= n) return;

    cd* __restrict__ A = static_cast<cd*>(P.A);
    const int64_t lda = P.lda;
    int64_t lds;
    const cd* __restrict__ S = first_source<cd>(P, c0 == 0, lds);

    __shared__ __attribute__((aligned(16))) double smem[kWaves * 16 * kTilePitch + LR * kBP + 4 * kInvBlock + 2 * LC * LC];
    double* const sT = smem;
    double* const sP = smem + kWaves * 16 * kTilePitch;  // real form of the current T_c, as Tt
    double* const sI = sP + LR * kBP;                    // inverses of its diagonal blocks
    cd* const sC = reinterpret_cast<cd*>(sI + 4 * kInvBlock);  // the factored block, by columns

    const int tid = threadIdx.x;
    if (tid < 64) {
        const int lane = tid;
        cd a[LC];
        {
            const int64_t base = c0 + c0 * lds;
            const __amdgpu_buffer_rsrc_t rb =
                strip_rsrc(S + base, ((n - 1) * lds + n - base) * (int64_t)sizeof(cd));
            const int cs = (int)(lds * (int64_t)sizeof(cd));
            const int lr = lane < LC ? lane : 0;
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const cd v = buf_load_c(rb, lr * (int)sizeof(cd), k * cs);
                a[k] = (lane < bs && k < bs) ? v : cd{0.0, 0.0};
            }
#pragma unroll
            for (int k = 0; k < LC; ++k) asm volatile("" : "+v"(a[k].x), "+v"(a[k].y));
        }
        const double ul = lane < bs ? P.u[c0 + lane] : 2.0;
        double mydp = 1.0;
        int mykeep = 0;
        int me = lane;
#pragma unroll
        for (int j = 0; j < LC; ++j) {
            asm volatile("" : "+v"(me));
            if (j < bs) {
                const cd p = readlane_c(a[j], j);
                const double uj = readlane_d(ul, j);
                const bool keep = uj < p.x;               // d = Re p
                const cd pp = keep ? p : cd{p.x - 1.0, p.y};  // Prop. 4 on rejection
                const double dp = pp.x;
                const double den = pp.x * pp.x + pp.y * pp.y;
                const cd inv = {pp.x / den, -pp.y / den};
                const bool isj = me == j, below = me > j;
                const cd l = below ? cmul(a[j], inv) : cd{0.0, 0.0};
#pragma unroll
                for (int kb = 0; kb < LC; kb += 16) {
                    cd v[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j) v[i] = readlane_c(a[kb + i], j);  // U[j][k]
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (kb + i > j) {
                            const cd m = cmul(l, v[i]);
                            a[kb + i].x -= m.x;
                            a[kb + i].y -= m.y;
                        }
                }
                asm volatile("" ::: "memory");
                __builtin_amdgcn_wave_barrier();
                a[j] = isj ? pp : (below ? l : a[j]);
                mydp = isj ? dp : mydp;
                mykeep = isj ? (keep ? 1 : 0) : mykeep;
            }
        }
        if (lane < LC) {
            // sC[t * LC + k] = block entry (k, t): L11 below the diagonal, U11
            // on and above it; a ragged block is padded with the identity.
#pragma unroll
            for (int t = 0; t < LC; ++t)
                sC[t * LC + lane] = lane < bs ? a[t] : (t == lane ? cd{1.0, 0.0} : cd{0.0, 0.0});
            if (bx == 0 && lane < bs) {
                cd* blk = reinterpret_cast<cd*>(P.diag) + (c0 / LC) * (LC * LC);
#pragma unroll
                for (int k = 0; k < LC; ++k) blk[k * LC + lane] = a[k];
                P.mask[c0 + lane] = (uint8_t)mykeep;
                P.piv[c0 + lane] = mydp;
            }
        }
    }
    __syncthreads();
    if (idx0 >= n) return;

    // Column panel: T_c = U11^T, T_c[k][t] = U11[t][k] = block entry (t, k).
    if (tid < LC) {
        const int k = tid;
        cd z[LC];
#pragma unroll
        for (int t = 0; t < LC; ++t) z[t] = t <= k ? sC[k * LC + t] : cd{0.0, 0.0};
        store_real_form(sP, z, k);
    }
    __syncthreads();
    {
        // Inverses of R(T_c)'s 16 x 16 diagonal blocks: forward substitution
        // on T_c's 8 x 8 diagonal blocks in complex arithmetic, one column per
        // lane (block lane / 8, column lane % 8), T_c[k][t] = sC[k * LC + t];
        // then sI[b * kInvBlock + i * kInvPitch + c] = R((T_c,bb)^{-1}) (R
        // carries inverses).
        const int lane = tid;
        if (lane < LC) {
            const int b = lane >> 3, c = lane & 7;
            cd y[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                cd acc = {k == c ? 1.0 : 0.0, 0.0};
#pragma unroll
                for (int t = 0; t < k; ++t) {
                    const cd m = cmul(sC[(8 * b + k) * LC + 8 * b + t], y[t]);
                    acc.x -= m.x;
                    acc.y -= m.y;
                }
                const cd dg = sC[(8 * b + k) * LC + 8 * b + k];
                const double den = dg.x * dg.x + dg.y * dg.y;
                y[k] = cmul(acc, cd{dg.x / den, -dg.y / den});
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                sI[b * kInvBlock + (2 * k) * kInvPitch + 2 * c] = y[k].x;
                sI[b * kInvBlock + (2 * k) * kInvPitch + 2 * c + 1] = -y[k].y;
                sI[b * kInvBlock + (2 * k + 1) * kInvPitch + 2 * c] = y[k].y;
                sI[b * kInvBlock + (2 * k + 1) * kInvPitch + 2 * c + 1] = y[k].x;
            }
        }
    }
    __syncthreads();

    const int lane = tid & 63;
    const int q = lane >> 4, i16 = lane & 15;
    const int64_t w0 = idx0 + (int64_t)(tid >> 6) * (16 * gpw);
    const int ngroups = w0 >= n ? 0 : ((int)((n - w0 + 15) / 16) < gpw ? (int)((n - w0 + 15) / 16) : gpw);
    double* const tile = sT + (tid >> 6) * (16 * kTilePitch);
    const int cstride = (int)(lda * (int64_t)sizeof(cd));
    const int istride = (int)(lds * (int64_t)sizeof(cd));

    // Planes from the tile (rows of the real form x' of a panel row): with
    // lprime (column panel), L' rows 2r and 2r + 1; else (row panel) W' row r.
    auto planes_from_tile = [&](int64_t gr0, bool lprime) {
        const int tr = lane >> 2, tc = 8 * (lane & 3);
        const int64_t rr = gr0 + tr;
        if (rr >= n) return;
        const int kk = 2 * (int)(c0 - j0) + tc;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            double v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = tile[tr * kTilePitch + 32 * half + tc + c];
            if (lprime) {
                double l0[8], l1[8];
                lprime_rows<false>(v, l0, l1);
                uint16_t* const lp = split_plane(P.split, 2 * n, n, ss, NPC, 0);
                store_pieces8_at<NPC>(lp, plane_rows(2 * n) * ss, ss, 2 * rr, kk + 32 * half, l0);
                store_pieces8_at<NPC>(lp, plane_rows(2 * n) * ss, ss, 2 * rr + 1, kk + 32 * half, l1);
            } else {
                uint16_t* const wp = split_plane(P.split, 2 * n, n, ss, NPC, NPC);
                store_pieces8_at<NPC>(wp, plane_rows(n) * ss, ss, rr, kk + 32 * half, v);
            }
        }
    };

    // ---- column panel: rows w0 + 16g + i16, real columns of [c0, c0 + 32)
    if (ngroups > 0) {
        const __amdgpu_buffer_rsrc_t rs =
            strip_rsrc(A + w0 + c0 * lda, (int64_t)LC * lda * (int64_t)sizeof(cd));
        const __amdgpu_buffer_rsrc_t rsi =
            strip_rsrc(S + w0 + c0 * lds, (int64_t)LC * lds * (int64_t)sizeof(cd));
        const int lane_a = (q & 1) * 8 + (q >> 1) * cstride;
        const int lane_s = (q & 1) * 8 + (q >> 1) * istride;
        auto row_of = [&](int g) {
            const int64_t r = w0 + 16 * g + i16;
            return (int)((r < n ? r : n - 1) - w0) * (int)sizeof(cd);
        };
        double nxt[16];
        {
            const int v = row_of(0) + lane_s;
#pragma unroll
            for (int k = 0; k < 16; ++k) nxt[k] = buf_load<double>(rsi, v, 2 * k * istride);
        }
        for (int g = 0; g < ngroups; ++g) {
            double cur[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) cur[k] = nxt[k];
            if (g + 1 < ngroups) {
                const int v = row_of(g + 1) + lane_s;
#pragma unroll
                for (int k = 0; k < 16; ++k) nxt[k] = buf_load<double>(rsi, v, 2 * k * istride);
            }
            d4 x[4];
            solve_group(sP, sI, cur, x, q, i16);  // L21' = A21' T^{-T}
            if (w0 + 16 * g + i16 < n) {
                const int v = row_of(g) + lane_a;
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        buf_store<double>(x[b][e], rs, v, (8 * b + 2 * e) * cstride);
            }
            if constexpr (NPC > 0) {
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) tile[i16 * kTilePitch + 16 * b + 4 * e + q] = x[b][e];
                __builtin_amdgcn_wave_barrier();
                planes_from_tile(w0 + 16 * g, true);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }

    // Row panel: T_c = L11 (unit lower), replacing the column panel's T once
    // every wavefront is done with it.
    __syncthreads();
    if (tid < LC) {
        const int k = tid;
        cd z[LC];
#pragma unroll
        for (int t = 0; t < LC; ++t)
            z[t] = t < k ? sC[t * LC + k] : (t == k ? cd{1.0, 0.0} : cd{0.0, 0.0});
        store_real_form(sP, z, k);
    }
    __syncthreads();
    if (tid < 64) invert_diag_blocks<true>(sP, sI, tid);
    __syncthreads();

    // ---- row panel: columns w0 + 16g + i of rows [c0, c0 + 32); lane l moves
    // column l/4, real entries 16(l%4) + [0, 16), through the tile.
    if (ngroups > 0) {
        const int tcl = lane >> 2, tk = 16 * (lane & 3);
        auto load_cols = [&](int g, double (&dst)[16]) {
            const int64_t col = w0 + 16 * g + tcl;
            const double* src = reinterpret_cast<const double*>(S + c0 + (col < n ? col : n - 1) * lds) + tk;
#pragma unroll
            for (int k = 0; k < 16; ++k) dst[k] = src[k];
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
            solve_group(sP, sI, cur, x, q, i16);  // U12^T' = A12^T' T^{-T}
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) tile[i16 * kTilePitch + 16 * b + 4 * e + q] = x[b][e];
            __builtin_amdgcn_wave_barrier();
            if (col < n) {
                double* dst = reinterpret_cast<double*>(A + c0 + col * lda) + tk;
#pragma unroll
                for (int k = 0; k < 16; ++k) dst[k] = tile[tcl * kTilePitch + tk + k];
            }
            if constexpr (NPC > 0) planes_from_tile(w0 + 16 * g, false);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

template <int NPC>
hipError_t launch_z(bool herm, const DevProb* probs, const GroupSpan* spans, int nspan, int64_t c0,
                    int64_t j0, int ss, hipStream_t s)
{
    GroupMap M;
    const int64_t total = leaf_map(spans, nspan, c0, LC, herm ? 2 : 1, M);
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)total), block(kThreads);
    if (herm) hipLaunchKernelGGL((leaf_zldlh<NPC>), grid, block, 0, s, probs, M, c0, j0, ss);
    else hipLaunchKernelGGL((leaf_zlu<NPC>), grid, block, 0, s, probs, M, c0, j0, ss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_complex(bool herm, int pieces, const DevProb* probs, const GroupSpan* spans,
                               int nspan, int64_t c0, int64_t j0, int ss, hipStream_t s)
{
    if (nspan > kMaxGroupsPerLaunch) return hipErrorInvalidValue;
    if (pieces == 3) return launch_z<3>(herm, probs, spans, nspan, c0, j0, ss, s);
    if (pieces == 2) return launch_z<2>(herm, probs, spans, nspan, c0, j0, ss, s);
    if (pieces == 0) return launch_z<0>(herm, probs, spans, nspan, c0, j0, ss, s);
    return hipErrorInvalidValue;
}

}  // namespace dpp
