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
//      block (and, for LU, of the row panel to its right) on the matrix
//      cores, in groups of 16 rows (columns), with the factored block and the
//      inverses of its 16x16 diagonal blocks in LDS (solve_group below).
// Every workgroup of a launch makes the same decisions from the same data
// (the chain is deterministic), so the panel solves need no second launch;
// workgroup 0 alone writes the block, the mask and the pivots.
// All arithmetic is FP64 whatever the storage type T.
#pragma once
#include "dpp_internal.h"

namespace dpp {
namespace leaf {

constexpr int L = kLeaf;
// Panel solves: 4 wavefronts per workgroup, each `gpw` groups of 16 panel rows
// (or columns); a staged 16 x 64 tile per wavefront.
constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;
// LDS pitches (in doubles), chosen so that a wavefront's FP64 accesses spread
// over the 64 four-byte banks (32 doubles wide) as evenly as 64 lanes allow,
// two per double-wide bank, or three where two patterns share a layout:
//   a factored 64 x 64 block, read by solve_group as Tt[(16c + 4s + q) * kBP
//     + 16b + i16]: lane (q, i16) at q * kBP + i16, two-way for kBP = 72;
//   the inverses of its 16 x 16 diagonal blocks, read as Inv[i16 * kInvPitch
//     + 4s + q]: two-way for kInvPitch = 18;
//   a staged 16 x 64 tile, written at i16 * kTilePitch + q (three-way) and
//     read at tr * kTilePitch + 8 m (two-way) for kTilePitch = 67.
constexpr int kBP = 72;
constexpr int kInvPitch = 18;
constexpr int kInvBlock = 16 * kInvPitch;  // doubles per inverse block; four per block
constexpr int kTilePitch = 67;
// Two workgroups per CU need at most half of the 160 KiB of LDS each.
constexpr int kLdsPerTwo = 80 * 1024;

// Every workgroup of a diagonal-block launch first runs the 64-step chain,
// then its share of the panel, one group of 16 rows after the other on each
// wavefront. With W workgroups per problem and `per_cu` resident per compute
// unit, the launch runs in rounds of cus * per_cu workgroups; each round costs
// about one chain plus the groups of one wavefront. The groups per wavefront
// (1 .. kMaxGroups) are chosen to minimize rounds * (chain + groups), with the
// chain and the first group (load latency included) at about 34 us and each
// further group at about 6 us (measured at n = 16384). A big batch of small
// problems thus gets one workgroup per problem instead of several that would
// each repeat the chain in later rounds. Returns the groups per wavefront;
// *gx receives the grid width (workgroups per problem).
constexpr int kMaxGroups = 16;
inline int groups_per_wave(int64_t rows, int nprob, int per_cu, int* gx)
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    if (rows <= 0) {
        *gx = 1;
        return 1;
    }
    const int64_t resident = (int64_t)cus * per_cu;
    int best = 1;
    int64_t best_cost = INT64_MAX;
    for (int g = 1; g <= kMaxGroups; ++g) {
        const int64_t w = (rows + kWaves * 16 * g - 1) / (kWaves * 16 * g);
        const int64_t rounds = (w * nprob + resident - 1) / resident;
        const int64_t cost = rounds * (34 + 6 * (int64_t)g);
        if (cost < best_cost) {
            best_cost = cost;
            best = g;
        }
    }
    *gx = (int)((rows + kWaves * 16 * best - 1) / (kWaves * 16 * best));
    return best;
}

// Group map of one diagonal-block launch at column c0 (block width bw): for
// each size group that has the block, its workgroups per problem and row
// groups per wavefront (groups_per_wave, with the rounds counted over every
// problem of the launch: the groups share the GPU, and each extra workgroup
// of a problem repeats its chain). Only the launch geometry depends on the
// batch; every workgroup of a problem computes the same chain and the rows
// are independent, so results do not. Returns the launch's workgroups (0: no
// group has the block).
inline int64_t leaf_map(const GroupSpan* spans, int nspan, int64_t c0, int bw, int per_cu,
                        GroupMap& M)
{
    M.ng = 0;
    M.off[0] = 0;
    int64_t off = 0;
    int64_t active = 0;  // problems of the launch that have this block
    for (int i = 0; i < nspan && i < kMaxGroupsPerLaunch; ++i)
        if (c0 < spans[i].nmax) active += spans[i].count;
    const int nprob = (int)(active < (int64_t)1 << 30 ? active : (int64_t)1 << 30);
    for (int i = 0; i < nspan && M.ng < kMaxGroupsPerLaunch; ++i) {
        const GroupSpan& g = spans[i];
        if (c0 >= g.nmax) continue;
        int gx = 1;
        const int gpw = groups_per_wave(g.nmax - c0 - bw, nprob, per_cu, &gx);
        M.p0[M.ng] = (int)g.p0;
        M.wpp[M.ng] = gx;
        M.aux[M.ng] = gpw;
        off += (int64_t)gx * g.count;
        M.off[++M.ng] = (int)off;
    }
    return off;
}

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

// BF16 pieces of one value: p_0 = bf16(x), p_i = bf16(x - p_0 - ... -
// p_{i-1}) (each remainder exact in FP64, rounded through FP32), so that the
// NPC pieces carry about 8 NPC significant bits of x.
template <int NPC>
__device__ __forceinline__ void split_pieces(double x, uint32_t (&p)[NPC])
{
    double r = x;
#pragma unroll
    for (int i = 0; i < NPC; ++i) {
        p[i] = bf16_bits((float)r);
        if (i + 1 < NPC) r -= (double)bf16_value(p[i]);
    }
}

// Writes the NPC pieces of 8 consecutive panel values v[0..7] of row r,
// columns kk .. kk+7 of the outer panel (kk a multiple of 8): piece i goes to
// the plane at first + i * stride (elements), one 16-byte store per plane.
template <int NPC>
__device__ __forceinline__ void store_pieces8_at(uint16_t* first, int64_t stride, int ss, int64_t r,
                                                 int kk, const double (&v)[8])
{
    if constexpr (NPC > 0) {
        uint32_t w[NPC][4];
#pragma unroll
        for (int p2 = 0; p2 < 4; ++p2) {
            uint32_t a[NPC], b[NPC];
            split_pieces<NPC>(v[2 * p2], a);
            split_pieces<NPC>(v[2 * p2 + 1], b);
#pragma unroll
            for (int i = 0; i < NPC; ++i) w[i][p2] = a[i] | (b[i] << 16);
        }
        const int64_t o = plane_off(r, kk, ss);
#pragma unroll
        for (int i = 0; i < NPC; ++i)
            *reinterpret_cast<uint4*>(first + i * stride + o) =
                make_uint4(w[i][0], w[i][1], w[i][2], w[i][3]);
    }
}
// Real kernels: the planes q0 .. q0 + NPC - 1 of a problem of size n.
template <int NPC>
__device__ __forceinline__ void store_pieces8(uint16_t* base, int64_t n, int ss, int q0, int64_t r,
                                              int kk, const double (&v)[8])
{
    store_pieces8_at<NPC>(split_plane(base, n, ss, q0), plane_rows(n) * ss, ss, r, kk, v);
}

// FP16 form: hi = fp16(y), lo = fp16(y - hi) of 8 consecutive (already
// scaled) values y[0..7] of row r, columns kk .. kk+7 of the outer panel;
// piece i goes to the plane at first + i * stride, one 16-byte store each.
// Both conversions go through FP32 (the hardware conversions; a direct FP64
// to FP16 conversion is a long software sequence): hi may then differ from
// the correctly rounded fp16(y) by one unit in rare cases, which the exact
// remainder y - hi absorbs, so the pair still carries about 22 bits of y.
__device__ __forceinline__ void store_f16_pieces8_at(uint16_t* first, int64_t stride, int ss,
                                                     int64_t r, int kk, const double (&y)[8])
{
    uint32_t w[2][4];
#pragma unroll
    for (int p2 = 0; p2 < 4; ++p2) {
        uint32_t h[2], l[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const double v = y[2 * p2 + t];
            // The empty asm keeps the code generator from merging the two
            // conversions back into one FP64 -> FP16 rounding.
            float vf = (float)v;
            asm volatile("" : "+v"(vf));
            const _Float16 hi = (_Float16)vf;
            float rf = (float)(v - (double)hi);
            asm volatile("" : "+v"(rf));
            const _Float16 lo = (_Float16)rf;
            h[t] = __builtin_bit_cast(uint16_t, hi);
            l[t] = __builtin_bit_cast(uint16_t, lo);
        }
        w[0][p2] = h[0] | (h[1] << 16);
        w[1][p2] = l[0] | (l[1] << 16);
    }
    const int64_t o = plane_off(r, kk, ss);
#pragma unroll
    for (int i = 0; i < 2; ++i)
        *reinterpret_cast<uint4*>(first + i * stride + o) = make_uint4(w[i][0], w[i][1], w[i][2], w[i][3]);
}

// The FP16 form's column balance rho = 2^h, h = floor(x / 2) for |d'| in
// [2^(x-1), 2^x) (about sqrt|d'|; h = 0 for d' = 0), so that l rho =
// (w / d') rho and w / rho are both near |w| / sqrt|d'| (returned: h, so that
// both scalings are exponent shifts); and the exponent e that brings a row
// block's largest magnitude m into (2^13, 2^14] (0 for m = 0).
__device__ __forceinline__ int f16_rho_exp(double d)
{
    if (d == 0.0) return 0;
    int x;
    (void)__builtin_frexp(d, &x);
    return x >> 1;
}
__device__ __forceinline__ int f16_row_exp(double m)
{
    if (!(m > 0.0)) return 0;
    int x;
    const double f = __builtin_frexp(m, &x);  // m = f 2^x, f in [0.5, 1): m <= 2^x, > 2^(x-1)
    return 14 - (f == 0.5 ? x - 1 : x);
}

// ------------------------------------------------------------ panel solves
// Rows of a panel solved against the factored 64x64 diagonal block on the
// matrix cores. A solve of the form X T^T = A (T lower triangular, 64 x 64)
// is cut into four 16-column blocks,
//   X_b^T = T_bb^{-1} (A_b^T - sum_{c<b} T_bc X_c^T),   b = 0..3,
// one v_mfma_f64_16x16x4f64 per 4-deep slab. The product leaves element e of
// lane l at row l/16 + 4e, column l%16 of the 16x16 result and takes its
// right-hand operand for slab s from row l/16, column l%16 of that slab, so
// element s of one product is, lane for lane, slab s of the right-hand operand
// of the next: a group of 16 rows never leaves registers.
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Where T[k][t] sits in LDS: Tt[t * LD + k] (T stored by columns with pitch
// LD), or with TR, Tt[k * LD + t] (T stored by rows, e.g. the transpose of an
// upper triangle stored by columns).
template <int LD, bool TR>
__device__ __forceinline__ int tidx(int t, int k)
{
    return TR ? k * LD + t : t * LD + k;
}

// One group of 16 rows. Lane (q, i16) = (lane / 16, lane % 16) holds in
// cur[4b + e] row i16, column 16b + 4e + q of A and receives the same entry
// of X in x[b][e]. T[k][t] is Tt[tidx<LD, TR>(t, k)]; only the blocks below
// the diagonal blocks are read. Inv[b * kInvBlock + i * kInvPitch + k] =
// (T_bb^{-1})[i][k].
template <int LD = kBP, bool TR = false>
__device__ __forceinline__ void solve_group(const double* Tt, const double* Inv,
                                            const double (&cur)[16], d4 (&x)[4], int q, int i16)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        d4 acc = {cur[4 * b], cur[4 * b + 1], cur[4 * b + 2], cur[4 * b + 3]};
#pragma unroll
        for (int c = 0; c < b; ++c)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc = mfma16(-Tt[tidx<LD, TR>(16 * c + 4 * s + q, 16 * b + i16)], x[c][s], acc);
        d4 xb = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) xb = mfma16(Inv[b * kInvBlock + i16 * kInvPitch + 4 * s + q], acc[s], xb);
        x[b] = xb;
    }
}

// Inverses of the four 16x16 diagonal blocks of T (lower triangular, unit
// diagonal if UNIT; T[k][t] = Tt[tidx<LD, TR>(t, k)] as for solve_group) by
// forward substitution, one column per lane of the calling wavefront.
template <bool UNIT, int LD = kBP, bool TR = false>
__device__ __forceinline__ void invert_diag_blocks(const double* Tt, double* Inv, int lane)
{
    const int b = lane >> 4, c = lane & 15;
    double y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        double acc = (k == c) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < k; ++t) acc -= Tt[tidx<LD, TR>(16 * b + t, 16 * b + k)] * y[t];
        y[k] = UNIT ? acc : acc / Tt[tidx<LD, TR>(16 * b + k, 16 * b + k)];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) Inv[b * kInvBlock + k * kInvPitch + c] = y[k];
}

}  // namespace leaf
}  // namespace dpp
