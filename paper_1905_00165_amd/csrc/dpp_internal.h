// Internal declarations shared by the gfx950 kernels and the host entry points.
// Not part of the public ABI (include/dpp.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpp {

// Width of the diagonal block whose keep/reject decisions one wavefront makes
// (one matrix row per lane of the 64-wide wavefront).
constexpr int kLeaf = 64;
// The same for complex kernels: 32 complex columns, whose real and imaginary
// parts are the 64 real columns of the block's real form (see below), so a
// lane's row still fits the same registers and the panel solves and updates
// see 64-wide real blocks.
constexpr int kLeafC = 32;

// Complex kernels (storage: interleaved real and imaginary parts, column-major,
// leading dimension in complex entries) run their solves and Schur updates in
// real arithmetic on real forms of the complex factors. Complex column p of a
// panel becomes real columns 2p (real part) and 2p + 1 (imaginary part); the
// Schur complement C, viewed as a real matrix with rows 2i + s (s = 0: real
// part, 1: imaginary part of complex row i) and complex columns j, lies in
// memory as a column-major real matrix with leading dimension 2 lda. Then
//   LDL^H: C -= L W^H, W = L D:  C'[2i + s][j] -= sum_k' L'[2i + s][k'] W'[j][k']
//     with W'[j] = (Re W_jp, Im W_jp)_p, L'[2i] = (Re L_ip, Im L_ip)_p and
//     L'[2i + 1] = (Im L_ip, -Re L_ip)_p;
//   LU: C -= L U, B = U^T: W'[j] = (Re B_jp, Im B_jp)_p, L'[2i] = (Re L_ip,
//     -Im L_ip)_p and L'[2i + 1] = (Im L_ip, Re L_ip)_p,
// i.e. a real product with twice the rows of L and twice the inner dimension.

// Per-problem descriptor as the kernels read it (device memory).
struct DevProb {
    void* A;          // column-major n x n, lda, storage type T
    int64_t n;
    int64_t lda;
    const void* K;    // the kernel, leading dimension ldk: read where an entry is
    int64_t ldk;      // read first (first_source below); K == A in place
    int64_t npiv;     // indices decided: [0, npiv), npiv = n or a multiple of 64
    const double* u;  // n uniforms
    uint8_t* mask;    // n
    double* piv;      // n, pivots after the decision
    double* loglik;   // 1
    int32_t* info;    // 1
    uint16_t* split;  // split-BF16 panel copies (see below), or nullptr
    double* diag;     // ceil(n/64) factored 64x64 diagonal blocks, column-major,
                      // block b at diag[b * 64 * 64]; copied into A at the end
    double* stats;    // 3 decision diagnostics (finalize.hip), or nullptr
    float* scale;     // FP16 split: per-row scales of the panel copies (below), or nullptr
};

// Out-of-place calls put the factor in A and leave K untouched. Every entry
// the factorization uses (the lower triangle for LDL^H, all of it for LU) is
// first read by exactly one launch: the diagonal-block launch at column 0 (its
// block, the panel below it and, for LU, the rows of U to its right), or an
// update whose factored columns start at k0 = 0 (the launch sequence gives
// each such update columns no earlier launch has touched). Those launches read
// K and write A; every other launch reads and writes A. In place, K is A.
template <typename T>
__device__ __forceinline__ const T* first_source(const DevProb& P, bool first, int64_t& ld)
{
    ld = first ? P.ldk : P.lda;
    return first ? static_cast<const T*>(P.K) : static_cast<const T*>(P.A);
}

// Split-BF16 panel copies of a problem: each factor value x is cut into
// `np` BF16 pieces (np = 2 or 3), p_0 = bf16(x) and p_i = bf16(x - p_0 - ...
// - p_{i-1}), so that their sum carries about 8 np significant bits of x. The
// 2 np planes are q = i: piece i of L, q = np + i: piece i of B, entry (r, kk)
// with r the global row of L (or the global column of the update for B) and
// kk = k - j0 the column within the current outer panel (ss columns per row,
// a multiple of 64). For LDL^H, B = L D (the scaled column, W); for LU,
// B = U^T. Values are bf16 bit patterns.
// Each plane is tiled in blocks of 32 rows x 32 columns (2 KiB), row blocks
// outer, and inside a block by halves of 16 columns: a half holds its 32 rows
// of 16 values (32 bytes) back to back. So the 16 rows x 32 columns an update
// stage copies are two contiguous 512-byte runs, and 32 rows x 16 columns one
// 1 KiB run; 8 consecutive columns of one row (16 bytes) stay contiguous.
// For complex kernels the planes of L hold the 2n rows of L' (one per real
// row of C) and those of B the n rows of W', both with ss real k columns.
//
// FP16 form (real LDL^H): np = 2 planes per side hold FP16 pieces hi =
// fp16(y), lo = fp16(y - hi) of scaled values y. Column k of the panel is
// balanced by a power of two rho_k near sqrt|d'_k|: the L side holds l_ik rho_k
// and the B side w_ik / rho_k, so their products are those of L and W while
// both sides stay near |w| / sqrt|d'_k| (every |w_ik| <= 1 for a marginal
// kernel); then each row's 64 values of one 64-column block are multiplied
// by the power of two 2^e that brings their largest magnitude into
// (2^13, 2^14], which keeps FP16's 11 bits for every value within 2^17 of the
// row's largest. The factor 2^-e that undoes it is kept per side s (0: L,
// 1: B), block c (kk / 64) and row r at scale[scale_off(n, ss, s, c, r)]; an
// update multiplies each 64-k partial sum of C by the factors of its row and
// column.
__host__ __device__ inline int64_t plane_rows(int64_t n) { return (n + 31) / 32 * 32; }
__host__ __device__ inline uint16_t* split_plane(uint16_t* base, int64_t nl, int64_t nb, int ss,
                                                 int np, int q)
{
    return q < np ? base + (int64_t)q * plane_rows(nl) * ss
                  : base + ((int64_t)np * plane_rows(nl) + (int64_t)(q - np) * plane_rows(nb)) * ss;
}
__host__ __device__ inline uint16_t* split_plane(uint16_t* base, int64_t n, int ss, int q)
{
    return base + (int64_t)q * plane_rows(n) * ss;
}
__host__ __device__ inline int64_t scale_off(int64_t n, int ss, int side, int c, int64_t r)
{
    return ((int64_t)side * (ss / 64) + c) * plane_rows(n) + r;
}
__host__ __device__ inline int64_t plane_off(int64_t r, int kk, int ss)
{
    return ((r >> 5) * (ss >> 5) + (kk >> 5)) * 1024 + ((kk >> 4) & 1) * 512 + (r & 31) * 16 +
           (kk & 15);
}

// ------------------------------------------------------------- size groups
// A batched call sorts its problems by n and cuts them into size groups; each
// step of the factorization is then one launch (or, for the updates, one per
// tile shape) covering every group that has that step. Within a launch group g
// owns the workgroups [off[g], off[g + 1]): wpp[g] of them for each of its
// problems [p0[g], p0[g] + (off[g + 1] - off[g]) / wpp[g]), and aux[g] is a
// per-group parameter of the kernel (the diagonal-block kernels: row groups
// per wavefront). The map travels in the kernel arguments.
struct GroupSpan {
    int64_t p0, count, nmax;  // first problem, problems, largest n of the group
};
constexpr int kMaxGroupsPerLaunch = 32;
struct GroupMap {
    int ng;
    int off[kMaxGroupsPerLaunch + 1];
    int wpp[kMaxGroupsPerLaunch];
    int p0[kMaxGroupsPerLaunch];
    int aux[kMaxGroupsPerLaunch];
};
// Problem, workgroup within the problem and aux of the launch's workgroup b
// (uniform across the workgroup); false past the last group.
__device__ __forceinline__ bool group_slot(const GroupMap& M, int64_t b, int& prob, int& w, int& aux)
{
    if (b >= M.off[M.ng]) return false;
    int g = 0;
    while (g + 1 < M.ng && b >= M.off[g + 1]) ++g;
    const int local = (int)(b - M.off[g]);
    prob = M.p0[g] + local / M.wpp[g];
    w = local % M.wpp[g];
    aux = M.aux[g];
    return true;
}
// Workgroup index b of a launch of G workgroups (G a multiple of 8) such that
// each of the 8 XCDs (workgroup i runs on XCD i % 8) takes a contiguous range.
__device__ __forceinline__ int64_t xcd_order(int64_t i, int64_t G) { return (i % 8) * (G / 8) + i / 8; }

// ------------------------------------------------------------------ launchers
// Each returns the launch status. `spans`/`nspan`: the size groups the launch
// covers (host array, problems indexed in `probs`); the kernels clamp per
// problem to its own n.

// Diagonal block [c0, c0+64) of every problem: decisions, L11/D1 (or L11/U11),
// and the panel solves for the rows below it (LU: and the columns to its
// right). With pieces = 2 or 3 also writes that many split-BF16 pieces of
// each panel value (0: none) at outer panel offset j0 with row stride ss;
// leaf_ldlh with f16 (pieces = 2) writes the FP16 form and its row scales.
hipError_t launch_leaf_ldlh(int dtype, int pieces, bool f16, const DevProb* probs,
                            const GroupSpan* spans, int nspan, int64_t c0, int64_t j0, int ss,
                            hipStream_t s);
hipError_t launch_leaf_lu(int dtype, int pieces, const DevProb* probs, const GroupSpan* spans,
                          int nspan, int64_t c0, int64_t j0, int ss, hipStream_t s);
// Complex kernels (storage dtype 2): the diagonal block [c0, c0 + kLeafC) in
// complex columns; the split planes hold the real forms L' and W' at real
// column 2 (c0 - j0) of the outer panel.
hipError_t launch_leaf_complex(bool herm, int pieces, const DevProb* probs, const GroupSpan* spans,
                               int nspan, int64_t c0, int64_t j0, int ss, hipStream_t s);

// Schur-complement update of rows [base, n) x cols [base, min(base+ncols, n))
// by the K range [k0, k0+kw) of the factored columns; herm: lower part only.
// Region of C an update writes: rows [r0, r0 + rlen), columns [c0, c0 + clen),
// each clipped to the problem's n. Hermitian updates take r0 == c0 and write
// the lower part only.
struct Region {
    int64_t r0, rlen, c0, clen;
};
// Rows [base, n) x columns [base, base + ncols): the lower-trapezoid updates
// of LDL^H and the trailing updates of LU.
inline Region trailing_region(int64_t base, int64_t ncols)
{
    return Region{base, (int64_t)1 << 62, base, ncols};
}

// dtype 0: FP64 storage, 1: FP32, 2: complex (FP64 parts; region, k0 and kw
// in complex rows and columns, the products on the real forms).
hipError_t launch_update_f64(bool herm, int dtype, const DevProb* probs, const GroupSpan* spans,
                             int nspan, Region rg, int64_t k0, int kw, hipStream_t s);
// Split-BF16 form: the products of the `pieces` (2 or 3) BF16 pieces of L and
// B whose orders sum to at most pieces - 1 (3 or 6 MFMA products). f16 (real
// Hermitian, pieces = 2): the FP16 form, hi*hi' + hi*lo' + lo*hi' on FP16
// MFMA, each 64-k partial sum scaled by its row and column factors.
// Groups whose updated columns call for different tile shapes go to separate
// launches (at most three).
hipError_t launch_update_split(bool herm, int dtype, int pieces, bool f16, const DevProb* probs,
                               const GroupSpan* spans, int nspan, Region rg, int64_t k0, int kw,
                               int64_t j0, int ss, hipStream_t s);

// Small Hermitian real problems (n <= kSmallMax, FP64 or FP32 storage), one
// workgroup each with the whole lower triangle in FP64 registers
// (small_ldlh.hip): the decisions, the factor or conditional kernel in A,
// mask and pivots; loglik and info come from launch_finalize as for the other
// problems.
constexpr int64_t kSmallMax = 192;
hipError_t launch_small_ldlh(int dtype, const DevProb* probs, int nprob, int64_t nmax,
                             hipStream_t s);

// loglik (fixed-order sum of ln|piv|) and info, one workgroup per problem.
hipError_t launch_finalize(const DevProb* probs, int nprob, hipStream_t s);

// Copies the factored diagonal blocks from each problem's strip into A (lower
// part for LDL^H, whole block for LU).
hipError_t launch_copy_lower(int dtype, void* dst, const void* src, int64_t n, int64_t ldd,
                             int64_t lds, hipStream_t s);
hipError_t launch_store_diag(bool herm, int dtype, const DevProb* probs, int nprob, int64_t nmax,
                             hipStream_t s);

// Copy `cnt` (<= kDescPerLaunch) host descriptors to dst through the kernel
// argument block of a one-workgroup launch.
constexpr int kDescPerLaunch = 34;  // 34 descriptors + count fit the 4 KiB argument block
hipError_t launch_store_descs(const DevProb* host, int cnt, DevProb* dst, hipStream_t s);

// L-ensemble conversion (lensemble.hip): one problem's device descriptor.
struct LensDesc {
    const void* L;     // n x n, ldl, storage type T (lower triangle read)
    void* K;           // n x n, ldk, storage type T (written in full)
    int64_t n, ldl, ldk;
    int64_t np;        // n rounded up to a multiple of 64; the augmented matrix is 2np x 2np
    double* aug;       // 2np x 2np FP64, column-major, leading dimension 2np
    double* u;         // 2np zeros (every pivot kept)
    uint8_t* mask;     // 2np, from the factorization of the first np pivots
    double* loglik;    // 1: sum of the logs of the first np pivots
    int32_t* sinfo;    // 1: the factorization's info word
    double* logdet;    // 1 or nullptr: ln det(L + I)
    int32_t* info;     // 1: 0, or 1 if L + I is not numerically positive definite
};
constexpr int kLensDescPerLaunch = 36;  // 36 descriptors + count fit the 4 KiB argument block
hipError_t launch_store_lens_descs(const LensDesc* host, int cnt, LensDesc* dst, hipStream_t s);
hipError_t launch_lens_augment(int dtype, const LensDesc* descs, int count, int64_t mmax,
                               hipStream_t s);
hipError_t launch_lens_extract(int dtype, const LensDesc* descs, int count, int64_t nmax,
                               hipStream_t s);
hipError_t launch_lens_status(const LensDesc* descs, int count, hipStream_t s);

}  // namespace dpp
