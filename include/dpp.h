/*
 * dpp.h - C ABI of the MI355X (gfx950) factorization-based DPP sampler.
 *
 * The library samples a finite Determinantal Point Process from its marginal
 * kernel K (Poulson, "High-performance sampling of generic Determinantal Point
 * Processes", Sec. 2 Theorem 2 and Sec. 3, blocked sampler) by running an
 * unpivoted right-looking factorization of K in which pivot j is modified by a
 * Bernoulli draw: with d_j the current diagonal entry (the inclusion
 * probability of j conditioned on the decisions for 0..j-1, Props. 3-5),
 * index j is kept iff u_j < d_j, otherwise d_j is replaced by d_j - 1; the
 * column is then scaled by the modified pivot and the trailing Schur
 * complement is updated. Hermitian (real symmetric) K uses the LDL^H
 * specialization, general K the LU form.
 *
 * Conventions shared by every entry point
 *   - Every pointer argument except `probs` of the batched calls and the
 *     return-value strings is a DEVICE pointer owned by the caller. The library
 *     allocates no memory: all scratch space comes from the caller's workspace
 *     `ws` of `ws_bytes` bytes (query the size with dpp_workspace_size*),
 *     which must be 256-byte aligned (DPP_ERR_INVALID_ARG otherwise; device
 *     allocations are). Its contents on entry are ignored.
 *   - Matrices are column-major with leading dimension max(1, n) <= lda <=
 *     2^20 (the kernels address strips of up to 256 columns with 32-bit
 *     byte offsets).
 *   - `stream` is a hipStream_t (NULL: the default stream). Calls are
 *     asynchronous: outputs are valid once the stream has reached the end of
 *     the call. The library issues one fixed launch sequence per call whose
 *     shape depends only on (n, dtype, precision), never on the decisions.
 *   - Argument errors (n < 1, lda < n, lda > 2^20, NULL pointers, workspace
 *     too small, unknown enum values) are returned synchronously and nothing
 *     is launched.
 *   - Numerical trouble never returns an error code; it is reported in `info`
 *     (LAPACK style, see below).
 *   - Calls on one stream are ordered. Two calls that share a workspace or an
 *     output buffer must not run concurrently on different streams.
 */
#ifndef DPP_H
#define DPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DPP_OK = 0,
    DPP_ERR_INVALID_ARG = 1, /* bad size, stride, pointer or enum value          */
    DPP_ERR_WORKSPACE = 2,   /* ws is NULL or ws_bytes below the required size     */
    DPP_ERR_HIP = 3,         /* a HIP runtime call (launch, copy) failed           */
    DPP_ERR_UNSUPPORTED = 4  /* no gfx950 device, or an unsupported combination    */
} dpp_status;

/* Storage type of A. The pivots, the keep/reject test and the log-likelihood
   are always computed in FP64; with DPP_F32 the Schur complements are rounded
   to FP32 when they are stored back.
   DPP_C128: complex entries, two FP64 parts (real, imaginary) each, leading
   dimensions counted in complex entries (at most 2^19). For the complex
   kernels of the paper (Sec. 1 domino tilings, Sec. 3 dense complex LU), a
   conditional inclusion probability is real: index j is kept iff u_j < d_j
   with d_j the real part of the current diagonal entry, and the pivot loses 1
   on a rejection (its imaginary part, nonzero only for LU, is kept). The
   Hermitian sampler forms K - 1_{Y^c} = L D L^H with D real; the LU sampler
   scales by the whole complex pivot. Outputs (mask, pivots = the real d'_j,
   loglik = sum ln|d'_j|, info) are as for real kernels; npiv (batched calls)
   must then be a multiple of 32. Not accepted by dpp_copy_lower and the
   L-ensemble conversion. */
typedef enum { DPP_F64 = 0, DPP_F32 = 1, DPP_C128 = 2 } dpp_dtype;

/* Arithmetic of the Schur-complement (trailing) updates.
   DPP_PREC_FP64: FP64 MFMA products, FP64 accumulation.
   DPP_PREC_SPLIT_BF16: each factor x is split as x = hi + lo with hi = bf16(x)
   and lo = bf16(x - hi); the update is hi*hi' + hi*lo' + lo*hi' on BF16 MFMA
   with FP32 accumulation (about 2^-16 of each product is lost).
   DPP_PREC_SPLIT_BF16X6: three pieces p0 = bf16(x), p1 = bf16(x - p0),
   p2 = bf16(x - p0 - p1) and the six products p0*p0' + p0*p1' + p1*p0' +
   p0*p2' + p2*p0' + p1*p1' on BF16 MFMA (about 2^-24 of each product is
   lost), at twice the matrix-core work of DPP_PREC_SPLIT_BF16; the FP32
   sum is two-level: the matrix cores accumulate 64 values of k at a time,
   and those chunk sums are added up in FP32, so no FP32 sum runs over more
   than max(64, k / 64) terms.
   DPP_PREC_SPLIT_FP16 (real Hermitian kernels, FP64 or FP32 storage, LDL^H
   calls only; others return DPP_ERR_INVALID_ARG and workspace size 0): each
   value is scaled by powers of two (per panel column from its pivot d'_k,
   so that both factors of a product stay near |w| / sqrt|d'_k|, and per row
   and 64-column block, to bring the row's largest value near 2^14) and
   split as hi = fp16(y), lo = fp16(y - hi), about 22 significant bits; the
   update is hi*hi' + hi*lo' + lo*hi' on FP16 MFMA (the matrix-core work of
   DPP_PREC_SPLIT_BF16), each 64-value partial sum over k multiplied back by
   its row and column factors and summed in FP32 as for
   DPP_PREC_SPLIT_BF16X6. About 2^-22 of each product is lost: between the
   three- and six-product BF16 forms (over whole projection-kernel samples
   at n = 16384 its worst error is nearer the three-product form's).
   Every form subtracts the sum from the stored value in the storage
   precision. The diagonal-block decisions, the panel solves and the
   log-likelihood stay in FP64 on every path. */
typedef enum {
    DPP_PREC_FP64 = 0,
    DPP_PREC_SPLIT_BF16 = 1,
    DPP_PREC_SPLIT_BF16X6 = 2,
    DPP_PREC_SPLIT_FP16 = 3
} dpp_precision;

/*
 * dpp_sample_ldlh - sample DPP(K) for Hermitian (real symmetric) K.
 *
 *   A       in/out, n x n, dtype dt. Only the LOWER triangle is read and written.
 *           On entry the lower triangle of K. On exit the strict lower triangle
 *           holds the unit-lower L and the diagonal holds D of
 *           K - 1_{Y^c} = L D L^T (the in-place factorization named in the
 *           caption of the paper's unblocked listing), with 1_{Y^c} the
 *           diagonal indicator of the rejected indices.
 *   u       in, n FP64 uniforms; u_j is consumed for index j. Values in [0,1)
 *           are the intended use; u_j = 1 forces a rejection.
 *   mask    out, n bytes: 1 if index j is in the sample, else 0.
 *   pivots  out, n FP64: d'_j, the pivot after the decision (d_j if kept,
 *           d_j - 1 if rejected), so the pre-decision probability is
 *           pivots[j] + 1 - mask[j].
 *   loglik  out, 1 FP64: sum_j ln|d'_j|, the natural log of the likelihood of
 *           the returned sample (Theorem 2), summed in a fixed order (the
 *           result is bitwise reproducible).
 *   info    out, 1 int32: 0, or j+1 for the first j whose pivot d'_j is exactly
 *           zero or NaN. Then loglik is -inf or NaN and the outputs for indices
 *           after j are unspecified.
 *   prec    trailing-update arithmetic (see dpp_precision).
 *   ws      device workspace of at least dpp_workspace_size(1, dt, n, prec)
 *           bytes; its contents on entry are ignored.
 */
dpp_status dpp_sample_ldlh(void* A, dpp_dtype dt, int64_t n, int64_t lda, const double* u,
                           uint8_t* mask, double* pivots, double* loglik, int32_t* info,
                           dpp_precision prec, void* ws, size_t ws_bytes, void* stream);

/*
 * dpp_sample_lu - sample DPP(K) for general (non-Hermitian) K, the unpivoted LU
 * form of the sampler (Sec. 2 listing, Sec. 3 blocked LU listing).
 *   A   in/out, all n x n entries. On exit the strict lower triangle holds the
 *       unit-lower L and the upper triangle (with the diagonal) holds U of
 *       K - 1_{Y^c} = L U.
 * The other arguments are as for dpp_sample_ldlh;
 * ws needs dpp_workspace_size(0, dt, n, prec) bytes.
 */
dpp_status dpp_sample_lu(void* A, dpp_dtype dt, int64_t n, int64_t lda, const double* u,
                         uint8_t* mask, double* pivots, double* loglik, int32_t* info,
                         dpp_precision prec, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for one problem. hermitian: 1 for dpp_sample_ldlh, 0 for
   dpp_sample_lu. Returns 0 for invalid arguments. */
size_t dpp_workspace_size(int hermitian, dpp_dtype dt, int64_t n, dpp_precision prec);

/* One problem of a batched call. All pointers are device pointers; the fields
   A ... info mean what the arguments of the same names mean for the single
   calls.
     K, ldk  out-of-place source (optional). K NULL (or K == A with ldk == lda):
             in place, A holds K on entry. Otherwise K is the n x n kernel with
             leading dimension ldk (n <= ldk <= 2^20), read only, in storage
             disjoint from A (checked; DPP_ERR_INVALID_ARG otherwise); A is
             then an output only: its contents on entry are ignored and on exit
             it holds the factor exactly as the in-place call would leave it
             (bit for bit), except that for LDL^H the strict upper triangle of
             A is not written. Each entry of K is read once, so no working copy
             of K is needed per sample. Several problems may share one K; no
             problem's A may overlap another problem's A or K.
     npiv    indices to decide (optional; 0 means n). 0 < npiv < n must be a
             multiple of 64: only indices [0, npiv) are decided (mask, pivots,
             loglik and info cover them; loglik is then the log-probability of
             those decisions), and on exit the trailing block A[npiv:n, npiv:n]
             (its lower triangle for LDL^H) holds the marginal kernel of the
             remaining indices conditioned on those decisions: the Schur
             complement of K - 1_{Y^c} restricted to the decided indices
             (Props. 3-5). Sampling that block with its own call continues the
             same chain. Argument error otherwise. (DPP_C128: a multiple of 32.)
     stats   out, optional (NULL: not computed), 3 FP64 diagnostics of the
             decisions over the decided indices j, with d_j the pre-decision
             probability (recovered as d'_j, or d'_j + 1 for a rejection):
               stats[0] = min_j |u_j - d_j|, how close any decision came to a
                          tie (the near-tie margin; +inf if no index decided);
               stats[1] = the number of j with d_j < -1e-12 or d_j > 1 + 1e-12
                          (probabilities pushed out of [0, 1] by rounding,
                          compared as they are: no clamping);
               stats[2] = max_j of the distance from d_j to [0, 1] (0 if none). */
typedef struct {
    void* A;
    int64_t n;
    int64_t lda;
    const double* u;
    uint8_t* mask;
    double* pivots;
    double* loglik;
    int32_t* info;
    const void* K;
    int64_t ldk;
    int64_t npiv;
    double* stats;
} dpp_problem;

/*
 * dpp_sample_ldlh_batched / dpp_sample_lu_batched - `count` independent
 * problems, each with its own n, lda, stream of uniforms and outputs, sampled
 * by one launch sequence on `stream`: the problems are sorted by size into
 * groups, and each step of the factorization is one launch covering every
 * group that has that step (an update: one launch per tile shape). Real
 * Hermitian problems with n at or below the small-problem cutover instead run
 * whole in one workgroup each, with FP64 arithmetic at every precision. The
 * cutover is tuned per precision at build time (0 turns the path off); the
 * environment variable DPP_SMALL_CUTOVER, read at every call, overrides it
 * with a value in 0..192 (anything else is ignored).
 *   probs   HOST array of `count` descriptors; it is read before the call
 *           returns and may be reused at once.
 *   ws      device workspace of dpp_workspace_size_batched(...) bytes.
 * Every problem's results equal those of the single call on that problem
 * (bit for bit): the blocking depends only on (n, dtype, precision), never on
 * the other problems, and the problems do not interact. Problems must not
 * share A or output buffers.
 */
dpp_status dpp_sample_ldlh_batched(const dpp_problem* probs, int64_t count, dpp_dtype dt,
                                   dpp_precision prec, void* ws, size_t ws_bytes, void* stream);
dpp_status dpp_sample_lu_batched(const dpp_problem* probs, int64_t count, dpp_dtype dt,
                                 dpp_precision prec, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for a batch whose problem sizes are ns[0..count-1] (host
   array). Returns 0 for invalid arguments. */
size_t dpp_workspace_size_batched(int hermitian, dpp_dtype dt, const int64_t* ns, int64_t count,
                                  dpp_precision prec);

/*
 * dpp_sample_ldlh_batched_noalloc - dpp_sample_ldlh_batched for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same launch sequence and
 * kernels, with the workspace taken from a scratch array the library holds
 * on each device (DPP_NOALLOC_SCRATCH_BYTES, held from the library's load on
 * that device until the process ends) instead of the caller's `ws`. The caller
 * still passes every input and output buffer. The call allocates nothing and
 * results equal dpp_sample_ldlh_batched's bit for bit.
 *   Returns DPP_ERR_WORKSPACE when the batch needs more than
 *   DPP_NOALLOC_SCRATCH_BYTES, i.e. when dpp_workspace_size_batched(1, dt,
 *   ns, count, prec) exceeds it (one problem fits up to n = 131008 on the
 *   FP64 path, n = 2848 with DPP_PREC_SPLIT_BF16, n = 2304 with
 *   DPP_PREC_SPLIT_BF16X6 and n = 2816 with DPP_PREC_SPLIT_FP16).
 *   Every call on one device shares that device's scratch, which keeps the
 *   last call's contents (no call needs it zeroed): calls that may overlap on
 *   one device (different streams, or different host threads without
 *   ordering) race on it and must be serialized by the caller.
 * The first call on a device looks up the scratch's device address (once per
 * device, with that device current).
 */
#define DPP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dpp_status dpp_sample_ldlh_batched_noalloc(const dpp_problem* probs, int64_t count, dpp_dtype dt,
                                           dpp_precision prec, void* stream);

/*
 * dpp_copy_lower - stage a working copy for dpp_sample_ldlh: copy the lower
 * triangle (with the diagonal) of the n x n column-major matrix src (leading
 * dimension ld_src) into dst (ld_dst). The in-place LDL^H sampler (Sec. 3,
 * Hermitian form) reads and overwrites only that triangle, so this restores a
 * working copy from K at half the bytes of a full copy; dst's strict upper
 * triangle is left as it was. Both are device buffers of storage type dt;
 * they must not overlap. Asynchronous on `stream`; argument errors (n < 1,
 * ld < n or > 2^20, NULL pointers, bad dt) return before any launch.
 */
dpp_status dpp_copy_lower(void* dst, const void* src, dpp_dtype dt, int64_t n, int64_t ld_dst,
                          int64_t ld_src, void* stream);

/*
 * dpp_lensemble_to_marginal_batched - on-device conversion of `count`
 * Hermitian (real symmetric) L-ensemble kernels into marginal kernels,
 * K = I - (L + I)^{-1}, the conversion the paper's closing section names as
 * the natural companion of the blocked sampler, run on the sampler's own
 * blocked LDL^H: the 2n' x 2n' matrix [[L + I, I], [I, 0]] (n' = n rounded up
 * to 64, L padded with zeros) is factored through its first n' pivots with
 * every pivot kept, which leaves -(L + I)^{-1} as the trailing Schur
 * complement. FP64 arithmetic throughout.
 *   probs  HOST array of `count` descriptors, read before the call returns:
 *     L, n, ldl   in, n x n, storage type dt, column-major; only the lower
 *                 triangle is read. L must be positive semi-definite.
 *     K, ldk      out, n x n, storage type dt: the symmetric marginal kernel,
 *                 both triangles written. K may be L itself (ldk == ldl);
 *                 otherwise the two must not overlap.
 *     logdet      out, optional (NULL): ln det(L + I), the log normalization
 *                 constant of the L-ensemble.
 *     info        out, int32: 0, or 1 if a pivot of L + I was not positive (L
 *                 not positive semi-definite to working precision); K is then
 *                 unspecified.
 *   ws     device workspace of dpp_lensemble_workspace_size(ns, count) bytes
 *          (about 32 n'^2 bytes per problem plus the factorization's).
 * Argument errors (n < 1, bad leading dimensions, 2n' > 2^20, NULL pointers,
 * overlapping L and K) return synchronously before any launch.
 */
typedef struct {
    const void* L;
    int64_t n;
    int64_t ldl;
    void* K;
    int64_t ldk;
    double* logdet;
    int32_t* info;
} dpp_lensemble;

dpp_status dpp_lensemble_to_marginal_batched(const dpp_lensemble* probs, int64_t count,
                                             dpp_dtype dt, void* ws, size_t ws_bytes,
                                             void* stream);
/* Workspace bytes for conversions of sizes ns[0..count-1] (host array); 0 for
   invalid arguments. */
size_t dpp_lensemble_workspace_size(const int64_t* ns, int64_t count);

/* Static, NUL-terminated description of a status code. */
const char* dpp_status_string(dpp_status s);

/*
 * Profiling of the library's own kernel launches (process-wide).
 * dpp_profile_begin() clears previous records and starts recording: every
 * subsequent launch of the library is bracketed by two hipEvents on its
 * stream, and its algorithmic work is noted (flops of the Schur updates with
 * the n^3/3 (LDL^H) / 2n^3/3 (LU) convention's per-element count, and the
 * minimum HBM bytes the launch must move). dpp_profile_end() waits for the
 * recorded events, fills up to `max` entries of `out` (one per kernel that
 * ran), stops recording and returns the number of entries (negative on a HIP
 * error). Recording adds two event records per launch; do not profile calls
 * from several host threads at once.
 */
typedef struct {
    char name[32];     /* kernel family, e.g. "update_bf16x3"            */
    int64_t launches;  /* launches recorded                               */
    double ms;         /* sum of event-measured durations (milliseconds) */
    double flops;      /* algorithmic flops of those launches            */
    double bytes;      /* algorithmic HBM bytes of those launches        */
} dpp_kernel_stats;

int dpp_profile_begin(void);
int dpp_profile_end(dpp_kernel_stats* out, int max);

#ifdef __cplusplus
}
#endif

#endif /* DPP_H */
