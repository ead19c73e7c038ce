// Host side of the C ABI declared in include/dpp.h: argument checks, workspace
// layout and the fixed launch sequence of the blocked sampler.
//
// Launch sequence (blocked right-looking sampler, Sec. 3; the unblocked
// sampler of Sec. 2 on each 64-wide diagonal block):
//
//   LDL^H, outer block width B0 (tuning.h: 4096 for FP64 and split updates):
//     for each outer panel [j0, j1 = j0 + B0):
//       factor_panel(j0, B0)                       -- recursive, below
//       update rows/cols [j1, n) by columns [j0, j1) -- the trailing update
//     factor_panel(c0, w), w = 64 * 2^k: w = 64 -> one diagonal-block
//       launch; else with mid = c0 + w/2: factor_panel(c0, w/2),
//       update rows [mid, n) x cols [mid, mid + w/2) by columns [c0, mid),
//       factor_panel(mid, w/2). Nodes at or past the largest n are skipped.
//   LU, outer block width B0 (tuning.h): for each outer panel [j0, j1),
//     lu_panel(j0, B0), the same binary tree: w = 64 -> one diagonal-block
//     launch (pivots, L below, U out to n); else factor the left half, update
//     rows [mid, n) x cols [mid, c0 + w) and rows [mid, c0 + w) x cols
//     [c0 + w, n) by columns [c0, mid), factor the right half. After the panel
//     the trailing update of [j1, n) x [j1, n) by its B0 columns.
//   Then one finalize launch (loglik, info).
//
// Every grouping of the Schur updates is exact in exact arithmetic: the -1 of
// a rejected pivot commutes with the outer-product updates (Prop. 5). The
// sequence depends only on (n, dtype, precision), never on the decisions, so
// there is no device-to-host traffic inside a call.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "dpp.h"
#include "dpp_internal.h"
#include "tuning.h"

namespace {

using dpp::DevProb;
using dpp::kLeaf;

struct Plan {
    bool herm;
    int dtype;   // 0 FP64 storage, 1 FP32 storage, 2 complex (FP64 parts)
    bool cplx;   // complex: blocks of kLeafC complex columns, real forms in the updates
    int leaf;    // diagonal-block width (kLeaf, or kLeafC for complex)
    int pieces;  // split updates: pieces per value (2 or 3), 0: FP64 updates
    bool f16;    // the FP16 form (pieces = 2, real Hermitian only)
    int B0;      // outer panel width (leaf times a power of two)
    int ss;      // row stride of the split panel copies (real k columns)
};

Plan make_plan(bool herm, dpp_dtype dt, dpp_precision prec, int64_t nmax)
{
    Plan p;
    p.herm = herm;
    p.dtype = dt == DPP_F32 ? 1 : dt == DPP_C128 ? 2 : 0;
    p.cplx = dt == DPP_C128;
    p.leaf = p.cplx ? dpp::kLeafC : kLeaf;
    p.f16 = prec == DPP_PREC_SPLIT_FP16;
    p.pieces = prec == DPP_PREC_SPLIT_BF16 || p.f16 ? 2 : prec == DPP_PREC_SPLIT_BF16X6 ? 3 : 0;
    // Outer panel width: each trailing update reads and writes the trailing
    // matrix once, so its HBM traffic per sample is ~ 8 n^3 / (3 B0) bytes for
    // FP64 storage; the split path needs the wider panel to stay MFMA-bound.
    // Inside a panel the binary tree passes over the panel's rows (and, for
    // LU, its rows of U to the right) once per level, log2(B0 / 64) times.
    // A complex column is two real columns of the products' real forms, so
    // complex panels are half as wide for the same real panel width.
    if (herm) p.B0 = p.pieces ? dpp::tuned::kB0LdlhSplit : dpp::tuned::kB0LdlhFp64;
    else p.B0 = dpp::tuned::kB0Lu;
    if (p.cplx) p.B0 /= 2;
    // The split copies hold the columns of one outer panel, at most B0 and no
    // more than the largest problem has (rounded to whole blocks), so small
    // batched problems keep small copies. B0 itself (the blocking) does not
    // depend on the sizes in the batch.
    const int64_t cap = (nmax + p.leaf - 1) / p.leaf * p.leaf;
    p.ss = (p.B0 < cap ? p.B0 : (int)cap) * (p.cplx ? 2 : 1);
    return p;
}

// Largest leading dimension: the kernels address a column strip (up to 256
// columns of A) with 32-bit byte offsets; complex entries take twice the bytes.
constexpr int64_t kMaxLda = (int64_t)1 << 20;
int64_t max_lda(dpp_dtype dt) { return dt == DPP_C128 ? kMaxLda / 2 : kMaxLda; }

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Planes of L have one row per real row of the Schur complement (two per
// complex row), planes of B one per column.
size_t split_bytes(const Plan& p, int64_t n)
{
    const size_t rows = (size_t)dpp::plane_rows(p.cplx ? 2 * n : n) + (size_t)dpp::plane_rows(n);
    return p.pieces ? align_up((size_t)p.pieces * rows * (size_t)p.ss * sizeof(uint16_t)) : 0;
}
// FP16 form: one float per side, row and 64-column block of the panel.
size_t scale_bytes(const Plan& p, int64_t n)
{
    return p.f16 ? align_up(2 * (size_t)(p.ss / 64) * (size_t)dpp::plane_rows(n) * sizeof(float)) : 0;
}
size_t diag_bytes(const Plan& p, int64_t n)
{
    const size_t elt = p.cplx ? 2 * sizeof(double) : sizeof(double);
    return align_up((size_t)((n + p.leaf - 1) / p.leaf) * p.leaf * p.leaf * elt);
}
// Per-problem workspace: [diagonal-block strip][split copies][row scales].
size_t problem_bytes(const Plan& p, int64_t n)
{
    return diag_bytes(p, n) + split_bytes(p, n) + scale_bytes(p, n);
}
// Workspace layout: [descriptors][per problem: diagonal strip, split copies].
size_t desc_bytes(int64_t count) { return align_up((size_t)count * sizeof(DevProb)); }

bool valid_enums(dpp_dtype dt, dpp_precision prec)
{
    return (dt == DPP_F64 || dt == DPP_F32 || dt == DPP_C128) &&
           (prec == DPP_PREC_FP64 || prec == DPP_PREC_SPLIT_BF16 || prec == DPP_PREC_SPLIT_BF16X6 ||
            prec == DPP_PREC_SPLIT_FP16);
}
// The FP16 form is built for real Hermitian kernels (its column balance uses
// the bound |w| <= 1 of their Schur complements).
bool supported(bool herm, dpp_dtype dt, dpp_precision prec)
{
    return prec != DPP_PREC_SPLIT_FP16 || (herm && dt != DPP_C128);
}

// gfx950 check, cached per device ordinal.
dpp_status device_ok()
{
    static std::mutex mu;
    static std::vector<int> state;  // 0 unknown, 1 ok, 2 unsupported
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DPP_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(mu);
    if ((int)state.size() <= dev) state.resize(dev + 1, 0);
    if (state[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DPP_ERR_UNSUPPORTED;
        state[dev] = (strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 2;
    }
    return state[dev] == 1 ? DPP_OK : DPP_ERR_UNSUPPORTED;
}

// ------------------------------------------------------------------ profiling
// Kernel families whose launches the profiler tells apart.
enum KernelId {
    K_LEAF_LDLH, K_LEAF_LU, K_LEAF_ZLDLH, K_LEAF_ZLU, K_UPDATE_F64, K_UPDATE_BF16X3,
    K_UPDATE_BF16X6, K_UPDATE_FP16X3, K_SMALL_LDLH, K_STORE_DIAG, K_FINALIZE, K_DESCS, K_COUNT
};
const char* const kKernelNames[K_COUNT] = {"leaf_ldlh",     "leaf_lu",       "leaf_zldlh",
                                           "leaf_zlu",      "update_f64",    "update_bf16x3",
                                           "update_bf16x6", "update_fp16x3", "small_ldlh",
                                           "store_diag",    "finalize",      "store_descs"};

struct ProfRecord {
    int id;
    hipEvent_t ev0, ev1;
    double flops, bytes;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;  // created once, reused
    size_t used = 0;
    std::vector<ProfRecord> recs;

    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};
Profiler& prof()
{
    static Profiler p;
    return p;
}

// The launches of a batch: every launch covers the size groups in `spans`
// (problems indexed in `probs`, the whole batch's descriptors).
struct Ctx {
    Plan plan;
    const DevProb* probs;  // device
    const dpp::GroupSpan* spans;
    int nspan;
    int64_t pfirst, count;  // the problems the spans cover: [pfirst, pfirst + count)
    int64_t nmax;
    int64_t pmax;          // largest npiv: no diagonal block at or past it is decided
    hipStream_t s;
    const std::vector<int64_t>* ns;  // host copy of the sizes of those problems
    bool profiling;
};

#define DPP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return DPP_ERR_HIP;  \
    } while (0)

// Runs `launch` (returning hipError_t); with profiling on, brackets it with
// events and notes its algorithmic work.
template <typename F>
dpp_status timed(const Ctx& c, int id, double flops, double bytes, F&& launch)
{
    if (!c.profiling) {
        DPP_TRY(launch());
        return DPP_OK;
    }
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    ProfRecord r{id, p.take(), p.take(), flops, bytes};
    if (!r.ev0 || !r.ev1) return DPP_ERR_HIP;
    DPP_TRY(hipEventRecord(r.ev0, c.s));
    DPP_TRY(launch());
    DPP_TRY(hipEventRecord(r.ev1, c.s));
    p.recs.push_back(r);
    return DPP_OK;
}

// Algorithmic work of a Schur update of rows [base, n) x cols [base, base+ncols)
// by kw factored columns, summed over the problems that have it.
void update_work(const Ctx& c, const dpp::Region& rg, int kw, double& flops, double& bytes)
{
    flops = bytes = 0.0;
    // Complex: four real products per complex one; entries of 16 bytes.
    const double cw = c.plan.cplx ? 4.0 : 1.0;
    const double elt = c.plan.dtype == 0 ? 8.0 : c.plan.dtype == 2 ? 16.0 : 4.0;
    // Operand bytes per row and k: BF16 pieces of L' (two real rows of two
    // real k per complex entry) and W' (one row of two), or the stored values.
    const double opnd_l = c.plan.pieces ? 2.0 * c.plan.pieces * (c.plan.cplx ? 4.0 : 1.0) : elt;
    const double opnd_w = c.plan.pieces ? 2.0 * c.plan.pieces * (c.plan.cplx ? 2.0 : 1.0) : elt;
    for (int64_t n : *c.ns) {
        const int64_t nr = (rg.r0 + rg.rlen < n ? rg.r0 + rg.rlen : n) - rg.r0;
        const int64_t nc = (rg.c0 + rg.clen < n ? rg.c0 + rg.clen : n) - rg.c0;
        if (nr <= 0 || nc <= 0) continue;
        const double e = c.plan.herm ? (double)nc * nr - (double)nc * (nc - 1) / 2.0
                                     : (double)nr * nc;
        flops += 2.0 * e * kw * cw;
        bytes += 2.0 * e * elt + ((double)nr * opnd_l + (double)nc * opnd_w) * kw;
    }
}

void leaf_work(const Ctx& c, int64_t c0, double& flops, double& bytes)
{
    flops = bytes = 0.0;
    const double elt = c.plan.dtype == 0 ? 8.0 : c.plan.dtype == 2 ? 16.0 : 4.0;
    const double sides = c.plan.herm ? 1.0 : 2.0;  // LU also solves the row panel
    const int64_t lw = c.plan.leaf;
    for (int64_t n : *c.ns) {
        if (c0 >= n) continue;
        const double bs = (double)((n - c0) < lw ? (n - c0) : lw);
        const double m = (double)(n - c0) - bs;
        flops += (bs * bs * bs / 3.0 * (c.plan.herm ? 1.0 : 2.0) + sides * m * bs * bs) *
                 (c.plan.cplx ? 4.0 : 1.0);
        bytes += (bs * bs + 2.0 * sides * m * bs) * elt +
                 sides * m * bs * 4.0 * c.plan.pieces * (c.plan.cplx ? 3.0 : 1.0);
    }
}

dpp_status update(const Ctx& c, const dpp::Region& rg, int64_t k0, int kw, int64_t j0)
{
    double fl = 0, by = 0;
    if (c.profiling) update_work(c, rg, kw, fl, by);
    if (c.plan.pieces)
        return timed(c, c.plan.f16 ? K_UPDATE_FP16X3 : c.plan.pieces == 2 ? K_UPDATE_BF16X3 : K_UPDATE_BF16X6,
                     fl, by, [&] {
            return dpp::launch_update_split(c.plan.herm, c.plan.dtype, c.plan.pieces, c.plan.f16,
                                            c.probs, c.spans, c.nspan, rg, k0, kw, j0, c.plan.ss, c.s);
        });
    return timed(c, K_UPDATE_F64, fl, by, [&] {
        return dpp::launch_update_f64(c.plan.herm, c.plan.dtype, c.probs, c.spans, c.nspan, rg,
                                      k0, kw, c.s);
    });
}

dpp_status leaf(const Ctx& c, int64_t c0, int64_t j0)
{
    double fl = 0, by = 0;
    if (c.profiling) leaf_work(c, c0, fl, by);
    if (c.plan.cplx)
        return timed(c, c.plan.herm ? K_LEAF_ZLDLH : K_LEAF_ZLU, fl, by, [&] {
            return dpp::launch_leaf_complex(c.plan.herm, c.plan.pieces, c.probs, c.spans, c.nspan,
                                            c0, j0, c.plan.ss, c.s);
        });
    if (c.plan.herm)
        return timed(c, K_LEAF_LDLH, fl, by, [&] {
            return dpp::launch_leaf_ldlh(c.plan.dtype, c.plan.pieces, c.plan.f16, c.probs, c.spans,
                                         c.nspan, c0, j0, c.plan.ss, c.s);
        });
    return timed(c, K_LEAF_LU, fl, by, [&] {
        return dpp::launch_leaf_lu(c.plan.dtype, c.plan.pieces, c.probs, c.spans, c.nspan, c0, j0,
                                   c.plan.ss, c.s);
    });
}

// Columns [c0, c0 + w) of the outer panel starting at j0, w = 64 * 2^k. The
// split points form a fixed binary tree over each outer panel, whatever the
// sizes in the batch: a problem sees the same sequence of operations (and
// bit-identical results) alone and in any batch.
dpp_status factor_panel(const Ctx& c, int64_t c0, int64_t w, int64_t j0)
{
    if (c0 >= c.pmax) return DPP_OK;
    if (w <= c.plan.leaf) return leaf(c, c0, j0);
    const int64_t h = w / 2, mid = c0 + h;
    dpp_status st = factor_panel(c, c0, h, j0);
    if (st != DPP_OK || mid >= c.nmax) return st;
    st = update(c, dpp::trailing_region(mid, h), c0, (int)h, j0);
    if (st != DPP_OK) return st;
    return factor_panel(c, mid, h, j0);
}

// LU columns [c0, c0 + w) of the outer panel starting at j0, w = leaf * 2^k:
// the same fixed binary tree as factor_panel. After the left half [c0, mid)
// is factored, its columns update, with k in [c0, mid), rows [mid, n) x
// columns [mid, c0 + w) (the right half's diagonal block, its rows of L, and
// its rows of U inside the node) and rows [mid, c0 + w) x columns
// [c0 + w, n) (the right half's rows of U past the node). A diagonal block at
// row block r then sees every k < r of the panel: the one node whose left
// half holds k and right half holds r applied it, and each of its launches
// solves its rows of L below it and its rows of U out to column n. The block
// [j1, n) x [j1, n) waits for one update with K = B0 after the panel.
dpp_status lu_panel(const Ctx& c, int64_t c0, int64_t w, int64_t j0)
{
    if (c0 >= c.pmax) return DPP_OK;
    if (w <= c.plan.leaf) return leaf(c, c0, j0);
    constexpr int64_t kAll = (int64_t)1 << 62;
    const int64_t h = w / 2, mid = c0 + h;
    dpp_status st = lu_panel(c, c0, h, j0);
    if (st != DPP_OK || mid >= c.nmax) return st;
    st = update(c, dpp::Region{mid, kAll, mid, h}, c0, (int)h, j0);
    if (st != DPP_OK) return st;
    if (c0 + w < c.nmax) {
        st = update(c, dpp::Region{mid, h, c0 + w, kAll}, c0, (int)h, j0);
        if (st != DPP_OK) return st;
    }
    return lu_panel(c, mid, h, j0);
}

// Largest n of the small-problem path: the tuned cutover of the precision,
// or DPP_SMALL_CUTOVER (a decimal in 0..kSmallMax) when that is set.
int64_t small_cutover(const Plan& plan)
{
    int64_t cut = dpp::tuned::kSmallCutover[plan.f16 ? 3 : plan.pieces ? plan.pieces - 1 : 0];
    if (const char* e = getenv("DPP_SMALL_CUTOVER")) {
        char* end = nullptr;
        const long v = strtol(e, &end, 10);
        if (end != e && *end == '\0' && v >= 0 && v <= dpp::kSmallMax) cut = v;
    }
    return std::min(dpp::kSmallMax, cut);
}

// Size groups of a batch (tuning.h): narrow widths up to kGroupSplitN, then wide.
int64_t size_group(int64_t n)
{
    using namespace dpp::tuned;
    const int64_t narrow = (kGroupSplitN + kGroupNarrow - 1) / kGroupNarrow;
    return n <= kGroupSplitN ? (n + kGroupNarrow - 1) / kGroupNarrow
                             : narrow + (n + kGroupWide - 1) / kGroupWide;
}

// The launch sequence of the problems the spans cover: one fixed sequence for
// the largest n, each launch covering every size group that has its step.
dpp_status run_groups(const Ctx& c)
{
    const Plan& plan = c.plan;
    for (int64_t j0 = 0; j0 < c.pmax; j0 += plan.B0) {
        const int64_t j1 = j0 + plan.B0;
        dpp_status st = plan.herm ? factor_panel(c, j0, plan.B0, j0) : lu_panel(c, j0, plan.B0, j0);
        if (st != DPP_OK) return st;
        if (j1 < c.nmax) {
            st = update(c, dpp::trailing_region(j1, c.nmax - j1), j0, plan.B0, j0);
            if (st != DPP_OK) return st;
        }
    }
    dpp_status st = timed(c, K_STORE_DIAG, 0.0, 0.0, [&] {
        return dpp::launch_store_diag(plan.herm, plan.dtype, c.probs + c.pfirst, (int)c.count, c.nmax,
                                      c.s);
    });
    if (st != DPP_OK) return st;
    return timed(c, K_FINALIZE, 0.0, 0.0,
                 [&] { return dpp::launch_finalize(c.probs + c.pfirst, (int)c.count, c.s); });
}

// An out-of-place problem's K: a valid leading dimension, and either A itself
// with the same leading dimension (in place) or storage disjoint from A's.
bool source_ok(const dpp_problem& q, dpp_dtype dt)
{
    if (q.ldk < q.n || q.ldk > max_lda(dt)) return false;
    if (q.K == q.A) return q.ldk == q.lda;
    const uintptr_t elt = dt == DPP_F64 ? 8 : dt == DPP_C128 ? 16 : 4;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(q.A), k0 = reinterpret_cast<uintptr_t>(q.K);
    const uintptr_t a1 = a0 + (uintptr_t)((q.n - 1) * q.lda + q.n) * elt;
    const uintptr_t k1 = k0 + (uintptr_t)((q.n - 1) * q.ldk + q.n) * elt;
    return a1 <= k0 || k1 <= a0;
}

dpp_status run(bool herm, const dpp_problem* probs, int64_t count, dpp_dtype dt,
               dpp_precision prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!probs || count < 1 || count > 65535 || !valid_enums(dt, prec) || !supported(herm, dt, prec))
        return DPP_ERR_INVALID_ARG;
    int64_t nmax = 0;
    for (int64_t i = 0; i < count; ++i) {
        const dpp_problem& q = probs[i];
        if (q.n < 1 || q.lda < q.n || q.lda > max_lda(dt) || !q.A || !q.u || !q.mask ||
            !q.pivots || !q.loglik || !q.info)
            return DPP_ERR_INVALID_ARG;
        if (q.K && !source_ok(q, dt)) return DPP_ERR_INVALID_ARG;
        const int64_t lw = dt == DPP_C128 ? dpp::kLeafC : dpp::kLeaf;
        if (q.npiv < 0 || q.npiv > q.n || (q.npiv % lw != 0 && q.npiv != q.n))
            return DPP_ERR_INVALID_ARG;
        nmax = q.n > nmax ? q.n : nmax;
    }
    const Plan plan = make_plan(herm, dt, prec, nmax);
    size_t need = desc_bytes(count);
    for (int64_t i = 0; i < count; ++i) need += problem_bytes(plan, probs[i].n);
    if (!ws || ws_bytes < need) return DPP_ERR_WORKSPACE;
    // The split planes take 16-byte stores and direct-to-LDS reads, the
    // diagonal strip 8-byte accesses; every piece starts at a multiple of
    // kAlign from ws.
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return DPP_ERR_INVALID_ARG;
    const dpp_status dev = device_ok();
    if (dev != DPP_OK) return dev;

    // Problems sorted by size (stable) and cut into groups of similar n. All
    // groups run one launch sequence (the one of the largest n); in each
    // launch a group gets workgroups sized for its own largest n (and, for
    // the updates, a tile shape for its own column count), so small problems
    // do not ride in grids sized for the largest, and the number of launches
    // does not grow with the number of groups. The blocking never depends on
    // the other sizes, so the grouping changes no result.
    std::vector<int64_t> order((size_t)count);
    for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return probs[a].n < probs[b].n; });

    std::vector<DevProb> host((size_t)count);  // descriptor slot p holds problem order[p]
    std::vector<char*> base_of((size_t)count);
    char* cursor = static_cast<char*>(ws) + desc_bytes(count);
    for (int64_t i = 0; i < count; ++i) {
        base_of[(size_t)i] = cursor;
        cursor += problem_bytes(plan, probs[i].n);
    }
    for (int64_t p = 0; p < count; ++p) {
        const int64_t i = order[(size_t)p];
        const dpp_problem& q = probs[i];
        DevProb& d = host[(size_t)p];
        d.A = q.A;
        d.n = q.n;
        d.lda = q.lda;
        d.K = q.K ? q.K : q.A;
        d.ldk = q.K ? q.ldk : q.lda;
        d.npiv = q.npiv ? q.npiv : q.n;
        d.u = q.u;
        d.mask = q.mask;
        d.piv = q.pivots;
        d.loglik = q.loglik;
        d.info = q.info;
        d.stats = q.stats;
        d.diag = reinterpret_cast<double*>(base_of[(size_t)i]);
        d.split = plan.pieces ? reinterpret_cast<uint16_t*>(base_of[(size_t)i] + diag_bytes(plan, q.n))
                              : nullptr;
        d.scale = plan.f16 ? reinterpret_cast<float*>(base_of[(size_t)i] + diag_bytes(plan, q.n) +
                                                      split_bytes(plan, q.n))
                           : nullptr;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool profiling;
    {
        std::lock_guard<std::mutex> g(prof().mu);
        profiling = prof().on;
    }
    std::vector<int64_t> ns_all((size_t)count);
    for (int64_t p = 0; p < count; ++p) ns_all[(size_t)p] = host[(size_t)p].n;
    Ctx c{plan, static_cast<const DevProb*>(ws), nullptr, 0, 0, count, nmax, nmax, s, &ns_all,
          profiling};

    // Descriptors reach the device as kernel arguments (copied at launch), so
    // the call neither reads host memory later nor blocks the host.
    for (int64_t i = 0; i < count; i += dpp::kDescPerLaunch) {
        const int cnt = (int)((count - i) < dpp::kDescPerLaunch ? (count - i) : dpp::kDescPerLaunch);
        const dpp_status st = timed(c, K_DESCS, 0.0, 0.0, [&] {
            return dpp::launch_store_descs(host.data() + i, cnt, static_cast<DevProb*>(ws) + i, s);
        });
        if (st != DPP_OK) return st;
    }

    // Small real Hermitian problems (the smallest, at the front of the sorted
    // order) run whole in LDS, one workgroup each, in one launch.
    int64_t nsmall = 0;
    if (plan.herm && !plan.cplx) {
        const int64_t cut = small_cutover(plan);
        while (nsmall < count && host[(size_t)nsmall].n <= cut) ++nsmall;
    }
    if (nsmall > 0) {
        const int64_t nm = host[(size_t)(nsmall - 1)].n;
        const std::vector<int64_t> ns_small(ns_all.begin(), ns_all.begin() + nsmall);
        const Ctx cs{plan, c.probs, nullptr, 0, 0, nsmall, nm, nm, s, &ns_small, profiling};
        double fl = 0.0;
        for (int64_t n : ns_small) fl += (double)n * n * n / 3.0;
        dpp_status st = timed(cs, K_SMALL_LDLH, fl, 0.0, [&] {
            return dpp::launch_small_ldlh(plan.dtype, c.probs, (int)nsmall, nm, s);
        });
        if (st != DPP_OK) return st;
        st = timed(cs, K_FINALIZE, 0.0, 0.0, [&] { return dpp::launch_finalize(c.probs, (int)nsmall, s); });
        if (st != DPP_OK) return st;
    }

    // Size groups, each sized in its launches for its own largest n; up to
    // kMaxGroupsPerLaunch of them share every launch.
    std::vector<dpp::GroupSpan> spans;
    for (int64_t p0 = nsmall; p0 < count;) {
        int64_t p1 = p0 + 1;
        while (p1 < count && size_group(host[(size_t)p1].n) == size_group(host[(size_t)p0].n)) ++p1;
        spans.push_back(dpp::GroupSpan{p0, p1 - p0, host[(size_t)(p1 - 1)].n});
        p0 = p1;
    }
    for (size_t g0 = 0; g0 < spans.size(); g0 += dpp::kMaxGroupsPerLaunch) {
        const size_t g1 = std::min(spans.size(), g0 + (size_t)dpp::kMaxGroupsPerLaunch);
        const int64_t pfirst = spans[g0].p0, plast = spans[g1 - 1].p0 + spans[g1 - 1].count;
        std::vector<int64_t> ns(ns_all.begin() + pfirst, ns_all.begin() + plast);
        int64_t pmax = 0;
        for (int64_t p = pfirst; p < plast; ++p) pmax = std::max(pmax, host[(size_t)p].npiv);
        const Ctx g{plan, c.probs, spans.data() + g0, (int)(g1 - g0), pfirst, plast - pfirst,
                    spans[g1 - 1].nmax, pmax, s, &ns, profiling};
        const dpp_status st = run_groups(g);
        if (st != DPP_OK) return st;
    }
    return DPP_OK;
}

size_t workspace_batched(bool herm, dpp_dtype dt, const int64_t* ns, int64_t count,
                         dpp_precision prec)
{
    if (!ns || count < 1 || !valid_enums(dt, prec) || !supported(herm, dt, prec)) return 0;
    int64_t nmax = 0;
    for (int64_t i = 0; i < count; ++i) {
        if (ns[i] < 1 || ns[i] > max_lda(dt)) return 0;
        nmax = ns[i] > nmax ? ns[i] : nmax;
    }
    const Plan plan = make_plan(herm, dt, prec, nmax);
    size_t need = desc_bytes(count);
    for (int64_t i = 0; i < count; ++i) need += problem_bytes(plan, ns[i]);
    return need;
}

// ------------------------------------------------- L-ensemble conversion
int64_t lens_np(int64_t n) { return (n + kLeaf - 1) / kLeaf * kLeaf; }

// Per-problem workspace of the conversion: the augmented matrix and the
// factorization's inputs and outputs for it.
size_t lens_problem_bytes(int64_t n)
{
    const size_t m = (size_t)(2 * lens_np(n));
    return align_up(m * m * sizeof(double)) + 2 * align_up(m * sizeof(double)) + align_up(m) +
           align_up(sizeof(double)) + align_up(sizeof(int32_t));
}

size_t lens_desc_bytes(int64_t count) { return align_up((size_t)count * sizeof(dpp::LensDesc)); }

size_t lens_workspace(const int64_t* ns, int64_t count, std::vector<int64_t>* ms_out = nullptr)
{
    if (!ns || count < 1 || count > 65535) return 0;
    std::vector<int64_t> ms((size_t)count);
    size_t need = lens_desc_bytes(count);
    for (int64_t i = 0; i < count; ++i) {
        if (ns[i] < 1 || 2 * lens_np(ns[i]) > kMaxLda) return 0;
        ms[(size_t)i] = 2 * lens_np(ns[i]);
        need += lens_problem_bytes(ns[i]);
    }
    const size_t sw = workspace_batched(true, DPP_F64, ms.data(), count, DPP_PREC_FP64);
    if (!sw) return 0;
    if (ms_out) *ms_out = ms;
    return need + sw;
}

// Input and output of one conversion: K may be L itself (same leading
// dimension: L is consumed before K is written), else the two must not overlap.
bool lens_args_ok(const dpp_lensemble& q, dpp_dtype dt)
{
    if (!q.L || !q.K || !q.info || q.n < 1 || q.ldl < q.n || q.ldk < q.n || q.ldl > kMaxLda ||
        q.ldk > kMaxLda)
        return false;
    if (q.K == q.L) return q.ldk == q.ldl;
    const uintptr_t elt = dt == DPP_F64 ? 8 : 4;
    const uintptr_t l0 = reinterpret_cast<uintptr_t>(q.L), k0 = reinterpret_cast<uintptr_t>(q.K);
    const uintptr_t l1 = l0 + (uintptr_t)((q.n - 1) * q.ldl + q.n) * elt;
    const uintptr_t k1 = k0 + (uintptr_t)((q.n - 1) * q.ldk + q.n) * elt;
    return l1 <= k0 || k1 <= l0;
}

// ------------------------------------------------- library-held scratch
// Workspace of dpp_sample_ldlh_batched_noalloc, for callers that cannot
// allocate device memory: one file-scope array per device, holding the last
// call's contents until the process ends. Host code never passes the array's
// name to a kernel (in host code it names a host-side stand-in); it uses the
// device address hipGetSymbolAddress returns, looked up once per device with
// that device current.
static __device__ __align__(256) unsigned char scratch[DPP_NOALLOC_SCRATCH_BYTES];

dpp_status scratch_address(void** out)
{
    static std::mutex mu;
    static std::vector<void*> addr;  // per device ordinal; nullptr: not looked up yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DPP_ERR_HIP;
    std::lock_guard<std::mutex> g(mu);
    if ((int)addr.size() <= dev) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[(size_t)dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DPP_ERR_HIP;
        addr[(size_t)dev] = p;
    }
    *out = addr[(size_t)dev];
    return DPP_OK;
}

}  // namespace

extern "C" {

dpp_status dpp_sample_ldlh_batched_noalloc(const dpp_problem* probs, int64_t count, dpp_dtype dt,
                                           dpp_precision prec, void* stream)
{
    if (!probs || count < 1 || count > 65535 || !valid_enums(dt, prec)) return DPP_ERR_INVALID_ARG;
    std::vector<int64_t> ns((size_t)count);
    for (int64_t i = 0; i < count; ++i) ns[(size_t)i] = probs[i].n;
    const size_t need = workspace_batched(true, dt, ns.data(), count, prec);
    if (need == 0) return DPP_ERR_INVALID_ARG;
    if (need > (size_t)DPP_NOALLOC_SCRATCH_BYTES) return DPP_ERR_WORKSPACE;
    const dpp_status dev = device_ok();
    if (dev != DPP_OK) return dev;
    void* ws = nullptr;
    const dpp_status st = scratch_address(&ws);
    if (st != DPP_OK) return st;
    // Nothing in the workspace needs to start at zero: every launch writes
    // what a later launch of the same call reads.
    return run(true, probs, count, dt, prec, ws, (size_t)DPP_NOALLOC_SCRATCH_BYTES, stream);
}


size_t dpp_lensemble_workspace_size(const int64_t* ns, int64_t count)
{
    return lens_workspace(ns, count);
}

dpp_status dpp_lensemble_to_marginal_batched(const dpp_lensemble* probs, int64_t count,
                                             dpp_dtype dt, void* ws, size_t ws_bytes,
                                             void* stream)
{
    if (!probs || count < 1 || count > 65535 || (dt != DPP_F64 && dt != DPP_F32))
        return DPP_ERR_INVALID_ARG;
    std::vector<int64_t> ns((size_t)count);
    int64_t nmax = 0, mmax = 0;
    for (int64_t i = 0; i < count; ++i) {
        if (!lens_args_ok(probs[i], dt)) return DPP_ERR_INVALID_ARG;
        ns[(size_t)i] = probs[i].n;
        nmax = std::max(nmax, probs[i].n);
    }
    std::vector<int64_t> ms;
    const size_t need = lens_workspace(ns.data(), count, &ms);
    if (need == 0) return DPP_ERR_INVALID_ARG;
    if (!ws || ws_bytes < need) return DPP_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return DPP_ERR_INVALID_ARG;
    const dpp_status dev = device_ok();
    if (dev != DPP_OK) return dev;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int dcode = dt == DPP_F64 ? 0 : 1;

    // Workspace: descriptors, then per problem the augmented matrix, u,
    // pivots, mask, loglik and info, then the factorization's own workspace.
    char* cursor = static_cast<char*>(ws) + lens_desc_bytes(count);
    std::vector<dpp::LensDesc> host((size_t)count);
    std::vector<dpp_problem> fact((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const dpp_lensemble& q = probs[i];
        const int64_t m = ms[(size_t)i];
        dpp::LensDesc& d = host[(size_t)i];
        d.L = q.L;
        d.K = q.K;
        d.n = q.n;
        d.ldl = q.ldl;
        d.ldk = q.ldk;
        d.np = m / 2;
        d.aug = reinterpret_cast<double*>(cursor);
        cursor += align_up((size_t)(m * m) * sizeof(double));
        d.u = reinterpret_cast<double*>(cursor);
        cursor += align_up((size_t)m * sizeof(double));
        double* piv = reinterpret_cast<double*>(cursor);
        cursor += align_up((size_t)m * sizeof(double));
        d.mask = reinterpret_cast<uint8_t*>(cursor);
        cursor += align_up((size_t)m);
        d.loglik = reinterpret_cast<double*>(cursor);
        cursor += align_up(sizeof(double));
        d.sinfo = reinterpret_cast<int32_t*>(cursor);
        cursor += align_up(sizeof(int32_t));
        d.logdet = q.logdet;
        d.info = q.info;
        mmax = std::max(mmax, m);
        fact[(size_t)i] = dpp_problem{d.aug, m, m, d.u, d.mask, piv, d.loglik, d.sinfo,
                                      nullptr, 0, d.np, nullptr};
    }
    dpp::LensDesc* ddesc = static_cast<dpp::LensDesc*>(ws);
    for (int64_t i = 0; i < count; i += dpp::kLensDescPerLaunch) {
        const int cnt = (int)std::min<int64_t>(count - i, dpp::kLensDescPerLaunch);
        if (dpp::launch_store_lens_descs(host.data() + i, cnt, ddesc + i, s) != hipSuccess)
            return DPP_ERR_HIP;
    }
    if (dpp::launch_lens_augment(dcode, ddesc, (int)count, mmax, s) != hipSuccess) return DPP_ERR_HIP;
    const size_t rest = ws_bytes - (size_t)(cursor - static_cast<char*>(ws));
    const dpp_status st =
        run(true, fact.data(), count, DPP_F64, DPP_PREC_FP64, cursor, rest, stream);
    if (st != DPP_OK) return st;
    if (dpp::launch_lens_extract(dcode, ddesc, (int)count, nmax, s) != hipSuccess) return DPP_ERR_HIP;
    if (dpp::launch_lens_status(ddesc, (int)count, s) != hipSuccess) return DPP_ERR_HIP;
    return DPP_OK;
}

dpp_status dpp_copy_lower(void* dst, const void* src, dpp_dtype dt, int64_t n, int64_t ld_dst,
                          int64_t ld_src, void* stream)
{
    if (!dst || !src || n < 1 || ld_dst < n || ld_src < n || ld_dst > kMaxLda || ld_src > kMaxLda ||
        (dt != DPP_F64 && dt != DPP_F32))
        return DPP_ERR_INVALID_ARG;
    const dpp_status dev = device_ok();
    if (dev != DPP_OK) return dev;
    if (dpp::launch_copy_lower(dt == DPP_F64 ? 0 : 1, dst, src, n, ld_dst, ld_src,
                               static_cast<hipStream_t>(stream)) != hipSuccess)
        return DPP_ERR_HIP;
    return DPP_OK;
}

dpp_status dpp_sample_ldlh(void* A, dpp_dtype dt, int64_t n, int64_t lda, const double* u,
                           uint8_t* mask, double* pivots, double* loglik, int32_t* info,
                           dpp_precision prec, void* ws, size_t ws_bytes, void* stream)
{
    const dpp_problem p{A, n, lda, u, mask, pivots, loglik, info};
    return run(true, &p, 1, dt, prec, ws, ws_bytes, stream);
}

dpp_status dpp_sample_lu(void* A, dpp_dtype dt, int64_t n, int64_t lda, const double* u,
                         uint8_t* mask, double* pivots, double* loglik, int32_t* info,
                         dpp_precision prec, void* ws, size_t ws_bytes, void* stream)
{
    const dpp_problem p{A, n, lda, u, mask, pivots, loglik, info};
    return run(false, &p, 1, dt, prec, ws, ws_bytes, stream);
}

dpp_status dpp_sample_ldlh_batched(const dpp_problem* probs, int64_t count, dpp_dtype dt,
                                   dpp_precision prec, void* ws, size_t ws_bytes, void* stream)
{
    return run(true, probs, count, dt, prec, ws, ws_bytes, stream);
}

dpp_status dpp_sample_lu_batched(const dpp_problem* probs, int64_t count, dpp_dtype dt,
                                 dpp_precision prec, void* ws, size_t ws_bytes, void* stream)
{
    return run(false, probs, count, dt, prec, ws, ws_bytes, stream);
}

size_t dpp_workspace_size(int hermitian, dpp_dtype dt, int64_t n, dpp_precision prec)
{
    return workspace_batched(hermitian != 0, dt, &n, 1, prec);
}

size_t dpp_workspace_size_batched(int hermitian, dpp_dtype dt, const int64_t* ns, int64_t count,
                                  dpp_precision prec)
{
    return workspace_batched(hermitian != 0, dt, ns, count, prec);
}

int dpp_profile_begin(void)
{
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.recs.clear();
    p.used = 0;
    p.on = true;
    return 0;
}

int dpp_profile_end(dpp_kernel_stats* out, int max)
{
    Profiler& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = false;
    dpp_kernel_stats acc[K_COUNT];
    memset(acc, 0, sizeof acc);
    for (const ProfRecord& r : p.recs) {
        if (hipEventSynchronize(r.ev1) != hipSuccess) return -1;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.ev0, r.ev1) != hipSuccess) return -1;
        acc[r.id].launches += 1;
        acc[r.id].ms += ms;
        acc[r.id].flops += r.flops;
        acc[r.id].bytes += r.bytes;
    }
    p.recs.clear();
    p.used = 0;
    int k = 0;
    for (int id = 0; id < K_COUNT; ++id) {
        if (acc[id].launches == 0) continue;
        if (out && k < max) {
            out[k] = acc[id];
            strncpy(out[k].name, kKernelNames[id], sizeof(out[k].name) - 1);
            out[k].name[sizeof(out[k].name) - 1] = 0;
        }
        ++k;
    }
    return k < max ? k : max;
}

const char* dpp_status_string(dpp_status s)
{
    switch (s) {
    case DPP_OK: return "success";
    case DPP_ERR_INVALID_ARG: return "invalid argument";
    case DPP_ERR_WORKSPACE: return "workspace missing or too small";
    case DPP_ERR_HIP: return "HIP runtime error";
    case DPP_ERR_UNSUPPORTED: return "unsupported device or configuration";
    }
    return "unknown status";
}

}  // extern "C"
