// Tuned constants of the launch sequence, each a function of (storage,
// precision, problem size) only, so that a result never depends on the rest
// of its batch. paper_1905_00165_amd/autotune.py measures the candidates on
// the GPU and writes this file; its record of the measurements is the comment
// block below.
#pragma once
#include <stdint.h>

namespace dpp {
namespace tuned {

// Outer panel width of real kernels (complex kernels: half as many complex
// columns): the trailing update re-reads the trailing matrix once per panel.
constexpr int kB0LdlhSplit = 4096;  // Hermitian, split-BF16 updates
constexpr int kB0LdlhFp64 = 2048;   // Hermitian, FP64 updates
constexpr int kB0Lu = 512;          // LU

// Size groups of a batch: widths of kGroupNarrow up to n = kGroupSplitN,
// then of kGroupWide (the blocking never depends on them, only the launches).
constexpr int64_t kGroupNarrow = 128;
constexpr int64_t kGroupSplitN = 2048;
constexpr int64_t kGroupWide = 1024;

// Largest n of a real Hermitian problem that runs in one workgroup with the
// whole matrix in LDS (small_ldlh.hip), by precision (FP64, split x3, split
// x6); 0 disables the path. At most kSmallMax.
constexpr int64_t kSmallCutover[3] = {128, 128, 128};

}  // namespace tuned
}  // namespace dpp
