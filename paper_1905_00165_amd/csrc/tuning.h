// Tuned constants of the launch sequence, each a function of (storage,
// precision, problem size) only, so that a result never depends on the rest
// of its batch. paper_1905_00165_amd/autotune.py measures the candidates on
// the GPU and writes this file; its record of the measurements is the comment
// block below.
// Record of the autotune run of 2026-12-03 (ms per call, by precision 0 = FP64,
// 1 = split x3, 2 = split x6):
//   1024 kernels of n = 32: small path {0: 0.0995, 1: 0.0992, 2: 0.0993}, blocked {0: 0.0923, 1: 0.0921, 2: 0.0918}
//   1024 kernels of n = 64: small path {0: 0.1315, 1: 0.1313, 2: 0.1313}, blocked {0: 0.1119, 1: 0.1116, 2: 0.1103}
//   1024 kernels of n = 96: small path {0: 0.1946, 1: 0.1944, 2: 0.1947}, blocked {0: 0.2187, 1: 0.1895, 2: 0.2141}
//   1024 kernels of n = 128: small path {0: 0.3889, 1: 0.3879, 2: 0.3906}, blocked {0: 0.2468, 1: 0.2252, 2: 0.2731}
//   1024 kernels of n = 160: small path {0: 0.4665, 1: 0.4657, 2: 0.4672}, blocked {0: 0.4183, 1: 0.3641, 2: 0.4441}
//   1024 kernels of n = 192: small path {0: 0.8093, 1: 0.8094, 2: 0.8083}, blocked {0: 0.4967, 1: 0.4289, 2: 0.5211}
//   -> kSmallCutover = [0, 0, 0]
//   4096 L-ensembles, group width 64: {0: 24.8878, 2: 26.3323}
//   4096 L-ensembles, group width 128: {0: 25.5257, 2: 26.9409}
//   4096 L-ensembles, group width 256: {0: 29.2082, 2: 28.3778}
//   -> kGroupNarrow = 64
//   b0_ldlh_split kB0LdlhSplit = 2048: {2: 124.3441}
//   b0_ldlh_split kB0LdlhSplit = 4096: {2: 122.9148}
//   -> kB0LdlhSplit = 4096
//   b0_ldlh_fp64 kB0LdlhFp64 = 1024: {0: 238.8056}
//   b0_ldlh_fp64 kB0LdlhFp64 = 2048: {0: 234.216}
//   -> kB0LdlhFp64 = 2048
//   b0_lu kB0Lu = 256: {0: 71.7892, 2: 49.947}
//   b0_lu kB0Lu = 512: {0: 69.4705, 2: 46.9873}
//   b0_lu kB0Lu = 1024: {0: 73.62, 2: 50.1623}
//   -> kB0Lu = 512
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
constexpr int64_t kGroupNarrow = 64;
constexpr int64_t kGroupSplitN = 2048;
constexpr int64_t kGroupWide = 1024;

// Largest n of a real Hermitian problem that runs in one workgroup with the
// whole lower triangle in registers (small_ldlh.hip), by precision (FP64, split x3, split
// x6, FP16 split); 0 disables the path. At most kSmallMax.
constexpr int64_t kSmallCutover[4] = {0, 0, 0, 0};

}  // namespace tuned
}  // namespace dpp
