// Tuned constants of the launch sequence, each a function of (storage,
// precision, problem size) only, so that a result never depends on the rest
// of its batch. paper_1905_00165_amd/autotune.py measures the candidates on
// the GPU and writes this file; its record of the measurements is the comment
// block below.
// Record of the autotune run of 2026-12-03 (ms per call, by precision 0 = FP64,
// 1 = split x3, 2 = split x6, 3 = FP16 split):
//   1024 kernels of n = 32: small path {0: 0.103, 1: 0.1028, 2: 0.103, 3: 0.1032}, blocked {0: 0.095, 1: 0.0954, 2: 0.0959, 3: 0.0958}
//   1024 kernels of n = 64: small path {0: 0.1345, 1: 0.1344, 2: 0.1342, 3: 0.1341}, blocked {0: 0.1163, 1: 0.1156, 2: 0.1147, 3: 0.1147}
//   1024 kernels of n = 96: small path {0: 0.2029, 1: 0.2008, 2: 0.2004, 3: 0.1998}, blocked {0: 0.2206, 1: 0.1963, 2: 0.1994, 3: 0.1963}
//   1024 kernels of n = 128: small path {0: 0.3957, 1: 0.3944, 2: 0.3926, 3: 0.3941}, blocked {0: 0.2476, 1: 0.2238, 2: 0.2409, 3: 0.2255}
//   1024 kernels of n = 160: small path {0: 0.4735, 1: 0.4759, 2: 0.4739, 3: 0.4762}, blocked {0: 0.4196, 1: 0.3689, 2: 0.3871, 3: 0.3712}
//   1024 kernels of n = 192: small path {0: 0.8183, 1: 0.8187, 2: 0.818, 3: 0.818}, blocked {0: 0.5001, 1: 0.4285, 2: 0.4501, 3: 0.4319}
//   -> kSmallCutover = [0, 0, 0, 0]
//   4096 L-ensembles, group width 64: {0: 24.4684, 2: 18.8064}
//   4096 L-ensembles, group width 128: {0: 25.6612, 2: 19.695}
//   4096 L-ensembles, group width 256: {0: 29.1797, 2: 20.371}
//   -> kGroupNarrow = 64
//   b0_ldlh_split kB0LdlhSplit = 2048: {2: 82.4463}
//   b0_ldlh_split kB0LdlhSplit = 4096: {2: 80.7221}
//   -> kB0LdlhSplit = 4096
//   b0_ldlh_fp64 kB0LdlhFp64 = 1024: {0: 217.4429}
//   b0_ldlh_fp64 kB0LdlhFp64 = 2048: {0: 212.4692}
//   b0_ldlh_fp64 kB0LdlhFp64 = 4096: {0: 210.3904}
//   -> kB0LdlhFp64 = 4096
//   b0_lu kB0Lu = 256: {0: 71.8761, 2: 37.8041}
//   b0_lu kB0Lu = 512: {0: 69.6748, 2: 34.6524}
//   b0_lu kB0Lu = 1024: {0: 73.3292, 2: 38.1667}
//   -> kB0Lu = 512
// LU outer panels as a binary tree (the same blocking as LDL^H), measured on
// the LU n = 8192 leg of the bench (32 samples; samples/s, split x3 / FP64):
//   kB0Lu = 512: 308.8 / 118.1 (64 columns at a time before: 267.5 / 113.9)
//   kB0Lu = 1024: 337.7 / 120.1
//   kB0Lu = 2048: 350.5 / 123.5
//   -> kB0Lu = 2048
#pragma once
#include <stdint.h>

namespace dpp {
namespace tuned {

// Outer panel width of real kernels (complex kernels: half as many complex
// columns): the trailing update re-reads the trailing matrix once per panel.
constexpr int kB0LdlhSplit = 4096;  // Hermitian, split-BF16 updates
constexpr int kB0LdlhFp64 = 4096;   // Hermitian, FP64 updates
constexpr int kB0Lu = 2048;         // LU

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
