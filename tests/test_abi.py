"""The C ABI library loads and exports every function include/dpp.h declares,
and rejects bad arguments synchronously. No GPU needed: every call here fails
its argument checks before any device work."""
import ctypes
import os
import re

import pytest

from paper_1905_00165_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "dpp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["dpp_sample_ldlh", "dpp_sample_lu", "dpp_sample_ldlh_batched",
                 "dpp_sample_lu_batched", "dpp_workspace_size", "dpp_workspace_size_batched",
                 "dpp_status_string", "dpp_profile_begin", "dpp_profile_end"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    for s in range(5):
        assert B.dpp_status_string(s)
    assert B.dpp_status_string(99) == "unknown status"


def test_workspace_sizes():
    assert B.dpp_workspace_size(True, B.DPP_F64, 0, B.DPP_PREC_FP64) == 0
    assert B.dpp_workspace_size(True, 7, 10, B.DPP_PREC_FP64) == 0
    fp = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_FP64)
    sp = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_SPLIT_BF16)
    assert 0 < fp < sp
    # split copies: 4 planes of n x (outer panel width) bf16
    assert sp - fp >= 4 * 1000 * 512 * 2
    b = B.dpp_workspace_size_batched(True, B.DPP_F64, [100, 200], B.DPP_PREC_SPLIT_BF16)
    assert b >= (B.dpp_workspace_size(True, B.DPP_F64, 100, B.DPP_PREC_SPLIT_BF16) +
                 B.dpp_workspace_size(True, B.DPP_F64, 200, B.DPP_PREC_SPLIT_BF16) - 1024)
    assert B.dpp_workspace_size_batched(True, B.DPP_F64, [100, 0], B.DPP_PREC_FP64) == 0
    # The split copies are no wider than the largest problem (rounded up to
    # 64 columns), with rows padded to blocks of 32: n = 100 alone needs 4
    # planes of 128 x 128.
    s100 = B.dpp_workspace_size(True, B.DPP_F64, 100, B.DPP_PREC_SPLIT_BF16)
    f100 = B.dpp_workspace_size(True, B.DPP_F64, 100, B.DPP_PREC_FP64)
    assert s100 - f100 == (4 * 128 * 128 * 2 + 255) // 256 * 256
    # ... and in a batch, as wide as the batch's largest problem.
    b2 = B.dpp_workspace_size_batched(True, B.DPP_F64, [100, 1000], B.DPP_PREC_SPLIT_BF16)
    f2 = B.dpp_workspace_size_batched(True, B.DPP_F64, [100, 1000], B.DPP_PREC_FP64)
    assert b2 - f2 == sum((4 * ((n + 31) // 32 * 32) * 1024 * 2 + 255) // 256 * 256 for n in (100, 1000))
    assert B.dpp_workspace_size(True, B.DPP_F64, (1 << 20) + 1, B.DPP_PREC_FP64) == 0


@pytest.mark.parametrize("name", ["dpp_sample_ldlh", "dpp_sample_lu"])
def test_argument_errors_return_before_any_launch(name):
    f = getattr(B.lib(), name)
    p = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    ws = ctypes.c_void_p(0x2000)
    big = 1 << 40
    # n < 1
    assert f(p, 0, 0, 1, p, p, p, p, p, 0, ws, big, None) == 1
    # lda < n, lda > 2^20
    assert f(p, 0, 10, 9, p, p, p, p, p, 0, ws, big, None) == 1
    assert f(p, 0, 10, (1 << 20) + 1, p, p, p, p, p, 0, ws, big, None) == 1
    # null A / u / outputs
    assert f(None, 0, 10, 10, p, p, p, p, p, 0, ws, big, None) == 1
    assert f(p, 0, 10, 10, None, p, p, p, p, 0, ws, big, None) == 1
    assert f(p, 0, 10, 10, p, p, p, p, None, 0, ws, big, None) == 1
    # bad enums
    assert f(p, 5, 10, 10, p, p, p, p, p, 0, ws, big, None) == 1
    assert f(p, 0, 10, 10, p, p, p, p, p, 9, ws, big, None) == 1
    # workspace
    assert f(p, 0, 10, 10, p, p, p, p, p, 0, None, big, None) == 2
    assert f(p, 0, 10, 10, p, p, p, p, p, 1, ws, 16, None) == 2


def test_copy_lower_argument_errors():
    f = B.lib().dpp_copy_lower
    p = ctypes.c_void_p(0x1000)
    assert f(None, p, 0, 10, 10, 10, None) == 1
    assert f(p, p, 0, 0, 10, 10, None) == 1
    assert f(p, p, 0, 10, 9, 10, None) == 1
    assert f(p, p, 0, 10, 10, (1 << 20) + 1, None) == 1
    assert f(p, p, 7, 10, 10, 10, None) == 1


def test_batched_argument_errors():
    lib = B.lib()
    p = 0x1000
    probs = (B.dpp_problem * 2)(B.dpp_problem(p, 10, 10, p, p, p, p, p),
                                B.dpp_problem(p, 10, 8, p, p, p, p, p))
    assert lib.dpp_sample_ldlh_batched(probs, 2, 0, 0, ctypes.c_void_p(p), 1 << 40, None) == 1
    assert lib.dpp_sample_lu_batched(probs, 0, 0, 0, ctypes.c_void_p(p), 1 << 40, None) == 1
    assert lib.dpp_sample_lu_batched(None, 1, 0, 0, ctypes.c_void_p(p), 1 << 40, None) == 1


def test_out_of_place_source_errors():
    """A source K needs n <= ldk <= 2^20 and storage disjoint from A (K == A
    with ldk == lda is the in-place call)."""
    lib = B.lib()
    p, n = 0x100000, 10
    ws = ctypes.c_void_p(p)

    def call(K, ldk, lda=n):
        probs = (B.dpp_problem * 1)(B.dpp_problem(p, n, lda, p, p, p, p, p, K, ldk))
        return lib.dpp_sample_ldlh_batched(probs, 1, 0, 0, ws, 1 << 40, None)

    assert call(p + 8 * 50, n) == 1              # overlaps A's n x n footprint
    assert call(p - 8 * 50, n) == 1              # A starts inside K
    assert call(p + 8 * 200, n - 1) == 1         # ldk < n
    assert call(p + 8 * 200, (1 << 20) + 1) == 1  # ldk > 2^20
    assert call(p, n + 1) == 1                   # K == A with another leading dimension


def test_partial_and_lensemble_argument_errors():
    """npiv must be 0, n, or a multiple of 64 below n; an L-ensemble output may
    not overlap its input unless it is the same buffer with the same leading
    dimension; sizes whose augmented matrix exceeds 2^20 are refused."""
    lib = B.lib()
    p, n = 0x100000, 200
    ws = ctypes.c_void_p(p)
    for bad in (-64, 100, n + 64):
        probs = (B.dpp_problem * 1)(B.dpp_problem(p, n, n, p, p, p, p, p, None, 0, bad))
        assert lib.dpp_sample_ldlh_batched(probs, 1, 0, 0, ws, 1 << 40, None) == 1
    q = (B.dpp_lensemble * 1)(B.dpp_lensemble(p, 10, 10, p + 8 * 40, 10, None, p))
    assert lib.dpp_lensemble_to_marginal_batched(q, 1, 0, ws, 1 << 40, None) == 1
    q = (B.dpp_lensemble * 1)(B.dpp_lensemble(p, 10, 10, p, 12, None, p))
    assert lib.dpp_lensemble_to_marginal_batched(q, 1, 0, ws, 1 << 40, None) == 1
    assert B.dpp_lensemble_workspace_size([(1 << 19) + 1]) == 0
    assert B.dpp_lensemble_workspace_size([100]) > 32 * 128 * 128


def test_profile_without_launches_is_empty():
    B.dpp_profile_begin()
    assert B.dpp_profile_end() == {}


def test_misaligned_workspace_is_refused():
    """The workspace must be 256-byte aligned (the split planes take 16-byte
    stores and direct-to-LDS reads); an offset into an arena is refused before
    any launch."""
    lib = B.lib()
    p = 0x100000
    probs = (B.dpp_problem * 1)(B.dpp_problem(p, 10, 10, p, p, p, p, p))
    for off in (8, 16, 128):
        assert lib.dpp_sample_ldlh_batched(probs, 1, 0, 0, ctypes.c_void_p(p + off), 1 << 40,
                                           None) == 1
        assert lib.dpp_sample_lu_batched(probs, 1, 0, 1, ctypes.c_void_p(p + off), 1 << 40,
                                         None) == 1
    f = lib.dpp_sample_ldlh
    assert f(ctypes.c_void_p(p), 0, 10, 10, ctypes.c_void_p(p), ctypes.c_void_p(p),
             ctypes.c_void_p(p), ctypes.c_void_p(p), ctypes.c_void_p(p), 0,
             ctypes.c_void_p(p + 64), 1 << 40, None) == 1
    q = (B.dpp_lensemble * 1)(B.dpp_lensemble(p, 10, 10, p, 10, None, p))
    assert lib.dpp_lensemble_to_marginal_batched(q, 1, 0, ctypes.c_void_p(p + 8), 1 << 40,
                                                 None) == 1


def test_binding_checks_output_buffers_and_streams():
    """Outputs and streams on the wrong device, of the wrong dtype or too short
    are refused by the binding before the library sees a pointer (a host
    buffer would otherwise reach the kernels)."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cpu")
    ok = {"mask": torch.empty(5, dtype=torch.uint8), "pivots": torch.empty(5, dtype=torch.float64),
          "loglik": torch.empty(1, dtype=torch.float64), "info": torch.empty(1, dtype=torch.int32),
          "stats": torch.empty(3, dtype=torch.float64)}
    B.check_outputs(ok, 5, dev)
    bad = [("mask", torch.empty(5, dtype=torch.uint8, device="meta")),     # other device
           ("pivots", torch.empty(5, dtype=torch.float32)),               # dtype
           ("pivots", torch.empty(4, dtype=torch.float64)),               # too short
           ("info", torch.empty(1, dtype=torch.int64)),
           ("stats", torch.empty(2, dtype=torch.float64)),
           ("mask", torch.empty(10, dtype=torch.uint8)[::2])]             # not contiguous
    for key, t in bad:
        o = dict(ok)
        o[key] = t
        with pytest.raises(ValueError):
            B.check_outputs(o, 5, dev)
    with pytest.raises(ValueError):
        B.check_outputs({"extra": torch.empty(1)}, 5, dev)
    B.check_stream(torch.empty(5, dtype=torch.float64), 5, dev)
    for u in (torch.empty(5, dtype=torch.float64, device="meta"), torch.empty(5),
              torch.empty(4, dtype=torch.float64), torch.empty(10, dtype=torch.float64)[::2]):
        with pytest.raises(ValueError):
            B.check_stream(u, 5, dev)


def test_six_product_workspace_holds_six_planes():
    """DPP_PREC_SPLIT_BF16X6 keeps three BF16 pieces of L and of W: six planes
    where the three-product form keeps four."""
    f = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_FP64)
    s3 = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_SPLIT_BF16)
    s6 = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_SPLIT_BF16X6)
    planes = 1024 * 1024 * 2   # rows padded to 32, columns to the 64-wide blocks
    assert s3 - f == 4 * planes and s6 - f == 6 * planes
    assert B.dpp_workspace_size(True, B.DPP_F64, 1000, 4) == 0   # unknown precision


def test_fp16_workspace_holds_four_planes_and_row_factors():
    """DPP_PREC_SPLIT_FP16 keeps two FP16 pieces of L and of W (four planes)
    and one FP32 factor per row, side and 64-column block; it serves real
    Hermitian problems only (LU and complex kernels: size 0, i.e. invalid)."""
    f = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_FP64)
    s16 = B.dpp_workspace_size(True, B.DPP_F64, 1000, B.DPP_PREC_SPLIT_FP16)
    planes = 1024 * 1024 * 2
    factors = 2 * (1024 // 64) * 1024 * 4   # sides x blocks x padded rows x FP32
    assert s16 - f == 4 * planes + factors
    assert B.dpp_workspace_size(True, B.DPP_F32, 1000, B.DPP_PREC_SPLIT_FP16) > 0
    assert B.dpp_workspace_size(False, B.DPP_F64, 1000, B.DPP_PREC_SPLIT_FP16) == 0
    assert B.dpp_workspace_size(True, B.DPP_C128, 1000, B.DPP_PREC_SPLIT_FP16) == 0
    assert B.dpp_workspace_size(False, B.DPP_C128, 1000, B.DPP_PREC_SPLIT_FP16) == 0


def test_noalloc_argument_errors_return_before_any_launch():
    """The no-allocation entry point checks its arguments, and that the batch
    fits the library's scratch, before touching the device."""
    f = B.lib().dpp_sample_ldlh_batched_noalloc
    p = ctypes.c_void_p(0x1000)
    ok = B.dpp_problem(p, 100, 100, p, p, p, p, p, None, 0, 0, None)
    arr = (B.dpp_problem * 1)(ok)
    assert f(None, 1, 0, 0, None) == 1                 # no descriptors
    assert f(arr, 0, 0, 0, None) == 1                  # count < 1
    assert f(arr, 1, 0, 7, None) == 1                  # unknown precision
    assert f(arr, 1, 5, 0, None) == 1                  # unknown dtype
    bad = (B.dpp_problem * 1)(B.dpp_problem(p, 0, 100, p, p, p, p, p, None, 0, 0, None))
    assert f(bad, 1, 0, 0, None) == 1                  # n < 1
    # one six-product problem of n = 3072 needs more than the 64 MiB scratch
    big = (B.dpp_problem * 1)(B.dpp_problem(p, 3072, 3072, p, p, p, p, p, None, 0, 0, None))
    assert B.dpp_workspace_size(True, B.DPP_F64, 3072, 2) > B.DPP_NOALLOC_SCRATCH_BYTES
    assert f(big, 1, 0, 2, None) == 2                  # DPP_ERR_WORKSPACE
    # the largest single problems the header states for each precision
    cap = B.DPP_NOALLOC_SCRATCH_BYTES
    for prec, nmax in ((0, 131008), (1, 2848), (2, 2304), (3, 2816)):
        assert 0 < B.dpp_workspace_size_batched(True, B.DPP_F64, [nmax], prec) <= cap, prec
        assert B.dpp_workspace_size_batched(True, B.DPP_F64, [nmax + 1], prec) > cap, prec
    assert f(big, 1, 0, 4, None) == 1                  # precision 4 is not defined


def test_complex_workspace_and_arguments():
    """Complex storage (DPP_C128): diagonal blocks of 32 x 32 complex entries
    (16 KiB each), split planes holding two real rows of L' per complex row;
    leading dimensions up to 2^19; partial problems in multiples of 32."""
    n = 1000
    f = B.dpp_workspace_size(True, B.DPP_C128, n, B.DPP_PREC_FP64)
    # one 256-byte descriptor slot, then the strip of diagonal blocks
    assert f == 256 + ((n + 31) // 32) * 32 * 32 * 16
    s3 = B.dpp_workspace_size(True, B.DPP_C128, n, B.DPP_PREC_SPLIT_BF16)
    ss = 2 * 1024   # real k columns of a 1024-wide complex panel (the whole n rounded to 32)
    # two pieces of L' (2n rows, padded to 32) and of W' (n rows, padded)
    assert s3 - f == 2 * (2016 + 1024) * ss * 2
    assert B.dpp_workspace_size(True, B.DPP_C128, (1 << 19) + 1, B.DPP_PREC_FP64) == 0
    f = B.lib().dpp_sample_ldlh_batched
    p = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x2000)
    bad_lda = (B.dpp_problem * 1)(B.dpp_problem(p, 10, (1 << 19) + 1, p, p, p, p, p, None, 0, 0, None))
    assert f(bad_lda, 1, B.DPP_C128, 0, ws, 1 << 40, None) == 1
    bad_npiv = (B.dpp_problem * 1)(B.dpp_problem(p, 100, 100, p, p, p, p, p, None, 0, 48, None))
    assert f(bad_npiv, 1, B.DPP_C128, 0, ws, 1 << 40, None) == 1
