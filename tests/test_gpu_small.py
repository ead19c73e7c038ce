"""The small-problem path: real Hermitian problems with n up to the cutover run
in one workgroup each with the whole lower triangle in registers (the
unblocked sampler of Sec. 2 as written, FP64 arithmetic). The tuned cutover
may turn the path off; these tests set it through DPP_SMALL_CUTOVER (read by
the library at every call) and check through the library's profiler that the
path ran exactly for the problems at or below it. Oracle parity on both sides
of the cutover, every precision and both storage types; partial problems
(npiv) leave the conditional kernel as the blocked path does; a batch mixing
small and blocked problems equals the single calls."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_1905_00165_amd import workloads as W
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding
    return binding


@pytest.fixture
def cutover():
    """Sets DPP_SMALL_CUTOVER for one test and restores it afterwards."""
    old = os.environ.get("DPP_SMALL_CUTOVER")

    def set_(v):
        os.environ["DPP_SMALL_CUTOVER"] = str(v)
        return v
    yield set_
    if old is None:
        os.environ.pop("DPP_SMALL_CUTOVER", None)
    else:
        os.environ["DPP_SMALL_CUTOVER"] = old


DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
TOL = {0: (1e-9, 1e-10), 1: (1e-4, 1e-5), 2: (1e-4, 1e-5), 3: (1e-4, 1e-5)}


@pytest.mark.parametrize("cut", [128, 192])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["fp64", "split", "split6", "fp16"])
def test_parity_on_both_sides_of_the_cutover(B, cutover, prec, dtype, cut):
    cutover(cut)
    worst = 0.0
    for n in sorted({1, 2, 33, 64, 100, cut - 1, cut, cut + 1, cut + 64}):
        K = W.hermitian_kernel(n, seed=500 + n)
        u = W.uniform_stream(n, seed=50000 + n)
        Kw = K if dtype == torch.float64 else np.asarray(K).astype(np.float32).astype(np.float64)
        ref = oracle.ldlh(Kw, u)
        A = B.colmajor(K, device=DEV, dtype=dtype)
        B.dpp_profile_begin()
        out = B.dpp_sample_ldlh(A, torch.from_numpy(u).to(DEV), prec=prec)
        torch.cuda.synchronize()
        prof = B.dpp_profile_end()
        small = n <= cut
        assert prof.get("small_ldlh", {}).get("launches", 0) == (1 if small else 0), (n, prof)
        t, h = TOL[prec]
        if dtype == torch.float32 and (prec == 0 or small):
            t, h = 1e-5, 1e-6   # FP32 storage: the stored kernel's rounding
        v = compare(out["mask"].cpu().numpy(), out["pivots"].cpu().numpy(),
                    float(out["loglik"].cpu()[0]), ref, u, t, h)
        assert int(out["info"].item()) == 0
        assert v.ok, (n, v.why)
        # the factor: L D L^T = K - 1_{Y^c} on the lower triangle
        F = A.cpu().numpy().astype(np.float64)
        R = oracle.reconstruct_ldlh(F)
        target = Kw - np.diag(1.0 - out["mask"].cpu().numpy())
        low = np.tril(np.ones((n, n), dtype=bool))
        err = float(np.max(np.abs(R[low] - target[low])))
        assert err <= (1e-12 if dtype == torch.float64 and (prec == 0 or small) else 1e-4), (n, err)
        worst = max(worst, v.max_dd)
    print(f"[accuracy] small path prec={prec} {dtype}: cutover {cut}, max |d - d_oracle| = {worst:.3e}")


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["fp64", "split", "split6", "fp16"])
def test_partial_small_problem_leaves_the_conditional_kernel(B, cutover, prec):
    cutover(192)
    for n in (65, 128, 192):
        K = W.hermitian_kernel(n, seed=510)
        u = W.uniform_stream(n, seed=51000)
        A = B.colmajor(K, device=DEV)
        out = B.dpp_sample_ldlh_batched([A], [torch.from_numpy(u).to(DEV)], prec=prec,
                                        npivs=[64])[0]
        torch.cuda.synchronize()
        ref = oracle.ldlh(K, u, npiv=64)
        got = A.cpu().numpy()
        low = np.tril(np.ones((n - 64, n - 64), dtype=bool))
        S_ref = oracle.conditional_kernel(K, ref["mask"][:64])
        assert np.array_equal(out["mask"].cpu().numpy()[:64], ref["mask"][:64])
        assert np.max(np.abs(got[64:, 64:][low] - S_ref[low])) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["fp64", "split", "split6", "fp16"])
def test_mixed_batch_equals_single_calls(B, cutover, prec):
    cut = cutover(128)
    ns = [5, cut, cut + 1, 300, 40, 1]
    Ks = [B.colmajor(W.hermitian_kernel(n, seed=520 + i), device=DEV) for i, n in enumerate(ns)]
    us = [torch.from_numpy(W.uniform_stream(n, seed=52000 + i)).to(DEV) for i, n in enumerate(ns)]
    As = [torch.empty_like(K) for K in Ks]
    B.dpp_profile_begin()
    outs = B.dpp_sample_ldlh_batched(As, us, prec=prec, Ks=Ks)
    torch.cuda.synchronize()
    assert B.dpp_profile_end()["small_ldlh"]["launches"] == 1
    for i, n in enumerate(ns):
        A1 = Ks[i].clone()
        single = B.dpp_sample_ldlh(A1, us[i], prec=prec)
        torch.cuda.synchronize()
        for key in ("mask", "pivots", "loglik", "info"):
            assert torch.equal(single[key], outs[i][key]), (n, key)
        low = torch.tril(torch.ones(n, n, dtype=torch.bool, device=DEV))
        assert torch.equal(A1[low], As[i][low])


def _tuned_cutover(prec):
    path = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1905_00165_amd", "csrc",
                        "tuning.h")
    m = re.search(r"kSmallCutover\[4\] = \{([^}]*)\}", open(path).read())
    return [int(x) for x in m.group(1).split(",")][prec]


@pytest.mark.parametrize("value", ["100000", "-1", "abc", "64x"])
def test_invalid_override_is_ignored(B, cutover, value):
    """A value that is not a decimal in 0..192 leaves the tuned cutover in force."""
    cutover(value)
    n = 100
    K = B.colmajor(W.hermitian_kernel(n, seed=530), device=DEV)
    u = torch.from_numpy(W.uniform_stream(n, seed=53000)).to(DEV)
    B.dpp_profile_begin()
    out = B.dpp_sample_ldlh(K, u)
    torch.cuda.synchronize()
    ran = "small_ldlh" in B.dpp_profile_end()
    assert ran == (n <= _tuned_cutover(0))
    assert int(out["info"].item()) == 0
