"""The small-problem path: real Hermitian problems with n up to the tuned
cutover run in one workgroup each with the whole lower triangle in LDS (the
unblocked sampler of Sec. 2 as written, FP64 arithmetic). Oracle parity on
both sides of the cutover, every precision and both storage types; partial
problems (npiv) leave the conditional kernel as the blocked path does; a
batch mixing small and blocked problems equals the single calls."""
import re
import os

import numpy as np
import pytest

import oracle
from paper_1905_00165_amd import workloads as W
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TUNING = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1905_00165_amd", "csrc",
                      "tuning.h")


def _cutover():
    text = open(TUNING).read()
    return [int(x) for x in re.search(r"kSmallCutover\[3\] = \{([^}]*)\}", text).group(1).split(",")]


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding
    return binding


DEV = torch.device("cuda:0") if torch.cuda.is_available() else None
TOL = {0: (1e-9, 1e-10), 1: (1e-4, 1e-5), 2: (1e-4, 1e-5)}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "split", "split6"])
def test_parity_on_both_sides_of_the_cutover(B, prec, dtype):
    cut = _cutover()[prec]
    worst = 0.0
    for n in sorted({1, 2, 33, max(cut - 1, 1), max(cut, 1), cut + 1, cut + 64}):
        K = W.hermitian_kernel(n, seed=500 + n)
        u = W.uniform_stream(n, seed=50000 + n)
        Kw = K if dtype == torch.float64 else np.asarray(K).astype(np.float32).astype(np.float64)
        ref = oracle.ldlh(Kw, u)
        A = B.colmajor(K, device=DEV, dtype=dtype)
        out = B.dpp_sample_ldlh(A, torch.from_numpy(u).to(DEV), prec=prec)
        torch.cuda.synchronize()
        t, h = TOL[prec]
        if dtype == torch.float32 and (prec == 0 or n <= cut):
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
        err = float(np.max(np.abs(R[low] - target[low]))) if n else 0.0
        assert err <= (1e-12 if dtype == torch.float64 and (prec == 0 or n <= cut) else 1e-4), (n, err)
        worst = max(worst, v.max_dd)
    print(f"[accuracy] small path prec={prec} {dtype}: cutover {cut}, max |d - d_oracle| = {worst:.3e}")


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "split", "split6"])
def test_partial_small_problem_leaves_the_conditional_kernel(B, prec):
    cut = _cutover()[prec]
    if cut < 64:
        pytest.skip("small path off for this precision")
    n = min(cut, 128)
    K = W.hermitian_kernel(n, seed=510)
    u = W.uniform_stream(n, seed=51000)
    A = B.colmajor(K, device=DEV)
    out = B.dpp_sample_ldlh_batched([A], [torch.from_numpy(u).to(DEV)], prec=prec, npivs=[64])[0]
    torch.cuda.synchronize()
    ref = oracle.ldlh(K, u, npiv=64)
    got = A.cpu().numpy()
    low = np.tril(np.ones((n - 64, n - 64), dtype=bool))
    S_ref = oracle.conditional_kernel(K, ref["mask"][:64])
    assert np.array_equal(out["mask"].cpu().numpy()[:64], ref["mask"][:64])
    assert np.max(np.abs(got[64:, 64:][low] - S_ref[low])) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp64", "split", "split6"])
def test_mixed_batch_equals_single_calls(B, prec):
    cut = _cutover()[prec]
    ns = [5, max(cut, 1), cut + 1, 300, 40]
    Ks = [B.colmajor(W.hermitian_kernel(n, seed=520 + i), device=DEV) for i, n in enumerate(ns)]
    us = [torch.from_numpy(W.uniform_stream(n, seed=52000 + i)).to(DEV) for i, n in enumerate(ns)]
    As = [torch.empty_like(K) for K in Ks]
    outs = B.dpp_sample_ldlh_batched(As, us, prec=prec, Ks=Ks)
    torch.cuda.synchronize()
    for i, n in enumerate(ns):
        A1 = Ks[i].clone()
        single = B.dpp_sample_ldlh(A1, us[i], prec=prec)
        torch.cuda.synchronize()
        for key in ("mask", "pivots", "loglik", "info"):
            assert torch.equal(single[key], outs[i][key]), (n, key)
        low = torch.tril(torch.ones(n, n, dtype=torch.bool, device=DEV))
        assert torch.equal(A1[low], As[i][low])
