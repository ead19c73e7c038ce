"""GPU parity of the complex samplers (DPP_C128 storage) against the complex
FP64 oracle, through the C ABI: the complex Hermitian LDL^H form and the
complex LU form (the paper's complex kernels: the domino-tiling examples of
Sec. 1 and the dense complex LU experiment of Sec. 3).

Tolerances are those of the real paths (tests/test_gpu_parity.py): FP64
1e-9 (near-tie threshold 1e-10), split-BF16 1e-4 (threshold 1e-5), on the
pre-decision probabilities (real parts of the diagonal) and relative on the
log-likelihood; a mask difference is allowed only as a counted near tie.
Sizes cover one 32-column block, ragged tails, several blocks and tiles, and
(n = 2600 LDL^H, n = 700 LU) more than one outer panel.
"""
import numpy as np
import pytest

import oracle
from paper_1905_00165_amd import workloads as W
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {0: (1e-9, 1e-10), 1: (1e-4, 1e-5), 2: (1e-4, 1e-5)}
PRECS = [0, 1, 2]
PREC_ID = {0: "fp64", 1: "split", 2: "split6"}


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding
    return binding


DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def _run(B, herm, K, u, prec):
    A = B.colmajor(np.asarray(K), device=DEV, dtype=torch.complex128)
    ut = torch.from_numpy(np.ascontiguousarray(u)).to(DEV)
    fn = B.dpp_sample_ldlh if herm else B.dpp_sample_lu
    out = fn(A, ut, prec=prec)
    torch.cuda.synchronize()
    return {"mask": out["mask"].cpu().numpy(), "pivots": out["pivots"].cpu().numpy(),
            "loglik": float(out["loglik"].cpu()[0]), "info": int(out["info"].cpu()[0]),
            "A": A.cpu().numpy()}


def _check(B, herm, K, u, prec):
    t, h = TOL[prec]
    ref = (oracle.zldlh if herm else oracle.zlu)(K, u)
    got = _run(B, herm, K, u, prec)
    v = compare(got["mask"], got["pivots"], got["loglik"], ref, u, t, h)
    assert got["info"] == 0
    assert v.ok, v.why
    return v, got, ref


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("n", [1, 5, 31, 32, 33, 64, 65, 100, 257, 700])
def test_complex_ldlh_small_sizes(B, n, prec):
    K = W.complex_hermitian_kernel(n, seed=300 + n)
    u = W.uniform_stream(n, seed=30000 + n)
    _check(B, True, K, u, prec)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("n", [1, 5, 31, 32, 33, 64, 65, 100, 257, 700])
def test_complex_lu_small_sizes(B, n, prec):
    K, _ = W.complex_similarity_kernel(n, seed=310 + n)
    u = W.uniform_stream(n, seed=31000 + n)
    _check(B, False, K, u, prec)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_complex_similarity_samples_the_hermitian_law(B, prec):
    """Prop. 2: K = S H S^{-1} (complex diagonal S) gives the same decisions
    as H on a shared stream, up to a counted near tie; with a unit-modulus S
    the LU of K equals the LDL^H of H to rounding."""
    n = 600
    K, H = W.complex_similarity_kernel(n, seed=320)
    u = W.uniform_stream(n, seed=32000)
    lu = _run(B, False, K, u, prec)
    ld = _run(B, True, H, u, prec)
    t, h = TOL[prec]
    ref = {"mask": ld["mask"], "predec": ld["pivots"] + 1.0 - ld["mask"], "loglik": ld["loglik"]}
    v = compare(lu["mask"], lu["pivots"], lu["loglik"], ref, u, 2 * t, h)
    assert v.ok, v.why


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_aztec_diamond_tilings(B, prec):
    """The paper's order-10 Aztec diamond (Kenyon's kernel, complex and
    non-Hermitian): every GPU sample is a domino tiling (each square covered
    exactly once) with log-likelihood -(d(d+1)/2) ln 2 = -38.1231, as
    printed."""
    d = 10
    K, eb, ew, _ = W.aztec_diamond_kernel(d)
    n = K.shape[0]
    for s in range(4):
        u = W.uniform_stream(n, seed=33000 + s)
        got = _run(B, False, K, u, prec)
        assert got["info"] == 0
        m = got["mask"].astype(bool)
        assert m.sum() == d * (d + 1)
        assert np.array_equal(np.sort(eb[m]), np.arange(d * (d + 1)))
        assert np.array_equal(np.sort(ew[m]), np.arange(d * (d + 1)))
        assert got["loglik"] == pytest.approx(-d * (d + 1) / 2 * np.log(2), rel=1e-4 if prec else 1e-9)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_complex_factor_reconstructs(B, prec):
    """On exit A holds L and D of K - 1_{Y^c} = L D L^H (Hermitian form) and L,
    U of K - 1_{Y^c} = L U (LU form)."""
    n = 300
    K = W.complex_hermitian_kernel(n, seed=340)
    u = W.uniform_stream(n, seed=34000)
    got = _run(B, True, K, u, prec)
    target = np.array(K) - np.diag(1.0 - got["mask"])
    low = np.tril(np.ones((n, n), dtype=bool))
    err = np.max(np.abs(oracle.reconstruct_ldlh(got["A"])[low] - target[low]))
    Kl, _ = W.complex_similarity_kernel(n, seed=341)
    gl = _run(B, False, Kl, u, prec)
    errl = np.max(np.abs(oracle.reconstruct_lu(gl["A"]) - (np.array(Kl) - np.diag(1.0 - gl["mask"]))))
    print(f"[accuracy] complex prec={PREC_ID[prec]} reconstruction ldlh {err:.3e} lu {errl:.3e}")
    assert err <= (1e-10 if prec == 0 else 1e-4)
    assert errl <= (1e-10 if prec == 0 else 1e-4)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
def test_complex_past_the_outer_panel(B, herm, prec):
    """Sizes whose later pivots depend on trailing updates of a full outer
    panel (complex panels: 2048 (split) / 1024 (FP64) columns for LDL^H, 1024
    for LU), against whole oracle runs."""
    n = 2600 if herm else 1100
    K = W.complex_hermitian_kernel(n, seed=350) if herm else W.complex_similarity_kernel(n, seed=351)[0]
    u = W.uniform_stream(n, seed=35000)
    v, _, _ = _check(B, herm, K, u, prec)
    print(f"[accuracy] complex {'ldlh' if herm else 'lu'} n={n} prec={PREC_ID[prec]}: "
          f"max |d - d_oracle| = {v.max_dd:.3e}, |dll|/|ll| = {v.ll_rel:.3e}")


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
def test_complex_batched_out_of_place_equals_single(B, herm, prec):
    """A batch of uneven complex problems read out of place from resident
    kernels equals the single in-place calls bit for bit."""
    ns = [100, 33, 257, 1]
    Ks = [W.complex_hermitian_kernel(n, seed=360 + i) if herm else
          W.complex_similarity_kernel(n, seed=360 + i)[0] for i, n in enumerate(ns)]
    us = [torch.from_numpy(W.uniform_stream(n, seed=36000 + i)).to(DEV) for i, n in enumerate(ns)]
    src = [B.colmajor(K, device=DEV, dtype=torch.complex128) for K in Ks]
    As = [torch.empty_like(K) for K in src]
    fb = B.dpp_sample_ldlh_batched if herm else B.dpp_sample_lu_batched
    outs = fb(As, us, prec=prec, Ks=src)
    torch.cuda.synchronize()
    fs = B.dpp_sample_ldlh if herm else B.dpp_sample_lu
    for i, n in enumerate(ns):
        A1 = src[i].clone()
        single = fs(A1, us[i], prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(single["mask"], outs[i]["mask"])
        assert torch.equal(single["pivots"], outs[i]["pivots"])
        assert torch.equal(single["loglik"], outs[i]["loglik"])
        part = torch.tril(torch.ones(n, n, dtype=torch.bool, device=DEV)) if herm else \
            torch.ones(n, n, dtype=torch.bool, device=DEV)
        assert torch.equal(A1[part], As[i][part])
