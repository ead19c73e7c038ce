"""GPU parity: the HIP sampler against the FP64 oracle, element by element, on
the same seeded inputs and uniform streams, through the C ABI.

Tolerances (per run):
  FP64 path: pre-decision probabilities |d_gpu - d_oracle| <= 1e-9 and
             |ll_gpu - ll_oracle| <= 1e-9 |ll_oracle|; near-tie threshold 1e-10.
  split-BF16 paths (three and six products) and the FP16 form (real
             Hermitian only): 1e-4 and near-tie threshold 1e-5.
  FP32 storage (FP64 updates): 1e-5, threshold 1e-6 (each stored Schur
             complement entry is rounded to FP32, relative 6e-8 per step).
A mask difference is allowed only as a counted near tie (tests/parity.py).
"""
import numpy as np
import pytest

import oracle
from paper_1905_00165_amd import workloads as W
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = None
DEV = None


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    global B, DEV
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding
    B = binding
    DEV = torch.device("cuda:0")
    yield


TOL = {0: (1e-9, 1e-10), 1: (1e-4, 1e-5), 2: (1e-4, 1e-5), 3: (1e-4, 1e-5)}
PRECS = [0, 1, 2, 3]
PRECS_LU = [0, 1, 2]
PREC_ID = {0: "fp64", 1: "split", 2: "split6", 3: "fp16"}


def _need(herm, prec):
    if prec == 3 and not herm:
        pytest.skip("the FP16 form serves real Hermitian problems; LU rejects it "
                    "(test_fp16_form_rejects_lu_and_complex)")


def _run(herm, K, u, prec, dtype=torch.float64):
    _need(herm, prec)
    A = B.colmajor(np.asarray(K), device=DEV, dtype=dtype)
    ut = torch.from_numpy(np.ascontiguousarray(u)).to(DEV)
    fn = B.dpp_sample_ldlh if herm else B.dpp_sample_lu
    out = fn(A, ut, prec=prec)
    torch.cuda.synchronize()
    return {"mask": out["mask"].cpu().numpy(), "pivots": out["pivots"].cpu().numpy(),
            "loglik": float(out["loglik"].cpu()[0]), "info": int(out["info"].cpu()[0]),
            "A": A.cpu().numpy()}


def _check(herm, K, u, prec, tol=None, thr=None, dtype=torch.float64):
    t, h = TOL[prec]
    tol = tol or t
    thr = thr or h
    Kw = np.asarray(K, dtype=np.float64) if dtype == torch.float64 else \
        np.asarray(K).astype(np.float32).astype(np.float64)
    ref = (oracle.ldlh if herm else oracle.lu)(Kw, u)
    got = _run(herm, K, u, prec, dtype=dtype)
    v = compare(got["mask"], got["pivots"], got["loglik"], ref, u, tol, thr)
    assert got["info"] == 0
    assert v.ok, v.why
    return v, got, ref


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 127, 129, 200, 300, 513, 777])
def test_ldlh_small_sizes(n, prec):
    K = W.hermitian_kernel(n, seed=10 + n)
    u = W.uniform_stream(n, seed=20 + n)
    _check(True, K, u, prec)


@pytest.mark.parametrize("prec", PRECS_LU, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 200, 300, 513])
def test_lu_small_sizes(n, prec):
    K, _ = W.similarity_kernel(n, seed=30 + n)
    u = W.uniform_stream(n, seed=40 + n)
    _check(False, K, u, prec)


@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_greedy_mode(herm, prec):
    """u = 1/2 everywhere (greedy maximum-likelihood mode): the decisions,
    pivots and log-likelihood match the oracle's greedy run at n = 700 (ten
    full blocks and a ragged one), Hermitian K and a diagonal similarity of it."""
    n = 700
    K = W.hermitian_kernel(n, seed=16)
    if not herm:
        s = np.exp(np.random.default_rng(17).normal(0.0, 0.5, size=n))
        K = np.asfortranarray((s[:, None] * K) / s[None, :])
    v, got, _ = _check(herm, K, W.greedy_stream(n), prec)
    assert 0 < int(got["mask"].sum()) < n


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_ldlh_dense_kernel_n1024_streams(prec):
    """The plain workload at n = 1024: K = Q diag(lam) Q^T, lam ~ U(0,1)."""
    K = W.hermitian_kernel(1024, seed=1)
    ties = 0
    for s in range(6):
        u = W.uniform_stream(1024, seed=1000 + s)
        v, _, _ = _check(True, K, u, prec)
        ties += v.near_tie
    assert ties <= 1


@pytest.mark.parametrize("prec", PRECS_LU, ids=lambda p: PREC_ID[p])
def test_lu_similarity_kernel_n1024(prec):
    """K = S H S^-1 sampled by the LU path matches the oracle, and its mask
    equals the LDL^H path's on H (Prop. 2)."""
    K, H = W.similarity_kernel(1024, seed=3)
    u = W.uniform_stream(1024, seed=3000)
    v, got, ref = _check(False, K, u, prec)
    gh = _run(True, H, u, prec)
    # Prop. 2 on the GPU alone: the LU run on K against the LDL^H run on H,
    # each within the tolerance of the oracle, so within twice it of each other
    t, h = TOL[prec]
    w = compare(got["mask"], got["pivots"], got["loglik"],
                {"mask": gh["mask"], "predec": gh["pivots"] + 1.0 - gh["mask"],
                 "loglik": gh["loglik"]}, u, 2 * t, h)
    assert w.ok, w.why


def test_fp32_storage_lensemble():
    """FP32-stored L-ensemble marginal kernel; FP64 decisions and updates."""
    K = W.lensemble_kernel(300, seed=4)
    u = W.uniform_stream(300, seed=4000)
    _check(True, K, u, 0, tol=1e-5, thr=1e-6, dtype=torch.float32)


def test_fp32_storage_split():
    K = W.lensemble_kernel(700, seed=5)
    u = W.uniform_stream(700, seed=5000)
    _check(True, K, u, 1, tol=1e-4, thr=1e-5, dtype=torch.float32)


@pytest.mark.parametrize("prec", PRECS_LU, ids=lambda p: PREC_ID[p])
def test_fp32_storage_lu(prec):
    """LU on an FP32-stored non-symmetric kernel (a diagonal similarity, n =
    700: ten full blocks and a ragged one) against the oracle on the same
    FP32 values widened to FP64."""
    K, _ = W.similarity_kernel(700, seed=6)
    u = W.uniform_stream(700, seed=6000)
    tol, thr = (1e-5, 1e-6) if prec == 0 else (1e-4, 1e-5)
    _check(False, K, u, prec, tol=tol, thr=thr, dtype=torch.float32)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_factor_reconstructs_k_minus_indicator(prec):
    n = 500
    K = W.hermitian_kernel(n, seed=6)
    u = W.uniform_stream(n, seed=6000)
    got = _run(True, K, u, prec)
    R = oracle.reconstruct_ldlh(got["A"])
    target = K - np.diag(1.0 - got["mask"])
    err = np.max(np.abs(np.tril(R) - np.tril(target)))
    assert err <= (1e-10 if prec == 0 else 1e-4)
    # the decision rule on the GPU's own probabilities
    d = got["pivots"] + 1.0 - got["mask"]
    assert np.array_equal(got["mask"], (u < d).astype(np.uint8))


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_projection_sample_size(prec):
    n, k = 1024, 256
    K = W.projection_kernel(n, k, seed=7)
    for s in range(4):
        got = _run(True, K, W.uniform_stream(n, seed=7000 + s), prec)
        assert int(got["mask"].sum()) == k


def test_zero_pivot_sets_info():
    K = np.diag([0.5, 1.0, 0.25])
    got = _run(True, K, np.array([0.1, 1.0, 0.1]), 0)
    assert got["info"] == 2
    assert got["pivots"][1] == 0.0
    assert not np.isfinite(got["loglik"])


def test_lda_padding_untouched():
    n, pad = 150, 5
    K = W.hermitian_kernel(n, seed=8)
    u = W.uniform_stream(n, seed=8000)
    storage = torch.full((n, n + pad), 7.0, dtype=torch.float64, device=DEV)
    storage[:, :n] = torch.as_tensor(K.T, device=DEV)
    A = storage.t()[:n, :]  # column-major view, lda = n + pad
    assert A.stride() == (1, n + pad)
    out = B.dpp_sample_ldlh(A, torch.from_numpy(u).to(DEV), prec=0)
    torch.cuda.synchronize()
    full = storage.cpu().numpy()
    assert np.all(full[:, n:] == 7.0)
    ref = oracle.ldlh(K, u)
    v = compare(out["mask"].cpu().numpy(), out["pivots"].cpu().numpy(),
                float(out["loglik"].cpu()[0]), ref, u, 1e-9, 1e-10)
    assert v.ok, v.why


@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_largest_leading_dimension(herm, prec):
    """lda = 2^20, the documented maximum (strips of 256 columns then span
    just under 2^31 bytes): the results match the oracle and sampled padding
    entries are untouched."""
    _need(herm, prec)
    n, lda = 300, 1 << 20
    K = W.hermitian_kernel(n, seed=14) if herm else W.similarity_kernel(n, seed=14)[0]
    u = W.uniform_stream(n, seed=1400)
    storage = torch.full((n, lda), 3.0, dtype=torch.float64, device=DEV)
    storage[:, :n] = torch.as_tensor(np.ascontiguousarray(K.T), device=DEV)
    A = storage.t()[:n, :]
    assert A.stride() == (1, lda)
    fn = B.dpp_sample_ldlh if herm else B.dpp_sample_lu
    out = fn(A, torch.from_numpy(u).to(DEV), prec=prec)
    torch.cuda.synchronize()
    ref = (oracle.ldlh if herm else oracle.lu)(K, u)
    tol, thr = TOL[prec]
    v = compare(out["mask"].cpu().numpy(), out["pivots"].cpu().numpy(),
                float(out["loglik"].cpu()[0]), ref, u, tol, thr)
    assert int(out["info"].cpu()[0]) == 0
    assert v.ok, v.why
    cols = torch.tensor([n, n + 1, 4096, lda // 2, lda - 1], device=DEV)
    assert bool(torch.all(storage[:, cols] == 3.0))
    del storage


@pytest.mark.parametrize("ns", [[100, 257, 64, 1], [700, 1000, 300, 129, 1100]],
                         ids=["small", "uneven"])
@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_batched_equals_single_bitwise(herm, prec, ns):
    """Each problem of a batch with uneven sizes equals its single call bit for
    bit (the blocking never depends on the other sizes in the batch)."""
    _need(herm, prec)
    Ks = [W.hermitian_kernel(n, seed=90 + n) if herm else W.similarity_kernel(n, seed=90 + n)[0]
          for n in ns]
    us = [W.uniform_stream(n, seed=9000 + n) for n in ns]
    As = [B.colmajor(K, device=DEV) for K in Ks]
    uts = [torch.from_numpy(u).to(DEV) for u in us]
    fb = B.dpp_sample_ldlh_batched if herm else B.dpp_sample_lu_batched
    outs = fb(As, uts, prec=prec)
    torch.cuda.synchronize()
    for K, u, A, o in zip(Ks, us, As, outs):
        single = _run(herm, K, u, prec)
        assert np.array_equal(o["mask"].cpu().numpy(), single["mask"])
        assert np.array_equal(o["pivots"].cpu().numpy(), single["pivots"])
        assert float(o["loglik"].cpu()[0]) == single["loglik"]
        assert np.array_equal(A.cpu().numpy(), single["A"])


@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_out_of_place_equals_in_place(herm, prec):
    """With a read-only source K per problem (two problems sharing one K, a
    padded leading dimension on another), each A receives exactly the in-place
    factor (the lower triangle for LDL^H, whose strict upper triangle of A is
    left unwritten), the outputs match bit for bit, and K is unchanged."""
    _need(herm, prec)
    ns = [700, 700, 1100, 129]
    Ks = [W.hermitian_kernel(n, seed=60 + i) if herm else W.similarity_kernel(n, seed=60 + i)[0]
          for i, n in enumerate(ns)]
    Ks[1] = Ks[0]
    us = [W.uniform_stream(n, seed=6000 + i) for i, n in enumerate(ns)]
    src = [B.colmajor(K, device=DEV) for K in Ks]
    src[1] = src[0]                                   # shared source
    pad = torch.zeros((ns[2], ns[2] + 3), dtype=torch.float64, device=DEV)
    pad[:, : ns[2]] = src[2].t()
    src[2] = pad.t()[: ns[2], :]                      # column-major, ldk = n + 3
    assert src[2].stride() == (1, ns[2] + 3)
    before = [s.cpu().numpy().copy() for s in src]
    As = [torch.full((n, n), float("nan"), dtype=torch.float64, device=DEV).t() for n in ns]
    uts = [torch.from_numpy(u).to(DEV) for u in us]
    fb = B.dpp_sample_ldlh_batched if herm else B.dpp_sample_lu_batched
    outs = fb(As, uts, prec=prec, Ks=src)
    torch.cuda.synchronize()
    for i, (K, u, A, o) in enumerate(zip(Ks, us, As, outs)):
        single = _run(herm, K, u, prec)
        assert np.array_equal(o["mask"].cpu().numpy(), single["mask"])
        assert np.array_equal(o["pivots"].cpu().numpy(), single["pivots"])
        assert float(o["loglik"].cpu()[0]) == single["loglik"]
        got = A.cpu().numpy()
        if herm:
            low = np.tril(np.ones_like(got, dtype=bool))
            assert np.array_equal(got[low], single["A"][low])
            assert np.all(np.isnan(got[~low]))
        else:
            assert np.array_equal(got, single["A"])
        assert np.array_equal(src[i].cpu().numpy(), before[i])


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_deterministic(prec):
    n = 700
    K = W.hermitian_kernel(n, seed=11)
    u = W.uniform_stream(n, seed=11000)
    a, b = _run(True, K, u, prec), _run(True, K, u, prec)
    assert np.array_equal(a["A"], b["A"]) and a["loglik"] == b["loglik"]


def test_uniform_spanning_tree_grid40():
    """The paper's 40 x 40 grid example on the GPU: a spanning tree with
    likelihood exp(-1794.24)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "worked_examples.json")))["uniform_spanning_tree_grid_40"]
    K, edges = W.grid_transfer_current_kernel(40)
    got = _run(True, K, W.uniform_stream(K.shape[0], seed=901), 0)
    assert got["info"] == 0
    chosen = edges[got["mask"].astype(bool)]
    assert len(chosen) == 40 * 40 - 1
    parent = list(range(1600))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in chosen:
        ra, rb = find(a), find(b)
        assert ra != rb
        parent[ra] = rb
    assert got["loglik"] == pytest.approx(gold["loglik_printed"], abs=0.005)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_batched_more_workgroups_than_fit_at_once(prec):
    """12 projection kernels of n = 6144 in one batched call: each diagonal-block
    launch has more workgroups (23 per problem) than the GPU runs at once, so
    late workgroups start after workgroup 0 has finished its block. Every sample
    must still have |Y| = rank and equal the single-problem result."""
    n, k, count = 6144, 1536, 12
    K = W.projection_kernel(n, k, seed=12, device=DEV).to(torch.float64)
    us = [torch.from_numpy(W.uniform_stream(n, seed=12000 + i)).to(DEV) for i in range(count)]
    As = [K.clone() for _ in range(count)]
    outs = B.dpp_sample_ldlh_batched([A.t() for A in As], us, prec=prec)
    torch.cuda.synchronize()
    sizes = [int(o["mask"].sum().item()) for o in outs]
    assert sizes == [k] * count
    for i in (0, count - 1):
        A1 = K.clone()
        single = B.dpp_sample_ldlh(A1.t(), us[i], prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(single["mask"], outs[i]["mask"])
        assert torch.equal(single["pivots"], outs[i]["pivots"])
        assert torch.equal(A1, As[i])


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_graph_capture_replays_equal_eager(prec):
    """A batched call captured in a HIP graph together with the restore copies
    and replayed several times, with eager work and host syncs in between,
    gives the eager result bit for bit on every replay."""
    n, count = 700, 3
    Ks = [B.colmajor(W.hermitian_kernel(n, seed=130 + i), device=DEV) for i in range(count)]
    us = [torch.from_numpy(W.uniform_stream(n, seed=13000 + i)).to(DEV) for i in range(count)]
    As = [torch.empty_like(K) for K in Ks]
    ws = torch.empty(B.dpp_workspace_size_batched(True, B.DPP_F64, [n] * count, prec),
                     dtype=torch.uint8, device=DEV)
    outs = [{"mask": torch.empty(n, dtype=torch.uint8, device=DEV),
             "pivots": torch.empty(n, dtype=torch.float64, device=DEV),
             "loglik": torch.empty(1, dtype=torch.float64, device=DEV),
             "info": torch.empty(1, dtype=torch.int32, device=DEV)} for _ in range(count)]

    def step():
        for A, K in zip(As, Ks):
            A.copy_(K)
        B.dpp_sample_ldlh_batched(As, us, prec=prec, ws=ws, outs=outs)

    step()
    torch.cuda.synchronize()
    eager = [(o["mask"].clone(), o["pivots"].clone(), o["loglik"].clone()) for o in outs]
    eager_A = [A.clone() for A in As]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for _ in range(4):
        for o, A in zip(outs, As):
            o["mask"].fill_(7)
            o["pivots"].fill_(-3.0)
            o["loglik"].fill_(0.0)
            A.fill_(0.5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e, eA, A in zip(outs, eager, eager_A, As):
            assert torch.equal(o["mask"], e[0])
            assert torch.equal(o["pivots"], e[1])
            assert torch.equal(o["loglik"], e[2])
            assert torch.equal(A, eA)


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_batched_lensembles_uneven_n_fp32(prec):
    """The batched L-ensemble workload at reduced count: 48 rank-64 kernels
    with n_i ~ U{64..1024}, formed in FP64 and stored FP32, one batched LDL^H
    call; every instance against the oracle on the same FP32 bytes (widened)
    and its own stream, |Y_i| <= 64, and two instances equal to single calls."""
    count = 48
    ns = [int(x) for x in W.lensemble_batch_sizes(count, seed=4)]
    Ks = [W.lensemble_kernel(n, seed=400000 + i) for i, n in enumerate(ns)]
    us = [W.uniform_stream(n, seed=4000 + i) for i, n in enumerate(ns)]
    As = [B.colmajor(K, device=DEV, dtype=torch.float32) for K in Ks]
    uts = [torch.from_numpy(u).to(DEV) for u in us]
    outs = B.dpp_sample_ldlh_batched(As, uts, prec=prec)
    torch.cuda.synchronize()
    tol, thr = (1e-5, 1e-6) if prec == 0 else TOL[prec]
    worst, ties = 0.0, 0
    for K, u, o in zip(Ks, us, outs):
        ref = oracle.ldlh(np.asarray(K, dtype=np.float64), u)
        v = compare(o["mask"].cpu().numpy(), o["pivots"].cpu().numpy(), float(o["loglik"].cpu()[0]),
                    ref, u, tol, thr)
        assert v.ok, v.why
        ties += int(v.near_tie)
        worst = max(worst, v.max_dd)
        assert int(o["mask"].sum().item()) <= 64
    print(f"[accuracy] L-ensemble batch prec={PREC_ID[prec]}: max |d - d_oracle| = {worst:.3e}, "
          f"near ties {ties}/{count}")
    for i in (0, count - 1):
        A1 = B.colmajor(Ks[i], device=DEV, dtype=torch.float32)
        single = B.dpp_sample_ldlh(A1, uts[i], prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(single["mask"], outs[i]["mask"])
        assert torch.equal(single["pivots"], outs[i]["pivots"])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_copy_lower_stages_the_triangle(dtype):
    """dpp_copy_lower copies the lower triangle with the diagonal, leaves the
    strict upper triangle of the destination alone, and a sample from the
    staged copy equals a sample from a full copy (ragged n, padded lda)."""
    n, lda = 1000, 1037
    K = W.hermitian_kernel(n, seed=140)
    buf = torch.empty(lda * n, dtype=dtype, device=DEV)
    src = torch.as_strided(buf, (n, n), (1, lda))
    src.copy_(torch.from_numpy(K))
    dst = B.colmajor(torch.full((n, n), -7.0, dtype=dtype), device=DEV)
    B.dpp_copy_lower(dst, src)
    torch.cuda.synchronize()
    d, sK = dst.cpu().numpy(), src.cpu().numpy()
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.array_equal(d[low], sK[low])
    assert np.all(d[~low] == -7.0)
    u = torch.from_numpy(W.uniform_stream(n, seed=14000)).to(DEV)
    full = src.clone()
    a = B.dpp_sample_ldlh(dst, u, prec=1)
    b = B.dpp_sample_ldlh(full, u, prec=1)
    torch.cuda.synchronize()
    assert torch.equal(a["mask"], b["mask"]) and torch.equal(a["pivots"], b["pivots"])


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_greedy_ml_mode(prec):
    """Greedy maximum-likelihood selection is the same sampler with u = 1/2
    for every index (keep j iff its conditional inclusion probability exceeds
    1/2): the GPU's decisions and pivots match the oracle's under that stream."""
    n = 700
    K = W.hermitian_kernel(n, seed=150)
    u = np.full(n, 0.5)
    t, h = TOL[prec]
    ref = oracle.ldlh(K, u)
    got = _run(True, K, u, prec)
    v = compare(got["mask"], got["pivots"], got["loglik"], ref, u, t, h)
    assert v.ok, v.why
    d = got["pivots"] + 1.0 - got["mask"]
    assert np.array_equal(got["mask"], (d > 0.5).astype(np.uint8))


_BIG = {}


def _big_kernel(which):
    """Kernels past the first outer panel (4096 columns on both paths):
    a projection kernel n = 6144 of rank 1536 and a dense Hermitian kernel
    n = 8192, generated on the device; host copies for the oracle."""
    if which not in _BIG:
        if which == "proj6144":
            K = W.projection_kernel(6144, 1536, seed=12, device=DEV)
        else:
            # row-major storage of the symmetric kernel: its transpose view
            # is the column-major matrix the calls take
            K = W.hermitian_kernel(8192, seed=21, device=DEV).contiguous()
        torch.cuda.synchronize()
        _BIG[which] = (K, K.cpu().numpy(), {})
    return _BIG[which]


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
@pytest.mark.parametrize("which", ["proj6144", "dense8192"])
def test_ldlh_past_the_outer_panel(which, prec):
    """Two samples of one resident K in a batched out-of-place call (the
    benchmark's launch form), every pivot against whole oracle runs on the
    same bytes and streams, at sizes whose later pivots depend on trailing
    updates of the full outer-panel depth."""
    K, Kh, cache = _big_kernel(which)
    n = Kh.shape[0]
    seeds = (21000, 21001)
    us = [W.uniform_stream(n, seed=s) for s in seeds]
    As = [torch.empty_like(K) for _ in seeds]
    outs = B.dpp_sample_ldlh_batched([A.t() for A in As],
                                     [torch.from_numpy(u).to(DEV) for u in us], prec=prec,
                                     Ks=[K.t()] * len(seeds))
    torch.cuda.synchronize()
    t, h = TOL[prec]
    for s, u, o in zip(seeds, us, outs):
        if s not in cache:
            r = oracle.ldlh(np.array(Kh.T, order="F", copy=True), u, inplace=True)
            cache[s] = {k: r[k] for k in ("mask", "predec", "loglik", "info")}
        ref = cache[s]
        v = compare(o["mask"].cpu().numpy(), o["pivots"].cpu().numpy(),
                    float(o["loglik"].cpu()[0]), ref, u, t, h)
        print(f"[accuracy] {which} prec={PREC_ID[prec]} stream {s}: first mask diff "
              f"{v.first_diff}, near tie {v.near_tie}, max |d - d_oracle| = {v.max_dd:.3e}, "
              f"|dll|/|ll| = {v.ll_rel:.3e}")
        assert int(o["info"].item()) == 0
        assert v.ok, v.why
        if which == "proj6144":
            assert int(o["mask"].sum().item()) == 1536
    del As, outs


@pytest.mark.parametrize("herm", [True, False], ids=["ldlh", "lu"])
@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_nan_in_kernel_sets_info(herm, prec):
    """A NaN in K reaches a pivot: info names the first NaN pivot (as the
    oracle's does), loglik is NaN, and the pivots before it are unaffected.
    A NaN on the diagonal at 70 is that pivot; one at (150, 3) (and (3, 150)
    for LU) reaches pivot 150 through the updates of column 3."""
    n = 200
    for pos, first in (((70, 70), 70), ((150, 3), 150)):
        K = W.hermitian_kernel(n, seed=160)
        if not herm:
            K = W.similarity_kernel(n, seed=160)[0]
        K = np.array(K)
        i, k = pos
        K[i, k] = np.nan
        K[k, i] = np.nan
        u = W.uniform_stream(n, seed=16000)
        ref = (oracle.ldlh if herm else oracle.lu)(K, u)
        got = _run(herm, K, u, prec)
        assert ref["info"] == first + 1
        assert got["info"] == first + 1, (pos, got["info"])
        assert np.isnan(got["loglik"])
        t, h = TOL[prec]
        pre = {"mask": ref["mask"][:first], "predec": ref["predec"][:first], "loglik": 0.0}
        v = compare(got["mask"][:first], got["pivots"][:first], 0.0, pre, u[:first], t, h)
        assert v.first_diff < 0 and v.max_dd <= t, v.why


@pytest.mark.parametrize("prec", PRECS, ids=lambda p: PREC_ID[p])
def test_decision_diagnostics(prec):
    """The library's per-problem diagnostics: the smallest |u_j - d_j| equals
    the oracle's to the path's tolerance (the margin of the decisions), and
    no probability leaves [0, 1] by more than the tolerance; partial problems
    report over their decided indices only."""
    n = 700
    Ks = [W.hermitian_kernel(n, seed=170), W.hermitian_kernel(n, seed=171)]
    us = [W.uniform_stream(n, seed=17000), W.uniform_stream(n, seed=17001)]
    As = [B.colmajor(K, device=DEV) for K in Ks]
    outs = B.dpp_sample_ldlh_batched(As, [torch.from_numpy(u).to(DEV) for u in us], prec=prec,
                                     npivs=[0, 256])
    torch.cuda.synchronize()
    t, h = TOL[prec]
    for K, u, o, npiv in zip(Ks, us, outs, (n, 256)):
        st = o["stats"].cpu().numpy()
        ref = oracle.ldlh(K, u, npiv=npiv)
        gap = float(np.min(np.abs(u[:npiv] - ref["predec"][:npiv])))
        assert abs(st[0] - gap) <= t, (st[0], gap)
        d = ref["predec"][:npiv]
        assert st[1] == pytest.approx(float(np.sum((d < -1e-12) | (d > 1 + 1e-12))), abs=2)
        assert 0.0 <= st[2] <= t


def test_fp16_form_rejects_lu_and_complex():
    """The FP16 form serves real Hermitian problems only: LU calls and complex
    kernels with it return DPP_ERR_INVALID_ARG before any launch, leaving A
    and the outputs unwritten."""
    n = 200
    K, _ = W.similarity_kernel(n, seed=180)
    A = B.colmajor(K, device=DEV)
    before = A.clone()
    with pytest.raises(B.DppError) as e:
        B.dpp_sample_lu(A, torch.from_numpy(W.uniform_stream(n, seed=18000)).to(DEV), prec=3)
    assert e.value.status == 1
    Z = B.colmajor(W.complex_hermitian_kernel(n, seed=181), device=DEV)
    zb = Z.clone()
    with pytest.raises(B.DppError) as e:
        B.dpp_sample_ldlh(Z, torch.from_numpy(W.uniform_stream(n, seed=18001)).to(DEV), prec=3)
    assert e.value.status == 1
    torch.cuda.synchronize()
    assert torch.equal(A, before) and torch.equal(Z, zb)
