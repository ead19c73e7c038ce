"""GPU checks at the full benchmark size, in the benchmark's launch
configuration: the projection kernel K = Q_r Q_r^T with n = 16384, rank 4096,
FP64 storage, eight samples per batched LDL^H call reading the resident K out
of place, both precisions.

  - full-length parity: samples on streams 2000 and 2001 against whole oracle
    runs on the same bytes and streams (Sec. 2, Theorem 2 and the unblocked
    listing; Sec. 3 blocked form with Prop. 5), every pivot and the
    log-likelihood, under the near-tie rule of tests/parity.py;
  - |Y| = rank for every sample of 64 distinct streams (Sec. 1: projection
    kernels give samples of size exactly their rank);
  - the decision rule on the GPU's own probabilities: keep j iff u_j < d_j,
    and the library's decision diagnostics against a recomputation;
  - sampled entries of L D L^T equal K - 1_{Y^c} (the factor is the in-place
    LDL^H of K - 1_{Y^c});
  - at sampled indices j in every outer panel, the GPU's d_j equals the
    conditional inclusion probability given the GPU's own decisions for
    0..j-1, computed from K by a library solve (Props. 3-5).
Tolerances: FP64 1e-9 (near-tie threshold 1e-10); split-BF16 1e-4 (threshold
1e-5), on probabilities, relative on the log-likelihood and on factor entries
(scaled by the magnitude of the entries involved). The three-product split
form keeps about 16 bits of each product; over a whole sample at this size
its last pivots (the conditional kernel there is a nearly exhausted
projection) amplify that to about 2e-4, so its full-length comparison is held
to 1e-3 and the six-product form is the split path held to 1e-4 at this size.
The FP16 form (pieces relative to each row's 64-column block, 22 bits of
each value) measured 5.8e-5 and 2.6e-5 on streams 2000/2001, but over the
64 benchmark streams a pre-decision probability leaves [0, 1] by up to
3.1e-4 (a lower bound of that stream's error), so like the three-product
form it is held to 1e-3 over whole samples at this size and to 1e-4 in the
other checks.
"""
import numpy as np
import pytest

import oracle
from paper_1905_00165_amd import workloads as W
from parity import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, RANK, BATCH = 16384, 4096, 8
TOL = {0: 1e-9, 1: 1e-4, 2: 1e-4, 3: 1e-4}
THR = {0: 1e-10, 1: 1e-5, 2: 1e-5, 3: 1e-5}
FULL_TOL = {0: 1e-9, 1: 1e-3, 2: 1e-4, 3: 1e-3}   # whole-sample comparison (see above)
NAME = {0: "fp64", 1: "split", 2: "split6", 3: "fp16"}


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding as B
    dev = torch.device("cuda:0")
    print(f"[fullsize] generating K: n={N} rank={RANK}", flush=True)
    K = W.projection_kernel(N, RANK, seed=2, device=dev)
    torch.cuda.synchronize()
    Kh = K.cpu().numpy()
    us = [W.uniform_stream(N, seed=2000 + i) for i in range(BATCH)]
    return B, dev, K, Kh, us


def _call(B, K, uts, prec, As, outs=None):
    """One batched out-of-place call, as the benchmark makes it."""
    Kc = K.t()  # column-major view (K is symmetric)
    return B.dpp_sample_ldlh_batched([A.t() for A in As], uts, prec=prec, Ks=[Kc] * len(As),
                                     outs=outs)


@pytest.fixture(scope="module", params=[0, 1, 2, 3], ids=["fp64", "split", "split6", "fp16"])
def run(request, setup):
    B, dev, K, Kh, us = setup
    prec = request.param
    print(f"[fullsize] {NAME[prec]}: {BATCH} samples, one batched call", flush=True)
    As = [torch.empty_like(K) for _ in range(BATCH)]
    uts = [torch.from_numpy(u).to(dev) for u in us]
    outs = _call(B, K, uts, prec, As)
    torch.cuda.synchronize()
    res = []
    for i, (A, o) in enumerate(zip(As, outs)):
        res.append({"mask": o["mask"].cpu().numpy(), "pivots": o["pivots"].cpu().numpy(),
                    "loglik": float(o["loglik"].cpu()[0]), "info": int(o["info"].cpu()[0]),
                    "stats": o["stats"].cpu().numpy(),
                    # factor of the first two samples, as a host copy of the
                    # column-major buffer (row-major view of its transpose)
                    "A": A.cpu() if i < 2 else None})
    del As, outs
    torch.cuda.empty_cache()
    return prec, res


_ORACLE = {}


def _oracle(Kh, us, i):
    """A whole oracle run on stream 2000 + i (about a minute on 16 cores),
    computed once per module."""
    if i not in _ORACLE:
        print(f"[fullsize] oracle run on stream {2000 + i}", flush=True)
        A = np.array(Kh.T, order="F", copy=True)   # column-major copy of symmetric K
        r = oracle.ldlh(A, us[i], inplace=True)
        del A
        _ORACLE[i] = {k: r[k] for k in ("mask", "predec", "loglik", "info")}
    return _ORACLE[i]


@pytest.mark.parametrize("i", [0, 1])
def test_full_length_parity_with_oracle(run, setup, i):
    prec, res = run
    Kh, us = setup[3], setup[4]
    ref = _oracle(Kh, us, i)
    r = res[i]
    assert ref["info"] == 0 and r["info"] == 0
    v = compare(r["mask"], r["pivots"], r["loglik"], ref, us[i], FULL_TOL[prec], THR[prec])
    print(f"[accuracy] prec={NAME[prec]} stream {2000 + i}, all {N} pivots: first mask diff "
          f"{v.first_diff}, near tie {v.near_tie}, max |d_gpu - d_oracle| = {v.max_dd:.3e}, "
          f"|dll|/|ll| = {v.ll_rel:.3e}, min |u - d| = {v.min_gap:.3e}")
    assert v.ok, v.why


def test_sample_size_and_info(run):
    prec, res = run
    for r in res:
        assert r["info"] == 0
        assert int(r["mask"].sum()) == RANK


def test_rank_invariant_on_64_streams(setup):
    """Each of 64 samples on its own stream (2000-2063), eight batched calls
    of eight, both precisions: |Y| = 4096 exactly and info = 0."""
    B, dev, K = setup[0], setup[1], setup[2]
    As = [torch.empty_like(K) for _ in range(BATCH)]
    for prec in (0, 1, 2, 3):
        sizes, infos = [], []
        for c in range(64 // BATCH):
            uts = [torch.from_numpy(W.uniform_stream(N, seed=2000 + BATCH * c + i)).to(dev)
                   for i in range(BATCH)]
            outs = _call(B, K, uts, prec, As)
            torch.cuda.synchronize()
            sizes += [int(o["mask"].sum().item()) for o in outs]
            infos += [int(o["info"].item()) for o in outs]
        assert sizes == [RANK] * 64, (NAME[prec], sizes)
        assert infos == [0] * 64
    del As
    torch.cuda.empty_cache()


def test_decision_rule_and_diagnostics(run, setup):
    """keep j iff u_j < d_j on the GPU's own probabilities; loglik is the sum
    of ln|d'_j|; the library's diagnostics (smallest |u_j - d_j|, count and
    size of d_j outside [0, 1]) equal their recomputation from the outputs."""
    prec, res = run
    us = setup[4]
    for r, u in zip(res, us):
        d = np.where(r["mask"] == 1, r["pivots"], r["pivots"] + 1.0)
        assert np.array_equal(r["mask"], (u < d).astype(np.uint8))
        ll = float(np.sum(np.log(np.abs(r["pivots"]))))
        assert r["loglik"] == pytest.approx(ll, rel=1e-12)
        gap = float(np.min(np.abs(u - d)))
        outside = int(np.sum((d < -1e-12) | (d > 1.0 + 1e-12)))
        far = float(np.max(np.maximum(-d, d - 1.0).clip(min=0.0)))
        assert r["stats"][0] == gap
        assert r["stats"][1] == outside
        assert r["stats"][2] == far
        # rounding pushes a probability out of [0, 1] by no more than the tolerance
        assert far <= TOL[prec]
    print(f"[accuracy] prec={NAME[prec]} d_j outside [-1e-12, 1+1e-12]: "
          f"{sum(int(r['stats'][1]) for r in res)} over {BATCH} samples, worst by "
          f"{max(r['stats'][2] for r in res):.3e}")


def test_factor_reconstructs_sampled_entries(run, setup):
    """(L D L^T)[i,k] = K[i,k] - [i == k] (1 - mask_i) on sampled (i, k)."""
    prec, res = run
    Kh = setup[3]
    rng = np.random.default_rng(77)
    worst = 0.0
    for r in res[:2]:
        F = r["A"].numpy().T                # column-major factor as a numpy matrix
        d = np.diag(F).copy()
        for _ in range(40):
            i = int(rng.integers(0, N))
            k = int(rng.integers(0, i + 1))
            m = min(i, k)
            Li = F[i, :m]
            Lk = F[k, :m]
            acc = float(np.dot(Li * d[:m], Lk))
            # unit diagonal of L: add the diagonal terms of the product
            if i == k:
                acc += d[i]
            else:
                acc += F[i, k] * d[k]
            target = Kh[i, k] - (1.0 - r["mask"][i] if i == k else 0.0)
            scale = 1.0 + float(np.dot(np.abs(Li * d[:m]), np.abs(Lk)))
            worst = max(worst, abs(acc - target) / scale)
            assert abs(acc - target) <= TOL[prec] * scale, (i, k, acc, target)
    print(f"[accuracy] prec={NAME[prec]} reconstruction max |LDL^T - (K - 1_Yc)| / scale = {worst:.3e}")


@pytest.mark.parametrize("j", [700, 2500, 4000, 6000, 10000, 15000])
def test_conditional_probability_deep_in_the_factorization(run, setup, j):
    """d_j from the GPU equals P[j in Y | the GPU's decisions for 0..j-1],
    the Schur complement of Props. 3-5 evaluated with a library solve; j
    covers every 4096-column outer panel."""
    prec, res = run
    Kh = setup[3]
    r = res[1]
    d_gpu = r["pivots"][j] + 1.0 - r["mask"][j]
    d_ref = oracle.conditional_pivot(Kh[: j + 1, : j + 1], r["mask"][:j], j)
    print(f"[accuracy] prec={NAME[prec]} j={j} |d_gpu - d_ref| = {abs(d_gpu - d_ref):.3e}")
    assert abs(d_gpu - d_ref) <= TOL[prec], (d_gpu, d_ref)
