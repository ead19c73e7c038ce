"""The serving loop: admission policy on the CPU; on the GPU, a served trace
whose every result matches the oracle on the kernel's stored bytes and equals
the standalone call (bit for bit), and whose batches overlapped on the
device."""
import numpy as np
import pytest

import oracle
from paper_1905_00165_amd import serve
from paper_1905_00165_amd import workloads as W
from parity import compare

torch = pytest.importorskip("torch")


class _R:
    def __init__(self, rid, f):
        self.rid, self.f = rid, f


def test_admit_takes_oldest_prefix_within_memory_and_batch():
    pend = [_R(i, f) for i, f in enumerate([3, 4, 2, 1, 1])]
    take, used = serve.admit(pend, lambda r: r.f, free_mem=9, max_batch=10)
    assert [r.rid for r in take] == [0, 1, 2] and used == 9
    take, used = serve.admit(pend, lambda r: r.f, free_mem=100, max_batch=2)
    assert [r.rid for r in take] == [0, 1] and used == 7


def test_admit_is_first_come_first_served():
    # the head does not fit: nothing behind it jumps the queue
    pend = [_R(0, 10), _R(1, 1)]
    take, used = serve.admit(pend, lambda r: r.f, free_mem=5, max_batch=4)
    assert take == [] and used == 0


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["fp64", "split", "split6", "fp16"])
def test_served_results_equal_standalone_and_overlap(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding as B
    dev = torch.device("cuda:0")
    sizes = [96, 300, 700, 1100, 180, 520]
    kernels = [B.colmajor(W.lensemble_kernel(n, seed=500 + i), device=dev, dtype=torch.float32)
               for i, n in enumerate(sizes)]
    rng = np.random.default_rng(5)
    reqs = []
    t = 0.0
    for i in range(60):
        k = int(rng.integers(0, len(sizes)))
        u = torch.from_numpy(W.uniform_stream(sizes[k], seed=5_000_000 + i)).to(dev)
        t += float(rng.exponential(2e-4))
        reqs.append(serve.Request(rid=i, kernel=k, u=u, arrival=t))
    before = [K.clone() for K in kernels]
    torch.cuda.synchronize()
    srv = serve.Server(kernels, prec=prec, slots=3, mem_budget=1 << 30, max_batch=6)
    import gc
    collecting = gc.isenabled()
    srv.run(reqs)
    assert gc.isenabled() == collecting   # the loop restores the collector's state
    torch.cuda.synchronize()
    assert srv.batches > 3 and srv.max_inflight >= 2
    assert all(torch.equal(K, K0) for K, K0 in zip(kernels, before))  # resident kernels only read
    # the oracle on each kernel's FP32 bytes widened to FP64 (FP32 storage:
    # 1e-5 with FP64 updates, 1e-4 split; near-tie thresholds 1e-6 / 1e-5)
    tol, thr = (1e-5, 1e-6) if prec == 0 else (1e-4, 1e-5)
    host = [K.cpu().numpy().astype(np.float64) for K in kernels]
    worst, ties = 0.0, 0
    for r in reqs:
        A = kernels[r.kernel].clone()
        alone = B.dpp_sample_ldlh(A, r.u, prec=prec)
        torch.cuda.synchronize()
        assert int(r.info.item()) == 0
        assert torch.equal(alone["mask"], r.mask), r.rid
        assert torch.equal(alone["pivots"], r.pivots), r.rid
        assert torch.equal(alone["loglik"], r.loglik), r.rid
        assert int(r.mask.sum().item()) <= 64
        u = r.u.cpu().numpy()
        ref = oracle.ldlh(host[r.kernel], u)
        v = compare(r.mask.cpu().numpy(), r.pivots.cpu().numpy(), float(r.loglik.cpu()[0]),
                    ref, u, tol, thr)
        assert v.ok, (r.rid, v.why)
        worst = max(worst, v.max_dd)
        ties += int(v.near_tie)
    print(f"[accuracy] served prec={prec}: max |d - d_oracle| = {worst:.3e}, near ties {ties}")
    st = serve.latency_stats(reqs)
    print(f"[serve] prec={prec} batches={srv.batches} max_inflight={srv.max_inflight} "
          f"p50={st['p50_ms']:.2f} ms p99={st['p99_ms']:.2f} ms")
