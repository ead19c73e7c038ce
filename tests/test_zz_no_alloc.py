"""The no-allocation entry point dpp_sample_ldlh_batched_noalloc: the same
launch sequence as dpp_sample_ldlh_batched with the library's per-device
scratch as the workspace, so its results must equal that call's bit for bit
(and hence the oracle's, as the parity tests show for the batched call).

Two calls in a row, the second on a smaller batch, each compared with the
workspace call on the same inputs; then a batch whose workspace would exceed
the scratch is refused before anything is launched.
"""
import numpy as np
import pytest

from paper_1905_00165_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _outs(ns, dev):
    return [{"mask": torch.empty(n, dtype=torch.uint8, device=dev),
             "pivots": torch.empty(n, dtype=torch.float64, device=dev),
             "loglik": torch.empty(1, dtype=torch.float64, device=dev),
             "info": torch.empty(1, dtype=torch.int32, device=dev),
             "stats": torch.empty(3, dtype=torch.float64, device=dev)} for n in ns]


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["fp64", "split", "split6", "fp16"])
def test_noalloc_equals_workspace_call(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding as B
    dev = torch.device("cuda:0")
    print(f"[noalloc] prec={prec}", flush=True)
    for call, ns in enumerate(([700, 1100, 129, 1], [300, 64])):   # second call smaller
        Ks = [W.hermitian_kernel(n, seed=180 + 10 * call + i) for i, n in enumerate(ns)]
        us = [torch.from_numpy(W.uniform_stream(n, seed=18000 + 10 * call + i)).to(dev)
              for i, n in enumerate(ns)]
        src = [B.colmajor(K, device=dev) for K in Ks]
        a_ws = [torch.empty_like(K) for K in src]
        a_na = [torch.empty_like(K) for K in src]
        ref = B.dpp_sample_ldlh_batched(a_ws, us, prec=prec, Ks=src, outs=_outs(ns, dev))
        got = B.dpp_sample_ldlh_batched_noalloc(a_na, us, prec=prec, Ks=src, outs=_outs(ns, dev))
        torch.cuda.synchronize()
        for i, n in enumerate(ns):
            for key in ("mask", "pivots", "loglik", "info", "stats"):
                assert torch.equal(got[i][key], ref[i][key]), (call, i, key)
            low = torch.tril(torch.ones(n, n, dtype=torch.bool, device=dev))
            assert torch.equal(a_na[i][low], a_ws[i][low]), (call, i)
            assert int(got[i]["info"].item()) == 0


def test_noalloc_refuses_a_batch_beyond_the_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_00165_amd import binding as B
    dev = torch.device("cuda:0")
    n = 2048 + 1024   # the six-product split workspace of one problem exceeds 64 MiB
    assert B.dpp_workspace_size(True, B.DPP_F64, n, 2) > B.DPP_NOALLOC_SCRATCH_BYTES
    A = torch.empty((n, n), dtype=torch.float64, device=dev).t()
    u = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(B.DppError) as e:
        B.dpp_sample_ldlh_batched_noalloc([A], [u], prec=2)
    assert e.value.status == 2   # DPP_ERR_WORKSPACE
