"""The entry point that allocates nothing (mlvs_mlp_eval_noalloc) against the
allocating one (mlvs_mlp_eval) on the same inputs, through the C ABI: two
calls in a row, the second with a smaller batch, outputs equal bit for bit
(the same kernels on the same float inputs; only where the intermediates live
differs)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _m():
    import paper_2609_35258_amd as m
    return m


def _net(K, B, seed):
    th = W.mlp_init_params(K, seed)
    rng = np.random.default_rng(seed + 1)
    X = rng.normal(size=(B, 10))
    y = rng.integers(0, K, size=B)
    th[-20:-10] = rng.normal(size=10) * 0.1
    th[-10:] = rng.uniform(0.5, 2.0, size=10)
    return th.astype(np.float32), X.astype(np.float32), y.astype(np.int32)


def _noalloc(P, K, X, y, B):
    import torch
    m = _m()
    dev = torch.device("cuda", torch.cuda.current_device())
    tP = torch.from_numpy(P).to(dev)
    tX = torch.from_numpy(np.ascontiguousarray(X[:B])).to(dev)
    ty = torch.from_numpy(np.ascontiguousarray(y[:B])).to(dev)
    probs = torch.full((B, K), float("nan"), dtype=torch.float32, device=dev)
    grad = torch.full((len(P),), float("nan"), dtype=torch.float32, device=dev)
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev)
    m.mlp_eval_noalloc(tP.data_ptr(), K, tX.data_ptr(), ty.data_ptr(), B, probs.data_ptr(), grad.data_ptr(),
                       loss.data_ptr(), st.cuda_stream)
    torch.cuda.synchronize()
    return probs.cpu().numpy(), grad.cpu().numpy(), float(loss.cpu().numpy()[0])


def test_noalloc_eval_matches_the_allocating_entry_point():
    m = _m()
    K = 5
    P, X, y = _net(K, 4096, 11)
    for B in (4096, 700):                       # two calls in a row, the second smaller; 4096 the limit
        print("noalloc eval, batch", B, flush=True)
        p_ref, g_ref, l_ref = m.mlp_eval(P, K, X[:B], y[:B])
        p, g, lsum = _noalloc(P, K, X, y, B)
        assert np.array_equal(p, p_ref)
        assert np.array_equal(g, g_ref)
        assert np.all(g[-20:] == 0.0)
        assert lsum / B == l_ref


def test_noalloc_eval_rejects_batches_beyond_its_array():
    m = _m()
    K = 3
    P, X, y = _net(K, 4, 2)
    with pytest.raises(m.MLVSError):
        m.mlp_eval_noalloc(1, K, 1, 1, 4097)      # argument check before any device work
    with pytest.raises(m.MLVSError):
        m.mlp_eval_noalloc(1, K, 1, 1, 0)
