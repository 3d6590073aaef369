"""The allocation-free gradient entry point (through the C ABI) against the one that takes
a workspace: the same kernels, so the same bits, on two calls in a row (the second with a
smaller batch, over the partial sums the first one left), and a clear refusal of a batch
beyond its built-in scratch."""
import numpy as np
import pytest

from oracle import learned as L

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
stgv = pytest.importorskip("paper_2605_14505_amd.stgv")

DEV = "cuda:0"


def _t32(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)


def test_gradient_without_workspace_equals_the_workspace_entry_point():
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(11)
    theta = L.init_params(6) + 0.01 * rng.standard_normal(L.N_PARAMS)
    norm = np.concatenate([0.1 * rng.standard_normal(47), 1.0 + 0.2 * rng.uniform(-1, 1, 47),
                           1e-3 * (1.0 + rng.uniform(0, 1, 41))])
    packed = torch.empty(stgv.lbm_mlp_packed_bytes(), dtype=torch.uint8, device=DEV)
    stgv.lbm_mlp_pack(_t32(theta), _t32(norm), packed, stream)
    n = 1000
    x = _t32(rng.standard_normal((n, 47)) * 0.7 + norm[:47])
    y = _t32(rng.standard_normal((n, 41)) * norm[94:])
    for batch in (700, 77):                          # the second call is smaller
        idx = torch.tensor(rng.permutation(n)[:batch], dtype=torch.int64, device=DEV)
        g_ws = torch.empty(L.N_PARAMS, dtype=torch.float32, device=DEV)
        l_ws = torch.empty(1, dtype=torch.float64, device=DEV)
        work = torch.empty(stgv.lbm_mlp_grad_work_bytes(batch), dtype=torch.uint8, device=DEV)
        stgv.lbm_mlp_grad(packed, x, y, idx, batch, g_ws, l_ws, work, stream)
        g_st = torch.full((L.N_PARAMS,), float("nan"), dtype=torch.float32, device=DEV)
        l_st = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
        stgv.lbm_mlp_grad_static(packed, x, y, idx, batch, g_st, l_st, stream)
        torch.cuda.synchronize()
        a, b = g_ws.cpu().numpy(), g_st.cpu().numpy()
        print(f"\nbatch {batch}: {int((a != b).sum())} of {a.size} gradient entries differ; "
              f"loss {l_ws.item():.9e} / {l_st.item():.9e}")
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert l_ws.item() == l_st.item()
        assert np.isfinite(b).all() and np.abs(b).max() > 0


def test_gradient_without_workspace_refuses_a_batch_beyond_its_scratch():
    stream = torch.cuda.current_stream().cuda_stream
    big = stgv.LBM_MLP_STATIC_MAX_BATCH + 1
    packed = torch.zeros(stgv.lbm_mlp_packed_bytes(), dtype=torch.uint8, device=DEV)
    x = torch.zeros((big, 47), dtype=torch.float32, device=DEV)
    y = torch.zeros((big, 41), dtype=torch.float32, device=DEV)
    idx = torch.zeros(big, dtype=torch.int64, device=DEV)
    grad = torch.zeros(L.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    with pytest.raises(stgv.LbmError) as ei:
        stgv.lbm_mlp_grad_static(packed, x, y, idx, big, grad, loss, stream)
    assert ei.value.status == stgv.LBM_ESIZE
    assert "exceeds" in str(ei.value)
    torch.cuda.synchronize()
    assert float(grad.abs().sum()) == 0.0           # nothing was queued
