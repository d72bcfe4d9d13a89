"""The gradient entry point that allocates nothing, against the one that takes
a workspace: two calls in a row (the second on fewer samples) through the C
ABI, bit-identical while the sample count keeps the block count at or below
the scratch's 256 rows, and within FP32 summation-order rounding beyond."""
import numpy as np
import pytest

from paper_2010_00180_amd import binding, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    binding.load()
    return torch


def _data(torch, n, seed):
    rng = np.random.default_rng(seed)
    feat = torch.tensor(rng.normal(size=(n, 4)).astype(np.float32), device="cuda")
    lab = torch.tensor((rng.random(n) < 0.2).astype(np.uint8), device="cuda")
    return feat, lab


def _both(torch, P, feat, lab, n, pos_w):
    st = torch.cuda.current_stream().cuda_stream
    wsb = binding.mlp_workspace_bytes()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    g_ws = torch.full((binding.MLP_NPARAM,), float("nan"), device="cuda")
    l_ws = torch.full((1,), float("nan"), device="cuda")
    binding.mlp_loss_grad(P.data_ptr(), feat.data_ptr(), lab.data_ptr(), n, pos_w, g_ws.data_ptr(), l_ws.data_ptr(),
                          ws.data_ptr(), wsb, st)
    g_na = torch.full((binding.MLP_NPARAM,), float("nan"), device="cuda")
    l_na = torch.full((1,), float("nan"), device="cuda")
    binding.mlp_loss_grad_noalloc(P.data_ptr(), feat.data_ptr(), lab.data_ptr(), n, pos_w, g_na.data_ptr(),
                                  l_na.data_ptr(), st)
    torch.cuda.synchronize()
    return g_ws.cpu().numpy(), l_ws.cpu().numpy(), g_na.cpu().numpy(), l_na.cpu().numpy()


def test_noalloc_gradient_matches_workspace_gradient(torch_cuda):
    torch = torch_cuda
    P = torch.tensor(workloads.network_params(3).astype(np.float32), device="cuda")
    # two calls in a row, the second smaller: at most 256 blocks either way, so bit-identical
    for n, seed in ((16000, 1), (3001, 2)):
        print(f"[noalloc] n={n} seed={seed}", flush=True)
        feat, lab = _data(torch, n, seed)
        g_ws, l_ws, g_na, l_na = _both(torch, P, feat, lab, n, 3.5)
        assert np.all(np.isfinite(g_ws)) and np.isfinite(l_ws[0])
        assert np.array_equal(g_na, g_ws), f"n={n}: max diff {np.max(np.abs(g_na - g_ws))}"
        assert np.array_equal(l_na, l_ws)
    # more samples than 256 blocks of 64: the same sums in another grouping
    n = 200000
    print(f"[noalloc] n={n}", flush=True)
    feat, lab = _data(torch, n, 3)
    g_ws, l_ws, g_na, l_na = _both(torch, P, feat, lab, n, 3.5)
    scale = np.max(np.abs(g_ws))
    assert np.max(np.abs(g_na - g_ws)) <= 1e-5 * scale
    assert abs(l_na[0] - l_ws[0]) <= 1e-5 * abs(l_ws[0])


def test_noalloc_gradient_rejects_bad_arguments(torch_cuda):
    torch = torch_cuda
    P = torch.zeros(binding.MLP_NPARAM, device="cuda")
    g = torch.zeros(binding.MLP_NPARAM, device="cuda")
    feat, lab = _data(torch, 64, 4)
    with pytest.raises(binding.IsingError):
        binding.mlp_loss_grad_noalloc(P.data_ptr(), feat.data_ptr(), lab.data_ptr(), 0, 1.0, g.data_ptr(), 0)
    with pytest.raises(binding.IsingError):
        binding.mlp_loss_grad_noalloc(P.data_ptr(), feat.data_ptr(), lab.data_ptr(), 64, 0.0, g.data_ptr(), 0)
