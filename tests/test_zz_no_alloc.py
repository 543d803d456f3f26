"""rx_mlp_grad_static, the entry point that allocates nothing (its gradient
partials live in a static device array), against rx_mlp_grad on the same
inputs: two calls in a row, the second on fewer rows; the row limit."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _rows(seed, n):
    r = np.random.default_rng(seed)
    x = np.zeros((n, 32), dtype=np.float32)
    x[:, :31] = r.standard_normal((n, 31))
    t = (2 * r.integers(0, 8, n) - 7).astype(np.float32)
    return x, t


def _params(seed):
    r = np.random.default_rng(seed)
    p = np.zeros(oracle.MLP_PARAMS)
    p[:64 * 31] = r.uniform(-1, 1, 64 * 31) * math.sqrt(6 / 31)
    o = 64 * 31 + 64
    p[o:o + 4096] = r.uniform(-1, 1, 4096) * math.sqrt(6 / 64)
    o += 4096 + 64
    p[o:o + 64] = r.uniform(-1, 1, 64) * math.sqrt(6 / 64)
    return p.astype(np.float32)


def test_static_gradient_equals_allocating_gradient():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2010_14333_amd as rx
    r = rx.Receiver(rx.RX_PAM8, 1, max_samples=1 << 16, equalizer=rx.RX_EQ_MLP)
    rx.rx_set_mlp(r.h, _params(3))
    for call, n in enumerate((8192, 1000)):   # the maximum, then fewer rows (a partial last workgroup)
        print(f"[no-alloc] call {call} rows {n}", flush=True)
        x, t = _rows(10 + call, n)
        gx = torch.from_numpy(x).to("cuda:0")
        gt = torch.from_numpy(t).to("cuda:0")
        g_ref = torch.zeros(oracle.MLP_PARAMS, dtype=torch.float32, device="cuda:0")
        g_sta = torch.full((oracle.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda:0")
        l_ref = rx.rx_mlp_grad(r.h, gx.data_ptr(), gt.data_ptr(), n, g_ref.data_ptr())
        l_sta = rx.rx_mlp_grad_static(r.h, gx.data_ptr(), gt.data_ptr(), n, g_sta.data_ptr())
        assert np.array_equal(g_sta.cpu().numpy(), g_ref.cpu().numpy())
        assert l_sta == l_ref
        # and both against the FP64 oracle's gradient (the kernels' own bar)
        lo, go = oracle.mlp_grad(_params(3).astype(np.float64), x[:, :31].astype(np.float64), t.astype(np.float64))
        gs = g_sta.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(gs - go) <= 1e-5 * np.linalg.norm(go)
        assert abs(l_sta - lo) <= 1e-6 * lo
    big = torch.zeros((8193, 32), dtype=torch.float32, device="cuda:0")
    tt = torch.zeros(8193, dtype=torch.float32, device="cuda:0")
    with pytest.raises(rx.RxError):
        rx.rx_mlp_grad_static(r.h, big.data_ptr(), tt.data_ptr(), 8193, g_sta.data_ptr())
    k = rx.Receiver(rx.RX_KK_16QAM, 1, max_samples=1 << 16)
    with pytest.raises(rx.RxError):
        rx.rx_mlp_grad_static(k.h, big.data_ptr(), tt.data_ptr(), 100, g_sta.data_ptr())
    k.close()
    r.close()
