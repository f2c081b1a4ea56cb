"""BF16 MFMA convolution kernels vs the FP64 oracle (oracle.convnet) on
bf16-rounded inputs and weights: forward (with and without ReLU), data
gradient (mirrored taps, transposed weights) and weight gradient.  FP32
accumulation of at most 27*16 products: relative error bar 1e-5."""
import numpy as np
import pytest

from oracle import convnet as C
from tests.helpers import rel

pytestmark = pytest.mark.gpu


def _data(seed, shape, periodic):
    rng = np.random.default_rng(seed)
    B, T, X, Y = shape
    x = C.bf16_round(rng.standard_normal((B, T, X, Y, 16)))
    w = C.bf16_round(rng.standard_normal((27, 16, 16)) * 0.2)
    b = rng.standard_normal(16).astype(np.float32)
    return x, w, b


@pytest.mark.parametrize("shape,periodic", [((2, 5, 6, 7), (False, True, True)), ((1, 8, 9, 1), (False, False, False)),
                                            ((3, 4, 4, 4), (True, True, True))])
def test_conv_forward(shape, periodic):
    import torch
    from paper_2502_18377_amd.learned import conv3d
    x, w, b = _data(1, shape, periodic)
    xt = torch.from_numpy(x).to("cuda", torch.bfloat16)
    wt = torch.from_numpy(w).to("cuda", torch.bfloat16)
    bt = torch.from_numpy(b).cuda()
    y, yb = conv3d(xt, wt, bt, periodic, relu=True, want=("f32", "bf16"))
    for i in range(shape[0]):
        ref = C.conv_fwd(x[i], w, b, periodic)
        assert rel(y[i].double().cpu().numpy(), ref) <= 1e-5
        assert np.array_equal(yb[i].float().cpu().numpy(), C.bf16_round(np.maximum(y[i].cpu().numpy(), 0)).astype(np.float32))


@pytest.mark.parametrize("periodic", [(False, True, True), (True, False, False)])
def test_conv_data_gradient(periodic):
    import torch
    from paper_2502_18377_amd.learned import conv3d
    x, w, _ = _data(2, (2, 5, 6, 7), periodic)
    dy = x                                    # any bf16 field serves as dY
    wtr = np.ascontiguousarray(np.transpose(w, (0, 2, 1)))   # [tap][in][out]
    g, _ = conv3d(torch.from_numpy(dy).to("cuda", torch.bfloat16), torch.from_numpy(wtr).to("cuda", torch.bfloat16),
                  None, periodic, sign=-1)
    for i in range(2):
        ref = C.conv_bwd_data(dy[i], w, periodic)
        assert rel(g[i].double().cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("periodic", [(False, True, True), (True, True, False)])
def test_conv_weight_gradient(periodic):
    import torch
    from paper_2502_18377_amd.learned import conv3d_wgrad
    x, _, _ = _data(3, (2, 6, 5, 8), periodic)
    dy = C.bf16_round(np.random.default_rng(4).standard_normal(x.shape))
    dw = conv3d_wgrad(torch.from_numpy(x).to("cuda", torch.bfloat16), torch.from_numpy(dy).to("cuda", torch.bfloat16),
                      periodic)
    ref = sum(C.conv_bwd_weight(x[i], dy[i], periodic)[0] for i in range(2))
    assert rel(dw.double().cpu().numpy(), ref) <= 1e-5
