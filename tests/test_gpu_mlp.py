"""GPU warm-start network kernels (BF16 matrix cores, FP32 accumulation) against the FP64
oracle network and exact BF16 arithmetic.

Tolerances: a single layer with BF16-rounded operands is exact up to FP32 accumulation
(1e-5 relative).  Through three 256-wide ReLU layers the BF16 rounding of weights and
activations (2^-9 relative each) accumulates; forward outputs and gradients are
compared norm-wise per layer against the FP64 oracle at 3e-2 (forward) and 6e-2
(gradients), about ten times the observed BF16 error, far below a layout or index error
(which gives O(1) differences).
"""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu


def bf16_round(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mlp(widths, batch):
    from paper_2302_14344_amd.solver import Mlp
    return Mlp(widths, batch)


def _init(widths, rng):
    parts = []
    for k in range(len(widths) - 1):
        fan_in = widths[k]
        parts.append(rng.standard_normal(widths[k + 1] * widths[k]) * np.sqrt(2.0 / fan_in))
        parts.append(rng.standard_normal(widths[k + 1]) * 0.1)
    return np.concatenate(parts)


@pytest.mark.parametrize("batch,k,n", [(1, 16, 16), (70, 9, 256), (257, 256, 15), (64, 33, 40)])
def test_single_layer_is_exact_in_bf16(batch, k, n):
    """y = bf16(x) bf16(W)^T + b, accumulated in FP32: pins the MFMA operand and result
    lane layout, the tile edges and the bias epilogue."""
    rng = np.random.default_rng(batch + k + n)
    widths = [k, n]
    p = _init(widths, rng)
    x = rng.standard_normal((batch, k))
    net = _mlp(widths, batch)
    net.set_params(p)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    W = bf16_round(p[:n * k]).reshape(n, k)
    b = np.asarray(p[n * k:], np.float32).astype(np.float64)
    ref = bf16_round(x) @ W.T + b
    np.testing.assert_allclose(y, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("widths,batch", [([12, 256, 256, 256, 6], 1000), ([26, 256, 256, 256, 15], 333)])
def test_forward_and_gradients_match_fp64_oracle(widths, batch):
    rng = np.random.default_rng(len(widths) + batch)
    p = _init(widths, rng)
    x = rng.standard_normal((batch, widths[0]))
    t = rng.standard_normal((batch, widths[-1]))
    wt = rng.uniform(0.5, 1.5, t.shape)
    net = _mlp(widths, batch)
    net.set_params(p)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    y_ref = O.mlp_forward(widths, p, x)
    assert np.linalg.norm(y - y_ref) <= 3e-2 * np.linalg.norm(y_ref)
    loss, g = net.backward(t, wt, want_grad=True)
    g = g.cpu().numpy().astype(np.float64)
    l_ref, g_ref = O.mlp_backward(widths, p, x, t, wt)
    assert abs(float(loss.item()) - l_ref) <= 3e-2 * l_ref
    off = 0
    for k in range(len(widths) - 1):
        nw = widths[k + 1] * widths[k]
        for sl in (slice(off, off + nw), slice(off + nw, off + nw + widths[k + 1])):
            assert np.linalg.norm(g[sl] - g_ref[sl]) <= 6e-2 * np.linalg.norm(g_ref[sl]), (k, sl)
        off += nw + widths[k + 1]


def test_adam_step_matches_formula():
    rng = np.random.default_rng(3)
    widths = [10, 32, 4]
    p = _init(widths, rng)
    x = rng.standard_normal((50, 10))
    t = rng.standard_normal((50, 4))
    net = _mlp(widths, 50)
    net.set_params(p)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pw = np.asarray(p, np.float64)
    for step in (1, 2, 3):
        net.forward(torch.as_tensor(x, dtype=torch.float32, device="cuda"))
        _, g = net.backward(t, want_grad=True)
        g = g.cpu().numpy().astype(np.float64)
        net.adam(1e-3, step)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        pw = pw - 1e-3 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
        np.testing.assert_allclose(net.get_params().cpu().numpy(), pw, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss():
    """A few hundred Adam steps on a smooth target drive the loss down by 10x."""
    rng = np.random.default_rng(4)
    widths = [4, 64, 64, 2]
    p = _init(widths, rng)
    x = rng.uniform(-1, 1, (512, 4))
    t = np.stack([np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2], np.cos(x[:, 3])], 1)
    net = _mlp(widths, 512)
    net.set_params(p)
    xs = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 301):
        net.forward(xs)
        loss, _ = net.backward(t)
        net.adam(3e-3, step)
        losses.append(float(loss.item()))
    assert losses[-1] < 0.1 * losses[0]


def test_minibatch_gather_rows():
    """The training minibatch gather: each row equals numpy indexing of the source bit for
    bit; an index outside the source gives a row of NaN."""
    from paper_2302_14344_amd.solver import Mlp
    rng = np.random.default_rng(12)
    src = rng.standard_normal((1000, 27)).astype(np.float32)
    idx = rng.integers(0, 1000, 4096).astype(np.int32)
    idx[[7, 100]] = [-1, 1000]
    net = Mlp([27, 16, 15], 64)
    s = torch.as_tensor(src, device=net.device)
    i = torch.as_tensor(idx, device=net.device)
    d = torch.empty((4096, 27), dtype=torch.float32, device=net.device)
    net.gather_rows(s, i, d)
    out = d.cpu().numpy()
    ok = (idx >= 0) & (idx < 1000)
    np.testing.assert_array_equal(out[ok], src[idx[ok]])
    assert np.isnan(out[~ok]).all()


@pytest.mark.parametrize("widths", [[12, 256, 256, 256, 6], [27, 256, 256, 256, 15], [5, 40, 33, 7], [9, 300, 5]])
@pytest.mark.parametrize("affine", [False, True])
def test_fused_inference_equals_forward(widths, affine):
    """The learned start's one-launch inference gives the per-layer forward's output bit for
    bit (same BF16 inputs, same k-block order, same matrix instruction), for full and ragged
    tiles; a backward pass needs a forward first.  A width above 256 takes the per-layer
    forward inside the same call."""
    from paper_2302_14344_amd import _lib as L
    from paper_2302_14344_amd.solver import Mlp
    rng = np.random.default_rng(sum(widths) + affine)
    net = Mlp(widths, 2048)
    n_par = net.n_params
    net.set_params((rng.standard_normal(n_par) * 0.1).astype(np.float32))
    if affine:
        net.set_input_affine(rng.uniform(0.5, 2.0, widths[0]).astype(np.float32),
                             rng.uniform(-1.0, 1.0, widths[0]).astype(np.float32))
    for batch in (2048, 1, 63, 65, 1000):
        x = torch.as_tensor(rng.standard_normal((batch, widths[0])).astype(np.float32), device=net.device)
        yf = net.forward(x).cpu().numpy()
        yi = net.infer(x).cpu().numpy()
        assert np.isfinite(yf).all()
        np.testing.assert_array_equal(yi, yf)
    if max(widths) <= 256:
        with pytest.raises(L.SubadmmError):
            net.backward(torch.zeros((1000, widths[-1]), device=net.device))
