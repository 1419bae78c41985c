"""The surrogate network's kernels (quapi_mlp_*) against a plain torch CPU
reference in float64.

Forward: the reference rounds to bf16 where the kernels do (the operands of
every product but an input layer of at most 16 inputs, which runs in FP32, and
the hidden activations); the rest of the difference is FP32 accumulation and
the FP32 erf, so outputs agree to a few bf16 units of the largest output.
Gradients: against torch autograd of the unrounded network in float64; bf16
rounding of the product operands leaves a relative error of the order of
2^-8 per element, so the bar is on whole layers (relative norm error < 3e-2,
cosine > 0.999).  Adam: one step against the textbook update, in float64.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_03127_amd import quapi
    quapi.lib()
    return quapi


def _split(net, p):
    """flat parameters -> [(W [fin][fout], b [fout])]"""
    out, o = [], 0
    for fin, fout in net.layers():
        W = p[o:o + fin * fout].reshape(fin, fout)
        o += fin * fout
        b = p[o:o + fout]
        o += fout
        out.append((W, b))
    return out


def _bf16(a):
    import torch
    return torch.as_tensor(a).to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _ref_forward(net, p, x, rounded):
    """rounded: bf16 where the kernels round -- every product's operands but
    those of an input layer of at most 16 inputs, which runs in FP32."""
    import torch
    fp32_in = net.n_in <= 16
    a = _bf16(x) if rounded and not fp32_in else torch.as_tensor(x, dtype=torch.float64)
    layers = _split(net, p)
    for l, (W, b) in enumerate(layers):
        Wt = _bf16(W) if rounded and not (l == 0 and fp32_in) else torch.as_tensor(W, dtype=torch.float64)
        z = a @ Wt + torch.as_tensor(b, dtype=torch.float64)
        if l == len(layers) - 1:
            return z
        g = torch.nn.functional.gelu(z)
        a = _bf16(g) if rounded else g


# the last shape has a bf16 input layer (more than 16 inputs)
SHAPES = [(6, 256, 4, 4, 1000), (5, 96, 2, 3, 77), (6, 64, 3, 4, 4096), (40, 128, 2, 4, 500)]


@pytest.mark.parametrize("n_in,width,depth,n_out,batch", SHAPES)
def test_forward_matches_reference(Q, n_in, width, depth, n_out, batch):
    import torch
    print(f"[mlp] forward {n_in}->{width}x{depth}->{n_out} batch {batch}", flush=True)
    net = Q.MLP(n_in, width, depth, n_out, max_batch=batch, seed=3)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (batch, n_in)).astype(np.float32)
    xd = torch.as_tensor(x, device="cuda")
    yd = torch.zeros((batch, n_out), dtype=torch.float32, device="cuda")
    net.forward(xd, yd)
    net.sync()
    y = yd.cpu().numpy()
    r = _ref_forward(net, net.params(), x, rounded=True).numpy()
    scale = max(1.0, np.abs(r).max())
    assert np.abs(y - r).max() < 1e-2 * scale, np.abs(y - r).max()


@pytest.mark.parametrize("n_in,width,depth,n_out,batch", SHAPES)
def test_gradients_match_autograd(Q, n_in, width, depth, n_out, batch):
    import torch
    print(f"[mlp] gradients {n_in}->{width}x{depth}->{n_out} batch {batch}", flush=True)
    net = Q.MLP(n_in, width, depth, n_out, max_batch=batch, seed=5)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (batch, n_in)).astype(np.float32)
    t = rng.normal(0, 1, (batch, n_out)).astype(np.float32)
    loss_d = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.backward(torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda"), loss_d)
    net.sync()
    g = net.grads()
    p = net.params()
    # autograd of the unrounded network, float64
    params = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for wb in _split(net, p) for a in wb]
    a = torch.as_tensor(x, dtype=torch.float64)
    for l in range(len(params) // 2):
        z = a @ params[2 * l] + params[2 * l + 1]
        a = z if l == len(params) // 2 - 1 else torch.nn.functional.gelu(z)
    loss = ((a - torch.as_tensor(t, dtype=torch.float64)) ** 2).mean()
    loss.backward()
    assert abs(loss_d.item() - loss.item()) < 2e-2 * loss.item()
    o = 0
    for q in params:
        n = q.numel()
        gr, gg = q.grad.numpy().ravel(), g[o:o + n].astype(np.float64)
        o += n
        rel = np.linalg.norm(gg - gr) / np.linalg.norm(gr)
        cos = gg @ gr / (np.linalg.norm(gg) * np.linalg.norm(gr))
        assert rel < 3e-2 and cos > 0.999, (q.shape, rel, cos)


def test_adam_step_matches_formula(Q):
    import torch
    net = Q.MLP(6, 64, 2, 4, max_batch=256, seed=7)
    rng = np.random.default_rng(3)
    x = torch.as_tensor(rng.uniform(-1, 1, (256, 6)).astype(np.float32), device="cuda")
    t = torch.as_tensor(rng.normal(0, 1, (256, 4)).astype(np.float32), device="cuda")
    p0 = net.params().astype(np.float64)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for step in range(1, 4):
        net.backward(x, t)
        net.sync()
        g = net.grads().astype(np.float64)
        net.adam(lr, b1, b2, eps)
        net.sync()
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p0 = p0 - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
        assert np.abs(net.params() - p0).max() < 1e-6, step


def test_training_reduces_loss(Q):
    """A smooth 6 -> 4 map: Adam on the library's kernels brings the loss down."""
    import torch
    rng = np.random.default_rng(4)
    B = 2048
    x = rng.uniform(-1, 1, (B, 6)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) * np.cos(x[:, 5]), x[:, 1] * x[:, 2], np.exp(-x[:, 3] ** 2),
                  0.5 * x[:, 4] + 0.1 * x[:, 0] ** 2], axis=1).astype(np.float32)
    net = Q.MLP(6, 256, 4, 4, max_batch=B, seed=11)
    xd, td = torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.backward(xd, td, loss)
    net.sync()
    first = loss.item()
    for _ in range(300):
        net.backward(xd, td, loss)
        net.adam(1e-3)
    net.sync()
    print(f"[mlp] loss {first:.3e} -> {loss.item():.3e}", flush=True)
    assert loss.item() < first / 20


def test_batch_bounds(Q):
    import torch
    net = Q.MLP(6, 32, 1, 4, max_batch=100, seed=1)
    x = torch.zeros((101, 6), device="cuda")
    y = torch.zeros((101, 4), device="cuda")
    with pytest.raises(Q.QuapiError) as e:
        net.forward(x, y)
    assert e.value.code == Q.QUAPI_EINVAL
    with pytest.raises(Q.QuapiError):
        net.forward(x[:0], y[:0])
    with pytest.raises(Q.QuapiError):
        net.adam(-1.0)
