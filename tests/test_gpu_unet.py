"""GPU U-Net kernels against the NumPy reference (oracle/unet.py): forward
output, gradients of every layer, and training progress.  The reference is
evaluated with the same bfloat16 rounding points as the kernels, so the
remaining differences come from accumulation order (forward) and from the
bfloat16 storage of gradient tensors between layers (backward)."""
import numpy as np
import pytest

from oracle import unet as ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2009_02281_amd import binding  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def grid_c64(shape_zyx, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(shape_zyx + (2,)).astype(np.float32)
    return g


def to_dev(g):
    return torch.from_numpy(np.ascontiguousarray(g)).view(torch.complex64)[..., 0].cuda()


@pytest.mark.parametrize("shape", [(8, 8, 16), (12, 8, 8)])
def test_forward_matches_reference(shape):
    net = binding.UNet(seed=5)
    p = binding.unet_params_to_layers(net.params())
    x = grid_c64(shape, 7)
    out = net.forward(to_dev(x)).cpu().numpy()
    out = np.stack([out.real, out.imag], axis=-1)
    want = ref.UNet(p, bf16=True).forward(x.astype(np.float64))
    err = rel(out, want)
    print(f"[gpu] unet forward {shape}: rel err {err:.2e}", flush=True)
    assert err <= 1e-2
    net.close()


def test_gradients_match_reference():
    net = binding.UNet(seed=11)
    rng = np.random.default_rng(12)
    flat = net.params()
    layers = binding.unet_params_to_layers(flat)
    # small random biases so that no layer is silent
    off = 0
    for W, b in layers:
        off += W.size
        flat[off:off + b.size] = 0.05 * rng.standard_normal(b.size)
        off += b.size
    net.set_params(flat)
    layers = binding.unet_params_to_layers(flat)
    shape = (8, 8, 16)
    x = grid_c64(shape, 13)
    t = grid_c64(shape, 14)
    loss = net.train_grid(to_dev(x), to_dev(t), apply=False)
    g = binding.unet_params_to_layers(net.grads())
    r = ref.UNet(layers, bf16=True)
    want_loss = r.loss(x.astype(np.float64), t.astype(np.float64))
    gw = r.backward(t.astype(np.float64))
    assert loss == pytest.approx(want_loss, rel=1e-2)
    for i, ((dW, db), (rW, rb)) in enumerate(zip(g, gw)):
        e_w, e_b = rel(dW, rW), rel(db, rb)
        print(f"    layer {i}: dW {e_w:.2e} db {e_b:.2e}", flush=True)
        assert e_w <= 3e-2 and e_b <= 3e-2, i
    net.close()


def test_batched_forward_equals_each_sample():
    """A batch is stacked along z; each sample's output must equal the one it
    gets alone, bit for bit (the same products in the same order), also
    where a 4-plane brick straddles two samples (12 planes deep: the coarsest
    level is 3 planes per sample)."""
    net = binding.UNet(seed=5)
    shape = (12, 8, 16)
    xs = [grid_c64(shape, 40 + i) for i in range(3)]
    out = net.forward(torch.stack([to_dev(x) for x in xs]))
    for i, x in enumerate(xs):
        assert torch.equal(out[i], net.forward(to_dev(x))), i
    net.close()


def test_batched_gradients_match_reference():
    """Loss and gradients of a batch of two: the batch mean of the oracle's
    per-sample losses and gradients."""
    net = binding.UNet(seed=15)
    layers = binding.unet_params_to_layers(net.params())
    shape = (12, 8, 8)
    xs = [grid_c64(shape, 50 + i) for i in range(2)]
    ts = [grid_c64(shape, 60 + i) for i in range(2)]
    loss = net.train_grid(torch.stack([to_dev(x) for x in xs]),
                          torch.stack([to_dev(t) for t in ts]), apply=False)
    g = binding.unet_params_to_layers(net.grads())
    r = ref.UNet(layers, bf16=True)
    want_loss, want = 0.0, None
    for x, t in zip(xs, ts):
        want_loss += 0.5 * r.loss(x.astype(np.float64), t.astype(np.float64))
        gi = r.backward(t.astype(np.float64))
        gi = [(0.5 * W, 0.5 * b) for W, b in gi]
        want = gi if want is None else [(W + a, b + c) for (W, b), (a, c) in zip(want, gi)]
    assert loss == pytest.approx(want_loss, rel=1e-2)
    for i, ((dW, db), (rW, rb)) in enumerate(zip(g, want)):
        e_w, e_b = rel(dW, rW), rel(db, rb)
        print(f"    layer {i}: dW {e_w:.2e} db {e_b:.2e}", flush=True)
        assert e_w <= 3e-2 and e_b <= 3e-2, i
    net.close()


def test_training_reduces_loss_and_weights_roundtrip(tmp_path):
    net = binding.UNet(seed=21)
    shape = (8, 8, 8)
    xs = [to_dev(grid_c64(shape, 30 + i)) for i in range(4)]
    # a fixed, learnable target: a smoothed copy of the input
    ts = []
    for x in xs:
        h = x.cpu().numpy()
        sm = (np.roll(h, 1, 0) + h + np.roll(h, -1, 0)) / 3.0
        ts.append(torch.from_numpy(sm.astype(np.complex64)).cuda())
    X = torch.stack(xs)
    T = torch.stack(ts)
    first = net.train_grid(X, T, lr=2e-3)
    for _ in range(60):
        last = net.train_grid(X, T, lr=2e-3)
    print(f"[gpu] unet training loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.5 * first
    path = str(tmp_path / "w.bin")
    net.save(path)
    net2 = binding.UNet.load(path)
    assert np.array_equal(net.params(), net2.params())
    assert torch.equal(net.forward(X), net2.forward(X))
    net.close()
    net2.close()


def test_64cubed_forward_and_gradients_match_reference():
    """One 64^3 grid, the size the benchmark's U-Net leg times.  At this size
    the full-resolution layers with 16 output channels give at least 1,024
    four-row bricks, so the four-row ("tall") convolution variants run, for
    the forward pass and for the data gradients, together with the weight
    gradient kernels of every layer at this size.  The calls are the ones
    the benchmark makes (forward of one grid; a training step of one grid),
    so every kernel variant it times is compared here with the oracle."""
    net = binding.UNet(seed=31)
    rng = np.random.default_rng(32)
    flat = net.params()
    off = 0
    for W, b in binding.unet_params_to_layers(flat):
        off += W.size
        flat[off:off + b.size] = 0.05 * rng.standard_normal(b.size)
        off += b.size
    net.set_params(flat)
    layers = binding.unet_params_to_layers(flat)
    shape = (64, 64, 64)
    x = grid_c64(shape, 33)
    t = grid_c64(shape, 34)
    print(f"[gpu] unet 64^3 forward + gradients", flush=True)
    out = net.forward(to_dev(x)).cpu().numpy()
    out = np.stack([out.real, out.imag], axis=-1)
    r = ref.UNet(layers, bf16=True)
    want = r.forward(x.astype(np.float64))
    err = rel(out, want)
    print(f"    forward rel err {err:.2e}", flush=True)
    assert err <= 1e-2
    loss = net.train_grid(to_dev(x), to_dev(t), apply=False)
    g = binding.unet_params_to_layers(net.grads())
    want_loss = r.loss(x.astype(np.float64), t.astype(np.float64))
    gw = r.backward(t.astype(np.float64))
    assert loss == pytest.approx(want_loss, rel=1e-2)
    for i, ((dW, db), (rW, rb)) in enumerate(zip(g, gw)):
        e_w, e_b = rel(dW, rW), rel(db, rb)
        print(f"    layer {i}: dW {e_w:.2e} db {e_b:.2e}", flush=True)
        assert e_w <= 3e-2 and e_b <= 3e-2, i
    net.close()
