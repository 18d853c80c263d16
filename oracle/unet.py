"""NumPy reference of the learned grid preconditioner -- TEST INFRASTRUCTURE.

The paper has no learned component; this is the project's addition on top of
the AIMx solve (a 3-D U-Net mapping the projected residual on the AIM grid to
a correction on the grid).  The reference fixes the network's definition so
that the GPU kernels can be checked against it:

* tensors are channels-last, [z][y][x][c], float64 here;
* conv3(x, W, b)[p, co] = b[co] + sum_{t, ci} x[p + d(t), ci] W[co, t, ci]
  over the 27 offsets d(t) = (dx, dy, dz) in {-1,0,1}^3 with t = (dz+1)*9 +
  (dy+1)*3 + (dx+1), zero outside the grid ("same" padding);
* pool: 2x2x2 average; up: nearest-neighbour x2; cat: channel concatenation;
* layers (channels): c0 = C, c1 = 2C, c2 = 4C
    a0 = relu(conv3(in, 2 -> c0));  s0 = relu(conv3(a0, c0 -> c0))
    a1 = relu(conv3(pool(s0), c0 -> c1)); s1 = relu(conv3(a1, c1 -> c1))
    a2 = relu(conv3(pool(s1), c1 -> c2)); a3 = relu(conv3(a2, c2 -> c2))
    a4 = relu(conv3(cat(up(a3), s1), c2 + c1 -> c1)); a5 = relu(conv3(a4, c1 -> c1))
    a6 = relu(conv3(cat(up(a5), s0), c1 + c0 -> c0)); a7 = relu(conv3(a6, c0 -> c0))
    out = a7 W10^T + b10   (1x1x1, c0 -> 2)
* loss = mean over all entries of (out - target)^2.

``bf16=True`` rounds weights and every stored activation to bfloat16 (round
to nearest even) at the points where the GPU stores them, so that the device
result can be compared at accumulation-order accuracy.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even)."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layer_shapes(C: int = 16):
    """(name, cout, cin, taps) of every layer, in parameter order."""
    c0, c1, c2 = C, 2 * C, 4 * C
    return [("conv0", c0, 2, 27), ("conv1", c0, c0, 27), ("conv2", c1, c0, 27),
            ("conv3", c1, c1, 27), ("conv4", c2, c1, 27), ("conv5", c2, c2, 27),
            ("conv6", c1, c2 + c1, 27), ("conv7", c1, c1, 27), ("conv8", c0, c1 + c0, 27),
            ("conv9", c0, c0, 27), ("out", 2, c0, 1)]


def init_params(C: int = 16, seed: int = 0):
    """He-normal weights W[co, t, ci] and zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for name, co, ci, t in layer_shapes(C):
        std = np.sqrt(2.0 / (ci * t)) if name != "out" else np.sqrt(1.0 / (ci * t))
        params.append((rng.standard_normal((co, t, ci)) * std, np.zeros(co)))
    return params


def shift(x, d):
    """y[z, y, x] = x[z + dz, y + dy, x + dx] with zeros outside."""
    dx, dy, dz = d
    D, H, W = x.shape[:3]
    out = np.zeros_like(x)
    zs = slice(max(0, -dz), min(D, D - dz))
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    zi = slice(max(0, dz), min(D, D + dz))
    yi = slice(max(0, dy), min(H, H + dy))
    xi = slice(max(0, dx), min(W, W + dx))
    out[zs, ys, xs] = x[zi, yi, xi]
    return out


def conv3(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, d in enumerate(TAPS):
        y += shift(x, d) @ W[:, t, :].T
    return y + b


def conv3_bruteforce(x, W, b):
    D, H, Wd, Ci = x.shape
    y = np.zeros((D, H, Wd, W.shape[0]))
    for z in range(D):
        for yy in range(H):
            for xx in range(Wd):
                acc = b.copy()
                for t, (dx, dy, dz) in enumerate(TAPS):
                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                    if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < Wd:
                        acc += W[:, t, :] @ x[zz, y2, x2]
                y[z, yy, xx] = acc
    return y


def conv3_backward(x, W, dy):
    """Gradients of sum(dy * conv3(x, W, b)) w.r.t. x, W and b."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, d in enumerate(TAPS):
        xs = shift(x, d)
        dW[:, t, :] = dy.reshape(-1, dy.shape[-1]).T @ xs.reshape(-1, xs.shape[-1])
        dx += shift(dy @ W[:, t, :], tuple(-v for v in d))
    return dx, dW, dy.reshape(-1, dy.shape[-1]).sum(axis=0)


def pool(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_backward(dy):
    D, H, W, C = dy.shape
    return dy.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


class UNet:
    def __init__(self, params, bf16: bool = False):
        self.bf16 = bf16
        r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
        self.params = [(r(W), np.asarray(b, dtype=np.float64)) for W, b in params]
        self._r = r

    def forward(self, x):
        r = self._r
        P = self.params
        act = {}
        act["in"] = r(x)
        act["a0"] = r(relu(conv3(act["in"], *P[0])))
        act["s0"] = r(relu(conv3(act["a0"], *P[1])))
        act["p0"] = r(pool(act["s0"]))
        act["a1"] = r(relu(conv3(act["p0"], *P[2])))
        act["s1"] = r(relu(conv3(act["a1"], *P[3])))
        act["p1"] = r(pool(act["s1"]))
        act["a2"] = r(relu(conv3(act["p1"], *P[4])))
        act["a3"] = r(relu(conv3(act["a2"], *P[5])))
        act["c1"] = np.concatenate([up(act["a3"]), act["s1"]], axis=-1)
        act["a4"] = r(relu(conv3(act["c1"], *P[6])))
        act["a5"] = r(relu(conv3(act["a4"], *P[7])))
        act["c0"] = np.concatenate([up(act["a5"]), act["s0"]], axis=-1)
        act["a6"] = r(relu(conv3(act["c0"], *P[8])))
        act["a7"] = r(relu(conv3(act["a6"], *P[9])))
        W, b = P[10]
        act["out"] = act["a7"] @ W[:, 0, :].T + b
        self.act = act
        return act["out"]

    def loss(self, x, target):
        out = self.forward(x)
        return float(np.mean((out - target) ** 2))

    def backward(self, target):
        """Parameter gradients of the mean-squared loss after forward()."""
        a = self.act
        return self.backward_from(2.0 * (a["out"] - target) / a["out"].size)

    def backward_from(self, dout):
        """Parameter gradients of a loss whose gradient with respect to the
        output is ``dout`` (same shape as the output), after forward()."""
        a = self.act
        P = self.params
        g = [None] * len(P)
        W, _ = P[10]
        g[10] = (np.einsum("zyxo,zyxi->oi", dout, a["a7"])[:, None, :], dout.reshape(-1, 2).sum(0))
        d = (dout @ W[:, 0, :]) * (a["a7"] > 0)

        def step(i, xin, dy, mask_src=None):
            dx, dW, db = conv3_backward(xin, P[i][0], dy)
            g[i] = (dW, db)
            return dx

        d = step(9, a["a6"], d) * (a["a6"] > 0)
        dc0 = step(8, a["c0"], d)
        c_up = a["a5"].shape[-1]
        d_s0 = dc0[..., c_up:]
        d = up_backward(dc0[..., :c_up]) * (a["a5"] > 0)
        d = step(7, a["a4"], d) * (a["a4"] > 0)
        dc1 = step(6, a["c1"], d)
        c_up = a["a3"].shape[-1]
        d_s1 = dc1[..., c_up:]
        d = up_backward(dc1[..., :c_up]) * (a["a3"] > 0)
        d = step(5, a["a2"], d) * (a["a2"] > 0)
        d = step(4, a["p1"], d)
        d = (pool_backward(d) + d_s1) * (a["s1"] > 0)
        d = step(3, a["a1"], d) * (a["a1"] > 0)
        d = step(2, a["p0"], d)
        d = (pool_backward(d) + d_s0) * (a["s0"] > 0)
        d = step(1, a["a0"], d) * (a["a0"] > 0)
        step(0, a["in"], d)
        return g
