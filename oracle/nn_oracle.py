"""FP64 CPU oracle of the learned warm start's network: periodic 3-D convolutions, pooling,
upsampling, the 4-level encoder-decoder, its weighted loss, the hand-written backward pass and
Adam, plus the restriction/prolongation that carry fields between the solver grid and the
network grid.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU baseline may use it;
the product path never does.  Plain numpy in float64, one library matmul per convolution tap; no
blocking or fusion.  Pinned in tests/test_nn_oracle_pins.py by the convolution theorem (FFT
cross-correlation), brute-force loops on tiny inputs, central finite differences of every
backward, and closed-form properties of Adam and of the trilinear prolongation.

Network (not in the paper, whose solver always starts from zero; Sec. 2 eq. galres fixes only the
system the start is fed into):
  input  [B, n, n, n, 16]: channel 0 = voxel solid fraction phi, channels 1-15 zero
  level l = 0..3 at n / 2^l voxels per axis with C = (16, 32, 64, 128) channels:
    encoder: a_0 = input, a_l = pool2(e_{l-1});  h_l = relu(conv3(a_l)),  e_l = relu(conv3(h_l))
    decoder: d_3 = e_3;  c_l = concat(up2(d_{l+1}), e_l);  g_l = relu(conv3(c_l)),  d_l = relu(conv3(g_l))
  head: out = conv1(d_0), 48 FP32 channels; channel 6J + c is component c of the strain
        fluctuation for unit Mandel macro strain e_J (J, c < 6), channels 36-47 unused.
Weights are W[tap][n][k], tap = (dz+1)*9 + (dy+1)*3 + (dx+1), biases b[n].
"""
from __future__ import annotations

import numpy as np

CHANNELS = (16, 32, 64, 128)
IN_CH = 16
OUT_CH = 48
N_TARGET = 36


def layer_specs():
    """(name, cin, cout, ksize) of every convolution, in forward order."""
    c = CHANNELS
    specs = [("enc0a", IN_CH, c[0], 3), ("enc0b", c[0], c[0], 3)]
    for l in range(1, 4):
        specs += [(f"enc{l}a", c[l - 1], c[l], 3), (f"enc{l}b", c[l], c[l], 3)]
    for l in (2, 1, 0):
        specs += [(f"dec{l}a", c[l + 1] + c[l], c[l], 3), (f"dec{l}b", c[l], c[l], 3)]
    specs.append(("head", c[0], OUT_CH, 1))
    return specs


def _offsets(ksize):
    if ksize == 1:
        return [(0, 0, 0)]
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, off):
    """s[v] = x[v + off] with periodic wrap (x: [B, D, H, W, C])."""
    return np.roll(x, shift=(-off[0], -off[1], -off[2]), axis=(1, 2, 3))


def conv3d(x, w, b, ksize):
    """y[v][n] = sum_tap sum_k x[v + off(tap)][k] w[tap][n][k] + b[n]  (periodic)."""
    B, D, H, W, K = x.shape
    N = w.shape[1]
    y = np.zeros((B, D, H, W, N))
    for t, off in enumerate(_offsets(ksize)):
        y += (_shift(x, off).reshape(-1, K) @ w[t].T).reshape(B, D, H, W, N)
    if b is not None:
        y += b
    return y


def conv3d_backward(x, w, dy, ksize):
    """Gradients of conv3d: (dx, dw, db)."""
    B, D, H, W, K = x.shape
    N = w.shape[1]
    dyf = dy.reshape(-1, N)
    dx = np.zeros_like(x, dtype=np.float64)
    dw = np.zeros_like(w, dtype=np.float64)
    for t, off in enumerate(_offsets(ksize)):
        dw[t] = dyf.T @ _shift(x, off).reshape(-1, K)
        # y[v] reads x[v + off]  =>  x[u] receives dy[u - off]
        dx += _shift((dyf @ w[t]).reshape(B, D, H, W, K), (-off[0], -off[1], -off[2]))
    db = dyf.sum(axis=0)
    return dx, dw, db


def relu(x):
    return np.maximum(x, 0.0)


def pool2(x):
    B, D, H, W, C = x.shape
    return x.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(dy):
    B, D, H, W, C = dy.shape
    return dy.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


def init_params(seed: int = 0, scale: float = 1.0):
    """He-normal weights, zero biases, as float64 (name -> (w, b))."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, cin, cout, k in layer_specs():
        taps = 27 if k == 3 else 1
        std = scale * np.sqrt(2.0 / (taps * cin))
        p[name] = (rng.standard_normal((taps, cout, cin)) * std, np.zeros(cout))
    return p


def forward(params, x):
    """Encoder-decoder forward; returns (out [B,n,n,n,48], cache of every activation)."""
    cache = {"in": x}
    a = x
    for l in range(4):
        if l > 0:
            a = pool2(cache[f"e{l - 1}"])
            cache[f"a{l}"] = a
        wa, ba = params[f"enc{l}a"]
        wb, bb = params[f"enc{l}b"]
        h = relu(conv3d(a, wa, ba, 3))
        cache[f"h{l}"] = h
        cache[f"e{l}"] = relu(conv3d(h, wb, bb, 3))
    d = cache["e3"]
    for l in (2, 1, 0):
        c = np.concatenate([up2(d), cache[f"e{l}"]], axis=-1)
        cache[f"c{l}"] = c
        wa, ba = params[f"dec{l}a"]
        wb, bb = params[f"dec{l}b"]
        g = relu(conv3d(c, wa, ba, 3))
        cache[f"g{l}"] = g
        d = relu(conv3d(g, wb, bb, 3))
        cache[f"d{l}"] = d
    w, b = params["head"]
    out = conv3d(d, w, b, 1)
    return out, cache


def backward(params, cache, dout):
    """Gradients of every parameter given dL/dout: name -> (dw, db)."""
    grads = {}
    C = CHANNELS
    dx, dw, db = conv3d_backward(cache["d0"], params["head"][0], dout, 1)
    grads["head"] = (dw, db)
    dd = dx * (cache["d0"] > 0)
    de_skip = {}
    for l in (0, 1, 2):
        dx, dw, db = conv3d_backward(cache[f"g{l}"], params[f"dec{l}b"][0], dd, 3)
        grads[f"dec{l}b"] = (dw, db)
        dg = dx * (cache[f"g{l}"] > 0)
        dx, dw, db = conv3d_backward(cache[f"c{l}"], params[f"dec{l}a"][0], dg, 3)
        grads[f"dec{l}a"] = (dw, db)
        dc = dx
        dup = dc[..., :C[l + 1]]
        de_skip[l] = dc[..., C[l + 1]:]
        dd = up2_backward(dup)
        src = "e3" if l == 2 else f"d{l + 1}"
        dd = dd * (cache[src] > 0)
    # dd is now dL/d(pre-activation of e3)
    de = dd
    for l in (3, 2, 1, 0):
        if l < 3:
            de = (de_skip[l] + pool2_backward(da)) * (cache[f"e{l}"] > 0)  # noqa: F821 (da from level l+1)
        dx, dw, db = conv3d_backward(cache[f"h{l}"], params[f"enc{l}b"][0], de, 3)
        grads[f"enc{l}b"] = (dw, db)
        dh = dx * (cache[f"h{l}"] > 0)
        a = cache["in"] if l == 0 else cache[f"a{l}"]
        dx, dw, db = conv3d_backward(a, params[f"enc{l}a"][0], dh, 3)
        grads[f"enc{l}a"] = (dw, db)
        da = dx
    return grads


def loss_weight(phi, weight3):
    """w(v) = weight3[0] + weight3[1] phi[v] + weight3[2] (1 if 0 < phi[v] < 1 else 0)."""
    a, b, c = weight3
    return a + b * phi + c * ((phi > 0) & (phi < 1))


def weighted_loss(pred, target, phi, weight3, inv_norm, n_target=N_TARGET):
    """L = inv_norm * sum_v sum_{c < n_target} w(v) (pred[v][c] - target[v][c])^2, w = loss_weight(phi, weight3).

    pred [B,n,n,n,48], target [B,n,n,n,n_target] (channels-last here), phi [B,n,n,n].
    Returns (L, dL/dpred)."""
    w = loss_weight(phi, weight3)[..., None]
    d = pred[..., :n_target] - target
    L = inv_norm * float(np.sum(w * d * d))
    g = np.zeros_like(pred, dtype=np.float64)
    g[..., :n_target] = 2.0 * w * d * inv_norm
    return L, g


def adam_step(p, g, m, v, lr, beta1, beta2, eps, step, weight_decay=0.0):
    """One Adam step with bias correction (returns new p, m, v)."""
    g = g + weight_decay * p
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def restrict(phi, factor):
    """Mean of phi [n0,n1,n2] over factor^3 blocks."""
    n0, n1, n2 = phi.shape
    return phi.reshape(n0 // factor, factor, n1 // factor, factor, n2 // factor, factor).mean(axis=(1, 3, 5))


def prolong(pred, factor, macro_strain):
    """Fine starting field [6, f n0, f n1, f n2] from a coarse prediction pred [n0,n1,n2,>=36]:
    eps[c] = sum_J E[J] * periodic trilinear interpolation of pred[..., 6J + c] at the fine voxel
    centres, the centre of coarse voxel i lying at fine coordinate (i + 1/2) f - 1/2."""
    c0, c1, c2 = pred.shape[:3]
    E = np.asarray(macro_strain, dtype=np.float64)
    field = np.einsum("xyzjc,j->cxyz", pred[..., :36].reshape(c0, c1, c2, 6, 6), E)
    out = field
    for axis, n in ((1, c0), (2, c1), (3, c2)):
        out = _lerp_axis(out, axis, n, factor)
    return out


def _lerp_axis(a, axis, n, f):
    pos = (np.arange(n * f) + 0.5) / f - 0.5
    i0 = np.floor(pos).astype(int)
    t = pos - i0
    lo = np.take(a, i0 % n, axis=axis)
    hi = np.take(a, (i0 + 1) % n, axis=axis)
    shape = [1] * a.ndim
    shape[axis] = n * f
    t = t.reshape(shape)
    return (1 - t) * lo + t * hi
