"""Pins of the FP64 network oracle (oracle/nn_oracle.py) against facts that do not come from it:
the convolution theorem, brute-force index loops, central finite differences of every backward,
and closed-form properties of Adam and of the trilinear prolongation."""
import numpy as np
import pytest

from oracle import nn_oracle as nn


def _corr_fft(x, k):
    """Periodic cross-correlation y[v] = sum_u x[u] k[u - v] via the convolution theorem."""
    return np.real(np.fft.ifftn(np.fft.fftn(x) * np.conj(np.fft.fftn(k))))


def test_conv3d_matches_fft_cross_correlation():
    rng = np.random.default_rng(1)
    B, n, cin, cout = 2, (6, 5, 4), 3, 2
    x = rng.standard_normal((B,) + n + (cin,))
    w = rng.standard_normal((27, cout, cin))
    b = rng.standard_normal(cout)
    y = nn.conv3d(x, w, b, 3)
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    for bi in range(B):
        for o in range(cout):
            ref = np.full(n, b[o])
            for k in range(cin):
                ker = np.zeros(n)
                for t, (dz, dy, dx) in enumerate(offs):
                    ker[dz % n[0], dy % n[1], dx % n[2]] += w[t, o, k]
                ref = ref + _corr_fft(x[bi, ..., k], ker)
            assert np.max(np.abs(y[bi, ..., o] - ref)) < 1e-12


def test_conv3d_brute_force_loops():
    rng = np.random.default_rng(2)
    n = (3, 4, 2)
    x = rng.standard_normal((1,) + n + (2,))
    w = rng.standard_normal((27, 3, 2))
    y = nn.conv3d(x, w, None, 3)
    for z in range(n[0]):
        for yy in range(n[1]):
            for xx in range(n[2]):
                for o in range(3):
                    s = 0.0
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                src = x[0, (z + dz) % n[0], (yy + dy) % n[1], (xx + dx) % n[2]]
                                s += float(np.dot(w[t, o], src))
                    assert abs(y[0, z, yy, xx, o] - s) < 1e-12
    # 1x1x1: a plain channel mix
    w1 = rng.standard_normal((1, 3, 2))
    assert np.allclose(nn.conv3d(x, w1, None, 1), x @ w1[0].T, atol=1e-14)


def _dd(f, x, d, h):
    return (f(x + h * d) - f(x - h * d)) / (2 * h)


@pytest.mark.parametrize("ksize", [1, 3])
def test_conv3d_backward_finite_differences(ksize):
    rng = np.random.default_rng(3 + ksize)
    taps = 27 if ksize == 3 else 1
    x = rng.standard_normal((2, 4, 3, 5, 3))
    w = rng.standard_normal((taps, 4, 3))
    b = rng.standard_normal(4)
    R = rng.standard_normal((2, 4, 3, 5, 4))
    dx, dw, db = nn.conv3d_backward(x, w, R, ksize)
    L = lambda xx, ww, bb: float(np.sum(R * nn.conv3d(xx, ww, bb, ksize)))
    for _ in range(3):
        d = rng.standard_normal(x.shape)
        assert abs(_dd(lambda t: L(t, w, b), x, d, 1e-3) - np.sum(dx * d)) < 1e-9
        d = rng.standard_normal(w.shape)
        assert abs(_dd(lambda t: L(x, t, b), w, d, 1e-3) - np.sum(dw * d)) < 1e-9
        d = rng.standard_normal(b.shape)
        assert abs(_dd(lambda t: L(x, w, t), b, d, 1e-3) - np.sum(db * d)) < 1e-9


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 4, 6, 2, 3))
    y = rng.standard_normal((2, 2, 3, 1, 3))
    # <pool2(x), y> = <x, pool2_backward(y)>, <up2(y), x> = <y, up2_backward(x)>
    assert abs(np.sum(nn.pool2(x) * y) - np.sum(x * nn.pool2_backward(y))) < 1e-12
    assert abs(np.sum(nn.up2(y) * x) - np.sum(y * nn.up2_backward(x))) < 1e-12
    # pool2 of an upsampled field returns it; pool2 of a constant is that constant
    assert np.allclose(nn.pool2(nn.up2(y)), y, atol=1e-15)
    assert np.allclose(nn.pool2(np.full((1, 4, 4, 4, 2), 3.5)), 3.5)
    assert nn.pool2(x)[0, 1, 2, 0, 1] == pytest.approx(x[0, 2:4, 4:6, 0:2, 1].mean(), abs=1e-15)


def test_architecture_shapes():
    specs = nn.layer_specs()
    assert [s[0] for s in specs] == ["enc0a", "enc0b", "enc1a", "enc1b", "enc2a", "enc2b", "enc3a", "enc3b",
                                     "dec2a", "dec2b", "dec1a", "dec1b", "dec0a", "dec0b", "head"]
    assert dict((s[0], (s[1], s[2])) for s in specs)["dec2a"] == (192, 64)
    p = nn.init_params(0)
    x = np.zeros((1, 8, 8, 8, 16))
    out, cache = nn.forward(p, x)
    assert out.shape == (1, 8, 8, 8, 48)
    assert cache["e3"].shape == (1, 1, 1, 1, 128) and cache["c0"].shape == (1, 8, 8, 8, 48)


def _unet_setup(seed, n=8, B=1):
    rng = np.random.default_rng(seed)
    p = nn.init_params(seed)
    p = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in p.items()}
    x = np.zeros((B, n, n, n, 16))
    x[..., 0] = rng.uniform(0, 1, (B, n, n, n))
    target = rng.standard_normal((B, n, n, n, 36))
    phi = x[..., 0]
    return rng, p, x, target, phi


def test_unet_backward_finite_differences():
    rng, p, x, target, phi = _unet_setup(7)
    inv = 1.0 / (phi.size * 36)

    def loss(params):
        out, _ = nn.forward(params, x)
        return nn.weighted_loss(out, target, phi, (0.1, 1.0, 0.5), inv)[0]

    out, cache = nn.forward(p, x)
    L, dout = nn.weighted_loss(out, target, phi, (0.1, 1.0, 0.5), inv)
    grads = nn.backward(p, cache, dout)
    # small enough that no ReLU pre-activation crosses zero along the probe for these seeds
    h = 1e-7
    for name, _, _, _ in nn.layer_specs():
        w, b = p[name]
        dw_dir = rng.standard_normal(w.shape)
        db_dir = rng.standard_normal(b.shape)
        pp = dict(p)
        pp[name] = (w + h * dw_dir, b + h * db_dir)
        lp = loss(pp)
        pp[name] = (w - h * dw_dir, b - h * db_dir)
        lm = loss(pp)
        fd = (lp - lm) / (2 * h)
        an = np.sum(grads[name][0] * dw_dir) + np.sum(grads[name][1] * db_dir)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, fd, an)


def test_weighted_loss_gradient():
    rng = np.random.default_rng(9)
    pred = rng.standard_normal((2, 2, 3, 2, 48))
    target = rng.standard_normal((2, 2, 3, 2, 36))
    phi = rng.uniform(0, 1, (2, 2, 3, 2))
    phi[0, 0, 0, :] = [0.0, 1.0]
    w3 = (0.25, 1.0, 2.0)
    L, g = nn.weighted_loss(pred, target, phi, w3, 0.01)
    assert np.all(g[..., 36:] == 0)
    d = rng.standard_normal(pred.shape)
    fd = _dd(lambda t: nn.weighted_loss(t, target, phi, w3, 0.01)[0], pred, d, 1e-4)
    assert abs(fd - np.sum(g * d)) < 1e-9
    # a perfect prediction has zero loss
    p2 = pred.copy()
    p2[..., :36] = target
    assert nn.weighted_loss(p2, target, phi, w3, 0.01)[0] == 0.0
    # one unit error in one voxel costs that voxel's weight: void 0.25, full 1.25, partial 0.25 + phi + 2
    one = np.zeros_like(pred)
    for ph, w in ((0.0, 0.25), (1.0, 1.25), (0.375, 2.625)):
        one[:] = 0.0
        one[0, 0, 0, 0, 0] = 1.0
        phi1 = np.zeros_like(phi)
        phi1[0, 0, 0, 0] = ph
        assert nn.weighted_loss(one, np.zeros_like(target), phi1, w3, 1.0)[0] == pytest.approx(w)


def test_adam_closed_forms():
    # constant gradient: bias correction makes every step lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    for step in range(1, 6):
        pn, m, v = nn.adam_step(p, g, m, v, 0.01, 0.9, 0.999, 1e-8, step)
        assert np.allclose(p - pn, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
        p = pn
    # minimises a quadratic
    p = np.array([3.0, -1.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for step in range(1, 3001):
        p, m, v = nn.adam_step(p, 2 * (p - np.array([0.5, 0.25])), m, v, 0.01, 0.9, 0.999, 1e-8, step)
    assert np.allclose(p, [0.5, 0.25], atol=1e-3)
    # decoupled from the sign convention: weight decay pulls towards zero
    pn, _, _ = nn.adam_step(np.array([1.0]), np.array([0.0]), np.zeros(1), np.zeros(1), 0.1, 0.9, 0.999, 1e-8, 1,
                            weight_decay=0.5)
    assert pn[0] == pytest.approx(0.9, abs=1e-6)


def test_restrict_and_prolong_properties():
    rng = np.random.default_rng(11)
    phi = rng.uniform(0, 1, (8, 12, 4))
    r = nn.restrict(phi, 4)
    assert r.shape == (2, 3, 1)
    assert r[1, 2, 0] == pytest.approx(phi[4:8, 8:12, 0:4].mean(), abs=1e-15)
    assert r.mean() == pytest.approx(phi.mean(), abs=1e-14)
    pred = rng.standard_normal((3, 4, 2, 48))
    E = rng.standard_normal(6)
    contracted = np.einsum("xyzjc,j->cxyz", pred[..., :36].reshape(3, 4, 2, 6, 6), E)
    # factor 1: fine centres coincide with coarse ones
    assert np.allclose(nn.prolong(pred, 1, E), contracted, atol=1e-13)
    # unit macro strain e_J selects channels 6J..6J+5
    e = np.zeros(6)
    e[4] = 1.0
    assert np.allclose(nn.prolong(pred, 1, e), np.moveaxis(pred[..., 24:30], -1, 0), atol=1e-15)
    # constants stay constant; periodic linear interpolation preserves the mean
    const = np.zeros((2, 2, 2, 48))
    const[..., :36] = 0.7
    f = nn.prolong(const, 4, np.ones(6))
    assert np.allclose(f, 4.2, atol=1e-13)
    f3 = nn.prolong(pred, 3, E)
    assert f3.shape == (6, 9, 12, 6)
    assert np.allclose(f3.mean(axis=(1, 2, 3)), contracted.mean(axis=(1, 2, 3)), atol=1e-12)
    # a fine centre midway between two coarse centres (factor 2, along the last axis) is their average
    p1 = np.zeros((1, 1, 4, 48))
    p1[0, 0, :, 0] = [1.0, 3.0, 5.0, 11.0]
    e0 = np.zeros(6)
    e0[0] = 1.0
    line = nn.prolong(p1, 2, e0)[0, 0, 0]
    # fine x=1 lies at coarse 0.25 between centres 0 and 1; x=0 at -0.25 between 3 (wrap) and 0
    assert line[1] == pytest.approx(0.75 * 1.0 + 0.25 * 3.0)
    assert line[0] == pytest.approx(0.25 * 11.0 + 0.75 * 1.0)
