"""Pins of the FP64 reference of the warm-start network (CPU).

The convolution is checked against its definition written as plain loops and
against scipy's n-dimensional correlation; the backward pass against central
finite differences of the forward pass; the subspace loss against finite
differences and its invariance under rotations of the predicted basis.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def _loops_conv(x, w, b, s):
    n, c, d = x.shape[0], x.shape[1], x.shape[2]
    od = (d - 1) // s + 1
    y = np.zeros((n, w.shape[0], od, od, od))
    for a in range(n):
        for o in range(w.shape[0]):
            for i in range(od):
                for j in range(od):
                    for k in range(od):
                        t = b[o]
                        for cc in range(c):
                            for p in range(3):
                                for q in range(3):
                                    for r in range(3):
                                        zi, zj, zk = s * i + p - 1, s * j + q - 1, s * k + r - 1
                                        if 0 <= zi < d and 0 <= zj < d and 0 <= zk < d:
                                            t += w[o, cc, p, q, r] * x[a, cc, zi, zj, zk]
                        y[a, o, i, j, k] = t
    return y


@pytest.mark.parametrize("stride", [1, 2])
def test_conv3d_matches_definition(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 2, 5, 5, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(cnn.conv3d(x, w, b, stride), _loops_conv(x, w, b, stride), rtol=1e-13, atol=1e-12)


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 1, 7, 7, 7))
    w = rng.standard_normal((1, 1, 3, 3, 3))
    ref = ndimage.correlate(x[0, 0], w[0, 0], mode="constant", cval=0.0)
    assert np.allclose(cnn.conv3d(x, w, np.zeros(1), 1)[0, 0], ref, rtol=1e-13, atol=1e-12)
    # stride 2 samples every other output of the stride-1 map
    assert np.allclose(cnn.conv3d(x, w, np.zeros(1), 2)[0, 0], ref[::2, ::2, ::2], rtol=1e-13, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = cnn.init_params(c_in=2, width=3, n_out=4, seed=7)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)   # nonzero biases, generic ReLU pattern
    x = rng.standard_normal((2, 2, 6, 6, 6))
    gout = rng.standard_normal((2, 4))
    _, acts = cnn.forward(p, x)
    grads = cnn.backward(p, acts, gout)
    f = lambda q: float(np.sum(gout * cnn.forward(q, x)[0]))
    eps = 1e-6
    for name in ("w0", "b0", "w2", "b3", "wl", "bl"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            q = {k: v.copy() for k, v in p.items()}
            q[name].reshape(-1)[idx] += eps
            fp = f(q)
            q[name].reshape(-1)[idx] -= 2 * eps
            fm = f(q)
            fd = (fp - fm) / (2 * eps)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)


def test_projector_loss_gradient_and_rotation_invariance():
    rng = np.random.default_rng(4)
    cs, _ = np.linalg.qr(rng.standard_normal((8, 3)))
    c = rng.standard_normal((1, 8, 3))
    loss, g = cnn.projector_loss(c, cs[None])
    eps = 1e-6
    for idx in range(0, 24, 5):
        d = np.zeros(24)
        d[idx] = eps
        lp, _ = cnn.projector_loss(c + d.reshape(1, 8, 3), cs[None])
        lm, _ = cnn.projector_loss(c - d.reshape(1, 8, 3), cs[None])
        assert abs((lp - lm) / (2 * eps) - g.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(g.reshape(-1)[idx]))
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    lq, _ = cnn.projector_loss(c @ q, cs[None])
    assert abs(lq - loss) <= 1e-10 * max(1.0, loss)
    # an orthonormal basis of the same subspace has zero loss
    l0, g0 = cnn.projector_loss((cs @ q)[None], cs[None])
    assert l0 <= 1e-24 and np.abs(g0).max() <= 1e-12


def test_bf16_rounding_ties_to_even_and_matches_torch():
    u = 2.0 ** -7                               # bfloat16 spacing on [1, 2)
    assert cnn.bf16(np.array([1 + u / 2]))[0] == 1.0            # tie, even neighbour 1
    assert cnn.bf16(np.array([1 + 1.5 * u]))[0] == 1 + 2 * u    # tie, even neighbour 1 + 2u
    assert cnn.bf16(np.array([1 + 0.51 * u]))[0] == 1 + u
    assert cnn.bf16(np.array([-3.0]))[0] == -3.0 and cnn.bf16(np.array([0.0]))[0] == 0.0
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(4096) * np.exp(rng.uniform(-20, 20, 4096))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(x.astype(np.float64)), ref)


def test_bf16_network_rounds_only_the_stored_values():
    rng = np.random.default_rng(6)
    p = cnn.init_params(c_in=2, width=3, n_out=4, seed=8)
    x = rng.standard_normal((2, 2, 5, 5, 5))
    out, acts = cnn.forward(p, x, use_bf16=True)
    for a in acts[:5]:
        assert np.array_equal(cnn.bf16(a), a)
    # weights that are already bfloat16 values and a bfloat16 input: the
    # rounded network differs from the exact one only by the rounding of the
    # stored activations, a relative 2^-9 per layer
    q = {k: (cnn.bf16(v) if k in ("w0", "w1", "w2", "w3") else v) for k, v in p.items()}
    ref, _ = cnn.forward(q, cnn.bf16(x))
    assert np.linalg.norm(out - ref) <= 4 * 5 * 2.0 ** -9 * np.linalg.norm(ref)
    # the BF16 backward equals the FP64 backward of the network with rounded weights at the rounded activations
    gout = rng.standard_normal((2, 4))
    g1 = cnn.backward(p, acts, gout, use_bf16=True)
    g2 = cnn.backward(q, acts, gout)
    for k in g1:
        assert np.array_equal(g1[k], g2[k])
