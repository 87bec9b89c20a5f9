"""Pins of the proposal network's oracle (oracle/cnn.py) against brute force,
finite differences, closed-form special cases and gauge invariants."""
import numpy as np
import pytest

import synth
from oracle import cnn


def _brute_conv(x, W, b):
    n, cin, H, Wd = x.shape
    co = W.shape[0]
    y = np.zeros((n, co, H, Wd))
    for q in range(n):
        for o in range(co):
            for i in range(H):
                for j in range(Wd):
                    s = b[o]
                    for c in range(cin):
                        for di in range(3):
                            for dj in range(3):
                                s += W[o, c, di, dj] * x[q, c, (i + di - 1) % H, (j + dj - 1) % Wd]
                    y[q, o, i, j] = s
    return y


def test_conv3x3_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 6))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(cnn.conv3x3(x, W, b), _brute_conv(x, W, b), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("di,dj", [(0, 0), (0, 2), (2, 1), (1, 1)])
def test_conv3x3_delta_kernel_is_a_shift(di, dj):
    # a kernel with one unit tap reads x at (i + di - 1, j + dj - 1): the
    # orientation the C ABI documents for the weight layout
    x = np.arange(1 * 1 * 4 * 5, dtype=float).reshape(1, 1, 4, 5)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, di, dj] = 1.0
    y = cnn.conv3x3(x, W, np.zeros(1))
    for i in range(4):
        for j in range(5):
            assert y[0, 0, i, j] == x[0, 0, (i + di - 1) % 4, (j + dj - 1) % 5]


def test_conv3x3_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 4, 4))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    R = rng.standard_normal((2, 2, 4, 4))      # loss = sum(R * y)
    dx, dW, db = cnn.conv3x3_backward(x, W, R)
    h = 1e-6

    def f(x_, W_, b_):
        return float(np.sum(R * cnn.conv3x3(x_, W_, b_)))

    for idx in [(0, 0, 0, 0), (1, 2, 3, 1), (0, 1, 2, 3)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, W, b) - f(x - e, W, b)) / (2 * h) - dx[idx]) < 1e-7
    for idx in [(0, 0, 0, 0), (1, 2, 2, 1), (0, 1, 1, 2)]:
        e = np.zeros_like(W)
        e[idx] = h
        assert abs((f(x, W + e, b) - f(x, W - e, b)) / (2 * h) - dW[idx]) < 1e-7
    for o in range(2):
        e = np.zeros_like(b)
        e[o] = h
        assert abs((f(x, W, b + e) - f(x, W, b - e)) / (2 * h) - db[o]) < 1e-7


def test_output_channel_mapping():
    # channel 4k + 2s + c is component c (re, im) of spin s of vector k
    L1, L2 = 3, 2
    out = np.zeros((32, L2, L1))
    out[4 * 5 + 2 * 1 + 0, 1, 2] = 7.0
    out[4 * 5 + 2 * 1 + 1, 1, 2] = -3.0
    v = cnn.output_to_vectors(out)
    site = 1 * L1 + 2
    assert v[5, site, 1] == 7.0 - 3.0j
    assert np.count_nonzero(v) == 1
    rng = np.random.default_rng(3)
    o = rng.standard_normal((32, L2, L1))
    np.testing.assert_array_equal(cnn.vectors_to_output(cnn.output_to_vectors(o)).reshape(o.shape), o)


def _random_vecs(rng, nvec, V):
    return rng.standard_normal((nvec, V, 2)) + 1j * rng.standard_normal((nvec, V, 2))


def _block_sites(L1, L2, b=4):
    x2, x1 = np.meshgrid(np.arange(L2), np.arange(L1), indexing="ij")
    blk = ((x2 // b) * (L1 // b) + x1 // b).ravel()
    return [np.nonzero(blk == j)[0] for j in range(blk.max() + 1)]


def test_projection_loss_special_cases():
    rng = np.random.default_rng(4)
    L1 = L2 = 8
    V = L1 * L2
    t = _random_vecs(rng, 8, V)
    # predictions = targets mixed by an invertible matrix per block and spin: the span is
    # the same, only eps separates the loss from 0 (1 - sigma^2/(sigma^2 + eps) per direction)
    pred = np.empty_like(t)
    for sites in _block_sites(L1, L2):
        for s in range(2):
            M = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)) + 4 * np.eye(8)
            pred[:, sites, s] = M.T @ t[:, sites, s]
    l_same, _ = cnn.projection_loss(pred, t, (L1, L2), eps=1e-3)
    assert 0.0 <= l_same < 1e-3
    l0, _ = cnn.projection_loss(pred, t, (L1, L2), eps=0.0)
    assert abs(l0) < 1e-10
    # predictions supported on the first half of every block, targets on the second half:
    # every target is orthogonal to the predicted span, so each term is exactly 1
    p2 = np.zeros_like(t)
    t2 = np.zeros_like(t)
    for sites in _block_sites(L1, L2):
        p2[:, sites[:8], :] = _random_vecs(rng, 8, 8)
        t2[:, sites[8:], :] = _random_vecs(rng, 8, 8)
    l1, _ = cnn.projection_loss(p2, t2, (L1, L2))
    assert abs(l1 - 1.0) < 1e-14
    # loss does not depend on the normalisation or the phase of the targets
    l_a, _ = cnn.projection_loss(pred + 0.3 * p2, t, (L1, L2))
    l_b, _ = cnn.projection_loss(pred + 0.3 * p2, t * 2.5 * np.exp(0.7j), (L1, L2))
    assert abs(l_a - l_b) < 1e-14


def test_projection_loss_gradient_finite_differences():
    rng = np.random.default_rng(5)
    L1 = L2 = 8
    V = L1 * L2
    pred = _random_vecs(rng, 8, V)
    t = _random_vecs(rng, 8, V)
    _, g = cnn.projection_loss(pred, t, (L1, L2))
    h = 1e-6
    for idx in [(0, 0, 0), (3, 17, 1), (7, 63, 0), (5, 40, 1)]:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            e = np.zeros_like(pred)
            e[idx] = h * unit
            fd = (cnn.projection_loss(pred + e, t, (L1, L2))[0] - cnn.projection_loss(pred - e, t, (L1, L2))[0]) / (2 * h)
            assert abs(fd - 2.0 * part(g[idx])) < 1e-8


def test_tree_gauge_fixing():
    rng = synth.rng_for(7, 1)
    L1, L2 = 8, 12
    theta = synth.u1_heatbath(L1, L2, 3.0, 5, rng)
    phi = cnn.tree_gauge_phase(theta, (4, 4))
    tf = cnn.gauge_transform_u1(theta, phi)
    for y in range(L2):
        for x in range(L1):
            if x % 4 != 3:                  # x_1 links inside a block row
                assert abs(np.angle(np.exp(1j * tf[0, y, x]))) < 1e-12
            if x % 4 == 0 and y % 4 != 3:   # x_2 links along the first block column
                assert abs(np.angle(np.exp(1j * tf[1, y, x]))) < 1e-12
            if x % 4 == 0 and y % 4 == 0:
                assert phi[y, x] == 0.0
    # gauge invariants are unchanged
    np.testing.assert_allclose(np.cos(synth.u1_plaquette_angles(tf)), np.cos(synth.u1_plaquette_angles(theta)),
                               atol=1e-12)


def test_network_gradients_finite_differences():
    rng = np.random.default_rng(6)
    L1 = L2 = 8
    theta = rng.uniform(-np.pi, np.pi, (2, L2, L1))
    target = _random_vecs(rng, 8, L1 * L2)
    params = cnn.init_params(rng)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    loss, grads = cnn.loss_and_param_grads(params, theta, target)
    assert 0.0 < loss < 1.0
    h = 1e-5

    def f(ps):
        return cnn.loss_and_param_grads(ps, theta, target)[0]

    checks = [(0, "W", (5, 2, 1, 2)), (1, "W", (10, 33, 0, 0)), (2, "W", (63, 7, 2, 2)), (3, "W", (31, 1, 1, 0)),
              (0, "b", (3,)), (2, "b", (40,)), (3, "b", (17,))]
    for l, kind, idx in checks:
        def shifted(d):
            ps = [(W.copy(), b.copy()) for W, b in params]
            (ps[l][0] if kind == "W" else ps[l][1])[idx] += d
            return ps
        fd = (f(shifted(h)) - f(shifted(-h))) / (2 * h)
        an = (grads[l][0] if kind == "W" else grads[l][1])[idx]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (l, kind, idx, fd, an)
