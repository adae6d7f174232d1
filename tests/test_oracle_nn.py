"""Pins of the proposal network's CPU oracle (no GPU).

The convolution is checked against scipy's n-dimensional correlation, the
backward pieces against adjoint identities and central finite differences of
the forward function, the BF16 rounding against an integer bit-trick on float32
inputs, and Adam's first step against its closed form."""
import numpy as np
import pytest
from scipy import ndimage

import tdgl_inputs as I
from oracle import nn_oracle as N


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_bf16_rounding_ties_and_steps():
    e = 2.0 ** -8
    assert N.round_bf16(1.0 + e) == 1.0                       # tie -> even
    assert N.round_bf16(1.0 + 3 * e) == 1.0 + 4 * e           # tie -> even (upwards)
    assert N.round_bf16(1.0 + e + 2.0 ** -20) == 1.0 + 2 * e  # above the tie
    assert N.round_bf16(-1.5) == -1.5
    assert N.round_bf16(0.0) == 0.0
    assert N.round_bf16(255.0) == 255.0                      # 8 significant bits
    assert N.round_bf16(257.0) == 256.0                      # tie -> even
    assert N.round_bf16(259.0) == 260.0


def test_bf16_rounding_matches_bit_trick():
    x = _rng(1).normal(size=20000).astype(np.float32) * 10.0 ** _rng(2).integers(-8, 8, 20000)
    x = x.astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    want = r.astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(N.round_bf16(x.astype(np.float64)), want)


def test_conv3_matches_scipy_correlate():
    rng = _rng(3)
    x = rng.normal(size=(2, 3, 4, 5, 6))
    W = rng.normal(size=(4, 27, 3))
    b = rng.normal(size=4)
    out = N.conv3(x, W, b)
    for bb in range(2):
        for o in range(4):
            want = np.full(x.shape[2:], b[o])
            for c in range(3):
                k = W[o, :, c].reshape(3, 3, 3)          # [dz+1][dy+1][dx+1]
                want += ndimage.correlate(x[bb, c], k, mode="constant", cval=0.0)
            np.testing.assert_allclose(out[bb, o], want, rtol=1e-12, atol=1e-12)


def test_conv3_single_tap_is_a_shift():
    x = _rng(4).normal(size=(1, 1, 4, 4, 4))
    W = np.zeros((1, 27, 1))
    t = N.taps().index((1, 0, -1))
    W[0, t, 0] = 1.0
    out = N.conv3(x, W, np.zeros(1))[0, 0]
    want = np.zeros((4, 4, 4))
    want[:3, :, 1:] = x[0, 0, 1:, :, :3]
    np.testing.assert_array_equal(out, want)


def test_conv3_adjoints():
    rng = _rng(5)
    x = rng.normal(size=(2, 3, 4, 4, 6))
    g = rng.normal(size=(2, 5, 4, 4, 6))
    W = rng.normal(size=(5, 27, 3))
    b = rng.normal(size=5)
    lhs = (N.conv3(x, W, np.zeros(5)) * g).sum()
    assert abs(lhs - (x * N.conv3_input_grad(g, W)).sum()) < 1e-10 * abs(lhs)
    gW, gb = N.conv3_weight_grad(g, x)
    dW, db = rng.normal(size=W.shape), rng.normal(size=5)
    lhs = (N.conv3(x, dW, db) * g).sum()
    assert abs(lhs - (gW * dW).sum() - (gb * db).sum()) < 1e-10 * abs(lhs)


def test_pool_and_up():
    rng = _rng(6)
    x = rng.normal(size=(2, 3, 2, 4, 4))
    g = rng.normal(size=(2, 3, 4, 8, 8))
    np.testing.assert_allclose(N.pool(N.up(x)), x, rtol=0, atol=1e-15)
    assert abs((N.up(x) * g).sum() - (x * N.up_adjoint(g)).sum()) < 1e-12
    y = rng.normal(size=(2, 3, 4, 8, 8))
    assert abs((N.pool(y) * x).sum() - (y * N.pool_adjoint(x)).sum()) < 1e-12
    assert N.pool(np.full((1, 1, 2, 2, 2), 3.5))[0, 0, 0, 0, 0] == 3.5
    assert N.up(x)[1, 2, 3, 7, 6] == x[1, 2, 1, 3, 3]


def test_act():
    z = np.array([-2.0, -0.5, 0.0, 0.25, 3.0])
    np.testing.assert_array_equal(N.act(z), [-0.25, -0.0625, 0.0, 0.25, 3.0])
    np.testing.assert_array_equal(N.act_slope(N.act(z)), [0.125, 0.125, 0.125, 1.0, 1.0])


def test_net_input_channels():
    shape = (8, 8, 8)
    T, th, noise = I.net_conditions(2, shape, 4, seed=7, thickness_range=(3, 6))
    x, m = N.net_input(T, th, noise, shape)
    assert x.shape == (2, 5, 8, 8, 8)
    for b in range(2):
        t = int(th[b])
        assert (x[b, 1, :t] == 1).all() and (x[b, :, t:] == 0).all()
        np.testing.assert_allclose(x[b, 0, 0, 0, 0], (float(T[b]) - 350.0) / 100.0, rtol=1e-12)
        # noise cell (1, 0, 1) of the 2x2x2 noise grid covers z 4..7, y 0..3, x 4..7
        if t > 4:
            np.testing.assert_allclose(x[b, 2 + 1, 4, 3, 7], noise[b, 1, 1, 0, 1] * 10.0, rtol=1e-7)


def test_param_layout():
    assert N.layer_shapes(8) == I.net_layer_shapes(8)
    assert N.num_params(32) == 1721859
    th = I.net_params(8, seed=1)
    assert len(th) == N.num_params(8)
    L = N.unpack(th, 8)
    np.testing.assert_array_equal(N.pack(L), th.astype(np.float64))
    assert L[0][0].shape == (8, 27, 5) and L[11][0].shape == (3, 27, 8)


def _small_problem(width=4, seed=11, B=2, shape=(4, 8, 8), noise_div=4):
    T, th, noise = I.net_conditions(B, shape, noise_div, seed=seed, thickness_range=(2, 4))
    theta = I.net_params(width, seed=seed).astype(np.float64)
    rng = _rng(seed + 1)
    target = rng.uniform(-0.3, 0.3, size=(B, 3) + shape) * N.film_mask(th, shape)
    return theta, T, th, noise, target, shape


def test_loss_gradient_matches_finite_differences():
    theta, T, th, noise, target, shape = _small_problem()
    width = 4
    loss, P, g = N.loss_and_grad(theta, width, T, th, noise, target, shape)
    f = lambda t: N.loss_and_grad(t, width, T, th, noise, target, shape)[0]
    rng = _rng(12)
    # small steps: a larger one can carry a pre-activation across the kink of
    # the leaky ReLU
    for _ in range(3):                       # random directions
        v = rng.normal(size=theta.shape)
        h = 1e-7
        fd = (f(theta + h * v) - f(theta - h * v)) / (2 * h)
        assert abs(fd - g @ v) < 1e-6 * max(abs(fd), 1e-12), (fd, g @ v)
    # single coordinates in every layer: a weight and the bias
    k = 0
    for ci, co in N.layer_shapes(width):
        for idx in (k + rng.integers(co * 27 * ci), k + co * 27 * ci + rng.integers(co)):
            e = np.zeros_like(theta)
            e[idx] = 1.0
            h = 1e-7
            fd = (f(theta + h * e) - f(theta - h * e)) / (2 * h)
            assert abs(fd - g[idx]) < 1e-6 * max(abs(g).max(), 1e-12), (idx, fd, g[idx])
        k += co * 27 * ci + co


def test_loss_zero_at_target_and_masked():
    theta, T, th, noise, _, shape = _small_problem()
    P, _ = N.forward(theta, 4, T, th, noise, shape)
    for b in range(2):
        assert (P[b, :, int(th[b]):] == 0).all()
    loss, _, g = N.loss_and_grad(theta, 4, T, th, noise, P, shape)
    assert loss == 0.0 and not g.any()


def test_bf16_mode_is_close_to_exact():
    theta, T, th, noise, target, shape = _small_problem()
    l0, P0, g0 = N.loss_and_grad(theta, 4, T, th, noise, target, shape)
    l1, P1, g1 = N.loss_and_grad(theta, 4, T, th, noise, target, shape, bf16=True)
    assert np.linalg.norm(P1 - P0) < 0.05 * np.linalg.norm(P0)
    assert np.linalg.norm(g1 - g0) < 0.05 * np.linalg.norm(g0)


def test_adam_first_step_closed_form():
    rng = _rng(13)
    th, g = rng.normal(size=50), rng.normal(size=50)
    new, m, v = N.adam(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    np.testing.assert_allclose(new, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_symmetry_ops_are_symmetries_of_the_film_model():
    """The TDGL effective field of the open BaTiO3 box commutes with every
    in-plane op (all terms, a film under vacuum), which pins the op's
    position and component conventions."""
    from oracle import tdgl_oracle as O
    cfg = I.c5_recipe(3, (4, 6, 6))
    cfg["T"] = 280.0
    cfg["mimg"] = 0
    prob = O.Problem(cfg)
    P = _rng(21).uniform(-0.2, 0.2, size=(3, 4, 6, 6))
    P[:, 3:] = 0.0
    E = O.effective_field(P, prob)
    scale = np.abs(E).max()
    for op in range(8):
        got = O.effective_field(N.apply_op(P, op), prob)
        np.testing.assert_allclose(got, N.apply_op(E, op), rtol=0, atol=1e-12 * scale)


def test_symmetry_op_group_structure():
    F = _rng(22).normal(size=(2, 3, 2, 4, 4))
    for op in range(8):
        if op & 4 == 0:        # mirrors are involutions
            np.testing.assert_array_equal(N.apply_op(N.apply_op(F, op), op), F)
    np.testing.assert_array_equal(N.apply_op(N.apply_op(F, 4), 4), F)
    # swap then both mirrors is a rotation by pi/2: four times is the identity
    G = F
    for _ in range(4):
        G = N.apply_op(G, 5)
    np.testing.assert_array_equal(G, F)
    assert not np.array_equal(N.apply_op(F, 5), F)
