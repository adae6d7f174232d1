"""GPU parity of the proposal network's kernels against the CPU oracle.

Single convolutions and weight gradients are compared bit for bit: their
inputs are small multiples of 1/4 and 1/8, so every product and partial sum
is exact in FP32 and the only rounding is the final one to BF16, which both
sides take from the same exact value.  The whole network is compared with
the oracle in its BF16 mode (the same rounding points as the kernels); the
remaining differences come from FP32 accumulation order, which can move a
stored value across a BF16 rounding boundary (one unit of 2^-8 relative) --
the tolerances below allow a few such flips per layer."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import tdgl_inputs as I  # noqa: E402
from oracle import nn_oracle as N  # noqa: E402
from tests.gpu_helpers import announce  # noqa: E402


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def to_bf16_bits(x):
    """Exact BF16 encoding of values that are BF16 numbers (test data only)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32)
    assert not (u & 0xFFFF).any(), "value is not a BF16 number"
    return (u >> 16).astype(np.uint16)


def from_bf16_bits(h):
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def channels_last(x, c_p):
    """[B][C][Z][Y][X] -> [B*Z*Y*X][c_p] (zero padding)."""
    B, C = x.shape[:2]
    out = np.zeros((B,) + x.shape[2:] + (c_p,))
    out[..., :C] = np.moveaxis(x, 1, -1)
    return out.reshape(-1, c_p)


def from_channels_last(y, B, C, shape):
    return np.moveaxis(y.reshape((B,) + tuple(shape) + (y.shape[-1],))[..., :C], -1, 1)


def dev_bf16(x_cl):
    return torch.from_numpy(to_bf16_bits(x_cl).view(np.int16)).cuda()


def host_bf16(t):
    return from_bf16_bits(t.cpu().numpy().view(np.uint16))


def weights_dev(W, cin_p, cout_p):
    cout, _, cin = W.shape
    Wp = np.zeros((cout_p, 27, cin_p))
    Wp[:cout, :, :cin] = W
    return dev_bf16(Wp.reshape(cout_p, 27 * cin_p))


CONV_CASES = [  # cin, cout, cin_p, cout_p, nb, (lz, ly, lx), up2
    (5, 8, 16, 16, 3, (2, 3, 3), 0),
    (16, 32, 16, 32, 5, (3, 2, 2), 0),      # 160 positions: a ragged last group
    (32, 64, 32, 64, 2, (2, 3, 3), 1),      # input read through 2x repetition
    (64, 128, 64, 128, 2, (2, 2, 3), 0),
    (128, 64, 128, 64, 1, (2, 3, 3), 1),
    (32, 256, 32, 256, 1, (2, 2, 2), 0),    # two channel blocks
    # grids of at least 8 x 16 (y, x) take the LDS-tiled kernel
    (5, 32, 16, 32, 2, (2, 3, 4), 0),
    (32, 64, 32, 64, 1, (2, 4, 5), 1),
    (64, 128, 64, 128, 2, (1, 3, 4), 0),
    (128, 32, 128, 32, 1, (2, 3, 4), 1),
    (16, 16, 16, 16, 3, (1, 3, 4), 0),
]


@pytest.mark.parametrize("case", CONV_CASES, ids=lambda c: "c%d-%d_nb%d_up%d" % (c[0], c[1], c[4], c[6]))
def test_conv3_epilogues_bit_exact(case):
    cin, cout, cin_p, cout_p, nb, (lz, ly, lx), up2 = case
    announce("nn conv3 %s" % (case,))
    rng = _rng(100 + cin + cout)
    shape = (1 << lz, 1 << ly, 1 << lx)
    in_shape = tuple(s // 2 for s in shape) if up2 else shape
    x = rng.integers(-4, 5, size=(nb, cin) + in_shape) / 4.0
    W = rng.integers(-4, 5, size=(cout, 27, cin)) / 8.0
    b = rng.integers(-8, 9, size=cout) / 16.0
    aux = rng.integers(-4, 5, size=(nb, cout) + shape) / 4.0
    xin = N.up(x) if up2 else x
    acc = N.conv3(xin, W, np.zeros(cout))
    t = N.round_bf16(N.act(acc + b[None, :, None, None, None]))
    want = {
        0: (t, None),
        1: (t, N.round_bf16(t + aux)),
        3: (N.round_bf16(acc), None),
        4: (N.round_bf16(acc * N.act_slope(aux)), None),
        5: (N.round_bf16(acc), N.round_bf16(acc * N.act_slope(aux))),
    }
    din = dev_bf16(channels_last(x, cin_p))
    dw = weights_dev(W, cin_p, cout_p)
    bias = torch.zeros(cout_p, dtype=torch.float32, device="cuda")
    bias[:cout] = torch.from_numpy(b.astype(np.float32)).cuda()
    daux = dev_bf16(channels_last(aux, cout_p))
    npos = nb * shape[0] * shape[1] * shape[2]
    from paper_2605_28800_amd import proposal as PR
    for epi, (w1, w2) in want.items():
        out = torch.full((npos, cout_p), 0x7FC0, dtype=torch.int16, device="cuda")
        out2 = torch.full((npos, cout_p), 0x7FC0, dtype=torch.int16, device="cuda")
        PR.nn_conv3(epi, din, dw, bias, nb, lx, ly, lz, cin_p, cout_p, out=out, out2=out2,
                    aux=daux, in_up2=up2)
        torch.cuda.synchronize()
        got = from_channels_last(host_bf16(out), nb, cout, shape)
        np.testing.assert_array_equal(got, w1, err_msg="epilogue %d out" % epi)
        if w2 is not None:
            got2 = from_channels_last(host_bf16(out2), nb, cout, shape)
            np.testing.assert_array_equal(got2, w2, err_msg="epilogue %d out2" % epi)


def test_conv3_output_epilogue_exact():
    announce("nn conv3 P epilogue")
    rng = _rng(7)
    nb, (lz, ly, lx), cin = 3, (3, 2, 3), 32
    shape = (1 << lz, 1 << ly, 1 << lx)
    x = rng.integers(-4, 5, size=(nb, cin) + shape) / 4.0
    W = rng.integers(-4, 5, size=(3, 27, cin)) / 8.0
    b = rng.integers(-8, 9, size=3) / 16.0
    thick = np.array([8.0, 3.0, 5.0], dtype=np.float32)
    want = N.film_mask(thick, shape) * N.conv3(x, W, b)
    bias = torch.zeros(16, dtype=torch.float32, device="cuda")
    bias[:3] = torch.from_numpy(b.astype(np.float32)).cuda()
    P = torch.full((nb, 3) + shape, float("nan"), dtype=torch.float32, device="cuda")
    from paper_2605_28800_amd import proposal as PR
    PR.nn_conv3(PR.EPI_P, dev_bf16(channels_last(x, cin)), weights_dev(W, cin, 16), bias, nb,
                lx, ly, lz, cin, 16, P=P, thick=torch.from_numpy(thick).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(P.cpu().numpy().astype(np.float64), want)


WGRAD_CASES = [  # cin, cout, cin_p, cout_p, nb, (lz, ly, lx), up2
    (5, 8, 16, 16, 3, (2, 3, 3), 0),
    (16, 32, 16, 32, 5, (3, 2, 2), 0),
    (32, 64, 32, 64, 9, (3, 3, 3), 0),      # several position splits
    (64, 32, 64, 32, 2, (2, 3, 3), 1),
    (128, 128, 128, 128, 1, (2, 2, 3), 0),
    (16, 256, 16, 256, 2, (2, 2, 2), 0),
]


@pytest.mark.parametrize("case", WGRAD_CASES, ids=lambda c: "c%d-%d_nb%d_up%d" % (c[0], c[1], c[4], c[6]))
def test_conv3_weight_gradient_bit_exact(case):
    cin, cout, cin_p, cout_p, nb, (lz, ly, lx), up2 = case
    announce("nn wgrad %s" % (case,))
    rng = _rng(200 + cin + cout)
    shape = (1 << lz, 1 << ly, 1 << lx)
    in_shape = tuple(s // 2 for s in shape) if up2 else shape
    x = rng.integers(-4, 5, size=(nb, cin) + in_shape) / 4.0
    g = rng.integers(-4, 5, size=(nb, cout) + shape) / 4.0
    gW, gb = N.conv3_weight_grad(g, N.up(x) if up2 else x)
    from paper_2605_28800_amd import proposal as PR
    grad = PR.nn_conv3_wgrad(dev_bf16(channels_last(g, cout_p)), dev_bf16(channels_last(x, cin_p)),
                             nb, lx, ly, lz, cin_p, cout_p, in_up2=up2)
    torch.cuda.synchronize()
    grad = grad.cpu().numpy().astype(np.float64)
    gw = grad[:cout_p * 27 * cin_p].reshape(cout_p, 27, cin_p)
    np.testing.assert_array_equal(gw[:cout, :, :cin], gW)
    assert not gw[cout:].any() and not gw[:, :, cin:].any()
    np.testing.assert_array_equal(grad[cout_p * 27 * cin_p:][:cout], gb)


# ------------------------------------------------------------------ network
def _net_problem(width=8, shape=(8, 16, 16), noise_div=4, B=3, seed=5):
    T, th, noise = I.net_conditions(B, shape, noise_div, seed=seed, thickness_range=(3, shape[0]))
    theta = I.net_params(width, seed=seed)
    rng = _rng(seed + 1)
    target = (rng.uniform(-0.3, 0.3, size=(B, 3) + shape) * N.film_mask(th, shape)).astype(np.float32)
    return theta, T, th, noise, target


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - b) / max(np.linalg.norm(b), 1e-300))


def _ulps(got, ref):
    """Per-element |got - ref| in BF16 units in the last place (2^-8) of the
    element's magnitude, or of the array's RMS where the element is smaller."""
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), np.sqrt(np.mean(ref ** 2)))
    return np.abs(np.asarray(got, dtype=np.float64) - ref) / (scale * 2.0 ** -8)


@pytest.mark.parametrize("width,shape,noise_div", [(8, (8, 16, 16), 4), (16, (4, 8, 8), 2)])
def test_network_forward_backward_against_oracle(width, shape, noise_div):
    announce("net forward/backward w=%d shape=%s" % (width, shape))
    from paper_2605_28800_amd.proposal import Net
    theta, T, th, noise, target = _net_problem(width, shape, noise_div)
    B = len(T)
    net = Net(shape, width=width, noise_div=noise_div, max_batch=4)
    try:
        net.set_params(theta)
        np.testing.assert_array_equal(net.get_params(), theta)
        dT, dth, dn, dt = _dev(T), _dev(th), _dev(noise), _dev(target)
        P = net.forward(dT, dth, dn).cpu().numpy()
        loss, g = net.loss_grad(dT, dth, dn, dt)
        # the same rows through an index array, in another order
        perm = np.array([2, 0, 1], dtype=np.int32)
        Pp = net.forward(dT, dth, dn, idx=_dev(perm, torch.int32)).cpu().numpy()
    finally:
        net.close()
    ol, oP, og = N.loss_and_grad(theta.astype(np.float64), width, T, th, noise, target, shape,
                                 bf16=True)
    np.testing.assert_array_equal(Pp, P[perm])
    for b in range(B):
        assert not P[b, :, int(th[b]):].any()
    assert _rel(P, oP) < 5e-3, _rel(P, oP)
    assert abs(loss - ol) < 5e-3 * ol, (loss, ol)
    assert _rel(g, og) < 1e-2, _rel(g, og)
    # element by element against the oracle's BF16 mode: the two round the
    # same sums in different orders, so a few BF16 roundings flip; measured
    # at most 0.45 (output) and 1.0 (gradient) units of 2^-8
    film = np.broadcast_to((N.film_mask(th, shape)[:, 0] > 0)[:, None], P.shape)
    assert _ulps(P, oP)[film].max() <= 2.0
    assert _ulps(g, og).max() <= 4.0
    k = 0
    for li, (ci, co) in enumerate(N.layer_shapes(width)):
        n = co * 27 * ci + co
        assert _rel(g[k:k + n], og[k:k + n]) < 3e-2, (li, _rel(g[k:k + n], og[k:k + n]))
        k += n
    # and the exact function, for scale: BF16 storage moves it by about 2^-8
    el, eP, eg = N.loss_and_grad(theta.astype(np.float64), width, T, th, noise, target, shape)
    assert _rel(P, eP) < 5e-2 and _rel(g, eg) < 1e-1


def test_adam_first_step_from_zero_weights():
    """All weights zero: P = 0, only the output biases get a gradient, and
    Adam's first step moves each by about -lr * sign(gradient)."""
    announce("net adam first step")
    from paper_2605_28800_amd.proposal import Net
    width, shape = 8, (4, 8, 8)
    _, T, th, noise, target = _net_problem(width, shape, 2, B=2, seed=9)
    theta = np.zeros(N.num_params(width), dtype=np.float32)
    _, _, og = N.loss_and_grad(theta.astype(np.float64), width, T, th, noise, target, shape,
                               bf16=True)
    net = Net(shape, width=width, noise_div=2, max_batch=2)
    try:
        net.set_params(theta)
        loss, g = net.loss_grad(_dev(T), _dev(th), _dev(noise), _dev(target))
        net.adam(1e-3)
        new = net.get_params()
    finally:
        net.close()
    nz = np.flatnonzero(og)
    np.testing.assert_array_equal(nz, np.arange(len(theta) - 3, len(theta)))
    np.testing.assert_allclose(g[-3:], og[-3:], rtol=1e-5)
    assert not g[:-3].any()
    # the first step of Adam from zero moments: -lr g / (|g| + eps)
    np.testing.assert_allclose(new[-3:], -1e-3 * og[-3:] / (np.abs(og[-3:]) + 1e-8), rtol=2e-6)
    assert not new[:-3].any()


def test_training_lowers_the_loss():
    announce("net training steps")
    from paper_2605_28800_amd.proposal import Net
    width, shape = 8, (4, 8, 8)
    theta, T, th, noise, _ = _net_problem(width, shape, 2, B=4, seed=11)
    target = I.noise_start(noise, th, shape)       # a learnable map of the inputs
    net = Net(shape, width=width, noise_div=2, max_batch=4)
    try:
        net.set_params(theta)
        idx = _dev(np.tile(np.arange(4, dtype=np.int32), 60), torch.int32)
        losses = net.train(idx, 4, _dev(T), _dev(th), _dev(noise), _dev(target), 3e-3)
    finally:
        net.close()
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])


def test_symmetry_ops_in_the_loss_against_oracle():
    """Samples under in-plane symmetry ops: the kernels read the noise field
    and the target through the op; the oracle applies the op to the arrays."""
    announce("net loss under symmetry ops")
    from paper_2605_28800_amd.proposal import Net
    width, shape, nd = 8, (8, 16, 16), 4
    theta, T, th, noise, target = _net_problem(width, shape, nd, B=4, seed=17)
    ops = np.array([0, 3, 5, 6], dtype=np.int32)
    noise_op = np.stack([N.apply_op(noise[i], int(o)) for i, o in enumerate(ops)])
    target_op = np.stack([N.apply_op(target[i], int(o)) for i, o in enumerate(ops)])
    ol, oP, og = N.loss_and_grad(theta.astype(np.float64), width, T, th, noise_op, target_op,
                                 shape, bf16=True)
    net = Net(shape, width=width, noise_div=nd, max_batch=4)
    try:
        net.set_params(theta)
        loss, g = net.loss_grad(_dev(T), _dev(th), _dev(noise), _dev(target),
                                ops=_dev(ops, torch.int32))
        loss0, _ = net.loss_grad(_dev(T), _dev(th), _dev(noise), _dev(target))
    finally:
        net.close()
    assert abs(loss - ol) < 5e-3 * ol, (loss, ol)
    assert _rel(g, og) < 1e-2, _rel(g, og)
    assert abs(loss - loss0) > 1e-3 * loss0        # the ops do change the samples


def test_network_error_paths_leave_it_usable():
    announce("net error paths")
    import ctypes
    import paper_2605_28800_amd as T
    from paper_2605_28800_amd.proposal import Net
    width, shape = 8, (4, 8, 8)
    theta, Tk, th, noise, target = _net_problem(width, shape, 2, B=2, seed=23)
    net = Net(shape, width=width, noise_div=2, max_batch=2)
    try:
        L = T.lib()
        dT, dth, dn, dt = _dev(Tk), _dev(th), _dev(noise), _dev(target)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())
        # Adam before any gradient
        assert L.tdgl_net_adam(net.h, 1e-3, 0.9, 0.999, 1e-8) == T.TDGL_E_STATE
        # batch above max_batch, zero steps, bad hyper-parameters, wrong count
        assert L.tdgl_net_forward(net.h, 3, None, ptr(dT), ptr(dth), ptr(dn), None) == T.TDGL_E_ARG
        idx = _dev(np.zeros(2, dtype=np.int32), torch.int32)
        assert L.tdgl_net_train(net.h, 0, 2, ptr(idx), None, ptr(dT), ptr(dth), ptr(dn), ptr(dt),
                                1e-3, 0.9, 0.999, 1e-8, None) == T.TDGL_E_ARG
        assert L.tdgl_net_train(net.h, 1, 2, ptr(idx), None, ptr(dT), ptr(dth), ptr(dn), ptr(dt),
                                -1.0, 0.9, 0.999, 1e-8, None) == T.TDGL_E_ARG
        short = np.zeros(10, dtype=np.float32)
        assert L.tdgl_net_set_params(net.h, short.ctypes.data_as(ctypes.c_void_p), 10) == T.TDGL_E_ARG
        # still usable, and the profile leaves the parameters as they were
        net.set_params(theta)
        P = net.forward(dT, dth, dn)
        assert torch.isfinite(P).all()
        ms = net.profile(2, dT, dth, dn, dt, reps=2)
        assert all(v > 0 for v in ms)
        np.testing.assert_array_equal(net.get_params(), theta)
        P2 = net.forward(dT, dth, dn)
        assert torch.equal(P, P2)
    finally:
        net.close()


@pytest.mark.timeout(600)
def test_network_forward_at_the_workload_size():
    """One 64x64x16 sample through the width-32 network (the shapes, tiles
    and kernels the learned-proposal workload runs) against the oracle.

    At this size BF16 storage alone moves the output by ~9e-3 (relative L2)
    from the exact FP64 function, and two BF16 computations whose FP32 sums
    run in different orders flip different roundings, so they differ by
    about half of that (measured 5.1e-3, uniform over tiles, rows, layers
    and components).  The test therefore asks (1) the GPU to be within 1e-2
    of the oracle's BF16 mode and (2) to be as far from the exact function
    as the oracle's BF16 mode is, to 10 % -- an indexing or epilogue error
    would add to (2).  The oracle's two forward passes take about two
    minutes on the host."""
    announce("net forward 64x64x16 width 32")
    from paper_2605_28800_amd.proposal import Net
    shape, width = (16, 64, 64), 32
    T, th, noise = I.net_conditions(2, shape, 8, seed=31, thickness_range=(8, 16))
    theta = I.net_params(width, seed=31)
    net = Net(shape, width=width, noise_div=8, max_batch=2)
    try:
        net.set_params(theta)
        P = net.forward(_dev(T), _dev(th), _dev(noise)).cpu().numpy()
    finally:
        net.close()
    th64 = theta.astype(np.float64)
    ref, _ = N.forward(th64, width, T[:1], th[:1], noise[:1], shape, bf16=True)
    exact, _ = N.forward(th64, width, T[:1], th[:1], noise[:1], shape, bf16=False)
    e_bf16 = _rel(ref, exact)
    assert _rel(P[:1], ref) < 1e-2, _rel(P[:1], ref)
    assert abs(_rel(P[:1], exact) - e_bf16) < 0.1 * e_bf16, (_rel(P[:1], exact), e_bf16)
    # element by element: flipped BF16 roundings spread through twelve
    # layers (measured: median 0.6, max 9.4 units of 2^-8, 0.8 % of the film
    # cells above 4); an indexing error moves whole tiles by ~2^8 units
    film = np.broadcast_to((N.film_mask(th[:1], shape)[:, 0] > 0)[:, None], P[:1].shape)
    u = _ulps(P[:1], ref)[film]
    assert u.max() <= 16.0, u.max()
    assert (u > 4.0).mean() <= 0.02, (u > 4.0).mean()
    assert not P[1, :, int(th[1]):].any()


def _sparse_dyadic_params(width, rng):
    """Every output channel of every layer reads one input channel at one
    tap, with weight +-1/2 or +-1, and a bias in multiples of 1/8: each
    convolution output is one product plus the bias, so every FP32 sum the
    kernels form is exact and both sides round the same numbers to BF16."""
    parts = []
    for ci, co in N.layer_shapes(width):
        W = np.zeros((co, 27, ci))
        W[np.arange(co), rng.integers(0, 27, co), rng.integers(0, ci, co)] = \
            rng.choice([-1.0, -0.5, 0.5, 1.0], co)
        parts += [W.ravel(), rng.integers(-4, 5, co) / 8.0]
    return np.concatenate(parts).astype(np.float32)


def _exact_in_fp32(theta, width, T, th, noise, shape):
    """The oracle's pre-rounding values of every layer are FP32 numbers
    (the construction's premise, checked rather than assumed)."""
    P, c = N.forward(theta, width, T, th, noise, shape, bf16=True)
    L = c["L"]
    pre = [N.conv3(c["x"], *L[0]), N.conv3(c["e0a"], *L[1]), N.pool(c["e0"]),
           N.conv3(c["p1"], *L[2]), N.conv3(c["e1a"], *L[3]), N.pool(c["e1"]),
           N.conv3(c["p2"], *L[4]), N.conv3(c["b1"], *L[5]), N.conv3(c["b2"], *L[6]),
           N.conv3(N.up(c["b3"]), *L[7]), c["t8"] + c["e1"], N.conv3(c["u1"], *L[8]),
           N.conv3(N.up(c["u1b"]), *L[9]), c["t10"] + c["e0"], N.conv3(c["u0"], *L[10]), P]
    return all(np.array_equal(v.astype(np.float32).astype(np.float64), v) for v in pre), P


@pytest.mark.parametrize("width,shape,noise_div", [(8, (8, 16, 16), 4), (16, (8, 32, 32), 8)])
def test_network_forward_bit_exact_on_a_sparse_dyadic_network(width, shape, noise_div):
    """Whole-network parity element by element: with one product per
    convolution output (sparse weights of +-1/2, +-1 and dyadic biases,
    dyadic noise, T at the centre of the temperature scale) no FP32 sum
    depends on its order, so the GPU's output equals the oracle's BF16 mode
    bit for bit at every element -- through every tap, channel, pooling,
    repetition, skip sum, mask and the output layer's layout."""
    announce("net sparse dyadic forward w=%d shape=%s" % (width, shape))
    from paper_2605_28800_amd.proposal import Net
    rng = _rng(41 + width)
    B = 3
    Z, Y, X = shape
    T = np.full(B, 350.0, np.float32)
    th = np.array([Z, Z // 2 + 1, 3], np.float32)
    noise = (rng.integers(-100, 101, size=(B, 3, Z // noise_div, Y // noise_div, X // noise_div))
             / 1024.0).astype(np.float32)
    theta = _sparse_dyadic_params(width, rng)
    exact, ref = _exact_in_fp32(theta.astype(np.float64), width, T, th, noise, shape)
    assert exact
    assert np.count_nonzero(ref) > 0.3 * ref.size * th.mean() / Z
    net = Net(shape, width=width, noise_div=noise_div, max_batch=B)
    try:
        net.set_params(theta)
        P = net.forward(_dev(T), _dev(th), _dev(noise)).cpu().numpy()
    finally:
        net.close()
    np.testing.assert_array_equal(P.astype(np.float64), ref)
