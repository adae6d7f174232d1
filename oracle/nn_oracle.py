"""CPU oracle of the learned initial-state proposal -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy definition of the small 3-D convolutional encoder-decoder
that proposes an initial polarisation for the TDGL relaxation.  The network is
not part of the paper's method; the paper notes (section 5) that the solver
can generate datasets for data-driven methods, and this network is trained on
states the solver relaxed.  Imported only by the tests and the benchmark; the
product library shares no code with it.

Definition (all arrays [batch][channel][z][y][x]):

* Input, 5 channels, every one multiplied by the film mask m (1 in the layers
  z < thickness, 0 in the vacuum above): (T - 350 K)/100 K, m, and the three
  components of a low-resolution noise field (C/m^2, upsampled by repetition
  to the cell grid) times 10 m^2/C.
* conv3: 3x3x3 cross-correlation with zero padding and a bias,
  out[o, p] = b[o] + sum_t sum_c W[o, t, c] x[c, p + d_t], where tap
  t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) and d_t = (dz, dy, dx).
* act: leaky ReLU with slope 1/8 for negative arguments.
* pool: mean over 2x2x2 blocks; up: nearest-neighbour repetition by 2.
* Layers (width w): e0a = act(conv(x; 5->w)), e0 = act(conv(e0a; w->w)),
  e1a = act(conv(pool e0; w->2w)), e1 = act(conv(e1a; 2w->2w)),
  b1 = act(conv(pool e1; 2w->4w)), b2, b3 = act(conv(.; 4w->4w)),
  u1 = act(conv(up b3; 4w->2w)) + e1, u1b = act(conv(u1; 2w->2w)),
  u0 = act(conv(up u1b; 2w->w)) + e0, u0b = act(conv(u0; w->w)),
  P = m * conv(u0b; w->3)  (C/m^2, no activation).
* Loss: sum over samples, components and film cells of (P - P_target)^2
  divided by 3 x the number of film cells in the batch.
* Adam (Kingma and Ba 2015) with bias correction on FP32 master weights.
* Training augmentation: a sample may be taken under an in-plane symmetry op
  (apply_op on its noise field and target); the open film is invariant
  under these ops.

Parameters are one flat vector: per layer, W as [cout][27][cin] in C order,
then b [cout].

With ``bf16=True`` the oracle rounds (to nearest, ties to even, to 8
significant bits) exactly where the GPU kernels store BF16 values: the
weights used by the convolutions, the input tensor, every activation, the
skip sums, the pooled tensors and the back-propagated activation gradients.
Weight gradients, biases, the output P and the loss stay unrounded.  With
``bf16=False`` it is the exact FP64 function, which the finite-difference
pins test.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.125        # leaky ReLU slope for negative arguments
T_CENTER, T_SCALE = 350.0, 100.0
NOISE_GAIN = 10.0    # m^2/C


# --------------------------------------------------------------- rounding
def round_bf16(x):
    """Round FP64 values to the nearest BF16 number (8 significant bits),
    ties to even; zeros, infinities and NaNs pass through."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    # 8 significant bits: a multiple of 2^-8 for m
    r = np.ldexp(np.round(np.ldexp(m, 8)), e - 8)
    return np.where(np.isfinite(x), r, x)


def _ident(x):
    return x


# ----------------------------------------------------------------- layers
def taps():
    """The 27 tap offsets (dz, dy, dx) in tap order."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(x, d):
    """y[..., z, y, x] = x[..., z + dz, y + dy, x + dx], zero outside."""
    Z, Y, X = x.shape[-3:]
    p = np.pad(x, [(0, 0)] * (x.ndim - 3) + [(1, 1)] * 3)
    dz, dy, dx = d
    return p[..., 1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X]


def conv3(x, W, b):
    """3x3x3 zero-padded cross-correlation: x [B][Cin][Z][Y][X], W [Cout][27][Cin]."""
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for t, d in enumerate(taps()):
        out += np.einsum("oc,bczyx->bozyx", W[:, t, :], _shifted(x, d))
    return out + b[None, :, None, None, None]


def conv3_input_grad(g, W):
    """Adjoint of conv3 in x: gx[c, p] = sum_t sum_o W[o, t, c] g[o, p - d_t]."""
    out = np.zeros((g.shape[0], W.shape[2]) + g.shape[2:])
    for t, d in enumerate(taps()):
        out += np.einsum("oc,bozyx->bczyx", W[:, t, :], _shifted(g, tuple(-v for v in d)))
    return out


def conv3_weight_grad(g, x):
    """Gradients of sum(g * conv3(x, W, b)) in W [Cout][27][Cin] and b."""
    gW = np.zeros((g.shape[1], 27, x.shape[1]))
    for t, d in enumerate(taps()):
        gW[:, t, :] = np.einsum("bozyx,bczyx->oc", g, _shifted(x, d))
    return gW, g.sum(axis=(0, 2, 3, 4))


def act(z):
    return np.where(z > 0, z, SLOPE * z)


def act_slope(y):
    """Derivative of act, read from its output (same sign as its input)."""
    return np.where(y > 0, 1.0, SLOPE)


def pool(x):
    B, C, Z, Y, X = x.shape
    return x.reshape(B, C, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(3, 5, 7))


def pool_adjoint(g):
    return np.repeat(np.repeat(np.repeat(g, 2, 2), 2, 3), 2, 4) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 2), 2, 3), 2, 4)


def up_adjoint(g):
    B, C, Z, Y, X = g.shape
    return g.reshape(B, C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(axis=(3, 5, 7))


# ---------------------------------------------------------------- network
def layer_shapes(width):
    """(cin, cout) of the twelve convolutions."""
    w = width
    return [(5, w), (w, w), (w, 2 * w), (2 * w, 2 * w), (2 * w, 4 * w), (4 * w, 4 * w),
            (4 * w, 4 * w), (4 * w, 2 * w), (2 * w, 2 * w), (2 * w, w), (w, w), (w, 3)]


def num_params(width):
    return sum(co * 27 * ci + co for ci, co in layer_shapes(width))


def unpack(theta, width):
    """Flat parameter vector -> list of (W [cout][27][cin], b [cout])."""
    out, k = [], 0
    for ci, co in layer_shapes(width):
        W = np.asarray(theta[k:k + co * 27 * ci], dtype=np.float64).reshape(co, 27, ci)
        k += co * 27 * ci
        b = np.asarray(theta[k:k + co], dtype=np.float64)
        k += co
        out.append((W, b))
    assert k == len(theta)
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def film_mask(thickness, shape):
    """m [B][1][Z][Y][X]: 1 in the layers z < thickness of each sample."""
    Z, Y, X = shape
    z = np.arange(Z)
    m = (z[None, :] < np.asarray(thickness, float)[:, None]).astype(np.float64)
    return np.broadcast_to(m[:, None, :, None, None], (len(thickness), 1, Z, Y, X)).copy()


def net_input(T, thickness, noise, shape):
    """The 5-channel input.  noise [B][3][Z/s][Y/s][X/s] (C/m^2)."""
    Z, Y, X = shape
    noise = np.asarray(noise, dtype=np.float64)
    s = Z // noise.shape[2]
    assert noise.shape[2] * s == Z and noise.shape[3] * s == Y and noise.shape[4] * s == X
    n = np.repeat(np.repeat(np.repeat(noise, s, 2), s, 3), s, 4)
    m = film_mask(thickness, shape)
    Tn = (np.asarray(T, float)[:, None, None, None, None] - T_CENTER) / T_SCALE
    return np.concatenate([m * Tn, m, m * n * NOISE_GAIN], axis=1), m


def forward(theta, width, T, thickness, noise, shape, bf16=False):
    """P [B][3][Z][Y][X] and the stored tensors the backward pass needs."""
    r = round_bf16 if bf16 else _ident
    L = [(r(W), b) for W, b in unpack(theta, width)]
    x, m = net_input(T, thickness, noise, shape)
    c = {"x": r(x), "m": m, "L": L}
    c["e0a"] = r(act(conv3(c["x"], *L[0])))
    c["e0"] = r(act(conv3(c["e0a"], *L[1])))
    c["p1"] = r(pool(c["e0"]))
    c["e1a"] = r(act(conv3(c["p1"], *L[2])))
    c["e1"] = r(act(conv3(c["e1a"], *L[3])))
    c["p2"] = r(pool(c["e1"]))
    c["b1"] = r(act(conv3(c["p2"], *L[4])))
    c["b2"] = r(act(conv3(c["b1"], *L[5])))
    c["b3"] = r(act(conv3(c["b2"], *L[6])))
    c["t8"] = r(act(conv3(up(c["b3"]), *L[7])))
    c["u1"] = r(c["t8"] + c["e1"])
    c["u1b"] = r(act(conv3(c["u1"], *L[8])))
    c["t10"] = r(act(conv3(up(c["u1b"]), *L[9])))
    c["u0"] = r(c["t10"] + c["e0"])
    c["u0b"] = r(act(conv3(c["u0"], *L[10])))
    P = m * conv3(c["u0b"], *L[11])
    return P, c


def loss_and_grad(theta, width, T, thickness, noise, target, shape, bf16=False):
    """Loss and its gradient in the flat parameter vector."""
    r = round_bf16 if bf16 else _ident
    P, c = forward(theta, width, T, thickness, noise, shape, bf16)
    m, L = c["m"], c["L"]
    count = 3.0 * m.sum()
    diff = P - np.asarray(target, dtype=np.float64)
    loss = float((m * diff * diff).sum() / count)
    grads = [None] * 12
    gy = r(m * 2.0 * diff / count)                       # dL/d(conv12 output)
    grads[11] = conv3_weight_grad(gy, c["u0b"])
    g = r(conv3_input_grad(gy, L[11][0]) * act_slope(c["u0b"]))      # pre-act of L11
    grads[10] = conv3_weight_grad(g, c["u0"])
    acc = conv3_input_grad(g, L[10][0])                 # d/d u0
    g_u0 = r(acc)                                       # to e0 through the skip
    g = r(acc * act_slope(c["t10"]))                    # pre-act of L10
    grads[9] = conv3_weight_grad(g, up(c["u1b"]))
    g_q0 = r(conv3_input_grad(g, L[9][0]))
    g = r(up_adjoint(g_q0) * act_slope(c["u1b"]))       # pre-act of L9
    grads[8] = conv3_weight_grad(g, c["u1"])
    acc = conv3_input_grad(g, L[8][0])                  # d/d u1
    g_u1 = r(acc)
    g = r(acc * act_slope(c["t8"]))                     # pre-act of L8
    grads[7] = conv3_weight_grad(g, up(c["b3"]))
    g_q1 = r(conv3_input_grad(g, L[7][0]))
    g = r(up_adjoint(g_q1) * act_slope(c["b3"]))        # pre-act of L7
    grads[6] = conv3_weight_grad(g, c["b2"])
    g = r(conv3_input_grad(g, L[6][0]) * act_slope(c["b2"]))
    grads[5] = conv3_weight_grad(g, c["b1"])
    g = r(conv3_input_grad(g, L[5][0]) * act_slope(c["b1"]))
    grads[4] = conv3_weight_grad(g, c["p2"])
    g_p2 = r(conv3_input_grad(g, L[4][0]))
    g = r((pool_adjoint(g_p2) + g_u1) * act_slope(c["e1"]))     # pre-act of L4
    grads[3] = conv3_weight_grad(g, c["e1a"])
    g = r(conv3_input_grad(g, L[3][0]) * act_slope(c["e1a"]))
    grads[2] = conv3_weight_grad(g, c["p1"])
    g_p1 = r(conv3_input_grad(g, L[2][0]))
    g = r((pool_adjoint(g_p1) + g_u0) * act_slope(c["e0"]))     # pre-act of L2
    grads[1] = conv3_weight_grad(g, c["e0a"])
    g = r(conv3_input_grad(g, L[1][0]) * act_slope(c["e0a"]))
    grads[0] = conv3_weight_grad(g, c["x"])
    return loss, P, pack(grads)


def apply_op(F, op):
    """Image of vector fields F [..][3][Z][Y][X] under an in-plane symmetry
    op (bits: 1 mirror x, 2 mirror y, 4 swap x and y): the swap first, then
    the x mirror, then the y mirror, each moving positions and components
    (a mirror negates the normal component)."""
    G = np.array(F, dtype=np.float64, copy=True)
    if op & 4:
        G = np.swapaxes(G, -1, -2)[..., [1, 0, 2], :, :, :].copy()
    if op & 1:
        G = G[..., ::-1].copy()
        G[..., 0, :, :, :] *= -1
    if op & 2:
        G = G[..., ::-1, :].copy()
        G[..., 1, :, :, :] *= -1
    return G


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new theta, m, v."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
