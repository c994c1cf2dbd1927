"""Plain FP64 CPU oracle for the operations of the learned surrogate.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU baseline may import this module. The product path never calls it, and it
shares no code with the HIP kernels.

The surrogate is a convolutional U-Net that maps the five SEIRD densities
(plus constant planes holding the rates and diffusivities) to the state a
fixed number of SSLBM steps later. Its operations are standard; each function
here is the textbook definition written out in FP64, one tap or one window at
a time, with NumPy's tensordot (a matrix product) as the only library step:

  conv3x3      out[n,y,x,o] = b[o] + sum_{dy,dx in -1..1} sum_i
                              W[o, 3(dy+1)+(dx+1), i] X[n, (y+dy) mod H, (x+dx) mod W, i]
               (cross-correlation with periodic padding, as the lattice is periodic)
  conv3x3_bwd_data    dX = d(sum dZ * conv(X)) / dX
  conv3x3_bwd_weight  dW, db = d(sum dZ * conv(X)) / dW, db
  leaky / leaky_bwd   y = z for z > 0, slope z otherwise
  pool2 / pool2_bwd   2x2 average pooling and its adjoint
  up2 / up2_bwd       2x nearest-neighbour upsampling and its adjoint
  adam                one step of Adam (Kingma and Ba, 2015, Algorithm 1)

Arrays are NHWC (image, row, column, channel); weights are [out][tap][in]
with tap = 3 (dy + 1) + (dx + 1). The pins in tests/test_oracle_surrogate.py
tie each function to something it does not compute itself: FFT circular
convolution, shifted identities, inner-product (adjoint) identities, finite
differences and Adam's closed form for a constant gradient.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[n, y, x, :] = x[n, (y + dy) mod H, (x + dx) mod W, :]."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv3x3(x, w, b=None):
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        out += np.tensordot(_shift(x, dy, dx), w[:, t, :], axes=([3], [1]))
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3x3_bwd_data(dz, w):
    """dX[n, y', x', i] = sum_t sum_o dZ[n, y' - dy, x' - dx, o] W[o, t, i]."""
    dz = np.asarray(dz, np.float64)
    w = np.asarray(w, np.float64)
    dx_ = np.zeros(dz.shape[:3] + (w.shape[2],))
    for t, (dy, dx) in enumerate(TAPS):
        dx_ += _shift(np.tensordot(dz, w[:, t, :], axes=([3], [0])), -dy, -dx)
    return dx_


def conv3x3_bwd_weight(x, dz):
    """dW[o, t, i] = sum_{n,y,x} dZ[n,y,x,o] X[n, y+dy, x+dx, i]; db[o] = sum dZ[..., o]."""
    x = np.asarray(x, np.float64)
    dz = np.asarray(dz, np.float64)
    dw = np.zeros((dz.shape[3], 9, x.shape[3]))
    for t, (dy, dx) in enumerate(TAPS):
        dw[:, t, :] = np.tensordot(dz, _shift(x, dy, dx), axes=([0, 1, 2], [0, 1, 2]))
    return dw, dz.sum(axis=(0, 1, 2))


def leaky(z, slope):
    z = np.asarray(z, np.float64)
    return np.where(z > 0, z, slope * z)


def leaky_bwd(dy, y, slope):
    """dZ from dY and the activation's output y (y > 0 exactly where z > 0)."""
    return np.where(np.asarray(y) > 0, np.asarray(dy, np.float64), slope * np.asarray(dy, np.float64))


def pool2(x):
    x = np.asarray(x, np.float64)
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool2_bwd(dy):
    """Adjoint of pool2: every input of a window receives a quarter."""
    return 0.25 * up2(dy)


def up2(x):
    x = np.asarray(x, np.float64)
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_bwd(dy):
    """Adjoint of up2: the sum over each 2x2 window."""
    dy = np.asarray(dy, np.float64)
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


# ------------------------------------------------------ input and output --

def pack_input(rho, planes, scale_in):
    """Network input [b, h, w, 16] from densities rho [b, 5, h, w]: rho_c /
    scale_in[c], then the 9 parameter values of each instance, then zeros."""
    rho = np.asarray(rho, np.float64)
    b, _, h, w = rho.shape
    x = np.zeros((b, h, w, 16))
    for c in range(5):
        x[..., c] = rho[:, c] / scale_in[c]
    for k in range(9):
        x[..., 5 + k] = np.asarray(planes, np.float64)[:, k][:, None, None]
    return x


def apply_output(rho, out, scale_out):
    """rho + scale_out[c] out[..., c] for the five compartments."""
    rho = np.asarray(rho, np.float64)
    nxt = rho.copy()
    for c in range(5):
        nxt[:, c] += scale_out[c] * np.asarray(out, np.float64)[..., c]
    return nxt


def mse_loss(out, rho, target, scale_out):
    """Mean over (b, y, x, c < 5) of (out_c - (target - rho)_c / scale_out[c])^2
    and its gradient with respect to out (zero for channels >= 5)."""
    out = np.asarray(out, np.float64)
    d = np.zeros_like(out)
    for c in range(5):
        d[..., c] = out[..., c] - (np.asarray(target, np.float64)[:, c]
                                   - np.asarray(rho, np.float64)[:, c]) / scale_out[c]
    count = out.shape[0] * out.shape[1] * out.shape[2] * 5
    return float(np.sum(d * d) / count), 2.0 * d / count


# ------------------------------------------------------ storage precision --

def bf16_round(a):
    """Round to the nearest BF16 value, ties to even: BF16 keeps the upper 16
    bits of the IEEE binary32 encoding (sign, 8 exponent bits, 7 fraction
    bits). Input is first rounded to binary32. Finite values only."""
    a32 = np.asarray(a, np.float64).astype(np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- network --

def unet_spec(levels: int = 4, base: int = 32, cin: int = 16, cout: int = 16):
    """Layer list of the U-Net in forward order: ('conv', in, out, act),
    ('pool',), ('up',), ('save', level), ('cat', level). Encoder level l has
    base * 2^l channels (two 3x3 convolutions each, pooled between levels);
    each decoder level upsamples, appends the saved encoder output of the
    same level after the upsampled channels, and applies two convolutions;
    a final 3x3 convolution without activation maps to cout channels."""
    ch = [base * 2 ** l for l in range(levels)]
    spec = []
    c = cin
    for l in range(levels):
        if l:
            spec.append(("pool",))
        spec.append(("conv", c, ch[l], True))
        spec.append(("conv", ch[l], ch[l], True))
        spec.append(("save", l))
        c = ch[l]
    for l in range(levels - 2, -1, -1):
        spec.append(("up",))
        spec.append(("cat", l))
        spec.append(("conv", c + ch[l], ch[l], True))
        spec.append(("conv", ch[l], ch[l], True))
        c = ch[l]
    spec.append(("conv", c, cout, False))
    return spec


def _exact(a):
    return np.asarray(a, np.float64)


def unet_forward(x, weights, spec, slope, store=_exact):
    """Forward pass; weights is a list of (W, b) per conv in spec order.
    Returns the output and the tape of activations for unet_backward.
    `store` is applied to every tensor a layer hands on (each activated
    convolution output and each pooled tensor; the last convolution's
    output is kept exact): identity by default, bf16_round to model a
    network whose activations are stored in BF16."""
    tape = []
    saved = {}
    k = 0
    h = np.asarray(x, np.float64)
    n_conv = sum(1 for op in spec if op[0] == "conv")
    for op in spec:
        if op[0] == "conv":
            w, b = weights[k]
            k += 1
            z = conv3x3(h, w, b)
            y = leaky(z, slope) if op[3] else z
            if k < n_conv:
                y = store(y)
            tape.append(("conv", h, y, op[3]))
            h = y
        elif op[0] == "pool":
            tape.append(("pool", h.shape))
            h = store(pool2(h))
        elif op[0] == "up":
            tape.append(("up",))
            h = up2(h)
        elif op[0] == "save":
            saved[op[1]] = h
            tape.append(("save", op[1]))
        elif op[0] == "cat":
            skip = saved[op[1]]
            tape.append(("cat", op[1], h.shape[3]))
            h = np.concatenate([h, skip], axis=3)
    return h, tape


def unet_backward(dout, weights, tape, slope, store=_exact):
    """Gradients (dW, db) per conv, in spec order, and dX of the input.
    `store` is applied where a gradient tensor is handed on: dZ after the
    activation, dX of each convolution, the upsampling adjoint, and an
    encoder output's gradient after the skip and pooled parts are added."""
    grads = [None] * len(weights)
    k = len(weights)
    skip_grad = {}
    g = store(dout)
    for entry in reversed(tape):
        if entry[0] == "conv":
            k -= 1
            _, x_in, y, act = entry
            dz = store(leaky_bwd(g, y, slope)) if act else g
            grads[k] = conv3x3_bwd_weight(x_in, dz)
            g = store(conv3x3_bwd_data(dz, weights[k][0]))
        elif entry[0] == "pool":
            g = pool2_bwd(g)
        elif entry[0] == "up":
            g = store(up2_bwd(g))
        elif entry[0] == "cat":
            _, level, c_up = entry
            skip_grad[level] = g[..., c_up:]
            g = g[..., :c_up]
        elif entry[0] == "save":
            if entry[1] in skip_grad:
                g = store(g + skip_grad.pop(entry[1]))
    return grads, g
