"""The surrogate's FP64 oracle operations against independent definitions
(CPU only): FFT circular convolution, shifted identities, adjoint
(inner-product) identities, finite differences and Adam's closed form."""
import numpy as np
import pytest

from oracle import surrogate as S

RNG = np.random.default_rng(7)


def _inner(a, b):
    return float(np.sum(np.asarray(a) * np.asarray(b)))


def test_conv_matches_fft_circular_correlation():
    """Each (out, in) channel pair is a circular cross-correlation with the
    3x3 kernel embedded in an H x W image: IFFT(conj(FFT(k)) FFT(x))."""
    n, h, w, ci, co = 2, 9, 12, 3, 4
    x = RNG.normal(size=(n, h, w, ci))
    wt = RNG.normal(size=(co, 9, ci))
    b = RNG.normal(size=co)
    got = S.conv3x3(x, wt, b)
    for o in range(co):
        want = np.full((n, h, w), b[o])
        for i in range(ci):
            k = np.zeros((h, w))
            for t, (dy, dx) in enumerate(S.TAPS):
                k[dy % h, dx % w] = wt[o, t, i]
            kf = np.conj(np.fft.fft2(k))
            for m in range(n):
                want[m] += np.real(np.fft.ifft2(kf * np.fft.fft2(x[m, :, :, i])))
        assert np.max(np.abs(got[..., o] - want)) < 1e-12


def test_conv_centre_and_shift_taps():
    x = RNG.normal(size=(1, 5, 7, 3))
    w = np.zeros((3, 9, 3))
    w[:, 4, :] = np.eye(3)  # centre tap, identity
    assert np.array_equal(S.conv3x3(x, w), x)
    w = np.zeros((3, 9, 3))
    w[:, 5, :] = np.eye(3)  # tap (dy, dx) = (0, +1): reads the east neighbour
    assert np.array_equal(S.conv3x3(x, w)[0, 2, 3], x[0, 2, 4])
    assert np.array_equal(S.conv3x3(x, w)[0, 2, 6], x[0, 2, 0])  # periodic wrap
    w = np.zeros((3, 9, 3))
    w[:, 1, :] = np.eye(3)  # tap (-1, 0): reads the row above
    assert np.array_equal(S.conv3x3(x, w)[0, 0, 3], x[0, 4, 3])


def test_conv_adjoint_identities():
    """<dZ, conv(X, W)> = <bwd_data(dZ, W), X> = <bwd_weight(X, dZ), W>,
    and <dZ, b> summed = <db, b>."""
    n, h, w, ci, co = 2, 6, 8, 5, 3
    x = RNG.normal(size=(n, h, w, ci))
    wt = RNG.normal(size=(co, 9, ci))
    dz = RNG.normal(size=(n, h, w, co))
    b = RNG.normal(size=co)
    lhs = _inner(dz, S.conv3x3(x, wt))
    assert abs(lhs - _inner(S.conv3x3_bwd_data(dz, wt), x)) < 1e-10 * abs(lhs) + 1e-10
    dw, db = S.conv3x3_bwd_weight(x, dz)
    assert abs(lhs - _inner(dw, wt)) < 1e-10 * abs(lhs) + 1e-10
    bias_part = _inner(dz, S.conv3x3(x, wt, b)) - lhs
    assert abs(bias_part - _inner(db, b)) < 1e-10 * (abs(bias_part) + 1)


def test_pool_and_upsample_adjoints():
    a = RNG.normal(size=(2, 4, 6, 3))
    big = RNG.normal(size=(2, 8, 12, 3))
    assert abs(_inner(S.up2(a), big) - _inner(a, S.up2_bwd(big))) < 1e-12
    assert abs(_inner(S.pool2(big), a) - _inner(big, S.pool2_bwd(a))) < 1e-12
    assert np.allclose(S.pool2(S.up2(a)), a, rtol=0, atol=1e-15)
    assert S.pool2(np.arange(16.0).reshape(1, 4, 4, 1))[0, 0, 0, 0] == (0 + 1 + 4 + 5) / 4


def test_leaky_derivative_fd():
    z = RNG.normal(size=200)
    z = z[np.abs(z) > 1e-3]
    c = RNG.normal(size=z.size)
    h = 1e-7
    fd = (S.leaky(z + h, 0.1) - S.leaky(z - h, 0.1)) / (2 * h) * c
    assert np.allclose(S.leaky_bwd(c, S.leaky(z, 0.1), 0.1), fd, rtol=1e-7, atol=1e-9)


def test_adam_constant_gradient_closed_form():
    """For a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves theta by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    theta, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 26):
        theta, m, v = S.adam(theta, g, m, v, t, lr=0.01)
    assert np.allclose(theta, -25 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_unet_shapes_and_parameter_count():
    spec = S.unet_spec(levels=4, base=32, cin=16, cout=16)
    convs = [op for op in spec if op[0] == "conv"]
    assert len(convs) == 15
    params = sum(9 * ci * co + co for _, ci, co, _ in convs)
    assert 1.9e6 < params < 2.0e6
    assert convs[8][1:3] == (256 + 128, 128)  # first decoder conv: upsampled + skip


@pytest.mark.parametrize("slope", [0.1])
def test_unet_gradient_fd(slope):
    """Whole-network gradients (a small U-Net) against central differences
    of the forward pass, for the input and for weights of every layer."""
    spec = S.unet_spec(levels=3, base=4, cin=3, cout=2)
    rng = np.random.default_rng(11)
    weights = []
    for op in spec:
        if op[0] == "conv":
            _, ci, co, _ = op
            weights.append((rng.normal(size=(co, 9, ci)) / np.sqrt(9 * ci), rng.normal(size=co) * 0.1))
    x = rng.normal(size=(2, 8, 8, 3))
    target = rng.normal(size=(2, 8, 8, 2))

    def loss(ws, xx):
        out, _ = S.unet_forward(xx, ws, spec, slope)
        return 0.5 * np.sum((out - target) ** 2)

    out, tape = S.unet_forward(x, weights, spec, slope)
    grads, dx = S.unet_backward(out - target, weights, tape, slope)
    h = 1e-6
    for k in range(len(weights)):
        w, b = weights[k]
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            up = [(wp, b) if j == k else weights[j] for j in range(len(weights))]
            dn = [(wm, b) if j == k else weights[j] for j in range(len(weights))]
            fd = (loss(up, x) - loss(dn, x)) / (2 * h)
            assert abs(grads[k][0][idx] - fd) <= 1e-5 * max(1.0, abs(fd)), (k, idx)
        o = rng.integers(0, b.size)
        bp, bm = b.copy(), b.copy()
        bp[o] += h
        bm[o] -= h
        fd = (loss([(w, bp) if j == k else weights[j] for j in range(len(weights))], x)
              - loss([(w, bm) if j == k else weights[j] for j in range(len(weights))], x)) / (2 * h)
        assert abs(grads[k][1][o] - fd) <= 1e-5 * max(1.0, abs(fd)), (k, "bias")
    for _ in range(4):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (loss(weights, xp) - loss(weights, xm)) / (2 * h)
        assert abs(dx[idx] - fd) <= 1e-5 * max(1.0, abs(fd)), idx


def test_loss_gradient_fd_and_io_roundtrip():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0, 1, size=(2, 5, 4, 6))
    target = rho + rng.normal(scale=0.01, size=rho.shape)
    scale = [0.5, 0.01, 0.02, 0.03, 0.001]
    out = rng.normal(size=(2, 4, 6, 16))
    loss, grad = S.mse_loss(out, rho, target, scale)
    assert np.all(grad[..., 5:] == 0)
    for _ in range(5):
        idx = (int(rng.integers(2)), int(rng.integers(4)), int(rng.integers(6)), int(rng.integers(5)))
        h = 1e-6
        op, om = out.copy(), out.copy()
        op[idx] += h
        om[idx] -= h
        fd = (S.mse_loss(op, rho, target, scale)[0] - S.mse_loss(om, rho, target, scale)[0]) / (2 * h)
        assert abs(grad[idx] - fd) < 1e-7
    # the output that makes the loss zero reproduces the target exactly
    exact = np.zeros_like(out)
    for c in range(5):
        exact[..., c] = (target[:, c] - rho[:, c]) / scale[c]
    assert S.mse_loss(exact, rho, target, scale)[0] < 1e-28
    assert np.allclose(S.apply_output(rho, exact, scale), target, rtol=0, atol=1e-15)
    x = S.pack_input(rho, rng.normal(size=(2, 9)), [1, 2, 3, 4, 5])
    assert np.allclose(x[1, 2, 3, 4], rho[1, 4, 2, 3] / 5) and np.all(x[..., 14:] == 0)


def test_bf16_round_definition():
    """Ties go to the even neighbour, 8 significant bits, and the result is
    the nearest BF16 value (checked by brute force against the two BF16
    neighbours built from the bit pattern)."""
    assert S.bf16_round(1.0) == 1.0
    assert S.bf16_round(1.0 + 2.0 ** -8) == 1.0            # tie -> even (1.0)
    assert S.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even
    assert S.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert S.bf16_round(-3.0) == -3.0
    vals = np.random.default_rng(1).normal(size=2000) * 10.0 ** np.random.default_rng(2).integers(-5, 5, 2000)
    got = S.bf16_round(vals)
    f32 = vals.astype(np.float32)
    lo = (f32.view(np.uint32) & 0xFFFF0000).view(np.float32).astype(np.float64)
    hi = ((f32.view(np.uint32) & 0xFFFF0000) + 0x10000).view(np.float32).astype(np.float64)
    best = np.where(np.abs(f32 - lo) <= np.abs(hi - f32), lo, hi)
    tie = np.abs(f32 - lo) == np.abs(hi - f32)
    assert np.array_equal(got[~tie], best[~tie])


def test_unet_storage_hook_changes_only_rounding():
    spec = S.unet_spec(levels=2, base=8, cin=8, cout=8)
    rng = np.random.default_rng(4)
    weights = [(rng.normal(size=(op[2], 9, op[1])) * 0.2, rng.normal(size=op[2]) * 0.1)
               for op in spec if op[0] == "conv"]
    x = rng.normal(size=(1, 8, 8, 8))
    exact, tape = S.unet_forward(x, weights, spec, 0.1)
    rounded, tape16 = S.unet_forward(x, weights, spec, 0.1, store=S.bf16_round)
    assert np.linalg.norm(rounded - exact) / np.linalg.norm(exact) < 2e-2
    g, _ = S.unet_backward(exact, weights, tape, 0.1)
    g16, _ = S.unet_backward(exact, weights, tape16, 0.1, store=S.bf16_round)
    for (a, _), (b, _) in zip(g, g16):
        assert np.linalg.norm(a - b) / np.linalg.norm(a) < 0.2


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_receptive_radius_brute_force(levels):
    """The rollout's prefilter pads its tiles by the network's receptive
    radius: perturbing one input pixel of the oracle U-Net (every alignment
    to the pooling grid) changes outputs exactly that far away."""
    from paper_2603_19789_amd.surrogate import receptive_radius
    spec = S.unet_spec(levels=levels, base=4, cin=2, cout=2)
    rng = np.random.default_rng(7)
    weights = [(rng.normal(size=(op[2], 9, op[1])) * 0.5, rng.normal(size=op[2]) * 0.1)
               for op in spec if op[0] == "conv"]
    n = 128
    x = rng.normal(size=(1, n, n, 2))
    base, _ = S.unet_forward(x, weights, spec, 0.1)
    reach = 0
    for off in range(2 ** (levels - 1)):
        c = n // 2 + off
        x2 = x.copy()
        x2[0, c, c, :] += 1.0
        out, _ = S.unet_forward(x2, weights, spec, 0.1)
        ys, xs = np.nonzero(np.abs(out - base).max(axis=(0, 3)) > 0)
        reach = max(reach, int(max(np.abs(ys - c).max(), np.abs(xs - c).max())))
    assert reach == receptive_radius(levels)


def test_training_initial_states_from_separable_factors():
    """The surrogate's training data starts from Gaussian-foci states built
    on the device from their separable factors: the factors' outer-product
    sum, clipped, is the generator's infected field (periodic wrap included:
    foci at the grid's edges, a non-square grid)."""
    from paper_2603_19789_amd.inputs import gaussian_foci_factors, gaussian_foci_state
    centres = [(3, 199), (100, 7), (255, 128), (0, 0)]
    gy, gx = gaussian_foci_factors(256, 200, centres, 0.03, 4.5)
    assert gy.shape == (4, 200) and gx.shape == (4, 256)
    field = np.minimum(gy.T @ gx, 1.0)
    want = gaussian_foci_state(256, 200, centres, 0.03, 4.5)
    assert np.max(np.abs(field - want[2])) < 1e-15
    assert np.max(np.abs(1.0 - field - want[0])) < 1e-15
