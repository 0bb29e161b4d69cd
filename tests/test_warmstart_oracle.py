"""Pins of the learned warm-start oracle: each checks it against something other than itself
(finite differences, closed forms of special stencils, symmetry, the published Adam update
on a scalar, bit patterns of BF16)."""
import numpy as np
import pytest

from oracle import warmstart_oracle as WO


def _small(seed=1, B=3, n=12):
    rng = np.random.default_rng(seed)
    params = []
    for li in range(len(WO.WIDTHS) - 1):
        cin, cout = WO.WIDTHS[li], WO.WIDTHS[li + 1]
        params.append((rng.normal(size=(cout, cin, WO.KW)) * 0.3, rng.normal(size=cout) * 0.1))
    x = rng.normal(size=(B, 3, n))
    return params, x


def test_parameter_count():
    # 3*32*5+32 + 2*(32*32*5+32) + 32*5+1
    assert WO.n_params() == 10977


def test_delta_stencil_is_identity_and_shift():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 9))
    W = np.zeros((4, 4, 5))
    for c in range(4):
        W[c, c, 2] = 1.0
    assert np.array_equal(WO.conv1d_circ(x, W, np.zeros(4)), x)
    W[:] = 0.0
    for c in range(4):
        W[c, c, 3] = 1.0                      # tap t = 3 reads x[i + 1]
    z = WO.conv1d_circ(x, W, np.zeros(4))
    assert np.array_equal(z[..., :-1], x[..., 1:]) and np.array_equal(z[..., -1], x[..., 0])


def test_conv_matches_dense_circulant():
    rng = np.random.default_rng(2)
    n = 7
    x = rng.normal(size=(1, 2, n))
    W = rng.normal(size=(3, 2, 5))
    b = rng.normal(size=3)
    z = WO.conv1d_circ(x, W, b)
    for co in range(3):
        M = np.zeros((n, 2 * n))
        for i in range(n):
            for ci in range(2):
                for t in range(5):
                    M[i, ci * n + (i + t - 2) % n] += W[co, ci, t]
        ref = M @ x[0].reshape(-1) + b[co]
        assert np.allclose(z[0, co], ref, rtol=0, atol=1e-13)


def test_shift_equivariance():
    params, x = _small()
    y = WO.forward(params, x)[-1]
    y2 = WO.forward(params, np.roll(x, 3, axis=2))[-1]
    assert np.allclose(np.roll(y, 3, axis=2), y2, atol=1e-12)


@pytest.mark.parametrize("layer", [0, 1, 3])
def test_gradients_match_finite_differences(layer):
    params, x = _small()
    rng = np.random.default_rng(5)
    target = rng.normal(size=(x.shape[0], 1, x.shape[2]))

    def loss(ps):
        return WO.loss_and_grad_out(WO.forward(ps, x)[-1], target)[0]

    acts = WO.forward(params, x)
    _, gy = WO.loss_and_grad_out(acts[-1], target)
    grads = WO.backward(params, acts, gy)
    W, b = params[layer]
    h = 1e-6
    for idx in [(0, 0, 0), (W.shape[0] - 1, W.shape[1] - 1, 4), (0, W.shape[1] - 1, 2)]:
        Wp = W.copy(); Wp[idx] += h
        Wm = W.copy(); Wm[idx] -= h
        pp = list(params); pp[layer] = (Wp, b)
        pm = list(params); pm[layer] = (Wm, b)
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grads[layer][0][idx])
    bp = b.copy(); bp[0] += h
    bm = b.copy(); bm[0] -= h
    pp = list(params); pp[layer] = (W, bp)
    pm = list(params); pm[layer] = (W, bm)
    fd = (loss(pp) - loss(pm)) / (2 * h)
    assert abs(fd - grads[layer][1][0]) <= 1e-6 * max(1.0, abs(fd))


def test_zero_last_layer_predicts_linear_extrapolation():
    params = WO.init_params(seed=3)
    rng = np.random.default_rng(4)
    up, uc = rng.normal(size=(5, 16)), rng.normal(size=(5, 16))
    assert np.array_equal(WO.predict_columns(params, up, uc, np.ones(5)), 2.0 * uc - up)


def test_target_is_exact_for_quadratic_trajectories():
    # a column moving on a quadratic path u(t) = a + b t + c t^2 has the constant second
    # difference 2c: the target is 2c / (OUT s), and the perfect output recovers u(t+1)
    rng = np.random.default_rng(6)
    a, b, c = rng.normal(size=(3, 4, 24))
    u = [a + b * t + c * t * t for t in (0.0, 1.0, 2.0)]
    _, s = WO.make_inputs(u[0], u[1], np.zeros(4))
    tgt = WO.training_target(u[0], u[1], u[2])
    assert WO.OUT == 2.0 ** -12
    assert np.allclose(tgt * WO.OUT, 2.0 * c / s[:, None], rtol=1e-11, atol=1e-12)
    assert np.allclose(WO.predict_columns_from_output(u[0], u[1], tgt), u[2], rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    # first Adam step moves every parameter by -lr * sign(g) (bias-corrected moments)
    params = [(np.array([[[1.0, -2.0, 0.5, 0.0, 3.0]]]), np.array([0.25]))]
    grads = [(np.array([[[0.3, -0.7, 1e-3, 2.0, -5.0]]]), np.array([-0.1]))]
    new = WO.adam_step(params, grads, {}, lr=0.01)
    assert np.allclose(new[0][0], params[0][0] - 0.01 * np.sign(grads[0][0]), atol=1e-9)
    assert np.allclose(new[0][1], params[0][1] + 0.01, atol=1e-9)


def test_bf16_rounding_bit_patterns():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 and rounds to even (1); 1 + 3*2^-8 rounds up
    v = WO.bf16_round(np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 1e-40, 3.0e38]))
    assert v[0] == 1.0 and v[1] == 1.0 and v[2] == 1.0 + 2.0 ** -6 and v[3] == -2.5
    assert v[4] == np.float64(np.float32(1e-40)) or abs(v[4]) < 1e-38
    # the largest finite BF16 is 0x7F7F = (2 - 2^-7) * 2^127
    assert WO.bf16_round(np.array([3.3895313892515355e38]))[0] == (2 - 2.0 ** -7) * 2.0 ** 127
