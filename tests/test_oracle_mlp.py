"""Pins of the cost-model oracle (oracle/mlp.py) -- CPU only.

Each pin fixes the oracle by something other than itself: finite differences
of the forward pass, the closed form of an all-active (affine) network, a dead
layer's constant output, the BF16 format's definition and Adam's closed forms
(first step, constant gradient, a hand-worked two-step sequence).
Planted mistakes in the backward pass must fail at least one of them.
"""
import numpy as np
import pytest

from oracle import mlp


def _rand_params(seed, bias=0.0):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-0.5, 0.5, mlp.PARAMS)
    p[mlp.B1:mlp.W2] += bias
    p[mlp.B2:mlp.W3] += bias
    return p


def _rand_data(seed, rows=13):
    rng = np.random.default_rng(seed + 100)
    X = rng.normal(2.0, 3.0, (rows, mlp.IN))
    Y = rng.normal(0.0, 2.0, rows)
    norm = np.concatenate([rng.normal(1.0, 0.5, mlp.IN), rng.uniform(0.2, 1.5, mlp.IN)])
    return X, Y, norm


def _fd_grad(p, norm, X, Y, scale, idx, h=1e-6):
    g = np.zeros(len(idx))
    for k, i in enumerate(idx):
        a = p.copy()
        b = p.copy()
        a[i] += h
        b[i] -= h
        g[k] = (mlp.loss(a, norm, X, Y, scale) - mlp.loss(b, norm, X, Y, scale)) / (2 * h)
    return g


def _sample_idx(seed):
    rng = np.random.default_rng(seed)
    blocks = [(mlp.W1, mlp.B1), (mlp.B1, mlp.W2), (mlp.W2, mlp.B2), (mlp.B2, mlp.W3),
              (mlp.W3, mlp.B3), (mlp.B3, mlp.PARAMS)]
    idx = []
    for a, b in blocks:
        idx.extend(rng.choice(np.arange(a, b), size=min(12, b - a), replace=False).tolist())
    return np.array(idx)


@pytest.mark.parametrize("seed", range(4))
def test_grad_matches_finite_differences(seed):
    p = _rand_params(seed, bias=0.2)
    X, Y, norm = _rand_data(seed)
    scale = 1.0 / len(Y)
    idx = _sample_idx(seed)
    g = mlp.grad(p, norm, X, Y, scale)
    fd = _fd_grad(p, norm, X, Y, scale, idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-7)


def test_all_active_network_is_affine():
    # large positive biases keep every unit active: f = ((x_n W1 + b1) W2 + b2) W3 + b3
    p = _rand_params(7, bias=40.0)
    p[mlp.W2:mlp.B2] = np.abs(p[mlp.W2:mlp.B2])  # positive h1 then keeps z2 positive
    X, Y, norm = _rand_data(7)
    w1, b1, w2, b2, w3, b3 = mlp.unpack(p)
    _, (_, z1, _, z2, _) = mlp.forward(p, norm, X)
    assert (z1 > 0).all() and (z2 > 0).all()
    xn = (X - norm[:8]) * norm[8:]
    M = w1 @ w2 @ w3
    c = b1 @ w2 @ w3 + b2 @ w3 + b3
    f, _ = mlp.forward(p, norm, X)
    assert np.allclose(f, xn @ M + c, rtol=1e-12, atol=1e-9)
    # and the loss gradient with respect to b3 and W1 has the affine closed form
    g = mlp.grad(p, norm, X, Y, 0.5)
    r = 2 * 0.5 * (f - Y)
    assert np.isclose(g[mlp.B3], r.sum())
    gw1 = np.einsum("r,ri,j->ij", r, xn, w2 @ w3)
    assert np.allclose(g[mlp.W1:mlp.B1].reshape(8, 64), gw1, rtol=1e-10, atol=1e-10)


def test_dead_first_layer_is_constant():
    p = _rand_params(3)
    p[mlp.B1:mlp.W2] = -1e6
    X, Y, norm = _rand_data(3)
    f, _ = mlp.forward(p, norm, X)
    w1, b1, w2, b2, w3, b3 = mlp.unpack(p)
    assert np.allclose(f, np.maximum(b2, 0) @ w3 + b3)
    g = mlp.grad(p, norm, X, Y, 1.0)
    assert not np.any(g[mlp.W1:mlp.W2])


def test_bf16_rounding_definition():
    one = np.float32(1.0)
    ulp = 2.0 ** -7  # BF16 keeps 7 explicit mantissa bits
    cases = [
        (1.0, 1.0),
        (1.0 + 2.0 ** -8, 1.0),                # half an ulp, tie -> even (1.0)
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2 * ulp),  # 1.5 ulp, tie -> even mantissa 2
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + ulp),  # just above half -> up
        (-3.0, -3.0),
        (0.0, 0.0),
        (65504.0, 65536.0),
    ]
    for x, want in cases:
        assert mlp.bf16_round(np.float32(x)) == np.float32(want), x
    assert mlp.bf16_round(one).dtype == np.float32


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    g = rng.normal(size=50)
    w0 = rng.normal(size=50)
    w1, m, v = mlp.adam(w0, np.zeros(50), np.zeros(50), g, 0.01, 1, eps=0.0)
    # with bias correction the first step is exactly -lr * sign(g)
    assert np.allclose(w1, w0 - 0.01 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


_MUTATIONS = [
    ("relu mask of layer 2 from layer 1", "* (z2 > 0)", "* (z1[:, :64] > 0)"),
    ("W2 not transposed", "d_z2 @ w2.T", "d_z2 @ w2"),
    ("missing factor 2", "2.0 * scale", "1.0 * scale"),
    ("bias grad as mean", "g_b2 = d_z2.sum(axis=0)", "g_b2 = d_z2.mean(axis=0)"),
    ("raw inputs for W1", "g_w1 = xn.T @ d_z1", "g_w1 = (xn + 1).T @ d_z1"),
]


@pytest.mark.parametrize("name,old,new", _MUTATIONS, ids=[m[0] for m in _MUTATIONS])
def test_pins_catch_planted_backward_mistakes(name, old, new):
    src = open(mlp.__file__).read()
    assert old in src, name
    ns = {"__name__": "mutant"}
    exec(compile(src.replace(old, new), "mutant_mlp.py", "exec"), ns)
    caught = False
    for seed in range(3):
        p = _rand_params(seed, bias=0.2)
        X, Y, norm = _rand_data(seed)
        idx = _sample_idx(seed)
        g = ns["grad"](p, norm, X, Y, 0.25)
        fd = _fd_grad(p, norm, X, Y, 0.25, idx)
        if not np.allclose(g[idx], fd, rtol=1e-5, atol=1e-7):
            caught = True
            break
    assert caught, f"mutation '{name}' escaped the pins"


def test_adam_constant_gradient_moves_by_signed_lr_every_step():
    # with g_t = g for all t the moments are m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2, so the bias-corrected ratio is g / |g| at every
    # step t and each update is exactly -lr * sign(g)
    rng = np.random.default_rng(1)
    g = rng.normal(size=40)
    w0 = rng.normal(size=40)
    w, m, v = w0.copy(), np.zeros(40), np.zeros(40)
    for t in range(1, 6):
        w, m, v = mlp.adam(w, m, v, g, 0.01, t, eps=0.0)
        assert np.allclose(w, w0 - 0.01 * t * np.sign(g), rtol=0, atol=1e-12), t
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)


def test_adam_two_steps_with_sign_change_by_hand():
    # g_1 = +1, g_2 = -1 (eps = 0), worked by hand:
    #   step 1: m = 0.1, v = 0.001, m/(1-0.9) = 1, v/(1-0.999) = 1 -> w -= lr
    #   step 2: m = 0.09 - 0.1 = -0.01, v = 0.000999 + 0.001 = 0.001999,
    #           m/(1-0.81) = -1/19, v/(1-0.998001) = 1              -> w += lr/19
    lr = 0.5
    w, m, v = mlp.adam(np.array([2.0]), np.zeros(1), np.zeros(1), np.array([1.0]), lr, 1, eps=0.0)
    assert np.allclose(w, [2.0 - lr], rtol=0, atol=1e-15)
    w, m, v = mlp.adam(w, m, v, np.array([-1.0]), lr, 2, eps=0.0)
    assert np.allclose(m, [-0.01], rtol=0, atol=1e-15)
    assert np.allclose(v, [0.001999], rtol=0, atol=1e-15)
    assert np.allclose(w, [2.0 - lr + lr / 19.0], rtol=0, atol=1e-12)


_ADAM_MUTATIONS = [
    ("first moment not bias-corrected by step", "mh = m / (1 - b1 ** step)", "mh = m / (1 - b1)"),
    ("second moment exponent off by one", "vh = v / (1 - b2 ** step)",
     "vh = v / (1 - b2 ** (step + 1))"),
    ("second moment from the raw gradient", "v = b2 * v + (1 - b2) * g * g",
     "v = b2 * v + (1 - b2) * np.abs(g)"),
    ("moment decay swapped", "m = b1 * m + (1 - b1) * g", "m = (1 - b1) * m + b1 * g"),
]


@pytest.mark.parametrize("name,old,new", _ADAM_MUTATIONS, ids=[m[0] for m in _ADAM_MUTATIONS])
def test_adam_pins_catch_planted_mistakes(name, old, new):
    src = open(mlp.__file__).read()
    assert old in src, name
    ns = {"__name__": "mutant"}
    exec(compile(src.replace(old, new), "mutant_mlp.py", "exec"), ns)
    caught = False
    for pin in (test_adam_first_step_is_signed_lr,
                test_adam_constant_gradient_moves_by_signed_lr_every_step,
                test_adam_two_steps_with_sign_change_by_hand):
        saved = mlp.adam
        mlp.adam = ns["adam"]
        try:
            pin()
        except AssertionError:
            caught = True
        finally:
            mlp.adam = saved
        if caught:
            break
    assert caught, f"mutation '{name}' escaped the Adam pins"
