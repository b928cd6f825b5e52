"""Pins of the FP64 closure-network oracle (CPU only).

The learned closure is an extension, not in arXiv:2211.06142; what fixes its
oracle here is mathematics: the error function, finite differences, exact
reductions of the network (zero weights, the linear regime of GELU), the closed
form of the first Adam step, bfloat16 rounding by definition, and a two-sphere
scene whose features follow from its geometry (delta/R*) and from eq 11.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from synth import scenes


def test_gelu_values():
    # gelu(s) = s Phi(s); Phi(1) from the normal distribution table
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    s = np.linspace(-5, 5, 41)
    # Phi(-s) = 1 - Phi(s)  =>  gelu(-s) = gelu(s) - s
    np.testing.assert_allclose(mlp.gelu(-s), mlp.gelu(s) - s, rtol=0, atol=1e-14)
    # saturation: gelu(s) = s exactly for large s in FP64, 0 for very negative s
    assert mlp.gelu(np.array([60.0]))[0] == 60.0
    assert abs(mlp.gelu(np.array([-60.0]))[0]) < 1e-300


def test_gelu_grad_finite_difference():
    s = np.linspace(-4, 4, 33)
    h = 1e-6
    fd = (mlp.gelu(s + h) - mlp.gelu(s - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(s), fd, rtol=0, atol=1e-9)


def test_gradient_finite_difference():
    rng = np.random.default_rng(3)
    p = mlp.init_params(5)
    p[6 * 64:6 * 64 + 64] = rng.normal(0, 0.3, 64)          # nonzero b1
    x = rng.normal(size=(7, 6))
    t = rng.normal(size=(7, 2))
    L, g = mlp.grad(p, x, t)
    assert L == pytest.approx(mlp.loss(p, x, t), rel=1e-15)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False),
                          [0, 383, 384, 447, 448, mlp.N_PARAMS - 131, mlp.N_PARAMS - 1]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, x, t) - mlp.loss(p - e, x, t)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def _layers_zero_hidden(seed):
    rng = np.random.default_rng(seed)
    layers = [(np.zeros((6, 64)), rng.normal(size=64)), (np.zeros((64, 64)), rng.normal(size=64)),
              (np.zeros((64, 64)), rng.normal(size=64)), (np.zeros((64, 2)), rng.normal(size=2))]
    return mlp.pack(layers), layers


def test_zero_weights_give_output_bias():
    p, layers = _layers_zero_hidden(1)
    x = np.random.default_rng(2).normal(size=(4, 6))
    np.testing.assert_array_equal(mlp.forward(p, x), np.tile(layers[3][1], (4, 1)))
    np.testing.assert_array_equal(oracle.mlp_forward(p, x), np.tile(layers[3][1], (4, 1)))


def _affine_regime(seed):
    """hidden biases 100 and small weights: every hidden pre-activation stays
    far above 40, where gelu(s) = s in FP64, so the network is affine"""
    rng = np.random.default_rng(seed)
    W = [rng.normal(0, 0.05, (6, 64)), rng.normal(0, 0.01, (64, 64)), rng.normal(0, 0.01, (64, 64)),
         rng.normal(0, 0.1, (64, 2))]
    b = [np.full(64, 100.0), np.full(64, 100.0), np.full(64, 100.0), rng.normal(size=2)]
    p = mlp.pack(list(zip(W, b)))
    x = rng.normal(size=(5, 6))
    M = W[0] @ W[1] @ W[2] @ W[3]
    c = ((b[0] @ W[1] + b[1]) @ W[2] + b[2]) @ W[3] + b[3]
    return p, x, x @ M + c


def test_affine_regime_numpy_and_c():
    p, x, y = _affine_regime(4)
    np.testing.assert_allclose(mlp.forward(p, x), y, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.mlp_forward(p, x), y, rtol=1e-12, atol=1e-12)


def test_c_forward_matches_numpy_forward():
    p = mlp.init_params(9)
    x = np.random.default_rng(10).normal(size=(16, 6))
    np.testing.assert_allclose(oracle.mlp_forward(p, x), mlp.forward(p, x), rtol=0, atol=1e-13)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(6)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    p1, m1, v1 = mlp.adam_step(p, g, z, z, 1, 1e-3)
    # m_hat = g, v_hat = g^2: the step is lr g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(p1, p - 1e-3 * np.sign(g), rtol=0, atol=1e-9)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_factors_bounds():
    c = mlp.factors(np.array([[0.0, 0.0], [10.0, -10.0], [math.log(1.5), -math.log(1.5)]]))
    np.testing.assert_allclose(c, [[1, 1], [2, 0.5], [1.5, 1 / 1.5]], rtol=1e-15)


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e-3])
    r = mlp.bf16_round(v)
    # 8 significant bits: 1 + 2^-8 is a tie (to even: 1), 1 + 3 2^-8 a tie to 1 + 2^-6
    np.testing.assert_array_equal(r[:5], [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5])
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_closure_features_two_spheres():
    """Two overlapping spheres at rest in a uniform flow on a single fluid cell:
    the features follow from the geometry and eq 11."""
    r, delta = 1.0e-4, 1.0e-6
    x, rr, _ = scenes.two_spheres(r, r, -delta, 0.0, offset=(1e-3, 1e-3, 1e-3))
    mat = scenes.material(k_cg=1.0)
    fluid = dict(rho_f=1000.0, mu_f=1e-3, n_min=0.3, voidfrac=oracle.VOID_CIC, u_superficial=0, couple_every=1)
    grid = ((0.0, 0.0, 0.0), (2e-3, 2e-3, 2e-3), (1, 1, 1))
    op = oracle.make_params(mat, 1e-8, g=(0.0, 0.0, 0.0), grid=grid, fluid=fluid)
    o = oracle.OracleSim(op, x, rr, bond_at_init=True)
    u = np.array([[0.1, 0.0, 0.0]])
    o.set_fluid(u, np.zeros((1, 3)))
    f = o.closure_features()
    V = 2 * (4.0 / 3.0) * math.pi * r ** 3
    n_exp = 1.0 - V / (2e-3) ** 3
    Rs = r / 2
    Re = 1000.0 * (2 * r) * 0.1 / 1e-3
    for i in range(2):
        assert f[i, 0] == pytest.approx(n_exp, rel=1e-14)
        assert f[i, 1] == pytest.approx(0.1, rel=1e-14)
        assert f[i, 2] == pytest.approx(Re, rel=1e-14)
        assert f[i, 3] == 1.0
        assert f[i, 4] == pytest.approx(delta / Rs, rel=1e-9)
        assert f[i, 5] == 1.0
