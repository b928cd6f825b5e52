"""GPU parity of the learned closure (an extension; not in arXiv:2211.06142):
the BF16 matrix-core network against the FP64 oracle network, its gradient,
its Adam step, training, and the closure inside the DEM coupling.

Tolerances.  The GPU rounds the inputs, weights and every hidden activation
to bfloat16 (unit roundoff 2^-9) and accumulates in FP32; the oracle gets the
same bfloat16 weights and FP32 biases and computes in FP64.  Over 20 random
He-initialised networks and 4000 standard-normal inputs each, a model of those
rounding points gives |dy| <= 0.027 (1 + |y|); the tests allow that bound.
Gradients pass through four more roundings (the backward signals) and are
compared per layer in relative L2 norm (<= 0.02) and direction (cosine >= 0.9999).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import cg, mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2211_06142_amd import dem  # noqa: E402

LAYER_SLICES = []
_o = 0
for _i in range(4):
    _k, _m = mlp.SIZES[_i], mlp.SIZES[_i + 1]
    LAYER_SLICES.append(slice(_o, _o + _k * _m + _m))
    _o += _k * _m + _m


def fp32_params(seed, scale=1.0):
    return mlp.init_params(seed, scale).astype(np.float32).astype(np.float64)


def oracle_view(p):
    """the values the GPU network multiplies with: BF16 weights, FP32 biases"""
    return mlp.pack([(mlp.bf16_round(W), b) for W, b in mlp.unpack(p)])


@pytest.mark.parametrize("batch", [1, 16, 1000, 4099])
def test_forward_matches_oracle(batch):
    p = fp32_params(3)
    x = np.random.default_rng(batch).normal(size=(batch, 6)).astype(np.float32).astype(np.float64)
    net = dem.Mlp(p)
    y = net.forward(x)
    yo = mlp.forward(oracle_view(p), mlp.bf16_round(x))
    assert y.shape == (batch, 2)
    err = np.max(np.abs(y - yo) / (1.0 + np.abs(yo)))
    print("forward batch %d: max |dy| / (1 + |y|) = %.4f" % (batch, err))
    assert err <= 0.027


def test_forward_special_cases():
    """zero hidden weights: y = b4 exactly; zero batch is a no-op"""
    rng = np.random.default_rng(1)
    layers = [(np.zeros((6, 64)), rng.normal(size=64)), (np.zeros((64, 64)), rng.normal(size=64)),
              (np.zeros((64, 64)), rng.normal(size=64)), (np.zeros((64, 2)), np.array([0.25, -1.5]))]
    net = dem.Mlp(mlp.pack(layers))
    y = net.forward(rng.normal(size=(37, 6)))
    np.testing.assert_array_equal(y, np.tile([0.25, -1.5], (37, 1)))
    assert dem.dem_mlp_forward(net.h, None, None, 0) == 0


def test_params_roundtrip_and_errors():
    p = fp32_params(4)
    net = dem.Mlp(p)
    np.testing.assert_array_equal(net.params(), p.astype(np.float32))
    assert dem.dem_mlp_forward(net.h, None, None, -1) == -1
    assert dem.dem_mlp_train_step(net.h, None, None, 16, 0.1)[0] == -1
    assert dem.dem_mlp_train_step(net.h, 1, 1, 16, -1.0)[0] == -1


@pytest.mark.parametrize("batch", [40, 3000])
def test_gradient_matches_oracle(batch):
    rng = np.random.default_rng(7)
    p = fp32_params(8)
    x = rng.normal(size=(batch, 6)).astype(np.float32).astype(np.float64)
    t = rng.normal(0, 0.5, size=(batch, 2)).astype(np.float32).astype(np.float64)
    net = dem.Mlp(p)
    loss, g = net.grad(x, t)
    lo, go = mlp.grad(oracle_view(p), mlp.bf16_round(x), t)
    assert loss == pytest.approx(lo, rel=0.05)
    for li, sl in enumerate(LAYER_SLICES):
        a, b = g[sl].astype(np.float64), go[sl]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        print("gradient batch %d layer %d: relative L2 %.4f, cosine %.6f" % (batch, li, rel, cos))
        assert rel <= 0.02
        assert cos >= 0.9999


def test_gradient_is_deterministic():
    rng = np.random.default_rng(9)
    x = rng.normal(size=(2500, 6))
    t = rng.normal(size=(2500, 2))
    net = dem.Mlp(fp32_params(10))
    l1, g1 = net.grad(x, t)
    l2, g2 = net.grad(x, t)
    assert l1 == l2
    np.testing.assert_array_equal(g1, g2)


def test_first_adam_step_matches_oracle():
    """The first Adam step moves every parameter by lr sign(g) (bias-corrected
    moments); compared where the oracle gradient's sign is unambiguous."""
    rng = np.random.default_rng(11)
    p = fp32_params(12)
    x = rng.normal(size=(2048, 6))
    t = rng.normal(0, 0.5, size=(2048, 2))
    lr = 1e-3
    net = dem.Mlp(p)
    net.train_step(x, t, lr)
    p1 = net.params().astype(np.float64)
    _, go = mlp.grad(oracle_view(p), mlp.bf16_round(x.astype(np.float32).astype(np.float64)),
                     t.astype(np.float32).astype(np.float64))
    p1o, _, _ = mlp.adam_step(p, go, np.zeros_like(p), np.zeros_like(p), 1, lr)
    assert np.all(np.abs(p1 - p) <= lr * (1 + 1e-5) + 1e-7)
    clear = np.abs(go) > 0.02 * np.abs(go).max()
    assert clear.sum() > 100
    np.testing.assert_allclose(p1[clear], p1o[clear], rtol=0, atol=1e-6)


def test_training_reduces_loss_and_is_reproducible():
    rng = np.random.default_rng(13)
    x = rng.normal(size=(4096, 6))
    t = np.stack([0.5 * np.tanh(x[:, 0] - x[:, 1]), 0.3 * np.sin(x[:, 2]) + 0.1 * x[:, 5]], axis=1)
    runs = []
    for _ in range(2):
        net = dem.Mlp(fp32_params(14, 0.5))
        losses = [net.train_step(x, t, 2e-3) for _ in range(150)]
        runs.append((losses, net.params()))
    losses = runs[0][0]
    assert losses[-1] < 0.2 * losses[0]
    assert runs[0][0] == runs[1][0]
    np.testing.assert_array_equal(runs[0][1], runs[1][1])


# ---------------------------------------------------------------------------
# the closure inside the DEM coupling
# ---------------------------------------------------------------------------
def _c0_closure_case(n=1500):
    w = dict(synth.c0())
    w["x"], w["r"] = w["x"][:n], w["r"][:n]
    p = fp32_params(21, 0.5)
    norm = np.array([0.6, 0.05, 2.0, 1.0, 0.01, 4.0, 0.2, 0.05, 2.0, 1.0, 0.02, 3.0])
    return w, p, norm


def _closure_pair(w, p, norm):
    mat = cg.scale_material(w["material"], w.get("k", 1.0))
    op = oracle.make_params(mat, w["dt"], g=w["g"], walls=w["walls"], grid=w["grid"], fluid=w["fluid"],
                            outlet=w["outlet"])
    o = oracle.OracleSim(op, w["x"], w["r"], bond_at_init=True)
    o.set_fluid(w["u_cell"], w["gradp_cell"])
    o.set_closure_mlp(oracle_view(p), norm)
    g = dem.Simulation(dem.params_from_workload(w, precision="fp64"), w["x"], w["r"])
    g.map_fluid(w["u_cell"], w["gradp_cell"])
    net = dem.Mlp(p)
    g.set_closure(net, norm)
    return g, o, net


def test_closure_features_and_factors_match_oracle():
    """first coupling evaluation (step 0): features in FP64 on both sides,
    factors through the BF16 network"""
    w, p, norm = _c0_closure_case()
    g, o, _ = _closure_pair(w, p, norm)
    g.step(1)
    o.step(1)
    cl = g.read_closure()
    fo = o.closure_last_features()
    col = np.abs(fo).max(axis=0) + 1e-300
    assert np.all(np.abs(cl["features"] - fo) <= 1e-9 * col)
    assert fo[:, 5].max() >= 3 and fo[:, 0].min() > 0
    cdo, cco = o.closure_factors()
    yo = np.log(np.stack([cdo, cco], axis=1))
    yg = np.log(np.stack([cl["c_drag"], cl["c_coh"]], axis=1))
    err = np.max(np.abs(yg - yo) / (1.0 + np.abs(yo)))
    print("closure factors: max |dy| / (1 + |y|) = %.4f" % err)
    assert err <= 0.027
    assert np.all((cl["c_drag"] >= 0.5) & (cl["c_drag"] <= 2.0))
    assert np.all((cl["c_coh"] >= 0.5) & (cl["c_coh"] <= 2.0))


def test_closure_constant_factors_dynamics_match_oracle():
    """A network with zero weights and output bias (ln 1.5, ln 0.7) applies
    c_drag = 1.5 and c_coh = 0.7 everywhere (to FP32 rounding of exp): forces
    after two coupling intervals agree with the oracle's."""
    w, p, norm = _c0_closure_case()
    layers = [(np.zeros_like(W), np.zeros_like(b)) for W, b in mlp.unpack(p)]
    layers[3] = (layers[3][0], np.array([math.log(1.5), math.log(0.7)]))
    pc = mlp.pack(layers).astype(np.float32).astype(np.float64)
    g, o, _ = _closure_pair(w, pc, norm)
    ce = w["fluid"]["couple_every"]
    g.step(2 * ce + 1)
    o.step(2 * ce + 1)
    cl = g.read_closure()
    np.testing.assert_allclose(cl["c_drag"], 1.5, rtol=2e-7)
    np.testing.assert_allclose(cl["c_coh"], 0.7, rtol=2e-7)
    gs, os_ = g.state(), o.state()
    err = np.linalg.norm(gs["F"] - os_["F"], axis=1) / (os_["fscale"] + 1e-300)
    assert err.max() < 1e-5
    np.testing.assert_array_equal(g.pairs()["pairs"], o.pairs()["pairs"])


def test_closure_off_restores_unit_factors():
    w, p, norm = _c0_closure_case(400)
    g = dem.Simulation(dem.params_from_workload(w, precision="fp64"), w["x"], w["r"])
    g.map_fluid(w["u_cell"], w["gradp_cell"])
    base = dem.Simulation(dem.params_from_workload(w, precision="fp64"), w["x"], w["r"])
    base.map_fluid(w["u_cell"], w["gradp_cell"])
    net = dem.Mlp(mlp.pack([(np.zeros_like(W), np.zeros_like(b)) for W, b in mlp.unpack(p)]))
    g.set_closure(net, norm)          # y = 0: every factor is exactly 1
    g.step(3)
    base.step(3)
    np.testing.assert_array_equal(g.state()["F"], base.state()["F"])
    g.set_closure(None)
    with pytest.raises(dem.DemError):
        g.read_closure()
    with pytest.raises(dem.DemError):
        g.set_closure(net, np.zeros(12))
