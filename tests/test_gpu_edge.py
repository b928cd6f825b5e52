"""Edge cases of the GPU path against the oracle: empty input, a single free
particle, every particle leaving through the outlet (steps and rebuilds with
no particle alive), an empty sample inside an ensemble, and a coarse-grained
material (k = 2, section 2.4) in FP64."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import cg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2211_06142_amd import dem  # noqa: E402


def _no_fluid(w):
    w = dict(w)
    w["fluid"] = None
    return w


def _oracle(w, x=None, r=None, **kw):
    mat = cg.scale_material(w["material"], w.get("k", 1.0))
    op = oracle.make_params(mat, w["dt"], g=w["g"], walls=w["walls"], grid=w["grid"], fluid=w["fluid"],
                            outlet=w["outlet"])
    o = oracle.OracleSim(op, w["x"] if x is None else x, w["r"] if r is None else r, **kw)
    if w["fluid"] is not None:
        o.set_fluid(w["u_cell"], w["gradp_cell"])
    return o


def _gpu(w, precision="fp64", x=None, r=None, **kw):
    g = dem.Simulation(dem.params_from_workload(w, precision=precision), w["x"] if x is None else x,
                       w["r"] if r is None else r, **kw)
    if w["fluid"] is not None:
        g.map_fluid(w["u_cell"], w["gradp_cell"])
    return g


def test_empty_input_rejected():
    w = _no_fluid(synth.c0())
    with pytest.raises(dem.DemError):
        dem.Simulation(dem.params_from_workload(w), np.zeros((0, 3)), np.zeros(0))


def test_single_free_particle():
    """no pairs, no walls: exact free fall under gravity (eq 1-2)"""
    w = _no_fluid(synth.c0())
    w["walls"] = []
    x = np.array([[1e-3, 1e-3, 2e-3]])
    r = np.array([1e-4])
    v = np.array([[0.01, -0.02, 0.3]])
    g = _gpu(w, x=x, r=r, v=v)
    o = _oracle(w, x=x, r=r, v=v)
    g.step(150)
    o.step(150)
    gs, os_ = g.state(), o.state()
    np.testing.assert_allclose(gs["x"], os_["x"], rtol=1e-15, atol=1e-18)
    np.testing.assert_allclose(gs["v"], os_["v"], rtol=1e-13, atol=1e-16)
    # the initial force is an input (zero here), so the first half kick adds
    # nothing: v = v0 + (t - dt/2) g
    t = (150 - 0.5) * w["dt"]
    np.testing.assert_allclose(gs["v"][0], v[0] + t * np.asarray(w["g"]), rtol=1e-12)
    assert g.pairs(which=2)["pairs"].shape[0] == 0


def test_every_particle_leaves_through_the_outlet():
    """A cavity wider than the box removes every sphere at the first drift; the
    steps, a forced rebuild and the coupling then run with nothing alive."""
    w = dict(synth.c0())
    n = 600
    w["x"], w["r"] = w["x"][:n], w["r"][:n]
    w["outlet"] = (1.5e-3, 1.5e-3, 10e-3)
    g = _gpu(w)
    o = _oracle(w, bond_at_init=True)
    g.step(12)
    g.request_rebuild()
    g.step(12)
    o.step(24)
    gs, os_ = g.state(), o.state()
    assert gs["n_alive"] == 0 and int(os_["alive"].sum()) == 0
    m = synth.MATERIAL["rho"] * (4.0 / 3.0) * math.pi * np.sum(w["r"] ** 3)
    assert gs["produced_mass"] == pytest.approx(m, rel=1e-12)
    assert gs["produced_mass"] == pytest.approx(o.scalars()["produced_mass"], rel=1e-12)
    assert g.pairs()["pairs"].shape[0] == 0
    assert gs["n_contacts"] == 0


def test_ensemble_with_an_empty_sample():
    base = synth.c1()
    a = synth.c3_crop(2, 800, 0.4, base)
    b = synth.c3_crop(5, 1200, 0.8, base)
    empty = dict(a)
    empty["x"], empty["r"] = np.zeros((0, 3)), np.zeros(0)
    ws = [a, empty, b]
    params = [dem.params_from_workload(s, precision="fp64") for s in ws]
    offs = np.array([0, len(a["r"]), len(a["r"]), len(a["r"]) + len(b["r"])], np.int64)
    sim = dem.Simulation(params, np.concatenate([s["x"] for s in ws]), np.concatenate([s["r"] for s in ws]),
                         sample_offsets=offs)
    sim.map_fluid(np.concatenate([s["u_cell"] for s in ws]), np.concatenate([s["gradp_cell"] for s in ws]))
    sim.step(15)
    st = sim.state()
    agg = sim.aggregates()
    assert agg["n_alive"][1] == 0 and agg["produced_mass"][1] == 0.0
    for k, (s, lo, hi) in enumerate([(a, 0, len(a["r"])), (b, offs[2], offs[3])]):
        o = _oracle(s, bond_at_init=True)
        o.step(15)
        os_ = o.state()
        err = np.linalg.norm(st["F"][lo:hi] - os_["F"], axis=1) / (os_["fscale"] + 1e-300)
        assert err.max() < 1e-12, k


@pytest.mark.parametrize("scheme", ["ssw", "ssp"])
def test_coarse_grained_material_fp64(scheme):
    """k = 2: the library scales the fine material (gamma x k, drag k^3 f(d/k),
    Table 3); the oracle gets the grain-scale material from oracle.cg"""
    w = dict(synth.c0())
    n = 1200
    w["x"], w["r"] = w["x"][:n], w["r"][:n]
    w["k"] = 2.0
    w["scheme"] = scheme
    g = _gpu(w)
    o = _oracle(w, bond_at_init=True)
    g.step(15)
    o.step(15)
    gs, os_ = g.state(), o.state()
    err = np.linalg.norm(gs["F"] - os_["F"], axis=1) / (os_["fscale"] + 1e-300)
    assert err.max() < 1e-12
    np.testing.assert_array_equal(g.pairs()["pairs"], o.pairs()["pairs"])
    eg, fg = g.fluid_out()
    fo = o.fluid()
    np.testing.assert_allclose(eg, fo["eps_s"], rtol=0, atol=1e-12)
    scale = np.abs(fo["fdrag_cell"]).max() + 1e-300
    np.testing.assert_allclose(fg, fo["fdrag_cell"], rtol=0, atol=1e-12 * scale)
