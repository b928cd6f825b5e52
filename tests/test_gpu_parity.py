"""GPU path (through the C ABI) against the FP64 oracle on the same inputs.

Bars (stated by the method's target): contact sets bit-exact; per-step
forces and torques within 1e-12 (FP64) or 1e-5 (mixed: FP32 forces)
relative to the magnitude scale of each particle's force terms (the sum of
the magnitudes of every term that enters it, so that cancelling terms, e.g.
JKR at point B or a resting packing, do not inflate relative error).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import cg
from synth import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2211_06142_amd import dem  # noqa: E402


def oracle_for(wk, x=None, r=None, **kw):
    mat = cg.scale_material(wk["material"], wk.get("k", 1.0))
    op = oracle.make_params(mat, wk["dt"], g=wk["g"], walls=wk["walls"], grid=wk["grid"], fluid=wk["fluid"],
                            outlet=wk["outlet"])
    sim = oracle.OracleSim(op, wk["x"] if x is None else x, wk["r"] if r is None else r, **kw)
    if wk["fluid"] is not None:
        sim.set_fluid(wk["u_cell"], wk["gradp_cell"])
    return sim


def gpu_for(w, precision, x=None, r=None, **kw):
    p = dem.params_from_workload(w, precision=precision)
    sim = dem.Simulation(p, w["x"] if x is None else x, w["r"] if r is None else r, **kw)
    if w["fluid"] is not None:
        sim.map_fluid(w["u_cell"], w["gradp_cell"])
    return sim


def scaled_err(a, b, scale):
    return np.max(np.linalg.norm(a - b, axis=1) / (scale + 1e-300))


def c0_sub(n=2000):
    w = synth.c0()
    if n < len(w["r"]):
        w = dict(w)
        w["x"], w["r"] = w["x"][:n], w["r"][:n]
    return w


# ---------------------------------------------------------------------------
# contact sets
# ---------------------------------------------------------------------------
def test_contact_sets_bit_exact_c0():
    w = c0_sub()
    g = gpu_for(w, "fp64")
    margin = g.info()["cutoff_margin"]
    touch = g.pairs(which=1)["pairs"]
    cand = g.pairs(which=2)["pairs"]
    np.testing.assert_array_equal(touch, oracle.pairs(w["x"], w["r"], extra=0.0, method="brute"))
    np.testing.assert_array_equal(cand, oracle.pairs(w["x"], w["r"], extra=margin, method="brute"))
    # bonds at t = 0: every touching pair
    act = g.pairs(which=0)
    np.testing.assert_array_equal(act["pairs"], touch)
    assert np.all(act["bonded"] == 1)


@pytest.mark.parametrize("seed", [11, 12])
def test_contact_sets_random_polydisperse(seed):
    rng = np.random.default_rng(seed)
    n = 3000
    x = rng.uniform(0, 2.5e-3, (n, 3))
    r = np.exp(rng.normal(math.log(6e-5), 0.4, n))
    w = dict(synth.c0())
    w["fluid"] = None
    w["walls"] = []
    g = gpu_for(w, "fp64", x=x, r=r)
    margin = g.info()["cutoff_margin"]
    np.testing.assert_array_equal(g.pairs(which=1)["pairs"], oracle.pairs(x, r, extra=0.0))
    np.testing.assert_array_equal(g.pairs(which=2)["pairs"], oracle.pairs(x, r, extra=margin))


@pytest.mark.parametrize("lanes", [1, 4])
def test_long_rows_and_crowded_cells(lanes):
    """Rows longer than the scratch stride and binning cells too full for LDS
    (a large sphere with a shell of 100 touching small ones, in a dense gas):
    contact sets bit-exact, then 10 FP64 steps against the oracle, so the
    half-pair slots of the long rows must be right for the history to agree.
    With one lane per particle the step kernel's per-wave contact queue fills
    and its rows span several rounds."""
    x, r = scenes.shells_in_gas(np.random.default_rng(5))
    w = dict(synth.c0())
    w["fluid"] = None
    w["walls"] = []
    g = gpu_for(w, "fp64", x=x, r=r)
    g.set_lanes(lanes)
    margin = g.info()["cutoff_margin"]
    cand = oracle.pairs(x, r, extra=margin)
    assert np.bincount(cand.ravel(), minlength=len(r)).max() > 64
    np.testing.assert_array_equal(g.pairs(which=1)["pairs"], oracle.pairs(x, r, extra=0.0))
    np.testing.assert_array_equal(g.pairs(which=2)["pairs"], cand)
    o = oracle_for(w, x=x, r=r, bond_at_init=True)
    g.step(5)
    g.request_rebuild()       # the history of the long rows is carried through a rebuild
    g.step(5)
    o.step(10)
    gs, os_ = g.state(), o.state()
    assert scaled_err(gs["F"], os_["F"], os_["fscale"]) < 1e-12
    assert scaled_err(gs["T"], os_["T"], os_["tscale"]) < 1e-12
    np.testing.assert_allclose(gs["x"], os_["x"], rtol=0, atol=1e-16)
    gp, op_ = g.pairs(which=0), o.pairs()
    np.testing.assert_array_equal(gp["pairs"], op_["pairs"])
    np.testing.assert_array_equal(gp["bonded"], op_["bonded"])
    dts = np.abs(op_["dt"]).max() + 1e-30
    np.testing.assert_allclose(gp["dt"], op_["dt"], rtol=0, atol=1e-11 * dts)


# ---------------------------------------------------------------------------
# one and several steps, FP64
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nsteps", [1, 10, 40])
def test_c0_fp64_steps(nsteps):
    w = c0_sub()
    g = gpu_for(w, "fp64")
    o = oracle_for(w, bond_at_init=True)
    g.step(nsteps)
    o.step(nsteps)
    gs, os_ = g.state(), o.state()
    assert scaled_err(gs["F"], os_["F"], os_["fscale"]) < 1e-12
    assert scaled_err(gs["T"], os_["T"], os_["tscale"]) < 1e-12
    np.testing.assert_allclose(gs["x"], os_["x"], rtol=0, atol=1e-16)
    vs = np.abs(os_["v"]).max()
    np.testing.assert_allclose(gs["v"], os_["v"], rtol=0, atol=1e-11 * vs)
    np.testing.assert_array_equal(gs["alive"], os_["alive"])
    gp = g.pairs(which=0)
    op_ = o.pairs()
    np.testing.assert_array_equal(gp["pairs"], op_["pairs"])
    np.testing.assert_array_equal(gp["bonded"], op_["bonded"])
    dts = np.abs(op_["dt"]).max() + 1e-30
    np.testing.assert_allclose(gp["dt"], op_["dt"], rtol=0, atol=1e-11 * dts)
    sc = o.scalars()
    assert gs["broken_bonds"] == sc["broken_bonds"]
    assert gs["n_contacts"] == sc["n_contacts"]


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_c0_fp64_lanes_per_particle(lanes):
    """the step kernel's lane-group size is a tuning knob: any setting matches
    the oracle to rounding"""
    w = c0_sub()
    g = gpu_for(w, "fp64")
    g.set_lanes(lanes)
    o = oracle_for(w, bond_at_init=True)
    g.step(10)
    o.step(10)
    gs, os_ = g.state(), o.state()
    assert scaled_err(gs["F"], os_["F"], os_["fscale"]) < 1e-12
    assert scaled_err(gs["T"], os_["T"], os_["tscale"]) < 1e-12
    with pytest.raises(dem.DemError):
        g.set_lanes(5)


def test_c0_fluid_cells_fp64():
    w = c0_sub()
    g = gpu_for(w, "fp64")
    o = oracle_for(w, bond_at_init=True)
    g.step(1)
    o.step(1)
    eps, fd = g.fluid_out()
    of = o.fluid()
    np.testing.assert_allclose(eps, of["eps_s"], rtol=1e-12, atol=1e-15)
    fs = np.abs(of["fdrag_cell"]).max()
    np.testing.assert_allclose(fd, of["fdrag_cell"], rtol=0, atol=1e-12 * fs)


@pytest.mark.parametrize("gn", [4, 5])
def test_coarse_grid_bucket_overflow_fp64(gn):
    """The c0 bed on a coarse fluid grid, so that buckets hold far more members
    than a bucket's list (64) or a lane (16) keeps: gn 5 is the sparse path of
    the solid-volume pass (31 particles per bucket on average, up to 163 in a
    bucket: its second scan, and the drag pass scanning overflowed buckets
    again), gn 4 the dense one (74 on average, up to 275).  Porosity and cell
    drag source against the oracle after one step (eq 6, eq 7)."""
    w = dict(c0_sub())
    lo, hi, _ = w["grid"]
    w["grid"] = (lo, hi, (gn, gn, gn))
    w["u_cell"], w["gradp_cell"] = synth.uniform_field(w["grid"], (0.0, 0.0, 0.05))
    ndual = (gn - 1) ** 3
    assert (len(w["r"]) > 32 * ndual) == (gn == 4)
    g = gpu_for(w, "fp64")
    o = oracle_for(w, bond_at_init=True)
    g.step(1)
    o.step(1)
    eps, fd = g.fluid_out()
    of = o.fluid()
    np.testing.assert_allclose(eps, of["eps_s"], rtol=1e-12, atol=1e-15)
    fs = np.abs(of["fdrag_cell"]).max()
    np.testing.assert_allclose(fd, of["fdrag_cell"], rtol=0, atol=1e-12 * fs)
    gs, os_ = g.state(), o.state()
    assert scaled_err(gs["F"], os_["F"], os_["fscale"]) < 1e-12


def test_c0_mixed_one_step():
    w = c0_sub()
    g = gpu_for(w, "mixed")
    o = oracle_for(w, bond_at_init=True)
    g.step(1)
    o.step(1)
    gs, os_ = g.state(), o.state()
    assert scaled_err(gs["F"], os_["F"], os_["fscale"]) < 1e-5
    assert scaled_err(gs["T"], os_["T"], os_["tscale"]) < 1e-5
    np.testing.assert_array_equal(g.pairs(which=0)["pairs"], o.pairs()["pairs"])


def test_determinism_bitwise():
    w = c0_sub()
    outs = []
    for _ in range(2):
        g = gpu_for(w, "mixed")
        g.step(30)
        s = g.state()
        outs.append((s["x"].copy(), s["F"].copy(), s["T"].copy()))
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def _moving_c0(n=2000, sigma=1.0, seed=31):
    w = c0_sub(n)
    v = np.random.default_rng(seed).normal(0.0, sigma, (len(w["r"]), 3))
    return w, v


def test_natural_rebuilds_mid_window_match_oracle():
    """Random velocities of about 1 m/s force list rebuilds inside the step
    windows (the displacement trigger, not a request): the steps after each
    rebuild must continue from the complete state of the step before it."""
    w, v = _moving_c0()
    g = gpu_for(w, "fp64", v=v)
    o = oracle_for(w, v=v, bond_at_init=True)
    g.step(90)
    o.step(90)
    assert g.info()["rebuilds"] >= 3
    gs, os_ = g.state(), o.state()
    assert scaled_err(gs["F"], os_["F"], os_["fscale"]) < 1e-12
    np.testing.assert_allclose(gs["x"], os_["x"], rtol=0, atol=1e-16)
    np.testing.assert_array_equal(g.pairs()["pairs"], o.pairs()["pairs"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_windows_identical_to_direct_launches(precision):
    """Recorded step windows replay the same launches: bit-identical states,
    across natural rebuilds and coupling evaluations, over several calls."""
    w, v = _moving_c0(1500, 1.0, 37)
    sims = []
    for graphs in (False, True):
        g = gpu_for(w, precision, v=v)
        g.set_graphs(graphs)
        for k in (70, 5, 64, 1):
            g.step(k)
        sims.append(g)
    a, b = sims[0].state(), sims[1].state()
    assert sims[0].info()["rebuilds"] >= 3
    assert sims[0].info()["rebuilds"] == sims[1].info()["rebuilds"]
    for key in ("x", "v", "w", "F", "T"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


def test_rebuild_invariance():
    """The neighbour list is an acceleration: forcing a rebuild every step must
    not change the contact set, bonds or forces beyond rounding."""
    w = c0_sub(1200)
    a = gpu_for(w, "fp64")
    b = gpu_for(w, "fp64")
    for _ in range(15):
        a.step(1)
        b.request_rebuild()
        b.step(1)
    sa, sb = a.state(), b.state()
    o = oracle_for(w, x=w["x"], r=w["r"], bond_at_init=True)
    o.step(15)
    sc = o.state()["fscale"]
    assert scaled_err(sa["F"], sb["F"], sc) < 1e-12
    np.testing.assert_array_equal(a.pairs()["pairs"], b.pairs()["pairs"])
    assert b.info()["rebuilds"] >= 15


# ---------------------------------------------------------------------------
# tiny scenes: restitution, incline, pull-off
# ---------------------------------------------------------------------------
def _scene_pair(model, mat, speed, dt, precision="fp64", **kw):
    x, r, v = scenes.two_spheres(7.5e-5, 7.5e-5, 1e-9, speed)
    p = dem.make_params(mat, dt, g=(0, 0, 0), normal_model=model, bond_at_init=False, precision=precision, **kw)
    op = oracle.make_params(mat, dt, g=(0, 0, 0), normal_model=model, k_lin=kw.get("k_lin", 0.0))
    return dem.Simulation(p, x, r, v=v), oracle.OracleSim(op, x, r, v=v, bond_at_init=False)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cor_matches_oracle(precision):
    mat = scenes.material(e=0.5, mu=0.0, gamma=0.0)
    g, o = _scene_pair(dem.DEM_NORMAL_HERTZ, mat, 0.2, 5e-9, precision)
    g.step(6000)
    o.step(6000)
    vg = g.state()["v"]
    vo = o.state()["v"]
    cor_g = -(vg[0, 0] - vg[1, 0]) / 0.2
    cor_o = -(vo[0, 0] - vo[1, 0]) / 0.2
    assert 0.4 < cor_o < 0.7
    assert cor_g == pytest.approx(cor_o, rel=1e-10 if precision == "fp64" else 1e-4)


def test_linear_law_cor_equals_e():
    mat = scenes.material(e=0.5, mu=0.0, gamma=0.0)
    g, _ = _scene_pair(dem.DEM_NORMAL_LINEAR, mat, 0.1, 2e-9, k_lin=500.0)
    g.step(40000)
    v = g.state()["v"]
    assert -(v[0, 0] - v[1, 0]) / 0.1 == pytest.approx(0.5, abs=2e-3)


@pytest.mark.parametrize("theta,rolls", [(math.radians(20), True), (math.radians(70), False)])
def test_incline_gpu(theta, rolls):
    r = 1e-4
    mu = 0.5
    mat = scenes.material(mu=mu, gamma=0.0)
    gvec = scenes.incline_gravity(theta)
    Es, _ = oracle.effective_moduli(mat["E"], mat["nu"])
    m = mat["rho"] * 4 / 3 * math.pi * r ** 3
    d0 = (m * 9.81 * math.cos(theta) / (4 / 3 * (2 * Es) * math.sqrt(r))) ** (2 / 3)
    p = dem.make_params(mat, 1e-7, g=gvec, walls=[scenes.plane((0, 0, 1), 0.0)],
                        normal_model=dem.DEM_NORMAL_HERTZ, bond_at_init=False)
    sim = dem.Simulation(p, np.array([[0, 0, r - d0]]), np.array([r]))
    sim.step(5000)
    t, vx = [], []
    for k in range(20):
        sim.step(1000)
        t.append(k * 1e-4)
        vx.append(sim.state()["v"][0, 0])
    a = np.polyfit(t, vx, 1)[0]
    expect = 5 / 7 * 9.81 * math.sin(theta) if rolls else 9.81 * (math.sin(theta) - mu * math.cos(theta))
    assert a == pytest.approx(expect, rel=3e-3)


def test_pull_off_gpu_matches_oracle():
    r = 7.5e-5
    Es, _ = oracle.effective_moduli(70e6, 0.3)
    Rs = r / 2
    X = (math.pi ** 2 * 0.25 * Rs / Es ** 2) ** (1 / 3)
    mat = scenes.material(e=1.0, mu=0.0, rho=1e9)
    x, rr, v = scenes.two_spheres(r, r, -0.5 * X, -2e-3)
    p = dem.make_params(mat, 1e-7, g=(0, 0, 0), bond_at_init=False)
    g = dem.Simulation(p, x, rr, v=v, pairs=np.array([[0, 1]]), pair_bonded=np.array([1]))
    op = oracle.make_params(mat, 1e-7, g=(0, 0, 0))
    o = oracle.OracleSim(op, x, rr, v=v, pairs=np.array([[0, 1]]), pair_bonded=np.array([1]), bond_at_init=False)
    broke_g = broke_o = None
    fmin = 0.0
    for k in range(3000):
        g.step(1)
        o.step(1)
        sg = g.state()
        if broke_g is None and sg["broken_bonds"] == 1:
            broke_g = k
        if broke_o is None and o.scalars()["broken_bonds"] == 1:
            broke_o = k
        if broke_g is None:
            fmin = min(fmin, -sg["F"][0, 0])
        if broke_g is not None and broke_o is not None:
            break
    assert broke_g is not None and broke_g == broke_o
    assert fmin == pytest.approx(-3 * math.pi * 0.5 * Rs, rel=1e-6)


# ---------------------------------------------------------------------------
# error paths through the ABI
# ---------------------------------------------------------------------------
def test_invalid_params_rejected():
    w = c0_sub(100)
    for bad in (dict(dt=-1.0), dict(nu=0.6), dict(e=0.0), dict(k=0.5)):
        p = dem.params_from_workload(w)
        for key, val in bad.items():
            setattr(p, key, val)
        with pytest.raises(dem.DemError) as ei:
            dem.Simulation(p, w["x"], w["r"])
        assert ei.value.code == dem.DEM_E_INVAL
    p = dem.params_from_workload(w, dt_rayleigh_max_frac=1e-3)
    with pytest.raises(dem.DemError):
        dem.Simulation(p, w["x"], w["r"])


def test_nonfinite_input_rejected():
    w = c0_sub(100)
    v = np.zeros((100, 3))
    v[3, 1] = np.nan
    with pytest.raises(dem.DemError) as ei:
        dem.Simulation(dem.params_from_workload(w), w["x"], w["r"], v=v)
    assert ei.value.code == dem.DEM_E_INVAL


def test_step_without_fluid_fields_is_state_error():
    w = c0_sub(100)
    sim = dem.Simulation(dem.params_from_workload(w), w["x"], w["r"])
    assert dem.dem_step(sim.ctx, 1) == dem.DEM_E_STATE


# ---------------------------------------------------------------------------
# full size: the 200 000-particle cylinder in the launch configuration of the
# benchmark (mixed precision) against the oracle
# ---------------------------------------------------------------------------
def test_c1_full_size_against_oracle():
    """The 200 000-sphere cylinder, built exactly as bench.py builds it (mixed
    precision, its skin and lanes per particle), over its first 5 steps, each
    judged from one identical state: before every step the oracle is seeded
    from the GPU's state (positions, velocities, angular velocities, forces,
    torques, alive flags, active pairs with elongation and bond flag, wall
    history, held fluid force, step count), then both take the step.  Forces
    and torques within 1e-5 of each particle's force scale, pair and bond
    sets and alive flags exact, and the cells of the coupling evaluation of
    step 0 (FP64 in mixed mode too) within 1e-12."""
    import bench
    w = synth.c1()
    g = bench.build_sim([w], bench.SKIN_FACTOR["c1"], bench.LANES, 0)
    np.testing.assert_array_equal(g.pairs(which=0)["pairs"], oracle.pairs(w["x"], w["r"], extra=0.0))
    nw = len(w["walls"])
    for k in range(5):
        s = g.state(held=True)
        pr = g.pairs(which=0)
        o = oracle_for(w, x=s["x"], v=s["v"], w=s["w"], F=s["F"], T=s["T"], alive=s["alive"], pairs=pr["pairs"],
                       pair_dt=pr["dt"], pair_bonded=pr["bonded"], bond_at_init=False,
                       wall_dt=np.ascontiguousarray(s["wall_dt"][:, :nw, :]))
        o.set_held(s["step"], s["fluid_force"])
        g.step(1)
        o.step(1)
        gs, os_ = g.state(), o.state()
        np.testing.assert_array_equal(gs["alive"], os_["alive"])
        ef = scaled_err(gs["F"], os_["F"], os_["fscale"])
        et = scaled_err(gs["T"], os_["T"], os_["tscale"])
        print("c1 step %d: scaled force error %.2e, torque %.2e" % (k, ef, et))
        assert ef < 1e-5 and et < 1e-5
        gp, op_ = g.pairs(which=0), o.pairs()
        np.testing.assert_array_equal(gp["pairs"], op_["pairs"])
        np.testing.assert_array_equal(gp["bonded"], op_["bonded"])
        assert gs["broken_bonds"] - s["broken_bonds"] == o.scalars()["broken_bonds"]
        if k == 0:
            eps, fd = g.fluid_out()
            of = o.fluid()
            np.testing.assert_allclose(eps, of["eps_s"], rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(fd, of["fdrag_cell"], rtol=0, atol=1e-12 * np.abs(of["fdrag_cell"]).max())


def test_c0_full_run_aggregates():
    """The whole c0 configuration (2 000 spheres, FP64, 1 000 steps) against
    the oracle on aggregates, the comparison for horizons where the
    trajectories may part by rounding: contacts within 2 %, broken bonds
    within 2 % (or 2 bonds), kinetic energy within 5 %, produced mass equal
    (the walled box has no outlet)."""
    w = synth.c0()
    g = gpu_for(w, "fp64")
    o = oracle_for(w, bond_at_init=True)
    g.step(1000)
    o.step(1000)
    gs, sc = g.state(), o.scalars()
    assert gs["step"] == sc["step"] == 1000
    assert gs["n_contacts"] == pytest.approx(sc["n_contacts"], rel=0.02)
    assert abs(gs["broken_bonds"] - sc["broken_bonds"]) <= max(2, 0.02 * sc["broken_bonds"])
    assert gs["kinetic"] == pytest.approx(sc["kinetic"], rel=0.05)
    assert gs["produced_mass"] == sc["produced_mass"] == 0.0
