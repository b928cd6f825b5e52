"""GPU parity of the batched ensemble (an extension; not in arXiv:2211.06142):
independent samples with their own surface energy, walls and fluid grid share
one context and one launch per kernel; each must reproduce the oracle run of
that sample alone, and its own single-sample GPU run bit for bit."""
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

SIZES = [(0, 700, 0.15), (3, 1500, 0.9), (7, 300, 0.5), (11, 2200, 0.3), (19, 1000, 0.7)]


def _samples(precision="fp64"):
    base = synth.c1()
    ws = [synth.c3_crop(s, n, g, base) for s, n, g in SIZES]
    for w in ws:
        w["precision"] = precision
    return ws


def _batched(ws, precision):
    params = [dem.params_from_workload(w, precision=precision) for w in ws]
    offs = np.cumsum([0] + [len(w["r"]) for w in ws]).astype(np.int64)
    x = np.concatenate([w["x"] for w in ws])
    r = np.concatenate([w["r"] for w in ws])
    sim = dem.Simulation(params, x, r, sample_offsets=offs)
    sim.map_fluid(np.concatenate([w["u_cell"] for w in ws]), np.concatenate([w["gradp_cell"] for w in ws]))
    return sim, offs


def _oracle(w):
    mat = cg.scale_material(w["material"], w.get("k", 1.0))
    op = oracle.make_params(mat, w["dt"], g=w["g"], walls=w["walls"], grid=w["grid"], fluid=w["fluid"],
                            outlet=w["outlet"])
    o = oracle.OracleSim(op, w["x"], w["r"], bond_at_init=True)
    o.set_fluid(w["u_cell"], w["gradp_cell"])
    return o


def test_ensemble_matches_oracle_per_sample():
    ws = _samples()
    sim, offs = _batched(ws, "fp64")
    nsteps = 2 * ws[0]["fluid"]["couple_every"] + 3
    sim.step(nsteps)
    st = sim.state()
    pairs = sim.pairs()["pairs"]
    agg = sim.aggregates()
    for s, w in enumerate(ws):
        o = _oracle(w)
        o.step(nsteps)
        os_ = o.state()
        a, b = offs[s], offs[s + 1]
        err = np.linalg.norm(st["F"][a:b] - os_["F"], axis=1) / (os_["fscale"] + 1e-300)
        assert err.max() < 1e-12, s
        np.testing.assert_allclose(st["x"][a:b], os_["x"], rtol=0, atol=1e-16)
        mine = pairs[(pairs[:, 0] >= a) & (pairs[:, 0] < b)] - a
        np.testing.assert_array_equal(mine, o.pairs()["pairs"])
        assert agg["broken_bonds"][s] == o.scalars()["broken_bonds"]


def test_ensemble_sample_equals_its_single_run():
    ws = _samples("mixed")
    sim, offs = _batched(ws, "mixed")
    k = 3
    one = dem.Simulation(dem.params_from_workload(ws[k], precision="mixed"), ws[k]["x"], ws[k]["r"])
    one.map_fluid(ws[k]["u_cell"], ws[k]["gradp_cell"])
    sim.step(25)
    one.step(25)
    a, b = offs[k], offs[k + 1]
    # no rebuild after the initial one on either side, so the rows (and the
    # summation order of every force) are the same
    assert sim.info()["rebuilds"] == 1 and one.info()["rebuilds"] == 1
    sb, so = sim.state(), one.state()
    for key in ("x", "v", "w", "F", "T"):
        np.testing.assert_array_equal(sb[key][a:b], so[key], err_msg=key)


def test_c3_full_size_sampled_against_oracle():
    """The whole 256-sample ensemble (2.66 M spheres), built exactly as the
    bench builds it, stepped 3 times; sampled samples (the three smallest, one
    in the middle of the sweep, the last) against their own oracle runs: the
    same contact and bond sets, forces to the mixed-precision bar."""
    import bench
    ws = synth.c3()
    sim = bench.build_sim(ws, bench.SKIN_FACTOR["c3"], bench.LANES, 0)
    offs = np.cumsum([0] + [len(w["r"]) for w in ws]).astype(np.int64)
    sim.step(3)
    st = sim.state()
    pairs = sim.pairs()["pairs"]
    sizes = np.array([len(w["r"]) for w in ws])
    picks = list(np.argsort(sizes, kind="stable")[:3]) + [128, 255]
    for s in picks:
        w = ws[s]
        o = _oracle(w)
        o.step(3)
        os_ = o.state()
        a, b = offs[s], offs[s + 1]
        err = np.linalg.norm(st["F"][a:b] - os_["F"], axis=1) / (os_["fscale"] + 1e-300)
        assert err.max() < 1e-5, s
        mine = pairs[(pairs[:, 0] >= a) & (pairs[:, 0] < b)] - a
        np.testing.assert_array_equal(mine, o.pairs()["pairs"])


# (sample index, size in parcels, surface energy, coarse-graining factor k)
K_SIZES = [(0, 900, 0.2, 1), (4, 400, 0.8, 2), (8, 150, 0.5, 3), (13, 1200, 0.35, 1), (17, 260, 0.6, 3),
           (22, 500, 0.95, 2)]


def _k_samples(precision):
    bases = {1: synth.c1(), 2: synth.c2(2), 3: synth.c2(3)}
    ws = [synth.c3_crop(s, n, g, bases[k]) for s, n, g, k in K_SIZES]
    for w in ws:
        w["precision"] = precision
    return ws


def test_ensemble_per_sample_k_matches_oracle():
    """Samples with their own coarse-graining factor (k = 1, 2, 3: gamma x k,
    drag k^3 f(d/k)) in one context: each reproduces the FP64 oracle run of that
    sample alone with its grain-scale material."""
    ws = _k_samples("fp64")
    assert sorted({w["k"] for w in ws}) == [1.0, 2.0, 3.0]
    sim, offs = _batched(ws, "fp64")
    nsteps = 2 * ws[0]["fluid"]["couple_every"] + 3
    sim.step(nsteps)
    st = sim.state()
    pairs = sim.pairs()["pairs"]
    agg = sim.aggregates()
    for s, w in enumerate(ws):
        o = _oracle(w)
        o.step(nsteps)
        os_ = o.state()
        a, b = offs[s], offs[s + 1]
        err = np.linalg.norm(st["F"][a:b] - os_["F"], axis=1) / (os_["fscale"] + 1e-300)
        assert err.max() < 1e-12, (s, w["k"])
        terr = np.linalg.norm(st["T"][a:b] - os_["T"], axis=1) / (os_["tscale"] + 1e-300)
        assert terr.max() < 1e-12, (s, w["k"])
        np.testing.assert_allclose(st["x"][a:b], os_["x"], rtol=0, atol=1e-16)
        mine = pairs[(pairs[:, 0] >= a) & (pairs[:, 0] < b)] - a
        np.testing.assert_array_equal(mine, o.pairs()["pairs"])
        assert agg["broken_bonds"][s] == o.scalars()["broken_bonds"]


def test_ensemble_graph_windows_identical_to_direct_launches():
    """The mixed-k ensemble with recorded step windows replayed (as the bench
    times it) gives the states of direct launches bit for bit, over several
    calls and coupling evaluations."""
    ws = _k_samples("mixed")
    out = []
    for graphs in (False, True):
        sim, _ = _batched(ws, "mixed")
        sim.set_graphs(graphs)
        for k in (23, 5, 31, 1):
            sim.step(k)
        out.append(sim.state())
    for key in ("x", "v", "w", "F", "T"):
        np.testing.assert_array_equal(out[0][key], out[1][key], err_msg=key)
