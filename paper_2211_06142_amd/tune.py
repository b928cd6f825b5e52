"""Autotuner of the free numerical parameters of the DEM step.

Neither parameter changes the physics: the neighbour skin trades list length
(pair entries the step kernel walks) against rebuild frequency, and the lanes
per particle trade parallelism against group-reduction work; results differ
between settings by rounding only.  Each trial is a short run through the
library (C-ABI) timed with HIP events on the context's stream; the tuner only
chooses.
"""
import numpy as np

from . import dem


def _time_steps(sim, steps):
    torch = sim.torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def tune(make_sim, skins, lanes=(1, 2, 4, 8), warmup=40, steps=1000, log=None):
    """make_sim(skin) -> a fresh dem.Simulation with that skin (metres).
    Returns (best, table): best = dict(skin, lanes, ms_per_step), table = all
    trials as (skin, lanes, ms_per_step, rebuilds)."""
    table = []
    for skin in skins:
        sim = make_sim(skin)
        sim.step(warmup)
        for ln in lanes:
            sim.set_lanes(ln)
            r0 = sim.info()["rebuilds"]
            ms = _time_steps(sim, steps) / steps
            table.append((float(skin), int(ln), float(ms), sim.info()["rebuilds"] - r0))
            if log:
                log("tune: skin %.3g m, %d lanes: %.4f ms/step" % (skin, ln, ms))
        sim.close()
    k = int(np.argmin([t[2] for t in table]))
    best = {"skin": table[k][0], "lanes": table[k][1], "ms_per_step": table[k][2]}
    return best, table


def tune_workload(w, skin_factors=(0.4, 0.8, 1.2, 1.6), precision=None, **kw):
    """Tune a workload dict (or a list of ensemble samples): skins are
    multiples of the smallest radius."""
    ws = w if isinstance(w, list) else [w]
    rmin = min(float(np.min(s["r"])) for s in ws)

    def make_sim(skin):
        params = [dem.params_from_workload(s, precision=precision, skin=skin) for s in ws]
        offs = np.cumsum([0] + [len(s["r"]) for s in ws]).astype(np.int64)
        sim = dem.Simulation(params if len(ws) > 1 else params[0], np.concatenate([s["x"] for s in ws]),
                             np.concatenate([s["r"] for s in ws]), sample_offsets=offs if len(ws) > 1 else None)
        sim.map_fluid(np.concatenate([s["u_cell"] for s in ws]), np.concatenate([s["gradp_cell"] for s in ws]))
        return sim

    return tune(make_sim, [f * rmin for f in skin_factors], **kw)
