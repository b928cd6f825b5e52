"""The paper's own sample run (arXiv:2211.06142 section 3.1) driven through
the library: the generated sand is compressed by the top plate to the
overburden stress, the compressed sample is perforated under the outlet, and
the sand-production run follows (bench.py --workload f2 --f2-protocol).

compress(): the bed of synth.f2_bed (the generation stage: geometric packing,
original JKR law) in a context of its own; between calls of dem_step the top
plate is moved by a proportional servo on the stress it carries (the
particles' force on it over the box's cross-section, dem_read_wall_forces),
down while the stress is below the target, up while above, by at most
`move_max` per cycle, until the stress has stayed within `tol` of the target
for `hold` cycles.  A plate moved between calls is quasi-static: its speed does
not enter the contact law (dem_set_walls).

perforate(): the compressed state with the tunnel under the outlet carved
(the grains whose centres lie within the penetrometer's radius of its axis
removed) in place of the penetrometer's push, the top plate replaced by the
plate with the outlet hole at the compressed height, the outlet above it, the
modified JKR law with every touching pair bonded (the paper applies it from
the perforation stage on), and the paper's fluid grid over the compressed
height; a workload dict in the layout of synth.f2.
"""
import math

import numpy as np

from . import dem


def _box_area(walls):
    """cross-section of the box from its side planes (normals +-x, +-y)"""
    lo, hi = [0.0, 0.0], [0.0, 0.0]
    for kind, p in walls:
        if kind != dem.DEM_WALL_PLANE:
            continue
        for ax in (0, 1):
            if p[ax] > 0.5:
                lo[ax] = p[3]
            elif p[ax] < -0.5:
                hi[ax] = -p[3]
    return (hi[0] - lo[0]) * (hi[1] - lo[1])


def compress(w, sigma=1.0e6, cycle_steps=200, move_max=0.5e-6, tol=0.03, hold=5, max_cycles=20000, log=None):
    """Servo-controlled compression of the bed w (synth.f2_bed) to the stress
    sigma on its top plate (the last wall, a plane facing down).  Returns the
    context (left in the compressed state), the plate's final height, the
    stress history and the porosity of the sample under the plate."""
    p = dem.params_from_workload(w, normal_model=dem.DEM_NORMAL_JKR_ORIG, bond_at_init=False)
    sim = dem.Simulation(p, w["x"], w["r"])
    walls = list(w["walls"])
    top = len(walls) - 1
    kind, prm = walls[top]
    assert kind == dem.DEM_WALL_PLANE and prm[2] < 0.0, "the last wall must be the top plate (normal -z)"
    area = _box_area(walls)
    z = -prm[3]
    hist = []
    inside = 0
    for cyc in range(max_cycles):
        sim.step(cycle_steps)
        s = float(sim.wall_forces()[0][top][2]) / area   # the bed pushes the plate up
        hist.append((cyc, z, s))
        err = (sigma - s) / sigma
        inside = inside + 1 if abs(err) <= tol else 0
        if log and cyc % 200 == 0:
            log("compress: cycle %d plate %.4f mm stress %.4g Pa" % (cyc, z * 1e3, s))
        if inside >= hold:
            break
        z -= max(-move_max, min(move_max, err * move_max))
        walls[top] = (kind, (0.0, 0.0, -1.0, -z))
        sim.set_walls(walls)
    vs = float(np.sum(4.0 / 3.0 * math.pi * w["r"] ** 3))
    return {"sim": sim, "plate_z": z, "history": np.array(hist), "stress": hist[-1][2], "cycles": len(hist),
            "steps": len(hist) * cycle_steps, "converged": inside >= hold, "porosity": 1.0 - vs / (area * z),
            "walls": walls}


def perforate(res, w_bed, r_perf=0.85e-3, r_hole=1.3e-3, grid_n=(12, 12, 6), couple_every=100, n_min=0.3,
              rho_f=998.2, mu_f=1.0e-3):
    """The sand-production workload from a compressed context (compress()): the
    tunnel carved under the hole, the plate with the hole at the compressed
    height, the outlet above it, the fluid grid over the compressed height."""
    st = res["sim"].state()
    x = st["x"]
    alive = st["alive"].astype(bool)
    walls = list(res["walls"])
    zp = res["plate_z"]
    lo = [0.0, 0.0]
    hi = [0.0, 0.0]
    for kind, p in walls[:-1]:
        for ax in (0, 1):
            if kind == dem.DEM_WALL_PLANE and p[ax] > 0.5:
                lo[ax] = p[3]
            elif kind == dem.DEM_WALL_PLANE and p[ax] < -0.5:
                hi[ax] = -p[3]
    cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
    keep = alive & (np.hypot(x[:, 0] - cx, x[:, 1] - cy) >= r_perf)
    walls[-1] = (dem.DEM_WALL_PLANE_HOLE, (cx, cy, zp, -1.0, r_hole))
    grid = ((lo[0], lo[1], 0.0), (hi[0], hi[1], zp), tuple(grid_n))
    ncell = int(np.prod(grid_n))
    out = dict(w_bed)
    out.update(name=w_bed["name"] + "_perforated", x=np.ascontiguousarray(x[keep]),
               r=np.ascontiguousarray(w_bed["r"][keep]), walls=walls, grid=grid,
               u_cell=np.zeros((ncell, 3)), gradp_cell=np.zeros((ncell, 3)),
               fluid=dict(rho_f=rho_f, mu_f=mu_f, n_min=n_min, voidfrac=dem.DEM_VOID_CIC, u_superficial=1,
                          couple_every=couple_every),
               outlet={"above": zp}, hole=(cx, cy, r_hole), normal_model="mod")
    return out
