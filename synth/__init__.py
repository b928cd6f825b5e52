"""Seeded synthetic inputs for the DEM + coupling workloads.

This module is shared by the oracle side and the GPU side and holds none of the
method's arithmetic: particle size samples, geometric packings (pure placement,
see packing.c), prescribed fluid fields, and the workload definitions.

The paper's own workload (a laboratory sand sample from a Kazakhstan reservoir,
its PSD in Table 2, Aspherix runs) is not available; these synthetic inputs stand
in for it.  Sizes, PSD, materials and geometry follow the workload list:

  c0  2 000 spheres, walled 3 mm box, 8^3 fluid grid, uniform upflow, FP64
  c1  200 000 spheres, hollow cylinder R 12 mm / cavity 2 mm / H 6 mm,
      48x48x24 grid, radial Darcy inflow to the cavity, mixed precision
  c2  c1 coarse-grained at k = 2, 3 (SSW and SSP)
  c3  256 boxes, N ~ U{500..20000}, surface energy swept 0.1-1.0 J/m^2
  c4  2 000 000-particle fine-equivalent cylinder at k = 3 (74 074 parcels)
"""
import ctypes
import hashlib
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsynth.so")
CACHE = os.path.join(HERE, "_cache")
SEED0 = 2211061420

# lognormal PSD of the diameters: median 0.15 mm, sigma 0.3, truncated 0.05-0.5 mm
PSD = dict(median=0.15e-3, sigma=0.3, dmin=0.05e-3, dmax=0.5e-3)

MATERIAL = dict(rho=2650.0, E=70e6, nu=0.3, e=0.5, mu=0.5, mu_roll=0.0, gamma=0.5)
WATER = dict(rho_f=998.2, mu_f=1.0e-3)          # Table 4
DT = 1.0e-7
COUPLE_EVERY = 10                                 # CFD step 1e-6 s (section 3.1) / DEM 1e-7 s
N_MIN = 0.3
GRAV = (0.0, 0.0, -9.81)

WALL_PLANE, WALL_CYL_IN, WALL_CYL_OUT, WALL_PLANE_HOLE = 0, 1, 2, 3


def build(force=True):
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                           os.path.join(HERE, "packing.c"), "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.settle_packing.restype = ctypes.c_double
        L.settle_packing.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double]
        L.settle_packing_jacobi.restype = ctypes.c_double
        L.settle_packing_jacobi.argtypes = L.settle_packing.argtypes
        L.settle_packing_colored.restype = ctypes.c_double
        L.settle_packing_colored.argtypes = L.settle_packing.argtypes
        L.deep_overlaps.restype = ctypes.c_int64
        L.deep_overlaps.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_void_p]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# particle sizes
# ---------------------------------------------------------------------------
def sample_diameters(rng, n, psd=PSD):
    """Lognormal diameters truncated to [dmin, dmax] by resampling."""
    out = np.empty(0)
    mu = math.log(psd["median"])
    while out.size < n:
        d = np.exp(rng.normal(mu, psd["sigma"], size=max(2 * (n - out.size), 16)))
        d = d[(d >= psd["dmin"]) & (d <= psd["dmax"])]
        out = np.concatenate([out, d])
    return out[:n].copy()


# ---------------------------------------------------------------------------
# packings
# ---------------------------------------------------------------------------
def settle(r, region_kind, region, rng, phi_start=0.25, shrink=0.998, iters=2000,
           settle_iters=600, relax=1.0, parallel=False, colored=False):
    """Random start in a dilute column, then geometric settling (packing.c).
    region_kind 0: box (x0,y0,z0,x1,y1,z1); 1: annulus (cx,cy,r_in,r_out,z0,z1).
    parallel: the OpenMP Jacobi sweep (deterministic for any thread count);
    colored: the OpenMP Gauss-Seidel sweep over colour classes of spatial
    blocks (deterministic for any thread count); else the serial Gauss-Seidel
    sweep.  The Jacobi sweep is not used: under the same drop schedule it falls
    behind and leaves a tail of deep overlaps (1 % of the contacts above 7 % of
    the smaller radius, against 1.3 % for the serial sweep), which stiff
    materials turn into bursts.  The coloured sweep matches the serial one (the
    c1 inputs: median overlap 0.5 % of the smaller radius in both, 0.006 % of the
    contacts above 7 % against 0.007 %, bed top 2.447 against 2.445 mm) and
    serves the 2 000 000-grain cylinder."""
    n = r.size
    vs = float(np.sum(4.0 / 3.0 * math.pi * r ** 3))
    if region_kind == 0:
        x0, y0, z0, x1, y1, z1 = region
        area = (x1 - x0) * (y1 - y0)
    else:
        cx, cy, rin, rout, z0, z1 = region
        area = math.pi * (rout ** 2 - rin ** 2)
    h_start = vs / (phi_start * area)
    h_bed = vs / (0.6 * area)
    x = np.empty((n, 3))
    if region_kind == 0:
        x[:, 0] = rng.uniform(x0 + r, x1 - r)
        x[:, 1] = rng.uniform(y0 + r, y1 - r)
    else:
        # uniform in the annulus by area
        u = rng.uniform(0.0, 1.0, n)
        rho = np.sqrt(rin ** 2 + u * (rout ** 2 - rin ** 2))
        th = rng.uniform(0.0, 2.0 * math.pi, n)
        rho = np.clip(rho, rin + r, rout - r)
        x[:, 0] = cx + rho * np.cos(th)
        x[:, 1] = cy + rho * np.sin(th)
    x[:, 2] = z0 + r + rng.uniform(0.0, 1.0, n) * h_start
    drop = 2.0 * (h_start - h_bed) / settle_iters
    prm = np.ascontiguousarray(region, dtype=np.float64)
    x = np.ascontiguousarray(x)
    rr = np.ascontiguousarray(r, dtype=np.float64)
    fn = (_L().settle_packing_jacobi if parallel else
          _L().settle_packing_colored if colored else _L().settle_packing)
    worst = fn(n, x.ctypes.data_as(ctypes.c_void_p), rr.ctypes.data_as(ctypes.c_void_p),
                                region_kind, prm.ctypes.data_as(ctypes.c_void_p), shrink, iters,
                                settle_iters, drop, relax)
    return x, worst


def relax(x, r, region_kind, region, sweeps, chunk=100, shrink=0.998, log=None):
    """More overlap-projection sweeps on a settled packing (no further drop),
    by the coloured sweep, in calls of `chunk` sweeps (each starting from a
    fresh pair list); returns the positions and the last sweep's largest
    overlap."""
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    rr = np.ascontiguousarray(r, dtype=np.float64)
    prm = np.ascontiguousarray(region, dtype=np.float64)
    worst = 0.0
    for done in range(0, sweeps, chunk):
        k = min(chunk, sweeps - done)
        worst = _L().settle_packing_colored(len(rr), x.ctypes.data_as(ctypes.c_void_p),
                                            rr.ctypes.data_as(ctypes.c_void_p), region_kind,
                                            prm.ctypes.data_as(ctypes.c_void_p), shrink, k, 0, 0.0, 1.0)
        if log:
            log("relax: %d of %d sweeps, largest overlap %.4f" % (done + k, sweeps, worst))
    return x, worst


def deep_overlap_mask(x, r, thresh):
    """True for the smaller sphere of every pair overlapping by more than
    thresh times the smaller radius"""
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    flags = np.zeros(len(r), np.uint8)
    _L().deep_overlaps(len(r), x.ctypes.data_as(ctypes.c_void_p), r.ctypes.data_as(ctypes.c_void_p), thresh,
                       flags.ctypes.data_as(ctypes.c_void_p))
    return flags.astype(bool)


def _cache_path(name):
    os.makedirs(CACHE, exist_ok=True)
    return os.path.join(CACHE, name + ".npz")


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def cached(name, fn):
    path = _cache_path(name)
    if os.path.exists(path):
        z = np.load(path)
        d = {k: z[k] for k in z.files}
        if "sha256" in d and digest(d["x"], d["r"]) == str(d["sha256"]):
            return d
    d = fn()
    d["sha256"] = np.array(digest(d["x"], d["r"]))
    tmp = path + ".tmp.npz"
    np.savez(tmp, **d)
    os.replace(tmp, path)
    return d


# ---------------------------------------------------------------------------
# fluid fields (prescribed: the CFD solve lies outside the DEM step)
# ---------------------------------------------------------------------------
def grid_centres(grid):
    lo, hi, nn = grid
    axes = [lo[c] + (np.arange(nn[c]) + 0.5) * (hi[c] - lo[c]) / nn[c] for c in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)   # x fastest


def uniform_field(grid, U):
    nc = grid[2][0] * grid[2][1] * grid[2][2]
    u = np.tile(np.asarray(U, dtype=np.float64), (nc, 1))
    gp = np.zeros((nc, 3))
    return u, gp


def radial_darcy_field(grid, r_cav, r_out, U_cav, mu_f, kappa):
    """Steady radial inflow to the cavity: superficial U(rho) = U_cav r_cav / rho
    inward and p(rho) = p_cav + dp ln(rho/r_cav)/ln(R/r_cav) with
    dp = U_cav mu_f r_cav ln(R/r_cav) / kappa (Darcy)."""
    c = grid_centres(grid)
    rho = np.hypot(c[:, 0], c[:, 1])
    lnr = math.log(r_out / r_cav)
    dp = U_cav * mu_f * r_cav * lnr / kappa
    er = np.zeros((rho.size, 3))
    nz = rho > 0
    er[nz, 0] = c[nz, 0] / rho[nz]
    er[nz, 1] = c[nz, 1] / rho[nz]
    mag = np.where(rho >= r_cav, U_cav * r_cav / np.maximum(rho, 1e-30), U_cav * rho / r_cav)
    u = -mag[:, None] * er
    dpdr = np.where(rho >= r_cav, dp / (np.maximum(rho, 1e-30) * lnr), 0.0)
    gp = dpdr[:, None] * er
    return u, gp


def kozeny_carman(d, n):
    return d * d * n ** 3 / (180.0 * (1.0 - n) ** 2)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def box_walls(lo, hi):
    return [(WALL_PLANE, (1.0, 0.0, 0.0, lo[0])), (WALL_PLANE, (-1.0, 0.0, 0.0, -hi[0])),
            (WALL_PLANE, (0.0, 1.0, 0.0, lo[1])), (WALL_PLANE, (0.0, -1.0, 0.0, -hi[1])),
            (WALL_PLANE, (0.0, 0.0, 1.0, lo[2])), (WALL_PLANE, (0.0, 0.0, -1.0, -hi[2]))]


def box_workload(n, side, seed, gamma=0.5, grid_n=8, name=None, U=0.05):
    """A walled cube of the given side with n settled spheres and a uniform
    upward superficial flow."""
    rng = np.random.default_rng(seed)
    name = name or "box_n%d_s%d" % (n, seed)

    def make():
        d = sample_diameters(rng, n)
        r = 0.5 * d
        x, worst = settle(r, 0, (0.0, 0.0, 0.0, side, side, side), rng)
        return {"x": x, "r": r, "worst": np.array(worst)}

    pk = cached(name, make)
    lo, hi = (0.0, 0.0, 0.0), (side, side, side)
    grid = (lo, hi, (grid_n, grid_n, grid_n))
    u, gp = uniform_field(grid, (0.0, 0.0, U))
    mat = dict(MATERIAL)
    mat["gamma"] = gamma
    return dict(name=name, x=pk["x"], r=pk["r"], material=mat, k=1.0, scheme="ssw",
                walls=box_walls(lo, hi), grid=grid, u_cell=u, gradp_cell=gp,
                fluid=dict(WATER, n_min=N_MIN, voidfrac=0, u_superficial=1, couple_every=COUPLE_EVERY),
                outlet=None, dt=DT, g=GRAV, sha256=str(pk["sha256"]))


def c0():
    """2 000 spheres in a walled 3x3x3 mm box, FP64, 1 000 steps."""
    w = box_workload(2000, 3.0e-3, SEED0 + 0, name="c0")
    w.update(precision="fp64", steps=1000, n_fine=2000)
    return w


def cylinder_workload(n, seed, name, k=1.0, scheme="ssw", R=12e-3, r_cav=2e-3, H=6e-3,
                      grid_n=(48, 48, 24), U_cav=0.5, psd_sample_n=None, colored=False, relax_sweeps=0):
    """Hollow cylinder (axis z), outer Hertz wall, floor and a top plate on the
    settled bed; the cavity r < r_cav is the outlet.  k > 1: grains, SSW (each
    sampled fine diameter times k) or SSP (one diameter, k times the mass-mean
    diameter of a fine sample)."""
    rng = np.random.default_rng(seed)

    def make():
        if scheme == "ssp" and k > 1.0:
            dref = sample_diameters(rng, psd_sample_n or 200000)
            dbar = float(np.cbrt(np.mean(dref ** 3)))
            d = np.full(n, k * dbar)
        else:
            d = k * sample_diameters(rng, n)
        r = 0.5 * d
        x, worst = settle(r, 1, (0.0, 0.0, r_cav, R, 0.0, H), rng, colored=colored)
        if relax_sweeps:
            x, worst = relax(x, r, 1, (0.0, 0.0, r_cav, R, 0.0, H), relax_sweeps,
                             log=lambda s: print("%s %s" % (name, s), flush=True))
            # spheres still wedged deep into a neighbour (against a wall, where
            # the confinement undoes the projection) are taken out
            keep = ~deep_overlap_mask(x, r, DEEP_OVERLAP)
            x, r = np.ascontiguousarray(x[keep]), np.ascontiguousarray(r[keep])
        return {"x": x, "r": r, "worst": np.array(worst)}

    pk = cached(name, make)
    x, r = pk["x"], pk["r"]
    top = float(np.max(x[:, 2] + r))
    walls = [(WALL_CYL_IN, (0.0, 0.0, R)), (WALL_PLANE, (0.0, 0.0, 1.0, 0.0)),
             (WALL_PLANE, (0.0, 0.0, -1.0, -top))]
    grid = ((-R, -R, 0.0), (R, R, H), grid_n)
    kappa = kozeny_carman(PSD["median"] * math.exp(0.5 * PSD["sigma"] ** 2), 0.41)
    u, gp = radial_darcy_field(grid, r_cav, R, U_cav, WATER["mu_f"], kappa)
    return dict(name=name, x=x, r=r, material=dict(MATERIAL), k=k, scheme=scheme, walls=walls,
                grid=grid, u_cell=u, gradp_cell=gp,
                fluid=dict(WATER, n_min=N_MIN, voidfrac=0, u_superficial=1, couple_every=COUPLE_EVERY),
                outlet=(0.0, 0.0, r_cav), dt=DT, g=GRAV, sha256=str(pk["sha256"]), bed_top=top)


def c1(n=200000, seed=0):
    """seed 0: the benchmark's packing; seeds 1, 2, ...: other packings of the
    same configuration (held-out runs of the learned closure)"""
    if seed == 0:
        w = cylinder_workload(n, SEED0 + 1, "c1" if n == 200000 else "c1_n%d" % n)
    else:
        w = cylinder_workload(n, SEED0 + 1 + 100 * seed, "c1_n%d_s%d" % (n, seed))
    w.update(precision="mixed", steps=5000, n_fine=n)
    return w


def c2(k=2, scheme="ssw", n_fine=200000, seed=0):
    n = int(round(n_fine / k ** 3))
    if seed == 0:
        w = cylinder_workload(n, SEED0 + 2 + 10 * int(k) + (1 if scheme == "ssp" else 0),
                              "c2_k%d_%s_n%d" % (k, scheme, n_fine), k=float(k), scheme=scheme)
    else:
        w = cylinder_workload(n, SEED0 + 2 + 10 * int(k) + (1 if scheme == "ssp" else 0) + 100 * seed,
                              "c2_k%d_%s_n%d_s%d" % (k, scheme, n_fine, seed), k=float(k), scheme=scheme)
    w.update(precision="mixed", steps=5000, n_fine=n_fine)
    return w


# the 2 000 000-grain column is 10^(1/3) times as tall as c1's, so the drop
# schedule moves it further per sweep and leaves its lower part compressed; this
# many more projection sweeps relax it
C4_RELAX_SWEEPS = 1000
DEEP_OVERLAP = 0.2   # overlap / smaller radius above which the relaxed column drops the smaller sphere


def c4(k=1, scheme="ssw"):
    """Fine-equivalent 2 000 000 grains: the c1 cylinder scaled by 10^(1/3)
    (R 25.85 mm, cavity 4.31 mm, H 12.93 mm) with c1's fluid cell size
    (grid 103 x 103 x 52); k > 1: the coarse-grained model (k = 3: 74 074
    parcels).  Packed by the coloured parallel sweep."""
    s = 10.0 ** (1.0 / 3.0)
    n_fine = 2000000
    n = int(round(n_fine / k ** 3))
    w = cylinder_workload(n, SEED0 + 4 + 10 * int(k) + (1 if scheme == "ssp" else 0),
                          "c4_k%d_%s_colr" % (k, scheme), k=float(k), scheme=scheme, R=12e-3 * s, r_cav=2e-3 * s,
                          H=6e-3 * s, grid_n=(103, 103, 52), colored=True, relax_sweeps=C4_RELAX_SWEEPS)
    w.update(precision="mixed", steps=5000, n_fine=n_fine)
    return w


def c3_sizes(n_samples=256, seed=SEED0 + 3):
    rng = np.random.default_rng(seed)
    ns = rng.integers(500, 20001, size=n_samples)
    gam = 0.1 + 0.9 * np.arange(n_samples) / max(n_samples - 1, 1)
    return ns, gam


def c3_sample(s, n_s, gamma):
    side = 3.0e-3 * (n_s / 2000.0) ** (1.0 / 3.0)
    gn = int(min(16, max(8, round(8 * (n_s / 2000.0) ** (1.0 / 3.0)))))
    w = box_workload(int(n_s), side, SEED0 + 1000 + s, gamma=gamma, grid_n=gn,
                     name="c3_s%d_n%d" % (s, n_s))
    w.update(precision="mixed", steps=2000, n_fine=int(n_s))
    return w


def c3_crop(s, n_s, gamma, base=None):
    """Ensemble sample s: the spheres of the settled C1 bed (annulus 2-12 mm) whose centres lie in
    an axis-aligned box of the bed's height (0.05 mm to 2.4 mm) and a square
    footprint holding about n_s of them, centred at radius 7 mm and angle
    2 pi s / 37 in the annulus; shifted to the origin, with six walls one
    largest radius outside the box (no initial wall overlap), a grid of 8-16
    cells per side and a uniform upward flow.  Dense, settled and cheap: no
    packing run per sample.  A coarse-grained base (c2) gives a sample of its
    parcels, with the base's k and scheme."""
    base = base if base is not None else c1()
    x, r = base["x"], base["r"]
    z0, z1 = 0.05e-3, 2.4e-3
    dens = len(r) / (math.pi * (12e-3 ** 2 - 2e-3 ** 2) * base["bed_top"])   # C1 annulus
    a = math.sqrt(n_s / (dens * (z1 - z0)))
    th = 2.0 * math.pi * s / 37.0
    cx, cy = 7.0e-3 * math.cos(th), 7.0e-3 * math.sin(th)
    lo = np.array([cx - a / 2, cy - a / 2, z0])
    hi = np.array([cx + a / 2, cy + a / 2, z1])
    sel = np.all((x >= lo) & (x < hi), axis=1)
    xs, rs = x[sel] - lo, r[sel].copy()
    pad = rs.max()
    wlo, whi = -pad * np.ones(3), (hi - lo) + pad
    gn = int(min(16, max(8, round(8 * (len(rs) / 2000.0) ** (1.0 / 3.0)))))
    grid = (tuple(wlo), tuple(whi), (gn, gn, gn))
    u, gp = uniform_field(grid, (0.0, 0.0, 0.02))
    mat = dict(MATERIAL)
    mat["gamma"] = gamma
    k = float(base.get("k", 1.0))
    return dict(name="c3_s%d_n%d_k%g" % (s, n_s, k), x=xs, r=rs, material=mat, k=k,
                scheme=base.get("scheme", "ssw"),
                walls=box_walls(tuple(wlo), tuple(whi)), grid=grid, u_cell=u, gradp_cell=gp,
                fluid=dict(WATER, n_min=N_MIN, voidfrac=0, u_superficial=1, couple_every=COUPLE_EVERY),
                outlet=None, dt=DT, g=GRAV, sha256=base["sha256"], precision="mixed", steps=2000,
                n_fine=int(round(len(rs) * k ** 3)))


def c3(n_samples=256, seed=SEED0 + 3, k_sweep=False):
    """The batched ensemble: n_samples crops with sizes 500-20 000 and surface
    energies 0.1-1.0 J/m^2 (c3_sizes).  k_sweep: sample s is coarse-grained
    with k = 1 + (s mod 3), a crop of the k-scaled bed (c1, c2(2), c2(3))
    holding the sample's size in fine-equivalent grains (size / k^3 parcels, at
    least 60)."""
    ns, gam = c3_sizes(n_samples, seed)
    if not k_sweep:
        base = c1()
        return [c3_crop(s, int(ns[s]), float(gam[s]), base) for s in range(n_samples)]
    bases = {1: c1(), 2: c2(2), 3: c2(3)}
    out = []
    for s in range(n_samples):
        k = 1 + s % 3
        out.append(c3_crop(s, max(60, int(round(ns[s] / k ** 3))), float(gam[s]), bases[k]))
    return out


# The paper's own setting (section 3.1): Table 2, mass fraction of each of the
# eight diameters (mm) of the original particles; Table 3, the sand's material
# (fine scale); the time step and the coupling interval of that run.
TABLE2 = [(0.058, 0.15), (0.075, 0.18), (0.088, 0.20), (0.1216, 0.22), (0.2264, 0.25), (0.1705, 0.275),
          (0.121, 0.30), (0.1395, 0.355)]
PAPER_MATERIAL = dict(rho=2605.0, E=2.0e10, nu=0.3, e=0.8, mu=0.2, mu_roll=0.0, gamma=30.0)
PAPER_DT = 1.0e-8
PAPER_COUPLE_EVERY = 100                            # CFD step 1e-6 s / DEM 1e-8 s


def table2_diameters(rng, n):
    """n diameters from the eight classes of Table 2, drawn with probabilities
    in proportion to mass fraction / d^3 (the number fraction of each class)."""
    w = np.array([m for m, _ in TABLE2])
    d = np.array([dd for _, dd in TABLE2]) * 1e-3
    p = w / d ** 3
    return d[rng.choice(d.size, size=n, p=p / p.sum())]


def table2_mean_diameter():
    """the mass-equivalent mean diameter of Table 2, (sum w / sum w / d^3)^(1/3)"""
    w = np.array([m for m, _ in TABLE2])
    d = np.array([dd for _, dd in TABLE2]) * 1e-3
    return float(np.cbrt(w.sum() / np.sum(w / d ** 3)))


F2_SIDE, F2_HEIGHT = 18e-3, 9e-3                 # the box of section 3.1 after compression
F2_R_PERF, F2_R_HOLE = 0.85e-3, 1.3e-3             # perforation tunnel, outlet hole (radii)


def _f2_settle(k, scheme, n_fine, seed):
    """the geometric packing of the paper's box: Table 2 sand settled in the
    18 x 18 mm box (positions, radii, worst overlap)"""
    L, H = F2_SIDE, F2_HEIGHT
    n = int(round(n_fine / k ** 3))
    rng = np.random.default_rng(SEED0 + 5 + 10 * int(k) + (1 if scheme == "ssp" else 0) + 100 * seed)
    if scheme == "ssp" and k > 1:
        d = np.full(n, k * table2_mean_diameter())
    else:
        d = k * table2_diameters(rng, n)
    r = 0.5 * d
    x, worst = settle(r, 0, (0.0, 0.0, 0.0, L, L, 3.0 * H), rng)
    return x, r, worst


def f2_bed(k=1, scheme="ssw", n_fine=250000, seed=0):
    """The paper's box before compression (section 3.1, generation stage):
    every grain of the geometric packing of f2 (nothing cut, no tunnel), five
    plane walls and a top plate one largest radius above the bed, no outlet,
    no fluid, the original JKR law of the generation stage (normal_model
    "orig"), Table 3 material, dt 1e-8 s.  paper_setting.compress moves the plate
    down to the overburden stress."""
    L = F2_SIDE
    name = "f2bed_k%d_%s_n%d_s%d" % (k, scheme, n_fine, seed)

    def make():
        x, r, worst = _f2_settle(k, scheme, n_fine, seed)
        return {"x": x, "r": r, "worst": np.array(worst)}

    pk = cached(name, make)
    x, r = pk["x"], pk["r"]
    top = float(np.max(x[:, 2] + r)) + float(r.max())
    walls = [(WALL_PLANE, (1.0, 0.0, 0.0, 0.0)), (WALL_PLANE, (-1.0, 0.0, 0.0, -L)),
             (WALL_PLANE, (0.0, 1.0, 0.0, 0.0)), (WALL_PLANE, (0.0, -1.0, 0.0, -L)),
             (WALL_PLANE, (0.0, 0.0, 1.0, 0.0)), (WALL_PLANE, (0.0, 0.0, -1.0, -top))]
    return dict(name=name, x=x, r=r, material=dict(PAPER_MATERIAL), k=float(k), scheme=scheme, walls=walls,
                grid=None, u_cell=None, gradp_cell=None, fluid=None, outlet=None, dt=PAPER_DT, g=GRAV,
                sha256=str(pk["sha256"]), precision="mixed", n_fine=n_fine, normal_model="orig")


def f2(k=1, scheme="ssw", n_fine=250000, seed=0):
    """The paper's own setting (section 3.1) after its perforation stage: an
    18 x 18 mm box of height 9 mm, sand of Table 2 (k = 1: n_fine grains; k > 1:
    SSW parcels k times each sampled diameter, or SSP parcels of k times the
    mean diameter, n_fine / k^3 of them) and Table 3, dt 1e-8 s, a 12 x 12 x 6
    grid of 1.5 mm cells, a top plate with the 2.6 mm outlet hole over the
    centre (outlet: centres above the plate's level), and the perforation, a
    vertical tunnel of 1.7 mm diameter through the whole height under the
    hole.  Stand-ins for the paper's stages: the grains are settled
    geometrically (no generation with the original JKR law, no 1 MPa
    compression, so the porosity is that of the geometric packing, not 41 %),
    and the tunnel is carved (the grains whose centres lie within it are
    removed) instead of pushed open by the penetrometer.  The fluid fields
    start at rest; the run's own pressure solve (model A, dem_fluid_solve with
    f2_cell_kinds) gives them."""
    L, H = F2_SIDE, F2_HEIGHT
    cx = cy = 0.5 * L
    r_perf, r_hole = F2_R_PERF, F2_R_HOLE
    name = "f2_k%d_%s_n%d_s%d" % (k, scheme, n_fine, seed)

    def make():
        x, r, worst = _f2_settle(k, scheme, n_fine, seed)
        keep = (x[:, 2] + r <= H) & (np.hypot(x[:, 0] - cx, x[:, 1] - cy) >= r_perf)
        return {"x": x[keep], "r": r[keep], "worst": np.array(worst)}

    pk = cached(name, make)
    walls = [(WALL_PLANE, (1.0, 0.0, 0.0, 0.0)), (WALL_PLANE, (-1.0, 0.0, 0.0, -L)),
             (WALL_PLANE, (0.0, 1.0, 0.0, 0.0)), (WALL_PLANE, (0.0, -1.0, 0.0, -L)),
             (WALL_PLANE, (0.0, 0.0, 1.0, 0.0)), (WALL_PLANE_HOLE, (cx, cy, H, -1.0, r_hole))]
    grid = ((0.0, 0.0, 0.0), (L, L, H), (12, 12, 6))
    ncell = 12 * 12 * 6
    mat = dict(PAPER_MATERIAL)
    return dict(name=name, x=pk["x"], r=pk["r"], material=mat, k=float(k), scheme=scheme, walls=walls,
                grid=grid, u_cell=np.zeros((ncell, 3)), gradp_cell=np.zeros((ncell, 3)),
                fluid=dict(WATER, n_min=N_MIN, voidfrac=0, u_superficial=1, couple_every=PAPER_COUPLE_EVERY),
                outlet={"above": H}, dt=PAPER_DT, g=GRAV, sha256=str(pk["sha256"]), precision="mixed",
                n_fine=n_fine, hole=(cx, cy, r_hole), steps=4000000)


def f2_cell_kinds(w, p_in=1.0):
    """Boundary conditions of the paper's fluid run (section 3.1) as cell kinds
    of the pressure solve: the layers of cells next to the two faces normal to
    y take the injection pressure p_in, the cells under the top and over the
    bottom hole (centres within the hole radius of the axis) are outlets at the
    reference pressure (dynamic pressure 0); every other cell is open and the
    remaining faces carry no flow.  Returns (kind, p_fixed)."""
    (lo, hi, nn) = w["grid"]
    nx, ny, nz = nn
    h = [(hi[c] - lo[c]) / nn[c] for c in range(3)]
    cx, cy, rh = w["hole"]
    kind = np.zeros(nx * ny * nz, np.int8)
    p = np.zeros(nx * ny * nz)
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                c = (iz * ny + iy) * nx + ix
                xc, yc = lo[0] + (ix + 0.5) * h[0], lo[1] + (iy + 0.5) * h[1]
                if (iz == 0 or iz == nz - 1) and math.hypot(xc - cx, yc - cy) < rh:
                    kind[c] = 1
                elif iy == 0 or iy == ny - 1:
                    kind[c], p[c] = 1, p_in
    return kind, p


def hole_box(v_up=2.0, r_hole=0.6e-3, depth=0.25e-3, precision="fp64"):
    """c0's settled spheres under a top plate with a hole over the centre
    (PLANE_HOLE a depth below the bed top) and the outlet at the plate's level,
    without cohesion: the spheres that would cut the plate outside the hole are
    left out, the column under the hole stands above the plate's level (its
    centres above it leave at the first step) and starts upwards at v_up, so
    spheres keep crossing the level and leaving while their neighbours are
    pushed against the plate (the parity runs of the paper's top outlet)."""
    base = c0()
    x, r = base["x"], base["r"]
    side = 3.0e-3
    cx = cy = 0.5 * side
    zp = float(np.max(x[:, 2] + r)) - depth
    under = np.hypot(x[:, 0] - cx, x[:, 1] - cy) < r_hole
    keep = (x[:, 2] + r <= zp) | under
    x, r, under = x[keep], r[keep], under[keep]
    walls = [wl for wl in base["walls"] if not (wl[0] == WALL_PLANE and wl[1][2] < 0.0)]
    walls.append((WALL_PLANE_HOLE, (cx, cy, zp, -1.0, r_hole)))
    mat = dict(MATERIAL)
    mat["gamma"] = 0.0
    v = np.zeros_like(x)
    v[under, 2] = v_up
    return dict(base, name="hole_box", x=x, r=r, material=mat, walls=walls, outlet={"above": zp}, v=v,
                precision=precision, hole=(cx, cy, r_hole))


def c1_ring(r_crop=2.8e-3, U_cav=2.0, outlet_shift=0.06e-3, v_in=0.3, precision="fp64"):
    """A ring of the settled c1 bed next to the cavity, for parity runs in which
    spheres leave: the spheres whose centres lie within r_crop of the axis (about
    5 500), an outer cylinder wall one largest radius beyond them, c1's floor and
    top plate, c1's grid with the radial inflow at U_cav, the outlet radius moved
    out by outlet_shift (so that the innermost spheres sit just outside it), and an
    inward radial start velocity v_in (returned as "v")."""
    base = c1()
    x, r = base["x"], base["r"]
    rho = np.hypot(x[:, 0], x[:, 1])
    sel = rho < r_crop
    xs, rs = x[sel].copy(), r[sel].copy()
    R = r_crop + rs.max()
    walls = [(WALL_CYL_IN, (0.0, 0.0, R))] + [wl for wl in base["walls"] if wl[0] == WALL_PLANE]
    grid = base["grid"]
    r_cav = 2e-3
    kappa = kozeny_carman(PSD["median"] * math.exp(0.5 * PSD["sigma"] ** 2), 0.41)
    u, gp = radial_darcy_field(grid, r_cav, 12e-3, U_cav, WATER["mu_f"], kappa)
    rr = np.hypot(xs[:, 0], xs[:, 1])
    v = np.zeros_like(xs)
    v[:, 0] = -v_in * xs[:, 0] / rr
    v[:, 1] = -v_in * xs[:, 1] / rr
    return dict(name="c1_ring", x=xs, r=rs, v=v, material=dict(MATERIAL), k=1.0, scheme="ssw", walls=walls,
                grid=grid, u_cell=u, gradp_cell=gp,
                fluid=dict(WATER, n_min=N_MIN, voidfrac=0, u_superficial=1, couple_every=COUPLE_EVERY),
                outlet=(0.0, 0.0, r_cav + outlet_shift), dt=DT, g=GRAV, sha256=base["sha256"],
                precision=precision, n_fine=len(rs), bed_top=base["bed_top"])
