"""FP64 CPU oracle of the coarse-grained CFD-DEM step (arXiv:2211.06142).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2211_06142_amd/``: the C part (dem_oracle.c) is
compiled by gcc on its own, and the Python parts (coarse-graining, MLP) are plain
numpy written from the paper.

Contents
  dem_oracle.c  single-contact laws (section 2.3), Di Felice drag (section 2.2),
                brute-force and plain-grid contact sets, the full step
  cg.py         coarse-graining transform (section 2.4, eq 14-35, Table 3)
  mlp.py        FP64 forward/backward of the learned closure network
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "dem_oracle.c")

MAX_WALLS = 8
WALL_PLANE, WALL_CYL_IN, WALL_CYL_OUT, WALL_PLANE_HOLE = 0, 1, 2, 3
NORMAL_JKR_MOD, NORMAL_HERTZ, NORMAL_LINEAR, NORMAL_JKR_ORIG = 0, 1, 2, 3
VOID_CIC, VOID_CENTROID = 0, 1
OUTLET_NONE, OUTLET_CAVITY, OUTLET_ABOVE = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrWall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_double * 6)]


class OrGrid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("n", ctypes.c_int * 3)]


class OrParams(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_double), ("E", ctypes.c_double), ("nu", ctypes.c_double),
        ("e", ctypes.c_double), ("mu", ctypes.c_double), ("mu_roll", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("k_cg", ctypes.c_double), ("k_lin", ctypes.c_double), ("normal_model", ctypes.c_int),
        ("fluid_on", ctypes.c_int), ("rho_f", ctypes.c_double), ("mu_f", ctypes.c_double),
        ("n_min", ctypes.c_double), ("voidfrac", ctypes.c_int), ("u_superficial", ctypes.c_int),
        ("couple_every", ctypes.c_int), ("grid", OrGrid),
        ("g", ctypes.c_double * 3), ("dt", ctypes.c_double),
        ("outlet_kind", ctypes.c_int), ("outlet", ctypes.c_double * 4),
        ("n_walls", ctypes.c_int), ("walls", OrWall * MAX_WALLS),
        ("use_grid_search", ctypes.c_int),
    ]


_lib = None
_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d, i64, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        L.or_jkr_delta_of_a.restype = d
        L.or_jkr_delta_of_a.argtypes = [d, d, d, d]
        L.or_jkr_force_of_a.restype = d
        L.or_jkr_force_of_a.argtypes = [d, d, d, d]
        L.or_jkr_a_of_delta.restype = d
        L.or_jkr_a_of_delta.argtypes = [d, d, d, d]
        L.or_bond_holds.restype = ctypes.c_int
        L.or_bond_holds.argtypes = [d, d, d, d, d]
        L.or_contact_holds_to_S.restype = ctypes.c_int
        L.or_contact_holds_to_S.argtypes = [d, d, d, d, d]
        L.or_beta_of_e.restype = d
        L.or_beta_of_e.argtypes = [d]
        L.or_drag.restype = None
        L.or_drag.argtypes = [vp, d, d, d, d, d, d, vp]
        L.or_pairs_brute.restype = i64
        L.or_pairs_brute.argtypes = [i64, vp, vp, vp, d, i64, vp, vp]
        L.or_pairs_grid.restype = i64
        L.or_pairs_grid.argtypes = [i64, vp, vp, vp, d, i64, vp, vp]
        L.or_create.restype = vp
        L.or_create.argtypes = [ctypes.POINTER(OrParams), i64, vp, vp, vp, vp, vp, vp, vp,
                                i64, vp, vp, vp, vp, ctypes.c_int, vp]
        L.or_destroy.restype = None
        L.or_destroy.argtypes = [vp]
        L.or_set_fluid.restype = ctypes.c_int
        L.or_set_fluid.argtypes = [vp, vp, vp]
        L.or_set_held.restype = ctypes.c_int
        L.or_set_held.argtypes = [vp, i64, vp]
        L.or_set_closure.restype = ctypes.c_int
        L.or_set_closure.argtypes = [vp, vp, vp]
        L.or_set_closure_mlp.restype = ctypes.c_int
        L.or_set_closure_mlp.argtypes = [vp, vp, vp]
        L.or_closure_features.restype = ctypes.c_int
        L.or_closure_features.argtypes = [vp, vp]
        L.or_mlp_forward.restype = None
        L.or_mlp_forward.argtypes = [vp, vp, vp]
        L.or_get_closure.restype = None
        L.or_get_closure.argtypes = [vp, vp, vp]
        L.or_get_closure_features.restype = None
        L.or_get_closure_features.argtypes = [vp, vp]
        L.or_step.restype = ctypes.c_int
        L.or_step.argtypes = [vp, i64]
        L.or_get_state.restype = None
        L.or_get_state.argtypes = [vp] + [vp] * 8
        L.or_get_scalars.restype = None
        L.or_get_scalars.argtypes = [vp, vp, vp, vp, vp, vp]
        L.or_get_pairs.restype = i64
        L.or_get_pairs.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.or_get_wall_dt.restype = None
        L.or_get_wall_dt.argtypes = [vp, vp]
        L.or_get_wall_forces.restype = None
        L.or_get_wall_forces.argtypes = [vp, vp]
        L.or_set_walls.restype = ctypes.c_int
        L.or_set_walls.argtypes = [vp, ctypes.c_int, vp]
        L.or_get_fluid.restype = None
        L.or_get_fluid.argtypes = [vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------------------
# single-contact laws
# ---------------------------------------------------------------------------
def jkr_delta_of_a(a, Rs, Es, gamma):
    return lib().or_jkr_delta_of_a(a, Rs, Es, gamma)


def jkr_force_of_a(a, Rs, Es, gamma):
    return lib().or_jkr_force_of_a(a, Rs, Es, gamma)


def jkr_a_of_delta(delta, Rs, Es, gamma):
    return lib().or_jkr_a_of_delta(delta, Rs, Es, gamma)


def bond_holds(d2, c, Rs, Es, gamma):
    return bool(lib().or_bond_holds(d2, c, Rs, Es, gamma))


def contact_holds_to_S(d2, c, Rs, Es, gamma):
    return bool(lib().or_contact_holds_to_S(d2, c, Rs, Es, gamma))


def beta_of_e(e):
    return lib().or_beta_of_e(e)


def mlp_forward(params, xh):
    """the C oracle's forward pass of the closure network, one row at a time"""
    pp = _f64(params, (8898,))
    xs = np.ascontiguousarray(np.asarray(xh, np.float64).reshape(-1, 6))
    y = np.zeros((xs.shape[0], 2))
    for k in range(xs.shape[0]):
        row, out = np.ascontiguousarray(xs[k]), np.zeros(2)
        lib().or_mlp_forward(_ptr(pp), _ptr(row), _ptr(out))
        y[k] = out
    return y


def drag(slip, d, k_cg, n, rho_f, mu_f, c_drag=1.0):
    s = _f64(slip, (3,))
    out = np.zeros(3)
    lib().or_drag(_ptr(s), d, k_cg, n, rho_f, mu_f, c_drag, _ptr(out))
    return out


def effective_moduli(E, nu):
    """E* and G* of two identical materials (section 2.3 definition of E*)."""
    Es = E / (2.0 * (1.0 - nu * nu))
    Gs = E / (4.0 * (2.0 - nu) * (1.0 + nu))
    return Es, Gs


# ---------------------------------------------------------------------------
# contact sets
# ---------------------------------------------------------------------------
def pairs(x, r, alive=None, extra=0.0, method="grid"):
    x = _f64(x, (-1, 3))
    r = _f64(r)
    n = r.shape[0]
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    f = lib().or_pairs_grid if method == "grid" else lib().or_pairs_brute
    cnt = f(n, _ptr(x), _ptr(r), _ptr(al), float(extra), 0, None, None)
    pi = np.zeros(max(cnt, 1), np.int64)
    pj = np.zeros(max(cnt, 1), np.int64)
    f(n, _ptr(x), _ptr(r), _ptr(al), float(extra), cnt, _ptr(pi), _ptr(pj))
    return np.stack([pi[:cnt], pj[:cnt]], axis=1)


# ---------------------------------------------------------------------------
# simulation
# ---------------------------------------------------------------------------
def make_params(mat, dt, g=(0.0, 0.0, -9.81), walls=(), grid=None, fluid=None, outlet=None,
                normal_model=NORMAL_JKR_MOD, k_lin=0.0, use_grid_search=True):
    """Build OrParams from GRAIN-scale material (see oracle.cg for the scaling).

    mat: dict rho, E, nu, e, mu, mu_roll, gamma, k_cg
    walls: sequence of (kind, params[<=6])
    grid: (lo[3], hi[3], n[3]) or None
    fluid: dict rho_f, mu_f, n_min, voidfrac, u_superficial, couple_every or None
    outlet: (x, y, radius) cavity, {"above": z} (centres above z leave) or None
    """
    p = OrParams()
    p.rho, p.E, p.nu, p.e = mat["rho"], mat["E"], mat["nu"], mat["e"]
    p.mu, p.mu_roll, p.gamma = mat["mu"], mat.get("mu_roll", 0.0), mat["gamma"]
    p.k_cg = mat.get("k_cg", 1.0)
    p.k_lin = k_lin
    p.normal_model = normal_model
    p.dt = dt
    for c in range(3):
        p.g[c] = g[c]
    p.n_walls = len(walls)
    for k, (kind, prm) in enumerate(walls):
        p.walls[k].kind = kind
        for q, val in enumerate(prm):
            p.walls[k].p[q] = val
    if grid is not None:
        lo, hi, nn = grid
        for c in range(3):
            p.grid.lo[c], p.grid.hi[c], p.grid.n[c] = lo[c], hi[c], nn[c]
    else:
        for c in range(3):
            p.grid.lo[c], p.grid.hi[c], p.grid.n[c] = 0.0, 1.0, 1
    if fluid is not None:
        p.fluid_on = 1
        p.rho_f, p.mu_f = fluid["rho_f"], fluid["mu_f"]
        p.n_min = fluid.get("n_min", 0.3)
        p.voidfrac = fluid.get("voidfrac", VOID_CIC)
        p.u_superficial = fluid.get("u_superficial", 1)
        p.couple_every = fluid.get("couple_every", 1)
    else:
        p.fluid_on = 0
        p.couple_every = 1
    if isinstance(outlet, dict):
        p.outlet_kind = OUTLET_ABOVE
        p.outlet[3] = outlet["above"]
    elif outlet is not None:
        p.outlet_kind = OUTLET_CAVITY
        for c in range(3):
            p.outlet[c] = outlet[c]
    p.use_grid_search = 1 if use_grid_search else 0
    return p


class OracleSim:
    """One oracle system.  State lives in C; arrays cross as float64 copies."""

    def __init__(self, params, x, r, v=None, w=None, F=None, T=None, alive=None,
                 pairs=None, pair_dt=None, pair_bonded=None, bond_at_init=True, wall_dt=None):
        L = lib()
        self.params = params
        x = _f64(x, (-1, 3))
        self.n = n = x.shape[0]
        z = np.zeros((n, 3))
        self._keep = []
        arrs = [x, _f64(v if v is not None else z, (-1, 3)), _f64(w if w is not None else z, (-1, 3)),
                _f64(F if F is not None else z, (-1, 3)), _f64(T if T is not None else z, (-1, 3)),
                _f64(r)]
        al = np.ascontiguousarray(alive if alive is not None else np.ones(n), dtype=np.uint8)
        npairs = 0
        pi = pj = pdt = pb = None
        if pairs is not None and len(pairs) > 0:
            pp = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
            npairs = pp.shape[0]
            pi = np.ascontiguousarray(pp[:, 0])
            pj = np.ascontiguousarray(pp[:, 1])
            pdt = _f64(pair_dt if pair_dt is not None else np.zeros((npairs, 3)), (-1, 3))
            pb = np.ascontiguousarray(pair_bonded if pair_bonded is not None else np.zeros(npairs),
                                      dtype=np.uint8)
        wd = None if wall_dt is None else _f64(wall_dt)
        self.h = L.or_create(ctypes.byref(params), n, *[_ptr(a) for a in arrs], _ptr(al),
                             npairs, _ptr(pi), _ptr(pj), _ptr(pdt), _ptr(pb),
                             1 if bond_at_init else 0, _ptr(wd))

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    def set_fluid(self, u_cell, gradp_cell):
        u = _f64(u_cell)
        gp = _f64(gradp_cell)
        lib().or_set_fluid(self.h, _ptr(u), _ptr(gp))

    def set_held(self, step, fluid_force=None):
        """Resume at absolute step `step` (the coupling schedule) with the fluid
        force (n x 3, drag plus buoyancy) held since the last coupling evaluation."""
        ff = None if fluid_force is None else _f64(fluid_force, (-1, 3))
        lib().or_set_held(self.h, int(step), _ptr(ff))

    def set_closure(self, c_drag=None, c_coh=None):
        cd = None if c_drag is None else _f64(c_drag)
        cc = None if c_coh is None else _f64(c_coh)
        lib().or_set_closure(self.h, _ptr(cd), _ptr(cc))

    def set_closure_mlp(self, params=None, norm=None):
        """Learned closure: FP64 parameters (8898) and norm = (mean[6], sd[6]);
        params None switches it off."""
        if params is None:
            lib().or_set_closure_mlp(self.h, None, None)
            return
        pp = _f64(params, (8898,))
        nn = _f64(norm, (12,))
        lib().or_set_closure_mlp(self.h, _ptr(pp), _ptr(nn))

    def closure_features(self):
        f = np.zeros((self.n, 6))
        lib().or_closure_features(self.h, _ptr(f))
        return f

    def closure_last_features(self):
        """features of the latest coupling evaluation that ran the closure"""
        f = np.zeros((self.n, 6))
        lib().or_get_closure_features(self.h, _ptr(f))
        return f

    def closure_factors(self):
        """(c_drag, c_coh) of the last coupling evaluation (ones when unset)"""
        cd, cc = np.zeros(self.n), np.zeros(self.n)
        lib().or_get_closure(self.h, _ptr(cd), _ptr(cc))
        return cd, cc

    def step(self, nsteps=1):
        rc = lib().or_step(self.h, int(nsteps))
        if rc != 0:
            raise RuntimeError("oracle step failed (fluid fields not set?)")

    def state(self):
        n = self.n
        out = {k: np.zeros((n, 3)) for k in ("x", "v", "w", "F", "T")}
        alive = np.zeros(n, np.uint8)
        fs = np.zeros(n)
        ts = np.zeros(n)
        lib().or_get_state(self.h, *[_ptr(out[k]) for k in ("x", "v", "w", "F", "T")], _ptr(alive),
                           _ptr(fs), _ptr(ts))
        out["alive"] = alive
        out["fscale"] = fs
        out["tscale"] = ts
        return out

    def scalars(self):
        pm = ctypes.c_double()
        bb = ctypes.c_int64()
        st = ctypes.c_int64()
        nc = ctypes.c_int64()
        ke = ctypes.c_double()
        lib().or_get_scalars(self.h, ctypes.byref(pm), ctypes.byref(bb), ctypes.byref(st),
                             ctypes.byref(nc), ctypes.byref(ke))
        return {"produced_mass": pm.value, "broken_bonds": bb.value, "step": st.value,
                "n_contacts": nc.value, "kinetic": ke.value}

    def pairs(self):
        L = lib()
        cnt = L.or_get_pairs(self.h, 0, None, None, None, None, None)
        pi = np.zeros(max(cnt, 1), np.int64)
        pj = np.zeros(max(cnt, 1), np.int64)
        pdt = np.zeros((max(cnt, 1), 3))
        pb = np.zeros(max(cnt, 1), np.uint8)
        pt = np.zeros(max(cnt, 1), np.uint8)
        L.or_get_pairs(self.h, cnt, _ptr(pi), _ptr(pj), _ptr(pdt), _ptr(pb), _ptr(pt))
        return {"pairs": np.stack([pi[:cnt], pj[:cnt]], 1), "dt": pdt[:cnt], "bonded": pb[:cnt],
                "touch": pt[:cnt]}

    def wall_forces(self):
        """(MAX_WALLS, 3): the particles' total force on each wall at the last evaluation"""
        out = np.zeros((MAX_WALLS, 3))
        lib().or_get_wall_forces(self.h, _ptr(out))
        return out

    def set_walls(self, walls):
        """replace the walls, [(kind, params), ...] with the same count"""
        arr = (OrWall * MAX_WALLS)()
        for k, (kind, prm) in enumerate(walls):
            arr[k].kind = kind
            for q, val in enumerate(prm):
                arr[k].p[q] = val
        if lib().or_set_walls(self.h, len(walls), ctypes.cast(arr, ctypes.c_void_p)) != 0:
            raise ValueError("set_walls: the wall count must stay the same")
        for k in range(len(walls)):
            self.params.walls[k] = arr[k]

    def wall_dt(self):
        nw = self.params.n_walls
        out = np.zeros((self.n, max(nw, 0), 3))
        if nw > 0:
            lib().or_get_wall_dt(self.h, _ptr(out))
        return out

    def fluid(self):
        g = self.params.grid
        nc = g.n[0] * g.n[1] * g.n[2]
        eps = np.zeros(nc)
        fd = np.zeros((nc, 3))
        fp = np.zeros((self.n, 3))
        fb = np.zeros((self.n, 3))
        lib().or_get_fluid(self.h, _ptr(eps), _ptr(fd), _ptr(fp), _ptr(fb))
        return {"eps_s": eps, "fdrag_cell": fd, "f_part": fp, "fb_part": fb}
