"""ctypes binding of include/dem.h (argument marshalling only).

Every name below mirrors the C ABI one for one; all stepping, coupling and
reduction work runs in the HIP kernels of libdem.so.  PyTorch provides device
memory and the HIP stream.  There is no fallback: if libdem.so is missing or
no GPU is present the calls raise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdem.so")

DEM_OK, DEM_E_INVAL, DEM_E_NOMEM, DEM_E_CAPACITY, DEM_E_NONFINITE, DEM_E_DEVICE, DEM_E_STATE = 0, -1, -2, -3, -4, -5, -6
DEM_MAX_WALLS = 8
DEM_WALL_PLANE, DEM_WALL_CYL_IN, DEM_WALL_CYL_OUT, DEM_WALL_PLANE_HOLE = 0, 1, 2, 3
DEM_NORMAL_JKR_MOD, DEM_NORMAL_HERTZ, DEM_NORMAL_LINEAR, DEM_NORMAL_JKR_ORIG = 0, 1, 2, 3
DEM_VOID_CIC, DEM_VOID_CENTROID = 0, 1
DEM_OUTLET_NONE, DEM_OUTLET_CAVITY, DEM_OUTLET_ABOVE = 0, 1, 2
DEM_PREC_FP64, DEM_PREC_MIXED = 0, 1
DEM_CG_SSW, DEM_CG_SSP = 0, 1
DEM_FLAG_AUTO_REGROW = 1
DEM_MAX_SIZE_CLASSES = 16

DEM_PAIRS_FULL_ROWS, DEM_PAIRS_HALF = 0, 1
DEM_CELL_OPEN, DEM_CELL_PRESSURE, DEM_CELL_SOLID = 0, 1, 2
DEM_PROF_PROLOGUE, DEM_PROF_REBUILD, DEM_PROF_FLUID, DEM_PROF_STEP, DEM_PROF_N = 0, 1, 2, 3, 4
PROF_NAMES = ["prologue", "rebuild", "fluid", "step"]

EXPORTS = sorted(["dem_init", "dem_step", "dem_map_fluid", "dem_read_state", "dem_read_pairs",
                  "dem_read_wall_forces", "dem_set_walls",
                  "dem_read_aggregates", "dem_info", "dem_request_rebuild", "dem_destroy", "dem_status_str",
                  "dem_cg_material", "dem_cg_diameters", "dem_rayleigh_dt", "dem_profile", "dem_read_profile",
                  "dem_read_fault", "dem_mlp_create", "dem_mlp_destroy", "dem_mlp_set_params", "dem_mlp_get_params",
                  "dem_mlp_forward", "dem_mlp_grad", "dem_mlp_train_step", "dem_set_closure", "dem_read_closure", "dem_set_graphs", "dem_set_lanes",
                  "dem_set_size_classes", "dem_read_produced_classes", "dem_mlp_train_step_noalloc", "dem_set_pair_mode", "dem_fluid_solve"])
MLP_NPARAMS = 8898
MLP_NOALLOC_MAX_BATCH = 4096


class dem_wall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("p", ctypes.c_double * 6)]


class dem_grid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("n", ctypes.c_int32 * 3),
                ("reserved", ctypes.c_int32)]


class dem_params(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_double), ("E", ctypes.c_double), ("nu", ctypes.c_double), ("e", ctypes.c_double),
        ("mu", ctypes.c_double), ("mu_roll", ctypes.c_double), ("gamma", ctypes.c_double),
        ("k", ctypes.c_double), ("cg_scheme", ctypes.c_int32), ("normal_model", ctypes.c_int32),
        ("k_lin", ctypes.c_double),
        ("fluid_on", ctypes.c_int32), ("voidfrac", ctypes.c_int32), ("u_superficial", ctypes.c_int32),
        ("couple_every", ctypes.c_int32),
        ("rho_f", ctypes.c_double), ("mu_f", ctypes.c_double), ("n_min", ctypes.c_double),
        ("grid", dem_grid), ("g", ctypes.c_double * 3), ("dt", ctypes.c_double), ("skin", ctypes.c_double),
        ("dt_rayleigh_max_frac", ctypes.c_double),
        ("outlet_kind", ctypes.c_int32), ("n_walls", ctypes.c_int32), ("outlet", ctypes.c_double * 4),
        ("walls", dem_wall * DEM_MAX_WALLS),
        ("precision", ctypes.c_int32), ("bond_at_init", ctypes.c_int32),
        ("pair_capacity", ctypes.c_int64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32),
    ]


_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


class dem_state(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("omega", ctypes.c_void_p),
        ("force", ctypes.c_void_p), ("torque", ctypes.c_void_p), ("radius", ctypes.c_void_p),
        ("alive", ctypes.c_void_p),
        ("n_pairs", ctypes.c_int64), ("pair_idx", ctypes.c_void_p), ("pair_dt", ctypes.c_void_p),
        ("pair_bonded", ctypes.c_void_p),
        ("produced_mass", ctypes.c_double), ("time", ctypes.c_double), ("coordination", ctypes.c_double),
        ("kinetic", ctypes.c_double),
        ("step", ctypes.c_int64), ("broken_bonds", ctypes.c_int64), ("n_alive", ctypes.c_int64),
        ("n_contacts", ctypes.c_int64),
        ("fluid_force", ctypes.c_void_p), ("wall_dt", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libdem.so (built by paper_2211_06142_amd.build).  Raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdem.so is not built: run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.dem_init.restype = i32
        L.dem_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(dem_params), i32, vp,
                               ctypes.POINTER(dem_state), i32, vp]
        L.dem_step.restype = i32
        L.dem_step.argtypes = [vp, i64]
        L.dem_map_fluid.restype = i32
        L.dem_map_fluid.argtypes = [vp, vp, vp, vp, vp]
        L.dem_read_state.restype = i32
        L.dem_read_state.argtypes = [vp, ctypes.POINTER(dem_state)]
        L.dem_read_pairs.restype = i32
        L.dem_read_pairs.argtypes = [vp, i32, i64, vp, vp, vp, vp]
        L.dem_read_aggregates.restype = i32
        L.dem_read_aggregates.argtypes = [vp, vp, vp, vp, vp]
        L.dem_read_wall_forces.restype = i32
        L.dem_read_wall_forces.argtypes = [vp, vp]
        L.dem_set_walls.restype = i32
        L.dem_set_walls.argtypes = [vp, i32, i32, vp]
        L.dem_info.restype = i32
        L.dem_info.argtypes = [vp, vp, vp, vp, vp, vp]
        L.dem_request_rebuild.restype = i32
        L.dem_request_rebuild.argtypes = [vp]
        L.dem_profile.restype = i32
        L.dem_profile.argtypes = [vp, i32]
        L.dem_read_profile.restype = i32
        L.dem_read_profile.argtypes = [vp, vp, vp]
        L.dem_read_fault.restype = i32
        L.dem_read_fault.argtypes = [vp, vp]
        L.dem_destroy.restype = None
        L.dem_destroy.argtypes = [vp]
        L.dem_status_str.restype = ctypes.c_char_p
        L.dem_status_str.argtypes = [i32]
        L.dem_cg_material.restype = i32
        L.dem_cg_material.argtypes = [ctypes.POINTER(dem_params), vp, vp]
        L.dem_cg_diameters.restype = i32
        L.dem_cg_diameters.argtypes = [i32, d, vp, i64, vp, i64]
        L.dem_rayleigh_dt.restype = d
        L.dem_rayleigh_dt.argtypes = [d, d, d, d]
        L.dem_mlp_create.restype = i32
        L.dem_mlp_create.argtypes = [ctypes.POINTER(vp), i32, vp]
        L.dem_mlp_destroy.restype = None
        L.dem_mlp_destroy.argtypes = [vp]
        L.dem_mlp_set_params.restype = i32
        L.dem_mlp_set_params.argtypes = [vp, vp]
        L.dem_mlp_get_params.restype = i32
        L.dem_mlp_get_params.argtypes = [vp, vp]
        L.dem_mlp_forward.restype = i32
        L.dem_mlp_forward.argtypes = [vp, vp, vp, i64]
        L.dem_mlp_grad.restype = i32
        L.dem_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp]
        L.dem_mlp_train_step.restype = i32
        L.dem_mlp_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float, vp]
        L.dem_mlp_train_step_noalloc.restype = i32
        L.dem_mlp_train_step_noalloc.argtypes = [vp, vp, vp, i64, ctypes.c_float, vp]
        L.dem_set_lanes.restype = i32
        L.dem_set_lanes.argtypes = [vp, i32]
        L.dem_fluid_solve.restype = i32
        L.dem_fluid_solve.argtypes = [vp, vp, vp, i32, d, vp, vp, vp, vp, vp]
        L.dem_set_pair_mode.restype = i32
        L.dem_set_pair_mode.argtypes = [vp, i32]
        L.dem_set_graphs.restype = i32
        L.dem_set_graphs.argtypes = [vp, i32]
        L.dem_set_closure.restype = i32
        L.dem_set_closure.argtypes = [vp, vp, vp]
        L.dem_read_closure.restype = i32
        L.dem_read_closure.argtypes = [vp, vp, vp, vp]
        L.dem_set_size_classes.restype = i32
        L.dem_set_size_classes.argtypes = [vp, i32, vp]
        L.dem_read_produced_classes.restype = i32
        L.dem_read_produced_classes.argtypes = [vp, vp]
        _lib = L
    return _lib


class DemError(RuntimeError):
    def __init__(self, code, where, fault=0):
        self.code = code
        self.fault = fault
        super().__init__("%s: %s (%d, fault bits %d)" % (where, dem_status_str(code), code, fault))


def _check(code, where, ctx=None):
    if code != DEM_OK:
        fault = 0
        if ctx is not None:
            fault = dem_read_fault(ctx)[1]
        raise DemError(code, where, fault)


# ---------------------------------------------------------------------------
# one-to-one wrappers
# ---------------------------------------------------------------------------
def dem_status_str(code):
    return lib().dem_status_str(int(code)).decode()


def dem_init(params, n_samples, sample_offsets, init_state, device, hip_stream):
    """params: dem_params or an array of n_samples; sample_offsets: int64 numpy
    array of n_samples+1 or None; init_state: dem_state; hip_stream: int handle."""
    ctx = ctypes.c_void_p()
    if isinstance(params, dem_params):
        parr = params
    else:
        parr = (dem_params * len(params))(*params)
    offs = None
    if sample_offsets is not None:
        offs = np.ascontiguousarray(sample_offsets, dtype=np.int64)
    rc = lib().dem_init(ctypes.byref(ctx), ctypes.cast(ctypes.byref(parr), ctypes.POINTER(dem_params)),
                        int(n_samples), None if offs is None else offs.ctypes.data, ctypes.byref(init_state),
                        int(device), ctypes.c_void_p(hip_stream))
    return rc, ctx


def dem_step(ctx, nsteps):
    return lib().dem_step(ctx, int(nsteps))


def dem_map_fluid(ctx, u_cell_ptr, gradp_cell_ptr, eps_out_ptr, fdrag_out_ptr):
    return lib().dem_map_fluid(ctx, u_cell_ptr, gradp_cell_ptr, eps_out_ptr, fdrag_out_ptr)


def dem_read_state(ctx, state):
    return lib().dem_read_state(ctx, ctypes.byref(state))


def dem_read_pairs(ctx, which, cap, pair_idx_ptr, pair_dt_ptr, pair_bonded_ptr):
    n = ctypes.c_int64()
    rc = lib().dem_read_pairs(ctx, int(which), int(cap), pair_idx_ptr, pair_dt_ptr, pair_bonded_ptr,
                              ctypes.byref(n))
    return rc, n.value


def dem_read_aggregates(ctx, produced_ptr, coordination_ptr, broken_ptr, nalive_ptr):
    return lib().dem_read_aggregates(ctx, produced_ptr, coordination_ptr, broken_ptr, nalive_ptr)


def dem_info(ctx):
    nc, npr, cap, rb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    mg = ctypes.c_double()
    rc = lib().dem_info(ctx, ctypes.byref(nc), ctypes.byref(npr), ctypes.byref(cap), ctypes.byref(rb),
                        ctypes.byref(mg))
    return rc, {"ncell": nc.value, "n_pairs": npr.value, "pair_capacity": cap.value, "rebuilds": rb.value,
                "cutoff_margin": mg.value}


def dem_request_rebuild(ctx):
    return lib().dem_request_rebuild(ctx)


def dem_destroy(ctx):
    lib().dem_destroy(ctx)


def dem_read_fault(ctx):
    b = ctypes.c_int32()
    rc = lib().dem_read_fault(ctx, ctypes.byref(b))
    return rc, b.value


def dem_profile(ctx, enable):
    return lib().dem_profile(ctx, int(enable))


def dem_read_profile(ctx):
    ms = np.zeros(DEM_PROF_N)
    cnt = np.zeros(DEM_PROF_N, np.int64)
    rc = lib().dem_read_profile(ctx, ms.ctypes.data, cnt.ctypes.data)
    return rc, ms, cnt


def dem_cg_material(params):
    g, f = ctypes.c_double(), ctypes.c_double()
    rc = lib().dem_cg_material(ctypes.byref(params), ctypes.byref(g), ctypes.byref(f))
    return rc, g.value, f.value


def dem_cg_diameters(scheme, k, d_fine, n_out):
    d = np.ascontiguousarray(d_fine, dtype=np.float64)
    out = np.zeros(max(int(n_out), 1))
    rc = lib().dem_cg_diameters(int(scheme), float(k), d.ctypes.data, d.size, out.ctypes.data, int(n_out))
    return rc, out[:n_out]


def dem_rayleigh_dt(radius, rho, E, nu):
    return lib().dem_rayleigh_dt(radius, rho, E, nu)


# ---------------------------------------------------------------------------
# parameter marshalling from a workload description
# ---------------------------------------------------------------------------
def dem_mlp_create(device, hip_stream):
    h = ctypes.c_void_p()
    rc = lib().dem_mlp_create(ctypes.byref(h), device, hip_stream)
    return rc, h


def dem_mlp_destroy(mlp):
    lib().dem_mlp_destroy(mlp)


def dem_mlp_set_params(mlp, params_ptr):
    return lib().dem_mlp_set_params(mlp, params_ptr)


def dem_mlp_get_params(mlp, params_ptr):
    return lib().dem_mlp_get_params(mlp, params_ptr)


def dem_mlp_forward(mlp, x_ptr, y_ptr, batch):
    return lib().dem_mlp_forward(mlp, x_ptr, y_ptr, batch)


def dem_mlp_grad(mlp, x_ptr, t_ptr, batch, grad_ptr):
    loss = ctypes.c_float()
    rc = lib().dem_mlp_grad(mlp, x_ptr, t_ptr, batch, grad_ptr, ctypes.byref(loss))
    return rc, loss.value


def dem_mlp_train_step(mlp, x_ptr, t_ptr, batch, lr):
    loss = ctypes.c_float()
    rc = lib().dem_mlp_train_step(mlp, x_ptr, t_ptr, batch, lr, ctypes.byref(loss))
    return rc, loss.value


def dem_set_size_classes(ctx, n_edges, edges_ptr):
    return lib().dem_set_size_classes(ctx, int(n_edges), edges_ptr)


def dem_read_produced_classes(ctx, mass_ptr):
    return lib().dem_read_produced_classes(ctx, mass_ptr)


def dem_mlp_train_step_noalloc(mlp, x_ptr, t_ptr, batch, lr):
    loss = ctypes.c_float()
    rc = lib().dem_mlp_train_step_noalloc(mlp, x_ptr, t_ptr, batch, lr, ctypes.byref(loss))
    return rc, loss.value


def dem_set_closure(ctx, mlp, norm_ptr):
    return lib().dem_set_closure(ctx, mlp, norm_ptr)


def dem_read_closure(ctx, feat_ptr, cd_ptr, cc_ptr):
    return lib().dem_read_closure(ctx, feat_ptr, cd_ptr, cc_ptr)


class Mlp:
    """Owns one dem_mlp (the learned closure network).  Inputs and targets are
    torch CUDA (HIP) tensors; every product runs in libdem.so."""

    def __init__(self, params=None, device=0, stream=None):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        rc, h = dem_mlp_create(device, self.stream.cuda_stream)
        _check(rc, "dem_mlp_create")
        self.h = h
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "h", None):
            dem_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(MLP_NPARAMS))
        _check(dem_mlp_set_params(self.h, p.ctypes.data), "dem_mlp_set_params")

    def params(self):
        p = np.zeros(MLP_NPARAMS, np.float32)
        _check(dem_mlp_get_params(self.h, p.ctypes.data), "dem_mlp_get_params")
        return p

    def _dev32(self, a, cols):
        t = self.torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, cols)),
                                 device=self.dev)
        return t

    def forward(self, x):
        xt = self._dev32(x, 6)
        y = self.torch.zeros((xt.shape[0], 2), dtype=self.torch.float32, device=self.dev)
        _check(dem_mlp_forward(self.h, xt.data_ptr(), y.data_ptr(), xt.shape[0]), "dem_mlp_forward")
        self.torch.cuda.synchronize(self.dev)
        return y.cpu().numpy()

    def grad(self, x, t):
        xt, tt = self._dev32(x, 6), self._dev32(t, 2)
        g = np.zeros(MLP_NPARAMS, np.float32)
        rc, loss = dem_mlp_grad(self.h, xt.data_ptr(), tt.data_ptr(), xt.shape[0], g.ctypes.data)
        _check(rc, "dem_mlp_grad")
        return loss, g

    def train_step(self, x, t, lr):
        xt, tt = self._dev32(x, 6), self._dev32(t, 2)
        rc, loss = dem_mlp_train_step(self.h, xt.data_ptr(), tt.data_ptr(), xt.shape[0], lr)
        _check(rc, "dem_mlp_train_step")
        return loss


def make_params(material, dt, k=1.0, scheme="ssw", g=(0.0, 0.0, -9.81), walls=(), grid=None, fluid=None,
                outlet=None, precision="fp64", normal_model=DEM_NORMAL_JKR_MOD, k_lin=0.0, bond_at_init=True,
                skin=0.0, pair_capacity=0, dt_rayleigh_max_frac=0.0):
    p = dem_params()
    p.rho, p.E, p.nu, p.e = material["rho"], material["E"], material["nu"], material["e"]
    p.mu, p.mu_roll, p.gamma = material["mu"], material.get("mu_roll", 0.0), material["gamma"]
    p.k = float(k)
    p.cg_scheme = DEM_CG_SSP if scheme == "ssp" else DEM_CG_SSW
    p.normal_model = normal_model
    p.k_lin = k_lin
    p.dt = dt
    p.skin = skin
    p.dt_rayleigh_max_frac = dt_rayleigh_max_frac
    for c in range(3):
        p.g[c] = g[c]
    p.n_walls = len(walls)
    for q, (kind, prm) in enumerate(walls):
        p.walls[q].kind = kind
        for a, val in enumerate(prm):
            p.walls[q].p[a] = val
    if fluid is not None:
        p.fluid_on = 1
        p.rho_f, p.mu_f = fluid["rho_f"], fluid["mu_f"]
        p.n_min = fluid.get("n_min", 0.3)
        p.voidfrac = fluid.get("voidfrac", DEM_VOID_CIC)
        p.u_superficial = fluid.get("u_superficial", 1)
        p.couple_every = fluid.get("couple_every", 1)
        lo, hi, nn = grid
        for c in range(3):
            p.grid.lo[c], p.grid.hi[c], p.grid.n[c] = lo[c], hi[c], nn[c]
    else:
        p.couple_every = 1
    if isinstance(outlet, dict):   # {"above": z}: centres above z leave
        p.outlet_kind = DEM_OUTLET_ABOVE
        p.outlet[3] = outlet["above"]
    elif outlet is not None:       # (x, y, radius): the cavity
        p.outlet_kind = DEM_OUTLET_CAVITY
        for c in range(3):
            p.outlet[c] = outlet[c]
    p.precision = DEM_PREC_MIXED if precision == "mixed" else DEM_PREC_FP64
    p.bond_at_init = 1 if bond_at_init else 0
    p.pair_capacity = pair_capacity
    return p


def params_from_workload(w, precision=None, **kw):
    return make_params(w["material"], w["dt"], k=w.get("k", 1.0), scheme=w.get("scheme", "ssw"), g=w["g"],
                       walls=w["walls"], grid=w["grid"], fluid=w["fluid"], outlet=w["outlet"],
                       precision=precision or w.get("precision", "fp64"), **kw)


# ---------------------------------------------------------------------------
# a context with torch-owned device buffers
# ---------------------------------------------------------------------------
class Simulation:
    """Owns one dem_ctx.  Inputs go in as torch CUDA (HIP) tensors; every
    computation happens in libdem.so."""

    def __init__(self, params, x, r, v=None, w=None, F=None, T=None, alive=None, pairs=None, pair_dt=None,
                 pair_bonded=None, sample_offsets=None, device=0, stream=None, fluid_force=None, wall_dt=None,
                 step=0, size_edges=None):
        import torch
        self.torch = torch
        dev = torch.device("cuda", device)
        self.dev = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        n = int(np.asarray(r).shape[0])
        self.n = n

        def t64(a, shape):
            if a is None:
                return None
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(shape), device=dev)

        bufs = dict(x=t64(x, (n, 3)), v=t64(v, (n, 3)), omega=t64(w, (n, 3)), force=t64(F, (n, 3)),
                    torque=t64(T, (n, 3)), radius=t64(r, (n,)), fluid_force=t64(fluid_force, (n, 3)),
                    wall_dt=t64(wall_dt, (n, DEM_MAX_WALLS, 3)))
        st = dem_state()
        st.n = n
        st.step = int(step)
        for k, t in bufs.items():
            setattr(st, k, None if t is None else t.data_ptr())
        al = None
        if alive is not None:
            al = torch.as_tensor(np.ascontiguousarray(alive, dtype=np.uint8), device=dev)
            st.alive = al.data_ptr()
        keep = [bufs, al]
        if pairs is not None and len(pairs) > 0:
            pp = torch.as_tensor(np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2), device=dev)
            st.n_pairs = pp.shape[0]
            st.pair_idx = pp.data_ptr()
            keep.append(pp)
            if pair_dt is not None:
                pd = t64(pair_dt, (-1, 3))
                st.pair_dt = pd.data_ptr()
                keep.append(pd)
            if pair_bonded is not None:
                pb = torch.as_tensor(np.ascontiguousarray(pair_bonded, dtype=np.uint8), device=dev)
                st.pair_bonded = pb.data_ptr()
                keep.append(pb)
        if isinstance(params, dem_params):
            plist = [params]
        else:
            plist = list(params)
        self.params = plist
        rc, ctx = dem_init(plist[0] if len(plist) == 1 else plist, len(plist), sample_offsets, st, device,
                           self.stream.cuda_stream)
        _check(rc, "dem_init")
        self.ctx = ctx
        self.ncell = self.info()["ncell"]
        if size_edges is not None:
            self.set_size_classes(size_edges)

    def close(self):
        if getattr(self, "ctx", None):
            dem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        _check(dem_step(self.ctx, nsteps), "dem_step", self.ctx)

    def map_fluid(self, u_cell, gradp_cell):
        torch = self.torch
        u = torch.as_tensor(np.ascontiguousarray(u_cell, dtype=np.float64), device=self.dev)
        g = torch.as_tensor(np.ascontiguousarray(gradp_cell, dtype=np.float64), device=self.dev)
        eps = torch.zeros(max(self.ncell, 1), dtype=torch.float64, device=self.dev)
        fd = torch.zeros(max(self.ncell, 1) * 3, dtype=torch.float64, device=self.dev)
        _check(dem_map_fluid(self.ctx, u.data_ptr(), g.data_ptr(), eps.data_ptr(), fd.data_ptr()),
               "dem_map_fluid")
        return eps[:self.ncell].cpu().numpy(), fd[:3 * self.ncell].reshape(-1, 3).cpu().numpy()

    def fluid_out(self):
        torch = self.torch
        eps = torch.zeros(max(self.ncell, 1), dtype=torch.float64, device=self.dev)
        fd = torch.zeros(max(self.ncell, 1) * 3, dtype=torch.float64, device=self.dev)
        _check(dem_map_fluid(self.ctx, None, None, eps.data_ptr(), fd.data_ptr()), "dem_map_fluid")
        return eps[:self.ncell].cpu().numpy(), fd[:3 * self.ncell].reshape(-1, 3).cpu().numpy()

    def state(self, held=False):
        """positions, velocities, forces, alive flags and scalars; held=True
        adds the held fluid force (n x 3) and the wall history (n x 8 x 3)"""
        torch = self.torch
        n = self.n
        out = {k: torch.zeros((n, 3), dtype=torch.float64, device=self.dev) for k in ("x", "v", "w", "F", "T")}
        alive = torch.zeros(n, dtype=torch.uint8, device=self.dev)
        st = dem_state()
        st.x, st.v, st.omega = out["x"].data_ptr(), out["v"].data_ptr(), out["w"].data_ptr()
        st.force, st.torque = out["F"].data_ptr(), out["T"].data_ptr()
        st.alive = alive.data_ptr()
        if held:
            out["fluid_force"] = torch.zeros((n, 3), dtype=torch.float64, device=self.dev)
            out["wall_dt"] = torch.zeros((n, DEM_MAX_WALLS, 3), dtype=torch.float64, device=self.dev)
            st.fluid_force, st.wall_dt = out["fluid_force"].data_ptr(), out["wall_dt"].data_ptr()
        _check(dem_read_state(self.ctx, st), "dem_read_state")
        res = {k: t.cpu().numpy() for k, t in out.items()}
        res["alive"] = alive.cpu().numpy()
        for k in ("produced_mass", "time", "coordination", "kinetic", "step", "broken_bonds", "n_alive",
                  "n_contacts"):
            res[k] = getattr(st, k)
        return res

    def pairs(self, which=0, sort=True):
        rc, cnt = dem_read_pairs(self.ctx, which, 0, None, None, None)
        _check(rc, "dem_read_pairs")
        pi = np.zeros((max(cnt, 1), 2), np.int64)
        pdt = np.zeros((max(cnt, 1), 3))
        pb = np.zeros(max(cnt, 1), np.uint8)
        rc, cnt = dem_read_pairs(self.ctx, which, cnt, pi.ctypes.data, pdt.ctypes.data, pb.ctypes.data)
        _check(rc, "dem_read_pairs")
        if not sort:
            return {"pairs": pi[:cnt], "dt": pdt[:cnt], "bonded": pb[:cnt]}
        order = np.lexsort((pi[:cnt, 1], pi[:cnt, 0]))
        return {"pairs": pi[:cnt][order], "dt": pdt[:cnt][order], "bonded": pb[:cnt][order]}

    def aggregates(self):
        ns = len(self.params)
        pm = np.zeros(ns)
        z = np.zeros(ns)
        bb = np.zeros(ns, np.int64)
        na = np.zeros(ns, np.int64)
        _check(dem_read_aggregates(self.ctx, pm.ctypes.data, z.ctypes.data, bb.ctypes.data, na.ctypes.data),
               "dem_read_aggregates")
        return {"produced_mass": pm, "coordination": z, "broken_bonds": bb, "n_alive": na}

    def wall_forces(self):
        """(n_samples, DEM_MAX_WALLS, 3): the particles' total force on each wall"""
        f = np.zeros((len(self.params), DEM_MAX_WALLS, 3))
        _check(lib().dem_read_wall_forces(self.ctx, f.ctypes.data), "dem_read_wall_forces")
        return f

    def set_walls(self, walls, sample=0):
        """replace a sample's walls, given as [(kind, params), ...] (the same count)"""
        arr = (dem_wall * DEM_MAX_WALLS)()
        for k, (kind, prm) in enumerate(walls):
            arr[k].kind = kind
            for q, val in enumerate(prm):
                arr[k].p[q] = val
        _check(lib().dem_set_walls(self.ctx, int(sample), len(walls), ctypes.cast(arr, ctypes.c_void_p)),
               "dem_set_walls")

    def set_size_classes(self, edges):
        """produced-sand size classes by fine-scale diameter (edges in m)"""
        if edges is None:
            _check(dem_set_size_classes(self.ctx, 0, None), "dem_set_size_classes")
            self.n_classes = 0
            return
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        _check(dem_set_size_classes(self.ctx, e.size, e.ctypes.data), "dem_set_size_classes")
        self.n_classes = e.size - 1

    def produced_classes(self):
        """produced mass per sample and size class (n_samples x n_classes), kg"""
        m = np.zeros((len(self.params), self.n_classes))
        _check(dem_read_produced_classes(self.ctx, m.ctypes.data), "dem_read_produced_classes")
        return m

    def info(self):
        rc, inf = dem_info(self.ctx)
        _check(rc, "dem_info")
        return inf

    def profile(self, enable):
        _check(dem_profile(self.ctx, enable), "dem_profile")

    def read_profile(self):
        rc, ms, cnt = dem_read_profile(self.ctx)
        _check(rc, "dem_read_profile")
        return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(PROF_NAMES)}

    def request_rebuild(self):
        _check(dem_request_rebuild(self.ctx), "dem_request_rebuild")

    def set_lanes(self, lanes):
        _check(lib().dem_set_lanes(self.ctx, int(lanes)), "dem_set_lanes")

    def fluid_solve(self, cell_kind, p_fixed, max_iter=2000, rel_tol=1e-10):
        """model-A pressure solve on the latest coupling evaluation; returns
        (p, superficial u, grad p, iterations, relative residual)"""
        kd = np.ascontiguousarray(np.asarray(cell_kind, dtype=np.int8))
        pf = np.ascontiguousarray(np.asarray(p_fixed, dtype=np.float64))
        nc = self.ncell
        p = np.zeros(nc)
        u = np.zeros((nc, 3))
        gp = np.zeros((nc, 3))
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        _check(lib().dem_fluid_solve(self.ctx, kd.ctypes.data, pf.ctypes.data, int(max_iter), float(rel_tol),
                                     p.ctypes.data, u.ctypes.data, gp.ctypes.data, ctypes.byref(it),
                                     ctypes.byref(rr)), "dem_fluid_solve")
        return p, u, gp, it.value, rr.value

    def set_pair_mode(self, mode):
        """DEM_PAIRS_FULL_ROWS or DEM_PAIRS_HALF (or "full" / "half")"""
        m = {"full": DEM_PAIRS_FULL_ROWS, "half": DEM_PAIRS_HALF}.get(mode, mode)
        _check(lib().dem_set_pair_mode(self.ctx, int(m)), "dem_set_pair_mode")

    def set_graphs(self, enable):
        _check(lib().dem_set_graphs(self.ctx, 1 if enable else 0), "dem_set_graphs")

    def set_closure(self, mlp=None, norm=None):
        """learned closure from the current parameters of `mlp` (an Mlp), with
        norm = (mean[6], sd[6]); None switches it off"""
        if mlp is None:
            _check(dem_set_closure(self.ctx, None, None), "dem_set_closure")
            return
        nn = np.ascontiguousarray(np.asarray(norm, dtype=np.float64).reshape(12))
        _check(dem_set_closure(self.ctx, mlp.h, nn.ctypes.data), "dem_set_closure")

    def read_closure(self):
        f = np.zeros((self.n, 6))
        cd, cc = np.zeros(self.n), np.zeros(self.n)
        _check(dem_read_closure(self.ctx, f.ctypes.data, cd.ctypes.data, cc.ctypes.data), "dem_read_closure")
        return {"features": f, "c_drag": cd, "c_coh": cc}
