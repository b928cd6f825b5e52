"""CPU checks of the C ABI: the library loads, exports every declared symbol,
the ctypes layouts equal the C layouts, and the host-only helpers agree with
the oracle's independent coarse-graining code.  No compute call needs a GPU."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import cg
from paper_2211_06142_amd import dem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dem.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:dem_status|void|const char\*|double)\s+(dem_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    L = dem.lib()
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(L, name), name
    assert dem.EXPORTS == names


def _c_layout():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "dem.h"
#define F(T, m) printf("%s %s %zu\n", #T, #m, offsetof(T, m));
int main(void) {
  printf("dem_params SIZE %zu\n", sizeof(dem_params));
  printf("dem_state SIZE %zu\n", sizeof(dem_state));
  printf("dem_grid SIZE %zu\n", sizeof(dem_grid));
  printf("dem_wall SIZE %zu\n", sizeof(dem_wall));
  %FIELDS%
  return 0;
}
"""
    fields = []
    for cls in (dem.dem_params, dem.dem_state, dem.dem_grid, dem.dem_wall):
        for name, _ in cls._fields_:
            fields.append("F(%s, %s)" % (cls.__name__, name))
    prog = prog.replace("%FIELDS%", "\n  ".join(fields))
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "l.c")
        exe = os.path.join(td, "l")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    res = {}
    for line in out:
        if line.strip():
            t, m, v = line.split()
            res[(t, m)] = int(v)
    return res


def test_ctypes_layout_matches_c():
    lay = _c_layout()
    for cls in (dem.dem_params, dem.dem_state, dem.dem_grid, dem.dem_wall):
        assert ctypes.sizeof(cls) == lay[(cls.__name__, "SIZE")], cls.__name__
        for name, _ in cls._fields_:
            assert getattr(cls, name).offset == lay[(cls.__name__, name)], (cls.__name__, name)


def test_cg_helpers_match_oracle():
    rng = np.random.default_rng(0)
    d = rng.uniform(1e-4, 4e-4, 1000)
    for k in (1.0, 2.0, 3.0):
        rc, out = dem.dem_cg_diameters(dem.DEM_CG_SSW, k, d, 500)
        assert rc == dem.DEM_OK
        np.testing.assert_allclose(out, cg.ssw_diameters(d[:500], k), rtol=1e-15)
        rc, out = dem.dem_cg_diameters(dem.DEM_CG_SSP, k, d, 7)
        assert rc == dem.DEM_OK
        np.testing.assert_allclose(out, cg.ssp_diameter(d, k), rtol=1e-13)
        p = dem.make_params(dict(rho=2650, E=70e6, nu=0.3, e=0.5, mu=0.5, gamma=0.5), 1e-7, k=k)
        rc, gam, fac = dem.dem_cg_material(p)
        assert rc == dem.DEM_OK
        assert gam == cg.scale_material(dict(gamma=0.5), k)["gamma"]
        assert fac == k ** 3
    assert dem.dem_rayleigh_dt(1.1474e-4, 2605, 2e10, 0.3) == pytest.approx(
        cg.rayleigh_dt(1.1474e-4, 2605, 2e10, 0.3), rel=1e-14)
    rc, _ = dem.dem_cg_diameters(dem.DEM_CG_SSW, 0.5, d, 10)
    assert rc == dem.DEM_E_INVAL


def test_init_validation_is_host_side():
    """Invalid parameters are refused before any device call."""
    x = np.zeros((2, 3))
    x[1, 0] = 1e-3
    r = np.array([1e-4, 1e-4])
    st = dem.dem_state()
    st.n = 2
    st.x = x.ctypes.data
    st.radius = r.ctypes.data
    mat = dict(rho=2650, E=70e6, nu=0.3, e=0.5, mu=0.5, gamma=0.5)
    for key, val in (("dt", 0.0), ("nu", 0.5), ("e", 1.5), ("k", 0.9), ("rho", -1.0)):
        p = dem.make_params(mat, 1e-7)
        setattr(p, key, val)
        rc, ctx = dem.dem_init(p, 1, None, st, 0, 0)
        assert rc == dem.DEM_E_INVAL, key
        assert not ctx.value
    assert dem.dem_status_str(dem.DEM_E_CAPACITY) == "pair capacity exceeded"
