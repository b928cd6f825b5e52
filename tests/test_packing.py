"""Input generator checks (no GPU): the coloured parallel Gauss-Seidel packing
sweep gives the same packing for any thread count and settles as well as the
serial sweep."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# settle a small annulus bed; print the positions' digest, the radii and positions
_SCRIPT = r"""
import sys, json, hashlib, numpy as np
sys.path.insert(0, %r)
import synth
n, seed, iters, colored = int(sys.argv[1]), int(sys.argv[2]), int(sys.argv[3]), sys.argv[4] == "1"
rng = np.random.default_rng(seed)
r = 0.5 * synth.sample_diameters(rng, n)
x, worst = synth.settle(r, 1, (0.0, 0.0, 0.5e-3, 2.0e-3, 0.0, 2e-3), rng, iters=iters, settle_iters=iters // 2,
                        colored=colored)
print(json.dumps({"sha": hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest(), "worst": worst,
                  "r": r.tolist(), "x": x.tolist()}))
""" % ROOT
REGION = (0.0, 0.0, 0.5e-3, 2.0e-3, 0.0, 2e-3)
SHRINK = 0.998   # settle()'s default: the radii are confined and separated at 0.998 r


def _run(n, seed, iters, colored, threads=1):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_WAIT_POLICY="passive")
    out = subprocess.run([sys.executable, "-c", _SCRIPT, str(n), str(seed), str(iters), "1" if colored else "0"],
                         env=env, capture_output=True, text=True, check=True)
    d = json.loads(out.stdout)
    return d["sha"], d["worst"], np.array(d["r"]), np.array(d["x"])


def test_colored_sweep_is_thread_count_independent():
    a = _run(3000, 7, 300, True, threads=1)
    b = _run(3000, 7, 300, True, threads=2)
    assert a[0] == b[0]
    assert a[1] == b[1]


def _overlaps(x, r):
    d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=2)
    i, j = np.triu_indices(len(r), 1)
    ov = (r[i] + r[j] - d[i, j]) / np.minimum(r[i], r[j])
    return ov[ov > 0]


@pytest.mark.parametrize("colored", [False, True])
def test_sweeps_settle_the_bed(colored):
    _, _, r, x = _run(1500, 11, 600, colored)
    rs = SHRINK * r
    ov = _overlaps(x, rs)
    # every sphere inside the annulus and above the floor
    rho = np.hypot(x[:, 0], x[:, 1])
    assert np.all(rho >= REGION[2] + rs - 1e-12) and np.all(rho <= REGION[3] - rs + 1e-12)
    assert np.all(x[:, 2] >= rs - 1e-12)
    # settled: a contact network (about 3.6 contacts per sphere) with small overlaps
    assert len(ov) > len(r)
    assert np.median(ov) < 0.01 and np.percentile(ov, 99) < 0.05


def test_colored_sweep_matches_serial_quality():
    _, _, r, xs = _run(1500, 11, 600, False)
    _, _, _, xc = _run(1500, 11, 600, True)
    os_, oc = _overlaps(xs, SHRINK * r), _overlaps(xc, SHRINK * r)
    # as many contacts, no deeper tail of residual overlaps, the same bed height
    assert abs(len(oc) - len(os_)) < 0.05 * len(os_)
    assert np.percentile(oc, 99) < 1.5 * np.percentile(os_, 99) + 1e-3
    top_s, top_c = np.max(xs[:, 2] + r), np.max(xc[:, 2] + r)
    assert abs(top_c - top_s) < 0.02 * top_s
