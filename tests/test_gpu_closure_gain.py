"""What the trained closure gains over the plain coarse-grained model (an
extension; not in arXiv:2211.06142): paired fine (200 000 grains) and coarse
(k = 2, SSW) runs of the cylinder, the dataset from them, training on the GPU,
and the produced mass of the plain and of the learned coarse model against
the fine run.  The closure is kept only when it is not worse than the plain
model (the fallback); the test checks that this rule is applied, that the
training lowers its loss, and that the coarse model (whichever is kept) is
faster than the fine one."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2211_06142_amd import closure_train as ct  # noqa: E402


def test_closure_gain_k2():
    res = ct.gain_test(synth.c1(), synth.c2(2), horizon=6000, window=500, epochs=10,
                       log=lambda *a: print(*a, flush=True))
    print({k: v for k, v in res.items() if k not in ("net", "norm", "mass_series")})
    assert res["train_samples"] > 10000
    assert res["loss_last"] < res["loss_first"]
    assert res["mass_fine"] > 0.0
    for k in ("err_plain_cg", "err_learned_cg"):
        assert math.isfinite(res[k])
    assert res["closure_accepted"] == (res["err_learned_cg"] <= res["err_plain_cg"])
    kept = res["err_learned_cg"] if res["closure_accepted"] else res["err_plain_cg"]
    assert kept == min(res["err_learned_cg"], res["err_plain_cg"])
    assert res["speedup_vs_fine"] > 1.0
    m = res["mass_series"]
    assert np.all(np.diff(m["fine"]) >= 0.0) and np.all(np.diff(m["plain"]) >= 0.0)
