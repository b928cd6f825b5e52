"""The training step that allocates nothing (dem_mlp_train_step_noalloc)
against the training step that grows its own buffers, through the C ABI: the
same kernels on the same inputs, so parameters and loss must agree bit for
bit, on two calls in a row (the second with a smaller batch, which must not
see the first call's leftovers in the shared scratch array)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2211_06142_amd import dem  # noqa: E402
from oracle import mlp  # noqa: E402


def test_noalloc_train_step_equals_train_step():
    rng = np.random.default_rng(21)
    p0 = mlp.init_params(22, 1.0).astype(np.float32)
    a, b = dem.Mlp(p0), dem.Mlp(p0)
    for batch, lr in ((dem.MLP_NOALLOC_MAX_BATCH, 2e-3), (1777, 1e-3)):
        x = torch.as_tensor(rng.normal(size=(batch, 6)).astype(np.float32), device="cuda")
        t = torch.as_tensor(rng.normal(0, 0.5, size=(batch, 2)).astype(np.float32), device="cuda")
        rc1, la = dem.dem_mlp_train_step(a.h, x.data_ptr(), t.data_ptr(), batch, lr)
        assert rc1 == dem.DEM_OK
        rc2, lb = dem.dem_mlp_train_step_noalloc(b.h, x.data_ptr(), t.data_ptr(), batch, lr)
        assert rc2 == dem.DEM_OK
        assert la == lb and np.isfinite(la)
        np.testing.assert_array_equal(a.params(), b.params())
        assert not np.array_equal(a.params(), p0)
    # batch beyond the scratch: rejected on the host, nothing launched
    x = torch.zeros((dem.MLP_NOALLOC_MAX_BATCH + 1, 6), dtype=torch.float32, device="cuda")
    t = torch.zeros((dem.MLP_NOALLOC_MAX_BATCH + 1, 2), dtype=torch.float32, device="cuda")
    rc, _ = dem.dem_mlp_train_step_noalloc(b.h, x.data_ptr(), t.data_ptr(), dem.MLP_NOALLOC_MAX_BATCH + 1, 1e-3)
    assert rc == dem.DEM_E_INVAL
    np.testing.assert_array_equal(a.params(), b.params())
    a.close()
    b.close()
