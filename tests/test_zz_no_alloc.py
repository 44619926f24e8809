"""lbm_closure_samples_noalloc (the work area in the library's fixed device
array) against lbm_closure_samples (work area allocated per call), through
the C ABI: bit-identical samples on two calls in a row, the second on a
smaller grid, and the size limits rejected with EINVAL."""
import numpy as np
import pytest

from paper_2206_15454_amd import inputs
from tests.gpu_common import make_gpu, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def fine_run(nx, ny, nz, seed):
    w = inputs.scaled(inputs.C1, nx, ny, nz, noise=0.3)
    g = make_gpu(w, "f32")
    rho, u = inputs.init_fields(w, seed)
    g.init(rho, u)
    g.step(6)
    return g


def test_noalloc_samples_equal_allocating_call_twice():
    import torch

    from paper_2206_15454_amd import lbm

    # first call: 128x64x64 fine (65536 coarse cells), then a smaller,
    # ragged 36x20x28 fine grid (2520 coarse cells) reusing the array
    for (nx, ny, nz), seed in (((128, 64, 64), 21), ((36, 20, 28), 22)):
        g = fine_run(nx, ny, nz, seed)
        lad_c = np.linspace(0.3, 0.0, ny // 2)
        Xa, ya = g.closure_samples(0.52, 4.0, lad_c)
        nc = (nx // 2) * (ny // 2) * (nz // 2)
        Xn = torch.full((nc, 9), float("nan"), dtype=torch.float32, device="cuda")
        yn = torch.full((nc,), float("nan"), dtype=torch.float32, device="cuda")
        g.closure_samples(0.52, 4.0, lad_c, out=(Xn, yn), noalloc=True)
        torch.cuda.synchronize()
        Xa, ya, Xn, yn = (t.cpu().numpy() for t in (Xa, ya, Xn, yn))
        print(f"{nx}x{ny}x{nz}: {nc} coarse cells, max target {ya.max():.3e}", flush=True)
        assert ya.max() > 0
        np.testing.assert_array_equal(Xn, Xa)
        np.testing.assert_array_equal(yn, ya)
        g.close()
    assert lbm.NOALLOC_MAX_COARSE == 262144


def test_noalloc_rejects_grids_beyond_its_array():
    import torch

    from paper_2206_15454_amd import lbm

    # 130x64x258 fine is 65x32x129 = 268320 coarse cells: beyond the limit
    g = fine_run(130, 64, 258, 23)
    nc = 65 * 32 * 129
    assert nc > lbm.NOALLOC_MAX_COARSE
    X = torch.empty((nc, 9), dtype=torch.float32, device="cuda")
    y = torch.empty(nc, dtype=torch.float32, device="cuda")
    with pytest.raises(lbm.LBMError) as ei:
        g.closure_samples(0.52, 4.0, np.zeros(32), out=(X, y), noalloc=True)
    assert ei.value.status == 1 and "at most" in str(ei.value)
    g.close()
    # more coarse rows than the LAD part holds
    ny = 2 * (lbm.NOALLOC_MAX_LAD + 1)
    g = fine_run(2, ny, 2, 24)
    X = torch.empty((ny // 2, 9), dtype=torch.float32, device="cuda")
    y = torch.empty(ny // 2, dtype=torch.float32, device="cuda")
    with pytest.raises(lbm.LBMError) as ei:
        g.closure_samples(0.52, 4.0, np.zeros(ny // 2), out=(X, y), noalloc=True)
    assert ei.value.status == 1
    g.close()
