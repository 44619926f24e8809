"""Storage precision on the 128x64x64 crop (physics of the 64x32x32 canopy
case, seed 3): every storage type after 1000 steps against the FP64 oracle.

Per field (rho, u, nu_t) the error is reported as max |gpu - oracle| and
RMS(gpu - oracle), both divided by max |oracle|.  Bounds are about twice the
values measured on MI355X (FP64 keeps the 1e-12 parity bar).  Stochastic
rounding (bf16sr) halves the velocity error of round-to-nearest BF16.
"""
import numpy as np
import pytest

from paper_2206_15454_amd import inputs
from tests.gpu_common import make_pair, require_gpu

pytestmark = pytest.mark.gpu

BOUNDS = {  # storage: {field: (max, rms)}; measured (max, rms) in the comments
    "f64": {"rho": (1e-12, 1e-12), "u": (1e-12, 1e-12), "nut": (1e-12, 1e-12)},  # 1e-13
    # rho (1.7e-6, 3.2e-7), u (6.4e-5, 2.5e-5), nu_t (1.1e-4, 1.7e-5); before the
    # paired collision (another rounding order) rho (2.9e-6, 1.2e-6), u (3.4e-5, 1.1e-5)
    "f32": {"rho": (6e-6, 3e-6), "u": (1.5e-4, 6e-5), "nut": (3e-4, 4e-5)},
    # rho (8.8e-5, 1.6e-5), u (1.4e-3, 2.0e-4), nu_t (2.9e-2, 5.0e-3)
    "f16s": {"rho": (2e-4, 4e-5), "u": (3e-3, 4e-4), "nut": (6e-2, 1e-2)},
    # rho (8.0e-4, 1.5e-4), u (3.0e-2, 4.3e-3), nu_t (2.5e-1, 6.1e-2)
    "bf16s": {"rho": (2e-3, 3e-4), "u": (6e-2, 9e-3), "nut": (5e-1, 1.2e-1)},
    # rho (9.8e-4, 1.8e-4), u (1.3e-2, 2.1e-3), nu_t (3.4e-1, 9.2e-2)
    "bf16sr": {"rho": (2e-3, 4e-4), "u": (3e-2, 5e-3), "nut": (7e-1, 2e-1)},
}


@pytest.fixture(scope="module")
def oracle_run():
    require_gpu()
    w = inputs.CROP
    o, _ = make_pair(w, storage="f64")
    o.step(w.steps)
    rho, u, nut, _ = o.moments()
    return rho, u, nut


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s", "bf16sr"])
def test_crop_1000_steps(oracle_run, storage):
    w = inputs.CROP
    _, g = make_pair(w, storage=storage)
    g.step(w.steps)
    rg, ug, ng, _ = g.moments()
    ro, uo, no = oracle_run
    out = {}
    for name, a, b in (("rho", rg, ro), ("u", ug, uo), ("nut", ng, no)):
        den = np.max(np.abs(b))
        d = np.abs(a - b)
        out[name] = (float(d.max() / den), float(np.sqrt(np.mean(d * d)) / den))
    print(f"crop 128x64x64 1000 steps {storage}: " +
          ", ".join(f"{k} max {v[0]:.2e} rms {v[1]:.2e}" for k, v in out.items()))
    for k, (mx, rms) in BOUNDS[storage].items():
        assert out[k][0] <= mx and out[k][1] <= rms, (k, out[k])
