"""The paper's own set-ups on the GPU: the ABL over a homogeneous forest
(Sec. 5; forced-equilibrium top, LAD cases 1-3 of Table tab:forest_cases)
and the Re_tau = 180 validation channel (Sec. 4)."""
import numpy as np
import pytest

from paper_2206_15454_amd import inputs
from tests.gpu_common import make_gpu, make_pair, normwise, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("case", [inputs.ABL1, inputs.ABL2])
def test_abl_physics_matches_oracle(case):
    """FP64 parity with the forced-equilibrium top on a 64x40x32 section of
    the fine-mesh set-up (same per-cell parameters)."""
    w = inputs.scaled(case, 64, 40, 32, storage="f64")
    o, g = make_pair(w, seed=8)
    o.step(40)
    g.step(40)
    ro, uo, no, do = o.moments()
    rg, ug, ng, dg = g.moments()
    e = {"rho": normwise(rg, ro), "u": normwise(ug, uo), "nut": normwise(ng, no)}
    print(case.name, e)
    assert max(e.values()) <= 1e-12
    assert dg["mass"] == pytest.approx(do["mass"], rel=1e-13)


def test_abl_fine_mesh_forest_cases():
    """350x140x280 (the paper's fine mesh, 7 forest cells), 400 steps in FP32
    for the three LAD cases: stable, and the forest drag slows the canopy
    rows relative to the case without forest."""
    import torch

    means = {}
    for w in (inputs.ABL1, inputs.ABL2, inputs.ABL3):
        g = make_gpu(w)
        rho, u = inputs.init_fields_torch(w, torch.device("cuda"))
        g.init(rho, u)
        g.step(400)
        r, uu, nt, d = g.moments()
        assert d["nonfinite"] == 0 and d["max_u"] < 0.2
        means[w.name] = uu[0].mean(axis=(0, 2))
        g.close()
    c1, c2, c3 = (means[w.name] for w in (inputs.ABL1, inputs.ABL2, inputs.ABL3))
    print("mean u in the forest rows: case1 %.4f case2 %.4f case3 %.4f" % (
        c1[:7].mean(), c2[:7].mean(), c3[:7].mean()))
    assert c1[:7].mean() < c3[:7].mean() and c2[:7].mean() < c3[:7].mean()
    # far above the forest the three cases still agree closely
    assert abs(c1[100:].mean() - c3[100:].mean()) < 0.02 * c3[100:].mean()


def test_channel_matches_oracle_and_stays_mirror_symmetric():
    w = inputs.scaled(inputs.CHANNEL, 48, 20, 16, storage="f64")
    o, g = make_pair(w, init=False)
    rho, u = inputs.init_fields(w, seed=3)
    # mirror-symmetric start about the mid-plane: u, w even and v odd in y
    u[0] = 0.5 * (u[0] + u[0][:, ::-1, :])
    u[1] = 0.5 * (u[1] - u[1][:, ::-1, :])
    u[2] = 0.5 * (u[2] + u[2][:, ::-1, :])
    o.init(rho, u)
    g.init(rho, u)
    o.step(100)
    g.step(100)
    _, uo, _, _ = o.moments()
    _, ug, _, _ = g.moments()
    assert normwise(ug, uo) <= 1e-12
    scale = np.max(np.abs(ug[0]))
    assert np.max(np.abs(ug[0] - ug[0][:, ::-1, :])) <= 1e-12 * scale
    assert np.max(np.abs(ug[1] + ug[1][:, ::-1, :])) <= 1e-12 * scale
