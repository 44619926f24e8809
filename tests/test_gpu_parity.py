"""Parity of the HIP fused step (through the C ABI) against the FP64 oracle.

Tolerances:
  * FP64 storage: normwise max|gpu - oracle| / max|oracle| <= 1e-12 per field
    after 200 steps of the 64x32x32 canopy case (the arithmetic differs only in
    operation order: shifted moments, fused multiply-adds).
  * One step from a stored state S (any storage T): the GPU result equals the
    oracle step of decode(S) rounded into T, up to one unit in the last place
    of T plus the FP32 arithmetic error (a few FP32 ulps of the population
    magnitude) where T is not FP64.
  * Multi-step, low precision: per-field normwise bounds stated in each test.
"""
import numpy as np
import pytest

from oracle import ref
from paper_2206_15454_amd import inputs
from tests.gpu_common import make_pair, normwise, require_gpu, round_storage, ulp

pytestmark = pytest.mark.gpu

_, W = ref.lattice()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _compare_moments(o, g):
    ro, uo, no, do = o.moments()
    rg, ug, ng, dg = g.moments()
    return {"rho": normwise(rg, ro), "u": normwise(ug, uo), "nut": normwise(ng, no)}, do, dg


def test_f64_canopy_200_steps_matches_oracle():
    w = inputs.C1
    o, g = make_pair(w)
    o.step(w.steps)
    g.step(w.steps)
    err, do, dg = _compare_moments(o, g)
    print("f64 64x32x32 200 steps normwise:", err)
    assert err["rho"] <= 1e-12 and err["u"] <= 1e-12 and err["nut"] <= 1e-12
    assert dg["t"] == 200 and dg["nonfinite"] == 0
    assert dg["mass"] == pytest.approx(do["mass"], rel=1e-13)
    for k in ("mom_x", "mom_y", "mom_z"):
        assert dg[k] == pytest.approx(do[k], rel=1e-10, abs=1e-14)
    for k in ("imp_x", "imp_y", "imp_z"):
        assert dg[k] == pytest.approx(do[k], rel=1e-12, abs=1e-18)
    assert dg["max_u"] == pytest.approx(do["max_u"], rel=1e-12)


@pytest.mark.parametrize("shape,bcs", [
    ((37, 5, 3), (1, 2)),     # ragged x, tiny y
    ((70, 4, 5), (1, 1)),     # channel: bounce-back both walls
    ((65, 3, 7), (2, 2)),     # free slip both
    ((64, 6, 4), (0, 0)),     # fully periodic
    ((300, 3, 2), (2, 1)),    # several x tiles with a ragged tail
    ((8, 1, 9), (1, 2)),      # a single row between the walls
    ((40, 6, 5), (1, 3)),     # forced-equilibrium top (the paper's ABL top)
    ((33, 4, 3), (3, 3)),     # forced equilibrium at both ends
    ((20, 1, 4), (2, 3)),     # one row: free slip below, equilibrium above
    ((1, 5, 1), (1, 2)),      # one column: x and z periodic onto the cell itself
    ((1, 4, 6), (1, 1)),      # one cell wide in x
    ((5, 3, 1), (2, 1)),      # one cell deep in z
])
def test_f64_boundaries_and_ragged_grids(shape, bcs):
    nx, ny, nz = shape
    w = inputs.scaled(inputs.C1, nx, ny, nz, bc_lo=bcs[0], bc_hi=bcs[1],
                      canopy_rows=max(1, ny // 2), g=(2e-5, 1e-6, -3e-6),
                      u_wall=(0.06, 0.0, 0.01))
    o, g = make_pair(w, seed=17, vector_drag=(nx % 2 == 1))
    o.step(25)
    g.step(25)
    err, do, dg = _compare_moments(o, g)
    print(shape, bcs, err)
    assert max(err.values()) <= 1e-12
    assert dg["mass"] == pytest.approx(do["mass"], rel=1e-13)


@pytest.mark.parametrize("nx", [67, 512])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s", "bf16sr"])
def test_one_step_from_stored_state(storage, nx):
    """Both AA parities: step 1 (neighbour access) and step 2 (local).
    nx = 67: 128-wide tiles with a ragged tail, default cache policy.
    nx = 512: the launch shape of the 512x128x256 benchmark (256-wide tiles,
    streaming accesses on whole-line rows, row-major tile order; FP32 with
    one buffer resource per plane)."""
    w = inputs.scaled(inputs.C1, nx, 9, 5, canopy_rows=4)
    o, g = make_pair(w, storage=storage, init=False)
    S = inputs.random_populations(w.shape, seed=5, base=W, scale=0.02)
    shifted = round_storage(S - W[:, None, None, None], storage)
    S = shifted + W[:, None, None, None]
    # both parities start from the same stored state S: lbm_set_f stores it
    # where the next step reads it (a neighbour step first; after one step,
    # a local step)
    for step in (1, 2):
        o.set_f(S)
        g.set_f(S)
        np.testing.assert_array_equal(g.get_f() - W[:, None, None, None], shifted)
        o.step(1)
        g.step(1)
        fo = o.get_f()
        fg = g.get_f()
        so = fo - W[:, None, None, None]
        sg = fg - W[:, None, None, None]
        err = np.abs(sg - so)
        if storage == "f64":
            # the oracle rounds relative to |f| (unshifted), the GPU relative to
            # |f - w|: 16 FP64 ulps of the largest population
            bound = 16 * 2.0 ** -53 * np.max(np.abs(fo))
        else:
            # 1 ulp of T at the value + FP32 arithmetic slack (8 FP32 ulps of
            # the largest shifted population of the cell's direction)
            scale = np.max(np.abs(so), axis=(1, 2, 3), keepdims=True)
            bound = ulp(so, storage) + 8 * 2.0 ** -24 * scale
        worst = float(np.max(err / bound))
        print(storage, "step", step, "max err/bound", worst)
        assert worst <= 1.0
        # the state after the step is representable in T
        np.testing.assert_array_equal(round_storage(sg, storage), sg)


@pytest.mark.parametrize("storage,bounds", [
    ("f32", {"rho": 1e-6, "u": 2e-5, "nut": 1e-4}),
    ("f16s", {"rho": 1e-4, "u": 2e-3, "nut": 5e-2}),
    ("bf16s", {"rho": 1e-3, "u": 2e-2, "nut": 2e-1}),
    ("bf16sr", {"rho": 1e-3, "u": 2e-2, "nut": 2e-1}),
])
def test_low_precision_canopy_200_steps(storage, bounds):
    w = inputs.C1
    o, g = make_pair(w, storage=storage)
    o.step(w.steps)
    g.step(w.steps)
    err, do, dg = _compare_moments(o, g)
    print(storage, "64x32x32 200 steps normwise:", err)
    for k, b in bounds.items():
        assert err[k] <= b, (k, err[k], b)


def test_stats_match_oracle():
    w = inputs.scaled(inputs.C1, 40, 10, 6)
    o, g = make_pair(w, seed=3)
    for s in (o, g):
        s.stats_reset()
        s.stats_enable(3)
    o.step(20)
    g.step(11)
    g.step(9)
    po, no = o.stats_read()
    pg, ng = g.stats_read()
    assert no == ng == 6
    # means of signed quantities cancel: the tolerance is relative to the
    # largest value of each column
    atol = 1e-11 * np.max(np.abs(po), axis=0, keepdims=True)
    assert np.all(np.abs(pg - po) <= 1e-12 * np.abs(po) + atol)
    g.stats_reset()
    assert g.stats_read()[1] == 0


def test_checkpoint_roundtrip_is_bit_identical():
    w = inputs.scaled(inputs.C1, 48, 12, 8)
    _, a = make_pair(w, storage="f32", seed=9)
    _, b = make_pair(w, storage="f32", seed=9)
    a.step(21)
    b.step(10)
    f = b.get_f()
    b.set_f(f)
    b.step(11)
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    np.testing.assert_array_equal(a.moments()[1], b.moments()[1])


def test_tile_width_does_not_change_fp64_results(monkeypatch):
    """Tiles 64, 128 or 256 cells wide (covering 4, 2 or 1 z rows of a row
    j; 300x6x5 leaves the last z block ragged), with and without the XCD
    remap: bit-identical FP64 populations, and the plane statistics, which
    each tile sums over its cells, equal up to their FP64 summation order."""
    w = inputs.scaled(inputs.C1, 300, 6, 5)
    res, stats = [], []
    for bx in ("64", "128", "256"):
        monkeypatch.setenv("LBMX_BX", bx)
        for remap in ("0", "1"):
            monkeypatch.setenv("LBMX_XCD_REMAP", remap)
            _, g = make_pair(w, seed=4)
            g.stats_reset()
            g.stats_enable(3)
            g.step(12)
            res.append(g.get_f())
            stats.append(g.stats_read())
    for r in res[1:]:
        np.testing.assert_array_equal(r, res[0])
    for p, n in stats[1:]:
        assert n == stats[0][1] == 4
        np.testing.assert_allclose(p, stats[0][0], rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16sr"])
def test_buffer_and_64bit_addressing_agree(monkeypatch, storage):
    """The step addresses populations through one buffer resource (arrays
    below 4 GiB) or 64-bit pointers (larger arrays; forced here with
    LBMX_WIDE): bit-identical populations, both AA parities, walls."""
    w = inputs.scaled(inputs.C1, 70, 9, 6, canopy_rows=4)
    res = []
    for wide in ("0", "1"):
        monkeypatch.setenv("LBMX_WIDE", wide)
        _, g = make_pair(w, storage=storage, seed=7)
        g.step(7)
        res.append(g.get_f())
    np.testing.assert_array_equal(res[1], res[0])


@pytest.mark.parametrize("storage,nx", [("f32", 64), ("bf16sr", 128), ("f64", 70)])
def test_streaming_cache_policy_changes_nothing(monkeypatch, storage, nx):
    """Rows of whole 128-byte lines use non-temporal accesses (LBMX_STREAMING
    forces the policy on or off): a cache hint, so the populations are
    bit-identical, both AA parities, walls included."""
    w = inputs.scaled(inputs.C1, nx, 9, 6, canopy_rows=4)
    res = []
    for stream in ("0", "1"):
        monkeypatch.setenv("LBMX_STREAMING", stream)
        _, g = make_pair(w, storage=storage, seed=8)
        g.step(7)
        res.append(g.get_f())
    np.testing.assert_array_equal(res[1], res[0])


@pytest.mark.parametrize("storage,nx", [("f32", 70), ("bf16sr", 67), ("f16s", 100), ("f64", 35)])
def test_row_pitch_changes_nothing(monkeypatch, storage, nx):
    """Population rows padded to whole 128-byte lines (the default when a row
    is not; LBMX_PITCH=0 keeps them dense), and z-layers padded beyond px ny
    cells (LBMX_ZALIGN, LBMX_ZPAD), give bit-identical populations, moments
    and diagnostics, both AA parities, walls included; with the learned
    closure too."""
    from paper_2206_15454_amd import closure

    w = inputs.scaled(inputs.C1, nx, 9, 6, canopy_rows=4)
    blob = closure.timing_blob(10.0)
    res = []
    # dense, padded rows, padded rows in z-layers rounded to 4 KiB, dense
    # rows in z-layers widened by 384 B
    for pitch, zalign, zpad in (("0", "", ""), ("1", "", ""), ("1", "4096", ""), ("0", "", "384")):
        monkeypatch.setenv("LBMX_PITCH", pitch)
        monkeypatch.setenv("LBMX_ZALIGN", zalign)
        monkeypatch.setenv("LBMX_ZPAD", zpad)
        out = []
        for learned in (False, True):
            _, g = make_pair(w, storage=storage, seed=10)
            if learned:
                g.set_closure(blob)
            g.step(7)
            r, u, nt, d = g.moments()
            out.append((g.get_f(), r, u, nt, d["mass"], d["mlp_fallback"]))
            g.close()
        res.append(out)
    for other in res[1:]:
        for a, b in zip(res[0], other):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(np.asarray(y), np.asarray(x))


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16sr"])
def test_x_only_force_kernels_change_nothing(monkeypatch, storage):
    """With the driving force along x and x-only drag (F_y = F_z = 0), the
    step runs kernels that leave out the y and z force terms (LBMX_FX=0
    forces the general ones): bit-identical populations and moments, canopy
    rows and walls included, plain and learned closure."""
    from paper_2206_15454_amd import closure

    w = inputs.scaled(inputs.C1, 96, 12, 8, canopy_rows=5)
    blob = closure.timing_blob(10.0)
    res = []
    for fx in ("0", "1"):
        monkeypatch.setenv("LBMX_FX", fx)
        out = []
        for learned in (False, True):
            _, g = make_pair(w, storage=storage, seed=12)
            if learned:
                g.set_closure(blob)
            g.step(9)
            r, u, nt, d = g.moments()
            out.append((g.get_f(), r, u, nt, d["mass"], d["imp_x"]))
            g.close()
        res.append(out)
    for a, b in zip(res[0], res[1]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(np.asarray(y), np.asarray(x))


@pytest.mark.parametrize("storage", ["f32", "bf16sr"])
def test_tile_order_changes_nothing(monkeypatch, storage):
    """Row-major and memory-order tile numbering (LBMX_TILE_ORDER forces
    either) give bit-identical populations, walls included."""
    w = inputs.scaled(inputs.C1, 96, 7, 5, canopy_rows=3)
    res = []
    for order in ("0", "1"):
        monkeypatch.setenv("LBMX_TILE_ORDER", order)
        _, g = make_pair(w, storage=storage, seed=9)
        g.step(6)
        res.append(g.get_f())
    np.testing.assert_array_equal(res[1], res[0])


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16sr"])
def test_xcd_runs_change_nothing(monkeypatch, storage):
    """The XCDs taking turns in runs of 1, 2, 4 or 6 tiles (LBMX_XCD_RUN;
    the tiles past the last whole round keep their block), one contiguous
    range per XCD and no remap give bit-identical populations and moments,
    in both tile orders.  200x9x12 has 108 tiles: a run of 4 or 6 covers
    96 of them in whole rounds."""
    w = inputs.scaled(inputs.C1, 200, 9, 12, canopy_rows=3)
    res = []
    for order in ("0", "1"):
        for remap, run in (("1", ""), ("0", ""), ("1", "1"), ("1", "2"), ("1", "4"), ("1", "6")):
            monkeypatch.setenv("LBMX_TILE_ORDER", order)
            monkeypatch.setenv("LBMX_XCD_REMAP", remap)
            monkeypatch.setenv("LBMX_XCD_RUN", run)
            _, g = make_pair(w, storage=storage, seed=12)
            g.step(5)
            r, u, nt, d = g.moments()
            res.append((g.get_f(), r, u, nt))
            g.close()
    for other in res[1:]:
        for x, y in zip(res[0], other):
            np.testing.assert_array_equal(np.asarray(y), np.asarray(x))


def test_errors_and_state_machine():
    from paper_2206_15454_amd import lbm

    with pytest.raises(lbm.LBMError):
        lbm.LBM(8, 4, 4, "f32", tau0=0.5)
    with pytest.raises(lbm.LBMError):
        lbm.LBM(8, 4, 4, "f32", bc_lo="periodic", bc_hi="freeslip")
    g = lbm.LBM(8, 4, 4, "f32")
    with pytest.raises(lbm.LBMError) as e:
        g.step(1)
    assert e.value.status == 4  # ESTATE before init
    # zero steps change nothing; a negative count is invalid
    rho0 = 1.0 + 0.01 * np.arange(g.n).reshape(g.shape) / g.n
    u0 = np.full((3,) + g.shape, 0.01)
    g.init(rho0, u0)
    g.step(0)
    r, u, nt, d = g.moments()
    assert d["t"] == 0
    np.testing.assert_allclose(r, rho0, rtol=1e-6)
    np.testing.assert_allclose(u, u0, rtol=1e-5)
    with pytest.raises(lbm.LBMError) as e:
        g.step(-1)
    assert e.value.status == 1
    with pytest.raises(lbm.LBMError):
        g.set_canopy(0.2, np.zeros(3))
    with pytest.raises(lbm.LBMError):
        g.set_canopy(0.2, -np.ones(4))
    # an unstable state is reported and blocks further steps
    g.init(np.ones(g.shape), np.full((3,) + g.shape, 0.3))
    with pytest.raises(lbm.LBMError) as e:
        g.moments()
    assert e.value.status == 5
    with pytest.raises(lbm.LBMError) as e:
        g.step(1)
    assert e.value.status == 4


def test_momentum_balance_periodic_f32():
    """Fully periodic without canopy: sum(rho u) gains sum(F) per step; the
    FP64 impulse accumulator equals t * M * g."""
    w = inputs.scaled(inputs.C1, 64, 8, 8, bc_lo=0, bc_hi=0, canopy_rows=0,
                      g=(1e-5, 0.0, 0.0))
    _, g = make_pair(w, storage="f32", seed=2)
    g.step(1)
    d0 = g.diag()
    g.step(50)
    d1 = g.diag()
    M = d0["mass"]
    # each step rounds every stored population to FP32 (<= 2^-24 |f~| each,
    # |f~| <= 0.01 here): the momentum of 4096 cells can move by up to
    # 4096 * 18 * 2^-24 * 0.01 ~ 4.4e-5 per step if the roundings line up
    assert abs(d1["mom_x"] - d0["mom_x"] - 50 * M * 1e-5) <= 50 * 4.4e-5
    assert d1["imp_x"] == pytest.approx(51 * M * 1e-5, rel=1e-6)


def test_stochastic_rounding_is_unbiased():
    """BF16SR: one step from a stored state rounds each population to one of
    its two BF16 neighbours with zero-mean error (in units of the BF16 ulp),
    while round-to-nearest keeps the error within half an ulp."""
    w = inputs.scaled(inputs.C1, 128, 16, 8, canopy_rows=4)
    errs = {}
    for st in ("bf16s", "bf16sr"):
        o, g = make_pair(w, storage=st, init=False)
        S = inputs.random_populations(w.shape, seed=21, base=W, scale=0.02)
        S = round_storage(S - W[:, None, None, None], st) + W[:, None, None, None]
        o.set_f(S)
        g.set_f(S)
        o.step(1)
        g.step(1)
        so = o.get_f() - W[:, None, None, None]
        sg = g.get_f() - W[:, None, None, None]
        # only values well above the FP32 arithmetic error of the step (a few
        # 1e-9 absolute), so that the rounding into BF16 is what is measured
        big = np.abs(so) > 1e-5
        errs[st] = ((sg - so) / ulp(so, st))[big]
    e_rn, e_sr = errs["bf16s"], errs["bf16sr"]
    print("signed error in ulps: RN mean %.4f max %.3f; SR mean %.4f max %.3f std %.3f" % (
        e_rn.mean(), np.abs(e_rn).max(), e_sr.mean(), np.abs(e_sr).max(), e_sr.std()))
    assert np.abs(e_rn).max() <= 0.5 + 1e-3
    assert np.abs(e_sr).max() <= 1.0 + 1e-3
    assert abs(e_sr.mean()) <= 0.02
    assert 0.2 <= e_sr.std() <= 0.5  # stochastic: not always the nearest neighbour


def test_momentum_balance_periodic_f64():
    """FP64 storage, fully periodic without canopy: the momentum gains
    exactly M g per step (Guo forcing: the force enters half before and
    half after the collision) and the FP64 impulse accumulator holds
    (t + 1) M g after t steps; both to round-off."""
    w = inputs.scaled(inputs.C1, 64, 8, 8, bc_lo=0, bc_hi=0, canopy_rows=0,
                      g=(1e-5, -2e-6, 3e-6))
    _, g = make_pair(w, storage="f64", seed=2)
    g.step(1)
    d0 = g.diag()
    g.step(50)
    d1 = g.diag()
    M = d0["mass"]
    assert d1["mass"] == pytest.approx(M, rel=1e-14)
    for k, gk in zip(("mom_x", "mom_y", "mom_z"), w.g):
        dm = d1[k] - d0[k]
        print(k, "gain", dm, "expected", 50 * M * gk)
        assert dm == pytest.approx(50 * M * gk, rel=1e-12)
    for k, gk in zip(("imp_x", "imp_y", "imp_z"), w.g):
        assert d1[k] == pytest.approx(51 * M * gk, rel=1e-12)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_diagnostics_after_init_and_after_steps(storage):
    """lbm_moments reduces the moment planes after lbm_init and the step's
    per-wavefront records after steps: both equal the oracle's diagnostics
    (sums over the same moments), for a grid with a ragged tile tail."""
    w = inputs.scaled(inputs.C1, 300, 7, 5, canopy_rows=3)
    o, g = make_pair(w, storage=storage, seed=12)
    tol = 1e-13 if storage == "f64" else 1e-6
    for nsteps in (0, 1, 6):
        o.step(nsteps)
        g.step(nsteps)
        _, uo, _, do = o.moments()
        _, ug, _, dg = g.moments()
        print(storage, nsteps, {k: (do[k], dg[k]) for k in ("mass", "mom_x", "max_u")})
        assert dg["mass"] == pytest.approx(do["mass"], rel=tol)
        umax = np.max(np.abs(uo))
        for k in ("mom_x", "mom_y", "mom_z"):
            assert dg[k] == pytest.approx(do[k], rel=tol * 100, abs=tol * w.n * umax)
        assert dg["max_u"] == pytest.approx(do["max_u"], rel=tol * 10)
        assert dg["nonfinite"] == 0
        # the records reduce the moments the step wrote: the sums of those
        # moments on the host agree
        rg, ug2, _, _ = g.moments()
        assert dg["mass"] == pytest.approx(float(np.sum(rg)), rel=1e-13)
        assert dg["mom_x"] == pytest.approx(float(np.sum(rg * ug2[0])), rel=1e-12,
                                            abs=1e-15 * w.n)


def test_instability_found_from_the_step_records():
    """After steps the diagnostics come from the step's records: a speed
    above 0.35 and non-finite populations are both reported (EUNSTABLE) and
    the non-finite cells are counted."""
    from paper_2206_15454_amd import lbm

    w = inputs.scaled(inputs.C1, 64, 6, 4, bc_lo=0, bc_hi=0, canopy_rows=0)
    g = lbm.LBM(w.nx, w.ny, w.nz, "f32", w.tau0, w.c_smag, w.g, 0, 0)
    g.init(np.ones(g.shape), np.concatenate([np.full((1,) + g.shape, 0.4),
                                            np.zeros((2,) + g.shape)]))
    g.step(2)
    with pytest.raises(lbm.LBMError) as e:
        g.moments()
    assert e.value.status == 5
    rho, u, nut, d = g.moments(check=False)
    assert d["max_u"] > 0.35 and d["nonfinite"] == 0
    # NaN in one population of 3 cells: those cells (and their downstream
    # neighbours after streaming) are non-finite
    f = np.tile(W[:, None, None, None], (1,) + g.shape)
    f[1, 0, 0, :3] = np.nan
    g.set_f(f)
    g.step(1)
    rho, u, nut, d = g.moments(check=False)
    bad = ~(np.isfinite(rho) & np.isfinite(u).all(axis=0) & np.isfinite(nut))
    assert d["nonfinite"] == int(bad.sum()) and d["nonfinite"] >= 3
    assert np.isfinite(d["mass"])
    assert d["mass"] == pytest.approx(float(np.sum(rho[~bad])), rel=1e-12)
