"""Learned closure in the fused step (MFMA inference) against the oracle.

Tolerance: the GPU evaluates the network with BF16 operands (inputs and
hidden activations rounded to 8 significant bits) and FP32 accumulation; the
oracle evaluates the same BF16-rounded weights in FP64 on unrounded inputs.
Each rounding is <= 2^-9 relative; through two layers and the softplus this
bounds the error of nu_t by a few percent of its scale: the tests use 3e-2
of max |nu_t| (one step).  Where the closure falls back, nu_t is the
Smagorinsky value and follows the FP64 bound.
"""
import numpy as np
import pytest

from oracle import ref
from paper_2206_15454_amd import closure, inputs
from tests.gpu_common import make_pair, normwise, oracle_lad, require_gpu, round_storage, ulp

pytestmark = pytest.mark.gpu

MEAN = np.array([0, 0, 0, 0, 0, 1e-3, 1.5, 0.1, 1.0])
STD = np.array([1e-4, 1e-6, 1e-9, 1e-3, 1e-6, 1e-3, 1.0, 0.15, 1.0])


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def random_params(seed):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(64, 9)) / 3.0
    b1 = rng.normal(size=64) * 0.1
    W2 = rng.normal(size=(64, 64)) / 8.0
    b2 = rng.normal(size=64) * 0.1
    w3 = rng.normal(size=64) / 8.0
    return closure.join(W1, b1, W2, b2, w3, -0.5)


def blob_with_range(lo, hi, seed=1, scale=1e-4, h=10.0):
    return closure.make_blob(random_params(seed), MEAN, STD, lo, hi, scale, h)


_, W_ = ref.lattice()
WIDE_LO = np.full(9, -1e30)
WIDE_HI = np.full(9, 1e30)


def test_blob_validation():
    from paper_2206_15454_amd import lbm

    g = lbm.LBM(16, 4, 4, "f32")
    good = blob_with_range(WIDE_LO, WIDE_HI)
    g.set_closure(good)
    for bad in (good[:-1], b"XXXX" + good[4:], good[:4] + b"\x02" + good[5:]):
        with pytest.raises(lbm.LBMError):
            g.set_closure(bad)
    std0 = closure.make_blob(random_params(1), MEAN, np.zeros(9), WIDE_LO, WIDE_HI, 1e-4, 10.0)
    with pytest.raises(lbm.LBMError):
        g.set_closure(std0)
    g.set_closure(None)


@pytest.mark.parametrize("storage", ["f32", "bf16s"])
def test_all_fallback_equals_smagorinsky_bitwise(storage):
    w = inputs.scaled(inputs.C1, 96, 12, 8)
    _, a = make_pair(w, storage=storage, seed=2)
    _, b = make_pair(w, storage=storage, seed=2)
    lo = WIDE_LO.copy()
    hi = WIDE_HI.copy()
    lo[8], hi[8] = 2.0, 3.0  # the width feature is 1: every cell is out of range
    b.set_closure(blob_with_range(lo, hi))
    a.step(15)
    b.step(15)
    # the populations (which carry the dynamics) are bit-identical
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    ra, ua, na, da = a.moments()
    rb, ub, nb, db = b.moments()
    np.testing.assert_array_equal(ua, ub)
    # the FP32 nu_t output may differ in its last bit (instruction selection
    # differs between the two kernels; tau and everything after it agree)
    assert np.max(np.abs(na - nb) / np.maximum(np.abs(nb), 1e-30)) <= 2 * 2.0 ** -23
    assert db["mlp_fallback"] == w.n and da["mlp_fallback"] == 0


def test_learned_closure_matches_oracle():
    w = inputs.scaled(inputs.C1, 48, 16, 8, canopy_rows=5)
    o, g = make_pair(w, storage="f64", seed=6)
    lo = WIDE_LO.copy()
    hi = WIDE_HI.copy()
    hi[7] = 0.15  # LAD above 0.15: the canopy rows fall back to Smagorinsky
    blob = blob_with_range(lo, hi, seed=3)
    m = ref.MLP(blob)
    o.set_closure(m)
    g.set_closure(blob)
    o.step(1)
    g.step(1)
    ro, uo, no, do = o.moments()
    rg, ug, ng, dg = g.moments()
    canopy = np.zeros(w.shape, dtype=bool)
    canopy[:, :5, :] = True
    assert do["mlp_fallback"] == dg["mlp_fallback"] == canopy.sum()
    # fallback rows: Smagorinsky in FP64
    assert normwise(ng[canopy], no[canopy]) <= 1e-12
    # learned rows: BF16 operands
    e_mlp = normwise(ng[~canopy], no[~canopy])
    print("learned nu_t normwise error after 1 step:", e_mlp, "max nu_t", no[~canopy].max())
    assert e_mlp <= 3e-2
    assert normwise(ug, uo) <= 1e-6
    # a few more steps stay close
    o.step(9)
    g.step(9)
    ro, uo, no, do = o.moments()
    rg, ug, ng, dg = g.moments()
    print("after 10 steps: u", normwise(ug, uo), "nu_t", normwise(ng, no))
    assert normwise(ug, uo) <= 1e-5
    assert normwise(ng, no) <= 5e-2


def test_learned_closure_persistent_walk_matches_oracle():
    """More tiles than the persistent kernel has blocks (256x64x32: 2048
    tiles of 256 cells), so each block walks several tiles; the closure is
    restricted to y/h <= 2, so the wavefronts of the upper rows skip the
    network and fall back to Smagorinsky."""
    w = inputs.scaled(inputs.C1, 256, 64, 32, canopy_rows=12)
    o, g = make_pair(w, storage="f64", seed=11)
    hi = WIDE_HI.copy()
    hi[6] = 2.0  # y/h = (j + 1/2) / 10: rows j >= 20 fall back
    blob = blob_with_range(WIDE_LO.copy(), hi, seed=5)
    o.set_closure(ref.MLP(blob))
    g.set_closure(blob)
    o.step(1)
    g.step(1)
    _, uo, no, do = o.moments()
    _, ug, ng, dg = g.moments()
    upper = np.zeros(w.shape, dtype=bool)
    upper[:, 20:, :] = True
    assert do["mlp_fallback"] == dg["mlp_fallback"] == upper.sum()
    assert normwise(ng[upper], no[upper]) <= 1e-12
    e_mlp = normwise(ng[~upper], no[~upper])
    print("persistent walk: learned nu_t normwise error", e_mlp)
    assert e_mlp <= 3e-2
    assert normwise(ug, uo) <= 1e-6


def test_closure_interval_matches_oracle():
    """Learned closure evaluated every 3 steps: the steps in between reuse
    the nu_t of the last evaluation, on the GPU as in the oracle."""
    w = inputs.scaled(inputs.C1, 48, 16, 8, canopy_rows=5)
    o, g = make_pair(w, storage="f64", seed=6)
    hi = WIDE_HI.copy()
    hi[7] = 0.15  # canopy rows fall back to Smagorinsky
    blob = blob_with_range(WIDE_LO.copy(), hi, seed=3)
    m = ref.MLP(blob)
    o.set_closure(m)
    g.set_closure(blob)
    o.set_closure_interval(3)
    g.set_closure_interval(3)
    nut = {}
    for t in range(1, 8):
        o.step(1)
        g.step(1)
        _, uo, no, do = o.moments()
        _, ug, ng, dg = g.moments()
        nut[t] = ng
        assert do["mlp_fallback"] == dg["mlp_fallback"] == 48 * 5 * 8
        assert normwise(ng, no) <= 5e-2 and normwise(ug, uo) <= 1e-5, t
    np.testing.assert_array_equal(nut[2], nut[1])
    np.testing.assert_array_equal(nut[3], nut[1])
    np.testing.assert_array_equal(nut[6], nut[4])
    assert np.max(np.abs(nut[4] - nut[3])) > 0


@pytest.mark.parametrize("storage", ["f32", "bf16sr"])
def test_closure_interval_with_a_constant_network_is_exact(storage):
    """With a network whose output does not depend on its input, reusing its
    nu_t changes nothing: populations bit-identical to evaluating every step;
    interval 1 is the default."""
    p = random_params(4)
    p[-65:-1] = 0.0  # w3 = 0: the output is softplus(b3)
    blob = closure.make_blob(p, MEAN, STD, WIDE_LO, WIDE_HI, 1e-4, 10.0)
    w = inputs.scaled(inputs.C1, 64, 12, 8)
    sims = []
    for every in (None, 1, 5):
        _, g = make_pair(w, storage=storage, seed=3)
        g.set_closure(blob)
        if every is not None:
            g.set_closure_interval(every)
        g.step(12)
        sims.append(g)
    f0 = sims[0].get_f()
    np.testing.assert_array_equal(sims[1].get_f(), f0)
    np.testing.assert_array_equal(sims[2].get_f(), f0)
    from paper_2206_15454_amd import lbm

    with pytest.raises(lbm.LBMError):
        sims[2].set_closure_interval(0)


# the 200-step bounds of the Smagorinsky step per storage type (the
# low-precision parity tests): the learned runs below stay within them
STEP_BOUNDS = {"f32": {"rho": 1e-6, "u": 2e-5}, "f16s": {"rho": 1e-4, "u": 2e-3},
               "bf16s": {"rho": 1e-3, "u": 2e-2}, "bf16sr": {"rho": 1e-3, "u": 2e-2}}


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s", "bf16sr"])
def test_learned_closure_each_storage_matches_oracle(storage):
    """The learned-closure kernel in every reduced-precision storage type,
    at the 512-wide launch shape (256-wide tiles, streaming rows), against
    the oracle.  The stored state S is physical: the oracle's own state
    after 3 steps from the seeded start, rounded into the storage type (so
    that the network's standardised inputs lie where it was set up).  From
    S, one step in each AA parity; then ten steps.

    Bounds (one step): rho and u as the plain step from a stored state (both
    sides decode the same S; the GPU adds FP32 arithmetic); nu_t within 3e-2
    of its largest value where the network runs (the FP64-storage bound;
    measured there 3.3e-3) and at FP32 Smagorinsky precision (1e-3) in the
    rows that fall back; the populations within 1 ulp of the storage type
    plus 8 FP32 ulps of their direction's largest value plus the effect of
    the nu_t bound on the relaxation, |f - f_eq| * 3 dnu / tau^2 with
    |f - f_eq| <= 2 max|f~|."""
    W4 = W_[:, None, None, None]
    w = inputs.scaled(inputs.C1, 512, 12, 8, canopy_rows=5)
    o, g = make_pair(w, storage=storage, seed=6)
    o.step(3)
    shifted = round_storage(o.get_f() - W4, storage)
    S = shifted + W4
    hi = WIDE_HI.copy()
    hi[7] = 0.15  # LAD above 0.15: the canopy rows fall back to Smagorinsky
    blob = blob_with_range(WIDE_LO.copy(), hi, seed=3)
    o.set_closure(ref.MLP(blob))
    g.set_closure(blob)
    canopy = np.zeros(w.shape, dtype=bool)
    canopy[:, :5, :] = True
    for parity in (0, 1):
        o.set_f(S)
        g.set_f(S)
        o.step(1)
        g.step(1)
        ro, uo, no, do = o.moments()
        rg, ug, ng, dg = g.moments()
        assert do["mlp_fallback"] == dg["mlp_fallback"] == canopy.sum()
        e = {"rho": normwise(rg, ro), "u": normwise(ug, uo),
             "nut_fallback": normwise(ng[canopy], no[canopy]),
             "nut_learned": normwise(ng[~canopy], no[~canopy])}
        print(storage, "parity", parity, e, "max nu_t", no.max())
        assert e["rho"] <= 1e-6 and e["u"] <= 1e-5
        assert e["nut_fallback"] <= 1e-3
        assert e["nut_learned"] <= 3e-2
        so = o.get_f() - W4
        sg = g.get_f() - W4
        dnu = 3e-2 * np.max(np.abs(no))
        relax = 2 * np.max(np.abs(shifted)) * 3 * dnu / w.tau0 ** 2
        scale = np.max(np.abs(so), axis=(1, 2, 3), keepdims=True)
        bound = ulp(so, storage) + 8 * 2.0 ** -24 * scale + relax
        worst = float(np.max(np.abs(sg - so) / bound))
        print(storage, "parity", parity, "populations: max err/bound", worst)
        assert worst <= 1.0
        np.testing.assert_array_equal(round_storage(sg, storage), sg)
    # Ten steps from S (the GPU continues from its own rounded states).  The
    # states of the two sides then differ by ten steps of storage rounding,
    # which the network may amplify without limit (its standardised inputs
    # include tr Pi^3 on a 1e-9 scale), so its 10-step nu_t difference is
    # reported, not bounded.  What is bounded: rho and u by the 200-step
    # bounds of the Smagorinsky step in this storage, and the tenth step
    # itself, taken by both sides from the GPU's own state after nine steps
    # (that state is representable in the storage type), by the one-step
    # bounds above: the kernel stays consistent with the oracle along its
    # own trajectory.
    o.set_f(S)
    g.set_f(S)
    o.step(10)
    g.step(9)
    G9 = g.get_f()
    g.step(1)
    ro, uo, no, do = o.moments()
    rg, ug, ng, dg = g.moments()
    e = {"rho": normwise(rg, ro), "u": normwise(ug, uo), "nut": normwise(ng, no)}
    assert e["rho"] <= STEP_BOUNDS[storage]["rho"]
    assert e["u"] <= max(STEP_BOUNDS[storage]["u"], 1e-5)
    oc = ref.RefLBM(w.nx, w.ny, w.nz, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi)
    oc.set_wall_velocity(w.u_wall)
    oc.set_canopy(w.cd, oracle_lad(w))
    oc.set_closure(ref.MLP(blob))
    oc.set_f(G9)
    oc.step(1)
    r1, u1, n1, d1 = oc.moments()
    e1 = {"rho": normwise(rg, r1), "u": normwise(ug, u1),
          "nut_fallback": normwise(ng[canopy], n1[canopy]),
          "nut_learned": normwise(ng[~canopy], n1[~canopy])}
    print(storage, "10 steps from S:", e, "; step 10 from the GPU's state:", e1)
    assert d1["mlp_fallback"] == dg["mlp_fallback"]
    assert e1["rho"] <= 1e-6 and e1["u"] <= 1e-5
    assert e1["nut_fallback"] <= 1e-3
    assert e1["nut_learned"] <= 3e-2


def test_learned_kernel_statistics_equal_plain_when_every_cell_falls_back():
    """The persistent learned-closure kernel accumulates the plane
    statistics through the block's shared staging area once per tile; with
    more tiles than blocks (512x64x32: 4096 tiles), and every cell falling
    back to Smagorinsky, its statistics equal the plain kernel's: the
    velocity columns bit for bit (identical populations, identical
    accumulation order), the nu_t column to its FP32 last bits."""
    w = inputs.scaled(inputs.C1, 512, 64, 32, canopy_rows=12)
    _, a = make_pair(w, storage="f32", seed=2)
    _, b = make_pair(w, storage="f32", seed=2)
    lo = WIDE_LO.copy()
    hi = WIDE_HI.copy()
    lo[8], hi[8] = 2.0, 3.0  # the width feature is 1: every cell is out of range
    b.set_closure(blob_with_range(lo, hi))
    for sim in (a, b):
        sim.stats_reset()
        sim.stats_enable(2)
        sim.step(8)
    pa, na = a.stats_read()
    pb, nb = b.stats_read()
    assert na == nb == 4
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    np.testing.assert_array_equal(pb[:, :9], pa[:, :9])
    assert np.max(np.abs(pb[:, 9] - pa[:, 9]) / np.maximum(np.abs(pa[:, 9]), 1e-30)) <= 1e-6


@pytest.mark.parametrize("storage,every,yh_lo", [("f32", 1, None), ("bf16sr", 1, None),
                                                 ("bf16sr", 3, None), ("f16s", 1, 1.0)])
def test_row_split_of_the_canopy_layer_closure_changes_nothing(monkeypatch, storage, every, yh_lo):
    """The trained network restricted to the canopy layer (y/h <= 4 through
    its feature range) on 128x64x16, h = 12: the evaluating steps run the
    learned kernel on the rows whose y/h is in range and the plain step on
    the rows above, whose cells would all fall back (LBMX_MLP_SPLIT=0: one
    learned launch over every row), in turn on one stream or with the plain
    rows on the library's second stream beside the network's kernel
    (LBMX_MLP_OVERLAP=2, the default).  Populations, moments, nu_t and the
    fallback count are bit for bit the same, every step and with the
    network every 3rd step, and with the range starting at y/h = 1 (plain
    rows below and above the network's); the plane statistics and FP64 diagnostics agree
    up to their summation order (the impulse of the plain rows is summed per
    wave in FP32 instead of per thread in FP64)."""
    w = inputs.scaled(inputs.C2, 128, 64, 16)
    blob = closure.canopy_layer_blob()
    if yh_lo is not None:  # rows below the range too: plain launches on both sides
        blob = closure.with_range(blob, "y_over_h", lo=yh_lo)
    runs = []
    # (split, overlap): one learned launch; the split in turn on one stream;
    # the split with the plain rows on the second stream beside the network
    for split, overlap in (("0", "0"), ("1", "0"), ("1", "2")):
        monkeypatch.setenv("LBMX_MLP_SPLIT", split)
        monkeypatch.setenv("LBMX_MLP_OVERLAP", overlap)
        _, g = make_pair(w, storage=storage, seed=14)
        g.set_closure(blob)
        g.set_closure_interval(every)
        g.stats_reset()
        g.stats_enable(2)
        g.step(9)
        runs.append((g.get_f(), g.moments(), g.stats_read()))
        g.close()
    (f0, m0, (p0, n0)) = runs[0]
    for f1, m1, (p1, n1) in runs[1:]:
        np.testing.assert_array_equal(f1, f0)
        for x, y in zip(m0[:3], m1[:3]):
            np.testing.assert_array_equal(np.asarray(y), np.asarray(x))
        assert m1[3]["mlp_fallback"] == m0[3]["mlp_fallback"] > 0
        for key, v in m0[3].items():
            rtol = 1e-5 if key.startswith("imp") and storage != "f64" else 1e-12
            np.testing.assert_allclose(m1[3][key], v, rtol=rtol, atol=1e-300)
        assert n0 == n1 == 4
        np.testing.assert_allclose(p1, p0, rtol=1e-12, atol=1e-18)
    # the two split runs differ only in the streams: bit for bit the same
    # diagnostics and statistics as well
    (_, ma, (pa, _)), (_, mb, (pb, _)) = runs[1], runs[2]
    assert ma[3] == mb[3]
    np.testing.assert_array_equal(pb, pa)
