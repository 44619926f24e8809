"""Pins of the oracle's learned closure (FP64 MLP forward/backward, blob).

The network is a design choice of this project (the paper uses Smagorinsky
and names other SGS models as future work), so the pins are mathematical:
known values of GELU/softplus, the composition on a one-path network (fixes
which index is input and which output), central finite differences of the
loss (fixes the backward pass), and the blob layout written here
independently with ``struct``.
"""
import math
import struct

import numpy as np
import pytest

from oracle import ref

NIN, NH1, NH2 = 9, 64, 64
NP = NH1 * NIN + NH1 + NH2 * NH1 + NH2 + NH2 + 1


def _bf16_bits(x):
    """Round-to-nearest-even float32 -> bfloat16 bits (test-local)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def _bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _blob(W1, b1, W2, b2, w3, b3, mean, std, lo, hi, scale, h):
    out = bytearray(b"LBMC")
    out += struct.pack("<5I", 1, NIN, NH1, NH2, 0)
    out += struct.pack("<36f", *mean, *std, *lo, *hi)
    out += struct.pack("<4f", scale, h, 0, 0)
    out += struct.pack("<132f", *b1, *b2, b3, 0, 0, 0)
    out += _bf16_bits(np.concatenate([W1.ravel(), W2.ravel(), w3.ravel()])).tobytes()
    assert len(out) == 10184
    return bytes(out)


def _flat(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def test_gelu_softplus_values():
    assert ref.gelu(0.0) == 0.0
    assert ref.gelu(10.0) == pytest.approx(10.0, abs=1e-12)
    assert abs(ref.gelu(-10.0)) < 1e-12
    for x in np.linspace(-4, 4, 33):
        exact = 0.5 * x * (1 + math.erf(x / math.sqrt(2)))  # GELU by definition
        assert abs(ref.gelu(x) - exact) < 5e-4  # tanh form approximates it
    assert ref.softplus(0.0) == pytest.approx(math.log(2.0), rel=1e-15)
    assert ref.softplus(50.0) == pytest.approx(50.0, rel=1e-15)
    assert ref.softplus(-50.0) == pytest.approx(math.exp(-50.0), rel=1e-12)
    assert ref.softplus(800.0) == 800.0


def test_one_path_network_fixes_indexing():
    W1 = np.zeros((NH1, NIN)); b1 = np.zeros(NH1)
    W2 = np.zeros((NH2, NH1)); b2 = np.zeros(NH2)
    w3 = np.zeros(NH2)
    a, bb, c, b3 = 0.7, -1.3, 2.1, 0.25
    W1[3, 5] = a   # hidden unit 3 reads input 5
    W2[7, 3] = bb  # hidden unit 7 of layer 2 reads unit 3 of layer 1
    w3[7] = c
    p = _flat(W1, b1, W2, b2, w3, b3)
    Z = np.random.default_rng(1).normal(size=(20, NIN))
    o = ref.mlp_apply(p, Z)
    expect = b3 + c * np.array([ref.gelu(bb * ref.gelu(a * z[5])) for z in Z])
    np.testing.assert_allclose(o, expect, rtol=1e-14, atol=1e-15)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = rng.normal(size=NP) * 0.3
    Z = rng.normal(size=(16, NIN))
    y = rng.uniform(0.1, 2.0, size=16)
    loss, g = ref.mlp_loss_grad(p, Z, y)
    o = ref.mlp_apply(p, Z)
    assert loss == pytest.approx(np.mean((np.log1p(np.exp(o)) - y) ** 2), rel=1e-13)
    idx = rng.choice(NP, size=120, replace=False)
    idx = np.concatenate([idx, [0, NP - 1, NH1 * NIN, NH1 * NIN + NH1]])
    def central(i, h):
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        return (ref.mlp_loss_grad(pp, Z, y)[0] - ref.mlp_loss_grad(pm, Z, y)[0]) / (2 * h)

    for i in idx:
        h = 1e-3 * max(1.0, abs(p[i]))
        fd = (4 * central(i, h / 2) - central(i, h)) / 3  # Richardson, O(h^4)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_blob_roundtrip_and_fallback():
    rng = np.random.default_rng(3)
    W1 = rng.normal(size=(NH1, NIN)) * 0.2; b1 = rng.normal(size=NH1) * 0.1
    W2 = rng.normal(size=(NH2, NH1)) * 0.1; b2 = rng.normal(size=NH2) * 0.1
    w3 = rng.normal(size=NH2) * 0.1; b3 = -1.0
    mean = rng.normal(size=NIN).astype(np.float32)
    std = rng.uniform(0.5, 2, size=NIN).astype(np.float32)
    lo = np.full(NIN, -5.0); hi = np.full(NIN, 5.0)
    blob = _blob(W1, b1, W2, b2, w3, b3, mean, std, lo, hi, 1e-4, 12.0)
    m = ref.MLP(blob)
    X = rng.uniform(-4, 4, size=(50, NIN))
    X[0, 2] = 7.0  # out of range -> Smagorinsky value
    smag = rng.uniform(0, 1e-4, 50)
    nut, fb = m.predict(X, smag)
    assert fb[0] == 1 and nut[0] == smag[0]
    assert fb[1:].sum() == 0
    # the same network from the BF16-rounded flat parameters
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    p = _flat(_bf16_value(_bf16_bits(W1)).reshape(W1.shape), f32(b1),
              _bf16_value(_bf16_bits(W2)).reshape(W2.shape), f32(b2),
              _bf16_value(_bf16_bits(w3)), float(np.float32(b3)))
    Zs = (X[1:] - mean.astype(np.float64)) / std.astype(np.float64)
    o = ref.mlp_apply(p, Zs)
    np.testing.assert_allclose(nut[1:], float(np.float32(1e-4)) * np.log1p(np.exp(o)),
                               rtol=1e-12)
    # the range test is taken in FP32: a feature just above an FP32 bound in
    # FP64 that rounds onto it is inside; one that rounds above it is outside
    top = float(np.float32(5.0))
    ulp32 = float(np.spacing(np.float32(5.0)))
    X2 = np.tile(X[1], (3, 1))
    X2[0, 4] = top + 0.25 * ulp32  # rounds to 5.0: in range
    X2[1, 4] = top + 0.75 * ulp32  # rounds to the next FP32 number: out
    X2[2, 4] = -top - 0.25 * ulp32  # rounds to -5.0: in range
    _, fb2 = m.predict(X2, smag[:3])
    assert fb2.tolist() == [0, 1, 0]
    with pytest.raises(ValueError):
        ref.MLP(blob[:-2])
    with pytest.raises(ValueError):
        ref.MLP(b"XXXX" + blob[4:])


def test_features_invariants():
    """Rotation about the wall normal leaves all stress features unchanged;
    tr P^2 = (Q^(1/2) / (rho c_s^2))^2."""
    rng = np.random.default_rng(4)
    blob = _blob(np.zeros((NH1, NIN)), np.zeros(NH1), np.zeros((NH2, NH1)), np.zeros(NH2),
                 np.zeros(NH2), 0.0, np.zeros(NIN), np.ones(NIN), -np.ones(NIN),
                 np.ones(NIN), 1.0, 12.0)
    m = ref.MLP(blob)
    A = rng.normal(size=(3, 3)) * 1e-3
    Pineq = A + A.T
    rho = 1.01
    x = m.features(0.5005, rho, Pineq, 0.3, 0.2)
    th = 0.7
    R = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0], [-math.sin(th), 0, math.cos(th)]])
    x2 = m.features(0.5005, rho, R @ Pineq @ R.T, 0.3, 0.2)
    np.testing.assert_allclose(x, x2, rtol=1e-12, atol=1e-18)
    Qh = math.sqrt(np.sum(Pineq * Pineq))
    assert x[5] == pytest.approx(Qh / (rho / 3), rel=1e-14)
    assert x[1] == pytest.approx((Qh / (rho / 3)) ** 2, rel=1e-14)
    assert x[0] == pytest.approx(np.trace(Pineq) / (rho / 3), rel=1e-14, abs=1e-18)
    assert tuple(x[6:]) == (0.3, 0.2, 1.0)


def _feature_mlp():
    blob = _blob(np.zeros((NH1, NIN)), np.zeros(NH1), np.zeros((NH2, NH1)), np.zeros(NH2),
                 np.zeros(NH2), 0.0, np.zeros(NIN), np.ones(NIN), -np.ones(NIN),
                 np.ones(NIN), 1.0, 12.0)
    return ref.MLP(blob)


@pytest.mark.parametrize("th", [0.0, 0.4, 1.1, 2.5])
def test_features_closed_form_from_eigenvalues(th):
    """P = Q diag(l) Q^T with Q a rotation about e_z (which moves e_y): tr P^k
    = sum l^k, and with (s, c) = (sin th, cos th) the second row of Q,
    n.P.n = l1 s^2 + l2 c^2 and n.P^2.n = l1^2 s^2 + l2^2 c^2.  A wrong
    index, a transposed factor, tr P tr P^2 for tr P^3 or (P_yy)^2 for
    (P^2)_yy fails one of these."""
    m = _feature_mlp()
    lam = np.array([3.0e-3, -1.2e-3, 0.7e-3])
    c, s = math.cos(th), math.sin(th)
    Q = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    P = Q @ np.diag(lam) @ Q.T
    rho = 0.97
    x = m.features(0.5005, rho, P * (rho / 3.0), 0.25, 0.1)
    scale = np.max(np.abs(lam))
    assert x[0] == pytest.approx(lam.sum(), abs=1e-15 * scale)
    assert x[1] == pytest.approx(np.sum(lam ** 2), rel=1e-13)
    assert x[2] == pytest.approx(np.sum(lam ** 3), rel=1e-12, abs=1e-15 * scale ** 3)
    assert x[3] == pytest.approx(lam[0] * s * s + lam[1] * c * c, abs=1e-15 * scale)
    assert x[4] == pytest.approx(lam[0] ** 2 * s * s + lam[1] ** 2 * c * c, rel=1e-12,
                                 abs=1e-15 * scale ** 2)
    assert x[5] == pytest.approx(math.sqrt(np.sum(lam ** 2)), rel=1e-13)


def test_features_newton_identity_and_column_norm():
    """Any symmetric P: tr P^3 = e1^3 - 3 e1 e2 + 3 e3 (Newton's identity with
    e1 = tr P, e2 = (e1^2 - tr P^2)/2, e3 = det P) and n.P^2.n = |P n|^2 =
    P_xy^2 + P_yy^2 + P_yz^2.  Off-diagonal-only tensors (xy and yz entries)
    and a traceless one (tr P^3 = 3 det P) are among the cases."""
    m = _feature_mlp()
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(20):
        A = rng.normal(size=(3, 3)) * 1e-3
        cases.append(A + A.T)
    cases.append(np.array([[0.0, 2e-3, 0.0], [2e-3, 0.0, -1e-3], [0.0, -1e-3, 0.0]]))
    T = rng.normal(size=(3, 3)) * 1e-3
    T = T + T.T
    cases.append(T - np.trace(T) / 3.0 * np.eye(3))
    for P in cases:
        rho = 1.02
        x = m.features(0.5005, rho, P * (rho / 3.0), 0.5, 0.0)
        e1 = np.trace(P)
        p2 = np.sum(P * P)
        e2 = 0.5 * (e1 * e1 - p2)
        e3 = np.linalg.det(P)
        scale3 = np.max(np.abs(P)) ** 3
        assert x[2] == pytest.approx(e1 ** 3 - 3 * e1 * e2 + 3 * e3, abs=1e-12 * scale3)
        assert x[4] == pytest.approx(P[0, 1] ** 2 + P[1, 1] ** 2 + P[1, 2] ** 2, rel=1e-13)
        if abs(e1) < 1e-18:
            assert x[2] == pytest.approx(3 * e3, abs=1e-12 * scale3)
    # the off-diagonal case: P^2 has (a^2 + b^2) at yy, its cube has zero trace
    x = m.features(0.5005, 1.0, cases[20] / 3.0, 0.5, 0.0)
    assert x[4] == pytest.approx(2e-3 ** 2 + 1e-3 ** 2, rel=1e-13)
    assert abs(x[2]) <= 1e-21


def _closure_sim(blob, every=None, seed=4):
    from paper_2206_15454_amd import inputs

    w = inputs.scaled(inputs.C1, 12, 8, 6, canopy_rows=3)
    s = ref.RefLBM(w.nx, w.ny, w.nz, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi)
    s.set_canopy(w.cd, inputs.lad_constant(w))
    m = ref.MLP(blob)
    s.set_closure(m)
    s._keep = m
    if every is not None:
        s.set_closure_interval(every)
    rho, u = inputs.init_fields(w, seed)
    s.init(rho, 5 * u)
    return s


def _random_blob(rng, lo, hi, w3_scale=0.1):
    W1 = rng.normal(size=(NH1, NIN)) * 0.2; b1 = rng.normal(size=NH1) * 0.1
    W2 = rng.normal(size=(NH2, NH1)) * 0.1; b2 = rng.normal(size=NH2) * 0.1
    w3 = rng.normal(size=NH2) * w3_scale
    mean = np.zeros(NIN, dtype=np.float32)
    std = np.array([1e-3, 1e-6, 1e-9, 1e-3, 1e-6, 1e-3, 1.0, 0.1, 1.0], dtype=np.float32)
    return _blob(W1, b1, W2, b2, w3, -1.0, mean, std, lo, hi, 2e-3, 3.0)


def test_closure_interval_reuses_the_last_evaluation():
    """Evaluated every 3 steps: nu_t stays, cell by cell, that of the last
    evaluation; interval 1 is the plain per-step closure; the first step after
    set-up, set_f or a new interval always evaluates."""
    rng = np.random.default_rng(8)
    # feature 7 (LAD) above 0.1 falls back: the canopy rows use Smagorinsky
    hi = np.full(NIN, 1e30); hi[7] = 0.1
    blob = _random_blob(rng, np.full(NIN, -1e30), hi)
    a, b, c = _closure_sim(blob), _closure_sim(blob, 1), _closure_sim(blob, 3)
    nut = {}
    for t in range(1, 7):
        for s in (a, b, c):
            s.step(1)
        ra, ua, na, da = a.moments()
        rb, ub, nb, db = b.moments()
        _, uc, nc, dc = c.moments()
        np.testing.assert_array_equal(ub, ua)
        np.testing.assert_array_equal(nb, na)
        nut[t] = nc
        if t == 1:
            np.testing.assert_array_equal(nc, na)
            np.testing.assert_array_equal(uc, ua)
        # the fallback count is that of the last evaluation (the canopy rows)
        assert dc["mlp_fallback"] == da["mlp_fallback"] == 12 * 3 * 6
    np.testing.assert_array_equal(nut[2], nut[1])
    np.testing.assert_array_equal(nut[3], nut[1])
    assert np.max(np.abs(nut[4] - nut[3])) > 0  # re-evaluated at step 4
    np.testing.assert_array_equal(nut[6], nut[4])
    # set_f: the next step evaluates again
    c.set_f(c.get_f())
    c.step(1)
    assert np.max(np.abs(c.moments()[2] - nut[6])) > 0


def test_closure_interval_with_a_constant_network_changes_nothing():
    """A network whose output does not depend on its input (w3 = 0) gives the
    same nu_t in every cell at every step, so reusing it is exact."""
    rng = np.random.default_rng(9)
    blob = _random_blob(rng, np.full(NIN, -1e30), np.full(NIN, 1e30), w3_scale=0.0)
    a, c = _closure_sim(blob), _closure_sim(blob, 4)
    a.step(9)
    c.step(9)
    _, ua, na, _ = a.moments()
    _, uc, nc, _ = c.moments()
    assert np.ptp(na) == 0 and na.flat[0] > 0
    np.testing.assert_array_equal(uc, ua)
    np.testing.assert_array_equal(nc, na)
    with pytest.raises(ValueError):
        c.set_closure_interval(0)


def test_closure_with_range_keeps_the_network():
    """closure.with_range changes one feature's range and nothing else; the
    oracle then falls back exactly where that feature leaves it."""
    from paper_2206_15454_amd import closure

    rng = np.random.default_rng(11)
    blob = _random_blob(rng, np.full(NIN, -1e30), np.full(NIN, 1e30))
    low = closure.with_range(blob, "y_over_h", hi=4.0)
    assert len(low) == len(blob)
    p0, m0, s0, lo0, hi0, sc0, h0 = closure.read_blob(blob)
    p1, m1, s1, lo1, hi1, sc1, h1 = closure.read_blob(low)
    np.testing.assert_array_equal(p0, p1)
    np.testing.assert_array_equal(lo0, lo1)
    assert hi1[6] == 4.0 and np.all(np.delete(hi1, 6) == np.delete(hi0, 6))
    X = rng.normal(size=(40, NIN)) * 1e-3
    X[:, 6] = np.linspace(0.1, 8.0, 40)
    smag = np.full(40, 7e-5)
    n0, f0 = ref.MLP(blob).predict(X, smag)
    n1, f1 = ref.MLP(low).predict(X, smag)
    above = X[:, 6] > 4.0
    assert np.all(f1 == above) and not f0.any()
    np.testing.assert_array_equal(n1[~above], n0[~above])
    np.testing.assert_array_equal(n1[above], smag[above])
