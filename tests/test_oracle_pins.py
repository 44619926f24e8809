"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: lattice
isotropy, exact moment identities of the equilibrium and of the Guo force,
the physical derivation behind the Smagorinsky closed form, particle
kinematics of streaming and walls, conservation laws, a scalar recurrence,
the Poiseuille closed form, and Taylor-Green viscous decay.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import ref

BB, FS, PER = ref.BC_BOUNCEBACK, ref.BC_FREESLIP, ref.BC_PERIODIC


# ---------------------------------------------------------------------------
# lattice (D3Q19; the paper names the lattice, the tables are standard)
# ---------------------------------------------------------------------------

def test_lattice_isotropy():
    c, w = ref.lattice()
    assert c.shape == (19, 3)
    assert len({tuple(v) for v in c}) == 19
    assert abs(w.sum() - 1.0) < 1e-15
    # isotropy up to 4th order with c_s^2 = 1/3
    for a in range(3):
        assert abs((w * c[:, a]).sum()) < 1e-16
        for b in range(3):
            m2 = (w * c[:, a] * c[:, b]).sum()
            assert abs(m2 - (1.0 / 3.0) * (a == b)) < 1e-15
            for g in range(3):
                assert abs((w * c[:, a] * c[:, b] * c[:, g]).sum()) < 1e-16
                for d in range(3):
                    m4 = (w * c[:, a] * c[:, b] * c[:, g] * c[:, d]).sum()
                    iso = ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g)) / 9.0
                    assert abs(m4 - iso) < 1e-15


def test_lattice_interface_order():
    """Direction order of the interface: rest, +x -x +y -y +z -z, then the
    twelve edge vectors, each immediately followed by its opposite."""
    c, w = ref.lattice()
    assert tuple(c[0]) == (0, 0, 0)
    axis = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    assert [tuple(v) for v in c[1:7]] == axis
    for q in range(1, 19, 2):
        assert tuple(c[q + 1]) == tuple(-c[q])
    assert all(np.abs(c[7:]).sum(axis=1) == 2)
    np.testing.assert_array_equal(w, [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


# ---------------------------------------------------------------------------
# equilibrium and Guo forcing: exact moment identities
# ---------------------------------------------------------------------------

def _random_states(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = rng.uniform(0.9, 1.1)
        u = rng.uniform(-1, 1, 3)
        u *= rng.uniform(0, 0.1) / np.linalg.norm(u)
        yield rho, u


def test_equilibrium_moments():
    c, w = ref.lattice()
    for rho, u in _random_states(50, 11):
        f = ref.feq(rho, u)
        assert abs(f.sum() - rho) < 1e-15
        np.testing.assert_allclose(c.T @ f, rho * u, rtol=0, atol=1e-16)
        Pi = np.einsum("q,qa,qb->ab", f, c, c)
        np.testing.assert_allclose(Pi, rho / 3 * np.eye(3) + rho * np.outer(u, u), rtol=0,
                                   atol=1e-15)


def test_equilibrium_rest_is_weights():
    _, w = ref.lattice()
    np.testing.assert_allclose(ref.feq(1.0, np.zeros(3)), w, rtol=0, atol=1e-17)
    np.testing.assert_allclose(ref.feq(1.7, np.zeros(3)), 1.7 * w, rtol=0, atol=1e-16)


def test_guo_moments():
    c, _ = ref.lattice()
    rng = np.random.default_rng(12)
    for rho, u in _random_states(50, 13):
        tau = rng.uniform(0.5005, 2.0)
        F = rng.uniform(-1e-3, 1e-3, 3)
        Fi = ref.guo(tau, u, F)
        k = 1.0 - 1.0 / (2.0 * tau)
        assert abs(Fi.sum()) < 1e-18
        np.testing.assert_allclose(c.T @ Fi, k * F, rtol=0, atol=1e-18)
        M2 = np.einsum("q,qa,qb->ab", Fi, c, c)
        np.testing.assert_allclose(M2, k * (np.outer(u, F) + np.outer(F, u)), rtol=0, atol=1e-18)


def test_moments_of_sums():
    c, _ = ref.lattice()
    f = np.random.default_rng(3).uniform(0, 0.1, 19)
    rho, j, Pi = ref.moments_of(f)
    assert rho == pytest.approx(f.sum(), abs=1e-16)
    np.testing.assert_allclose(j, c.T @ f, atol=1e-16)
    np.testing.assert_allclose(Pi, np.einsum("q,qa,qb->ab", f, c, c), atol=1e-16)


# ---------------------------------------------------------------------------
# Smagorinsky closure (Sec. 2.2)
# ---------------------------------------------------------------------------

def test_smagorinsky_zero_stress_gives_tau0():
    for tau0 in (0.5005, 0.52, 0.8, 1.3):
        tau, nut = ref.smag(tau0, 0.01, 1.03, np.zeros((3, 3)))
        assert tau == tau0 and nut == 0.0
    tau, nut = ref.smag(0.6, 0.0, 1.0, np.ones((3, 3)) * 1e-3)
    assert tau == 0.6 and nut == 0.0


def test_smagorinsky_physical_consistency():
    """With Pi_neq = -2 rho c_s^2 tau S for a strain S (Chapman-Enskog) and
    tau = tau0 + 3 C |S|, |S| = sqrt(2 S:S), the closure must return exactly
    nu_t = C |S| -- this fixes both the 18 sqrt(2) constant and the root."""
    rng = np.random.default_rng(5)
    for _ in range(40):
        tau0 = rng.uniform(0.5005, 1.0)
        C = rng.uniform(0.005, 0.04)
        rho = rng.uniform(0.95, 1.05)
        A = rng.normal(size=(3, 3)) * 10 ** rng.uniform(-5, -2)
        S = 0.5 * (A + A.T)
        S -= np.trace(S) / 3 * np.eye(3)
        Smag = math.sqrt(2.0 * np.sum(S * S))
        tau = tau0 + 3.0 * C * Smag
        Pineq = -2.0 * rho / 3.0 * tau * S
        tau_o, nut_o = ref.smag(tau0, C, rho, Pineq)
        assert nut_o == pytest.approx(C * Smag, rel=1e-12)
        assert tau_o == pytest.approx(tau, rel=1e-14)


def test_smagorinsky_quadratic_and_monotone():
    rng = np.random.default_rng(6)
    prev = None
    base = rng.normal(size=(3, 3))
    base = base + base.T
    for s in np.geomspace(1e-8, 1e-2, 30):
        tau0, C, rho = 0.5005, 0.01, 1.02
        Pineq = s * base
        tau, nut = ref.smag(tau0, C, rho, Pineq)
        Sabs = nut / C
        Qh = math.sqrt(np.sum(Pineq * Pineq))
        resid = 3 * C * Sabs ** 2 + tau0 * Sabs - 3 * Qh / (math.sqrt(2) * rho)
        assert abs(resid) <= 1e-14 * (3 * Qh / (math.sqrt(2) * rho)) + 1e-24
        if prev is not None:
            assert tau > prev
        prev = tau


# ---------------------------------------------------------------------------
# LAD profile, Eq. (af_theory)
# ---------------------------------------------------------------------------

def test_lad_peak_branches_and_normalisation():
    h, ym, afm = 10.0, 6.5, 0.38
    ny = 16
    a = ref.lad_lalic(h, ym, ny, afm=afm)
    y = np.arange(ny) + 0.5
    assert a[6] == pytest.approx(afm, rel=1e-15)  # y = 6.5 = y_m
    assert np.all(a[y >= h] == 0.0)
    assert np.all(a <= afm * (1 + 1e-15))
    assert np.argmax(a) == 6
    # recover the exponent n from the values: ln(a/afm) = n (ln r + 1 - r)
    for j in range(ny):
        if y[j] >= h or y[j] == ym:
            continue
        r = (h - ym) / (h - y[j])
        n = math.log(a[j] / afm) / (math.log(r) + 1 - r)
        assert n == pytest.approx(6.0 if y[j] < ym else 0.5, rel=1e-10)
    b = ref.lad_lalic(12.0, 8.4, 128, lai=2.0)
    assert b.sum() == pytest.approx(2.0, rel=1e-14)
    assert np.all(b[12:] == 0) and np.all(b[:12] > 0)
    assert np.argmax(b) == 8  # cell centre 8.5 nearest to y_m = 8.4
    # the continuous profile -> 0 as y -> h from below
    c = ref.lad_lalic(1000.0, 700.0, 1000, afm=1.0)
    assert c[999] < 0.05 and c[990] > c[999]


def test_lad_rejects_bad_parameters():
    with pytest.raises(ValueError):
        ref.lad_lalic(10.0, 12.0, 8)
    with pytest.raises(ValueError):
        ref.lad_lalic(-1.0, 0.5, 8)


# ---------------------------------------------------------------------------
# streaming and walls: particle kinematics, brute force on tiny grids
# ---------------------------------------------------------------------------

def _landing(c, q, i, j, k, shape, bc_lo, bc_hi):
    """Where a particle that leaves the centre of cell (i,j,k) with velocity
    c_q is after one unit of time.  Walls are the planes y = 0 and y = ny
    (cell centres at j + 1/2).  A no-slip wall reverses the whole velocity at
    the wall (half a step out, half a step back); a free-slip wall reverses
    only the normal component, tangential motion continues for the full step."""
    nz, ny, nx = shape
    v = np.array(c[q], dtype=float)
    pos = np.array([i + 0.5, j + 0.5, k + 0.5])
    if bc_lo == PER and bc_hi == PER:  # no walls: the domain wraps in y as well
        pos = pos + v
        qq = [tuple(x) for x in c].index(tuple(int(s) for s in v))
        return (qq, int(math.floor(pos[2])) % nz, int(math.floor(pos[1])) % ny,
                int(math.floor(pos[0])) % nx)
    t = 0.0
    while t < 1.0 - 1e-12:
        # time to reach a wall plane moving with v
        dt = 1.0 - t
        hit = None
        if v[1] < 0 and pos[1] + v[1] * dt < 0:
            dt, hit = (0 - pos[1]) / v[1], "lo"
        elif v[1] > 0 and pos[1] + v[1] * dt > ny:
            dt, hit = (ny - pos[1]) / v[1], "hi"
        bc = {"lo": bc_lo, "hi": bc_hi}.get(hit)
        pos = pos + v * dt
        t += dt
        if hit is not None:
            if bc == BB:
                v = -v
            else:
                v[1] = -v[1]
    ii = int(math.floor(pos[0])) % nx
    jj = int(math.floor(pos[1]))
    kk = int(math.floor(pos[2])) % nz
    qq = [tuple(x) for x in c].index(tuple(int(s) for s in v))
    return qq, kk, jj, ii


@pytest.mark.parametrize("shape", [(3, 4, 3), (4, 2, 5), (2, 1, 3)])
@pytest.mark.parametrize("bcs", [(BB, FS), (BB, BB), (FS, FS), (FS, BB), (PER, PER)])
def test_streaming_is_the_particle_permutation(shape, bcs):
    nz, ny, nx = shape
    c, _ = ref.lattice()
    sim = ref.RefLBM(nx, ny, nz, tau0=0.8, bc_lo=bcs[0], bc_hi=bcs[1])
    n = nx * ny * nz
    ids = np.arange(19 * n, dtype=np.float64).reshape((19,) + shape)
    sim.set_f(ids)
    pulled = sim.pull()
    assert sorted(pulled.ravel().tolist()) == list(range(19 * n))  # a permutation
    for q in range(19):
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            qq, kk, jj, ii = _landing(c, q, i, j, k, shape, bcs[0], bcs[1])
            assert pulled[qq, kk, jj, ii] == ids[q, k, j, i]


# ---------------------------------------------------------------------------
# conservation laws and exact balances of the whole step
# ---------------------------------------------------------------------------

def _c1_like(nx, ny, nz, **kw):
    from paper_2206_15454_amd import inputs

    w = inputs.scaled(inputs.C1, nx, ny, nz, **kw)
    sim = ref.RefLBM(w.nx, w.ny, w.nz, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi)
    lad = np.zeros(w.ny)
    lad[: w.canopy_rows] = w.lad_const
    sim.set_canopy(w.cd, lad)
    rho, u = inputs.init_fields(w)
    sim.init(rho, u)
    return w, sim


def test_mass_conserved_with_walls_canopy_and_sgs():
    w, sim = _c1_like(24, 16, 12)
    m0 = sim.moments()[3]["mass"]
    sim.step(200)
    rho, u, nut, d = sim.moments()
    # streaming permutes populations and the collision conserves mass up to
    # rounding: allow a few ulp per step (a dropped or wrong term gives >1e-8)
    assert abs(d["mass"] - m0) <= 200 * 5e-16 * m0
    assert d["nonfinite"] == 0 and d["t"] == 200
    assert nut.max() > 0  # the closure is active


def test_body_force_momentum_gain_periodic():
    """Fully periodic, no canopy: the reported momentum sum(rho u) gains
    exactly M g per step for any tau (Guo forcing, half-force velocity)."""
    from paper_2206_15454_amd import inputs

    g = (2e-5, -1e-5, 3e-6)
    sim = ref.RefLBM(10, 6, 8, tau0=0.55, csmag=0.02, g=g, bc_lo=PER, bc_hi=PER)
    w = inputs.scaled(inputs.C1, 10, 6, 8)
    rho, u = inputs.init_fields(w, seed=7)
    rho = rho * (1 + 0.01 * np.random.default_rng(8).uniform(-1, 1, rho.shape))
    sim.init(rho, u)
    sim.step(1)
    d0 = sim.moments()[3]
    M = d0["mass"]
    for _ in range(20):
        sim.step(1)
        d1 = sim.moments()[3]
        for a, key in enumerate(("mom_x", "mom_y", "mom_z")):
            assert d1[key] - d0[key] == pytest.approx(M * g[a], rel=1e-9, abs=1e-15)
        d0 = d1
    # impulse accumulated over the 21 steps is 21 M g
    assert d1["imp_x"] == pytest.approx(21 * M * g[0], rel=1e-13)


@pytest.mark.parametrize("vector", [False, True])
def test_canopy_drag_scalar_recurrence(vector):
    """Uniform flow, periodic, LAD = a everywhere: with s = j_x / rho,
    s_{n+1} = s_n + g + a_d(s_n + g/2), a_d(v) = -C_D a |v| v, and the
    reported velocity is u_n = s_n + g/2 + a_d/2."""
    g, cd, a, s = 3e-6, 0.2, 0.3, 0.05
    sim = ref.RefLBM(3, 2, 4, tau0=0.52, csmag=0.01, g=(g, 0, 0), bc_lo=PER, bc_hi=PER)
    sim.set_canopy(cd, np.full(2, a), vector_drag=vector)
    shape = (4, 2, 3)
    u0 = np.zeros((3,) + shape)
    u0[0] = s
    sim.init(np.ones(shape), u0)
    for _ in range(300):
        v = s + 0.5 * g
        ad = -cd * a * abs(v) * v
        u_expect = v + 0.5 * ad
        s = s + g + ad
        sim.step(1)
        _, u, _, _ = sim.moments()
        assert np.max(np.abs(u[0] - u_expect)) <= 1e-14
        assert np.max(np.abs(u[1:])) == 0.0


def test_poiseuille_closed_form():
    """Open channel: bounce-back bottom, free-slip top, body force g, no SGS.
    Steady BGK solution: u(y) = (g/nu) [H y - y^2/2 + (2/3) L - 1/8],
    L = (tau - 1/2)^2, nu = (tau - 1/2)/3 (uniform slip that vanishes at
    L = 3/16)."""
    H = 16
    g = 1e-6
    for tau in (0.6, 0.8, 0.5 + math.sqrt(3.0 / 16.0), 1.2):
        nu = (tau - 0.5) / 3.0
        sim = ref.RefLBM(1, H, 1, tau0=tau, csmag=0.0, g=(g, 0, 0), bc_lo=BB, bc_hi=FS)
        sim.init(np.ones((1, H, 1)), np.zeros((3, 1, H, 1)))
        T = int(12 * H * H / nu)
        sim.step(T)
        _, u, _, _ = sim.moments()
        y = np.arange(H) + 0.5
        L = (tau - 0.5) ** 2
        expect = (g / nu) * (H * y - y * y / 2 + (2.0 / 3.0) * L - 1.0 / 8.0)
        np.testing.assert_allclose(u[0, 0, :, 0], expect, rtol=1e-9)
        assert np.max(np.abs(u[1:])) < 1e-10 * np.max(expect)


def _taylor_green(n, U, tau, csmag, steps):
    k = 2 * math.pi / n
    sim = ref.RefLBM(n, 2, n, tau0=tau, csmag=csmag, bc_lo=PER, bc_hi=PER)
    x = np.arange(n) + 0.5
    X = x[None, None, :]
    Z = x[:, None, None]
    u = np.zeros((3, n, 2, n))
    u[0] = U * np.sin(k * X) * np.cos(k * Z) * np.ones((n, 2, n))
    u[2] = -U * np.cos(k * X) * np.sin(k * Z) * np.ones((n, 2, n))
    # pressure of the Taylor-Green vortex: rho = 1 + 3 p
    p = -U * U / 4 * (np.cos(2 * k * X) + np.cos(2 * k * Z))
    rho = (1 + 3 * p) * np.ones((n, 2, n))
    sim.init(rho, u)
    return sim, k, X, Z


def test_taylor_green_viscous_decay():
    n, U, tau = 64, 0.01, 0.8
    nu = (tau - 0.5) / 3
    sim, k, _, _ = _taylor_green(n, U, tau, 0.0, 0)
    sim.step(10)
    _, u, _, _ = sim.moments()
    e0 = np.sum(u[0] ** 2 + u[2] ** 2)
    sim.step(300)
    _, u, _, _ = sim.moments()
    e1 = np.sum(u[0] ** 2 + u[2] ** 2)
    rate = -math.log(e1 / e0) / 300
    assert rate == pytest.approx(4 * nu * k * k, rel=1e-2)
    assert np.max(np.abs(u[1])) < 1e-18


def test_taylor_green_smagorinsky_strain():
    """nu_t = C |S| with |S| of the analytic vortex (|S| = 2 U k |cos kx cos kz|),
    to O(k^2) at the cells of largest strain."""
    n, U, tau, C = 64, 0.02, 0.6, 0.02
    sim, k, X, Z = _taylor_green(n, U, tau, C, 0)
    sim.step(20)
    _, u, nut, _ = sim.moments()
    Ut = np.sqrt(np.mean(u[0] ** 2 + u[2] ** 2) * 4 / 2)  # current amplitude
    S = 2 * Ut * k * np.abs(np.cos(k * X) * np.cos(k * Z)) * np.ones((n, 2, n))
    big = S > 0.8 * S.max()
    np.testing.assert_allclose(nut[big], C * S[big], rtol=0.03)


def test_stats_means_of_sampled_steps():
    w, sim = _c1_like(8, 6, 4)
    sim.stats_reset()
    sim.stats_enable(2)
    acc = np.zeros((6, 10))
    for t in range(1, 7):
        sim.step(1)
        if t % 2 == 0:
            _, u, nut, _ = sim.moments()
            q = [u[0], u[1], u[2], u[0] ** 2, u[1] ** 2, u[2] ** 2, u[0] * u[1], u[0] * u[2],
                 u[1] * u[2], nut]
            acc += np.stack([x.mean(axis=(0, 2)) for x in q], axis=1)
    prof, ns = sim.stats_read()
    assert ns == 3
    np.testing.assert_allclose(prof, acc / 3, rtol=1e-12, atol=1e-20)


def test_thread_count_does_not_change_results():
    import subprocess
    import sys
    import os

    code = ("import numpy as np, sys; sys.path.insert(0, %r);"
            "from tests.test_oracle_pins import _c1_like;"
            "w, s = _c1_like(16, 8, 8); s.step(20); r,u,n,d = s.moments();"
            "np.save(sys.argv[1], np.concatenate([r.ravel(), u.ravel(), n.ravel()]))"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import tempfile

    outs = []
    with tempfile.TemporaryDirectory() as d:
        for th in ("1", "4"):
            path = os.path.join(d, f"o{th}.npy")
            env = dict(os.environ, OMP_NUM_THREADS=th)
            subprocess.run([sys.executable, "-c", code, path], check=True, env=env)
            outs.append(np.load(path))
    assert np.array_equal(outs[0], outs[1])


# ---------------------------------------------------------------------------
# forced-equilibrium boundary (Sec. 5.1: the top moves with the free stream)
# ---------------------------------------------------------------------------

def test_equilibrium_boundary_keeps_a_uniform_stream():
    """feq(1, U) everywhere is a fixed point when the boundary imposes U."""
    U = (0.05, 0.0, -0.02)
    sim = ref.RefLBM(6, 5, 4, tau0=0.6, csmag=0.01, bc_lo=ref.BC_FREESLIP,
                     bc_hi=ref.BC_EQUILIBRIUM)
    sim.set_wall_velocity(U)
    u = np.zeros((3, 4, 5, 6))
    u[0], u[2] = U[0], U[2]
    sim.init(np.ones((4, 5, 6)), u)
    f0 = sim.get_f()
    sim.step(20)
    np.testing.assert_allclose(sim.get_f(), f0, rtol=0, atol=20 * 4e-16)  # a few ulps per step


def test_equilibrium_boundary_couette_is_linear():
    """Bounce-back bottom, forced equilibrium at U on top, no force: the
    steady profile is a straight line from ~0 at the wall to ~U at the top."""
    H, U = 12, 0.02
    for tau in (0.6, 0.9):
        sim = ref.RefLBM(1, H, 1, tau0=tau, csmag=0.0, bc_lo=BB, bc_hi=ref.BC_EQUILIBRIUM)
        sim.set_wall_velocity((U, 0.0, 0.0))
        sim.init(np.ones((1, H, 1)), np.zeros((3, 1, H, 1)))
        sim.step(int(20 * H * H / ((tau - 0.5) / 3)))
        _, u, _, _ = sim.moments()
        ux = u[0, 0, :, 0]
        y = np.arange(H) + 0.5
        a, b = np.polyfit(y, ux, 1)
        assert np.max(np.abs(ux - (a * y + b))) <= 1e-10 * U
        assert abs(b) <= 0.05 * U and 0.8 * U / H <= a <= 1.2 * U / H
