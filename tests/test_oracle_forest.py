"""Pins of the oracle's heterogeneous forest (point cloud -> per-cell forest
code -> LAD, Sec. 3 forest description, Algorithm 1, Eq. (af_theory)).

The connected components are checked against an independent union-find
written here; the LAD against the homogeneous profile routine (Eq. af_theory
over rows), which is itself pinned in test_oracle_pins.py."""
import numpy as np
import pytest

from oracle import ref


def union_find_codes(points, nx, ny, nz, ym_frac):
    """Independent reference: union-find over face neighbours (periodic x, z)."""
    forest = np.zeros((nz, ny, nx), dtype=bool)
    for x, y, z in points:
        forest[int(np.floor(z)), int(np.floor(y)), int(np.floor(x))] = True
    parent = {}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    cells = [tuple(c) for c in np.argwhere(forest)]
    for c in cells:
        parent[c] = c
    for k, j, i in cells:
        for dk, dj, di in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
            jj = j + dj
            if jj >= ny:
                continue
            o = ((k + dk) % nz, jj, (i + di) % nx)
            if forest[o]:
                ra, rb = find((k, j, i)), find(o)
                if ra != rb:
                    parent[ra] = rb
    groups = {}
    for c in cells:
        groups.setdefault(find(c), []).append(c)
    qm = int(np.floor(ym_frac * 4096.0 + 0.5))
    codes = np.zeros((nz, ny, nx), dtype=np.uint32)
    for members in groups.values():
        rows = [c[1] for c in members]
        lo, h = min(rows), max(rows) - min(rows) + 1
        for k, j, i in members:
            codes[k, j, i] = h | ((j - lo) << 10) | (qm << 20)
    return codes, len(groups)


@pytest.mark.parametrize("seed", range(6))
def test_codes_match_union_find(seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = rng.integers(3, 9, size=3)
    npts = int(rng.integers(1, 3 * nx * ny * nz // 4 + 2))
    pts = rng.random((npts, 3)) * np.array([nx, ny, nz])
    frac = float(rng.random() * 0.99)
    codes, nobj = ref.forest_codes(pts, nx, ny, nz, frac)
    want, nwant = union_find_codes(pts, nx, ny, nz, frac)
    np.testing.assert_array_equal(codes, want)
    assert nobj == nwant


def test_hand_cases():
    # a column of rows 2..5, a diagonal neighbour (separate object), and a
    # pair joined across the periodic x boundary
    pts = [(1.5, y + 0.5, 1.5) for y in range(2, 6)]
    pts += [(2.5, 6.5, 2.5)]
    pts += [(0.2, 0.3, 4.5), (5.9, 0.1, 4.5), (5.1, 1.9, 4.5)]
    codes, nobj = ref.forest_codes(np.array(pts), 6, 8, 6, 0.7)
    assert nobj == 3
    for y in range(2, 6):
        assert ref.forest_decode(codes[1, y, 1]) == (4, y - 2, 2867)
    assert ref.forest_decode(codes[2, 6, 2])[:2] == (1, 0)
    assert ref.forest_decode(codes[4, 0, 0])[:2] == (2, 0)
    assert ref.forest_decode(codes[4, 1, 5])[:2] == (2, 1)
    assert int((codes > 0).sum()) == 8


def test_errors():
    with pytest.raises(ValueError):
        ref.forest_codes(np.array([[4.0, 0.5, 0.5]]), 4, 4, 4)  # x = nx is outside
    with pytest.raises(ValueError):
        ref.forest_codes(np.array([[-1e-9, 0.5, 0.5]]), 4, 4, 4)
    with pytest.raises(ValueError):
        ref.forest_codes(np.array([[0.5, 0.5, 0.5]]), 4, 4, 4, ym_frac=1.0)
    with pytest.raises(ValueError):
        ref.forest_codes(np.array([[0.5, np.nan, 0.5]]), 4, 4, 4)
    codes, n = ref.forest_codes(np.zeros((0, 3)), 4, 4, 4)
    assert n == 0 and not codes.any()


@pytest.mark.parametrize("h,afm", [(7, 0.38), (12, 0.3), (20, 1.0)])
def test_homogeneous_forest_equals_row_profile(h, afm):
    """A forest covering the whole ground up to row h-1 has, in every
    column, exactly the Eq. (af_theory) profile with y_m = h q_m / 4096."""
    nx, ny, nz = 3, h + 4, 2
    pts = [(i + 0.5, j + 0.5, k + 0.5) for i in range(nx) for j in range(h) for k in range(nz)]
    codes, nobj = ref.forest_codes(np.array(pts), nx, ny, nz, 0.7)
    assert nobj == 1
    ym = h * 2867 / 4096.0
    row = ref.lad_lalic(h, ym, ny, afm=afm)
    lad = np.array([[[ref.forest_lad(c, afm) for c in r] for r in pl] for pl in codes])
    for k in range(nz):
        for i in range(nx):
            np.testing.assert_array_equal(lad[k, :, i], row)


def test_lad_values():
    # y_m = 4.5 at h = 8 (q_m = 2304): the cell centred on y_m has the peak a_fm
    pts = np.array([(0.5, j + 0.5, 0.5) for j in range(8)])
    codes, _ = ref.forest_codes(pts, 1, 10, 1, 0.5625)
    lad = [ref.forest_lad(c, 0.4) for c in codes[0, :, 0]]
    assert lad[4] == 0.4
    assert all(0 < v < 0.4 for v in lad[:4] + lad[5:8]) and lad[8] == lad[9] == 0.0
    # n = 6 below the peak, 1/2 above: recover it from two values
    for j in (1, 6):
        yc, ym, h = j + 0.5, 4.5, 8.0
        r = (h - ym) / (h - yc)
        n = np.log(lad[j] / 0.4) / (np.log(r) + 1 - r)
        assert n == pytest.approx(6.0 if j < 4 else 0.5, rel=1e-12)
    # constant mode (Table tab:forest_cases case 1)
    assert [ref.forest_lad(c, 0.215, True) for c in codes[0, :, 0]] == [0.215] * 8 + [0.0] * 2


def test_step_with_homogeneous_codes_equals_row_profile():
    """Whole oracle step: per-cell LAD from codes == per-row LAD, bit for bit."""
    from paper_2206_15454_amd import inputs

    nx, ny, nz, h = 12, 10, 8, 6
    pts = [(i + 0.5, j + 0.5, k + 0.5) for i in range(nx) for j in range(h) for k in range(nz)]
    codes, _ = ref.forest_codes(np.array(pts), nx, ny, nz, 0.7)
    w = inputs.scaled(inputs.C1, nx, ny, nz)
    rho, u = inputs.init_fields(w, 5)
    a = ref.RefLBM(nx, ny, nz, 0.52, 0.01, (1e-5, 0, 0))
    b = ref.RefLBM(nx, ny, nz, 0.52, 0.01, (1e-5, 0, 0))
    a.set_canopy(0.3, ref.lad_lalic(h, h * 2867 / 4096.0, ny, afm=0.5))
    b.set_forest(0.3, 0.5, codes)
    for s in (a, b):
        s.init(rho, 3 * u)
        s.step(20)
    ra, ua, na, da = a.moments()
    rb, ub, nb, db = b.moments()
    np.testing.assert_array_equal(ua, ub)
    np.testing.assert_array_equal(na, nb)
    assert da["imp_x"] == db["imp_x"] and da["imp_x"] < 0
