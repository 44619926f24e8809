"""FP64 oracle of the learned closure's training samples (NumPy).

TEST INFRASTRUCTURE ONLY (see lbm_ref.c).  Written from the definitions,
independently of the HIP kernels:

  * box filter: the mean over each 2x2x2 block of fine cells;
  * fine strain S^f and coarse strain Sb: S = (grad u + grad u^T)/2 with
    central differences (periodic in x and z; one-sided forward / backward in
    y at the first / last row; zero if there is a single row);
  * subfilter stress tau = box(u u) - ub ub + box(-2 nu_t^f S^f);
  * target nu* = max(0, -dev(tau):Sb / (2 Sb:Sb)), 0 where Sb:Sb <= 1e-30;
  * features of P = -2 (tau0 + 3 nu*) Sb: tr P, tr P^2, tr P^3, P_yy,
    (P^2)_yy, sqrt(tr P^2), (j + 1/2)/h, lad[j], 1.

Arrays are [z][y][x]; velocity [3][z][y][x].
"""
import numpy as np


def grad(u):
    """g[a][b] = du_a/dx_b, shape (3, 3, nz, ny, nx)"""
    nz, ny, nx = u.shape[1:]
    g = np.zeros((3, 3) + u.shape[1:])
    for a in range(3):
        f = u[a]
        g[a, 0] = 0.5 * (np.roll(f, -1, axis=2) - np.roll(f, 1, axis=2))
        g[a, 2] = 0.5 * (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0))
        if ny > 1:
            d = np.zeros_like(f)
            d[:, 1:-1] = 0.5 * (f[:, 2:] - f[:, :-2])
            d[:, 0] = f[:, 1] - f[:, 0]
            d[:, -1] = f[:, -1] - f[:, -2]
            g[a, 1] = d
    return g


def strain(u):
    g = grad(u)
    return 0.5 * (g + g.transpose(1, 0, 2, 3, 4))


def box(f):
    """2x2x2 block means of the last three axes"""
    *lead, nz, ny, nx = f.shape
    r = f.reshape(*lead, nz // 2, 2, ny // 2, 2, nx // 2, 2)
    return r.mean(axis=(-5, -3, -1))


def samples(u, nut, tau0_coarse, canopy_h, lad_coarse):
    """(X [nc, 9], y [nc], extras) for fine velocity u [3][z][y][x] and fine
    nu_t [z][y][x]."""
    Sf = strain(u)
    ub = box(u)
    uu = box(u[:, None] * u[None, :])
    tf = box(-2.0 * nut[None, None] * Sf)
    tau = uu - ub[:, None] * ub[None, :] + tf
    Sb = strain(ub)
    dev = tau - np.trace(tau)[None, None] / 3.0 * np.eye(3)[:, :, None, None, None]
    dd = np.einsum("ab...,ab...->...", dev, Sb)
    ss = np.einsum("ab...,ab...->...", Sb, Sb)
    nus = np.zeros_like(ss)
    ok = ss > 1e-30
    nus[ok] = np.maximum(0.0, -dd[ok] / (2.0 * ss[ok]))
    P = -2.0 * (tau0_coarse + 3.0 * nus)[None, None] * Sb
    P2 = np.einsum("ab...,bc...->ac...", P, P)
    tr1 = np.trace(P)
    tr2 = np.trace(P2)
    tr3 = np.einsum("ab...,ba...->...", P2, P)
    cz, cy, cx = ss.shape
    yh = ((np.arange(cy) + 0.5) / canopy_h)[None, :, None] * np.ones((cz, cy, cx))
    lad = np.asarray(lad_coarse, dtype=np.float64)[None, :, None] * np.ones((cz, cy, cx))
    X = np.stack([tr1, tr2, tr3, P[1, 1], P2[1, 1], np.sqrt(tr2), yh, lad, np.ones_like(ss)],
                 axis=-1).reshape(-1, 9)
    return X, nus.reshape(-1), {"tau": tau, "Sb": Sb, "ub": ub}
