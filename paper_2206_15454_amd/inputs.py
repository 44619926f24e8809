"""Seeded synthetic inputs and the workload table.

This module holds no arithmetic of the method: only the sizes and physical
parameters of each workload and the seeded initial fields (density and
velocity).  It is the one module that both the oracle-based tests and the
GPU path read, so that both sides start from identical arrays.

Initial velocity (every workload): u_x = U_ref (y_j / Y)^(1/7) + A U_ref xi_x,
u_y = A U_ref xi_y, u_z = A U_ref xi_z, with xi ~ U[-1, 1) drawn i.i.d. per
cell and component by NumPy's PCG64 generator (``default_rng(seed)``) as one
array of shape (3, nz, ny, nx) in C order; y_j = j + 1/2; rho = 1 exactly.

Leaf-area density: a workload names either a constant value below a canopy
row (``lad_const``, ``canopy_rows``) or the Lalic-Mihailovic profile by its
parameters (``lad_lalic``: h, y_m, LAI normalisation; ``lad_profile``: h,
y_m, peak a_fm); the caller evaluates the profile with its own
implementation of the paper's Eq. (af_theory).
"""
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

BC_PERIODIC, BC_BOUNCEBACK, BC_FREESLIP, BC_EQUILIBRIUM = 0, 1, 2, 3
STORAGES = ("f64", "f32", "f16s", "bf16s", "bf16sr")


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    storage: str
    tau0: float
    c_smag: float
    g: Tuple[float, float, float]
    bc_lo: int
    bc_hi: int
    cd: float
    lad_const: float = 0.0
    canopy_rows: int = 0
    lad_lalic: Optional[Tuple[float, float, float]] = None  # (h, y_m, LAI) in cells
    u_ref: float = 0.05
    y_ref: float = 32.0
    noise: float = 0.02
    seed: int = 1
    steps: int = 200
    u_wall: Tuple[float, float, float] = (0.0, 0.0, 0.0)  # forced-equilibrium boundary
    lad_profile: Optional[Tuple[float, float, float]] = None  # (h, y_m, a_fm): Eq. af_theory peak
    channel: bool = False  # initial profile mirrored about the mid-plane (two walls)
    # heterogeneous forest from a synthetic point cloud: (trees per ground
    # cell, min and max tree height in cells, a_fm, y_m / h, points per cell)
    forest: Optional[Tuple[float, float, float, float, float, float]] = None
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


# canopy boundary layer, plain method in FP64: 64x32x32, 200 steps
C1 = Workload(name="canopy-abl-64x32x32-f64", nx=64, ny=32, nz=32, storage="f64", tau0=0.52,
              c_smag=0.01, g=(1e-6, 0.0, 0.0), bc_lo=BC_BOUNCEBACK, bc_hi=BC_FREESLIP, cd=0.2,
              lad_const=0.3, canopy_rows=8, u_ref=0.05, y_ref=32.0, noise=0.02, seed=1,
              steps=200)

# production canopy boundary layer in FP32: 512x128x256, h = 12, LAI 2, u_tau = 0.01
C2 = Workload(name="canopy-abl-512x128x256-f32", nx=512, ny=128, nz=256, storage="f32",
              tau0=0.5005, c_smag=0.01, g=(0.01 ** 2 / 128.0, 0.0, 0.0),
              bc_lo=BC_BOUNCEBACK, bc_hi=BC_FREESLIP, cd=0.15, lad_lalic=(12.0, 8.4, 2.0),
              u_ref=0.1, y_ref=128.0, noise=0.05, seed=2, steps=20000)

# precision study: physics of the 64x32x32 case on 1024x256x512 cells
C3 = replace(C1, name="canopy-abl-1024x256x512", nx=1024, ny=256, nz=512, storage="f32",
             seed=3, steps=1000)

# the same physics on a 128x64x64 crop that the oracle finishes
CROP = replace(C1, name="canopy-abl-128x64x64", nx=128, ny=64, nz=64, seed=3, steps=1000)

# learned-closure training data: the production setup at twice the resolution
# (acoustic scaling in coarse units: tau0_f = 1/2 + 2 (tau0 - 1/2), g_f = g / 2)
C4 = replace(C2, name="canopy-abl-fine-1024x256x512-f32", nx=1024, ny=256, nz=512,
             tau0=0.501, g=(C2.g[0] / 2.0, 0.0, 0.0), lad_lalic=(24.0, 16.8, 2.0),
             y_ref=256.0, seed=4, steps=40000)

# learned-closure inference: 1024x256x512 BF16 storage
C5 = replace(C3, name="canopy-abl-1024x256x512-bf16s-mlp", storage="bf16s", seed=3,
             steps=20000)

# The paper's ABL over a homogeneous forest (Sec. 5), fine mesh 350x140x280 of
# 1000x400x800 m (dx = 2.857 m): forest height h = 20 m = 7 cells, C_D = 0.15,
# bounce-back ground, forced-equilibrium top moving with the free stream
# (U = 0.08), periodic x and z.  LAD per cell = a_f [1/m] * dx:
#   case 1: constant 0.215/m -> 0.6143; case 2: Eq. (af_theory) with
#   y_m = 0.7 h, a_fm = 0.38/m -> peak 1.0857; case 3: no forest.
# The driving force of the paper cannot be recovered from its text; here
# g = u*^2 / Ny with u* = U/20.
_DX_ABL = 1000.0 / 350.0
ABL1 = Workload(name="paper-abl-350x140x280-case1", nx=350, ny=140, nz=280, storage="f32",
                tau0=0.5005, c_smag=0.01, g=((0.08 / 20) ** 2 / 140, 0.0, 0.0),
                bc_lo=BC_BOUNCEBACK, bc_hi=BC_EQUILIBRIUM, cd=0.15,
                lad_const=0.215 * _DX_ABL, canopy_rows=7, u_ref=0.08, y_ref=140.0, noise=0.05,
                seed=5, steps=20000, u_wall=(0.08, 0.0, 0.0))
# the coarse and medium meshes of the paper's mesh study (Table tab:mesh_cost,
# constant LAD): dx = 5 m and 4 m, forest 4 and 5 cells high
ABL_COARSE = replace(ABL1, name="paper-abl-200x80x160-case1", nx=200, ny=80, nz=160,
                     g=((0.08 / 20) ** 2 / 80, 0.0, 0.0), lad_const=0.215 * 5.0, canopy_rows=4,
                     y_ref=80.0)
ABL_MEDIUM = replace(ABL1, name="paper-abl-250x100x200-case1", nx=250, ny=100, nz=200,
                     g=((0.08 / 20) ** 2 / 100, 0.0, 0.0), lad_const=0.215 * 4.0, canopy_rows=5,
                     y_ref=100.0)
ABL2 = replace(ABL1, name="paper-abl-350x140x280-case2",
               lad_profile=(7.0, 0.7 * 7.0, 0.38 * _DX_ABL))
ABL3 = replace(ABL1, name="paper-abl-350x140x280-case3", lad_const=0.0, canopy_rows=0)

# The paper's validation channel (Sec. 4, Re_tau = 180): 12 x 2 x 4 H at 31
# cells per H -> 372 x 62 x 124, walls top and bottom; dx = 1/31, dt = 0.001,
# nu = 1/3250, F = 0.002986 in lattice units: tau0 = 0.5 + 3 nu dt/dx^2,
# g = F dt^2/dx.
CHANNEL = Workload(name="paper-channel-372x62x124", nx=372, ny=62, nz=124, storage="f32",
                   tau0=0.5 + 3.0 * (1.0 / 3250.0) * 0.001 * 31.0 ** 2, c_smag=0.01,
                   g=(0.002986 * 0.001 ** 2 * 31.0, 0.0, 0.0), bc_lo=BC_BOUNCEBACK,
                   bc_hi=BC_BOUNCEBACK, cd=0.0, u_ref=0.03, y_ref=31.0, noise=0.05, seed=6,
                   steps=20000, channel=True)

# A heterogeneous forest (Sec. 3 forest codes, Algorithm 1) on the production
# grid: about 1640 trees of 8-16 cells, crowns that overlap into patches,
# a_fm = 0.36 per cell (the peak of the LAI-2 profile above), y_m = 0.7 h.
FOREST = replace(C2, name="forest-patches-512x128x256-f32", lad_lalic=None,
                 forest=(1.0 / 80.0, 8.0, 16.0, 0.36, 0.7, 4.0), seed=7)

# One GPU's share of the 1024x256x512 case split into 8 slabs along x (the
# decomposition of a multi-GPU run): 128x256x512 cells, the same N as the
# production case, with the tile shape that a 128-wide slab gives.
SLAB = replace(C3, name="canopy-abl-slab-128x256x512", nx=128, ny=256, nz=512, storage="f32")

WORKLOADS = {w.name: w for w in (C1, C2, C3, CROP, C4, C5, ABL1, ABL2, ABL3, ABL_COARSE,
                                 ABL_MEDIUM, CHANNEL, FOREST, SLAB)}


def scaled(w: Workload, nx: int, ny: int, nz: int, **kw) -> Workload:
    """The same physics on another grid (test sizes)."""
    return replace(w, name=f"{w.name}@{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, **kw)


def lad_constant(w: Workload) -> Optional[np.ndarray]:
    """Constant-LAD canopy rows (None when the workload uses a profile)."""
    if w.lad_lalic is not None or w.lad_profile is not None or w.forest is not None:
        return None
    lad = np.zeros(w.ny)
    lad[: min(w.canopy_rows, w.ny)] = w.lad_const
    return lad


def init_fields(w: Workload, seed: Optional[int] = None):
    """Seeded initial density and velocity, float64, shapes (nz,ny,nx) and
    (3,nz,ny,nx)."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    xi = rng.uniform(-1.0, 1.0, size=(3,) + w.shape)
    y = np.arange(w.ny, dtype=np.float64) + 0.5
    if w.channel:
        y = np.minimum(y, w.ny - y)
    ubar = w.u_ref * (y / w.y_ref) ** (1.0 / 7.0)
    u = w.noise * w.u_ref * xi
    u[0] += ubar[None, :, None]
    rho = np.ones(w.shape)
    return rho, u


def init_fields_torch(w: Workload, device, seed: Optional[int] = None):
    """The same recipe drawn on the GPU with torch's generator (for grids too
    large to draw on the host quickly).  Not bit-identical to
    ``init_fields``; every storage type of one study receives the same
    arrays."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(w.seed if seed is None else seed)
    u = torch.rand((3,) + w.shape, generator=gen, device=device, dtype=torch.float64)
    u.mul_(2.0).sub_(1.0).mul_(w.noise * w.u_ref)
    y = torch.arange(w.ny, device=device, dtype=torch.float64) + 0.5
    if w.channel:
        y = torch.minimum(y, w.ny - y)
    u[0] += (w.u_ref * (y / w.y_ref) ** (1.0 / 7.0))[None, :, None]
    rho = torch.ones(w.shape, device=device, dtype=torch.float64)
    return rho, u


def random_populations(shape, seed: int, base, scale: float = 0.01):
    """Arbitrary population fields f_q = base_q (1 + scale * xi), xi ~ U[-1, 1)
    i.i.d., shape (19,) + shape; ``base`` (19 values) is supplied by the
    caller."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64).reshape((19,) + (1,) * len(shape))
    xi = rng.uniform(-1.0, 1.0, size=(19,) + tuple(shape))
    return base * (1.0 + scale * xi)


def forest_points(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Synthetic forest point cloud [npts][3] (x, y, z in cell units).

    Trees stand at uniform random ground positions (periodic in x and z),
    trees_per_cell * nx * nz of them, with height H ~ U[h_min, h_max].  Each
    has a trunk (points along the axis from the ground to 0.3 H) and a crown:
    an ellipsoid centred at 0.65 H with vertical semi-axis 0.35 H and
    horizontal radius R ~ U[0.2, 0.35] H, filled with uniformly drawn points
    at points_per_cell per unit volume (so some crown cells hold none, as in
    a scanned cloud).  NumPy PCG64 ``default_rng(seed)``."""
    density, hmin, hmax, _, _, ppc = w.forest
    rng = np.random.default_rng(w.seed if seed is None else seed)
    ntrees = max(1, int(round(density * w.nx * w.nz)))
    cx = rng.random(ntrees) * w.nx
    cz = rng.random(ntrees) * w.nz
    H = rng.uniform(hmin, hmax, ntrees)
    R = rng.uniform(0.2, 0.35, ntrees) * H
    out = []
    for t in range(ntrees):
        m = max(1, int(round(0.3 * H[t] * 2)))  # trunk: 2 points per cell of height
        out.append(np.stack([np.full(m, cx[t]), rng.random(m) * 0.3 * H[t], np.full(m, cz[t])], 1))
        a, b = R[t], 0.35 * H[t]
        m = int(round(ppc * 4.0 / 3.0 * np.pi * a * a * b))
        d = rng.normal(size=(m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d *= rng.random((m, 1)) ** (1.0 / 3.0)
        out.append(np.stack([cx[t] + a * d[:, 0], 0.65 * H[t] + b * d[:, 1],
                             cz[t] + a * d[:, 2]], 1))
    p = np.concatenate(out)
    p[:, 0] %= w.nx
    p[:, 2] %= w.nz
    p[p[:, 0] >= w.nx, 0] = 0.0  # a tiny negative value wraps to exactly nx
    p[p[:, 2] >= w.nz, 2] = 0.0
    p[:, 1] = np.clip(p[:, 1], 0.0, np.nextafter(w.ny, 0))
    return p
