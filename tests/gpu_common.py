"""Helpers shared by the GPU tests: build both sides from the same seeded
inputs (the oracle and the HIP library never see each other's arrays)."""
import numpy as np

from oracle import ref
from paper_2206_15454_amd import inputs

BC_NAMES = {0: "periodic", 1: "bounceback", 2: "freeslip"}


def require_gpu():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need an MI355X: torch.cuda.is_available() is False")
    from paper_2206_15454_amd import lbm

    lbm.lib()  # raises if the HIP library is not built


def oracle_lad(w):
    lad = inputs.lad_constant(w)
    if lad is None and w.lad_lalic is not None:
        h, ym, lai = w.lad_lalic
        lad = ref.lad_lalic(h, ym, w.ny, lai=lai)
    elif lad is None:
        h, ym, afm = w.lad_profile
        lad = ref.lad_lalic(h, ym, w.ny, afm=afm)
    return lad


def make_pair(w, storage=None, seed=None, init=True, vector_drag=False):
    """(oracle simulation, GPU simulation) of workload w, identically set up."""
    from paper_2206_15454_amd import lbm

    storage = storage or w.storage
    o = ref.RefLBM(w.nx, w.ny, w.nz, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi)
    o.set_wall_velocity(w.u_wall)
    g = lbm.LBM(w.nx, w.ny, w.nz, storage, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi,
                u_wall=w.u_wall)
    lad = oracle_lad(w)
    o.set_canopy(w.cd, lad, vector_drag)
    g.set_canopy(w.cd, lad, vector_drag)
    if init:
        rho, u = inputs.init_fields(w, seed)
        o.init(rho, u)
        g.init(rho, u)
    return o, g


def normwise(a, b):
    """max |a - b| / max |b| over the grid (per field)."""
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


# storage rounding on the host (independent of the library)
def round_storage(x, storage):
    if storage == "f64":
        return np.asarray(x, dtype=np.float64)
    if storage == "f32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    if storage == "f16s":
        return np.asarray(x, dtype=np.float16).astype(np.float64)
    if storage in ("bf16s", "bf16sr"):
        f = np.asarray(x, dtype=np.float32)  # exact for the values used (already f32)
        b = f.view(np.uint32).astype(np.uint64)
        b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        return b.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(storage)


def ulp(x, storage):
    """unit in the last place of |x| in the storage type (x is the shifted value)."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    mant = {"f64": 52, "f32": 23, "f16s": 10, "bf16s": 7, "bf16sr": 7}[storage]
    tiny = {"f64": 2.0 ** -1022, "f32": 2.0 ** -126, "f16s": 2.0 ** -14, "bf16s": 2.0 ** -126,
            "bf16sr": 2.0 ** -126}[storage]
    e = np.floor(np.log2(np.maximum(a, tiny)))
    return 2.0 ** (e - mant)


def make_gpu(w, storage=None):
    """GPU simulation of workload w (no oracle), canopy set, not initialised."""
    from paper_2206_15454_amd import lbm

    g = lbm.LBM(w.nx, w.ny, w.nz, storage or w.storage, w.tau0, w.c_smag, w.g, w.bc_lo,
                w.bc_hi, u_wall=w.u_wall)
    g.set_canopy(w.cd, oracle_lad(w))
    return g


def make_forest_pair(w, storage=None, seed=None, constant=False, vector_drag=False):
    """(oracle, GPU) simulations of a heterogeneous-forest workload: each side
    turns the same seeded point cloud into forest codes with its own routine."""
    from paper_2206_15454_amd import lbm

    _, _, _, afm, ym_frac, _ = w.forest
    pts = inputs.forest_points(w)
    oc, _ = ref.forest_codes(pts, w.nx, w.ny, w.nz, ym_frac)
    gc, _ = lbm.forest_codes(pts, w.nx, w.ny, w.nz, ym_frac)
    o = ref.RefLBM(w.nx, w.ny, w.nz, w.tau0, w.c_smag, w.g, w.bc_lo, w.bc_hi)
    o.set_wall_velocity(w.u_wall)
    g = lbm.LBM(w.nx, w.ny, w.nz, storage or w.storage, w.tau0, w.c_smag, w.g, w.bc_lo,
                w.bc_hi, u_wall=w.u_wall, forest_map=True)
    o.set_forest(w.cd, afm, oc, constant, vector_drag)
    g.set_forest(w.cd, afm, gc, constant, vector_drag)
    rho, u = inputs.init_fields(w, seed)
    o.init(rho, u)
    g.init(rho, u)
    return o, g, oc
