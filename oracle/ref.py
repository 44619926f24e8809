"""ctypes wrapper of the FP64 CPU oracle (``liblbm_ref.so``).

TEST INFRASTRUCTURE ONLY.  Arrays are NumPy float64, C order: populations
``[19][nz][ny][nx]``, scalars per cell ``[nz][ny][nx]``, vectors
``[3][nz][ny][nx]``.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

BC_PERIODIC, BC_BOUNCEBACK, BC_FREESLIP, BC_EQUILIBRIUM = 0, 1, 2, 3
DIAG_KEYS = ("mass", "mom_x", "mom_y", "mom_z", "imp_x", "imp_y", "imp_z", "max_u", "t",
             "nonfinite", "mlp_fallback")

_dp = C.POINTER(C.c_double)


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.ref_create.restype = C.c_void_p
        L.ref_create.argtypes = [C.c_int] * 3 + [C.c_double] * 5 + [C.c_int] * 2
        L.ref_destroy.argtypes = [C.c_void_p]
        L.ref_set_canopy.argtypes = [C.c_void_p, C.c_double, _dp, C.c_int, C.c_int]
        L.ref_init.argtypes = [C.c_void_p, _dp, _dp]
        L.ref_set_f.argtypes = [C.c_void_p, _dp]
        L.ref_get_f.argtypes = [C.c_void_p, _dp]
        L.ref_pull.argtypes = [C.c_void_p, _dp]
        L.ref_step.argtypes = [C.c_void_p, C.c_int64]
        L.ref_moments.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.ref_stats.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, C.POINTER(C.c_int64)]
        L.ref_set_closure.argtypes = [C.c_void_p, C.c_void_p]
        L.ref_set_closure_interval.argtypes = [C.c_void_p, C.c_int]
        L.ref_set_wall_velocity.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        L.ref_lattice.argtypes = [C.POINTER(C.c_int), _dp]
        L.ref_feq.argtypes = [C.c_double, _dp, _dp]
        L.ref_guo.argtypes = [C.c_double, _dp, _dp, _dp]
        L.ref_moments_of.argtypes = [_dp, _dp, _dp, _dp]
        L.ref_smag.restype = C.c_double
        L.ref_smag.argtypes = [C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.ref_lad_lalic.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, _dp]
        L.ref_mlp_load.restype = C.c_void_p
        L.ref_mlp_load.argtypes = [C.c_char_p, C.c_size_t]
        L.ref_mlp_free.argtypes = [C.c_void_p]
        L.ref_mlp_apply.argtypes = [_dp, _dp, C.c_int64, _dp]
        L.ref_mlp_loss_grad.restype = C.c_double
        L.ref_mlp_loss_grad.argtypes = [_dp, _dp, _dp, C.c_int64, _dp]
        L.ref_mlp_predict.argtypes = [C.c_void_p, _dp, C.c_int64, _dp, _dp, C.POINTER(C.c_int)]
        L.ref_mlp_features.argtypes = [C.c_void_p, C.c_double, C.c_double, _dp, C.c_double,
                                       C.c_double, _dp]
        L.ref_gelu.restype = C.c_double
        L.ref_gelu.argtypes = [C.c_double]
        L.ref_softplus.restype = C.c_double
        L.ref_softplus.argtypes = [C.c_double]
        L.ref_threads.restype = C.c_int
        L.ref_forest_codes.argtypes = [_dp, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_double,
                                       C.POINTER(C.c_uint32), C.POINTER(C.c_int64)]
        L.ref_forest_lad.restype = C.c_double
        L.ref_forest_lad.argtypes = [C.c_uint32, C.c_double, C.c_int]
        L.ref_forest_decode.argtypes = [C.c_uint32] + [C.POINTER(C.c_int)] * 3
        L.ref_set_forest.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int,
                                     C.POINTER(C.c_uint32), C.c_int]
        _LIB = L
    return _LIB


# --------------------------------------------------------------------------
# per-cell formulas
# --------------------------------------------------------------------------

def lattice():
    c = (C.c_int * 57)()
    w = np.zeros(19)
    lib().ref_lattice(c, _ptr(w))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w


def feq(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib().ref_feq(float(rho), _ptr(u), _ptr(out))
    return out


def guo(tau, u, F):
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().ref_guo(float(tau), _ptr(u), _ptr(F), _ptr(out))
    return out


def moments_of(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.zeros(1)
    j = np.zeros(3)
    Pi = np.zeros(9)
    lib().ref_moments_of(_ptr(f), _ptr(rho), _ptr(j), _ptr(Pi))
    return rho[0], j, Pi.reshape(3, 3)


def smag(tau0, csmag, rho, Pineq):
    P = np.ascontiguousarray(Pineq, dtype=np.float64).reshape(9)
    nut = np.zeros(1)
    tau = lib().ref_smag(float(tau0), float(csmag), float(rho), _ptr(P), _ptr(nut))
    return tau, nut[0]


def lad_lalic(h, ym, ny, afm=1.0, lai=0.0):
    out = np.zeros(ny)
    rc = lib().ref_lad_lalic(float(h), float(ym), float(afm), float(lai), int(ny), _ptr(out))
    if rc != 0:
        raise ValueError("invalid LAD parameters")
    return out


def forest_codes(points, nx, ny, nz, ym_frac=0.7):
    """(codes uint32 [nz][ny][nx], number of forest objects) from a point
    cloud [npts][3] in cell units."""
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    codes = np.zeros((nz, ny, nx), dtype=np.uint32)
    nobj = C.c_int64(0)
    rc = lib().ref_forest_codes(_ptr(p), p.shape[0], nx, ny, nz, float(ym_frac),
                                codes.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(nobj))
    if rc != 0:
        raise ValueError("invalid point cloud or y_m fraction")
    return codes, nobj.value


def forest_decode(code):
    h, y, q = C.c_int(), C.c_int(), C.c_int()
    lib().ref_forest_decode(int(code), C.byref(h), C.byref(y), C.byref(q))
    return h.value, y.value, q.value


def forest_lad(code, afm, constant=False):
    return lib().ref_forest_lad(int(code), float(afm), int(constant))


def gelu(x):
    return lib().ref_gelu(float(x))


def softplus(x):
    return lib().ref_softplus(float(x))


def threads():
    return lib().ref_threads()


# --------------------------------------------------------------------------
# learned closure (FP64)
# --------------------------------------------------------------------------

NPARAM = 4865


def mlp_apply(params, Z):
    p = np.ascontiguousarray(params, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    o = np.zeros(Z.shape[0])
    lib().ref_mlp_apply(_ptr(p), _ptr(Z), Z.shape[0], _ptr(o))
    return o


def mlp_loss_grad(params, Z, y):
    p = np.ascontiguousarray(params, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(NPARAM)
    loss = lib().ref_mlp_loss_grad(_ptr(p), _ptr(Z), _ptr(y), Z.shape[0], _ptr(g))
    return loss, g


class MLP:
    """Oracle view of a closure blob."""

    def __init__(self, blob: bytes):
        self._blob = bytes(blob)
        self.h = lib().ref_mlp_load(self._blob, len(self._blob))
        if not self.h:
            raise ValueError("bad closure blob")

    def predict(self, X, smag_nut=None):
        X = np.ascontiguousarray(X, dtype=np.float64)
        n = X.shape[0]
        nut = np.zeros(n)
        fb = (C.c_int * n)()
        s = None if smag_nut is None else np.ascontiguousarray(smag_nut, dtype=np.float64)
        lib().ref_mlp_predict(self.h, _ptr(X), n, _ptr(s), _ptr(nut), fb)
        return nut, np.array(list(fb), dtype=np.int32)

    def features(self, tau0, rho, Pineq, yh, lad):
        P = np.ascontiguousarray(Pineq, dtype=np.float64).reshape(9)
        x = np.zeros(9)
        lib().ref_mlp_features(self.h, tau0, rho, _ptr(P), yh, lad, _ptr(x))
        return x

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.ref_mlp_free(self.h)
            self.h = None


# --------------------------------------------------------------------------
# simulation
# --------------------------------------------------------------------------

class RefLBM:
    """FP64 double-buffered pull-scheme LBM; one object per simulation."""

    def __init__(self, nx, ny, nz, tau0, csmag=0.0, g=(0.0, 0.0, 0.0),
                 bc_lo=BC_BOUNCEBACK, bc_hi=BC_FREESLIP):
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.h = lib().ref_create(nx, ny, nz, float(tau0), float(csmag), float(g[0]),
                                  float(g[1]), float(g[2]), int(bc_lo), int(bc_hi))
        if not self.h:
            raise ValueError("invalid oracle parameters")
        self._mlp = None

    def close(self):
        if self.h:
            lib().ref_destroy(self.h)
            self.h = None

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.ref_destroy(self.h)
            self.h = None

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def set_canopy(self, cd, lad, vector_drag=False):
        lad = np.ascontiguousarray(lad, dtype=np.float64)
        if lib().ref_set_canopy(self.h, float(cd), _ptr(lad), lad.size, int(vector_drag)) != 0:
            raise ValueError("lad length must equal ny")

    def set_forest(self, cd, afm, codes, constant=False, vector_drag=False):
        codes = np.ascontiguousarray(codes, dtype=np.uint32).reshape(self.shape)
        if lib().ref_set_forest(self.h, float(cd), float(afm), int(constant),
                                codes.ctypes.data_as(C.POINTER(C.c_uint32)),
                                int(vector_drag)) != 0:
            raise MemoryError("oracle forest")

    def set_wall_velocity(self, u):
        lib().ref_set_wall_velocity(self.h, float(u[0]), float(u[1]), float(u[2]))

    def set_closure(self, mlp):
        self._mlp = mlp
        lib().ref_set_closure(self.h, mlp.h if mlp is not None else None)

    def set_closure_interval(self, every):
        if lib().ref_set_closure_interval(self.h, int(every)) != 0:
            raise ValueError("every must be >= 1")

    def init(self, rho, u):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        lib().ref_init(self.h, _ptr(rho), _ptr(u))

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape((19,) + self.shape)
        lib().ref_set_f(self.h, _ptr(f))

    def get_f(self):
        f = np.zeros((19,) + self.shape)
        lib().ref_get_f(self.h, _ptr(f))
        return f

    def pull(self):
        f = np.zeros((19,) + self.shape)
        lib().ref_pull(self.h, _ptr(f))
        return f

    def step(self, n=1):
        lib().ref_step(self.h, int(n))

    def moments(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        nut = np.zeros(self.shape)
        d = np.zeros(11)
        lib().ref_moments(self.h, _ptr(rho), _ptr(u), _ptr(nut), _ptr(d))
        return rho, u, nut, dict(zip(DIAG_KEYS, d.tolist()))

    def stats(self, op, every=0):
        prof = np.zeros((self.ny, 10))
        ns = C.c_int64(0)
        if lib().ref_stats(self.h, int(op), int(every), _ptr(prof), C.byref(ns)) != 0:
            raise ValueError("bad stats op")
        return prof, ns.value

    def stats_reset(self):
        self.stats(0)

    def stats_enable(self, every):
        self.stats(1, every)

    def stats_read(self):
        return self.stats(2)
