"""Thin Python binding of the C ABI in ``include/lbm.h`` (ctypes).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbmx.so``.  PyTorch supplies device memory (one uint8 tensor per
simulation) and the stream (torch's current stream unless one is given).
There is no CPU fallback: without the built library every call raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBMX_LIB") or os.path.join(_HERE, "liblbmx.so")

STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3, "bf16sr": 4}
BC = {"periodic": 0, "bounceback": 1, "freeslip": 2, "equilibrium": 3}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EUNSTABLE"}


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("storage", C.c_int32), ("tau0", C.c_double), ("c_smag", C.c_double),
                ("g", C.c_double * 3), ("bc_ylo", C.c_int32), ("bc_yhi", C.c_int32),
                ("stream", C.c_void_p), ("u_wall", C.c_double * 3), ("forest_map", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("mom", C.c_double * 3), ("impulse", C.c_double * 3),
                ("max_u", C.c_double), ("t", C.c_int64), ("nonfinite", C.c_int64),
                ("mlp_fallback", C.c_int64)]

    def as_dict(self):
        return {"mass": self.mass, "mom_x": self.mom[0], "mom_y": self.mom[1],
                "mom_z": self.mom[2], "imp_x": self.impulse[0], "imp_y": self.impulse[1],
                "imp_z": self.impulse[2], "max_u": self.max_u, "t": self.t,
                "nonfinite": self.nonfinite, "mlp_fallback": self.mlp_fallback}


class TrainParams(C.Structure):
    _fields_ = [("mean", C.c_float * 9), ("std", C.c_float * 9), ("out_scale", C.c_float),
                ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("max_batch", C.c_int32), ("stream", C.c_void_p)]


EXPORTS = ("lbm_lattice", "lbm_required_bytes", "lbm_create", "lbm_destroy", "lbm_last_error",
           "lbm_set_stream", "lbm_set_canopy", "lbm_set_closure", "lbm_init", "lbm_step",
           "lbm_moments", "lbm_stats", "lbm_set_f", "lbm_get_f", "lbm_lad_lalic",
           "lbm_closure_samples", "lbm_train_create", "lbm_train_step", "lbm_train_get",
           "lbm_train_destroy", "lbm_train_last_error", "lbm_forest_codes", "lbm_set_forest",
           "lbm_set_closure_interval", "lbm_closure_samples_noalloc")

# capacity of lbm_closure_samples_noalloc's fixed work area (include/lbm.h)
NOALLOC_MAX_COARSE = 262144
NOALLOC_MAX_LAD = 4096

_lib = None


def lib():
    """Load liblbmx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
        L.lbm_lattice.restype = i32
        L.lbm_lattice.argtypes = [C.POINTER(i32), dp]
        L.lbm_required_bytes.restype = C.c_size_t
        L.lbm_required_bytes.argtypes = [C.POINTER(Params)]
        L.lbm_create.restype = i32
        L.lbm_create.argtypes = [C.POINTER(Params), vp, C.c_size_t, C.POINTER(vp)]
        L.lbm_destroy.restype = i32
        L.lbm_destroy.argtypes = [vp]
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_last_error.argtypes = [vp]
        L.lbm_set_stream.restype = i32
        L.lbm_set_stream.argtypes = [vp, vp]
        L.lbm_set_canopy.restype = i32
        L.lbm_set_canopy.argtypes = [vp, C.c_double, dp, i32, i32]
        L.lbm_set_closure.restype = i32
        L.lbm_set_closure.argtypes = [vp, i32, C.c_char_p, C.c_size_t]
        L.lbm_init.restype = i32
        L.lbm_init.argtypes = [vp, vp, vp, i32]
        L.lbm_step.restype = i32
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_moments.restype = i32
        L.lbm_moments.argtypes = [vp, vp, vp, vp, i32, C.POINTER(Diag)]
        L.lbm_stats.restype = i32
        L.lbm_stats.argtypes = [vp, i32, i32, dp, C.POINTER(i64)]
        L.lbm_set_f.restype = i32
        L.lbm_set_f.argtypes = [vp, vp, i32]
        L.lbm_get_f.restype = i32
        L.lbm_get_f.argtypes = [vp, vp, i32]
        L.lbm_lad_lalic.restype = i32
        L.lbm_lad_lalic.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, i32, dp]
        L.lbm_closure_samples.restype = i32
        L.lbm_closure_samples.argtypes = [vp, C.c_double, C.c_double, dp, vp, vp, i64]
        L.lbm_closure_samples_noalloc.restype = i32
        L.lbm_closure_samples_noalloc.argtypes = [vp, C.c_double, C.c_double, dp, vp, vp, i64]
        L.lbm_train_create.restype = i32
        L.lbm_train_create.argtypes = [C.POINTER(TrainParams), C.POINTER(C.c_float), C.POINTER(vp)]
        L.lbm_train_step.restype = i32
        L.lbm_train_step.argtypes = [vp, vp, vp, i64, i32, C.POINTER(C.c_float)]
        L.lbm_train_get.restype = i32
        L.lbm_train_get.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.lbm_train_destroy.restype = i32
        L.lbm_train_destroy.argtypes = [vp]
        L.lbm_train_last_error.restype = C.c_char_p
        L.lbm_train_last_error.argtypes = [vp]
        L.lbm_forest_codes.restype = i32
        L.lbm_forest_codes.argtypes = [dp, i64, i32, i32, i32, C.c_double,
                                       C.POINTER(C.c_uint32), C.POINTER(i64)]
        L.lbm_set_closure_interval.restype = i32
        L.lbm_set_closure_interval.argtypes = [vp, i32]
        L.lbm_set_forest.restype = i32
        L.lbm_set_forest.argtypes = [vp, C.c_double, C.c_double, i32, C.POINTER(C.c_uint32), i32]
        _lib = L
    return _lib


def lattice():
    c = (C.c_int32 * 57)()
    w = np.zeros(19)
    lib().lbm_lattice(c, w.ctypes.data_as(C.POINTER(C.c_double)))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w


def lad_lalic(h, ym, ny, afm=1.0, lai=0.0):
    """Eq. (af_theory) at cell centres (the library's host routine)."""
    out = np.zeros(ny)
    st = lib().lbm_lad_lalic(float(h), float(ym), float(afm), float(lai), int(ny),
                             out.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise LBMError(st, "invalid LAD parameters")
    return out


def forest_codes(points, nx, ny, nz, ym_frac=0.7):
    """Per-cell forest codes [nz][ny][nx] (uint32) and the number of forest
    objects from a point cloud [npts][3] in cell units (the library's host
    routine)."""
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    codes = np.zeros((nz, ny, nx), dtype=np.uint32)
    nobj = C.c_int64(0)
    st = lib().lbm_forest_codes(p.ctypes.data_as(C.POINTER(C.c_double)), p.shape[0], int(nx),
                                int(ny), int(nz), float(ym_frac),
                                codes.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(nobj))
    if st != 0:
        raise LBMError(st, "invalid point cloud or y_m fraction")
    return codes, nobj.value


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class LBM:
    """One simulation context on the current GPU."""

    def __init__(self, nx, ny, nz, storage="f32", tau0=0.52, c_smag=0.01, g=(0.0, 0.0, 0.0),
                 bc_lo="bounceback", bc_hi="freeslip", stream=None, u_wall=(0.0, 0.0, 0.0),
                 forest_map=False):
        import torch

        self.torch = torch
        L = lib()
        bc_lo = BC[bc_lo] if isinstance(bc_lo, str) else int(bc_lo)
        bc_hi = BC[bc_hi] if isinstance(bc_hi, str) else int(bc_hi)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.p = Params(nx, ny, nz, STORAGE[storage], float(tau0), float(c_smag),
                        (C.c_double * 3)(*map(float, g)), bc_lo, bc_hi,
                        C.c_void_p(self.stream.cuda_stream),
                        (C.c_double * 3)(*map(float, u_wall)), int(bool(forest_map)))
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.storage = storage
        nbytes = L.lbm_required_bytes(C.byref(self.p))
        if nbytes == 0:
            raise LBMError(1, "invalid parameters")
        # device memory from torch's allocator (one buffer, 256-byte aligned)
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = self.buf.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        h = C.c_void_p()
        self._check(L.lbm_create(C.byref(self.p), C.c_void_p(aligned), nbytes, C.byref(h)),
                    "lbm_create")
        self.h = h

    # -- helpers ----------------------------------------------------------
    def _check(self, st, what):
        if st != 0:
            msg = lib().lbm_last_error(getattr(self, "h", None)).decode() if getattr(
                self, "h", None) else what
            raise LBMError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None
            self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _in(self, a, count):
        """(pointer, on_device, keepalive) for an FP64 input array."""
        if _is_torch(a):
            t = a.detach().to(dtype=self.torch.float64).contiguous()
            if t.numel() != count:
                raise ValueError(f"expected {count} values, got {t.numel()}")
            return C.c_void_p(t.data_ptr()), int(t.is_cuda), t
        arr = np.ascontiguousarray(a, dtype=np.float64)
        if arr.size != count:
            raise ValueError(f"expected {count} values, got {arr.size}")
        return C.c_void_p(arr.ctypes.data), 0, arr

    # -- ABI ----------------------------------------------------------------
    def set_canopy(self, cd, lad, vector_drag=False):
        lad = np.ascontiguousarray(lad, dtype=np.float64)
        self._check(lib().lbm_set_canopy(self.h, float(cd),
                                         lad.ctypes.data_as(C.POINTER(C.c_double)), lad.size,
                                         int(bool(vector_drag))), "lbm_set_canopy")

    def set_forest(self, cd, afm, codes, constant=False, vector_drag=False):
        """Per-cell LAD from forest codes (needs forest_map=True)."""
        codes = np.ascontiguousarray(codes, dtype=np.uint32)
        if codes.size != self.n:
            raise ValueError("codes must have nx*ny*nz entries")
        self._check(lib().lbm_set_forest(self.h, float(cd), float(afm), int(bool(constant)),
                                         codes.ctypes.data_as(C.POINTER(C.c_uint32)),
                                         int(bool(vector_drag))), "lbm_set_forest")

    def set_closure(self, blob=None):
        if blob is None:
            self._check(lib().lbm_set_closure(self.h, 0, None, 0), "lbm_set_closure")
        else:
            blob = bytes(blob)
            self._check(lib().lbm_set_closure(self.h, 1, blob, len(blob)), "lbm_set_closure")

    def set_closure_interval(self, every):
        """Evaluate the learned closure every `every` steps, reuse its nu_t between."""
        self._check(lib().lbm_set_closure_interval(self.h, int(every)), "lbm_set_closure_interval")

    def init(self, rho, u):
        pr, dr, kr = self._in(rho, self.n)
        pu, du, ku = self._in(u, 3 * self.n)
        if dr != du:
            raise ValueError("rho and u must both be host or both be device arrays")
        self._check(lib().lbm_init(self.h, pr, pu, dr), "lbm_init")

    def step(self, n=1):
        self._check(lib().lbm_step(self.h, int(n)), "lbm_step")

    def moments(self, device=False, check=True):
        """(rho, u, nu_t, diag): numpy arrays, or torch cuda tensors with
        device=True.  check=False returns the outputs of an unstable state
        instead of raising."""
        torch = self.torch
        if device:
            rho = torch.empty(self.shape, dtype=torch.float64, device="cuda")
            u = torch.empty((3,) + self.shape, dtype=torch.float64, device="cuda")
            nut = torch.empty(self.shape, dtype=torch.float64, device="cuda")
            ptrs = [C.c_void_p(t.data_ptr()) for t in (rho, u, nut)]
        else:
            rho = np.zeros(self.shape)
            u = np.zeros((3,) + self.shape)
            nut = np.zeros(self.shape)
            ptrs = [C.c_void_p(a.ctypes.data) for a in (rho, u, nut)]
        d = Diag()
        st = lib().lbm_moments(self.h, *ptrs, int(device), C.byref(d))
        if st != 0 and (check or st != 5):
            self._check(st, "lbm_moments")
        return rho, u, nut, d.as_dict()

    def diag(self):
        d = Diag()
        self._check(lib().lbm_moments(self.h, None, None, None, 0, C.byref(d)), "lbm_moments")
        return d.as_dict()

    def stats(self, op, every=0):
        prof = np.zeros((self.shape[1], 10))
        ns = C.c_int64(0)
        self._check(lib().lbm_stats(self.h, int(op), int(every),
                                    prof.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ns)),
                    "lbm_stats")
        return prof, ns.value

    def stats_reset(self):
        self.stats(0)

    def stats_enable(self, every):
        self.stats(1, every)

    def stats_read(self):
        return self.stats(2)

    def set_f(self, f):
        p, dev, keep = self._in(f, 19 * self.n)
        self._check(lib().lbm_set_f(self.h, p, dev), "lbm_set_f")

    def get_f(self, device=False):
        if device:
            out = self.torch.empty((19,) + self.shape, dtype=self.torch.float64, device="cuda")
            p = C.c_void_p(out.data_ptr())
        else:
            out = np.zeros((19,) + self.shape)
            p = C.c_void_p(out.ctypes.data)
        self._check(lib().lbm_get_f(self.h, p, int(device)), "lbm_get_f")
        return out

    def closure_samples(self, tau0_coarse, canopy_h, lad_coarse, out=None, noalloc=False):
        """(X [nc, 9], y [nc]) float32 torch tensors on the device: training
        samples of the learned closure from this (fine) simulation.  out:
        (X, y) device tensors to write (allocated here if None).  noalloc:
        call lbm_closure_samples_noalloc (no device allocation, no
        synchronisation) instead of lbm_closure_samples."""
        torch = self.torch
        nz, ny, nx = self.shape
        nc = (nx // 2) * (ny // 2) * (nz // 2)
        if out is None:
            X = torch.empty((nc, 9), dtype=torch.float32, device="cuda")
            y = torch.empty(nc, dtype=torch.float32, device="cuda")
        else:
            X, y = out
        lad = np.ascontiguousarray(lad_coarse, dtype=np.float64)
        name = "lbm_closure_samples_noalloc" if noalloc else "lbm_closure_samples"
        self._check(getattr(lib(), name)(self.h, float(tau0_coarse), float(canopy_h),
                                         lad.ctypes.data_as(C.POINTER(C.c_double)),
                                         C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                                         nc), name)
        return X, y


class Trainer:
    """GPU trainer of the closure network (MFMA forward/backward + Adam)."""

    NPARAM = 4865

    def __init__(self, params, mean, std, out_scale, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 max_batch=8192, stream=None):
        import torch

        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        prm = TrainParams((C.c_float * 9)(*map(float, mean)), (C.c_float * 9)(*map(float, std)),
                          float(out_scale), float(lr), float(betas[0]), float(betas[1]),
                          float(eps), int(max_batch), C.c_void_p(self.stream.cuda_stream))
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.NPARAM:
            raise ValueError("expected 4865 parameters")
        h = C.c_void_p()
        st = lib().lbm_train_create(C.byref(prm), p.ctypes.data_as(C.POINTER(C.c_float)),
                                    C.byref(h))
        if st != 0:
            raise LBMError(st, "lbm_train_create")
        self.h = h
        self.max_batch = int(max_batch)

    def _check(self, st, what):
        if st != 0:
            raise LBMError(st, f"{what}: {lib().lbm_train_last_error(self.h).decode()}")

    def step(self, X, y, update=True, loss=True):
        """One batch (torch float32 cuda tensors X [n, 9], y [n]); returns the
        loss (before the update) if requested."""
        X = X.contiguous()
        y = y.contiguous()
        out = C.c_float(0.0)
        self._check(lib().lbm_train_step(self.h, C.c_void_p(X.data_ptr()),
                                         C.c_void_p(y.data_ptr()), int(y.numel()), int(update),
                                         C.byref(out) if loss else None), "lbm_train_step")
        return out.value if loss else None

    def get(self):
        p = np.zeros(self.NPARAM, dtype=np.float32)
        g = np.zeros(self.NPARAM, dtype=np.float32)
        self._check(lib().lbm_train_get(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                        g.ctypes.data_as(C.POINTER(C.c_float))), "lbm_train_get")
        return p, g

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_train_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
