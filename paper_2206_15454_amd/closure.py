"""Closure blob: the serialized learned eddy-viscosity closure that
``lbm_set_closure`` loads (layout documented in include/lbm.h).

Weights are stored as bfloat16 (round to nearest even), biases and the
feature standardisation as float32.  Flat parameter order:
W1[64][9], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
import struct

import numpy as np

NIN, NH1, NH2 = 9, 64, 64
NPARAM = NH1 * NIN + NH1 + NH2 * NH1 + NH2 + NH2 + 1
BLOB_BYTES = 10184
FEATURES = ("trP", "trP2", "trP3", "nPn", "nP2n", "sqrt_trP2", "y_over_h", "lad", "width")


def bf16_bits(x):
    """float32 -> bfloat16 bits, round to nearest even (finite values)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def bf16_round(x):
    """values rounded to bfloat16, as float64"""
    return (bf16_bits(x).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def split(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAM
    o = 0
    W1 = p[o:o + NH1 * NIN].reshape(NH1, NIN); o += NH1 * NIN
    b1 = p[o:o + NH1]; o += NH1
    W2 = p[o:o + NH2 * NH1].reshape(NH2, NH1); o += NH2 * NH1
    b2 = p[o:o + NH2]; o += NH2
    w3 = p[o:o + NH2]; o += NH2
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def join(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def stored_params(p):
    """The flat parameters as the blob stores them (weights bf16, biases f32)."""
    W1, b1, W2, b2, w3, b3 = split(p)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return join(bf16_round(W1), f32(b1), bf16_round(W2), f32(b2), bf16_round(w3),
                float(np.float32(b3)))


def make_blob(params, mean, std, lo, hi, scale, canopy_h):
    W1, b1, W2, b2, w3, b3 = split(params)
    vec = lambda a: np.asarray(a, dtype=np.float64).reshape(NIN)
    out = bytearray(b"LBMC")
    out += struct.pack("<5I", 1, NIN, NH1, NH2, 0)
    out += struct.pack("<36f", *vec(mean), *vec(std), *vec(lo), *vec(hi))
    out += struct.pack("<4f", float(scale), float(canopy_h), 0.0, 0.0)
    out += struct.pack("<132f", *b1, *b2, float(b3), 0.0, 0.0, 0.0)
    out += bf16_bits(np.concatenate([np.ravel(W1), np.ravel(W2), np.ravel(w3)])).tobytes()
    assert len(out) == BLOB_BYTES
    return bytes(out)


def read_blob(blob):
    """(params as stored, mean, std, lo, hi, scale, canopy_h)"""
    b = bytes(blob)
    if len(b) != BLOB_BYTES or b[:4] != b"LBMC":
        raise ValueError("not a closure blob")
    f = np.frombuffer(b, dtype="<f4", count=36, offset=24).astype(np.float64)
    mean, std, lo, hi = f[0:9], f[9:18], f[18:27], f[27:36]
    scale, h = struct.unpack_from("<2f", b, 168)
    bias = np.frombuffer(b, dtype="<f4", count=129, offset=184).astype(np.float64)
    w = np.frombuffer(b, dtype="<u2", offset=712).astype(np.uint32)
    wv = (w << 16).view(np.float32).astype(np.float64)
    W1 = wv[:NH1 * NIN].reshape(NH1, NIN)
    W2 = wv[NH1 * NIN:NH1 * NIN + NH2 * NH1].reshape(NH2, NH1)
    w3 = wv[NH1 * NIN + NH2 * NH1:]
    p = join(W1, bias[:64], W2, bias[64:128], w3, bias[128])
    return p, mean, std, lo, hi, scale, h


def with_range(blob, feature, lo=None, hi=None):
    """The same closure with the valid range of one raw feature (index or
    name in FEATURES) changed; cells outside it use Smagorinsky.  The
    weights are carried over bit for bit."""
    k = FEATURES.index(feature) if isinstance(feature, str) else int(feature)
    p, mean, std, rlo, rhi, scale, h = read_blob(blob)
    rlo, rhi = rlo.copy(), rhi.copy()
    if lo is not None:
        rlo[k] = lo
    if hi is not None:
        rhi[k] = hi
    return make_blob(p, mean, std, rlo, rhi, scale, h)


def everywhere(blob):
    """The same network with every input range opened: every cell evaluates
    it (no Smagorinsky fallback except for non-finite outputs).  For timing
    it on workloads other than the one it was trained on."""
    p, mean, std, _, _, scale, h = read_blob(blob)
    return make_blob(p, mean, std, np.full(NIN, -3e38), np.full(NIN, 3e38), scale, h)


def timing_blob(canopy_h, seed=0):
    """A random network whose input ranges admit every cell (for timing the
    closure kernel; its nu_t is small and positive)."""
    rng = np.random.default_rng(seed)
    p = join(rng.normal(size=(NH1, NIN)) / 3.0, rng.normal(size=NH1) * 0.1,
             rng.normal(size=(NH2, NH1)) / 8.0, rng.normal(size=NH2) * 0.1,
             rng.normal(size=NH2) / 8.0, -2.0)
    mean = np.array([0, 0, 0, 0, 0, 1e-3, 1.5, 0.1, 1.0])
    std = np.array([1e-4, 1e-6, 1e-9, 1e-3, 1e-6, 1e-3, 1.0, 0.15, 1.0])
    return make_blob(p, mean, std, np.full(NIN, -3e38), np.full(NIN, 3e38), 1e-5, canopy_h)


def trained_blob():
    """The closure trained on the production canopy case (512x128x256, h = 12
    cells) from a run at twice the resolution; see data/*.json for the record."""
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                        "closure_canopy_512x128x256.bin")
    with open(path, "rb") as f:
        return f.read()


def canopy_layer_blob(cut=4.0):
    """The trained closure used only in the canopy layer, y/h <= cut
    (Smagorinsky above, through the y/h feature range).  Measured on the
    production canopy case, it keeps the spanwise fluctuations that the
    unrestricted closure damps in the upper layer."""
    return with_range(trained_blob(), "y_over_h", hi=cut)
