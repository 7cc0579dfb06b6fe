"""ctypes marshalling for the C oracle (``liborc.so``) -- TEST INFRASTRUCTURE ONLY.

Argument marshalling only; every computation happens in ``orc.c``.  Bunches
are numpy arrays of shape (6, n) (rows x, y, t, px, py, pt), FP64, C order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORC_SANITIZE=1 builds and loads an AddressSanitizer + UndefinedBehaviorSanitizer
# copy (liborc_san.so); the interpreter then needs the sanitizer runtimes
# preloaded, e.g. LD_PRELOAD="$(gcc -print-file-name=libasan.so)
# $(gcc -print-file-name=libubsan.so)" ASAN_OPTIONS=detect_leaks=0.
_SANITIZE = os.environ.get("ORC_SANITIZE", "") not in ("", "0")
_SO = os.path.join(_HERE, "liborc_san.so" if _SANITIZE else "liborc.so")
_SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all"]
MEC2_MEV = 0.51099895000   # electron rest energy (CODATA 2018)


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               *(_SAN_FLAGS if _SANITIZE else []),
               "-o", _SO + ".tmp", os.path.join(_HERE, "orc.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Elem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nsub", C.c_int32), ("L", C.c_double), ("k", C.c_double),
                ("angle", C.c_double), ("f", C.c_double), ("n0_m3", C.c_double),
                ("dE_MeV", C.c_double), ("chirp", C.c_double), ("chromatic", C.c_int32),
                ("pad", C.c_int32)]


class _Ref(C.Structure):
    _fields_ = [("mass_MeV", C.c_double), ("gamma", C.c_double), ("s", C.c_double)]


class _Shape(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("hidden", C.c_int32),
                ("n_out", C.c_int32)]


_KIND = {"drift": 1, "quad": 2, "sbend": 3, "thin_lens": 4, "stage": 5}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp, i64, i32 = C.POINTER(C.c_double), C.c_int64, C.c_int32
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_fill_gaussian.argtypes = [dp, i64, i64, C.c_uint64, dp, dp, i64, C.POINTER(C.c_int64)]
        L.orc_push.argtypes = [dp, i64, i64, C.POINTER(_Elem), i32, C.POINTER(_Ref)]
        L.orc_moments.argtypes = [dp, i64, i64, dp, dp]
        L.orc_emittances.argtypes = [dp, dp]
        L.orc_compare.argtypes = [dp, dp, i64, i64, dp, dp, dp]
        L.orc_bf16.argtypes = [C.c_float]
        L.orc_bf16.restype = C.c_float
        fp = C.POINTER(C.c_float)
        L.orc_prelu_nparams.argtypes = [C.POINTER(_Shape)]
        L.orc_prelu_nparams.restype = i64
        L.orc_prelu_init.argtypes = [C.POINTER(_Shape), C.c_uint64, fp]
        L.orc_prelu_apply.argtypes = [C.POINTER(_Shape), fp, dp, C.c_int, dp, dp, i64, i64]
        L.orc_prelu_loss_grad.argtypes = [C.POINTER(_Shape), fp, dp, dp, dp, i64,
                                          C.POINTER(C.c_int64), i64, dp, dp]
        L.orc_mlp_nparams.argtypes = [C.POINTER(_Shape)]
        L.orc_mlp_nparams.restype = i64
        L.orc_mlp_init.argtypes = [C.POINTER(_Shape), C.c_uint64, fp]
        L.orc_mlp_apply.argtypes = [C.POINTER(_Shape), fp, dp, C.c_int, dp, dp, i64, i64]
        L.orc_mlp_loss_grad.argtypes = [C.POINTER(_Shape), fp, dp, C.c_int, dp, dp, i64,
                                        C.POINTER(C.c_int64), i64, dp, dp]
        L.orc_adam_step.argtypes = [i64, fp, dp, dp, dp, i64, C.c_double, C.c_double,
                                    C.c_double, C.c_double]
        L.orc_norm_stats.argtypes = [dp, dp, i64, i64, dp]
        L.orc_lr_at.argtypes = [i64, i64, C.c_double, C.c_double]
        L.orc_lr_at.restype = C.c_double
        L.orc_epoch_perm.argtypes = [i64, C.c_uint64, i64, C.POINTER(C.c_int64)]
        L.orc_mlp_train.argtypes = [C.POINTER(_Shape), fp, dp, C.c_int, dp, dp, i64, i64, i64, i64,
                                    i64, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_uint64, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def _bunch(z):
    z = np.asarray(z)
    if z.dtype != np.float64 or z.ndim != 2 or z.shape[0] != 6 or not z.flags.c_contiguous:
        raise TypeError("bunch must be a C-contiguous float64 array of shape (6, n)")
    return z


@dataclass
class Ref:
    """Reference particle: total energy via gamma, path length s."""
    gamma: float
    s: float = 0.0
    mass_MeV: float = MEC2_MEV

    @staticmethod
    def from_energy(E_MeV: float) -> "Ref":
        return Ref(gamma=E_MeV / MEC2_MEV)


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def fill_gaussian(n, seed, mean=(0.0,) * 6, sigma=(1.0,) * 6, i0=0, idx=None):
    idx_arr = None
    if idx is not None:
        idx_arr = np.ascontiguousarray(idx, dtype=np.int64)
        n = len(idx_arr)
    z = np.empty((6, n), dtype=np.float64)
    m = np.ascontiguousarray(mean, dtype=np.float64)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    ip = idx_arr.ctypes.data_as(C.POINTER(C.c_int64)) if idx_arr is not None else None
    _check(lib().orc_fill_gaussian(_dp(z), n, n, seed, _dp(m), _dp(s), i0, ip), "fill")
    return z


def _elements(seq):
    arr = (_Elem * max(1, len(seq)))()
    for i, e in enumerate(seq):
        kind = e.kind if hasattr(e, "kind") else "stage"
        if kind == "stage" or not hasattr(e, "kind"):
            arr[i] = _Elem(5, int(e.nsub), float(e.L), 0.0, 0.0, 0.0, float(e.n0_m3), float(e.dE_MeV),
                           float(getattr(e, "chirp", 0.0)), 0, 0)
        else:
            arr[i] = _Elem(_KIND[kind], 0, float(e.L), float(e.k), float(e.angle), float(e.f), 0.0, 0.0,
                           0.0, int(bool(getattr(e, "chromatic", False))), 0)
    return arr


def push(z, seq, ref: Ref):
    """Track bunch z in place through elements/stages; updates ref."""
    z = _bunch(z)
    r = _Ref(ref.mass_MeV, ref.gamma, ref.s)
    _check(lib().orc_push(_dp(z), z.shape[1], z.shape[1], _elements(seq), len(seq), C.byref(r)), "push")
    ref.gamma, ref.s = r.gamma, r.s
    return z


def track(z, beamline, ref: Ref):
    """Beamline = list of segments (element lists or Stage objects)."""
    for seg in beamline:
        push(z, seg if isinstance(seg, list) else [seg], ref)
    return z


def moments(z):
    z = _bunch(z)
    m = np.empty(6)
    c21 = np.empty(21)
    _check(lib().orc_moments(_dp(z), z.shape[1], z.shape[1], _dp(m), _dp(c21)), "moments")
    return m, c21


def cov_matrix(c21):
    c = np.empty((6, 6))
    q = 0
    for j in range(6):
        for k in range(j, 6):
            c[j, k] = c[k, j] = c21[q]
            q += 1
    return c


def emittances(c21):
    c21 = np.ascontiguousarray(c21, dtype=np.float64)
    e = np.empty(3)
    lib().orc_emittances(_dp(c21), _dp(e))
    return e


def compare(s, f):
    s, f = _bunch(s), _bunch(f)
    assert s.shape == f.shape
    rms, cen, er = np.empty(6), np.empty(6), np.empty(3)
    _check(lib().orc_compare(_dp(s), _dp(f), s.shape[1], s.shape[1], _dp(rms), _dp(cen), _dp(er)), "compare")
    return rms, cen, er


def bf16(x):
    f = lib().orc_bf16
    return np.array([f(float(v)) for v in np.ravel(x)], dtype=np.float32).reshape(np.shape(x))


# ---------------------------------------------------------------- MLP
def shape(n_in=6, width=64, hidden=3, n_out=6):
    return _Shape(n_in, width, hidden, n_out)


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def mlp_nparams(sh):
    return int(lib().orc_mlp_nparams(C.byref(sh)))


def mlp_init(sh, seed):
    p = np.empty(mlp_nparams(sh), dtype=np.float32)
    lib().orc_mlp_init(C.byref(sh), seed, _fp(p))
    return p


def mlp_apply(sh, params, norm, zin, mode=0):
    zin = _bunch(zin)
    params = np.ascontiguousarray(params, dtype=np.float32)
    norm = np.ascontiguousarray(norm, dtype=np.float64)
    out = np.empty_like(zin)
    _check(lib().orc_mlp_apply(C.byref(sh), _fp(params), _dp(norm), mode, _dp(zin), _dp(out),
                               zin.shape[1], zin.shape[1]), "mlp_apply")
    return out


def mlp_loss_grad(sh, params, norm, zin, zout, idx, mode=0):
    zin, zout = _bunch(zin), _bunch(zout)
    params = np.ascontiguousarray(params, dtype=np.float32)
    norm = np.ascontiguousarray(norm, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    g = np.empty(mlp_nparams(sh))
    loss = C.c_double()
    _check(lib().orc_mlp_loss_grad(C.byref(sh), _fp(params), _dp(norm), mode, _dp(zin), _dp(zout),
                                   zin.shape[1], idx.ctypes.data_as(C.POINTER(C.c_int64)), len(idx),
                                   _dp(g), C.byref(loss)), "loss_grad")
    return loss.value, g


def adam_step(params, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    params = np.ascontiguousarray(params, dtype=np.float32).copy()
    m, v = m.copy(), v.copy()
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    _check(lib().orc_adam_step(len(params), _fp(params), _dp(m), _dp(v), _dp(grad), t, lr, b1, b2, eps), "adam")
    return params, m, v


def norm_stats(zin, zout, n_train):
    zin, zout = _bunch(zin), _bunch(zout)
    norm = np.empty(24)
    _check(lib().orc_norm_stats(_dp(zin), _dp(zout), n_train, zin.shape[1], _dp(norm)), "norm_stats")
    return norm


def lr_at(t, planned, lr, lr_final):
    return float(lib().orc_lr_at(t, planned, lr, lr_final))


def epoch_perm(n, seed, epoch):
    p = np.empty(n, dtype=np.int64)
    lib().orc_epoch_perm(n, seed, epoch, p.ctypes.data_as(C.POINTER(C.c_int64)))
    return p


def mlp_train(sh, params, zin, zout, batch, epochs, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8,
              train_frac=0.7, shuffle_seed=0, mode=1, max_steps=-1, lr_final=None):
    zin, zout = _bunch(zin), _bunch(zout)
    params = np.ascontiguousarray(params, dtype=np.float32).copy()
    norm = np.empty(24)
    log = np.zeros(2 * epochs)
    _check(lib().orc_mlp_train(C.byref(sh), _fp(params), _dp(norm), mode, _dp(zin), _dp(zout),
                               zin.shape[1], zin.shape[1], batch, epochs, max_steps, lr,
                               lr if lr_final is None else lr_final, b1, b2, eps,
                               train_frac, shuffle_seed, _dp(log)), "train")
    return params, norm, log.reshape(epochs, 2)


# ---------------------------------------------------------------- PReLU network
def prelu_nparams(sh):
    return int(lib().orc_prelu_nparams(C.byref(sh)))


def prelu_init(sh, seed):
    p = np.empty(prelu_nparams(sh), dtype=np.float32)
    lib().orc_prelu_init(C.byref(sh), seed, _fp(p))
    return p


def prelu_apply(sh, params, norm, zin, mode=0):
    zin = _bunch(zin)
    params = np.ascontiguousarray(params, dtype=np.float32)
    norm = np.ascontiguousarray(norm, dtype=np.float64)
    out = np.empty_like(zin)
    _check(lib().orc_prelu_apply(C.byref(sh), _fp(params), _dp(norm), mode, _dp(zin), _dp(out),
                                 zin.shape[1], zin.shape[1]), "prelu_apply")
    return out


def prelu_loss_grad(sh, params, norm, zin, zout, idx):
    zin, zout = _bunch(zin), _bunch(zout)
    params = np.ascontiguousarray(params, dtype=np.float32)
    norm = np.ascontiguousarray(norm, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    g = np.empty(prelu_nparams(sh))
    loss = C.c_double()
    _check(lib().orc_prelu_loss_grad(C.byref(sh), _fp(params), _dp(norm), _dp(zin), _dp(zout),
                                     zin.shape[1], idx.ctypes.data_as(C.POINTER(C.c_int64)), len(idx),
                                     _dp(g), C.byref(loss)), "prelu_loss_grad")
    return loss.value, g
