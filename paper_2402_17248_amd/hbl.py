"""Thin Python binding of libhbl (argument marshalling only).

Every step of the hot path runs in libhbl's HIP kernels; this module converts
arguments, owns no computation, and raises :class:`HblError` on any non-zero
status.  Torch is used for device memory (bunch tensors of shape (6, ld),
FP64, contiguous) and for the current HIP stream.  If libhbl.so is missing
the import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libhbl.so")

HBL_OK, HBL_EINVAL, HBL_EHIP, HBL_ENOMEM, HBL_ENONFINITE, HBL_ESTATE, HBL_EIO = 0, -1, -2, -3, -4, -5, -6
DRIFT, QUAD, SBEND, THIN_LENS, STAGE = 1, 2, 3, 4, 5
FUSED, UNFUSED = 0, 1
MEC2_MEV = 0.51099895000

_KIND = {"drift": DRIFT, "quad": QUAD, "sbend": SBEND, "thin_lens": THIN_LENS, "stage": STAGE}


class HblError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class Element(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nsub", C.c_int32), ("L", C.c_double), ("k", C.c_double),
                ("angle", C.c_double), ("f", C.c_double), ("n0_m3", C.c_double), ("dE_MeV", C.c_double),
                ("chirp", C.c_double), ("chromatic", C.c_int32), ("reserved", C.c_int32)]


class Ref(C.Structure):
    _fields_ = [("mass_MeV", C.c_double), ("gamma", C.c_double), ("s", C.c_double)]

    @staticmethod
    def from_energy(E_MeV: float, s: float = 0.0) -> "Ref":
        return Ref(MEC2_MEV, E_MeV / MEC2_MEV, s)

    def copy(self) -> "Ref":
        return Ref(self.mass_MeV, self.gamma, self.s)


class MlpShape(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("hidden", C.c_int32), ("n_out", C.c_int32)]


class TrainCfg(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("max_steps", C.c_int64), ("lr", C.c_float),
                ("lr_final", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("train_frac", C.c_double), ("shuffle_seed", C.c_uint64), ("keep_best", C.c_int32),
                ("resume", C.c_int32)]


def _load():
    # torch's HIP runtime must be the one libhbl binds to: import torch first,
    # so that libhbl's libamdhip64.so.7 dependency resolves (by soname) to the
    # copy torch already loaded, and the process holds a single HIP runtime.
    import torch  # noqa: F401
    if not os.path.exists(SO_PATH):
        raise ImportError(f"libhbl.so not built at {SO_PATH}: run `python -m paper_2402_17248_amd.build` "
                          "(the HIP library is required; there is no CPU fallback)")
    L = C.CDLL(SO_PATH)
    vp, dp, i64, i32, st = C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.c_int32, C.c_int32
    sigs = {
        "hbl_last_error": ([], C.c_char_p),
        "hbl_version": ([], C.c_char_p),
        "hbl_bunch_fill_gaussian": ([vp, i64, i64, C.c_uint64, dp, dp, i64, vp], st),
        "hbl_lattice_create": ([C.POINTER(Element), i32, C.POINTER(Ref), C.POINTER(vp)], st),
        "hbl_lattice_destroy": ([vp], st),
        "hbl_lattice_info": ([vp, dp, C.POINTER(i32)], st),
        "hbl_push_lattice": ([vp, i64, i64, vp, C.POINTER(Ref), C.c_uint32, vp], st),
        "hbl_apply_stage": ([vp, i64, i64, C.POINTER(Element), C.POINTER(Ref), vp, i64, vp], st),
        "hbl_stage_newton_steps": ([C.POINTER(Element), C.POINTER(Ref), C.POINTER(i32)], st),
        "hbl_apply_stage_gaps": ([vp, i64, i64, vp, C.POINTER(Element), vp, C.POINTER(Ref), vp, i64, vp], st),
        "hbl_moments": ([vp, i64, i64, dp, dp, vp], st),
        "hbl_moments_async": ([vp, i64, i64, vp, vp], st),
        "hbl_moments_async_noalloc": ([vp, i64, i64, vp, vp], st),
        "hbl_emittances": ([dp, dp], st),
        "hbl_compare": ([vp, vp, i64, i64, dp, dp, dp, vp], st),
        "hbl_surrogate_create": ([C.POINTER(MlpShape), C.c_uint64, C.POINTER(vp)], st),
        "hbl_surrogate_destroy": ([vp], st),
        "hbl_surrogate_num_params": ([vp, C.POINTER(i64)], st),
        "hbl_surrogate_get_params": ([vp, C.POINTER(C.c_float), i64], st),
        "hbl_surrogate_set_params": ([vp, C.POINTER(C.c_float), i64], st),
        "hbl_surrogate_get_norm": ([vp, dp], st),
        "hbl_surrogate_set_norm": ([vp, dp], st),
        "hbl_surrogate_set_stage": ([vp, C.POINTER(Element), C.POINTER(Ref)], st),
        "hbl_surrogate_train": ([vp, vp, vp, i64, i64, C.POINTER(TrainCfg), C.POINTER(C.c_float), vp], st),
        "hbl_surrogate_loss_grad": ([vp, vp, vp, i64, C.POINTER(C.c_int32), i32, C.POINTER(C.c_float),
                                     dp, vp], st),
        "hbl_surrogate_apply": ([vp, i64, i64, vp, C.POINTER(Ref), vp], st),
        "hbl_surrogate_apply_gaps": ([vp, i64, i64, vp, vp, vp, C.POINTER(Ref), vp], st),
        "hbl_surrogate_save": ([vp, C.c_char_p], st),
        "hbl_surrogate_load": ([C.c_char_p, C.POINTER(vp)], st),
        "hbl_prelu_create": ([C.POINTER(MlpShape), C.c_uint64, C.POINTER(vp)], st),
        "hbl_prelu_destroy": ([vp], st),
        "hbl_prelu_num_params": ([vp, C.POINTER(i64)], st),
        "hbl_prelu_get_params": ([vp, C.POINTER(C.c_float), i64], st),
        "hbl_prelu_set_params": ([vp, C.POINTER(C.c_float), i64], st),
        "hbl_prelu_get_norm": ([vp, dp], st),
        "hbl_prelu_set_norm": ([vp, dp], st),
        "hbl_prelu_set_stage": ([vp, C.POINTER(Element), C.POINTER(Ref)], st),
        "hbl_prelu_apply": ([vp, i64, i64, vp, C.POINTER(Ref), vp], st),
        "hbl_prelu_apply_gaps": ([vp, i64, i64, vp, vp, vp, C.POINTER(Ref), vp], st),
        "hbl_prelu_loss_grad": ([vp, vp, vp, i64, C.POINTER(C.c_int32), i32, C.POINTER(C.c_float), dp, vp], st),
        "hbl_prelu_train": ([vp, vp, vp, i64, i64, C.POINTER(TrainCfg), C.POINTER(C.c_float), vp], st),
        "hbl_prelu_save": ([vp, C.c_char_p], st),
        "hbl_prelu_set_chunk": ([vp, i64], st),
        "hbl_prelu_load": ([C.c_char_p, C.POINTER(vp)], st),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _call(name, *args):
    rc = getattr(lib, name)(*args)
    if rc != HBL_OK:
        raise HblError(rc, name, lib.hbl_last_error().decode())
    return rc


def exported_symbols() -> Sequence[str]:
    return [n for n in dir(lib) if n.startswith("hbl_")]


def version() -> str:
    return lib.hbl_version().decode()


# ------------------------------------------------------------------ helpers
def _torch():
    import torch
    return torch


def current_stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def new_bunch(n: int, device="cuda"):
    """Device tensor (6, ld) FP64 with ld = n rounded up to even (16-B rows)."""
    torch = _torch()
    ld = n + (n & 1)
    return torch.empty((6, max(ld, 2)), dtype=torch.float64, device=device)


def _on_current_device(t, what):
    """Raise unless tensor t lives on the current HIP device (the library
    launches there; a host tensor or another device's memory would fault)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor, got one on {t.device}")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{what} is on {t.device}, the current device is cuda:{torch.cuda.current_device()}")


def _bunch_args(z, n=None, what="bunch"):
    torch = _torch()
    if not isinstance(z, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if z.dtype != torch.float64 or z.dim() != 2 or z.shape[0] != 6 or z.stride(1) != 1:
        raise TypeError(f"{what} must be a (6, ld) float64 tensor with unit column stride")
    ld = z.stride(0)
    n = z.shape[1] if n is None else int(n)
    if not 0 <= n <= z.shape[1]:
        raise ValueError(f"{what}: n = {n} outside [0, {z.shape[1]}] (the tensor's particle count)")
    _on_current_device(z, what)
    return C.c_void_p(z.data_ptr()), n, ld


def _index_args(idx, limit, what):
    import numpy as np
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim != 1:
        raise ValueError(f"{what}: indices must be one-dimensional")
    if len(idx) and (idx.min() < 0 or idx.max() >= limit):
        raise ValueError(f"{what}: indices must lie in [0, {limit})")
    return idx


def element(e) -> Element:
    """From a workloads.Element / workloads.Stage description."""
    if hasattr(e, "kind"):
        return Element(_KIND[e.kind], 0, float(e.L), float(e.k), float(e.angle), float(e.f), 0.0, 0.0, 0.0,
                       int(bool(getattr(e, "chromatic", False))), 0)
    return Element(STAGE, int(e.nsub), float(e.L), 0.0, 0.0, 0.0, float(e.n0_m3), float(e.dE_MeV),
                   float(getattr(e, "chirp", 0.0)), 0, 0)


# ------------------------------------------------------------------ verbs
def fill_gaussian(z, seed, mean, sigma, n=None, i0=0, stream=None):
    ptr, n, ld = _bunch_args(z, n)
    m = (C.c_double * 6)(*mean)
    s = (C.c_double * 6)(*sigma)
    _call("hbl_bunch_fill_gaussian", ptr, n, ld, seed, m, s, i0, stream or current_stream())


class Lattice:
    """Compiled sequence of linear elements for one reference energy."""

    def __init__(self, elems, ref: Ref):
        arr = (Element * max(1, len(elems)))(*[element(e) if not isinstance(e, Element) else e for e in elems])
        h = C.c_void_p()
        _call("hbl_lattice_create", arr, len(elems), C.byref(ref), C.byref(h))
        self._h = h
        L = C.c_double()
        ne = C.c_int32()
        _call("hbl_lattice_info", h, C.byref(L), C.byref(ne))
        self.length, self.n_elem = L.value, ne.value

    def push(self, z, ref: Ref, fused=True, n=None, stream=None):
        ptr, n, ld = _bunch_args(z, n)
        _call("hbl_push_lattice", ptr, n, ld, self._h, C.byref(ref), FUSED if fused else UNFUSED,
              stream or current_stream())

    def close(self):
        if getattr(self, "_h", None):
            lib.hbl_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_stage(z, stage, ref: Ref, record=None, n=None, stream=None, pre=None, post=None):
    """Fine-step stage; with pre/post (Lattice) the gaps around it run in the same pass."""
    ptr, n, ld = _bunch_args(z, n)
    el = stage if isinstance(stage, Element) else element(stage)
    rp, rld = (None, 0)
    if record is not None:
        rp, _, rld = _bunch_args(record, n, "record")
    if pre is None and post is None:
        _call("hbl_apply_stage", ptr, n, ld, C.byref(el), C.byref(ref), rp, rld, stream or current_stream())
    else:
        _call("hbl_apply_stage_gaps", ptr, n, ld, pre._h if pre else None, C.byref(el),
              post._h if post else None, C.byref(ref), rp, rld, stream or current_stream())


def stage_newton_steps(stage, ref: Ref) -> int:
    """Newton steps per substep the stage integrator will use (0 = divide)."""
    el = stage if isinstance(stage, Element) else element(stage)
    k = C.c_int32()
    _call("hbl_stage_newton_steps", C.byref(el), C.byref(ref), C.byref(k))
    return k.value


def moments(z, n=None, stream=None):
    ptr, n, ld = _bunch_args(z, n)
    m = (C.c_double * 6)()
    c = (C.c_double * 21)()
    _call("hbl_moments", ptr, n, ld, m, c, stream or current_stream())
    return list(m), list(c)


def _out27_arg(out27):
    torch = _torch()
    _on_current_device(out27, "moments output")
    if out27.dtype != torch.float64 or not out27.is_contiguous() or out27.numel() < 27:
        raise TypeError("moments output must be a contiguous float64 device tensor of >= 27 elements")
    return C.c_void_p(out27.data_ptr())


def moments_async(z, out27, n=None, stream=None):
    ptr, n, ld = _bunch_args(z, n)
    _call("hbl_moments_async", ptr, n, ld, _out27_arg(out27), stream or current_stream())


def moments_async_noalloc(z, out27, n=None, stream=None):
    """hbl_moments_async through the library's fixed scratch (no allocation)."""
    ptr, n, ld = _bunch_args(z, n)
    _call("hbl_moments_async_noalloc", ptr, n, ld, _out27_arg(out27), stream or current_stream())


def emittances(cov21):
    c = (C.c_double * 21)(*cov21)
    e = (C.c_double * 3)()
    _call("hbl_emittances", c, e)
    return list(e)


def compare(zs, zf, n=None, stream=None):
    ps, n, ld = _bunch_args(zs, n)
    pf, _, ldf = _bunch_args(zf, n)
    if ldf != ld:
        raise ValueError("compare: both bunches need the same leading dimension")
    r, c, e = (C.c_double * 6)(), (C.c_double * 6)(), (C.c_double * 3)()
    _call("hbl_compare", ps, pf, n, ld, r, c, e, stream or current_stream())
    return list(r), list(c), list(e)


class Surrogate:
    """Neural-network stage surrogate (tanh MLP 6-64-64-64-6) owned by libhbl."""

    def __init__(self, seed: int = 0, _handle=None):
        if _handle is None:
            h = C.c_void_p()
            _call("hbl_surrogate_create", C.byref(MlpShape(6, 64, 3, 6)), seed, C.byref(h))
            _handle = h
        self._h = _handle
        n = C.c_int64()
        _call("hbl_surrogate_num_params", self._h, C.byref(n))
        self.n_params = n.value

    @staticmethod
    def load(path: str) -> "Surrogate":
        h = C.c_void_p()
        _call("hbl_surrogate_load", path.encode(), C.byref(h))
        return Surrogate(_handle=h)

    def save(self, path: str):
        _call("hbl_surrogate_save", self._h, path.encode())

    def get_params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        _call("hbl_surrogate_get_params", self._h, out.ctypes.data_as(C.POINTER(C.c_float)), self.n_params)
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        _call("hbl_surrogate_set_params", self._h, p.ctypes.data_as(C.POINTER(C.c_float)), len(p))

    def get_norm(self):
        out = (C.c_double * 24)()
        _call("hbl_surrogate_get_norm", self._h, out)
        return list(out)

    def set_norm(self, norm):
        _call("hbl_surrogate_set_norm", self._h, (C.c_double * 24)(*norm))

    def set_stage(self, stage, ref_at_entry: Ref):
        el = stage if isinstance(stage, Element) else element(stage)
        _call("hbl_surrogate_set_stage", self._h, C.byref(el), C.byref(ref_at_entry))

    def train(self, zin, zout, n_pairs, batch=4096, epochs=1, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              train_frac=0.7, shuffle_seed=0, max_steps=-1, lr_final=None, keep_best=False, resume=False,
              stream=None):
        """keep_best: 0/False the last epoch's parameters; 1/True those of the
        lowest test loss; 2 those (among the last quarter of the epochs) whose
        test-split emittances in x and y are closest to the true ones.
        resume: continue an earlier training (normalisation, Adam state and
        epoch numbering kept)."""
        import numpy as np
        pin, _, ld = _bunch_args(zin, n_pairs, "input pairs")
        pout, _, ldo = _bunch_args(zout, n_pairs, "output pairs")
        if ldo != ld:
            raise ValueError("train: input and output pairs need the same leading dimension")
        cfg = TrainCfg(batch, epochs, max_steps, lr, lr if lr_final is None else lr_final, beta1, beta2, eps,
                       train_frac, shuffle_seed, int(keep_best), int(bool(resume)))
        log = np.zeros(2 * max(epochs, 1), dtype=np.float32)
        _call("hbl_surrogate_train", self._h, pin, pout, n_pairs, ld, C.byref(cfg),
              log.ctypes.data_as(C.POINTER(C.c_float)), stream or current_stream())
        return log[: 2 * epochs].reshape(epochs, 2)

    def loss_grad(self, zin, zout, idx, stream=None):
        import numpy as np
        pin, _, ld = _bunch_args(zin, what="input pairs")
        pout, _, ldo = _bunch_args(zout, what="output pairs")
        if ldo != ld:
            raise ValueError("loss_grad: input and output pairs need the same leading dimension")
        idx = _index_args(idx, min(zin.shape[1], zout.shape[1]), "loss_grad")
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_double()
        _call("hbl_surrogate_loss_grad", self._h, pin, pout, ld, idx.ctypes.data_as(C.POINTER(C.c_int32)),
              len(idx), g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss), stream or current_stream())
        return loss.value, g

    def apply(self, z, ref: Optional[Ref] = None, n=None, stream=None, pre=None, post=None):
        """Inference in place; with pre/post (Lattice) the gaps around the stage run in the same pass."""
        ptr, n, ld = _bunch_args(z, n)
        if pre is None and post is None:
            _call("hbl_surrogate_apply", ptr, n, ld, self._h, C.byref(ref) if ref is not None else None,
                  stream or current_stream())
        else:
            _call("hbl_surrogate_apply_gaps", ptr, n, ld, pre._h if pre else None, self._h,
                  post._h if post else None, C.byref(ref) if ref is not None else None,
                  stream or current_stream())

    def close(self):
        if getattr(self, "_h", None):
            lib.hbl_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreluNet:
    """The paper-shaped stage surrogate owned by libhbl: H hidden layers of
    width W with PReLU (one learned slope each), e.g. 3 x 700 or 5 x 900."""

    def __init__(self, width: int, hidden: int, seed: int = 0, _handle=None):
        if _handle is None:
            h = C.c_void_p()
            _call("hbl_prelu_create", C.byref(MlpShape(6, width, hidden, 6)), seed, C.byref(h))
            _handle = h
        self._h = _handle
        self.width, self.hidden = width, hidden
        n = C.c_int64()
        _call("hbl_prelu_num_params", self._h, C.byref(n))
        self.n_params = n.value

    @staticmethod
    def load(path: str) -> "PreluNet":
        import struct
        h = C.c_void_p()
        _call("hbl_prelu_load", path.encode(), C.byref(h))
        with open(path, "rb") as f:             # shape from the file header (after the 8-byte tag)
            _, width, hidden, _ = struct.unpack("<4i", f.read(24)[8:24])
        return PreluNet(width, hidden, _handle=h)

    def save(self, path: str):
        _call("hbl_prelu_save", self._h, path.encode())

    def flops_per_particle(self) -> int:
        """Multiply-adds x 2 of one forward pass (the network as defined, unpadded)."""
        W, H = self.width, self.hidden
        return 2 * (6 * W + (H - 1) * W * W + 6 * W)

    def get_params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        _call("hbl_prelu_get_params", self._h, out.ctypes.data_as(C.POINTER(C.c_float)), self.n_params)
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        _call("hbl_prelu_set_params", self._h, p.ctypes.data_as(C.POINTER(C.c_float)), len(p))

    def set_chunk(self, particles: int):
        _call("hbl_prelu_set_chunk", self._h, particles)

    def get_norm(self):
        out = (C.c_double * 24)()
        _call("hbl_prelu_get_norm", self._h, out)
        return list(out)

    def set_norm(self, norm):
        _call("hbl_prelu_set_norm", self._h, (C.c_double * 24)(*norm))

    def set_stage(self, stage, ref_at_entry: Ref):
        el = stage if isinstance(stage, Element) else element(stage)
        _call("hbl_prelu_set_stage", self._h, C.byref(el), C.byref(ref_at_entry))

    def loss_grad(self, zin, zout, idx, stream=None):
        import numpy as np
        pin, _, ld = _bunch_args(zin, what="input pairs")
        pout, _, ldo = _bunch_args(zout, what="output pairs")
        if ldo != ld:
            raise ValueError("loss_grad: input and output pairs need the same leading dimension")
        idx = _index_args(idx, min(zin.shape[1], zout.shape[1]), "loss_grad")
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_double()
        _call("hbl_prelu_loss_grad", self._h, pin, pout, ld, idx.ctypes.data_as(C.POINTER(C.c_int32)),
              len(idx), g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss), stream or current_stream())
        return loss.value, g

    def train(self, zin, zout, n_pairs, batch=1200, epochs=1, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8,
              train_frac=0.7, shuffle_seed=0, max_steps=-1, lr_final=None, stream=None):
        import numpy as np
        pin, _, ld = _bunch_args(zin, n_pairs, "input pairs")
        pout, _, ldo = _bunch_args(zout, n_pairs, "output pairs")
        if ldo != ld:
            raise ValueError("train: input and output pairs need the same leading dimension")
        cfg = TrainCfg(batch, epochs, max_steps, lr, lr if lr_final is None else lr_final, beta1, beta2, eps,
                       train_frac, shuffle_seed, 0, 0)
        log = np.zeros(2 * max(epochs, 1), dtype=np.float32)
        _call("hbl_prelu_train", self._h, pin, pout, n_pairs, ld, C.byref(cfg),
              log.ctypes.data_as(C.POINTER(C.c_float)), stream or current_stream())
        return log[: 2 * epochs].reshape(epochs, 2)

    def apply(self, z, ref: Optional[Ref] = None, n=None, stream=None, pre=None, post=None):
        """Inference in place; with pre/post (Lattice) the gaps run in the same launches."""
        ptr, n, ld = _bunch_args(z, n)
        if pre is None and post is None:
            _call("hbl_prelu_apply", ptr, n, ld, self._h, C.byref(ref) if ref is not None else None,
                  stream or current_stream())
        else:
            _call("hbl_prelu_apply_gaps", ptr, n, ld, pre._h if pre else None, self._h,
                  post._h if post else None, C.byref(ref) if ref is not None else None,
                  stream or current_stream())

    def close(self):
        if getattr(self, "_h", None):
            lib.hbl_prelu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
