"""Python binding of libqcmet (argument marshalling only).

Every function named ``qm_*`` mirrors the C entry point of the same name in
include/qcmet.h.  Device buffers are torch CUDA tensors (PyTorch supplies
device memory and streams, nothing else); every step of a decode runs in the
library's HIP kernels.  There is no fallback: if ``libqcmet.so`` is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcmet.so")

QM_OK = 0
QM_ERR_INVALID_ARG = -1
QM_ERR_SHAPE = -2
QM_ERR_SCHEDULE_CONFLICT = -3
QM_ERR_NO_WORKSPACE = -4
QM_ERR_OOM = -5
QM_ERR_HIP = -6
QM_ERR_INPUT = -7
QM_ERR_UNSUPPORTED = -8
QM_ERR_STATE = -9

QM_MSG_FP32 = 0x0
QM_MSG_FP16 = 0x1
QM_MSG_FP8 = 0x2
QM_VALIDATE = 0x4
QM_GRAPH = 0x8
QM_EARLY_STOP = 0x10
QM_FLOODING = 0x20

# every symbol include/qcmet.h declares
EXPORTED = [
    "qm_abi_version", "qm_last_error", "qm_code_create", "qm_code_destroy", "qm_code_get_info",
    "qm_code_set_schedule", "qm_code_get_schedule", "qm_decoder_create", "qm_decoder_destroy",
    "qm_decoder_workspace_bytes", "qm_decoder_bind_workspace", "qm_decoder_set_tuning",
    "qm_decoder_get_tuning", "qm_decode", "qm_decode_early", "qm_autotune", "qm_decoder_set_profiling",
    "qm_decoder_get_profile", "qm_nms_workspace_bytes", "qm_nms_bind_workspace", "qm_nms_decode",
    "qm_nms_loss_grad", "qm_adam_step", "qm_generate_frames", "qm_decode_noalloc", "qm_nms_train_grad",
]

QM_NOALLOC_SCRATCH_BYTES = 64 << 20


class QMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class qm_code_info(ctypes.Structure):
    _fields_ = [("mb", ctypes.c_int32), ("nb", ctypes.c_int32), ("Z", ctypes.c_int32),
                ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("n_type1_cols", ctypes.c_int32), ("n_deg1_cols", ctypes.c_int32),
                ("n_type1_entries", ctypes.c_int32), ("max_row_type1", ctypes.c_int32),
                ("edges", ctypes.c_int64), ("G", ctypes.c_int32)]


class qm_tuning(ctypes.Structure):
    _fields_ = [("frames_per_tile", ctypes.c_int32), ("block", ctypes.c_int32),
                ("merge", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("frames_per_lane", ctypes.c_int32), ("fuse_codes", ctypes.c_int32),
                ("stream_hint", ctypes.c_int32), ("lds_resident", ctypes.c_int32),
                ("tile_groups", ctypes.c_int32), ("spread_codes", ctypes.c_int32),
                ("frames_per_batch", ctypes.c_int32), ("resident_cap", ctypes.c_int32)]


class qm_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("layer_ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("layer_bytes", ctypes.c_double), ("checks", ctypes.c_double),
                ("lds_launches", ctypes.c_int32), ("lds_ms", ctypes.c_double), ("lds_bytes", ctypes.c_double),
                ("et_narrowings", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libqcmet (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(python -m paper_2004_09084_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        i32, p, sz = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
        L.qm_abi_version.restype = ctypes.c_int
        L.qm_last_error.restype = ctypes.c_char_p
        L.qm_code_create.argtypes = [i32, i32, i32, p, ctypes.POINTER(p)]
        L.qm_code_destroy.argtypes = [p]
        L.qm_code_get_info.argtypes = [p, ctypes.POINTER(qm_code_info)]
        L.qm_code_set_schedule.argtypes = [p, i32, p, p]
        L.qm_code_get_schedule.argtypes = [p, ctypes.POINTER(i32), p, p]
        L.qm_decoder_create.argtypes = [p, i32, p, i32, ctypes.POINTER(p)]
        L.qm_decoder_destroy.argtypes = [p]
        L.qm_decoder_workspace_bytes.argtypes = [p]
        L.qm_decoder_workspace_bytes.restype = sz
        L.qm_decoder_bind_workspace.argtypes = [p, p, sz]
        L.qm_decoder_set_tuning.argtypes = [p, ctypes.POINTER(qm_tuning)]
        L.qm_decoder_get_tuning.argtypes = [p, ctypes.POINTER(qm_tuning)]
        L.qm_decode.argtypes = [p, p, p, i32, p, p, p, p]
        L.qm_decode_early.argtypes = [p, p, p, i32, p, p, p, p, p]
        L.qm_decode_noalloc.argtypes = [p, p, p, i32, p, p, p, p]
        L.qm_autotune.argtypes = [p, p, p, i32, p, p, p, ctypes.c_char_p, p]
        L.qm_decoder_set_profiling.argtypes = [p, i32]
        L.qm_decoder_get_profile.argtypes = [p, ctypes.POINTER(qm_profile), i32]
        L.qm_nms_workspace_bytes.argtypes = [p, i32, i32]
        L.qm_nms_workspace_bytes.restype = sz
        L.qm_nms_bind_workspace.argtypes = [p, p, sz, i32, i32]
        L.qm_nms_decode.argtypes = [p, p, p, p, i32, i32, p, p, p, p, p]
        L.qm_nms_loss_grad.argtypes = [p, p, p, p, p, i32, p, p, p]
        L.qm_nms_train_grad.argtypes = [p, p, p, p, p, i32, i32, i32, p, p, p, p]
        f32 = ctypes.c_float
        L.qm_adam_step.argtypes = [p, p, p, p, i32, f32, f32, f32, f32, i32, p]
        u64 = ctypes.c_uint64
        L.qm_generate_frames.argtypes = [p, i32, u64, u64, f32, i32, p, p, p, p]
        for name in EXPORTED:
            f = getattr(L, name)
            if name not in ("qm_last_error", "qm_decoder_workspace_bytes", "qm_abi_version",
                            "qm_nms_workspace_bytes"):
                f.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != QM_OK:
        raise QMError(rc, lib().qm_last_error().decode())
    return rc


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t) -> int | None:
    """Device address of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device buffer expected (torch CUDA tensor)")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _stream_handle(stream) -> int | None:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# ----------------------------------------------------------- thin wrappers --

def qm_abi_version() -> int:
    return lib().qm_abi_version()


def qm_code_create(shifts: np.ndarray, Z: int) -> ctypes.c_void_p:
    sh = np.ascontiguousarray(shifts, dtype=np.int32)
    mb, nb = sh.shape
    out = ctypes.c_void_p()
    _check(lib().qm_code_create(mb, nb, int(Z), _np_ptr(sh), ctypes.byref(out)))
    return out


def qm_code_destroy(code) -> None:
    _check(lib().qm_code_destroy(code))


def qm_code_get_info(code) -> qm_code_info:
    info = qm_code_info()
    _check(lib().qm_code_get_info(code, ctypes.byref(info)))
    return info


def qm_code_set_schedule(code, group_ptr, rows) -> None:
    gp = np.ascontiguousarray(group_ptr, dtype=np.int32)
    rw = np.ascontiguousarray(rows, dtype=np.int32)
    _check(lib().qm_code_set_schedule(code, len(gp) - 1, _np_ptr(gp), _np_ptr(rw)))


def qm_code_get_schedule(code):
    info = qm_code_get_info(code)
    G = ctypes.c_int32(0)
    gp = np.zeros(info.mb + 1, dtype=np.int32)
    rw = np.zeros(info.mb, dtype=np.int32)
    _check(lib().qm_code_get_schedule(code, ctypes.byref(G), _np_ptr(gp), _np_ptr(rw)))
    return gp[:G.value + 1].copy(), rw


def qm_decoder_create(codes, frames_per_code, flags: int = 0) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(codes))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in codes])
    fpc = np.ascontiguousarray(frames_per_code, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(lib().qm_decoder_create(arr, len(codes), _np_ptr(fpc), int(flags), ctypes.byref(out)))
    return out


def qm_decoder_destroy(dec) -> None:
    _check(lib().qm_decoder_destroy(dec))


def qm_decoder_workspace_bytes(dec) -> int:
    return int(lib().qm_decoder_workspace_bytes(dec))


def qm_decoder_bind_workspace(dec, ws) -> None:
    _check(lib().qm_decoder_bind_workspace(dec, _dptr(ws), ws.numel() * ws.element_size()))


def qm_decoder_set_tuning(dec, frames_per_tile=0, block=0, merge=1, graph=0, frames_per_lane=0, fuse_codes=2,
                          stream_hint=1, lds_resident=2, tile_groups=1, spread_codes=1,
                          frames_per_batch=0, resident_cap=10) -> None:
    t = qm_tuning(frames_per_tile, block, merge, graph, frames_per_lane, fuse_codes, stream_hint, lds_resident,
                  tile_groups, spread_codes, frames_per_batch, resident_cap)
    _check(lib().qm_decoder_set_tuning(dec, ctypes.byref(t)))


def qm_decoder_get_tuning(dec) -> dict:
    t = qm_tuning()
    _check(lib().qm_decoder_get_tuning(dec, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in qm_tuning._fields_}


def qm_decode(dec, llr, syndrome, iters: int, hard, app, flags, stream=None) -> None:
    _check(lib().qm_decode(dec, _dptr(llr), _dptr(syndrome), int(iters), _dptr(hard), _dptr(app),
                           _dptr(flags), _stream_handle(stream)))


def qm_decode_noalloc(dec, llr, syndrome, iters: int, hard, app, flags, stream=None) -> None:
    _check(lib().qm_decode_noalloc(dec, _dptr(llr), _dptr(syndrome), int(iters), _dptr(hard), _dptr(app),
                                   _dptr(flags), _stream_handle(stream)))


def qm_decode_early(dec, llr, syndrome, max_iters: int, hard, app, flags, iters_used=None, stream=None) -> None:
    _check(lib().qm_decode_early(dec, _dptr(llr), _dptr(syndrome), int(max_iters), _dptr(hard), _dptr(app),
                                 _dptr(flags), _dptr(iters_used), _stream_handle(stream)))


def qm_autotune(dec, llr, syndrome, iters: int, hard, app, flags, cache_path: str | None = None,
                stream=None) -> None:
    _check(lib().qm_autotune(dec, _dptr(llr), _dptr(syndrome), int(iters), _dptr(hard), _dptr(app),
                             _dptr(flags), cache_path.encode() if cache_path else None, _stream_handle(stream)))


def qm_decoder_set_profiling(dec, enable: bool) -> None:
    _check(lib().qm_decoder_set_profiling(dec, 1 if enable else 0))


def qm_decoder_get_profile(dec, reset: bool = True) -> dict:
    p = qm_profile()
    _check(lib().qm_decoder_get_profile(dec, ctypes.byref(p), 1 if reset else 0))
    return {f: getattr(p, f) for f, _ in qm_profile._fields_}


def qm_nms_workspace_bytes(dec, T: int, train: bool) -> int:
    return int(lib().qm_nms_workspace_bytes(dec, int(T), 1 if train else 0))


def qm_nms_bind_workspace(dec, ws, T: int, train: bool) -> None:
    _check(lib().qm_nms_bind_workspace(dec, _dptr(ws), ws.numel() * ws.element_size(), int(T), 1 if train else 0))


def qm_nms_decode(dec, weights, llr, syndrome, T: int, early_stop: bool, hard, app, flags, iters_used,
                  stream=None) -> None:
    _check(lib().qm_nms_decode(dec, _dptr(weights), _dptr(llr), _dptr(syndrome), int(T), 1 if early_stop else 0,
                               _dptr(hard), _dptr(app), _dptr(flags), _dptr(iters_used), _stream_handle(stream)))


def qm_nms_loss_grad(dec, weights, llr, syndrome, x, T: int, loss, grad, stream=None) -> None:
    _check(lib().qm_nms_loss_grad(dec, _dptr(weights), _dptr(llr), _dptr(syndrome), _dptr(x), int(T), _dptr(loss),
                                  _dptr(grad), _stream_handle(stream)))


def qm_nms_train_grad(dec, weights, llr, syndrome, x, T: int, every_sweep: bool, window: int, loss, grad,
                      clamped=None, stream=None) -> None:
    _check(lib().qm_nms_train_grad(dec, _dptr(weights), _dptr(llr), _dptr(syndrome), _dptr(x), int(T),
                                   1 if every_sweep else 0, int(window), _dptr(loss), _dptr(grad), _dptr(clamped),
                                   _stream_handle(stream)))


def qm_generate_frames(dec, code_index: int, seed: int, first_frame: int, snr: float, F: int, x, llr, syndrome,
                       stream=None) -> None:
    _check(lib().qm_generate_frames(dec, int(code_index), int(seed), int(first_frame), float(snr), int(F), _dptr(x),
                                    _dptr(llr), _dptr(syndrome), _stream_handle(stream)))


def qm_adam_step(w, g, m, v, lr: float, b1: float, b2: float, eps: float, step: int, stream=None) -> None:
    _check(lib().qm_adam_step(_dptr(w), _dptr(g), _dptr(m), _dptr(v), w.numel(), float(lr), float(b1), float(b2),
                              float(eps), int(step), _stream_handle(stream)))


# ------------------------------------------------------ convenience layer --

class Code:
    """A QC base matrix loaded into the library."""

    def __init__(self, shifts: np.ndarray, Z: int):
        self.shifts = np.ascontiguousarray(shifts, dtype=np.int32)
        self.Z = int(Z)
        self.handle = qm_code_create(self.shifts, self.Z)
        self.info = qm_code_get_info(self.handle)

    @property
    def n(self) -> int:
        return int(self.info.n)

    @property
    def m(self) -> int:
        return int(self.info.m)

    def schedule(self):
        return qm_code_get_schedule(self.handle)

    def set_schedule(self, group_ptr, rows):
        qm_code_set_schedule(self.handle, group_ptr, rows)
        self.info = qm_code_get_info(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.qm_code_destroy(h)
            self.handle = None


class Decoder:
    """Decoder for frames_per_code[c] frames of codes[c] with a torch-owned
    device workspace."""

    def __init__(self, codes, frames_per_code, flags: int = 0, device="cuda", tuning: dict | None = None):
        import torch
        self.codes = list(codes)          # keep the codes alive
        self.frames = [int(f) for f in frames_per_code]
        self.flags = int(flags)
        self.device = torch.device(device)
        self.handle = qm_decoder_create([c.handle for c in self.codes], self.frames, self.flags)
        self.workspace = None
        if tuning:
            qm_decoder_set_tuning(self.handle, **tuning)
        self._bind()

    def _bind(self):
        import torch
        nbytes = qm_decoder_workspace_bytes(self.handle)
        if self.workspace is None or self.workspace.numel() < nbytes:
            self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        qm_decoder_bind_workspace(self.handle, self.workspace)

    def set_tuning(self, **kw):
        cur = qm_decoder_get_tuning(self.handle)
        cur.update(kw)
        qm_decoder_set_tuning(self.handle, **cur)
        self._bind()

    def tuning(self) -> dict:
        return qm_decoder_get_tuning(self.handle)

    @property
    def n_total(self) -> int:
        return sum(f * c.n for f, c in zip(self.frames, self.codes))

    @property
    def m_total(self) -> int:
        return sum(f * c.m for f, c in zip(self.frames, self.codes))

    @property
    def F_total(self) -> int:
        return sum(self.frames)

    def alloc_outputs(self, want_app: bool = True):
        import torch
        hard = torch.empty(self.n_total, dtype=torch.uint8, device=self.device)
        app = torch.empty(self.n_total, dtype=torch.float32, device=self.device) if want_app else None
        flags = torch.empty(self.F_total, dtype=torch.uint8, device=self.device)
        return hard, app, flags

    def decode(self, llr, syndrome, iters: int, out=None, want_app: bool = True, stream=None):
        """llr: float32 [sum F_c n_c], syndrome: uint8 [sum F_c m_c] (device).
        Returns (hard, app, flags) device tensors."""
        if llr.numel() != self.n_total or syndrome.numel() != self.m_total:
            raise ValueError("llr/syndrome size does not match the decoder's frames")
        hard, app, flags = out if out is not None else self.alloc_outputs(want_app)
        qm_decode(self.handle, llr.reshape(-1), syndrome.reshape(-1), iters, hard, app, flags, stream)
        return hard, app, flags

    def decode_early(self, llr, syndrome, max_iters: int, out=None, want_app: bool = True, stream=None):
        """Early-terminating decode (decoder created with QM_EARLY_STOP).
        Returns (hard, app, flags, iters_used) device tensors."""
        import torch
        if llr.numel() != self.n_total or syndrome.numel() != self.m_total:
            raise ValueError("llr/syndrome size does not match the decoder's frames")
        hard, app, flags = out if out is not None else self.alloc_outputs(want_app)
        iters = torch.empty(self.F_total, dtype=torch.int32, device=self.device)
        qm_decode_early(self.handle, llr.reshape(-1), syndrome.reshape(-1), max_iters, hard, app, flags, iters, stream)
        return hard, app, flags, iters

    def set_profiling(self, enable: bool):
        qm_decoder_set_profiling(self.handle, enable)

    def profile(self, reset: bool = True) -> dict:
        return qm_decoder_get_profile(self.handle, reset)

    def autotune(self, llr, syndrome, iters: int, cache_path: str | None = None, stream=None, out=None):
        hard, app, flags = out if out is not None else self.alloc_outputs(True)
        qm_autotune(self.handle, llr.reshape(-1), syndrome.reshape(-1), iters, hard, app, flags, cache_path, stream)
        return self.tuning()

    # ---- learned decoder (normalized/offset min-sum) ----
    def nms_bind(self, T: int, train: bool = False):
        import torch
        nbytes = qm_nms_workspace_bytes(self.handle, T, train)
        if nbytes == 0:
            raise QMError(QM_ERR_UNSUPPORTED, "min-sum needs exactly one code with float32 messages")
        self.nms_workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        qm_nms_bind_workspace(self.handle, self.nms_workspace, T, train)

    def nms_decode(self, weights, llr, syndrome, T: int, early_stop: bool = False, out=None, stream=None):
        import torch
        hard, app, flags = out if out is not None else self.alloc_outputs(True)
        iters = torch.empty(self.F_total, dtype=torch.int32, device=self.device)
        qm_nms_decode(self.handle, weights.reshape(-1), llr.reshape(-1), syndrome.reshape(-1), T, early_stop,
                      hard, app, flags, iters, stream)
        return hard, app, flags, iters

    def nms_loss_grad(self, weights, llr, syndrome, x, T: int, stream=None):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty_like(weights)
        qm_nms_loss_grad(self.handle, weights.reshape(-1), llr.reshape(-1), syndrome.reshape(-1), x.reshape(-1), T,
                         loss, grad, stream)
        return loss, grad

    def nms_train_grad(self, weights, llr, syndrome, x, T: int, every_sweep: bool = True, window: int = 1,
                       stream=None):
        """Returns (loss, grad, clamped) device tensors (qm_nms_train_grad)."""
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty_like(weights)
        clamped = torch.empty(1, dtype=torch.int32, device=self.device)
        qm_nms_train_grad(self.handle, weights.reshape(-1), llr.reshape(-1), syndrome.reshape(-1), x.reshape(-1), T,
                          every_sweep, window, loss, grad, clamped, stream)
        return loss, grad, clamped

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.qm_decoder_destroy(h)
            self.handle = None
