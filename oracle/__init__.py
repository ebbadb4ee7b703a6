"""FP64 CPU oracle for layered belief-propagation decoding (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never touches the GPU library and the GPU library
never touches it.  The C source ``qcmet_oracle.c`` documents which passage of
the paper each routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qcmet_oracle.c")
_LIB = os.path.join(_HERE, "libqcmet_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics kept)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load(path: str):
    L = ctypes.CDLL(path)
    d, i32, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    L.qo_phi.restype = d; L.qo_phi.argtypes = [d]
    L.qo_clip.restype = d; L.qo_clip.argtypes = [d]
    L.qo_x_lo.restype = d; L.qo_x_hi.restype = d
    L.qo_round_half.restype = d; L.qo_round_half.argtypes = [d]
    L.qo_round_e4m3.restype = d; L.qo_round_e4m3.argtypes = [d]
    L.qo_greedy_schedule.restype = i32
    L.qo_greedy_schedule.argtypes = [i32, i32, p, p, p, p]
    L.qo_check_schedule.restype = i32
    L.qo_check_schedule.argtypes = [i32, i32, p, i32, p, p]
    L.qo_decode_sp.restype = i32
    L.qo_decode_sp.argtypes = [i32, i32, i32, p, i32, p, p, i32, p, p, i32, i32, p, p, p, i32]
    L.qo_decode_sp_early.restype = i32
    L.qo_decode_sp_early.argtypes = [i32, i32, i32, p, i32, p, p, i32, p, p, i32, i32, p, p, p, p, i32]
    L.qo_decode_flood.restype = i32
    L.qo_decode_flood.argtypes = [i32, i32, i32, p, i32, p, p, i32, i32, p, p, p, i32]
    L.qo_nms_decode.restype = i32
    L.qo_nms_decode.argtypes = [i32, i32, i32, p, i32, p, p, i32, p, p, i32, p, p, i32,
                                p, p, p, p, i32]
    L.qo_nms_train_grad.restype = i32
    L.qo_nms_train_grad.argtypes = [i32, i32, i32, p, i32, p, p, i32, p, p, p, i32, p, p, i32, i32,
                                    p, p, p, p, i32]
    L.qo_nms_loss_grad.restype = i32
    L.qo_nms_loss_grad.argtypes = [i32, i32, i32, p, i32, p, p, i32, p, p, p, i32, p, p,
                                   p, p, p, p, i32]
    return L


def build_variant(source: str, path: str) -> str:
    """Compile C source text (a planted-mistake copy of the oracle) to path."""
    src = path + ".c"
    with open(src, "w") as fh:
        fh.write(source)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                           "-ffp-contract=off", src, "-o", path, "-lm", "-lpthread"])
    return path


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def use_library(path: str | None):
    """Swap in another build of the oracle (the mutation tests plant mistakes
    in copies of the source); None restores the default build."""
    global _lib
    _lib = None if path is None else _load(path)


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _load(_LIB)
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def phi(x: float) -> float:
    return lib().qo_phi(float(x))


def clip(x: float) -> float:
    return lib().qo_clip(float(x))


def x_lo() -> float:
    return lib().qo_x_lo()


def x_hi() -> float:
    return lib().qo_x_hi()


def round_half(v: float) -> float:
    return lib().qo_round_half(float(v))


def round_e4m3(v: float) -> float:
    return lib().qo_round_e4m3(float(v))


def greedy_schedule(shifts: np.ndarray):
    """Greedy layer merge: (group_ptr int32 [G+1], rows int32 [mb])."""
    sh = np.ascontiguousarray(shifts, dtype=np.int32)
    mb, nb = sh.shape
    gptr = np.zeros(mb + 1, dtype=np.int32)
    rows = np.zeros(mb, dtype=np.int32)
    G = ctypes.c_int(0)
    rc = lib().qo_greedy_schedule(mb, nb, _ptr(sh), ctypes.byref(G), _ptr(gptr), _ptr(rows))
    if rc != 0:
        raise RuntimeError(f"qo_greedy_schedule failed: {rc}")
    return gptr[:G.value + 1].copy(), rows


def check_schedule(shifts, group_ptr, rows) -> int:
    sh = np.ascontiguousarray(shifts, dtype=np.int32)
    gp = np.ascontiguousarray(group_ptr, dtype=np.int32)
    rw = np.ascontiguousarray(rows, dtype=np.int32)
    return lib().qo_check_schedule(sh.shape[0], sh.shape[1], _ptr(sh), len(gp) - 1, _ptr(gp), _ptr(rw))


def serial_schedule(mb: int, order=None):
    rows = np.arange(mb, dtype=np.int32) if order is None else np.asarray(order, dtype=np.int32)
    return np.arange(mb + 1, dtype=np.int32), rows


def _prep(shifts, Z, llr, syn, schedule):
    sh = np.ascontiguousarray(shifts, dtype=np.int32)
    mb, nb = sh.shape
    n, m = nb * Z, mb * Z
    L = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float32)
    S = np.ascontiguousarray(np.atleast_2d(syn), dtype=np.uint8)
    if L.shape[1] != n or S.shape[1] != m or L.shape[0] != S.shape[0]:
        raise ValueError("shape mismatch")
    if schedule is None:
        schedule = greedy_schedule(sh)
    gp = np.ascontiguousarray(schedule[0], dtype=np.int32)
    rw = np.ascontiguousarray(schedule[1], dtype=np.int32)
    return sh, mb, nb, n, m, L, S, gp, rw


def _msg_mode(fp16_messages, fp8_messages):
    if fp16_messages and fp8_messages:
        raise ValueError("fp16_messages and fp8_messages exclude each other")
    return 1 if fp16_messages else 2 if fp8_messages else 0


def decode_sp(shifts, Z, llr, syn, T, schedule=None, fp16_messages=False, threads=0, fp8_messages=False):
    """Layered sum-product in FP64.  Returns (app f64 [F,n], hard u8 [F,n],
    flags u8 [F], threads_used)."""
    sh, mb, nb, n, m, L, S, gp, rw = _prep(shifts, Z, llr, syn, schedule)
    F = L.shape[0]
    app = np.empty((F, n), dtype=np.float64)
    hard = np.empty((F, n), dtype=np.uint8)
    flags = np.empty(F, dtype=np.uint8)
    rc = lib().qo_decode_sp(mb, nb, Z, _ptr(sh), len(gp) - 1, _ptr(gp), _ptr(rw), F, _ptr(L), _ptr(S),
                            int(T), _msg_mode(fp16_messages, fp8_messages), _ptr(app), _ptr(hard), _ptr(flags),
                            int(threads))
    if rc <= 0:
        raise RuntimeError(f"qo_decode_sp failed: {rc}")
    return app, hard, flags, rc


def decode_sp_early(shifts, Z, llr, syn, T, schedule=None, fp16_messages=False, threads=0, fp8_messages=False):
    """Layered sum-product with early termination: each frame stops at the
    first sweep count in [0, T] whose hard decisions satisfy the syndrome.
    Returns (app, hard, flags, iters_used)."""
    sh, mb, nb, n, m, L, S, gp, rw = _prep(shifts, Z, llr, syn, schedule)
    F = L.shape[0]
    app = np.empty((F, n), dtype=np.float64)
    hard = np.empty((F, n), dtype=np.uint8)
    flags = np.empty(F, dtype=np.uint8)
    iters = np.empty(F, dtype=np.int32)
    rc = lib().qo_decode_sp_early(mb, nb, Z, _ptr(sh), len(gp) - 1, _ptr(gp), _ptr(rw), F, _ptr(L), _ptr(S),
                                  int(T), _msg_mode(fp16_messages, fp8_messages), _ptr(app), _ptr(hard), _ptr(flags),
                                  _ptr(iters), int(threads))
    if rc <= 0:
        raise RuntimeError(f"qo_decode_sp_early failed: {rc}")
    return app, hard, flags, iters


def decode_flood(shifts, Z, llr, syn, T, fp16_messages=False, threads=0, fp8_messages=False):
    """Flooding-schedule sum-product in FP64.  Returns (app, hard, flags,
    threads_used)."""
    sh, mb, nb, n, m, L, S, gp, rw = _prep(shifts, Z, llr, syn, None)
    F = L.shape[0]
    app = np.empty((F, n), dtype=np.float64)
    hard = np.empty((F, n), dtype=np.uint8)
    flags = np.empty(F, dtype=np.uint8)
    rc = lib().qo_decode_flood(mb, nb, Z, _ptr(sh), F, _ptr(L), _ptr(S), int(T),
                               _msg_mode(fp16_messages, fp8_messages), _ptr(app), _ptr(hard), _ptr(flags),
                               int(threads))
    if rc <= 0:
        raise RuntimeError(f"qo_decode_flood failed: {rc}")
    return app, hard, flags, rc


def nms_decode(shifts, Z, llr, syn, T, alpha, beta, early_stop=False, schedule=None, threads=0):
    """Normalised/offset min-sum.  alpha, beta: [T, mb, 2].  Returns
    (app, hard, flags, iters_used)."""
    sh, mb, nb, n, m, L, S, gp, rw = _prep(shifts, Z, llr, syn, schedule)
    F = L.shape[0]
    a = np.ascontiguousarray(np.broadcast_to(alpha, (T, mb, 2)), dtype=np.float64)
    b = np.ascontiguousarray(np.broadcast_to(beta, (T, mb, 2)), dtype=np.float64)
    app = np.empty((F, n), dtype=np.float64)
    hard = np.empty((F, n), dtype=np.uint8)
    flags = np.empty(F, dtype=np.uint8)
    iters = np.empty(F, dtype=np.int32)
    rc = lib().qo_nms_decode(mb, nb, Z, _ptr(sh), len(gp) - 1, _ptr(gp), _ptr(rw), F, _ptr(L), _ptr(S),
                             int(T), _ptr(a), _ptr(b), 1 if early_stop else 0, _ptr(app), _ptr(hard),
                             _ptr(flags), _ptr(iters), int(threads))
    if rc <= 0:
        raise RuntimeError(f"qo_nms_decode failed: {rc}")
    return app, hard, flags, iters


def nms_loss_grad(shifts, Z, llr, syn, x, T, alpha, beta, schedule=None, threads=0):
    """Mean BCE of the final APP after T NMS iterations and its gradients
    w.r.t. alpha and beta.  Returns (loss, g_alpha [T,mb,2], g_beta, app)."""
    sh, mb, nb, n, m, L, S, gp, rw = _prep(shifts, Z, llr, syn, schedule)
    F = L.shape[0]
    X = np.ascontiguousarray(np.atleast_2d(x), dtype=np.uint8)
    a = np.ascontiguousarray(np.broadcast_to(alpha, (T, mb, 2)), dtype=np.float64)
    b = np.ascontiguousarray(np.broadcast_to(beta, (T, mb, 2)), dtype=np.float64)
    app = np.empty((F, n), dtype=np.float64)
    loss = ctypes.c_double(0.0)
    ga = np.zeros((T, mb, 2), dtype=np.float64)
    gb = np.zeros((T, mb, 2), dtype=np.float64)
    rc = lib().qo_nms_loss_grad(mb, nb, Z, _ptr(sh), len(gp) - 1, _ptr(gp), _ptr(rw), F, _ptr(L), _ptr(S),
                                _ptr(X), int(T), _ptr(a), _ptr(b), _ptr(app), ctypes.byref(loss),
                                _ptr(ga), _ptr(gb), int(threads))
    if rc <= 0:
        raise RuntimeError(f"qo_nms_loss_grad failed: {rc}")
    return loss.value, ga, gb, app


def nms_train_grad(shifts, Z, llr, syn, x, T, alpha, beta, every_sweep, window, schedule=None, threads=0):
    """Min-sum training objective and its gradient: every_sweep False gives
    the mean BCE of the APPs after the last sweep, True the mean over the T
    sweeps of the mean BCE after each sweep; the gradient of each loss term
    runs back through at most `window` sweeps (its own and the ones before),
    holding the state before them fixed.  Returns (loss, g_alpha [T,mb,2],
    g_beta, app)."""
    sh, mb, nb, n, m, L, S, gp, rw = _prep(shifts, Z, llr, syn, schedule)
    F = L.shape[0]
    X = np.ascontiguousarray(np.atleast_2d(x), dtype=np.uint8)
    a = np.ascontiguousarray(np.broadcast_to(alpha, (T, mb, 2)), dtype=np.float64)
    b = np.ascontiguousarray(np.broadcast_to(beta, (T, mb, 2)), dtype=np.float64)
    app = np.empty((F, n), dtype=np.float64)
    loss = ctypes.c_double(0.0)
    ga = np.zeros((T, mb, 2), dtype=np.float64)
    gb = np.zeros((T, mb, 2), dtype=np.float64)
    rc = lib().qo_nms_train_grad(mb, nb, Z, _ptr(sh), len(gp) - 1, _ptr(gp), _ptr(rw), F, _ptr(L), _ptr(S),
                                 _ptr(X), int(T), _ptr(a), _ptr(b), 1 if every_sweep else 0, int(window),
                                 _ptr(app), ctypes.byref(loss), _ptr(ga), _ptr(gb), int(threads))
    if rc <= 0:
        raise RuntimeError(f"qo_nms_train_grad failed: {rc}")
    return loss.value, ga, gb, app
