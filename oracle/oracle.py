"""ctypes marshalling for the FP64 C oracle (test infrastructure only).

Every function converts numpy arrays to the layout the C code expects and
returns numpy arrays; no arithmetic of the method lives here.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

NCH = 13
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "efunc_oracle.c")
# EFUNC_ORACLE_LIB selects another build (the sanitised one of build_oracle)
_LIB_PATH = os.environ.get("EFUNC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None
# AddressSanitizer + UndefinedBehaviorSanitizer, every UB report fatal
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]


def build_oracle(force: bool = True, sanitize: bool = False, out: str = None) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics: no fast-math);
    sanitize=True builds an ASan/UBSan copy (load it with the gcc sanitizer
    runtimes preloaded) at out."""
    out = out or _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        opt = SANITIZE_FLAGS if sanitize else ["-O2"]
        subprocess.check_call(
            ["gcc", *opt, "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, out)
    return out


class _Grid(C.Structure):
    _fields_ = [("R", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("offsets", C.c_int32), ("raw_beta", C.c_int32)]


@dataclass
class Grid:
    R: int
    lo: float = -1.0
    hi: float = 1.0
    offsets: int = 1
    raw_beta: int = 0

    def c(self) -> _Grid:
        return _Grid(self.R, self.lo, self.hi, self.offsets, self.raw_beta)

    @property
    def I(self) -> int:  # noqa: E743 - the paper's symbol
        return self.R ** 3


_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_G = C.POINTER(_Grid)
_I64 = C.c_int64


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_oracle(force=True)
        lib = C.CDLL(_LIB_PATH)
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = C.c_int
        lib.oracle_num_keys.argtypes = [_G]
        lib.oracle_num_keys.restype = _I64
        lib.oracle_lattice.argtypes = [_G, _I64]
        lib.oracle_lattice.restype = C.c_double
        lib.oracle_build_keys.argtypes = [_G, _F, _D]
        lib.oracle_eval.argtypes = [_D, _I64, _D, _I64, _D, _D, _D]
        lib.oracle_eval_qgrad.argtypes = [_D, _I64, _D, _I64, _D]
        lib.oracle_eval_qgrad_scales.argtypes = [_D, _I64, _D, _I64, C.c_double, _D, _D, _D, _D]
        lib.oracle_eval_cond.argtypes = [_D, _I64, _D, _I64, _D, C.c_double, _D]
        lib.oracle_grad.argtypes = [_D, _I64, _D, _I64, _D, _D, _D, C.c_double, _D]
        lib.oracle_grad_theta.argtypes = [_G, _F, _D, _D]
        lib.oracle_eval_trunc.argtypes = [_G, _D, _D, _I64, C.c_double, _D, _D, _D]
        lib.oracle_eval_trunc.restype = C.c_int
        lib.oracle_grad_trunc.argtypes = [_G, _D, _D, _I64, C.c_double, _D, _D, _D,
                                          C.c_double, C.c_double, _D]
        lib.oracle_grad_trunc.restype = C.c_int
        lib.oracle_adam.argtypes = [_D, _D, _D, _D, _I64, _I64, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_double]
        lib.oracle_meanshift.argtypes = [_G, _D, _I64, C.c_double, _D]
        lib.oracle_fit_step.argtypes = [_G, _F, _D, _D, _I64, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_double, _D, _D, _I64,
                                        C.c_int, C.c_double, _D, _D, _D, _D, _D, _D]
        lib.oracle_fit_step.restype = C.c_int
        _lib = lib
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Temporarily route every call through another build of the oracle
    (used by the mutation test, which compiles deliberately broken copies)."""
    global _lib
    load()
    saved = _lib
    _lib = None
    real = _LIB_PATH
    try:
        globals()["_LIB_PATH"] = path
        load()
        yield
    finally:
        globals()["_LIB_PATH"] = real
        _lib = saved


def _d(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f(a):
    return a.ctypes.data_as(_F)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def threads() -> int:
    return int(load().oracle_threads())


def num_keys(g: Grid) -> int:
    gc = g.c()
    return int(load().oracle_num_keys(C.byref(gc)))


def lattice(g: Grid) -> np.ndarray:
    gc = g.c()
    lib = load()
    return np.array([lib.oracle_lattice(C.byref(gc), n) for n in range(g.R)])


def build_keys(g: Grid, theta) -> np.ndarray:
    theta = _f32(theta).reshape(-1)
    assert theta.size == g.I * NCH
    keys = np.empty((num_keys(g), 8), np.float64)
    gc = g.c()
    load().oracle_build_keys(C.byref(gc), _f(theta), _d(keys))
    return keys


def eval_global(keys, q):
    """Return (O, lse, sigma) over all keys (the definition)."""
    keys, q = _f64(keys), _f64(q).reshape(-1, 3)
    J = q.shape[0]
    O, lse, sig = (np.empty(J) for _ in range(3))
    load().oracle_eval(_d(keys), keys.shape[0], _d(q), J, _d(O), _d(lse), _d(sig))
    return O, lse, sig


def eval_cond(keys, q, T: float = float("inf"), with_tail: bool = False):
    """Tolerance scales: kappa_j = sum_a w_a |s_a| |f_a - O_j|, and with
    with_tail also tail_j = sum over keys with weight below e^-T of
    w_a |f_a - O_j|."""
    keys, q = _f64(keys), _f64(q).reshape(-1, 3)
    kap = np.empty(q.shape[0])
    tail = np.empty(q.shape[0]) if with_tail else None
    load().oracle_eval_cond(_d(keys), keys.shape[0], _d(q), q.shape[0], _d(kap), T, _d(tail))
    return (kap, tail) if with_tail else kap


def eval_qgrad(keys, q):
    keys, q = _f64(keys), _f64(q).reshape(-1, 3)
    out = np.empty_like(q)
    load().oracle_eval_qgrad(_d(keys), keys.shape[0], _d(q), q.shape[0], _d(out))
    return out


def eval_qgrad_scales(keys, q, T: float = float("inf")):
    """Tolerance scales of dO/dq (J x 3 each): (qsig, qkap, qtail, qbx), see
    oracle_eval_qgrad_scales."""
    keys, q = _f64(keys), _f64(q).reshape(-1, 3)
    qs, qk, qt, qb = (np.empty_like(q) for _ in range(4))
    load().oracle_eval_qgrad_scales(_d(keys), keys.shape[0], _d(q), q.shape[0], T, _d(qs),
                                    _d(qk), _d(qt), _d(qb))
    return qs, qk, qt, qb


def eval_trunc(g: Grid, keys, q, T: float = 20.0):
    keys, q = _f64(keys), _f64(q).reshape(-1, 3)
    J = q.shape[0]
    O, lse, sig = (np.empty(J) for _ in range(3))
    gc = g.c()
    rc = load().oracle_eval_trunc(C.byref(gc), _d(keys), _d(q), J, T, _d(O), _d(lse), _d(sig))
    if rc != 0:
        raise MemoryError("oracle_eval_trunc failed")
    return O, lse, sig


def grad_global(keys, q, dLdO, T: float = None):
    """Return (gk, ak): key gradients and their running-error scales (nkeys x 8);
    with T also bk, the part of ak from pairs with weight below e^-T."""
    keys, q, dLdO = _f64(keys), _f64(q).reshape(-1, 3), _f64(dLdO)
    gk = np.empty((keys.shape[0], 8))
    ak = np.empty((keys.shape[0], 8))
    bk = np.empty((keys.shape[0], 8)) if T is not None else None
    load().oracle_grad(_d(keys), keys.shape[0], _d(q), q.shape[0], _d(dLdO), _d(gk), _d(ak),
                       float("inf") if T is None else T, _d(bk))
    return (gk, ak) if T is None else (gk, ak, bk)


def grad_trunc(g: Grid, keys, q, dLdO, T: float = 20.0, Tb: float = None, T2: float = None):
    """(gk, ak) of the truncated gradient; with Tb also bk, the part of the
    scale from pairs below e^-Tb among those with logit >= M_j - T2 (T2
    defaults to T + 10)."""
    keys, q, dLdO = _f64(keys), _f64(q).reshape(-1, 3), _f64(dLdO)
    gk = np.empty((keys.shape[0], 8))
    ak = np.empty((keys.shape[0], 8))
    bk = np.empty((keys.shape[0], 8)) if Tb is not None else None
    T2 = T + 10.0 if T2 is None else T2
    gc = g.c()
    rc = load().oracle_grad_trunc(C.byref(gc), _d(keys), _d(q), q.shape[0], T, _d(dLdO),
                                  _d(gk), _d(ak), 0.0 if Tb is None else Tb, T2, _d(bk))
    if rc != 0:
        raise MemoryError("oracle_grad_trunc failed")
    return (gk, ak) if Tb is None else (gk, ak, bk)


def grad_theta(g: Grid, theta, gk) -> np.ndarray:
    """Key gradients (or their scales) mapped onto the [R,R,R,13] channels."""
    theta = _f32(theta).reshape(-1)
    gk = _f64(gk)
    out = np.empty(g.I * NCH)
    gc = g.c()
    load().oracle_grad_theta(C.byref(gc), _f(theta), _d(gk), _d(out))
    return out.reshape(g.R, g.R, g.R, NCH)


def adam(theta, m, v, grad, step, lr=6e-4, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    theta, m, v = _f64(theta).copy(), _f64(m).copy(), _f64(v).copy()
    grad = _f64(grad)
    load().oracle_adam(_d(theta), _d(m), _d(v), _d(grad), theta.size, step, lr, beta1,
                       beta2, eps, wd)
    return theta, m, v


def meanshift(g: Grid, surf, bandwidth: float = 100.0) -> np.ndarray:
    surf = _f64(surf).reshape(-1, 3)
    out = np.empty((g.I, 3))
    gc = g.c()
    load().oracle_meanshift(C.byref(gc), _d(surf), surf.shape[0], bandwidth, _d(out))
    return out


def fit_step(g: Grid, theta, m, v, step, q, o, lr=6e-4, beta1=0.9, beta2=0.999, eps=1e-8,
             wd=0.0, mode: int = 0, T: float = 20.0):
    """One oracle fitting iteration.  Returns dict(theta, m, v, grad, O, loss, l1)."""
    theta = _f32(theta).reshape(-1)
    m, v = _f64(m).reshape(-1), _f64(v).reshape(-1)
    q, o = _f64(q).reshape(-1, 3), _f64(o).reshape(-1)
    n = g.I * NCH
    th, mo, vo, gr = (np.empty(n) for _ in range(4))
    O = np.empty(q.shape[0])
    loss = np.empty(2)
    gc = g.c()
    rc = load().oracle_fit_step(C.byref(gc), _f(theta), _d(m), _d(v), step, lr, beta1, beta2,
                                eps, wd, _d(q), _d(o), q.shape[0], mode, T, _d(th), _d(mo),
                                _d(vo), _d(gr), _d(O), _d(loss))
    if rc != 0:
        raise MemoryError("oracle_fit_step failed")
    shp = (g.R, g.R, g.R, NCH)
    return dict(theta=th.reshape(shp), m=mo.reshape(shp), v=vo.reshape(shp),
                grad=gr.reshape(shp), O=O, loss=float(loss[0]), l1=float(loss[1]))
