"""ctypes marshalling for the FP64 variant oracle (efunc_oracle_var.c):
polynomial degree 0/1/2, grid and/or moved key sets, learnable or fixed
scales.  Test infrastructure only; no arithmetic of the method lives here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "efunc_oracle_var.c")
# EFUNC_ORACLE_VAR_LIB selects another build (the sanitised one of build_var_oracle)
_LIB_PATH = os.environ.get("EFUNC_ORACLE_VAR_LIB") or os.path.join(_HERE, "liboracle_var.so")
_lib = None
KEYW = 16
GRADW = 14


def build_var_oracle(force: bool = True, src: str = None, out: str = None, sanitize: bool = False) -> str:
    """Compile the variant oracle with gcc (-O2, OpenMP, IEEE semantics);
    sanitize=True builds an ASan/UBSan copy."""
    from .oracle import SANITIZE_FLAGS
    src = src or _SRC
    out = out or _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        opt = SANITIZE_FLAGS if sanitize else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-I", _HERE, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class _Model(C.Structure):
    _fields_ = [("R", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("degree", C.c_int32), ("grid_keys", C.c_int32), ("moved_keys", C.c_int32),
                ("learn_scale", C.c_int32), ("rho_fixed", C.c_double)]


@dataclass
class Model:
    R: int
    degree: int = 1
    grid_keys: int = 1
    moved_keys: int = 1
    learn_scale: int = 1
    rho_fixed: float = 7.0
    lo: float = -1.0
    hi: float = 1.0

    def c(self) -> _Model:
        return _Model(self.R, self.lo, self.hi, self.degree, self.grid_keys, self.moved_keys,
                      self.learn_scale, self.rho_fixed)

    @property
    def I(self) -> int:  # noqa: E743 - the paper's symbol
        return self.R ** 3


_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_M = C.POINTER(_Model)
_I64 = C.c_int64


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_var_oracle(force=True)
        lib = C.CDLL(_LIB_PATH)
        lib.ovar_num_values.argtypes = [C.c_int]
        lib.ovar_num_values.restype = C.c_int
        lib.ovar_layout.argtypes = [_M, C.POINTER(C.c_int32)]
        lib.ovar_layout.restype = C.c_int
        lib.ovar_num_keys.argtypes = [_M]
        lib.ovar_num_keys.restype = _I64
        lib.ovar_build_keys.argtypes = [_M, _F, _D]
        lib.ovar_eval.argtypes = [_D, _I64, C.c_int, _D, _I64, _D, _D, _D]
        lib.ovar_eval_cond.argtypes = [_D, _I64, C.c_int, _D, _I64, _D, C.c_double, _D]
        lib.ovar_eval_qgrad.argtypes = [_D, _I64, C.c_int, _D, _I64, _D]
        lib.ovar_eval_qgrad_scales.argtypes = [_D, _I64, C.c_int, _D, _I64, C.c_double, _D, _D,
                                               _D, _D]
        lib.ovar_grad.argtypes = [_D, _I64, C.c_int, _D, _I64, _D, _D, _D, C.c_double, _D]
        lib.ovar_grad_theta.argtypes = [_M, _F, _D, _D]
        lib.ovar_fit_step.argtypes = [_M, _F, _D, _D, _I64, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _D, _D, _I64, _D, _D, _D, _D, _D, _D]
        lib.ovar_fit_step.restype = C.c_int
        _lib = lib
    return _lib


def use_library(path: str):
    """Route later calls through another build (mutation tests); returns the
    previous handle so that the caller can restore it with restore()."""
    global _lib
    prev = _lib
    lib_path = globals()["_LIB_PATH"]
    globals()["_LIB_PATH"] = path
    _lib = None
    load()
    globals()["_LIB_PATH"] = lib_path
    return prev


def restore(prev):
    global _lib
    _lib = prev


def _d(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_values(degree: int) -> int:
    return int(load().ovar_num_values(degree))


def layout(m: Model) -> dict:
    out = (C.c_int32 * 6)()
    mc = m.c()
    load().ovar_layout(C.byref(mc), out)
    names = ["grid_values", "grid_rho", "moved_delta", "moved_values", "moved_rho", "nch"]
    return dict(zip(names, list(out)))


def channels(m: Model) -> int:
    return layout(m)["nch"]


def build_keys(m: Model, theta) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float32)
    assert th.size == m.I * channels(m)
    mc = m.c()
    n = int(load().ovar_num_keys(C.byref(mc)))
    keys = np.empty((n, KEYW), np.float64)
    load().ovar_build_keys(C.byref(mc), th.ctypes.data_as(_F), _d(keys))
    return keys


def eval_global(keys, degree, q):
    keys, q = _f64(keys), _f64(q)
    J = len(q)
    O, lse, sig = np.empty(J), np.empty(J), np.empty(J)
    load().ovar_eval(_d(keys), len(keys), degree, _d(q), J, _d(O), _d(lse), _d(sig))
    return O, lse, sig


def eval_cond(keys, degree, q, T: float = float("inf"), with_tail: bool = False):
    keys, q = _f64(keys), _f64(q)
    J = len(q)
    kap, tail = np.empty(J), np.empty(J)
    load().ovar_eval_cond(_d(keys), len(keys), degree, _d(q), J, _d(kap), T, _d(tail))
    return (kap, tail) if with_tail else kap


def eval_qgrad(keys, degree, q):
    keys, q = _f64(keys), _f64(q)
    out = np.empty((len(q), 3))
    load().ovar_eval_qgrad(_d(keys), len(keys), degree, _d(q), len(q), _d(out))
    return out


def eval_qgrad_scales(keys, degree, q, T: float = float("inf")):
    """Tolerance scales of dO/dq (J x 3 each): (qsig, qkap, qtail, qbx)."""
    keys, q = _f64(keys), _f64(q)
    qs, qk, qt, qb = (np.empty((len(q), 3)) for _ in range(4))
    load().ovar_eval_qgrad_scales(_d(keys), len(keys), degree, _d(q), len(q), T, _d(qs), _d(qk),
                                  _d(qt), _d(qb))
    return qs, qk, qt, qb


def grad_global(keys, degree, q, dLdO, T: float = None):
    keys, q, dl = _f64(keys), _f64(q), _f64(dLdO)
    n = len(keys)
    gk, ak = np.empty((n, GRADW)), np.empty((n, GRADW))
    bk = np.empty((n, GRADW)) if T is not None else None
    load().ovar_grad(_d(keys), n, degree, _d(q), len(q), _d(dl), _d(gk), _d(ak),
                     float("inf") if T is None else T, _d(bk))
    return (gk, ak) if T is None else (gk, ak, bk)


def grad_theta(m: Model, theta, gk) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float32)
    gk = _f64(gk)
    out = np.empty(m.I * channels(m))
    mc = m.c()
    load().ovar_grad_theta(C.byref(mc), th.ctypes.data_as(_F), _d(gk), _d(out))
    return out


def fit_step(m: Model, theta, mom1, mom2, step, q, o, lr=6e-4, beta1=0.9, beta2=0.999,
             eps=1e-8, wd=0.0):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    n = th.size
    q, o = _f64(q), _f64(o)
    m1, m2 = _f64(mom1).reshape(-1), _f64(mom2).reshape(-1)
    to, mo, vo, go, Oo = np.empty(n), np.empty(n), np.empty(n), np.empty(n), np.empty(len(q))
    loss = np.empty(2)
    mc = m.c()
    rc = load().ovar_fit_step(C.byref(mc), th.ctypes.data_as(_F), _d(m1), _d(m2), step, lr, beta1,
                              beta2, eps, wd, _d(q), _d(o), len(q), _d(to), _d(mo), _d(vo), _d(go),
                              _d(Oo), _d(loss))
    assert rc == 0
    return {"theta": to, "m": mo, "v": vo, "grad": go, "O": Oo, "loss": loss[0], "l1": loss[1]}
