"""Python binding of the efunc C ABI (include/efunc.h).

Argument marshalling only: every function below checks tensor placement,
dtype and contiguity, passes raw device pointers and the current HIP stream
to the function of the same name in libefunc.so, and turns a negative return
code into EfuncError.  All computation runs in the library's HIP kernels;
if the library is missing, importing the binding succeeds but every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# EFUNC_LIBRARY selects another build of the same library (e.g. the host-
# sanitised one); by default the in-tree libefunc.so next to this file.
LIB_PATH = os.environ.get("EFUNC_LIBRARY") or os.path.join(HERE, "libefunc.so")
NCH = 13

EFUNC_OK = 0
EFUNC_EINVAL = -1
EFUNC_EHIP = -2
EFUNC_ESIZE = -3
EFUNC_ENONFINITE = -4
EFUNC_EUNSUPPORTED = -5


class EfuncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"efunc error {code}: {msg}")
        self.code = code


class efunc_config(C.Structure):
    _fields_ = [("R", C.c_int32), ("lo", C.c_float), ("hi", C.c_float), ("offsets", C.c_int32),
                ("t_cut", C.c_float), ("window", C.c_int32), ("deterministic", C.c_int32),
                ("check_finite", C.c_int32), ("degree", C.c_int32), ("grid_keys", C.c_int32),
                ("learn_scale", C.c_int32), ("rho_fixed", C.c_float)]


class efunc_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float)]


class efunc_tuning(C.Structure):
    _fields_ = [("tile_cap", C.c_int32), ("group_cells", C.c_int32), ("blocks_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class efunc_stats(C.Structure):
    _fields_ = [("W", C.c_int32), ("n_tiles", C.c_int32), ("n_uncertified", C.c_int64),
                ("pairs", C.c_int64), ("pairs_moved", C.c_int64), ("bwd_pairs", C.c_int64),
                ("bwd_pairs_moved", C.c_int64), ("beta_min", C.c_float),
                ("beta_grid_max", C.c_float), ("n_nonfinite", C.c_int32),
                ("workspace_bytes", C.c_int64), ("window_keys", C.c_int64), ("kept_keys", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol declared in include/efunc.h
EXPORTS = ["efunc_default_config", "efunc_channels", "efunc_default_adam", "efunc_create", "efunc_destroy",
           "efunc_init_params", "efunc_eval", "efunc_grad", "efunc_fit_step", "efunc_get_stats",
           "efunc_set_timing", "efunc_read_timing", "efunc_default_tuning", "efunc_set_tuning",
           "efunc_get_tuning", "efunc_batch_create", "efunc_batch_destroy", "efunc_batch_bind",
           "efunc_batch_fit", "efunc_batch_set_tuning", "efunc_batch_get_tuning",
           "efunc_batch_autotune", "efunc_batch_get_stats", "efunc_batch_set_timing",
           "efunc_batch_read_timing", "efunc_initnet_create", "efunc_initnet_destroy",
           "efunc_initnet_num_params", "efunc_initnet_forward", "efunc_initnet_backward",
           "efunc_conv3d_bf16", "efunc_conv3d_wgrad_bf16", "efunc_conv3d_pack_weights",
           "efunc_adam_update", "efunc_loss_grad", "efunc_fit_step_static", "efunc_initnet_theta",
           "efunc_initnet_theta_backward", "efunc_last_error"]

_lib = None


def lib() -> C.CDLL:
    """Load libefunc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise EfuncError(EFUNC_EUNSUPPORTED,
                             f"{LIB_PATH} is missing: build it with paper_2505_21319_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.efunc_default_config.argtypes = [C.POINTER(efunc_config), C.c_int32]
        L.efunc_default_config.restype = None
        L.efunc_channels.argtypes = [C.POINTER(efunc_config)]
        L.efunc_channels.restype = C.c_int
        L.efunc_default_adam.argtypes = [C.POINTER(efunc_adam)]
        L.efunc_default_adam.restype = None
        L.efunc_create.argtypes = [C.POINTER(efunc_config), i64, C.POINTER(vp)]
        L.efunc_destroy.argtypes = [vp]
        L.efunc_init_params.argtypes = [vp, vp, vp, i64, C.c_float, C.c_float, vp]
        L.efunc_eval.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp]
        L.efunc_grad.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp]
        L.efunc_fit_step.argtypes = [vp, vp, vp, vp, i64, C.POINTER(efunc_adam), vp, vp, i64, vp, vp]
        L.efunc_get_stats.argtypes = [vp, C.POINTER(efunc_stats)]
        L.efunc_set_timing.argtypes = [vp, C.c_int32]
        L.efunc_read_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.efunc_default_tuning.argtypes = [C.POINTER(efunc_tuning)]
        L.efunc_default_tuning.restype = None
        L.efunc_set_tuning.argtypes = [vp, C.POINTER(efunc_tuning)]
        L.efunc_get_tuning.argtypes = [vp, C.POINTER(efunc_tuning)]
        pp = C.POINTER(vp)
        L.efunc_batch_create.argtypes = [C.POINTER(efunc_config), C.POINTER(i64), C.c_int32, pp]
        L.efunc_batch_destroy.argtypes = [vp]
        L.efunc_batch_bind.argtypes = [vp, pp, pp, pp, pp, pp, C.POINTER(i64), vp]
        L.efunc_batch_fit.argtypes = [vp, C.POINTER(efunc_adam), i64, i64, C.c_int32, vp]
        L.efunc_batch_set_tuning.argtypes = [vp, C.POINTER(efunc_tuning)]
        L.efunc_batch_get_tuning.argtypes = [vp, C.POINTER(efunc_tuning)]
        L.efunc_batch_autotune.argtypes = [vp, C.POINTER(efunc_adam), C.c_int32,
                                           C.POINTER(efunc_tuning), C.POINTER(C.c_double), vp]
        L.efunc_batch_get_stats.argtypes = [vp, C.c_int32, C.POINTER(efunc_stats)]
        L.efunc_batch_set_timing.argtypes = [vp, C.c_int32]
        L.efunc_batch_read_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        i32 = C.c_int32
        L.efunc_initnet_create.argtypes = [i32, i32, i32, C.POINTER(i32), pp]
        L.efunc_initnet_destroy.argtypes = [vp]
        L.efunc_initnet_num_params.argtypes = [vp]
        L.efunc_initnet_num_params.restype = i64
        L.efunc_initnet_forward.argtypes = [vp, vp, vp, i32, vp, vp]
        L.efunc_initnet_backward.argtypes = [vp, vp, i32, vp, vp]
        L.efunc_conv3d_bf16.argtypes = [vp, i32, vp, i32, i32, vp, i32, vp, i32, i64, vp, vp, vp, vp]
        L.efunc_conv3d_wgrad_bf16.argtypes = [vp, i32, vp, i32, i32, i64, vp, vp, vp]
        L.efunc_conv3d_pack_weights.argtypes = [vp, i32, i32, vp, vp, vp]
        L.efunc_adam_update.argtypes = [vp, vp, vp, vp, i64, i64, C.POINTER(efunc_adam), vp]
        L.efunc_loss_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
        L.efunc_fit_step_static.argtypes = [C.POINTER(efunc_config), vp, vp, vp, i64,
                                             C.POINTER(efunc_adam), vp, vp, i64, vp, vp]
        L.efunc_initnet_theta.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_float, C.c_float, vp, vp, vp, vp]
        L.efunc_initnet_theta_backward.argtypes = [vp, C.c_int32, C.c_int32, vp, vp]
        L.efunc_last_error.argtypes = []
        L.efunc_last_error.restype = C.c_char_p
        for name in ("efunc_create", "efunc_destroy", "efunc_init_params", "efunc_eval",
                     "efunc_grad", "efunc_fit_step", "efunc_get_stats", "efunc_set_timing",
                     "efunc_read_timing", "efunc_set_tuning", "efunc_get_tuning",
                     "efunc_batch_create", "efunc_batch_destroy", "efunc_batch_bind",
                     "efunc_batch_fit", "efunc_batch_set_tuning", "efunc_batch_get_tuning",
                     "efunc_batch_autotune", "efunc_batch_get_stats", "efunc_batch_set_timing",
                     "efunc_batch_read_timing", "efunc_initnet_create", "efunc_initnet_destroy",
                     "efunc_initnet_forward", "efunc_initnet_backward", "efunc_conv3d_bf16",
                     "efunc_conv3d_wgrad_bf16", "efunc_conv3d_pack_weights", "efunc_adam_update",
                     "efunc_loss_grad", "efunc_fit_step_static", "efunc_initnet_theta",
                     "efunc_initnet_theta_backward"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != EFUNC_OK:
        raise EfuncError(rc, lib().efunc_last_error().decode())


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, name: str, numel: Optional[int] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def efunc_default_config(R: int) -> efunc_config:
    c = efunc_config()
    lib().efunc_default_config(C.byref(c), R)
    return c


def efunc_channels(cfg: efunc_config) -> int:
    n = lib().efunc_channels(C.byref(cfg))
    if n < 0:
        _check(n)
    return n


def efunc_default_adam() -> efunc_adam:
    a = efunc_adam()
    lib().efunc_default_adam(C.byref(a))
    return a


def efunc_create(cfg: efunc_config, max_points: int) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().efunc_create(C.byref(cfg), max_points, C.byref(out)))
    return out


def efunc_destroy(ctx) -> None:
    _check(lib().efunc_destroy(ctx))


def efunc_init_params(ctx, theta, surf, R: int, bandwidth=100.0, rho0=7.0, stream=None, nch=NCH):
    ns = 0 if surf is None else surf.numel() // 3
    _check(lib().efunc_init_params(ctx, _ptr(theta, torch.float32, "theta", R ** 3 * nch),
                                   _ptr(surf, torch.float32, "surf"), ns, bandwidth, rho0,
                                   _stream(stream)))


def efunc_eval(ctx, theta, q, O, lse=None, dOdq=None, n_uncertified=None, stream=None, n_theta=None):
    """n_theta: the context's parameter count R^3 x channels; theta must hold
    exactly that many floats (the C ABI cannot check a pointer's extent)."""
    J = q.numel() // 3
    _check(lib().efunc_eval(ctx, _ptr(theta, torch.float32, "theta", n_theta),
                            _ptr(q, torch.float32, "q", 3 * J), J,
                            _ptr(O, torch.float32, "O", J), _ptr(lse, torch.float32, "lse", J),
                            _ptr(dOdq, torch.float32, "dOdq", 3 * J),
                            _ptr(n_uncertified, torch.int64, "n_uncertified", 1),
                            _stream(stream)))


def efunc_grad(ctx, theta, q, O, lse, dLdO, grad, stream=None, n_theta=None):
    J = q.numel() // 3
    _check(lib().efunc_grad(ctx, _ptr(theta, torch.float32, "theta", n_theta),
                            _ptr(q, torch.float32, "q", 3 * J), _ptr(O, torch.float32, "O", J),
                            _ptr(lse, torch.float32, "lse", J),
                            _ptr(dLdO, torch.float32, "dLdO", J), J,
                            _ptr(grad, torch.float32, "grad", theta.numel()), _stream(stream)))


def efunc_fit_step(ctx, theta, m, v, step: int, q, o, loss_out=None, adam: Optional[efunc_adam] = None,
                   stream=None, n_theta=None):
    J = q.numel() // 3
    n = theta.numel()
    _check(lib().efunc_fit_step(ctx, _ptr(theta, torch.float32, "theta", n_theta),
                                _ptr(m, torch.float32, "m", n), _ptr(v, torch.float32, "v", n),
                                step, C.byref(adam) if adam is not None else None,
                                _ptr(q, torch.float32, "q", 3 * J), _ptr(o, torch.float32, "o", J),
                                J, _ptr(loss_out, torch.float64, "loss_out", 2), _stream(stream)))


def efunc_fit_step_static(cfg: efunc_config, theta, m, v, step: int, q, o, loss_out=None,
                          adam: Optional[efunc_adam] = None, stream=None):
    """efunc_fit_step without a context: the workspace lives in the library's
    fixed per-GPU scratch array (no device allocation)."""
    J = q.numel() // 3
    n = cfg.R ** 3 * efunc_channels(cfg)
    _check(lib().efunc_fit_step_static(C.byref(cfg), _ptr(theta, torch.float32, "theta", n),
                                       _ptr(m, torch.float32, "m", n), _ptr(v, torch.float32, "v", n),
                                       step, C.byref(adam) if adam is not None else None,
                                       _ptr(q, torch.float32, "q", 3 * J), _ptr(o, torch.float32, "o", J),
                                       J, _ptr(loss_out, torch.float64, "loss_out", 2), _stream(stream)))


def efunc_initnet_theta(sdf, R: int, res=None, rho0: float = 7.0, rho_min: float = float("-inf"),
                        theta=True, mask=False, grad=False, stream=None):
    """Starting parameters from coarse fields sdf [B, R^3] (or [R^3]): returns
    (theta [B, R^3, 13] or None, mask [B, R^3, 2] uint8 or None, grad
    [B, R^3, 3] or None) as requested; res [B, R^3, 13] is added before the
    log-scale floor rho_min."""
    B = sdf.numel() // R ** 3
    n = B * R ** 3
    dev = sdf.device
    th = torch.empty(B, R ** 3, 13, device=dev) if theta else None
    mk = torch.empty(B, R ** 3, 2, device=dev, dtype=torch.uint8) if mask else None
    gr = torch.empty(B, R ** 3, 3, device=dev) if grad else None
    _check(lib().efunc_initnet_theta(_ptr(sdf, torch.float32, "sdf", n), R, B,
                                     _ptr(res, torch.float32, "res", 13 * n), rho0, rho_min,
                                     _ptr(th, torch.float32, "theta", 13 * n),
                                     _ptr(mk, torch.uint8, "mask", 2 * n),
                                     _ptr(gr, torch.float32, "grad", 3 * n), _stream(stream)))
    return th, mk, gr


def efunc_initnet_theta_backward(mask, R: int, dtheta, stream=None) -> None:
    """Zero dtheta's log-scale channels where mask records a floored value."""
    B = mask.numel() // (2 * R ** 3)
    _check(lib().efunc_initnet_theta_backward(_ptr(mask, torch.uint8, "mask", 2 * B * R ** 3), R, B,
                                              _ptr(dtheta, torch.float32, "dtheta", 13 * B * R ** 3),
                                              _stream(stream)))


def efunc_loss_grad(ctx, theta, q, o, grad, loss_out=None, stream=None, n_theta=None):
    J = q.numel() // 3
    _check(lib().efunc_loss_grad(ctx, _ptr(theta, torch.float32, "theta", n_theta),
                                 _ptr(q, torch.float32, "q", 3 * J),
                                 _ptr(o, torch.float32, "o", J), J,
                                 _ptr(grad, torch.float32, "grad", theta.numel()),
                                 _ptr(loss_out, torch.float64, "loss_out", 2), _stream(stream)))


def efunc_get_stats(ctx) -> dict:
    s = efunc_stats()
    _check(lib().efunc_get_stats(ctx, C.byref(s)))
    return s.as_dict()


def efunc_set_timing(ctx, enable: bool) -> None:
    _check(lib().efunc_set_timing(ctx, 1 if enable else 0))


def efunc_read_timing(ctx):
    """(summed tile-kernel milliseconds, launches) since timing was enabled/read."""
    ms, n = C.c_double(), C.c_int64()
    _check(lib().efunc_read_timing(ctx, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def efunc_default_tuning() -> efunc_tuning:
    t = efunc_tuning()
    lib().efunc_default_tuning(C.byref(t))
    return t


def efunc_set_tuning(ctx, t: efunc_tuning) -> None:
    _check(lib().efunc_set_tuning(ctx, C.byref(t)))


def efunc_get_tuning(ctx) -> efunc_tuning:
    t = efunc_tuning()
    _check(lib().efunc_get_tuning(ctx, C.byref(t)))
    return t


def _ptr_array(ts, dtype, name, numels=None):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t, dtype, f"{name}[{i}]", None if numels is None else numels[i])
    return arr


def efunc_batch_create(cfgs, max_points) -> C.c_void_p:
    n = len(cfgs)
    carr = (efunc_config * n)(*cfgs)
    marr = (C.c_int64 * n)(*[int(x) for x in max_points])
    out = C.c_void_p()
    _check(lib().efunc_batch_create(carr, marr, n, C.byref(out)))
    return out


def efunc_batch_destroy(b) -> None:
    _check(lib().efunc_batch_destroy(b))


def efunc_batch_bind(b, thetas, ms, vs, qs, os_, loss_out=None, n_thetas=None) -> None:
    """n_thetas: each shape's parameter count R^3 x channels (checked before
    the call; the C ABI cannot check a pointer's extent)."""
    n = len(thetas)
    if not (len(ms) == len(vs) == len(qs) == len(os_) == n):
        raise ValueError("one tensor per shape in every list")
    if n_thetas is not None and len(n_thetas) != n:
        raise ValueError("one parameter count per shape")
    nth = [t.numel() for t in thetas] if n_thetas is None else [int(x) for x in n_thetas]
    Js = [q.numel() // 3 for q in qs]
    Jarr = (C.c_int64 * n)(*Js)
    _check(lib().efunc_batch_bind(
        b, _ptr_array(thetas, torch.float32, "theta", nth), _ptr_array(ms, torch.float32, "m", nth),
        _ptr_array(vs, torch.float32, "v", nth), _ptr_array(qs, torch.float32, "q", [3 * J for J in Js]),
        _ptr_array(os_, torch.float32, "o", Js), Jarr,
        _ptr(loss_out, torch.float64, "loss_out", 2 * n)))


def efunc_batch_fit(b, first_step: int, n_steps: int, use_graph: bool = False,
                    adam: Optional[efunc_adam] = None, stream=None) -> None:
    _check(lib().efunc_batch_fit(b, C.byref(adam) if adam is not None else None, first_step, n_steps,
                                 1 if use_graph else 0, _stream(stream)))


def efunc_batch_set_tuning(b, t: efunc_tuning) -> None:
    _check(lib().efunc_batch_set_tuning(b, C.byref(t)))


def efunc_batch_get_tuning(b) -> efunc_tuning:
    t = efunc_tuning()
    _check(lib().efunc_batch_get_tuning(b, C.byref(t)))
    return t


def efunc_batch_autotune(b, reps: int = 3, adam: Optional[efunc_adam] = None, stream=None):
    """(chosen tuning as a dict, its median iteration milliseconds)."""
    t = efunc_tuning()
    ms = C.c_double()
    _check(lib().efunc_batch_autotune(b, C.byref(adam) if adam is not None else None, reps,
                                      C.byref(t), C.byref(ms), _stream(stream)))
    return t.as_dict(), ms.value


def efunc_batch_get_stats(b, shape: int) -> dict:
    s = efunc_stats()
    _check(lib().efunc_batch_get_stats(b, shape, C.byref(s)))
    return s.as_dict()


def efunc_batch_set_timing(b, enable: bool) -> None:
    _check(lib().efunc_batch_set_timing(b, 1 if enable else 0))


def efunc_batch_read_timing(b):
    ms, n = C.c_double(), C.c_int64()
    _check(lib().efunc_batch_read_timing(b, C.byref(ms), C.byref(n)))
    return ms.value, n.value


class BatchEngine:
    """Owns one efunc batch: S shapes fitted together (see efunc_batch_*)."""

    def __init__(self, Rs, max_points, **cfg):
        cfgs = []
        for R in Rs:
            c = efunc_default_config(int(R))
            for k, v in cfg.items():
                setattr(c, k, v)
            cfgs.append(c)
        self.Rs = [int(R) for R in Rs]
        self.n_thetas = [int(R) ** 3 * efunc_channels(c) for R, c in zip(self.Rs, cfgs)]
        self.b = efunc_batch_create(cfgs, max_points)
        self._bound = None

    def close(self):
        if self.b:
            efunc_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def bind(self, thetas, ms, vs, qs, os_, loss_out=None):
        efunc_batch_bind(self.b, thetas, ms, vs, qs, os_, loss_out, self.n_thetas)
        self._bound = (thetas, ms, vs, qs, os_, loss_out)  # keep the tensors alive

    def fit(self, first_step, n_steps, use_graph=False, adam=None):
        efunc_batch_fit(self.b, first_step, n_steps, use_graph, adam)

    def set_tuning(self, tile_cap=512, group_cells=2, blocks_per_cu=8):
        t = efunc_tuning(tile_cap, group_cells, blocks_per_cu)
        efunc_batch_set_tuning(self.b, t)

    def tuning(self):
        return efunc_batch_get_tuning(self.b).as_dict()

    def autotune(self, reps=3, adam=None):
        return efunc_batch_autotune(self.b, reps, adam)

    def stats(self, shape):
        return efunc_batch_get_stats(self.b, shape)


def kpad(k: int) -> int:
    return (k + 31) // 32 * 32


def efunc_conv3d_pack_weights(W, Cin: int, Cout: int, stream=None):
    """(wf [Cout][kpad(27 Cin)], wd [Cin][kpad(27 Cout)]) bf16 packings of fp32 W[co][tap][ci]."""
    wf = torch.empty(Cout, kpad(27 * Cin), device=W.device, dtype=torch.bfloat16)
    wd = torch.empty(Cin, kpad(27 * Cout), device=W.device, dtype=torch.bfloat16)
    _check(lib().efunc_conv3d_pack_weights(_ptr(W, torch.float32, "W", Cout * 27 * Cin), Cin, Cout,
                                           wf.data_ptr(), wd.data_ptr(), _stream(stream)))
    return wf, wd


def blocked_size(V: int, C: int) -> int:
    """Elements of a blocked channel-major copy ([ceil(V/32)][C][32])."""
    return (V + 31) // 32 * 32 * C


def efunc_conv3d_bf16(x, Cin: int, w, Cout: int, R: int, bias=None, relu=False, mask=None,
                      y_bf16=None, y_f32=None, yT_bf16=None, stream=None):
    """yT_bf16, if given, receives the blocked channel-major copy (blocked_size(V, Cout) bf16)."""
    V = x.numel() // Cin
    _check(lib().efunc_conv3d_bf16(_ptr(x, torch.bfloat16, "x", V * Cin), Cin,
                                   _ptr(w, torch.bfloat16, "w", Cout * w.shape[1]), w.shape[1], Cout,
                                   _ptr(bias, torch.float32, "bias", Cout), 1 if relu else 0,
                                   _ptr(mask, torch.bfloat16, "mask", V * Cout), R, V,
                                   _ptr(y_bf16, torch.bfloat16, "y_bf16", V * Cout),
                                   _ptr(y_f32, torch.float32, "y_f32", V * Cout),
                                   _ptr(yT_bf16, torch.bfloat16, "yT_bf16", blocked_size(V, Cout)), _stream(stream)))


def efunc_conv3d_wgrad_bf16(xT, Cin: int, dyT, Cout: int, R: int, V: int, dw, db=None, stream=None):
    """xT and dyT in the blocked channel-major layout (blocked_size(V, C) bf16 each)."""
    _check(lib().efunc_conv3d_wgrad_bf16(_ptr(xT, torch.bfloat16, "xT", blocked_size(V, Cin)), Cin,
                                         _ptr(dyT, torch.bfloat16, "dyT", blocked_size(V, Cout)), Cout, R, V,
                                         _ptr(dw, torch.float32, "dw", Cout * 27 * Cin),
                                         _ptr(db, torch.float32, "db", Cout), _stream(stream)))


def efunc_adam_update(p, m, v, g, step: int, adam: Optional[efunc_adam] = None, stream=None):
    n = p.numel()
    _check(lib().efunc_adam_update(_ptr(p, torch.float32, "p", n), _ptr(m, torch.float32, "m", n),
                                   _ptr(v, torch.float32, "v", n), _ptr(g, torch.float32, "g", n), n,
                                   step, C.byref(adam) if adam is not None else None, _stream(stream)))


class InitNet:
    """The learned-initialiser network (efunc_initnet_*): sdf [B][R^3] -> [B][R^3][C_L]."""

    def __init__(self, R: int, max_shapes: int, channels):
        self.R, self.channels = R, list(channels)
        arr = (C.c_int32 * len(channels))(*channels)
        out = C.c_void_p()
        _check(lib().efunc_initnet_create(R, max_shapes, len(channels) - 1, arr, C.byref(out)))
        self.net = out
        self.n_params = int(lib().efunc_initnet_num_params(out))

    def close(self):
        if self.net:
            _check(lib().efunc_initnet_destroy(self.net))
            self.net = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def forward(self, params, sdf, out=None):
        B = sdf.numel() // self.R ** 3
        if out is None:
            out = torch.empty(B, self.R ** 3, self.channels[-1], device=sdf.device, dtype=torch.float32)
        _check(lib().efunc_initnet_forward(self.net, _ptr(params, torch.float32, "params", self.n_params),
                                           _ptr(sdf, torch.float32, "sdf", B * self.R ** 3), B,
                                           _ptr(out, torch.float32, "out", B * self.R ** 3 * self.channels[-1]),
                                           _stream(None)))
        return out

    def backward(self, dout, dparams):
        B = dout.numel() // (self.R ** 3 * self.channels[-1])
        _check(lib().efunc_initnet_backward(self.net, _ptr(dout, torch.float32, "dout", dout.numel()), B,
                                            _ptr(dparams, torch.float32, "dparams", self.n_params),
                                            _stream(None)))


class Engine:
    """Owns one efunc context (convenience wrapper over the functions above)."""

    def __init__(self, R: int, max_points: int, **cfg):
        c = efunc_default_config(R)
        for k, v in cfg.items():
            setattr(c, k, v)
        self.R = R
        self.cfg = c
        self.nch = efunc_channels(c)
        self.n_theta = R ** 3 * self.nch
        self.max_points = max_points
        self.ctx = efunc_create(c, max_points)

    def close(self):
        if self.ctx:
            efunc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def eval(self, theta, q, with_lse=True, with_qgrad=False):
        J = q.shape[0]
        O = torch.empty(J, device=q.device, dtype=torch.float32)
        lse = torch.empty(J, device=q.device, dtype=torch.float32) if with_lse else None
        dq = torch.empty(J, 3, device=q.device, dtype=torch.float32) if with_qgrad else None
        nu = torch.zeros(1, device=q.device, dtype=torch.int64)
        efunc_eval(self.ctx, theta, q, O, lse, dq, nu, n_theta=self.n_theta)
        return O, lse, dq, nu

    def grad(self, theta, q, O, lse, dLdO, grad=None):
        if grad is None:
            grad = torch.zeros_like(theta)
        efunc_grad(self.ctx, theta, q, O, lse, dLdO, grad, n_theta=self.n_theta)
        return grad

    def fit_step(self, theta, m, v, step, q, o, loss_out=None, adam=None):
        efunc_fit_step(self.ctx, theta, m, v, step, q, o, loss_out, adam, n_theta=self.n_theta)

    def loss_grad(self, theta, q, o, grad, loss_out=None):
        efunc_loss_grad(self.ctx, theta, q, o, grad, loss_out, n_theta=self.n_theta)

    def init_params(self, theta, surf, bandwidth=100.0, rho0=7.0):
        efunc_init_params(self.ctx, theta, surf, self.R, bandwidth, rho0, nch=self.nch)

    def stats(self):
        return efunc_get_stats(self.ctx)

    def set_tuning(self, tile_cap=512, group_cells=2, blocks_per_cu=8):
        efunc_set_tuning(self.ctx, efunc_tuning(tile_cap, group_cells, blocks_per_cu))

    def tuning(self):
        return efunc_get_tuning(self.ctx).as_dict()
