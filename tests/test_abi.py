"""The C-ABI library loads and exports every entry point declared in
include/efunc.h; host-side argument validation runs without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "efunc.h")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(efunc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2505_21319_amd import efunc
    if not os.path.exists(efunc.LIB_PATH):
        from paper_2505_21319_amd import build
        build.build()
    return efunc.lib()


def test_header_declares_the_boundary():
    names = declared()
    for n in ["efunc_create", "efunc_destroy", "efunc_init_params", "efunc_eval", "efunc_grad",
              "efunc_fit_step", "efunc_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    from paper_2505_21319_amd import efunc
    assert sorted(efunc.EXPORTS) == declared()
    for n in declared():
        assert hasattr(L, n), n


def test_defaults(L):
    from paper_2505_21319_amd import efunc as E
    c = E.efunc_default_config(32)
    assert (c.R, c.lo, c.hi, c.offsets, c.t_cut, c.window) == (32, -1.0, 1.0, 1, 20.0, 0)
    a = E.efunc_default_adam()
    assert abs(a.lr - 6e-4) < 1e-9 and abs(a.beta2 - 0.999) < 1e-7 and a.weight_decay == 0.0


def test_invalid_arguments_are_rejected_before_any_device_work(L):
    from paper_2505_21319_amd import efunc as E
    out = C.c_void_p()
    assert L.efunc_create(None, 10, C.byref(out)) == E.EFUNC_EINVAL
    c = E.efunc_default_config(1)
    assert L.efunc_create(C.byref(c), 10, C.byref(out)) == E.EFUNC_EINVAL
    assert b"R = 1" in L.efunc_last_error()
    c = E.efunc_default_config(513)
    assert L.efunc_create(C.byref(c), 10, C.byref(out)) == E.EFUNC_EINVAL
    assert b"R = 513" in L.efunc_last_error()
    c = E.efunc_default_config(8)
    c.lo, c.hi = 1.0, -1.0
    assert L.efunc_create(C.byref(c), 10, C.byref(out)) == E.EFUNC_EINVAL
    c = E.efunc_default_config(8)
    assert L.efunc_create(C.byref(c), -5, C.byref(out)) == E.EFUNC_EINVAL
    c.deterministic = 2
    assert L.efunc_create(C.byref(c), 5, C.byref(out)) == E.EFUNC_EINVAL
    c.deterministic = 1
    batch = C.c_void_p()
    assert L.efunc_batch_create(C.byref(c), (C.c_int64 * 1)(5), 1, C.byref(batch)) == E.EFUNC_EUNSUPPORTED
    assert b"deterministic" in L.efunc_last_error()
    assert L.efunc_fit_step_static(C.byref(c), None, None, None, 1, None, None, None, 0, None, None) == \
        E.EFUNC_EUNSUPPORTED
    assert L.efunc_eval(None, None, None, 0, None, None, None, None, None) == E.EFUNC_EINVAL
    assert L.efunc_fit_step(None, None, None, None, 1, None, None, None, 0, None, None) == E.EFUNC_EINVAL
    assert L.efunc_destroy(None) == E.EFUNC_OK


def test_channel_counts_of_paper_variants():
    """efunc_channels (host-only) against the channel counts the paper prints
    for its ablation variants (Tab. ablation)."""
    import json
    from paper_2505_21319_amd import efunc as E
    E.lib()
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_param_counts.json")))
    for e in d["variants"]:
        c = E.efunc_default_config(e["R"])
        c.degree, c.grid_keys, c.offsets, c.learn_scale = (e["degree"], e["grid_keys"],
                                                           e["moved_keys"], e["learn_scale"])
        assert E.efunc_channels(c) == e["channels"], e["config"]
        assert E.efunc_channels(c) * e["R"] ** 3 == e["params"], e["config"]
    c = E.efunc_default_config(8)
    c.degree = 3
    with pytest.raises(E.EfuncError):
        E.efunc_channels(c)
    c = E.efunc_default_config(8)
    c.grid_keys, c.offsets = 0, 0
    with pytest.raises(E.EfuncError):
        E.efunc_channels(c)


def test_network_and_convolution_arguments_are_rejected_before_any_device_work(L):
    """The learned-initialiser entry points validate on the host: every call
    here fails one check before a kernel could be launched (the pointers are
    never dereferenced)."""
    from paper_2505_21319_amd import efunc as E
    fake = C.c_void_p(4096)       # 16-byte aligned, never touched
    odd = C.c_void_p(4096 + 2)    # misaligned
    out = C.c_void_p()
    ch = (C.c_int32 * 3)(1, 16, 13)
    assert L.efunc_initnet_create(1, 2, 2, ch, C.byref(out)) == E.EFUNC_EINVAL      # R < 2
    assert L.efunc_initnet_create(8, 2, 0, ch, C.byref(out)) == E.EFUNC_EINVAL      # no layer
    bad = (C.c_int32 * 3)(1, 65, 13)
    assert L.efunc_initnet_create(8, 2, 2, bad, C.byref(out)) == E.EFUNC_EINVAL     # > 64 channels
    assert b"channels[1] = 65" in L.efunc_last_error()
    assert L.efunc_initnet_forward(None, fake, fake, 1, fake, None) == E.EFUNC_EINVAL
    assert L.efunc_initnet_backward(None, fake, 1, fake, None) == E.EFUNC_EINVAL
    # conv3d: NULL output, channel range, Kpad, V not a multiple of R^3, alignment
    assert L.efunc_conv3d_bf16(fake, 16, fake, 448, 16, None, 0, None, 4, 64, None, None, None, None) \
        == E.EFUNC_EINVAL
    assert L.efunc_conv3d_bf16(fake, 65, fake, 1760, 16, None, 0, None, 4, 64, fake, None, None, None) \
        == E.EFUNC_EINVAL
    assert L.efunc_conv3d_bf16(fake, 16, fake, 440, 16, None, 0, None, 4, 64, fake, None, None, None) \
        == E.EFUNC_EINVAL                                                              # Kpad % 32 != 0
    assert L.efunc_conv3d_bf16(fake, 16, fake, 448, 16, None, 0, None, 4, 65, fake, None, None, None) \
        == E.EFUNC_EINVAL                                                              # V % R^3 != 0
    assert L.efunc_conv3d_bf16(odd, 16, fake, 448, 16, None, 0, None, 4, 64, fake, None, None, None) \
        == E.EFUNC_EINVAL                                                              # x misaligned
    assert b"16-byte" in L.efunc_last_error()
    assert L.efunc_conv3d_bf16(fake, 16, fake, 448, 16, None, 0, None, 4, 64, None, None, odd, None) \
        == E.EFUNC_EINVAL                                                              # yT misaligned
    assert L.efunc_conv3d_wgrad_bf16(None, 16, fake, 16, 4, 64, fake, None, None) == E.EFUNC_EINVAL
    assert L.efunc_conv3d_wgrad_bf16(fake, 16, odd, 16, 4, 64, fake, None, None) == E.EFUNC_EINVAL
    assert L.efunc_conv3d_wgrad_bf16(fake, 0, fake, 16, 4, 64, fake, None, None) == E.EFUNC_EINVAL
    assert L.efunc_conv3d_pack_weights(None, 16, 16, fake, fake, None) == E.EFUNC_EINVAL
    assert L.efunc_adam_update(None, fake, fake, fake, 10, 1, None, None) == E.EFUNC_EINVAL
    assert L.efunc_adam_update(fake, fake, fake, fake, 10, 0, None, None) == E.EFUNC_EINVAL  # step 0
    assert L.efunc_loss_grad(None, fake, fake, fake, 10, fake, None, None) == E.EFUNC_EINVAL
