"""The C-ABI library loads and exports what include/pic.h declares (CPU only).

Only calls that validate arguments before touching the GPU are made here.
"""

import ctypes
import os
import re

import pytest

from paper_2410_18414_amd import pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b([A-Za-z_]\w*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_library_exports_every_declared_symbol():
    lib = pic.load()
    decl = declared_functions()
    assert len(decl) >= 16
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(pic.EXPORTS) == decl


def _cfg(**kw):
    base = dict(nx=32, ny=32, lx=1.0, ly=1.0, dt=0.01, degree=2, scheme="bdf", bdf_order=1,
                dtype="f64", max_particles=100)
    base.update(kw)
    return pic.make_config(**base)


@pytest.mark.parametrize("bad", [
    dict(nx=7), dict(ny=4), dict(nx=2048), dict(ny=1025), dict(degree=6), dict(degree=0), dict(bdf_order=7),
    dict(dt=0.0), dict(dt=2.0), dict(c=2.0), dict(max_particles=0), dict(m=0.0), dict(lx=-1.0),
    dict(flags=256)])
def test_invalid_configs_rejected(bad):
    cfg = _cfg(**bad)
    assert pic.load().pic_workspace_bytes(ctypes.byref(cfg)) == 0
    assert pic.load().pic_last_error(None)


def test_valid_config_and_history_counts():
    assert pic.workspace_bytes(_cfg()) > 0
    assert pic.workspace_bytes(_cfg(nx=30, ny=1021)) > 0      # any side in [8, 1024]
    assert pic.history_fields(_cfg(scheme="bdf", bdf_order=2)) == 18
    assert pic.history_fields(_cfg(scheme="bdf", bdf_order=3)) == 27
    assert pic.history_fields(_cfg(scheme="cdf2")) == 18
    assert pic.history_fields(_cfg(scheme="cdf2_semi")) == 18
    assert pic.history_fields(_cfg(scheme="cdf2_explicit")) == 18
    assert pic.history_fields(_cfg(scheme="dirk2")) == 17
    assert pic.history_fields(_cfg(scheme="dirk3")) == 17
    cfg = _cfg()
    cfg.scheme = 6                       # no such scheme
    assert pic.load().pic_workspace_bytes(ctypes.byref(cfg)) == 0
    assert b"scheme" in pic.load().pic_last_error(None)


def test_create_rejects_bad_workspace_without_gpu():
    lib = pic.load()
    cfg = _cfg()
    h = ctypes.c_void_p()
    st = lib.pic_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h))
    assert st == 3 and not h.value          # PIC_ERR_WORKSPACE
    st = lib.pic_create(ctypes.byref(cfg), ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert st == 3 and b"too small" in lib.pic_last_error(None)
    cfg.abi_version = 99
    assert lib.pic_create(ctypes.byref(cfg), ctypes.c_void_p(256), 1 << 40, None,
                          ctypes.byref(h)) == 1


@pytest.mark.parametrize("flags,scheme", [(pic.FLAG_JVSTAR | pic.FLAG_ADJOINT, "bdf"),
                                          (pic.FLAG_NAIVE_RHO | pic.FLAG_ADJOINT, "bdf"),
                                          (pic.FLAG_NAIVE_RHO, "cdf2_semi"),
                                          (pic.FLAG_DIRK_SUBSTEP, "bdf"),
                                          (pic.FLAG_DIRK_SUBSTEP | pic.FLAG_NAIVE_RHO, "dirk2"),
                                          (pic.FLAG_ADJOINT, "bdf-odd"),
                                          (pic.FLAG_DETERMINISTIC | pic.FLAG_NO_SORT, "bdf"),
                                          (pic.FLAG_DETERMINISTIC | pic.FLAG_NAIVE_RHO, "bdf"),
                                          (pic.FLAG_DETERMINISTIC | pic.FLAG_ADJOINT, "bdf")])
def test_create_rejects_unsupported_combinations_without_gpu(flags, scheme):
    """Unsupported flag/scheme combinations fail (PIC_ERR_UNSUPPORTED) before
    the workspace is looked at."""
    lib = pic.load()
    cfg = _cfg(flags=flags, scheme="bdf", nx=30) if scheme == "bdf-odd" else _cfg(flags=flags, scheme=scheme)
    h = ctypes.c_void_p()
    assert lib.pic_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h)) == 2
    assert not h.value


def test_null_context_calls_fail_cleanly():
    lib = pic.load()
    for name in ("deposit_current", "field_solve", "gather_push"):
        assert getattr(lib, name)(None) == 1
    assert lib.step(None, 1) == 1


def test_batch_config_rules_without_gpu():
    lib = pic.load()
    a = _cfg(nx=32, ny=32)
    b = _cfg(nx=64, ny=16, max_particles=500)
    arr = (pic.ConfigStruct * 2)(a, b)
    assert lib.pic_batch_workspace_bytes(arr, 2) > 0
    c = _cfg(scheme="cdf2")
    arr2 = (pic.ConfigStruct * 2)(a, c)
    assert lib.pic_batch_workspace_bytes(arr2, 2) == 0
    assert b"share" in lib.pic_last_error(None)
    assert lib.pic_batch_workspace_bytes(arr, 0) == 0


def test_checkpoint_keys_are_config_fields():
    from paper_2410_18414_amd import state
    names = [n for n, _ in pic.ConfigStruct._fields_]
    assert all(k in names for k in state._KEYS)
