"""The C-ABI library without a GPU: it loads, exports every symbol include/ljmd.h declares,
validates arguments before touching a device, and reports a missing device as
LJMD_E_DEVICE with a message. No compute call is made here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1308_5587_amd import ljmd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(ljmd_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ljmd.LIB_PATH):
        from paper_1308_5587_amd import build_lib

        build_lib.build()
    return ljmd.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared_functions()
    assert len(declared) >= 16
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
    assert set(ljmd.EXPORTED) <= declared


def test_version(lib):
    assert "gfx950" in ljmd.version()


def _cfg(**kw):
    cfg = ljmd.LjmdConfig()
    for a in range(3):
        cfg.box[a] = kw.get("L", 10.0)
    cfg.ntypes = kw.get("ntypes", 1)
    cfg.dt = kw.get("dt", 0.005)
    cfg.skin = kw.get("skin", 0.4)
    cfg.precision = kw.get("precision", 0)
    cfg.threads_per_particle = kw.get("tpp", 0)
    cfg.block_size = kw.get("block", 0)
    cfg.graph_steps = kw.get("graph", 0)
    return cfg


def _create(lib, cfg, n=4, types=None, pos=None):
    pos = np.ones((n, 3)) if pos is None else pos
    vel = np.zeros((n, 3))
    typ = np.zeros(n, np.int32) if types is None else np.asarray(types, np.int32)
    h = C.c_void_p()
    rc = lib.ljmd_system_create(C.byref(cfg), n, pos.ctypes.data_as(C.POINTER(C.c_double)),
                                vel.ctypes.data_as(C.POINTER(C.c_double)),
                                typ.ctypes.data_as(C.POINTER(C.c_int32)), None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("kw,why", [
    (dict(dt=0.0), "dt"), (dict(dt=-1.0), "dt"), (dict(skin=-0.1), "skin"),
    (dict(L=0.0), "box"), (dict(L=float("nan")), "box"), (dict(ntypes=0), "ntypes"),
    (dict(ntypes=17), "ntypes"), (dict(precision=5), "precision"), (dict(tpp=3), "threads"),
    (dict(block=100), "block"), (dict(graph=3), "graph"),
])
def test_invalid_config_rejected_before_device(lib, kw, why):
    rc, h = _create(lib, _cfg(**kw))
    assert rc == ljmd.LJMD_E_INVAL
    assert not h.value
    assert lib.ljmd_last_error().decode()


def test_invalid_arrays_rejected(lib):
    rc, _ = _create(lib, _cfg(), types=[0, 0, 1, 0])
    assert rc == ljmd.LJMD_E_INVAL and "type" in lib.ljmd_last_error().decode()
    bad = np.ones((4, 3))
    bad[2, 1] = np.inf
    rc, _ = _create(lib, _cfg(), pos=bad)
    assert rc == ljmd.LJMD_E_INVAL
    rc, _ = _create(lib, _cfg(), n=0, pos=np.ones((1, 3)))
    assert rc == ljmd.LJMD_E_INVAL


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.ljmd_step(None, 1) == ljmd.LJMD_E_INVAL
    assert lib.ljmd_pair_lj_set(None, 0, 0, 1.0, 1.0, 2.5) == ljmd.LJMD_E_INVAL
    out = np.zeros(6)
    assert lib.ljmd_get_virial(None, out.ctypes.data_as(C.POINTER(C.c_double))) == ljmd.LJMD_E_INVAL
    lib.ljmd_system_destroy(None)


def test_no_device_reports_device_error(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible; this checks the no-device path")
    rc, h = _create(lib, _cfg())
    assert rc == ljmd.LJMD_E_DEVICE
    assert "device" in lib.ljmd_last_error().decode().lower()
    with pytest.raises(ljmd.LjmdError) as e:
        ljmd.System(np.array([10.0] * 3), np.ones((2, 3)), np.zeros((2, 3)), np.zeros(2, np.int32),
                    pairs=[(0, 0, 1.0, 1.0, 2.5)])
    assert e.value.code == ljmd.LJMD_E_DEVICE


def test_struct_layout_matches_header(lib, tmp_path):
    """The ctypes mirrors of ljmd_config and ljmd_stats have the C compiler's layout."""
    import subprocess

    fields_cfg = [f for f, _ in ljmd.LjmdConfig._fields_]
    fields_st = [f for f, _ in ljmd.LjmdStats._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ljmd.h"', "int main(void){",
             'printf("%zu %zu\\n", sizeof(ljmd_config), sizeof(ljmd_stats));']
    lines += [f'printf("%zu\\n", offsetof(ljmd_config, {f}));' for f in fields_cfg]
    lines += [f'printf("%zu\\n", offsetof(ljmd_stats, {f}));' for f in fields_st]
    lines += ["return 0;}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == C.sizeof(ljmd.LjmdConfig) and vals[1] == C.sizeof(ljmd.LjmdStats)
    offs = vals[2:]
    for k, f in enumerate(fields_cfg):
        assert getattr(ljmd.LjmdConfig, f).offset == offs[k], f
    for k, f in enumerate(fields_st):
        assert getattr(ljmd.LjmdStats, f).offset == offs[len(fields_cfg) + k], f
