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


STRUCTS = [("ljmd_config", "LjmdConfig"), ("ljmd_stats", "LjmdStats"),
           ("ljmd_batch_config", "LjmdBatchConfig"), ("ljmd_replica_spec", "LjmdReplicaSpec"),
           ("ljmd_batch_stats", "LjmdBatchStats"), ("ljmd_tuning_entry", "LjmdTuningEntry")]


@pytest.mark.parametrize("cname,pyname", STRUCTS)
def test_struct_layout_matches_header(lib, tmp_path, cname, pyname):
    """The ctypes mirrors of the C structs have the C compiler's size and offsets."""
    import subprocess

    cls = getattr(ljmd, pyname)
    fields = [f for f, _ in cls._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ljmd.h"', "int main(void){",
             f'printf("%zu\\n", sizeof({cname}));']
    lines += [f'printf("%zu\\n", offsetof({cname}, {f}));' for f in fields]
    lines += ["return 0;}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == C.sizeof(cls)
    for k, f in enumerate(fields):
        assert getattr(cls, f).offset == vals[1 + k], f


def _bcfg(**kw):
    cfg = ljmd.LjmdBatchConfig()
    cfg.budget_bytes = kw.get("budget", 64 << 20)
    cfg.max_slots = kw.get("slots", 4)
    cfg.precision = kw.get("precision", 1)
    cfg.dt = kw.get("dt", 0.005)
    cfg.skin = kw.get("skin", 0.4)
    cfg.block_steps = kw.get("steps", 0)
    cfg.threads_per_particle = kw.get("tpp", 0)
    cfg.block_size = kw.get("block", 0)
    return cfg


@pytest.mark.parametrize("kw", [
    dict(slots=0), dict(precision=7), dict(dt=0.0), dict(skin=-1.0), dict(steps=3),
    dict(steps=-2), dict(tpp=5), dict(block=96), dict(budget=1000),
])
def test_invalid_batch_config_rejected_before_device(lib, kw):
    h = C.c_void_p()
    rc = lib.ljmd_batch_create(C.byref(_bcfg(**kw)), C.byref(h))
    assert rc == ljmd.LJMD_E_INVAL
    assert not h.value
    assert lib.ljmd_last_error().decode()


def test_batch_null_handles(lib):
    assert lib.ljmd_batch_run_block(None) == ljmd.LJMD_E_INVAL
    assert lib.ljmd_batch_release(None, 0) == ljmd.LJMD_E_INVAL
    k = C.c_int32(0)
    assert lib.ljmd_batch_poll(None, None, C.byref(k)) == ljmd.LJMD_E_INVAL
    lib.ljmd_batch_destroy(None)


def test_batch_no_device(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible; this checks the no-device path")
    h = C.c_void_p()
    assert lib.ljmd_batch_create(C.byref(_bcfg()), C.byref(h)) == ljmd.LJMD_E_DEVICE
    assert not h.value


def test_tuning_table_round_trip(lib, tmp_path):
    """The tuning table is host state: entries set are read back in key order, survive a
    JSON round trip, replace entries of the same key, and an invalid entry stores nothing."""
    mine = [dict(precision=1, multi_type=1, size_bucket=25, threads_per_particle=4, block_size=448),
            dict(precision=0, multi_type=0, size_bucket=26, threads_per_particle=2, block_size=512)]
    ljmd.set_tuning(mine)
    table = ljmd.tuning_table()
    keys = [(e["precision"], e["multi_type"], e["size_bucket"]) for e in table]
    assert keys == sorted(keys)
    for e in mine:
        assert e in table
    path = tmp_path / "tuning.json"
    ljmd.save_tuning(path)
    ljmd.set_tuning([dict(mine[0], threads_per_particle=8)])  # same key: replaced
    assert dict(mine[0], threads_per_particle=8) in ljmd.tuning_table()
    ljmd.load_tuning(path)
    assert mine[0] in ljmd.tuning_table()
    n = len(ljmd.tuning_table())
    bad = [dict(mine[0], size_bucket=3), dict(mine[1], block_size=96)]
    with pytest.raises(ljmd.LjmdError) as e:
        ljmd.set_tuning(bad)
    assert e.value.code == ljmd.LJMD_E_INVAL
    assert len(ljmd.tuning_table()) == n  # the valid first entry was not stored either
    for field, value in (("threads_per_particle", 3), ("precision", 2), ("multi_type", 2),
                         ("size_bucket", 27), ("block_size", 64)):
        with pytest.raises(ljmd.LjmdError):
            ljmd.set_tuning([dict(mine[1], **{field: value})])
    cnt = C.c_int32(-1)
    assert lib.ljmd_tuning_get(None, 4, C.byref(cnt)) == ljmd.LJMD_E_INVAL
    assert lib.ljmd_tuning_get(None, 0, None) == ljmd.LJMD_E_INVAL
    assert lib.ljmd_tuning_set(None, 1) == ljmd.LJMD_E_INVAL
