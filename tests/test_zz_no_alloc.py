"""ljmd_batch_read_noalloc (no device allocation, fixed staging array) against
ljmd_batch_read through the C ABI: bitwise equal results on two calls in a row, the second
with a smaller replica; a replica beyond the staging limit is refused before device work."""

import ctypes as C

import numpy as np
import pytest

from paper_1308_5587_amd import inputs as gen
from parity import print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ljmd_mod():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1308_5587_amd import ljmd

    ljmd.load()
    return ljmd


def _read(lib, h, slot, n, noalloc):
    pos, vel, f = np.empty((n, 3)), np.empty((n, 3)), np.empty((n, 3))
    e, w = np.empty(2), np.empty(6)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    fn = lib.ljmd_batch_read_noalloc if noalloc else lib.ljmd_batch_read
    rc = fn(h, slot, dp(pos), dp(vel), dp(f), dp(e), dp(w))
    return rc, (pos, vel, f, e, w)


def test_noalloc_read_matches_read(ljmd_mod):
    print_case("batch read without allocation vs batch read")
    big = gen.make_lj_fluid(20000, rho=0.8442, T=1.2, seed=41)
    small = gen.make_lj_fluid(900, rho=0.7, T=1.0, seed=42)
    b = ljmd_mod.Batch(256 << 20, 4, precision="mixed", block_steps=10)
    sb = b.admit(big, 20)
    ss = b.admit(small, 30)
    while len(b.poll()) < 2:
        b.run_block()
    lib = ljmd_mod.load()
    for slot, n in ((sb, big.n), (ss, small.n)):  # second call: the smaller replica
        rc0, ref = _read(lib, b._h, slot, n, False)
        rc1, got = _read(lib, b._h, slot, n, True)
        assert rc0 == 0 and rc1 == 0, lib.ljmd_last_error()
        for x, y in zip(ref, got):
            assert np.array_equal(x, y)
    # the larger replica again after the smaller one (the array keeps the last contents)
    rc0, ref = _read(lib, b._h, sb, big.n, False)
    rc1, got = _read(lib, b._h, sb, big.n, True)
    assert rc0 == 0 and rc1 == 0
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)
    b.close()


def test_noalloc_read_refuses_beyond_limit(ljmd_mod):
    print_case("batch read without allocation: replica beyond the staging limit")
    n = 360_000  # 3 doubles each exceed the 8 MiB staging array
    spec = gen.make_lj_fluid(n, rho=0.8442, T=1.2, seed=43)
    b = ljmd_mod.Batch(1 << 30, 1, precision="mixed", block_steps=2,
                       threads_per_particle=2, block_size=256)
    s = b.admit(spec, 2)
    b.run_block()
    assert b.poll() == [s]
    with pytest.raises(ljmd_mod.LjmdError) as e:
        b.read(s, noalloc=True)
    assert e.value.code == ljmd_mod.LJMD_E_INVAL
    got = b.read(s)  # the allocating read still works
    assert got["pos"].shape == (n, 3)
    b.close()
