"""Host logic of the batched solver, on the CPU (no device call): the tile table
covers every row of every system exactly once, in 64-row-aligned tiles of at most
the tile size, numbered 0..G-1 inside each system; whole systems go to one XCD
(tile t runs on XCD t % 8) and the XCDs get nearly equal numbers of tiles."""
import numpy as np
import pytest

from paper_2302_04180_amd import rpk


@pytest.fixture(scope="module", autouse=True)
def lib():
    import torch  # noqa: F401  (one HIP runtime shared with torch)
    rpk.load()


def check_plan(sizes, tile):
    t = rpk.plan_tiles(sizes, tile)
    assert len(t) % 8 == 0
    real = t[t[:, 0] >= 0]
    for k, n in enumerate(sizes):
        mine = real[real[:, 0] == k]
        g = max(1, -(-n // tile))
        assert len(mine) == g                                   # G_k tiles
        assert sorted(mine[:, 3].tolist()) == list(range(g))    # record indices 0..G-1
        order = np.argsort(mine[:, 1])
        lo, hi = mine[order, 1], mine[order, 2]
        assert lo[0] == 0 and hi[-1] == n and np.all(lo[1:] == hi[:-1])  # exact cover, no overlap
        assert np.all(lo % 64 == 0) and np.all(hi - lo <= tile) and np.all(hi > lo)
        xcd = {int(p) % 8 for p in np.nonzero((t[:, 0] == k))[0]}
        assert len(xcd) == 1                                    # one XCD per system
    per_xcd = [int(np.sum(t[x::8, 0] >= 0)) for x in range(8)]
    assert max(per_xcd) - min(per_xcd) <= max(-(-n // tile) for n in sizes)
    assert np.all(t[t[:, 0] < 0, 1:3] == 0)
    return t


def test_plan_uneven_systems():
    rng = np.random.default_rng(5)
    sizes = [int(e) ** 3 for e in rng.integers(8, 49, size=256)]
    for tile in (1024, 4096, 16384):
        check_plan(sizes, tile)


def test_plan_edge_cases():
    check_plan([1], 64)                        # one row
    check_plan([64, 65, 127, 128, 129], 64)    # ragged tails
    check_plan([10 ** 6], 4096)                # one large system over many tiles
    check_plan([5] * 100, 1024)                # many tiny systems
    with pytest.raises(rpk.RpkError):
        rpk.plan_tiles([100], 100)             # tile not a multiple of 64
    with pytest.raises(rpk.RpkError):
        rpk.plan_tiles([0], 64)                # empty system


def test_server_rejects_bad_options_without_device_work():
    import ctypes
    lib = rpk.load()
    o = rpk.ServerOpts(0, 4, 0, rpk.Opts(1e-9, 10, 1, 0, 0, 0, rpk._launch(), None, None))
    h = ctypes.c_void_p()
    assert lib.rpk_server_create(ctypes.byref(o), ctypes.byref(h)) == 1          # no budget
    o = rpk.ServerOpts(1 << 20, 0, 0, rpk.Opts(1e-9, 10, 1, 0, 0, 0, rpk._launch(), None, None))
    assert lib.rpk_server_create(ctypes.byref(o), ctypes.byref(h)) == 1          # no slot
    o = rpk.ServerOpts(1 << 20, 4, 0, rpk.Opts(1e-9, 10, 1, 0, 0, 1, rpk._launch(), None, None))
    assert lib.rpk_server_create(ctypes.byref(o), ctypes.byref(h)) == 1          # resume is not for servers
