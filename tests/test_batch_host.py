"""CPU checks of the batched entry points' host side: workspace sizing of the
round schedule, tile-choice state, and argument validation before anything
is enqueued (no GPU needed)."""
import ctypes
import os

import pytest

pytest.importorskip("torch")
from paper_1909_04573_amd import prnu  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(prnu.LIB_PATH):
        pytest.fail("libprnu.so is not built (python -m paper_1909_04573_amd.build)")
    return prnu.lib()


def _cams(specs, base=0x10000000):
    """Fake device pointers, never dereferenced: (n, H, W, C, group) per camera."""
    arr = (prnu.Camera * len(specs))()
    addr = base
    for i, (n, H, W, C, d) in enumerate(specs):
        acc = C * H * W * 8
        arr[i] = prnu.Camera(0x1000, n, H, W, C, d, addr, addr + acc)
        addr += 2 * acc + 4096
    return arr


def _ws(lib, specs, budget=0, p=None):
    p = p or prnu.denoise_params()
    n = ctypes.c_size_t(0)
    rc = lib.prnu_batch_workspace_size(_cams(specs), len(specs), ctypes.byref(p), budget, ctypes.byref(n))
    return rc, n.value


def _pyramid_bytes(H, W, C, ng, levels=4):
    Hp, Wp = -(-H // 16) * 16, -(-W // 16) * 16
    al = lambda x: -(-x // 256) * 256  # noqa: E731
    b = al(ng * C * H * W * 4)
    for l in range(1, levels + 1):
        b += al(ng * C * 4 * (Hp >> l) * (Wp >> l) * 4)
    return b


def test_workspace_single_round(lib):
    specs = [(10, 72, 104, 3, 4), (40, 48, 48, 1, 2)]
    rc, n = _ws(lib, specs)
    assert rc == 0
    need = _pyramid_bytes(72, 104, 3, 3) + _pyramid_bytes(48, 48, 1, 20)
    assert need <= n <= need + 64 * 1024  # plus work tables and counters


def test_budget_limits_round_area(lib):
    specs = [(400, 1080, 1920, 1, 1), (300, 720, 1280, 1, 3), (100, 2160, 3840, 1, 10)]
    rc, big = _ws(lib, specs, 1 << 40)
    assert rc == 0
    total = _pyramid_bytes(1080, 1920, 1, 400) + _pyramid_bytes(720, 1280, 1, 100) + \
        _pyramid_bytes(2160, 3840, 1, 10)
    assert total <= big <= total + (1 << 20)
    rc, small = _ws(lib, specs, 1 << 30)
    assert rc == 0 and small < (1 << 30) + (1 << 22)
    # a budget below one group still schedules one group per round
    rc, tiny = _ws(lib, specs, 1024)
    assert rc == 0 and tiny >= _pyramid_bytes(2160, 3840, 1, 1)


def test_batch_validation(lib):
    p = prnu.denoise_params()
    P = ctypes.byref(p)
    ws = ctypes.c_void_p(0x40000000)
    h = ctypes.c_void_p()
    ok = [(10, 72, 104, 3, 4), (9, 64, 80, 1, 3)]
    n = ctypes.c_size_t(0)
    assert lib.prnu_batch_workspace_size(None, 1, P, 0, ctypes.byref(n)) == prnu.PRNU_E_INVAL
    assert lib.prnu_batch_workspace_size(_cams(ok), 0, P, 0, ctypes.byref(n)) == prnu.PRNU_E_INVAL
    assert lib.prnu_batch_workspace_size(_cams([(10, 15, 64, 1, 1)]), 1, P, 0, ctypes.byref(n)) == \
        prnu.PRNU_E_INVAL
    assert lib.prnu_batch_workspace_size(_cams([(10, 64, 64, 2, 1)]), 1, P, 0, ctypes.byref(n)) == \
        prnu.PRNU_E_INVAL
    assert lib.prnu_batch_workspace_size(_cams([(10, 64, 64, 1, 0)]), 1, P, 0, ctypes.byref(n)) == \
        prnu.PRNU_E_INVAL
    bad = prnu.denoise_params(taps=6)
    assert lib.prnu_batch_workspace_size(_cams(ok), 2, ctypes.byref(bad), 0, ctypes.byref(n)) == \
        prnu.PRNU_E_UNSUPPORTED
    # create: every failure below is found before any HIP call
    assert lib.prnu_batch_create(_cams(ok), 2, 5, P, 0, 0, 0, ws, 1 << 30, None, ctypes.byref(h)) == \
        prnu.PRNU_E_INVAL
    assert lib.prnu_batch_create(_cams(ok), 2, 0, P, 7, 0, 0, ws, 1 << 30, None, ctypes.byref(h)) == \
        prnu.PRNU_E_INVAL
    assert lib.prnu_batch_create(_cams(ok), 2, 0, P, 0, 8, 0, ws, 1 << 30, None, ctypes.byref(h)) == \
        prnu.PRNU_E_INVAL
    assert lib.prnu_batch_create(_cams(ok), 2, 0, P, 0, 0, 0, ws, 1024, None, ctypes.byref(h)) == \
        prnu.PRNU_E_WORKSPACE
    assert lib.prnu_batch_create(_cams(ok), 2, 0, P, 0, 0, 0, None, 1 << 30, None, ctypes.byref(h)) == \
        prnu.PRNU_E_WORKSPACE
    assert lib.prnu_batch_create(_cams(ok), 2, 0, P, 0, 0, 0, ctypes.c_void_p(0x40000010), 1 << 30, None,
                                 ctypes.byref(h)) == prnu.PRNU_E_WORKSPACE
    overlap = _cams(ok)
    overlap[1].A = overlap[0].B + 8  # inside camera 0's B
    assert lib.prnu_batch_create(overlap, 2, 0, P, 0, 0, 0, ws, 1 << 30, None, ctypes.byref(h)) == \
        prnu.PRNU_E_INVAL
    assert "overlap" in lib.prnu_last_error().decode()
    same = _cams(ok)
    same[0].B = same[0].A  # A and B of one camera
    assert lib.prnu_fingerprint_batch(same, 2, 0, P, 0, 0, ws, 1 << 30, None) == prnu.PRNU_E_INVAL
    nul = _cams(ok)
    nul[1].frames = None
    assert lib.prnu_fingerprint_batch(nul, 2, 0, P, 0, 0, ws, 1 << 30, None) == prnu.PRNU_E_INVAL
    assert lib.prnu_batch_launch(None, None) == prnu.PRNU_E_INVAL
    assert lib.prnu_batch_destroy(None) == prnu.PRNU_OK


def test_tile_state(lib):
    """Forward levels take strips of 64 (default) or 32 columns, inverse and
    MLE levels tiles of 32 (default) or 16, per kind, filter length and size."""
    assert prnu.get_tile(prnu.TILE_FWD, 16, 1000, 999) == 64
    prnu.set_tile(prnu.TILE_FWD, 16, 1000, 999, 32)
    assert prnu.get_tile(prnu.TILE_FWD, 16, 1000, 999) == 32
    assert prnu.get_tile(prnu.TILE_INV, 16, 1000, 999) == 32  # per kind
    prnu.set_tile(prnu.TILE_INV, 16, 1000, 999, 16)
    assert prnu.get_tile(prnu.TILE_INV, 16, 1000, 999) == 16
    assert prnu.get_tile(prnu.TILE_FWD, 8, 1000, 999) == 64  # per filter length
    prnu.set_tile(prnu.TILE_FWD, 16, 1000, 999, 0)
    prnu.set_tile(prnu.TILE_INV, 16, 1000, 999, 0)
    assert prnu.get_tile(prnu.TILE_FWD, 16, 1000, 999) == 64
    assert prnu.get_tile(prnu.TILE_INV, 16, 1000, 999) == 32
    # the forward strip's segment target: 6 workgroups per CU by default, 3 or 12
    assert prnu.get_tile(prnu.TILE_SEG, 16, 1000, 999) == 6
    for k in (3, 12):
        prnu.set_tile(prnu.TILE_SEG, 16, 1000, 999, k)
        assert prnu.get_tile(prnu.TILE_SEG, 16, 1000, 999) == k
    prnu.set_tile(prnu.TILE_SEG, 16, 1000, 999, 0)
    assert prnu.get_tile(prnu.TILE_SEG, 16, 1000, 999) == 6
    with pytest.raises(prnu.PrnuError, match="segment target"):
        prnu.set_tile(prnu.TILE_SEG, 16, 1000, 999, 32)
    for args in [(3, 16, 8, 8, 16), (0, 6, 8, 8, 32), (0, 16, 0, 8, 32), (0, 16, 8, 8, 24), (0, 16, 8, 8, 16),
                 (1, 16, 8, 8, 64), (2, 16, 8, 8, 64)]:
        with pytest.raises(prnu.PrnuError):
            prnu.set_tile(*args)


def test_autotune_workspace(lib):
    p = prnu.denoise_params()
    n = ctypes.c_size_t(0)
    assert lib.prnu_autotune_workspace_size(1080, 1920, 1, ctypes.byref(p), ctypes.byref(n)) == 0
    assert n.value >= 8 * 1080 * 1920 * 4
    assert lib.prnu_autotune_workspace_size(1080, 1920, 2, ctypes.byref(p), ctypes.byref(n)) == prnu.PRNU_E_INVAL
    assert lib.prnu_autotune(1080, 1920, 1, ctypes.byref(p), ctypes.c_void_p(0x40000000), 16, None, None) == \
        prnu.PRNU_E_WORKSPACE


def test_set_tiles_layout(lib):
    """set_tiles applies autotune's layout: forward levels 1..4, inverse 2..4,
    MLE, and the forward levels' segment targets from entry 12 on."""
    tiles = [32, 64, 32, 64, 0, 32, 16, 32, 16, 0, 0, 0, 3, 12, 0, 6]
    try:
        prnu.set_tiles(1080, 1920, tiles)
        Hp, Wp = 1088, 1920
        assert [prnu.get_tile(prnu.TILE_FWD, 16, Hp >> l, Wp >> l) for l in range(1, 5)] == tiles[0:4]
        assert [prnu.get_tile(prnu.TILE_INV, 16, Hp >> l, Wp >> l) for l in range(2, 5)] == tiles[5:8]
        assert prnu.get_tile(prnu.TILE_MLE, 16, Hp >> 1, Wp >> 1) == 16
        assert prnu.get_tile(prnu.TILE_INV, 16, Hp >> 1, Wp >> 1) == 32  # untouched: entry 4 is unused
        assert [prnu.get_tile(prnu.TILE_SEG, 16, Hp >> l, Wp >> l) for l in range(1, 5)] == [3, 12, 6, 6]
    finally:
        for l in range(1, 5):
            for kind in (prnu.TILE_FWD, prnu.TILE_INV, prnu.TILE_MLE, prnu.TILE_SEG):
                prnu.set_tile(kind, 16, 1088 >> l, 1920 >> l, 0)


def test_batch_planning_under_sanitizers(host_check):
    """Round packing of 40 mixed cameras under shrinking budgets, the batch
    validation and the tile table run clean under ASan + UBSan."""
    rc, out = host_check("batch")
    assert rc == 0 and "0 failed" in out, out
    assert "Sanitizer" not in out and "runtime error" not in out, out
