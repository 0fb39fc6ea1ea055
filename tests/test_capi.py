"""The C ABI library without a GPU: it loads, exports every function that
include/sun.h declares, and validates arguments on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sun.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sun_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    """The library, built first if nothing is built (these tests make no
    GPU calls)."""
    import os
    from paper_1112_4533_amd import build, sun
    if not os.path.exists(sun.LIB_PATH):
        build.build()
    return sun.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _bytes(lib, nc, L, dtype):
    lb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib.sun_lattice_bytes(nc, (ctypes.c_int * 4)(*L), dtype, ctypes.byref(lb), ctypes.byref(sb))
    return rc, lb.value, sb.value


def test_lattice_bytes(lib):
    rc, lb, sb = _bytes(lib, 3, (32, 32, 32, 32), 0)
    assert rc == 0 and lb == 4 * 32 ** 4 * 18 * 4 and sb >= 16 * 4 * 32 ** 4 // 256
    rc, lb, _ = _bytes(lib, 2, (8, 8, 8, 8), 1)
    assert rc == 0 and lb == 4 * 8 ** 4 * 4 * 8           # SU(2): 4 reals per link
    rc, lb, _ = _bytes(lib, 8, (12, 12, 12, 12), 1)
    assert rc == 0 and lb == 4 * 12 ** 4 * 128 * 8
    # SU(3) two-row storage: 12 reals per link
    rc, lb, _ = _bytes(lib, 3, (32, 32, 32, 32), 2)
    assert rc == 0 and lb == 4 * 32 ** 4 * 12 * 4
    rc, lb, _ = _bytes(lib, 3, (8, 8, 8, 8), 3)
    assert rc == 0 and lb == 4 * 8 ** 4 * 12 * 8
    for nc in (2, 4):
        assert _bytes(lib, nc, (8, 8, 8, 8), 2)[0] == -4
    # the workgroup-per-link path: Nc^2 complex entries per link, one FP64
    # partial pair per link in the scratch buffer
    for nc, dt, size in [(5, 0, 4), (9, 0, 4), (16, 1, 8), (32, 0, 4), (4, 4, 4), (8, 5, 8), (32, 1, 8), (29, 5, 8)]:
        rc, lb, sb = _bytes(lib, nc, (8, 8, 8, 8), dt)
        assert rc == 0 and lb == 4 * 8 ** 4 * 2 * nc * nc * size, (nc, dt)
        assert sb >= 16 * 4 * 8 ** 4, (nc, dt)
    for nc, dt in [(3, 4), (2, 5)]:    # the workgroup-per-link path starts at Nc = 4
        assert _bytes(lib, nc, (8, 8, 8, 8), dt)[0] == -4, (nc, dt)


@pytest.mark.parametrize("nc,L,dtype", [
    (1, (8, 8, 8, 8), 0), (33, (8, 8, 8, 8), 0), (3, (7, 8, 8, 8), 0), (3, (1, 8, 8, 8), 0),
    (3, (8, 8, 3, 8), 0), (3, (8, 8, 8, 8), 6), (3, (8, 8, 8, 8), -1), (3, (256, 256, 256, 256), 0)])
def test_lattice_bytes_rejects(lib, nc, L, dtype):
    rc, _, _ = _bytes(lib, nc, L, dtype)
    assert rc == -1
    assert lib.sun_last_error()


def test_create_validates_buffers_without_touching_them(lib):
    L = (4, 4, 4, 4)
    rc, lb, sb = _bytes(lib, 3, L, 0)
    h = ctypes.c_void_p()
    args = lambda links, lbytes, scr, sbytes: (3, (ctypes.c_int * 4)(*L), 0, ctypes.c_void_p(links), lbytes,
                                               ctypes.c_void_p(scr), sbytes, ctypes.byref(h))
    assert lib.sun_lattice_create(*args(0, lb, 0x20000, sb)) == -2          # null links
    assert lib.sun_lattice_create(*args(0x10000, lb - 1, 0x20000, sb)) == -2
    assert lib.sun_lattice_create(*args(0x10000, lb, 0x20000, sb - 256)) == -2
    assert lib.sun_lattice_create(*args(0x10010, lb, 0x20000, sb)) == -1    # misaligned
    assert lib.sun_lattice_create(*args(0x10000, lb, 0x20000, sb)) == 0
    v = ctypes.c_uint64()
    assert lib.sun_get_step(h, ctypes.byref(v)) == 0 and v.value == 0
    assert lib.sun_set_step(h, 77) == 0
    assert lib.sun_get_step(h, ctypes.byref(v)) == 0 and v.value == 77
    # bad phase arguments are rejected before any launch
    assert lib.sun_phase(h, 2, 0, 0, 6.0, 1, 0, None) == -1
    assert lib.sun_phase(h, 0, 4, 0, 6.0, 1, 0, None) == -1
    assert lib.sun_phase(h, 0, 0, 2, 6.0, 1, 0, None) == -1
    assert lib.sun_sweep(h, 6.0, -1, 0, 1, 1, None) == -1
    assert lib.sun_plaquette(h, None, None) == -2
    assert lib.sun_profile_read(h, 9, None, None) == -1
    assert lib.sun_profile(h, -2) == -1
    assert lib.sun_profile(h, -1) == 0          # run-timing mode
    assert lib.sun_profile(h, 0) == 0
    # launch shapes: only the instantiated workgroup sizes, wave caps and walks
    b, x, w, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    get = lambda k: (lib.sun_get_launch(h, k, ctypes.byref(b), ctypes.byref(x), ctypes.byref(w), ctypes.byref(t)),
                     b.value, x.value, w.value, t.value)
    # (a 4^4 plane holds 8 checkerboard sites: the default t-blocked walk
    # falls back to the linear one and reports 0)
    # (18-real FP32 links, 72 bytes: the overrelaxation default caps at 8)
    assert get(0) == (0, 256, 1, 16, 0) and get(1) == (0, 256, 1, 8, 0)
    assert lib.sun_set_launch(h, -1, 100, 1, 8, 0) == -1
    assert lib.sun_set_launch(h, -1, 64, 1, 5, 0) == -1
    assert lib.sun_set_launch(h, 2, 64, 1, 8, 0) == -1
    assert lib.sun_set_launch(h, -1, 64, 1, 8, 3) == -1
    assert lib.sun_set_launch(h, 1, 64, 0, 16, 0) == 0
    assert get(0) == (0, 256, 1, 16, 0) and get(1) == (0, 64, 0, 16, 0)
    assert lib.sun_set_launch(h, -1, 128, 1, 8, 0) == 0
    assert get(0) == (0, 128, 1, 8, 0) and get(1) == (0, 128, 1, 8, 0)
    assert lib.sun_get_launch(h, 0, None, None, None, None) == -1
    # sites per work-item: 1, 2 or 4 per kind, kept by sun_set_launch
    s = ctypes.c_int()
    assert lib.sun_get_sites_per_item(h, 0, ctypes.byref(s)) == 0 and s.value == 1   # small lattice
    assert lib.sun_get_sites_per_item(h, 1, ctypes.byref(s)) == 0 and s.value == 1
    assert lib.sun_set_sites_per_item(h, -1, 3) == -1
    assert lib.sun_set_sites_per_item(h, 2, 2) == -1
    assert lib.sun_set_sites_per_item(None, -1, 2) == -1
    assert lib.sun_set_sites_per_item(h, 1, 4) == 0
    assert lib.sun_get_sites_per_item(h, 1, ctypes.byref(s)) == 0 and s.value == 4
    assert lib.sun_get_sites_per_item(h, 0, ctypes.byref(s)) == 0 and s.value == 1
    assert lib.sun_set_launch(h, -1, 128, 1, 8, 0) == 0
    assert lib.sun_get_sites_per_item(h, 1, ctypes.byref(s)) == 0 and s.value == 4
    assert lib.sun_get_sites_per_item(h, 1, None) == -1
    assert lib.sun_set_sites_per_item(h, -1, 1) == 0
    # a 4^4 plane holds 8 checkerboard sites: no whole workgroup, linear walk
    assert lib.sun_set_launch(h, -1, 64, 1, 0, 4) == 0
    assert get(1) == (0, 64, 1, 0, 0)
    lib.sun_lattice_destroy(h)
    # the t-blocked walk needs L_t % tblock == 0 and L_x L_y / 2 % block == 0
    L2 = (16, 16, 4, 8)
    rc, lb, sb = _bytes(lib, 3, L2, 0)
    assert lib.sun_lattice_create(3, (ctypes.c_int * 4)(*L2), 0, ctypes.c_void_p(0x10000), lb,
                                  ctypes.c_void_p(0x20000), sb, ctypes.byref(h)) == 0
    assert get(0) == (0, 256, 1, 16, 0)          # 128 sites per plane: no whole 256-item tile
    assert lib.sun_set_launch(h, -1, 128, 1, 0, 4) == 0
    assert get(0) == (0, 128, 1, 0, 4) and get(1) == (0, 128, 1, 0, 4)
    for block, tb, want in [(64, 4, 4), (128, 8, 8), (128, 2, 2), (256, 4, 0), (64, 1, 0), (64, 0, 0)]:
        assert lib.sun_set_launch(h, 1, block, 1, 12, tb) == 0
        assert get(1) == (0, block, 1, 12, want), (block, tb)
    lib.sun_lattice_destroy(h)


def test_batch_argument_checks(lib):
    tb = ctypes.c_size_t()
    assert lib.sun_batch_bytes(0, ctypes.byref(tb)) == -1
    assert lib.sun_batch_bytes(64, ctypes.byref(tb)) == 0 and tb.value >= 64 * 64
    out = ctypes.c_void_p()
    one = (ctypes.c_void_p * 1)(None)
    d = (ctypes.c_double * 1)(1.0)
    s = (ctypes.c_uint64 * 1)(1)
    assert lib.sun_batch_create(1, one, d, s, ctypes.c_void_p(0x10000), tb.value, ctypes.byref(out)) == -1
    # a lattice on the workgroup-per-link path passes the checks (here the
    # table upload then fails for want of a device, never as unsupported)
    L = (ctypes.c_int * 4)(4, 4, 2, 2)
    lb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.sun_lattice_bytes(9, L, 0, ctypes.byref(lb), ctypes.byref(sb)) == 0
    h = ctypes.c_void_p()
    assert lib.sun_lattice_create(9, L, 0, ctypes.c_void_p(0x100000), lb.value, ctypes.c_void_p(0x200000), sb.value,
                                  ctypes.byref(h)) == 0
    wide = (ctypes.c_void_p * 1)(h.value)
    rc = lib.sun_batch_create(1, wide, d, s, ctypes.c_void_p(0x10000), tb.value, ctypes.byref(out))
    assert rc in (0, -3), rc
    if rc == 0:
        lib.sun_batch_destroy(out)
    else:
        assert b"batch table upload" in lib.sun_last_error()
    lib.sun_lattice_destroy(h)
    # a lattice listed twice, or two lattices over overlapping buffers, would
    # update the same links in one launch: refused before the table is written
    assert lib.sun_lattice_bytes(3, L, 0, ctypes.byref(lb), ctypes.byref(sb)) == 0
    hs = []
    for links, scr in [(0x1000000, 0x2000000), (0x3000000, 0x4000000), (0x1000000 + 256, 0x5000000),
                       (0x6000000, 0x4000000 + sb.value - 256)]:
        h = ctypes.c_void_p()
        assert lib.sun_lattice_create(3, L, 0, ctypes.c_void_p(links), lb.value, ctypes.c_void_p(scr), sb.value,
                                      ctypes.byref(h)) == 0
        hs.append(h.value)
    two = (ctypes.c_double * 2)(6.0, 6.0)
    s2 = (ctypes.c_uint64 * 2)(1, 2)
    for pair in [(0, 0), (0, 2), (1, 3)]:
        arr = (ctypes.c_void_p * 2)(hs[pair[0]], hs[pair[1]])
        assert lib.sun_batch_create(2, arr, two, s2, ctypes.c_void_p(0x10000), tb.value, ctypes.byref(out)) == -1, pair
        assert b"share device memory" in lib.sun_last_error(), pair
    for hv in hs:
        lib.sun_lattice_destroy(ctypes.c_void_p(hv))
    assert lib.sun_batch_sweep(None, 1, 1, 1, None, None) == -1
    assert lib.sun_batch_replay(None, None) == -1


def test_watchdog_argument_checks(lib):
    """The watchdog's threshold must be finite and >= 0, and sun_check needs
    a preceding sun_watchdog; both refusals come before any launch."""
    L = (4, 4, 4, 4)
    rc, lb, sb = _bytes(lib, 3, L, 0)
    h = ctypes.c_void_p()
    assert lib.sun_lattice_create(3, (ctypes.c_int * 4)(*L), 0, ctypes.c_void_p(0x10000), lb, ctypes.c_void_p(0x200000),
                                  sb, ctypes.byref(h)) == 0
    for bad in (-1e-3, float("nan"), float("inf")):
        assert lib.sun_watchdog(h, bad, None) == -1
        assert b"threshold" in lib.sun_last_error()
    assert lib.sun_watchdog(None, 1e-4, None) == -1
    d = ctypes.c_double()
    assert lib.sun_check(h, ctypes.byref(d), None) == -1
    assert b"never set" in lib.sun_last_error()
    assert lib.sun_check(None, ctypes.byref(d), None) == -1
    lib.sun_lattice_destroy(h)
    # the watchdog state adds 256 bytes to the scratch buffer
    from paper_1112_4533_amd import sun
    assert sun.SUN_ENUMERIC == -5
    assert issubclass(sun.SunNumericError, sun.SunError)


def test_sampler_hook_argument_checks(lib):
    """The SU(2) draw hook checks its arguments before any launch: the
    register-path and wide storage codes are accepted (the wide ones select
    the batched draw), the two-row codes are not; a negative count or a null
    buffer is refused and an empty draw is a no-op."""
    p = ctypes.c_void_p(0x10000)
    for dtype in (2, 3, 6, -1):
        assert lib.sun_sample_su2(dtype, p, 8, 1, 0, 0, p, p, None) == -1
    for dtype in (0, 1, 4, 5):
        assert lib.sun_sample_su2(dtype, p, -1, 1, 0, 0, p, p, None) == -1
        assert lib.sun_sample_su2(dtype, None, 8, 1, 0, 0, p, p, None) == -2
        assert lib.sun_sample_su2(dtype, p, 8, 1, 0, 0, p, None, None) == -2
        assert lib.sun_sample_su2(dtype, p, 0, 1, 0, 0, p, p, None) == 0


def test_tile_order_argument_checks(lib):
    """The race-check tile order needs a handle; any seed is accepted (0
    restores the default order)."""
    assert lib.sun_set_tile_order(None, 1) == -1
    L = (4, 4, 4, 4)
    rc, lb, sb = _bytes(lib, 3, L, 0)
    h = ctypes.c_void_p()
    assert lib.sun_lattice_create(3, (ctypes.c_int * 4)(*L), 0, ctypes.c_void_p(0x10000), lb,
                                  ctypes.c_void_p(0x200000), sb, ctypes.byref(h)) == 0
    for seed in (0, 1, 2 ** 64 - 1):
        assert lib.sun_set_tile_order(h, seed) == 0
    lib.sun_lattice_destroy(h)


def test_heatbath_takes_two_tiles_on_large_lattices_only(lib):
    """Default sites per work-item of the heatbath: 2 where the grid keeps
    at least 1024 workgroups (32^4: 2048 tiles of 256), else 1."""
    s = ctypes.c_int()
    for L, want in (((32, 32, 32, 32), 2), ((24, 24, 24, 24), 1), ((12, 12, 12, 12), 1)):
        rc, lb, sb = _bytes(lib, 3, L, 2)
        h = ctypes.c_void_p()
        assert lib.sun_lattice_create(3, (ctypes.c_int * 4)(*L), 2, ctypes.c_void_p(0x10000), lb,
                                      ctypes.c_void_p(0x10000 + ((lb + 255) // 256) * 256), sb, ctypes.byref(h)) == 0
        assert lib.sun_get_sites_per_item(h, 0, ctypes.byref(s)) == 0 and s.value == want, (L, s.value)
        assert lib.sun_get_sites_per_item(h, 1, ctypes.byref(s)) == 0 and s.value == 1
        lib.sun_lattice_destroy(h)
