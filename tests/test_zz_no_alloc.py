"""The plaquette entry point that allocates nothing (sun_plaquette_static):
argument checks on the host, and on the GPU the same bits as sun_plaquette
on a handle over the same field, on calls in a row whose inputs shrink (the
static partials array keeps the previous call's contents)."""
import ctypes

import pytest
import torch

from gpu_common import gpu_lattice


@pytest.fixture(scope="module")
def lib():
    import os
    from paper_1112_4533_amd import build, sun
    if not os.path.exists(sun.LIB_PATH):
        build.build()
    return sun.load()


def test_static_plaquette_argument_checks(lib):
    """Refusals come before any HIP call: bad geometry or storage, null or
    misaligned buffers, and lattices whose partials exceed the array."""
    L4 = ctypes.c_int * 4
    p = ctypes.c_void_p(0x10000)
    assert lib.sun_plaquette_static(3, L4(8, 7, 8, 8), 0, p, p, None) == -1
    assert lib.sun_plaquette_static(1, L4(8, 8, 8, 8), 0, p, p, None) == -1
    assert lib.sun_plaquette_static(2, L4(8, 8, 8, 8), 2, p, p, None) == -4
    assert lib.sun_plaquette_static(3, L4(8, 8, 8, 8), 0, None, p, None) == -2
    assert lib.sun_plaquette_static(3, L4(8, 8, 8, 8), 0, p, None, None) == -2
    assert lib.sun_plaquette_static(3, L4(8, 8, 8, 8), 0, ctypes.c_void_p(0x10010), p, None) == -1
    # register path: 16 bytes per 256 sites; 76^4 = 33.4M sites fits, 78^4 does not
    assert lib.sun_plaquette_static(3, L4(78, 78, 78, 78), 0, p, p, None) == -2
    assert b"static scratch" in lib.sun_last_error()
    # workgroup-per-link path: 16 bytes per site; 20^4 = 160000 sites does not fit
    assert lib.sun_plaquette_static(6, L4(20, 20, 20, 20), 0, p, p, None) == -2


CASES = [  # calls in a row on one GPU, each smaller than the one before
    (3, (16, 16, 16, 16), "f32r12", 6.0),
    (3, (6, 4, 4, 2), "f32", 5.7),
    (2, (4, 4, 2, 2), "f64", 2.3),
    (5, (4, 4, 2, 2), "f64", 17.3),
    (3, (2, 2, 2, 2), "f64r12", 5.0),
]


@pytest.mark.gpu
def test_static_plaquette_is_the_handle_plaquette(gpu):
    sun = gpu
    for rep in range(2):
        for nc, L, dtype, beta in CASES:
            lat = gpu_lattice(sun, nc, L, dtype, hot=True, seed=7 + rep)
            lat.sweep(beta, 1, 1, seed=7 + rep)
            want = lat.plaquette()
            got = sun.plaquette_static(nc, L, dtype, lat.links)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (rep, nc, L, dtype, got, want)
            assert abs(float(got[0])) < 1.0
