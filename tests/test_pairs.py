"""The order in which the large-Nc update runs its SU(2) subgroup steps, two
at a time (sun_pairs.hpp), checked on the host: the table is compiled with
the host compiler from the same header the kernels use and printed.

Sec. 4's update left-multiplies the link by one SU(2) element per index pair
(i, j), i < j, in the fixed order; step (i, j) reads the 2x2 block (i, j) of
W = U A and rewrites rows i and j of U and W.  A slot may therefore hold
two steps only if they share no index, and the steps touching any one
index must keep their fixed order; then the link is the same bit for bit,
which the last test checks by running both orders on random data."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1112_4533_amd", "csrc", "sun_pairs.hpp")
NONE = 0xFF

PROGRAM = r"""
#include "sun_pairs.hpp"
#include <cstdio>
constexpr sun::pairs::Table kT = sun::pairs::make_table();
int main() {
    for (int n = 2; n <= sun::pairs::kMaxN; ++n) {
        printf("%d", n);
        for (int s = kT.first[n]; s < kT.first[n + 1]; ++s) printf(" %u", kT.slot[s]);
        printf("\n");
    }
    for (int n = 2; n <= sun::pairs::kMaxN; ++n)
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) printf("%u ", sun::pairs::step_index(n, i, j));
    printf("\n");
}
"""


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("pairs")
    src, exe = d / "pairs.cpp", d / "pairs"
    src.write_text(PROGRAM)
    subprocess.run([gxx, "-std=c++17", "-O1", f"-I{os.path.dirname(HEADER)}", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.strip().split("\n")
    slots = {}
    for ln in lines[:-1]:
        v = [int(x) for x in ln.split()]
        slots[v[0]] = [(e & 0xFF, (e >> 8) & 0xFF, (e >> 16) & 0xFF, e >> 24) for e in v[1:]]
    return slots, [int(x) for x in lines[-1].split()]


def fixed_order(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def steps_of(slot):
    iA, jA, iB, jB = slot
    out = [(iA, jA)]
    if iB != NONE:
        assert jB != NONE
        out.append((iB, jB))
    else:
        assert jB == NONE
    return out


def test_every_step_once_and_slots_of_disjoint_pairs(table):
    slots, _ = table
    for n in range(2, 33):
        seen = []
        for sl in slots[n]:
            st = steps_of(sl)
            if len(st) == 2:
                assert not set(st[0]) & set(st[1]), (n, st)
            seen += st
        assert sorted(seen) == fixed_order(n), n


def test_the_steps_on_each_index_keep_the_fixed_order(table):
    slots, _ = table
    for n in range(2, 33):
        order = {s: k for k, s in enumerate(fixed_order(n))}
        pos = {}
        for t, sl in enumerate(slots[n]):
            for s in steps_of(sl):
                pos[s] = t
            if sl[2] != NONE:  # the first of a slot precedes the second
                assert order[sl[:2]] < order[sl[2:]], (n, sl)
        for k in range(n):
            touching = [s for s in fixed_order(n) if k in s]
            ts = [pos[s] for s in touching]
            assert ts == sorted(ts) and len(set(ts)) == len(ts), (n, k)


def test_slot_counts(table):
    """Greedy two at a time: ceil(S / 2) plus a short start-up (the first
    steps all touch index 0); SU(32) runs its 496 steps in 257 slots."""
    slots, _ = table
    for n in range(2, 33):
        S = n * (n - 1) // 2
        assert (S + 1) // 2 <= len(slots[n]) <= (S + 1) // 2 + n, n
    assert len(slots[32]) == 257 and len(slots[8]) == 17 and len(slots[3]) == 3


def test_step_index_is_the_position_in_the_fixed_order(table):
    _, idx = table
    expect = []
    for n in range(2, 33):
        expect += list(range(n * (n - 1) // 2))
    assert idx == expect


def _left_mul_rows(M, i, j, a):
    r_i, r_j = M[i].copy(), M[j].copy()
    M[i] = a[0, 0] * r_i + a[0, 1] * r_j
    M[j] = a[1, 0] * r_i + a[1, 1] * r_j


@pytest.mark.parametrize("n", [4, 5, 8, 13, 32])
def test_slot_order_gives_the_fixed_order_link_bit_for_bit(table, n):
    """Each step's 2x2 factor is a function of the block (i, j) of W it reads
    (here the normalised projection plus a per-step constant), as in the
    update; the slot order must reproduce the fixed order exactly."""
    slots, _ = table
    rng = np.random.default_rng(n)
    U0 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    cst = {s: rng.standard_normal(4) for s in fixed_order(n)}

    def step(U, W, i, j):
        # an SU(2) element from the block and a per-step constant (unitary,
        # so that nothing grows over hundreds of steps)
        c = cst[(i, j)]
        q = np.array([W[i, i].real + W[j, j].real, W[i, j].imag + W[j, i].imag,
                      W[i, j].real - W[j, i].real, W[i, i].imag - W[j, j].imag]) + c
        q = q / np.sqrt(q @ q)
        a = np.array([[q[0] + 1j * q[3], q[2] + 1j * q[1]], [-q[2] + 1j * q[1], q[0] - 1j * q[3]]])
        _left_mul_rows(U, i, j, a)
        _left_mul_rows(W, i, j, a)

    U1, W1 = U0.copy(), U0 @ A
    for i, j in fixed_order(n):
        step(U1, W1, i, j)
    U2, W2 = U0.copy(), U0 @ A
    for sl in slots[n]:
        for i, j in steps_of(sl):
            step(U2, W2, i, j)
    assert np.isfinite(U1).all() and not np.allclose(U1, U0)
    assert np.array_equal(U1, U2) and np.array_equal(W1, W2)
