"""Race check of the chessboard (paper Sec. 3: a direction's links are
updated on the even and then the odd sites, so that the updates of one
kernel call do not depend on each other): with the oracle's access log on,
no link a phase writes is read by another update of that phase, and every
link of the phase's parity and direction is written exactly once.  A
deliberately broken phase that updates both parities at once must be
caught.  The GPU's parity tests rest on this independence (each phase is
compared link by link with no cascade)."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("nc,L", [(3, (4, 4, 4, 4)), (2, (6, 4, 2, 4)), (3, (4, 4, 4, 1)), (2, (4, 4, 1, 1)),
                                  (4, (2, 2, 4, 2)), (3, (2, 2, 2, 2))])
def test_phase_writes_nothing_another_update_reads(nc, L):
    V = int(np.prod(L))
    U = O.new_field(nc, L, hot=True, seed=5)
    for mu in range(4):
        for kind in (0, 1):
            for par in (0, 1):
                multi, read_by_other, written = O.phase_access_check(U, nc, L, kind, mu, par, beta=6.0, seed=9)
                assert multi == 0 and read_by_other == 0, (mu, kind, par, multi, read_by_other)
                assert written == (V // 2 if L[mu] > 1 else 0)


@pytest.mark.parametrize("nc,L", [(3, (4, 4, 4, 4)), (2, (4, 4, 1, 1))])
def test_broken_schedule_is_caught(nc, L):
    """Updating both parities in one pass: every updated link is a staple
    link of its neighbours' updates."""
    U = O.new_field(nc, L, hot=True, seed=5)
    multi, read_by_other, written = O.phase_access_check(U, nc, L, 1, 0, 2)
    assert written == int(np.prod(L)) and read_by_other == written and multi == 0
