"""Seeded synthetic workloads (lattice sizes, couplings, seeds, batch mixes).

This module holds no arithmetic of the method: it only names the runs the
tests and the benchmark use, so that the HIP path and the CPU oracle are fed
the same inputs.  The paper generates its configurations in-process from
(Nc, lattice, beta, seed), so there is no dataset: a run is fully given by
these parameters.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Run:
    name: str
    nc: int
    L: tuple
    beta: float
    hot: bool
    dtype: str          # link storage: "f32" or "f64"
    n_hb: int
    n_or: int
    sweeps: int
    seed: int = 1234
    reunit: bool = True

    @property
    def volume(self):
        v = 1
        for x in self.L:
            v *= x
        return v


# SU(2) 8^4, beta 2.3, cold start, FP64 links, 1 HB + 3 OR, 20 sweeps.
SU2_8_COLD = Run("su2_8^4_cold_f64", 2, (8, 8, 8, 8), 2.3, False, "f64", 1, 3, 20)
# SU(3) 16^4, beta 6.0, hot start, FP32 links, 1 HB + 4 OR, 200 sweeps.
SU3_16_HOT = Run("su3_16^4_hot_f32", 3, (16, 16, 16, 16), 6.0, True, "f32", 1, 4, 200)
# SU(3) 32^4, beta 6.2, hot start, 1 HB + 4 OR, 100 sweeps, FP32 and FP64.
SU3_32_F32 = Run("su3_32^4_hot_f32", 3, (32, 32, 32, 32), 6.2, True, "f32", 1, 4, 100)
SU3_32_F64 = Run("su3_32^4_hot_f64", 3, (32, 32, 32, 32), 6.2, True, "f64", 1, 4, 100)
# The same with SU(3) links stored as two rows (12 reals, FP32).
SU3_32_F32_TWO_ROW = Run("su3_32^4_hot_f32_two_row", 3, (32, 32, 32, 32), 6.2, True, "f32r12", 1, 4, 100)


def large_nc_runs(dtype="f32"):
    """SU(4), SU(6), SU(8) on 12^4, hot start, 1 HB + 1 OR (+ re-unitarization),
    100 sweeps, with beta = 11.1 (Nc/4)^2 (the same beta / Nc^2 as SU(4) at 11.1)."""
    return [Run(f"su{n}_12^4_hot_{dtype}", n, (12, 12, 12, 12), round(11.1 * (n / 4.0) ** 2, 4), True, dtype, 1, 1,
                100) for n in (4, 6, 8)]


@dataclass(frozen=True)
class BatchSpec:
    chains: tuple = field(default_factory=tuple)


def batch_spec(n_chains=64, seed=1234):
    """64 independent chains: the first half SU(2), the second half SU(3);
    extents uniform over {8, 12, 16, 20} (hypercubic), beta uniform in
    [2.2, 2.6] (SU(2)) or [5.6, 6.4] (SU(3)); chain i uses seed 1234 + i.
    FP32 links, 1 HB + 4 OR, 100 sweeps each."""
    rng = np.random.default_rng(seed)
    runs = []
    for i in range(n_chains):
        nc = 2 if i < n_chains // 2 else 3
        ext = int(rng.choice([8, 12, 16, 20]))
        lo, hi = (2.2, 2.6) if nc == 2 else (5.6, 6.4)
        beta = float(rng.uniform(lo, hi))
        runs.append(Run(f"chain{i}", nc, (ext,) * 4, beta, True, "f32", 1, 4, 100, seed=1234 + i))
    return runs
