"""Helpers shared by the GPU parity tests: tolerances, lattice set-up and
the link-by-link comparison against the oracle's phase diagnostics (the
reasoning behind the tolerances is in test_gpu_parity's docstring)."""
import numpy as np
import torch

import oracle as O

TOL = {"f64": 1e-12, "f32": 1e-5, "f64r12": 1e-12, "f32r12": 1e-5, "f64w": 1e-12, "f32w": 1e-5}
FLIP_MARGIN = 1e-4


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_lattice(sun, nc, L, dtype, field=None, hot=True, seed=1234):
    lat = sun.Lattice(nc, L, dtype)
    if field is None:
        lat.init(hot=hot, seed=seed)
    else:
        lat.import_(torch.from_numpy(field))
    return lat


def rounded(field, dtype):
    """The field as the GPU stores it (FP32 rounding of each real)."""
    if dtype.startswith("f64"):
        return field.copy()
    r = field.real.astype(np.float32).astype(np.float64)
    i = field.imag.astype(np.float32).astype(np.float64)
    return r + 1j * i


EPS = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}   # unit roundoff of the storage precision
EVIDENCE = []            # one record per comparison (written out by conftest)


def record(**kw):
    """Keeps a parity measurement; conftest prints them all at the end of
    the session and writes them to $SUN_PARITY_EVIDENCE if set."""
    import os
    kw.setdefault("test", os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0])
    EVIDENCE.append(kw)


def compare_links(gpu_field, orc_field, dtype, margin=None, cond=None, what="", spread=None, spread_factor=100.0,
                  decisions=None):
    """Link-by-link comparison; margin and cond are (4, V) arrays from the
    oracle's phase diagnostics (entries < 0: link not updated).  decisions,
    if given, is the number of heatbath accept/reject decisions the phase
    took (updated links times subgroups).  spread, if
    given, is the oracle's own per-link sensitivity (twin_spread); a link
    may then also differ by up to spread_factor times it."""
    d = np.abs(gpu_field - orc_field).reshape(4, gpu_field.shape[1], -1).max(axis=2)
    base = np.ones_like(d)
    c = None
    if cond is not None:
        c = np.asarray(cond, dtype=np.float64)
        base = np.maximum(1.0, np.where(c > 0, c, 0.0) / (2.0 if dtype.startswith("f32") else 4.0))
    tol = TOL[dtype] * base
    if spread is not None:
        tol = np.maximum(tol, spread_factor * spread)
    bad = d > tol
    ok = ~bad
    rec = {"what": what, "dtype": dtype, "links": int(d.size), "max_dU": float(d.max()),
           "max_dU_over_tol": float((d / tol)[ok].max()) if ok.any() else None,
           "max_dU_over_ctol": float((d / (TOL[dtype] * base))[ok].max()) if ok.any() else None}
    if c is not None:
        upd = (c > 0) & ok
        if upd.any():
            eps = EPS[dtype[:3]]
            # the rounding model: |dU| ~ K eps (1 + c); K measured here
            rec["max_K"] = float((d[upd] / (eps * (1.0 + c[upd]))).max())
            rec["max_cond"] = float(c[upd].max())
    if spread is not None:
        sp = np.asarray(spread)
        m = (sp > 0) & ok
        if m.any():
            rec["max_dU_over_spread"] = float((d[m] / sp[m]).max())
        # links that only the spread term admits
        only = m & (d > TOL[dtype] * base)
        rec["spread_admitted"] = int(only.sum())
        if only.any():
            rec["max_dU_over_spread_admitted"] = float((d[only] / sp[only]).max())
    if decisions is not None:
        rec["decisions"] = int(decisions)
    if cond is not None or spread is not None:
        print(f"{what}: max |dU| {d.max():.2e}, max |dU| / tol {rec['max_dU_over_tol']}")
    if not bad.any():
        rec["flips"] = 0
        record(**rec)
        return 0
    idx = np.argwhere(bad)
    rec["flips"] = int(len(idx))
    if margin is not None:
        mm = np.asarray(margin)
        rec["flip_margins"] = [float(mm[a][b]) for a, b in idx[:50]]
        if c is not None:
            rec["flip_conds"] = [float(c[a][b]) for a, b in idx[:50]]
    record(**rec)
    if dtype.startswith("f64") or margin is None:
        mu, s = idx[0]
        raise AssertionError(f"{what}: {len(idx)} links out of tolerance, e.g. (mu={mu}, s={s}) "
                             f"|dU| = {d[mu, s]:.3e}, tol {tol[mu, s]:.2e}")
    m = np.where(np.asarray(margin) < 0, np.inf, margin)
    # the window of flippable decisions widens by the measured amplification
    window = FLIP_MARGIN * (np.maximum(1.0, spread_factor * spread / TOL[dtype]) if spread is not None
                            else np.ones_like(d))
    for mu, s in idx:
        assert m[mu][s] < window[mu][s], (
            f"{what}: link (mu={mu}, s={s}) differs by {d[mu, s]:.3e} with decision margin {m[mu][s]:.3e} "
            f"(window {window[mu][s]:.1e})")
    # a heatbath update takes one accept/reject decision per SU(2) subgroup
    # (paper Sec. 2), so where a caller gives the number of decisions the
    # budget also grows with it (1e-5 per decision)
    allowed = max(3, 1e-4 * d.size, 1e-5 * decisions if decisions else 0)
    assert len(idx) <= allowed, f"{what}: {len(idx)} flipped links (allowed {allowed:.0f})"
    return len(idx)


def oracle_phase_diag(field, nc, L, kind, mu, par, beta, seed, step):
    """Runs the oracle phase in place; returns (4, V) margin and conditioning maps."""
    margin, _, cond = O.phase(field, nc, L, kind, mu, par, beta, seed, step, want_margin=True)
    mfull = np.full((4, field.shape[1]), -1.0)
    cfull = np.full((4, field.shape[1]), -1.0)
    mfull[mu] = margin
    cfull[mu] = cond
    return mfull, cfull


def thermal_field(nc, L, beta, sweeps=2, seed=77):
    U = O.new_field(nc, L, hot=True, seed=seed)
    for k in range(sweeps):
        O.sweep(U, nc, L, beta, 1, 1, seed, k)
    return U


BETA = {2: 2.3, 3: 6.0, 4: 11.1, 5: 17.3, 6: 24.98, 7: 34.0, 8: 44.4}


def beta_for(nc):
    """Couplings of the tests: the table above for Nc <= 8, else the same
    beta / Nc^2 as SU(4) at 11.1."""
    return BETA[nc] if nc in BETA else round(11.1 * (nc / 4.0) ** 2, 4)


def twin_spread(field, nc, L, kind, mu, par, beta, seed, step, rel, noise_seed=12345):
    """Per-link (4, V) change of the oracle's phase output when its input is
    perturbed by relative noise `rel` (the storage precision's rounding
    level).  At large Nc one link update is a chain of Nc (Nc - 1) / 2
    subgroup steps, each dividing by its own k, so rounding compounds along
    the chain; this measures that amplification directly."""
    a = field.copy()
    O.phase(a, nc, L, kind, mu, par, beta, seed, step)
    rng = np.random.default_rng(noise_seed)
    b = field * (1.0 + rel * (rng.standard_normal(field.shape) + 1j * rng.standard_normal(field.shape)))
    O.phase(b, nc, L, kind, mu, par, beta, seed, step)
    return np.abs(a - b).reshape(4, field.shape[1], -1).max(axis=2)
