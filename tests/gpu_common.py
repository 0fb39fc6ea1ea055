"""Helpers shared by the GPU parity tests: tolerances, lattice set-up and
the link-by-link comparison against the oracle's phase diagnostics (the
reasoning behind the tolerances is in test_gpu_parity's docstring)."""
import numpy as np
import torch

import oracle as O

TOL = {"f64": 1e-12, "f32": 1e-5, "f64r12": 1e-12, "f32r12": 1e-5, "f64w": 1e-12, "f32w": 1e-5}

# Rounding model of one link update (the test module docstrings give the
# derivation): a link whose update has conditioning c = |A|_F / k_min (the
# staple's norm over the smallest subgroup weight k the update divides by)
# lands within K eps (1 + c) of the oracle, eps the unit roundoff of the
# storage precision.  K_LINK is that K.  The median K measured is about 1
# and the largest grows with the number of links compared: up to 29 (FP64)
# and 34 (FP32 links drifted by 6e-6 across a sweep without
# re-unitarization) over phases of at most 524k links, and 35 (FP64) and 60
# (FP32) over the 12.6M links of a hot-start heatbath phase on 64^3 x 96.
K_LINK = 64.0
# A decision (Creutz / Kennedy-Pendleton switch at alpha = 1.7, accept test
# r^2 <= 1 - x0^2 or r^2 <= 1 - lambda^2) compares quantities of order one
# computed from alpha = 2 beta k / Nc, whose relative error is that of the
# link's update; the factors alpha (at the switch) and 2 x0 bound the
# amplification by 2.  A decision may flip only inside K_FLIP eps (1 + c).
K_FLIP = 2 * K_LINK
# Typical rounding constant (the median K of the comparisons is about 1):
# a decision with margin m flips with probability about P(|error| > m), so
# over decisions whose margin density near 0 is at most 1 the expected
# number of flips is at most sum 2 K_TYP eps (1 + c) over the decisions.
K_TYP = 2.0
# Large Nc: the update is a chain of Nc (Nc - 1) / 2 subgroup steps and the
# oracle's own sensitivity to input rounding (twin_spread) grows along it;
# a link may also differ by SPREAD_FACTOR times that measured sensitivity.
# The largest ratio of GPU deviation to that sensitivity measured with one
# twin was 2.6 in FP64 and 70 in FP32 (SU(32) on 8^4, where the FP32
# arithmetic along the chain -- matrix-core products, hardware logarithms --
# adds rounding at every step that an input perturbation does not model).
SPREAD_FACTOR = {"f64": 10.0, "f32": 100.0}


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


def compare_links(gpu_field, orc_field, dtype, margin=None, cond=None, what="", spread=None,
                  spread_factor=None, decisions=None):
    """Link-by-link comparison of (D, V, Nc, Nc) fields (D directions, 4 or
    a slice of them).  margin and cond are (D, V) arrays from the oracle's
    phase diagnostics (entries < 0: link not updated, margin inf: no
    decision).  With cond, a link must agree to K_LINK eps (1 + c); without,
    to TOL[dtype].  spread, if given, is the oracle's own per-link
    sensitivity (twin_spread); a link may then also differ by up to
    spread_factor times it.  A link outside tolerance is a decision flip if
    its oracle margin lies within K_FLIP eps (1 + c) (FP32 only); the number
    of flips must stay within three times the expected count (K_TYP) or 3.
    decisions: the number of heatbath decisions the phase took, if known."""
    d = np.abs(gpu_field - orc_field).reshape(gpu_field.shape[0], gpu_field.shape[1], -1).max(axis=2)
    eps = EPS[dtype[:3]]
    c = None
    if cond is not None:
        c = np.maximum(np.asarray(cond, dtype=np.float64), 0.0)
        tol_model = K_LINK * eps * (1.0 + c)
    else:
        tol_model = np.full_like(d, TOL[dtype])
    tol = tol_model
    if spread is not None:
        if spread_factor is None:
            spread_factor = SPREAD_FACTOR[dtype[:3]]
        tol = np.maximum(tol, spread_factor * np.asarray(spread))
    bad = d > tol
    ok = ~bad
    rec = {"what": what, "dtype": dtype, "links": int(d.size), "max_dU": float(d.max()),
           "max_dU_over_tol": float((d / tol)[ok].max()) if ok.any() else None,
           "max_dU_over_ctol": float((d / tol_model)[ok].max()) if ok.any() else None}
    upd = None
    if c is not None:
        upd = (np.asarray(cond) > 0)
        u = upd & ok
        if u.any():
            # the rounding model: |dU| ~ K eps (1 + c); K measured here
            kk = d[u] / (eps * (1.0 + c[u]))
            rec["max_K"] = float(kk.max())
            rec["median_K"] = float(np.median(kk))
            rec["max_cond"] = float(c[u].max())
    if spread is not None:
        sp = np.asarray(spread)
        m = (sp > 0) & ok
        if m.any():
            rec["max_dU_over_spread"] = float((d[m] / sp[m]).max())
        # links that only the spread term admits
        only = m & (d > tol_model)
        rec["spread_admitted"] = int(only.sum())
        if only.any():
            rec["max_dU_over_spread_admitted"] = float((d[only] / sp[only]).max())
    mm = None
    expected = 0.0
    if margin is not None and c is not None:
        mm = np.asarray(margin)
        hb = upd & np.isfinite(mm)
        n_upd = int(hb.sum())
        if n_upd:
            nc = gpu_field.shape[-1]
            per_link = decisions / n_upd if decisions else 2 * max(1, nc * (nc - 1) // 2)
            expected = float(per_link * (2 * K_TYP * eps * (1.0 + c[hb])).sum())
            rec["decisions"] = int(decisions) if decisions else int(per_link * n_upd)
            rec["expected_flips"] = expected
            rec["at_risk"] = int((hb & (mm < K_FLIP * eps * (1.0 + c))).sum())
    if cond is not None or spread is not None:
        print(f"{what}: max |dU| {d.max():.2e}, max |dU| / tol {rec['max_dU_over_tol']}")
    if not bad.any():
        rec["flips"] = 0
        record(**rec)
        return 0
    idx = np.argwhere(bad)
    rec["flips"] = int(len(idx))
    if mm is not None:
        rec["flip_margins"] = [float(mm[a][b]) for a, b in idx[:50]]
        rec["flip_conds"] = [float(c[a][b]) for a, b in idx[:50]]
        rec["flip_windows"] = [float(K_FLIP * eps * (1.0 + c[a][b])) for a, b in idx[:50]]
    record(**rec)
    if dtype.startswith("f64") or mm is None:
        mu, s = idx[0]
        raise AssertionError(f"{what}: {len(idx)} links out of tolerance, e.g. (mu={mu}, s={s}) "
                             f"|dU| = {d[mu, s]:.3e}, tol {tol[mu, s]:.2e}")
    m = np.where(mm < 0, np.inf, mm)
    window = K_FLIP * eps * (1.0 + c)
    for mu, s in idx:
        assert m[mu][s] < window[mu][s], (
            f"{what}: link (mu={mu}, s={s}) differs by {d[mu, s]:.3e} with decision margin {m[mu][s]:.3e} "
            f"(window {window[mu][s]:.1e})")
    allowed = max(3.0, 3.0 * expected)
    assert len(idx) <= allowed, f"{what}: {len(idx)} flipped links (expected {expected:.2f}, allowed {allowed:.1f})"
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


def twin_spread(field, nc, L, kind, mu, par, beta, seed, step, rel, twins=3, noise_seed=12345):
    """Per-link (4, V) change of the oracle's phase output when its input is
    perturbed by relative noise `rel` (the storage precision's rounding
    level), the largest over `twins` independent perturbations (one sample
    of a random change has a long tail across links; the largest of three
    is a steadier per-link scale).  At large Nc one link update is a chain
    of Nc (Nc - 1) / 2 subgroup steps, each dividing by its own k, so
    rounding compounds along the chain; this measures that amplification
    directly."""
    a = field.copy()
    O.phase(a, nc, L, kind, mu, par, beta, seed, step)
    rng = np.random.default_rng(noise_seed)
    out = np.zeros((4, field.shape[1]))
    for _ in range(twins):
        b = field * (1.0 + rel * (rng.standard_normal(field.shape) + 1j * rng.standard_normal(field.shape)))
        O.phase(b, nc, L, kind, mu, par, beta, seed, step)
        out = np.maximum(out, np.abs(a - b).reshape(4, field.shape[1], -1).max(axis=2))
    return out
