"""Host logic of the launch-shape autotuner, with the timer and the lattice
replaced by stand-ins: it picks the fastest shape of each update kind, leaves
the chosen sites-per-item applied, and a cached choice is applied without
timing anything.  No GPU is touched."""
import json

from paper_1112_4533_amd import autotune, sun


class FakeLattice:
    """Records what the tuner applies."""
    nc, L, dtype = 3, (32, 32, 32, 32), 2

    def __init__(self):
        self.shapes, self.spt = {}, {}

    def set_launch(self, block, xcd, waves, tblock, kind=-1):
        self.shapes[kind] = (block, xcd, waves, tblock)

    def set_sites_per_item(self, spt, kind=-1):
        self.spt[kind] = spt


def fake_timer(table, state):
    """A stand-in for the event timer: the time of a step is looked up from
    the current (kind, setting)."""
    def _time(fn, reps):
        fn()
        return table[state["kind"], state["setting"]]
    return _time


def test_search_takes_the_fastest_shape_per_kind(monkeypatch):
    state = {}
    table = {(0, (256, 1, 16, 4)): 1.0, (0, (128, 0, 0, 0)): 2.0,
             (1, (256, 1, 16, 4)): 3.0, (1, (128, 0, 0, 0)): 2.5}
    monkeypatch.setattr(autotune, "_time", fake_timer(table, state))

    def set_shape(shape, kind):
        state["kind"], state["setting"] = kind, shape

    steps = []
    best, times = autotune._search([(256, 1, 16, 4), (128, 0, 0, 0)], set_shape,
                                   lambda: steps.append("hb"), lambda: steps.append("or"), reps=1)
    assert best == {sun.HEATBATH: (256, 1, 16, 4), sun.OVERRELAX: (128, 0, 0, 0)}
    assert times["heatbath"] == {"256/1/16/4": 1.0, "128/0/0/0": 2.0}
    assert times["overrelax"] == {"256/1/16/4": 3.0, "128/0/0/0": 2.5}
    # each kind is timed only with its own step
    assert steps == ["hb", "hb", "or", "or"]


def test_sites_per_item_search_leaves_the_best_applied(monkeypatch):
    state = {}
    table = {(0, 1): 2.0, (0, 2): 1.5, (0, 4): 1.7, (1, 1): 1.0, (1, 2): 1.1, (1, 4): 1.2}
    monkeypatch.setattr(autotune, "_time", fake_timer(table, state))
    applied = {}

    def set_spt(v, kind):
        state["kind"], state["setting"] = kind, v
        applied[kind] = v

    best, times = autotune._search_spt(set_spt, lambda: None, lambda: None, reps=1)
    assert best == {sun.HEATBATH: 2, sun.OVERRELAX: 1}
    assert applied == best
    assert times["heatbath_sites_per_item"] == {"1": 2.0, "2": 1.5, "4": 1.7}


def test_cached_choice_is_applied_without_timing(monkeypatch, tmp_path):
    lat = FakeLattice()
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    key = autotune.lattice_key(lat)
    assert key == f"gfx950:su3:32x32x32x32:{sun.DTYPE_NAMES[2]}"
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({key: {"shape": {"0": [256, 1, 16, 4], "1": [256, 1, 12, 4]},
                                       "sites_per_item": {"0": 1, "1": 2}, "ms": {"x": 1}}}))
    monkeypatch.setattr(autotune, "CACHE", str(cache))

    def no_timing(fn, reps):
        raise AssertionError("a cached choice must not be timed")
    monkeypatch.setattr(autotune, "_time", no_timing)
    best, ms = autotune.tune_lattice(lat)
    assert best == {0: (256, 1, 16, 4), 1: (256, 1, 12, 4)}
    assert lat.shapes == best and lat.spt == {0: 1, 1: 2}
    assert ms == {"x": 1}


def test_damaged_cache_reads_as_empty(monkeypatch, tmp_path):
    cache = tmp_path / "tune.json"
    cache.write_text("{not json")
    monkeypatch.setattr(autotune, "CACHE", str(cache))
    assert autotune._load_cache() == {}
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "absent.json"))
    assert autotune._load_cache() == {}


def test_cache_save_is_atomic_and_readable(monkeypatch, tmp_path):
    cache = tmp_path / "sub" / "tune.json"
    monkeypatch.setattr(autotune, "CACHE", str(cache))
    autotune._save_cache({"k": {"shape": {"0": [64, 1, 0, 0]}}})
    assert autotune._load_cache() == {"k": {"shape": {"0": [64, 1, 0, 0]}}}
    assert not (tmp_path / "sub" / "tune.json.tmp").exists()

