"""CPU tests of the tuning rules and the tuner's persistence (no GPU).

The rules are host state of the library: setting, reading back and refusing
out-of-range rules touch no device.  Saved plans load only on the device
and library version they were tuned on.
"""

import json

import pytest

from paper_1912_01884_amd import autotune, fhtp


@pytest.fixture(autouse=True)
def clean_rules():
    fhtp.tune_set([])
    yield
    fhtp.tune_set([])


def test_rules_round_trip_and_clear():
    rules = [autotune.rule(dtype=0, log2n=6, window=0, dc=8, steps=2, stripe=8, fht_grid=1),
             autotune.rule(window=1, fht_grid=0, w_min=10, w_max=99)]
    fhtp.tune_set(rules)
    assert fhtp.tune_get() == rules
    fhtp.tune_set([])
    assert fhtp.tune_get() == []


@pytest.mark.parametrize("bad", [dict(dc=12), dict(steps=4), dict(steps=-1), dict(small=2), dict(small=-1), dict(stripe=65), dict(stripe=-1),
                                 dict(fht_grid=2), dict(window=2), dict(dtype=3), dict(log2n=11),
                                 dict(w_min=5, w_max=4), dict(w_min=-1)])
def test_out_of_range_rules_are_refused_and_change_nothing(bad):
    good = autotune.rule(window=0, dc=16, steps=1)
    fhtp.tune_set([good])
    with pytest.raises(fhtp.FhtpError) as e:
        fhtp.tune_set([autotune.rule(), dict(autotune.rule(), **bad)])
    assert e.value.code == fhtp.ERR_OPTION
    assert fhtp.tune_get() == [good]


def test_rule_count_limit():
    with pytest.raises(fhtp.FhtpError):
        fhtp.tune_set([autotune.rule()] * 1025)
    fhtp.tune_set([autotune.rule()] * 1024)
    assert len(fhtp.tune_get()) == 1024


def test_rules_for_groups_cover_both_window_kinds_then_a_catch_all():
    dp = dict(dc=8, steps=3, stripe=4)
    rules = autotune._rules_for([(0, 6), (1, 7)], dp, {(1, 7): 1})
    assert len(rules) == 5
    assert rules[0] == autotune.rule(dtype=0, log2n=6, window=0, fht_grid=0, **dp)
    assert rules[1] == autotune.rule(dtype=0, log2n=6, window=1, fht_grid=0)
    assert rules[2] == autotune.rule(dtype=1, log2n=7, window=0, fht_grid=1, **dp)
    assert rules[4] == autotune.rule(window=0, **dp)
    fhtp.tune_set(rules)  # every generated rule is valid


def test_saved_plan_loads_only_on_the_same_device_and_library(tmp_path, monkeypatch):
    key = {"device": "MI355X", "arch": "gfx950", "library": fhtp.version()}
    monkeypatch.setattr(autotune, "device_key", lambda: dict(key))
    res = autotune.TuneResult(rules=autotune._rules_for([(0, 5)], dict(dc=16, steps=1, stripe=0),
                                                        {(0, 5): 1}),
                              default_ms=2.0, tuned_ms=1.5, dp_choice=dict(dc=16, steps=1, stripe=0),
                              fht_choice={"dtype0 log2n5": 1})
    path = str(tmp_path / "plan.json")
    autotune.save(res, path, workload="test")
    doc = json.load(open(path))
    assert doc["key"] == key and doc["workload"] == "test"
    assert autotune.load(path) == res.rules
    assert fhtp.tune_get() == res.rules
    fhtp.tune_set([])
    monkeypatch.setattr(autotune, "device_key", lambda: dict(key, library="other"))
    assert autotune.load(path) is None
    assert fhtp.tune_get() == []
    monkeypatch.setenv("FHTP_PLAN", path)
    monkeypatch.setattr(autotune, "device_key", lambda: dict(key))
    assert autotune.load_from_env() == res.rules


def test_tuner_logic_with_a_simulated_workload(monkeypatch):
    """tune() on a stand-in workload whose time depends on the installed rules:
    it must pick the fastest DP candidate, then the faster FHT grid per group,
    restore the previous rules, and refuse a candidate that changes a result."""
    costs = {}

    class FakeWorkload:
        def __init__(self, images, ks, bends=None, gammas=None, stream=None):
            self.groups = [(0, 5), (1, 7)]
            self.bad = False

        def time_ms(self, reps):
            rules = fhtp.tune_get()
            if not rules:
                return 10.0
            dp = rules[0]
            t = 5.0 + (0 if (dp["steps"], dp["stripe"]) == (2, 8) else 1.0)
            t -= 0.5 * sum(r["fht_grid"] for r in rules if r["window"] == 0 and r["log2n"] == 7)
            costs[len(costs)] = t
            return t

        def results(self):
            return [(1, [0, 1])] if not self.bad else [(2, [0, 1])]

    monkeypatch.setattr(autotune, "Workload", FakeWorkload)
    before = [autotune.rule(window=1, fht_grid=1)]
    fhtp.tune_set(before)
    res = autotune.tune([None], [1], install_result=False)
    assert fhtp.tune_get() == before
    assert res.dp_choice == dict(dc=8, steps=2, stripe=8)
    assert res.fht_choice == {"dtype0 log2n5": 0, "dtype1 log2n7": 1}
    assert res.default_ms == 10.0 and res.tuned_ms == 4.5
    assert res.rules == autotune._rules_for([(0, 5), (1, 7)], res.dp_choice, {(0, 5): 0, (1, 7): 1})
    res = autotune.tune([None], [1])
    assert fhtp.tune_get() == res.rules

    class Breaks(FakeWorkload):
        def time_ms(self, reps):
            self.bad = bool(fhtp.tune_get())
            return 1.0

    monkeypatch.setattr(autotune, "Workload", Breaks)
    fhtp.tune_set(before)
    with pytest.raises(RuntimeError, match="changed a result"):
        autotune.tune([None], [1])
    assert fhtp.tune_get() == before
