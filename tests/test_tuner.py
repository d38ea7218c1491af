"""CPU checks of the auto-tuner with a fake measurement (no GPU).

The tuner implements the paper's Eq. 1 (x* = argmin over the configuration
space of the measured run time), the "median configuration" of its Table 2
protocol (here: the valid configurations sorted by median time, the one at
index floor((N - 1) / 2)), the skipping of configurations the kernels cannot
run, and a resumable database of measurements.
"""
import json
import os

import pytest

from paper_2608_21227_amd import Config, Unsupported, tuner


def _fake_space(k=11):
    return [Config(tile=16 * (1 + i % 4), threads=64 << (i % 5), inner_block=1, sweep_width=1 + i % 8) for i in range(k)]


def _times(cfgs):
    # distinct, known run times (ms) per configuration; index 3 and 7 are invalid
    return {tuner.key_of(c): 10.0 + ((i * 7) % 11) for i, c in enumerate(cfgs)}


def test_argmin_lower_median_and_invalid_skip(tmp_path):
    cfgs = _fake_space()
    times = _times(cfgs)
    invalid = {tuner.key_of(cfgs[3]), tuner.key_of(cfgs[7])}
    calls = []

    def measure(c):
        calls.append(tuner.key_of(c))
        return [times[tuner.key_of(c)]] * 5

    recs = tuner.tune(512, "float32", cfgs, str(tmp_path / "db.jsonl"), measure,
                      is_valid=lambda c: tuner.key_of(c) not in invalid)
    assert not (invalid & set(calls)), "an invalid configuration was measured"
    summ = tuner.summarize(recs)
    valid = sorted((times[k], k) for k in times if k not in invalid)
    assert summ["valid"] == len(valid) == 9 and summ["invalid"] == 2
    # Eq. 1: the argmin
    assert tuner.key_of(Config(**summ["best"])) == valid[0][1]
    assert summ["best_ms"] == valid[0][0]
    # lower median: index (N - 1) // 2 of the sorted valid list (N = 9 -> index 4)
    assert tuner.key_of(Config(**summ["median"])) == valid[(len(valid) - 1) // 2][1]
    assert summ["ratio_median_over_best"] == pytest.approx(valid[4][0] / valid[0][0])


def test_even_count_takes_the_lower_median(tmp_path):
    cfgs = _fake_space(6)
    t = {tuner.key_of(c): float(v) for c, v in zip(cfgs, [5, 1, 4, 2, 6, 3])}
    recs = tuner.tune(64, "float64", cfgs, str(tmp_path / "db.jsonl"), lambda c: [t[tuner.key_of(c)]] * 3,
                      is_valid=lambda c: True)
    summ = tuner.summarize(recs)
    assert summ["median_ms"] == 3.0  # sorted 1..6, index (6 - 1) // 2 = 2
    assert summ["best_ms"] == 1.0


def test_unsupported_raised_by_the_measurement_is_recorded_invalid(tmp_path):
    cfgs = _fake_space(4)

    def measure(c):
        if c == cfgs[1]:
            raise Unsupported(-2, "exceeds LDS")
        return [1.0, 1.0]

    recs = tuner.tune(128, "float32", cfgs, str(tmp_path / "db.jsonl"), measure, is_valid=lambda c: True)
    by_key = {r["key"]: r for r in recs}
    assert by_key[tuner.key_of(cfgs[1])]["status"] == "invalid"
    assert tuner.summarize(recs)["valid"] == 3


def test_resume_skips_measured_configs_and_drops_a_torn_line(tmp_path):
    db = str(tmp_path / "db.jsonl")
    cfgs = _fake_space(5)
    first = []
    tuner.tune(256, "float32", cfgs[:3], db, lambda c: first.append(c) or [2.0, 2.0], is_valid=lambda c: True)
    assert len(first) == 3
    with open(db, "a") as f:
        f.write('{"n": 256, "dtype": "float32", "key": "torn')  # an interrupted write
    second = []
    recs = tuner.tune(256, "float32", cfgs, db, lambda c: second.append(c) or [3.0, 3.0], is_valid=lambda c: True)
    assert second == cfgs[3:], "resume must measure exactly the configurations not yet in the database"
    assert len(recs) == 5
    # other cells in the same file are not mixed in
    tuner.tune(512, "float64", cfgs[:1], db, lambda c: [9.0], is_valid=lambda c: True)
    assert len([r for r in tuner.read_db(db) if r.get("n") == 256]) == 5


def test_erratic_measurements_are_repeated_and_flagged(tmp_path):
    cfgs = _fake_space(2)
    seq = {tuner.key_of(cfgs[0]): [[1.0, 9.0], [1.0, 1.1]], tuner.key_of(cfgs[1]): [[2.0, 2.1]]}

    def measure(c):
        return seq[tuner.key_of(c)].pop(0)

    recs = tuner.tune(512, "float32", cfgs, str(tmp_path / "db.jsonl"), measure, is_valid=lambda c: True)
    by_key = {r["key"]: r for r in recs}
    r0 = by_key[tuner.key_of(cfgs[0])]
    assert r0["remeasured"] is True and r0["times_ms"] == [1.0, 1.1]  # spread 9x: measured again, last kept
    assert by_key[tuner.key_of(cfgs[1])]["remeasured"] is False


def test_summarize_of_no_valid_config():
    recs = [{"status": "invalid"}, {"status": "invalid"}]
    assert tuner.summarize(recs) == {"valid": 0, "invalid": 2}


def test_space_is_the_stated_cross_product():
    sp = tuner.space()
    assert len(sp) == 4 * 5 * 4 * 8 == 640
    assert len({tuner.key_of(c) for c in sp}) == 640
    assert tuner.PLAIN == Config(tile=32, threads=256, inner_block=1, sweep_width=1)


def test_table_lookup_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    table = {"4096_float32": {"best": Config(16, 1024, 1, 4).as_dict(), "median": Config(16, 64, 4, 8).as_dict(),
                              "best_ms": 1.0, "median_ms": 2.0}}
    tuner.save_table(table, path)
    t2 = tuner.load_table(path)
    assert tuner.lookup(t2, 4096, "float32") == Config(16, 1024, 1, 4)
    assert tuner.lookup_median(t2, 4096, "float32") == Config(16, 64, 4, 8)
    assert tuner.lookup(t2, 2048, "float32") is None
    with open(path) as f:
        json.load(f)


def test_library_default_is_the_tuned_argmin_of_each_measured_cell():
    """svd_values without a configuration runs the tuned table's best for a measured
    cell (the table is compiled into the library when it is built)."""
    import paper_2608_21227_amd as svdv
    table = tuner.load_table()
    if not table:
        pytest.skip("no tuned table")
    for key in table:
        n, dt = key.split("_")
        assert svdv.default_config(int(n), int(n), dt) == tuner.lookup(table, int(n), dt), key
