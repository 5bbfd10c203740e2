"""The tuner's result cache (CPU only): entries accumulate, a torn or missing file reads as
empty, and concurrent writers always leave a valid file behind."""

import json
import multiprocessing as mp
import os

from paper_0802_0748_amd import tune


def _writer(path, i):
    for k in range(20):
        tune._store(path, f"w{i}_{k}", {"block": 48, "shifts_per_wg": 64, "ms_per_iter": 0.1 * i})


def test_cache_round_trip_and_torn_file(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune._load(path) == {}
    tune._store(path, "a", {"block": 16})
    tune._store(path, "b", {"block": 24})
    assert tune._load(path) == {"a": {"block": 16}, "b": {"block": 24}}
    with open(path, "w") as f:
        f.write('{"a": {"blo')
    assert tune._load(path) == {}


def test_concurrent_writers_leave_a_valid_file(tmp_path):
    path = str(tmp_path / "tune.json")
    ctx = mp.get_context("fork")
    procs = [ctx.Process(target=_writer, args=(path, i)) for i in range(4)]
    for p in procs:
        p.start()
    for p in procs:
        p.join(60)
        assert p.exitcode == 0
    with open(path) as f:
        table = json.load(f)
    assert table and all(k.startswith("w") for k in table)
    assert not [f for f in os.listdir(tmp_path) if f.startswith(".tune-")]
