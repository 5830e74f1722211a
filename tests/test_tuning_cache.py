"""Host logic of the tuning cache (no GPU): size classes and the JSON file."""
import json
import os

import pytest

from paper_2308_13175_amd import tuning


def test_size_class_rounds_to_powers_of_two():
    assert tuning.size_class(1_000_000, 200_000, 1) == "q2^20-p2^18-single"
    assert tuning.size_class(32_000_000, 20_000_000, 1) == "q2^25-p2^24-single"
    assert tuning.size_class(43_397_030, 4_339_703, 64) == "q2^25-p2^22-batch"
    assert tuning.size_class(0, 0, 1) == "q2^0-p2^0-single"
    # the class boundary sits at the geometric midpoint between powers of two
    assert tuning.size_class(int(2 ** 20.49), 1, 1) == "q2^20-p2^0-single"
    assert tuning.size_class(int(2 ** 20.51), 1, 1) == "q2^21-p2^0-single"


def test_cache_round_trip_and_atomic_replace(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert tuning.load_cache(path) == {}
    entry = {"nn": [8, 1, 1, 0, 1, 8], "grad": [4096, 16, 2048, 16384]}
    tuning.save_cache(path, {"gfx950|q2^20-p2^18-single": entry})
    assert tuning.load_cache(path) == {"gfx950|q2^20-p2^18-single": entry}
    data = tuning.load_cache(path)
    data["gfx950|q2^25-p2^24-single"] = {"nn": [6, 1, 2, 1, 1, 8], "grad": [2048, 4, 0, 0]}
    tuning.save_cache(path, data)
    assert sorted(tuning.load_cache(path)) == ["gfx950|q2^20-p2^18-single", "gfx950|q2^25-p2^24-single"]
    assert [f for f in os.listdir(tmp_path / "sub") if f.startswith(".tuning-")] == []


def test_cache_rejects_a_foreign_file(tmp_path):
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps([1, 2, 3]))
    with pytest.raises(ValueError):
        tuning.load_cache(str(path))
