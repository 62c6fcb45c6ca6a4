"""Autotuner selection logic and cache round trip (CPU; timings injected)."""

import json
import math

import pytest

from paper_2201_08500_amd import autotune


def fake_timer(prec, Nx, sched, nz, reps):
    base = {"stockham": 3.0, "fourstep": 2.0, "split": 1.5}[sched]
    if Nx not in (1024, 2048) and sched == "split":
        base = 2.0            # split falls back to four-step elsewhere
    return base * Nx / 1024 * (2 if prec == "fp64" else 1)


def test_select_prefers_fastest_and_simpler_on_ties():
    assert autotune.select({"stockham": 3, "fourstep": 2, "split": 1.5}) == "split"
    assert autotune.select({"stockham": 2, "fourstep": 1.995, "split": 2.5}) == "stockham"
    with pytest.raises(ValueError):
        autotune.select({})


def test_tune_writes_cache_and_plan_reads_it(tmp_path, monkeypatch):
    out = tmp_path / "sched.json"
    res = autotune.tune(["fp32s", "fp64"], [512, 2048], nz=10, reps=1,
                        out=str(out), timer=fake_timer, device_name="test")
    data = json.loads(out.read_text())
    assert data == res
    assert data["choices"]["fp32s"]["2048"] == "split"
    assert data["choices"]["fp64"]["512"] == "fourstep"
    monkeypatch.setenv(autotune.ENV, str(out))
    assert autotune.cached_choice("fp32s", 2048) == "split"
    assert autotune.cached_choice("fp32", 2048) is None
    # Plan applies the cached schedule when none is given
    from paper_2201_08500_amd import Plan
    p = Plan(2048, 0.5e-6, 0.5e-6, 10, -1.5e-5, 3.8e-6, 3.8e-6, math.pi / 4,
             1.24e-10, 2, precision="fp64")
    assert p.schedule == 2     # cached choice for fp64 at Nx = 2048: split
    p = Plan(512, 0.5e-6, 0.5e-6, 10, -1.5e-5, 3.8e-6, 3.8e-6, math.pi / 4,
             1.24e-10, 2, precision="fp64")
    assert p.schedule == 1


def test_bad_cache_entry_is_rejected(tmp_path, monkeypatch):
    out = tmp_path / "bad.json"
    out.write_text(json.dumps({"choices": {"fp32": {"1024": "bogus"}}}))
    monkeypatch.setenv(autotune.ENV, str(out))
    with pytest.raises(ValueError):
        autotune.cached_choice("fp32", 1024)


def test_default_cache_file_applies_without_the_variable(tmp_path, monkeypatch):
    """With BPM_SCHEDULE_CACHE unset, a cache in the default location is the
    plans' default; set to an empty string, the variable disables it."""
    monkeypatch.delenv(autotune.ENV, raising=False)
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    assert autotune.cache_path() is None
    path = autotune.default_cache_path()
    assert path == str(tmp_path / "bpm_mi355x" / "schedules.json")
    (tmp_path / "bpm_mi355x").mkdir()
    autotune.tune(["fp64"], [2048], nz=10, reps=1, out=path, timer=fake_timer,
                  device_name="test")
    assert autotune.cached_choice("fp64", 2048) == "split"
    from paper_2201_08500_amd import Plan
    p = Plan(2048, 0.5e-6, 0.5e-6, 10, -1.5e-5, 3.8e-6, 3.8e-6, math.pi / 4,
             1.24e-10, 2, precision="fp64")
    assert p.schedule == 2
    monkeypatch.setenv(autotune.ENV, "")
    assert autotune.cached_choice("fp64", 2048) is None
