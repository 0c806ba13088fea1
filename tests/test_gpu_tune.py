"""Autotuner: times the candidate tilings, keeps the fastest, writes a JSON
cache line that a second plan reuses, and the tuned plan still meets parity."""
import json

import pytest

from paper_2408_03273_amd import workloads as wl
from tests import _harness as H

pytestmark = pytest.mark.gpu


def test_autotune_cache_and_parity(tmp_path):
    s = wl.random_system(51, 9, 4000, box=(21.0, 22.0, 23.0), alpha=0.33, rcut=9.0, kmax=(8, 9, 10))
    cache = str(tmp_path / "tune.jsonl")
    plan = H.make_plan(s)
    before = plan.describe()
    plan.autotune(s.nm, cache)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    assert {"key", "fwd", "ct", "xcd", "fwd_target", "bwd", "kc", "times_us"} <= set(entry)
    print("[tune]", before, "->", plan.describe(), entry["times_us"], flush=True)
    ref = H.oracle_outputs(s)
    got = H.gpu_outputs(s, plan=plan)
    errs = H.compare(got, ref, H.FWD_KEYS + H.BWD_KEYS)
    assert max(errs.values()) <= 1e-10, errs
    # a second plan finds the entry and does not append another one
    plan2 = H.make_plan(s)
    plan2.autotune(s.nm, cache)
    assert len(open(cache).read().strip().splitlines()) == 1
    assert plan2.describe() == plan.describe()
