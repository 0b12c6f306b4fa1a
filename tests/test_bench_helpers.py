"""bench.py's host-side helpers (CPU): the oracle baseline times one core and
all cores on the same counts, and counter summaries are used only for the
library build and workload they were taken on."""
import json
import os

import numpy as np
import pytest

import bench
import oracle
import xmgen


def test_cpu_baseline_counts_the_sample_once_per_run_on_one_and_all_cores():
    g = xmgen.rmat(9, seed=1)
    work = [(xmgen.named("ffl"), np.arange(0, 100, dtype=np.uint32), 0),
            (xmgen.named("c4"), np.arange(100, 300, dtype=np.uint32), 1)]
    want = sum(oracle.count(g, p, roots=r, root_vertex=v, mode="B") for p, r, v in work)
    rec = bench.cpu_baseline(g, work, "two work items")
    assert rec["kind"] == "oracle" and rec["cores"] == bench.host_cores()
    assert f"{want} embeddings" in rec["sample"] and rec["sample"].startswith("two work items")
    assert rec["value"] == pytest.approx(want / rec["seconds_all_cores"], rel=1e-3)
    assert rec["value_1core"] == pytest.approx(want / rec["seconds_1core"], rel=1e-3)


def test_profile_records_are_keyed_by_library_and_workload():
    name = "count_kernel_batch256_traffic.json"
    path = os.path.join(bench.ROOT, "profiles", name)
    stored = json.load(open(path))
    assert bench.profile_record(name, "some_other_workload") is None
    rec = bench.profile_record(name, stored["workload_id"])
    assert (rec is not None) == (stored["lib_sha256_16"] == bench.lib_hash())
    assert bench.profile_record("no_such_summary.json", stored["workload_id"]) is None
