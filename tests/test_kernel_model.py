"""CPU model of the count kernel's control flow: termination and parity.

Runs tests/kernel_model.py (which follows count.hip step by step and
asserts every buffer index) under extreme tunings that force hub splitting,
partial windows and reuse fallbacks, and compares with the oracle.
"""
import pytest

import oracle
import xmgen
from paper_2404_11105_amd import describe_plan
from tests.kernel_model import Model

TUNINGS = [dict(chunk=1, split=64, cap=64), dict(chunk=64, split=64, cap=128, split_work=4096),
           dict(chunk=7, split=100, cap=4096)]


@pytest.mark.parametrize("tune", TUNINGS, ids=lambda t: f"c{t['chunk']}s{t['split']}k{t['cap']}")
def test_model_terminates_and_matches_oracle(tune):
    g = xmgen.rmat(7, seed=7)  # hubs of degree > 64 exist, so roots get split
    assert max(g.out_deg().max(), g.in_deg().max()) > 64
    for name in ["bifan", "c4", "tt4p", "ffl", "c3", "mixed_star"]:
        pat = xmgen.named(name)
        want = oracle.count(g, pat)
        for reduced in (True, False):
            m = Model(describe_plan(pat, reduced), g, **tune, max_windows=200000)
            assert m.run() == want, (name, reduced)


def test_model_random_patterns_small_cap():
    g = xmgen.uniform_digraph(60, 500, 3)
    pat = xmgen.named("p7hub")
    for reduced in (True, False):
        assert Model(describe_plan(pat, reduced), g, chunk=3, split=64, cap=64).run() == oracle.count(g, pat)
    for k in range(3, 7):
        for s in range(3):
            pat = xmgen.random_pattern(k, 700 + 10 * k + s)
            want = oracle.count(g, pat)
            for reduced in (True, False):
                m = Model(describe_plan(pat, reduced), g, chunk=3, split=64, cap=64)
                assert m.run() == want, (k, s, reduced)
