"""GPU: xm_count_static, the entry point that allocates nothing (its
workspace is the library's static scratch array), gives exactly the counts
of xm_count, on two calls in a row with the second input smaller, and
refuses a launch whose workspace would not fit the array."""
import ctypes

import pytest

import xmgen
from tests.cases import CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def xa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_11105_amd as xa
    return xa


def static_count(xa, G, plans, **opts):
    """xm_count_static through the C ABI; returns (counts, statuses)."""
    import torch

    from paper_2404_11105_amd import _lib
    from paper_2404_11105_amd.api import _stream_ptr, make_opts
    n = len(plans)
    counts = torch.zeros(2 * n, dtype=torch.int64, device=G.device)
    status = torch.full((n,), 99, dtype=torch.int32, device=G.device)
    arr = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    o = make_opts(**opts) if opts else None
    torch.cuda.synchronize()
    rc = _lib.lib().xm_count_static(G.handle, n, arr, ctypes.byref(o) if o is not None else None,
                                     ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                                     _stream_ptr(None))
    if rc != 0:
        return rc, None
    torch.cuda.synchronize()
    c = counts.cpu().numpy().view("uint64")
    return [int(c[2 * i]) | (int(c[2 * i + 1]) << 64) for i in range(n)], [int(s) for s in status.cpu()]


def test_static_entry_point_equals_xm_count_on_two_calls(xa):
    cases = [("rmat11_named", dict(symmetry=False)), ("rand_uniform300", dict(symmetry=False))]
    for name, kw in cases:
        print(f"[case] xm_count_static on {name}", flush=True)
        c = CASES[name]
        g, pats = c["graph"](), c["patterns"]()
        G = xa.Graph(g)
        plans = [xa.Plan(p, reduced=True, graph=G, **kw) for p in pats]
        want = xa.count(G, plans)
        got, status = static_count(xa, G, plans)
        assert status == [0] * len(plans), status
        assert got == want, name
    # the second call above was smaller (fewer nodes and arcs) than the first;
    # a third, smaller still, with symmetry-broken plans and a root subset
    g = xmgen.uniform_digraph(200, 1200, 4)
    G = xa.Graph(g)
    plans = [xa.Plan(xmgen.named(n), reduced=True, graph=G, root_vertex=0, symmetry="above")
             for n in ("bifan", "c4")]
    import numpy as np
    roots = np.arange(0, 200, 3, dtype=np.uint32)
    cnt = xa.Counter(G, plans, roots=roots)
    cnt.run()
    want = cnt.results()[0]
    got, status = static_count(xa, G, plans, roots=cnt.roots, roots_host=cnt.roots_host)
    assert status == [0, 0] and got == want


def test_static_entry_point_refuses_a_workspace_past_the_array(xa):
    from paper_2404_11105_amd import _lib
    g = xmgen.rmat(11, seed=1)
    G = xa.Graph(g)
    plans = [xa.Plan(xmgen.named("c4"), reduced=False, graph=G)]
    rc, _ = static_count(xa, G, plans, cap=1 << 16, waves_per_cu=32)
    assert rc == _lib.XM_ERR_WORKSPACE
    assert b"static scratch" in _lib.lib().xm_last_error()
    # a launch that fits still runs after the refusal
    got, status = static_count(xa, G, plans)
    assert status == [0] and got == xa.count(G, plans)
