"""Seeded directed data graphs stored as uint32 out-CSR + in-CSR.

Every graph is simple: arcs are distinct ordered pairs (u, v) with u != v.
Adjacency lists are sorted ascending.  The in-CSR is the transpose of the
out-CSR.  Node ids are < 2**32 and the arc count is < 2**32.

Workload recipes (the paper evaluates on SNAP power-law digraphs that are not
available here; these synthetic graphs stand in for them):

* ``uniform_digraph(n, m, seed)``: m distinct ordered pairs drawn uniformly
  with numpy PCG64 ``default_rng(seed)``, loops and repeats rejected.
* ``rmat(scale, edge_factor, abcd, seed)``: ``edge_factor * 2**scale`` R-MAT
  draws with quadrant probabilities (a, b, c, d), no noise and no id
  permutation, then repeats and self-loops dropped.
"""
from __future__ import annotations

import dataclasses
import numpy as np

U32 = np.uint32


@dataclasses.dataclass
class Digraph:
    n: int
    out_off: np.ndarray  # uint32[n+1]
    out_adj: np.ndarray  # uint32[m]
    in_off: np.ndarray   # uint32[n+1]
    in_adj: np.ndarray   # uint32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.out_adj.shape[0])

    def out_deg(self) -> np.ndarray:
        return np.diff(self.out_off.astype(np.int64))

    def in_deg(self) -> np.ndarray:
        return np.diff(self.in_off.astype(np.int64))

    def arcs(self) -> np.ndarray:
        """(m, 2) int64 array of arcs in out-CSR order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.out_deg())
        return np.stack([src, self.out_adj.astype(np.int64)], axis=1)

    def reversed(self) -> "Digraph":
        return Digraph(self.n, self.in_off, self.in_adj, self.out_off, self.out_adj,
                       name=self.name + "^T")

    def relabeled(self, perm: np.ndarray) -> "Digraph":
        """Graph with node x renamed perm[x]."""
        a = self.arcs()
        p = np.asarray(perm, dtype=np.int64)
        return from_arcs(self.n, p[a[:, 0]], p[a[:, 1]], name=self.name + "^perm")

    def sizing(self) -> dict:
        od, idg = self.out_deg(), self.in_deg()
        return {"n": self.n, "m": self.m, "max_out": int(od.max(initial=0)),
                "max_in": int(idg.max(initial=0)),
                "isolated": int(np.count_nonzero((od + idg) == 0)),
                "sum_out_sq": int((od * od).sum())}


def _csr_from_sorted_keys(n: int, keys: np.ndarray):
    """keys = (major << 32) | minor, sorted, unique -> (off[n+1], adj[m])."""
    major = (keys >> np.uint64(32)).astype(np.int64)
    adj = (keys & np.uint64(0xFFFFFFFF)).astype(U32)
    cnt = np.bincount(major, minlength=n)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    return off.astype(U32), adj


def from_arcs(n: int, src, dst, name: str = "") -> Digraph:
    """Build a simple digraph from arc arrays: drops loops and repeats."""
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    if n >= 2 ** 32:
        raise ValueError("node ids must fit in uint32")
    keep = src != dst
    src, dst = src[keep], dst[keep]
    if src.size and (src.max() >= n or dst.max() >= n):
        raise ValueError("arc endpoint out of range")
    okey = np.unique((src << np.uint64(32)) | dst)
    if okey.size >= 2 ** 32:
        raise ValueError("arc count must fit in uint32")
    out_off, out_adj = _csr_from_sorted_keys(n, okey)
    s2 = okey >> np.uint64(32)
    d2 = okey & np.uint64(0xFFFFFFFF)
    ikey = np.sort((d2 << np.uint64(32)) | s2)
    del okey, s2, d2
    in_off, in_adj = _csr_from_sorted_keys(n, ikey)
    return Digraph(n, out_off, out_adj, in_off, in_adj, name=name)


def uniform_digraph(n: int, m: int, seed: int = 0) -> Digraph:
    """Exactly m distinct arcs u->v (u != v), uniform, numpy PCG64(seed).

    Pairs are drawn in batches; a pair is kept if it is not a loop and has not
    been drawn before (first occurrence wins), until m pairs are kept.
    """
    if m > n * (n - 1):
        raise ValueError("too many arcs for a simple digraph")
    rng = np.random.default_rng(seed)
    seen = np.empty(0, dtype=np.uint64)
    order_keys = []
    have = 0
    while have < m:
        batch = max(1024, 2 * (m - have))
        u = rng.integers(0, n, size=batch, dtype=np.uint64)
        v = rng.integers(0, n, size=batch, dtype=np.uint64)
        key = (u << np.uint64(32)) | v
        key = key[u != v]
        # first occurrence within the batch, then drop keys already kept
        _, first = np.unique(key, return_index=True)
        key = key[np.sort(first)]
        key = key[~np.isin(key, seen)]
        key = key[: m - have]
        order_keys.append(key)
        seen = np.union1d(seen, key)
        have += key.size
    keys = np.concatenate(order_keys)
    return from_arcs(n, keys >> np.uint64(32), keys & np.uint64(0xFFFFFFFF),
                     name=f"uniform(n={n},m={m},seed={seed})")


RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)
_RMAT_CHUNK = 1 << 22  # fixed: the draw sequence depends on it


def rmat(scale: int, edge_factor: int = 16, abcd=RMAT_ABCD, seed: int = 0) -> Digraph:
    """R-MAT digraph with 2**scale nodes from edge_factor * 2**scale draws.

    Each draw picks one quadrant per bit level (most significant first) with
    probabilities (a, b, c, d): a -> (0,0), b -> (0,1), c -> (1,0), d -> (1,1)
    for the (source bit, destination bit).  Repeated arcs and loops are dropped.
    """
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    n = 1 << scale
    total = edge_factor * n
    rng = np.random.default_rng(seed)
    t_ab, t_abc = np.float32(a + b), np.float32(a + b + c)
    t_a = np.float32(a)
    keys = []
    done = 0
    while done < total:
        cnt = min(_RMAT_CHUNK, total - done)
        u = np.zeros(cnt, dtype=np.uint64)
        v = np.zeros(cnt, dtype=np.uint64)
        for lvl in range(scale):
            r = rng.random(cnt, dtype=np.float32)
            bit = np.uint64(1 << (scale - 1 - lvl))
            ubit = r >= t_ab
            vbit = ((r >= t_a) & (r < t_ab)) | (r >= t_abc)
            u |= ubit.astype(np.uint64) * bit
            v |= vbit.astype(np.uint64) * bit
        k = (u << np.uint64(32)) | v
        keys.append(np.unique(k[u != v]))
        done += cnt
    allk = np.unique(np.concatenate(keys)) if len(keys) > 1 else keys[0]
    return from_arcs(n, allk >> np.uint64(32), allk & np.uint64(0xFFFFFFFF),
                     name=f"rmat(scale={scale},ef={edge_factor},seed={seed})")


def complete_digraph(n: int) -> Digraph:
    """Every ordered pair (u, v), u != v: both arc directions everywhere."""
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return from_arcs(n, u.ravel(), v.ravel(), name=f"complete({n})")


def star_hub(leaves: int, extra_nodes: int = 0) -> Digraph:
    """Node 0 with arcs 0->i for i in 1..leaves (an out-star hub)."""
    n = leaves + 1 + extra_nodes
    return from_arcs(n, np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1),
                     name=f"outstar({leaves})")


@dataclasses.dataclass
class DeviceDigraph:
    """A simple digraph whose uint32 CSR arrays live in device memory (int32
    tensors holding the uint32 bit patterns)."""
    n: int
    out_off: object
    out_adj: object
    in_off: object
    in_adj: object
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.out_off[-1])

    def to_host(self) -> Digraph:
        cv = lambda t: t.cpu().numpy().view(np.uint32)  # noqa: E731
        m = int(self.out_off[-1])
        return Digraph(self.n, cv(self.out_off), cv(self.out_adj)[:m], cv(self.in_off),
                       cv(self.in_adj)[:m], name=self.name)


def rmat_device(scale: int, edge_factor: int = 16, abcd=RMAT_ABCD, seed: int = 0,
                device: str = "cuda") -> DeviceDigraph:
    """R-MAT on the GPU with torch's seeded generator (same recipe as rmat():
    edge_factor * 2**scale draws, quadrant probabilities (a, b, c, d) per bit
    level, repeats and loops dropped).  The draws differ from rmat()'s numpy
    stream, so the graph differs; it is deterministic for a seed on one
    device type.  Built directly in device memory for graphs too large to
    generate on the host quickly."""
    import torch
    a, b, c, d = abcd
    n = 1 << scale
    total = edge_factor * n
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    t_a, t_ab, t_abc = float(a), float(a + b), float(a + b + c)
    keys = []
    chunk = 1 << 24
    done = 0
    while done < total:
        cnt = min(chunk, total - done)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for lvl in range(scale):
            r = torch.rand(cnt, generator=gen, device=device, dtype=torch.float32)
            bit = 1 << (scale - 1 - lvl)
            ub = r >= t_ab
            vb = ((r >= t_a) & (r < t_ab)) | (r >= t_abc)
            u += ub.to(torch.int64) * bit
            v += vb.to(torch.int64) * bit
        keep = u != v
        keys.append(torch.unique((u[keep] << 32) | v[keep]))
        done += cnt
        del u, v
    key = torch.unique(torch.cat(keys)) if len(keys) > 1 else keys[0]
    del keys
    src = key >> 32
    dst = key & 0xFFFFFFFF
    m = int(key.numel())
    out_off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    out_off[1:] = torch.cumsum(torch.bincount(src, minlength=n), 0)
    out_adj = dst.to(torch.int32)
    ikey, _ = torch.sort((dst << 32) | src)
    in_off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    in_off[1:] = torch.cumsum(torch.bincount(dst, minlength=n), 0)
    in_adj = (ikey & 0xFFFFFFFF).to(torch.int32)
    del key, src, dst, ikey
    if m == 0:
        out_adj = torch.zeros(1, dtype=torch.int32, device=device)
        in_adj = torch.zeros(1, dtype=torch.int32, device=device)
    return DeviceDigraph(n, out_off.to(torch.int32), out_adj, in_off.to(torch.int32), in_adj,
                         name=f"rmat_device(scale={scale},ef={edge_factor},seed={seed})")
