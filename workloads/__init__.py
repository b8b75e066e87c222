"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random inputs: it holds none of the sorting method's
arithmetic (no run detection, powers or merging) and imports neither the
oracle nor the GPU library, so both sides can be fed the same arrays.

The paper measures on synthetic data only (Section 4.3: integers with random
runs, 16-byte records, random permutations); its generator code is not
published, so the recipes below are this project's stand-ins for those inputs.
All host draws use numpy's PCG64 ``default_rng(seed)``.  The two large pools
(the batched workload at full size, about 3.5e9 keys, and the serving request
pool) are drawn on the GPU with a seeded torch generator instead, so that the
benchmark does not spend minutes on the host: sizes and run lengths still come
from PCG64, and the keys of each run are drawn already in ascending order as
order statistics (the ascending sample of L uniforms has the law of the
normalised partial sums S_1/S_{L+1} < ... < S_L/S_{L+1} of L+1 standard
exponential gaps), so no per-run sort is needed.

Workloads (sizes can be scaled down for tests; the recipe stays the same):
  runs_i32      n=2^20 int32; run lengths U{1..2048} (last run truncated);
                values uniform int32, sorted ascending, each run reversed
                with probability 1/2; payload = input index.
  runs_i64      n=2^28 int64 uniform over the full range; run lengths
                U{1..2*sqrt(n)}, each run sorted ascending; payload = index.
  perm_i64      n=2^28 int64 random permutation of 0..n-1 (no presortedness).
  ties_i32      n=2^27 int32 from 16 distinct values (14 uniform plus INT32_MIN
                and INT32_MAX); run lengths min(floor(U^(-1/1.5)), n/8)
                (Pareto alpha=1.5, minimum 1); with probability 0.2 a run is
                strictly descending (length min(L,16), distinct values), else
                L i.i.d. draws from the 16 values sorted ascending.
  batch_i32     m=8192 arrays, sizes floor(2^U), U~U[8,22]; int32 full range;
                run lengths U{1..floor(2*sqrt(size))}, sorted ascending;
                payload = index within the array.  Packed with uint64 offsets.
  batch_i32_device  the same recipe at full size on the GPU (order statistics).
  serve_f32     request pool: sizes floor(2^U), U~U[10,26]; float32 ~ N(0,1)
                redrawn while |x| < FLT_MIN (all normal numbers); about 1% of
                positions overwritten by copies of other keys of the same
                request; runs U{1..floor(2*sqrt(size))} sorted ascending;
                int32 payload = index.  Arrivals: Poisson process.
"""
from __future__ import annotations

import math

import numpy as np

I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1


def _run_lengths(rng: np.random.Generator, n: int, draw) -> np.ndarray:
    """Consecutive run lengths from ``draw(rng, count)`` until they cover n (last one truncated)."""
    out = []
    total = 0
    while total < n:
        need = n - total
        chunk = draw(rng, max(64, need // 8 + 64))
        cs = np.cumsum(chunk, dtype=np.int64)
        cut = int(np.searchsorted(cs, need, side="left"))
        if cut < chunk.size:
            chunk = chunk[: cut + 1].copy()
            chunk[-1] -= int(cs[cut] - need)
            out.append(chunk)
            total = n
        else:
            out.append(chunk)
            total += int(cs[-1])
    lens = np.concatenate(out) if out else np.zeros(0, np.int64)
    return lens[lens > 0].astype(np.int64)


def _sort_runs_inplace(vals: np.ndarray, lens: np.ndarray) -> None:
    pos = 0
    for L in lens.tolist():
        if L > 1:
            vals[pos:pos + L].sort(kind="stable")
        pos += L


def runs_i32(n: int = 1 << 20, seed: int = 1, max_run: int = 2048):
    rng = np.random.default_rng(seed)
    lens = _run_lengths(rng, n, lambda g, c: g.integers(1, max_run + 1, size=c))
    keys = rng.integers(I32_MIN, I32_MAX + 1, size=n, dtype=np.int64).astype(np.int32)
    _sort_runs_inplace(keys, lens)
    flips = rng.random(lens.size) < 0.5
    pos = 0
    for L, f in zip(lens.tolist(), flips.tolist()):
        if f and L > 1:
            keys[pos:pos + L] = keys[pos:pos + L][::-1].copy()
        pos += L
    return keys, np.arange(n, dtype=np.uint32)


def runs_i64(n: int = 1 << 28, seed: int = 2, max_run: int | None = None):
    rng = np.random.default_rng(seed)
    if max_run is None:
        max_run = max(1, int(2 * math.isqrt(n)))
    lens = _run_lengths(rng, n, lambda g, c: g.integers(1, max_run + 1, size=c))
    keys = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, size=n,
                        dtype=np.int64, endpoint=True)
    _sort_runs_inplace(keys, lens)
    return keys, np.arange(n, dtype=np.uint32)


def perm_i64(n: int = 1 << 28, seed: int = 3):
    rng = np.random.default_rng(seed)
    return rng.permutation(n).astype(np.int64), np.arange(n, dtype=np.uint32)


def ties_i32(n: int = 1 << 27, seed: int = 4, desc_prob: float = 0.2):
    rng = np.random.default_rng(seed)
    distinct = np.unique(rng.integers(I32_MIN + 1, I32_MAX, size=64, dtype=np.int64))
    distinct = rng.permutation(distinct)[:14]
    table = np.sort(np.concatenate([distinct, [I32_MIN, I32_MAX]])).astype(np.int32)
    assert table.size == 16
    cap = max(1, n // 8)

    def draw(g, c):
        u = 1.0 - g.random(c)                       # U in (0, 1]
        return np.minimum(np.floor(u ** (-1.0 / 1.5)), cap).astype(np.int64)

    # Run lengths; a descending run is cut to at most 16 (it needs distinct
    # values).  Draw until the (possibly cut) lengths cover n.
    lens_parts, desc_parts, total = [], [], 0
    while total < n:
        L = _run_lengths(rng, n - total, draw)
        d = rng.random(L.size) < desc_prob
        L = np.where(d, np.minimum(L, 16), L)
        lens_parts.append(L)
        desc_parts.append(d)
        total += int(L.sum())
    lens = np.concatenate(lens_parts)
    desc = np.concatenate(desc_parts)
    cs = np.cumsum(lens)
    keep = int(np.searchsorted(cs, n, side="left")) + 1
    lens, desc = lens[:keep].copy(), desc[:keep].copy()
    lens[-1] -= int(cs[keep - 1] - n)
    desc &= lens > 1

    vi = np.empty(n, dtype=np.int64)
    elem_desc = np.repeat(desc, lens)
    # ascending runs: i.i.d. value indices, sorted within each run
    asc_pos = np.flatnonzero(~elem_desc)
    asc_run = np.repeat(np.arange(lens.size, dtype=np.int64)[~desc], lens[~desc])
    comp = asc_run * 16 + rng.integers(0, 16, size=asc_pos.size, dtype=np.int64)
    comp.sort(kind="stable")
    vi[asc_pos] = comp % 16
    # descending runs: a random L-subset of the 16 indices, in decreasing order
    d_lens = lens[desc]
    chunks = []
    for c0 in range(0, d_lens.size, 1 << 20):
        dl = d_lens[c0:c0 + (1 << 20)]
        rank = np.argsort(np.argsort(rng.random((dl.size, 16)), axis=1), axis=1)
        chosen = (rank < dl[:, None])[:, ::-1]
        chunks.append(np.broadcast_to(np.arange(15, -1, -1), chosen.shape)[chosen])
    if chunks:
        vi[np.flatnonzero(elem_desc)] = np.concatenate(chunks)
    keys = table[vi]
    return keys, np.arange(n, dtype=np.uint32)


def batch_i32(m: int = 8192, seed: int = 5, lo_exp: float = 8.0, hi_exp: float = 22.0):
    """Returns (keys int32[N], payload uint32[N] local index, offsets uint64[m+1])."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=m)).astype(np.int64)
    offsets = np.zeros(m + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    keys = np.empty(total, dtype=np.int32)
    payload = np.empty(total, dtype=np.uint32)
    for i, sz in enumerate(sizes.tolist()):
        s = int(offsets[i])
        mr = max(1, int(2 * math.isqrt(sz)))
        lens = _run_lengths(rng, sz, lambda g, c, mr=mr: g.integers(1, mr + 1, size=c))
        v = rng.integers(I32_MIN, I32_MAX + 1, size=sz, dtype=np.int64)
        rid = np.repeat(np.arange(lens.size, dtype=np.int64), lens)
        comp = np.sort((rid << 32) | (v - I32_MIN))
        keys[s:s + sz] = ((comp & 0xFFFFFFFF) + I32_MIN).astype(np.int32)
        payload[s:s + sz] = np.arange(sz, dtype=np.uint32)
    return keys, payload, offsets


def serve_request_f32(size: int, rng: np.random.Generator):
    """One serving request: float32 keys (normal numbers, ~1% duplicates) in random runs."""
    x = rng.standard_normal(size).astype(np.float32)
    tiny = np.abs(x) < np.finfo(np.float32).tiny
    while tiny.any():
        x[tiny] = rng.standard_normal(int(tiny.sum())).astype(np.float32)
        tiny = np.abs(x) < np.finfo(np.float32).tiny
    ndup = size // 100
    if ndup and size > 1:
        dst = rng.integers(0, size, size=ndup)
        src = rng.integers(0, size, size=ndup)
        x[dst] = x[src]
    mr = max(1, int(2 * math.isqrt(size)))
    lens = _run_lengths(rng, size, lambda g, c: g.integers(1, mr + 1, size=c))
    _sort_runs_inplace(x, lens)
    return x, np.arange(size, dtype=np.uint32)


def serve_sizes(count: int, seed: int = 6, lo_exp: float = 10.0, hi_exp: float = 26.0):
    rng = np.random.default_rng(seed)
    return np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    expected = int(rate_per_s * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_per_s, size=expected)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate_per_s, size=expected)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


WORKLOADS = {
    "runs_i32": runs_i32,
    "runs_i64": runs_i64,
    "perm_i64": perm_i64,
    "ties_i32": ties_i32,
}


# ---------------------------------------------------------------- device pools
def _batch_layout(m: int, seed: int, lo_exp: float, hi_exp: float):
    """Array sizes, offsets and per-array run lengths (host, PCG64)."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=m)).astype(np.int64)
    offsets = np.zeros(m + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    lens = []
    for sz in sizes.tolist():
        mr = max(1, int(2 * math.isqrt(sz)))
        lens.append(_run_lengths(rng, sz, lambda g, c, mr=mr: g.integers(1, mr + 1, size=c)))
    return sizes, offsets, lens


def _sorted_uniform_runs(torch, gen, run_lens, device):
    """float64 tensor: for each run of length L, L ascending uniforms in (0,1) drawn
    as order statistics (partial sums of L+1 exponential gaps over their total)."""
    lens = torch.as_tensor(run_lens, dtype=torch.int64, device=device)
    R = lens.numel()
    T = int(lens.sum())
    gaps = torch.empty(T + R, dtype=torch.float64, device=device).exponential_(generator=gen)
    cs = gaps.cumsum_(0)
    run_id = torch.repeat_interleave(torch.arange(R, device=device), lens)
    slot = torch.arange(T, device=device) + run_id                  # run r owns L_r + 1 slots
    first = torch.cumsum(lens, 0) - lens + torch.arange(R, device=device)   # first slot of run r
    base = torch.where(first > 0, cs[(first - 1).clamp_min(0)], torch.zeros_like(cs[:1]))
    total = cs[first + lens] - base
    u = (cs[slot] - base[run_id]) / total[run_id]
    return u


def batch_i32_device(m: int = 8192, seed: int = 5, lo_exp: float = 8.0, hi_exp: float = 22.0,
                     device: str = "cuda:0", chunk_keys: int = 1 << 27):
    """The batched workload drawn on the GPU: (keys int32 tensor, payload int32 tensor =
    index within the array, host offsets uint64[m+1]).  Same sizes and run-length
    recipe as batch_i32; keys uniform over int32, ascending within runs."""
    import torch
    sizes, offsets, lens = _batch_layout(m, seed, lo_exp, hi_exp)
    total = int(offsets[-1])
    keys = torch.empty(total, dtype=torch.int32, device=device)
    pay = torch.empty(total, dtype=torch.int32, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    i = 0
    while i < m:
        j, n = i, 0
        while j < m and (j == i or n + sizes[j] <= chunk_keys):
            n += int(sizes[j])
            j += 1
        s0 = int(offsets[i])
        if n:
            u = _sorted_uniform_runs(torch, gen, np.concatenate(lens[i:j]), device)
            k = torch.floor(u * 4294967296.0) - 2147483648.0
            keys[s0:s0 + n] = k.clamp_(-2147483648.0, 2147483647.0).to(torch.int32)
            sz = torch.as_tensor(sizes[i:j], device=device)
            starts = torch.cumsum(sz, 0) - sz
            pay[s0:s0 + n] = (torch.arange(n, device=device)
                              - torch.repeat_interleave(starts, sz)).to(torch.int32)
        i = j
    return keys, pay, offsets


def serve_pool_device(count: int = 512, seed: int = 6, lo_exp: float = 10.0, hi_exp: float = 26.0,
                      device: str = "cuda:0"):
    """Serving request pool on the GPU: a list of (keys float32 tensor, payload int32 =
    index) per request.  Sizes floor(2^U), U~U[lo,hi] (PCG64, seed); keys N(0,1) in random
    runs U{1..floor(2*sqrt(size))}, ascending within a run (normal quantiles of sorted
    uniforms, kept away from 0 so every key is a normal float32), and about 1% of the
    positions repeat their left neighbour's key (duplicates)."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.floor(2.0 ** rng.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    tiny = float(np.finfo(np.float32).tiny)
    pool = []
    for sz in sizes.tolist():
        mr = max(1, int(2 * math.isqrt(sz)))
        lens = _run_lengths(rng, sz, lambda g, c: g.integers(1, mr + 1, size=c))
        u = _sorted_uniform_runs(torch, gen, lens, device)
        x = torch.special.ndtri(u).to(torch.float32)
        small = x.abs() < tiny
        x = torch.where(small, torch.where(x < 0, -tiny, tiny), x)   # no zeros or subnormals
        if sz > 1:
            nd = max(1, sz // 100)
            pos = torch.randint(1, sz, (nd,), generator=gen, device=device)
            x[pos] = x[pos - 1]
        pool.append((x, torch.arange(sz, dtype=torch.int32, device=device)))
    return pool
