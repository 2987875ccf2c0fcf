"""Full-size GPU parity at 2^28 keys, in the launch configuration bench.py times.

The uniform configuration (2^28 u64 keys, p = 1024, eps = 0.02) and the
Zipf-Morton configuration with a payload (2^28 u64 keys + u64 source index,
p = 4096, eps = 0.05) are compared with the CPU oracle bit for bit: outputs
and offsets of hss_partition and hss_sort, the splitters (chi, S keys and
tags), the piece matrix, and every round's domain, probe keys, tags and
ranks, local histograms c_s(e) and splitter state.  The oracle runs its
per-segment work on up to 16 host threads (its result does not depend on
the thread count).  The largest accepted size (2^32 - 1 u32 keys), which the
oracle cannot hold in host memory, is checked by properties that hold at any
size.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_01237_amd as lib
    return lib


def _dev(a):
    return torch.from_numpy(a.view(np.int64)).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint64)


def _check_offsets(off, n, p, tol):
    ideal = (np.arange(p + 1, dtype=np.uint64) * np.uint64(n)) // np.uint64(p)
    assert off[0] == 0 and off[p] == n
    assert np.all(np.diff(off.astype(np.int64)) >= 0)
    dev = np.abs(off.astype(np.int64) - ideal.astype(np.int64))
    assert int(dev.max()) <= tol, int(dev.max())


def _compare_full(plan, ref, p, tag):
    """Every round of the trace (level 2) and the splitters, exactly."""
    tr = plan.trace()
    assert len(tr) == len(ref.rounds), (len(tr), len(ref.rounds))
    for j, (a, b) in enumerate(zip(tr, ref.rounds)):
        _say(f"[fullsize] {tag}: round {j + 1}: domain {a.domain} probes {a.m}")
        assert (a.domain, a.m, a.thresh, a.all) == (b.domain, b.m, b.thresh, b.all), j
        for f in ("probe_key", "probe_tag", "probe_rank", "counts", "settled", "chi",
                  "lo_rank", "hi_rank"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), (j, f)
    del tr
    chi, sk, stg, pieces = plan.splitters()
    assert np.array_equal(chi, ref.chi)
    assert np.array_equal(sk[1:p], ref.s_key[1:p])
    assert np.array_equal(stg[1:p], ref.s_tag[1:p])
    assert np.array_equal(pieces, ref.pieces)


def _full_parity(hss, name, kind, n, p, eps, dseed, hseed, payload):
    """The plan bench.py times (default tuning: graph-replayed rounds, draws
    taken ahead) against the oracle's outputs and splitters; a second plan
    with trace level 2 (rounds read back one by one) against the oracle's
    whole round trace."""
    _say(f"[fullsize] {name}: {kind} u64 n={n} p={p} eps={eps} seeds={dseed}/{hseed} "
         f"payload={payload}: generating")
    keys = synth.make(kind, n, dseed)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    _say(f"[fullsize] {name}: oracle partition on {ORACLE_THREADS} host threads")
    ref = oracle.hss(keys, p, eps, hseed, vals=vals, mode="partition", trace_level=2,
                     threads=ORACLE_THREADS)
    assert ref.status == 0
    _say(f"[fullsize] {name}: oracle stages (s): {ref.times}")
    with hss.Plan(n, p, eps, payload=payload) as plan:
        tol = plan.constants(1)[0]
        _say(f"[fullsize] {name}: hss_partition on the GPU")
        ko, vo, off = plan.partition(kd, hseed, vd)
        offs = _host(off)
        _check_offsets(offs, n, p, tol)
        assert np.array_equal(offs, ref.offsets)
        assert np.array_equal(_host(ko), ref.keys)
        if payload:
            assert np.array_equal(_host(vo), ref.vals)
        del ko, vo
        chi, sk, stg, pieces = plan.splitters()
        assert np.array_equal(chi, ref.chi)
        assert np.array_equal(sk[1:p], ref.s_key[1:p])
        assert np.array_equal(stg[1:p], ref.s_tag[1:p])
        assert np.array_equal(pieces, ref.pieces)
        _say(f"[fullsize] {name}: hss_sort on the GPU")
        ks, vs, off2 = plan.sort(kd, hseed, vd)
        srt = _host(ks)
        sv = None if vs is None else _host(vs)
        assert np.array_equal(_host(off2), ref.offsets)
        del ks, vs
    with hss.Plan(n, p, eps, payload=payload, trace_level=2) as plan:
        _say(f"[fullsize] {name}: hss_partition with the round trace")
        ko, vo, off = plan.partition(kd, hseed, vd)
        assert np.array_equal(_host(off), ref.offsets)
        assert np.array_equal(_host(ko), ref.keys)
        del ko, vo
        _compare_full(plan, ref, p, name)
    del ref
    _say(f"[fullsize] {name}: oracle sort")
    ref = oracle.hss(keys, p, eps, hseed, vals=vals, mode="sort", trace_level=0,
                     threads=ORACLE_THREADS)
    assert ref.status == 0
    assert np.array_equal(srt, ref.keys)
    if payload:
        assert np.array_equal(sv, ref.vals)


@pytest.mark.timeout(1200)
def test_uniform_2p28_p1024_bit_exact(hss):
    _full_parity(hss, "uniform", "uniform64", 1 << 28, 1024, 0.02, 2, 2, False)


@pytest.mark.timeout(1200)
def test_zipf_morton_payload_2p28_p4096_bit_exact(hss):
    _full_parity(hss, "zipf+morton", "zipf_morton", 1 << 28, 4096, 0.05, 3, 3, True)


def _device_digest(x, chunk=1 << 28):
    """Order-independent digest of int32 keys on the device (wrapping int64
    sums of the keys, of a splitmix64 hash of each and of its square)."""
    mask = (1 << 32) - 1
    c1 = 0x9E3779B97F4A7C15 - (1 << 64)
    c2 = 0xBF58476D1CE4E5B9 - (1 << 64)
    c3 = 0x94D049BB133111EB - (1 << 64)

    def lsr(v, k):   # logical shift right of int64
        return (v >> k) & ((1 << (64 - k)) - 1)

    s0 = s1 = s2 = torch.zeros((), dtype=torch.int64, device=x.device)
    for a in range(0, x.numel(), chunk):
        v = x[a:a + chunk].to(torch.int64) & mask
        z = v + c1
        z = (z ^ lsr(z, 30)) * c2
        z = (z ^ lsr(z, 27)) * c3
        z = z ^ lsr(z, 31)
        s0 = s0 + v.sum()
        s1 = s1 + z.sum()
        s2 = s2 + (z * z).sum()
    return int(s0), int(s1), int(s2), x.numel()


def test_partition_and_sort_at_the_largest_size_u32(hss):
    """N = 2^32 - 1 u32 keys, the largest plan the library accepts (tags,
    counts and piece offsets are 32-bit): the sort is in unsigned order and a
    permutation of the input, every splitter lies in its target range, and
    every bucket of the partition holds exactly the keys of its rank range
    (the same keys as the sort's bucket, each between its first and last)."""
    n, p, eps, hseed = (1 << 32) - 1, 1024, 0.02, 5
    flip = -(1 << 31)   # xor with the sign bit: signed order of the result = unsigned order
    _say(f"[fullsize] largest: u32 n={n} p={p} eps={eps}: generating on the device")
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    kd = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, generator=g, device="cuda")
    digest_in = _device_digest(kd)
    with hss.Plan(n, p, eps, key_bytes=4) as plan:
        tol = plan.constants(1)[0]
        _say("[fullsize] largest: hss_sort")
        ks, _, off_s = plan.sort(kd, hseed)
        offs = _host(off_s).astype(np.int64)
        _check_offsets(offs.astype(np.uint64), n, p, tol)
        assert _device_digest(ks) == digest_in
        ks ^= flip
        for a in range(0, n - 1, 1 << 28):
            b = min(a + (1 << 28) + 1, n)
            assert bool((ks[a + 1:b] >= ks[a:b - 1]).all()), a
        _say("[fullsize] largest: hss_partition")
        ko, _, off_p = plan.partition(kd, hseed)
        assert np.array_equal(_host(off_p).astype(np.int64), offs)
        ko ^= flip
        for b0 in range(0, p, 64):
            b1 = min(b0 + 64, p)
            a0, a1 = int(offs[b0]), int(offs[b1])
            part = ko[a0:a1]
            lens = torch.tensor(np.diff(offs[b0:b1 + 1]), device="cuda")
            first = torch.tensor(offs[b0:b1], device="cuda")
            last = torch.tensor(offs[b0 + 1:b1 + 1] - 1, device="cuda")
            lo = torch.repeat_interleave(ks[first], lens)
            hi = torch.repeat_interleave(ks[last], lens)
            assert bool(((part >= lo) & (part <= hi)).all()), b0
            assert torch.equal(torch.sort(part).values, ks[a0:a1]), b0
            del lo, hi
