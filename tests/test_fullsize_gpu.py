"""Full-size GPU checks at 2^28 keys, in the launch configuration bench.py times.

The oracle cannot run these sizes in test time, so the outputs are checked by
properties that hold at any size (a permutation of the input, bucket order,
piece order, balance) and sampled splitters are recomputed one by one from
their definition: chi(i) is the rank of the splitter element S(i) in the order
(key, tag) of sections 2 and 6.1, counted segment by segment on the host.
"""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _mix(a):
    """splitmix64 finaliser of every key (wrapping uint64 arithmetic)."""
    with np.errstate(over="ignore"):
        z = a + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _multiset_digest(a):
    """Order-independent digest: wrapping sums of the keys and of a mixing hash, and xor."""
    with np.errstate(over="ignore"):
        h = _mix(a)
        return (int(a.sum(dtype=np.uint64)), int(h.sum(dtype=np.uint64)),
                int(np.bitwise_xor.reduce(h)), len(a))


def _check_offsets(off, n, p, tol):
    ideal = (np.arange(p + 1, dtype=np.uint64) * np.uint64(n)) // np.uint64(p)
    assert off[0] == 0 and off[p] == n
    assert np.all(np.diff(off.astype(np.int64)) >= 0)
    dev = np.abs(off.astype(np.int64) - ideal.astype(np.int64))
    assert int(dev.max()) <= tol, int(dev.max())


def _check_sampled_splitters(keys, p, chi, s_key, s_tag, which):
    """chi(i) = #{(k, g) < (s_key, s_tag)}: keys below s_key in every segment,
    plus the equal keys whose tag (local stable position) is below s_tag."""
    n = len(keys)
    ns = n // p
    seg = keys.reshape(p, ns)
    base = np.arange(p, dtype=np.int64) * ns
    for i in which:
        k, g = np.uint64(s_key[i]), int(s_tag[i])
        lt = (seg < k).sum(axis=1).astype(np.int64)
        eq = (seg == k).sum(axis=1).astype(np.int64)
        first_eq_tag = base + lt
        below = np.clip(g - first_eq_tag, 0, eq)
        rank = int(lt.sum() + below.sum())
        assert rank == int(chi[i]), (i, rank, int(chi[i]))
        # S(i) is the element with tag g: the x-th smallest of its segment
        t, x = g // ns, g % ns
        assert np.partition(seg[t], x)[x] == k, i


def _bucket_bounds_keys_only(out, off):
    """Every key of bucket b is <= every key of bucket b+1."""
    starts = off[:-1].astype(np.int64)
    ends = off[1:].astype(np.int64)
    nz = ends > starts
    mx = np.maximum.reduceat(out, starts[nz])
    mn = np.minimum.reduceat(out, starts[nz])
    assert np.all(mx[:-1] <= mn[1:])


def test_partition_and_sort_uniform_2p28_p1024(hss):
    n, p, eps, dseed, hseed = 1 << 28, 1024, 0.02, 2, 2
    _say(f"[fullsize] uniform u64 n={n} p={p} eps={eps} seed={hseed}: generating")
    keys = synth.make("uniform64", n, dseed)
    digest_in = _multiset_digest(keys)
    kd = _dev(keys)
    with hss.Plan(n, p, eps) as plan:
        tol = plan.constants(1)[0]
        _say("[fullsize] uniform: hss_partition")
        ko, _, off = plan.partition(kd, hseed)
        out, offs = _host(ko), _host(off)
        _check_offsets(offs, n, p, tol)
        assert _multiset_digest(out) == digest_in
        _bucket_bounds_keys_only(out, offs)
        chi, s_key, s_tag, _ = plan.splitters()
        assert np.array_equal(chi, offs)
        rng = np.random.default_rng(0)
        which = sorted(set(rng.integers(1, p, size=12).tolist()) | {1, p // 2, p - 1})
        _say(f"[fullsize] uniform: {len(which)} sampled splitters from their definition")
        _check_sampled_splitters(keys, p, chi, s_key, s_tag, which)
        del out
        _say("[fullsize] uniform: hss_sort")
        ks, _, off2 = plan.sort(kd, hseed)
        srt = _host(ks)
        assert np.all(srt[1:] >= srt[:-1])
        assert _multiset_digest(srt) == digest_in
        assert np.array_equal(_host(off2), offs)


def test_partition_and_sort_zipf_morton_payload_2p28_p4096(hss):
    n, p, eps, dseed, hseed = 1 << 28, 4096, 0.05, 3, 3
    _say(f"[fullsize] zipf+morton u64+payload n={n} p={p} eps={eps} seed={hseed}: generating")
    keys = synth.make("zipf_morton", n, dseed)
    vals = np.arange(n, dtype=np.uint64)
    ns = n // p
    kd, vd = _dev(keys), _dev(vals)
    with hss.Plan(n, p, eps, payload=True) as plan:
        tol = plan.constants(1)[0]
        _say("[fullsize] zipf+morton: hss_partition")
        ko, vo, off = plan.partition(kd, hseed, vd)
        out, ov, offs = _host(ko), _host(vo), _host(off)
        _check_offsets(offs, n, p, tol)
        # the payload (source index) names a permutation carrying its key
        seen = np.zeros(n, dtype=np.uint8)
        seen[ov.astype(np.int64)] = 1
        assert int(seen.sum()) == n
        del seen
        assert np.array_equal(keys[ov.astype(np.int64)], out)
        # inside a bucket: pieces by ascending source segment, each in (key,
        # source index) order; between buckets: (key, source index) order
        src_seg = ov // np.uint64(ns)
        start = np.zeros(n, dtype=bool)
        start[offs[:-1][offs[:-1] < n].astype(np.int64)] = True
        step_seg = src_seg[1:].astype(np.int64) - src_seg[:-1].astype(np.int64)
        assert np.all((step_seg >= 0) | start[1:])
        same = (step_seg == 0) & ~start[1:]
        inc = (out[1:] > out[:-1]) | ((out[1:] == out[:-1]) & (ov[1:] > ov[:-1]))
        assert np.all(inc | ~same)
        del src_seg, step_seg, same, inc, start
        _say("[fullsize] zipf+morton: bucket order")
        for b in range(p - 1):
            a0, a1, a2 = int(offs[b]), int(offs[b + 1]), int(offs[b + 2])
            if a0 == a1 or a1 == a2:
                continue
            kb, vb = out[a0:a1], ov[a0:a1]
            kc, vc = out[a1:a2], ov[a1:a2]
            mxk, mnk = kb.max(), kc.min()
            assert mxk <= mnk, b
            if mxk == mnk:
                assert vb[kb == mxk].max() < vc[kc == mnk].min(), b
        chi, s_key, s_tag, _ = plan.splitters()
        assert np.array_equal(chi, offs)
        rng = np.random.default_rng(1)
        which = sorted(set(rng.integers(1, p, size=12).tolist()) | {1, p // 2, p - 1})
        _say(f"[fullsize] zipf+morton: {len(which)} sampled splitters from their definition")
        _check_sampled_splitters(keys, p, chi, s_key, s_tag, which)
        del out, ov
        _say("[fullsize] zipf+morton: hss_sort")
        ks, vs, off2 = plan.sort(kd, hseed, vd)
        srt, sv = _host(ks), _host(vs)
        assert np.array_equal(keys[sv.astype(np.int64)], srt)
        assert np.all((srt[1:] > srt[:-1]) | ((srt[1:] == srt[:-1]) & (sv[1:] > sv[:-1])))
        assert np.array_equal(_host(off2), offs)


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
