"""GPU tests of the request server: every served request equals the plain
hss_partition (or hss_sort) of the same request bit for bit (keys, payload,
offsets), whatever else was batched with it; a few small ones also equal the
oracle."""
import sys
import time

import numpy as np
import pytest

import oracle
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


def _requests(count, seed):
    """Mixed small requests: u32 and u64 keys, with and without payload."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(2 ** rng.uniform(10, 17))
        p = int(min(n, np.exp(rng.uniform(np.log(4), np.log(300)))))
        eps = float(rng.choice([0.02, 0.05, 0.1]))
        kb = 4 if rng.integers(0, 3) == 0 else 8
        pay = bool(rng.integers(0, 2))
        out.append((n, max(p, 1), eps, kb, pay, 7000 + i))
    return out


def _inputs(n, kb, pay, dseed):
    keys = synth.make("uniform64", n, dseed)
    if kb == 4:
        keys = (keys >> np.uint64(32)).astype(np.uint32)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if pay else None
    return keys, vals


def _dev(a):
    return torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()


def test_served_requests_equal_plain_partitions(hss):
    reqs = _requests(48, 3)
    _say(f"[server] {len(reqs)} requests in bursts")
    with hss.Server(max_batch_keys=1 << 20, max_batch_requests=16) as srv:
        tickets, held = [], []
        for i, (n, p, eps, kb, pay, dseed) in enumerate(reqs):
            keys, vals = _inputs(n, kb, pay, dseed)
            kd = _dev(keys)
            vd = _dev(vals) if pay else None
            tickets.append(srv.submit(kd, p, eps, dseed, vd))
            held.append((keys, vals, kd, vd))
            if i % 8 == 7:
                time.sleep(0.002)
        done = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert st["requests"] == len(reqs)
        assert 1 <= st["batches"] <= len(reqs)
        _say(f"[server] {st['batches']} batches; comparing with plain partitions")
        for i, ((n, p, eps, kb, pay, dseed), r) in enumerate(zip(reqs, done)):
            keys, vals, kd, vd = held[i]
            assert r.t_done >= r.t_submit
            with hss.Plan(n, p, eps, key_bytes=kb, payload=pay) as plan:
                ko, vo, off = plan.partition(kd, dseed, vd)
                torch.cuda.synchronize()
                assert torch.equal(off, r.offsets), i
                assert torch.equal(ko, r.keys_out), i
                if pay:
                    assert torch.equal(vo, r.vals_out), i
            if i < 6:
                ref = oracle.hss(keys, p, eps, dseed, vals=vals, mode="partition", trace_level=0)
                assert np.array_equal(r.offsets.cpu().numpy().view(np.uint64), ref.offsets), i
                kt = np.uint64 if kb == 8 else np.uint32
                assert np.array_equal(r.keys_out.cpu().numpy().view(kt), ref.keys), i


def test_server_polls_and_reuses_memory(hss):
    """Two waves of identical shapes: the second runs from the block cache;
    poll reports a request only once."""
    with hss.Server() as srv:
        for wave in range(2):
            tickets = []
            for i in range(6):
                keys, vals = _inputs(50_000 + 1000 * i, 8, True, 900 + i)
                tickets.append((srv.submit(_dev(keys), 32, 0.05, 11 + i, _dev(vals)), keys, vals))
            for i, (t, keys, vals) in enumerate(tickets):
                r = None
                while r is None:
                    r = srv.poll(t)
                    time.sleep(0.001)
                with pytest.raises(hss.HssError):
                    srv.poll(t)                       # retired
                ref = oracle.hss(keys, 32, 0.05, 11 + i, vals=vals, mode="partition", trace_level=0)
                assert np.array_equal(r.offsets.cpu().numpy().view(np.uint64), ref.offsets)
                assert np.array_equal(r.vals_out.cpu().numpy().view(np.uint64), ref.vals)


def test_server_rejects_bad_requests(hss):
    import ctypes as C
    with hss.Server() as srv:
        k = torch.zeros(100, dtype=torch.int64, device="cuda")
        with pytest.raises(hss.HssError):
            srv.submit(k, 200, 0.05, 1)                # p > N
        with pytest.raises(hss.HssError):
            srv.submit(k, 4, 1.5, 1)                   # eps >= 1
        with pytest.raises(hss.HssError):
            srv.submit(k[1:], 4, 0.05, 1)              # misaligned keys
        with pytest.raises(ValueError):
            srv.submit(k, 4, 0.05, 1, op="merge")      # no such operation
        ko = torch.empty_like(k)
        off = torch.empty(5, dtype=torch.int64, device="cuda")
        req = hss._Request(100, 4, hss.HSS_U64, 0.05, 1, k.data_ptr(), None, ko.data_ptr(), None,
                           off.data_ptr(), 7)           # an operation code the library does not know
        t = C.c_uint64()
        assert hss._lib.hss_server_submit(srv._h, C.byref(req), C.byref(t)) == -1   # invalid argument
        assert srv.stats()["requests"] == 0


def test_served_sorts_and_partitions_equal_plain_calls(hss):
    """A stream mixing sort and partition requests: a sort request runs as a
    batch of its own, partitions batch together; every result equals the
    plain hss_sort or hss_partition of the same request, and small sorts the
    oracle's."""
    reqs = _requests(24, 8)
    reqs.append(((1 << 20) + 5, 96, 0.02, 8, True, 7999))   # a sort above the early-draw size
    ops = ["sort" if i % 2 == 0 else "partition" for i in range(len(reqs))]
    ops[-1] = "sort"
    _say(f"[server] {len(reqs)} requests, sorts and partitions mixed")
    with hss.Server(max_batch_keys=1 << 20, max_batch_requests=16) as srv:
        tickets, held = [], []
        for i, ((n, p, eps, kb, pay, dseed), op) in enumerate(zip(reqs, ops)):
            keys, vals = _inputs(n, kb, pay, dseed)
            kd = _dev(keys)
            vd = _dev(vals) if pay else None
            tickets.append(srv.submit(kd, p, eps, dseed, vd, op=op))
            held.append((keys, vals, kd, vd))
        done = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert st["requests"] == len(reqs)
        assert st["batches"] >= ops.count("sort")
        for i, ((n, p, eps, kb, pay, dseed), op, r) in enumerate(zip(reqs, ops, done)):
            keys, vals, kd, vd = held[i]
            with hss.Plan(n, p, eps, key_bytes=kb, payload=pay) as plan:
                fn = plan.sort if op == "sort" else plan.partition
                ko, vo, off = fn(kd, dseed, vd)
                torch.cuda.synchronize()
                assert torch.equal(off, r.offsets), (i, op)
                assert torch.equal(ko, r.keys_out), (i, op)
                if pay:
                    assert torch.equal(vo, r.vals_out), (i, op)
            if op == "sort" and n < (1 << 17):
                ref = oracle.hss(keys, p, eps, dseed, vals=vals, mode="sort", trace_level=0)
                assert np.array_equal(r.offsets.cpu().numpy().view(np.uint64), ref.offsets), i
                kt = np.uint64 if kb == 8 else np.uint32
                assert np.array_equal(r.keys_out.cpu().numpy().view(kt), ref.keys), i
                if pay:
                    assert np.array_equal(r.vals_out.cpu().numpy().view(np.uint64), ref.vals), i


def test_batches_overlap_and_match_alone(hss):
    """Continuous batching: with several workers and a full queue, batches run
    at once on their streams; each result is still the one the request gets
    alone."""
    reqs = [(int(2 ** (14 + (i % 5))), 16 + (i % 7) * 8, 0.05, 8, i % 2 == 0, 8100 + i)
            for i in range(24)]
    with hss.Server(max_batch_requests=4, workers=3) as srv:
        tickets, held = [], []
        for (n, p, eps, kb, pay, dseed) in reqs:
            keys, vals = _inputs(n, kb, pay, dseed)
            held.append((_dev(keys), _dev(vals) if pay else None))
        torch.cuda.synchronize()
        for (n, p, eps, kb, pay, dseed), (kd, vd) in zip(reqs, held):
            tickets.append(srv.submit(kd, p, eps, dseed, vd, sync=False))
        done = [srv.wait(t) for t in tickets]
        st = srv.stats()
    _say(f"[server] overlap: {st}")
    assert st["requests"] == len(reqs)
    assert st["max_concurrent_batches"] >= 2
    for (n, p, eps, kb, pay, dseed), (kd, vd), r in zip(reqs, held, done):
        with hss.Plan(n, p, eps, key_bytes=kb, payload=pay) as plan:
            ko, vo, off = plan.partition(kd, dseed, vd)
            torch.cuda.synchronize()
            assert torch.equal(off, r.offsets) and torch.equal(ko, r.keys_out)
            if pay:
                assert torch.equal(vo, r.vals_out)


def test_budget_bounds_admission(hss):
    """The HBM budget bounds what runs at once: with room for two requests,
    no more than two are admitted together, whatever the workers."""
    n, p = 1 << 16, 32
    fp = hss.Server.footprint(n, p, 8, True)
    with hss.Server(workers=4, hbm_budget=2 * fp, max_batch_requests=1) as srv:
        tickets = []
        for i in range(12):
            keys, vals = _inputs(n, 8, True, 8200 + i)
            tickets.append((srv.submit(_dev(keys), p, 0.05, 40 + i, _dev(vals)), keys, vals, 40 + i))
        for t, keys, vals, seed in tickets:
            r = srv.wait(t)
            ref = oracle.hss(keys, p, 0.05, seed, vals=vals, mode="partition", trace_level=0)
            assert np.array_equal(r.vals_out.cpu().numpy().view(np.uint64), ref.vals)
        st = srv.stats()
    assert st["max_admitted_bytes"] <= 2 * fp
    assert st["max_concurrent_batches"] <= 2


def test_cache_stays_within_the_budget(hss):
    """After a stream of mixed sizes the device memory the server holds
    (blocks in use and idle) is within its HBM budget: idle blocks are freed,
    largest first, whenever the total would go over it."""
    budget = 192 << 20
    rng = np.random.default_rng(11)
    sizes = [int(2 ** rng.uniform(12, 21)) for _ in range(40)]
    _say(f"[server] cache budget {budget}: {len(sizes)} requests of 2^12..2^21 keys")
    checked = []
    with hss.Server(workers=2, hbm_budget=budget) as srv:
        for b0 in range(0, len(sizes), 8):   # in bursts, so that sizes mix in the cache
            burst = []
            for i in range(b0, min(b0 + 8, len(sizes))):
                n = sizes[i]
                keys, vals = _inputs(n, 8, True, 8600 + i)
                p = max(1, min(n, 64))
                burst.append((srv.submit(_dev(keys), p, 0.05, 90 + i, _dev(vals)), keys, vals, p, 90 + i))
            for t, keys, vals, p, seed in burst:
                r = srv.wait(t)
                if len(checked) < 4:
                    checked.append((r.vals_out.cpu().numpy().view(np.uint64), keys, vals, p, seed))
        mem = srv.memory()
        _say(f"[server] held {mem['held_bytes']} max {mem['max_held_bytes']}")
        assert 0 < mem["held_bytes"] <= budget
    for got, keys, vals, p, seed in checked:
        ref = oracle.hss(keys, p, 0.05, seed, vals=vals, mode="partition", trace_level=0)
        assert np.array_equal(got, ref.vals)


def test_batching_wait_gathers_a_lone_request(hss):
    """With a batching wait, a partition request queued alone waits for a
    second of its class (submitted 5 ms later, well inside the wait) and both
    run as one batch; a request that stays alone runs once its wait ends.
    Results equal the oracle."""
    _say("[server] batching wait")
    with hss.Server(workers=1, batch_wait_us=500_000) as srv:
        a = _inputs(40_000, 8, True, 1201)
        b = _inputs(30_000, 8, True, 1202)
        ta = srv.submit(_dev(a[0]), 16, 0.05, 21, _dev(a[1]))
        time.sleep(0.005)
        tb = srv.submit(_dev(b[0]), 16, 0.05, 22, _dev(b[1]))
        ra, rb = srv.wait(ta), srv.wait(tb)
        assert srv.stats()["batches"] == 1
        for (keys, vals), seed, r in ((a, 21, ra), (b, 22, rb)):
            ref = oracle.hss(keys, 16, 0.05, seed, vals=vals, mode="partition", trace_level=0)
            assert np.array_equal(r.offsets.cpu().numpy().view(np.uint64), ref.offsets)
            assert np.array_equal(r.keys_out.cpu().numpy().view(np.uint64), ref.keys)
            assert np.array_equal(r.vals_out.cpu().numpy().view(np.uint64), ref.vals)
        c, _ = _inputs(20_000, 8, False, 1203)
        rc = srv.wait(srv.submit(_dev(c), 8, 0.05, 23))
        assert rc.t_done - rc.t_submit >= 0.45
        assert srv.stats()["batches"] == 2
        ref = oracle.hss(c, 8, 0.05, 23, mode="partition", trace_level=0)
        assert np.array_equal(rc.keys_out.cpu().numpy().view(np.uint64), ref.keys)


def test_cancel_takes_a_queued_request_out(hss):
    """A request queued behind a running one is cancelled: waiting on it
    raises 'cancelled' and its output is untouched; the others complete and
    equal the oracle; a retired ticket is unknown to cancel."""
    _say("[server] cancel")
    with hss.Server(workers=1, max_batch_requests=1) as srv:
        big = synth.make("uniform64", 1 << 25, 1301)         # keeps the worker busy
        tb = srv.submit(_dev(big), 1024, 0.05, 31)
        small = [_inputs(20_000 + 1000 * i, 8, False, 1310 + i)[0] for i in range(3)]
        outs = [torch.zeros(len(k), dtype=torch.int64, device="cuda") for k in small]
        ts = [srv.submit(_dev(k), 8, 0.05, 40 + i, keys_out=o) for i, (k, o) in enumerate(zip(small, outs))]
        assert srv.cancel(ts[1]) is True
        srv.wait(tb)
        done = {i: srv.wait(ts[i]) for i in (0, 2)}
        with pytest.raises(hss.HssError) as err:
            srv.wait(ts[1])
        assert err.value.status == hss.HSS_ERR_CANCELLED
        assert int(outs[1].abs().sum()) == 0
        with pytest.raises(hss.HssError):
            srv.cancel(ts[1])                                 # retired
        for i, r in done.items():
            ref = oracle.hss(small[i], 8, 0.05, 40 + i, mode="partition", trace_level=0)
            assert np.array_equal(r.keys_out.cpu().numpy().view(np.uint64), ref.keys)
            assert np.array_equal(r.offsets.cpu().numpy().view(np.uint64), ref.offsets)
        # a request the idle worker has taken (running or done) is not cancelled
        t = srv.submit(_dev(small[0]), 8, 0.05, 40)
        time.sleep(0.05)
        assert srv.cancel(t) is False
        r = srv.wait(t)
        ref = oracle.hss(small[0], 8, 0.05, 40, mode="partition", trace_level=0)
        assert np.array_equal(r.keys_out.cpu().numpy().view(np.uint64), ref.keys)
