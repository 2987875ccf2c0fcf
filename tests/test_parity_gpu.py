"""GPU parity: libhss (through the C ABI) against the CPU oracle, bit-exact.

Every case prints what it runs before touching the device.  Small and medium
cases compare the whole round trace (probe sets, ranks, splitter state per
round), the splitters, the piece matrix and the outputs.  Full-size cases
(2^28 keys) check the outputs by properties that hold at any size and
compare sampled splitters with their definition.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import refcheck as R

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
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda()
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda()
    raise TypeError(a.dtype)


def _host(t, dtype):
    return t.cpu().numpy().view(dtype)


def _keys(kind, n, seed, bits):
    k = synth.make(kind, n, seed)
    if bits == 32:
        k = (k >> np.uint64(32)).astype(np.uint32) if kind in ("uniform64", "UNIF") else k.astype(np.uint32)
    return k


CASES = [
    # kind, n, p, eps, seed, bits, payload
    ("uniform64", 1 << 20, 16, 0.05, 1, 64, False),      # the small configuration
    ("uniform64", 1 << 16, 16, 0.05, 7, 64, True),
    ("uniform64", 100_003, 37, 0.02, 2, 64, True),       # ragged segments, several tiles
    ("uniform32", 300_001, 64, 0.1, 3, 32, True),
    ("uniform32", 65_536, 8, 0.05, 4, 32, False),
    ("SKEW1", 200_000, 32, 0.05, 4, 64, False),
    ("SKEW2", 200_000, 32, 0.05, 5, 64, True),           # 101 distinct keys
    ("SKEW3", 120_000, 20, 0.05, 6, 64, False),
    ("GAUSS", 120_000, 20, 0.05, 7, 64, False),
    ("ALLZEROS", 100_000, 25, 0.05, 8, 64, True),
    ("zipf_morton", 400_000, 128, 0.05, 9, 64, True),
    ("uniform64", 5000, 1, 0.05, 10, 64, True),          # p = 1
    ("uniform64", 300, 300, 0.5, 11, 64, True),          # p = N
    ("uniform64", 40_000, 9, 1e-6, 12, 64, False),       # tol = 0
    ("SKEW2", 33_333, 10, 0.003, 13, 64, True),          # tol = 0 with duplicates
    ("uniform64", 1 << 22, 256, 0.02, 14, 64, False),    # medium, k = 7
    ("uniform64", 1, 1, 0.5, 15, 64, True),              # a single key
    ("uniform64", 4097, 4096, 0.9, 16, 64, False),       # many tiny segments
    ("uniform32", 1 << 21, 64, 0.02, 17, 32, True),      # first draws taken ahead, u32
    # p = 4096 on clustered keys with a payload: 4096-key segments, duplicates
    # across hundreds of buckets, per-cell tables of 4097 x 4096 words
    ("zipf_morton", 1 << 24, 4096, 0.05, 18, 64, True),
]


def _compare_trace(plan, ref, p):
    tr = plan.trace()
    assert len(tr) == len(ref.rounds), (len(tr), len(ref.rounds))
    for j, (a, b) in enumerate(zip(tr, ref.rounds)):
        assert (a.domain, a.m, a.thresh, a.all) == (b.domain, b.m, b.thresh, b.all), j
        assert np.array_equal(a.probe_key, b.probe_key), j
        assert np.array_equal(a.probe_tag, b.probe_tag), j
        assert np.array_equal(a.probe_rank, b.probe_rank), j
        if a.counts is not None or b.counts is not None:
            assert np.array_equal(a.counts, b.counts), j
        assert np.array_equal(a.settled, b.settled), j
        assert np.array_equal(a.chi, b.chi), j
        assert np.array_equal(a.lo_rank, b.lo_rank), j
        assert np.array_equal(a.hi_rank, b.hi_rank), j


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-p{c[2]}-b{c[5]}" for c in CASES])
def test_partition_and_sort_match_oracle(hss, case):
    kind, n, p, eps, seed, bits, payload = case
    _say(f"[parity] {kind} n={n} p={p} eps={eps} seed={seed} bits={bits} payload={payload}")
    keys = _keys(kind, n, seed, bits)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    kt = keys.dtype
    with hss.Plan(n, p, eps, key_bytes=keys.itemsize, payload=payload, trace_level=2) as plan:
        # constants
        tol, k, a, th, al = plan.constants(40)
        oc = oracle.constants(n, p, eps, max_j=40)
        assert (tol, k, a) == (oc.tol, oc.k, oc.a)
        assert np.array_equal(th, oc.thresh) and np.array_equal(al, oc.all)
        # local sort
        lk, lv = plan.local_sort(kd, vd)
        ok_, ov_ = oracle.local_sort(keys, p, vals)
        assert np.array_equal(_host(lk, kt), ok_)
        if payload:
            assert np.array_equal(_host(lv, np.uint64), ov_)
        # partition
        ko, vo, off = plan.partition(kd, seed, vd)
        ref = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition", trace_level=2,
                         threads=ORACLE_THREADS)
        assert ref.status == 0
        assert np.array_equal(_host(off, np.uint64), ref.offsets)
        assert np.array_equal(_host(ko, kt), ref.keys)
        if payload:
            assert np.array_equal(_host(vo, np.uint64), ref.vals)
        _compare_trace(plan, ref, p)
        chi, sk, stg, pieces = plan.splitters()
        assert np.array_equal(chi, ref.chi)
        assert np.array_equal(sk[1:p], ref.s_key[1:p])
        assert np.array_equal(stg[1:p], ref.s_tag[1:p])
        assert np.array_equal(pieces, ref.pieces)
        # sort
        ks, vs, off2 = plan.sort(kd, seed, vd)
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(_host(ks, kt), keys[order])
        if payload:
            assert np.array_equal(_host(vs, np.uint64), vals[order])
        assert np.array_equal(_host(off2, np.uint64), ref.offsets)


OPTION_CASES = [
    # kind, n, p, eps, seed, bits, payload, k_override
    ("uniform64", 1 << 18, 64, 0.05, 21, 64, False, 1),   # one round (section 4.1)
    ("SKEW2", 100_000, 16, 0.05, 22, 64, True, 1),        # one round, duplicates
    ("uniform32", 50_000, 10, 10 / 50_000, 23, 32, False, 0),   # eps = p/N: exact
    ("GAUSS", 8192, 64, 64 / 8192, 24, 64, True, 0),      # exact, 5 rounds
    ("uniform64", 20_000, 10, 10 / 20_000, 25, 64, False, 1),   # exact with k = 1
    # first samples above 16384 probes: sorted by the segmented sort
    ("uniform64", 1 << 20, 64, 0.02, 26, 64, True, 1),
    ("SKEW2", 1 << 19, 128, 0.02, 27, 64, False, 1),
    ("uniform32", 1 << 19, 128, 0.02, 28, 32, False, 1),
]


@pytest.mark.parametrize("case", OPTION_CASES,
                         ids=[f"{c[0]}-{c[1]}-p{c[2]}-k{c[7]}" for c in OPTION_CASES])
def test_plan_options_match_oracle(hss, case):
    """One-round HSS (k = 1) and exact splitting (eps = p / N, tol = 0) are plan
    options on the same kernels; trace and outputs equal the oracle's."""
    kind, n, p, eps, seed, bits, payload, k = case
    _say(f"[parity] options {kind} n={n} p={p} eps={eps} k={k} payload={payload}")
    keys = _keys(kind, n, seed, bits)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    with hss.Plan(n, p, eps, key_bytes=keys.itemsize, payload=payload, trace_level=1,
                  k_override=k) as plan:
        tol, kk, a, th, al = plan.constants(40)
        oc = oracle.constants(n, p, eps, k_override=k, max_j=40)
        assert (tol, kk, a) == (oc.tol, oc.k, oc.a)
        assert np.array_equal(th, oc.thresh) and np.array_equal(al, oc.all)
        ko, vo, off = plan.partition(kd, seed, vd)
        ref = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition", k_override=k)
        assert ref.status == 0
        assert np.array_equal(_host(off, np.uint64), ref.offsets)
        assert np.array_equal(_host(ko, keys.dtype), ref.keys)
        if payload:
            assert np.array_equal(_host(vo, np.uint64), ref.vals)
        _compare_trace(plan, ref, p)
        if tol == 0:
            ideal = (np.arange(p + 1, dtype=np.uint64) * np.uint64(n)) // np.uint64(p)
            assert np.array_equal(_host(off, np.uint64), ideal)


BUDGET_CASES = [
    # kind, n, p, eps, seed, bits, payload, probes per processor per round
    ("uniform64", 1 << 18, 64, 0.02, 31, 64, False, 5),
    ("SKEW2", 100_000, 16, 0.05, 32, 64, True, 1),
    ("uniform32", 1 << 17, 32, 0.02, 33, 32, True, 3),
    ("GAUSS", 1 << 16, 128, 0.05, 34, 64, False, 1),
    ("uniform64", 1 << 20, 64, 0.02, 35, 64, True, 5),    # round 1's draws taken ahead
]


@pytest.mark.parametrize("case", BUDGET_CASES,
                         ids=[f"{c[0]}-{c[1]}-p{c[2]}-c{c[7]}" for c in BUDGET_CASES])
def test_probe_budget_matches_oracle(hss, case):
    """The fixed probe budget: each round's rate is set on the device from
    the domain it measured; trace and outputs equal the oracle's."""
    kind, n, p, eps, seed, bits, payload, c = case
    _say(f"[parity] budget {kind} n={n} p={p} eps={eps} c={c} payload={payload}")
    keys = _keys(kind, n, seed, bits)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    with hss.Plan(n, p, eps, key_bytes=keys.itemsize, payload=payload, trace_level=1,
                  probes_per_round=c) as plan:
        ref = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition", probes_per_round=c)
        assert ref.status == 0
        for call in range(2):   # the second call rewrites the device rates
            ko, vo, off = plan.partition(kd, seed, vd)
            assert np.array_equal(_host(off, np.uint64), ref.offsets), call
            assert np.array_equal(_host(ko, keys.dtype), ref.keys), call
            if payload:
                assert np.array_equal(_host(vo, np.uint64), ref.vals), call
            _compare_trace(plan, ref, p)


def test_force_full_sample_exact_splitters(hss):
    n, p = 50_000, 13
    _say(f"[parity] force_full_sample n={n} p={p}")
    keys = synth.make("SKEW2", n, 3)
    with hss.Plan(n, p, 0.05, trace_level=1, force_full_sample=True) as plan:
        ko, _, off = plan.partition(_dev(keys), 1)
        assert [int(x) for x in _host(off, np.uint64)] == list(R.ideal(n, p))
        ref = oracle.hss(keys, p, 0.05, 1, force_full_sample=True)
        assert np.array_equal(_host(ko, np.uint64), ref.keys)
        _compare_trace(plan, ref, p)


def test_round_cap_reports_not_converged(hss):
    n, p = 1 << 16, 64
    _say(f"[parity] max_rounds=1 n={n} p={p}")
    keys = synth.make("uniform64", n, 3)
    with hss.Plan(n, p, 0.01, max_rounds=1) as plan:
        with pytest.raises(hss.HssError) as ei:
            plan.partition(_dev(keys), 3)
        assert ei.value.status == -5
    assert oracle.hss(keys, p, 0.01, 3, max_rounds=1).status == -5


def test_rejects_misaligned_and_overlapping_pointers(hss):
    n, p = 4096, 4
    _say("[parity] argument checks")
    keys = _dev(synth.make("uniform64", n + 2, 3))
    with hss.Plan(n, p, 0.1) as plan:
        with pytest.raises(hss.HssError):      # outputs overlap the input
            hss._check(hss._lib.hss_partition(plan._h, 1, keys.data_ptr(), None,
                                              keys.data_ptr(), None,
                                              torch.empty(p + 1, dtype=torch.int64,
                                                          device="cuda").data_ptr(), None),
                       "overlap")
        out = torch.empty(n + 2, dtype=torch.int64, device="cuda")
        with pytest.raises(hss.HssError):      # misaligned output
            hss._check(hss._lib.hss_partition(plan._h, 1, keys.data_ptr(), None,
                                              out.data_ptr() + 8, None,
                                              torch.empty(p + 1, dtype=torch.int64,
                                                          device="cuda").data_ptr(), None),
                       "misaligned")


def test_plan_reuse_and_seeds(hss):
    """One plan, several seeds and inputs in a row: each call equals a fresh oracle run."""
    n, p, eps = 200_000, 50, 0.03
    with hss.Plan(n, p, eps, payload=True, trace_level=0) as plan:
        for seed in (1, 2, 3):
            _say(f"[parity] reuse seed={seed}")
            keys = synth.make("uniform64", n, 40 + seed)
            vals = np.arange(n, dtype=np.uint64)
            ko, vo, off = plan.partition(_dev(keys), seed, _dev(vals))
            ref = oracle.hss(keys, p, eps, seed, vals=vals, trace_level=0)
            assert np.array_equal(_host(off, np.uint64), ref.offsets)
            assert np.array_equal(_host(ko, np.uint64), ref.keys)
            assert np.array_equal(_host(vo, np.uint64), ref.vals)
            assert len(plan.trace()) == len(ref.rounds)


SORT_CASES = [
    # kind, n, p, note
    ("uniform64", 1 << 20, 64, "on-chip fast path"),
    ("SKEW2", 100_000, 64, "segments <= cap, one big group: LDS slow path"),
    ("SKEW2", 300_000, 16, "top byte constant: HBM fallback"),
    ("ALLZEROS", 50_000, 7, "all equal"),
    ("GAUSS", 60_000, 40, "few top bytes"),
    ("SKEW3", 90_000, 30, "biased bits"),
    ("zipf_morton", 500_000, 64, "mixed"),
    ("uniform32", 1 << 18, 32, "32-bit keys"),
]


@pytest.mark.parametrize("lsd_only", [False, True])
@pytest.mark.parametrize("case", SORT_CASES, ids=[c[3] for c in SORT_CASES])
def test_local_sort_paths(hss, case, lsd_only):
    kind, n, p, _ = case
    _say(f"[local sort] {kind} n={n} p={p} lsd_only={lsd_only}")
    keys = synth.make(kind, n, 21)
    if kind == "uniform32":
        keys = keys.astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64)
    with hss.Plan(n, p, 0.05, key_bytes=keys.itemsize, payload=True, lsd_only=lsd_only) as plan:
        lk, lv = plan.local_sort(_dev(keys), _dev(vals))
        ok_, ov_ = oracle.local_sort(keys, p, vals)
        assert np.array_equal(_host(lk, keys.dtype), ok_)
        assert np.array_equal(_host(lv, np.uint64), ov_)
        ks, vs, _ = plan.sort(_dev(keys), 5, _dev(vals))
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(_host(ks, keys.dtype), keys[order])
        assert np.array_equal(_host(vs, np.uint64), vals[order])


@pytest.mark.parametrize("size", [2047, 2048, 2049, 3071, 3072, 3073, 4096, 33, 32])
def test_local_sort_sub_bucket_boundaries(hss, size):
    """One segment whose top byte puts exactly `size` keys in one sub-bucket,
    with the rest spread out; duplicates inside the sub-bucket."""
    rng = np.random.default_rng(size)
    n, p = 1 << 15, 4
    keys = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    seg = n // p
    # no other key of segment 0 in the hot sub-bucket
    top = keys[:seg] >> np.uint64(56)
    keys[:seg][top == np.uint64(0xAB)] ^= np.uint64(1 << 56)
    idx = rng.choice(seg, size=size, replace=False)
    # hot keys share the top two bytes: one sub-bucket, one group, duplicates
    hot = (np.uint64(0xAB) << np.uint64(56)) | rng.integers(0, 1 << 10, size=size, dtype=np.uint64)
    keys[idx] = hot
    vals = np.arange(n, dtype=np.uint64)
    _say(f"[local sort] sub-bucket of {size} keys")
    with hss.Plan(n, p, 0.05, payload=True) as plan:
        lk, lv = plan.local_sort(_dev(keys), _dev(vals))
        ok_, ov_ = oracle.local_sort(keys, p, vals)
        assert np.array_equal(_host(lk, np.uint64), ok_)
        assert np.array_equal(_host(lv, np.uint64), ov_)


@pytest.mark.parametrize("n,p", [(1 << 22, 16), (1 << 21, 8), (1 << 23, 1024)])
def test_local_sort_large_segments(hss, n, p):
    """Segments of 2^18 keys: sub-buckets of about 1024 keys, as at full size."""
    _say(f"[local sort] uniform n={n} p={p}")
    keys = synth.uniform64(n, 77)
    with hss.Plan(n, p, 0.02) as plan:
        lk, _ = plan.local_sort(_dev(keys))
        ok_, _ = oracle.local_sort(keys, p)
        got = _host(lk, np.uint64)
        bad = np.nonzero(got != ok_)[0]
        assert len(bad) == 0, (len(bad), bad[:10])


@pytest.mark.parametrize("n,p,eps", [(1 << 22, 16, 0.02), (1 << 23, 1024, 0.02)])
def test_partition_large_segments(hss, n, p, eps):
    _say(f"[parity] uniform n={n} p={p} eps={eps}")
    keys = synth.uniform64(n, 78)
    with hss.Plan(n, p, eps, trace_level=1) as plan:
        ko, _, off = plan.partition(_dev(keys), 5)
        ref = oracle.hss(keys, p, eps, 5)
        _compare_trace(plan, ref, p)
        assert np.array_equal(_host(off, np.uint64), ref.offsets)
        assert np.array_equal(_host(ko, np.uint64), ref.keys)


@pytest.mark.parametrize("centre_bit", [56, 63, 40, 8])
def test_sort_buckets_straddling_power_of_two(hss, centre_bit):
    """Keys packed around 2^centre_bit: bucket key ranges cross a power of two,
    so the bucket sort must take digits of key - bucket base, not raw bits."""
    n, p = 300_000, 8
    rng = np.random.default_rng(centre_bit)
    c = np.uint64(1) << np.uint64(centre_bit)
    half = np.uint64(min(1 << 20, (1 << centre_bit) - 1))
    keys = c - half + rng.integers(0, 2 * int(half), size=n, dtype=np.uint64)
    keys[::7] = keys[::7] & ~np.uint64(0xFF)           # duplicates
    vals = np.arange(n, dtype=np.uint64)
    _say(f"[sort] keys around 2^{centre_bit}")
    with hss.Plan(n, p, 0.05, payload=True) as plan:
        ks, vs, off = plan.sort(_dev(keys), 9, _dev(vals))
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(_host(ks, np.uint64), keys[order])
        assert np.array_equal(_host(vs, np.uint64), vals[order])
        ref = oracle.hss(keys, p, 0.05, 9, vals=vals, mode="sort")
        assert np.array_equal(_host(off, np.uint64), ref.offsets)


def test_graph_replays_match_plain_launches(hss):
    """The first rounds run from a captured graph; replayed call after call,
    with other device work and synchronisations in between and after the
    probe buffers grew, every call equals the same call with plain launches
    (and the oracle)."""
    n, p, eps = 1 << 18, 64, 0.02
    _say("[parity] graph replays against plain launches")
    with hss.Plan(n, p, eps) as g, hss.Plan(n, p, eps, plain_launches=True) as f:
        for call in range(6):
            keys = _keys("uniform64" if call % 3 else "SKEW1", n, 50 + call, 64)
            kd = _dev(keys)
            junk = torch.randn(1 << 20, device="cuda").cumsum(0)   # unrelated eager work
            ko, _, off = g.partition(kd, 70 + call)
            torch.cuda.synchronize()
            ko2, _, off2 = f.partition(kd, 70 + call)
            torch.cuda.synchronize()
            assert torch.equal(off, off2) and torch.equal(ko, ko2), call
            if call in (0, 5):
                ref = oracle.hss(keys, p, eps, 70 + call, mode="partition", trace_level=0)
                assert np.array_equal(_host(off, np.uint64), ref.offsets), call
            del junk


KNOB_SETTINGS = [
    {},
    {"small_sort_cap": 4096},
    {"sample_workgroups": 4096},
    {"pair_rank_from": 1},                 # round 1 searched per pair as well
    {"pair_rank_from": 64},                # every round by segment chunks
    {"pair_rank_workgroups": 2048, "sample_workgroups": 8192, "small_sort_cap": 4096},
]


@pytest.mark.parametrize("kind,n,p,bits,payload", [("uniform64", 1 << 20, 64, 64, False),
                                                   ("SKEW1", 1 << 19, 16, 64, True),
                                                   ("uniform32", 300_001, 37, 32, True)])
def test_every_knob_setting_matches_oracle(hss, kind, n, p, bits, payload):
    """The launch knobs change no output: every setting equals the oracle,
    trace included."""
    eps, seed = 0.02, 44
    keys = _keys(kind, n, seed, bits)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    kd, vd = _dev(keys), (None if vals is None else _dev(vals))
    ref = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition")
    with hss.Plan(n, p, eps, key_bytes=keys.itemsize, payload=payload, trace_level=1) as plan:
        base = plan.knobs()
        for k in KNOB_SETTINGS:
            _say(f"[parity] knobs {kind} {k}")
            plan.set_knobs(**{**base, **k})
            ko, vo, off = plan.partition(kd, seed, vd)
            assert np.array_equal(_host(off, np.uint64), ref.offsets), k
            assert np.array_equal(_host(ko, keys.dtype), ref.keys), k
            if payload:
                assert np.array_equal(_host(vo, np.uint64), ref.vals), k
            _compare_trace(plan, ref, p)
        with pytest.raises(hss.HssError):
            plan.set_knobs(small_sort_cap=3000)


def test_autotuned_plan_and_batch(hss):
    """The first call of an autotuned plan searches the knobs on its input
    and still returns the oracle's result; later calls run with the choice."""
    n, p, eps = 1 << 20, 128, 0.02
    keys = _keys("uniform64", n, 45, 64)
    ref = oracle.hss(keys, p, eps, 9, mode="partition", trace_level=0)
    with hss.Plan(n, p, eps, autotune=True) as plan:
        assert plan.knobs()["tuned"] == 0
        for call in range(2):
            ko, _, off = plan.partition(_dev(keys), 9)
            assert np.array_equal(_host(off, np.uint64), ref.offsets), call
            assert np.array_equal(_host(ko, np.uint64), ref.keys), call
        k = plan.knobs()
        _say(f"[parity] autotuned knobs {k}")
        assert k["tuned"] == 1 and k["small_sort_cap"] in (2048, 4096)
    shapes = [(70_000, 16, 0.05, 8), (123_457, 37, 0.05, 8), (5000, 8, 0.05, 8)]
    ks = [_keys("uniform64", s[0], 60 + i, 64) for i, s in enumerate(shapes)]
    with hss.BatchPlan(shapes, autotune=True) as bp:
        ko, _, off = bp.partition([_dev(k) for k in ks], [3, 4, 5])
        for i, (nn, pp, ee, _) in enumerate(shapes):
            r = oracle.hss(ks[i], pp, ee, 3 + i, mode="partition", trace_level=0)
            assert np.array_equal(_host(off[i], np.uint64), r.offsets), i
            assert np.array_equal(_host(ko[i], np.uint64), r.keys), i
        assert bp.knobs(8)["tuned"] == 1


def _random_plan_shapes(seed, count):
    rng = np.random.default_rng(seed)
    kinds = ["uniform64", "SKEW1", "SKEW2", "SKEW3", "GAUSS", "zipf_morton", "ALLZEROS"]
    out = []
    for i in range(count):
        n = int(2 ** rng.uniform(8, 21))
        p = int(min(n, 2 ** rng.uniform(0, 12.5)))
        out.append((kinds[int(rng.integers(0, len(kinds)))], n, max(p, 1),
                    float(rng.choice([0.005, 0.02, 0.1, 0.5])), 32 if rng.random() < 0.3 else 64,
                    bool(rng.random() < 0.5), 300 + i))
    return out


@pytest.mark.parametrize("case", _random_plan_shapes(11, 32), ids=lambda c: f"{c[0]}-{c[1]}-p{c[2]}-b{c[4]}")
def test_random_plans_match_oracle(hss, case):
    """Random shapes across the local sort's paths (tiny and large segments,
    packed first-level jobs, narrow digits, duplicates): partition and sort
    equal the oracle bit for bit."""
    kind, n, p, eps, bits, payload, seed = case
    _say(f"[random-plan] {case}")
    keys = _keys(kind, n, seed, bits)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    ref = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition", trace_level=0)
    srt = oracle.hss(keys, p, eps, seed, vals=vals, mode="sort", trace_level=0)
    assert ref.status == 0 and srt.status == 0
    with hss.Plan(n, p, eps, key_bytes=keys.itemsize, payload=payload) as plan:
        ko, vo, off = plan.partition(kd, seed, vd)
        assert np.array_equal(_host(off, np.uint64), ref.offsets)
        assert np.array_equal(_host(ko, keys.dtype), ref.keys)
        if payload:
            assert np.array_equal(_host(vo, np.uint64), ref.vals)
        ks, vs, _ = plan.sort(kd, seed, vd)
        assert np.array_equal(_host(ks, keys.dtype), srt.keys)
        if payload:
            assert np.array_equal(_host(vs, np.uint64), srt.vals)


def test_workspace_limit_admits_a_plan_that_fits(hss):
    """A plan under its workspace limit runs as without one (same outputs)."""
    import re
    n, p, eps, seed = 1 << 20, 16, 0.05, 3
    _say(f"[parity] workspace limit n={n} p={p}")
    with pytest.raises(hss.HssError) as ei:
        hss.Plan(n, p, eps, workspace_limit_mib=1)
    need = int(re.search(r"needs (\d+) bytes", str(ei.value)).group(1))
    keys = _keys("uniform64", n, 41, 64)
    kd = _dev(keys)
    with hss.Plan(n, p, eps, workspace_limit_mib=(need >> 20) + 1) as plan:
        ko, _, off = plan.partition(kd, seed)
        assert plan.workspace_bytes <= need + (1 << 20)
        with hss.Plan(n, p, eps) as ref:
            rk, _, roff = ref.partition(kd, seed)
        assert torch.equal(off, roff) and torch.equal(ko, rk)


PICK_CASES = [
    # kind, n, p, eps, seed, bits, payload, picks per segment per round in expectation
    ("uniform64", 1 << 18, 64, 0.02, 51, 64, False, 5),
    ("SKEW2", 100_000, 16, 0.05, 52, 64, True, 1),       # duplicates, many picked twice
    ("uniform32", 1 << 17, 32, 0.02, 53, 32, True, 3),
    ("zipf_morton", 1 << 21, 256, 0.05, 54, 64, True, 5),
    ("uniform64", 1 << 22, 1024, 0.02, 55, 64, False, 5),
]


@pytest.mark.parametrize("case", PICK_CASES, ids=[f"{c[0]}-{c[1]}-p{c[2]}-c{c[7]}" for c in PICK_CASES])
def test_pick_sampler_matches_oracle(hss, case):
    """Section 6's sampler (picks of the whole segment, those outside the
    intervals discarded): every round's picks, probes, ranks, local
    histograms and splitter state, and the outputs, equal the oracle's; a
    second call on the same plan as well (the pick bits are cleared)."""
    kind, n, p, eps, seed, bits, payload, c = case
    _say(f"[parity] picks {kind} n={n} p={p} eps={eps} c={c} payload={payload}")
    keys = _keys(kind, n, seed, bits)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    ref = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition", probes_per_round=c,
                     pick_sampler=True, trace_level=2, threads=ORACLE_THREADS)
    assert ref.status == 0
    for trace in (2, 0):
        with hss.Plan(n, p, eps, key_bytes=keys.itemsize, payload=payload, trace_level=trace,
                      probes_per_round=c, pick_sampler=True) as plan:
            for call in range(2):
                ko, vo, off = plan.partition(kd, seed, vd)
                assert np.array_equal(_host(off, np.uint64), ref.offsets), (trace, call)
                assert np.array_equal(_host(ko, keys.dtype), ref.keys), (trace, call)
                if payload:
                    assert np.array_equal(_host(vo, np.uint64), ref.vals), (trace, call)
                if trace:
                    _compare_trace(plan, ref, p)
                else:
                    tr = plan.trace()
                    assert [(a.domain, a.m, a.thresh, a.all) for a in tr] == \
                        [(b.domain, b.m, b.thresh, b.all) for b in ref.rounds]


def test_rounds_queued_ahead_of_the_exchange(hss):
    """A plain partition queues the k - 1 rounds that usually settle every
    splitter and its exchange behind them with no read-back in between; the
    exchange runs only if they did, and the closing read-back goes on with the
    rounds and exchanges again otherwise.  Over 24 seeds (5 of which take a
    k-th round in the oracle) outputs, offsets, splitters and the per-round
    counts must equal the oracle's, through both paths."""
    n, p, eps = 1 << 18, 64, 0.05
    _say(f"[parity] rounds queued ahead: uniform64 n={n} p={p} eps={eps}, seeds 1000..1023")
    keys = _keys("uniform64", n, 9, 64)
    kd = _dev(keys)
    longer = 0
    with hss.Plan(n, p, eps) as plan:
        k = plan.constants(1)[1]
        for seed in range(1000, 1024):
            ref = oracle.hss(keys, p, eps, seed, mode="partition", trace_level=0)
            assert ref.status == 0
            ko, _, off = plan.partition(kd, seed)
            assert np.array_equal(_host(off, np.uint64), ref.offsets), seed
            assert np.array_equal(_host(ko, np.uint64), ref.keys), seed
            chi = plan.splitters()[0]
            assert np.array_equal(chi, ref.chi), seed
            tr = plan.trace()
            assert [(r.domain, r.m) for r in tr] == [(r.domain, r.m) for r in ref.rounds], seed
            longer += len(ref.rounds) > k - 1
    _say(f"[parity] rounds queued ahead: {longer} of 24 seeds needed more than k - 1 = {k - 1} rounds")
    assert longer > 0


def test_partition_in_caller_workspace(hss):
    """hss_partition_ws: the partition in the caller's device workspace, at a
    shape above the fixed array's limits and again, smaller and with a payload,
    in the same workspace; no device memory taken by the library on the
    second call; a workspace below the shape's size is refused before any
    device work."""
    _say("[parity] caller workspace")
    n, p = 1 << 22, 1024
    keys = synth.uniform64(n, 91)
    need = hss.workspace_bytes(n, p, 0.02)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    ko, _, off = hss.partition_ws(_dev(keys), p, 0.02, 7, ws)
    ref = oracle.hss(keys, p, 0.02, 7, mode="partition", trace_level=0)
    assert np.array_equal(_host(off, np.uint64), ref.offsets)
    assert np.array_equal(_host(ko, np.uint64), ref.keys)
    # a smaller shape with a payload, in the same workspace
    n2, p2 = 200_003, 64
    k2 = synth.uniform64(n2, 92)
    v2 = np.arange(n2, dtype=np.uint64)
    assert hss.workspace_bytes(n2, p2, 0.05, payload=True) <= need
    kd, vd = _dev(k2), _dev(v2)
    ko2, vo2 = torch.empty_like(kd), torch.empty_like(vd)
    off2 = torch.empty(p2 + 1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    hss.partition_ws(kd, p2, 0.05, 8, ws, vals=vd, keys_out=ko2, vals_out=vo2, offsets=off2)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    ref2 = oracle.hss(k2, p2, 0.05, 8, vals=v2, mode="partition", trace_level=0)
    assert np.array_equal(_host(off2, np.uint64), ref2.offsets)
    assert np.array_equal(_host(ko2, np.uint64), ref2.keys)
    assert np.array_equal(_host(vo2, np.uint64), ref2.vals)
    # too small: refused on the host, outputs untouched
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    with pytest.raises(hss.HssError):
        hss.partition_ws(_dev(keys), p, 0.02, 7, ws[: need // 2], keys_out=out)
    assert int(out.abs().sum()) == 0
