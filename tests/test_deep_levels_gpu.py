"""GPU parity of the local sort's deeper MSD levels against the oracle.

Inputs are built to reach each path of the hybrid sort with segments far above
the on-chip capacity: segments whose top digit holds every key (all equal, or
varying only in low bits), clusters that stay above the capacity for two more
levels (so one level sorts in place in the output), clustered duplicates
that end in the slow path (an on-chip sample sort) from an in-place level, and
segments of at most 2048 keys whose 64 sampled places all hold one value, so
that the sample sort is left with one class of almost every key to rank.
Keys from the top sixth of a Zipf-Morton draw (few heavy values near the
largest key) take splitters at the first level and again below it, where the
last class of an entry ends at the largest key of the key width.
Local sort, partition and sort must equal the oracle bit for bit, keys alone
and with a payload.
"""
import sys

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


def _dev(a):
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda()
    return torch.from_numpy(a.view(np.int32)).cuda()


def _host(t, dtype):
    return t.cpu().numpy().view(dtype)


def _keys(kind, n, seed, bits, p):
    rng = np.random.default_rng(seed)
    top = np.uint64(1) << np.uint64(bits - 1)
    if kind == "planted_samples":    # top bits agree; the sampled places of every segment hold 7
        # (the slow path samples stratum j of 64 at offset (37 j + 11) mod 64 of 64)
        k = top + rng.integers(0, 1 << (bits - 12), n).astype(np.uint64)
        j = np.arange(64)
        for s in range(p):
            a, b = s * n // p, (s + 1) * n // p
            k[a + (((64 * j + ((37 * j + 11) & 63)) * (b - a)) >> 12)] = 7
    elif kind == "narrow_gauss":       # around 0.7 2^b, sigma 2^(b-24): the top bits agree
        sig = 2.0 ** (bits - 24)
        k = (0.7 * 2.0 ** bits + rng.normal(0.0, sig, n)).astype(np.uint64)
    elif kind == "clustered_dups":   # 3000 values 2^(b-13) apart, ~n/3000 copies each
        step = np.uint64(1) << np.uint64(bits - 13)
        k = top + rng.integers(0, 3000, n).astype(np.uint64) * step
    elif kind == "top_zipf":         # the largest sixth of 6 n Zipf-Morton keys, shuffled
        k = synth.make("zipf_morton", 6 * n, seed)
        k = np.sort(k)[-n:]
        if bits == 32:
            k = k >> np.uint64(32)
        k = k[rng.permutation(n)]
    elif kind == "low7":             # only the lowest 7 bits vary
        k = rng.integers(0, 101, n).astype(np.uint64)
    else:
        k = synth.make(kind, n, seed)
        if bits == 32 and kind not in ("ALLZEROS", "SKEW2"):
            k = k >> np.uint64(32)
    return k.astype(np.uint32) if bits == 32 else k


CASES = [
    # kind, n, p, bits, payload
    ("ALLZEROS", 1 << 21, 4, 64, False),       # every segment equal: copied whole
    ("ALLZEROS", 1 << 20, 2, 32, True),
    ("low7", 1 << 21, 4, 64, True),            # top digit uniform; retried on 7 bits
    ("low7", 1 << 20, 8, 32, False),
    ("narrow_gauss", 1 << 22, 4, 64, True),    # retry, then two deeper levels
    ("narrow_gauss", 1 << 21, 4, 32, False),
    ("GAUSS", 1 << 22, 4, 64, False),          # central sub-buckets sorted in place
    ("GAUSS", 1 << 21, 4, 64, True),
    ("clustered_dups", 1 << 22, 4, 64, True),  # slow list from an in-place level
    ("clustered_dups", 1 << 21, 4, 32, False),
    ("SKEW1", 1 << 21, 4, 64, True),           # half the keys in a 1000-wide range
    ("low7", 200_000, 32, 64, False),          # many small entries, 101 sub-buckets each
    ("clustered_dups", 300_000, 16, 64, True),
    ("SKEW1", 400_000, 16, 32, False),
    ("planted_samples", 2048 * 8, 8, 64, True),   # sample sort: one class of 1984 keys
    ("planted_samples", 1500 * 16, 16, 32, False),
    ("top_zipf", 320_000, 4, 64, True),        # splitter classes up to the largest key
    ("top_zipf", 320_000, 4, 32, True),
    ("top_zipf", 1 << 20, 16, 64, False),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-p{c[2]}-b{c[3]}-pay{int(c[4])}" for c in CASES])
def test_deep_levels_match_oracle(hss, case):
    kind, n, p, bits, payload = case
    seed = 31
    _say(f"[deep] {kind} n={n} p={p} bits={bits} payload={payload}")
    keys = _keys(kind, n, seed, bits, p)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    kd = _dev(keys)
    vd = None if vals is None else _dev(vals)
    kt = keys.dtype
    with hss.Plan(n, p, 0.05, key_bytes=keys.itemsize, payload=payload) as plan:
        lk, lv = plan.local_sort(kd, vd)
        ok_, ov_ = oracle.local_sort(keys, p, vals)
        assert np.array_equal(_host(lk, kt), ok_)
        if payload:
            assert np.array_equal(_host(lv, np.uint64), ov_)
        ko, vo, off = plan.partition(kd, 5, vd)
        ref = oracle.hss(keys, p, 0.05, 5, vals=vals, mode="partition", trace_level=0)
        assert ref.status == 0
        assert np.array_equal(_host(off, np.uint64), ref.offsets)
        assert np.array_equal(_host(ko, kt), ref.keys)
        if payload:
            assert np.array_equal(_host(vo, np.uint64), ref.vals)
        ks, vs, off2 = plan.sort(kd, 5, vd)
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(_host(ks, kt), keys[order])
        if payload:
            assert np.array_equal(_host(vs, np.uint64), vals[order])
        assert np.array_equal(_host(off2, np.uint64), ref.offsets)
