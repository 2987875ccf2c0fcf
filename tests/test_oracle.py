"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses numpy's stable
sort (the closed form of a sort), brute-force counting, rocRAND's Philox, a
special case with a known answer, or an invariant the paper states.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests import refcheck as R

U64 = np.uint64


def _keys(kind, n, seed, bits=64):
    k = synth.make(kind, n, seed)
    return k if bits == 64 else (k >> U64(32)).astype(np.uint32)


# ---------------------------------------------------------------- Philox ----

def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(7)
    seeds = [0, 1, 2, 0xFFFFFFFF, 1 << 32, (1 << 64) - 1] + [int(x) for x in rng.integers(0, 2**63, 20)]
    js = [1, 2, 3, 7, 14, 1 << 20]
    gs = [0, 1, 2, 3, 4, 5, 1023, 1 << 20, (1 << 34) + 3, (1 << 40) + 2]
    S, J, G = [], [], []
    for s in seeds:
        for j in js:
            for g in gs:
                S.append(s); J.append(j); G.append(g)
    ref = rocrand_philox(S, J, G)
    got = [oracle.philox_word(s, g, j) for s, j, g in zip(S, J, G)]
    assert got == ref


def test_philox_block_words_are_distinct_words():
    # word g & 3 of one block: four consecutive tags share one counter
    blk = oracle.philox4x32_10([5, 0, 3, 0], [9, 0])
    assert [oracle.philox_word(9, 20 + w, 3) for w in range(4)] == [int(x) for x in blk]


# ------------------------------------------------------------- constants ----

@pytest.mark.parametrize("n,p,eps", [(1 << 20, 16, 0.05), (1 << 28, 1024, 0.02),
                                     (1 << 28, 4096, 0.05), (1000, 7, 0.3), (12345, 100, 0.9),
                                     (64, 64, 0.5), (1 << 40, 1 << 20, 0.01)])
def test_constants_closed_forms(n, p, eps):
    c = oracle.constants(n, p, eps)
    # target range half-width: tol <= N eps / (2p) < tol + 1 (section 2)
    x = Fraction(n) * Fraction(eps) / (2 * p)
    assert c.tol <= x < c.tol + 1
    # final ratio s_k = 2 ln p / eps (lemma on the k-th round)
    assert c.a == pytest.approx(2 * math.log(p) / eps, rel=1e-15)
    # k = ceil(ln a): e^(k-1) < a <= e^k, at least one round
    if c.a > math.e:
        assert math.exp(c.k - 1) < c.a <= math.exp(c.k) * (1 + 1e-12)
    else:
        assert c.k == 1
    # per-round acceptance probability p s_j / N with s_j = a^(j/k) (section 4.2)
    for j in range(1, 40):
        q = p * c.a ** (j / c.k) / n
        if q >= 1:
            assert c.all[j - 1] == 1
        else:
            assert c.all[j - 1] == 0
            assert abs(c.thresh[j - 1] / 2**32 - q) <= 2**-32 + q * 1e-12
    # thresholds grow round over round by the ratio a^(1/k)
    th = [int(t) for t, a in zip(c.thresh, c.all) if not a]
    assert all(x <= y for x, y in zip(th, th[1:]))
    if len(th) >= 3 and th[1] > 1 << 16:
        assert th[2] / th[1] == pytest.approx(c.a ** (1 / c.k), rel=1e-4)


def test_constants_one_round_rate():
    # k = 1 is the one-round method of section 4.1: rate 2 p ln p / (eps N)
    n, p, eps = 1 << 26, 512, 0.05
    c = oracle.constants(n, p, eps, k_override=1)
    assert c.k == 1
    assert c.thresh[0] / 2**32 == pytest.approx(2 * p * math.log(p) / (eps * n), abs=2**-32)


def test_constants_section7_worked_numbers():
    # Section 7.2: with p = 2048 and eps = 2%, 2p max(1/eps, log p) is about 100 p.
    p, eps = 2048, 0.02
    assert 2 * p * max(1 / eps, math.log2(p)) == pytest.approx(100 * p)
    # and the final HSS ratio 2 ln p / eps for that run
    c = oracle.constants(2048 * 1_000_000, p, eps)
    assert c.a == pytest.approx(2 * math.log(2048) / 0.02)
    # section 4.1: (p-1)/p^2 < 1/p
    assert (p - 1) / p**2 < 1 / p


# ------------------------------------------------------------ local sort ----

@pytest.mark.parametrize("kind,bits", [("uniform64", 64), ("SKEW2", 64), ("uniform32", 32),
                                       ("ALLZEROS", 64), ("zipf_morton", 64)])
@pytest.mark.parametrize("n,p", [(1000, 7), (4096, 16), (513, 512)])
def test_local_sort_is_stable_sort_per_segment(kind, bits, n, p):
    keys = synth.make(kind, n, 11)
    if bits == 32:
        keys = keys.astype(np.uint32) if kind == "uniform32" else (keys & U64(0xFFFF)).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64) * U64(3)
    ko, vo = oracle.local_sort(keys, p, vals)
    lo = R.local_order(keys, p)
    assert np.array_equal(ko, keys[lo])
    assert np.array_equal(vo, vals[lo])


# ------------------------------------------------- whole-method outputs ----

CASES = [
    # kind, n, p, eps, seed, bits, payload
    ("uniform64", 1 << 16, 16, 0.05, 1, 64, False),
    ("uniform64", 50_000, 37, 0.02, 2, 64, True),
    ("uniform32", 30_001, 64, 0.1, 3, 32, True),
    ("SKEW1", 20_000, 32, 0.05, 4, 64, False),
    ("SKEW2", 20_000, 32, 0.05, 5, 64, True),
    ("SKEW3", 20_000, 20, 0.05, 6, 64, False),
    ("GAUSS", 20_000, 20, 0.05, 7, 64, False),
    ("ALLZEROS", 10_000, 25, 0.05, 8, 64, True),
    ("zipf_morton", 40_000, 128, 0.05, 9, 64, True),
    ("uniform64", 5000, 1, 0.05, 10, 64, True),       # p = 1: one segment, no rounds
    ("uniform64", 300, 300, 0.5, 11, 64, True),       # p = N
    ("uniform64", 4000, 9, 1e-6, 12, 64, False),      # tol = 0: exact splitting
    ("SKEW2", 3333, 10, 0.003, 13, 64, True),         # tol = 0 with duplicates
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[2]}" for c in CASES])
def test_sort_equals_stable_sort(case):
    kind, n, p, eps, seed, bits, payload = case
    keys = synth.make(kind, n, seed)
    if bits == 32:
        keys = keys.astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    r = oracle.hss(keys, p, eps, seed, vals=vals, mode="sort")
    assert r.status == 0
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(r.keys, keys[order])
    if payload:
        assert np.array_equal(r.vals, vals[order])
    R.check_balance(r.offsets, n, p, r.tol)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[2]}" for c in CASES])
def test_partition_matches_definition(case):
    kind, n, p, eps, seed, bits, payload = case
    keys = synth.make(kind, n, seed)
    if bits == 32:
        keys = keys.astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    r = oracle.hss(keys, p, eps, seed, vals=vals, mode="partition")
    assert r.status == 0
    R.check_balance(r.chi, n, p, r.tol)
    assert np.array_equal(r.offsets, r.chi)
    ek, ev = R.expected_partition(keys, vals, p, r.chi)
    assert np.array_equal(r.keys, ek)
    if payload:
        assert np.array_equal(r.vals, ev)
    # splitter S(i) is the element of global rank chi(i)
    tr = R.tag_rank(keys, p)
    for i in range(1, p):
        assert tr[int(r.s_tag[i])] == int(r.chi[i])
    # piece matrix row b = per-segment counts of S(b)
    if n <= 50_000 and p <= 64:
        for i in range(1, p):
            assert np.array_equal(r.pieces[i], R.brute_counts(keys, p, int(r.s_tag[i])))


def test_full_sample_settles_exactly():
    # every key is a probe in round 1, so each splitter lands on N i / p exactly
    for kind, n, p in [("uniform64", 3000, 13), ("SKEW2", 2000, 16), ("ALLZEROS", 999, 10)]:
        keys = synth.make(kind, n, 3)
        r = oracle.hss(keys, p, 0.05, 1, force_full_sample=True)
        assert r.status == 0
        assert len(r.rounds) == (1 if p > 1 else 0)
        assert [int(c) for c in r.chi] == list(R.ideal(n, p))
        assert r.rounds[0].m == n


def test_ranks_and_counts_by_brute_force():
    keys = synth.make("SKEW2", 1500, 21)      # many duplicates across segments
    p = 7
    r = oracle.hss(keys, p, 0.05, 5, trace_level=2)
    assert r.status == 0
    tr = R.tag_rank(keys, p)
    for rd in r.rounds:
        assert rd.m == len(rd.probe_tag)
        for e in range(rd.m):
            g = int(rd.probe_tag[e])
            c = R.brute_counts(keys, p, g)
            assert np.array_equal(rd.counts[e], c)
            assert int(rd.probe_rank[e]) == int(c.sum()) == int(tr[g])
        # probes listed in the strict order (key, tag)
        ks = [(int(a), int(b)) for a, b in zip(rd.probe_key, rd.probe_tag)]
        assert ks == sorted(ks)
        assert np.all(np.diff(rd.probe_rank.astype(np.int64)) > 0)


def _domain_from_state(n, p, tr_rank, prev, ideal, tol):
    """Tags strictly inside an unsettled interval, from the previous round's state."""
    if prev is None:
        return np.ones(n, dtype=bool)
    dom = np.zeros(n, dtype=bool)
    for i in range(1, p):
        if prev.settled[i - 1]:
            continue
        lo = -1 if int(prev.lo_rank[i - 1]) == R.NONE else int(prev.lo_rank[i - 1])
        hi = n if int(prev.hi_rank[i - 1]) == R.NONE else int(prev.hi_rank[i - 1])
        dom |= (tr_rank > lo) & (tr_rank < hi)
    return dom


@pytest.mark.parametrize("kind,n,p,eps,seed", [("uniform64", 20_000, 16, 0.05, 3),
                                               ("SKEW2", 8000, 12, 0.02, 4),
                                               ("zipf_morton", 30_000, 40, 0.05, 5),
                                               ("uniform64", 6000, 33, 0.01, 6)])
def test_round_probe_sets_follow_sampling_rule(kind, n, p, eps, seed, rocrand_philox):
    """Each round's probes are exactly the keys of the previous round's
    unsettled intervals whose rocRAND Philox word is below the threshold; the
    state after each round is the tightest one the probes allow."""
    keys = synth.make(kind, n, seed)
    r = oracle.hss(keys, p, eps, seed)
    assert r.status == 0
    tr = R.tag_rank(keys, p)
    idl = R.ideal(n, p)
    seen = []          # ranks of all probes so far
    prev = None
    for j, rd in enumerate(r.rounds, start=1):
        dom = _domain_from_state(n, p, tr, prev, idl, r.tol)
        assert rd.domain == int(dom.sum())
        tags = np.nonzero(dom)[0]
        if rd.all:
            chosen = tags
        else:
            w = np.array(rocrand_philox([seed] * len(tags), [j] * len(tags), tags.tolist()),
                         dtype=np.uint64) if len(tags) else np.zeros(0, dtype=np.uint64)
            chosen = tags[w < rd.thresh]
        assert sorted(chosen.tolist()) == sorted(int(t) for t in rd.probe_tag)
        seen_before = list(seen)
        seen += [int(x) for x in rd.probe_rank]
        this = sorted(int(x) for x in rd.probe_rank)
        for i in range(1, p):
            ideal_i = int(idl[i])
            was = prev is not None and prev.settled[i - 1]
            if was:
                assert rd.settled[i - 1] and rd.chi[i - 1] == prev.chi[i - 1]
                continue
            # never settled earlier: no earlier probe was inside the target range
            assert all(abs(x - ideal_i) > r.tol for x in seen_before)
            if rd.settled[i - 1]:
                c = int(rd.chi[i - 1])
                assert c in this and abs(c - ideal_i) <= r.tol
                # no probe of this round strictly closer; ties go to the lower rank
                for x in this:
                    assert abs(x - ideal_i) > abs(c - ideal_i) or (abs(x - ideal_i) == abs(c - ideal_i) and x >= c)
            else:
                lo = int(rd.lo_rank[i - 1]); hi = int(rd.hi_rank[i - 1])
                lo = -1 if lo == R.NONE else lo
                hi = n if hi == R.NONE else hi
                assert lo < ideal_i - r.tol and hi > ideal_i + r.tol
                assert lo == -1 or lo in seen
                assert hi == n or hi in seen
                assert not any(lo < x < hi for x in seen)   # tightest bounds
        # unsettled intervals are disjoint or identical (section 4.2.2)
        ivs = sorted({(int(rd.lo_rank[i]), int(rd.hi_rank[i])) for i in range(p - 1)
                      if not rd.settled[i]})
        for (a1, b1), (a2, b2) in zip(ivs, ivs[1:]):
            a1 = -1 if a1 == R.NONE else a1
            a2 = -1 if a2 == R.NONE else a2
            b1 = n if b1 == R.NONE else b1
            assert b1 <= a2 + 0 or (a1, b1) == (a2, b2)
        prev = rd
    assert all(prev.settled) if prev is not None else p == 1


def test_bounds_monotone_across_rounds():
    keys = synth.make("uniform64", 1 << 15, 2)
    n, p = len(keys), 64
    r = oracle.hss(keys, p, 0.01, 9)
    for a, b in zip(r.rounds, r.rounds[1:]):
        for i in range(p - 1):
            if b.settled[i]:
                continue
            la = -1 if int(a.lo_rank[i]) == R.NONE else int(a.lo_rank[i])
            lb = -1 if int(b.lo_rank[i]) == R.NONE else int(b.lo_rank[i])
            ha = n if int(a.hi_rank[i]) == R.NONE else int(a.hi_rank[i])
            hb = n if int(b.hi_rank[i]) == R.NONE else int(b.hi_rank[i])
            assert la <= lb and hb <= ha


# ----------------------------------------------------------- statistics ----

def test_sampling_statistics_round1():
    """Round 1 takes each key with probability p s_1 / N (section 4.2.1)."""
    n, p, eps = 1 << 17, 64, 0.05
    c = oracle.constants(n, p, eps)
    q = c.thresh[0] / 2**32
    ms = []
    for seed in range(40):
        keys = synth.make("uniform64", n, 100 + seed)
        r = oracle.hss(keys, p, eps, seed, trace_level=0)
        ms.append(r.rounds[0].m)
    mean = np.mean(ms)
    sd = math.sqrt(n * q * (1 - q) / len(ms))
    assert abs(mean - n * q) < 5 * sd
    assert n * q == pytest.approx(p * c.a ** (1 / c.k), rel=1e-6)


def test_interval_union_and_sample_size_lemmas():
    """E|gamma_j| <= 2N/s_j (section 4.2, expectation lemma) and
    Z_j <= 5 p s_j / s_{j-1} (sample-size lemma), checked loosely over seeds."""
    n, p, eps = 1 << 18, 256, 0.02
    c = oracle.constants(n, p, eps)
    sj = lambda j: c.a ** (j / c.k)
    dom = {}
    over = 0
    total = 0
    rounds = []
    for seed in range(12):
        keys = synth.make("uniform64", n, 500 + seed)
        r = oracle.hss(keys, p, eps, seed, trace_level=0)
        rounds.append(len(r.rounds))
        for j, rd in enumerate(r.rounds, start=1):
            dom.setdefault(j, []).append(rd.domain)
            if j >= 2:
                total += 1
                over += rd.m > 5 * p * sj(j) / sj(j - 1)
    for j in range(2, 5):
        # the domain of round j+1 is gamma_j; rounds that never happen have 0
        vals = dom.get(j + 1, []) + [0] * (12 - len(dom.get(j + 1, [])))
        assert np.mean(vals) <= 1.25 * 2 * n / sj(j)
    assert over <= max(1, total // 10)
    assert np.mean(rounds) <= c.k + 1


def test_rounds_independent_of_distribution_in_law():
    # The rank process does not depend on key values (section 7.5): with the
    # same seed, an all-equal input and a uniform input sample the same tags
    # in round 1.
    n, p = 20_000, 16
    a = oracle.hss(synth.make("uniform64", n, 1), p, 0.05, 77)
    b = oracle.hss(synth.make("ALLZEROS", n, 1), p, 0.05, 77)
    assert sorted(a.rounds[0].probe_tag.tolist()) == sorted(b.rounds[0].probe_tag.tolist())


# ----------------------------------------------------------- arguments ----

@pytest.mark.parametrize("n,p,eps", [(10, 0, 0.1), (10, 11, 0.1), (10, 2, 0.0), (10, 2, 1.0),
                                     (10, 2, -0.5), (0, 1, 0.1)])
def test_invalid_arguments(n, p, eps):
    keys = np.arange(max(n, 1), dtype=np.uint64)[:n]
    r = oracle.hss(keys, p, eps, 1)
    assert r.status == -1


def test_round_cap_reports_not_converged():
    keys = synth.make("uniform64", 1 << 16, 3)
    r = oracle.hss(keys, 64, 0.01, 3, max_rounds=1)
    assert r.status == -5


def test_one_round_lemma():
    """k = 1 is HSS with one round (section 4.1): at the rate 2 p ln p / (eps N)
    each target range of N eps / p keys misses every probe with probability at
    most 1/p^2, so all p - 1 splitters settle in the first round except with
    probability below 1/p.  Over 60 seeds at p = 16 that bound allows about
    3.5 runs with a second round; far more would mean a wrong rate, range or
    settle rule."""
    n, p, eps = 1 << 15, 16, 0.05
    c = oracle.constants(n, p, eps, k_override=1)
    assert c.k == 1
    extra = 0
    for seed in range(60):
        keys = synth.make("uniform64", n, 500 + seed)
        r = oracle.hss(keys, p, eps, seed, k_override=1, trace_level=0)
        assert r.status == 0
        off = r.offsets.astype(np.int64)
        assert np.all(np.abs(off - np.array(R.ideal(n, p), dtype=np.int64)) <= r.tol)
        extra += len(r.rounds) > 1
    assert extra <= 12, extra


@pytest.mark.parametrize("n,p,kind", [(20_000, 10, "uniform64"), (30_011, 7, "SKEW2"),
                                      (8192, 64, "GAUSS")])
def test_exact_splitting(n, p, kind):
    """eps = p / N gives tol = 0 (section 4.2, exact splitting): every splitter
    lands on rank floor(N i / p) and every bucket holds floor((i+1)N/p) -
    floor(iN/p) keys.  The schedule reaches rate 1 after finitely many rounds,
    which bounds the round count."""
    eps = p / n
    keys = synth.make(kind, n, 40 + p)
    c = oracle.constants(n, p, eps, max_j=64)
    assert c.tol == 0
    j_full = 1 + int(np.argmax(c.all))
    assert c.all[j_full - 1] and not any(c.all[:j_full - 1])
    r = oracle.hss(keys, p, eps, 9, trace_level=0)
    assert r.status == 0
    assert [int(x) for x in r.offsets] == list(R.ideal(n, p))
    assert 1 <= len(r.rounds) <= j_full
    # every bucket holds exactly its slice of the sorted input
    srt = np.sort(keys, kind="stable")
    for b in range(p):
        lo, hi = int(r.offsets[b]), int(r.offsets[b + 1])
        assert np.array_equal(np.sort(r.keys[lo:hi]), srt[lo:hi]), b


def test_probe_budget_draws_cp_probes_per_round():
    """A fixed budget of c p probes per round (section 6, the theorem with
    O(p) samples per round): each key of the round's domain is a probe with
    probability c p / |gamma|, so every round below rate 1 draws c p probes in
    expectation whatever its domain.  Over 40 seeds the mean per round is
    within 5 sigma of c p (Bernoulli counts: variance at most c p)."""
    n, p, eps, c = 1 << 17, 64, 0.02, 5
    counts = []
    for seed in range(40):
        keys = synth.make("uniform64", n, 300 + seed)
        r = oracle.hss(keys, p, eps, seed, trace_level=0, probes_per_round=c)
        assert r.status == 0
        off = r.offsets.astype(np.int64)
        assert np.all(np.abs(off - np.array(R.ideal(n, p), dtype=np.int64)) <= r.tol)
        counts += [rd.m for rd in r.rounds if not rd.all]
    mean = float(np.mean(counts))
    assert abs(mean - c * p) <= 5 * math.sqrt(c * p / len(counts)), (mean, len(counts))


def test_probe_budget_round_counts():
    """With 5p probes per round at eps = 2% the splitters settle within the
    6 rounds the paper reports (section 7.2, at p = 2048; the rank process
    does not depend on p much); one probe per processor per round (the
    iteration study of section 7.1) needs more rounds but stays bounded."""
    n, p, eps = 1 << 21, 256, 0.02
    r5, r1 = [], []
    for seed in range(3):
        keys = synth.make("uniform64", n, 600 + seed)
        a = oracle.hss(keys, p, eps, seed, trace_level=0, probes_per_round=5)
        b = oracle.hss(keys, p, eps, seed, trace_level=0, probes_per_round=1)
        assert a.status == 0 and b.status == 0
        r5.append(len(a.rounds))
        r1.append(len(b.rounds))
    assert all(3 <= x <= 6 for x in r5), r5
    assert min(r1) > max(r5) and max(r1) <= 16, (r1, r5)


# ------------------------------------------- fewer buckets, two stages ----

BUCKET_CASES = [
    # kind, n, p, q, eps, seed, bits, payload
    ("uniform64", 40_000, 64, 8, 0.05, 3, 64, True),
    ("SKEW2", 20_000, 32, 5, 0.05, 4, 64, False),
    ("GAUSS", 30_000, 48, 12, 0.02, 5, 64, True),
    ("uniform32", 10_007, 20, 3, 0.1, 6, 32, False),
    ("ALLZEROS", 9_000, 16, 4, 0.05, 7, 64, True),
    ("uniform64", 5_000, 10, 10, 0.05, 8, 64, False),     # q = p
]


@pytest.mark.parametrize("case", BUCKET_CASES, ids=[f"{c[0]}-{c[2]}-{c[3]}" for c in BUCKET_CASES])
def test_buckets_partition_matches_definition(case):
    """q < p buckets over p segments (one stage of section 5.3): splitters sit
    within N eps/(2q) of N i/q, the output is the partition the splitter ranks
    define (bucket, then source segment, then local order), and every row of
    the piece matrix is the per-segment count of its splitter."""
    kind, n, p, q, eps, seed, bits, payload = case
    keys = _keys(kind, n, seed, bits)
    vals = np.arange(n, dtype=np.uint64) * U64(7) if payload else None
    r = oracle.hss(keys, p, eps, seed, vals=vals, buckets=q)
    assert r.status == 0
    assert r.tol == math.floor(n * eps / (2 * q))
    assert r.k == max(1, math.ceil(math.log(2 * math.log(q) / eps))) if q > 1 else True
    assert len(r.offsets) == q + 1 and r.pieces.shape == (q + 1, p)
    R.check_balance(r.chi, n, q, r.tol)
    assert np.array_equal(r.offsets, r.chi)
    ek, ev = R.expected_partition(keys, vals, p, r.chi)
    assert np.array_equal(r.keys, ek)
    if payload:
        assert np.array_equal(r.vals, ev)
    tr = R.tag_rank(keys, p)
    for i in range(1, q):
        assert tr[int(r.s_tag[i])] == int(r.chi[i])
        assert np.array_equal(r.pieces[i], R.brute_counts(keys, p, int(r.s_tag[i])))
    assert np.array_equal(r.pieces[q], np.diff(R.seg_bounds(n, p)))


def test_buckets_full_sample_settles_exactly():
    for kind, n, p, q in [("uniform64", 3000, 13, 4), ("SKEW2", 2000, 16, 7), ("ALLZEROS", 999, 10, 2)]:
        keys = synth.make(kind, n, 3)
        r = oracle.hss(keys, p, 0.05, 1, force_full_sample=True, buckets=q)
        assert r.status == 0
        assert len(r.rounds) == 1 and r.rounds[0].m == n
        assert [int(c) for c in r.chi] == list(R.ideal(n, q))


def test_one_bucket_is_the_local_sort():
    keys = synth.make("SKEW1", 7000, 2)
    vals = np.arange(7000, dtype=np.uint64)
    r = oracle.hss(keys, 9, 0.05, 1, vals=vals, buckets=1)
    assert r.status == 0 and len(r.rounds) == 0
    lo = R.local_order(keys, 9)
    assert np.array_equal(r.keys, keys[lo]) and np.array_equal(r.vals, vals[lo])
    assert [int(x) for x in r.offsets] == [0, 7000]


def test_bucket_count_above_segments_is_invalid():
    keys = synth.make("uniform64", 100, 1)
    assert oracle.hss(keys, 4, 0.1, 1, buckets=5).status == -1
    assert oracle.hss(keys, 4, 0.1, 1, buckets=0).status == -1


TWO_STAGE_CASES = [
    # kind, n, p, r, eps1, eps2, seed, payload
    ("uniform64", 60_000, 64, 8, 0.05, 0.05, 11, True),
    ("SKEW2", 30_000, 32, 4, 0.02, 0.05, 12, False),
    ("GAUSS", 40_000, 36, 6, 0.05, 0.02, 13, True),
    ("ALLZEROS", 8_000, 16, 4, 0.05, 0.05, 14, False),
    ("zipf_morton", 50_000, 64, 16, 0.05, 0.05, 15, True),
]


@pytest.mark.parametrize("case", TWO_STAGE_CASES, ids=[f"{c[0]}-{c[2]}-{c[3]}" for c in TWO_STAGE_CASES])
def test_two_stage_composition(case):
    """Two-stage HSS (section 5.3): group boundaries within N eps1/(2r) of
    N g/r; inside each group, bucket boundaries within N_g eps2 r/(2p) of
    N_g i r/p; the output of each stage is the partition its splitter ranks
    define, applied to the previous stage's output; and the whole is a
    permutation whose buckets are in key order."""
    kind, n, p, r, eps1, eps2, seed, payload = case
    keys = synth.make(kind, n, seed)
    vals = np.arange(n, dtype=np.uint64) ^ U64(0xABCDEF) if payload else None
    t = oracle.hss_two_stage(keys, p, r, eps1, eps2, seed, vals=vals)
    assert t.status == 0
    pg = p // r
    chi1 = [int(c) for c in t.groups]
    R.check_balance(chi1, n, r, math.floor(n * eps1 / (2 * r)))
    k1, v1 = R.expected_partition(keys, vals, p, chi1)
    off = [int(x) for x in t.offsets]
    assert off[0] == 0 and off[p] == n
    for g in range(r):
        lo, hi = chi1[g], chi1[g + 1]
        ng = hi - lo
        st2 = t.stage2[g]
        tol2 = math.floor(ng * eps2 / (2 * pg))
        assert st2.tol == tol2
        loc = [x - lo for x in off[g * pg:(g + 1) * pg + 1]]
        R.check_balance(loc, ng, pg, tol2)
        ek, ev = R.expected_partition(k1[lo:hi], None if v1 is None else v1[lo:hi], pg, loc)
        assert np.array_equal(t.keys[lo:hi], ek)
        if payload:
            assert np.array_equal(t.vals[lo:hi], ev)
    # every final bucket lies between its neighbours in key order
    srt = np.sort(keys)
    for b in range(p):
        seg = np.sort(t.keys[off[b]:off[b + 1]])
        assert np.array_equal(seg, srt[off[b]:off[b + 1]]), b
    if payload:
        # the payload travels with its key
        assert np.array_equal(np.sort(t.vals), np.sort(vals))
        pos = {int(v): i for i, v in enumerate(vals)}
        assert all(keys[pos[int(v)]] == k for v, k in zip(t.vals[:500], t.keys[:500]))


def test_two_stage_with_one_group_is_single_stage():
    """r = 1: the first stage only concatenates the locally sorted segments,
    whose local sort the second stage leaves unchanged, so the result is the
    single-stage run with the group's seed."""
    keys = synth.make("SKEW3", 20_000, 21)
    vals = np.arange(20_000, dtype=np.uint64)
    p, eps, seed = 32, 0.03, 9
    t = oracle.hss_two_stage(keys, p, 1, 0.05, eps, seed, vals=vals)
    s = oracle.hss(keys, p, eps, oracle.stage_seed(seed, 0), vals=vals, trace_level=0)
    assert t.status == 0 and s.status == 0
    assert np.array_equal(t.keys, s.keys) and np.array_equal(t.vals, s.vals)
    assert np.array_equal(t.offsets, s.offsets)


def test_two_stage_with_p_groups_is_single_stage_sort():
    """r = p: every group is one processor, whose second stage is a stable
    sort of its bucket, which is the single-stage sort."""
    keys = synth.make("GAUSS", 20_000, 22)
    vals = np.arange(20_000, dtype=np.uint64)
    p, eps, seed = 16, 0.05, 4
    t = oracle.hss_two_stage(keys, p, p, eps, 0.05, seed, vals=vals)
    s = oracle.hss(keys, p, eps, seed, vals=vals, mode="sort", trace_level=0)
    assert t.status == 0 and s.status == 0
    assert np.array_equal(t.keys, s.keys) and np.array_equal(t.vals, s.vals)
    assert np.array_equal(t.offsets, s.offsets)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(t.keys, keys[order]) and np.array_equal(t.vals, vals[order])


def test_two_stage_invalid_group_counts():
    keys = synth.make("uniform64", 1000, 1)
    assert oracle.hss_two_stage(keys, 16, 3, 0.05, 0.05, 1).status == -1
    assert oracle.hss_two_stage(keys, 16, 0, 0.05, 0.05, 1).status == -1


# --------------------------------------------------------------- threads ----

THREAD_CASES = [
    # kind, n, p, q, eps, seed, bits, payload, mode, budget
    ("uniform64", 60_000, 37, None, 0.02, 2, 64, True, "partition", 0),
    ("SKEW2", 20_000, 32, None, 0.05, 5, 64, True, "sort", 0),
    ("zipf_morton", 40_000, 128, None, 0.05, 9, 64, True, "partition", 0),
    ("uniform32", 30_001, 64, 8, 0.1, 3, 32, False, "sort", 0),
    ("uniform64", 50_000, 50, None, 0.05, 4, 64, False, "partition", 5),
    ("uniform64", 300, 300, None, 0.5, 11, 64, True, "partition", 0),
]


@pytest.mark.parametrize("case", THREAD_CASES, ids=[f"{c[0]}-{c[1]}-{c[2]}-{c[8]}" for c in THREAD_CASES])
def test_threads_do_not_change_the_result(case):
    """The per-segment and per-bucket work split over host threads gives the
    run of one thread, field by field (outputs, splitters, pieces and every
    round's probes, ranks, local histograms and splitter state)."""
    kind, n, p, q, eps, seed, bits, payload, mode, budget = case
    keys = synth.make(kind, n, seed)
    if bits == 32:
        keys = keys.astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    one = oracle.hss(keys, p, eps, seed, vals=vals, mode=mode, trace_level=2, buckets=q,
                     probes_per_round=budget, threads=1)
    assert one.status == 0
    for t in (3, 8):
        many = oracle.hss(keys, p, eps, seed, vals=vals, mode=mode, trace_level=2, buckets=q,
                          probes_per_round=budget, threads=t)
        assert many.status == 0
        for f in ("keys", "vals", "offsets", "chi", "s_key", "s_tag", "pieces"):
            a, b = getattr(one, f), getattr(many, f)
            assert (a is None and b is None) or np.array_equal(a, b), f
        assert len(one.rounds) == len(many.rounds)
        for ra, rb in zip(one.rounds, many.rounds):
            assert (ra.domain, ra.m, ra.thresh, ra.all) == (rb.domain, rb.m, rb.thresh, rb.all)
            for f in ("probe_key", "probe_tag", "probe_rank", "counts", "lo_rank", "hi_rank",
                      "settled", "chi"):
                assert np.array_equal(getattr(ra, f), getattr(rb, f)), f
    assert all(x >= 0 for x in one.times) and one.times[0] > 0


# ------------------------------------------------- section 6 pick sampler ----

@pytest.mark.parametrize("kind,n,p,eps,c,seed", [("uniform64", 20_000, 16, 0.02, 5, 3),
                                                 ("SKEW2", 12_000, 12, 0.05, 1, 4),
                                                 ("zipf_morton", 30_001, 40, 0.05, 5, 5)])
def test_pick_sampler_follows_section6(kind, n, p, eps, c, seed, rocrand_philox):
    """Each round's probes are exactly the distinct positions, among
    ceil(c N / |gamma|) picks of every segment (rocRAND Philox words of
    counter (pick, segment, round, 1) scaled to the segment), that lie
    strictly inside an unsettled interval; every key of the intervals once the
    picks reach the largest segment."""
    keys = synth.make(kind, n, seed)
    r = oracle.hss(keys, p, eps, seed, probes_per_round=c, pick_sampler=True)
    assert r.status == 0
    tr = R.tag_rank(keys, p)
    idl = R.ideal(n, p)
    starts = [(s * n) // p for s in range(p + 1)]
    max_seg = max(starts[s + 1] - starts[s] for s in range(p))
    prev = None
    for j, rd in enumerate(r.rounds, start=1):
        dom = _domain_from_state(n, p, tr, prev, idl, r.tol)
        domain = int(dom.sum())
        assert rd.domain == domain
        picks = math.ceil(float(c) * float(n) / float(domain))
        if picks >= max_seg:
            assert rd.all == 1
            chosen = set(np.nonzero(dom)[0].tolist())
        else:
            assert rd.all == 0 and rd.thresh == picks
            S, J, G, where = [], [], [], []
            for s in range(p):
                for l in range(picks):
                    # rocRAND's counter: word 0 of block (offset / 4) in
                    # subsequence j + 2^32, i.e. counter (l, s, j, 1)
                    S.append(seed); J.append(j + (1 << 32)); G.append(4 * (l + (s << 32)))
                    where.append(s)
            words = rocrand_philox(S, J, G)
            chosen = set()
            for s, w in zip(where, words):
                ns = starts[s + 1] - starts[s]
                g = starts[s] + ((w * ns) >> 32)
                if dom[g]:
                    chosen.add(g)
        assert sorted(chosen) == sorted(int(t) for t in rd.probe_tag)
        prev = rd
    assert all(prev.settled)


def test_pick_sampler_draws_cp_probes_per_round():
    """In expectation c p probes per round: the mean over seeds of every
    round's probe count lies near c p (the pick count is rounded up, and a
    position picked twice counts once)."""
    n, p, c = 1 << 17, 64, 5
    keys = synth.make("uniform64", n, 9)
    ms = []
    for seed in range(12):
        r = oracle.hss(keys, p, 0.02, 100 + seed, probes_per_round=c, pick_sampler=True,
                       trace_level=0)
        assert r.status == 0
        ms += [rd.m / (c * p) for rd in r.rounds if not rd.all]
    assert 0.85 < float(np.mean(ms)) < 1.3, np.mean(ms)
