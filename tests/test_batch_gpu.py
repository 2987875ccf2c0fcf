"""GPU parity of batches: every instance of hss_batch_partition equals the
oracle's hss_partition of that instance alone (keys, payload, offsets),
bit for bit, whatever the other instances of the batch are."""
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


def _keys(kind, n, seed, kb):
    k = synth.make(kind, n, seed)
    if kb == 4:
        k = (k >> np.uint64(32)).astype(np.uint32) if kind == "uniform64" else k.astype(np.uint32)
    return k


MIXED = [
    # n, p, eps, key bytes, kind, seed
    (5000, 8, 0.05, 8, "uniform64", 1),
    (70_000, 16, 0.05, 4, "uniform64", 2),        # u32, segments take the MSD pass
    (300_000, 64, 0.02, 8, "uniform64", 3),
    (4096, 256, 0.05, 8, "uniform64", 4),         # segments of 16 keys, sorted whole
    (1_000_000, 8, 0.05, 8, "uniform64", 5),      # segments of 125 000 keys
    (200_000, 32, 0.05, 8, "SKEW2", 6),           # 101 distinct keys
    (50_000, 10, 0.05, 8, "ALLZEROS", 7),
    (1000, 1, 0.05, 8, "uniform64", 8),           # p = 1
    (300, 300, 0.5, 8, "uniform64", 9),           # p = N
    (40_000, 9, 1e-6, 4, "uniform64", 10),        # tol = 0, u32
    (123_457, 37, 0.05, 8, "GAUSS", 11),          # ragged segments
    (20_000, 100, 0.05, 4, "SKEW1", 12),          # u32, segments of 200 keys
]


def _run_batch(hss, cases, payload, seeds, budget=0):
    shapes = [(n, p, eps, kb) for (n, p, eps, kb, _, _) in cases]
    host_keys = [_keys(kind, n, s, kb) for (n, p, eps, kb, kind, s) in cases]
    host_vals = ([(np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) ^ np.uint64(i)
                  for i, (n, *_r) in enumerate(cases)] if payload else None)
    with hss.BatchPlan(shapes, payload=payload, probes_per_round=budget) as bp:
        ko, vo, off = bp.partition([_dev(k) for k in host_keys], seeds,
                                   [_dev(v) for v in host_vals] if payload else None)
        torch.cuda.synchronize()
        for i, (n, p, eps, kb, kind, s) in enumerate(cases):
            ref = oracle.hss(host_keys[i], p, eps, seeds[i],
                             vals=host_vals[i] if payload else None, mode="partition",
                             probes_per_round=budget)
            assert ref.status == 0
            dt = np.uint64 if kb == 8 else np.uint32
            assert np.array_equal(_host(off[i], np.uint64), ref.offsets), i
            assert np.array_equal(_host(ko[i], dt), ref.keys), i
            if payload:
                assert np.array_equal(_host(vo[i], np.uint64), ref.vals), i


@pytest.mark.parametrize("payload", [False, True])
def test_batch_matches_oracle(hss, payload):
    _say(f"[batch] {len(MIXED)} mixed instances, payload={payload}")
    seeds = [1000 + i for i in range(len(MIXED))]
    _run_batch(hss, MIXED, payload, seeds)


@pytest.mark.parametrize("budget", [1, 5])
def test_batch_with_probe_budget_matches_oracle(hss, budget):
    """A probe budget in a batch: every instance draws at its own rate
    c q / |gamma| from its own domain, as its plain plan would."""
    _say(f"[batch] {len(MIXED)} mixed instances, budget {budget} q probes per round")
    seeds = [2000 + i for i in range(len(MIXED))]
    _run_batch(hss, MIXED, budget == 5, seeds, budget=budget)


def test_batch_reuse_with_new_seeds(hss):
    cases = MIXED[:6]
    _say("[batch] two calls on one batch with different seeds")
    with hss.BatchPlan([(n, p, e, kb) for (n, p, e, kb, _, _) in cases]) as bp:
        for call in range(2):
            seeds = [77 * call + i for i in range(len(cases))]
            keys = [_keys(kind, n, s + call, kb) for (n, p, e, kb, kind, s) in cases]
            ko, _, off = bp.partition([_dev(k) for k in keys], seeds)
            for i, (n, p, e, kb, kind, s) in enumerate(cases):
                ref = oracle.hss(keys[i], p, e, seeds[i], mode="partition")
                dt = np.uint64 if kb == 8 else np.uint32
                assert np.array_equal(_host(off[i], np.uint64), ref.offsets), (call, i)
                assert np.array_equal(_host(ko[i], dt), ref.keys), (call, i)


def test_batch_of_uneven_instances(hss):
    """The batched configuration's mix at reduced sizes: sizes log-uniform on
    [2^12, 2^18], p log-uniform on [8, 256], half u32 and half u64 keys."""
    rng = np.random.default_rng(4)
    cases = []
    for i in range(64):
        n = int(2 ** rng.uniform(12, 18))
        p = int(np.clip(np.exp(rng.uniform(np.log(8), np.log(257))), 8, 256))
        cases.append((n, p, 0.05, 4 if i < 32 else 8, "uniform64", 100 + i))
    _say(f"[batch] 64 uneven instances, {sum(c[0] for c in cases)} keys")
    _run_batch(hss, cases, False, [1000 + i for i in range(64)])


def test_batch_rejects_bad_shapes(hss):
    with pytest.raises(hss.HssError):
        hss.BatchPlan([(100, 200, 0.05, 8)])       # p > N
    with pytest.raises(hss.HssError):
        hss.BatchPlan([(100, 4, 1.5, 8)])          # eps >= 1
