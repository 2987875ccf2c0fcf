"""hss_partition_static, the entry point that allocates nothing, against
hss_partition: two calls in a row through the C ABI (the second on a smaller
input of another key width), each compared bit for bit with a plan's
hss_partition of the same shape, seed and input.  Around each of the two
calls the device's free memory is read: the library takes none (the fixed
array is reserved when its code is loaded, which a first call does)."""
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
    return torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()


def _case(kind, n, bits, seed, payload):
    keys = synth.make(kind, n, seed)
    if bits == 32:
        keys = (keys >> np.uint64(32)).astype(np.uint32) if kind == "uniform64" else keys.astype(np.uint32)
    vals = (np.arange(n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) if payload else None
    return keys, vals


def test_static_partition_equals_plan_partition(hss):
    # a first call on the device looks the array up and loads the library's code
    _say("[no-alloc] first call: uniform64 n=4096 p=8 (loads the code)")
    k0, _ = _case("uniform64", 4096, 64, 1, False)
    hss.partition_static(_dev(k0), 8, 0.05, 1)
    torch.cuda.synchronize()
    cases = [
        # kind, n, p, eps, data seed, hss seed, key bits, payload
        ("zipf_morton", 1 << 20, 256, 0.02, 3, 11, 64, True),   # the largest accepted shape
        ("SKEW2", 100_003, 37, 0.05, 4, 12, 32, False),        # smaller, ragged, duplicates
    ]
    for kind, n, p, eps, dseed, hseed, bits, payload in cases:
        _say(f"[no-alloc] {kind} n={n} p={p} eps={eps} bits={bits} payload={payload}")
        st, need, cap = hss.static_workspace_bytes(n, p, eps, bits // 8, payload)
        assert st == 0 and 0 < need <= cap
        keys, vals = _case(kind, n, bits, dseed, payload)
        kd = _dev(keys)
        vd = None if vals is None else _dev(vals)
        ko = torch.empty_like(kd)
        vo = None if vd is None else torch.empty_like(vd)
        off = torch.empty(p + 1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        hss.partition_static(kd, p, eps, hseed, vd, ko, vo, off)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        _say(f"[no-alloc] free device memory before/after: {free0} {free1}")
        assert free1 >= free0, (free0, free1)
        with hss.Plan(n, p, eps, key_bytes=bits // 8, payload=payload) as plan:
            rk, rv, roff = plan.partition(kd, hseed, vd)
            torch.cuda.synchronize()
        assert torch.equal(off, roff)
        assert torch.equal(ko, rk)
        if payload:
            assert torch.equal(vo, rv)
