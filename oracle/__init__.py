"""CPU oracle of Histogram Sort with Sampling -- TEST INFRASTRUCTURE ONLY.

A plain, slow C++ statement of the method (``hss_oracle.cpp``), loaded with
ctypes.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product library never does.  It shares
no code with the HIP path.

Parity status of each entry point (what pins it, besides the GPU):
  philox4x32_10  -- pinned: rocRAND's independent Philox4x32-10 engine.
  constants      -- pinned: closed forms of section 4.2 and section 7.2 numbers.
  local_sort     -- pinned: numpy stable argsort per segment.
  hss            -- pinned: outputs against numpy's stable sort (closed form),
                    ranks against brute-force counting, the full-sample case
                    (every splitter exactly at N i / p), the balance
                    invariants of section 2, and the sampling statistics of
                    section 4.2.  The exact probe sets and which probe settles a
                    splitter depend on the random stream; beyond the Philox pin
                    and the definitions they are "parity unpinned".
                    With q < p buckets (one stage of section 5.3): the same
                    invariants, and q = 1 is the local sort.
  hss_two_stage  -- pinned: r = 1 reduces to single-stage HSS of the locally
                    sorted input, r = p to the single-stage sort; outputs
                    against numpy's sort, group and bucket bounds of section 2
                    for both stages.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hss_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle_hss.so")
_lib = None

NONE = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-pthread",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        u64, u32, dbl, vp = C.c_uint64, C.c_uint32, C.c_double, C.c_void_p
        L.oracle_philox4x32_10.argtypes = [vp, vp, vp]
        L.oracle_constants.argtypes = [u64, u32, dbl, u32, vp, vp, vp, u32, vp, vp]
        L.oracle_philox_word.argtypes = [u64, u64, u32]
        L.oracle_philox_word.restype = u32
        L.oracle_hss.argtypes = [u64, u32, u32, dbl, C.c_int, vp, vp, u64, C.c_int, u32, u32,
                                 C.c_int, u32, C.c_int, vp, vp, vp, C.c_int, C.c_int]
        L.oracle_times.argtypes = [vp, vp]
        L.oracle_hss.restype = vp
        L.oracle_local_sort.argtypes = [u64, u32, C.c_int, vp, vp, vp, vp]
        L.oracle_local_sort.restype = C.c_int
        L.oracle_status.argtypes = [vp]
        L.oracle_status.restype = C.c_int
        L.oracle_num_rounds.argtypes = [vp]
        L.oracle_num_rounds.restype = u32
        L.oracle_tol.argtypes = [vp]
        L.oracle_tol.restype = u64
        L.oracle_k.argtypes = [vp]
        L.oracle_k.restype = u32
        L.oracle_round_info.argtypes = [vp, u32, vp, vp, vp, vp]
        L.oracle_round_probes.argtypes = [vp, u32, vp, vp, vp, vp]
        L.oracle_round_state.argtypes = [vp, u32, vp, vp, vp, vp]
        L.oracle_splitters.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_free.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(ctr), _ptr(key), _ptr(out))
    return out


def philox_word(seed: int, g: int, j: int) -> int:
    return int(lib().oracle_philox_word(seed, g, j))


@dataclass
class Constants:
    tol: int
    k: int
    a: float
    thresh: np.ndarray   # per round j = 1..len, acceptance threshold
    all: np.ndarray      # per round, 1 when every domain key is a probe


def constants(n: int, p: int, eps: float, k_override: int = 0, max_j: int = 64) -> Constants:
    tol, k, a = C.c_uint64(), C.c_uint32(), C.c_double()
    th = np.zeros(max_j, dtype=np.uint32)
    al = np.zeros(max_j, dtype=np.uint32)
    lib().oracle_constants(n, p, eps, k_override, C.byref(tol), C.byref(k), C.byref(a),
                           max_j, _ptr(th), _ptr(al))
    return Constants(int(tol.value), int(k.value), float(a.value), th, al)


def local_sort(keys: np.ndarray, p: int, vals: np.ndarray | None = None):
    keys = np.ascontiguousarray(keys)
    bits = 32 if keys.dtype == np.uint32 else 64
    ko = np.empty_like(keys)
    vo = None if vals is None else np.empty(len(keys), dtype=np.uint64)
    vi = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint64)
    rc = lib().oracle_local_sort(len(keys), p, bits, _ptr(keys), _ptr(vi), _ptr(ko), _ptr(vo))
    if rc != 0:
        raise ValueError("invalid arguments")
    return ko, vo


@dataclass
class Round:
    domain: int
    m: int
    thresh: int
    all: int
    probe_key: np.ndarray | None = None
    probe_tag: np.ndarray | None = None
    probe_rank: np.ndarray | None = None
    counts: np.ndarray | None = None     # (m, p), trace level 2
    lo_rank: np.ndarray | None = None    # (p-1,), NONE = -infinity or settled
    hi_rank: np.ndarray | None = None
    settled: np.ndarray | None = None
    chi: np.ndarray | None = None


@dataclass
class Result:
    status: int
    keys: np.ndarray | None = None
    vals: np.ndarray | None = None
    offsets: np.ndarray | None = None
    tol: int = 0
    k: int = 0
    rounds: list = field(default_factory=list)
    chi: np.ndarray | None = None
    s_key: np.ndarray | None = None
    s_tag: np.ndarray | None = None
    pieces: np.ndarray | None = None     # (q+1, p)
    # seconds per stage: local sort, splitter rounds, exchange, bucket sort
    times: tuple = (0.0, 0.0, 0.0, 0.0)


def hss(keys: np.ndarray, p: int, eps: float, seed: int, vals: np.ndarray | None = None,
        mode: str = "partition", k_override: int = 0, max_rounds: int = 0,
        force_full_sample: bool = False, trace_level: int = 1,
        probes_per_round: int = 0, buckets: int | None = None, threads: int = 1,
        pick_sampler: bool = False) -> Result:
    """Run the whole method on the host; returns outputs and the round trace.
    threads: host threads over which the per-segment work (local sort,
    slices, draws, local histograms, piece rows) and the per-bucket work
    (exchange, bucket sort) are split; the result does not depend on it.
    probes_per_round = c > 0: a fixed budget of c q probes per round (rate
    c q / |gamma|) instead of the rate schedule; with pick_sampler, drawn as
    the implementation of section 6 does: ceil(c N / |gamma|) uniform picks
    of every segment (with replacement), those outside the intervals
    discarded, each position once (round info's thresh is then the pick
    count).  buckets = q (default p):
    the p segments are split into q <= p buckets, as in one stage of
    multi-stage HSS (section 5.3); offsets, chi and the splitter state then
    have q+1 (resp. q-1) entries."""
    keys = np.ascontiguousarray(keys)
    if keys.dtype not in (np.uint32, np.uint64):
        raise TypeError("keys must be uint32 or uint64")
    bits = 32 if keys.dtype == np.uint32 else 64
    n = len(keys)
    q = p if buckets is None else int(buckets)
    if q <= 0 or q > max(p, 0):
        return Result(status=-1)
    ko = np.empty(max(n, 1), dtype=keys.dtype)
    vi = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint64)
    vo = None if vals is None else np.empty(max(n, 1), dtype=np.uint64)
    off = np.zeros(q + 1, dtype=np.uint64)
    kin = keys if n else np.zeros(1, dtype=keys.dtype)
    L = lib()
    h = L.oracle_hss(n, p, q, eps, bits, _ptr(kin), _ptr(vi), seed & NONE,
                     1 if mode == "sort" else 0, k_override, max_rounds,
                     1 if force_full_sample else 0, probes_per_round, trace_level,
                     _ptr(ko), _ptr(vo), _ptr(off), int(threads), 1 if pick_sampler else 0)
    try:
        st = L.oracle_status(h)
        res = Result(status=st)
        if st != 0:
            return res
        res.keys, res.vals, res.offsets = ko[:n], (None if vo is None else vo[:n]), off
        res.tol, res.k = int(L.oracle_tol(h)), int(L.oracle_k(h))
        tm = np.zeros(4, dtype=np.float64)
        L.oracle_times(h, _ptr(tm))
        res.times = tuple(float(x) for x in tm)
        for j in range(L.oracle_num_rounds(h)):
            d, m, th, al = C.c_uint64(), C.c_uint64(), C.c_uint32(), C.c_uint32()
            L.oracle_round_info(h, j, C.byref(d), C.byref(m), C.byref(th), C.byref(al))
            r = Round(int(d.value), int(m.value), int(th.value), int(al.value))
            if trace_level >= 1:
                mm = r.m
                r.probe_key = np.zeros(mm, dtype=np.uint64)
                r.probe_tag = np.zeros(mm, dtype=np.uint64)
                r.probe_rank = np.zeros(mm, dtype=np.uint64)
                cnt = np.zeros(mm * p, dtype=np.uint32) if trace_level >= 2 else None
                L.oracle_round_probes(h, j, _ptr(r.probe_key), _ptr(r.probe_tag),
                                      _ptr(r.probe_rank), _ptr(cnt))
                if cnt is not None:
                    r.counts = cnt.reshape(mm, p)
                r.lo_rank = np.zeros(q - 1, dtype=np.uint64)
                r.hi_rank = np.zeros(q - 1, dtype=np.uint64)
                r.settled = np.zeros(q - 1, dtype=np.uint8)
                r.chi = np.zeros(q - 1, dtype=np.uint64)
                if q > 1:
                    L.oracle_round_state(h, j, _ptr(r.lo_rank), _ptr(r.hi_rank),
                                         _ptr(r.settled), _ptr(r.chi))
            res.rounds.append(r)
        res.chi = np.zeros(q + 1, dtype=np.uint64)
        res.s_key = np.zeros(q + 1, dtype=np.uint64)
        res.s_tag = np.zeros(q + 1, dtype=np.uint64)
        res.pieces = np.zeros((q + 1) * p, dtype=np.uint64)
        L.oracle_splitters(h, _ptr(res.chi), _ptr(res.s_key), _ptr(res.s_tag), _ptr(res.pieces))
        res.pieces = res.pieces.reshape(q + 1, p)
        return res
    finally:
        L.oracle_free(h)


@dataclass
class TwoStage:
    status: int
    keys: np.ndarray | None = None
    vals: np.ndarray | None = None
    offsets: np.ndarray | None = None    # p+1 final bucket boundaries
    groups: np.ndarray | None = None     # r+1 group boundaries of stage 1
    stage1: Result | None = None
    stage2: list = field(default_factory=list)


def stage_seed(seed: int, g: int) -> int:
    """Philox seed of group g in the second stage (READING: the paper leaves
    the random streams of the groups open; each group gets its own, seed+1+g,
    so that no two runs share one)."""
    return (seed + 1 + g) & NONE


def hss_two_stage(keys: np.ndarray, p: int, r: int, eps1: float, eps2: float, seed: int,
                  vals: np.ndarray | None = None, probes_per_round: int = 0) -> TwoStage:
    """Two-stage HSS (section 5.3), composed from single-stage runs.

    Stage 1: the p segments are split into r buckets, one per group of p/r
    processors (tolerance eps1); the exchange gives group g the keys ranked
    [chi1(g), chi1(g+1)).  READING: the group's keys are then dealt out evenly
    to its p/r processors in the order the exchange wrote them (segment s of
    the group holds positions floor(s N_g r/p) ..).  Stage 2: every group runs
    HSS on its own keys with p/r segments and buckets (tolerance eps2).  Final
    bucket g p/r + i is bucket i of group g.  Requires r | p and N_g >= p/r.
    probes_per_round = c > 0: both stages draw c q probes per round in
    expectation (q = r, then p/r).
    """
    keys = np.ascontiguousarray(keys)
    if r <= 0 or p % r != 0:
        return TwoStage(status=-1)
    pg = p // r
    st1 = hss(keys, p, eps1, seed, vals=vals, mode="partition", trace_level=0, buckets=r,
              probes_per_round=probes_per_round)
    if st1.status != 0:
        return TwoStage(status=st1.status)
    ko = np.empty_like(keys)
    vo = None if vals is None else np.empty(len(keys), dtype=np.uint64)
    off = np.zeros(p + 1, dtype=np.uint64)
    chi1 = st1.offsets.astype(np.uint64)
    res = TwoStage(status=0, stage1=st1, groups=chi1)
    for g in range(r):
        lo, hi = int(chi1[g]), int(chi1[g + 1])
        if hi - lo < pg:
            return TwoStage(status=-1, stage1=st1, groups=chi1)
        kg = st1.keys[lo:hi]
        vg = None if vals is None else st1.vals[lo:hi]
        st2 = hss(kg, pg, eps2, stage_seed(seed, g), vals=vg, mode="partition", trace_level=0,
                  probes_per_round=probes_per_round)
        if st2.status != 0:
            return TwoStage(status=st2.status, stage1=st1, groups=chi1)
        ko[lo:hi] = st2.keys
        if vo is not None:
            vo[lo:hi] = st2.vals
        off[g * pg:(g + 1) * pg] = lo + st2.offsets[:pg]
        res.stage2.append(st2)
    off[p] = len(keys)
    res.keys, res.vals, res.offsets = ko, vo, off
    return res
