"""Histogram Sort with Sampling on one MI355X -- Python binding of libhss.so.

Argument marshalling only: every step runs in the HIP kernels of libhss.so,
declared in include/hss.h.  PyTorch supplies device memory and the stream.
Importing this package fails loudly when the library has not been built.

    import paper_1803_01237_amd as hss
    keys_out, vals_out, offsets = hss.partition(keys, p=1024, eps=0.02, seed=2)
    keys_sorted, _, _ = hss.sort(keys, p=1024, eps=0.02, seed=2)

Keys are torch tensors of 4- or 8-byte integers (int32/uint32/int64/uint64),
compared as unsigned integers.  A payload is an 8-byte integer tensor.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhss.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build() or "
                      f"python -m paper_1803_01237_amd.build)")

# PyTorch ships its own HIP runtime under the same soname as the system one;
# load it first so that libhss.so and PyTorch share one runtime.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

HSS_U32, HSS_U64 = 0, 1
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "out of memory",
          -4: "device error", -5: "not converged", -6: "cancelled"}
HSS_ERR_CANCELLED = -6
NONE = (1 << 64) - 1

EXPORTS = [
    "hss_plan", "hss_plan_destroy", "hss_workspace_bytes", "hss_partition", "hss_sort",
    "hss_local_sort", "hss_get_constants", "hss_trace_rounds", "hss_trace_round_info",
    "hss_trace_round_probes", "hss_trace_round_counts", "hss_trace_round_state",
    "hss_trace_splitters",
    "hss_profile", "hss_profile_reset", "hss_profile_read",
    "hss_batch_plan", "hss_batch_destroy", "hss_batch_workspace_bytes", "hss_batch_partition",
    "hss_batch_profile", "hss_batch_profile_reset", "hss_batch_profile_read",
    "hss_server_create", "hss_server_destroy", "hss_server_submit", "hss_server_poll",
    "hss_server_wait", "hss_server_cancel", "hss_server_clock", "hss_server_stats", "hss_server_footprint",
    "hss_server_memory",
    "hss_plan_knobs", "hss_plan_set_knobs", "hss_batch_knobs", "hss_plan_buckets",
    "hss_staged_plan", "hss_staged_destroy", "hss_staged_workspace_bytes", "hss_staged_partition",
    "hss_staged_sort",
    "hss_staged_times", "hss_partition_static", "hss_partition_static_bytes", "hss_stream_copy",
    "hss_partition_ws", "hss_partition_workspace_bytes",
    "hss_status_string", "hss_last_error",
]

PROFILE_FAMILIES = ["radix_count", "radix_scan", "radix_scatter", "rounds",
                    "exchange_offsets", "exchange_copy", "small_sort"]


class HssError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.hss_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")
        self.status = status


class _Tuning(C.Structure):
    _fields_ = [("max_rounds", C.c_uint32), ("k_override", C.c_uint32),
                ("force_full_sample", C.c_uint32), ("trace_level", C.c_uint32),
                ("lsd_only", C.c_uint32), ("probes_per_round", C.c_uint32),
                ("plain_launches", C.c_uint32), ("autotune", C.c_uint32),
                ("workspace_limit_mib", C.c_uint32), ("pick_sampler", C.c_uint32),
                ("reserved", C.c_uint32 * 1)]


class _Knobs(C.Structure):
    _fields_ = [("small_sort_cap", C.c_uint32), ("sample_workgroups", C.c_uint32),
                ("pair_rank_from", C.c_uint32), ("pair_rank_workgroups", C.c_uint32),
                ("tuned", C.c_uint32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_vp, _u64, _u32, _dbl = C.c_void_p, C.c_uint64, C.c_uint32, C.c_double
_lib.hss_plan.argtypes = [C.POINTER(_vp), _u64, _u32, _dbl, C.c_int, C.c_int, C.POINTER(_Tuning)]
_lib.hss_plan.restype = C.c_int
_lib.hss_plan_buckets.argtypes = [C.POINTER(_vp), _u64, _u32, _u32, _dbl, C.c_int, C.c_int,
                                  C.POINTER(_Tuning)]
_lib.hss_plan_buckets.restype = C.c_int
_lib.hss_staged_plan.argtypes = [C.POINTER(_vp), _u64, _u32, _u32, _dbl, _dbl, C.c_int, C.c_int,
                                 C.POINTER(_Tuning)]
_lib.hss_staged_plan.restype = C.c_int
_lib.hss_staged_destroy.argtypes = [_vp]
_lib.hss_staged_destroy.restype = None
_lib.hss_staged_workspace_bytes.argtypes = [_vp]
_lib.hss_staged_workspace_bytes.restype = C.c_size_t
_lib.hss_staged_partition.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hss_staged_partition.restype = C.c_int
_lib.hss_staged_sort.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hss_staged_sort.restype = C.c_int
_lib.hss_staged_times.argtypes = [_vp, C.POINTER(_dbl), C.POINTER(_dbl), C.POINTER(_dbl)]
_lib.hss_staged_times.restype = C.c_int
_lib.hss_plan_destroy.argtypes = [_vp]
_lib.hss_plan_destroy.restype = None
_lib.hss_workspace_bytes.argtypes = [_vp]
_lib.hss_workspace_bytes.restype = C.c_size_t
for _f in (_lib.hss_partition, _lib.hss_sort):
    _f.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp]
    _f.restype = C.c_int
_lib.hss_local_sort.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.hss_local_sort.restype = C.c_int
_lib.hss_get_constants.argtypes = [_vp, _vp, _vp, _vp, _u32, _vp, _vp]
_lib.hss_get_constants.restype = C.c_int
_lib.hss_trace_rounds.argtypes = [_vp]
_lib.hss_trace_rounds.restype = _u32
_lib.hss_trace_round_info.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp]
_lib.hss_trace_round_info.restype = C.c_int
_lib.hss_trace_round_probes.argtypes = [_vp, _u32, _vp, _vp, _vp]
_lib.hss_trace_round_probes.restype = C.c_int
_lib.hss_trace_round_counts.argtypes = [_vp, _u32, _vp]
_lib.hss_trace_round_counts.restype = C.c_int
_lib.hss_trace_round_state.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp]
_lib.hss_trace_round_state.restype = C.c_int
_lib.hss_trace_splitters.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.hss_trace_splitters.restype = C.c_int
_lib.hss_profile.argtypes = [_vp, C.c_int]
_lib.hss_profile.restype = C.c_int
_lib.hss_profile_reset.argtypes = [_vp]
_lib.hss_profile_reset.restype = C.c_int
_lib.hss_profile_read.argtypes = [_vp, _u32, _vp, _vp, _vp]
_lib.hss_profile_read.restype = C.c_int


class _Shape(C.Structure):
    _fields_ = [("n", C.c_uint64), ("p", C.c_uint32), ("key_type", C.c_int), ("eps", C.c_double)]


class _IO(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("keys_in", C.c_void_p), ("vals_in", C.c_void_p),
                ("keys_out", C.c_void_p), ("vals_out", C.c_void_p), ("offsets", C.c_void_p)]


_lib.hss_batch_plan.argtypes = [C.POINTER(_vp), C.POINTER(_Shape), _u32, C.c_int, C.POINTER(_Tuning)]
_lib.hss_batch_plan.restype = C.c_int
_lib.hss_batch_destroy.argtypes = [_vp]
_lib.hss_batch_destroy.restype = None
_lib.hss_batch_workspace_bytes.argtypes = [_vp]
_lib.hss_batch_workspace_bytes.restype = C.c_size_t
_lib.hss_batch_partition.argtypes = [_vp, C.POINTER(_IO), _vp]
_lib.hss_batch_partition.restype = C.c_int
_lib.hss_batch_profile.argtypes = [_vp, C.c_int]
_lib.hss_batch_profile.restype = C.c_int
_lib.hss_batch_profile_reset.argtypes = [_vp]
_lib.hss_batch_profile_reset.restype = C.c_int
_lib.hss_batch_profile_read.argtypes = [_vp, _u32, _vp, _vp, _vp]
_lib.hss_batch_profile_read.restype = C.c_int


class _Request(C.Structure):
    _fields_ = [("n", C.c_uint64), ("p", C.c_uint32), ("key_type", C.c_int), ("eps", C.c_double),
                ("seed", C.c_uint64), ("keys_in", C.c_void_p), ("vals_in", C.c_void_p),
                ("keys_out", C.c_void_p), ("vals_out", C.c_void_p), ("offsets", C.c_void_p),
                ("op", C.c_int)]


HSS_OP_PARTITION, HSS_OP_SORT = 0, 1
_OPS = {"partition": HSS_OP_PARTITION, "sort": HSS_OP_SORT}


class _ServerConfig(C.Structure):
    _fields_ = [("max_batch_keys", C.c_uint64), ("max_batch_requests", C.c_uint32),
                ("workers", C.c_uint32), ("hbm_budget", C.c_uint64), ("batch_wait_us", C.c_uint32)]


_lib.hss_server_create.argtypes = [C.POINTER(_vp), C.POINTER(_ServerConfig)]
_lib.hss_server_create.restype = C.c_int
_lib.hss_server_footprint.argtypes = [C.POINTER(_Request)]
_lib.hss_server_footprint.restype = _u64
_lib.hss_server_destroy.argtypes = [_vp]
_lib.hss_server_destroy.restype = None
_lib.hss_server_submit.argtypes = [_vp, C.POINTER(_Request), C.POINTER(_u64)]
_lib.hss_server_submit.restype = C.c_int
_lib.hss_server_poll.argtypes = [_vp, _u64, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(_dbl), C.POINTER(_dbl)]
_lib.hss_server_poll.restype = C.c_int
_lib.hss_server_wait.argtypes = [_vp, _u64, C.POINTER(C.c_int), C.POINTER(_dbl), C.POINTER(_dbl)]
_lib.hss_server_wait.restype = C.c_int
_lib.hss_server_cancel.argtypes = [_vp, _u64, C.POINTER(C.c_int)]
_lib.hss_server_cancel.restype = C.c_int
_lib.hss_server_clock.argtypes = []
_lib.hss_server_clock.restype = _dbl
_lib.hss_server_stats.argtypes = [_vp, C.POINTER(_u64), C.POINTER(_u64), C.POINTER(_u64),
                                  C.POINTER(_u32), C.POINTER(_u64)]
_lib.hss_server_stats.restype = C.c_int
_lib.hss_server_memory.argtypes = [_vp, C.POINTER(_u64), C.POINTER(_u64)]
_lib.hss_server_memory.restype = C.c_int
_lib.hss_plan_knobs.argtypes = [_vp, C.POINTER(_Knobs)]
_lib.hss_plan_knobs.restype = C.c_int
_lib.hss_plan_set_knobs.argtypes = [_vp, C.POINTER(_Knobs)]
_lib.hss_plan_set_knobs.restype = C.c_int
_lib.hss_batch_knobs.argtypes = [_vp, C.c_int, C.POINTER(_Knobs)]
_lib.hss_batch_knobs.restype = C.c_int
_lib.hss_status_string.argtypes = [C.c_int]
_lib.hss_status_string.restype = C.c_char_p
_lib.hss_last_error.argtypes = []
_lib.hss_last_error.restype = C.c_char_p


def _check(st: int, where: str):
    if st != 0:
        raise HssError(st, where)


def _np_ptr(a):
    return None if a is None else a.ctypes.data


def _torch():
    import torch
    return torch


def _stream_handle():
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


def _key_type(t) -> int:
    if t.element_size() == 8:
        return HSS_U64
    if t.element_size() == 4:
        return HSS_U32
    raise TypeError("keys must be 4- or 8-byte integers")


@dataclass
class RoundTrace:
    domain: int
    m: int
    thresh: int
    all: int
    probe_key: np.ndarray | None = None
    probe_tag: np.ndarray | None = None
    probe_rank: np.ndarray | None = None
    counts: np.ndarray | None = None     # (m, p): c_s(e), trace level 2
    lo_rank: np.ndarray | None = None
    hi_rank: np.ndarray | None = None
    settled: np.ndarray | None = None
    chi: np.ndarray | None = None


class Plan:
    """A plan for (N, p, eps, key type, payload).  Owns its device workspace.
    buckets = q < p splits the p segments into q buckets (one stage of
    multi-stage HSS); offsets and splitters then have q+1 entries."""

    def __init__(self, n: int, p: int, eps: float, key_bytes: int = 8, payload: bool = False,
                 max_rounds: int = 0, k_override: int = 0, force_full_sample: bool = False,
                 trace_level: int = 0, lsd_only: bool = False, probes_per_round: int = 0,
                 plain_launches: bool = False, autotune: bool = False, buckets: int | None = None,
                 workspace_limit_mib: int = 0, pick_sampler: bool = False):
        tun = _Tuning(max_rounds, k_override, 1 if force_full_sample else 0, trace_level,
                      1 if lsd_only else 0, probes_per_round, 1 if plain_launches else 0,
                      1 if autotune else 0, workspace_limit_mib, 1 if pick_sampler else 0)
        h = _vp()
        kt = HSS_U64 if key_bytes == 8 else HSS_U32
        if buckets is None:
            _check(_lib.hss_plan(C.byref(h), n, p, eps, kt, 1 if payload else 0, C.byref(tun)),
                   "hss_plan")
        else:
            _check(_lib.hss_plan_buckets(C.byref(h), n, p, buckets, eps, kt, 1 if payload else 0,
                                         C.byref(tun)), "hss_plan_buckets")
        self._h = h
        self.n, self.p, self.eps = n, p, eps
        self.q = p if buckets is None else int(buckets)
        self.key_bytes, self.payload = key_bytes, payload
        self.trace_level = trace_level

    def close(self):
        if getattr(self, "_h", None):
            _lib.hss_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.hss_workspace_bytes(self._h))

    def knobs(self) -> dict:
        k = _Knobs()
        _check(_lib.hss_plan_knobs(self._h, C.byref(k)), "hss_plan_knobs")
        return k.as_dict()

    def set_knobs(self, **kw):
        k = _Knobs()
        _check(_lib.hss_plan_knobs(self._h, C.byref(k)), "hss_plan_knobs")
        for f, v in kw.items():
            setattr(k, f, v)
        _check(_lib.hss_plan_set_knobs(self._h, C.byref(k)), "hss_plan_set_knobs")

    def _outputs(self, keys, vals, keys_out, vals_out, offsets):
        torch = _torch()
        if keys_out is None:
            keys_out = torch.empty_like(keys)
        if vals is not None and vals_out is None:
            vals_out = torch.empty_like(vals)
        if offsets is None:
            offsets = torch.empty(self.q + 1, dtype=torch.int64, device=keys.device)
        return keys_out, vals_out, offsets

    def _validate(self, keys, vals):
        if not keys.is_cuda or not keys.is_contiguous():
            raise ValueError("keys must be a contiguous device tensor")
        if keys.numel() != self.n or keys.element_size() != self.key_bytes:
            raise ValueError("keys do not match the plan")
        if (vals is not None) != self.payload:
            raise ValueError("payload presence does not match the plan")
        if vals is not None and (vals.numel() != self.n or vals.element_size() != 8
                                 or not vals.is_contiguous() or not vals.is_cuda):
            raise ValueError("payload must be a contiguous device tensor of N 8-byte words")

    def _run(self, fn, name, keys, seed, vals, keys_out, vals_out, offsets):
        self._validate(keys, vals)
        keys_out, vals_out, offsets = self._outputs(keys, vals, keys_out, vals_out, offsets)
        st = fn(self._h, seed & NONE, keys.data_ptr(),
                None if vals is None else vals.data_ptr(), keys_out.data_ptr(),
                None if vals_out is None else vals_out.data_ptr(), offsets.data_ptr(),
                _stream_handle())
        _check(st, name)
        return keys_out, vals_out, offsets

    def partition(self, keys, seed: int, vals=None, keys_out=None, vals_out=None, offsets=None):
        return self._run(_lib.hss_partition, "hss_partition", keys, seed, vals, keys_out,
                         vals_out, offsets)

    def sort(self, keys, seed: int, vals=None, keys_out=None, vals_out=None, offsets=None):
        return self._run(_lib.hss_sort, "hss_sort", keys, seed, vals, keys_out, vals_out, offsets)

    def local_sort(self, keys, vals=None, keys_out=None, vals_out=None):
        self._validate(keys, vals)
        torch = _torch()
        if keys_out is None:
            keys_out = torch.empty_like(keys)
        if vals is not None and vals_out is None:
            vals_out = torch.empty_like(vals)
        st = _lib.hss_local_sort(self._h, keys.data_ptr(),
                                 None if vals is None else vals.data_ptr(), keys_out.data_ptr(),
                                 None if vals_out is None else vals_out.data_ptr(),
                                 _stream_handle())
        _check(st, "hss_local_sort")
        return keys_out, vals_out

    def constants(self, max_j: int = 64):
        tol, k, a = C.c_uint64(), C.c_uint32(), C.c_double()
        th = np.zeros(max_j, dtype=np.uint32)
        al = np.zeros(max_j, dtype=np.uint32)
        _check(_lib.hss_get_constants(self._h, C.byref(tol), C.byref(k), C.byref(a), max_j,
                                      _np_ptr(th), _np_ptr(al)), "hss_get_constants")
        return int(tol.value), int(k.value), float(a.value), th, al

    def trace(self) -> list:
        out = []
        for j in range(_lib.hss_trace_rounds(self._h)):
            d, m, th, al = C.c_uint64(), C.c_uint64(), C.c_uint32(), C.c_uint32()
            _check(_lib.hss_trace_round_info(self._h, j, C.byref(d), C.byref(m), C.byref(th),
                                             C.byref(al)), "hss_trace_round_info")
            r = RoundTrace(int(d.value), int(m.value), int(th.value), int(al.value))
            if self.trace_level >= 1:
                r.probe_key = np.zeros(r.m, dtype=np.uint64)
                r.probe_tag = np.zeros(r.m, dtype=np.uint64)
                r.probe_rank = np.zeros(r.m, dtype=np.uint64)
                _check(_lib.hss_trace_round_probes(self._h, j, _np_ptr(r.probe_key),
                                                   _np_ptr(r.probe_tag), _np_ptr(r.probe_rank)),
                       "hss_trace_round_probes")
                if self.trace_level >= 2:
                    cnt = np.zeros(r.m * self.p, dtype=np.uint32)
                    _check(_lib.hss_trace_round_counts(self._h, j, _np_ptr(cnt)),
                           "hss_trace_round_counts")
                    r.counts = cnt.reshape(r.m, self.p)
                q = self.q - 1
                r.lo_rank = np.zeros(q, dtype=np.uint64)
                r.hi_rank = np.zeros(q, dtype=np.uint64)
                r.settled = np.zeros(q, dtype=np.uint8)
                r.chi = np.zeros(q, dtype=np.uint64)
                _check(_lib.hss_trace_round_state(self._h, j, _np_ptr(r.lo_rank),
                                                  _np_ptr(r.hi_rank), _np_ptr(r.settled),
                                                  _np_ptr(r.chi)), "hss_trace_round_state")
            out.append(r)
        return out

    def profile(self, enable: bool = True):
        _check(_lib.hss_profile(self._h, 1 if enable else 0), "hss_profile")

    def profile_reset(self):
        _check(_lib.hss_profile_reset(self._h), "hss_profile_reset")

    def profile_read(self) -> dict:
        """{family: (ms, launches, algorithmic bytes)} summed since the last reset."""
        out = {}
        for i, name in enumerate(PROFILE_FAMILIES):
            ms, n, b = C.c_double(), C.c_uint64(), C.c_uint64()
            _check(_lib.hss_profile_read(self._h, i, C.byref(ms), C.byref(n), C.byref(b)),
                   "hss_profile_read")
            out[name] = (float(ms.value), int(n.value), int(b.value))
        return out

    def splitters(self):
        p, q = self.p, self.q
        chi = np.zeros(q + 1, dtype=np.uint64)
        sk = np.zeros(q + 1, dtype=np.uint64)
        stg = np.zeros(q + 1, dtype=np.uint64)
        pieces = np.zeros((q + 1) * p, dtype=np.uint64)
        _check(_lib.hss_trace_splitters(self._h, _np_ptr(chi), _np_ptr(sk), _np_ptr(stg),
                                        _np_ptr(pieces)), "hss_trace_splitters")
        return chi, sk, stg, pieces.reshape(q + 1, p)


class StagedPlan:
    """Two-stage HSS: r groups of p/r processors (r divides p).  Stage 1
    splits into r group buckets (eps1), stage 2 partitions every group with
    its p/r processors (eps2, seed + 1 + g for group g)."""

    def __init__(self, n: int, p: int, groups: int, eps1: float, eps2: float, key_bytes: int = 8,
                 payload: bool = False, max_rounds: int = 0, k_override: int = 0,
                 force_full_sample: bool = False, plain_launches: bool = False,
                 autotune: bool = False, probes_per_round: int = 0):
        tun = _Tuning(max_rounds, k_override, 1 if force_full_sample else 0, 0, 0, probes_per_round,
                      1 if plain_launches else 0, 1 if autotune else 0)
        h = _vp()
        kt = HSS_U64 if key_bytes == 8 else HSS_U32
        _check(_lib.hss_staged_plan(C.byref(h), n, p, groups, eps1, eps2, kt, 1 if payload else 0,
                                    C.byref(tun)), "hss_staged_plan")
        self._h = h
        self.n, self.p, self.r = n, p, groups
        self.key_bytes, self.payload = key_bytes, payload

    def close(self):
        if getattr(self, "_h", None):
            _lib.hss_staged_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.hss_staged_workspace_bytes(self._h))

    def times(self):
        """Host seconds of the last call: (stage 1, stage-2 layout, stage 2)."""
        a, b, c = _dbl(), _dbl(), _dbl()
        _check(_lib.hss_staged_times(self._h, C.byref(a), C.byref(b), C.byref(c)), "hss_staged_times")
        return float(a.value), float(b.value), float(c.value)

    def partition(self, keys, seed: int, vals=None, keys_out=None, vals_out=None, offsets=None,
                  groups_out=None):
        return self._run(_lib.hss_staged_partition, "hss_staged_partition", keys, seed, vals, keys_out,
                         vals_out, offsets, groups_out)

    def sort(self, keys, seed: int, vals=None, keys_out=None, vals_out=None, offsets=None, groups_out=None):
        """The two-stage partition, then every final bucket sorted (stably)."""
        return self._run(_lib.hss_staged_sort, "hss_staged_sort", keys, seed, vals, keys_out, vals_out,
                         offsets, groups_out)

    def _run(self, fn, name, keys, seed, vals, keys_out, vals_out, offsets, groups_out):
        torch = _torch()
        if not keys.is_cuda or not keys.is_contiguous():
            raise ValueError("keys must be a contiguous device tensor")
        if keys.numel() != self.n or keys.element_size() != self.key_bytes:
            raise ValueError("keys do not match the plan")
        if (vals is not None) != self.payload:
            raise ValueError("payload presence does not match the plan")
        if vals is not None and (vals.numel() != self.n or vals.element_size() != 8
                                 or not vals.is_contiguous() or not vals.is_cuda):
            raise ValueError("payload must be a contiguous device tensor of N 8-byte words")
        if keys_out is None:
            keys_out = torch.empty_like(keys)
        if vals is not None and vals_out is None:
            vals_out = torch.empty_like(vals)
        if offsets is None:
            offsets = torch.empty(self.p + 1, dtype=torch.int64, device=keys.device)
        if groups_out is None:
            groups_out = torch.empty(self.r + 1, dtype=torch.int64, device=keys.device)
        st = fn(self._h, seed & NONE, keys.data_ptr(), None if vals is None else vals.data_ptr(),
                keys_out.data_ptr(), None if vals_out is None else vals_out.data_ptr(),
                offsets.data_ptr(), groups_out.data_ptr(), _stream_handle())
        _check(st, name)
        return keys_out, vals_out, offsets, groups_out


class BatchPlan:
    """Many independent instances partitioned in the same launches.

    shapes: list of (n, p, eps, key_bytes).  Every call passes one
    (keys, seed[, vals]) per instance, in the same order."""

    def __init__(self, shapes, payload: bool = False, max_rounds: int = 0, k_override: int = 0,
                 force_full_sample: bool = False, autotune: bool = False, probes_per_round: int = 0,
                 workspace_limit_mib: int = 0):
        self.shapes = [(int(n), int(p), float(e), int(kb)) for (n, p, e, kb) in shapes]
        arr = (_Shape * len(self.shapes))()
        for i, (n, p, e, kb) in enumerate(self.shapes):
            arr[i] = _Shape(n, p, HSS_U64 if kb == 8 else HSS_U32, e)
        tun = _Tuning(max_rounds, k_override, 1 if force_full_sample else 0, 0, 0, probes_per_round,
                      0, 1 if autotune else 0, workspace_limit_mib)
        h = _vp()
        _check(_lib.hss_batch_plan(C.byref(h), arr, len(self.shapes), 1 if payload else 0,
                                   C.byref(tun)), "hss_batch_plan")
        self._h = h
        self.payload = payload

    def close(self):
        if getattr(self, "_h", None):
            _lib.hss_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.hss_batch_workspace_bytes(self._h))

    def partition(self, keys, seeds, vals=None, keys_out=None, vals_out=None, offsets=None):
        """keys: list of device tensors (one per instance); seeds: list of ints.
        Returns (keys_out, vals_out, offsets), lists in instance order."""
        torch = _torch()
        B = len(self.shapes)
        if len(keys) != B or len(seeds) != B:
            raise ValueError("one key tensor and one seed per instance")
        if (vals is not None) != self.payload:
            raise ValueError("payload presence does not match the batch")
        keys_out = keys_out or [torch.empty_like(k) for k in keys]
        vals_out = vals_out or ([torch.empty_like(v) for v in vals] if vals is not None else None)
        offsets = offsets or [torch.empty(s[1] + 1, dtype=torch.int64, device=keys[0].device)
                              for s in self.shapes]
        io = (_IO * B)()
        for i, (n, p, _, kb) in enumerate(self.shapes):
            k = keys[i]
            if (not k.is_cuda or not k.is_contiguous() or k.numel() != n
                    or k.element_size() != kb):
                raise ValueError(f"keys of instance {i} do not match its shape")
            io[i] = _IO(seeds[i] & NONE, k.data_ptr(),
                        vals[i].data_ptr() if vals is not None else None,
                        keys_out[i].data_ptr(),
                        vals_out[i].data_ptr() if vals_out is not None else None,
                        offsets[i].data_ptr())
        _check(_lib.hss_batch_partition(self._h, io, _stream_handle()), "hss_batch_partition")
        return keys_out, vals_out, offsets

    def knobs(self, key_bytes: int = 8) -> dict:
        k = _Knobs()
        _check(_lib.hss_batch_knobs(self._h, HSS_U64 if key_bytes == 8 else HSS_U32, C.byref(k)),
               "hss_batch_knobs")
        return k.as_dict()

    def profile(self, enable: bool = True):
        _check(_lib.hss_batch_profile(self._h, 1 if enable else 0), "hss_batch_profile")

    def profile_reset(self):
        _check(_lib.hss_batch_profile_reset(self._h), "hss_batch_profile_reset")

    def profile_read(self) -> dict:
        out = {}
        for i, name in enumerate(PROFILE_FAMILIES):
            ms, n, b = C.c_double(), C.c_uint64(), C.c_uint64()
            _check(_lib.hss_batch_profile_read(self._h, i, C.byref(ms), C.byref(n), C.byref(b)),
                   "hss_batch_profile_read")
            out[name] = (float(ms.value), int(n.value), int(b.value))
        return out


@dataclass
class Served:
    """A finished request: its outputs and its times on the server clock."""
    keys_out: object
    vals_out: object
    offsets: object
    t_submit: float
    t_done: float


class Server:
    """Requests of any shape served as they arrive, with continuous batching:
    the library's worker threads (each on its own stream) run the queued
    requests (same operation, key width and payload choice) as batches, a
    sort request alone, admitted under an HBM budget, so batches overlap on
    the device; each result equals the plain partition (or sort) of that
    request."""

    def __init__(self, max_batch_keys: int = 0, max_batch_requests: int = 0, workers: int = 0,
                 hbm_budget: int = 0, batch_wait_us: int = 0):
        h = _vp()
        cfg = _ServerConfig(max_batch_keys, max_batch_requests, workers, hbm_budget, batch_wait_us)
        _check(_lib.hss_server_create(C.byref(h), C.byref(cfg)), "hss_server_create")
        self._h = h
        self._live = {}

    @staticmethod
    def clock() -> float:
        return float(_lib.hss_server_clock())

    def submit(self, keys, p: int, eps: float, seed: int, vals=None, keys_out=None, vals_out=None,
               offsets=None, sync: bool = True, op: str = "partition") -> int:
        """Queue one request (op "partition" or "sort"); returns its ticket.
        With sync, the current stream is synchronised first, so that the
        inputs are complete."""
        torch = _torch()
        if not keys.is_cuda or not keys.is_contiguous():
            raise ValueError("keys must be a contiguous device tensor")
        n = keys.numel()
        keys_out = torch.empty_like(keys) if keys_out is None else keys_out
        if vals is not None and vals_out is None:
            vals_out = torch.empty_like(vals)
        offsets = (torch.empty(p + 1, dtype=torch.int64, device=keys.device)
                   if offsets is None else offsets)
        if sync:
            torch.cuda.current_stream().synchronize()
        if op not in _OPS:
            raise ValueError(f"op must be one of {sorted(_OPS)}")
        req = _Request(n, p, _key_type(keys), eps, seed & NONE, keys.data_ptr(),
                       vals.data_ptr() if vals is not None else None, keys_out.data_ptr(),
                       vals_out.data_ptr() if vals_out is not None else None, offsets.data_ptr(),
                       _OPS[op])
        t = _u64()
        _check(_lib.hss_server_submit(self._h, C.byref(req), C.byref(t)), "hss_server_submit")
        self._live[int(t.value)] = (keys, vals, keys_out, vals_out, offsets)
        return int(t.value)

    def _retire(self, ticket, st, ts, td) -> Served:
        keys, vals, ko, vo, off = self._live.pop(ticket)
        _check(st, f"request {ticket}")
        return Served(ko, vo, off, ts, td)

    def poll(self, ticket: int):
        """None while the request runs, else its Served record."""
        done, st, ts, td = C.c_int(), C.c_int(), _dbl(), _dbl()
        _check(_lib.hss_server_poll(self._h, ticket, C.byref(done), C.byref(st), C.byref(ts),
                                    C.byref(td)), "hss_server_poll")
        if not done.value:
            return None
        return self._retire(ticket, st.value, ts.value, td.value)

    def wait(self, ticket: int) -> Served:
        st, ts, td = C.c_int(), _dbl(), _dbl()
        _check(_lib.hss_server_wait(self._h, ticket, C.byref(st), C.byref(ts), C.byref(td)),
               "hss_server_wait")
        return self._retire(ticket, st.value, ts.value, td.value)

    def cancel(self, ticket: int) -> bool:
        """Take a queued request out of the queue (True); False when a worker
        already took it (it finishes).  A cancelled ticket is still retired by
        poll or wait, which raise HssError with status "cancelled"."""
        c = C.c_int()
        _check(_lib.hss_server_cancel(self._h, ticket, C.byref(c)), "hss_server_cancel")
        return bool(c.value)

    def stats(self) -> dict:
        b, r, k, mc, ma = _u64(), _u64(), _u64(), _u32(), _u64()
        _check(_lib.hss_server_stats(self._h, C.byref(b), C.byref(r), C.byref(k), C.byref(mc),
                                     C.byref(ma)), "hss_server_stats")
        return {"batches": int(b.value), "requests": int(r.value), "keys": int(k.value),
                "max_concurrent_batches": int(mc.value), "max_admitted_bytes": int(ma.value)}

    def memory(self) -> dict:
        """Device bytes held by the server's block cache, now and at most."""
        h, m = _u64(), _u64()
        _check(_lib.hss_server_memory(self._h, C.byref(h), C.byref(m)), "hss_server_memory")
        return {"held_bytes": int(h.value), "max_held_bytes": int(m.value)}

    @staticmethod
    def footprint(n: int, p: int, key_bytes: int = 8, payload: bool = False) -> int:
        """Budget bytes of a request of this shape."""
        req = _Request(n, p, HSS_U64 if key_bytes == 8 else HSS_U32, 0.05, 0, None,
                       1 if payload else None, None, None, None)
        return int(_lib.hss_server_footprint(C.byref(req)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.hss_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _plan_for(keys, p, eps, vals, tuning):
    return Plan(keys.numel(), p, eps, key_bytes=keys.element_size(), payload=vals is not None,
                **tuning)


def partition(keys, p: int, eps: float, seed: int, vals=None, **tuning):
    """HSS partition of `keys` into p buckets; returns (keys_out, vals_out, offsets)."""
    with _plan_for(keys, p, eps, vals, tuning) as plan:
        return plan.partition(keys, seed, vals)


def sort(keys, p: int, eps: float, seed: int, vals=None, **tuning):
    """Stable sort of `keys` through HSS; returns (keys_out, vals_out, offsets)."""
    with _plan_for(keys, p, eps, vals, tuning) as plan:
        return plan.sort(keys, seed, vals)


_lib.hss_partition_static.argtypes = [_u64, _u32, C.c_double, C.c_int, _u64, _vp, _vp, _vp, _vp,
                                      _vp, _vp]
_lib.hss_partition_static.restype = C.c_int
_lib.hss_partition_static_bytes.argtypes = [_u64, _u32, C.c_double, C.c_int, C.c_int, _vp, _vp]
_lib.hss_partition_static_bytes.restype = C.c_int
_lib.hss_partition_ws.argtypes = [_u64, _u32, C.c_double, C.c_int, _u64, _vp, _vp, _vp, _vp, _vp, _vp,
                                  C.c_size_t, _vp]
_lib.hss_partition_ws.restype = C.c_int
_lib.hss_partition_workspace_bytes.argtypes = [_u64, _u32, C.c_double, C.c_int, C.c_int,
                                               C.POINTER(C.c_size_t)]
_lib.hss_partition_workspace_bytes.restype = C.c_int


def partition_static(keys, p: int, eps: float, seed: int, vals=None, keys_out=None,
                     vals_out=None, offsets=None):
    """hss_partition_static: the partition of hss_partition with the library's
    fixed device workspace (no device allocation by the library); outputs
    are allocated here unless given.  Returns (keys_out, vals_out, offsets)."""
    torch = _torch()
    if not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous device tensor")
    if vals is not None and (vals.numel() != keys.numel() or vals.element_size() != 8
                             or not vals.is_contiguous() or not vals.is_cuda):
        raise ValueError("payload must be a contiguous device tensor of N 8-byte words")
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    if offsets is None:
        offsets = torch.empty(p + 1, dtype=torch.int64, device=keys.device)
    st = _lib.hss_partition_static(keys.numel(), p, eps, _key_type(keys), seed & NONE,
                                   keys.data_ptr(), None if vals is None else vals.data_ptr(),
                                   keys_out.data_ptr(),
                                   None if vals_out is None else vals_out.data_ptr(),
                                   offsets.data_ptr(), _stream_handle())
    _check(st, "hss_partition_static")
    return keys_out, vals_out, offsets


def partition_ws(keys, p: int, eps: float, seed: int, workspace, vals=None, keys_out=None,
                 vals_out=None, offsets=None):
    """hss_partition_ws: the partition of hss_partition in the caller's device
    workspace (a contiguous device tensor of at least workspace_bytes(...)
    bytes); the library allocates no device memory.  Returns (keys_out,
    vals_out, offsets)."""
    torch = _torch()
    if not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous device tensor")
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("the workspace must be a contiguous device tensor")
    if vals is not None and (vals.numel() != keys.numel() or vals.element_size() != 8
                             or not vals.is_contiguous() or not vals.is_cuda):
        raise ValueError("payload must be a contiguous device tensor of N 8-byte words")
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    if offsets is None:
        offsets = torch.empty(p + 1, dtype=torch.int64, device=keys.device)
    st = _lib.hss_partition_ws(keys.numel(), p, eps, _key_type(keys), seed & NONE,
                               keys.data_ptr(), None if vals is None else vals.data_ptr(),
                               keys_out.data_ptr(), None if vals_out is None else vals_out.data_ptr(),
                               offsets.data_ptr(), workspace.data_ptr(),
                               workspace.numel() * workspace.element_size(), _stream_handle())
    _check(st, "hss_partition_ws")
    return keys_out, vals_out, offsets


def workspace_bytes(n: int, p: int, eps: float, key_bytes: int = 8, payload: bool = False) -> int:
    """Bytes of workspace a hss_partition_ws call of this shape needs."""
    b = C.c_size_t()
    _check(_lib.hss_partition_workspace_bytes(n, p, eps, HSS_U64 if key_bytes == 8 else HSS_U32,
                                              1 if payload else 0, C.byref(b)),
           "hss_partition_workspace_bytes")
    return int(b.value)


def static_workspace_bytes(n: int, p: int, eps: float, key_bytes: int = 8,
                           payload: bool = False):
    """(status, bytes of the fixed workspace a call of this shape takes, its size)."""
    b, c = C.c_size_t(), C.c_size_t()
    st = _lib.hss_partition_static_bytes(n, p, eps, HSS_U64 if key_bytes == 8 else HSS_U32,
                                         1 if payload else 0, C.byref(b), C.byref(c))
    return int(st), int(b.value), int(c.value)


_lib.hss_stream_copy.argtypes = [_vp, _vp, C.c_size_t, _u32, C.c_int, _vp]
_lib.hss_stream_copy.restype = C.c_int


def stream_copy(dst, src, workgroups: int = 4096, nontemporal: bool = False):
    """Copy the device tensor src into dst (same byte size, a multiple of 16)
    with the library's streaming copy kernel (a bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    _check(_lib.hss_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, workgroups,
                                1 if nontemporal else 0, _stream_handle()), "hss_stream_copy")


def exported_symbols():
    """Names of the C-ABI entry points present in the loaded library."""
    return [name for name in EXPORTS if hasattr(_lib, name)]
