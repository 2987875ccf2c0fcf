"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the sorting method: it only draws keys and
payloads with numpy's PCG64 so that the CPU oracle and the GPU library see the
same host arrays.

Workloads (keys are unsigned integers, compared as unsigned):
  uniform64(n, seed)        -- uniform on [0, 2^64)
  uniform32(n, seed)        -- uniform on [0, 2^32)
  zipf_morton(n, seed)      -- half Zipf(s=1.1) over 1024 distinct 64-bit values,
                               half 63-bit Morton codes of 3-D points drawn from
                               a mixture of 8 Gaussians (sigma 0.01) in the unit
                               cube; shuffled
  paper_distribution(name)  -- the input distributions of the paper's section on
                               the effect of the input distribution: UNIF, SKEW1,
                               SKEW2, SKEW3, GAUSS, ALLZEROS
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    # name: (n, p, eps, data seed, hss seed, generator, payload)
    "uniform_2^20_p16": (1 << 20, 16, 0.05, 1, 1, "uniform64", False),
    "uniform_2^28_p1024": (1 << 28, 1024, 0.02, 2, 2, "uniform64", False),
    "zipf_morton_2^28_p4096": (1 << 28, 4096, 0.05, 3, 3, "zipf_morton", True),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform64(n: int, seed: int) -> np.ndarray:
    return np.random.PCG64(seed).random_raw(n).astype(np.uint64, copy=False)


def uniform32(n: int, seed: int) -> np.ndarray:
    return (np.random.PCG64(seed).random_raw(n) >> np.uint64(32)).astype(np.uint32)


def _part1by2(x: np.ndarray) -> np.ndarray:
    """Spread the low 21 bits of x so that bit b moves to bit 3b."""
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    x = (x | (x << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x1249249249249249)
    return x


def morton63(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray) -> np.ndarray:
    """Interleave three 21-bit coordinates: x at bit 3b, y at 3b+1, z at 3b+2."""
    return _part1by2(ix) | (_part1by2(iy) << np.uint64(1)) | (_part1by2(iz) << np.uint64(2))


def zipf_morton(n: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    nz = n // 2
    nm = n - nz
    # Zipf half: 1024 distinct random 64-bit values, bounded Zipf weights r^-1.1.
    vals = np.unique(rng.integers(0, 2**64, size=1024, dtype=np.uint64, endpoint=False))
    while len(vals) < 1024:
        extra = rng.integers(0, 2**64, size=1024 - len(vals), dtype=np.uint64, endpoint=False)
        vals = np.unique(np.concatenate([vals, extra]))
    vals = rng.permutation(vals)
    w = np.arange(1, 1025, dtype=np.float64) ** -1.1
    w /= w.sum()
    zipf = vals[rng.choice(1024, size=nz, p=w)]
    # Morton half: 8 Gaussian clusters in the unit cube, sigma 0.01.
    centres = rng.random((8, 3))
    which = rng.integers(0, 8, size=nm)
    pts = centres[which] + 0.01 * rng.standard_normal((nm, 3))
    pts = np.clip(pts, 0.0, 1.0 - 2.0 ** -21)
    q = np.floor(pts * (1 << 21)).astype(np.uint64)
    mort = morton63(q[:, 0], q[:, 1], q[:, 2])
    keys = np.concatenate([zipf, mort])
    return keys[rng.permutation(n)].astype(np.uint64)


def paper_distribution(name: str, n: int, seed: int) -> np.ndarray:
    """64-bit keys following one of the paper's six test distributions."""
    rng = _rng(seed)
    name = name.upper()
    if name == "UNIF":
        return rng.integers(0, 2**64, size=n, dtype=np.uint64)
    if name == "SKEW1":
        a = rng.integers(0, 2**64, size=n - n // 2, dtype=np.uint64)
        base = rng.integers(0, 2**64 - 1000, dtype=np.uint64)
        b = base + rng.integers(0, 1000, size=n // 2, dtype=np.uint64)
        return rng.permutation(np.concatenate([a, b]))
    if name == "SKEW2":
        return rng.integers(0, 101, size=n, dtype=np.uint64)
    if name == "SKEW3":
        return (rng.integers(0, 2**64, size=n, dtype=np.uint64)
                & rng.integers(0, 2**64, size=n, dtype=np.uint64))
    if name == "GAUSS":
        x = rng.normal(2.0**63, 2.0**60, size=n)
        x = np.clip(x, 0.0, 2.0**64 - 4096.0)
        return x.astype(np.uint64)
    if name == "ALLZEROS":
        return np.zeros(n, dtype=np.uint64)
    raise ValueError(name)


def make(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "uniform64":
        return uniform64(n, seed)
    if kind == "uniform32":
        return uniform32(n, seed)
    if kind == "zipf_morton":
        return zipf_morton(n, seed)
    return paper_distribution(kind, n, seed)


def config(name: str, n_override: int | None = None):
    """Keys (and payload = source index, where the config carries one)."""
    n, p, eps, dseed, hseed, kind, payload = CONFIGS[name]
    if n_override is not None:
        n = n_override
    keys = make(kind, n, dseed)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    return keys, vals, p, eps, hseed


def batched_shapes(count: int = 512, seed: int = 4, lo_bits: float = 12.0, hi_bits: float = 22.0):
    """Instance shapes of the batched workload: N log-uniform on
    [2^lo_bits, 2^hi_bits], p = clamp(floor(e^U(ln 8, ln 257)), 8, 256),
    eps = 0.05; the first half of the instances has 32-bit keys, the rest
    64-bit.  Returns [(n, p, eps, key_bytes, data_seed, hss_seed)]."""
    rng = _rng(seed)
    out = []
    for i in range(count):
        n = int(np.floor(2.0 ** rng.uniform(lo_bits, hi_bits)))
        p = int(np.clip(np.floor(np.exp(rng.uniform(np.log(8.0), np.log(257.0)))), 8, 256))
        p = min(p, n)
        kb = 4 if i < count // 2 else 8
        out.append((n, p, 0.05, kb, seed * 100_000 + i, 1000 + i))
    return out


def batched_keys(shape) -> np.ndarray:
    """Uniform keys of one batched instance (32-bit: the top half of a 64-bit draw)."""
    n, _p, _eps, kb, dseed, _hseed = shape
    k = uniform64(n, dseed)
    return (k >> np.uint64(32)).astype(np.uint32) if kb == 4 else k


def served_shapes(count: int = 20_000, seed: int = 5, lo_bits: float = 14.0, hi_bits: float = 26.0):
    """Request shapes of the served workload: N log-uniform on
    [2^lo_bits, 2^hi_bits], p = clamp(floor(e^U(ln 64, ln 2049)), 64, 2048)
    (at most N), eps drawn from {0.02, 0.05}; 64-bit keys with a payload.
    Returns [(n, p, eps, data_seed, hss_seed)]."""
    rng = _rng(seed)
    out = []
    for i in range(count):
        n = int(np.floor(2.0 ** rng.uniform(lo_bits, hi_bits)))
        p = int(np.clip(np.floor(np.exp(rng.uniform(np.log(64.0), np.log(2049.0)))), 64, 2048))
        eps = 0.02 if rng.integers(0, 2) == 0 else 0.05
        out.append((n, min(p, n), eps, seed * 1_000_000 + i, 1_000_000 + i))
    return out


def device_keys(n: int, data_seed: int, device):
    """Uniform 64-bit keys drawn on the device (the served workload's inputs,
    too many to stage from the host): torch's generator seeded with
    data_seed.  Returns an int64 tensor (keys compare as unsigned)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(data_seed)
    return torch.randint(-(1 << 63), (1 << 63) - 1, (n,), dtype=torch.int64, device=device, generator=g)
