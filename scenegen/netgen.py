"""Seeded inputs for the proposal network's tests: feature maps, parameter
vectors and training targets whose values are exactly representable in
bfloat16, so that the device (bf16 storage) and the float64 reference see the
same numbers.  Generation only: no network arithmetic lives here."""
from __future__ import annotations

import numpy as np


def bf16_representable(x) -> np.ndarray:
    """float32 copy of x rounded to the nearest bfloat16 value (ties to even)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def random_features(seed: int, n: int, h: int, w: int, c: int = 16) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return bf16_representable(rng.standard_normal((n, h, w, c)))


def random_params(seed: int, layers, scale: float = 1.0) -> np.ndarray:
    """Canonical flat vector for a layer table of (name, c_in, c_out, k): He-scaled
    weights [c_out][k][k][c_in], small biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, k in layers:
        parts.append(rng.standard_normal(co * k * k * ci) * scale * np.sqrt(2.0 / (k * k * ci)))
        parts.append(rng.standard_normal(co) * 0.1)
    return bf16_representable(np.concatenate(parts))


def random_targets(seed: int, n: int, h: int, w: int, d_min: float = 2.0, d_max: float = 6.0) -> np.ndarray:
    """(n, h, w, 6) float32: depth, unit normal facing -z, confidence target, weight 0/1."""
    rng = np.random.default_rng(seed)
    t = np.zeros((n, h, w, 6), np.float32)
    t[..., 0] = rng.uniform(d_min, d_max, (n, h, w))
    nv = rng.standard_normal((n, h, w, 3)) * 0.3
    nv[..., 2] = -1.0
    t[..., 1:4] = nv / np.linalg.norm(nv, axis=-1, keepdims=True)
    t[..., 4] = rng.uniform(0, 1, (n, h, w))
    t[..., 5] = (rng.uniform(0, 1, (n, h, w)) < 0.8)
    return t


def random_q_ref(seed: int, n: int, h: int, w: int, d_min: float = 2.0, d_max: float = 6.0) -> np.ndarray:
    """(n, h, w) float32 inverse depths inside [1/d_max, 1/d_min] (a plane sweep's winners)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(1.0 / d_max, 1.0 / d_min, (n, h, w)).astype(np.float32)
