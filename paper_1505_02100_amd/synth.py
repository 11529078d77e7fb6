"""Seeded synthetic samples shaped like the workloads of the PLUGIN selector.

This module only draws random numbers; it holds none of the selector's
arithmetic, so both the HIP path and the FP64 oracle consume its bytes.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used as a counter-based stream: the k-th
64-bit word of stream ``seed`` is ``mix64(seed + (k + 1) * 0x9E3779B97F4A7C15)``.
Uniforms take the top 53 bits; normals use the Box-Muller transform.

Workload shapes (the paper publishes neither its datasets nor their
distributions; these stand in for them):
  * ``normal``    N(0, 1)
  * ``bimodal``   0.5 N(-1, (2/3)^2) + 0.5 N(1, (2/3)^2)
  * ``lognormal`` a * exp(Z) + b with Z ~ N(0, 1)
  * ``t3``        Student t with 3 degrees of freedom
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_scalar(x: int) -> int:
    """One SplitMix64 step on a Python int (used to derive per-dataset seeds)."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


class Stream:
    """Counter-based SplitMix64 stream; draws are consumed in order."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & _MASK)
        self.counter = 0

    def words(self, m: int) -> np.ndarray:
        k = np.arange(self.counter + 1, self.counter + 1 + m, dtype=np.uint64)
        self.counter += m
        with np.errstate(over="ignore"):
            return _mix64(self.seed + k * _GAMMA)

    def uniform(self, m: int) -> np.ndarray:
        """Uniforms in [0, 1) with 53 random bits."""
        return (self.words(m) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def uniform_open(self, m: int) -> np.ndarray:
        """Uniforms in (0, 1]."""
        return 1.0 - self.uniform(m)

    def normal(self, m: int) -> np.ndarray:
        half = (m + 1) // 2
        u1 = self.uniform_open(half)
        u2 = self.uniform(half)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)])
        return z[:m]


def normal(n: int, seed: int, mu: float = 0.0, sigma: float = 1.0) -> np.ndarray:
    return mu + sigma * Stream(seed).normal(n)


def bimodal(n: int, seed: int) -> np.ndarray:
    """0.5 N(-1, (2/3)^2) + 0.5 N(1, (2/3)^2); (2/3)^2 read as the variance."""
    s = Stream(seed)
    pick = s.uniform(n) < 0.5
    z = s.normal(n)
    return np.where(pick, -1.0, 1.0) + (2.0 / 3.0) * z


def lognormal(n: int, seed: int, a: float = 1.0, b: float = 0.0) -> np.ndarray:
    """a * exp(Z) + b with Z ~ N(0, 1)."""
    return a * np.exp(Stream(seed).normal(n)) + b


def student_t3(n: int, seed: int) -> np.ndarray:
    s = Stream(seed)
    z = s.normal(n)
    w = s.normal(3 * n).reshape(3, n)
    chi2 = (w * w).sum(axis=0)
    return z / np.sqrt(chi2 / 3.0)


DISTS = ("normal", "bimodal", "t3")


def draw(dist: str, n: int, seed: int) -> np.ndarray:
    if dist == "normal":
        return normal(n, seed)
    if dist == "bimodal":
        return bimodal(n, seed)
    if dist == "t3":
        return student_t3(n, seed)
    if dist == "lognormal":
        return lognormal(n, seed)
    raise ValueError(f"unknown distribution {dist!r}")


def sha256(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x, dtype=np.float64).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# The five workloads (sizes and mixes).
# ---------------------------------------------------------------------------

def workload_single_normal(n: int = 1024, seed: int = 0) -> np.ndarray:
    """One dataset of n draws from N(0, 1)."""
    return normal(n, seed)


def workload_single_bimodal(n: int = 65536, seed: int = 1) -> np.ndarray:
    """One dataset of n draws from the bimodal mixture."""
    return bimodal(n, seed)


def workload_single_lognormal(n: int = 1 << 20, seed: int = 2, a: float = 1e3,
                              b: float = -5e2) -> np.ndarray:
    """One dataset a * exp(Z) + b: heavy right tail, large offset."""
    return lognormal(n, seed, a, b)


def workload_batch(count: int = 512, master: int = 3, n_lo: int = 256, n_hi: int = 65536):
    """``count`` datasets; n log-uniform in [n_lo, n_hi]; distribution chosen
    uniformly among normal / bimodal / t3.  Returns (list of arrays, list of
    distribution names)."""
    meta = Stream(master)
    u_n = meta.uniform(count)
    u_d = meta.uniform(count)
    xs, names = [], []
    for k in range(count):
        n = int(round(math.exp(math.log(n_lo) + u_n[k] * (math.log(n_hi) - math.log(n_lo)))))
        d = DISTS[min(int(u_d[k] * 3.0), 2)]
        xs.append(draw(d, n, splitmix64_scalar(master ^ k)))
        names.append(d)
    return xs, names


def serving_trace(rate: float = 200.0, duration: float = 60.0, master: int = 4,
                  n_lo: float = 1e3, n_hi: float = 4e6):
    """Poisson arrivals: returns a list of (arrival_time_s, n, dist, seed)."""
    meta = Stream(master)
    out = []
    t = 0.0
    k = 0
    while True:
        u = meta.uniform_open(3)
        t += -math.log(u[0]) / rate
        if t >= duration:
            break
        n = int(round(math.exp(math.log(n_lo) + (1.0 - u[1]) * (math.log(n_hi) - math.log(n_lo)))))
        d = DISTS[min(int((1.0 - u[2]) * 3.0), 2)]
        out.append((t, n, d, splitmix64_scalar(master ^ (k + 0x5151))))
        k += 1
    return out


# ---------------------------------------------------------------------------
# The same counter-based generator written with torch integer ops, so that
# serving workloads can draw their samples directly in device memory.  The
# uniforms are bit-identical to Stream's; the normals go through the device
# libm's log / cos / sin and may differ from numpy's in the last bit, so any
# check of a device-drawn sample copies those exact bytes back first.
# ---------------------------------------------------------------------------

def _i64(v: int) -> int:
    """Two's-complement int64 value of an unsigned 64-bit constant."""
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(z, s: int):
    """Logical right shift of an int64 tensor."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix64_t(z):
    z = (z ^ _srl(z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _srl(z, 27)) * _i64(0x94D049BB133111EB)
    return z ^ _srl(z, 31)


class TorchStream:
    """Stream's counter-based SplitMix64 sequence on a torch device."""

    def __init__(self, seed: int, device):
        self.seed = _i64(seed & _MASK)
        self.counter = 0
        self.device = device

    def words(self, m: int):
        import torch
        k = torch.arange(self.counter + 1, self.counter + 1 + m, dtype=torch.int64, device=self.device)
        self.counter += m
        return _mix64_t(self.seed + k * _i64(0x9E3779B97F4A7C15))

    def uniform(self, m: int):
        import torch
        return _srl(self.words(m), 11).to(torch.float64) * (1.0 / 9007199254740992.0)

    def uniform_open(self, m: int):
        return 1.0 - self.uniform(m)

    def normal(self, m: int):
        import torch
        half = (m + 1) // 2
        u1 = self.uniform_open(half)
        u2 = self.uniform(half)
        r = torch.sqrt(-2.0 * torch.log(u1))
        z = torch.cat([r * torch.cos(2.0 * math.pi * u2), r * torch.sin(2.0 * math.pi * u2)])
        return z[:m]


def draw_torch(dist: str, n: int, seed: int, device="cuda"):
    """draw() on a torch device (same streams and transforms)."""
    import torch
    s = TorchStream(seed, device)
    if dist == "normal":
        return s.normal(n)
    if dist == "bimodal":
        pick = s.uniform(n) < 0.5
        z = s.normal(n)
        return torch.where(pick, -1.0, 1.0).to(torch.float64) + (2.0 / 3.0) * z
    if dist == "t3":
        z = s.normal(n)
        w = s.normal(3 * n).reshape(3, n)
        return z / torch.sqrt((w * w).sum(dim=0) / 3.0)
    if dist == "lognormal":
        return torch.exp(s.normal(n))
    raise ValueError(f"unknown distribution {dist!r}")
