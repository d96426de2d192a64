"""Seeded, chunk-addressable synthetic workloads.

This module only draws random numbers and lays out channel descriptors.  It
holds none of the filtering arithmetic, so both the GPU path and the FP64
oracle can be fed from it.

Every sample is complex Gaussian CN(0,1): real and imaginary parts are i.i.d.
N(0, 1/2).  Sample t of channel c depends only on (seed, config, c, t): it is
element t mod 2^16 of chunk t // 2^16, drawn from
``numpy.random.default_rng([seed, config, c, 1, chunk])``, so any block can be
regenerated on its own.  Per-channel parameters are drawn from
``default_rng([seed, config, c, 0])`` in the fixed order (len, N, f, L_V,
f_switch); a parameter that a configuration fixes is still drawn and ignored,
so the draw order never shifts.

Transition values V (one shared set per (N, L_V) key) are L_V uniform (0,1)
draws sorted in decreasing order, redrawn until they stay strictly decreasing
and inside (0,1) after rounding to float32; they are returned as float64
holding float32-exact values, which is what the filter and the oracle both use.

Passband width: a fraction f of the half band maps to the first transition bin
k1 = max(1, round(f N / 2)), i.e. passband bins [0, k1) and their mirror.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 16
DEFAULT_SEED = 2406


@dataclass
class Channel:
    n: int
    hop: int
    lv: int
    length: int
    k1: int
    v_key: tuple
    schedule: list = field(default_factory=list)  # [(from_block, k1)], sorted

    def full_schedule(self):
        return [(0, self.k1)] + list(self.schedule)

    def n_blocks(self) -> int:
        return 0 if self.length <= 0 else -(-self.length // self.hop)


@dataclass
class Workload:
    name: str
    seed: int
    config: int
    channels: list
    v_sets: dict            # v_key -> float64 array (float32-exact)
    storage: str = "c64"    # "c64", "c128", "f16", "bf16"
    description: str = ""

    def total_samples(self) -> int:
        return int(sum(c.length for c in self.channels))

    def v_pool(self):
        """Concatenate the V sets; returns (pool, {v_key: offset})."""
        offs, parts, o = {}, [], 0
        for key in sorted(self.v_sets):
            offs[key] = o
            parts.append(self.v_sets[key])
            o += len(self.v_sets[key])
        pool = np.concatenate(parts) if parts else np.zeros(0)
        return pool.astype(np.float64), offs


def draw_v(seed: int, config: int, n: int, lv: int) -> np.ndarray:
    rng = np.random.default_rng([seed, config, 1 << 20, n, lv])
    while True:
        v = np.sort(rng.random(lv))[::-1].astype(np.float32)
        ok = lv == 0 or (v[0] < 1.0 and v[-1] > 0.0 and np.all(np.diff(v) < 0))
        if ok:
            return v.astype(np.float64)


def _param_draws(seed: int, config: int, ch: int) -> np.ndarray:
    return np.random.default_rng([seed, config, ch, 0]).random(5)


def k1_of(f: float, n: int) -> int:
    return max(1, int(round(f * n / 2)))


def _chunk(seed: int, config: int, ch: int, c: int) -> np.ndarray:
    z = np.random.default_rng([seed, config, ch, 1, c]).standard_normal((CHUNK, 2))
    x = np.empty(CHUNK, dtype=np.complex128)
    x.real = z[:, 0]
    x.imag = z[:, 1]
    x *= 1.0 / math.sqrt(2.0)
    return x


def samples(seed: int, config: int, ch: int, start: int, count: int,
            dtype=np.complex128) -> np.ndarray:
    """Samples [start, start+count) of channel ch (complex128 or complex64)."""
    out = np.empty(count, dtype=dtype)
    if count <= 0:
        return out
    c0, c1 = start // CHUNK, (start + count - 1) // CHUNK
    for c in range(c0, c1 + 1):
        lo = max(start, c * CHUNK)
        hi = min(start + count, (c + 1) * CHUNK)
        out[lo - start:hi - start] = _chunk(seed, config, ch, c)[lo - c * CHUNK:hi - c * CHUNK]
    return out


def channel_samples(w: Workload, ch: int, dtype=np.complex128, threads: int = 0) -> np.ndarray:
    """All samples of one channel, chunks drawn in parallel threads."""
    length = w.channels[ch].length
    out = np.empty(length, dtype=dtype)
    nchunks = -(-length // CHUNK)

    def fill(c):
        lo, hi = c * CHUNK, min(length, (c + 1) * CHUNK)
        out[lo:hi] = _chunk(w.seed, w.config, ch, c)[:hi - lo]

    threads = threads or min(16, os.cpu_count() or 1)
    if nchunks <= 1 or threads <= 1:
        for c in range(nchunks):
            fill(c)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, range(nchunks)))
    return out


def _make(name, seed, config, chans, storage="c64", description=""):
    v_sets = {}
    for c in chans:
        if c.v_key not in v_sets:
            v_sets[c.v_key] = draw_v(seed, config, c.v_key[0], c.v_key[1])
    return Workload(name=name, seed=seed, config=config, channels=chans,
                    v_sets=v_sets, storage=storage, description=description)


def config1(seed: int = DEFAULT_SEED) -> Workload:
    """One channel of 65,536 complex128 samples; N=256, hop 192; passband bins
    [0,24) (k1 = 24) and mirror; 8 transition values per edge."""
    n, hop, lv = 256, 192, 8
    _param_draws(seed, 1, 0)
    chans = [Channel(n=n, hop=hop, lv=lv, length=65536, k1=24, v_key=(n, lv))]
    return _make("plain-1ch-n256", seed, 1, chans, storage="c128",
                 description="1 ch x 65536 complex128, N=256, hop=192, k1=24, L_V=8")


def config2(seed: int = DEFAULT_SEED, n_channels: int = 64, length: int = 1 << 20) -> Workload:
    """64 channels x 2^20 complex64; N=1024, hop 768; passband width f ~ U[5%,45%]
    per channel; 16 shared transition values per edge; every channel switches
    to a second independent width draw at block 512."""
    n, hop, lv = 1024, 768, 16
    chans = []
    for c in range(n_channels):
        u = _param_draws(seed, 2, c)
        k1 = k1_of(0.05 + 0.40 * u[2], n)
        k1s = k1_of(0.05 + 0.40 * u[4], n)
        chans.append(Channel(n=n, hop=hop, lv=lv, length=length, k1=k1,
                             v_key=(n, lv), schedule=[(512, k1s)]))
    return _make("fp32-64ch-n1024-switch512", seed, 2, chans,
                 description=f"{n_channels} ch x {length} complex64, N=1024, hop=768, "
                             "L_V=16, switch at block 512")


def config3(seed: int = DEFAULT_SEED, n_channels: int = 512) -> Workload:
    """512 channels, length log-uniform in [2^14, 2^20], N uniform over
    {256, 512, 1024, 2048} with hop 3N/4, f ~ U[1%,50%], L_V ~ U{8..32};
    V shared per (N, L_V)."""
    chans = []
    for c in range(n_channels):
        u = _param_draws(seed, 3, c)
        length = int(round(2.0 ** (14.0 + 6.0 * u[0])))
        n = (256, 512, 1024, 2048)[min(3, int(4 * u[1]))]
        lv = 8 + min(24, int(25 * u[3]))
        k1 = k1_of(0.01 + 0.49 * u[2], n)
        chans.append(Channel(n=n, hop=3 * n // 4, lv=lv, length=length, k1=k1,
                             v_key=(n, lv)))
    return _make("batched-512ch-mixedN", seed, 3, chans,
                 description=f"{n_channels} ch, len log-uniform [2^14,2^20], "
                             "N in {256,512,1024,2048}, hop=3N/4, L_V 8..32")


def config4(seed: int = DEFAULT_SEED, storage: str = "f16", n_channels: int = 256,
            length: int = 1 << 20) -> Workload:
    """256 channels x 2^20 samples stored as FP16 or BF16 pairs; N=256, hop 192;
    f ~ U[5%,45%]; L_V = 8."""
    n, hop, lv = 256, 192, 8
    chans = []
    for c in range(n_channels):
        u = _param_draws(seed, 4, c)
        chans.append(Channel(n=n, hop=hop, lv=lv, length=length,
                             k1=k1_of(0.05 + 0.40 * u[2], n), v_key=(n, lv)))
    return _make(f"{storage}-256ch-n256", seed, 4, chans, storage=storage,
                 description=f"{n_channels} ch x {length} {storage} pairs, N=256, hop=192, L_V=8")


def config5(seed: int = DEFAULT_SEED, n_channels: int = 256, length: int = 1 << 22) -> Workload:
    """256 channels x 2^22 complex64; N=4096, hop 3072; f ~ U[0.5%,10%];
    32 transition values per edge (narrow band, pruned inverse)."""
    n, hop, lv = 4096, 3072, 32
    chans = []
    for c in range(n_channels):
        u = _param_draws(seed, 5, c)
        chans.append(Channel(n=n, hop=hop, lv=lv, length=length,
                             k1=k1_of(0.005 + 0.095 * u[2], n), v_key=(n, lv)))
    return _make("narrow-256ch-n4096", seed, 5, chans,
                 description=f"{n_channels} ch x {length} complex64, N=4096, hop=3072, L_V=32")


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def custom(channels, seed: int = DEFAULT_SEED, config: int = 99, storage: str = "c64",
           name: str = "custom") -> Workload:
    """Workload from explicit channel descriptors (test cases)."""
    return _make(name, seed, config, list(channels), storage=storage)
