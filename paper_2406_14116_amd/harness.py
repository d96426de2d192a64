"""Device-side plumbing for workloads: upload seeded inputs as torch tensors in
the storage layout of include/vbw.h, allocate outputs, read slices back.

Marshalling only; the filtering itself runs in libvbw.so.
"""
from __future__ import annotations

import numpy as np

from . import workloads as wl


def _torch():
    import torch
    return torch


def host_to_storage(x: np.ndarray, dtype: str):
    """complex numpy array -> torch CPU tensor in the storage layout."""
    torch = _torch()
    if dtype == "c64":
        return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64)))
    if dtype == "r32":                      # real input: the real parts
        return torch.from_numpy(np.ascontiguousarray(x.real.astype(np.float32)))
    pairs = np.stack([x.real, x.imag], axis=1).astype(np.float32)
    t = torch.from_numpy(np.ascontiguousarray(pairs))
    # float32 -> float16 / bfloat16 conversion rounds to nearest-even
    return t.to(torch.float16 if dtype == "f16" else torch.bfloat16)


def storage_to_c128(t) -> np.ndarray:
    """torch tensor in a storage layout (any device) -> complex128 numpy."""
    torch = _torch()
    t = t.detach().to("cpu")
    if t.dtype == torch.complex64:
        return t.numpy().astype(np.complex128)
    if t.dtype == torch.float32 and t.dim() == 1:     # real storage
        return t.numpy().astype(np.complex128)
    f = t.to(torch.float32).numpy().reshape(-1, 2).astype(np.float64)
    return f[:, 0] + 1j * f[:, 1]


def upload_channel(w: wl.Workload, ch: int, dtype: str, device="cuda"):
    x = wl.channel_samples(w, ch, dtype=np.complex64 if dtype in ("c64", "r32") else np.complex128)
    return host_to_storage(x, dtype).to(device)


def upload_inputs(w: wl.Workload, dtype: str, device="cuda"):
    return [upload_channel(w, c, dtype, device) for c in range(len(w.channels))]


def alloc_outputs(w: wl.Workload, dtype: str, f32_out: bool = False, device="cuda"):
    torch = _torch()
    outs = []
    for c in w.channels:
        if dtype == "r32":
            outs.append(torch.empty(c.length, dtype=torch.float32, device=device))
        elif dtype == "c64" or f32_out:
            outs.append(torch.empty(c.length, dtype=torch.complex64, device=device))
        else:
            tdt = torch.float16 if dtype == "f16" else torch.bfloat16
            outs.append(torch.empty((c.length, 2), dtype=tdt, device=device))
    return outs


def block_slice(t, hop: int, block: int, length: int):
    """Output samples of one block (truncated at the channel length)."""
    lo = block * hop
    hi = min(length, lo + hop)
    return t[lo:hi]


def sample_blocks(n_blocks: int, rng: np.random.Generator, switch_block=None, n_random: int = 8):
    """Blocks {0, 1, last-1, last}, {s-1, s, s+1} around the band switch s
    (an int, or every one of an iterable), plus seeded random ones."""
    s = {0, 1, n_blocks - 2, n_blocks - 1}
    switches = [] if switch_block is None else ([switch_block] if np.isscalar(switch_block) else list(switch_block))
    for sw in switches:
        s |= {int(sw) - 1, int(sw), int(sw) + 1}
    if n_blocks > 0:
        s |= set(int(b) for b in rng.integers(0, n_blocks, size=n_random))
    return sorted(b for b in s if 0 <= b < n_blocks)
