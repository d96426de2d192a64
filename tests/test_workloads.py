"""Seeded workload generator: determinism, chunk addressing, statistics and the
shapes of the five benchmark configurations."""
import numpy as np
import pytest

from paper_2406_14116_amd import workloads as wl


def test_chunk_addressable_and_deterministic():
    w = wl.config3(n_channels=4)
    ch = 2
    full = wl.channel_samples(w, ch)
    assert len(full) == w.channels[ch].length
    for start, count in [(0, 10), (wl.CHUNK - 3, 7), (5, 3 * wl.CHUNK // 2)]:
        count = min(count, len(full) - start)
        if count <= 0:
            continue
        part = wl.samples(w.seed, w.config, ch, start, count)
        assert np.array_equal(part, full[start:start + count])
    assert np.array_equal(full, wl.channel_samples(wl.config3(n_channels=4), ch, threads=1))


def test_unit_variance_complex_gaussian():
    x = wl.samples(1, 2, 0, 0, 1 << 18)
    assert abs(np.mean(x)) < 0.01
    assert abs(np.mean(np.abs(x) ** 2) - 1.0) < 0.01
    assert abs(np.var(x.real) - 0.5) < 0.01 and abs(np.var(x.imag) - 0.5) < 0.01


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_config_shapes(cfg):
    w = wl.CONFIGS[cfg]()
    for c in w.channels:
        assert c.n & (c.n - 1) == 0 and (c.n - c.hop) % 2 == 0
        for _, k1 in c.full_schedule():
            assert 1 <= k1 and k1 + c.lv - 1 <= c.n // 2 - 1
        v = w.v_sets[c.v_key]
        assert len(v) == c.lv
        assert np.all(np.diff(v) < 0) and v[0] < 1 and v[-1] > 0
        assert np.array_equal(v, v.astype(np.float32).astype(np.float64))
    if cfg == 1:
        assert (w.channels[0].k1, w.channels[0].length, w.storage) == (24, 65536, "c128")
    if cfg == 2:
        assert len(w.channels) == 64 and all(c.schedule[0][0] == 512 for c in w.channels)
        assert w.channels[0].n_blocks() == 1366
    if cfg == 3:
        assert len(w.channels) == 512
        assert {c.n for c in w.channels} == {256, 512, 1024, 2048}
        lens = [c.length for c in w.channels]
        assert min(lens) >= 2 ** 14 and max(lens) <= 2 ** 20
        assert {c.lv for c in w.channels} <= set(range(8, 33))
    if cfg == 5:
        k2 = [c.k1 + c.lv - 1 for c in w.channels]
        assert 2 * max(k2) + 1 <= 473
