"""Pins for the FP64 oracle: each test checks it against something other than
itself -- a library routine, a closed form from the paper, brute force on tiny
sizes, or a structural property of overlap-save -- chosen so that a dropped
term, a wrong sign or index, or a transposed operand fails at least one.

Paper: Moryakova & Johansson, arXiv 2406.14116.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import ols


def crandn(rng, n):
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)


def db(a, b):
    return ols.error_db(a, b)


def run_generic(x, n, hop, H):
    """Whole-channel output of the generic-H oracle, truncated to len(x)."""
    out = ols.blocks_generic(x, n, hop, H)
    return out.reshape(-1)[: len(x)]


# --- transforms: library routine, closed forms, Parseval --------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 64, 256])
def test_dft_matches_numpy_fft(n):
    rng = np.random.default_rng(n)
    s = crandn(rng, n)
    X = ols.dft(s)
    np.testing.assert_allclose(X, np.fft.fft(s), rtol=0, atol=1e-12 * max(1, n))


@pytest.mark.parametrize("n", [4, 16, 128])
def test_idft_sign_and_scale(n):
    """Eq. (4): a unit bin at k0 inverts to exp(+j 2 pi k0 q / N) / N."""
    for k0 in (0, 1, n // 2 - 1, n - 1):
        Y = np.zeros(n, complex)
        Y[k0] = 1.0
        z = ols.idft(Y)
        q = np.arange(n)
        np.testing.assert_allclose(z, np.exp(2j * np.pi * k0 * q / n) / n, atol=1e-15)


@pytest.mark.parametrize("n", [16, 1024])
def test_dft_parseval_and_tone(n):
    rng = np.random.default_rng(7)
    s = crandn(rng, n)
    X = ols.dft(s)
    assert abs(np.sum(abs(s) ** 2) - np.sum(abs(X) ** 2) / n) <= 1e-12 * np.sum(abs(s) ** 2)
    k0 = 3
    tone = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    X = ols.dft(tone)
    expect = np.zeros(n, complex)
    expect[k0] = n
    np.testing.assert_allclose(X, expect, atol=1e-9)
    np.testing.assert_allclose(ols.idft(ols.dft(s)), s, atol=1e-13)


# --- time-invariant special case: exact linear convolution ----------------------

@pytest.mark.parametrize("n,hop,length", [(16, 12, 100), (16, 10, 97), (64, 48, 64 * 5 + 1),
                                          (256, 192, 65536 // 16), (32, 2, 50), (8, 6, 1)])
def test_ti_case_is_linear_convolution(n, hop, length):
    """Sec. II: with H = DFT_N(h) and h zero from index L = N - M + 1 on, OLS is
    exactly the linear convolution; the zero-history framing makes the output
    equal (h * x)[:len]."""
    rng = np.random.default_rng(n * 1000 + hop)
    x = crandn(rng, length)
    lfilt = n - hop + 1
    h = crandn(rng, lfilt)
    H = np.fft.fft(np.concatenate([h, np.zeros(n - lfilt)]))
    y = run_generic(x, n, hop, H)
    ref = np.convolve(x, h)[:length]
    assert db(y, ref) < -270


def test_ti_case_fails_one_tap_too_long():
    """A filter one tap longer than N - M + 1 aliases: the condition is tight."""
    n, hop = 64, 48
    rng = np.random.default_rng(5)
    x = crandn(rng, 2000)
    h = crandn(rng, n - hop + 2)
    H = np.fft.fft(np.concatenate([h, np.zeros(n - len(h))]))
    assert db(run_generic(x, n, hop, H), np.convolve(x, h)[:2000]) > -60


# --- HFSO coefficients: delay, closed form, realness ------------------------------

@pytest.mark.parametrize("n,hop", [(16, 12), (64, 48), (256, 192), (1024, 768), (128, 96)])
def test_allpass_is_pure_delay(n, hop):
    """H_R = 1 on every bin (L_V = 0, k1 = N/2 + 1) leaves only the phase of
    eq. (5): y(t) = x(t - D), D = (L-1)/2 = (N-M)/2."""
    rng = np.random.default_rng(n)
    length = 5 * hop + 7
    x = crandn(rng, length)
    d = (n - hop) // 2
    y = ols.channel_hfso(x, n, hop, [], [(0, n // 2 + 1)])
    ref = np.concatenate([np.zeros(d, complex), x[: length - d]])
    assert db(y, ref) < -270


def cosine_form(n, hop, k1, v, q):
    """Eq. (8), the real closed form of d_{M-1}(q) = IDFT(H)(q)."""
    d = (n - hop) / 2.0
    acc = np.ones_like(q, dtype=float)
    for k in range(1, k1):
        acc += 2 * np.cos(2 * np.pi * k / n * (q - d))
    for r, vr in enumerate(v):
        k = k1 + r
        acc += 2 * vr * np.cos(2 * np.pi * k / n * (q - d))
    return acc / n


@pytest.mark.parametrize("n,hop,k1,lv", [(128, 96, 41, 15), (128, 96, 48, 15), (256, 192, 24, 8),
                                         (1024, 768, 230, 16), (16, 12, 1, 3), (16, 10, 7, 1),
                                         (64, 48, 5, 0)])
def test_coefficients_match_cosine_closed_form(n, hop, k1, lv):
    rng = np.random.default_rng(k1)
    v = np.sort(rng.random(lv))[::-1]
    H = ols.hfso_coeffs(n, hop, k1, v)
    d = np.fft.ifft(H)
    q = np.arange(n)
    np.testing.assert_allclose(d.real, cosine_form(n, hop, k1, v, q), atol=1e-15)
    assert np.max(np.abs(d.imag)) < 1e-15


def test_magnitude_regions_and_mirror():
    """Eq. (6) regions; the mirrored transition edge carries V in reverse."""
    n, k1, v = 32, 5, np.array([0.9, 0.6, 0.3])
    hr = ols.hfso_magnitude(n, k1, v)
    assert np.all(hr[:k1] == 1) and np.all(hr[n - k1 + 1:] == 1)
    assert list(hr[k1:k1 + 3]) == [0.9, 0.6, 0.3]
    assert list(hr[n - k1 - 2:n - k1 + 1]) == [0.3, 0.6, 0.9]
    assert np.all(hr[k1 + 3:n - k1 - 2] == 0)
    np.testing.assert_array_equal(hr[1:], hr[1:][::-1])


# --- brute force on tiny sizes -----------------------------------------------------

def brute_force_channel(x, n, hop, k1, v):
    """Per block: explicit circular convolution with the real impulse response
    of eq. (8), then keep z(N-M .. N-1) (Sec. II steps 1-5), in plain loops."""
    length = len(x)
    h = cosine_form(n, hop, k1, v, np.arange(n))
    y = np.zeros(length, complex)
    nb = -(-length // hop)
    for m in range(nb):
        start = m * hop - (n - hop)
        s = [x[start + i] if 0 <= start + i < length else 0.0 for i in range(n)]
        for j in range(hop):
            t = m * hop + j
            if t >= length:
                break
            i = n - hop + j
            y[t] = sum(h[(i - ip) % n] * s[ip] for ip in range(n))
    return y


def tiny_cases():
    for n in (4, 8, 16):
        for hop in range(1, n):
            if (n - hop) % 2:
                continue
            for lv in range(0, n // 2):
                for k1 in range(1, n // 2 + 1):
                    if k1 + lv - 1 <= n // 2 - 1:
                        yield n, hop, k1, lv


def test_brute_force_tiny_sizes():
    rng = np.random.default_rng(11)
    worst, count = -np.inf, 0
    for n, hop, k1, lv in tiny_cases():
        v = np.sort(rng.random(lv))[::-1]
        length = 3 * hop + (count % hop) + 1
        x = crandn(rng, length)
        y = ols.channel_hfso(x, n, hop, v, [(0, k1)])
        ref = brute_force_channel(x, n, hop, k1, v)
        worst = max(worst, db(y, ref))
        count += 1
    assert count > 150
    assert worst < -270


# --- structure: LPTV block phase, linearity, realness, tones ------------------------

def test_hop_shift_invariance_and_time_variance():
    """OLS with HFSO coefficients is M-periodic time-varying (Sec. II): a shift
    by M shifts the output exactly, a shift by 1 does not."""
    n, hop, k1 = 64, 48, 9
    v = np.array([0.8, 0.5, 0.2])
    rng = np.random.default_rng(3)
    x = crandn(rng, 20 * hop)
    y = ols.channel_hfso(x, n, hop, v, [(0, k1)])
    xs = np.concatenate([np.zeros(hop, complex), x])
    ys = ols.channel_hfso(xs, n, hop, v, [(0, k1)])
    assert np.array_equal(ys[hop:], y)
    x1 = np.concatenate([np.zeros(1, complex), x])
    y1 = ols.channel_hfso(x1, n, hop, v, [(0, k1)])
    assert db(y1[1:], y) > -80


def test_linearity_and_real_response():
    n, hop, k1 = 128, 96, 20
    v = np.linspace(0.9, 0.1, 7)
    rng = np.random.default_rng(4)
    a, b = crandn(rng, 1000), crandn(rng, 1000)
    ya = ols.channel_hfso(a, n, hop, v, [(0, k1)])
    yb = ols.channel_hfso(b, n, hop, v, [(0, k1)])
    yab = ols.channel_hfso(2.0 * a - 0.5j * b, n, hop, v, [(0, k1)])
    assert db(yab, 2.0 * ya - 0.5j * yb) < -280
    yr = ols.channel_hfso(a.real, n, hop, v, [(0, k1)])
    assert np.max(np.abs(yr.imag)) < 1e-14


@pytest.mark.parametrize("n,hop,k1,lv", [(64, 48, 10, 4), (256, 192, 24, 8)])
def test_bin_centred_tones(n, hop, k1, lv):
    """A tone exactly on bin k0 is N-periodic, so every interior block sees it
    circularly: the output is H_R(k0) times the tone delayed by D.  Pass bins
    give amplitude 1, transition bins V(r) (mirror: reversed), stop bins 0."""
    v = np.sort(np.random.default_rng(1).random(lv))[::-1]
    k2 = k1 + lv - 1
    d = (n - hop) // 2
    length = 8 * hop
    t = np.arange(length)
    expected = {0: 1.0, k1 - 1: 1.0, k1: v[0], k2: v[-1], k2 + 1: 0.0, n // 2: 0.0,
                n - k1 + 1: 1.0, n - k1: v[0], n - k2: v[-1], n - k2 - 1: 0.0, k1 + 1: v[1]}
    for k0, amp in expected.items():
        x = np.exp(2j * np.pi * k0 * t / n)
        y = ols.channel_hfso(x, n, hop, v, [(0, k1)])
        interior = slice(hop, (length // hop - 1) * hop)
        ref = amp * np.exp(2j * np.pi * k0 * (t - d) / n)
        assert np.max(np.abs(y[interior] - ref[interior])) < 1e-11, k0


# --- schedule, block selection, arguments --------------------------------------------

def test_bandwidth_switch_splices_whole_blocks():
    n, hop = 64, 48
    v = np.array([0.7, 0.4])
    rng = np.random.default_rng(9)
    x = crandn(rng, 30 * hop + 5)
    s = 12
    y = ols.channel_hfso(x, n, hop, v, [(0, 6), (s, 20)])
    ya = ols.channel_hfso(x, n, hop, v, [(0, 6)])
    yb = ols.channel_hfso(x, n, hop, v, [(0, 20)])
    assert np.array_equal(y[: s * hop], ya[: s * hop])
    assert np.array_equal(y[s * hop:], yb[s * hop:])
    # duplicate from_block: the later pair in the schedule list wins after sorting
    y2 = ols.channel_hfso(x, n, hop, v, [(0, 6), (s, 20), (s + 3, 6)])
    assert np.array_equal(y2[(s + 3) * hop:], ya[(s + 3) * hop:])


def test_block_subset_equals_full_run():
    n, hop = 128, 96
    v = np.array([0.9, 0.5, 0.1])
    rng = np.random.default_rng(10)
    x = crandn(rng, 40 * hop - 17)
    full = ols.blocks_hfso(x, n, hop, v, [(0, 30)])
    sel = [0, 1, 17, 38, 39]
    part = ols.blocks_hfso(x, n, hop, v, [(0, 30)], blocks=sel)
    assert np.array_equal(part, full[sel])
    y = ols.channel_hfso(x, n, hop, v, [(0, 30)])
    assert np.array_equal(y, full.reshape(-1)[: len(x)])


@pytest.mark.parametrize("length", [0, 1, 95, 96, 97])
def test_ragged_and_empty_lengths(length):
    n, hop = 128, 96
    x = crandn(np.random.default_rng(length), length)
    y = ols.channel_hfso(x, n, hop, [0.5], [(0, 10)])
    assert y.shape == (length,)
    if length:
        h = np.zeros(n)
        h[(n - hop) // 2] = 1.0
        yd = ols.channel_hfso(x, n, hop, [], [(0, n // 2 + 1)])
        d = (n - hop) // 2
        np.testing.assert_allclose(yd, np.concatenate([np.zeros(d), x])[:length], atol=1e-14)


@pytest.mark.parametrize("args", [
    dict(n=64, hop=47, k1=5, v=[0.5]),        # N - M odd: D not an integer
    dict(n=64, hop=48, k1=0, v=[0.5]),        # k1 < 1
    dict(n=64, hop=48, k1=31, v=[0.5, 0.4]),  # k2 = 32 = N/2: mirrored edges collide
    dict(n=64, hop=64, k1=5, v=[0.5]),        # hop must be < N
])
def test_invalid_arguments_rejected(args):
    with pytest.raises(ols.OracleError):
        ols.hfso_coeffs(args["n"], args["hop"], args["k1"], args["v"])
