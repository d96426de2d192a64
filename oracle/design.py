"""Design-side relations of the paper, written out plainly (test infrastructure).

Paper: Moryakova & Johansson, arXiv 2406.14116.

* ``bin_edges``       -- Sec. III-B, eq. (7) and the discretisation that follows
                         it: first/last transition bins k1, k2, the transition
                         width Delta_N and L_V = Delta_N - 1.
* ``order_estimate``  -- Sec. III-E, eq. (12): estimated filter order.
* ``dft_size``        -- Sec. III-E: N estimated as 0.9 L log2 L, rounded to the
                         nearest power of two, and M = N - L + 1.
* ``complexity``      -- Sec. III-D, Table I: multiplication/addition rates per
                         output sample and memory, optionally with the cheaper
                         exponent multiplies that Sec. IV applies when
                         (L-1)/N = 1/(2c).

None of this runs on the filtering path; the path takes integer k1 and L_V.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class BinEdges:
    k1: float
    k2: float
    delta_n: float
    lv: float
    b_n: float


def bin_edges(b: float, delta: float, n: int) -> BinEdges:
    """Eq. (7): k1 = (b - Delta/2) N/(2 pi) + 1, k2 = (b + Delta/2) N/(2 pi) - 1.

    With Delta = Delta_N 2 pi/N and b = b_N 2 pi/N this is k1 = b_N - Delta_N/2 + 1,
    and Delta_N = k2 - k1 + 2, L_V = Delta_N - 1.
    """
    k1 = (b - delta / 2.0) * n / (2.0 * math.pi) + 1.0
    k2 = (b + delta / 2.0) * n / (2.0 * math.pi) - 1.0
    delta_n = k2 - k1 + 2.0
    return BinEdges(k1=k1, k2=k2, delta_n=delta_n, lv=delta_n - 1.0,
                    b_n=b * n / (2.0 * math.pi))


def b_n_range(delta_n: int, n: int) -> tuple[float, float]:
    """Admissible b_N range stated after eq. (7): Delta_N/2 <= b_N <= N/2 - Delta_N/2 - 1."""
    return delta_n / 2.0, n / 2.0 - delta_n / 2.0 - 1.0


def order_estimate(delta_p: float, delta_s: float, delta: float) -> float:
    """Eq. (12): N_D = -4 pi log10(10 delta_p delta_s) / (3 Delta)."""
    return -4.0 * math.pi * math.log10(10.0 * delta_p * delta_s) / (3.0 * delta)


def even_order(nd_hat: float) -> int:
    """Reading of Sec. IV: the printed initial order is the estimate rounded up
    to an even integer (26.67 -> 28), i.e. an odd length L = N_D + 1."""
    k = math.ceil(nd_hat)
    return k + (k & 1)


def dft_size(L: int) -> tuple[float, int, int]:
    """Sec. III-E: N_hat = 0.9 L log2 L, N = nearest power of two, M = N - L + 1."""
    n_hat = 0.9 * L * math.log2(L)
    q = round(math.log2(n_hat))
    n = 1 << q
    return n_hat, n, n - L + 1


@dataclass(frozen=True)
class Rates:
    r_mf: float
    r_mv: float
    r_a: float
    memory: int


def complexity(n: int, L: int, lv: int, odd_k_rule: bool = False) -> Rates:
    """Table I rates per output sample for real segments and N = 2^Q.

    Each FFT/IFFT costs C_mf,F = N/2 log2 N - 3N/2 + 2 multiplications and
    C_a,F = 3N/2 log2 N - 5N/2 + 4 additions (the addition count as Table I
    implies; the inline formula of Sec. III-D lacks a factor N on its first
    term).  The multiply by H costs C_mf,H = 3N/2 fixed multiplications,
    C_mv,H = 2 L_V variable ones and C_a,H = 3N/2 additions.  With
    ``odd_k_rule`` the exponent multiply costs 2 multiplications and 2
    additions for every odd k and nothing for even k, over the N/2 bins kept by
    conjugate symmetry (Sec. IV, (L-1)/N = 1/4).
    """
    q = math.log2(n)
    m = n - L + 1
    c_mf_f = n / 2.0 * q - 1.5 * n + 2.0
    c_a_f = 1.5 * n * q - 2.5 * n + 4.0
    if odd_k_rule:
        c_mf_h = 2.0 * (n / 4.0)
        c_a_h = 2.0 * (n / 4.0)
    else:
        c_mf_h = 1.5 * n
        c_a_h = 1.5 * n
    return Rates(r_mf=(2.0 * c_mf_f + c_mf_h) / m,
                 r_mv=2.0 * lv / m,
                 r_a=(2.0 * c_a_f + c_a_h) / m,
                 memory=lv)
