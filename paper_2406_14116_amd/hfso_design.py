"""HFSO design: the step before the filtering path (Moryakova & Johansson,
arXiv 2406.14116, Sec. III-C to III-E).

The filtering library takes the L_V transition values V(r) as an input.  This
module computes them:

* ``impulse_terms``  -- eq. (8): the zero-phase-delayed impulse response of the
  DFT coefficients of eqs. (5)-(6), affine in V (the passband part plus one
  cosine per transition value).
* ``ptvir``          -- the overlap-save system is M-periodically time varying;
  output position j of a block (j < M) sees a time-invariant response G_j
  (eqs. (2)-(4)).  With the framing used by the library (block m reads
  samples m M - (N - M) .. m M + M - 1 and keeps samples N - M + j of the
  inverse transform) the response of position j is the circular impulse
  response h(q) placed at lag q for q <= j + N - M and at lag q - N otherwise.
  These are the paper's H_n up to the common delay of M - 1 samples that its
  causal convention adds (the footnote to eq. (9)), which changes no
  magnitude.
* ``minimax_v``      -- eq. (10)-(11): the V(r) minimising the largest error
  |G_j(w) - D(w)| over the passband and stopband grid, every position j and
  every b in the design range; D is exp(-j w (N - M)/2) on the passband and 0 on
  the stopband.  The complex modulus constraint is enforced on P directions
  (|z| <= delta is replaced by Re(z exp(-j theta_p)) <= delta, a regular
  P-gon, so the true maximum is at most delta / cos(pi / P)); the linear
  program is solved by HiGHS on a growing set of grid points (each round adds
  the worst points of the full grid) until the full-grid maximum agrees with
  the program's value.
* ``measure_ptvir_gpu`` -- the same responses measured on the GPU library:
  one vbw_filter call over a grid of complex exponentials.
* ``rates``          -- Table I: multiplications and additions per output
  sample, with the cheaper exponent multiplies of Sec. III-D when
  (L - 1)/N = 1/(2c).
* ``design``         -- Sec. III-E: order estimate of eq. (12), N = 0.9 L log2 L
  rounded to a power of two, M = N - L + 1, the search over the order for the
  smallest one whose minimax error meets the specification, and among that
  order and a few above it (which meet it too) the one with the fewest
  multiplications per output sample.

The design itself is float64 on the host (scipy's HiGHS); it runs once per
design, not per sample.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def impulse_terms(n: int, m: int, k1: int, lv: int):
    """Eq. (8): h(q) = a(q) + sum_r C(q, r) V(r), q < N, with D = (N - M)/2.

    a(q) = (1 + 2 sum_{k=1}^{k1-1} cos(2 pi k (q - D)/N)) / N
    C(q, r) = 2 cos(2 pi (k1 + r)(q - D)/N) / N
    """
    if (n - m) % 2:
        raise ValueError("N - M must be even (integer delay D)")
    d = (n - m) // 2
    q = np.arange(n, dtype=np.float64)
    ang = 2.0 * np.pi * (q - d) / n
    a = np.ones(n)
    for k in range(1, k1):
        a += 2.0 * np.cos(k * ang)
    a /= n
    c = np.empty((n, lv))
    for r in range(lv):
        c[:, r] = 2.0 * np.cos((k1 + r) * ang) / n
    return a, c


def ptvir(h: np.ndarray, n: int, m: int, w: np.ndarray) -> np.ndarray:
    """Responses G_j(w) of output positions j = 0..M-1 (rows) at the
    frequencies w (columns) for circular impulse responses h (last axis N;
    leading axes are carried along: h of shape (..., N) gives (..., M, K)).

    G_j(w) = sum_{q <= j+N-M} h(q) exp(-j w q) + exp(j w N) sum_{q > j+N-M} h(q) exp(-j w q)
    """
    h = np.asarray(h, dtype=np.float64)
    phase = np.exp(-1j * np.outer(np.arange(n), w))                 # (N, K)
    terms = h[..., :, None] * phase                                # (..., N, K)
    cs = np.cumsum(terms, axis=-2)                                 # prefix sums over q
    total = cs[..., -1:, :]
    lo = cs[..., n - m: n, :]                                      # q <= j + N - M, j = 0..M-1
    return lo + np.exp(1j * w * n)[None, :] * (total - lo)


def desired(w: np.ndarray, d: int, passband: np.ndarray) -> np.ndarray:
    """exp(-j w D) on the passband, 0 on the stopband."""
    return np.where(passband, np.exp(-1j * w * d), 0.0)


@dataclass
class MinimaxResult:
    v: np.ndarray                 # L_V transition values
    delta: float                  # largest |error| over the full grid, all b, all positions
    delta_lp: float               # the linear program's value
    rounds: int
    worst_db_per_b: dict = field(default_factory=dict)


def _band_grid(k: int, b_n: int, delta_n: int, n: int):
    w = np.linspace(0.0, np.pi, k)
    wp = (b_n - delta_n / 2.0) * 2.0 * np.pi / n
    ws = (b_n + delta_n / 2.0) * 2.0 * np.pi / n
    keep = (w <= wp + 1e-12) | (w >= ws - 1e-12)
    return w[keep], (w[keep] <= wp + 1e-12)


def minimax_v(n: int, m: int, delta_n: int, b_range: tuple[int, int], k: int = 1000, p: int = 16,
              tol: float = 1e-3, max_rounds: int = 40, add_per_round: int = 4) -> MinimaxResult:
    """Eqs. (10)-(11) for b_N in [b_range[0], b_range[1]] (integers), transition
    width Delta_N bins (L_V = Delta_N - 1, k1 = b_N - Delta_N/2 + 1), K grid
    points on [0, pi], P directions for the modulus."""
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix

    if delta_n % 2:
        raise ValueError("Delta_N must be even (integer band edges)")
    lv = delta_n - 1
    d = (n - m) // 2
    # per b: E = A + B V on its grid, A (M, K_b) complex, B (M, K_b, L_V) complex
    data = []
    for b_n in range(b_range[0], b_range[1] + 1):
        k1 = b_n - delta_n // 2 + 1
        if k1 < 1 or k1 + lv - 1 > n // 2 - 1:
            raise ValueError(f"b_N = {b_n}: band edges outside [1, N/2 - 1]")
        w, pb = _band_grid(k, b_n, delta_n, n)
        a, c = impulse_terms(n, m, k1, lv)
        basis = np.concatenate([a[None, :], c.T], axis=0)          # (1 + L_V, N)
        g = ptvir(basis, n, m, w)                                  # (1 + L_V, M, K_b)
        A = g[0] - desired(w, d, pb)[None, :]
        B = np.moveaxis(g[1:], 0, -1)                              # (M, K_b, L_V)
        data.append((b_n, w, A, B))

    theta = 2.0 * np.pi * np.arange(p) / p
    rot = np.exp(-1j * theta)
    shrink = 1.0 / math.cos(math.pi / p)

    def errors(v):
        return [np.abs(A + B @ v) for (_, _, A, B) in data]

    # start: for every (b, position) the grid points that are worst for V = 0.5
    active = []
    v = np.full(lv, 0.5)
    for bi, err in enumerate(errors(v)):
        for j in range(err.shape[0]):
            for i in np.argsort(err[j])[-add_per_round:]:
                active.append((bi, j, int(i)))
    active = set(active)
    res_v, delta_lp = v, float("inf")
    rounds = 0
    for rounds in range(1, max_rounds + 1):
        pts = sorted(active)
        rows_a = np.array([data[bi][2][j, i] for bi, j, i in pts])            # complex
        rows_b = np.array([data[bi][3][j, i] for bi, j, i in pts])            # complex (n_pts, L_V)
        # Re(rot (A + B V)) <= delta  ->  Re(rot B) V - delta <= -Re(rot A)
        lhs = (rot[None, :, None] * rows_b[:, None, :]).real.reshape(-1, lv)
        rhs = -(rot[None, :] * rows_a[:, None]).real.reshape(-1)
        a_ub = np.concatenate([lhs, -np.ones((lhs.shape[0], 1))], axis=1)
        cost = np.zeros(lv + 1)
        cost[-1] = 1.0
        sol = linprog(cost, A_ub=csr_matrix(a_ub), b_ub=rhs, bounds=[(None, None)] * lv + [(0, None)],
                      method="highs")
        if sol.status != 0:
            raise RuntimeError(f"linear program failed: {sol.message}")
        res_v, delta_lp = sol.x[:lv], float(sol.x[-1])
        errs = errors(res_v)
        worst = max(float(e.max()) for e in errs)
        if worst <= delta_lp * shrink * (1.0 + tol):
            break
        added = 0
        for bi, err in enumerate(errs):
            over = err > delta_lp * shrink
            for j in np.nonzero(over.any(axis=1))[0]:
                for i in np.argsort(err[j])[-add_per_round:]:
                    if (bi, int(j), int(i)) not in active:
                        active.add((bi, int(j), int(i)))
                        added += 1
        if added == 0:
            break
    errs = errors(res_v)
    worst = max(float(e.max()) for e in errs)
    per_b = {data[bi][0]: 20.0 * math.log10(float(e.max())) for bi, e in enumerate(errs)}
    return MinimaxResult(v=res_v, delta=worst, delta_lp=delta_lp, rounds=rounds, worst_db_per_b=per_b)


def order_estimate(delta_p: float, delta_s: float, delta: float) -> float:
    """Eq. (12): N_D = -4 pi log10(10 delta_p delta_s) / (3 Delta)."""
    return -4.0 * math.pi * math.log10(10.0 * delta_p * delta_s) / (3.0 * delta)


def sizes_for_length(L: int) -> tuple[int, int]:
    """Sec. III-E: N = 0.9 L log2 L rounded to the nearest power of two, M = N - L + 1."""
    n = 1 << round(math.log2(0.9 * L * math.log2(L)))
    return n, n - L + 1


@dataclass
class Rates:
    r_mf: float        # fixed multiplications per output sample
    r_mv: float        # variable (general) multiplications per output sample
    r_a: float         # additions per output sample
    memory: int        # stored values (L_V)


def rates(n: int, L: int, lv: int) -> Rates:
    """Table I for real segments, split-radix FFT and IFFT, N = 2^Q:
    per transform (N/2) log2 N - 3N/2 + 2 multiplications and
    (3N/2) log2 N - 5N/2 + 4 additions; the multiply by H costs 2 L_V general
    multiplications, and its fixed exponent factor exp(-j 2 pi k (L-1)/(2N))
    over the N/2 bins kept by conjugate symmetry costs 3 multiplications and 3
    additions per bin, except (Sec. III-D) when (L - 1)/N = 1/(2c): nothing for
    k = m c, 2 and 2 for k = m c + floor(c/2) (c >= 2)."""
    q = math.log2(n)
    m = n - L + 1
    mf_f = n / 2.0 * q - 1.5 * n + 2.0
    a_f = 1.5 * n * q - 2.5 * n + 4.0
    c = None
    if (L - 1) > 0 and n % (2 * (L - 1)) == 0:
        c = n // (2 * (L - 1))
    mf_h = a_h = 0.0
    for k in range(n // 2):
        if c is not None and k % c == 0:
            continue
        cost = 2.0 if (c is not None and c >= 2 and k % c == c // 2) else 3.0
        mf_h += cost
        a_h += cost
    return Rates(r_mf=(2.0 * mf_f + mf_h) / m, r_mv=2.0 * lv / m, r_a=(2.0 * a_f + a_h) / m, memory=lv)


@dataclass
class Design:
    L: int
    n: int
    m: int
    delta_n: int
    b_range: tuple
    result: MinimaxResult
    tried: list                    # (L, N, M, delta) of every order tried


def design(delta_p: float, delta_s: float, delta_over_pi: float, b_over_pi: tuple[float, float],
           k: int = 1000, p: int = 16, max_steps: int = 12, extra_orders: int = 3) -> Design:
    """Sec. III-E procedure: start from the even order at or above eq. (12)'s
    estimate (odd L, integer delay), size N and M from L, solve eq. (10); raise
    the order while the error exceeds delta_E = min(delta_p, delta_s), lower it
    while it still meets it.  The smallest order that meets it and the next
    ``extra_orders`` even orders are then ranked by multiplications per output
    sample (Table I, fixed plus variable) and the cheapest that meets the
    specification is returned (a longer L can cost less when (L - 1)/N makes
    the exponents cheap)."""
    delta = delta_over_pi * math.pi
    nd = math.ceil(order_estimate(delta_p, delta_s, delta))
    nd += nd & 1
    target = min(delta_p, delta_s)
    tried, results = [], {}

    def solve(nd_):
        L = nd_ + 1
        n, m = sizes_for_length(L)
        delta_n = round(delta_over_pi * n / 2.0)
        b_lo = math.ceil(b_over_pi[0] * n / 2.0 - 1e-9)
        b_hi = math.floor(b_over_pi[1] * n / 2.0 + 1e-9)
        r = minimax_v(n, m, delta_n, (b_lo, b_hi), k=k, p=p)
        tried.append((L, n, m, r.delta))
        results[nd_] = (L, n, m, delta_n, (b_lo, b_hi), r)
        return r.delta <= target

    ok = solve(nd)
    step = 0
    if ok:
        while nd > 2 and step < max_steps and solve(nd - 2):
            nd -= 2
            step += 1
    else:
        while not ok and step < max_steps:
            nd += 2
            step += 1
            ok = solve(nd)
        if not ok:
            raise RuntimeError(f"no order up to {nd + 1} meets delta_E = {target}")
    def cost(nd_):
        L = nd_ + 1
        n, _ = sizes_for_length(L)
        rr = rates(n, L, round(delta_over_pi * n / 2.0) - 1)
        return rr.r_mf + rr.r_mv

    for cand in sorted(range(nd, nd + 2 * extra_orders + 1, 2), key=lambda c: (cost(c), c)):
        if cand in results or solve(cand):
            if results[cand][5].delta <= target:
                nd = cand
                break
    L, n, m, delta_n, br, r = results[nd]
    return Design(L=L, n=n, m=m, delta_n=delta_n, b_range=br, result=r, tried=tried)


def measure_ptvir_gpu(n: int, m: int, k1: int, v, w, stream=None) -> np.ndarray:
    """The responses G_j(w) (shape (M, K)) of the filter as the GPU library
    actually runs it: one channel per frequency carries exp(j w t) for three
    blocks, and output position j of block 2 (whose segment lies inside the
    input) gives y[2M + j] exp(-j w (2M + j)) = G_j(w).  One vbw_filter call
    evaluates the whole grid (float32 arithmetic)."""
    import torch

    from . import vbw
    w = np.asarray(w, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    length = 3 * m
    t = np.arange(length)
    x = np.exp(1j * np.outer(w, t)).astype(np.complex64)          # (K, 3M)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    chans = [dict(n=n, hop=m, lv=v.size, v_offset=0, k1=k1, len=length) for _ in range(w.size)]
    with vbw.Plan(chans, v) as plan:
        plan.filter([xd[i] for i in range(w.size)], [yd[i] for i in range(w.size)], stream)
        torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.complex128)
    tt = 2 * m + np.arange(m)
    return (y[:, tt] * np.exp(-1j * np.outer(w, tt))).T
