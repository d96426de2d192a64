"""GPU test of vbw_filter_noalloc, the entry point that allocates no device
memory: its output against vbw_filter's (plan path) on the same inputs, on two
calls in a row (the second smaller, so the shared static scratch holds the
first call's tables when it starts), and against the FP64 oracle."""
import numpy as np
import pytest

from oracle import ols
from paper_2406_14116_amd import vbw
from paper_2406_14116_amd import workloads as wl

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FP32_DB = -110.0


def say(*a):
    print(*a, flush=True)


def crandn(rng, n):
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)


def make_case(seed, specs):
    """specs: (n, hop, lv, k1, len); returns channel dicts, V pool, V per
    channel, inputs, band switches (channel, k1, from_block)."""
    rng = np.random.default_rng(seed)
    chans, pool, vs, xs, switches = [], [], [], [], []
    off = 0
    for i, (n, hop, lv, k1, length) in enumerate(specs):
        v = wl.draw_v(seed, i, n, lv)
        chans.append(dict(n=n, hop=hop, lv=lv, v_offset=off, k1=k1, len=length))
        pool.append(v)
        vs.append(v)
        off += lv
        xs.append(crandn(rng, length))
        nb = -(-length // hop)
        if nb > 3:
            k1b = int(rng.integers(1, n // 2 - lv + 1))
            switches.append((i, k1b, int(rng.integers(1, nb))))
    return chans, np.concatenate(pool), vs, xs, switches


def run_both(chans, pool, xs_host, switches, dtype="c64", engine="fft", flags=0):
    xs = [torch.from_numpy(x).cuda() for x in xs_host]
    y_plan = [torch.full_like(x, complex(np.nan, np.nan)) for x in xs]
    y_free = [torch.full_like(x, complex(np.nan, np.nan)) for x in xs]
    plan = vbw.Plan(chans, pool, dtype=dtype, engine=engine, flags=flags)
    for c, k1, b in switches:
        plan.set_bandwidth(c, k1, b)
    plan.filter(xs, y_plan)
    vbw.filter_noalloc(chans, pool, xs, y_free, dtype=dtype, engine=engine, flags=flags, switches=switches)
    torch.cuda.synchronize()
    plan.close()
    return [y.cpu().numpy() for y in y_plan], [y.cpu().numpy() for y in y_free]


def check_against_oracle(chans, vs, xs_host, switches, outs):
    for i, (c, x, y) in enumerate(zip(chans, xs_host, outs)):
        if c["len"] == 0:
            continue
        sched = [(0, c["k1"])] + sorted((b, k) for (ch, k, b) in switches if ch == i)
        ref = ols.channel_hfso(x.astype(np.complex128), c["n"], c["hop"], vs[i], sched)
        err = ols.error_db(y, ref)
        say(f"  channel {i} N={c['n']} len={c['len']}: {err:.1f} dB vs oracle")
        assert err <= FP32_DB, (i, err)


def test_noalloc_matches_plan_path_two_calls():
    first = [(1024, 768, 16, 40, 300_000), (256, 192, 8, 24, 77_777), (4096, 3072, 32, 100, 200_001),
             (64, 48, 4, 5, 9_999), (2048, 1536, 24, 300, 0), (512, 384, 12, 60, 50_000)]
    second = [(256, 192, 8, 30, 20_001), (1024, 768, 16, 200, 5_000)]
    for call, specs in enumerate((first, second)):
        say(f"noalloc call {call}: {len(specs)} channels")
        chans, pool, vs, xs, sw = make_case(11 + call, specs)
        y_plan, y_free = run_both(chans, pool, xs, sw)
        for i, (a, b) in enumerate(zip(y_plan, y_free)):
            # same kernels, same work partition: the same bits
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), i
        check_against_oracle(chans, vs, xs, sw, y_free)


def test_noalloc_16bit_matrix_core_engine():
    rng = np.random.default_rng(3)
    for call, lens in enumerate(((100_000, 33_333), (10_000,))):
        say(f"noalloc gemm call {call}")
        chans, pool, vs, xs, sw = make_case(21 + call, [(256, 192, 8, 20 + 7 * i, n) for i, n in enumerate(lens)])
        xt = [torch.from_numpy(np.stack([x.real, x.imag], 1)).to(torch.float16).cuda() for x in xs]
        outs = []
        for use_plan in (True, False):
            ys = [torch.full_like(x, float("nan")) for x in xt]
            if use_plan:
                plan = vbw.Plan(chans, pool, dtype="f16", engine="gemm")
                for c, k1, b in sw:
                    plan.set_bandwidth(c, k1, b)
                plan.filter(xt, ys)
                torch.cuda.synchronize()
                plan.close()
            else:
                vbw.filter_noalloc(chans, pool, xt, ys, dtype="f16", engine="gemm", switches=sw)
            torch.cuda.synchronize()
            outs.append([y.cpu().view(torch.int16).numpy() for y in ys])
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
    del rng


@pytest.mark.parametrize("dtype,flags", [("r32", 0), ("c64", vbw.NO_PRUNE), ("bf16", vbw.F32_OUT)])
def test_noalloc_other_storage_and_flags(dtype, flags):
    """Real input, the unpruned inverse and 16-bit input with float32 output:
    the same bits as the plan path, and the oracle's result on the stored
    input."""
    specs = [(1024, 768, 16, 100, 200_003), (256, 192, 8, 30, 50_000), (2048, 1536, 16, 400, 30_001)]
    chans, pool, vs, xs, sw = make_case(31, specs)
    if dtype == "r32":
        xt = [torch.from_numpy(np.ascontiguousarray(x.real)).cuda() for x in xs]
        stored = [x.real.astype(np.complex128) for x in xs]
    elif dtype == "bf16":
        xt = [torch.from_numpy(np.stack([x.real, x.imag], 1)).to(torch.bfloat16).cuda() for x in xs]
        stored = [t.float().cpu().numpy() @ np.array([1.0, 1.0j]) for t in xt]
    else:
        xt = [torch.from_numpy(x).cuda() for x in xs]
        stored = [x.astype(np.complex128) for x in xs]
    outs = []
    for use_plan in (True, False):
        if dtype == "bf16":
            ys = [torch.full((t.shape[0], 2), float("nan"), device="cuda") for t in xt]
        else:
            ys = [torch.full_like(t, float("nan")) for t in xt]
        if use_plan:
            plan = vbw.Plan(chans, pool, dtype=dtype, flags=flags)
            for c, k1, b in sw:
                plan.set_bandwidth(c, k1, b)
            plan.filter(xt, ys)
            torch.cuda.synchronize()
            plan.close()
        else:
            vbw.filter_noalloc(chans, pool, xt, ys, dtype=dtype, flags=flags, switches=sw)
        torch.cuda.synchronize()
        outs.append([y.cpu().numpy() for y in ys])
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    for i, (c, x, y) in enumerate(zip(chans, stored, outs[1])):
        sched = [(0, c["k1"])] + sorted((bb, k) for (ch, k, bb) in sw if ch == i)
        ref = ols.channel_hfso(x, c["n"], c["hop"], vs[i], sched)
        if dtype == "r32":          # a real filter on real input: the oracle's real part
            got, ref = y.astype(np.float64), ref.real
        elif dtype == "bf16":       # float32 output pairs
            got = y.astype(np.float64) @ np.array([1.0, 1.0j])
        else:
            got = y.astype(np.complex128)
        err = ols.error_db(got, ref)
        say(f"  {dtype} channel {i}: {err:.1f} dB vs oracle")
        assert err <= FP32_DB, (i, err)


def test_noalloc_rejects_what_it_cannot_serve():
    chans = [dict(n=256, hop=192, lv=4, v_offset=0, k1=10, len=1000)]
    pool = np.array([0.9, 0.7, 0.4, 0.1])
    x = torch.zeros(1000, dtype=torch.complex64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(vbw.VbwError) as e:
        vbw.filter_noalloc(chans, pool, [x], [y], flags=vbw.GRAPH)
    assert e.value.status == vbw.VBW_EUNSUPPORTED
    with pytest.raises(vbw.VbwError) as e:
        vbw.filter_noalloc(chans, pool, [x], [y], switches=[(0, 200, 3)])
    assert e.value.status == vbw.VBW_ERANGE
    # tables beyond the static scratch: 40,000 one-sample channels need
    # 56 bytes of per-call table each (2.2 MB > 2 MiB); nothing is launched
    n = 40_000
    xb = torch.zeros(n, dtype=torch.complex64, device="cuda")
    yb = torch.zeros(n, dtype=torch.complex64, device="cuda")
    many = [dict(n=16, hop=12, lv=0, v_offset=0, k1=1, len=1)] * n
    with pytest.raises(vbw.VbwError) as e:
        vbw.filter_noalloc(many, pool, [xb[i:i + 1] for i in range(n)], [yb[i:i + 1] for i in range(n)])
    assert e.value.status == vbw.VBW_ETOOLARGE
    torch.cuda.synchronize()
