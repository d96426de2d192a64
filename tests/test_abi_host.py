"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every declared function, validation returns the documented codes,
the integer planner and bandwidth schedule agree with an independent
enumeration, and the float32 twiddle table is correctly rounded."""
import math
import os

import numpy as np
import pytest

from paper_2406_14116_amd import vbw


def chan(n=256, hop=192, lv=8, k1=24, length=65536, v_offset=0):
    return dict(n=n, hop=hop, lv=lv, v_offset=v_offset, k1=k1, len=length)


def host_plan(chans, v=None, **kw):
    if v is None:
        v = np.linspace(0.9, 0.1, 64)
    return vbw.Plan(chans, v, flags=vbw.HOST_ONLY | kw.pop("flags", 0), **kw)


def test_library_exports_every_declared_function():
    names = vbw.header_functions()
    assert {"vbw_plan", "vbw_set_bandwidth", "vbw_filter", "vbw_destroy", "vbw_strerror"} <= set(names)
    L = vbw.lib()
    for name in names:
        assert hasattr(L, name), name


def test_library_exports_only_declared_c_functions():
    """The C symbols the library exports are exactly those the header declares
    (everything else has C++ or internal linkage)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm missing")
    out = subprocess.run([nm, "-D", "--defined-only", vbw.LIB_PATH], check=True, capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines()
                if len(line.split()) == 3 and line.split()[1] == "T" and not line.split()[-1].startswith("_")}
    assert exported == set(vbw.header_functions())


def test_strerror_codes():
    for code in (0, -1, -2, -3, -4, -5):
        assert vbw.strerror(code) and vbw.strerror(code) != "unknown status"
    assert vbw.strerror(-99) == "unknown status"


@pytest.mark.parametrize("n", [2, 16, 256, 1024, 4096])
def test_twiddle_table_correctly_rounded(n):
    tw = vbw.twiddle_table(n).astype(np.float64)
    r = np.arange(n)
    ang = 2.0 * np.pi * r / n
    exact = np.stack([np.cos(ang), -np.sin(ang)], axis=1)
    # within half an ulp of float32 (plus the float64 reference's own error)
    ulp = np.spacing(np.abs(exact).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(tw - exact) <= 0.5 * ulp + 4e-16)
    # exact symmetries of the table
    assert tw[0, 0] == 1.0 and tw[0, 1] == 0.0
    if n >= 4:
        assert tw[n // 4, 0] == 0.0 and tw[n // 4, 1] == -1.0
        assert np.array_equal(tw[1:, 0], tw[1:, 0][::-1])
        assert np.array_equal(tw[1:, 1], -tw[1:, 1][::-1])


def test_twiddle_subtables_are_strided_views():
    big = vbw.twiddle_table(4096)
    for n in (16, 512):
        assert np.array_equal(vbw.twiddle_table(n), big[:: 4096 // n])


@pytest.mark.parametrize("bad,code", [
    (dict(n=300), vbw.VBW_EINVAL),           # not a power of two
    (dict(n=8, hop=6, k1=2, lv=1), vbw.VBW_EINVAL),   # N below 16
    (dict(n=8192, hop=6144), vbw.VBW_EINVAL),  # N above 4096
    (dict(hop=191), vbw.VBW_EINVAL),           # N - M odd: no integer delay
    (dict(hop=256), vbw.VBW_EINVAL),           # M must be < N
    (dict(hop=0), vbw.VBW_EINVAL),
    (dict(lv=-1), vbw.VBW_EINVAL),
    (dict(len=-5), vbw.VBW_EINVAL),
    (dict(v_offset=60), vbw.VBW_EINVAL),       # V range outside the pool
    (dict(k1=0), vbw.VBW_ERANGE),
    (dict(k1=121), vbw.VBW_ERANGE),            # k2 = 128 = N/2
    (dict(k1=130, lv=0), vbw.VBW_ERANGE),
    (dict(k1=129, lv=1), vbw.VBW_ERANGE),
])
def test_validation_codes(bad, code):
    c = chan()
    c.update(bad)
    with pytest.raises(vbw.VbwError) as e:
        host_plan([c])
    assert e.value.status == code


def test_admissible_edges():
    host_plan([chan(k1=129, lv=0)]).close()   # all-pass: every bin is passband
    host_plan([chan(k1=120, lv=8)]).close()   # k2 = N/2 - 1
    host_plan([chan(k1=1, lv=0)]).close()     # only the DC bin passes
    host_plan([chan(length=0)]).close()       # empty channel


def test_validation_of_descriptor_fields():
    with pytest.raises(vbw.VbwError) as e:
        host_plan([chan()], v=[0.5, float("nan")] + [0.1] * 20)
    assert e.value.status == vbw.VBW_EINVAL
    with pytest.raises(vbw.VbwError) as e:
        host_plan([chan()], flags=1 << 20)
    assert e.value.status == vbw.VBW_EINVAL
    with pytest.raises(vbw.VbwError) as e:
        host_plan([])
    assert e.value.status == vbw.VBW_EINVAL
    with pytest.raises(vbw.VbwError) as e:
        host_plan([chan()], engine="gemm")    # float32 storage has no GEMM engine
    assert e.value.status == vbw.VBW_EUNSUPPORTED


def test_host_only_plan_refuses_to_filter():
    p = host_plan([chan()])
    with pytest.raises(vbw.VbwError) as e:
        p.filter_ptrs([0x1000], [0x100000])
    assert e.value.status == vbw.VBW_EUNSUPPORTED


def enumerate_items(chans):
    """Independent enumeration: ceil(len/M) blocks per channel, tiled into
    groups of 4096/N consecutive blocks."""
    items, blocks = [], 0
    for ci, c in enumerate(chans):
        nb = -(-c["len"] // c["hop"]) if c["len"] > 0 else 0
        blocks += nb
        per = 4096 // c["n"]
        first = 0
        while first < nb:
            items.append((ci, first, min(per, nb - first)))
            first += per
    return items, blocks


def test_planner_counts_match_enumeration():
    rng = np.random.default_rng(0)
    chans = []
    for i in range(40):
        n = int(2 ** rng.integers(4, 13))
        hop = int(n - 2 * rng.integers(1, n // 2))
        length = int(rng.choice([0, 1, hop - 1, hop, hop + 1, int(rng.integers(1, 50000))]))
        lv = int(rng.integers(0, min(8, n // 2 - 1) + 1))
        chans.append(chan(n=n, hop=hop, lv=lv, k1=1, length=max(0, length)))
    p = host_plan(chans)
    items, blocks = enumerate_items(chans)
    assert p.query(vbw.Q_N_ITEMS) == len(items)
    assert p.query(vbw.Q_TOTAL_BLOCKS) == blocks
    assert p.query(vbw.Q_TOTAL_SAMPLES) == sum(c["len"] for c in chans)
    assert p.query(vbw.Q_N_CHANNELS) == 40
    assert p.query(vbw.Q_WORKGROUP) == 256


def test_schedule_semantics():
    """Block m uses the entry with the largest from_block <= m; an equal
    from_block replaces; a failed call changes nothing."""
    p = host_plan([chan(), chan(k1=30)])
    p.set_bandwidth(0, 40, 512)
    p.set_bandwidth(0, 50, 100)
    p.set_bandwidth(0, 60, 512)          # replaces (512, 40)
    expect = {0: 24, 99: 24, 100: 50, 511: 50, 512: 60, 10 ** 6: 60}
    for m, k1 in expect.items():
        assert p.block_k1(0, m) == k1
    assert p.block_k1(1, 5000) == 30
    for args, code in [((0, 0, 10), vbw.VBW_ERANGE), ((0, 121, 10), vbw.VBW_ERANGE),
                       ((2, 30, 0), vbw.VBW_EINVAL), ((0, 30, -1), vbw.VBW_EINVAL)]:
        with pytest.raises(vbw.VbwError) as e:
            p.set_bandwidth(*args)
        assert e.value.status == code
    for m, k1 in expect.items():
        assert p.block_k1(0, m) == k1
    p.set_bandwidth(0, 33, 0)            # replaces the initial edge
    assert p.block_k1(0, 0) == 33 and p.block_k1(0, 512) == 60
    assert p.block_k1(0, -1) == vbw.VBW_EINVAL


def test_schedule_matches_oracle_rule():
    """Random schedules: the library's lookup equals the oracle's rule applied
    by plain Python (largest from_block <= m, later duplicates win)."""
    rng = np.random.default_rng(1)
    p = host_plan([chan(n=1024, hop=768, lv=16, k1=30, length=1 << 20)])
    entries = [(0, 30)]
    for _ in range(50):
        frm, k1 = int(rng.integers(0, 1400)), int(rng.integers(1, 496))
        p.set_bandwidth(0, k1, frm)
        entries.append((frm, k1))
    for m in range(0, 1400, 7):
        # the last call among those with the largest from_block <= m
        cands = [(frm, i, k1) for i, (frm, k1) in enumerate(entries) if frm <= m]
        want = max(cands)[2]
        assert p.block_k1(0, m) == want


def test_plan_copies_descriptors():
    chans = [chan()]
    v = np.linspace(0.9, 0.1, 64)
    p = vbw.Plan(chans, v, flags=vbw.HOST_ONLY)
    v[:] = 0.0
    chans[0]["len"] = 1
    assert p.query(vbw.Q_TOTAL_SAMPLES) == 65536


def test_stream_plan_validation():
    """A streaming plan's calls carry whole blocks and at least the N - hop
    samples of history the next call needs; the matrix-core engine does not
    stream; reset is refused where there is no device stream state."""
    ok = host_plan([chan(length=192 * 10), chan(n=1024, hop=768, lv=16, k1=100, length=0)], flags=vbw.STREAM)
    with pytest.raises(vbw.VbwError) as e:
        ok.stream_reset(0)
    assert e.value.status == vbw.VBW_EUNSUPPORTED
    ok.close()
    for bad in (chan(length=192 * 10 + 1), chan(n=256, hop=2, lv=8, k1=24, length=200)):
        with pytest.raises(vbw.VbwError) as e:
            host_plan([bad], flags=vbw.STREAM)
        assert e.value.status == vbw.VBW_EINVAL, bad
    with pytest.raises(vbw.VbwError) as e:
        host_plan([chan(length=192 * 10)], flags=vbw.STREAM, dtype="f16", engine="gemm")
    assert e.value.status == vbw.VBW_EUNSUPPORTED
    plain = host_plan([chan()])
    with pytest.raises(vbw.VbwError) as e:
        plain.stream_reset(0)
    assert e.value.status == vbw.VBW_EINVAL
    plain.close()


def test_binding_checks_tensor_types_and_sizes():
    """The binding refuses tensors whose element type does not match the
    plan's storage or that hold fewer than len samples (the kernels would read
    or write past them), before any pointer reaches the library."""
    torch = pytest.importorskip("torch")
    p = host_plan([chan(length=1000)])
    ok_x = torch.zeros(1000, dtype=torch.complex64)
    with pytest.raises(ValueError, match="fewer than"):
        p.filter([torch.zeros(999, dtype=torch.complex64)], [ok_x])
    with pytest.raises(ValueError, match="fewer than"):
        p.filter([ok_x], [torch.zeros(10, dtype=torch.complex64)])
    with pytest.raises(ValueError, match="input must be"):
        p.filter([torch.zeros((1000, 2), dtype=torch.float16)], [ok_x])
    with pytest.raises(ValueError, match="on the GPU"):      # right type and size, but host memory
        p.filter([ok_x], [torch.zeros(1000, dtype=torch.complex64)])
    p.close()
    p = host_plan([chan(length=1000)], dtype="f16", flags=vbw.F32_OUT)
    with pytest.raises(ValueError, match="on the GPU"):
        p.filter([torch.zeros((1000, 2), dtype=torch.float16)], [torch.zeros(1000, dtype=torch.complex64)])
    with pytest.raises(ValueError, match="fewer than"):
        p.filter([torch.zeros((1000, 2), dtype=torch.float16)], [torch.zeros((1000, 1), dtype=torch.float32)])
    p.close()
    p = host_plan([chan(length=1000)], dtype="r32")
    with pytest.raises(ValueError, match="input must be"):
        p.filter([torch.zeros(1000, dtype=torch.complex64)], [torch.zeros(1000, dtype=torch.float32)])
    p.close()


def test_binding_event_handles():
    """The timed calls (Plan.filter_timed, a bound run with events) take both
    events, and only events that exist: a torch event that was never recorded
    has no HIP event yet, and a null handle would reach the library."""
    with pytest.raises(ValueError, match="both"):
        vbw._event_handles(None, 0x10)
    with pytest.raises(ValueError, match="must exist"):
        vbw._event_handles(0x10, 0)
    assert vbw._event_handles(0x10, 0x20) == (0x10, 0x20)

    class Ev:
        def __init__(self, h):
            self.cuda_event = h
    assert vbw._event_handles(Ev(0x30), Ev(0x40)) == (0x30, 0x40)
    with pytest.raises(ValueError, match="must exist"):
        vbw._event_handles(Ev(0), Ev(0x40))


def test_binding_fails_loudly_without_the_library(tmp_path):
    """With the HIP library absent the binding raises (there is no CPU
    fallback): a fresh interpreter pointed at a missing library path."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2406_14116_amd import vbw\n"
            "try:\n"
            "    vbw.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "    raise SystemExit(3)\n"
            "raise SystemExit(0)\n")
    env = dict(os.environ, VBW_LIBRARY=str(tmp_path / "absent" / "libvbw.so"), PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 3, (r.returncode, r.stdout, r.stderr)
    assert "missing" in r.stdout
