"""Host-side checks of the C ABI: the library loads, exports every symbol
the header declares, and its planner follows the paper's row counts
(Section 3) and the byte model of the five-pass schedule.  No device calls."""

import ctypes
import itertools
import json
import os
import re
from fractions import Fraction

import pytest

import paper_1211_5244_amd as P
from paper_1211_5244_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_ratios.json")))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "poisson.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*\s*|int\s+)(poisson_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = header_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTED) == names


@pytest.mark.parametrize("n,bc", [((256, 256, 256), 7), ((192, 192, 384), 3), ((384, 192, 384), 2),
                                  ((128, 128, 128), 0), ((32, 32, 32), 7)])
def test_byte_model(n, bc):
    d = P.poisson_plan_describe(*n, bc)
    S = [n[j] * (2 if (bc >> j) & 1 else 1) for j in range(3)]
    assert d["S"] == tuple(S)
    p, q, r = d["axis_order"]
    H = S[p] // 2 + 1
    want = (8 * n[0] * n[1] * n[2] + 32 * H * n[q] * n[r] + 32 * H * S[q] * n[r]
            + 4 * H * (S[q] // 2 + 1) * (S[r] // 2 + 1))
    assert d["alg_bytes"] == want
    ws = 8 * H * n[q] * n[r] + 8 * H * S[q] * n[r]
    assert ws <= d["workspace_bytes"] < ws + 512


def test_headline_byte_counts():
    assert P.poisson_plan_describe(256, 256, 256, 7)["alg_bytes"] == pytest.approx(1819.0e6, rel=1e-4)
    assert P.poisson_plan_describe(192, 192, 384, 3)["alg_bytes"] == pytest.approx(825.0e6, rel=1e-4)
    assert P.poisson_plan_describe(384, 192, 384, 2)["alg_bytes"] == pytest.approx(1165.9e6, rel=1e-4)


@pytest.mark.parametrize("bc", range(8))
def test_axis_order_puts_periodic_axes_first(bc):
    d = P.poisson_plan_describe(64, 64, 64, bc)
    free = [(bc >> a) & 1 for a in d["axis_order"]]
    assert free == sorted(free), (bc, d["axis_order"])
    # among orders with the same free pattern, x leads when it can
    if not (bc & 1):
        assert d["axis_order"][0] == 0


def _work(n, bc):
    rows, lens = P.poisson_plan_rows(*n, bc)
    return sum(r * l for r, l in zip(rows, lens))


def test_fft_work_ratios_of_the_paper():
    N = 64
    g = GOLDEN["fft_work_ratios"]
    # fully free vs the full padded grid (3 * S^3 points of 1D transforms)
    S = 2 * N
    assert Fraction(_work((N, N, N), 7), 3 * S ** 3) == Fraction(*g["free"])
    # wire: periodic z first; reference = full padded 3D FFT of (N, 2N, 2N)
    assert Fraction(_work((N, N, N), 3), 3 * N * S * S) == Fraction(*g["wire_periodic_axis_first"])
    # surface with free y last vs the periodic problem of the same FFT size
    per = _work((N, S, N), 0)
    assert Fraction(_work((N, N, N), 2), per) == Fraction(*g["surface_free_axis_last_vs_periodic"])


def _work_ordered(n, bc, order):
    d = P.poisson_plan_describe_ordered(*n, bc, axis_order=order)
    lens = [d["S"][a] for a in d["axis_order"]]
    return sum(r * l for r, l in zip(d["rows"], lens))


@pytest.mark.parametrize("bc", range(8))
def test_forced_orders_and_the_automatic_choice(bc):
    n = (48, 32, 24)
    auto = P.poisson_plan_describe(*n, bc)
    best = None
    for order in itertools.permutations(range(3)):
        d = P.poisson_plan_describe_ordered(*n, bc, axis_order=order)
        assert d["axis_order"] == order
        assert d["S"] == auto["S"]
        # rows of Section 3 in this order: N_q N_r, S_p N_r, S_p S_q
        p, q, r = order
        assert d["rows"] == (n[q] * n[r], d["S"][p] * n[r], d["S"][p] * d["S"][q])
        best = d["alg_bytes"] if best is None else min(best, d["alg_bytes"])
    assert auto["alg_bytes"] == best
    assert P.poisson_plan_describe_ordered(*n, bc)["axis_order"] == auto["axis_order"]


def test_axis_order_ablation_ratios():
    """Section 3's row rule in the orders it compares.  Wire (x, y free, z
    periodic, N^3 data): z first costs N^3 + 2N^3 + 4N^3 of the full 12N^3
    (7/12, as free); z last 2N^3 + 4N^3 + 4N^3 (5/6).  Surface (y free):
    y last costs 4N^3 of 6N^3 (2/3); y first 6N^3 (no gain)."""
    N = 64
    S = 2 * N
    wire_full = 3 * S * S * N          # full padded 3D transform of (2N, 2N, N)
    assert Fraction(_work_ordered((N, N, N), 3, (2, 0, 1)), wire_full) == Fraction(7, 12)
    assert Fraction(_work_ordered((N, N, N), 3, (0, 1, 2)), wire_full) == Fraction(5, 6)
    surf_full = 3 * N * S * N          # (N, 2N, N), y free
    assert Fraction(_work_ordered((N, N, N), 2, (0, 2, 1)), surf_full) == Fraction(2, 3)
    assert Fraction(_work_ordered((N, N, N), 2, (1, 0, 2)), surf_full) == Fraction(1, 1)


@pytest.mark.parametrize("order", [(0, 0, 1), (0, 1, 3), (-1, 1, 2), (2, 2, 2)])
def test_forced_order_must_be_a_permutation(order):
    with pytest.raises(P.PoissonError) as e:
        P.poisson_plan_describe_ordered(16, 16, 16, 7, axis_order=order)
    assert e.value.code == P._lib.POISSON_E_ARG


def test_transfer_fractions_of_the_paper():
    g = GOLDEN["transfer_fractions"]
    N = 32
    for name, bc in (("free", 7), ("wire", 3), ("surface", 2), ("periodic", 0)):
        d = P.poisson_plan_describe(N, N, N, bc)
        frac = Fraction(N ** 3, d["S"][0] * d["S"][1] * d["S"][2])
        assert frac == Fraction(*g[name]), name


def test_rows_follow_section_3():
    rows, lens = P.poisson_plan_rows(48, 32, 24, 7)
    # x, y, z all free: N_y N_z rows of S_x, S_x N_z rows of S_y, S_x S_y rows of S_z
    assert rows == (32 * 24, 96 * 24, 96 * 64) and lens == (96, 64, 48)


@pytest.mark.parametrize("args,code", [
    ((5, 8, 8, 7), P._lib.POISSON_E_UNSUPPORTED),   # S = 10
    ((8, 8, 1, 7), P._lib.POISSON_E_ARG),           # n < 2
    ((8, 8, 8, 8), P._lib.POISSON_E_ARG),           # mask out of range
    ((2048, 8, 8, 0), P._lib.POISSON_E_ARG),        # too long
    ((1024, 8, 8, 1), P._lib.POISSON_E_UNSUPPORTED),  # S = 2048
    ((7, 8, 8, 0), P._lib.POISSON_E_UNSUPPORTED),   # prime factor 7
])
def test_describe_rejects_bad_arguments(args, code):
    with pytest.raises(P.PoissonError) as e:
        P.poisson_plan_describe(*args)
    assert e.value.code == code
    assert P.poisson_last_error()


def test_precision_modes():
    for prec in (P.POISSON_FP32, P.POISSON_SPLIT_FP16, P.POISSON_SPLIT_BF16):
        assert P.poisson_plan_describe(64, 64, 64, 7, prec)["alg_bytes"] > 0
    with pytest.raises(P.PoissonError) as e:
        P.poisson_plan_describe(64, 64, 64, 7, 9)
    assert e.value.code == P._lib.POISSON_E_ARG


def test_null_and_bad_host_arguments():
    lib = P.load_library()
    assert lib.poisson_plan(None, 8, 8, 8, 7, 0.3, 0) == P._lib.POISSON_E_ARG
    out = ctypes.c_void_p()
    assert lib.poisson_plan(ctypes.byref(out), 8, 8, 8, 7, -1.0, 0) == P._lib.POISSON_E_ARG
    assert lib.poisson_plan(ctypes.byref(out), 8, 8, 8, 7, float("nan"), 0) == P._lib.POISSON_E_ARG
    assert lib.poisson_solve(None, None, None, None) == P._lib.POISSON_E_ARG
    assert lib.poisson_kernel_set(None, None, 0) == P._lib.POISSON_E_ARG
    assert lib.poisson_kernel_build_isf(None, 16, None) == P._lib.POISSON_E_ARG
    assert lib.poisson_batch_kernel_build_isf(None, 16, None) == P._lib.POISSON_E_ARG
    assert lib.poisson_batch_create(ctypes.byref(out), 0, None, None, None, 0) == P._lib.POISSON_E_ARG
    assert lib.poisson_plan_destroy(None) == 0


def test_null_handles_of_the_later_entry_points():
    """Schedules, tuning, host-buffer solves and plan queries reject a NULL
    plan or array before touching any device."""
    lib = P.load_library()
    E = P._lib.POISSON_E_ARG
    sel = (ctypes.c_int * 5)()
    assert lib.poisson_plan_set_schedule(None, sel) == E
    assert lib.poisson_plan_get_schedule(None, sel, sel) == E
    assert lib.poisson_plan_tune(None, None, None, 0, None, None) == E
    assert lib.poisson_batch_tune(None, None, None, 0, None, None) == E
    assert lib.poisson_solve_host(None, None, None, None) == E
    assert lib.poisson_solve_host_many(None, 1, None, None, None) == E
    assert lib.poisson_plan_info(None, None, None, None, None) == E
    assert lib.poisson_batch_set_streams(None, 2) == E
    assert lib.poisson_set_tune_cache(None) == 0  # host only: switches the cache off
    assert lib.poisson_batch_get_streams(None, None) == E
    assert lib.poisson_rel_l2_noalloc(None, None, 0, None, None) == E
    assert lib.poisson_rel_l2_noalloc(None, None, 16, None, None) == E
    assert lib.poisson_batch_set_mode(None, 1) == E
    assert lib.poisson_batch_get_mode(None, None) == E
    assert lib.poisson_batch_set_queue_radix(None, 64, 0) == E
    assert lib.poisson_batch_get_queue_radix(None, 64, None) == E
    assert lib.poisson_batch_set_queue_shape(None, 2048, 256) == E
    assert lib.poisson_batch_set_queue_spin(None, 1) == E
    assert lib.poisson_batch_queue_status(None, None) == E
    assert lib.poisson_queue_radices(64, 0, None) == E
    assert lib.poisson_queue_simulate(0, None, 1, 0, 1, None) == E
    out = ctypes.c_void_p()
    bad = (ctypes.c_int * 3)(0, 0, 1)
    assert lib.poisson_plan_ordered(ctypes.byref(out), 8, 8, 8, 7, 0.3, 0, bad) == E
    assert out.value is None


def test_batch_rejects_one_bad_entry_before_any_device_call():
    with pytest.raises(P.PoissonError) as e:
        P.poisson_batch_create([(8, 8, 8), (5, 8, 8)], [7, 7], [0.3, 0.3])
    assert e.value.code == P._lib.POISSON_E_UNSUPPORTED
    assert "entry 1" in str(e.value)
    with pytest.raises(P.PoissonError) as e:
        P.poisson_batch_create([(8, 8, 8), (8, 8, 8)], [7, 7], [0.3, 0.0])
    assert e.value.code == P._lib.POISSON_E_ARG
