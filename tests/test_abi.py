"""Host-side checks of the C ABI: the library loads, exports every symbol
the header declares, and its planner follows the paper's row counts
(Section 3) and the byte model of the five-pass schedule.  No device calls."""

import ctypes
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
    assert lib.poisson_batch_create(ctypes.byref(out), 0, None, None, None, 0) == P._lib.POISSON_E_ARG
    assert lib.poisson_plan_destroy(None) == 0


def test_batch_rejects_one_bad_entry_before_any_device_call():
    with pytest.raises(P.PoissonError) as e:
        P.poisson_batch_create([(8, 8, 8), (5, 8, 8)], [7, 7], [0.3, 0.3])
    assert e.value.code == P._lib.POISSON_E_UNSUPPORTED
    assert "entry 1" in str(e.value)
    with pytest.raises(P.PoissonError) as e:
        P.poisson_batch_create([(8, 8, 8), (8, 8, 8)], [7, 7], [0.3, 0.0])
    assert e.value.code == P._lib.POISSON_E_ARG
