"""Host logic: the pass descriptors of plan.cpp against the arrays they
address.  Every GPU kernel trusts these strides and extents, so for many
sizes, boundary conditions and forced axis orders the tests check, on the
CPU, that every element a pass reads or writes lies inside its array, that
no two lines of a pass write the same element, and that each pass covers
exactly the elements the next one reads (Section 3's row counts)."""

import itertools
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1211_5244_amd", "csrc")


@pytest.fixture(scope="module")
def dump():
    out = os.path.join(tempfile.mkdtemp(prefix="plan_dump_"), "plan_dump")
    cmd = ["g++", "-std=c++17", "-O1", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "plan_dump.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)

    def run(n, bc, order=None):
        args = [out, *map(str, n), str(bc)] + ([] if order is None else list(map(str, order)))
        lines = subprocess.run(args, check=True, capture_output=True, text=True).stdout.split("\n")
        if lines[0].startswith("error"):
            return None
        g = list(map(int, lines[0].split()[1:]))
        passes = [list(map(int, ln.split()[1:])) for ln in lines[1:6]]
        return g, passes
    return run


# element offsets a pass touches: per line (a, b) and element j
def _offsets(count, ext_tile, ext_batch, s):
    j = np.arange(count)[:, None, None]
    a = np.arange(ext_tile)[None, :, None]
    b = np.arange(ext_batch)[None, None, :]
    return (j * s[0] + a * s[1] + b * s[2]).ravel()


def _check(n, bc, g, passes):
    order, S, a1, a2 = g[:3], g[3:6], g[6], g[7]
    p, q, r = order
    grid = n[0] * n[1] * n[2]
    H = S[p] // 2 + 1
    sizes_in = [grid, a1, a2, a2, a1]
    sizes_out = [a1, a2, a2, a1, grid]
    # values read / written per line, from the kind and the padding alone
    # (R2C, FWD, CONV, INV, C2R): a padded line holds its first L/2 values,
    # a cropped one keeps its first L/2, a real transform keeps L/2+1
    for k, (idx, kind, L, n_in, n_out, et, eb, i0, i1, i2, o0, o1, o2, it, ot, pad, crop) in \
            enumerate(passes):
        assert idx == k and kind == k
        half_or_full_in = L // 2 if pad else L
        half_or_full_out = L // 2 if crop else L
        reads = [half_or_full_in, half_or_full_in, half_or_full_in, L, L // 2 + 1][kind]
        writes = [L // 2 + 1, L, half_or_full_out, half_or_full_out, half_or_full_out][kind]
        assert (n_in, n_out) == (reads, writes), (k, n, bc, order)
        ins = _offsets(reads, et, eb, (i0, i1, i2))
        outs = _offsets(writes, et, eb, (o0, o1, o2))
        assert ins.min() >= 0 and ins.max() < sizes_in[k], (k, n, bc, order)
        assert outs.min() >= 0 and outs.max() < sizes_out[k], (k, n, bc, order)
        # no element written twice, and every element of the output array
        # written (the next pass reads all of it)
        assert len(np.unique(outs)) == len(outs), (k, n, bc, order)
        assert len(outs) == sizes_out[k], (k, n, bc, order, len(outs), sizes_out[k])
        # tiled / line sides are what the kernels assume
        assert (i0 == 1) != bool(it) and (o0 == 1) != bool(ot)
        if it:
            assert i1 == 1
        if ot:
            assert o1 == 1
    # Section 3 row counts: N_q N_r, S_p N_r, S_p S_q (complex rows after
    # the real first step: H instead of S_p)
    assert passes[0][5] * passes[0][6] == n[q] * n[r]
    assert passes[1][5] * passes[1][6] == H * n[r]
    assert passes[2][5] * passes[2][6] == H * S[q]


SIZES = [(6, 8, 12), (16, 16, 16), (24, 32, 48), (12, 48, 32), (2, 4, 2), (96, 6, 4), (4, 6, 384)]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("bc", range(8))
def test_pass_descriptors_stay_in_bounds(dump, n, bc):
    res = dump(n, bc)
    if res is None:
        pytest.skip("length not supported for this mask")
    _check(n, bc, *res)


@pytest.mark.parametrize("order", list(itertools.permutations(range(3))))
@pytest.mark.parametrize("bc", [0, 2, 3, 7])
def test_forced_orders_stay_in_bounds(dump, order, bc):
    n = (24, 16, 12)
    res = dump(n, bc, order)
    assert res is not None
    assert tuple(res[0][:3]) == order
    _check(n, bc, *res)


def _plane_ok(g, passes):
    """Whether the library enables the plane kernel for this geometry (the
    flag plan_dump prints from plane_geometry_ok).  Where it does, the
    kernel's structural preconditions must hold: q-lines contiguous in A1,
    pass 3 writing back exactly where pass 1 reads, one plane of N_r lines
    per p index."""
    if not g[8]:
        return False
    H = g[3 + g[0]] // 2 + 1
    p2, p3, p4 = passes[1], passes[2], passes[3]
    LR, pr = p3[2], p3[15]
    assert (p2[7] == 1 and p4[10] == 1 and p4[11] == p2[8] and p4[12] == p2[9]
            and p4[5] == p2[5] and p4[6] == p2[6] and p2[6] == H
            and p2[5] == (LR // 2 if pr else LR)), (g, passes)
    return True


@pytest.mark.parametrize("e", [32, 48, 64])
@pytest.mark.parametrize("bc", [0, 2, 3, 7])
def test_plane_kernel_indexing(dump, e, bc):
    """The small-grid plane kernel's own addressing, on the CPU: plane kp of
    solve j reads and rewrites A1 at kp*s_p + r*s_r + q (q < N_q, r < N_r)
    and K^F row (kp, min(k_q, L_q - k_q)) up to k_r = L_r/2.  Where the
    library enables it, those offsets must stay inside A1 and the K^F table
    and be exactly the elements pass 1 reads and pass 3 writes."""
    n = (e, e, e)
    res = dump(n, bc)
    assert res is not None
    g, passes = res
    if not _plane_ok(g, passes):
        pytest.skip("no plane kernel for this geometry")
    a1 = g[6]
    p2, p3 = passes[1], passes[2]
    LQ, LR, pq, pr = p2[2], p3[2], p2[15], p3[15]
    NQ, NR = (LQ // 2 if pq else LQ), (LR // 2 if pr else LR)
    s_r, s_p, H = p2[8], p2[9], p2[6]
    kp = np.arange(H)[:, None, None]
    r = np.arange(NR)[None, :, None]
    q = np.arange(NQ)[None, None, :]
    offs = (kp * s_p + r * s_r + q).ravel()
    assert offs.min() >= 0 and offs.max() < a1
    assert len(np.unique(offs)) == len(offs) == a1
    reads = _offsets(p2[3], p2[5], p2[6], p2[7:10])
    writes = _offsets(passes[3][4], passes[3][5], passes[3][6], passes[3][10:13])
    assert set(offs.tolist()) == set(reads.tolist()) == set(writes.tolist())
    kq_half, KR = LQ // 2 + 1, LR // 2 + 1
    kq = np.arange(LQ)
    kqf = np.minimum(kq, LQ - kq)
    krow_max = ((H - 1) * kq_half + kqf.max()) * KR + LR // 2
    assert kqf.max() < kq_half and krow_max < H * kq_half * KR


def test_plane_cases_of_the_gpu_tests_are_enabled(dump):
    """Every geometry the GPU plane-kernel test selects has the kernel."""
    for n, bc in [((32, 32, 32), 0), ((48, 48, 48), 0), ((64, 64, 64), 0), ((32, 32, 32), 7),
                  ((32, 32, 32), 3), ((48, 48, 48), 7), ((64, 64, 64), 7), ((32, 32, 32), 2),
                  ((48, 48, 48), 2), ((64, 64, 64), 2), ((96, 96, 96), 0), ((128, 128, 128), 0),
                  ((96, 96, 96), 2), ((128, 128, 128), 2)]:
        g, passes = dump(n, bc)
        assert _plane_ok(g, passes), (n, bc)
