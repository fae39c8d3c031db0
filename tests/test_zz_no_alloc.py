"""The allocation-free residual (poisson_rel_l2_noalloc) against the
allocating one (poisson_rel_l2), through the C ABI.

Its partial sums live in the library's static device scratch, which keeps the
last call's contents: two calls in a row, the second on a smaller input, must
each match poisson_rel_l2 on the same data, and so must every replay of a
HIP graph that captured it (with other work between the replays)."""

import numpy as np
import pytest

import paper_1211_5244_amd as P

pytestmark = pytest.mark.gpu

REL = 1e-15  # float64: same partial sums, summed in the same order


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load_library()
    return torch


def _pair(torch, count, seed):
    g = np.random.default_rng(seed)
    ref = g.standard_normal(count)
    v = (ref * (1.0 + 1e-6 * g.standard_normal(count))).astype(np.float32)
    return torch.from_numpy(v).cuda(), torch.from_numpy(ref).cuda()


def _noalloc(torch, v, ref, count):
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    P.poisson_rel_l2_noalloc(v, ref, count, out, stream)
    torch.cuda.synchronize()
    return float(out.item())


def test_two_calls_second_smaller(torch_dev):
    torch = torch_dev
    for count, seed in ((1 << 24, 1), (1000, 2)):  # 1024 block partials, then 4
        v, ref = _pair(torch, count, seed)
        want = P.poisson_rel_l2(v, ref, count)
        got = _noalloc(torch, v, ref, count)
        print(f"count {count}: noalloc {got!r} vs allocating {want!r}", flush=True)
        assert got == pytest.approx(want, rel=REL, abs=0.0)


def test_zero_reference_and_exact_match(torch_dev):
    torch = torch_dev
    v = torch.zeros(4096, dtype=torch.float32, device="cuda")
    ref = torch.zeros(4096, dtype=torch.float64, device="cuda")
    assert _noalloc(torch, v, ref, 4096) == P.poisson_rel_l2(v, ref, 4096) == 0.0
    v2, _ = _pair(torch, 5000, 3)
    exact = v2.double()  # the float32 values themselves: zero residual
    assert _noalloc(torch, v2, exact, 5000) == 0.0


def test_graph_replays(torch_dev):
    torch = torch_dev
    count = 300_000
    v, ref = _pair(torch, count, 4)
    want = P.poisson_rel_l2(v, ref, count)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            P.poisson_rel_l2_noalloc(v, ref, count, out, torch.cuda.current_stream())
    torch.cuda.synchronize()
    other_v, other_ref = _pair(torch, 2048, 5)
    for rep in range(4):
        out.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert float(out.item()) == pytest.approx(want, rel=REL, abs=0.0), rep
        # eager work between the replays leaves other partials in the scratch
        assert _noalloc(torch, other_v, other_ref, 2048) == pytest.approx(
            P.poisson_rel_l2(other_v, other_ref, 2048), rel=REL, abs=0.0)
