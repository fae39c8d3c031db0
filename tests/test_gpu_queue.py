"""The persistent batched solve (one launch over a pass-ordered work queue):
parity with the float64 oracle (paper Eqs. 2-3 and Section 3 define what a
solve computes), bitwise equality of a batch with lone queue solves, every
radix choice, graph replay, the bounded-wait error path and the tuner."""

import numpy as np
import pytest

import oracle
import paper_1211_5244_amd as P
from densities import batch_density

pytestmark = pytest.mark.gpu

H = 0.3
REL_L2 = 1e-6
ELEM = 4e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load_library()
    return torch


def _check(V, rho, bc, what):
    ref = oracle.solve(rho.astype(np.float64), bc, H)
    err = oracle.rel_l2(V, ref)
    emax = float(np.max(np.abs(V.astype(np.float64) - ref)) / np.max(np.abs(ref)))
    print(f"{what}: relL2 {err:.3e} max elementwise {emax:.3e}", flush=True)
    assert err <= REL_L2, (what, err)
    assert emax <= ELEM, (what, emax)


def _queue_batch(cases, **shape):
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    B.mode = P.POISSON_BATCH_QUEUE
    if shape:
        B.set_queue_shape(**shape)
    return B


def _solve(torch, B, rhos):
    Vs = [torch.full_like(r, float("nan")) for r in rhos]
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    assert B.queue_status() == 0
    return Vs


# mixed sizes and classes: ragged extents, odd sizes, 3*2^k lengths
MIXED = [((32, 32, 32), 7), ((24, 12, 16), 0), ((12, 48, 6), 3), ((48, 8, 24), 5),
         ((16, 16, 64), 2), ((6, 8, 12), 6), ((24, 6, 3), 4), ((8, 12, 96), 1), ((3, 6, 12), 7)]


def test_queue_matches_oracle_and_lone_solves(torch_dev):
    """A mixed batch in one queue launch meets the oracle bar per solve and
    equals each solve run alone through the queue, bit for bit."""
    torch = torch_dev
    cases = [(n, bc, 2000 + i) for i, (n, bc) in enumerate(MIXED)]
    print("queue mixed batch", [c[:2] for c in cases], flush=True)
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    B = _queue_batch(cases)
    Vs = _solve(torch, B, rhos)
    for i, (n, bc, _) in enumerate(cases):
        _check(Vs[i].cpu().numpy(), rhos[i].cpu().numpy(), bc, f"queue {n} bc={bc}")
        lone = _queue_batch([cases[i]])
        Vl = _solve(torch, lone, [rhos[i]])
        assert torch.equal(Vl[0], Vs[i]), (i, n, bc)
        lone.close()
    # a second launch reuses the counters the first one returned to zero
    again = _solve(torch, B, rhos)
    for i in range(len(cases)):
        assert torch.equal(again[i], Vs[i]), i
    B.close()


@pytest.mark.parametrize("sel", [0, 1, 2])
def test_queue_radix_choices(torch_dev, sel):
    """Every radix decomposition of every length in the batch meets the
    oracle bar; small tiles and items (many items per solve) too."""
    torch = torch_dev
    cases = [((32, 32, 32), 7, 2100), ((48, 48, 48), 0, 2101), ((24, 48, 12), 3, 2102),
             ((64, 32, 16), 2, 2103), ((96, 3, 6), 2, 2104)]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    B = _queue_batch(cases, tile_elems=256, item_kb=8)
    lengths = {2 * e if (bc >> j) & 1 else e for n, bc, _ in cases for j, e in enumerate(n)}
    for L in sorted(lengths):
        B.set_queue_radix(L, sel)
        assert B.queue_radix(L) == sel
    Vs = _solve(torch, B, rhos)
    for i, (n, bc, _) in enumerate(cases):
        _check(Vs[i].cpu().numpy(), rhos[i].cpu().numpy(), bc, f"queue radix {sel} {n} bc={bc}")
    B.close()


EXTREME = [((512, 6, 8), 7), ((1024, 4, 6), 0), ((2, 4, 2), 7), ((384, 8, 6), 7), ((12, 24, 3), 7),
           ((2, 2, 2), 7)]


@pytest.mark.parametrize("n,bc", EXTREME)
def test_queue_extreme_lengths(torch_dev, n, bc):
    """Lengths 4 and 1024, the tiniest grids and odd extents."""
    torch = torch_dev
    print(f"queue extreme {n} bc={bc}", flush=True)
    rho = torch.from_numpy(batch_density(n, bc, 2200).astype(np.float32)).cuda()
    B = _queue_batch([(n, bc, 0)])
    V = _solve(torch, B, [rho])[0]
    _check(V.cpu().numpy(), rho.cpu().numpy(), bc, f"queue {n} bc={bc}")
    B.close()


def test_queue_batch_edges_match_grouped(torch_dev):
    """Edges 32..128 in all four classes: at the default radix choices the
    queue computes every butterfly as the grouped launches do and gives their
    results bit for bit; edges 96 and 128 meet the oracle bar."""
    torch = torch_dev
    from densities import BATCH_BCS, BATCH_EDGES
    cases = [((e, e, e), bc, 2300 + 4 * k + j) for k, e in enumerate(BATCH_EDGES) for j, bc in enumerate(BATCH_BCS)]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    G = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    Vg = [torch.empty_like(r) for r in rhos]
    G.solve(rhos, Vg)
    Q = _queue_batch(cases)
    Vq = _solve(torch, Q, rhos)
    for i, (n, bc, _) in enumerate(cases):
        assert torch.equal(Vq[i], Vg[i]), (n, bc)
        if n[0] >= 96:
            _check(Vq[i].cpu().numpy(), rhos[i].cpu().numpy(), bc, f"queue {n} bc={bc}")
    G.close()
    Q.close()


def test_queue_graph_replay(torch_dev):
    """The queue launch captured in a graph replays to the eager result,
    replay after replay, with eager work between the replays."""
    torch = torch_dev
    cases = [(n, bc, 2400 + i) for i, (n, bc) in enumerate(MIXED)]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    B = _queue_batch(cases)
    Vs = _solve(torch, B, rhos)
    eager = [v.clone() for v in Vs]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            P.poisson_batch_solve(B.handle, rhos, Vs, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        for v in Vs:
            v.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(cases)):
            assert torch.equal(Vs[i], eager[i]), (rep, i)
        B.solve(rhos, Vs)
        torch.cuda.synchronize()
    assert B.queue_status() == 0
    # new arrays cannot be uploaded inside a capture
    other = [torch.empty_like(v) for v in Vs]
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(P.PoissonError) as e:
        with torch.cuda.stream(side):
            with torch.cuda.graph(g2):
                P.poisson_batch_solve(B.handle, rhos, other, torch.cuda.current_stream())
    assert e.value.code == P._lib.POISSON_E_STATE
    torch.cuda.synchronize()
    B.close()


def test_queue_bounded_wait_reports_and_recovers(torch_dev):
    """A spin limit of one poll makes waits run out: the launch still ends,
    the sticky flag reports it, and with the default limit the next launch
    is correct again."""
    torch = torch_dev
    cases = [(n, bc, 2500 + i) for i, (n, bc) in enumerate(MIXED)]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    B = _queue_batch(cases, tile_elems=256, item_kb=4)
    good = _solve(torch, B, rhos)
    B.set_queue_spin(1)
    Vs = [torch.empty_like(r) for r in rhos]
    for _ in range(3):
        B.solve(rhos, Vs)
    torch.cuda.synchronize()
    assert B.queue_status() & P._lib.QUEUE_ERR_SPIN
    assert B.queue_status() == 0  # cleared by the read
    B.set_queue_spin(1 << 20)
    again = _solve(torch, B, rhos)
    for i in range(len(cases)):
        assert torch.equal(again[i], good[i]), i
    B.close()


def test_queue_tuner_and_modes(torch_dev):
    """The batch tuner times the queue against the grouped launches and
    keeps the faster; results meet the oracle bar in the mode it chose, and
    split-precision batches refuse the queue."""
    torch = torch_dev
    cases = [(n, bc, 2600 + i) for i, (n, bc) in enumerate(MIXED)]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    Vs = [torch.empty_like(r) for r in rhos]
    B.tune(rhos, Vs, reps=2)
    mode = B.mode
    print("tuned mode", mode, flush=True)
    assert mode in (P.POISSON_BATCH_GROUPED, P.POISSON_BATCH_QUEUE)
    Vs = _solve(torch, B, rhos)
    for i, (n, bc, _) in enumerate(cases):
        _check(Vs[i].cpu().numpy(), rhos[i].cpu().numpy(), bc, f"tuned {n} bc={bc}")
    B.close()
    S = P.Batch([(16, 16, 16)], [7], [H], precision=P.POISSON_SPLIT_FP16)
    with pytest.raises(P.PoissonError) as e:
        S.mode = P.POISSON_BATCH_QUEUE
    assert e.value.code == P._lib.POISSON_E_UNSUPPORTED
    assert S.mode == P.POISSON_BATCH_GROUPED
    S.close()


def test_queue_full_batch512(torch_dev):
    """The whole 512-solve batch the bench times, as one queue launch: every
    solve equals the grouped launches' result bit for bit (which equals the
    lone solves' and meets the oracle bar in the tests above), and the launch
    reports no flags.  Other radix choices agree to float32 rounding."""
    torch = torch_dev
    from densities import batch_workload
    items = batch_workload(512)
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in items]
    G = P.Batch([c[0] for c in items], [c[1] for c in items], [H] * len(items))
    Vg = [torch.empty_like(r) for r in rhos]
    G.solve(rhos, Vg)
    Q = _queue_batch(items)
    Vq = _solve(torch, Q, rhos)
    for i, (n, bc, _) in enumerate(items):
        assert torch.equal(Vq[i], Vg[i]), (i, n, bc)
    for L in (32, 48, 64, 96, 128, 192, 256):
        Q.set_queue_radix(L, 1)
    Vr = _solve(torch, Q, rhos)
    worst = 0.0
    for i in range(len(items)):
        d = float(torch.linalg.vector_norm(Vr[i] - Vg[i]) / torch.linalg.vector_norm(Vg[i]))
        worst = max(worst, d)
    print(f"queue batch512, radix-4 stages, vs grouped: worst relL2 {worst:.2e}", flush=True)
    assert worst <= 5e-7
    G.close()
    Q.close()


def test_queue_runs_isf_kernels(torch_dev):
    """The queue takes each plan's K^F as built, so an ISF batch (free,
    surface, wire) gives its grouped launches' results bit for bit."""
    torch = torch_dev
    cases = [((32, 32, 32), 7, 2700), ((24, 48, 12), 3, 2701), ((16, 16, 64), 2, 2702)]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    n_list, bc_list = [c[0] for c in cases], [c[1] for c in cases]
    G = P.Batch(n_list, bc_list, [H] * len(cases), kernel="isf")
    Vg = [torch.empty_like(r) for r in rhos]
    G.solve(rhos, Vg)
    Q = P.Batch(n_list, bc_list, [H] * len(cases), kernel="isf")
    Q.mode = P.POISSON_BATCH_QUEUE
    Vq = _solve(torch, Q, rhos)
    for i, (n, bc, _) in enumerate(cases):
        assert torch.equal(Vq[i], Vg[i]), (n, bc)
    G.close()
    Q.close()


def test_queue_full_free256(torch_dev):
    """The headline problem (free 256^3, FFT grid 512^3) as a queue launch: it
    equals the plain solve bit for bit, launch after launch."""
    torch = torch_dev
    from densities import workload_density
    n, bc, rho = workload_density("free256", H)
    r = torch.from_numpy(rho.astype(np.float32)).cuda()
    plan = P.Plan(n, bc, H)
    ref = plan.solve(r)
    torch.cuda.synchronize()
    B = _queue_batch([(n, bc, 0)])
    for _ in range(2):
        V = _solve(torch, B, [r])[0]
        assert torch.equal(V, ref)
    B.close()
    plan.close()
