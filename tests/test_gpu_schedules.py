"""GPU: pass schedules (tile width, XCD workgroup order) and the autotuner.

Tile widths and workgroup orders only change which lines a workgroup stages
together and where it runs, so each must give results bitwise equal to
schedule 0 (whose parity against the oracle the parity tests establish), on
regular and ragged tiles.  The small-grid plane kernel (bit 3 of pass 2)
must agree to float32 rounding and meet the oracle bar.  The autotuner must
leave a valid schedule and equal results.
"""

import numpy as np
import pytest

import oracle
import paper_1211_5244_amd as P
from densities import batch_density, draw_gaussians, gaussian_mixture

pytestmark = pytest.mark.gpu

H = 0.3


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load_library()
    return torch


def _rho(torch, n, bc, seed):
    gs = draw_gaussians(n, H, 5, (1.0, 3.0), seed)
    return torch.from_numpy(gaussian_mixture(n, bc, H, gs).astype(np.float32)).cuda()


def _compiled(plan):
    """Per pass, the schedules compiled for it (distinct tile widths)."""
    out = []
    for k in range(5):
        ok = []
        for ts in range(P.TILE_SCHEDULES):
            sel = [0] * 5
            sel[k] = ts
            try:
                plan.set_schedule(sel)
                ok.append(ts)
            except P.PoissonError as e:
                assert e.code == P._lib.POISSON_E_UNSUPPORTED, e
        out.append(ok)
    plan.set_schedule([0] * 5)
    return out


# (n, bc): 512-length lines, ragged tiles (extents not multiples of the tile
# width), mixed radix, all four boundary classes
CASES = [((256, 256, 256), 7), ((24, 48, 12), 7), ((48, 24, 64), 3), ((12, 48, 24), 2),
         ((32, 24, 48), 0), ((96, 64, 48), 5)]


SPLIT_CASES = [((256, 256, 256), 7, P.POISSON_SPLIT_FP16), ((48, 24, 64), 3, P.POISSON_SPLIT_FP16),
               ((32, 24, 48), 0, P.POISSON_SPLIT_BF16), ((96, 64, 48), 5, P.POISSON_SPLIT_BF16)]


@pytest.mark.parametrize("n,bc,precision", [(n, bc, P.POISSON_FP32) for n, bc in CASES] + SPLIT_CASES)
def test_every_schedule_keeps_results(torch_dev, n, bc, precision):
    torch = torch_dev
    r = _rho(torch, n, bc, seed=700 + bc)
    plan = P.Plan(n, bc, H, precision=precision)
    ref = plan.solve(r).clone()
    compiled = _compiled(plan)
    print(f"{n} bc={bc}: compiled schedules per pass {compiled}", flush=True)
    # the fused conv pass: no tile width, both orders, maybe the plane kernel
    assert set(compiled[2]) in ({0, 4}, {0, 4, 8, 12})
    assert all(0 in c and 4 in c for c in compiled)  # the XCD order works everywhere
    assert not any(sel & P.PLANE_BIT for k in (0, 1, 3, 4) for sel in compiled[k])
    # one pass at a time, then all passes together
    trials = []
    for k in range(5):
        for ts in compiled[k][1:]:
            sel = [0] * 5
            sel[k] = ts
            trials.append(sel)
    for ts in range(1, P.TILE_SCHEDULES):  # every pass on schedule ts where compiled
        if any(ts in c for c in compiled):
            trials.append([ts if ts in c else 0 for c in compiled])
    for sel in trials:
        plan.set_schedule(sel)
        got_sel, lines = plan.schedule
        assert list(got_sel) == sel
        assert lines[2] == 0 and all(lines[k] > 0 for k in (0, 1, 3, 4))
        V = plan.solve(r)
        torch.cuda.synchronize()
        _assert_same_solve(V, ref, sel[2] & P.PLANE_BIT)


# every compiled plane-kernel geometry: periodic, free, wire and surface cubes
PLANE_CASES = [((32, 32, 32), 0), ((48, 48, 48), 0), ((64, 64, 64), 0), ((32, 32, 32), 7),
               ((32, 32, 32), 3), ((48, 48, 48), 7), ((64, 64, 64), 7), ((32, 32, 32), 2),
               ((48, 48, 48), 2), ((64, 64, 64), 2), ((96, 96, 96), 0), ((128, 128, 128), 0),
               ((96, 96, 96), 2), ((128, 128, 128), 2)]


@pytest.mark.parametrize("n,bc", PLANE_CASES)
def test_plane_kernel_matches_three_passes(torch_dev, n, bc):
    """Passes 1-3 as one LDS-resident plane kernel (schedule bit 3 of pass 2)
    against the three separate passes, and against the oracle; single solves
    and a batch chunk of three.

    The plane kernel evaluates the same butterflies as the separate passes
    with the rounding of each operation fixed in the source (no compiler
    contraction), so results are bitwise equal to them.  Its own accuracy
    against the oracle must meet the float32 bar.  Between two plane-kernel
    runs (XCD order on or off, single or batched) results are bitwise equal
    as well."""
    torch = torch_dev
    r = _rho(torch, n, bc, seed=900 + bc)
    plan = P.Plan(n, bc, H)
    ref = plan.solve(r).clone()
    plan.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    V = plan.solve(r).clone()
    torch.cuda.synchronize()
    d = oracle.rel_l2(V.cpu().numpy(), ref.cpu().numpy().astype(np.float64))
    assert torch.equal(V, ref), (n, bc, d)
    err = oracle.rel_l2(V.cpu().numpy(), oracle.solve(r.cpu().numpy().astype(np.float64), bc, H))
    assert err <= 1e-6
    plan.set_schedule([0, 0, P.PLANE_BIT | 4, 0, 0])  # with the XCD order bit too
    V2 = plan.solve(r)
    torch.cuda.synchronize()
    assert torch.equal(V2, V)
    # batches: one plane-kernel launch covers every solve of a chunk, each
    # solve bitwise equal to its single plane-kernel solve
    rhos = [_rho(torch, n, bc, seed=910 + i) for i in range(3)]
    B = P.Batch([n] * 3, [bc] * 3, [H] * 3)
    B.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    assert all(B.schedule(i) == (0, 0, P.PLANE_BIT, 0, 0) for i in range(3))
    Vs = [torch.empty_like(x) for x in rhos]
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    plan.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    for x, v in zip(rhos, Vs):
        assert torch.equal(plan.solve(x), v)


@pytest.mark.parametrize("precision", [P.POISSON_SPLIT_FP16, P.POISSON_SPLIT_BF16])
@pytest.mark.parametrize("n,bc", [((32, 32, 32), 7), ((48, 48, 48), 0), ((64, 64, 64), 2),
                                  ((32, 32, 32), 3), ((64, 64, 64), 7), ((128, 128, 128), 0),
                                  ((96, 96, 96), 2)])
def test_split_plane_kernel_equals_three_passes(torch_dev, n, bc, precision):
    """The plane kernel in the split modes.  The split line transform fixes
    its rounding order (matrix-core products, twiddle products with a fixed
    fused form), so unlike float32 the fused kernel gives results bitwise
    equal to the separate passes; they must meet the oracle bar, single and
    batched."""
    torch = torch_dev
    r = _rho(torch, n, bc, seed=960 + bc)
    plan = P.Plan(n, bc, H, precision=precision)
    ref = plan.solve(r).clone()
    plan.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    V = plan.solve(r).clone()
    torch.cuda.synchronize()
    d = oracle.rel_l2(V.cpu().numpy(), ref.cpu().numpy().astype(np.float64))
    err = oracle.rel_l2(V.cpu().numpy(), oracle.solve(r.cpu().numpy().astype(np.float64), bc, H))
    print(f"{n} bc={bc} precision={precision}: plane vs passes {d:.2e}, vs oracle {err:.2e}", flush=True)
    assert torch.equal(V, ref), d
    assert err <= 1e-6, err
    rhos = [_rho(torch, n, bc, seed=970 + i) for i in range(3)]
    B = P.Batch([n] * 3, [bc] * 3, [H] * 3, precision=precision)
    B.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    Vs = [torch.empty_like(x) for x in rhos]
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    for x, v in zip(rhos, Vs):
        assert torch.equal(plan.solve(x), v)


def test_batch_schedule_applies_to_every_problem(torch_dev):
    """poisson_batch_set_schedule: all distinct problems or none."""
    torch = torch_dev
    cases = [((32, 32, 32), 7), ((48, 48, 48), 0), ((24, 48, 12), 7)]  # the last has no plane kernel
    rhos = [_rho(torch, n, bc, seed=950 + i) for i, (n, bc) in enumerate(cases)]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * 3)
    ref = [torch.empty_like(x) for x in rhos]
    B.solve(rhos, ref)
    with pytest.raises(P.PoissonError) as e:
        B.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    assert e.value.code == P._lib.POISSON_E_UNSUPPORTED
    with pytest.raises(P.PoissonError) as e:
        B.set_schedule([0, 0, 0, P.TILE_SCHEDULES, 0])
    assert e.value.code == P._lib.POISSON_E_ARG
    assert all(B.schedule(i) == (0,) * 5 for i in range(3))
    with pytest.raises(P.PoissonError) as e:
        B.schedule(3)
    assert e.value.code == P._lib.POISSON_E_ARG
    Vs = [torch.empty_like(x) for x in rhos]
    B.solve(rhos, Vs)  # unchanged after the rejected calls
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(Vs, ref))
    B.set_schedule([4, 4, 4, 4, 4])  # XCD order: compiled everywhere, bitwise equal
    assert all(B.schedule(i) == (4,) * 5 for i in range(3))
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(Vs, ref))


def _assert_same_solve(V, ref, plane):
    """Bitwise equal under every schedule, the plane kernel included
    (test_plane_kernel_matches_three_passes)."""
    d = oracle.rel_l2(V.cpu().numpy(), ref.cpu().numpy().astype(np.float64))
    assert (V == ref).all(), (plane, d)


def test_schedule_rejects_bad_values(torch_dev):
    plan = P.Plan((32, 32, 32), 7, H)
    with pytest.raises(P.PoissonError) as e:
        plan.set_schedule([P.TILE_SCHEDULES, 0, 0, 0, 0])
    assert e.value.code == P._lib.POISSON_E_ARG
    with pytest.raises(P.PoissonError) as e:
        plan.set_schedule([0, 0, 1, 0, 0])
    assert e.value.code == P._lib.POISSON_E_UNSUPPORTED
    assert list(plan.schedule[0]) == [0] * 5  # unchanged after a rejected call
    split = P.Plan((32, 32, 32), 7, H, precision=P.POISSON_SPLIT_FP16)
    with pytest.raises(P.PoissonError) as e:
        split.set_schedule([0, 0, 1, 0, 0])  # the conv pass has no tile width
    assert e.value.code == P._lib.POISSON_E_UNSUPPORTED
    split.set_schedule([5, 4, 4, 4, 5])  # split modes compile the tile widths too
    assert list(split.schedule[0]) == [5, 4, 4, 4, 5]


@pytest.mark.parametrize("n,bc", [((256, 256, 256), 7), ((64, 96, 48), 3)])
def test_tune_keeps_results(torch_dev, n, bc):
    torch = torch_dev
    r = _rho(torch, n, bc, seed=800 + bc)
    plan = P.Plan(n, bc, H)
    ref = plan.solve(r).clone()
    scratch = torch.empty_like(r)
    ms = plan.tune(r, scratch, reps=3)
    sel, lines = plan.schedule
    print(f"{n} bc={bc}: tuned {sel} lines {lines} ms {[round(x, 4) for x in ms]}", flush=True)
    assert all(np.isfinite(ms)) and all(x > 0 for x in ms)
    V = plan.solve(r)
    torch.cuda.synchronize()
    _assert_same_solve(V, ref, sel[2] & P.PLANE_BIT)
    if n == (64, 96, 48):
        err = oracle.rel_l2(V.cpu().numpy(), oracle.solve(r.cpu().numpy().astype(np.float64), bc, H))
        assert err <= 1e-6


def test_batch_tune_keeps_results(torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(4999)
    cases = [((int(e),) * 3, int(b), 9000 + i)
             for i, (e, b) in enumerate(zip(rng.choice([32, 48, 64], 24), rng.choice([0, 3, 5, 7], 24)))]
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    ref = [torch.empty_like(r) for r in rhos]
    B.solve(rhos, ref)
    scratch = [torch.empty_like(r) for r in rhos]
    mb = B.tune(rhos, scratch, reps=2)
    print(f"batch tune: {mb} MiB per launch; schedules {sorted(set(B.schedule(i) for i in range(len(cases))))}",
          flush=True)
    assert mb in (32.0, 64.0, 96.0, 128.0, 192.0, 256.0, 384.0, 512.0)
    Vs = [torch.empty_like(r) for r in rhos]
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    for i in range(len(cases)):
        # the tuner may pick the plane kernel for some problems
        _assert_same_solve(Vs[i], ref[i], True)


@pytest.mark.parametrize("precision", [P.POISSON_FP32, P.POISSON_SPLIT_FP16])
def test_plane_kernel_batch_in_a_graph(torch_dev, precision):
    """A batch on the plane kernel captured in a HIP graph: every replay,
    with eager work between replays, equals the eager batch bitwise."""
    torch = torch_dev
    cases = [((32, 32, 32), 7), ((48, 48, 48), 0), ((64, 64, 64), 2), ((32, 32, 32), 7)]
    rhos = [_rho(torch, n, bc, seed=990 + i) for i, (n, bc) in enumerate(cases)]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases), precision=precision)
    B.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    Vs = [torch.empty_like(r) for r in rhos]
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
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
        B.solve(rhos, Vs)  # eager work between replays
        torch.cuda.synchronize()


def test_solve_passes_with_the_plane_bit(torch_dev):
    """poisson_solve_passes with the plane kernel selected: a range over
    passes 1-3 runs the plane kernel (equal to poisson_solve bitwise), any
    other split of the passes runs them separately (equal to the solve
    without the plane kernel bitwise)."""
    torch = torch_dev
    n, bc = (32, 32, 32), 7
    r = _rho(torch, n, bc, seed=995)
    plan = P.Plan(n, bc, H)
    separate = plan.solve(r).clone()
    plan.set_schedule([0, 0, P.PLANE_BIT, 0, 0])
    fused = plan.solve(r).clone()
    s = torch.cuda.current_stream()
    V = torch.empty_like(r)
    P.poisson_solve_passes(plan.handle, r, V, 0, 4, s)
    torch.cuda.synchronize()
    assert torch.equal(V, fused)
    V.zero_()
    P.poisson_solve_passes(plan.handle, r, V, 0, 3, s)
    P.poisson_solve_passes(plan.handle, r, V, 4, 4, s)
    torch.cuda.synchronize()
    assert torch.equal(V, fused)
    V.zero_()
    for first, last in ((0, 1), (2, 4)):
        P.poisson_solve_passes(plan.handle, r, V, first, last, s)
    torch.cuda.synchronize()
    assert torch.equal(V, separate)
    assert torch.equal(separate, fused)  # fixed rounding: the same bits either way


def test_tune_cache_round_trip(torch_dev, tmp_path):
    """poisson_plan_tune records its schedule; new plans of the same problem
    start from it (same results); unknown lines and schedules the build does
    not compile are ignored."""
    torch = torch_dev
    path = tmp_path / "tuned.txt"
    P.poisson_set_tune_cache(str(path))
    try:
        n, bc = (48, 24, 64), 3
        r = _rho(torch, n, bc, seed=41)
        plan = P.Plan(n, bc, H)
        assert plan.schedule[0] == (0, 0, 0, 0, 0)  # nothing cached yet
        ref = plan.solve(r).clone()
        plan.tune(r)
        tuned = plan.schedule[0]
        lines = path.read_text().splitlines()
        assert len(lines) == 1, lines
        key, vals = lines[0].split(" : ")
        assert tuple(int(v) for v in vals.split()) == tuned
        again = P.Plan(n, bc, H)
        assert again.schedule[0] == tuned
        assert torch.equal(again.solve(r), ref)
        # other problems and precisions have their own lines
        assert P.Plan(n, bc, H, precision=P.POISSON_SPLIT_FP16).schedule[0] == (0, 0, 0, 0, 0)
        again.tune(r)
        assert len(path.read_text().splitlines()) == 1  # replaced, not appended
        path.write_text("not a cache line\n" + key + " : 3 3 3 3 3\n")
        assert P.Plan(n, bc, H).schedule[0] == (0, 0, 0, 0, 0)
    finally:
        P.poisson_set_tune_cache(None)
    assert P.Plan(n, bc, H).schedule[0] == (0, 0, 0, 0, 0)
