"""GPU parity: the HIP path against the FP64 oracle.

Every case feeds the same float32-rounded density to both sides (seeded
Gaussian mixtures or seeded noise).  The bar is the relative L2 error of
1e-6 (float32 solver against the float64 definition), plus an element-wise
envelope; the float64 K^F built on the GPU must match the oracle's to 1e-12.
"""

import numpy as np
import pytest

import oracle
import paper_1211_5244_amd as P
from densities import WORKLOADS, draw_gaussians, gaussian_mixture, workload_density

pytestmark = pytest.mark.gpu

H = 0.3
REL_L2 = 1e-6        # float32 solver vs float64 definition
ELEM = 4e-6          # |dV_i| <= ELEM * max|V_ref|
KF_REL = 1e-12       # float64 kernel build vs float64 oracle kernel


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load_library()  # raises if the HIP library is missing: no fallback
    return torch


def _density(n, bc, seed, count=6):
    gs = draw_gaussians(n, H, count, (1.0, 3.0), seed)
    rho = gaussian_mixture(n, bc, H, gs)
    return rho.astype(np.float32)


def _gpu_solve(torch, n, bc, rho32, plan=None, precision=P.POISSON_FP32):
    plan = plan or P.Plan(n, bc, H, precision=precision)
    r = torch.from_numpy(rho32).cuda()
    V = plan.solve(r)
    torch.cuda.synchronize()
    return V.cpu().numpy(), plan


def _check(V, ref, what):
    err = oracle.rel_l2(V, ref)
    emax = float(np.max(np.abs(V.astype(np.float64) - ref)) / np.max(np.abs(ref)))
    print(f"{what}: relL2 {err:.3e} max elementwise {emax:.3e}", flush=True)
    assert err <= REL_L2, (what, err)
    assert emax <= ELEM, (what, emax)
    return err


SMALL_SHAPES = [(32, 24, 48), (12, 64, 16), (6, 8, 12)]


@pytest.mark.parametrize("bc", range(8))
@pytest.mark.parametrize("n", [(6, 8, 12), (16, 16, 16), (12, 48, 32)])
def test_kernel_build_matches_oracle(torch_dev, n, bc):
    plan = P.Plan(n, bc, H)
    kf = plan.kernel()
    ref = oracle.kernel_octant(n, bc, H)
    d = float(np.max(np.abs(kf - ref)) / np.max(np.abs(ref)))
    print(f"K^F {n} bc={bc}: {d:.2e}", flush=True)
    assert d <= KF_REL


@pytest.mark.parametrize("n,bc", [((256, 256, 256), 7), ((192, 192, 384), 3), ((384, 192, 384), 2)])
def test_kernel_build_matches_oracle_full_size(torch_dev, n, bc):
    """The float64 builder at the benchmark sizes: the 257-point DCT-I sums of
    the free 256^3 problem and the K0 of large kappa r on the 384-length
    wire and surface grids, against the oracle's FFT of the sampled kernel."""
    plan = P.Plan(n, bc, H)
    kf = plan.kernel()
    plan.close()
    ref = oracle.kernel_octant(n, bc, H)
    d = float(np.max(np.abs(kf - ref)) / np.max(np.abs(ref)))
    print(f"K^F {n} bc={bc}: {d:.2e}", flush=True)
    assert d <= KF_REL


@pytest.mark.parametrize("bc", range(8))
@pytest.mark.parametrize("n", SMALL_SHAPES)
def test_solve_parity_small(torch_dev, n, bc):
    rho = _density(n, bc, seed=100 + bc)
    V, _ = _gpu_solve(torch_dev, n, bc, rho)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"{n} bc={bc}")


@pytest.mark.parametrize("bc", range(8))
def test_solve_parity_noise(torch_dev, bc):
    """Unstructured density: every Fourier mode carries weight."""
    n = (24, 32, 16)
    rng = np.random.default_rng(bc)
    rho = rng.standard_normal((n[2], n[1], n[0]))
    if bc == 0:
        rho -= rho.mean()
    rho = rho.astype(np.float32)
    V, _ = _gpu_solve(torch_dev, n, bc, rho)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"noise {n} bc={bc}")


@pytest.mark.parametrize("name", ["free128", "wire128", "surface128", "periodic128"])
def test_solve_parity_128(torch_dev, name):
    n, bc, rho = workload_density(name)
    rho = rho.astype(np.float32)
    V, _ = _gpu_solve(torch_dev, n, bc, rho)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), name)


@pytest.mark.parametrize("n,bc", [((64, 96, 48), 7), ((64, 96, 48), 3), ((96, 64, 48), 2),
                                  ((48, 64, 96), 0), ((96, 48, 64), 5), ((48, 96, 64), 6),
                                  ((64, 48, 96), 1), ((96, 96, 48), 4)])
def test_solve_parity_mixed_radix(torch_dev, n, bc):
    rho = _density(n, bc, seed=7, count=8)
    V, _ = _gpu_solve(torch_dev, n, bc, rho)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"{n} bc={bc}")


@pytest.mark.parametrize("bc", [7, 3, 2, 5, 0])
def test_every_axis_order_matches_oracle(torch_dev, bc):
    """Forced forward axis orders (Section 3's axis-order study) change the
    passes' layouts and row counts, not V."""
    import itertools
    n = (24, 32, 48) if bc else (24, 32, 12)
    rho = _density(n, bc, seed=300 + bc)
    ref = oracle.solve(rho.astype(np.float64), bc, H)
    for order in itertools.permutations(range(3)):
        plan = P.Plan(n, bc, H, axis_order=order)
        assert tuple(plan.info["axis_order"]) == order
        V, _ = _gpu_solve(torch_dev, n, bc, rho, plan=plan)
        _check(V, ref, f"{n} bc={bc} order={order}")


@pytest.mark.parametrize("n,bc", [((32, 24, 16), 7), ((24, 16, 32), 3), ((32, 12, 24), 2)])
def test_full_padded_comparator_matches_oracle(torch_dev, n, bc):
    """The benchmark's "3D FFT library" comparator (a periodic plan over the
    whole padded grid with the problem's K^F set through poisson_kernel_set,
    pad and crop around it) gives the same V as the definition."""
    import bench
    torch = torch_dev
    rho = _density(n, bc, seed=350 + bc)
    fp = bench.FullPaddedSolve(P, n, bc, H)
    r = torch.from_numpy(rho).cuda()
    V = torch.empty_like(r)
    fp.solve(r, V)
    torch.cuda.synchronize()
    _check(V.cpu().numpy(), oracle.solve(rho.astype(np.float64), bc, H), f"full padded {n} bc={bc}")
    fp.close()


def test_host_buffer_solves(torch_dev):
    """Upload, solve and download through pinned host buffers: one at a time,
    in place, and the overlapped many-solve pipeline, all bitwise equal to
    device-resident solves."""
    torch = torch_dev
    n, bc = (64, 48, 32), 7
    plan = P.Plan(n, bc, H)
    rhos = [torch.from_numpy(_density(n, bc, seed=400 + i)).pin_memory() for i in range(5)]
    ref = [plan.solve(r.cuda()).cpu() for r in rhos]
    torch.cuda.synchronize()
    outs = [torch.empty_like(r).pin_memory() for r in rhos]
    plan.solve_host(rhos, outs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(outs, ref)):
        assert torch.equal(a, b), i
    x = rhos[1].clone().pin_memory()
    P.poisson_solve_host(plan.handle, x, x, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert torch.equal(x, ref[1])
    # a second pipelined call reuses the plan's buffers and streams
    outs2 = [torch.empty_like(r).pin_memory() for r in rhos[:3]]
    plan.solve_host(rhos[:3], outs2)
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(outs2[i], ref[i]), i


# extreme lengths: the longest compiled (1024, 768) and the shortest (4) FFT
# lines, on each kind of axis, and n = 2 on a free axis
EXTREME = [((512, 6, 8), 7), ((384, 8, 6), 7), ((2, 4, 2), 7), ((1024, 4, 6), 0),
           ((768, 4, 4), 6), ((4, 512, 4), 2), ((6, 4, 1024), 0), ((4, 6, 384), 3)]


@pytest.mark.parametrize("n,bc", EXTREME)
def test_extreme_lengths(torch_dev, n, bc):
    rho = _density(n, bc, seed=500 + bc, count=3)
    V, _ = _gpu_solve(torch_dev, n, bc, rho)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"{n} bc={bc}")


@pytest.mark.parametrize("prec", [P.POISSON_SPLIT_FP16, P.POISSON_SPLIT_BF16])
@pytest.mark.parametrize("n,bc", EXTREME)
def test_split_extreme_lengths(torch_dev, n, bc, prec):
    rho = _density(n, bc, seed=500 + bc, count=3)
    V, _ = _gpu_solve(torch_dev, n, bc, rho, precision=prec)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"split{prec} {n} bc={bc}")


@pytest.mark.parametrize("bc", [7, 3, 2, 0])
def test_zero_density_gives_zero(torch_dev, bc):
    n = (24, 32, 12)
    V, _ = _gpu_solve(torch_dev, n, bc, np.zeros((n[2], n[1], n[0]), np.float32))
    assert not np.any(V), bc  # exactly zero, no rounding residue


@pytest.mark.parametrize("bc", range(8))
def test_point_charge(torch_dev, bc):
    """A single grid charge: every Fourier mode carries the same weight."""
    n = (16, 24, 12)
    rho = np.zeros((n[2], n[1], n[0]), np.float32)
    rho[5, 7, 3] = 1.0 / H ** 3
    if bc == 0:
        rho -= rho.mean(dtype=np.float64)  # periodic: the k = 0 mode is projected out
    V, _ = _gpu_solve(torch_dev, n, bc, rho)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"point charge bc={bc}")


@pytest.mark.parametrize("n,bc", [((24, 32, 16), 7), ((24, 32, 16), 3), ((24, 16, 32), 4)])
def test_each_pass_against_numpy_fft(torch_dev, n, bc):
    """Pass by pass (Section 3's steps with the transposes folded into the
    layouts): each GPU pass output, read from a caller-owned workspace,
    against numpy's FFT of the GPU's previous intermediate, in float64.
    Order (x, y, z) is forced, so the layouts are
      A1[z][kx][y] (y fastest) after P1 and P4, A2[kx][ky][z] after P2, P3."""
    torch = torch_dev
    n1, n2, n3 = n
    plan = P.Plan(n, bc, H, axis_order=(0, 1, 2))
    S1, S2, S3 = plan.S
    Hx = S1 // 2 + 1
    ws_bytes = plan.info["workspace_bytes"]
    ws = torch.zeros(ws_bytes, dtype=torch.uint8, device="cuda")
    P.poisson_set_workspace(plan.handle, ws, ws_bytes)
    a1_bytes = (Hx * n2 * n3 * 8 + 255) // 256 * 256
    rho = _density(n, bc, seed=600 + bc)
    r = torch.from_numpy(rho).cuda()
    V = torch.empty_like(r)
    stream = torch.cuda.current_stream()
    kf = oracle.kernel_fourier(n, bc, H)  # (S3, S2, S1)

    def a1():
        b = ws[:Hx * n2 * n3 * 8].cpu().numpy().view(np.complex64)
        return b.reshape(n3, Hx, n2).astype(np.complex128)

    def a2():
        b = ws[a1_bytes:a1_bytes + Hx * S2 * n3 * 8].cpu().numpy().view(np.complex64)
        return b.reshape(Hx, S2, n3).astype(np.complex128)

    def rel(got, want):
        return float(np.linalg.norm(got - want) / np.linalg.norm(want))

    def run(k):
        P.poisson_solve_passes(plan.handle, r, V, k, k, stream)
        torch.cuda.synchronize()

    # P1: real-to-complex along x of the zero-padded density
    run(0)
    pad = np.zeros((n3, n2, S1))
    pad[:, :, :n1] = rho
    want = np.fft.rfft(pad, axis=2).transpose(0, 2, 1)          # [z][kx][y]
    e1 = rel(a1(), want)
    # P2: forward along y, zero-padded
    prev = a1()
    run(1)
    pad = np.zeros((n3, Hx, S2), complex)
    pad[:, :, :n2] = prev
    want = np.fft.fft(pad, axis=2).transpose(1, 2, 0)           # [kx][ky][z]
    e2 = rel(a2(), want)
    # P3: forward along z, times K^F / (S1 S2 S3), unnormalized inverse, crop
    prev = a2()
    run(2)
    pad = np.zeros((Hx, S2, S3), complex)
    pad[:, :, :n3] = prev
    kz = kf[:, :, :Hx].transpose(2, 1, 0) / (S1 * S2 * S3)     # [kx][ky][kz]
    want = (np.fft.ifft(kz * np.fft.fft(pad, axis=2), axis=2) * S3)[:, :, :n3]
    e3 = rel(a2(), want)
    # P4: unnormalized inverse along y, crop
    prev = a2()
    run(3)
    want = (np.fft.ifft(prev, axis=1) * S2)[:, :n2, :].transpose(2, 0, 1)  # [z][kx][y]
    e4 = rel(a1(), want)
    # P5: complex-to-real along x, unnormalized, crop
    prev = a1()
    run(4)
    want = (np.fft.irfft(prev.transpose(0, 2, 1), n=S1, axis=2) * S1)[:, :, :n1]
    e5 = rel(V.cpu().numpy().astype(np.float64), want)
    print(f"{n} bc={bc} per-pass relL2: {e1:.2e} {e2:.2e} {e3:.2e} {e4:.2e} {e5:.2e}", flush=True)
    for e in (e1, e2, e3, e4, e5):
        assert e <= 5e-7  # one float32 pass: a few units of 2^-24


def test_kernel_set_from_oracle_octant(torch_dev):
    """poisson_kernel_set with the oracle's octant gives the same solve."""
    n, bc = (32, 24, 48), 3
    rho = _density(n, bc, seed=3)
    V_build, _ = _gpu_solve(torch_dev, n, bc, rho)
    plan = P.Plan(n, bc, H, build_kernel=False)
    plan.set_kernel(oracle.kernel_octant(n, bc, H))
    V_set, _ = _gpu_solve(torch_dev, n, bc, rho, plan)
    assert oracle.rel_l2(V_set, V_build) < 1e-7
    _check(V_set, oracle.solve(rho.astype(np.float64), bc, H), "kernel_set")


def test_in_place_and_deterministic(torch_dev):
    torch = torch_dev
    n, bc = (48, 32, 64), 7
    rho = _density(n, bc, seed=5)
    plan = P.Plan(n, bc, H)
    r = torch.from_numpy(rho).cuda()
    V1 = plan.solve(r)
    V2 = plan.solve(r)
    x = r.clone()
    plan.solve(x, x)
    torch.cuda.synchronize()
    assert torch.equal(V1, V2)
    assert torch.equal(V1, x)


def test_solve_before_kernel_is_an_error(torch_dev):
    torch = torch_dev
    plan = P.Plan((16, 16, 16), 7, H, build_kernel=False)
    r = torch.zeros((16, 16, 16), device="cuda")
    with pytest.raises(P.PoissonError) as e:
        plan.solve(r)
    assert e.value.code == P._lib.POISSON_E_NO_KERNEL


def test_batch_equals_single_solves(torch_dev):
    torch = torch_dev
    cases = [((32, 32, 32), 7), ((48, 48, 48), 3), ((32, 32, 32), 7), ((64, 64, 64), 2),
             ((16, 16, 16), 0), ((48, 48, 48), 3)]
    rhos = [torch.from_numpy(_density(n, bc, seed=50 + i)).cuda() for i, (n, bc) in enumerate(cases)]
    Vs = [torch.empty_like(r) for r in rhos]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    for i, (n, bc) in enumerate(cases):
        single = P.Plan(n, bc, H).solve(rhos[i])
        torch.cuda.synchronize()
        assert torch.equal(single, Vs[i]), i


def test_gpu_residual_norm_matches_host(torch_dev):
    torch = torch_dev
    n, bc = (32, 32, 32), 7
    rho = _density(n, bc, seed=9)
    V, _ = _gpu_solve(torch, n, bc, rho)
    ref = oracle.solve(rho.astype(np.float64), bc, H)
    dev = P.poisson_rel_l2(torch.from_numpy(V).cuda(), torch.from_numpy(ref).cuda(), V.size)
    assert dev == pytest.approx(oracle.rel_l2(V, ref), rel=1e-9)


# ------------------------------------------------------------- full sizes
def _direct_free_samples(rho, h, points):
    """V at a few points by the direct sum of Eq. 2 with the sampled Coulomb
    kernel (free BCs), float64, no FFT."""
    n3, n2, n1 = rho.shape
    z = np.arange(n3)[:, None, None]
    y = np.arange(n2)[None, :, None]
    x = np.arange(n1)[None, None, :]
    out = []
    for (i1, i2, i3) in points:
        m2 = (x - i1) ** 2 + (y - i2) ** 2 + (z - i3) ** 2
        k = np.where(m2 > 0, -h * h / (4 * np.pi * np.sqrt(np.maximum(m2, 1))),
                     -(h * h / (4 * np.pi)) * 2.837297479480619)
        out.append(float(np.sum(k * rho)))
    return np.array(out)


def test_full_free256(torch_dev):
    """The 256^3 free-BC workload (padded 512^3) at full size, in the
    configuration the benchmark times."""
    torch = torch_dev
    n, bc, rho = workload_density("free256")
    rho32 = rho.astype(np.float32)
    V, plan = _gpu_solve(torch, n, bc, rho32)
    ref = oracle.solve(rho32.astype(np.float64), bc, H)
    err = _check(V, ref, "free256")
    dev = P.poisson_rel_l2(torch.from_numpy(V).cuda(), torch.from_numpy(ref).cuda(), V.size)
    assert dev == pytest.approx(err, rel=1e-6)
    rng = np.random.default_rng(0)
    pts = [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(6)] + [(0, 0, 0), (255, 255, 255)]
    direct = _direct_free_samples(rho32.astype(np.float64), H, pts)
    got = np.array([V[k, j, i] for (i, j, k) in pts], dtype=np.float64)
    assert np.max(np.abs(got - direct)) <= ELEM * np.max(np.abs(ref))


def test_max_size_periodic_1024_closed_form(torch_dev):
    """The largest grid (1024^3 periodic: the biggest intermediates, 537M
    complex elements each) against the closed form V = -rho/|k|^2 of a
    single cosine mode (Eq. 3 with the spectral wave numbers)."""
    torch = torch_dev
    n = (1024, 1024, 1024)
    f = (3, 5, 2)
    L = [v * H for v in n]
    ax = [torch.arange(v, device="cuda", dtype=torch.float64) * H for v in n]
    cx = torch.cos(2 * np.pi * f[0] * ax[0] / L[0])
    cy = torch.cos(2 * np.pi * f[1] * ax[1] / L[1])
    cz = torch.cos(2 * np.pi * f[2] * ax[2] / L[2])
    k2 = sum((2 * np.pi * f[j] / L[j]) ** 2 for j in range(3))
    rho = (cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).float()
    del ax
    plan = P.Plan(n, 0, H)
    V = plan.solve(rho)
    torch.cuda.synchronize()
    plan.close()
    # exact answer for the float32-rounded density: the mode's amplitude
    # scales by -1/|k|^2; rounding of rho adds other modes of relative size
    # ~1e-8, so compare against -rho/|k|^2 itself
    num = torch.linalg.vector_norm(V.double() + rho.double() / k2)
    den = torch.linalg.vector_norm(rho.double() / k2)
    err = float(num / den)
    print(f"periodic 1024^3 cosine mode: relL2 {err:.3e}", flush=True)
    assert err <= 1e-6


def test_max_size_free512_samples(torch_dev):
    """512^3 free (FFT grid 1024^3, the longest lines) at sampled points,
    each a float64 direct sum of Eq. 2 on the GPU (no FFT)."""
    torch = torch_dev
    n = (512, 512, 512)
    gs = draw_gaussians(n, H, 4, (2.0, 6.0), 77)
    ax = [torch.arange(v, device="cuda", dtype=torch.float64) * H for v in n]
    rho = torch.zeros((n[2], n[1], n[0]), device="cuda", dtype=torch.float64)
    for spec in gs:
        c, sig, q = spec.center, spec.sigma, spec.charge
        g = [torch.exp(-(ax[j] - c[j]) ** 2 / (2 * sig * sig)) for j in range(3)]
        rho += q * (2 * np.pi * sig * sig) ** -1.5 * (g[2][:, None, None] * g[1][None, :, None]
                                                       * g[0][None, None, :])
    rho = rho.float()
    plan = P.Plan(n, 7, H)
    V = plan.solve(rho)
    torch.cuda.synchronize()
    plan.close()
    z = torch.arange(n[2], device="cuda", dtype=torch.float64)[:, None, None]
    y = torch.arange(n[1], device="cuda", dtype=torch.float64)[None, :, None]
    x = torch.arange(n[0], device="cuda", dtype=torch.float64)[None, None, :]
    r64 = rho.double()
    pts = [(0, 0, 0), (511, 511, 511), (256, 100, 400), (17, 300, 255), (511, 0, 256)]
    got, want = [], []
    for (i1, i2, i3) in pts:
        m2 = (x - i1) ** 2 + (y - i2) ** 2 + (z - i3) ** 2
        k = torch.where(m2 > 0, -H * H / (4 * np.pi * torch.sqrt(torch.clamp(m2, min=1))),
                        torch.full_like(m2, -(H * H / (4 * np.pi)) * 2.837297479480619))
        want.append(float(torch.sum(k * r64)))
        got.append(float(V[i3, i2, i1]))
        del m2, k
    scale = float(torch.max(torch.abs(V)))
    d = np.max(np.abs(np.array(got) - np.array(want))) / scale
    print(f"free 512^3 direct-sum samples: max |dV| / max|V| = {d:.3e}", flush=True)
    assert d <= ELEM


@pytest.mark.parametrize("name", ["wire192x192x384", "surface384x192x384"])
def test_full_mixed_bc_large(torch_dev, name):
    n, bc, rho = workload_density(name)
    rho32 = rho.astype(np.float32)
    V, _ = _gpu_solve(torch_dev, n, bc, rho32)
    _check(V, oracle.solve(rho32.astype(np.float64), bc, H), name)


# ---------------------------------------------------------------- batches
def _batch_cases():
    from densities import BATCH_BCS, BATCH_EDGES
    cases = []
    i = 0
    for e in BATCH_EDGES[:3]:
        for bc in BATCH_BCS:
            for _ in range(3 if e == 32 else 1):
                cases.append(((e, e, e), bc, 900 + i))
                i += 1
    return cases


def test_batch_chunks_equal_single_solves(torch_dev, monkeypatch):
    """Chunked grouped launches (forced to 2 solves per launch) reproduce
    the single-solve results bit for bit."""
    torch = torch_dev
    from densities import batch_density
    monkeypatch.setenv("POISSON_BATCH_CHUNK_MB", "0.5")
    cases = _batch_cases()
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    Vs = [torch.full_like(r, float("nan")) for r in rhos]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    B.solve(rhos, Vs)
    torch.cuda.synchronize()
    for i, (n, bc, _) in enumerate(cases):
        single = P.Plan(n, bc, H).solve(rhos[i])
        torch.cuda.synchronize()
        assert torch.equal(single, Vs[i]), (i, n, bc)
    # and one entry of each class against the oracle
    seen = set()
    for i, (n, bc, _) in enumerate(cases):
        if bc in seen:
            continue
        seen.add(bc)
        _check(Vs[i].cpu().numpy(), oracle.solve(rhos[i].cpu().numpy().astype(np.float64), bc, H),
               f"batch {n} bc={bc}")


def test_batch_graph_replay(torch_dev):
    """A captured batch replays to the eager result, replay after replay,
    with eager work and synchronization in between."""
    torch = torch_dev
    from densities import batch_density
    cases = _batch_cases()
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    Vs = [torch.empty_like(r) for r in rhos]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
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
        # eager work between replays
        B.solve(rhos, Vs)
        torch.cuda.synchronize()


# ------------------------------------------------------- split precision
SPLITS = [pytest.param(P.POISSON_SPLIT_FP16, id="fp16x2"), pytest.param(P.POISSON_SPLIT_BF16, id="bf16x3")]


@pytest.mark.parametrize("prec", SPLITS)
@pytest.mark.parametrize("bc", range(8))
@pytest.mark.parametrize("n", SMALL_SHAPES)
def test_split_parity_small(torch_dev, n, bc, prec):
    """Radix-8 stages on the matrix cores with split operands keep the
    float32 bar against the float64 definition."""
    rho = _density(n, bc, seed=100 + bc)
    V, _ = _gpu_solve(torch_dev, n, bc, rho, precision=prec)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"split{prec} {n} bc={bc}")


@pytest.mark.parametrize("prec", SPLITS)
@pytest.mark.parametrize("name", ["free128", "wire128", "surface128", "periodic128"])
def test_split_parity_128(torch_dev, name, prec):
    n, bc, rho = workload_density(name)
    rho = rho.astype(np.float32)
    V, _ = _gpu_solve(torch_dev, n, bc, rho, precision=prec)
    _check(V, oracle.solve(rho.astype(np.float64), bc, H), f"split{prec} {name}")


@pytest.mark.parametrize("prec", SPLITS)
def test_split_full_free256(torch_dev, prec):
    n, bc, rho = workload_density("free256")
    rho32 = rho.astype(np.float32)
    V, _ = _gpu_solve(torch_dev, n, bc, rho32, precision=prec)
    _check(V, oracle.solve(rho32.astype(np.float64), bc, H), f"split{prec} free256")


@pytest.mark.parametrize("name", ["wire192x192x384", "surface384x192x384"])
def test_split_fp16_mixed_bc_large(torch_dev, name):
    n, bc, rho = workload_density(name)
    rho32 = rho.astype(np.float32)
    V, _ = _gpu_solve(torch_dev, n, bc, rho32, precision=P.POISSON_SPLIT_FP16)
    _check(V, oracle.solve(rho32.astype(np.float64), bc, H), f"split fp16 {name}")


def test_split_batch_equals_single_solves(torch_dev):
    torch = torch_dev
    from densities import batch_density
    cases = _batch_cases()
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    Vs = [torch.empty_like(r) for r in rhos]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases),
                precision=P.POISSON_SPLIT_FP16)
    B.solve(rhos, Vs)
    again = [torch.empty_like(r) for r in rhos]
    B.solve(rhos, again)
    torch.cuda.synchronize()
    for i, (n, bc, _) in enumerate(cases):
        # the same batch call twice: bit for bit
        assert torch.equal(Vs[i], again[i]), (i, n, bc)
        single = P.Plan(n, bc, H, precision=P.POISSON_SPLIT_FP16).solve(rhos[i])
        torch.cuda.synchronize()
        # a line's place in its wavefront differs between a batched and a
        # lone solve; the result must not depend on it
        assert torch.equal(single, Vs[i]), (i, n, bc)


def _all_edge_cases():
    """Every edge of the mixed batch (32 to 128) in every BC class, two of
    the smaller ones, so chunks hold several solves."""
    from densities import BATCH_BCS, BATCH_EDGES
    cases = []
    i = 0
    for e in BATCH_EDGES:
        for bc in BATCH_BCS:
            for _ in range(2 if e <= 64 else 1):
                cases.append(((e, e, e), bc, 1300 + i))
                i += 1
    return cases


@pytest.mark.parametrize("precision", [P.POISSON_FP32, P.POISSON_SPLIT_FP16])
def test_batch_all_edges_and_streams(torch_dev, precision):
    """Edges 32..128 in all four classes: the batch on one stream and spread
    over two and four concurrent streams gives the lone solves' results bit
    for bit, and edges 96 and 128 of every class meet the oracle bar."""
    torch = torch_dev
    from densities import batch_density
    cases = _all_edge_cases()
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    lone = []
    for n, bc, _ in cases:
        lone.append(P.Plan(n, bc, H, precision=precision).solve(rhos[len(lone)]))
    torch.cuda.synchronize()
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases), precision=precision)
    for streams in (1, 2, 4):
        B.streams = streams
        assert B.streams == streams
        Vs = [torch.full_like(r, float("nan")) for r in rhos]
        B.solve(rhos, Vs)
        torch.cuda.synchronize()
        for i, (n, bc, _) in enumerate(cases):
            assert torch.equal(lone[i], Vs[i]), (streams, i, n, bc)
    for i, (n, bc, _) in enumerate(cases):
        if n[0] >= 96:
            _check(Vs[i].cpu().numpy(), oracle.solve(rhos[i].cpu().numpy().astype(np.float64), bc, H),
                   f"batch {n} bc={bc} precision={precision}")
    with pytest.raises(P.PoissonError):
        B.streams = 5
    B.close()


def test_batch_streams_graph_replay(torch_dev):
    """A batch spread over three streams, captured on the caller's stream:
    every replay (with eager work in between) equals the eager result."""
    torch = torch_dev
    from densities import batch_density
    cases = _all_edge_cases()
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).cuda() for n, bc, seed in cases]
    Vs = [torch.empty_like(r) for r in rhos]
    B = P.Batch([c[0] for c in cases], [c[1] for c in cases], [H] * len(cases))
    B.streams = 3
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
        B.solve(rhos, Vs)
        torch.cuda.synchronize()
    B.close()
