"""Throughput of the Green's-function Poisson solve on one MI355X.

One step = one whole solve (all five passes) of the fully free 256^3 problem
(FFT grid 512^3) on a seeded 32-Gaussian density already resident in HBM.
Prints one JSON line with solves/s, the HBM roofline of the dominant pass and
of the whole solve, the accuracy against the FP64 oracle, and the FP64 CPU
oracle timed on this host's cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload free256]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "solves/s + % HBM roofline, 256^3 free BC; batched/split-prec vs plain FP32"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD spec
PASS_NAMES = ["p1_r2c", "p2_fwd", "p3_conv", "p4_inv", "p5_c2r"]
H = 0.3


PLANE_BIT = 8  # schedule bit of pass 2: passes 1-3 run as the small-grid plane kernel


def pass_bytes(n, info, plane=False):
    """Algorithmic HBM bytes of each launch (each array read and written
    once).  Five passes, or with the plane kernel three launches: pass 0,
    passes 1-3 (A1 read and rewritten, the K^F octant read; A2 stays in LDS)
    and pass 4."""
    S = info["S"]
    p, q, r = info["axis_order"]
    Hc = S[p] // 2 + 1
    grid = n[0] * n[1] * n[2]
    a1 = 8 * Hc * n[q] * n[r]
    a2 = 8 * Hc * S[q] * n[r]
    kf = 4 * Hc * (S[q] // 2 + 1) * (S[r] // 2 + 1)
    if plane:
        return [4 * grid + a1, 2 * a1 + kf, a1 + 4 * grid]
    return [4 * grid + a1, a1 + a2, 2 * a2 + kf, a2 + a1, a1 + 4 * grid]


def launches(tile_sel):
    """(name, first pass, last pass) of each launch a solve runs with the
    schedule tile_sel."""
    if tile_sel[2] & PLANE_BIT:
        return [("p1_r2c", 0, 0), ("p2_plane", 1, 3), ("p5_c2r", 4, 4)]
    return [(PASS_NAMES[k], k, k) for k in range(5)]


def solve_bytes(n, info, tile_sel):
    return float(sum(pass_bytes(n, info, plane=bool(tile_sel[2] & PLANE_BIT))))


TRAFFIC_SOURCES = ("paper_1211_5244_amd/csrc/passes.hip", "paper_1211_5244_amd/csrc/fft_core.h",
                   "paper_1211_5244_amd/csrc/fft_mfma.h")


def measured_traffic(kernel, mode="fp32"):
    """HBM bytes per launch of pass `kernel` in precision `mode` (that pass on
    its default tile schedule) from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since it was taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()[:16]
    path = os.path.join(root, "profiles", "pmc_traffic_free256.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) == 5 and parts[0] == "traffic" and parts[1] == kernel and parts[2] == mode:
            fields = dict(p.split("=", 1) for p in parts[3:])
            if fields.get("source_sha") == sha:
                return float(fields["bytes"])
    return None


def cpu_baseline(rho32, n, bc, reps=3, workers=None, warmup=True):
    """The FP64 oracle on this host, K^F prebuilt (as the GPU's is)."""
    import oracle
    rho64 = rho32.astype(np.float64)
    kf = oracle.kernel_fourier(n, bc, H)
    workers = workers or os.cpu_count() or 1
    if warmup:
        oracle.solve(rho64, bc, H, kf=kf, workers=workers)
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        V = oracle.solve(rho64, bc, H, kf=kf, workers=workers)
        t.append(time.perf_counter() - t0)
    med = float(np.median(t))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return V, {"value": 1.0 / med, "unit": "solves/s", "cores": workers, "kind": "oracle",
               "cpu_model": model,
               "sample": f"{reps} whole FP64 solves of the same workload"
                         f"{' after 1 warm-up' if warmup else ''} "
                         f"(scipy.fft, workers={workers}, K^F prebuilt); median {med:.3f} s"}


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=20):
    """Device-to-device copy rate (read + write bytes / time) of a plain copy."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def bench_batch(torch, P, dev, reps=5, precision=0):
    """512 mixed solves: a per-solve loop of poisson_solve, the grouped batch
    (poisson_batch_solve) and the same batch replayed from a HIP graph."""
    from densities import batch_density, batch_workload
    items = batch_workload(512)
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).to(dev)
            for n, bc, seed in items]
    Vs = [torch.empty_like(r) for r in rhos]
    alg = sum(P.poisson_plan_describe(*n, bc)["alg_bytes"] for n, bc, _ in items)
    stream = torch.cuda.current_stream(dev)
    plans = {}
    for n, bc, _ in items:
        if (n, bc) not in plans:
            plans[(n, bc)] = P.Plan(n, bc, H, precision=precision)
    B = P.Batch([it[0] for it in items], [it[1] for it in items], [H] * len(items),
                precision=precision)
    torch.cuda.synchronize()

    def loop():
        for (n, bc, _), r, v in zip(items, rhos, Vs):
            P.poisson_solve(plans[(n, bc)].handle, r, v, stream)

    def batched():
        P.poisson_batch_solve(B.handle, rhos, Vs, stream)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_loop = timed(loop)
    ref = [v.clone() for v in Vs]
    t_batch = timed(batched)
    descr = {key: P.poisson_plan_describe(*key[0], key[1]) for key in plans}

    def max_rel_diff():  # largest relative L2 difference from the per-solve loop
        return max(float((a.double() - b.double()).norm() / a.double().norm()) for a, b in zip(ref, Vs))

    same = all(torch.equal(a, b) for a, b in zip(ref, Vs))
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g):
            P.poisson_batch_solve(B.handle, rhos, Vs, torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    t_graph = timed(g.replay)
    same = same and all(torch.equal(a, b) for a, b in zip(ref, Vs))
    # the same grouped launches on one stream (the default spreads them over
    # four concurrent streams)
    default_streams = B.streams
    B.streams = 1
    t_one_stream = timed(batched)
    same = same and all(torch.equal(a, b) for a, b in zip(ref, Vs))
    B.streams = default_streams
    # float32: the persistent schedule, one launch over a pass-ordered device
    # queue (its own engine; at the default radix choices bitwise the loop)
    queue = {}
    if precision == 0:
        B.mode = P.POISSON_BATCH_QUEUE
        t_queue = timed(batched)
        queue_diff = max_rel_diff()
        g3 = torch.cuda.CUDAGraph()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(g3):
                P.poisson_batch_solve(B.handle, rhos, Vs, torch.cuda.current_stream(dev))
        torch.cuda.synchronize()
        t_queue_graph = timed(g3.replay)
        queue_diff = max(queue_diff, max_rel_diff())
        queue_flags = B.queue_status()
        B.mode = P.POISSON_BATCH_GROUPED
        queue = {"queue": t_queue, "queue_graph": t_queue_graph}
    # the autotuner: tile schedules per distinct plan, the per-launch budget,
    # the number of concurrent streams, then (float32) the queue's radix
    # choices and item size, keeping whichever schedule is faster
    chunk_mb = B.tune(rhos, Vs)
    t_tuned = timed(batched)
    # tuned schedules may use the small-grid plane kernel, equal to float32 rounding only
    tuned_diff = max_rel_diff()
    g2 = torch.cuda.CUDAGraph()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g2):
            P.poisson_batch_solve(B.handle, rhos, Vs, torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    t_tuned_graph = timed(g2.replay)
    tuned_diff = max(tuned_diff, max_rel_diff())
    # the tuned batch's bytes follow the schedules it runs (the plane kernel
    # keeps A2 in LDS)
    alg_tuned = sum(solve_bytes(n, descr[(n, bc)], B.schedule(i)) for i, (n, bc, _) in enumerate(items))
    out = {"solves": len(items), "alg_bytes": alg, "alg_bytes_tuned": alg_tuned,
           "tuned_identical_to_loop": tuned_diff == 0.0,
           "untuned_identical_to_loop": bool(same),
           "tuned_max_rel_l2_vs_loop": tuned_diff, "tuned_chunk_mb": chunk_mb,
           "default_streams": default_streams, "tuned_streams": B.streams,
           "tuned_mode": "queue" if B.mode == P.POISSON_BATCH_QUEUE else "grouped"}
    if queue:
        out["queue_max_rel_l2_vs_loop"] = queue_diff
        out["queue_identical_to_loop"] = queue_diff == 0.0
        out["queue_flags"] = queue_flags
    for name, t in (("loop", t_loop), ("batched", t_batch), ("batched_graph", t_graph),
                    ("batched_one_stream", t_one_stream),
                    ("batched_tuned", t_tuned), ("batched_tuned_graph", t_tuned_graph),
                    *queue.items()):
        # the queue runs the five-pass geometry (no plane kernel)
        a = alg_tuned if "tuned" in name and B.mode == P.POISSON_BATCH_GROUPED else alg
        out[name] = {"ms": t, "solves_per_s": len(items) / (t * 1e-3),
                     "alg_gbs": a / (t * 1e-3) / 1e9}
    return out


def queue_only(torch, P, dev, steps, warmup):
    """The 512-solve float32 batch as one persistent queue launch per solve of
    the batch: `warmup` untimed launches, then `steps` timed ones."""
    from densities import batch_density, batch_workload
    items = batch_workload(512)
    rhos = [torch.from_numpy(batch_density(n, bc, seed).astype(np.float32)).to(dev)
            for n, bc, seed in items]
    Vs = [torch.empty_like(r) for r in rhos]
    B = P.Batch([it[0] for it in items], [it[1] for it in items], [H] * len(items))
    B.mode = P.POISSON_BATCH_QUEUE
    stream = torch.cuda.current_stream(dev)
    for _ in range(max(warmup, 1)):  # the first launch uploads the descriptors
        P.poisson_batch_solve(B.handle, rhos, Vs, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        P.poisson_batch_solve(B.handle, rhos, Vs, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(steps, 1)
    alg = sum(P.poisson_plan_describe(*n, bc)["alg_bytes"] for n, bc, _ in items)
    return {"workload": "batch512 float32, persistent queue launch", "ms": ms,
            "solves_per_s": len(items) / (ms * 1e-3), "alg_gbs": alg / (ms * 1e-3) / 1e9,
            "flags": B.queue_status()}


def bench_host(torch, P, plan, r, count=20):
    """Transfer-inclusive rates (Sections 1 and 4 count the copies of rho to
    the device and of V back): one solve at a time through pinned host
    buffers (upload, solve, download, no overlap), and the pipeline that
    overlaps the copies of neighbouring solves with the current solve."""
    stream = torch.cuda.current_stream(r.device)
    rho_h = [r.cpu().pin_memory() for _ in range(2)]
    V_h = [torch.empty_like(rho_h[0]).pin_memory() for _ in range(2)]
    P.poisson_solve_host(plan.handle, rho_h[0], V_h[0], stream)  # first call allocates
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(count):
        P.poisson_solve_host(plan.handle, rho_h[i & 1], V_h[i & 1], stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_one = e0.elapsed_time(e1) / count
    rl = [rho_h[i & 1] for i in range(count)]
    vl = [V_h[i & 1] for i in range(count)]
    e0.record(stream)
    P.poisson_solve_host_many(plan.handle, rl, vl, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_pipe = e0.elapsed_time(e1) / count
    nbytes = 2 * r.numel() * 4
    return {"bytes_per_solve": nbytes,
            "one_at_a_time": {"ms": t_one, "solves_per_s": 1000.0 / t_one,
                              "pcie_gbs": nbytes / (t_one * 1e-3) / 1e9},
            "pipelined": {"ms": t_pipe, "solves_per_s": 1000.0 / t_pipe,
                          "pcie_gbs": nbytes / (t_pipe * 1e-3) / 1e9, "solves": count}}


# The other configurations, timed in the default run as extra keys (tuned
# FP32 and tuned split fp16): the four 128^3 BC classes and the 384-length
# wire and surface grids.  Timing does not depend on the density's values,
# so each solves a seeded normal field.
EXTRA_WORKLOADS = ["free128", "wire128", "surface128", "periodic128",
                   "wire192x192x384", "surface384x192x384"]


def window_median(torch, stream, fn, reps, windows=3):
    """Median over `windows` event-timed windows of the mean ms of one fn()
    in `reps` back-to-back calls on `stream`."""
    times = []
    for _ in range(windows):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / reps)
    return sorted(times)[len(times) // 2]


def bench_workloads(torch, P, dev, steps, warmup):
    from densities import WORKLOADS
    stream = torch.cuda.current_stream(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(13)
    out = {}
    for name in EXTRA_WORKLOADS:
        w = WORKLOADS[name]
        n, bc = w["n"], w["bc"]
        info = P.poisson_plan_describe(*n, bc)
        r = torch.randn((n[2], n[1], n[0]), generator=g, device=dev, dtype=torch.float32)
        V = torch.empty_like(r)
        rec = {"n": list(n), "bc_mask": bc}
        for prec, label in ((P.POISSON_FP32, "fp32"), (P.POISSON_SPLIT_FP16, "split_fp16")):
            plan = P.Plan(n, bc, H, precision=prec)
            plan.tune(r, V, stream=stream)
            sel = plan.schedule[0]
            for _ in range(warmup):
                plan.solve(r, V, stream)
            # median of three timed windows: the first solves after tuning
            # can run slow once, and one short window would keep that
            ms = window_median(torch, stream, lambda: P.poisson_solve(plan.handle, r, V, stream), steps)
            b = solve_bytes(n, info, sel)
            rec[label] = {"ms": ms, "solves_per_s": 1000.0 / ms, "alg_bytes": b,
                          "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "tile_schedule": list(sel)}
            plan.close()
        # the same problem as a batch of 16 independent densities (grouped
        # launches over the default concurrent streams): the throughput of
        # the kernels once a lone solve's launch ramps no longer dominate
        if max(n) <= 128:
            count = 16
            rs = [torch.randn((n[2], n[1], n[0]), generator=g, device=dev, dtype=torch.float32)
                  for _ in range(count)]
            vs = [torch.empty_like(x) for x in rs]
            B = P.Batch([n] * count, [bc] * count, [H] * count)
            for _ in range(warmup):
                B.solve(rs, vs, stream)
            reps = max(1, steps // 5)
            ms = window_median(torch, stream, lambda: P.poisson_batch_solve(B.handle, rs, vs, stream),
                               reps) / count
            b = solve_bytes(n, info, [0] * 5)
            rec["fp32_batch16"] = {"ms_per_solve": ms, "solves_per_s": 1000.0 / ms,
                                   "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            B.close()
            del rs, vs
        out[name] = rec
        del r, V
    return out


class FullPaddedSolve:
    """The "3D FFT library" comparator of Section 4 and 5: a problem with
    free axes solved as a periodic problem on the whole padded grid S1 x S2
    x S3, with no zero skipping and no crop inside the transforms.  The
    density is zero padded into an S-grid, the periodic plan of that grid
    gets the problem's own K^F octant (the octants have the same shape), and
    the potential is cropped back.  Same V as the customized solve; every
    1D transform runs over all S_p S_q (resp. S_p S_r, S_q S_r) rows."""

    def __init__(self, P, n, bc, h, precision=0):
        import torch
        own = P.Plan(n, bc, h, precision=precision)
        kf = own.kernel()
        own.close()
        self.n = tuple(n)
        self.S = tuple(int(v) * (2 if (bc >> j) & 1 else 1) for j, v in enumerate(n))
        self.plan = P.Plan(self.S, 0, h, precision=precision, build_kernel=False)
        self.plan.set_kernel(kf)
        self.pad = None
        self.torch = torch

    def solve(self, rho, V, stream=None):
        n, S = self.n, self.S
        if self.pad is None:
            self.pad = self.torch.zeros((S[2], S[1], S[0]), dtype=self.torch.float32, device=rho.device)
        self.pad.zero_()
        self.pad[:n[2], :n[1], :n[0]].copy_(rho)
        self.plan.solve(self.pad, self.pad, stream)
        V.copy_(self.pad[:n[2], :n[1], :n[0]])
        return V

    def solve_padded(self, stream=None):
        """The transforms alone, on the resident padded grid."""
        self.plan.solve(self.pad, self.pad, stream)

    def close(self):
        self.plan.close()


def fig1(torch, P, dev, steps, warmup):
    """Figure 1's experiment (Section 4): time of each BC class relative to the
    fully periodic solve of the same FFT size S^3, with Section 3's axis-order
    study (wire with its periodic axis last, surface with its free axis
    first) and the row-count prediction of each.  Timing does not depend on
    the density's values: each case solves a seeded normal field."""
    stream = torch.cuda.current_stream(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    out = []
    for S in (64, 128, 256, 512):
        N = S // 2
        cases = [("periodic", (S, S, S), 0, None),
                 ("free", (N, N, N), 7, None),
                 ("wire", (N, N, S), 3, None),                      # z periodic, first
                 ("wire_periodic_last", (N, N, S), 3, (0, 1, 2)),
                 ("surface", (S, N, S), 2, None),                   # y free, last
                 ("surface_free_first", (S, N, S), 2, (1, 0, 2))]
        base = None
        for name, n, bc, order in cases:
            plan = P.Plan(n, bc, H, axis_order=order)
            d = P.poisson_plan_describe_ordered(*n, bc, axis_order=plan.info["axis_order"])
            work = sum(rw * d["S"][a] for rw, a in zip(d["rows"], d["axis_order"]))
            r = torch.randn((n[2], n[1], n[0]), generator=g, device=dev, dtype=torch.float32)
            V = torch.empty_like(r)
            for _ in range(warmup):
                plan.solve(r, V, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                P.poisson_solve(plan.handle, r, V, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            if name == "periodic":
                base = (ms, work, d["alg_bytes"])
            out.append({"S": S, "case": name, "n": list(n), "bc_mask": bc,
                        "axis_order": list(d["axis_order"]), "ms": ms,
                        "time_vs_periodic": ms / base[0],
                        "fft_work_vs_periodic": work / base[1],
                        "alg_bytes_vs_periodic": d["alg_bytes"] / base[2]})
            plan.close()
            if order is None and bc != 0:
                # the same problem through the full-padded periodic solve
                fp = FullPaddedSolve(P, n, bc, H)
                for _ in range(warmup):
                    fp.solve(r, V, stream)
                e0.record(stream)
                for _ in range(steps):
                    fp.solve(r, V, stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms_fp = e0.elapsed_time(e1) / steps
                e0.record(stream)
                for _ in range(steps):
                    fp.solve_padded(stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms_fft = e0.elapsed_time(e1) / steps
                out.append({"S": S, "case": name + "_full_padded", "n": list(n), "bc_mask": bc,
                            "ms": ms_fp, "ms_transforms_only": ms_fft,
                            "time_vs_periodic": ms_fp / base[0],
                            "customized_vs_full_padded": ms / ms_fp})
                fp.close()
            del r, V
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="free256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-solve batch")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision modes")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default schedules (short runs under a profiler)")
    ap.add_argument("--no-host", action="store_true", help="skip the host-buffer transfer rates")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other configurations and the Figure 1 rows")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the 1 GiB copy (counter calibration)")
    ap.add_argument("--queue-only", action="store_true",
                    help="only run the 512-solve float32 batch as the persistent queue launch "
                         "(warmup + steps launches; short runs under a profiler)")
    ap.add_argument("--fig1", action="store_true",
                    help="only run the per-BC timing relative to periodic (Figure 1) and the "
                         "axis-order study")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1211_5244_amd as P
    from densities import WORKLOADS, workload_density

    dev = torch.device("cuda:0")
    if args.copy_only:
        print(json.dumps({"copy_gbs": copy_bandwidth(torch, dev)}), flush=True)
        return
    if args.queue_only:
        P.load_library()
        print(json.dumps(queue_only(torch, P, dev, args.steps, args.warmup)), flush=True)
        return
    if args.fig1:
        P.load_library()
        rows = fig1(torch, P, dev, steps=min(args.steps, 50), warmup=min(args.warmup, 5))
        print(json.dumps({"metric": "solve time relative to the fully periodic solve at equal "
                                    "FFT size S^3 (Figure 1)", "unit": "ratio",
                          "data": "synthetic", "rows": rows}), flush=True)
        return
    P.load_library()
    n, bc, rho = workload_density(args.workload, H)
    rho32 = rho.astype(np.float32)
    info = P.poisson_plan_describe(*n, bc)
    plan = P.Plan(n, bc, H)
    r = torch.from_numpy(rho32).to(dev)
    V = torch.empty_like(r)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        plan.solve(r, V, stream)
    torch.cuda.synchronize()

    # default tile schedules first, then the autotuner's choice (timed below)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        P.poisson_solve(plan.handle, r, V, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    untuned_ms = e0.elapsed_time(e1) / args.steps
    if not args.no_tune:
        plan.tune(r, V, stream=stream)
    tile_sel, tile_lines = plan.schedule
    for _ in range(args.warmup):
        plan.solve(r, V, stream)
    torch.cuda.synchronize()

    # timed region 1: back-to-back solves
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        P.poisson_solve(plan.handle, r, V, stream)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    # accuracy of exactly the path timed above (whole solves, tuned schedule)
    V_gpu = V.cpu().numpy()

    # timed region 2: the same solves with HIP events between the launches
    # the tuned schedule runs (passes 1-3 as one range with the plane kernel)
    runs = launches(tile_sel)
    nl = len(runs)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(nl + 1)] for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        for j, (_, first, last) in enumerate(runs):
            P.poisson_solve_passes(plan.handle, r, V, first, last, stream)
            ev[k][j + 1].record(stream)
    torch.cuda.synchronize()
    per_pass = [float(np.mean([ev[k][j].elapsed_time(ev[k][j + 1]) for k in range(args.steps)]))
                for j in range(nl)]
    step_ms = np.array([ev[k][0].elapsed_time(ev[k][nl]) for k in range(args.steps)])
    step_pct = {f"p{q}": float(np.percentile(step_ms, q)) for q in (10, 50, 90)}
    names = [name for name, _, _ in runs]

    copy_gbs = copy_bandwidth(torch, dev)
    pb = pass_bytes(n, info, plane=nl == 3)
    dom = int(np.argmax(per_pass))
    achieved = pb[dom] / (per_pass[dom] * 1e-3) / 1e9
    alg_solve = solve_bytes(n, info, tile_sel)
    solve_gbs = alg_solve / (ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": list(n), "bc_mask": bc, "S": list(info["S"]),
                   "axis_order": list(info["axis_order"]), "h": H,
                   "gaussians": WORKLOADS[args.workload]["gaussians"], "precision": "fp32",
                   "tile_schedule": list(tile_sel), "tile_lines": list(tile_lines)},
        "untuned_ms_per_step": untuned_ms,
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(names[dom])
                                 if args.workload == "free256" and tile_sel[runs[dom][1]] == 0
                                 and runs[dom][1] == runs[dom][2] else None),
                     "alg_bytes_per_launch": pb[dom],
                     "launch_ms": per_pass[dom]},
        "solve_roofline": {"alg_bytes": alg_solve, "achieved": solve_gbs,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": solve_gbs / HBM_PEAK_GBS},
        "copy_gbs": copy_gbs,
        "solve_vs_copy": solve_gbs / copy_gbs,
        "passes_ms": dict(zip(names, per_pass)),
        "step_ms_percentiles": step_pct,  # per solve, from the per-launch event loop
        "passes_gbs": {names[i]: pb[i] / (per_pass[i] * 1e-3) / 1e9 for i in range(nl)},
    }
    if not args.no_host:
        out["host_transfer"] = bench_host(torch, P, plan, r)
    # split-precision modes on the same workload: time and accuracy
    if not args.no_split:
        out["split"] = {}
        for prec, name in ((P.POISSON_SPLIT_FP16, "fp16x2"), (P.POISSON_SPLIT_BF16, "bf16x3")):
            sp = P.Plan(n, bc, H, precision=prec)
            Vs = torch.empty_like(r)
            if not args.no_tune:
                sp.tune(r, Vs, stream=stream)  # tuned, as the float32 plan
            for _ in range(3):
                sp.solve(r, Vs, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                P.poisson_solve(sp.handle, r, Vs, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / args.steps
            Vsplit = Vs.cpu().numpy()
            # per-launch times of the split solve, as for float32
            sruns = launches(sp.schedule[0])
            sev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(sruns) + 1)]
                   for _ in range(args.steps)]
            for k in range(args.steps):
                sev[k][0].record(stream)
                for j, (_, first, last) in enumerate(sruns):
                    P.poisson_solve_passes(sp.handle, r, Vs, first, last, stream)
                    sev[k][j + 1].record(stream)
            torch.cuda.synchronize()
            sms = [float(np.mean([sev[k][j].elapsed_time(sev[k][j + 1]) for k in range(args.steps)]))
                   for j in range(len(sruns))]
            spb = pass_bytes(n, info, plane=len(sruns) == 3)
            sdom = int(np.argmax(sms))
            sname = sruns[sdom][0]
            out["split"][name] = {"ms_per_solve": t, "solves_per_s": 1000.0 / t,
                                  "solve_roofline_frac": solve_bytes(n, info, sp.schedule[0]) / (t * 1e-3) / 1e9
                                  / HBM_PEAK_GBS,
                                  "passes_ms": {nm: v for (nm, _, _), v in zip(sruns, sms)},
                                  "passes_frac": {nm: b / (v * 1e-3) / 1e9 / HBM_PEAK_GBS
                                                  for (nm, _, _), b, v in zip(sruns, spb, sms)},
                                  "dominant": {"kernel": sname, "launch_ms": sms[sdom],
                                               "alg_bytes_per_launch": spb[sdom],
                                               "frac": spb[sdom] / (sms[sdom] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                               "traffic": (measured_traffic(sname, name)
                                                           if args.workload == "free256"
                                                           and sp.schedule[0][sruns[sdom][1]] == 0
                                                           and sruns[sdom][1] == sruns[sdom][2]
                                                           else None)},
                                  "tile_schedule": list(sp.schedule[0]), "V": Vsplit}
            sp.close()
    if not args.no_extra:
        out["workloads"] = bench_workloads(torch, P, dev, steps=min(args.steps, 50), warmup=10)
        out["fig1"] = fig1(torch, P, dev, steps=min(args.steps, 20), warmup=3)
    if not args.no_batch:
        out["batch"] = {"workload": "batch512 (edges 32..128, 4 BC classes, 4 Gaussians)",
                        "fp32": bench_batch(torch, P, dev),
                        "split_fp16x2": bench_batch(torch, P, dev, precision=P.POISSON_SPLIT_FP16)}
    if not args.no_cpu_baseline:
        V_ref, cb = cpu_baseline(rho32, n, bc)
        out["cpu_baseline"] = cb
        # one core, as the paper's single-core CPU comparison
        _, cb1 = cpu_baseline(rho32, n, bc, reps=1, workers=1, warmup=False)
        out["cpu_baseline_1core"] = cb1
        diff = V_gpu.astype(np.float64) - V_ref
        out["rel_l2_vs_oracle"] = float(np.linalg.norm(diff) / np.linalg.norm(V_ref))
        for name, rec in out.get("split", {}).items():
            d = rec["V"].astype(np.float64) - V_ref
            rec["rel_l2_vs_oracle"] = float(np.linalg.norm(d) / np.linalg.norm(V_ref))
    for rec in out.get("split", {}).values():
        rec.pop("V", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
