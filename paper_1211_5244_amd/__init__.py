"""MI355X (gfx950) Poisson solver for free, wire, surface and periodic BCs.

The solver computes V = crop(IDFT(K^F * DFT(pad(rho)))) with customized
zero-skipping 3D FFTs (Dugan, Genovese, Goedecker, Sections 2-3) in the
hand-written HIP kernels of libpoisson.so.  This package is its thin Python
binding: the C entry points under their own names (`_lib`), plus `Plan` and
`Batch`, which take PyTorch device tensors and pass their addresses.
PyTorch is only used for device memory and streams.
"""

from __future__ import annotations

from ._lib import (  # noqa: F401
    EXPORTED,
    LIB_PATH,
    POISSON_BATCH_GROUPED,
    POISSON_BATCH_QUEUE,
    POISSON_FP32,
    POISSON_FREE_X,
    POISSON_FREE_Y,
    POISSON_FREE_Z,
    POISSON_SPLIT_BF16,
    POISSON_SPLIT_FP16,
    PLANE_BIT,
    TILE_SCHEDULES,
    PoissonError,
    load_library,
    poisson_batch_create,
    poisson_batch_destroy,
    poisson_batch_kernel_build,
    poisson_batch_kernel_build_isf,
    poisson_batch_get_mode,
    poisson_batch_get_queue_radix,
    poisson_batch_get_schedule,
    poisson_batch_get_streams,
    poisson_batch_queue_status,
    poisson_batch_set_mode,
    poisson_batch_set_queue_radix,
    poisson_batch_set_queue_shape,
    poisson_batch_set_queue_spin,
    poisson_queue_radices,
    poisson_queue_simulate,
    poisson_batch_set_schedule,
    poisson_batch_set_streams,
    poisson_set_tune_cache,
    poisson_batch_solve,
    poisson_batch_tune,
    poisson_kernel_build,
    poisson_kernel_build_isf,
    poisson_kernel_get,
    poisson_kernel_set,
    poisson_last_error,
    poisson_plan,
    poisson_plan_describe,
    poisson_plan_describe_ordered,
    poisson_plan_destroy,
    poisson_plan_get_schedule,
    poisson_plan_info,
    poisson_plan_ordered,
    poisson_plan_rows,
    poisson_plan_set_schedule,
    poisson_plan_tune,
    poisson_rel_l2,
    poisson_rel_l2_noalloc,
    poisson_set_workspace,
    poisson_solve,
    poisson_solve_host,
    poisson_solve_host_many,
    poisson_solve_passes,
)


def _check_grid(t, n, what):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous float32 tensor")
    if tuple(t.shape) != (n[2], n[1], n[0]):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {(n[2], n[1], n[0])}")


class Plan:
    """One grid size, boundary-condition mask and spacing.

    rho and V are float32 device tensors of shape (n3, n2, n1) (x fastest).
    kernel="isf" builds the interpolating-scaling-function Green's function
    of order isf_order instead of the default (grids with a free axis)."""

    def __init__(self, n, bc_mask, h, precision=POISSON_FP32, build_kernel=True, stream=None,
                 axis_order=None, kernel="default", isf_order=16):
        self.n = tuple(int(v) for v in n)
        self.bc_mask = int(bc_mask)
        self.h = float(h)
        self.handle = poisson_plan_ordered(*self.n, self.bc_mask, self.h, precision, axis_order)
        self.info = poisson_plan_info(self.handle)
        if build_kernel:
            # asynchronous: solves enqueued later on the same stream see K^F
            if stream is None:
                import torch
                stream = torch.cuda.current_stream()
            if kernel == "isf":
                poisson_kernel_build_isf(self.handle, isf_order, stream)  # blocking
            elif kernel == "default":
                poisson_kernel_build(self.handle, stream)
            else:
                raise ValueError(f"unknown kernel {kernel!r}")

    @property
    def S(self):
        return self.info["S"]

    def set_kernel(self, kf_octant):
        poisson_kernel_set(self.handle, kf_octant)

    def kernel(self):
        return poisson_kernel_get(self.handle, self.S)

    def solve(self, rho, V=None, stream=None):
        import torch
        _check_grid(rho, self.n, "rho")
        if V is None:
            V = torch.empty_like(rho)
        _check_grid(V, self.n, "V")
        if stream is None:
            stream = torch.cuda.current_stream(rho.device)
        poisson_solve(self.handle, rho, V, stream)
        return V

    def solve_host(self, rho_list, V_list, stream=None):
        """Solves on pinned host tensors of shape (n3, n2, n1): uploads,
        solves and downloads with the copies overlapping the solves."""
        import torch
        for i, (r, v) in enumerate(zip(rho_list, V_list)):
            for t, what in ((r, f"rho[{i}]"), (v, f"V[{i}]")):
                if t.device.type != "cpu" or t.dtype != torch.float32 or not t.is_contiguous():
                    raise TypeError(f"{what} must be a contiguous float32 host tensor")
                if tuple(t.shape) != (self.n[2], self.n[1], self.n[0]):
                    raise ValueError(f"{what} has shape {tuple(t.shape)}")
        if stream is None:
            stream = torch.cuda.current_stream()
        poisson_solve_host_many(self.handle, rho_list, V_list, stream)

    @property
    def schedule(self):
        """Per-pass tile schedules (tile_sel[5], complex lines per tile[5])."""
        return poisson_plan_get_schedule(self.handle)

    def set_schedule(self, tile_sel):
        poisson_plan_set_schedule(self.handle, tile_sel)

    def tune(self, rho, V=None, reps=0, stream=None):
        """Autotune the tile schedules on this device (V receives scratch
        values); returns the chosen schedule's ms per pass."""
        import torch
        _check_grid(rho, self.n, "rho")
        if V is None:
            V = torch.empty_like(rho)
        _check_grid(V, self.n, "V")
        if stream is None:
            stream = torch.cuda.current_stream(rho.device)
        return poisson_plan_tune(self.handle, rho, V, reps, stream)

    def close(self):
        if getattr(self, "handle", None):
            poisson_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent solves (sizes and BC masks may differ)."""

    def __init__(self, n_list, bc_list, h_list, precision=POISSON_FP32, stream=None,
                 kernel="default", isf_order=16):
        self.n_list = [tuple(int(v) for v in n) for n in n_list]
        self.handle = poisson_batch_create(self.n_list, list(bc_list), list(h_list), precision)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        if kernel == "isf":
            poisson_batch_kernel_build_isf(self.handle, isf_order, stream)  # blocking
        elif kernel == "default":
            poisson_batch_kernel_build(self.handle, stream)
        else:
            raise ValueError(f"unknown kernel {kernel!r}")

    def solve(self, rho_list, V_list, stream=None):
        import torch
        for i, (r, v) in enumerate(zip(rho_list, V_list)):
            _check_grid(r, self.n_list[i], f"rho[{i}]")
            _check_grid(v, self.n_list[i], f"V[{i}]")
        if stream is None:
            stream = torch.cuda.current_stream(rho_list[0].device)
        poisson_batch_solve(self.handle, rho_list, V_list, stream)

    def set_schedule(self, tile_sel):
        """The same five pass schedules for every distinct problem."""
        poisson_batch_set_schedule(self.handle, tile_sel)

    def schedule(self, index):
        """The five pass schedules solve `index` runs with."""
        return poisson_batch_get_schedule(self.handle, index)

    @property
    def streams(self):
        """Concurrent streams a batch solve uses (1..4)."""
        return poisson_batch_get_streams(self.handle)

    @streams.setter
    def streams(self, k):
        poisson_batch_set_streams(self.handle, k)

    @property
    def mode(self):
        """POISSON_BATCH_GROUPED (per-pass launches) or POISSON_BATCH_QUEUE
        (one persistent launch over a work queue, float32 only)."""
        return poisson_batch_get_mode(self.handle)

    @mode.setter
    def mode(self, m):
        poisson_batch_set_mode(self.handle, m)

    def set_queue_radix(self, length, radix_sel):
        poisson_batch_set_queue_radix(self.handle, length, radix_sel)

    def queue_radix(self, length):
        return poisson_batch_get_queue_radix(self.handle, length)

    def set_queue_shape(self, tile_elems=2048, item_kb=512):
        poisson_batch_set_queue_shape(self.handle, tile_elems, item_kb)

    def set_queue_spin(self, spin_limit):
        poisson_batch_set_queue_spin(self.handle, spin_limit)

    def queue_status(self):
        """Sticky queue flags since the last call (waits for the device)."""
        return poisson_batch_queue_status(self.handle)

    def tune(self, rho_list, V_list, reps=0, stream=None):
        """Autotune tile schedules and the per-launch budget (V receives
        scratch values); returns the chosen budget in MiB."""
        import torch
        for i, (r, v) in enumerate(zip(rho_list, V_list)):
            _check_grid(r, self.n_list[i], f"rho[{i}]")
            _check_grid(v, self.n_list[i], f"V[{i}]")
        if stream is None:
            stream = torch.cuda.current_stream(rho_list[0].device)
        return poisson_batch_tune(self.handle, rho_list, V_list, reps, stream)

    def close(self):
        if getattr(self, "handle", None):
            poisson_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
