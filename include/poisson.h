/*
 * poisson.h - C ABI of libpoisson, an MI355X (gfx950) Poisson solver for
 * free, wire, surface and periodic boundary conditions.
 *
 * Operation (Dugan, Genovese, Goedecker, "A Customized 3D GPU Poisson Solver
 * for Free Boundary Conditions"): the potential V of lap V = rho (Eq. 1) is
 * the discrete convolution of rho with a Green's function K (Section 2,
 * Eq. 2), evaluated in Fourier space as V^F = K^F rho^F (Eq. 3).  Axes with
 * free boundary conditions are zero padded to twice their length (Section 2),
 * so the FFT lengths are S_j = N_j B_j with B_j = 1 (periodic) or 2 (free)
 * (Section 3).  The forward transform skips the all-zero half of every padded
 * axis and the inverse transform crops each free axis back to N_j
 * (Section 3, the customized 3D FFT); the first forward axis is real-to-complex
 * and keeps S_p/2+1 coefficients (Section 3, last paragraphs).
 *
 * Conventions shared by every entry point
 *  - Arrays of grid values are contiguous float32 with x fastest:
 *    element (i1, i2, i3) is at index i1 + n1*(i2 + n2*i3).  In PyTorch this
 *    is a contiguous tensor of shape (n3, n2, n1).
 *  - bc_mask bit j (POISSON_FREE_X/Y/Z) set = free along axis j, clear =
 *    periodic along axis j.
 *  - K^F convention: K^F = DFT_S(K_pad) (unnormalized forward DFT of the real,
 *    even, padded kernel) and V = crop(IDFT_S(K^F * DFT_S(pad(rho)))) with
 *    the inverse DFT carrying 1/(S1 S2 S3).  K^F is real and even in every
 *    axis, so only the octant 0 <= k_j <= S_j/2 is passed, as float64 with k1
 *    fastest: (S1/2+1)*(S2/2+1)*(S3/2+1) values.
 *  - Device pointers are HIP device pointers of the device that was current
 *    when the plan was created.  Streams are hipStream_t passed as void*;
 *    NULL means the legacy default stream.
 *  - Every call returns POISSON_OK (0) or a negative status and has no side
 *    effects when it fails; poisson_last_error() gives a message for the
 *    calling thread's last failure.  C++ exceptions never cross this ABI.
 *  - Solves are asynchronous on the given stream; a device fault surfaces as
 *    POISSON_E_HIP at a later call.
 *  - A plan (or batch) may be used from one stream at a time: two solves of
 *    one plan in flight on different streams share its workspace and race.
 */
#ifndef POISSON_H
#define POISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct poisson_plan_s *poisson_plan_t;
typedef struct poisson_batch_s *poisson_batch_t;

enum {
  POISSON_OK = 0,
  POISSON_E_ARG = -1,         /* invalid argument (size, mask, spacing, pointer) */
  POISSON_E_UNSUPPORTED = -2, /* an FFT length S_j outside the compiled set */
  POISSON_E_NO_KERNEL = -3,   /* solve before poisson_kernel_set/_build */
  POISSON_E_NOMEM = -4,       /* device allocation failed */
  POISSON_E_HIP = -5,         /* a HIP runtime call failed */
  POISSON_E_STATE = -6        /* call not valid in the object's current state */
};

enum { POISSON_FREE_X = 1, POISSON_FREE_Y = 2, POISSON_FREE_Z = 4 };

/* Precision of the line transforms.  Data, twiddles, K^F and accumulation
 * are float32 in every mode.  The split modes take a line of length
 * L = 16 B (32..512) as two dense DFT factors (DFT_B and DFT_16, four-step
 * form) on the matrix cores, with each line scaled by a power of two and
 * split into 16-bit parts whose cross products carry float32 accuracy;
 * lengths 768, 1024 and below 32 run their radix-8 stages as 16x16 DFT
 * matrix products instead. */
enum {
  POISSON_FP32 = 0,       /* all stages on the vector ALUs in float32 */
  POISSON_SPLIT_FP16 = 1, /* DFT products on MFMA: fp16 hi + lo, 3 products */
  POISSON_SPLIT_BF16 = 2  /* DFT products on MFMA: bf16 three-way split, 6 products */
};

/* Create a plan for an n1 x n2 x n3 grid with spacing h (> 0, finite).
 * Each S_j = n_j * (1 + bit j of bc_mask) must be of the form 2^a 3^b with
 * 4 <= S_j <= 1024 (n_j >= 2); otherwise POISSON_E_UNSUPPORTED.  Chooses
 * the axis order (periodic axes first, free axes last in the forward
 * transform: Section 3), builds the twiddle tables and allocates the device
 * buffers of the plan (not the workspace; see poisson_set_workspace).  The
 * plan is owned by the caller and released with poisson_plan_destroy. */
int poisson_plan(poisson_plan_t *out, int n1, int n2, int n3, unsigned bc_mask, double h,
                 int precision);

/* Host-only description of the plan the same arguments would create; touches
 * no device.  Any output pointer may be NULL.
 *  axis_order: the forward axis order (p, q, r), 0 = x; p is the
 *              real-to-complex axis.
 *  S:          FFT lengths per physical axis (x, y, z).
 *  workspace_bytes: device workspace a solve needs.
 *  alg_bytes:  minimum HBM bytes one solve moves with five passes that each
 *              read and write their data once (density, two intermediates,
 *              potential, the K^F octant in float32). */
int poisson_plan_describe(int n1, int n2, int n3, unsigned bc_mask, int precision,
                          int axis_order[3], int S[3], size_t *workspace_bytes,
                          double *alg_bytes);

/* A plan with a caller-chosen forward axis order (p, q, r), a permutation of
 * 0, 1, 2 (NULL: the automatic order of poisson_plan).  For the axis-order
 * study of Section 3: every order gives the same V up to rounding, but the
 * number of 1D transforms, the bytes moved and so the time depend on it. */
int poisson_plan_ordered(poisson_plan_t *out, int n1, int n2, int n3, unsigned bc_mask, double h,
                         int precision, const int axis_order[3]);

/* Host-only description as poisson_plan_describe, for a forced order
 * (force_order NULL: automatic), plus the rows of the three forward steps
 * (as poisson_plan_rows).  Any output pointer may be NULL. */
int poisson_plan_describe_ordered(int n1, int n2, int n3, unsigned bc_mask, int precision,
                                  const int force_order[3], int axis_order[3], int S[3],
                                  size_t *workspace_bytes, double *alg_bytes, long long rows[3]);

/* The same description of an existing plan (its actual axis order). */
int poisson_plan_info(poisson_plan_t plan, int axis_order[3], int S[3], size_t *workspace_bytes,
                      double *alg_bytes);

/* Host-only: per forward step s = 0, 1, 2 of the customized 3D FFT in the
 * chosen order, the number of 1D transforms (rows) and their length, counted
 * as in Section 3 (complex rows: the second step has S_p * N_r rows).  The
 * inverse transform has the same counts in reverse order. */
int poisson_plan_rows(int n1, int n2, int n3, unsigned bc_mask, long long rows[3],
                      int lengths[3]);

/* Hand the plan a caller-owned device workspace of at least the described
 * size (256-byte aligned).  The plan stops using (and frees) any workspace it
 * allocated itself.  Passing NULL returns the plan to self-allocation. */
int poisson_set_workspace(poisson_plan_t plan, void *dev_ptr, size_t bytes);

/* Set K^F from its float64 octant (layout above), on the host
 * (is_device_ptr = 0) or the device (1).  The plan keeps the float64 octant
 * and a float32 copy permuted to its pass order with 1/(S1 S2 S3) folded in
 * (Section 3: the kernel is transposed once so the last forward transform
 * needs no transpose).  Synchronous. */
int poisson_kernel_set(poisson_plan_t plan, const double *kf_octant, int is_device_ptr);

/* Build the default Green's function of the plan's boundary conditions on
 * the device in float64 and set it as with poisson_kernel_set.  Asynchronous
 * on `stream`: enqueues the build and returns; the plan's workspace serves
 * as float64 scratch (the first call on a plan without a workspace
 * allocates it, as poisson_kernel_set does), so nothing else is allocated
 * and the host does not wait.  Solves enqueued after it on the same stream
 * see the new K^F.  Kernel family (the paper cites but does not define it): on
 * periodic axes the spectral wave numbers k_j = 2 pi f_j / (S_j h), on the
 * d free axes the sampled Green's function of (lap_d - kappa^2), kappa^2 =
 * sum of periodic k_j^2, times h^d:
 *   d=0: -1/kappa^2 (0 at k=0);  d=1: -exp(-kappa r)/(2 kappa), r/2 at kappa=0;
 *   d=2: -K0(kappa r)/(2 pi), ln(r)/(2 pi) at kappa=0;  d=3: -1/(4 pi r),
 * with O(h^4) origin weights, then the DFT along the free axes. */
int poisson_kernel_build(poisson_plan_t plan, void *stream);

/* Build, in float64 on the device, the Green's function of the BigDFT
 * solver the paper implements (Sections 2-3 take their kernels from it) and
 * set it as with poisson_kernel_set.  Along the free axes the grid values
 * of the density are read as coefficients of Deslauriers-Dubuc
 * interpolating scaling functions phi of even `order` (8..32; 16 is the
 * usual choice), and the Green's function is integrated against them:
 *   free:     K(i) = -(h^2 / 4 pi) int phi3(u) / |i - u| d^3u;
 *   surface:  h int phi(u) G_kappa(h (n - u)) du, G = -exp(-kappa|y|)/(2 kappa)
 *             (|y|/2 at kappa = 0);
 *   wire:     h^2 int phi2(u) G_kappa(h |n - u|) d^2u, G = -K0(kappa r)/(2 pi)
 *             (ln(r)/(2 pi) at kappa = 0);
 * with kappa^2 = sum of the periodic k_j^2, k_j = 2 pi f_j / (S_j h), as in
 * poisson_kernel_build.  Each is evaluated through a Gaussian integral
 * representation that separates into 1-D projections of Gaussians onto
 * phi and their DCTs (no 3-D transform).  POISSON_E_UNSUPPORTED for a fully
 * periodic plan; an order out of range is POISSON_E_ARG.  Blocking:
 * allocates a temporary device table of a few MB, enqueues the build on
 * `stream`, waits for it and frees the table.  Solves see the new K^F
 * afterwards. */
int poisson_kernel_build_isf(poisson_plan_t plan, int order, void *stream);

/* Copy the plan's float64 K^F octant to host memory (same layout as
 * poisson_kernel_set).  Synchronous. */
int poisson_kernel_get(poisson_plan_t plan, double *kf_octant_host);

/* V = K * rho for one density (device pointers, float32, layout above):
 * the discrete convolution of Eq. 2 evaluated as Eq. 3, V^F = K^F rho^F,
 * with the customized zero-padded 3D FFT of Section 3 (padding skipped in
 * the forward transform, crops after the inverse).
 * rho == V (in place) is allowed.  Enqueues five passes on `stream` and
 * returns without waiting; performs no allocation and no host sync, so it
 * can be captured into a HIP graph once the workspace exists (the plan
 * allocates its own workspace in poisson_kernel_set/_build). */
int poisson_solve(poisson_plan_t plan, const float *rho_dev, float *V_dev, void *stream);

/* Run only passes first..last (0..4) of poisson_solve, in order, on
 * `stream`: 0 real-to-complex along p, 1 forward along q, 2 forward along r
 * times K^F and inverse along r, 3 inverse along q, 4 complex-to-real along p
 * (the step list of Section 3 with the transposes folded into the passes).
 * Passes exchange data through the plan's workspace, so a later range sees
 * the intermediates an earlier one left; running 0..4 equals poisson_solve.
 * For per-pass timing and inspection.  Workspace layout (complex64, axis
 * order (p, q, r), H = S_p/2+1): A1 at offset 0, H*N_q*N_r elements, with
 * t1 fastest (t1 = q if p is x, else x), then p, then the third axis,
 * written by pass 0 and 3; A2 at the next multiple of 256 bytes,
 * H*S_q*N_r elements, r fastest, then q, then p, written by passes 1 and 2.
 * The conv pass multiplies by K^F/(S1 S2 S3); inverse transforms are
 * unnormalized.  With the plane kernel selected (schedule bit 3 of pass 2),
 * a range that covers passes 1..3 runs them as that one kernel, which
 * writes A1 only (A2 keeps stale values); any other range runs them as
 * separate passes, whose results agree with the plane kernel's to float32
 * rounding. */
int poisson_solve_passes(poisson_plan_t plan, const float *rho_dev, float *V_dev, int first,
                         int last, void *stream);

/* Solves on host buffers (Sections 1 and 4 count the transfers of the
 * density to the device and of the potential back).  poisson_solve_host
 * copies rho_host to a device grid of the plan, solves in place and copies
 * V back, all ordered on `stream`; poisson_solve_host_many does this for
 * `count` densities through two device grids and two copy streams of the
 * plan, so the upload of density i+1 and the download of potential i-1
 * overlap the solve of density i.  rho_host[i] == V_host[i] is allowed.
 * Host buffers should be pinned (hipHostMalloc) for the copies to run
 * asynchronously and overlap.  Asynchronous: the caller's stream completes
 * after the last copy to the host.  The first call allocates the two grids
 * and creates the copy streams (default priority); later calls allocate
 * nothing.  Not graph-capturable (it uses the plan's own streams). */
int poisson_solve_host(poisson_plan_t plan, const float *rho_host, float *V_host, void *stream);
int poisson_solve_host_many(poisson_plan_t plan, int count, const float *const *rho_host,
                            float *const *V_host, void *stream);

/* Release the plan and every device buffer it owns (not a caller workspace).
 * Waits for the device to finish work that may use them. */
int poisson_plan_destroy(poisson_plan_t plan);

/* Batches of independent solves of different sizes and boundary conditions
 * (Section 5 motivates many densities per run).  n holds 3*count sizes,
 * bc_mask and h one entry per solve.  Solves with equal (n, bc_mask, h)
 * share one plan and one K^F.  The batch owns one workspace: each plan's
 * solves run in chunks of up to 64 whose intermediates fit a budget (384 MiB
 * by default, or the environment variable POISSON_BATCH_CHUNK_MB read at
 * creation), and every pass of a chunk is one kernel launch. */
int poisson_batch_create(poisson_batch_t *out, int count, const int *n,
                         const unsigned *bc_mask, const double *h, int precision);
/* Builds the default K^F of every distinct plan (as poisson_kernel_build). */
int poisson_batch_kernel_build(poisson_batch_t batch, void *stream);
/* Builds the ISF K^F of every distinct plan (as poisson_kernel_build_isf;
 * blocking).  POISSON_E_UNSUPPORTED, before any build, if one of them is
 * fully periodic. */
int poisson_batch_kernel_build_isf(poisson_batch_t batch, int order, void *stream);
/* rho_ptrs / V_ptrs: host arrays of `count` device pointers, in creation
 * order; solve i may be in place (rho_ptrs[i] == V_ptrs[i]).  Asynchronous,
 * no allocation, no host sync: capturable into a HIP graph. */
int poisson_batch_solve(poisson_batch_t batch, const float *const *rho_ptrs,
                        float *const *V_ptrs, void *stream);
int poisson_batch_destroy(poisson_batch_t batch);

/* Schedules and the autotuner.
 *
 * The grouped launches fix the radix decomposition of each FFT length (the
 * persistent schedule below tunes it).  Each pass has a schedule 0..15 (0
 * is the default):
 *  - bits 0-1, tile width: passes 0, 1, 3 and 4 stage their lines through
 *    LDS in tiles of W consecutive lines, W about 16, 8, 4 or 32 complex
 *    lines for values 0..3.  Every mode compiles every width that fits the
 *    LDS of a compute unit and differs from a lower one; pass 2 (the fused
 *    convolution) has no tile and takes width 0 only.
 *  - bit 2, workgroup order: 1 gives each of the chip's 8 XCDs (each with
 *    its own L2) a contiguous run of tiles (or kernel rows) per round
 *    instead of every eighth one.
 *  - bit 3, pass 2 only: run passes 1-3 as one kernel that holds each k_p
 *    plane in LDS (the intermediate A2 never reaches HBM).  Compiled for
 *    every precision and small grids: L_q = L_r in {32, 48, 64} periodic,
 *    {64, 96, 128} free, and (L_q, L_r) = (32, 64), (48, 96), (64, 128)
 *    with only r free, where the q-lines are contiguous in A1.  The
 *    schedules of passes 1 and 3 are then unused.
 * Bits 0-2 change which lines a workgroup transforms together, where it
 * runs and how long its HBM row segments are, never a line's arithmetic:
 * results are bitwise identical under all of them.  Bit 3 computes the same
 * butterflies in one kernel, with the rounding of every operation fixed in
 * the source, so it is bitwise equal too, in every precision. */

/* Set the five passes' schedules.  POISSON_E_ARG if one is outside 0..15,
 * POISSON_E_UNSUPPORTED if its tile width is not compiled for its pass
 * (then nothing changes). */
int poisson_plan_set_schedule(poisson_plan_t plan, const int tile_sel[5]);

/* The same five schedules for every distinct problem of a batch: checked
 * against all of them first (POISSON_E_ARG / POISSON_E_UNSUPPORTED as
 * poisson_plan_set_schedule if one of them rejects it; then nothing
 * changes). */
int poisson_batch_set_schedule(poisson_batch_t batch, const int tile_sel[5]);

/* The five schedules that solve `index` (creation order) runs with: those
 * of its distinct problem.  POISSON_E_ARG if index is outside 0..count-1. */
int poisson_batch_get_schedule(poisson_batch_t batch, int index, int tile_sel[5]);

/* Current schedules and, per pass, the complex lines per tile they give
 * (0 for pass 2).  Either pointer may be NULL. */
int poisson_plan_get_schedule(poisson_plan_t plan, int tile_sel[5], int tile_lines[5]);

/* Autotuner: coordinate descent over the five passes, pass 2 first (its
 * bit 3 decides whether passes 1 and 3 run) and once more at the end.  For
 * each pass, every compiled schedule is timed as whole solves on this
 * device (at least reps solves and about 2 ms per round after a warm-up,
 * best of two rounds, hipEvents on `stream`), so a candidate is charged for
 * what it leaves in the caches for the next pass; it replaces the current
 * choice only if the solve gets at least 1% faster, and the final schedule
 * is kept only if it still beats the starting one when both are timed
 * again (alternately, best of two each).  Runs solves on
 * rho_dev and V_dev: V_dev (and the workspace) receive scratch values.
 * pass_ms (may be NULL) receives the chosen schedule's per-launch times:
 * one per pass, or, when it runs passes 1-3 as the plane kernel, that
 * launch's time in pass_ms[1] and 0 in pass_ms[2] and pass_ms[3].
 * reps <= 0 means 10.  Needs K^F and a workspace; synchronous. */
int poisson_plan_tune(poisson_plan_t plan, const float *rho_dev, float *V_dev, int reps,
                      double pass_ms[5], void *stream);

/* Tuned-schedule cache: a text file (path; NULL or "" switches it off)
 * where poisson_plan_tune records the schedule it chose, one line per
 * problem (n, bc_mask, precision, axis order) and device kind (arch name,
 * compute units), replaced through a temporary file and a rename.  Plans
 * created afterwards (poisson_plan, the plans of a batch) start from the
 * cached schedule, so a process need not tune again.  The file is
 * advisory: unreadable files, unknown lines and schedules the library does
 * not compile are ignored.  Without a call, the environment variable
 * POISSON_TUNE_CACHE gives the path.  Host only; returns POISSON_OK. */
int poisson_set_tune_cache(const char *path);

/* Autotuner for a batch: tunes each distinct plan's schedules on its
 * first chunk, then times whole batch solves for intermediates budgets of
 * 32..512 MiB and keeps the fastest (chunk_mb, may be NULL, receives it),
 * then the number of concurrent streams (1..4, poisson_batch_set_streams)
 * at that budget.  A float32 batch then times the persistent schedule
 * (radix choice per line length, then tiles of 1024 or 2048 elements with
 * items of 128, 512 or 2048 KiB) and
 * keeps it as the batch's mode only if it beats the grouped launches
 * (poisson_batch_get_mode tells which).  The arrays are those of
 * poisson_batch_solve; V receives
 * scratch values.  May reallocate the batch workspace (graphs captured
 * before then must be captured again).  reps <= 0 means 5.  Synchronous. */
int poisson_batch_tune(poisson_batch_t batch, const float *const *rho_ptrs, float *const *V_ptrs,
                       int reps, double *chunk_mb, void *stream);

/* Concurrent streams of a batch solve (1..4; 4 by default).  The batch's
 * chunks (up to 64 solves of one distinct problem per launch) are spread
 * over `streams` streams, largest first to the stream with the fewest
 * algorithmic bytes so far: the caller's stream and streams-1 of the
 * batch's own (default priority), forked from and joined back into the
 * caller's stream with events, so a graph captured on the caller's stream
 * holds them all.  Each stream has its own workspace region; a solve's
 * result does not depend on its stream.  Kernels of different chunks then
 * overlap, filling the ramp and tail of each launch (paper Section 5: many
 * densities per run).  Creates the streams and events, may grow the
 * workspace, and synchronizes the device: call it outside a capture.
 * POISSON_E_ARG for streams outside 1..4. */
int poisson_batch_set_streams(poisson_batch_t batch, int streams);
int poisson_batch_get_streams(poisson_batch_t batch, int *streams);

/* The persistent schedule of a batch (paper Section 5: many densities per
 * run; each item runs a piece of one pass of Section 3).  With
 * POISSON_BATCH_QUEUE, poisson_batch_solve is ONE kernel launch: a fixed
 * grid of workgroups (as many as fit the device at once) takes work items
 * from a device queue that holds every (solve, pass) segment in pass order
 * (all pass-0 segments, then all pass-1 segments, ...), and an item of
 * pass k > 0 waits until every item of pass k - 1 of its solve is
 * complete.  Completion is counted per (solve, pass) and per pass level;
 * each wait is bounded (poisson_batch_set_queue_spin) and a wait that runs
 * out sets a sticky flag (poisson_batch_queue_status) instead of hanging.
 * The line transforms are generic in length: a tile of complex lines in LDS
 * and one Stockham step per radix (2, 3, 4, 8) in the order the radix
 * choice gives; float32 arithmetic, with the rounding of every operation
 * fixed, so a solve's result depends only on its radix choices, not on the
 * batch it runs in or the tile shape.  At the default radix choices it is
 * bitwise the result of the grouped launches.  Float32 batches only.  Every solve
 * gets its own intermediates (the sum of the distinct plans' workspaces
 * over all solves, allocated at the first queue solve after a change).  The
 * first queue solve after creation, a schedule change or with new arrays
 * uploads descriptors (blocking, outside graph capture: a capture then
 * fails with POISSON_E_STATE); later ones with the same arrays are a single
 * asynchronous launch and capturable.  Calls that overlap on one batch
 * race on its counters. */
#define POISSON_BATCH_GROUPED 0 /* per-pass launches of chunks over streams (default) */
#define POISSON_BATCH_QUEUE 1   /* one persistent launch over a work queue */
/* POISSON_E_UNSUPPORTED for POISSON_BATCH_QUEUE on a split-precision batch. */
int poisson_batch_set_mode(poisson_batch_t batch, int mode);
int poisson_batch_get_mode(poisson_batch_t batch, int *mode);
/* Radix decomposition of a length-L queue transform for choice `radix_sel`:
 * 0 the stages of the grouped float32 kernels' compiled shape (radix 8
 * first; at the default choice a queue solve computes every butterfly as
 * the grouped launches do and gives their results bit for bit), 1 radix-4
 * stages (then 2, then 3), 2 the stages of choice 0 in reverse order.
 * Writes the radices,
 * first stage first, and returns their count; POISSON_E_UNSUPPORTED for a
 * length outside the library's set, POISSON_E_ARG for another choice.  Host
 * only. */
int poisson_queue_radices(int length, int radix_sel, int radices[12]);
/* Radix choice of every queue transform of length `length` in this batch
 * (0 by default; poisson_batch_tune picks them). */
int poisson_batch_set_queue_radix(poisson_batch_t batch, int length, int radix_sel);
int poisson_batch_get_queue_radix(poisson_batch_t batch, int length, int *radix_sel);
/* Tile of the queue transforms: tile_elems complex elements (power of two,
 * 64..2048; default 2048) hold the largest power of two of lines of length
 * L that fits (at least one); an item is as many tiles as carry about
 * item_kb KiB in and out (default 512). */
int poisson_batch_set_queue_shape(poisson_batch_t batch, int tile_elems, int item_kb);
/* Spin limit of every queue wait (default 2^20 polls, on the order of a
 * second; > 0). */
int poisson_batch_set_queue_spin(poisson_batch_t batch, unsigned spin_limit);
/* Waits for the device, then returns and clears the batch's sticky queue
 * flags: bit 0 = a wait ran out (the results of the solve it belonged to
 * are undefined). */
int poisson_batch_queue_status(poisson_batch_t batch, unsigned *flags);
/* Host simulation of the queue protocol (no GPU): `workers` threads play
 * workgroups over (solve, pass) segments of seg_items[pass * nsolve +
 * solve] items (each >= 1), with the device kernel's queue order, release
 * and wait rules, and check that no item passed its wait before every item
 * of its dependency had finished its work, that every item ran once and
 * that the counters end at zero.  fault plants a protocol mistake for tests
 * of these checks: 1 releases held lower-level items after a wait instead
 * of before it, 2 counts an item complete before its work.  stats (may be
 * NULL) receives waits, releases, violations and waits that ran out.
 * POISSON_E_STATE if a check fails. */
int poisson_queue_simulate(int nsolve, const int *seg_items, int workers, int fault,
                           unsigned seed, long long stats[4]);

/* Residual check in float64 on the device: *out = ||v - ref||_2 / ||ref||_2
 * over `count` values, v float32 and ref float64, both device pointers.
 * Synchronous (waits on `stream`). */
int poisson_rel_l2(const float *v_dev, const double *ref_dev, size_t count, double *out,
                   void *stream);

/* The residual of poisson_rel_l2 for callers that cannot allocate (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * enqueues the same float64 reduction on `stream` and writes
 * ||v - ref||_2 / ||ref||_2 to the device double *out_dev, without
 * allocating and without waiting on the host (capturable into a HIP graph).
 * Its per-block partial sums (at most 1024 pairs) live in a 16 KiB static
 * device array of the library that every device holds until the process
 * ends; the reduction never needs more, so every count is accepted.  All
 * calls on one device share that array: calls that overlap on one device
 * (concurrent streams or threads) race.  The result equals poisson_rel_l2's
 * to float64 rounding (same partial sums, summed in the same order).
 * POISSON_E_ARG for NULL pointers or count == 0. */
int poisson_rel_l2_noalloc(const float *v_dev, const double *ref_dev, size_t count,
                           double *out_dev, void *stream);

/* Message of the calling thread's last failed call ("" if none). */
const char *poisson_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* POISSON_H */
