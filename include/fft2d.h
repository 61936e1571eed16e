/*
 * fft2d.h -- C ABI of the MI355X (gfx950) complex 2D FFT library.
 *
 * The operation is the 2D discrete Fourier transform of FP32 complex data,
 * computed as the paper computes it (Brown, Davies, Le Clair, "Exploring Fast
 * Fourier Transforms on the Tenstorrent Wormhole", arXiv 2506.15437): radix-2
 * Cooley-Tukey butterflies with precomputed twiddle factors on bit-reversal
 * reordered data (Section 2.2, Listing 1, Fig. 2), applied as one FFT along
 * every row followed by one FFT down every column (Section 5, Fig. 6).
 *
 * Definition (the paper does not write it out; this is the library's reading):
 *   forward  X[k][l] = sum_{m<M} sum_{n<N} x[m][n] exp(-2 pi i (k m/M + l n/N))
 *   inverse  x[m][n] = 1/(M N) sum_{k<M} sum_{l<N} X[k][l] exp(+2 pi i (k m/M + l n/N))
 * Results are in natural order, same shape as the input.
 *
 * Data layout: complex64 = { float re; float im; } interleaved, 8 bytes per
 * point. A uniform plan works on [batch][rows][cols] contiguous, cols fastest.
 * All data pointers are DEVICE pointers owned by the caller and must be 8-byte
 * aligned (16-byte alignment is recommended). Sizes must be powers of two in
 * [1, 16384] per dimension.
 *
 * Devices: a plan belongs to the HIP device that was current when it was
 * made; executing it requires that device to be current (and the stream and
 * data to be on it), else FFT2D_ERR_WRONG_DEVICE.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream). fft2d_exec, fft2d_exec_pass and fft2d_backward only enqueue work on
 * that stream; they never synchronise and never allocate, so they can be
 * captured in a HIP graph. fft2d_exec_batched enqueues the plan's own
 * instantiated graph; when the pointer set changed it first waits on the host
 * for the previous descriptor upload (from pinned memory) to finish, so it is
 * not meant to be captured.
 *
 * Errors: every function returns an fft2d_status and never throws. On failure
 * nothing is enqueued (except after a failed launch of a batch above 2^31
 * points, see fft2d_plan), outputs are untouched, and fft2d_last_error() gives
 * a thread-local detail string.
 *
 * Thread safety: a uniform plan is read-only during out-of-place execution and
 * may be used from several host threads and streams at once. In-place calls of
 * a split plan (large grids; see fft2d_plan) and every call of a batched plan
 * use mutable plan memory (work buffer; work counters and descriptor table):
 * such calls on one plan must not overlap (one stream at a time), and a batched
 * plan is used from one host thread at a time.
 */
#ifndef FFT2D_H
#define FFT2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sign of the exponent: FORWARD is unscaled, INVERSE is scaled by 1/(M N). */
#define FFT2D_FORWARD (-1)
#define FFT2D_INVERSE (+1)

/* Largest supported length along one dimension (2^14). */
#define FFT2D_MAX_LEN 16384

typedef enum fft2d_status {
  FFT2D_OK = 0,
  FFT2D_ERR_NULL_POINTER = 1,      /* a required pointer argument is NULL */
  FFT2D_ERR_INVALID_SIZE = 2,      /* a size is not a power of two in [1, 16384], or a count is < 1 */
  FFT2D_ERR_INVALID_DIRECTION = 3, /* direction is neither FFT2D_FORWARD nor FFT2D_INVERSE */
  FFT2D_ERR_MISALIGNED = 4,        /* a data pointer is not 8-byte aligned */
  FFT2D_ERR_WRONG_PLAN_KIND = 5,   /* uniform plan given to a batched call, or the reverse */
  FFT2D_ERR_OUT_OF_MEMORY = 6,     /* plan creation could not allocate host or device memory */
  FFT2D_ERR_HIP = 7,               /* a HIP runtime call failed; see fft2d_last_error() */
  FFT2D_ERR_INVALID_PLAN = 8,      /* the handle is not a live plan (e.g. already destroyed) */
  FFT2D_ERR_OVERLAP = 9,           /* input and output partially overlap (exact aliasing is allowed) */
  FFT2D_ERR_INCOMPLETE = 10,       /* an earlier fft2d_exec_batched on this plan gave up a bounded wait */
  FFT2D_ERR_WRONG_DEVICE = 11      /* the current HIP device is not the one the plan was made on */
} fft2d_status;

/* Opaque plan handle, owned by the library until fft2d_destroy(). */
typedef struct fft2d_plan_s* fft2d_plan_t;

/*
 * fft2d_plan -- create a plan for `batch` independent rows x cols transforms.
 *   out    : receives the handle (set to NULL on failure).
 *   batch  : number of grids, >= 1; grids are contiguous, rows*cols points apart;
 *            batch*rows*cols <= 2^35 points (256 GiB), else FFT2D_ERR_INVALID_SIZE.
 *   rows   : M, power of two in [1, 16384] (rows = 1 gives a batch of 1D FFTs).
 *   cols   : N, power of two in [1, 16384], the contiguous dimension.
 * Builds the FP32 twiddle tables (each entry computed in FP64 from its own
 * angle and rounded once; the paper precomputes its twiddles at start-up,
 * Section 4) in device memory on the current HIP device, and chooses the radix
 * schedule and tile shape for each pass. Grids of at least 2^22 points with
 * 1024 <= cols <= 8192, and grids of 16384 columns with at least 2048 rows,
 * use a split column transform (rows = M1 * M2: the row pass also applies the
 * first M1-point stage of the column FFT, the column pass the remaining
 * length-M2 stage). An out-of-place call keeps the intermediate in `out`; an
 * in-place call needs the plan-owned work buffer of batch*rows*cols complex64
 * points, allocated here. The environment variable FFT2D_SPLIT
 * (off | auto | M1) overrides the choice at plan time, FFT2D_SPLIT_COLUMN
 * (narrow | auto | wide) the column kernel's points per thread (32 | 64; auto
 * takes 64 where there is such a kernel). The split row pass runs the last
 * stage of its row FFT across its M1 rows, so that the M1-point combine needs
 * no LDS exchange of its own (FFT2D_COMBINE=xrow | classic; for 4096-point
 * rows and at most 1024 tiles with 64 points per thread, FFT2D_COMBINE_WIDE=
 * auto | on | off), and column
 * passes of 1024 and 2048 points use two radix stages (32 x 32, 64 x 32:
 * FFT2D_COLUMN_STAGES=two | classic), with nontemporal loads for grids of at
 * least 256 MiB (FFT2D_COLUMN_NT=auto | on | off). Grids of 32 x 32,
 * 32 x 64, 64 x 32, 64 x 64, 32 x 128, 128 x 32, 64 x 128, 128 x 64, 128 x 128,
 * 32 x 256, 256 x 32, 64 x 256 and 256 x 64 run both passes in one whole-grid
 * launch (one workgroup per grid, every point read and written once) when the
 * batch is large enough to fill the GPU (any batch for grids of up to 4096
 * points, at least 32 grids of 8192 points, 128 grids of 16384); FFT2D_GRID
 * (off | auto | on) overrides that choice. Plain passes that would run about
 * one tile per CU or fewer use narrower tiles (FFT2D_FEW_TILES
 * off | auto | on); for 1024-point rows that is one row per wave, whose
 * second exchange runs in registers across the wave's lanes
 * (FFT2D_ROW_SHUFFLE on | off). Batches of more than 2^31 points run
 * as several launches of whole grids (a HIP launch holds fewer than 2^32
 * work-items); if one of those launches fails, the earlier ones stay enqueued.
 * Must be called with a GPU present.
 */
fft2d_status fft2d_plan(fft2d_plan_t* out, int64_t batch, int64_t rows, int64_t cols);

/*
 * fft2d_plan_batched -- plan `count` independent transforms of different shapes
 * (rows[i] x cols[i], powers of two in [1, 16384]), executed by
 * fft2d_exec_batched in one persistent kernel launch replayed from a HIP graph.
 * rows and cols are host arrays of `count` entries (1 <= count <= 2^24), read
 * during the call only. The persistent grid size, the item order, the
 * work-group granularity and, for every row and column length of 32 points or
 * more, one of two radix schedules / tile shapes come from the library's
 * autotuner (FFT2D_BATCH_VARIANT=0|1 fixes the latter), cached per shape set in
 * a text file
 * (FFT2D_TUNE=off|cached|full, FFT2D_TUNE_CACHE=<path>, default
 * $HOME/.cache/fft2d_tune.txt). Tuning runs the kernel on two temporary device
 * buffers of the plan's total size, freed before the call returns; if they
 * cannot be allocated the call fails with FFT2D_ERR_OUT_OF_MEMORY (FFT2D_TUNE=off
 * avoids them). The plan also launches a small probe kernel once to learn
 * which XCD each workgroup runs on. Tall grids (rows >= 1024, 512 <= cols <=
 * 8192) are split as in fft2d_plan: their row pass combines M1 rows into a
 * plan-owned work buffer of rows*cols complex64 each, and their column pass
 * runs columns of rows/M1 points (FFT2D_BATCH_SPLIT=off disables this).
 * Grids of 64x64, 64x128, 128x64, 128x128, 64x256 and 256x64 are transformed
 * whole by one workgroup, with one read and one write of their data
 * (FFT2D_BATCH_GRID=off disables this). FFT2D_BATCH_GUIDED=1 groups the work
 * in large units first and small ones at the end of each queue (fewer tile
 * calls: less memory traffic, the same time on the 512-shape set).
 * In the persistent kernel every transform runs on one XCD; a grid of at
 * least 2^22 points that holds at least 1/16 of the plan's points (1/(2 nq),
 * nq the number of XCD queues) runs instead as a plain transform: the row and
 * column kernels of a uniform plan the batched plan owns, launched on the same
 * stream after the persistent kernel (FFT2D_BATCH_PLAIN=off disables this).
 * Plain transforms of one shape whose inputs, and outputs, follow each other
 * in memory in index order (slices of one tensor) run as one uniform batch:
 * two launches for all of them, as fft2d_plan with a batch count would. These
 * owned uniform plans hold device memory like any uniform plan (a split shape's
 * work buffer: one grid for the single-grid plan, all grids of the shape for
 * the batch plan).
 */
fft2d_status fft2d_plan_batched(fft2d_plan_t* out, int64_t count, const int64_t* rows, const int64_t* cols);

/*
 * fft2d_exec -- transform every grid of a uniform plan.
 *   in, out   : device pointers to batch*rows*cols complex64; in == out (in
 *               place) is allowed, partial overlap is rejected.
 *   direction : FFT2D_FORWARD or FFT2D_INVERSE (definition above).
 *   stream    : hipStream_t as void*.
 * Work: one row pass and one column pass (Section 5), each reading and writing
 * every point once.
 */
fft2d_status fft2d_exec(fft2d_plan_t plan, const void* in, void* out, int direction, void* stream);

/*
 * fft2d_exec_batched -- transform every grid of a batched plan.
 *   in, out : HOST arrays of `count` device pointers (grid i has the shape given
 *             at plan time); in[i] == out[i] is allowed. The arrays are read
 *             during the call only. When the pointer set differs from the
 *             previous call's, the device descriptor table is refreshed by a
 *             stream-ordered copy before the launch.
 *   direction, stream : as for fft2d_exec.
 * The persistent kernel's waits (a column tile waits for its grid's row
 * tiles) always end by construction; each is still bounded (about a second
 * of polling) so the launch drains even if that were broken. A wait that gives
 * up skips its tile and sets a flag in pinned host memory; the next call on
 * the plan then returns FFT2D_ERR_INCOMPLETE without launching (and clears the
 * flag), since the outputs of the earlier call are incomplete. The last
 * workgroup of every launch also checks that each XCD's queue was drained (a
 * queue whose XCD received no workgroup, e.g. under a CU mask on the stream,
 * leaves its transforms uncomputed) and sets the same flag if not. The
 * environment variables FFT2D_BATCH_SPIN_LIMIT (-1 gives up every wait) and
 * FFT2D_BATCH_DRAIN_SLACK (raises the pops the drain check expects) force both
 * reports from the host, for tests.
 */
fft2d_status fft2d_exec_batched(fft2d_plan_t plan, const void* const* in, void* const* out, int direction,
                                void* stream);

/*
 * fft2d_backward -- vector-Jacobian product (adjoint) of fft2d_exec, for
 * reverse-mode differentiation. With the convention grad = dL/dRe + i dL/dIm:
 *   forward_direction == FFT2D_FORWARD : grad_in = F^H grad_out, the unscaled
 *                                        opposite-sign transform;
 *   forward_direction == FFT2D_INVERSE : grad_in = (1/(M N)) F grad_out.
 * grad_out, grad_in : device pointers shaped like the plan's data; may alias.
 * This is not the inverse transform (that is fft2d_exec with FFT2D_INVERSE).
 */
fft2d_status fft2d_backward(fft2d_plan_t plan, const void* grad_out, void* grad_in, int forward_direction,
                            void* stream);

/*
 * fft2d_exec_pass -- enqueue only one of the two passes of fft2d_exec, for
 * profiling and per-pass timing. Pass 0 is the row pass (length-cols FFT along
 * every row; for split plans also the first, M1-point stage of the column
 * transform), pass 1 the column pass. Pass 0 reads `in` and writes the
 * intermediate result; pass 1 reads the intermediate and writes `out`. The
 * intermediate is `out`, except for in-place calls (in == out) of split
 * plans, where it is the plan's work buffer,
 * so pass 0 then pass 1 with the same arguments is exactly fft2d_exec (for a
 * plan that runs the whole-grid kernel: the same transform in two launches,
 * equal to it up to rounding). The
 * inverse's 1/(M N) scale is applied by the last pass. Returns
 * FFT2D_ERR_INVALID_SIZE if the plan has no such pass (that dimension has
 * length 1) and FFT2D_ERR_INVALID_DIRECTION for a pass index other than 0 or 1.
 * Uniform plans only.
 */
fft2d_status fft2d_exec_pass(fft2d_plan_t plan, const void* in, void* out, int direction, int pass, void* stream);

/*
 * fft2d_exec_pass_timed -- fft2d_exec_pass with timing: the same pass, same
 * arguments and results, launched with start_event and stop_event bound to the
 * pass's kernel launch (hipExtLaunchKernel), so that the elapsed time between
 * the two events (hipEventElapsedTime) is the kernel's own execution time,
 * without the marker packets that recording events between launches adds.
 * start_event and stop_event are hipEvent_t handles created by the caller
 * (with timing enabled) and still owned by it; both must be non-null
 * (FFT2D_ERR_NULL_POINTER). The pass must be a single launch: a plan whose
 * batch holds more than 2^31 points returns FFT2D_ERR_INVALID_SIZE. Other
 * errors as fft2d_exec_pass. Like it, this only enqueues work on `stream`;
 * it is a timing aid and not meant to be captured in a HIP graph.
 */
fft2d_status fft2d_exec_pass_timed(fft2d_plan_t plan, const void* in, void* out, int direction, int pass,
                                   void* start_event, void* stop_event, void* stream);

/* Ablations of fft2d_exec_pass_ablated. */
#define FFT2D_ABLATE_ARITHMETIC 1 /* loads, LDS exchanges and stores; no twiddles, no butterflies */
#define FFT2D_ABLATE_EXCHANGE 2   /* loads and stores only: a copy with the pass's access pattern */

/*
 * fft2d_exec_pass_ablated -- a measurement aid: one pass of a uniform plan
 * with part of its work switched off, the way the paper's Table 2 times its
 * FFT with single components (compute, reorderings, transfers) disabled
 * (Section 4). The pass keeps its kernel's workgroups, tiles, load and store
 * instructions, addresses and cache policies; with FFT2D_ABLATE_ARITHMETIC it
 * also keeps the LDS exchanges (the on-chip reorderings) but drops the
 * twiddle loads, multiplications and butterflies; with FFT2D_ABLATE_EXCHANGE
 * it drops the exchanges too and each thread stores the points it loaded.
 * Its duration is therefore the data-movement floor of that pass. The output
 * is a reordered copy of the input, not a transform.
 *   pass        : 0 (row pass) or 1 (column pass), as for fft2d_exec_pass;
 *                 in, out and the intermediate buffer as there.
 *   ablation    : FFT2D_ABLATE_ARITHMETIC or FFT2D_ABLATE_EXCHANGE
 *                 (else FFT2D_ERR_INVALID_DIRECTION).
 *   start_event, stop_event : both null, or hipEvent_t handles bound to the
 *                 launch as in fft2d_exec_pass_timed.
 * Only the pass kernels of the benchmarked grids carry these variants
 * (4096 x 4096, 8192 x 8192, 16384 x 2048, 8 x 2048 x 2048, 1024 x 1024,
 * batches of 16384-point rows): another pass returns FFT2D_ERR_INVALID_SIZE.
 */
fft2d_status fft2d_exec_pass_ablated(fft2d_plan_t plan, const void* in, void* out, int pass, int ablation,
                                     void* start_event, void* stop_event, void* stream);

/* Methods of fft2d_probe_dft16. */
#define FFT2D_DFT16_BUTTERFLY 0 /* radix-2 butterflies on the vector ALU (the library's radix-16 stage) */
#define FFT2D_DFT16_MFMA 1      /* dense DFT matrix on the matrix cores (v_mfma_f32_16x16x4_f32) */

/*
 * fft2d_probe_dft16 -- a measurement aid for the choice between the vector
 * ALU and the matrix cores for a radix-16 stage (the paper runs its FFT
 * arithmetic on either the vector unit or the matrix engine of a Tensix core,
 * Section 4). Applies x <- Pi F x `reps` times to each of `count` 16-point
 * complex64 vectors held in registers, where F is the unscaled forward
 * 16-point DFT and Pi moves point 4q + r to point q + 4r, scaling by 2^-16
 * (exactly) after every 8 applications: out = (Pi F / 4)^reps in. The work is
 * arithmetic only (one load and one store of each vector), so
 * count * reps / elapsed time is the method's DFT16 rate.
 *   method : FFT2D_DFT16_BUTTERFLY or FFT2D_DFT16_MFMA (else
 *            FFT2D_ERR_INVALID_DIRECTION);
 *   in, out : device pointers to count * 16 complex64, 8-byte aligned,
 *            vector v at points 16 v ... 16 v + 15; may alias exactly;
 *   count  : multiple of 64 in [64, 2^26]; reps : multiple of 8 in [8, 4096]
 *            (else FFT2D_ERR_INVALID_SIZE);
 *   start_event, stop_event : both null, or hipEvent_t handles bound to the
 *            kernel launch as in fft2d_exec_pass_timed.
 * Only enqueues work on `stream`; no plan is needed.
 */
fft2d_status fft2d_probe_dft16(int method, const void* in, void* out, int64_t count, int reps, void* start_event,
                               void* stop_event, void* stream);

/*
 * fft2d_probe_tile_copy -- a measurement aid for the column pass's access
 * pattern (the paper's 2D FFT reads its columns after a global transpose,
 * Section 5, Fig. 6): copies a rows x cols complex64 grid from `in` to `out`
 * in column tiles of `tile_cols` columns (row segments of 8 * tile_cols bytes)
 * by 512-thread workgroups, lanes over columns first. Tile (k1, hb, cb) holds
 * rows k1 + residues * (hb * H + m), m < H, H = 2048, 1024, 512 for 16, 32,
 * 64 columns (so a tile is 256 KiB in every case), the row set of a split
 * column pass with M1 = residues. out equals in afterwards.
 *   tile_cols   : 16, 32 or 64 (else FFT2D_ERR_INVALID_SIZE);
 *   rows, cols  : rows a multiple of residues * H, cols of tile_cols,
 *                 rows * cols <= 2^28 (else FFT2D_ERR_INVALID_SIZE);
 *   nontemporal : nonzero loads the input with the nontemporal hint;
 *   in, out     : device pointers, 8-byte aligned, not overlapping
 *                 (FFT2D_ERR_MISALIGNED, FFT2D_ERR_OVERLAP);
 *   start_event, stop_event : both null, or hipEvent_t handles bound to the
 *                 launch as in fft2d_exec_pass_timed.
 * Only enqueues work on `stream`.
 */
fft2d_status fft2d_probe_tile_copy(const void* in, void* out, int64_t rows, int64_t cols, int tile_cols, int residues,
                                   int nontemporal, void* start_event, void* stop_event, void* stream);

/*
 * fft2d_probe_lds -- a measurement aid for the LDS exchanges of the pass
 * kernels (the on-chip counterpart of the paper's reorderings, Section 4):
 * one 1024-thread workgroup per compute unit, each thread reading (write = 0)
 * or writing (write != 0) 4096 times `width_bytes` (4, 8 or 16) at
 * lane-consecutive addresses of a 128 KiB LDS array. *bytes receives the
 * bytes moved by the launch (divide by its duration for the bandwidth).
 *   sink        : device buffer of sink_floats floats, at least 1024 per
 *                 compute unit (else FFT2D_ERR_INVALID_SIZE), overwritten;
 *   width_bytes : 4, 8 or 16 (else FFT2D_ERR_INVALID_SIZE);
 *   start_event, stop_event : as for fft2d_probe_tile_copy.
 * Enqueues on `stream` after querying the current device.
 */
fft2d_status fft2d_probe_lds(int width_bytes, int write, void* sink, int64_t sink_floats, int64_t* bytes,
                             void* start_event, void* stop_event, void* stream);

/* fft2d_destroy -- free a plan and its device memory. NULL is a no-op. Waits for
 * no stream: the caller must make sure no enqueued work still uses the plan. */
fft2d_status fft2d_destroy(fft2d_plan_t plan);

/* Static English text for a status code. */
const char* fft2d_status_string(fft2d_status status);

/* Thread-local detail of the last failure on this host thread ("" if none). */
const char* fft2d_last_error(void);

/*
 * fft2d_plan_describe -- write a one-line, NUL-terminated description of the
 * plan's chosen kernels (radix schedules, tile shapes, grid sizes) into buf
 * (at most buflen bytes, truncated if needed).
 */
fft2d_status fft2d_plan_describe(fft2d_plan_t plan, char* buf, int64_t buflen);

/*
 * fft2d_plan_twiddles -- copy one of a uniform plan's FP32 twiddle tables to
 * host memory, for inspection and tests (synchronous: it waits for the copy).
 *   which    : 0 = the row pass's table, 1 = the column pass's table, 2 = the
 *              combine table of a split plan, W_rows^j = exp(-2 pi i j / rows)
 *              for j < rows.
 *   host_out : complex64 host buffer of `capacity` entries (may be NULL when
 *              capacity is 0); min(capacity, *count) entries are written.
 *   count    : receives the table's size (0 if the plan has no such table).
 * Pass tables cover passes p >= 1 of the pass's radix schedule (reported by
 * fft2d_plan_describe): with R = radix p and Ns the product of the earlier
 * radices, entry (r, k), r in [1, R), k in [0, Ns), is exp(-2 pi i k r / (Ns R)),
 * stored pass after pass, r-major within a pass. Every entry is computed in
 * FP64 from its own angle and rounded once to FP32 (the paper's Section 4
 * precomputes its twiddles once at start-up).
 * Errors: FFT2D_ERR_WRONG_PLAN_KIND for a batched plan,
 * FFT2D_ERR_INVALID_SIZE for another `which`.
 */
fft2d_status fft2d_plan_twiddles(fft2d_plan_t plan, int which, void* host_out, int64_t capacity, int64_t* count);

/* Work-buffer capacity of fft2d_exec_noalloc, in bytes (64 MiB). */
#define FFT2D_NOALLOC_WORK_BYTES (64 * 1024 * 1024)

/*
 * fft2d_exec_noalloc -- fft2d_exec without a plan and without any allocation,
 * for callers that cannot allocate device memory when they transform (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). It computes exactly what fft2d_exec computes for a plan made by
 * fft2d_plan(batch, rows, cols) on the current device, with the same kernels
 * (and the same environment overrides), on caller-owned buffers:
 *   batch, rows, cols : as for fft2d_plan (FFT2D_ERR_INVALID_SIZE otherwise);
 *   in, out           : device pointers to batch*rows*cols complex64, 8-byte
 *                       aligned; in == out allowed, partial overlap rejected;
 *   direction, stream : as for fft2d_exec.
 * Instead of plan memory it uses one library-owned device array of
 * 3*16384*8 bytes of twiddle tables plus FFT2D_NOALLOC_WORK_BYTES of work
 * buffer, which every GPU the library runs on holds from its first use until
 * the process ends. Each call first rewrites the tables on `stream` (one small
 * kernel computing every entry in FP64 and rounding it once to FP32), then
 * enqueues the passes; it never synchronises and calls no allocating routine.
 * Only in-place calls of split shapes (see fft2d_plan) need the work buffer:
 * such a call with batch*rows*cols*8 > FFT2D_NOALLOC_WORK_BYTES returns
 * FFT2D_ERR_INVALID_SIZE before enqueuing anything. Calls that overlap on one
 * GPU (several streams or host threads) race on the shared array and must not
 * be made; calls ordered on one stream are safe.
 */
fft2d_status fft2d_exec_noalloc(int64_t batch, int64_t rows, int64_t cols, const void* in, void* out,
                                int direction, void* stream);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int fft2d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFT2D_H */
