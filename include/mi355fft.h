/*
 * mi355fft - complex Cooley-Tukey FFT for AMD MI355X (gfx950), C ABI.
 *
 * Operation (Zhang, Hu, Yin, Hu, "A GPU Based Memory Optimized Parallel
 * Method For FFT Implementation", Sec. 2.1):
 *   forward, eq. 1:  X(k) = sum_{n<N} x(n) W_N^{nk},        W_N = exp(-2*pi*i/N)
 *   inverse, eq. 2:  x(n) = (1/N) sum_{k<N} X(k) W_N^{-nk}
 * The forward transform is unscaled and the inverse carries 1/N unless
 * fft_set_scale() overrides it.  2-D transforms apply eq. 1 / eq. 2 along
 * every row and then every column (Sec. 2.3.2); the default inverse scale is
 * then 1/(rows*cols).
 *
 * Method (Sec. 2.3): a transform that fits one workgroup runs all of its
 * butterfly stages in LDS and registers in one kernel.  Longer transforms
 * are split in global memory as N = N1*N2 (the reducibility of eq. 5) into
 * a pass of N1-point sub-transforms, a twiddle multiply W_N^{n2*k1}, and a
 * pass of N2-point sub-transforms; each pass is one kernel.  2-D transforms
 * with tall columns use three passes (the paper's three-exchange case):
 * two column sub-passes and a row pass.  Twiddle factors come from sin/cos
 * tables computed once per plan (Sec. 2.3.1).
 *
 * Data layout: complex values interleaved (re, im), row-major, batch
 * outermost, contiguous, natural order in and out.
 *   FFT_C64   - float32 pairs (8 bytes per point)
 *   FFT_C16F  - IEEE binary16 pairs (4 bytes per point)
 *   FFT_C16BF - bfloat16 pairs (4 bytes per point)
 * 16-bit data are converted to float32 on load and rounded to nearest even
 * on store; all arithmetic and twiddles are float32.  Twiddle tables are
 * computed in float64 and rounded to float32.
 *
 * Pointers: `in` and `out` are device pointers the caller owns; they must
 * stay valid until the work queued on `stream` has finished.  `stream` is a
 * hipStream_t passed as void* (NULL = the null stream).
 *
 * Errors: every call returns FFT_OK (0) or a negative FFT_ERR_* code; no
 * C++ exception crosses this interface and nothing aborts.  Faults inside a
 * kernel surface, as usual for HIP, at the caller's next synchronisation.
 */
#ifndef MI355FFT_H
#define MI355FFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft_plan_s *fft_plan_t;

/* dtype */
#define FFT_C64 0
#define FFT_C16F 1
#define FFT_C16BF 2

/* direction: sign of the exponent of W (eq. 1 uses -1, eq. 2 uses +1) */
#define FFT_FORWARD (-1)
#define FFT_INVERSE (+1)

/* status codes */
#define FFT_OK 0
#define FFT_ERR_INVALID_ARGUMENT (-1) /* null pointer, dims, batch, dtype, direction, schedule */
#define FFT_ERR_UNSUPPORTED_SIZE (-2) /* a length that is not a power of two, or out of range */
#define FFT_ERR_ALIGNMENT (-3)        /* in/out not aligned to the element size (8 B complex64,
                                         4 B 16-bit pairs: every access moves one element) */
#define FFT_ERR_INPLACE (-4)          /* in == out on a multi-pass plan with no workspace */
#define FFT_ERR_HIP (-5)              /* a HIP call failed; see fft_last_hip_error() */
#define FFT_ERR_NO_MEMORY (-6)        /* host or device allocation failed */
#define FFT_ERR_WATCHDOG (-7)         /* the batched kernel's bounded wait expired */
#define FFT_ERR_SCRATCH_LIMIT (-8)    /* fft_exec_static: the exec needs more than
                                         FFT_STATIC_SCRATCH_BYTES of scratch */

/* Size limits.  1-D lengths 1 .. 2^28 (three passes above 2^24); 2-D
 * extents 1 .. 2^14 each.  Batched plans (fft_plan_many*) take 1 .. 2^24. */
#define FFT_MAX_LOG2_1D 28
#define FFT_MAX_LOG2_2D 14

/*
 * Plan (Sec. 2.3.2: how many kernel calls a length needs, and the N = N1*N2
 * split of eq. 5 between them; Sec. 2.3.1: the sin/cos table built before
 * the transform).
 * Create a plan for `batch` transforms of shape n[0..dims) (dims 1 or 2;
 * for dims 2, n[0] = rows, n[1] = columns, row-major), element type `dtype`
 * and `direction`.  Builds the twiddle tables (float64 -> float32 on the
 * host; generated on the GPU in float64 for 1-D lengths >= 2^22) and
 * uploads them to the current device.  Blocking; not for use under stream
 * capture.  On success *out holds the plan; on failure *out is NULL.
 */
int fft_plan(const int64_t *n, int64_t batch, int dims, int dtype, int direction,
             fft_plan_t *out);

/*
 * As fft_plan, with an explicit schedule string (used by the autotuner and
 * by tests).  NULL or "" selects the built-in choice.  Grammar:
 *   schedule := item (';' item)*
 *   item     := 'split=' N1            (1-D two-pass: first-pass length; three-pass:
 *                                       first-pass length, default 2^10)
 *             | 'split2=' N2          (1-D three-pass (Sec. 2.3.3's "cube": N =
 *                                       N1*N2*N3, used above 2^24 or when given):
 *                                       second-pass length, 2 .. 2^7, default 2^7)
 *             | 'a=' variant | 'b=' variant | 'row=' variant | 'col=' variant
 *             | 'single=' variant
 *             | 'xcd=' digits         (one '0'/'1' for every pass, or one digit
 *                                       per pass, first pass first; 1: consecutive
 *                                       tiles run on one XCD, sharing its L2.
 *                                       Persistent variants ('q'): the workgroups
 *                                       of one XCD start on consecutive tiles)
 *             | 'col3=' 0|1           (2-D: columns as two sub-passes of sqrt(rows)
 *                                       points; rows a power of 4, at least 2 columns)
 *             | 'colt=' variant       (the first of those sub-passes)
 *             | 'blk=' 0|8|16|32      (2-D two-pass plan: the row pass writes its
 *                                       output in blocks of that many columns,
 *                                       each block's rows back to back, so that
 *                                       a column tile reads one contiguous run;
 *                                       the column pass writes the natural
 *                                       layout.  0, the default: natural order)
 *             | 'rowcol=' 0|2|4       (2-D, complex64: the row pass also takes the
 *                                       first radix-r step of the columns (R =
 *                                       r*M, eq. 5): a tile holds rows n1 + M*j,
 *                                       j < r, and writes rows r*n1 + k2; then
 *                                       M-point columns over rows r*n1 + k2,
 *                                       in place, whose tiles can be r times
 *                                       wider.  'row=' then names a fused
 *                                       variant ('f'), 'col=' an M-point column
 *                                       variant.  In place needs a workspace.)
 *             | 'method=' lds|levels  (1-D only.  'levels' is the method the
 *                                       paper replaces (Sec. 2.2, Fig. 2), kept
 *                                       for comparison: one radix-2 kernel per
 *                                       butterfly level, each reading and writing
 *                                       every point in global memory, ping-ponging
 *                                       through a plan-owned buffer of batch*N
 *                                       elements; in place as well, no workspace.
 *                                       fft_plan_info reports the whole sequence
 *                                       as one entry "levels_radix2".
 *                                       'mfma', 'xlane', 'xlane_bperm': N = 256
 *                                       complex64 only, 256 = 16 x 16 (eq. 5) in
 *                                       one kernel, kept as experiments beside
 *                                       the LDS path: the radix-16 stages as
 *                                       matrix-core products ("mfma_dft256"), or
 *                                       the exchange between the two stages as
 *                                       cross-lane moves instead of LDS, by DPP
 *                                       and ds_swizzle ("xlane_dft256") or by
 *                                       ds_bpermute ("xlane_bperm_dft256").)
 *   variant  := name as listed by fft_variant_name()
 * FFT_ERR_INVALID_ARGUMENT if the string does not parse or names a variant
 * that cannot run this size.
 */
int fft_plan_ex(const int64_t *n, int64_t batch, int dims, int dtype, int direction,
                const char *schedule, fft_plan_t *out);

/*
 * Plan `count` independent 1-D transforms whose lengths sizes[0..count) are
 * powers of two in 1 .. 2^24, packed back to back in the given order (the
 * offset of transform i is the sum of sizes[0..i)).  fft_exec runs them all
 * with one persistent kernel.  By default ('pipe=2' below) it is launched
 * twice per exec: the first launch runs every one-pass transform and the
 * first pass of every two-pass one, the second launch every second pass, so
 * the kernel boundary orders each transform's passes (Sec. 2.3.3); inside a
 * launch the workgroups claim work items from a device queue and never wait
 * for one another.  The single-launch kernels ('pipe=0|1') chain a
 * transform's passes by a completion counter instead.  The queue state lives
 * in the plan's workspace and is reset by the kernel itself, so the launches
 * can be captured in a hipGraph and replayed.  Two fft_exec calls that share one workspace must not run
 * concurrently.
 */
int fft_plan_many(const int64_t *sizes, int64_t count, int dtype, int direction,
                  fft_plan_t *out);

/*
 * As fft_plan_many with a schedule string of ';'-separated items:
 *   'p=' 8|16          points per lane (radix of the in-register stages)
 *   'threads=' 256|512 workgroup size (not every dtype has every size;
 *                      default 512)
 *   'pass2=' t         lengths of at least 2^t use two passes (1 <= t <= 1 +
 *                      log2 of the longest one-tile length, which is the default)
 *   'order=' bigfirst|given   order of the work queue
 *   'pipe=' 0|1|2      0: one launch, items from a shared atomic queue, a
 *                      second-pass tile waits on its transform's completion
 *                      counter; 1: one workgroup per CU that loads its next
 *                      item while it transforms the current one (compiled for
 *                      p=16, threads=256|512), items assigned round-robin in
 *                      queue order, completion counters as in 0 -- its
 *                      progress needs every workgroup of the launch resident
 *                      at once, so it is only for a GPU the launch has to
 *                      itself; 2 (the default): the same pipelining in two
 *                      launches per exec (first passes and one-pass tiles,
 *                      then second passes; the kernel boundary orders a
 *                      transform's passes and no workgroup waits for another),
 *                      items claimed from each launch's atomic queue head.
 *                      fft_plan_info names the kernel many_queue, many_pipe
 *                      or many_2launch
 *   'pass.L=' 1|2      length 2^L in one pass or two (one needs 2^L within
 *                      the longest tile)
 *   'n1.L=' l          two passes for length 2^L with a first pass of 2^l
 *                      points (both sub-lengths within the longest tile)
 *   'lag=' k           0 (default): every first-pass item ahead of every
 *                      second-pass item; k > 0: the second-pass items of the
 *                      i-th two-pass transform follow the first-pass items of
 *                      the (i+k)-th, so its intermediate is read back while it
 *                      is still in the last-level cache
 *   'ntst=' 0|1        pipe=2 only: 1 stores every item's results with the
 *                      nontemporal hint (default 0)
 *   'ntail=' k         pipe=2 only: the last k items of each launch store
 *                      with the nontemporal hint, so that less written data
 *                      is still dirty in the caches when the launch ends and
 *                      has to be written back before the next launch starts
 *                      (default 0)
 * FFT_ERR_INVALID_ARGUMENT for a malformed item or an uncompiled combination.
 * In-place exec (in == out) is refused with FFT_ERR_INPLACE when any length
 * uses two passes.
 */
int fft_plan_many_ex(const int64_t *sizes, int64_t count, int dtype, int direction,
                     const char *schedule, fft_plan_t *out);

/*
 * Host-only view of the work queue fft_plan_many_ex would build (no GPU use):
 * *n_items items; if `items` is not NULL it receives 4 ints per item in queue
 * order: kind (0 one-pass tile, 1 first-pass tile, 2 second-pass tile),
 * log2 of the tile's transform length, transform index (for a one-pass tile:
 * its first transform), and the tile number (one-pass: the number of
 * transforms in the tile).  first_len[i] / first_tiles[i] (each may be NULL)
 * receive N1 and the first-pass tile count of transform i (0 for one-pass
 * transforms).  FFT_ERR_INVALID_ARGUMENT if max_items is too small.
 */
int fft_describe_many(const int64_t *sizes, int64_t count, int dtype, const char *schedule,
                      int32_t *items, int64_t max_items, int64_t *n_items, int32_t *first_len,
                      int32_t *first_tiles);

/*
 * Host-only: how the launches of a batched exec split fft_describe_many's
 * item list: *n_q launches; if `q_off` is not NULL it receives n_q + 1
 * offsets, launch p running items q_off[p] .. q_off[p+1]-1 (the two-launch
 * kernel, schedule 'pipe=2': first passes and one-pass tiles, then second
 * passes; the other kernels: one launch).
 * FFT_ERR_INVALID_ARGUMENT if max_q < n_q + 1.
 */
int fft_describe_many_launches(const int64_t *sizes, int64_t count, int dtype, const char *schedule,
                               int32_t *q_off, int64_t max_q, int64_t *n_q);

/*
 * Batched plans only: a second-pass tile waits on its transform's counter for
 * at most a wall-clock bound (default 2 s per wait), then sets a watchdog
 * flag and goes on, so the kernel always finishes.  fft_many_watchdog()
 * reads (blocking) that flag, returning FFT_ERR_WATCHDOG if set (and clearing
 * it if `clear`); an expired wait means the results are invalid.
 * fft_many_set_wait_limit() sets the bound in microseconds (1 .. 2^40).
 */
int fft_many_watchdog(fft_plan_t plan, int clear);
int fft_many_set_wait_limit(fft_plan_t plan, int64_t microseconds);

/*
 * Execute (eq. 1 forward or eq. 2 inverse on every transform of the plan, by
 * the passes of Sec. 2.3.2; for 2-D, rows then columns).
 * Queue the transform on `stream`.  Asynchronous: no host synchronisation, no
 * allocation, no host reads of device data, so it may be captured into a
 * hipGraph.  `in` and `out` must not partially overlap; in == out is allowed
 * for one-pass plans, for three-pass plans, and for two-pass plans once a
 * workspace of fft_workspace_size() bytes is set (else FFT_ERR_INPLACE).  Input data are
 * not modified unless in == out.  A plan may be executed on several streams;
 * execs that share a workspace (in-place two-pass, three-pass and batched
 * plans) must not overlap in time, and calls on one plan from several host
 * threads must be serialised by the caller (the plan's timing state is not
 * locked).
 */
int fft_exec(fft_plan_t plan, const void *in, void *out, void *stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).
 * As fft_exec, except that the scratch an exec needs -- a batched plan's
 * queue and completion counters, the intermediate of an in-place two-pass
 * exec, or the intermediate of a three-pass plan -- is taken from one static
 * device array of FFT_STATIC_SCRATCH_BYTES (32 MiB) that the library holds on
 * every device it runs on until the process ends, instead of the plan's
 * workspace.  The plan's own workspace, if any, is neither used nor changed.
 * It calls no allocating routine: the array's device address is looked up
 * once per device (hipGetSymbolAddress) on the first call on that device,
 * which must be the device the plan was made on (else
 * FFT_ERR_INVALID_ARGUMENT).  A batched plan's counters are cleared by a
 * small fill kernel on `stream` before its launch.  Execs that need no
 * scratch run exactly as fft_exec.  Errors: as fft_exec, plus
 * FFT_ERR_SCRATCH_LIMIT when the exec needs more than the array holds (for
 * complex64: in-place two-pass or three-pass execs of more than 2^22 points
 * in all; batched plans of more than about 8 million transforms).
 * For a batched plan the bound on its dependency waits is as in fft_exec,
 * and an expired wait sets the flag in the plan's own workspace, which
 * fft_many_watchdog() reads.
 * Every call on one device shares that device's array and leaves its
 * contents behind: calls that need scratch and overlap in time on one device
 * (on different streams, or from different host threads) race and give
 * undefined results; the caller must order them.
 */
#define FFT_STATIC_SCRATCH_BYTES (32u << 20)
int fft_exec_static(fft_plan_t plan, const void *in, void *out, void *stream);

/*
 * Output scale (eq. 2 carries 1/N; eq. 1 none).
 * Scale applied to every output value (default 1 forward, 1/(product of
 * lengths) inverse, per transform for plan_many).  The adjoint of the forward
 * transform is the inverse-direction plan with scale 1.
 */
int fft_set_scale(fft_plan_t plan, double scale);

/*
 * Workspace for the global-memory exchanges between passes (Sec. 2.3.2/2.3.3).
 * Device scratch a plan needs to run in place (1-D two-pass), on every exec
 * (1-D three-pass plans, lengths above 2^24: one buffer of batch * N
 * elements, allocated by the plan) or, for plan_many, for its queue and
 * counters.  fft_set_workspace hands the plan caller-owned device memory of
 * at least that many bytes (NULL, 0 returns to the plan-owned default, if
 * any); the caller keeps it alive while the plan may run.
 */
int fft_workspace_size(fft_plan_t plan, size_t *bytes);
int fft_set_workspace(fft_plan_t plan, void *ptr, size_t bytes);

typedef struct {
  int64_t n[2];          /* shape (n[1] = 1 for 1-D) */
  int64_t batch;         /* transforms per exec (count for plan_many) */
  int dims, dtype, direction;
  int passes;            /* kernel launches per exec */
  int64_t split[2];      /* 1-D two-pass: N1, N2 (0 otherwise) */
  char pass_variant[4][32]; /* variant name of each launch */
  int64_t points;        /* complex points per exec */
  double flops;          /* nominal 5 N log2 N summed over transforms */
  double bytes_min;      /* bytes read + written once (in + out) */
  double bytes_pass[4];  /* algorithmic bytes read + written by each launch */
  int gpu_twiddles;      /* 1 if the tables were generated on the GPU */
} fft_plan_info_t;

/* What a plan runs (the passes of Sec. 2.3.2 and the nominal work of eq. 1
 * counted as 5 N log2 N).  FFT_ERR_INVALID_ARGUMENT for NULL arguments. */
int fft_plan_info(fft_plan_t plan, fft_plan_info_t *info);

/* Free the plan's tables and workspace.  NULL is a no-op. */
int fft_destroy(fft_plan_t plan);

/* Static text for a status code. */
const char *fft_error_string(int status);

/* The hipError_t of the last failing HIP call in this thread (0 if none). */
int fft_last_hip_error(void);

/*
 * Kernel variants compiled into the library: fft_variant_count() of them;
 * fft_variant_name(i) gives the i-th name (NULL if out of range) and
 * fft_variant_describe(i, ...) its sub-transform length L, points per lane
 * P, transforms per workgroup W, workgroup size and role (0 contiguous rows,
 * 1 first pass of a split, 2 strided columns, 3 strided columns with a
 * twiddle, 4 rows fused with a radix-W column step).  Names read
 * <role><L>p<P>w<W>[q|q2][x]_<dtype>: role r, a, c, t, f as above; q a
 * persistent kernel (one workgroup per CU walking the tiles)
 * with the next tile's loads in flight while one is computed, q2 with the
 * next two; x the exchange through LDS in two rounds (real, then
 * imaginary parts), which halves its LDS footprint.
 */
int fft_variant_count(void);
const char *fft_variant_name(int index);
int fft_variant_describe(int index, int *L, int *P, int *W, int *threads, int *role,
                         int *dtype);

/*
 * Host-only planning: the schedule fft_plan would choose, without touching
 * the GPU.  Writes the pass count and up to 4 variant names (as in
 * fft_plan_info_t.pass_variant) and the split.
 */
int fft_describe(const int64_t *n, int64_t batch, int dims, int dtype,
                 const char *schedule, int *passes, char names[4][32],
                 int64_t split[2]);

/*
 * Per-launch timing with HIP events on the exec stream (timing-only events,
 * without a system-scope fence, so that they do not write back and
 * invalidate caches between passes).  A pass that is one kernel launch
 * hands its two events to the launch itself (hipExtLaunchKernel), so they
 * take the kernel's own start and end, as a kernel trace does; other work
 * (a copy pass, a pass launched once per transform, the batched, per-level
 * and 256-point plans) is bracketed by events recorded before and after it.
 * fft_profile_enable(plan, slots) with slots >= 1 creates events for
 * `slots` execs (blocking) and clears the totals; every later fft_exec
 * records its launches into the next slot (a ring: execs beyond `slots`
 * between two collects overwrite the oldest).  slots = 0 turns timing off.
 * After the caller has synchronised the stream, fft_profile_collect() adds
 * the elapsed time of every pending exec's launches to running totals, and
 * fft_profile_read(plan, pass, &ms, &count) returns the total milliseconds
 * and the number of timed launches of pass `pass` (0-based launch index
 * within one exec).  Execs queued on a stream that is being captured into a
 * graph are not timed (their events could not be read back from replays).
 * fft_profile_sample(plan, every) times only one exec in `every` (the first,
 * then every `every`-th after it; default 1), so that the events' own cost
 * is spread thin over a long timed run; FFT_ERR_INVALID_ARGUMENT if
 * every < 1.  It restarts the count; enabling keeps the setting.
 */
int fft_profile_enable(fft_plan_t plan, int slots);
int fft_profile_sample(fft_plan_t plan, int every);
int fft_profile_collect(fft_plan_t plan);
int fft_profile_read(fft_plan_t plan, int pass, double *total_ms, int64_t *launches);

/*
 * The host twiddle generator, for inspection and tests: writes `count`
 * float32 pairs out[2i], out[2i+1] = W_M^{e(i)} (re, im) with
 * e(i) = (i / R) * (i % R) * mul for R > 0 and e(i) = i * mul for R == 0,
 * each the float64 value of Sec. 2.3.1's sin/cos table rounded to nearest.
 * M must be a power of two.  Host memory; no GPU use.
 */
int fft_twiddle_host(int64_t count, int64_t R, int64_t M, int64_t mul, float *out);

/*
 * Host-to-host execution in chunks, with the transfers overlapped.
 *
 * The paper times its transforms with the host-to-device and device-to-host
 * copies included (Sec. 3), finds them dominant for short signals, and names
 * the transfer as the next thing to improve (Sec. 4).  A pipe runs a plan
 * over data in host memory: chunk c of `chunks` (each the plan's batch of
 * transforms, contiguous) is copied in on one stream, transformed on a
 * second and copied out on a third, so that the copy in of chunk c + 1, the
 * transform of chunk c and the copy out of chunk c - 1 proceed together.
 *
 * fft_pipe_create(plan, slots, &pipe): `slots` >= 2 device staging pairs
 * (input, output) of one chunk each, three non-blocking streams of default
 * priority and their events, all owned by the pipe (blocking; allocates).
 * The plan must outlive the pipe.
 * fft_pipe_exec(pipe, host_in, host_out, chunks): queues every copy and
 * transform and returns; host_in / host_out hold chunks * (plan's points)
 * elements of the plan's type.  Page-locked host memory (hipHostMalloc, or
 * torch's pin_memory) is needed for the copies to overlap; pageable memory
 * gives the same results more slowly.  The host buffers must stay valid and
 * host_in unmodified until fft_pipe_wait returns.  in-place (host_in ==
 * host_out) is allowed.
 * fft_pipe_wait(pipe): blocks until the last copy out has finished.
 * fft_pipe_destroy(pipe): waits, then frees everything the pipe owns; NULL
 * is a no-op.
 * Errors: FFT_ERR_INVALID_ARGUMENT (null pointer, slots < 2, chunks < 0),
 * FFT_ERR_NO_MEMORY, FFT_ERR_HIP.
 */
typedef struct fft_pipe_s *fft_pipe_t;
int fft_pipe_create(fft_plan_t plan, int slots, fft_pipe_t *out);
int fft_pipe_exec(fft_pipe_t pipe, const void *host_in, void *host_out, int64_t chunks);
int fft_pipe_wait(fft_pipe_t pipe);
int fft_pipe_destroy(fft_pipe_t pipe);

#ifdef __cplusplus
}
#endif

#endif /* MI355FFT_H */
