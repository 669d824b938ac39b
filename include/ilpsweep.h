/*
 * ilpsweep - offered-ILP streaming-load library for MI355X (gfx950).
 *
 * Method: Manjunath & Ramachandra, "Concurrency Response of Plain Global
 * Loads on the NVIDIA H100".  Every lane of a wavefront issues K independent
 * loads per iteration over a buffer far larger than the caches (Section 3,
 * "The axis K"), folds every loaded 32-bit word into a per-lane sink that the
 * compiler cannot drop (Section 3, "Instruments"), and the library reports
 * the attained bandwidth under a fixed-work control that holds the total
 * of issued logical loads equal for every K (Section 3, "Fixed-work
 * control"; Section 4.2, "Exact-work accounting").
 *
 * Conventions for every entry point below
 * ---------------------------------------
 *  - Return value: SWEEP_OK (0) or a negative SWEEP_E* code; the text of the
 *    last error of the calling thread is available from sweep_last_error().
 *    No C++ exception crosses this boundary.
 *  - Validation errors leave every output untouched.
 *  - Device pointers are plain HIP device addresses owned by the caller, who
 *    keeps them alive until the call returns.  Host pointers are ordinary
 *    host memory owned by the caller.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  A
 *    call enqueues its kernels on that stream and returns after they finish
 *    (it synchronises on an event recorded on that stream), except where a
 *    function says otherwise.
 *  - The library allocates small internal device scratch (per-wave records,
 *    per-cell results) on first use per device and frees it in
 *    sweep_shutdown().  Entry points take one library-wide lock, so calls
 *    from several host threads are safe; they run one after another.
 *  - Work unit: a wave-group is one wavefront's K loads, each a contiguous,
 *    coalesced 64-lane segment of 64 * vec_width bytes.  Lane l of load j of
 *    wave-group q reads vector ((q*K + j)*64 + l) mod (bytes / vec_width).
 *    Wave w of the grid handles q = w, w + n_waves, ... (round robin).
 *    This is the default order; opts.order selects the blocked deal or the
 *    strided layout for the plain kernel (SWEEP_ORDER_*).
 *  - Sinks: per lane a wrapping 32-bit sum and a 32-bit XOR of every loaded
 *    word, reduced over lanes, waves and the grid with the same operators.
 *  - Bandwidth is issued logical bytes per calibrated nanosecond, in decimal
 *    GB/s (Section 3, "Timing, residency, statistics").
 */
#ifndef ILPSWEEP_H
#define ILPSWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define SWEEP_OK          0
#define SWEEP_EINVAL     -1   /* argument out of range                       */
#define SWEEP_EALIGN     -2   /* pointer / size alignment violated           */
#define SWEEP_EOCCUPANCY -3   /* requested residency not achievable          */
#define SWEEP_EHIP       -4   /* a HIP runtime call failed                   */
#define SWEEP_ENOMEM     -5   /* internal scratch allocation failed          */
#define SWEEP_ENODEV     -6   /* no usable gfx950 device                     */

/* ------------------------------------------------------------- work modes */
/* Fixed work (the library's control): Q = floor(L / (64 K)) wave-groups dealt
 * round robin, so issued loads 64 K Q match L to within 64 K - 1 loads. */
#define SWEEP_FIXED_WORK        0
/* Baseline arm of Section 4.2, Table 1: every wave runs `fixed_iters`
 * iterations, so issued work grows in proportion to K. */
#define SWEEP_FIXED_ITERS       1
/* The paper's own construction (Section 3): every thread runs
 * floor(L / (threads K)) iterations. */
#define SWEEP_PER_THREAD_FLOOR  2

/* ---------------------------------------------------------- cache policies */
#define SWEEP_CACHE_DEFAULT   0  /* global_load, default (wave-scope) caching */
#define SWEEP_CACHE_NT        1  /* global_load ... nt (streaming hint)        */
#define SWEEP_CACHE_BYPASS_L1 2  /* buffer_load ... sc1: device scope, misses
                                    the vector L1 (the analogue of .cg)        */
#define SWEEP_CACHE_BYPASS_L1_NT 3 /* buffer_load ... sc1 nt: L1 bypass plus the
                                    streaming (non-temporal) hint              */

/* ------------------------------------------------------- work-group order */
/* How wave-groups are dealt to the waves (the address ordering of Section
 * 4.2's proposed discriminating experiment; coalescing, occupancy and bytes
 * are the same under all three).  Plain kernel only. */
#define SWEEP_ORDER_ROUND_ROBIN 0  /* wave w: q = w, w + n_waves, ...        */
#define SWEEP_ORDER_BLOCKED     1  /* wave w: q = w*G .. w*G+G-1,
                                      G = ceil(Q / n_waves)                    */
#define SWEEP_ORDER_STRIDED     2  /* dealt round robin, but load j of group q
                                      reads segment j*Q + q: a group's K loads
                                      go to K regions Q segments apart instead
                                      of K adjacent segments (the vectors read
                                      over a cell, and so its global sinks,
                                      are those of the other orders)           */

/* ----------------------------------------------------------------- kinds */
#define SWEEP_KIND_PLAIN        0  /* K independent loads into registers      */
#define SWEEP_KIND_LDS_ASYNC    1  /* loads straight into LDS, no dest VGPR   */
#define SWEEP_KIND_LDS_MATCHED  2  /* loads into VGPRs, then ds_write/ds_read */

/* ------------------------------------------------------------- FP dtypes */
#define SWEEP_F32       0
#define SWEEP_BF16      1
#define SWEEP_FP8_E4M3  2          /* OCP e4m3fn: bias 7, max 448, no inf    */

/* Per-wave record written by every sweep kernel (32 bytes).  t0 / t1 are
 * the wave's start and end readings of the constant-rate device wall clock
 * (s_memrealtime); hw_id / xcc_id are the HW_REG_HW_ID and HW_REG_XCC_ID
 * hardware registers read by the wave, which identify its CU and XCD. */
typedef struct {
  uint32_t sum32;
  uint32_t xor32;
  uint32_t hw_id;
  uint32_t xcc_id;
  uint64_t t0;
  uint64_t t1;
} sweep_wave_rec_t;

typedef struct {
  void*     stream;        /* hipStream_t, NULL = null stream              */
  int       cache_policy;  /* SWEEP_CACHE_*                                */
  int       mode;          /* SWEEP_FIXED_WORK / _FIXED_ITERS / _PER_THREAD_FLOOR */
  uint32_t  fixed_iters;   /* iterations per wave for SWEEP_FIXED_ITERS    */
  uint32_t  grid_wgs;      /* 0: CUs * waves_per_cu / (waves per WG)       */
  int       pin_occupancy; /* nonzero: pad LDS so that no CU can hold more
                              than the requested workgroups                 */
  sweep_wave_rec_t* wave_out; /* device, n_waves records, or NULL           */
  uint32_t* lane_out;      /* device, 2 u32 (sum, xor) per thread, or NULL  */
  int       order;         /* SWEEP_ORDER_* (plain kernel)                  */
  uint64_t  wave_out_cap;  /* records wave_out holds; a call whose launch
                              has more waves fails with SWEEP_EINVAL and
                              writes nothing (required with wave_out)       */
  uint64_t  lane_out_cap;  /* (sum, xor) pairs lane_out holds, i.e. threads;
                              checked like wave_out_cap                      */
  int       fuse;          /* sweep_graph_create / sweep_batched only:
                              nonzero runs each run of consecutive plain,
                              fixed-work, round-robin cells that share K,
                              vector width, cache policy and launch shape as
                              one persistent launch over their concatenated
                              wave-groups (results per cell as before) */
} sweep_opts_t;

typedef struct {
  uint64_t target_loads;   /* L                                            */
  uint64_t issued_loads;   /* 64 K Q (exact)                               */
  uint64_t issued_bytes;   /* issued_loads * vec_width                     */
  double   mismatch;       /* (L - issued) / L; 0 for fixed-iteration modes*/
  uint32_t sum32, xor32;   /* global sinks                                 */
  uint32_t grid_wgs, wg_threads, waves;
  uint32_t iters_min, iters_max;   /* per-wave iteration counts            */
  uint32_t max_wgs_per_cu; /* residency limit of the kernel at this launch */
  uint32_t vgprs, sgprs, lds_bytes, scratch_bytes; /* kernel resources;
                                      sgprs is 0: the runtime does not report it */
  uint64_t window_ticks;   /* max(t1) - min(t0) over all waves             */
  double   window_ns;      /* window_ticks converted with the clock rate   */
  double   event_ms;       /* hipEvent time of the kernel's dispatch       */
  double   gbps;           /* issued_bytes / window_ns                     */
} sweep_result_t;

typedef struct {
  uint32_t grid_wgs, wg_threads, waves;
  uint64_t n_vec;          /* vectors in the buffer                        */
  uint64_t Q;              /* wave-groups                                  */
  uint64_t issued_loads, issued_bytes;
  uint32_t iters_min, iters_max;
  double   mismatch;       /* (L - issued) / L                             */
  uint32_t lds_pad_bytes;  /* dynamic LDS per WG when pinning occupancy    */
} sweep_plan_t;

typedef struct {
  int      ordinal;
  char     arch[64];         /* gcnArchName, e.g. "gfx950:sramecc+:xnack-" */
  uint32_t num_cus;
  uint32_t lds_per_cu;       /* bytes                                      */
  uint32_t lds_per_wg_max;   /* bytes                                      */
  uint32_t l2_bytes;
  uint64_t hbm_bytes;
  double   wall_clock_hz;    /* nominal s_memrealtime rate                 */
  double   calibrated_hz;    /* rate measured against the host clock, 0 if
                                sweep_calibrate_clock() was not called      */
  int      clock_khz;        /* shader clock reported by the runtime       */
  int      mem_clock_khz;
  int      mem_bus_bits;
} sweep_device_t;

/* One cell of a sweep (sweep_run, sweep_batched, sweep_autotune). */
typedef struct {
  int         kind;          /* SWEEP_KIND_*                               */
  int         K;             /* loads per iteration (plain) or in-flight
                                depth (LDS kinds), 1..16                    */
  int         vec_width;     /* 4, 8 or 16 bytes (LDS kinds: 16)           */
  int         waves_per_cu;  /* plain: 4..32, multiple of 4; LDS: 1..16    */
  int         cache_policy;
  int         mode;
  uint32_t    fixed_iters;
  uint32_t    grid_wgs;      /* 0 = automatic                              */
  const void* buf;           /* device                                     */
  size_t      bytes;
  uint64_t    total_logical_loads;
  int         order;         /* SWEEP_ORDER_* (plain kind only)            */
} sweep_cell_t;

/* Result of a pointer chase. */
typedef struct {
  uint32_t final_index;      /* index reached after warm + timed hops       */
  uint32_t hops;             /* timed hops                                  */
  uint64_t wall_ticks;       /* wall-clock ticks over the timed hops        */
  double   ns_per_hop;       /* mean latency (includes sampling overhead
                                when n_samples > 0)                         */
  double   shader_clock_hz;  /* shader clock measured in the same window    */
} sweep_chase_t;

/* One walker of sweep_chase_walkers. */
typedef struct {
  uint32_t final_index;      /* index reached after warm + timed hops       */
  uint32_t xcc_id;           /* XCD the walker ran on (0..7 on MI355X)       */
  uint32_t hops;             /* timed hops                                   */
  uint32_t reserved;
  uint64_t wall_ticks;       /* device wall-clock ticks over the timed hops  */
  double   ns_per_hop;       /* mean latency of one dependent load           */
} sweep_walker_t;

/* Initialise the library on HIP device `ordinal` (makes it current) and
 * allocate its scratch.  Optional: every other call initialises lazily on
 * the current device.  Errors: SWEEP_ENODEV, SWEEP_EHIP, SWEEP_ENOMEM. */
int sweep_init(int ordinal);

/* Free all library-owned device memory and events on every device. */
int sweep_shutdown(void);

/* Fill `out` with the current device's properties. */
int sweep_device_info(sweep_device_t* out);

/* Measure the device wall-clock rate against the host steady clock over
 * about `seconds` (>= 0.01) and use it for all later window conversions
 * (Section 3: cross-SM windows come from a runtime-calibrated timer).
 * Writes the rate in Hz to *hz.  Errors: SWEEP_EINVAL, SWEEP_EHIP. */
int sweep_calibrate_clock(double seconds, double* hz);

/* Host-only plan of a plain-load cell (no GPU needed).  `num_cus` is the CU
 * count the grid is sized for.  Errors: SWEEP_EINVAL (K not in 1..16,
 * vec_width not 4/8/16, waves_per_cu not a multiple of 4 in 4..32, bytes 0,
 * L too small for one wave-group in fixed-work mode, fixed_iters 0 in
 * fixed-iteration mode, unknown mode or order, more than 2^32 - 1
 * iterations for some wave, issued bytes beyond 64 bits), SWEEP_EALIGN
 * (bytes not a multiple of 64 * vec_width, so that no 64-lane segment
 * straddles the buffer end). */
int sweep_plan(size_t bytes, int K, int vec_width, int waves_per_cu,
               uint64_t total_logical_loads, int mode, uint32_t fixed_iters,
               uint32_t num_cus, uint32_t grid_wgs, int order,
               sweep_plan_t* out);

/* Seeded buffer fill: 32-bit word i of `buf` becomes the low half of
 * SplitMix64 output i for state `seed` (Steele, Lea and Flood, 2014), i.e.
 * the generator state seed + (i+1) * 0x9E3779B97F4A7C15 passed through the
 * SplitMix64 finaliser.  `buf` is a device pointer aligned to 16 bytes,
 * `bytes` a multiple of 4.  Asynchronous on `stream` (does not wait).
 * Errors: SWEEP_EALIGN, SWEEP_EINVAL (bytes 0), SWEEP_EHIP. */
int sweep_fill_u32(void* buf, size_t bytes, uint64_t seed, void* stream);

/* Plain-load K sweep cell (Section 3, "The axis K"; Section 4.2): every
 * lane issues K independent `vec_width`-byte global loads per iteration
 * before consuming any of them, then folds each 32-bit word into its sinks.
 * The grid is persistent: grid_wgs workgroups of 256 threads (4 waves), by
 * default CUs * waves_per_cu / 4, so waves_per_cu / 4 waves per SIMD.
 *   buf        device, 16-byte aligned, read only
 *   bytes      buffer size, a multiple of 64 * vec_width
 *   K          1..16
 *   vec_width  4, 8 or 16
 *   waves_per_cu  4..32, multiple of 4
 *   total_logical_loads  L (fixed-work and per-thread-floor modes)
 *   opt        may be NULL (defaults: null stream, SWEEP_CACHE_DEFAULT,
 *              fixed work, pinned occupancy)
 *   out        host result
 * Errors: SWEEP_EINVAL, SWEEP_EALIGN, SWEEP_EOCCUPANCY (the kernel's
 * registers or LDS do not allow waves_per_cu), SWEEP_EHIP. */
int sweep_plain(const void* buf, size_t bytes, int K, int vec_width,
                int waves_per_cu, uint64_t total_logical_loads,
                const sweep_opts_t* opt, sweep_result_t* out);

/* sweep_plain for callers that cannot allocate memory (code that must not
 * call hipMalloc: tight serving or measurement loops, harnesses that forbid
 * allocation).  Same arguments, kernels, validation and results as
 * sweep_plain, except:
 *  - The wave records, the cell result and the record offsets live in a
 *    static device array of 512 KiB + 256 bytes per GPU, held until the
 *    process ends; the call allocates nothing (no hipMalloc, hipFree, pinned
 *    host memory or events).  Its device address is resolved once per GPU,
 *    in sweep_init() or else on the first call on that GPU.
 *  - A launch of more than 16384 waves (CUs * waves_per_cu) fails with
 *    SWEEP_EINVAL unless opt->wave_out receives the records instead.
 *  - event_ms is 0: the call is timed by the kernel's own clock window
 *    (window_ns, gbps) and returns after a stream synchronisation.
 *  - Every call on a GPU shares that GPU's array, which keeps the last
 *    call's contents; each call writes everything it reads before reading
 *    it.  Calls take the library lock and return only when their work is
 *    done, so calls from one process do not overlap; work that overlapped
 *    it on the same GPU from outside the library would race on the array.
 * Errors: as sweep_plain. */
int sweep_plain_noalloc(const void* buf, size_t bytes, int K, int vec_width,
                        int waves_per_cu, uint64_t total_logical_loads,
                        const sweep_opts_t* opt, sweep_result_t* out);

/* LDS-direct asynchronous path (Section 4.3, the counterpart of cp.async:
 * loads that write LDS with no destination register).  Every wave keeps a
 * ring of `depth` 1 KiB LDS slots; each slot is filled by one
 * global_load_lds_dwordx4 (16 bytes per lane), waited for with
 * s_waitcnt vmcnt(depth - 1), read back by its own lane (ds_read_b128),
 * folded, and refilled, so `depth` requests stay in flight.  The address
 * map is the plain map with K = depth, so the sinks equal sweep_plain's.
 *   depth         1..16
 *   vec_width     16
 *   waves_per_cu  1..16 waves in the one workgroup per CU
 *                 (LDS: waves_per_cu * depth KiB per CU)
 * Errors as sweep_plain. */
int sweep_lds_async(const void* buf, size_t bytes, int depth, int vec_width,
                    int waves_per_cu, uint64_t total_logical_loads,
                    const sweep_opts_t* opt, sweep_result_t* out);

/* Matched plain path of Section 4.3: the same ring, depth and address map,
 * but each request is a global_load_dwordx4 into registers followed by a
 * ds_write_b128 into the slot and the ds_read_b128 back.  Arguments and
 * errors as sweep_lds_async. */
int sweep_lds_matched_plain(const void* buf, size_t bytes, int depth,
                            int vec_width, int waves_per_cu,
                            uint64_t total_logical_loads,
                            const sweep_opts_t* opt, sweep_result_t* out);

/* Two co-resident streams in one workgroup (Section 4.4).  Each workgroup
 * (one per CU) holds `waves_plain` waves of the plain K-load loop (K =
 * depth, 16-byte loads) over the first half of the buffer (stream A) and
 * `waves_async` waves of the LDS-direct ring (depth `depth`) over the
 * second half (stream B); either count may be 0 to measure a stream solo.
 * total_logical_loads is split evenly between the streams.  out[0] is
 * stream A, out[1] stream B (each with its own sinks and window).
 *   depth 1..16; waves_plain, waves_async 0..8, not both 0.
 * This is the cross-mechanism mix; sweep_two_stream_kind with kind_b =
 * SWEEP_KIND_PLAIN gives the same-mechanism one the section measures.
 * Errors as sweep_plain. */
int sweep_two_stream(const void* buf, size_t bytes, int depth,
                     int waves_plain, int waves_async,
                     uint64_t total_logical_loads, const sweep_opts_t* opt,
                     sweep_result_t out[2]);

/* The same two co-resident streams with stream B's mechanism chosen:
 * kind_b = SWEEP_KIND_LDS_ASYNC is sweep_two_stream; kind_b =
 * SWEEP_KIND_PLAIN runs the plain K-load loop in both streams (plain loads
 * beside plain loads in one workgroup, Section 4.4).  Stream B's sinks do
 * not depend on kind_b: both mechanisms read the same address map.
 *   waves_a, waves_b 0..8, not both 0; other arguments and errors as
 *   sweep_two_stream; SWEEP_EINVAL for any other kind_b. */
int sweep_two_stream_kind(const void* buf, size_t bytes, int depth, int waves_a,
                          int waves_b, int kind_b, uint64_t total_logical_loads,
                          const sweep_opts_t* opt, sweep_result_t out[2]);

/* The two streams placed on different CUs: the cross-SM placement that
 * Section 6 lists as confirmatory work for the same-CTA test of Section
 * 4.4.  Half of the workgroups run `waves_a` waves of stream A, the other
 * half `waves_b` waves of stream B (workgroups of max(waves_a, waves_b)
 * waves; the surplus waves of the smaller stream leave at once).  In every
 * run of 16 consecutive workgroups the first 8 are stream A's and the last
 * 8 stream B's; workgroups are dealt to the 8 XCDs in turn, so each XCD
 * holds as many of each.  With opt->pin_occupancy (the default) each CU
 * holds one workgroup, so no CU runs both streams.  A stream with 0 waves
 * leaves its workgroups empty: the solo runs keep the co-run's placement.
 * Equal total waves per stream to sweep_two_stream_kind(a, b) are
 * sweep_two_stream_split(2a, 2b).  The buffer halves, the split of
 * total_logical_loads, the sinks and out[] are as in sweep_two_stream_kind.
 *   waves_a, waves_b 0..16, not both 0; the grid (opt->grid_wgs, or one
 *   workgroup per CU) a multiple of 16, else SWEEP_EINVAL; other
 *   arguments and errors as sweep_two_stream_kind.
 * No passage of the paper measures this placement; it states only that
 * its two-stream result is same-CTA and names cross-SM placement as work
 * to do. */
int sweep_two_stream_split(const void* buf, size_t bytes, int depth, int waves_a,
                           int waves_b, int kind_b, uint64_t total_logical_loads,
                           const sweep_opts_t* opt, sweep_result_t out[2]);

/* Sweep driver: runs `n` cells back to back on opt->stream in the given
 * order (ascending or reversed sweeps are the caller's ordering, Section
 * 3), with per-cell hipEvents and per-wave clock windows, and one host
 * synchronisation at the end.  opt->stream is used for every cell; the
 * cells' own fields override the other options.  results[i] belongs to
 * cells[i].  Errors: the first failing cell's code (nothing is launched if
 * any cell fails validation). */
int sweep_run(const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
              sweep_result_t* results);

/* Batched sweep (no passage of the paper defines it: it batches the cells
 * of Section 3's sweeps the way a production sweep runs them): the same
 * cells captured into a hipGraph (one kernel node per cell, then one
 * finishing node) and launched with a single
 * hipGraphLaunch; equivalent to sweep_graph_create + sweep_graph_launch +
 * sweep_graph_destroy.  Per-cell windows come from the in-kernel clock
 * records; results[i].event_ms is 0 and *graph_ms receives the hipEvent
 * time of the whole launch.  Errors as sweep_run. */
int sweep_batched(const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
                  sweep_result_t* results, double* graph_ms);

/* A sweep captured once into a hipGraph and replayed (as sweep_batched, no
 * passage of the paper defines it): one kernel node per cell, in order,
 * then one finishing kernel.  The graph owns its scratch
 * (wave records, per-cell results, offsets; 32 B per wave plus 40 B per
 * cell), so other library calls between replays do not disturb it.  The
 * cells' buffers must stay allocated until the graph is destroyed; their
 * contents may change between replays.
 * sweep_graph_create: validates every cell (errors as sweep_run), captures
 *   and instantiates; *out receives the handle.  Only opt->pin_occupancy
 *   and opt->fuse are read (opt may be NULL).  SWEEP_ENOMEM if the scratch
 *   cannot be had.
 * sweep_graph_launch: replays on `stream` (a hipStream_t of the graph's
 *   device, NULL = default stream), waits, and fills results[0..n) in cell
 *   order (per-cell windows from the in-kernel clock records, event_ms 0)
 *   and *graph_ms (hipEvent time of the whole replay; may be NULL).
 *   Replays of one graph must not overlap.
 * sweep_graph_destroy: frees the graph and its scratch; NULL is allowed. */
typedef struct sweep_graph sweep_graph_t;
int sweep_graph_create(const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
                       sweep_graph_t** out);
int sweep_graph_launch(sweep_graph_t* graph, void* stream, sweep_result_t* results,
                       double* graph_ms);
int sweep_graph_destroy(sweep_graph_t* graph);

/* Autotuner (no passage of the paper defines it; it searches the axes the
 * method sweeps, Section 3 "The axis K" and occupancy): times every
 * candidate (vec_width, K, waves_per_cu) for a plain cell over `buf` /
 * `bytes` (one full pass per launch, fixed work), `reps`
 * launches each after one warm-up launch, and returns the candidate with
 * the best median bandwidth in *best (kind, K, vec_width, waves_per_cu,
 * cache_policy filled; buf, bytes and total_logical_loads set for one full
 * pass) and that median in *best_gbps.  Candidates that fail with
 * SWEEP_EOCCUPANCY are skipped.  Arrays are host memory.
 * Errors: SWEEP_EINVAL (empty candidate set, reps < 1), others as
 * sweep_plain. */
int sweep_autotune(const void* buf, size_t bytes,
                   const int* vec_widths, int n_vec_widths,
                   const int* Ks, int n_Ks,
                   const int* waves_per_cu, int n_waves,
                   int cache_policy, int reps,
                   sweep_cell_t* best, double* best_gbps);

/* Streaming sum of a floating-point payload (precision variant; no passage
 * of the paper defines it: it applies the streaming loop of Section 3 to
 * FP payloads and adds compensated accumulation): every lane
 * loads 16-byte vectors, decodes them to FP32 and accumulates them with
 * TwoSum into an (s, c) pair (Sum2 of Ogita, Rump and Oishi, 2005; FP8 in
 * chunks of 64 values, whose FP32 sum is exact); pairs are merged per wave
 * and per workgroup in FP32 with TwoSum, and only the final combine of the
 * per-workgroup pairs is done in FP64.  Every lane keeps eight 16-byte
 * loads in flight at waves_per_cu = 4 and four above.  Deterministic for a
 * fixed grid and waves_per_cu.
 *   payload  device, 16-byte aligned; n_elems elements of `dtype`
 *   n_elems  any count (0 gives 0.0) whose bytes fit 64 bits
 *   dtype    SWEEP_F32, SWEEP_BF16 or SWEEP_FP8_E4M3
 *   waves_per_cu  4..32, multiple of 4
 *   sum      host, receives the result
 *   out      host, may be NULL; receives timing, grid and byte counts
 *            (issued_bytes = payload bytes; checksums are 0)
 * NaN inputs propagate to the result.  Errors: SWEEP_EINVAL, SWEEP_EALIGN,
 * SWEEP_EHIP. */
int sweep_reduce_fp(const void* payload, size_t n_elems, int dtype,
                    int waves_per_cu, const sweep_opts_t* opt, double* sum,
                    sweep_result_t* out);

/* Unloaded load latency (Section 4.1, latency ladder): one lane of one
 * wave follows the dependent chain idx <- chain[idx] (32-bit word indices)
 * for `warm_hops` untimed and then `hops` timed hops, so exactly one load is
 * in flight at a time.  The first `n_samples` timed hops are also timed one
 * by one in shader-clock cycles and written to `samples`.
 *   chain        device, 16-byte aligned, `bytes` < 4 GiB, multiple of 4;
 *                every reachable word must hold an index < bytes / 4
 *   start        first index (< bytes / 4)
 *   cache_policy SWEEP_CACHE_* of the chasing loads (default = may hit the
 *                vector L1, bypass_l1 = .cg analogue)
 *   samples      device, n_samples u32, or NULL with n_samples 0
 *   n_samples    0..4096, <= hops
 * Synchronous on `stream`.  Errors: SWEEP_EINVAL, SWEEP_EALIGN, SWEEP_EHIP. */
int sweep_chase(const void* chain, size_t bytes, uint32_t start,
                uint32_t warm_hops, uint32_t hops, int cache_policy,
                uint32_t* samples, uint32_t n_samples, void* stream,
                sweep_chase_t* out);

/* Streaming read by a subset of the XCDs (no passage of the paper defines
 * it; it locates the ceiling the K sweep's plateau meets on MI355X, which
 * the paper's single-die view leaves open).  The launch has the shape of
 * the full-grid plain cell, num_cus * waves_per_cu / 4 workgroups of four
 * waves, pinned like sweep_plain.  A workgroup works only if the bit of
 * its XCD (read from HW_REG_XCC_ID) is set in xcd_mask; the others return
 * at once.  The dispatcher deals workgroups to the eight XCDs in turn, so
 * every round of eight workgroups puts one on each XCD, and the active
 * waves are numbered densely by (round, rank of their XCD in the mask).
 * Assumes one MI355X partition of eight XCDs.  The active waves run the
 * plain loop with K = 8 loads of 16-byte vectors, adjacent
 * segments, over groups dealt round robin, reading the first
 * n_act * groups * 512 vectors of the buffer once, with
 * groups = floor((bytes / 16) / (n_act * 512)).  Every active wave's record
 * carries its XCC_ID, so a caller can check that active wave w ran on the
 * XCD of rank (w / 4) mod popcount(mask) in the mask.
 *   xcd_mask      1..255
 *   waves_per_cu  as sweep_plain (4..32, a multiple of 4)
 *   opt           cache_policy, stream, pin_occupancy, wave_out (n_act
 *                 records, with wave_out_cap) are read; the rest is ignored
 * out: as sweep_plain; waves = n_act active waves, target = issued loads.
 * After the launch (outside its timed window) the library checks every
 * active wave's record: present, and from the XCD its number names.
 * Errors: SWEEP_EINVAL (mask, policy, size below one group per active
 * wave), SWEEP_EALIGN, SWEEP_EOCCUPANCY, SWEEP_EHIP, SWEEP_ENOMEM,
 * SWEEP_ENODEV (the placement check failed: workgroups were not dealt one
 * per XCD in each round of eight, so the read is not the one described). */
int sweep_xcd_subset(const void* buf, size_t bytes, int waves_per_cu, uint32_t xcd_mask,
                     const sweep_opts_t* opt, sweep_result_t* out);

/* Static split weighted per XCD (no passage of the paper defines it; the
 * method gives every wave an equal share, and this measures what unequal
 * service across XCDs costs that rule).  Same launch shape and loop as
 * sweep_xcd_subset, but XCD x (read from HW_REG_XCC_ID) owns a contiguous
 * share of floor(total * weights[x] / sum(weights)) groups, total =
 * floor((bytes / 16) / 512), dealt round robin over its own grid / 8 * 4
 * waves; the shares start at group 0 and follow each other in XCD order,
 * so the read covers the first sum(shares) * 512 vectors once.  XCDs whose
 * share is 0 return at once.  Active waves are numbered (rank of the XCD
 * among those with a share) * (waves per XCD) + (wave within the XCD), so
 * wave_out record i belongs to the XCD of rank i / (waves per XCD).
 *   weights       host array of 8 finite, non-negative weights, not all 0
 *   opt           as sweep_xcd_subset
 * out: as sweep_plain; iters_min / iters_max are the per-wave group counts
 * over the XCDs with a share.  Errors as sweep_xcd_subset. */
int sweep_xcd_split(const void* buf, size_t bytes, int waves_per_cu, const double* weights,
                    const sweep_opts_t* opt, sweep_result_t* out);

/* Dependent-chain walkers on several XCDs at once: the latency probe of
 * Section 4.1 resolved by XCD.  The paper's probe ran on one SM, so it
 * could not separate near and far paths; on MI355X every XCD has its own
 * L2 and its own route to the shared last-level cache and HBM.
 * Launches `n_walkers` workgroups of one wave; lane 0 of workgroup b
 * follows the chain from starts[b] (host array of n_walkers word indices)
 * for `warm_hops` untimed and `hops` timed dependent loads, as sweep_chase
 * does without samples.  The dispatcher deals workgroups to the XCDs in
 * turn; out[b].xcc_id is the XCD walker b ran on (HW_REG_XCC_ID).  With
 * the walkers spread along the chain they touch different lines, and with
 * at most 64 loads in flight the memory system is unloaded.
 *   n_walkers  1..64;  out: host array of n_walkers results
 * Synchronous on `stream`.  Errors: SWEEP_EINVAL, SWEEP_EALIGN, SWEEP_EHIP. */
int sweep_chase_walkers(const void* chain, size_t bytes, const uint32_t* starts,
                        int n_walkers, uint32_t warm_hops, uint32_t hops,
                        int cache_policy, void* stream, sweep_walker_t* out);

/* Text of an error code. */
const char* sweep_strerror(int code);

/* Text of the calling thread's last error (empty string if none). */
const char* sweep_last_error(void);

/* Library version string. */
const char* sweep_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ILPSWEEP_H */
