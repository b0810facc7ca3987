/*
 * xorsat.h -- C ABI of the MI355X quasi-greedy many-clone 3-XORSAT solver.
 *
 * Paper: Bernaschi et al., "How we are leading a 3-XORSAT challenge: from the energy landscape
 * to the algorithm and its efficient implementation on GPUs" (arXiv 2102.09510).
 *
 * The library runs the paper's quasi-greedy (QG) single-spin-flip dynamics on many clones of
 * one instance of H = -sum_t J_t s_a s_b s_c (Eq. (1); the paper has J_t = +1), 64 clones per
 * 64-bit word, on an AMD gfx950 GPU. All arithmetic is integer and bit-exact: for the same
 * instance, seed and configuration every result is reproducible to the bit, whatever tiling,
 * batching or serving mode produced it.
 *
 * Conventions
 *   - Every call returns xs_status; XS_OK is 0. No exception crosses the ABI. On an error
 *     xs_last_error() returns a message for the calling thread.
 *   - Spins: s = +1 or -1. Bits: x = 1 <=> s = -1. Clone c lives in bit (c & 63) of 64-bit word
 *     (c >> 6); the 32 clones c with the same c >> 5 form a "group" that shares every random
 *     number (Section "Basic information about the GPU implementation": one random number per
 *     32-clone word).
 *   - Device pointers are plain HIP device addresses (for example torch's data_ptr()). The
 *     stream argument is a hipStream_t passed as void* (NULL = the default stream).
 *   - Structs that may grow carry struct_size; set it to sizeof(the struct).
 */
#ifndef XORSAT_H
#define XORSAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XS_ABI_VERSION 2

typedef int32_t xs_status;
#define XS_OK 0
#define XS_EINVAL 1      /* an argument or an instance breaks a stated rule */
#define XS_ENOMEM 2      /* host or device allocation failed (or a thread could not start) */
#define XS_EDEVICE 3     /* a HIP call failed (the message names it) */
#define XS_EAGAIN 4      /* the server cannot admit the request now */
#define XS_ENOTFOUND 5   /* unknown ticket */
#define XS_ECANCELED 6   /* the request was cancelled */

/* Largest supported instance: the per-workgroup tables keep LDS byte offsets in 16 bits. */
#define XS_MAX_N 2048
/* Clone counts are multiples of this (one random-number block: 8 groups of 32 clones). */
#define XS_CLONE_QUANTUM 256
/* Largest clone count: clone indices (the winner) are int32 with INT32_MAX meaning none. */
#define XS_MAX_CLONES 0x7FFFFF00u

/* Run flags (xs_run_config.flags). */
#define XS_STOP_ON_FIRST 0x1u /* stop at the end of the first chunk after which some clone
                                 is in a ground state (E = -N) */
#define XS_RESUME 0x2u        /* state already holds the start configuration (checkpoint)     */
#define XS_PLACE_ROWS 0x4u    /* build the LDS row placement of tiles under eight blocks with
                                 its full search, even for a short run (speed only; a host
                                 cost of about 0.8 ms per spin, once per instance and tiling,
                                 kept for later runs). Without it, runs of fewer than 2^32
                                 clone-sweeps use a placement only if one already exists, and
                                 longer runs build one with a search sized to the run. */
#define XS_PER_CHUNK 0x8u     /* launch every chunk separately (one launch per launch shape,
                                 then a decision kernel) instead of the persistent work-queue
                                 launch; speed only. A batch runs per chunk if any of its
                                 configs sets it. */
#define XS_ONE_SWEEP_STEPS 0x10u /* run every sweep on its own steps: no overlap of the end of
                                 one sweep with the start of the next (which chunks without
                                 ground-state tracking otherwise use where the schedule has
                                 such a form); speed only, the results are identical. */

typedef struct xs_instance xs_instance;

/* ABI version the library was built with (XS_ABI_VERSION). */
int32_t xs_abi_version(void);
/* Name of a status code ("XS_EINVAL", ...). Static storage. */
const char *xs_status_str(xs_status status);
/* Message of the last failed call on this thread ("" if none). Valid until the next call. */
const char *xs_last_error(void);

/*
 * Load an instance (Section "The model and its energy landscape"): n spins, m = n triplets,
 * tri[3*t .. 3*t+2] the 0-based spins of triplet t, J[t] = +1 or -1 its coupling. Every spin
 * must appear in exactly three triplets, the three spins of a triplet must differ, and
 * 4 <= n <= XS_MAX_N; otherwise XS_EINVAL. Repeated triplets are allowed (each is counted).
 * The spins are partitioned once, on the host, into independent sets of at most colour_cap
 * spins (Supplementary Material, "Details on the GPU implementation": greedy repeated scans,
 * sets of 32 were best; 0 selects 32). The partition fixes the update order and therefore the
 * trajectories, so it is part of the instance. The library copies tri and J; the caller keeps
 * ownership of its arrays. Device tables are uploaded on first use.
 */
xs_status xs_instance_create(int32_t n, int32_t m, const int32_t *tri, const int8_t *J,
                             int32_t colour_cap, xs_instance **out);
void xs_instance_destroy(xs_instance *inst);

typedef struct {
    int32_t n;          /* spins (= triplets) */
    int32_t n_classes;  /* independent sets in the partition */
    int32_t colour_cap; /* largest allowed set */
    int32_t max_class;  /* largest actual set */
    int32_t n_levels;   /* parallel steps of a sweep on the device (<= n_classes): each spin one
                           step after the latest earlier spin in update order that shares a
                           triplet with it, which reproduces the sequential sweep exactly */
    int32_t max_level;  /* most spins in one step */
} xs_instance_info;

xs_status xs_instance_get_info(const xs_instance *inst, xs_instance_info *info);
/* The update order: perm[n] (spins set by set) and class_off[n_classes + 1] (set k holds
 * positions class_off[k] .. class_off[k+1]-1). Host arrays owned by the caller. */
xs_status xs_instance_get_partition(const xs_instance *inst, int32_t *perm, int32_t *class_off);
/* The execution schedule the kernels use for launches whose steps hold at most step_cap spins
 * (0: no limit): order[n] (spins step by step) and step_off[*n_steps + 1]. Each spin sits in a
 * later step than every spin before it in the update order that shares a triplet with it, so
 * running the steps in order reproduces the sequential sweep exactly. step_off needs room for
 * n + 1 entries. Host arrays owned by the caller. */
xs_status xs_instance_get_schedule(const xs_instance *inst, uint32_t step_cap, int32_t *order,
                                   int32_t *step_off, int32_t *n_steps);
/* The cross-sweep body of the schedule for steps of at most step_cap spins (1 .. 65535), which
 * chunks without ground-state tracking run when records are read from global memory. Sweep t
 * of spin j runs in step s(j) of iteration t + late[j], where s(j) is the step of j's position
 * in order[n] (steps step_off[0 .. *n_steps]); iteration k runs its steps in order, and the
 * iterations of a chunk [t0, t1) are t0 .. t1. Running them reproduces the sequential sweeps
 * exactly (rules in the source of make_body). XS_ENOTFOUND if the instance has no body for
 * this cap (its sweeps then run one after another). step_off needs room for n + 1 entries and
 * late for n (0 or 1, per spin). Host arrays owned by the caller. */
xs_status xs_instance_get_body(const xs_instance *inst, uint32_t step_cap, int32_t *order,
                               int32_t *step_off, uint8_t *late, int32_t *n_steps);

/*
 * Run configuration. The dynamics (Section "The quasi-greedy algorithm"): a sweep visits the
 * spins set by set in partition order; a spin in k unsatisfied triplets flips with
 * probability w_k, w2 = w3 = 1, w1 = accept_thr / 65536 (the paper uses w1 = 0.055,
 * accept_thr = 3604) and w0 = accept_thr0 / 65536 (0 for the quasi-greedy rule; w0 = w1^3 is
 * the Metropolis rule of the pseudo-temperature T = -2 / ln w1 that the same section relates it
 * to). A k = 1 spin flips iff its 16-bit draw d < accept_thr, a k = 0 spin iff d < accept_thr0.
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed low, seed high):
 *   start bit of spin i, clone c: bit (c & 31) of philox(i, 0xFFFFFFFF, g >> 2, id)[g & 3];
 *   draw of spin i, sweep t, group g = c >> 5:
 *       (philox(i, t, g >> 3, id)[(g & 7) >> 1] >> (16 * (g & 1))) & 0xFFFF.
 */
typedef struct {
    uint32_t struct_size;
    uint32_t instance_id;  /* part of every random counter; keeps instances independent */
    uint64_t seed;         /* Philox key */
    uint32_t n_clones;     /* > 0, multiple of XS_CLONE_QUANTUM, <= XS_MAX_CLONES */
    uint32_t accept_thr;   /* w1 threshold, 0 .. 65536 */
    uint32_t flags;        /* XS_STOP_ON_FIRST | XS_RESUME | XS_PLACE_ROWS | XS_PER_CHUNK |
                              XS_ONE_SWEEP_STEPS */
    uint32_t max_sweeps;   /* sweep budget of this call (0 = only check the start state) */
    uint32_t start_sweep;  /* absolute index of the first sweep (for resumed runs) */
    uint32_t chunk_sweeps; /* sweeps between stop checks, K (0 = 100, as in the paper) */
    uint32_t tile_blocks;  /* clone blocks of 256 per workgroup (power of two <= 32, dividing
                              n_clones / 256, n * tile_blocks <= 2048); 0 = chosen by the
                              library. Changes speed only, never results. */
    uint32_t wg_threads;   /* threads per workgroup: 64 .. 1024, a power of two, at least
                              8 * tile_blocks; 0 = chosen by the library. Speed only. */
    uint32_t col_bytes;    /* bytes of a spin row one thread updates per step: 4, 8 or 16
                              (32, 64 or 128 clones); 0 = chosen by the library. Speed only. */
    uint32_t rec_global;   /* where a workgroup reads the per-spin neighbour records: 1 = global
                              memory (through the caches; frees LDS for clone state), 2 = LDS,
                              0 = chosen by the library. Speed only. */
    uint32_t accept_thr0;  /* w0 threshold, 0 .. 65536 (0: quasi-greedy). With accept_thr0 > 0 a
                              ground state is not absorbing: no sweep is tested, first_hit is
                              end_sweep for a clone whose end configuration has E = -N and -1
                              otherwise, and XS_STOP_ON_FIRST is rejected (XS_EINVAL). */
    uint32_t reserved;     /* must be 0 */
} xs_run_config;

/*
 * Caller-owned buffers of one run.
 *   state      device, uint64 [n][n_clones / 64] (spin-major): bit b of state[i*W + w] is x_i of
 *              clone 64*w + b. Written with the start configuration unless XS_RESUME; holds the
 *              configuration at the end sweep on return. Required.
 *   first_hit  device, int32 [n_clones]: smallest sweep index t in [start_sweep, end_sweep] at
 *              which the clone's configuration (before sweep t) has E = -N, else -1. Required.
 *   energy     device, int32 [n_clones] or NULL: E = 2U - N at the end sweep.
 *   solved     host, int8 [n] or NULL: spins (+1/-1) of the winning clone (unchanged if none).
 * The device buffers must be addressable by the kernels (device or managed memory, or host
 * memory mapped at the same address); anything else is rejected with XS_EINVAL before any
 * launch.
 */
typedef struct {
    uint64_t *state;
    int32_t *first_hit;
    int32_t *energy;
    int8_t *solved;
} xs_run_buffers;

typedef struct {
    int64_t tts_sweeps;          /* min over clones of first_hit (Section "Numerical results":
                                    a run's TTS is its fastest clone), -1 if none */
    int32_t winner_clone;        /* lowest clone index attaining tts_sweeps, -1 if none */
    uint32_t end_sweep;          /* absolute sweep index at which the run stopped */
    uint32_t sweeps_done;        /* end_sweep - start_sweep */
    uint32_t tile_blocks;        /* tiling used (result-neutral) */
    uint32_t wg_threads;         /* workgroup size used (result-neutral) */
    uint32_t col_bytes;          /* task column width used (result-neutral) */
    uint32_t rec_global;         /* 1 if records were read from global memory (result-neutral) */
    uint32_t persistent;         /* 1 if the run used persistent work-queue launches, 0 if a
                                    launch per chunk (result-neutral) */
    uint64_t clone_spin_updates; /* n_clones * n * sweeps_done */
    double seconds;              /* wall time of the call */
} xs_run_result;

/*
 * Run one instance: draw the start configuration (unless XS_RESUME), then sweep in chunks of
 * chunk_sweeps until max_sweeps are done or, with XS_STOP_ON_FIRST, until the end of the first
 * chunk after which some clone is in a ground state (E = -N). With w0 = 0 a ground state is never left
 * (Section "The quasi-greedy algorithm", property (iii)), so the exact first sweep of every
 * clone is known and the chunk length changes only end_sweep, never first hits, TTS, winner
 * or solved configuration. Work is ordered on `stream`; the call returns after it finished.
 * XS_EINVAL for bad sizes, XS_EDEVICE for a HIP failure.
 */
xs_status xs_run(const xs_instance *inst, const xs_run_config *cfg, const xs_run_buffers *bufs,
                 void *stream, xs_run_result *result);

/*
 * Run `count` instances together (uneven sizes allowed): every chunk is one launch over the
 * workgroup tiles of all unfinished instances. Each instance's results are identical to
 * xs_run with the same instance, configuration and buffers. Buffers must not overlap.
 */
xs_status xs_run_batch(int32_t count, const xs_instance *const *insts, const xs_run_config *cfgs,
                       const xs_run_buffers *bufs, void *stream, xs_run_result *results);

/*
 * xs_run_batch for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). Same arguments, same checks and
 * bit-identical results and buffers; the differences:
 *   - everything the call needs on the device besides the caller's buffers (instance
 *     descriptors, the tile list, the running-instance counter, the winners' spins and the
 *     instances' tables, copied in by each call) lives in one library-owned scratch array of
 *     XS_NOALLOC_SCRATCH_BYTES per device, set aside when the library is loaded and held until
 *     the process ends; a batch that needs more is rejected with XS_EINVAL (the message gives
 *     the bytes needed) before anything is launched;
 *   - no device memory is allocated or freed and no graph, event or stream is created: the
 *     chunk loop is launched directly on `stream`, and these calls are not timed by
 *     xs_profile_enable (host bookkeeping still uses the C++ heap);
 *   - every such call on one device shares that device's scratch, so calls that overlap on one
 *     device (from several threads, or on several streams) race: serialise them. The call
 *     synchronises `stream` before it returns, like xs_run_batch.
 */
#define XS_NOALLOC_SCRATCH_BYTES 8388608u /* 8 MiB */
xs_status xs_run_batch_noalloc(int32_t count, const xs_instance *const *insts,
                               const xs_run_config *cfgs, const xs_run_buffers *bufs,
                               void *stream, xs_run_result *results);

/*
 * The same batch without blocking the caller: the arguments are checked and copied, the run is
 * driven from a library thread on `stream` (current device of the caller), and xs_wait blocks
 * until it ended, fills results[] and releases the handle (call it exactly once). Until then the
 * instances, buffers and results[] must stay alive and untouched, and the caller must not use
 * `stream`. Errors found before the run starts are returned here (no handle); errors during
 * the run are returned by xs_wait, with the message in its thread's xs_last_error.
 */
typedef struct xs_pending xs_pending;
xs_status xs_run_batch_async(int32_t count, const xs_instance *const *insts,
                             const xs_run_config *cfgs, const xs_run_buffers *bufs, void *stream,
                             xs_run_result *results, xs_pending **out);
xs_status xs_wait(xs_pending *pending);

/*
 * Server: continuous batching of many runs on one device. Requests are queued by
 * xs_server_submit; each xs_server_step admits queued requests in arrival order while their
 * device footprint (state n*n_clones/8 bytes, first_hit and energy 4*n_clones bytes each, n
 * bytes of solved spins) fits the server's memory budget and resident limit, runs one chunk of
 * sweeps (each request's own chunk_sweeps) over every resident request in the same launches,
 * and completes the requests that ended: their final pass runs, results are copied into the
 * host buffers given at submission and their device memory is released. Admission, tiling and
 * the mix of other requests never change a request's results: each one is bit-identical to
 * xs_run with the same instance and configuration (its random numbers are keyed by its own
 * seed and instance_id). The instance must stay alive until the request completed. Not
 * thread-safe: drive one server from one thread. XS_RESUME is not supported here.
 */
typedef struct xs_server xs_server;

typedef struct {
    uint32_t struct_size;
    uint32_t max_resident;     /* requests resident at once (0 = no limit besides memory) */
    uint64_t hbm_budget_bytes; /* device bytes the resident requests may hold; reserved as one
                                  allocation at the first admission and sub-allocated from then
                                  on (no device allocation while serving) */
    uint32_t max_pending;      /* queued, not yet admitted requests (0 = no limit); a submit
                                  beyond it returns XS_EAGAIN (back-pressure) */
    uint32_t reserved;         /* must be 0 */
} xs_server_config;

/* Host buffers filled when a request completes; each may be NULL. */
typedef struct {
    uint64_t *state;    /* [n][n_clones/64] final configuration */
    int32_t *first_hit; /* [n_clones] */
    int32_t *energy;    /* [n_clones] */
    int8_t *solved;     /* [n] spins of the winner (unchanged if no clone hit) */
} xs_server_outputs;

typedef struct {
    uint64_t ticket;
    xs_status status;      /* XS_OK, XS_ECANCELED, or XS_ENOMEM if it can never fit the budget */
    xs_run_result result;  /* result.seconds = submission to completion */
    double queued_s;       /* submission to admission */
} xs_server_completion;

typedef struct {
    uint64_t steps, admitted, completed, pending, resident;
    uint64_t clone_spin_updates; /* sweeps run by all requests so far */
    uint64_t bytes_in_use;       /* device bytes held by resident requests */
    double step_seconds;         /* wall time spent inside xs_server_step */
} xs_server_stats;

xs_status xs_server_create(const xs_server_config *cfg, void *stream, xs_server **out);
/* Releases every request's device memory; pending and resident requests are dropped. */
void xs_server_destroy(xs_server *srv);
/* Queue a request; the configuration and output pointers are copied, the instance is not.
 * XS_EINVAL for an invalid configuration, XS_EAGAIN (nothing queued) while max_pending requests
 * wait for admission. */
xs_status xs_server_submit(xs_server *srv, const xs_instance *inst, const xs_run_config *cfg,
                           const xs_server_outputs *outs, uint64_t *ticket);
/* One scheduling step (see above). n_active receives resident + pending requests after it. */
xs_status xs_server_step(xs_server *srv, int32_t *n_active);
/* Move up to cap completions (oldest first) into done[]; n_done receives how many. */
xs_status xs_server_poll(xs_server *srv, xs_server_completion *done, int32_t cap,
                         int32_t *n_done);
/* Cancel a queued or resident request (it completes with XS_ECANCELED at the next step).
 * XS_ENOTFOUND if the ticket is unknown or already completed. */
xs_status xs_server_cancel(xs_server *srv, uint64_t ticket);
xs_status xs_server_get_stats(const xs_server *srv, xs_server_stats *out);

/*
 * Autotuner of the result-neutral launch knobs (tile_blocks: clones per workgroup, in blocks of
 * 256; wg_threads: threads per workgroup; col_bytes: clones one thread updates per step, which
 * with the class size sets how a colour class is spread over the threads). It times the valid
 * combinations with short budget runs of `count` copies of
 * `inst` (fewer if their state would exceed 2 GiB) on `stream`, using HIP events around the
 * sweep launches, and records the fastest combination for workloads of the same N (rounded up to a
 * power of two), clone count and batch size (rounded up to a power of two, at most 64). Later
 * runs whose config leaves every knob 0 use the recorded choice. Allocates and frees its own
 * device buffers. Results of any run never depend on these knobs.
 */
#define XS_TUNE_MAX_TRIALS 64
typedef struct {
    uint32_t tile_blocks, wg_threads, col_bytes, rec_global;
    double updates_per_ns; /* sweep-kernel rate of this trial */
} xs_tune_trial;

typedef struct {
    uint32_t tile_blocks, wg_threads, col_bytes, rec_global; /* the fastest choice */
    double updates_per_ns;
    int32_t n_trials;
    xs_tune_trial trials[XS_TUNE_MAX_TRIALS];
} xs_tune_result;

xs_status xs_autotune(const xs_instance *inst, uint32_t n_clones, int32_t count, void *stream,
                      xs_tune_result *out);
/* Write / read the recorded choices as text ("n_bucket clones count_bucket B T CW GR rate"
 * lines, GR = 1 for records in global memory, 2 for LDS).
 * Loading adds to (and overrides) the table in memory. */
xs_status xs_tune_save(const char *path);
xs_status xs_tune_load(const char *path);
/* Forget every recorded choice. */
xs_status xs_tune_clear(void);

/*
 * Launch timing of the sweep kernel, for measurement tools. When enabled, the library records
 * a pair of HIP events on the run's stream around every sweep-chunk launch and adds the
 * elapsed times once the run has synchronised. Counters are process-wide.
 */
typedef struct {
    uint64_t launches;           /* sweep-chunk launches timed */
    double total_ms;             /* sum of their durations */
    uint64_t clone_spin_updates; /* updates those launches performed */
} xs_kernel_stats;

xs_status xs_profile_enable(int32_t on);
/* Copy the counters; reset them to zero if reset != 0. */
xs_status xs_profile_read(xs_kernel_stats *out, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* XORSAT_H */
