// Device-side descriptors shared by the host runtime (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace xs {

constexpr int kMaxTileBlocks = 32; // 256-clone blocks per workgroup tile
constexpr uint32_t kInitSweep = 0xFFFFFFFFu;

// One instance of a batched run as the kernels see it. Lives in device memory; the host fills
// the constant part, the kernels update the control part.
struct InstDev {
    // tables (device pointers owned by the instance)
    const uint4 *rec;        // [n] 16-byte records in step order: u16 LDS rows {i, a1, b1, a2, b2,
                             // a3, b3} of the spin and its partners, then meta = i | jbits << 13
    const int32_t *step_off; // [n_steps + 1] schedule steps (independent sets, run in order)
    const uint2 *tri;        // [n] triplets: x = a | b << 16, y = c | j << 16 (j = 1 <=> J = -1)
    const uint4 *grec;       // [n] records with row offsets for this tiling (global-record kernels)
    const uint16_t *rowmap;  // [n] LDS row of each spin, or null for row = spin
    // caller buffers
    uint64_t *state;         // [n][n_words]
    int32_t *first_hit;      // [n_clones]
    int32_t *energy;         // [n_clones] or null
    int8_t *solved;          // [n] device staging for the winner's spins
    // constants
    uint32_t n, n_words, n_steps, tile_blocks, log2_tile_blocks;
    uint32_t inst_id, thr, seed_lo, seed_hi;
    uint32_t flags, t_start, t_stop, chunk;
    // control (mutable)
    uint32_t t_cur;   // next sweep to run
    uint32_t done;    // nonzero once the run of this instance ended
    uint32_t hit;     // nonzero once some clone was seen in a ground state
    int32_t tts;      // min first_hit (final pass)
    int32_t winner;   // lowest clone with first_hit == tts (final pass)
    uint32_t wg_threads;  // workgroup size of this instance's chunk launches (host side)
    uint32_t track;       // nonzero once a chunk had to be replayed: later chunks test every sweep
    uint32_t col_bytes;   // task column width of this instance's launches (host side)
    uint32_t rec_global;  // records read from global memory (host side: selects the kernel)
    uint32_t thr0;        // w0 threshold: k = 0 spins flip iff the draw is below it (0: never)
    // persistent work-queue launches (qg_persist)
    uint32_t tile0, ntiles;  // this instance's tiles: tile list entries tile0 .. tile0 + ntiles - 1
    uint32_t arrived;        // tiles that finished the current chunk
    uint32_t epoch_left;     // chunks this instance may still run in the current launch
    uint32_t ring_off;       // first ring slot of its tiles in the current launch (set-up only)
    // Gauge (host decides j0 before the tables are attached; persistent launches only): with
    // j0 = 1 the state holds x_i ^ g_i from the start of the chunks to their end (gauge[n] = g,
    // 0 or 1) and every record's coupling bits are 0 (each J_t is +1 in that gauge).
    const uint8_t *gauge;
    uint32_t j0;
    // Cross-sweep body (records in global memory, w0 = 0 only; null: none): records with row
    // offsets for this tiling in body order (meta bit 12: the spin's update runs in the
    // iteration after its sweep's) and the step offsets of one iteration (n_bsteps steps).
    // Untracked chunks run iterations of the body; tracked sweeps and replays the plain steps.
    const uint4 *bgrec;
    const int32_t *bstep_off;
    uint32_t n_bsteps;
};

// Work queue of a persistent launch: tickets (head) are taken by workgroups, slots (tail) are
// reserved by pushes; a slot holds (launch tag << 32) | tile index once published.
struct QueueDev {
    uint64_t *ring;     // [cap] slots (tag 0: never written)
    uint32_t cap;       // slots: at least every push of one launch
    uint32_t head;      // tickets taken
    uint32_t tail;      // slots reserved
    uint32_t live;      // instances still running chunks in this launch
    uint32_t finished;  // set once live is 0 (nothing more is pushed) or a wait gave up
    uint32_t error;     // set if a workgroup's wait for its slot reached the time limit
    uint32_t active;    // instances not done (read by the host after each launch)
    uint32_t pad;
    uint64_t wait_limit;  // wall-clock ticks a workgroup waits for its slot before giving up
};

}  // namespace xs

// Launch wrappers implemented in kernels.hip (C++ linkage, internal to the library).
namespace xs {
hipError_t launch_init(InstDev *d_inst, const InstDev &h_inst, hipStream_t s);
// threads: 64, 128, 256, 512 or 1024, at least 8 * tile_blocks of every tile it runs;
// col_bytes: 4, 8 or 16 bytes of a spin row per task; rec_global: every tile's instance has
// grec set (records in global memory), else records are staged in LDS; met: every tile's
// instance has thr0 > 0 (w0 rule, no ground-state tracking).
hipError_t launch_chunk(InstDev *d_insts, const uint2 *d_tiles, int n_tiles, int threads,
                        int col_bytes, bool rec_global, bool met, size_t lds_bytes,
                        hipStream_t s);
hipError_t launch_decide(InstDev *d_insts, int count, uint32_t *d_active, hipStream_t s);
// The final pass (energies, end-sweep ground states, TTS, winner, its spins) of the count
// consecutive descriptors at d_insts; max_words and max_n bound their n_words and n.
hipError_t launch_final(InstDev *d_insts, int count, uint32_t max_words, uint32_t max_n,
                        hipStream_t s);
size_t chunk_lds_bytes(uint32_t n, uint32_t tile_blocks, bool rec_global, bool met);
// Persistent work-queue launches. A run clears the ring once (queue_clear); each launch then
// runs a one-workgroup set-up (queue_setup: the tiles of every unfinished instance in tile-list
// order, each instance allowed epoch_chunks chunks) and the persistent kernel (queue_run):
// `grid` workgroups of `threads` threads pop tiles, run one chunk of each, and the last tile
// of an instance's chunk decides (advance, end at the budget or the first ground state) and
// pushes the instance's tiles again while it may run more chunks. Every instance's col_bytes
// must be 8 or 16 and threads at least 8 * its tile_blocks; met as for launch_chunk.
// d_order: instance indices in tile-list order; gen: tag of this launch (> 0, increasing).
hipError_t launch_queue_clear(uint64_t *ring, uint32_t cap, hipStream_t s);
// Flip the state rows with g_i = 1 of every descriptor that has a gauge table (count
// consecutive descriptors; max_pieces bounds n * n_words / 2): the state enters its gauge
// before the chunks of a persistent run and leaves it before the final pass.
hipError_t launch_gauge_flip(InstDev *d_insts, int count, uint64_t max_pieces, hipStream_t s);
hipError_t launch_queue_setup(InstDev *d_insts, int count, const uint32_t *d_order,
                              const uint2 *d_tiles, uint32_t n_tiles, QueueDev *d_q,
                              uint32_t gen, uint32_t epoch_chunks, hipStream_t s);
hipError_t launch_queue_run(InstDev *d_insts, const uint2 *d_tiles, QueueDev *d_q, uint32_t gen,
                            int threads, bool met, size_t lds_bytes, int grid, hipStream_t s);
// Workgroups of the persistent kernel that fit on one CU at once.
hipError_t queue_blocks_per_cu(int threads, bool met, size_t lds_bytes, int *blocks);
// The no-allocation entry point's device scratch on the current device: its device address
// (looked up once per device with hipGetSymbolAddress, with that device current) and size.
hipError_t noalloc_scratch(uint8_t **ptr, size_t *bytes);
}  // namespace xs
