// Host-side internals shared by the run driver (api.cpp) and the server (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/xorsat.h"
#include "xs_internal.h"

namespace xsh {

// One execution schedule of the sweep on a device: records in schedule order and step offsets.
struct DevSched {
    uint4 *rec = nullptr;              // [n] records (LDS rows of the spins, meta)
    int32_t *off = nullptr;            // [steps + 1]
    uint16_t *rowmap = nullptr;        // [n] LDS row of each spin (null: identity)
    uint32_t steps = 0;
    std::map<uint32_t, uint4 *> grec;  // records as row offsets, per tile_blocks
    // cross-sweep body (HostSched::border): step offsets and records as row offsets
    int32_t *boff = nullptr;           // [bsteps + 1], null: no body
    uint32_t bsteps = 0;
    std::map<uint32_t, uint4 *> bgrec;  // per tile_blocks
};

struct DeviceTables {
    uint2 *tri = nullptr;
    uint8_t *gauge = nullptr;  // [n] gauge bits (0 or 1), uploaded on first use
    std::map<uint32_t, DevSched> sched;  // per (step cap, row slots)
};

// The host side of a schedule: the update order regrouped into parallel steps.
struct HostSched {
    std::vector<int32_t> order;    // spins in schedule order
    std::vector<int32_t> off;      // [steps + 1]
    std::vector<uint16_t> rec;     // [n][8] records in schedule order
    std::vector<uint16_t> rowmap;  // [n] LDS row of each spin (empty: identity)
    int32_t max_step = 0;
    // Cross-sweep body (empty: none): the steps of one iteration of overlapped sweeps. Spins in
    // body order, its step offsets, and records as `rec` whose meta bit 12 marks a spin whose
    // update runs one iteration after its sweep's (see make_body).
    std::vector<int32_t> border, boff;
    std::vector<uint16_t> brec;
};


}  // namespace xsh

struct xs_instance {
    int32_t n = 0;
    int32_t cap = 32;
    std::vector<int32_t> tri;        // [n][3]
    std::vector<int8_t> J;           // [n]
    std::vector<int32_t> perm;       // update order
    std::vector<int32_t> class_off;  // [n_classes + 1]
    // Caches filled on first use (under mu), so they may change behind a const instance.
    mutable std::map<uint32_t, xsh::HostSched> sched;  // per (step cap, row slots)
    std::vector<uint16_t> tri16;     // [n][4]: a, b, c, j
    int32_t max_class = 0;
    // Gauge bits g (g_a ^ g_b ^ g_c = [J_t = -1] for every triplet), found on first use (under
    // mu): state 0 = not tried, 1 = found, -1 = no such gauge (not every J_t can become +1).
    mutable std::vector<uint8_t> gauge;
    mutable int gauge_state = 0;
    mutable std::mutex mu;
    mutable std::map<int, xsh::DeviceTables> dev;  // per HIP device
};

// Return XS_EDEVICE (with the HIP message) from the enclosing function if a HIP call fails.
#define XS_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return xsh::fail(XS_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace xsh {

// A device allocation freed when the scope ends unless released (uploads that fail halfway
// leave nothing behind and nothing half-built).
struct DevAlloc {
    void *p = nullptr;
    DevAlloc() = default;
    DevAlloc(const DevAlloc &) = delete;
    DevAlloc &operator=(const DevAlloc &) = delete;
    ~DevAlloc() {
        if (p) (void)hipFree(p);
    }
    template <typename T> T *release() {
        T *q = static_cast<T *>(p);
        p = nullptr;
        return q;
    }
};

// Set the calling thread's last error message and return st.
xs_status fail(xs_status st, const char *fmt, ...);
// Run the body of a C entry point. Exceptions of the C++ library (a failed host allocation, a
// vector too long, a thread that cannot start) become XS_ENOMEM and a message: none crosses
// the C ABI.
template <class F>
xs_status guarded(F &&body) {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(XS_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(XS_ENOMEM, "host resource failure: %s", e.what());
    } catch (...) {
        return fail(XS_ENOMEM, "host resource failure");
    }
}
// Device tables of an instance on `device`, uploaded on first use.
xs_status ensure_tables(const xs_instance *I, int device, DeviceTables *out);
// Check a run configuration and its buffers (state buffer ignored if check_buffers is false).
xs_status validate_run(const xs_instance *I, const xs_run_config *cfg, const xs_run_buffers *b,
                       bool check_buffers);
// Fill the constant and initial control fields of a descriptor (tiling left to tile_instances).
void fill_desc(const xs_instance *I, const xs_run_config &c, const DeviceTables &t,
               uint64_t *state, int32_t *first_hit, int32_t *energy, xs::InstDev &d);

// One chunk launch per workgroup size over a list of tiles.
struct TileGroup {
    uint32_t threads, col_bytes, rec_global, met;
    size_t first, count, lds;
};
// After tiling: point every descriptor at its instance's schedule for the launch's step width
// (records, step offsets, and the global-memory records of its tiling if it reads records from
// global memory), built and uploaded on first use.
xs_status attach_tables(std::vector<xs::InstDev> &h, const xs_instance *const *insts, int count,
                        int device);
// Choose tiling for descriptors h[0..count) (explicit config knobs, then the tuned table, then
// the default rule), fill tile_blocks / log2 / wg_threads, and build the tile list and groups.
xs_status tile_instances(std::vector<xs::InstDev> &h, const xs_run_config *cfgs, int count,
                         std::vector<uint2> &tiles, std::vector<TileGroup> &groups);

}  // namespace xsh
