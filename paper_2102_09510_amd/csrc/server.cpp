// Continuous-batching server of the C ABI (xs_server_*): admission by device-memory footprint,
// one sweep chunk over all resident requests per step, completion and readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "../../include/xorsat.h"
#include "xs_host.h"

using xsh::fail;
using xsh::guarded;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    const xs_instance *inst = nullptr;
    xs_run_config cfg{};
    xs_server_outputs outs{};
    size_t bytes = 0;          // device footprint
    uint8_t *mem = nullptr;    // device memory while resident
    xs::InstDev desc{};        // descriptor, control fields carried across steps
    bool fresh = false;        // admitted, start configuration not drawn yet
    bool canceled = false;
    double t_submit = 0, t_admit = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// First-fit sub-allocator over one device allocation of the server's whole memory budget, so
// that admitting and completing requests never calls the device allocator. Free ranges are
// kept by offset and merged with their neighbours on release. Sizes are multiples of 256.
class DevicePool {
  public:
    ~DevicePool() {
        if (base_) (void)hipFree(base_);
    }
    // Allocate the budget on first use.
    xs_status reserve(size_t bytes) {
        if (base_) return XS_OK;
        XS_HIP(hipMalloc(&base_, bytes));
        size_ = bytes;
        free_[0] = bytes;
        return XS_OK;
    }
    // Offset of a free range of `bytes`, or false if none is large enough now.
    bool alloc(size_t bytes, uint8_t **out) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            *out = base_ + off;
            return true;
        }
        return false;
    }
    void release(uint8_t *p, size_t bytes) {
        size_t off = (size_t)(p - base_), len = bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }

  private:
    uint8_t *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

size_t footprint(const xs_instance *I, const xs_run_config &c) {
    const size_t n = (size_t)I->n, nc = c.n_clones;
    return align256(n * nc / 8) + 2 * align256(4 * nc) + align256(n);
}

}  // namespace

struct xs_server {
    xs_server_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t next_ticket = 1;
    std::deque<Request *> pending;
    std::vector<Request *> resident;
    std::deque<xs_server_completion> completed;
    xs_server_stats stats{};
    uint8_t *scratch = nullptr;  // descriptors | tiles | active counter | finished descriptors
    size_t scratch_bytes = 0;
    DevicePool pool;             // the resident requests' device memory

    ~xs_server() {
        for (Request *r : pending) delete r;
        for (Request *r : resident) delete r;
        if (scratch) (void)hipFree(scratch);
    }

    void complete(Request *r, xs_status st, const xs_run_result &res) {
        xs_server_completion c{};
        c.ticket = r->ticket;
        c.status = st;
        c.result = res;
        c.result.seconds = now_s() - r->t_submit;
        c.queued_s = r->t_admit > 0 ? r->t_admit - r->t_submit : c.result.seconds;
        completed.push_back(c);
        ++stats.completed;
    }

    void release(Request *r) {
        if (r->mem) {
            pool.release(r->mem, r->bytes);
            r->mem = nullptr;
            stats.bytes_in_use -= r->bytes;
        }
    }

    xs_status admit() {
        while (!pending.empty()) {
            Request *r = pending.front();
            if (r->canceled) {
                pending.pop_front();
                complete(r, XS_ECANCELED, xs_run_result{-1, -1, r->cfg.start_sweep, 0, 0, 0, 0, 0, 0, 0, 0});
                delete r;
                continue;
            }
            if (cfg.max_resident && resident.size() >= cfg.max_resident) break;
            if (r->bytes > cfg.hbm_budget_bytes) {  // can never fit
                pending.pop_front();
                complete(r, XS_ENOMEM, xs_run_result{-1, -1, r->cfg.start_sweep, 0, 0, 0, 0, 0, 0, 0, 0});
                delete r;
                continue;
            }
            xs_status st = pool.reserve(align256(cfg.hbm_budget_bytes));
            if (st != XS_OK) return st;
            if (!pool.alloc(r->bytes, &r->mem)) break;  // wait for memory to free up
            xsh::DeviceTables t;
            st = xsh::ensure_tables(r->inst, device, &t);
            if (st != XS_OK) {
                pool.release(r->mem, r->bytes);
                r->mem = nullptr;
                return st;
            }
            const size_t n = (size_t)r->inst->n, nc = r->cfg.n_clones;
            uint64_t *state = reinterpret_cast<uint64_t *>(r->mem);
            int32_t *fh = reinterpret_cast<int32_t *>(r->mem + align256(n * nc / 8));
            int32_t *en = reinterpret_cast<int32_t *>(r->mem + align256(n * nc / 8) +
                                                      align256(4 * nc));
            xsh::fill_desc(r->inst, r->cfg, t, state, fh, en, r->desc);
            r->desc.solved = reinterpret_cast<int8_t *>(r->mem + align256(n * nc / 8) +
                                                        2 * align256(4 * nc));
            r->fresh = true;
            r->t_admit = now_s();
            stats.bytes_in_use += r->bytes;
            ++stats.admitted;
            resident.push_back(r);
            pending.pop_front();
        }
        return XS_OK;
    }

    xs_status ensure_scratch(size_t bytes) {
        if (bytes <= scratch_bytes) return XS_OK;
        const size_t want = std::max(bytes, 2 * scratch_bytes);
        if (scratch) {
            XS_HIP(hipStreamSynchronize(stream));
            XS_HIP(hipFree(scratch));
            scratch = nullptr;
            scratch_bytes = 0;  // a failed allocation below leaves no stale size behind
        }
        XS_HIP(hipMalloc(&scratch, want));
        scratch_bytes = want;
        return XS_OK;
    }

    xs_status step(int32_t *n_active) {
        const double t0 = now_s();
        ++stats.steps;
        // Cancelled resident requests leave before the chunk.
        for (size_t k = 0; k < resident.size();) {
            Request *r = resident[k];
            if (!r->canceled) {
                ++k;
                continue;
            }
            xs_run_result res{-1, -1, r->desc.t_cur, r->desc.t_cur - r->desc.t_start, 0, 0, 0, 0,
                              0, (uint64_t)r->desc.n_words * 64 * r->desc.n *
                                  (r->desc.t_cur - r->desc.t_start),
                              0};
            release(r);
            complete(r, XS_ECANCELED, res);
            delete r;
            resident.erase(resident.begin() + k);
        }
        xs_status st = admit();
        if (st != XS_OK) return st;
        const int R = (int)resident.size();
        if (R > 0) {
            std::vector<xs::InstDev> h(R);
            std::vector<xs_run_config> cfgs(R);
            std::vector<uint32_t> t_before(R);
            for (int k = 0; k < R; ++k) {
                h[k] = resident[k]->desc;
                cfgs[k] = resident[k]->cfg;
                t_before[k] = h[k].t_cur;
            }
            std::vector<uint2> tiles;
            std::vector<xsh::TileGroup> groups;
            st = xsh::tile_instances(h, cfgs.data(), R, tiles, groups);
            if (st != XS_OK) return st;
            std::vector<const xs_instance *> insts(R);
            for (int k = 0; k < R; ++k) insts[k] = resident[k]->inst;
            st = xsh::attach_tables(h, insts.data(), R, device);
            if (st != XS_OK) return st;
            const size_t off_tiles = align256(sizeof(xs::InstDev) * R);
            const size_t off_active = off_tiles + align256(sizeof(uint2) * tiles.size());
            const size_t off_fin = off_active + 256;
            st = ensure_scratch(off_fin + align256(sizeof(xs::InstDev) * R));
            if (st != XS_OK) return st;
            xs::InstDev *d_inst = reinterpret_cast<xs::InstDev *>(scratch);
            uint2 *d_tiles = reinterpret_cast<uint2 *>(scratch + off_tiles);
            uint32_t *d_active = reinterpret_cast<uint32_t *>(scratch + off_active);
            xs::InstDev *d_fin = reinterpret_cast<xs::InstDev *>(scratch + off_fin);
            XS_HIP(hipMemcpyAsync(d_inst, h.data(), sizeof(xs::InstDev) * R,
                                  hipMemcpyHostToDevice, stream));
            XS_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(uint2) * tiles.size(),
                                  hipMemcpyHostToDevice, stream));
            for (int k = 0; k < R; ++k)
                if (resident[k]->fresh) {
                    XS_HIP(xs::launch_init(d_inst + k, h[k], stream));
                    resident[k]->fresh = false;
                }
            for (const xsh::TileGroup &g : groups)
                XS_HIP(xs::launch_chunk(d_inst, d_tiles + g.first, (int)g.count, (int)g.threads,
                                        (int)g.col_bytes, g.rec_global != 0, g.met != 0, g.lds,
                                        stream));
            XS_HIP(xs::launch_decide(d_inst, R, d_active, stream));
            XS_HIP(hipMemcpyAsync(h.data(), d_inst, sizeof(xs::InstDev) * R,
                                  hipMemcpyDeviceToHost, stream));
            XS_HIP(hipStreamSynchronize(stream));
            // The requests that ended in this chunk get their final pass (energies, TTS, winner,
            // solved spins) together: their descriptors are gathered into one array, so one
            // launch of each final kernel covers all of them, however many end at once.
            std::vector<int> fin;
            uint32_t fin_words = 0, fin_n = 0;
            for (int k = 0; k < R; ++k) {
                stats.clone_spin_updates +=
                    (uint64_t)h[k].n_words * 64 * h[k].n * (h[k].t_cur - t_before[k]);
                if (h[k].done) {
                    fin.push_back(k);
                    fin_words = std::max(fin_words, h[k].n_words);
                    fin_n = std::max(fin_n, h[k].n);
                }
            }
            if (!fin.empty()) {
                const int F = (int)fin.size();
                std::vector<xs::InstDev> hf(F);
                for (int i = 0; i < F; ++i) hf[i] = h[fin[i]];
                XS_HIP(hipMemcpyAsync(d_fin, hf.data(), sizeof(xs::InstDev) * F,
                                      hipMemcpyHostToDevice, stream));
                XS_HIP(xs::launch_final(d_fin, F, fin_words, fin_n, stream));
                XS_HIP(hipMemcpyAsync(hf.data(), d_fin, sizeof(xs::InstDev) * F,
                                      hipMemcpyDeviceToHost, stream));
                XS_HIP(hipStreamSynchronize(stream));
                for (int i = 0; i < F; ++i) h[fin[i]] = hf[i];
            }
            std::vector<Request *> still;
            std::vector<std::pair<Request *, xs_run_result>> ended;
            for (int k = 0; k < R; ++k) {
                Request *r = resident[k];
                r->desc = h[k];
                if (!h[k].done) {
                    still.push_back(r);
                    continue;
                }
                const xs::InstDev &d = h[k];
                xs_run_result res{};
                res.tts_sweeps = d.tts == INT32_MAX ? -1 : d.tts;
                res.winner_clone = d.winner == INT32_MAX ? -1 : d.winner;
                res.end_sweep = d.t_cur;
                res.sweeps_done = d.t_cur - d.t_start;
                res.tile_blocks = d.tile_blocks;
                res.wg_threads = d.wg_threads;
                res.col_bytes = d.col_bytes;
                res.rec_global = d.rec_global;
                res.clone_spin_updates = (uint64_t)d.n_words * 64 * d.n * res.sweeps_done;
                const size_t n = d.n, nc = (size_t)d.n_words * 64;
                if (r->outs.state)
                    XS_HIP(hipMemcpyAsync(r->outs.state, d.state, n * nc / 8,
                                          hipMemcpyDeviceToHost, stream));
                if (r->outs.first_hit)
                    XS_HIP(hipMemcpyAsync(r->outs.first_hit, d.first_hit, 4 * nc,
                                          hipMemcpyDeviceToHost, stream));
                if (r->outs.energy)
                    XS_HIP(hipMemcpyAsync(r->outs.energy, d.energy, 4 * nc,
                                          hipMemcpyDeviceToHost, stream));
                if (r->outs.solved && d.winner != INT32_MAX)
                    XS_HIP(hipMemcpyAsync(r->outs.solved, d.solved, n, hipMemcpyDeviceToHost,
                                          stream));
                ended.emplace_back(r, res);
            }
            if (!ended.empty()) XS_HIP(hipStreamSynchronize(stream));  // outputs copied
            for (auto &e : ended) {
                release(e.first);
                complete(e.first, XS_OK, e.second);
                delete e.first;
            }
            resident.swap(still);
        }
        stats.pending = pending.size();
        stats.resident = resident.size();
        stats.step_seconds += now_s() - t0;
        if (n_active) *n_active = (int32_t)(resident.size() + pending.size());
        return XS_OK;
    }
};

extern "C" {

xs_status xs_server_create(const xs_server_config *cfg, void *stream, xs_server **out) {
    return guarded([&]() -> xs_status {
        if (!cfg || !out) return fail(XS_EINVAL, "null argument");
        *out = nullptr;
        if (cfg->struct_size < sizeof(xs_server_config))
            return fail(XS_EINVAL, "xs_server_config.struct_size too small");
        if (cfg->hbm_budget_bytes == 0) return fail(XS_EINVAL, "hbm_budget_bytes is 0");
        if (cfg->reserved) return fail(XS_EINVAL, "xs_server_config.reserved must be 0");
        xs_server *S = new (std::nothrow) xs_server;
        if (!S) return fail(XS_ENOMEM, "host allocation failed");
        S->cfg = *cfg;
        S->stream = reinterpret_cast<hipStream_t>(stream);
        hipError_t e = hipGetDevice(&S->device);
        if (e != hipSuccess) {
            delete S;
            return fail(XS_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
        }
        *out = S;
        return XS_OK;
    });
}

void xs_server_destroy(xs_server *srv) {
    if (!srv) return;
    (void)hipStreamSynchronize(srv->stream);
    delete srv;
}

xs_status xs_server_submit(xs_server *srv, const xs_instance *inst, const xs_run_config *cfg,
                           const xs_server_outputs *outs, uint64_t *ticket) {
    return guarded([&]() -> xs_status {
        if (!srv || !inst || !cfg || !ticket) return fail(XS_EINVAL, "null argument");
        xs_run_buffers none{};
        xs_status st = xsh::validate_run(inst, cfg, &none, false);
        if (st != XS_OK) return st;
        if (cfg->flags & XS_RESUME) return fail(XS_EINVAL, "XS_RESUME is not supported by the server");
        if (srv->cfg.max_pending && srv->pending.size() >= srv->cfg.max_pending)
            return fail(XS_EAGAIN, "%zu requests already wait for admission", srv->pending.size());
        Request *r = new (std::nothrow) Request;
        if (!r) return fail(XS_ENOMEM, "host allocation failed");
        r->ticket = srv->next_ticket++;
        r->inst = inst;
        r->cfg = *cfg;
        if (outs) r->outs = *outs;
        r->bytes = footprint(inst, *cfg);
        r->t_submit = now_s();
        try {
            srv->pending.push_back(r);
        } catch (...) {
            delete r;
            throw;
        }
        srv->stats.pending = srv->pending.size();
        *ticket = r->ticket;
        return XS_OK;
    });
}

xs_status xs_server_step(xs_server *srv, int32_t *n_active) {
    return guarded([&]() -> xs_status {
        if (!srv) return fail(XS_EINVAL, "null server");
        return srv->step(n_active);
    });
}

xs_status xs_server_poll(xs_server *srv, xs_server_completion *done, int32_t cap,
                         int32_t *n_done) {
    return guarded([&]() -> xs_status {
        if (!srv || !n_done || (cap > 0 && !done)) return fail(XS_EINVAL, "null argument");
        int32_t k = 0;
        while (k < cap && !srv->completed.empty()) {
            done[k++] = srv->completed.front();
            srv->completed.pop_front();
        }
        *n_done = k;
        return XS_OK;
    });
}

xs_status xs_server_cancel(xs_server *srv, uint64_t ticket) {
    return guarded([&]() -> xs_status {
        if (!srv) return fail(XS_EINVAL, "null server");
        for (Request *r : srv->pending)
            if (r->ticket == ticket && !r->canceled) {
                r->canceled = true;
                return XS_OK;
            }
        for (Request *r : srv->resident)
            if (r->ticket == ticket && !r->canceled) {
                r->canceled = true;
                return XS_OK;
            }
        return fail(XS_ENOTFOUND, "ticket %llu is not queued or resident", (unsigned long long)ticket);
    });
}

xs_status xs_server_get_stats(const xs_server *srv, xs_server_stats *out) {
    return guarded([&]() -> xs_status {
        if (!srv || !out) return fail(XS_EINVAL, "null argument");
        *out = srv->stats;
        return XS_OK;
    });
}

}  // extern "C"
