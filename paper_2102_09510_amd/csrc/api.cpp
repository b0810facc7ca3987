// Host runtime of the C ABI declared in include/xorsat.h: instance validation, the greedy
// independent-set partition, device tables, and the chunked run driver (single and batched).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/xorsat.h"
#include "place.h"
#include "xs_host.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace xsh {

xs_status fail(xs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

}  // namespace xsh

using xsh::DeviceTables;
using xsh::fail;

namespace {

struct ProfileState {
    std::mutex mu;
    bool on = false;
    xs_kernel_stats stats{};
};
ProfileState g_prof;

}  // namespace

namespace xsh {

// Greedy partition into independent sets of at most `cap` spins: repeated ascending scans; a
// scan adds an unassigned spin unless the set is full or the spin shares a triplet with a spin
// the scan already added. The "blocked" stamps mark the neighbours of the current set.
void partition(xs_instance &I) {
    const int n = I.n;
    std::vector<std::vector<int32_t>> nbr(n);
    for (int t = 0; t < n; ++t)
        for (int q = 0; q < 3; ++q)
            for (int r = 0; r < 3; ++r)
                if (q != r) nbr[I.tri[3 * t + q]].push_back(I.tri[3 * t + r]);
    std::vector<char> assigned(n, 0);
    std::vector<int32_t> blocked(n, -1);
    I.perm.clear();
    I.class_off.assign(1, 0);
    I.max_class = 0;
    int pass = 0;
    while ((int)I.perm.size() < n) {
        int size = 0;
        for (int v = 0; v < n && size < I.cap; ++v) {
            if (assigned[v] || blocked[v] == pass) continue;
            assigned[v] = 1;
            I.perm.push_back(v);
            ++size;
            for (int32_t u : nbr[v]) blocked[u] = pass;
        }
        I.class_off.push_back((int32_t)I.perm.size());
        I.max_class = std::max(I.max_class, size);
        ++pass;
    }
}

// The rules of a body, checked for offsets tau and iteration length ii (see make_body).
bool body_valid(const xs_instance &I, uint32_t cap, const std::vector<int32_t> &inc,
                const std::vector<int32_t> &pos, const std::vector<int32_t> &tau, int ii) {
    const int n = I.n;
    std::vector<int32_t> width(ii, 0);
    for (int v = 0; v < n; ++v) {
        if (tau[v] < 0 || tau[v] >= 2 * ii) return false;
        if (++width[tau[v] % ii] > (int)cap && cap) return false;
        for (int q = 0; q < 3; ++q) {
            const int tr = inc[3 * v + q];
            for (int z = 0; z < 3; ++z) {
                const int u = I.tri[3 * tr + z];
                if (u == v) continue;
                if (tau[u] % ii == tau[v] % ii) return false;
                if (pos[u] < pos[v] ? !(tau[u] < tau[v]) : !(tau[u] < ii + tau[v])) return false;
            }
        }
    }
    return true;
}

// A body of a given length ii by modulo scheduling, for shapes where the sweep-by-sweep
// placement of make_body does not settle into one: spins are placed in update order, each at
// the earliest offset its placed partners allow (after its earlier partners, at most ii - 1
// before its later ones) whose step (offset mod ii) has room and holds none of its partners;
// passes repeat while a later partner's move raised some spin's earliest offset. Offsets only
// grow, so a pass limit ends it; the result is normalised to start at 0 and checked.
bool modulo_body(const xs_instance &I, uint32_t cap, const std::vector<int32_t> &inc,
                 const std::vector<int32_t> &pos, int ii, std::vector<int32_t> &tau) {
    const int n = I.n;
    constexpr int kPasses = 24;
    tau.assign(n, -1);
    std::vector<int32_t> fill(ii, 0);
    auto earliest = [&](int v) {
        int s = 0;
        for (int q = 0; q < 3; ++q) {
            const int tr = inc[3 * v + q];
            for (int z = 0; z < 3; ++z) {
                const int u = I.tri[3 * tr + z];
                if (u == v || tau[u] < 0) continue;
                s = std::max(s, pos[u] < pos[v] ? tau[u] + 1 : tau[u] + 1 - ii);
            }
        }
        return s;
    };
    auto fits = [&](int v, int s) {
        if (cap && fill[s % ii] >= (int)cap) return false;
        for (int q = 0; q < 3; ++q) {
            const int tr = inc[3 * v + q];
            for (int z = 0; z < 3; ++z) {
                const int u = I.tri[3 * tr + z];
                if (u != v && tau[u] >= 0 && tau[u] % ii == s % ii) return false;
            }
        }
        return true;
    };
    for (int pass = 0; pass < kPasses; ++pass) {
        bool moved = false;
        for (int p = 0; p < n; ++p) {
            const int v = I.perm[p];
            const int lb = earliest(v);
            if (tau[v] >= lb) continue;
            if (tau[v] >= 0) --fill[tau[v] % ii];
            tau[v] = -1;
            int s = lb;
            while (!fits(v, s)) {
                if (s - lb > 2 * ii) return false;  // no step of the iteration fits
                ++s;
            }
            tau[v] = s;
            ++fill[s % ii];
            moved = true;
        }
        if (!moved) {
            const int base = *std::min_element(tau.begin(), tau.end());
            const int shift = base - ((base % ii) + ii) % ii;  // keep residues: subtract a multiple of ii
            for (int v = 0; v < n; ++v) tau[v] -= shift;
            return body_valid(I, cap, inc, pos, tau, ii);
        }
    }
    return false;
}

// Cross-sweep body. Successive sweeps may overlap: the update of spin j in sweep t runs at
// step t * II + tau(j) of the run, for offsets tau(j) in [0, 2 II), i.e. in step tau(j) mod II
// of iteration t + tau(j) div II (a "late" spin runs in the iteration after its sweep's). The
// iterations then reproduce the sequential sweeps exactly when, for every two spins i and j
// that share a triplet: (1) tau(i) < tau(j) if i comes before j in the update order (sweep t
// of j reads sweep t of i); (2) tau(i) < II + tau(j) if i comes after j (sweep t + 1 of j reads
// sweep t of i, and writes j only after sweep t of i has read it); (3) tau(i) != tau(j) mod II
// (they never share a step); and (4) no step holds more than cap spins. Updates of one spin in
// successive sweeps are II steps apart, and (1)-(2) order every pair of updates that touch a
// common spin as the sequential sweeps do (pairs more than one sweep apart: |tau(i) - tau(j)| <
// 2 II). tau comes from placing the updates of successive sweeps each as early as these rules
// allow, into the first step with room (the single-sweep rule of make_schedule, across
// sweeps), for up to forty sweeps: once every spin's step moves by the same II from one
// sweep to the next over three sweeps, tau is one of them less its minimum; a pattern that
// only nearly settles is tried with the largest shift of its last sweeps (and one more) as
// II; otherwise modulo_body looks for an II below the single-sweep step count directly. The
// result is checked against (1)-(4) (body_valid) and kept only if II is below the
// single-sweep step count.
bool make_body(const xs_instance &I, uint32_t cap, int plain_steps,
               const std::vector<int32_t> &inc, const std::vector<int32_t> &pos,
               std::vector<int32_t> &tau, int &ii) {
    const int n = I.n;
    constexpr int kSweeps = 40, kTail = 8;
    std::vector<int32_t> prev(n, -1), cur(n), fill;
    std::vector<std::vector<int32_t>> last;  // steps of the last kTail sweeps
    std::vector<int32_t> first_step;         // first step of each sweep
    for (int t = 0; t < kSweeps; ++t) {
        for (int p = 0; p < n; ++p) {
            const int v = I.perm[p];
            int s = prev[v] + 1;
            for (int q = 0; q < 3; ++q) {
                const int tr = inc[3 * v + q];
                for (int z = 0; z < 3; ++z) {
                    const int u = I.tri[3 * tr + z];
                    if (u == v) continue;
                    s = std::max(s, pos[u] < p ? cur[u] + 1 : prev[u] + 1);
                }
            }
            while (cap && s < (int)fill.size() && fill[s] >= (int)cap) ++s;
            if (s >= (int)fill.size()) fill.resize(s + 1, 0);
            ++fill[s];
            cur[v] = s;
        }
        last.push_back(cur);
        if ((int)last.size() > kTail) last.erase(last.begin());
        prev = cur;
        // settled: every spin moved by the same shift over each of the last three sweeps
        if (last.size() >= 4) {
            const size_t m = last.size();
            const int d = last[m - 1][0] - last[m - 2][0];
            bool same = true;
            for (size_t k = m - 3; k < m && same; ++k)
                for (int v = 0; v < n && same; ++v) same = last[k][v] - last[k - 1][v] == d;
            if (same) break;
        }
    }
    // A settled pattern: every spin moves by the same II over the last three sweeps. Else, the
    // last sweep's offsets with the largest (then one more) shift seen over the last sweeps.
    auto take = [&](const std::vector<int32_t> &steps, int len) {
        const int base = *std::min_element(steps.begin(), steps.end());
        tau.assign(n, 0);
        for (int v = 0; v < n; ++v) tau[v] = steps[v] - base;
        ii = len;
        return len > 0 && len < plain_steps && body_valid(I, cap, inc, pos, tau, len);
    };
    const int m = (int)last.size();
    if (m >= 3) {
        const std::vector<int32_t> &a = last[m - 3], &b = last[m - 2], &c = last[m - 1];
        const int d = c[0] - b[0];
        bool periodic = true;
        for (int v = 0; v < n && periodic; ++v) periodic = c[v] - b[v] == d && b[v] - a[v] == d;
        if (periodic && take(b, d)) return true;
    }
    int most = 0;
    for (int k = 1; k < m; ++k)
        for (int v = 0; v < n; ++v) most = std::max(most, last[k][v] - last[k - 1][v]);
    for (int len = most; len <= most + 1; ++len)
        for (int k = m - 1; k >= std::max(0, m - 4); --k)
            if (take(last[k], len)) return true;
    // Modulo schedules of decreasing length, from one step below the single-sweep count down
    // to the width bound, keeping the last that works (a failure ends the search: shorter ones
    // rarely work where a longer one did not, and each try costs passes over the spins).
    const int lo = std::max(1, cap ? (n + (int)cap - 1) / (int)cap : 1);
    std::vector<int32_t> t;
    int found = 0;
    for (int k = plain_steps - 1; k >= lo && modulo_body(I, cap, inc, pos, k, t); --k) {
        tau = t;
        found = k;
    }
    ii = found;
    return found > 0;
}

// Execution schedule of the update order. The update of a spin reads its own value and those of
// the spins it shares a triplet with, and writes only its own, so two updates commute unless
// their spins share a triplet. Each spin is placed in a step after every earlier spin (in update
// order) it shares a triplet with -- the first such step with room when steps hold at most
// `cap` spins (cap 0: no limit) -- so running the steps one after another, the spins of a step
// in parallel, keeps the order of every pair that does not commute and gives exactly the
// sequential sweep. Steps are independent sets. Uncapped, there are at most as many steps as
// classes (a member of class c has no conflicting predecessor in c, so by induction its step is
// at most c) and far fewer when the class cap, not a shared triplet, closed the classes; the
// cap fits the steps to the threads of a launch. B > 0: the LDS rows are placed for tiles of B
// blocks read in CW-byte columns. j0: the records' coupling bits are 0 (runs in the gauge of
// solve_gauge, where every coupling is +1). body: also build the cross-sweep body (make_body)
// where one exists; the rows are then placed for the body's steps, which untracked chunks run.
xsh::HostSched make_schedule(const xs_instance &I, uint32_t cap, uint32_t B, uint32_t CW,
                             bool j0, bool body, int effort = 0) {
    const int n = I.n;
    std::vector<int32_t> inc(3 * (size_t)n), deg(n, 0), pos(n), step(n, 0), fill;
    for (int t = 0; t < n; ++t)
        for (int q = 0; q < 3; ++q) {
            const int v = I.tri[3 * t + q];
            inc[3 * v + deg[v]++] = t;
        }
    for (int p = 0; p < n; ++p) pos[I.perm[p]] = p;
    for (int p = 0; p < n; ++p) {
        const int v = I.perm[p];
        int s = 0;
        for (int q = 0; q < 3; ++q) {
            const int t = inc[3 * v + q];
            for (int z = 0; z < 3; ++z) {
                const int u = I.tri[3 * t + z];
                if (u != v && pos[u] < p) s = std::max(s, step[u] + 1);
            }
        }
        while (cap && s < (int)fill.size() && fill[s] >= (int)cap) ++s;
        if (s >= (int)fill.size()) fill.resize(s + 1, 0);
        ++fill[s];
        step[v] = s;
    }
    xsh::HostSched hs;
    const int steps = (int)fill.size();
    hs.off.assign(steps + 1, 0);
    for (int l = 0; l < steps; ++l) {
        hs.max_step = std::max(hs.max_step, fill[l]);
        hs.off[l + 1] = hs.off[l] + fill[l];
    }
    std::vector<int32_t> next(hs.off.begin(), hs.off.end() - 1);
    hs.order.assign(n, 0);
    for (int p = 0; p < n; ++p) hs.order[next[step[I.perm[p]]]++] = I.perm[p];
    // The body: spins grouped by tau mod II (in update order within a step).
    std::vector<int32_t> tau;
    int ii = 0;
    if (body && make_body(I, cap, steps, inc, pos, tau, ii)) {
        std::vector<int32_t> bfill(ii, 0);
        for (int v = 0; v < n; ++v) ++bfill[tau[v] % ii];
        hs.boff.assign(ii + 1, 0);
        for (int l = 0; l < ii; ++l) hs.boff[l + 1] = hs.boff[l] + bfill[l];
        std::vector<int32_t> bnext(hs.boff.begin(), hs.boff.end() - 1);
        hs.border.assign(n, 0);
        for (int p = 0; p < n; ++p) {
            const int v = I.perm[p];
            hs.border[bnext[tau[v] % ii]++] = v;
        }
    }
    // Roles of every spin: itself, then for each of its three triplets (ascending triplet index)
    // the two other spins; and its coupling bits (bit q: triplet q has J = -1).
    std::vector<int32_t> roles(7 * (size_t)n);
    std::vector<uint16_t> jbits(n, 0);
    for (int i = 0; i < n; ++i) {
        roles[7 * (size_t)i] = i;
        for (int q = 0; q < 3; ++q) {
            const int t = inc[3 * i + q];
            int k = 0;
            for (int z = 0; z < 3; ++z)
                if (I.tri[3 * t + z] != i) roles[7 * (size_t)i + 1 + 2 * q + k++] = I.tri[3 * t + z];
            if (I.J[t] < 0 && !j0) jbits[i] |= (uint16_t)(1u << q);
        }
    }
    // Rows placed for the steps the hot loop runs (the body's, where there is one); the
    // placement also re-orders those steps' spins and each spin's partner slots (coupling bits
    // follow their triplets), none of which changes a result.
    const RowModel model = row_model(B, CW);
    if (!model.sets.empty() && n >= 2 * (int)model.S) {
        std::vector<int32_t> &ord = hs.border.empty() ? hs.order : hs.border;
        const Placement pl =
            place_rows(ord, hs.border.empty() ? hs.off : hs.boff, roles, n, model, effort);
        hs.rowmap = pl.row;
        ord = pl.order;
        for (int i = 0; i < n; ++i) {
            const int sl = pl.slots[i];
            if (!sl) continue;
            int32_t *r = &roles[7 * (size_t)i];
            const int32_t was[7] = {r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
            for (int k = 1; k < 7; ++k) r[k] = was[slot_source(sl, k)];
            const uint16_t jb = jbits[i];
            jbits[i] = 0;
            for (int q = 0; q < 3; ++q) jbits[i] |= (uint16_t)(((jb >> kTripOrder[sl % 6][q]) & 1u) << q);
        }
    }
    // Records in schedule order: the LDS rows of the spin and of its six partners, then
    // meta = spin | coupling bits << 13 (body records: | late << 12).
    auto records = [&](const std::vector<int32_t> &order, std::vector<uint16_t> &rec,
                       bool mark_late) {
        rec.assign(8 * (size_t)n, 0);
        for (int p = 0; p < n; ++p) {
            const int i = order[p];
            uint16_t *r = &rec[8 * (size_t)p];
            for (int k = 0; k < 7; ++k) {
                const int32_t u = roles[7 * (size_t)i + k];
                r[k] = hs.rowmap.empty() ? (uint16_t)u : hs.rowmap[u];
            }
            const uint16_t late = mark_late && tau[i] >= ii ? 1u << 12 : 0u;
            r[7] = (uint16_t)(i | late | (jbits[i] << 13));
        }
    };
    records(hs.order, hs.rec, false);
    if (!hs.border.empty()) records(hs.border, hs.brec, true);
    return hs;
}

// Gauge of an instance: bits g with g_a ^ g_b ^ g_c = [J_t = -1] for every triplet t = (a, b, c),
// by Gaussian elimination over GF(2) (Section "The model and its energy landscape": a planted
// instance, J_t = tau_a tau_b tau_c, is the gauge image of the ferromagnet). Flipping the spins
// with g_i = 1 turns every coupling into +1 and leaves every k, and so every trajectory,
// unchanged. False if no such g exists (some coupling stays -1 in every gauge).
bool solve_gauge(const xs_instance &I, std::vector<uint8_t> &g) {
    const int n = I.n, W = n / 64 + 1;  // n unknowns, right-hand side at bit n
    std::vector<uint64_t> M((size_t)n * W, 0);
    auto row = [&](int r) { return M.data() + (size_t)r * W; };
    auto bit = [&](int r, int c) { return (row(r)[c >> 6] >> (c & 63)) & 1u; };
    for (int t = 0; t < n; ++t) {
        uint64_t *m = row(t);
        for (int q = 0; q < 3; ++q) {
            const int v = I.tri[3 * t + q];
            m[v >> 6] ^= 1ull << (v & 63);
        }
        if (I.J[t] < 0) m[n >> 6] ^= 1ull << (n & 63);
    }
    std::vector<int> pivot;  // pivot column of each row of the echelon form
    int rank = 0;
    for (int c = 0; c < n && rank < n; ++c) {
        int p = rank;
        while (p < n && !bit(p, c)) ++p;
        if (p == n) continue;
        if (p != rank) std::swap_ranges(row(p), row(p) + W, row(rank));
        const uint64_t *pr = row(rank);
        for (int r = rank + 1; r < n; ++r)
            if (bit(r, c)) {
                uint64_t *m = row(r);
                for (int w = c >> 6; w < W; ++w) m[w] ^= pr[w];
            }
        pivot.push_back(c);
        ++rank;
    }
    for (int r = rank; r < n; ++r)
        if (bit(r, n)) return false;  // 0 = 1: inconsistent
    // Back substitution, free unknowns 0.
    std::vector<uint64_t> x(W, 0);
    for (int k = rank - 1; k >= 0; --k) {
        const uint64_t *m = row(k);
        uint64_t par = bit(k, n);
        for (int w = 0; w < W; ++w) {
            uint64_t v = m[w] & x[w];
            if (w == (n >> 6)) v &= (1ull << (n & 63)) - 1;  // unknowns only
            par ^= (uint64_t)__builtin_popcountll(v) & 1u;
        }
        // the pivot's own bit is still 0 in x, so par = rhs ^ (the other unknowns of the row)
        if (par) x[pivot[k] >> 6] |= 1ull << (pivot[k] & 63);
    }
    g.assign(n, 0);
    for (int i = 0; i < n; ++i) g[i] = (uint8_t)((x[i >> 6] >> (i & 63)) & 1u);
    for (int t = 0; t < n; ++t)  // every coupling becomes +1
        if ((g[I.tri[3 * t]] ^ g[I.tri[3 * t + 1]] ^ g[I.tri[3 * t + 2]]) != (I.J[t] < 0 ? 1 : 0))
            return false;
    return true;
}

// Triplets as the final pass reads them: a, b, c, and j = 1 for J = -1.
void build_triplets(xs_instance &I) {
    const int n = I.n;
    I.tri16.assign(4 * (size_t)n, 0);
    for (int t = 0; t < n; ++t) {
        for (int q = 0; q < 3; ++q) I.tri16[4 * t + q] = (uint16_t)I.tri[3 * t + q];
        I.tri16[4 * t + 3] = I.J[t] < 0 ? 1 : 0;
    }
}

xs_status ensure_tables(const xs_instance *I, int device, DeviceTables *out) {
    std::lock_guard<std::mutex> lock(I->mu);
    auto it = I->dev.find(device);
    if (it != I->dev.end()) {
        *out = it->second;
        return XS_OK;
    }
    DeviceTables t;
    const size_t n = (size_t)I->n;
    DevAlloc tri;
    XS_HIP(hipMalloc(&tri.p, 8 * n));
    XS_HIP(hipMemcpy(tri.p, I->tri16.data(), 8 * n, hipMemcpyHostToDevice));
    t.tri = tri.release<uint2>();
    I->dev[device] = t;
    *out = t;
    return XS_OK;
}

// Steps of a launch hold one task round: wg_threads / (columns per row) spins.
uint32_t step_cap(const xs::InstDev &d) {
    return d.wg_threads * d.col_bytes / (32u * d.tile_blocks);
}

// Schedules are kept per (step cap, placement layout, coupling gauge, body); caps stay below
// 2^16. Layout 0: rows not placed; else tile blocks | column bytes << 8 (below bit 30).
uint32_t sched_key(uint32_t cap, uint32_t layout, bool j0 = false, bool body = false,
                   bool full = false) {
    return cap | layout << 16 | (full ? 1u << 29 : 0u) | (body ? 1u << 30 : 0u) |
           (j0 ? 1u << 31 : 0u);
}

// The cross-sweep body runs where records are read from global memory and w0 = 0 (ground
// states are absorbing and chunks without tracking are checked at their end), unless the run
// asks for one sweep at a time.
bool wants_body(const xs::InstDev &d) {
    return d.rec_global && d.thr0 == 0 && !(d.flags & XS_ONE_SWEEP_STEPS);
}
uint32_t place_layout(uint32_t B, uint32_t CW) { return B < 8 ? B | CW << 8 : 0u; }

// Clone-sweeps (clones x sweeps left) from which a run builds the row placement. The search
// costs about 0.5 µs of host time per spin and unit of effort (place_rows) and saves 5-10 % of
// the sweep time, both in proportion to N, so its effort is set from the clone-sweeps: a run
// spends at most about a tenth of its sweep time on it, and a run that asks for the placement
// (XS_PLACE_ROWS) gets the full effort. Batches build their instances' schedules on several host
// threads at once, which divides the cost (host_threads()).
constexpr uint64_t kPlaceMinWork = 1ull << 32;
constexpr int kPlaceEffort = 1600;

// Host threads that build the schedules of a batch.
uint32_t host_threads() {
    const uint32_t hc = std::thread::hardware_concurrency();
    return std::max(1u, std::min(hc ? hc : 1u, 16u));
}

// What a descriptor's schedule is made of (see host_sched).
struct SchedParams {
    uint32_t key, cap, layout;
    bool j0, body;
    int effort;  // of the row placement search
};

// The schedule a descriptor's launch uses: its step cap, row placement and body. The row
// placement is used if it exists or the run is long enough to pay for building it (runs of a
// batch share the host threads, `builders` of them); either gives the same results. Caller
// holds I->mu.
SchedParams sched_params(const xs_instance *I, const xs::InstDev &d, uint32_t builders) {
    SchedParams sp;
    sp.cap = step_cap(d);
    sp.layout = place_layout(d.tile_blocks, d.col_bytes);
    sp.j0 = d.j0 != 0;
    sp.body = wants_body(d);
    const uint64_t work = (uint64_t)d.n_words * 64u * (d.t_stop - d.t_cur);
    const uint32_t nb = std::max(builders, 1u);
    bool full = false;
    sp.effort = 0;
    if (sp.layout) {
        // a full placement serves every later run; a run that asks for one builds it
        full = (d.flags & XS_PLACE_ROWS) ||
               I->sched.count(sched_key(sp.cap, sp.layout, sp.j0, sp.body, true));
        if (full)
            sp.effort = kPlaceEffort;
        else if (work >= kPlaceMinWork / nb ||
                 I->sched.count(sched_key(sp.cap, sp.layout, sp.j0, sp.body)))
            sp.effort = (int)std::min<uint64_t>(std::max<uint64_t>(work * nb >> 29, 8), kPlaceEffort);
        else
            sp.layout = 0;
    }
    sp.key = sched_key(sp.cap, sp.layout, sp.j0, sp.body, full);
    return sp;
}

// The host schedule a descriptor's launch uses (built on first use; caller holds I->mu), and
// its key in the instance's caches.
const xsh::HostSched &host_sched(const xs_instance *I, const xs::InstDev &d, uint32_t *key_out,
                                 uint32_t builders = 1) {
    const SchedParams sp = sched_params(I, d, builders);
    auto hit = I->sched.find(sp.key);
    if (hit == I->sched.end())
        hit = I->sched
                  .emplace(sp.key, make_schedule(*I, sp.cap, sp.layout & 0xFF, sp.layout >> 8,
                                                 sp.j0, sp.body, sp.effort))
                  .first;
    *key_out = sp.key;
    return hit->second;
}

// Build the missing schedules of a batch's descriptors on several host threads (each instance
// and key once). make_schedule reads only fields an instance never changes after creation, so
// the builds run without the instance's lock; the results are inserted under it. Returns the
// number of builders the batch may count on (1 when at most one schedule is missing).
uint32_t prebuild_schedules(const std::vector<xs::InstDev> &h, const xs_instance *const *insts,
                            int count) {
    const uint32_t threads = host_threads();
    struct Job {
        const xs_instance *I;
        SchedParams sp;
        xsh::HostSched hs;
    };
    std::vector<Job> jobs;
    for (int k = 0; k < count; ++k) {
        const xs_instance *I = insts[k];
        std::lock_guard<std::mutex> lock(I->mu);
        const SchedParams sp = sched_params(I, h[k], threads);
        if (I->sched.count(sp.key)) continue;
        bool dup = false;
        for (const Job &j : jobs) dup |= j.I == I && j.sp.key == sp.key;
        if (!dup) jobs.push_back(Job{I, sp, {}});
    }
    if (jobs.size() < 2) return 1;
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t j; (j = next.fetch_add(1)) < jobs.size();) {
            Job &b = jobs[j];
            b.hs = make_schedule(*b.I, b.sp.cap, b.sp.layout & 0xFF, b.sp.layout >> 8, b.sp.j0,
                                 b.sp.body, b.sp.effort);
        }
    };
    std::vector<std::thread> pool;
    try {
        for (uint32_t t = 1; t < std::min<size_t>(threads, jobs.size()); ++t) pool.emplace_back(work);
    } catch (const std::system_error &) {
        // fewer threads: the caller's thread builds what the others do not
    }
    work();
    for (std::thread &t : pool) t.join();
    for (Job &j : jobs) {
        std::lock_guard<std::mutex> lock(j.I->mu);
        j.I->sched.emplace(j.sp.key, std::move(j.hs));
    }
    return threads;
}

// Records with the byte offsets of the rows in a tile of B blocks (32 * B bytes per row), as
// the kernels that read records from global memory take them.
std::vector<uint32_t> grec_image(const std::vector<uint16_t> &rec, int n, uint32_t B) {
    const uint32_t rowb = 32u * B;
    std::vector<uint32_t> g(4 * (size_t)n);
    for (int p = 0; p < n; ++p) {
        const uint16_t *r = &rec[8 * (size_t)p];
        g[4 * p + 0] = (r[0] * rowb) | ((r[1] * rowb) << 16);
        g[4 * p + 1] = (r[2] * rowb) | ((r[3] * rowb) << 16);
        g[4 * p + 2] = (r[4] * rowb) | ((r[5] * rowb) << 16);
        g[4 * p + 3] = (r[6] * rowb) | ((uint32_t)r[7] << 16);
    }
    return g;
}

xs_status attach_tables(std::vector<xs::InstDev> &h, const xs_instance *const *insts, int count,
                        int device) {
    const uint32_t builders = prebuild_schedules(h, insts, count);
    for (int k = 0; k < count; ++k) {
        xs::InstDev &d = h[k];
        const xs_instance *I = insts[k];
        std::lock_guard<std::mutex> lock(I->mu);
        uint32_t key = 0;
        const xsh::HostSched &hs = host_sched(I, d, &key, builders);
        xsh::DevSched &ds = I->dev[device].sched[key];
        if (!ds.rec) {
            const size_t n = (size_t)I->n, off_bytes = sizeof(int32_t) * hs.off.size();
            DevAlloc rec, off, rowmap;
            XS_HIP(hipMalloc(&rec.p, 16 * n));
            XS_HIP(hipMemcpy(rec.p, hs.rec.data(), 16 * n, hipMemcpyHostToDevice));
            XS_HIP(hipMalloc(&off.p, off_bytes));
            XS_HIP(hipMemcpy(off.p, hs.off.data(), off_bytes, hipMemcpyHostToDevice));
            if (!hs.rowmap.empty()) {
                XS_HIP(hipMalloc(&rowmap.p, 2 * n));
                XS_HIP(hipMemcpy(rowmap.p, hs.rowmap.data(), 2 * n, hipMemcpyHostToDevice));
            }
            ds.rec = rec.release<uint4>();
            ds.off = off.release<int32_t>();
            ds.rowmap = rowmap.release<uint16_t>();
            ds.steps = (uint32_t)hs.off.size() - 1;
        }
        d.rec = ds.rec;
        d.step_off = ds.off;
        d.rowmap = ds.rowmap;
        d.n_steps = ds.steps;
        d.gauge = nullptr;
        if (d.j0) {
            xsh::DeviceTables &dt = I->dev[device];
            if (!dt.gauge) {
                DevAlloc gb;
                XS_HIP(hipMalloc(&gb.p, (size_t)I->n));
                XS_HIP(hipMemcpy(gb.p, I->gauge.data(), (size_t)I->n, hipMemcpyHostToDevice));
                dt.gauge = gb.release<uint8_t>();
            }
            d.gauge = dt.gauge;
        }
        d.grec = nullptr;
        if (!d.rec_global) continue;
        auto it = ds.grec.find(d.tile_blocks);
        if (it == ds.grec.end()) {
            const std::vector<uint32_t> g = grec_image(hs.rec, I->n, d.tile_blocks);
            DevAlloc dp;
            XS_HIP(hipMalloc(&dp.p, 16 * (size_t)I->n));
            XS_HIP(hipMemcpy(dp.p, g.data(), 16 * (size_t)I->n, hipMemcpyHostToDevice));
            it = ds.grec.emplace(d.tile_blocks, dp.release<uint4>()).first;
        }
        d.grec = it->second;
        d.bgrec = nullptr;
        d.bstep_off = nullptr;
        d.n_bsteps = 0;
        if (hs.border.empty() || !wants_body(d)) continue;
        if (!ds.boff) {
            const size_t bytes = sizeof(int32_t) * hs.boff.size();
            DevAlloc off;
            XS_HIP(hipMalloc(&off.p, bytes));
            XS_HIP(hipMemcpy(off.p, hs.boff.data(), bytes, hipMemcpyHostToDevice));
            ds.boff = off.release<int32_t>();
            ds.bsteps = (uint32_t)hs.boff.size() - 1;
        }
        auto bt = ds.bgrec.find(d.tile_blocks);
        if (bt == ds.bgrec.end()) {
            const std::vector<uint32_t> g = grec_image(hs.brec, I->n, d.tile_blocks);
            DevAlloc dp;
            XS_HIP(hipMalloc(&dp.p, 16 * (size_t)I->n));
            XS_HIP(hipMemcpy(dp.p, g.data(), 16 * (size_t)I->n, hipMemcpyHostToDevice));
            bt = ds.bgrec.emplace(d.tile_blocks, dp.release<uint4>()).first;
        }
        d.bgrec = bt->second;
        d.bstep_off = ds.boff;
        d.n_bsteps = ds.bsteps;
    }
    return XS_OK;
}

uint32_t ilog2(uint32_t v) {
    uint32_t r = 0;
    while ((1u << (r + 1)) <= v) ++r;
    return r;
}

// Largest power-of-two tile (in 256-clone blocks) that divides the clone count and keeps the
// tile's spin rows within `max_row_blocks` (n * B <= max: state LDS of n * B * 32 bytes).
uint32_t max_tile_blocks(uint32_t n, uint32_t n_blocks, uint32_t max_nb) {
    uint32_t B = 1;
    while (n_blocks % (B * 2) == 0 && n * (B * 2) <= max_nb && B * 2 <= (uint32_t)xs::kMaxTileBlocks)
        B *= 2;
    return B;
}

// Default tiling: default_tile_blocks per instance, then tiles are halved across the batch
// while it has fewer than kTargetTiles workgroups, so that small batches still spread over the
// CUs.
constexpr size_t kTargetTiles = 1024;

// True if the kernels can address p: device or managed memory, or host memory mapped for the
// device at the same address.
bool device_addressable(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // an unknown host pointer: clear the error it leaves
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged ||
           a.type == hipMemoryTypeUnified || a.devicePointer == p;
}

xs_status validate_run(const xs_instance *I, const xs_run_config *cfg, const xs_run_buffers *b,
                       bool check_buffers) {
    if (!I || !cfg || !b) return fail(XS_EINVAL, "null argument");
    if (cfg->struct_size < sizeof(xs_run_config))
        return fail(XS_EINVAL, "xs_run_config.struct_size %u < %zu", cfg->struct_size,
                    sizeof(xs_run_config));
    if (cfg->n_clones == 0 || cfg->n_clones % XS_CLONE_QUANTUM != 0)
        return fail(XS_EINVAL, "n_clones %u is not a positive multiple of %d", cfg->n_clones,
                    XS_CLONE_QUANTUM);
    if (cfg->n_clones > XS_MAX_CLONES)
        return fail(XS_EINVAL, "n_clones %u > %u", cfg->n_clones, XS_MAX_CLONES);
    if (cfg->accept_thr > 65536) return fail(XS_EINVAL, "accept_thr %u > 65536", cfg->accept_thr);
    if (cfg->accept_thr0 > 65536)
        return fail(XS_EINVAL, "accept_thr0 %u > 65536", cfg->accept_thr0);
    if (cfg->reserved) return fail(XS_EINVAL, "xs_run_config.reserved must be 0");
    if (cfg->accept_thr0 && (cfg->flags & XS_STOP_ON_FIRST))
        return fail(XS_EINVAL, "XS_STOP_ON_FIRST needs accept_thr0 = 0 (with w0 > 0 a ground "
                               "state is not absorbing and no sweep is tested)");
    if (cfg->flags &
        ~(XS_STOP_ON_FIRST | XS_RESUME | XS_PLACE_ROWS | XS_PER_CHUNK | XS_ONE_SWEEP_STEPS))
        return fail(XS_EINVAL, "unknown flags 0x%x", cfg->flags);
    if ((uint64_t)cfg->start_sweep + cfg->max_sweeps >= 0xFFFFFFFFull)
        return fail(XS_EINVAL, "start_sweep + max_sweeps must stay below 2^32 - 1");
    if (check_buffers) {
        if (!b->state || !b->first_hit)
            return fail(XS_EINVAL, "state and first_hit are required");
        if (((uintptr_t)b->state & 15) != 0)
            return fail(XS_EINVAL, "state must be 16-byte aligned");
        if (!device_addressable(b->state) || !device_addressable(b->first_hit) ||
            (b->energy && !device_addressable(b->energy)))
            return fail(XS_EINVAL, "state, first_hit and energy must be device memory");
    }
    const uint32_t nb = cfg->n_clones / 256;
    if (cfg->tile_blocks) {
        const uint32_t B = cfg->tile_blocks;
        if ((B & (B - 1)) || B > (uint32_t)xs::kMaxTileBlocks || nb % B ||
            (uint32_t)I->n * B > 2048)
            return fail(XS_EINVAL,
                        "tile_blocks %u must be a power of two <= %d dividing n_clones/256 with "
                        "n * tile_blocks <= 2048",
                        B, xs::kMaxTileBlocks);
    }
    if (cfg->col_bytes && cfg->col_bytes != 4 && cfg->col_bytes != 8 && cfg->col_bytes != 16)
        return fail(XS_EINVAL, "col_bytes %u must be 4, 8 or 16", cfg->col_bytes);
    if (cfg->rec_global > 2) return fail(XS_EINVAL, "rec_global %u must be 0, 1 or 2", cfg->rec_global);
    if (cfg->wg_threads) {
        const uint32_t T = cfg->wg_threads;
        const uint32_t B = cfg->tile_blocks;
        if ((T & (T - 1)) || T < 64 || T > 1024)
            return fail(XS_EINVAL, "wg_threads %u must be a power of two in [64, 1024]", T);
        if (B && T < 8 * B)
            return fail(XS_EINVAL, "wg_threads %u must be at least 8 * tile_blocks (%u)", T, B);
    }
    return XS_OK;
}

// Default workgroup size for a tile of B blocks: about one thread per task of a typical sweep
// step (tasks = spins of the step x columns of the row), as measured: 256 up to four blocks,
// 512 from eight, and 512 for one-block tiles of more than 1024 spins, whose steps are large.
uint32_t default_threads(uint32_t B, uint32_t n) {
    if (B == 1 && n > 1024) return 512u;
    return B >= 8 ? 512u : 256u;
}

// Default tile: the largest with n * B <= 1024 (at most 32 KB of clone state, four workgroups
// per CU). Below n = 256, where the records stay in LDS, raised to eight blocks (256-byte rows:
// each pass of a 16-byte row read takes complementary quarters of two rows, free of bank
// conflicts whatever the rows) where n * 8 <= 2048 still leaves two workgroups per CU. At
// n = 256 four-block tiles with records in global memory (and the coupling gauge) measured
// 5.5 % faster than eight-block tiles with records in LDS.
uint32_t default_tile_blocks(uint32_t n, uint32_t nb) {
    uint32_t B = max_tile_blocks(n, nb, 1024);
    if (B < 8 && n < 256 && n * 8 <= 2048 && nb % 8 == 0) B = 8;
    return B;
}

// Default task column: 16 bytes, and 8 for one-block tiles, so that a step still spreads over
// the workgroup (a one-block tile has 64 tasks of 16 bytes per 32 spins, 128 of 8 bytes).
uint32_t default_col_bytes(uint32_t B) { return B >= 2 ? 16u : 8u; }

// Default record placement: global memory from n = 256 (4 KB of records or more), which also
// lets persistent launches run the instance in its coupling gauge; below, LDS.
uint32_t default_rec_global(uint32_t n) { return n >= 256 ? 1u : 0u; }

// Options of one driver call beyond the public configuration.
struct RunOpts {
    bool graph = true;             // replay the chunk loop as a captured hipGraph
    double *kernel_ms = nullptr;   // if set: time every sweep-chunk launch, add the sum here
    // If set: device memory of fixed_bytes that holds everything the call needs on the device
    // (descriptors, tiles, counter, staging, and the instances' tables, copied in per call).
    // The call then allocates no device memory and creates no graph, event or stream.
    uint8_t *fixed = nullptr;
    size_t fixed_bytes = 0;
};

// Tuned launch knobs (tile_blocks, wg_threads, col_bytes, rec_global) per workload key,
// filled by xs_autotune or xs_tune_load.
struct TuneKey {
    uint32_t n_bucket, clones, count_bucket;
    bool operator<(const TuneKey &o) const {
        return std::tie(n_bucket, clones, count_bucket) <
               std::tie(o.n_bucket, o.clones, o.count_bucket);
    }
};
struct TuneVal {
    uint32_t tile_blocks, wg_threads, col_bytes, rec_global;
    double rate;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

uint32_t pow2_ceil(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}
TuneKey tune_key(uint32_t n, uint32_t clones, int32_t count) {
    return TuneKey{pow2_ceil(n), clones, std::min<uint32_t>(64, pow2_ceil((uint32_t)count))};
}

// Capture of the chunk loop: `group` chunk iterations recorded once on a private stream and
// replayed on the caller's stream (the caller's stream may be the null stream, which cannot be
// captured).
// Chunks per captured graph of the chunk loop (a power of two).
constexpr int kGraphChunks = 8;

struct ChunkGraph {
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int group = 0;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        group = 0;
    }
    ~ChunkGraph() {
        reset();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

void fill_desc(const xs_instance *I, const xs_run_config &c, const DeviceTables &t,
               uint64_t *state, int32_t *first_hit, int32_t *energy, xs::InstDev &d) {
    std::memset(&d, 0, sizeof d);
    d.tri = t.tri;  // records and step offsets: attach_tables, once the launch is chosen
    d.state = state;
    d.first_hit = first_hit;
    d.energy = energy;
    d.n = (uint32_t)I->n;
    d.n_words = c.n_clones / 64;
    d.inst_id = c.instance_id;
    d.thr = c.accept_thr;
    d.thr0 = c.accept_thr0;
    d.seed_lo = (uint32_t)c.seed;
    d.seed_hi = (uint32_t)(c.seed >> 32);
    d.flags = c.flags;
    d.t_start = c.start_sweep;
    d.t_stop = c.start_sweep + c.max_sweeps;
    d.chunk = c.chunk_sweeps ? c.chunk_sweeps : 100;
    d.t_cur = c.start_sweep;
    d.done = c.max_sweeps == 0 ? 1u : 0u;
    d.tts = INT32_MAX;
    d.winner = INT32_MAX;
}

xs_status tile_instances(std::vector<xs::InstDev> &h, const xs_run_config *cfgs, int count,
                         std::vector<uint2> &tiles, std::vector<TileGroup> &groups) {
    for (int k = 0; k < count; ++k) {
        const xs_run_config &c = cfgs[k];
        xs::InstDev &d = h[k];
        const uint32_t nb = c.n_clones / 256;
        uint32_t B = c.tile_blocks ? c.tile_blocks : default_tile_blocks(d.n, nb);
        uint32_t tuned_T = 0, tuned_C = 0, tuned_G = 0;
        if (!c.tile_blocks && !c.wg_threads && !c.col_bytes && !c.rec_global) {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune.find(tune_key(d.n, c.n_clones, count));
            if (it != g_tune.end() && nb % it->second.tile_blocks == 0 &&
                d.n * it->second.tile_blocks <= 2048) {
                B = it->second.tile_blocks;
                tuned_T = it->second.wg_threads;
                tuned_C = it->second.col_bytes;
                tuned_G = it->second.rec_global;
            }
        }
        d.tile_blocks = B;
        d.wg_threads = tuned_T;  // 0 unless tuned
        d.col_bytes = tuned_C;
        d.rec_global = tuned_G;  // 0 = not tuned, 1 = global, 2 = LDS
    }
    // Shrink automatic tiles while the batch has too few workgroups.
    auto count_tiles = [&]() {
        size_t t = 0;
        for (int k = 0; k < count; ++k) t += (cfgs[k].n_clones / 256) / h[k].tile_blocks;
        return t;
    };
    for (;;) {
        if (count_tiles() >= kTargetTiles) break;
        bool changed = false;
        for (int k = 0; k < count; ++k)
            if (!cfgs[k].tile_blocks && !h[k].wg_threads && h[k].tile_blocks > 1) {
                h[k].tile_blocks /= 2;
                changed = true;
            }
        if (!changed) break;
    }
    // Tiles grouped by (workgroup size, column width, record placement, rule): one launch per
    // group and chunk.
    using LaunchKey = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>;
    std::map<LaunchKey, std::vector<uint2>> by_launch;
    std::map<LaunchKey, size_t> lds_of;
    for (int k = 0; k < count; ++k) {
        xs::InstDev &d = h[k];
        d.log2_tile_blocks = ilog2(d.tile_blocks);
        uint32_t T = cfgs[k].wg_threads ? cfgs[k].wg_threads
                     : d.wg_threads       ? d.wg_threads
                                          : default_threads(d.tile_blocks, d.n);
        T = std::max(T, 8 * d.tile_blocks);
        d.wg_threads = T;
        const uint32_t C = cfgs[k].col_bytes ? cfgs[k].col_bytes
                           : d.col_bytes      ? d.col_bytes
                                              : default_col_bytes(d.tile_blocks);
        d.col_bytes = C;
        const uint32_t GRc = cfgs[k].rec_global ? cfgs[k].rec_global
                             : d.rec_global       ? d.rec_global
                                                  : (default_rec_global(d.n) ? 1u : 2u);
        d.rec_global = GRc == 1 ? 1u : 0u;
        const uint32_t nb = cfgs[k].n_clones / 256;
        const uint32_t met = d.thr0 ? 1u : 0u;
        const auto key = std::make_tuple(T, C, d.rec_global, met);
        auto &v = by_launch[key];
        for (uint32_t b0 = 0; b0 < nb; b0 += d.tile_blocks) v.push_back(make_uint2((uint32_t)k, b0));
        lds_of[key] = std::max(lds_of[key], xs::chunk_lds_bytes(d.n, d.tile_blocks,
                                                                d.rec_global != 0, met != 0));
    }
    tiles.clear();
    groups.clear();
    for (auto &kv : by_launch) {
        groups.push_back(TileGroup{std::get<0>(kv.first), std::get<1>(kv.first),
                                   std::get<2>(kv.first), std::get<3>(kv.first), tiles.size(),
                                   kv.second.size(), lds_of[kv.first]});
        tiles.insert(tiles.end(), kv.second.begin(), kv.second.end());
    }
    for (const TileGroup &g : groups)
        if (g.lds > 160 * 1024)
            return fail(XS_EINVAL, "a tile needs %zu bytes of LDS (max 163840)", g.lds);
    return XS_OK;
}

// Device scratch of the allocating entry points, kept for later calls: a small pool per device
// of buffers that calls lease and give back once their stream has finished (idle() after the
// final synchronisation). A call that fails before that frees its buffer instead (hipFree waits
// for the device). The pool keeps at most kPoolKeep buffers per device and frees the smallest
// beyond that; what it holds at exit is left to the process teardown.
struct ScratchPool {
    std::mutex mu;
    std::map<int, std::vector<std::pair<size_t, uint8_t *>>> free;  // per device
};
ScratchPool g_pool;
constexpr size_t kPoolKeep = 4;

struct ScratchLease {
    int device = -1;
    size_t bytes = 0;
    uint8_t *p = nullptr;
    bool is_idle = false;
    void idle() { is_idle = true; }
    xs_status take(int dev, size_t need) {
        device = dev;
        {
            std::lock_guard<std::mutex> lock(g_pool.mu);
            auto &v = g_pool.free[dev];
            size_t best = SIZE_MAX;
            for (size_t k = 0; k < v.size(); ++k)
                if (v[k].first >= need && (best == SIZE_MAX || v[k].first < v[best].first))
                    best = k;
            if (best != SIZE_MAX) {
                bytes = v[best].first;
                p = v[best].second;
                v.erase(v.begin() + best);
                return XS_OK;
            }
        }
        bytes = std::max<size_t>(need, 1 << 16);
        void *q = nullptr;
        XS_HIP(hipMalloc(&q, bytes));
        p = static_cast<uint8_t *>(q);
        return XS_OK;
    }
    ~ScratchLease() {
        if (!p) return;
        if (!is_idle) {
            (void)hipFree(p);
            return;
        }
        std::vector<uint8_t *> drop;
        {
            std::lock_guard<std::mutex> lock(g_pool.mu);
            auto &v = g_pool.free[device];
            v.emplace_back(bytes, p);
            while (v.size() > kPoolKeep) {
                auto it = std::min_element(v.begin(), v.end());
                drop.push_back(it->second);
                v.erase(it);
            }
        }
        for (uint8_t *q : drop) (void)hipFree(q);
    }
};

// Batches run an instance whose tiles read their records from global memory in its gauge
// where one exists (every coupling +1, three fewer operations per task: measured 3-7 % faster
// at N = 512-1024; with records in LDS the gauged kernel measured slower, so those keep the
// couplings). Finding the gauge costs up to n^3/128 word operations, once per instance: done
// for n <= 512, for runs of 2^36 clone-spin updates or more, or with XS_PLACE_ROWS; otherwise
// a gauge found earlier is used.
void choose_gauge(std::vector<xs::InstDev> &h, const xs_instance *const *insts,
                  const xs_run_config *cfgs, int count) {
    for (int k = 0; k < count; ++k) {
        const xs_instance *I = insts[k];
        xs::InstDev &d = h[k];
        d.j0 = 0;
        if (!d.rec_global) continue;
        std::lock_guard<std::mutex> lock(I->mu);
        if (I->gauge_state == 0) {
            const double upd = 64.0 * d.n_words * d.n * (double)(d.t_stop - d.t_cur);
            if (I->n <= 512 || upd >= 68719476736.0 || (cfgs[k].flags & XS_PLACE_ROWS))
                I->gauge_state = solve_gauge(*I, I->gauge) ? 1 : -1;
        }
        d.j0 = I->gauge_state == 1 ? 1u : 0u;
    }
}

// A batch run as persistent work-queue launches (qg_queue_run): one launch per epoch of up to
// epoch_chunks chunks of every unfinished instance, instead of a launch per chunk and launch
// shape.
struct QueuePlan {
    bool on = false;
    uint32_t threads = 0;
    bool met = false;
    size_t lds = 0;
    int grid = 0;
    uint32_t epoch_chunks = 0;
    std::vector<uint2> tiles;     // largest tiles first, each instance's tiles together
    std::vector<uint32_t> order;  // instance indices in tile-list order
};

// Queue mode needs one workgroup size and one rule for the whole batch and column widths of 8
// or 16 bytes. The workgroup size is the configs' explicit one, else the default of the
// instance with the most work; every descriptor then takes it (its step cap follows). The ring
// takes 8 bytes per tile and chunk of an epoch, within ring_budget bytes. Leaves qp.on false
// (launch per chunk) when the batch does not qualify.
xs_status plan_queue(std::vector<xs::InstDev> &h_io, const xs_instance *const *insts,
                     const xs_run_config *cfgs, int count, int device, size_t ring_budget,
                     QueuePlan &qp) {
    qp.on = false;
    std::vector<xs::InstDev> h = h_io;  // committed only if the batch runs from the queue
    const bool met = h[0].thr0 != 0;
    uint32_t T = 0;
    int heavy = 0;
    double heavy_work = -1.0, upd_chunk = 0.0;
    size_t n_tiles = 0;
    for (int k = 0; k < count; ++k) {
        const xs::InstDev &d = h[k];
        if ((cfgs[k].flags & XS_PER_CHUNK) || (d.thr0 != 0) != met) return XS_OK;
        if (d.col_bytes != 8 && d.col_bytes != 16) return XS_OK;
        if (cfgs[k].wg_threads) {
            if (T && T != cfgs[k].wg_threads) return XS_OK;
            T = cfgs[k].wg_threads;
        }
        const double clones = 64.0 * d.n_words;
        const double work = clones * d.n * (double)(d.t_stop - d.t_cur);
        if (work > heavy_work) {
            heavy_work = work;
            heavy = k;
        }
        if (!d.done) upd_chunk += clones * d.n * d.chunk;
        n_tiles += d.n_words * 64 / 256 / d.tile_blocks;
    }
    if (!T) T = h[heavy].wg_threads;
    if (T != 256 && T != 512) return XS_OK;
    // Every workgroup of the launch reserves the largest tile's LDS. Tiles of library-chosen
    // size whose LDS would lower the number of workgroups per CU that the instance with the
    // most work gets are halved until they fit its share.
    auto lds_of = [&](const xs::InstDev &d) {
        return xs::chunk_lds_bytes(d.n, d.tile_blocks, d.rec_global != 0, met);
    };
    constexpr size_t kLdsCu = 160 * 1024 - 64;  // per CU, less the kernel's own 8 bytes
    int occ_threads = 0;
    XS_HIP(xs::queue_blocks_per_cu((int)T, met, 0, &occ_threads));
    const size_t lds_heavy = lds_of(h[heavy]);
    if (occ_threads <= 0 || lds_heavy > kLdsCu) return XS_OK;
    const size_t occ = std::min<size_t>((size_t)occ_threads, kLdsCu / lds_heavy);
    const size_t lds_cap = kLdsCu / occ;
    for (int k = 0; k < count; ++k) {
        xs::InstDev &d = h[k];
        if (cfgs[k].tile_blocks) continue;
        while (d.tile_blocks > 1 && lds_of(d) > lds_cap) {
            d.tile_blocks /= 2;
            d.log2_tile_blocks -= 1;
        }
        if (d.col_bytes == 16 && d.tile_blocks == 1 && !cfgs[k].col_bytes) d.col_bytes = 8;
    }
    size_t lds = 0;
    n_tiles = 0;
    for (int k = 0; k < count; ++k) {
        if (8 * h[k].tile_blocks > T) return XS_OK;
        lds = std::max(lds, lds_of(h[k]));
        n_tiles += h[k].n_words * 64 / 256 / h[k].tile_blocks;
    }
    if (lds > kLdsCu) return XS_OK;
    // Epoch: about two seconds of the batch's sweeps at 10 K updates/ns, 1 to 64 chunks, and
    // no more than the ring budget holds.
    uint32_t E = (uint32_t)std::max(1.0, std::min(64.0, 2.0 / (upd_chunk / 1e13 + 1e-12)));
    E = (uint32_t)std::min<size_t>(E, ring_budget / (8 * std::max<size_t>(n_tiles, 1)));
    if (E < 1 || n_tiles * E >= 0xFFFFFFFFull) return XS_OK;
    // Epochs of equal length over the longest budget (100 chunks at most 11 per epoch: ten of
    // ten, not nine of eleven and one of one).
    uint64_t most_chunks = 1;
    for (int k = 0; k < count; ++k)
        if (!h[k].done)
            most_chunks = std::max<uint64_t>(
                most_chunks, (h[k].t_stop - h[k].t_cur + h[k].chunk - 1) / h[k].chunk);
    const uint64_t epochs = (most_chunks + E - 1) / E;
    E = (uint32_t)((most_chunks + epochs - 1) / epochs);
    int per_cu = 0, cus = 0;
    XS_HIP(xs::queue_blocks_per_cu((int)T, met, lds, &per_cu));
    XS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    if (per_cu <= 0 || cus <= 0) return XS_OK;
    // Largest tiles (spins x blocks) first; an instance's tiles stay together.
    qp.order.resize(count);
    for (int k = 0; k < count; ++k) qp.order[k] = (uint32_t)k;
    std::stable_sort(qp.order.begin(), qp.order.end(), [&](uint32_t a, uint32_t b) {
        return (uint64_t)h[a].n * h[a].tile_blocks > (uint64_t)h[b].n * h[b].tile_blocks;
    });
    qp.tiles.clear();
    qp.tiles.reserve(n_tiles);
    for (uint32_t k : qp.order) {
        xs::InstDev &d = h[k];
        const uint32_t nb = d.n_words * 64 / 256;
        d.tile0 = (uint32_t)qp.tiles.size();
        d.ntiles = nb / d.tile_blocks;
        for (uint32_t b0 = 0; b0 < nb; b0 += d.tile_blocks) qp.tiles.push_back(make_uint2(k, b0));
        d.wg_threads = T;
    }
    choose_gauge(h, insts, cfgs, count);
    qp.threads = T;
    qp.met = met;
    qp.lds = lds;
    qp.grid = (int)std::min<size_t>((size_t)per_cu * cus, qp.tiles.size());
    qp.epoch_chunks = E;
    qp.on = true;
    h_io.swap(h);
    return XS_OK;
}

xs_status run_batch(int32_t count, const xs_instance *const *insts, const xs_run_config *cfgs,
                    const xs_run_buffers *bufs, hipStream_t stream, xs_run_result *results,
                    const RunOpts &opt) {
    const auto wall0 = std::chrono::steady_clock::now();
    if (count <= 0 || !insts || !cfgs || !bufs || !results)
        return fail(XS_EINVAL, "empty or null batch");
    int device = 0;
    XS_HIP(hipGetDevice(&device));

    std::vector<xs::InstDev> h(count);
    std::vector<uint2> tiles;
    const bool fixed = opt.fixed != nullptr;
    for (int k = 0; k < count; ++k) {
        xs_status st = validate_run(insts[k], &cfgs[k], &bufs[k], true);
        if (st != XS_OK) return st;
        DeviceTables t;
        if (!fixed) {
            st = ensure_tables(insts[k], device, &t);
            if (st != XS_OK) return st;
        }
        fill_desc(insts[k], cfgs[k], t, bufs[k].state, bufs[k].first_hit, bufs[k].energy, h[k]);
    }
    std::vector<TileGroup> groups;
    QueuePlan qp;
    {
        xs_status st = tile_instances(h, cfgs, count, tiles, groups);
        if (st != XS_OK) return st;
        st = plan_queue(h, insts, cfgs, count, device, fixed ? opt.fixed_bytes / 2 : SIZE_MAX,
                        qp);
        if (st != XS_OK) return st;
        if (qp.on)
            tiles.swap(qp.tiles);
        else
            choose_gauge(h, insts, cfgs, count);  // the launch per chunk runs gauges too
        if (!fixed) {
            st = attach_tables(h, insts, count, device);
            if (st != XS_OK) return st;
        }
    }
    // Device scratch of the call: descriptors, tiles, the running-instance counter and the
    // winners' spins (and, with fixed scratch, the instances' tables).
    auto a256 = [](size_t v) { return (v + 255) & ~size_t(255); };
    size_t solved_bytes = 0;
    std::vector<size_t> solved_off(count);
    for (int k = 0; k < count; ++k) {
        solved_off[k] = solved_bytes;
        solved_bytes += (h[k].n + 15) & ~15u;
    }
    const size_t off_tiles = a256(sizeof(xs::InstDev) * count);
    const size_t off_active = off_tiles + a256(sizeof(uint2) * tiles.size());
    const size_t off_solved = off_active + 256;
    size_t total = off_solved + solved_bytes;
    // Queue mode: the queue counters, the instance order and the ring.
    const size_t off_queue = a256(total);
    const size_t off_order = off_queue + a256(sizeof(xs::QueueDev));
    const size_t off_ring = off_order + a256(sizeof(uint32_t) * count);
    const uint32_t ring_cap = qp.on ? (uint32_t)(tiles.size() * qp.epoch_chunks) : 0u;
    if (qp.on) total = off_ring + sizeof(uint64_t) * ring_cap;
    // Fixed scratch: each distinct (instance, schedule, tiling, record placement) gets its
    // tables (triplets, records, step offsets, row map, global-memory records) in one host
    // image after the staging area, copied with one transfer; descriptors take their offsets.
    const size_t off_tables = a256(total);
    std::vector<uint8_t> image;
    struct TabOff {
        size_t tri, rec, off, rowmap, grec, gauge, boff, bgrec;
        uint32_t steps, bsteps;
    };
    std::vector<TabOff> tab_of(count);
    if (fixed) {
        std::map<std::tuple<const xs_instance *, uint32_t, uint32_t, uint32_t>, int> seen;
        auto put = [&](const void *src, size_t bytes) {
            const size_t at = image.size();
            image.resize(a256(at + bytes), 0);
            std::memcpy(image.data() + at, src, bytes);
            return at;
        };
        for (int k = 0; k < count; ++k) {
            const xs_instance *I = insts[k];
            std::lock_guard<std::mutex> lock(I->mu);
            uint32_t key = 0;
            const xsh::HostSched &hs = host_sched(I, h[k], &key);
            const auto id = std::make_tuple(I, key, h[k].tile_blocks, h[k].rec_global);
            auto it = seen.find(id);
            if (it != seen.end()) {
                tab_of[k] = tab_of[it->second];
                continue;
            }
            seen.emplace(id, k);
            const size_t n = (size_t)I->n;
            TabOff &o = tab_of[k];
            o.tri = put(I->tri16.data(), 8 * n);
            o.rec = put(hs.rec.data(), 16 * n);
            o.off = put(hs.off.data(), sizeof(int32_t) * hs.off.size());
            o.rowmap = hs.rowmap.empty() ? SIZE_MAX : put(hs.rowmap.data(), 2 * n);
            o.gauge = h[k].j0 ? put(I->gauge.data(), n) : SIZE_MAX;
            o.grec = SIZE_MAX;
            o.boff = o.bgrec = SIZE_MAX;
            o.bsteps = 0;
            if (h[k].rec_global) {
                const std::vector<uint32_t> g = grec_image(hs.rec, I->n, h[k].tile_blocks);
                o.grec = put(g.data(), 16 * n);
                if (!hs.border.empty() && wants_body(h[k])) {
                    const std::vector<uint32_t> gb = grec_image(hs.brec, I->n, h[k].tile_blocks);
                    o.bgrec = put(gb.data(), 16 * n);
                    o.boff = put(hs.boff.data(), sizeof(int32_t) * hs.boff.size());
                    o.bsteps = (uint32_t)hs.boff.size() - 1;
                }
            }
            o.steps = (uint32_t)hs.off.size() - 1;
        }
        total = off_tables + image.size();
        if (total > opt.fixed_bytes)
            return fail(XS_EINVAL,
                        "the batch needs %zu bytes of device scratch, more than the %zu the "
                        "no-allocation entry point has",
                        total, opt.fixed_bytes);
    }
    uint8_t *scratch = opt.fixed;
    ScratchLease lease;
    if (!fixed) {
        const xs_status st = lease.take(device, total);
        if (st != XS_OK) return st;
        scratch = lease.p;
    }
    for (int k = 0; k < count; ++k)
        h[k].solved = reinterpret_cast<int8_t *>(scratch + off_solved + solved_off[k]);
    if (fixed) {
        uint8_t *tb = scratch + off_tables;
        for (int k = 0; k < count; ++k) {
            const TabOff &o = tab_of[k];
            xs::InstDev &d = h[k];
            d.tri = reinterpret_cast<const uint2 *>(tb + o.tri);
            d.rec = reinterpret_cast<const uint4 *>(tb + o.rec);
            d.step_off = reinterpret_cast<const int32_t *>(tb + o.off);
            d.rowmap = o.rowmap == SIZE_MAX ? nullptr
                                            : reinterpret_cast<const uint16_t *>(tb + o.rowmap);
            d.grec = o.grec == SIZE_MAX ? nullptr : reinterpret_cast<const uint4 *>(tb + o.grec);
            d.gauge = o.gauge == SIZE_MAX ? nullptr : reinterpret_cast<const uint8_t *>(tb + o.gauge);
            d.n_steps = o.steps;
            d.bgrec = o.bgrec == SIZE_MAX ? nullptr : reinterpret_cast<const uint4 *>(tb + o.bgrec);
            d.bstep_off =
                o.boff == SIZE_MAX ? nullptr : reinterpret_cast<const int32_t *>(tb + o.boff);
            d.n_bsteps = o.bsteps;
        }
        if (!image.empty())
            XS_HIP(hipMemcpyAsync(tb, image.data(), image.size(), hipMemcpyHostToDevice, stream));
    }
    xs::InstDev *d_inst = reinterpret_cast<xs::InstDev *>(scratch);
    uint2 *d_tiles = reinterpret_cast<uint2 *>(scratch + off_tiles);
    uint32_t *d_active = reinterpret_cast<uint32_t *>(scratch + off_active);

    XS_HIP(hipMemcpyAsync(d_inst, h.data(), sizeof(xs::InstDev) * count, hipMemcpyHostToDevice,
                          stream));
    XS_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(uint2) * tiles.size(),
                          hipMemcpyHostToDevice, stream));
    xs::QueueDev *d_q = reinterpret_cast<xs::QueueDev *>(scratch + off_queue);
    uint32_t *d_order = reinterpret_cast<uint32_t *>(scratch + off_order);
    uint64_t *d_ring = reinterpret_cast<uint64_t *>(scratch + off_ring);
    xs::QueueDev q_init{};
    if (qp.on) {
        q_init.ring = d_ring;
        q_init.cap = ring_cap;
        int clock_khz = 0;  // wall-clock rate of wall_clock64()
        XS_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device));
        q_init.wait_limit = (uint64_t)std::max(clock_khz, 1) * 1000ull * 60ull;  // a minute
        XS_HIP(hipMemcpyAsync(d_q, &q_init, sizeof q_init, hipMemcpyHostToDevice, stream));
        XS_HIP(hipMemcpyAsync(d_order, qp.order.data(), sizeof(uint32_t) * count,
                              hipMemcpyHostToDevice, stream));
        XS_HIP(xs::launch_queue_clear(d_ring, ring_cap, stream));
    }
    for (int k = 0; k < count; ++k) XS_HIP(xs::launch_init(d_inst + k, h[k], stream));
    // Instances run in their gauge hold the flipped state from here to the final pass.
    uint64_t gauge_pieces = 0;
    for (int k = 0; k < count; ++k)
        if (h[k].j0) gauge_pieces = std::max<uint64_t>(gauge_pieces, (uint64_t)h[k].n * h[k].n_words / 2);
    if (gauge_pieces) XS_HIP(xs::launch_gauge_flip(d_inst, count, gauge_pieces, stream));

    bool any_running = false;
    for (int k = 0; k < count; ++k) any_running |= !h[k].done;
    int group = 1;
    bool profile;
    {
        std::lock_guard<std::mutex> lock(g_prof.mu);
        profile = g_prof.on;
    }
    const bool timed = !fixed && (profile || opt.kernel_ms);  // events are HIP objects
    std::vector<hipEvent_t> ev;
    struct Events {
        std::vector<hipEvent_t> *v;
        ~Events() { for (auto e : *v) (void)hipEventDestroy(e); }
    } ev_guard{&ev};
    xs_kernel_stats local{};
    ChunkGraph cg;
    auto enqueue_chunks = [&](hipStream_t s, int n, bool with_events) -> xs_status {
        for (int g = 0; g < n; ++g) {
            if (with_events) XS_HIP(hipEventRecord(ev[2 * g], s));
            for (const TileGroup &gr : groups)
                XS_HIP(xs::launch_chunk(d_inst, d_tiles + gr.first, (int)gr.count,
                                        (int)gr.threads, (int)gr.col_bytes, gr.rec_global != 0,
                                        gr.met != 0,
                                        gr.lds, s));
            if (with_events) XS_HIP(hipEventRecord(ev[2 * g + 1], s));
            XS_HIP(xs::launch_decide(d_inst, count, d_active, s));
        }
        return XS_OK;
    };
    // Queue mode: per epoch, the set-up kernel and one persistent launch; the host reads the
    // count of unfinished instances (and the queue's error flag) after each.
    for (uint32_t gen = 1; qp.on && any_running; ++gen) {
        if (timed)
            while (ev.size() < 2) {
                hipEvent_t e;
                XS_HIP(hipEventCreate(&e));
                ev.push_back(e);
            }
        XS_HIP(xs::launch_queue_setup(d_inst, count, d_order, d_tiles, (uint32_t)tiles.size(), d_q,
                                      gen, qp.epoch_chunks, stream));
        if (timed) XS_HIP(hipEventRecord(ev[0], stream));
        XS_HIP(xs::launch_queue_run(d_inst, d_tiles, d_q, gen, (int)qp.threads, qp.met, qp.lds,
                                    qp.grid, stream));
        if (timed) XS_HIP(hipEventRecord(ev[1], stream));
        xs::QueueDev qh;
        XS_HIP(hipMemcpyAsync(&qh, d_q, sizeof qh, hipMemcpyDeviceToHost, stream));
        XS_HIP(hipStreamSynchronize(stream));
        if (qh.error)
            return fail(XS_EDEVICE, "persistent launch: a workgroup's wait for work reached its "
                                    "time limit");
        if (timed) {
            float ms = 0.f;
            XS_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            local.total_ms += ms;
            local.launches += 1;
        }
        any_running = qh.active != 0;
    }
    // Chunk loop: chunk launches over all tiles, then the device-side decision. The host reads
    // the count of running instances every `group` chunks (finished instances' tiles exit at
    // once, so launching ahead changes no result). Untimed loops of two or more chunks are
    // replayed from a captured graph.
    while (any_running) {
        if (timed)
            while (ev.size() < 2 * (size_t)group) {
                hipEvent_t e;
                XS_HIP(hipEventCreate(&e));
                ev.push_back(e);
            }
        if (!timed && opt.graph && !fixed && group >= 2) {
            // A graph of at most kGraphChunks chunks, launched group / g times: larger groups
            // reuse it instead of capturing and instantiating a graph per size.
            const int g = std::min(group, kGraphChunks);
            if (cg.group != g) {
                cg.reset();
                if (!cg.cap) XS_HIP(hipStreamCreateWithFlags(&cg.cap, hipStreamNonBlocking));
                XS_HIP(hipStreamBeginCapture(cg.cap, hipStreamCaptureModeRelaxed));
                const xs_status st = enqueue_chunks(cg.cap, g, false);
                hipGraph_t gph = nullptr;
                const hipError_t e_end = hipStreamEndCapture(cg.cap, &gph);
                if (st != XS_OK) {
                    if (gph) (void)hipGraphDestroy(gph);
                    return st;
                }
                XS_HIP(e_end);
                cg.graph = gph;
                XS_HIP(hipGraphInstantiate(&cg.exec, cg.graph, nullptr, nullptr, 0));
                cg.group = g;
            }
            for (int r = 0; r < group / g; ++r) XS_HIP(hipGraphLaunch(cg.exec, stream));
        } else {
            const xs_status st = enqueue_chunks(stream, group, timed);
            if (st != XS_OK) return st;
        }
        uint32_t active = 0;
        XS_HIP(hipMemcpyAsync(&active, d_active, sizeof active, hipMemcpyDeviceToHost, stream));
        XS_HIP(hipStreamSynchronize(stream));
        any_running = active != 0;
        if (timed)
            for (int g = 0; g < group; ++g) {
                float ms = 0.f;
                XS_HIP(hipEventElapsedTime(&ms, ev[2 * g], ev[2 * g + 1]));
                local.total_ms += ms;
                local.launches += 1;
            }
        // Read back less and less often: chunks launched after every instance has finished cost
        // only their launch (every tile exits at once), while each read-back drains the GPU.
        if (group < 64) group *= 2;
    }
    {
        uint32_t max_words = 0, max_n = 0;
        for (int k = 0; k < count; ++k) {
            max_words = std::max(max_words, h[k].n_words);
            max_n = std::max(max_n, h[k].n);
        }
        if (gauge_pieces) XS_HIP(xs::launch_gauge_flip(d_inst, count, gauge_pieces, stream));
        XS_HIP(xs::launch_final(d_inst, count, max_words, max_n, stream));
    }
    std::vector<xs::InstDev> out(count);
    XS_HIP(hipMemcpyAsync(out.data(), d_inst, sizeof(xs::InstDev) * count, hipMemcpyDeviceToHost,
                          stream));
    std::vector<int8_t> solved(solved_bytes);
    if (solved_bytes)
        XS_HIP(hipMemcpyAsync(solved.data(), scratch + off_solved, solved_bytes,
                              hipMemcpyDeviceToHost, stream));
    XS_HIP(hipStreamSynchronize(stream));
    lease.idle();
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    for (int k = 0; k < count; ++k) {
        const xs::InstDev &d = out[k];
        xs_run_result &r = results[k];
        r.tts_sweeps = d.tts == INT32_MAX ? -1 : d.tts;
        r.winner_clone = d.winner == INT32_MAX ? -1 : d.winner;
        r.end_sweep = d.t_cur;
        r.sweeps_done = d.t_cur - d.t_start;
        r.tile_blocks = d.tile_blocks;
        r.wg_threads = d.wg_threads;
        r.col_bytes = d.col_bytes;
        r.rec_global = d.rec_global;
        r.persistent = qp.on ? 1u : 0u;
        r.clone_spin_updates = (uint64_t)d.n_words * 64 * d.n * r.sweeps_done;
        r.seconds = secs;
        if (bufs[k].solved && d.winner != INT32_MAX)
            std::memcpy(bufs[k].solved, solved.data() + solved_off[k], d.n);
        local.clone_spin_updates += r.clone_spin_updates;
    }
    if (opt.kernel_ms) *opt.kernel_ms += local.total_ms;
    if (profile) {
        std::lock_guard<std::mutex> lock(g_prof.mu);
        g_prof.stats.launches += local.launches;
        g_prof.stats.total_ms += local.total_ms;
        g_prof.stats.clone_spin_updates += local.clone_spin_updates;
    }
    return XS_OK;
}

}  // namespace xsh

using namespace xsh;

extern "C" {

int32_t xs_abi_version(void) { return XS_ABI_VERSION; }

const char *xs_status_str(xs_status s) {
    switch (s) {
        case XS_OK: return "XS_OK";
        case XS_EINVAL: return "XS_EINVAL";
        case XS_ENOMEM: return "XS_ENOMEM";
        case XS_EDEVICE: return "XS_EDEVICE";
        case XS_EAGAIN: return "XS_EAGAIN";
        case XS_ENOTFOUND: return "XS_ENOTFOUND";
        case XS_ECANCELED: return "XS_ECANCELED";
        default: return "XS_UNKNOWN";
    }
}

const char *xs_last_error(void) { return g_last_error.c_str(); }

xs_status xs_instance_create(int32_t n, int32_t m, const int32_t *tri, const int8_t *J,
                             int32_t colour_cap, xs_instance **out) {
    return guarded([&]() -> xs_status {
        if (!out) return fail(XS_EINVAL, "out is null");
        *out = nullptr;
        if (!tri || !J) return fail(XS_EINVAL, "tri and J are required");
        if (n < 4 || n > XS_MAX_N) return fail(XS_EINVAL, "n = %d outside [4, %d]", n, XS_MAX_N);
        if (m != n) return fail(XS_EINVAL, "m = %d must equal n = %d", m, n);
        if (colour_cap < 0 || colour_cap > XS_MAX_N)
            return fail(XS_EINVAL, "colour_cap = %d outside [0, %d]", colour_cap, XS_MAX_N);
        std::vector<int32_t> deg(n, 0);
        for (int t = 0; t < m; ++t) {
            const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
            if (a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= n)
                return fail(XS_EINVAL, "triplet %d has an index outside [0, %d)", t, n);
            if (a == b || a == c || b == c)
                return fail(XS_EINVAL, "triplet %d repeats a spin", t);
            if (J[t] != 1 && J[t] != -1) return fail(XS_EINVAL, "J[%d] = %d is not +1/-1", t, J[t]);
            ++deg[a];
            ++deg[b];
            ++deg[c];
        }
        for (int v = 0; v < n; ++v)
            if (deg[v] != 3) return fail(XS_EINVAL, "spin %d is in %d triplets, not 3", v, deg[v]);
        xs_instance *I = new (std::nothrow) xs_instance;
        if (!I) return fail(XS_ENOMEM, "host allocation failed");
        I->n = n;
        I->cap = colour_cap ? colour_cap : 32;
        I->tri.assign(tri, tri + 3 * (size_t)m);
        I->J.assign(J, J + m);
        partition(*I);
        build_triplets(*I);
        // uncapped steps, reported by get_info
        I->sched.emplace(sched_key(0, 0), make_schedule(*I, 0, 0, 0, false, false));
        *out = I;
        return XS_OK;
    });
}

void xs_instance_destroy(xs_instance *I) {
    if (!I) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto &kv : I->dev) {
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second.tri);
        (void)hipFree(kv.second.gauge);
        for (auto &s : kv.second.sched) {
            (void)hipFree(s.second.rec);
            (void)hipFree(s.second.off);
            (void)hipFree(s.second.rowmap);
            for (auto &g : s.second.grec) (void)hipFree(g.second);
            (void)hipFree(s.second.boff);
            for (auto &g : s.second.bgrec) (void)hipFree(g.second);
        }
    }
    if (cur >= 0 && !I->dev.empty()) (void)hipSetDevice(cur);
    delete I;
}

xs_status xs_instance_get_info(const xs_instance *I, xs_instance_info *info) {
    return guarded([&]() -> xs_status {
        if (!I || !info) return fail(XS_EINVAL, "null argument");
        info->n = I->n;
        info->n_classes = (int32_t)I->class_off.size() - 1;
        info->colour_cap = I->cap;
        info->max_class = I->max_class;
        std::lock_guard<std::mutex> lock(I->mu);
        const xsh::HostSched &lv = I->sched.at(sched_key(0, 0));
        info->n_levels = (int32_t)lv.off.size() - 1;
        info->max_level = lv.max_step;
        return XS_OK;
    });
}

xs_status xs_instance_get_partition(const xs_instance *I, int32_t *perm, int32_t *class_off) {
    return guarded([&]() -> xs_status {
        if (!I || !perm || !class_off) return fail(XS_EINVAL, "null argument");
        std::memcpy(perm, I->perm.data(), sizeof(int32_t) * I->perm.size());
        std::memcpy(class_off, I->class_off.data(), sizeof(int32_t) * I->class_off.size());
        return XS_OK;
    });
}

xs_status xs_instance_get_schedule(const xs_instance *I, uint32_t step_cap, int32_t *order,
                                   int32_t *step_off, int32_t *n_steps) {
    return guarded([&]() -> xs_status {
        if (!I || !order || !step_off || !n_steps) return fail(XS_EINVAL, "null argument");
        std::lock_guard<std::mutex> lock(I->mu);
        const uint32_t cap = std::min<uint32_t>(step_cap, 0xFFFFu);  // at least n: no limit
        auto it = I->sched.find(sched_key(cap, 0));
        if (it == I->sched.end())
            it = I->sched.emplace(sched_key(cap, 0), make_schedule(*I, cap, 0, 0, false, false)).first;
        const xsh::HostSched &hs = it->second;
        std::memcpy(order, hs.order.data(), sizeof(int32_t) * hs.order.size());
        std::memcpy(step_off, hs.off.data(), sizeof(int32_t) * hs.off.size());
        *n_steps = (int32_t)hs.off.size() - 1;
        return XS_OK;
    });
}

xs_status xs_instance_get_body(const xs_instance *I, uint32_t step_cap, int32_t *order,
                               int32_t *step_off, uint8_t *late, int32_t *n_steps) {
    return guarded([&]() -> xs_status {
        if (!I || !order || !step_off || !late || !n_steps) return fail(XS_EINVAL, "null argument");
        if (step_cap == 0 || step_cap > 0xFFFFu)
            return fail(XS_EINVAL, "step_cap %u outside [1, 65535]", step_cap);
        std::lock_guard<std::mutex> lock(I->mu);
        const uint32_t key = sched_key(step_cap, 0, false, true);
        auto it = I->sched.find(key);
        if (it == I->sched.end())
            it = I->sched.emplace(key, make_schedule(*I, step_cap, 0, 0, false, true)).first;
        const xsh::HostSched &hs = it->second;
        if (hs.border.empty()) return fail(XS_ENOTFOUND, "no cross-sweep body for this cap");
        std::memcpy(order, hs.border.data(), sizeof(int32_t) * hs.border.size());
        std::memcpy(step_off, hs.boff.data(), sizeof(int32_t) * hs.boff.size());
        for (int p = 0; p < I->n; ++p) late[hs.border[p]] = (hs.brec[8 * (size_t)p + 7] >> 12) & 1;
        *n_steps = (int32_t)hs.boff.size() - 1;
        return XS_OK;
    });
}

xs_status xs_autotune(const xs_instance *inst, uint32_t n_clones, int32_t count, void *stream_v,
                      xs_tune_result *out) {
    return guarded([&]() -> xs_status {
        if (!inst || !out || count <= 0) return fail(XS_EINVAL, "null argument or count <= 0");
        if (n_clones == 0 || n_clones % XS_CLONE_QUANTUM)
            return fail(XS_EINVAL, "n_clones %u is not a positive multiple of %d", n_clones,
                        XS_CLONE_QUANTUM);
        if (n_clones > XS_MAX_CLONES)
            return fail(XS_EINVAL, "n_clones %u > %u", n_clones, XS_MAX_CLONES);
        hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
        const uint32_t n = (uint32_t)inst->n, nb = n_clones / 256;
        const size_t state_bytes = (size_t)n * n_clones / 8;
        const int copies = (int)std::max<size_t>(1, std::min<size_t>((size_t)count,
                                                                     (size_t(2) << 30) / state_bytes));
        // Sweeps per trial: about 4e10 clone-spin updates, between 8 and 200.
        const double upd_per_sweep = (double)copies * n_clones * n;
        const uint32_t sweeps = (uint32_t)std::min(200.0, std::max(8.0, 4e10 / upd_per_sweep));
        uint8_t *mem = nullptr;
        const size_t fh_bytes = sizeof(int32_t) * n_clones;
        const size_t per = ((state_bytes + 255) & ~size_t(255)) + ((fh_bytes + 255) & ~size_t(255));
        XS_HIP(hipMalloc(&mem, per * copies));
        struct Free {
            uint8_t *p;
            ~Free() { if (p) (void)hipFree(p); }
        } guard{mem};
        std::vector<const xs_instance *> insts(copies, inst);
        std::vector<xs_run_config> cfgs(copies);
        std::vector<xs_run_buffers> bufs(copies);
        std::vector<xs_run_result> res(copies);
        for (int k = 0; k < copies; ++k) {
            xs_run_config &c = cfgs[k];
            std::memset(&c, 0, sizeof c);
            c.struct_size = sizeof c;
            c.instance_id = (uint32_t)k;
            c.seed = 0x5EEDull + k;
            c.n_clones = n_clones;
            c.accept_thr = 3604;
            c.max_sweeps = sweeps;
            c.chunk_sweeps = sweeps;
            bufs[k].state = reinterpret_cast<uint64_t *>(mem + per * k);
            bufs[k].first_hit = reinterpret_cast<int32_t *>(mem + per * k + ((state_bytes + 255) & ~size_t(255)));
            bufs[k].energy = nullptr;
            bufs[k].solved = nullptr;
        }
        std::memset(out, 0, sizeof *out);
        for (uint32_t B = 1; B <= (uint32_t)xs::kMaxTileBlocks; B *= 2) {
            if (nb % B || n * B > 2048 || xs::chunk_lds_bytes(n, B, true, false) > 160 * 1024) continue;
            for (uint32_t T = 128; T <= 1024; T *= 2) {
                if (T < 8 * B || (T == 128 && B > 2)) continue;
                for (uint32_t C = 4; C <= 16; C *= 2)
                    for (uint32_t G = (n >= 512 ? 1u : 2u); G <= 2; ++G) {
                        // skip columns that leave most threads without a task in a full step
                        if (32u * (8u * B / (C / 4)) < T / 4 || out->n_trials >= XS_TUNE_MAX_TRIALS)
                            continue;
                        if (xs::chunk_lds_bytes(n, B, G == 1, false) > 160 * 1024) continue;
                        for (auto &c : cfgs) {
                            c.tile_blocks = B;
                            c.wg_threads = T;
                            c.col_bytes = C;
                            c.rec_global = G;
                        }
                        RunOpts opt;
                        double ms = 0.0;
                        opt.kernel_ms = &ms;
                        xs_status st = run_batch(copies, insts.data(), cfgs.data(), bufs.data(),
                                                 stream, res.data(), opt);  // warm
                        if (st != XS_OK) return st;
                        ms = 0.0;
                        st = run_batch(copies, insts.data(), cfgs.data(), bufs.data(), stream,
                                       res.data(), opt);
                        if (st != XS_OK) return st;
                        uint64_t upd = 0;
                        for (auto &r : res) upd += r.clone_spin_updates;
                        const double rate = ms > 0 ? (double)upd / (ms * 1e6) : 0.0;
                        out->trials[out->n_trials++] = xs_tune_trial{B, T, C, G, rate};
                        if (rate > out->updates_per_ns) {
                            out->updates_per_ns = rate;
                            out->tile_blocks = B;
                            out->wg_threads = T;
                            out->col_bytes = C;
                            out->rec_global = G;
                        }
                    }
            }
        }
        if (!out->n_trials) return fail(XS_EINVAL, "no valid launch configuration");
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[tune_key(n, n_clones, count)] = TuneVal{out->tile_blocks, out->wg_threads,
                                                       out->col_bytes, out->rec_global,
                                                       out->updates_per_ns};
        return XS_OK;
    });
}

xs_status xs_tune_save(const char *path) {
    return guarded([&]() -> xs_status {
        if (!path) return fail(XS_EINVAL, "null path");
        FILE *f = std::fopen(path, "w");
        if (!f) return fail(XS_EINVAL, "cannot open %s for writing", path);
        std::lock_guard<std::mutex> lock(g_tune_mu);
        std::fprintf(f, "# n_bucket clones count_bucket tile_blocks wg_threads col_bytes "
                        "rec_global updates_per_ns\n");
        for (auto &kv : g_tune)
            std::fprintf(f, "%u %u %u %u %u %u %u %.1f\n", kv.first.n_bucket, kv.first.clones,
                         kv.first.count_bucket, kv.second.tile_blocks, kv.second.wg_threads,
                         kv.second.col_bytes, kv.second.rec_global, kv.second.rate);
        std::fclose(f);
        return XS_OK;
    });
}

xs_status xs_tune_load(const char *path) {
    return guarded([&]() -> xs_status {
        if (!path) return fail(XS_EINVAL, "null path");
        FILE *f = std::fopen(path, "r");
        if (!f) return fail(XS_ENOTFOUND, "cannot open %s", path);
        char line[256];
        std::lock_guard<std::mutex> lock(g_tune_mu);
        while (std::fgets(line, sizeof line, f)) {
            if (line[0] == '#') continue;
            unsigned nb_, cl, cb, B, T, C, G;
            double rate;
            if (std::sscanf(line, "%u %u %u %u %u %u %u %lf", &nb_, &cl, &cb, &B, &T, &C, &G,
                            &rate) != 8)
                continue;
            if (!B || (B & (B - 1)) || B > (unsigned)xs::kMaxTileBlocks || !T || (T & (T - 1)) ||
                T < 64 || T > 1024 || T < 8 * B || (C != 4 && C != 8 && C != 16) ||
                (G != 1 && G != 2))
                continue;
            g_tune[TuneKey{nb_, cl, cb}] = TuneVal{B, T, C, G, rate};
        }
        std::fclose(f);
        return XS_OK;
    });
}

xs_status xs_tune_clear(void) {
    return guarded([&]() -> xs_status {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune.clear();
        return XS_OK;
    });
}

xs_status xs_profile_enable(int32_t on) {
    return guarded([&]() -> xs_status {
        std::lock_guard<std::mutex> lock(g_prof.mu);
        g_prof.on = on != 0;
        return XS_OK;
    });
}

xs_status xs_profile_read(xs_kernel_stats *out, int32_t reset) {
    return guarded([&]() -> xs_status {
        if (!out) return fail(XS_EINVAL, "null argument");
        std::lock_guard<std::mutex> lock(g_prof.mu);
        *out = g_prof.stats;
        if (reset) g_prof.stats = xs_kernel_stats{};
        return XS_OK;
    });
}

xs_status xs_run(const xs_instance *inst, const xs_run_config *cfg, const xs_run_buffers *bufs,
                 void *stream, xs_run_result *result) {
    return guarded([&]() -> xs_status {
        return run_batch(1, &inst, cfg, bufs, reinterpret_cast<hipStream_t>(stream), result,
                         RunOpts{});
    });
}

xs_status xs_run_batch(int32_t count, const xs_instance *const *insts, const xs_run_config *cfgs,
                       const xs_run_buffers *bufs, void *stream, xs_run_result *results) {
    return guarded([&]() -> xs_status {
        return run_batch(count, insts, cfgs, bufs, reinterpret_cast<hipStream_t>(stream), results,
                         RunOpts{});
    });
}

xs_status xs_run_batch_noalloc(int32_t count, const xs_instance *const *insts,
                               const xs_run_config *cfgs, const xs_run_buffers *bufs,
                               void *stream, xs_run_result *results) {
    return guarded([&]() -> xs_status {
        RunOpts opt;
        opt.graph = false;
        XS_HIP(xs::noalloc_scratch(&opt.fixed, &opt.fixed_bytes));
        return run_batch(count, insts, cfgs, bufs, reinterpret_cast<hipStream_t>(stream), results,
                         opt);
    });
}

}  // extern "C"

struct xs_pending {
    std::vector<const xs_instance *> insts;
    std::vector<xs_run_config> cfgs;
    std::vector<xs_run_buffers> bufs;
    xs_run_result *results = nullptr;
    xs_status status = XS_OK;
    std::string error;
    std::thread worker;
};

extern "C" {

xs_status xs_run_batch_async(int32_t count, const xs_instance *const *insts,
                             const xs_run_config *cfgs, const xs_run_buffers *bufs, void *stream,
                             xs_run_result *results, xs_pending **out) {
    return guarded([&]() -> xs_status {
        if (!out) return fail(XS_EINVAL, "null argument");
        *out = nullptr;
        if (count <= 0 || !insts || !cfgs || !bufs || !results)
            return fail(XS_EINVAL, "empty or null batch");
        for (int k = 0; k < count; ++k) {
            xs_status st = validate_run(insts[k], &cfgs[k], &bufs[k], true);
            if (st != XS_OK) return st;
        }
        int device = 0;
        XS_HIP(hipGetDevice(&device));
        xs_pending *p = new (std::nothrow) xs_pending;
        if (!p) return fail(XS_ENOMEM, "host allocation failed");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        try {
            p->insts.assign(insts, insts + count);
            p->cfgs.assign(cfgs, cfgs + count);
            p->bufs.assign(bufs, bufs + count);
            p->results = results;
            p->worker = std::thread([p, device, s]() {
                if (hipSetDevice(device) != hipSuccess) {
                    p->status = XS_EDEVICE;
                    p->error = "hipSetDevice failed in the run thread";
                    return;
                }
                p->status = guarded([&]() -> xs_status {
                    return run_batch((int32_t)p->insts.size(), p->insts.data(), p->cfgs.data(),
                                     p->bufs.data(), s, p->results, RunOpts{});
                });
                if (p->status != XS_OK) {
                    try {
                        p->error = g_last_error;
                    } catch (...) {  // xs_wait still returns the status
                    }
                }
            });
        } catch (...) {
            delete p;
            return fail(XS_ENOMEM, "host allocation or run thread start failed");
        }
        *out = p;
        return XS_OK;
    });
}

xs_status xs_wait(xs_pending *p) {
    return guarded([&]() -> xs_status {
        if (!p) return fail(XS_EINVAL, "null argument");
        p->worker.join();
        const xs_status st = p->status;
        if (st != XS_OK) g_last_error = p->error;
        delete p;
        return st;
    });
}

}  // extern "C"
