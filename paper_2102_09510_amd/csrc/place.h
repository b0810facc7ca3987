// LDS row placement: which LDS row holds each spin, which spins of a step share an LDS pass,
// and in which order a task reads its partners. Host code only (the standard library), used by
// the schedule builder.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <utility>
#include <vector>

namespace xsh {

// LDS passes of a row access (measured on gfx950 with a probe of lane pairs and bank
// conflicts): ds_read_b64 serves lanes 0-31 and 32-63 in two passes; ds_read_b128 serves four
// passes of 16 lanes, lanes with the same l >> 5 and the same parity of the bits of
// (l >> 2) & 7 together; a ds_read_b32 is taken as one pass. Within a pass, lanes that read
// different rows of 32 * B < 256 bytes collide when they read the same column of rows equal
// modulo S = 8 / B. RowModel lists, for a tile of B blocks read in CW-byte columns, the sets of
// positions (relative to the first position of a wave, which takes P consecutive positions of
// a step) whose rows must differ modulo S for the access to be free of conflicts.
struct RowModel {
    uint32_t S = 1, P = 1;
    std::vector<std::vector<uint8_t>> sets;
};

inline RowModel row_model(uint32_t B, uint32_t CW) {
    RowModel m;
    if (B == 0 || B >= 8) return m;
    m.S = 8 / B;
    const uint32_t ncol = 32 * B / CW;
    m.P = 64 / ncol;
    std::map<std::pair<uint32_t, uint32_t>, std::vector<uint8_t>> by;  // (pass, column)
    for (uint32_t l = 0; l < 64; ++l) {
        const uint32_t pos = l / ncol, col = l % ncol;
        uint32_t pass = 0;
        if (CW == 16) pass = (l >> 5) * 2 + (__builtin_popcount((l >> 2) & 7) & 1);
        else if (CW == 8) pass = l >> 5;
        auto &v = by[{pass, col}];
        if (std::find(v.begin(), v.end(), (uint8_t)pos) == v.end()) v.push_back((uint8_t)pos);
    }
    for (auto &kv : by)
        if (kv.second.size() > 1 &&
            std::find(m.sets.begin(), m.sets.end(), kv.second) == m.sets.end())
            m.sets.push_back(kv.second);
    return m;
}

// Slot orders of a spin's partners: a task reads its own row, then the two other spins of each
// of its three triplets. Any order of the triplets, and of the two spins inside each, gives the
// same update (the rule sums the three triplets and each triplet's parity is symmetric), so a
// spin may take any of 3! * 2^3 = 48 slot orders; order s = o + 6 * w puts triplet
// kTripOrder[o][q] in slot pair q, its two spins swapped where bit q of w is set.
constexpr int kSlotOrders = 48;
constexpr uint8_t kTripOrder[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Role k (0 = own row, 1..6 = partner slots) of a spin under slot order s: the index (0..6) of
// the role it takes from the spin's roles in their given order.
inline int slot_source(int s, int k) {
    if (k == 0) return 0;
    const int q = (k - 1) >> 1, z = (k - 1) & 1;
    return 1 + 2 * kTripOrder[s % 6][q] + (z ^ ((s / 6 >> q) & 1));
}

struct Placement {
    std::vector<uint16_t> row;    // LDS row of each spin (a permutation of [0, n))
    std::vector<int32_t> order;   // the spins of each step, re-ordered inside the step
    std::vector<uint8_t> slots;   // slot order of each spin (slot_source)
};

// Placement for the steps off of `order` (roles: per spin, its own index and then the two other
// spins of each of its triplets). A cell is one read (role k) of one position set of one wave's
// share of a step (RowModel): its distinct rows collide when they fall on the same residue
// modulo S, and it costs its fullest residue's count minus one, twice for the own row (which
// the task also writes). Starting from the given order and slots, and residues that put each
// group's own rows on distinct residues as far as the residue counts allow, a seeded annealing search proposes moves around a costly cell: trade the residues of
// one of its colliding rows and a row of a residue the cell lacks, swap that row's position with
// another of its step, or give its spin another slot order. A move that does not raise the
// summed cost is kept, one that does with probability exp(-rise / T), T falling linearly to 0
// over the search. The rows of each residue are then numbered in spin order, so the map is a
// permutation of [0, n) (the residue counts never change), and the result is a fixed function
// of the inputs.
inline Placement place_rows(const std::vector<int32_t> &order, const std::vector<int32_t> &off,
                              const std::vector<int32_t> &roles, int n, const RowModel &m,
                              int effort = 400) {
    const uint32_t S = m.S;
    Placement pl;
    pl.order = order;
    pl.slots.assign(n, 0);
    // groups of positions (one per position set of each wave's share of each step)
    std::vector<int32_t> goff(1, 0), gpos, pstep(n, 0);
    for (size_t st = 0; st + 1 < off.size(); ++st) {
        for (int p = off[st]; p < off[st + 1]; ++p) pstep[p] = (int32_t)st;
        for (int g = off[st]; g < off[st + 1]; g += (int)m.P)
            for (const auto &set : m.sets) {
                const size_t first = gpos.size();
                for (uint8_t d : set)
                    if (g + d < off[st + 1]) gpos.push_back(g + d);
                if (gpos.size() - first < 2) {
                    gpos.resize(first);  // one row alone cannot collide
                    continue;
                }
                goff.push_back((int32_t)gpos.size());
            }
    }
    const int ng = (int)goff.size() - 1;
    pl.row.resize(n);
    if (ng == 0 || S < 2) {
        for (int r = 0; r < n; ++r) pl.row[r] = (uint16_t)r;
        return pl;
    }
    std::vector<int32_t> poff(n + 1, 0), pgrp;  // groups of each position
    for (int q = 0; q < ng; ++q)
        for (int j = goff[q]; j < goff[q + 1]; ++j) ++poff[gpos[j] + 1];
    for (int p = 0; p < n; ++p) poff[p + 1] += poff[p];
    pgrp.assign(poff[n], 0);
    {
        std::vector<int32_t> f(poff.begin(), poff.end() - 1);
        for (int q = 0; q < ng; ++q)
            for (int j = goff[q]; j < goff[q + 1]; ++j) pgrp[f[gpos[j]]++] = q;
    }
    std::vector<int32_t> posof(n);
    for (int p = 0; p < n; ++p) posof[pl.order[p]] = p;
    // Start: the own rows of each group on distinct residues where the residue counts allow
    // (they must stay those of r mod S, so that the final numbering is a permutation).
    std::vector<uint8_t> col(n, 0xFF);
    std::vector<int32_t> left(S, 0);
    for (int r = 0; r < n; ++r) ++left[r % S];
    for (int q = 0; q < ng; ++q) {
        uint32_t used = 0;
        for (int j = goff[q]; j < goff[q + 1]; ++j) {
            const int32_t r = pl.order[gpos[j]];
            if (col[r] != 0xFF) {
                used |= 1u << col[r];
                continue;
            }
            int best = -1;
            for (uint32_t z = 0; z < S; ++z)
                if (!(used >> z & 1) && left[z] > 0 && (best < 0 || left[z] > left[best])) best = (int)z;
            if (best < 0) continue;
            col[r] = (uint8_t)best;
            --left[best];
            used |= 1u << best;
        }
    }
    for (int r = 0, z = 0; r < n; ++r)
        if (col[r] == 0xFF) {
            while (left[z] == 0) ++z;
            col[r] = (uint8_t)z;
            --left[z];
        }
    std::vector<std::vector<int32_t>> of(S);
    std::vector<int32_t> at(n);
    for (int r = 0; r < n; ++r) {
        at[r] = (int32_t)of[col[r]].size();
        of[col[r]].push_back(r);
    }
    std::vector<int32_t> cur(roles.begin(), roles.begin() + 7 * (size_t)n);  // under pl.slots
    auto role = [&](int s, int k) { return cur[7 * (size_t)s + k]; };
    auto set_slots = [&](int s, uint8_t v) {
        pl.slots[s] = v;
        for (int k = 1; k < 7; ++k) cur[7 * (size_t)s + k] = roles[7 * (size_t)s + slot_source(v, k)];
    };
    // cost of cell (q, k), and its fullest residue
    auto cell = [&](int q, int k, int *hi) {
        int32_t rows[8];
        int nr = 0, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = goff[q]; j < goff[q + 1]; ++j) {
            const int32_t r = role(pl.order[gpos[j]], k);
            bool dup = false;
            for (int z = 0; z < nr; ++z) dup |= rows[z] == r;  // a row read twice is a broadcast
            if (dup || nr == 8) continue;
            rows[nr++] = r;
            ++cnt[col[r]];
        }
        int mx = 0, h = 0;
        for (uint32_t z = 0; z < S; ++z)
            if (cnt[z] > mx) mx = cnt[z], h = (int)z;
        if (hi) *hi = h;
        return mx > 1 ? (mx - 1) * (k ? 1 : 2) : 0;
    };
    std::vector<uint8_t> cost(7 * (size_t)ng);
    for (int q = 0; q < ng; ++q)
        for (int k = 0; k < 7; ++k) cost[7 * (size_t)q + k] = (uint8_t)cell(q, k, nullptr);
    uint64_t rng = 0x9E3779B97F4A7C15ull ^ (uint64_t)n;
    auto next = [&]() {  // xorshift64*
        rng ^= rng >> 12;
        rng ^= rng << 25;
        rng ^= rng >> 27;
        return (uint32_t)((rng * 0x2545F4914F6CDD1Dull) >> 32);
    };
    std::vector<int32_t> cells;  // affected cells of a move, as 7 * q + k
    std::vector<uint8_t> fresh;
    // cells that read row r: its own (role 0) and, for each spin u among its partners, the
    // roles of u that read r
    auto cells_of_row = [&](int32_t r) {
        for (int j = poff[posof[r]]; j < poff[posof[r] + 1]; ++j) cells.push_back(7 * pgrp[j]);
        for (int k = 1; k < 7; ++k) {
            const int32_t u = roles[7 * (size_t)r + k];
            for (int z = 1; z < 7; ++z)
                if (role(u, z) == r)
                    for (int j = poff[posof[u]]; j < poff[posof[u] + 1]; ++j)
                        cells.push_back(7 * pgrp[j] + z);
        }
    };
    auto cells_of_pos = [&](int p, int k0) {
        for (int j = poff[p]; j < poff[p + 1]; ++j)
            for (int k = k0; k < 7; ++k) cells.push_back(7 * pgrp[j] + k);
    };
    const double T0 = 0.3;
    const long evals = (long)effort * n, picks = 8 * evals;
    long e = 0;
    for (long pick = 0; pick < picks && e < evals; ++pick) {
        const int c = (int)(next() % (7 * (uint32_t)ng));
        if (!cost[c]) continue;
        const int q = c / 7, k = c % 7;
        int hi = 0;
        cell(q, k, &hi);
        // a member position whose row lies on the fullest residue
        int j0 = -1, seen = 0;
        for (int j = goff[q]; j < goff[q + 1]; ++j)
            if (col[role(pl.order[gpos[j]], k)] == hi && next() % ++seen == 0) j0 = gpos[j];
        if (j0 < 0) continue;
        const int s = pl.order[j0];
        const int32_t r = role(s, k);
        int kind = (int)(next() % 3);
        if (kind == 2 && k == 0) kind = (int)(next() % 2);
        ++e;
        cells.clear();
        int32_t b = -1, p2 = -1;
        uint8_t old_slot = 0;
        if (kind == 0) {  // trade residues with a row of a residue the cell lacks (or any other)
            uint32_t has = 0;
            for (int j = goff[q]; j < goff[q + 1]; ++j) has |= 1u << col[role(pl.order[gpos[j]], k)];
            int lo = (int)(next() % S);
            for (uint32_t t = 0; t < S; ++t)
                if (!(has >> ((lo + t) % S) & 1)) {
                    lo = (int)((lo + t) % S);
                    break;
                }
            if (lo == (int)col[r]) continue;
            b = of[lo][next() % of[lo].size()];
            cells_of_row(r);
            cells_of_row(b);
        } else if (kind == 1) {  // swap positions with another spin of the step
            const int st = pstep[j0];
            p2 = off[st] + (int)(next() % (uint32_t)(off[st + 1] - off[st]));
            if (p2 == j0) continue;
            cells_of_pos(j0, 0);
            cells_of_pos(p2, 0);
        } else {  // another slot order for the spin
            old_slot = pl.slots[s];
            cells_of_pos(j0, 1);
        }
        std::sort(cells.begin(), cells.end());
        cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
        int before = 0;
        for (int32_t x : cells) before += cost[x];
        auto apply = [&]() {
            if (kind == 0) {
                std::swap(col[r], col[b]);
            } else if (kind == 1) {
                const int32_t a = pl.order[j0], o = pl.order[p2];
                pl.order[j0] = o;
                pl.order[p2] = a;
                posof[a] = p2;
                posof[o] = j0;
            }
        };
        apply();
        if (kind == 2) set_slots(s, (uint8_t)(next() % kSlotOrders));
        fresh.resize(cells.size());
        int after = 0;
        for (size_t i = 0; i < cells.size(); ++i) {
            fresh[i] = (uint8_t)cell(cells[i] / 7, cells[i] % 7, nullptr);
            after += fresh[i];
        }
        const int rise = after - before;
        bool keep = rise <= 0;
        if (!keep) {
            const double T = T0 * (1.0 - (double)e / (double)evals);
            keep = T > 1e-3 && (double)(next() & 0xFFFFFF) < std::exp(-rise / T) * 16777216.0;
        }
        if (keep) {
            for (size_t i = 0; i < cells.size(); ++i) cost[cells[i]] = fresh[i];
            if (kind == 0) {
                std::swap(of[col[r]][at[b]], of[col[b]][at[r]]);
                std::swap(at[r], at[b]);
            }
        } else if (kind == 2) {
            set_slots(s, old_slot);
        } else {
            apply();  // both moves are their own inverse
        }
    }
    std::vector<int> rank(S, 0);
    for (int r = 0; r < n; ++r) pl.row[r] = (uint16_t)(col[r] + S * rank[col[r]]++);
    return pl;
}

// Total cost of a placement under the cell model of place_rows (for checks and tuning).
inline long placement_cost(const Placement &pl, const std::vector<int32_t> &off,
                           const std::vector<int32_t> &roles, const RowModel &m) {
    const uint32_t S = m.S;
    if (S < 2) return 0;
    long total = 0;
    for (size_t st = 0; st + 1 < off.size(); ++st)
        for (int g = off[st]; g < off[st + 1]; g += (int)m.P)
            for (const auto &set : m.sets)
                for (int k = 0; k < 7; ++k) {
                    std::vector<int32_t> rows;
                    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    for (uint8_t d : set) {
                        if (g + d >= off[st + 1]) continue;
                        const int s = pl.order[g + d];
                        const int32_t r = roles[7 * (size_t)s + slot_source(pl.slots[s], k)];
                        if (std::find(rows.begin(), rows.end(), r) != rows.end()) continue;
                        rows.push_back(r);
                        ++cnt[pl.row[r] % S];
                    }
                    int mx = 0;
                    for (uint32_t z = 0; z < S; ++z) mx = std::max(mx, cnt[z]);
                    if (rows.size() > 1 && mx > 1) total += (mx - 1) * (k ? 1 : 2);
                }
    return total;
}

}  // namespace xsh
