/*
 * Scalar CPU oracle of the quasi-greedy many-clone dynamics (TEST INFRASTRUCTURE ONLY).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this file's
 * library. It shares no code with the GPU path: it keeps one int8 spin (+1/-1) per site and
 * clone, walks the spins one at a time, and recomputes the energy from its definition after
 * every sweep. It is meant to be slow and easy to check by eye against the paper.
 *
 * Paper: Bernaschi et al., "How we are leading a 3-XORSAT challenge: from the energy landscape
 * to the algorithm and its efficient implementation on GPUs" (arXiv 2102.09510).
 *
 * What each function follows:
 *   or_energy        Eq. (1): H = -sum over triplets of J_t s_a s_b s_c (the paper has J = +1;
 *                    planted instances carry J_t = tau_a tau_b tau_c).
 *   or_colour        Supplementary Material, "Details on the GPU implementation": greedy
 *                    partition into independent sets of at most `cap` nodes, found by scanning
 *                    the graph repeatedly.
 *   or_philox        Philox4x32 with 10 rounds, from its published definition (Salmon, Moraes,
 *                    Dror, Shaw, SC'11, "Parallel random numbers: as easy as 1, 2, 3").
 *   or_run           Section "The quasi-greedy algorithm": a spin in k unsatisfied triplets
 *                    flips with probability w_k, w0 = thr0 / 2^16 (0 for the quasi-greedy rule;
 *                    w0 = w1^3 is the Metropolis rule the same section mentions),
 *                    w1 = thr / 2^16, w2 = w3 = 1;
 *                    Section "Basic information about the GPU implementation": one random
 *                    number shared by the 32 clones of a word; Supplementary Material: sets
 *                    processed one after the other, the exact sweep at which a clone reaches the
 *                    ground state is recorded.
 *
 * Readings where the paper leaves a choice open (shared with the GPU path by specification,
 * not by code):
 *   - random numbers: Philox4x32-10, key = (seed low 32 bits, seed high 32 bits);
 *       initial spin of site i, clone c (group g = c >> 5, bit b = c & 31):
 *         bit b of  philox(ctr = (i, 0xFFFFFFFF, g >> 2, instance_id))[g & 3],  bit 1 <=> s = -1;
 *       sweep t, site i, group g: the 16-bit draw
 *         d = (philox(ctr = (i, t, g >> 3, instance_id))[(g & 7) >> 1] >> (16 * (g & 1))) & 0xFFFF
 *       and the spin flips iff d < thr (k = 1) or d < thr0 (k = 0);
 *   - a sweep visits the sites in `perm` order (the colour classes one after another);
 *   - first_hit[c] = smallest t in [start_sweep, start_sweep + n_sweeps] with E(C_t) = -N,
 *     where C_t is the configuration before sweep t, or -1. With thr0 > 0 a ground state can be
 *     left again, and only the final configuration is tested: first_hit = the end sweep if it
 *     has E = -N, else -1.
 *
 * Parity unpinned (or_run, or_trace): the exact trajectories for 0 < w1 < 1 follow from the
 * random-number reading above, which the paper does not fix; the tests pin the rule itself
 * (per update, the deterministic w1 = 0 and w1 = 1 sweeps worked by hand, acceptance
 * frequencies, the energy change per flip, the absorbing ground state, the paramagnetic energy
 * of the w0 = w1^3 rule) and, at N <= 12, the law of first_hit (and of the end state with
 * w0 > 0) against the exact Markov chain over all configurations, not single trajectories.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox4x32-10 */

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    /* Philox-4x32: two 32x32->64 multiplications per round; the high halves are mixed with the
     * other two counter words and the round key, the low halves pass through. The key is bumped
     * by the Weyl constants after each round. Ten rounds. */
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_seeded(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                          uint32_t out[4]) {
    uint32_t ctr[4] = {a, b, c, d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* Initial spin of site i for clone c. */
int8_t or_initial_spin(uint64_t seed, uint32_t instance_id, int32_t i, int64_t c) {
    int64_t g = c >> 5;
    uint32_t out[4];
    philox_seeded(seed, (uint32_t)i, 0xFFFFFFFFu, (uint32_t)(g >> 2), instance_id, out);
    uint32_t bit = (out[g & 3] >> (c & 31)) & 1u;
    return bit ? -1 : 1;
}

/* The 16-bit draw compared with the threshold for site i, clone c, sweep t. */
uint32_t or_draw16(uint64_t seed, uint32_t instance_id, int32_t i, uint32_t t, int64_t c) {
    int64_t g = c >> 5;
    uint32_t out[4];
    philox_seeded(seed, (uint32_t)i, t, (uint32_t)(g >> 3), instance_id, out);
    uint32_t word = out[(g & 7) >> 1];
    return (word >> (16 * (g & 1))) & 0xFFFFu;
}

/* ---------------------------------------------------------------- energy, Eq. (1) */

int32_t or_energy(int32_t n, const int32_t *tri, const int8_t *J, const int8_t *s) {
    int32_t e = 0;
    for (int32_t t = 0; t < n; ++t) /* M = N triplets */
        e -= J[t] * s[tri[3 * t]] * s[tri[3 * t + 1]] * s[tri[3 * t + 2]];
    return e;
}

/* Triplets containing each site (exactly three per site for valid instances). */
static int build_incidence(int32_t n, const int32_t *tri, int32_t *inc /* n*3 */) {
    int32_t *deg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int bad = 0;
    for (int32_t t = 0; t < n && !bad; ++t)
        for (int q = 0; q < 3; ++q) {
            int32_t v = tri[3 * t + q];
            if (v < 0 || v >= n || deg[v] >= 3) { bad = 1; break; }
            inc[3 * v + deg[v]++] = t;
        }
    for (int32_t v = 0; v < n && !bad; ++v)
        if (deg[v] != 3) bad = 1;
    free(deg);
    return bad ? -1 : 0;
}

/* ---------------------------------------------------------------- colouring */

/* Do sites u and v appear together in some triplet? (inc: the three triplets of each site) */
static int shares_triplet(const int32_t *tri, const int32_t *inc, int32_t u, int32_t v) {
    for (int q = 0; q < 3; ++q) {
        int32_t t = inc[3 * u + q];
        if (tri[3 * t] == v || tri[3 * t + 1] == v || tri[3 * t + 2] == v) return 1;
    }
    return 0;
}

/* Greedy partition into independent sets (no two members share a triplet) of at most `cap`
 * sites. Each pass scans the unassigned sites in ascending order and adds a site to the set
 * being built when the set has room and the site shares no triplet with any member. perm
 * receives the sites set by set; class_off[k] .. class_off[k+1]-1 are the positions of set k
 * (class_off needs room for n+1 entries). Returns the number of sets, or -1 on bad input. */
int32_t or_colour(int32_t n, const int32_t *tri, int32_t cap, int32_t *perm, int32_t *class_off) {
    if (n <= 0 || cap <= 0) return -1;
    int32_t *inc = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    if (build_incidence(n, tri, inc) != 0) { free(inc); return -1; }
    char *assigned = (char *)calloc((size_t)n, 1);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t placed = 0, n_classes = 0;
    class_off[0] = 0;
    while (placed < n) {
        int32_t size = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (assigned[v] || size >= cap) continue;
            int ok = 1;
            for (int32_t q = 0; q < size && ok; ++q)
                if (shares_triplet(tri, inc, cur[q], v)) ok = 0;
            if (ok) cur[size++] = v;
        }
        for (int32_t q = 0; q < size; ++q) {
            assigned[cur[q]] = 1;
            perm[placed++] = cur[q];
        }
        class_off[++n_classes] = placed;
    }
    free(assigned);
    free(cur);
    free(inc);
    return n_classes;
}

/* ---------------------------------------------------------------- the dynamics */

/* Number of triplets of site i that are unsatisfied (J_t s_a s_b s_c = -1). */
static int unsatisfied_count(const int32_t *tri, const int8_t *J, const int32_t *inc,
                             const int8_t *s, int32_t i) {
    int k = 0;
    for (int q = 0; q < 3; ++q) {
        int32_t t = inc[3 * i + q];
        if (J[t] * s[tri[3 * t]] * s[tri[3 * t + 1]] * s[tri[3 * t + 2]] == -1) ++k;
    }
    return k;
}

/* One sweep of one clone over the sites in perm order (sweep index t). Optional trace arrays
 * (n entries each, in visiting order) receive k and whether the site flipped. */
static void sweep_one(int32_t n, const int32_t *tri, const int8_t *J, const int32_t *inc,
                      const int32_t *perm, uint64_t seed, uint32_t instance_id, uint32_t thr,
                      uint32_t thr0, uint32_t t, int64_t clone, int8_t *s, int8_t *trace_k,
                      int8_t *trace_flip) {
    for (int32_t pos = 0; pos < n; ++pos) {
        int32_t i = perm[pos];
        int k = unsatisfied_count(tri, J, inc, s, i);
        int flip;
        if (k >= 2)
            flip = 1; /* w2 = w3 = 1 */
        else if (k == 1)
            flip = or_draw16(seed, instance_id, i, t, clone) < thr; /* w1 = thr / 2^16 */
        else
            flip = thr0 > 0 && or_draw16(seed, instance_id, i, t, clone) < thr0; /* w0 */
        if (flip) s[i] = (int8_t)-s[i];
        if (trace_k) trace_k[pos] = (int8_t)k;
        if (trace_flip) trace_flip[pos] = (int8_t)flip;
    }
}

/*
 * Run clones [clone_begin, clone_begin + clone_count) for n_sweeps sweeps, sweep indices
 * start_sweep .. start_sweep + n_sweeps - 1.
 *   init_spins  optional [clone_count][n] (+1/-1); NULL draws the initial spins from the stream.
 *   first_hit   [clone_count]: smallest t in [start_sweep, start_sweep + n_sweeps] such that the
 *               configuration before sweep t (after the last sweep for the upper end) has
 *               E = -N; -1 if none.
 *   energy      optional [clone_count]: E after the last sweep.
 *   final_spins optional [clone_count][n].
 * Returns 0, or -1 on invalid input.
 */
int32_t or_run(int32_t n, const int32_t *tri, const int8_t *J, const int32_t *perm,
               uint64_t seed, uint32_t instance_id, uint32_t thr, uint32_t thr0,
               int64_t clone_begin,
               int64_t clone_count, uint32_t start_sweep, uint32_t n_sweeps,
               const int8_t *init_spins, int32_t *first_hit, int32_t *energy,
               int8_t *final_spins, int32_t n_threads) {
    if (n <= 0 || clone_count < 0) return -1;
    int32_t *inc = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    if (build_incidence(n, tri, inc) != 0) { free(inc); return -1; }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        int8_t *s = (int8_t *)malloc((size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < clone_count; ++q) {
            int64_t c = clone_begin + q;
            if (init_spins)
                memcpy(s, init_spins + q * n, (size_t)n);
            else
                for (int32_t i = 0; i < n; ++i) s[i] = or_initial_spin(seed, instance_id, i, c);
            int32_t hit = thr0 == 0 && or_energy(n, tri, J, s) == -n ? (int32_t)start_sweep : -1;
            for (uint32_t k = 0; k < n_sweeps; ++k) {
                uint32_t t = start_sweep + k;
                sweep_one(n, tri, J, inc, perm, seed, instance_id, thr, thr0, t, c, s, NULL, NULL);
                if (thr0 == 0 && hit < 0 && or_energy(n, tri, J, s) == -n) hit = (int32_t)(t + 1);
            }
            if (thr0 > 0 && or_energy(n, tri, J, s) == -n) hit = (int32_t)(start_sweep + n_sweeps);
            first_hit[q] = hit;
            if (energy) energy[q] = or_energy(n, tri, J, s);
            if (final_spins) memcpy(final_spins + q * n, s, (size_t)n);
        }
        free(s);
    }
    free(inc);
    return 0;
}

/*
 * Single-clone trajectory with a full trace, for invariant tests: for every sweep the k seen and
 * the flip taken at each visited position (trace_k / trace_flip: [n_sweeps][n]) and the energy
 * before every sweep plus after the last one (energies: [n_sweeps + 1]).
 */
int32_t or_trace(int32_t n, const int32_t *tri, const int8_t *J, const int32_t *perm,
                 uint64_t seed, uint32_t instance_id, uint32_t thr, uint32_t thr0, int64_t clone,
                 uint32_t start_sweep, uint32_t n_sweeps, int8_t *spins /* in/out [n] */,
                 int8_t *trace_k, int8_t *trace_flip, int32_t *energies) {
    int32_t *inc = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    if (build_incidence(n, tri, inc) != 0) { free(inc); return -1; }
    energies[0] = or_energy(n, tri, J, spins);
    for (uint32_t k = 0; k < n_sweeps; ++k) {
        sweep_one(n, tri, J, inc, perm, seed, instance_id, thr, thr0, start_sweep + k, clone, spins,
                  trace_k + (size_t)k * n, trace_flip + (size_t)k * n);
        energies[k + 1] = or_energy(n, tri, J, spins);
    }
    free(inc);
    return 0;
}
