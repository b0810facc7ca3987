// HIP kernels (gfx950) of the quasi-greedy many-clone dynamics.
//
// Paper: Bernaschi et al., arXiv 2102.09510. Section "The quasi-greedy algorithm" gives the
// rule (w0 = 0, w1, w2 = w3 = 1); Section "Basic information about the GPU implementation" the
// multispin coding (one random number per 32-clone word); the Supplementary Material the
// independent-set schedule, the LDS-resident state and the many sweeps per launch. The host
// hands the kernels the update order as steps: independent sets whose in-order execution is
// the sequential sweep (spins sharing a triplet keep their order).
//
// Data layout
//   global state   uint64 [n][W] spin-major, W = n_clones / 64 (bit = clone).
//   tile           B consecutive 256-clone blocks of one instance (4*B words per spin row),
//                  owned by one workgroup for a whole chunk of sweeps.
//   LDS            rec  [n]      16-byte records in step order, u16 fields: byte offsets of
//                               the spin's own row and of the two other spins of each of its
//                               three triplets, then meta = i | jbits << 13;
//                  state [n][32*B] the tile's rows, spin i in row rowmap[i] when the host
//                               placed the rows (tiles under eight blocks), else in row i;
//                  rbits [n][B]  k = 1 acceptance bits of the current sweep, one byte per
//                               (position, block): bit k belongs to group k of the block;
//                  acc   [8*B]   per-group OR of "some triplet of the visited spin is
//                               unsatisfied" over the current sweep.
//   task           one spin of the current step x one CW-byte column of its row (CW = 16, 8
//                  or 4: 128, 64 or 32 clones). Consecutive threads take consecutive columns
//                  of the same row, so a wave reads contiguous LDS runs.
//
// Per update, with p_t = x_a ^ x_b ^ j_t the value that satisfies triplet t of spin x:
//   k = #{t : x != p_t};  m = majority(p1, p2, p3) is the new spin when k != 1 (k = 0 keeps
//   x = m, k >= 2 flips to m = ~x); k == 1 <=> (x ^ p1 ^ p2 ^ p3) & ~(x ^ m); then the spin
//   flips iff the group's acceptance bit is set. All of it is bitwise over 32 clones.
//
// Ground-state detection (exact first hit): during the sweep that starts from C_t the OR of
// (k >= 1) over all visited spins is zero iff C_t has E = -N. If C_t has an unsatisfied triplet,
// the first visited spin of any unsatisfied triplet still sees it (every spin before it had
// k = 0 and kept its value), so the OR is one; if C_t is a ground state nothing moves.
#include <algorithm>
#include <atomic>
#include <mutex>

#include "xs_internal.h"

#include "../../include/xorsat.h"

namespace xs {
namespace {

// Three-input logic in one gfx950 instruction: result bit = lut[(a << 2) | (b << 1) | c], so a
// LUT is the function evaluated on the bit patterns a = 0xF0, b = 0xCC, c = 0xAA.
constexpr uint32_t kA = 0xF0, kB = 0xCC, kC = 0xAA;
constexpr uint32_t kXor3 = (kA ^ kB ^ kC) & 0xFF;
constexpr uint32_t kMaj3 = ((kA & kB) | (kA & kC) | (kB & kC)) & 0xFF;
constexpr uint32_t kXorAndN = (kA ^ (kB & ~kC)) & 0xFF;    // a ^ (b & ~c)
constexpr uint32_t kMux = ((kA & kB) | (~kA & kC)) & 0xFF; // a ? b : c, bitwise
constexpr uint32_t kXorAnd2 = ((kA ^ kB) & kC) & 0xFF;     // (a ^ b) & c
constexpr uint32_t kFlipIfEq = (kA ^ (kC & ~(kA ^ kB))) & 0xFF;  // a ^ (c & (a == b))
constexpr uint32_t kAnyDiff = ((kA ^ kB) | (kA ^ kC)) & 0xFF;    // (a ^ b) | (a ^ c)

template <uint32_t LUT>
__device__ __forceinline__ uint32_t lop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, LUT);
}

// Philox4x32-10 bijection (Salmon, Moraes, Dror, Shaw, SC'11): per round two 32x32->64
// products; high halves mixed with the other counter words and the round key, low halves
// passed on; key bumped by the Weyl increments between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(lop3<kXor3>((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                       lop3<kXor3>((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// The same bijection for the sweep draws, whose counter is (i, t, z, id) with t and id uniform
// over the workgroup and z fixed per thread: the caller passes z's first-round product pz and
// the uniform terms t ^ k0 and id ^ k1 of the first round, so only i varies per call.
__device__ __forceinline__ uint4 philox10_draw(uint32_t i, uint64_t pz, uint32_t t_k0,
                                               uint32_t id_k1, uint32_t k0, uint32_t k1) {
    const uint64_t pi = (uint64_t)0xD2511F53u * i;
    uint4 c = make_uint4((uint32_t)(pz >> 32) ^ t_k0, (uint32_t)pz,
                         (uint32_t)(pi >> 32) ^ id_k1, (uint32_t)pi);
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(lop3<kXor3>((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                       lop3<kXor3>((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
    }
    return c;
}


// One 32-clone word of one spin: seven three-input operations, two more when ground states are
// tracked (kAcc: acc collects "k >= 1"). With d_t = x ^ p_t: k is odd iff x ^ par = 1 (par =
// p1 ^ p2 ^ p3 = x ^ d1 ^ d2 ^ d3) and k <= 1 iff x = m (x ^ m = maj(d1, d2, d3)). So
// t = (x ^ par) & accept flips the spin exactly where k = 1 and the group accepts, provided
// x = m; where x != m (k >= 2) the new spin is m = ~x whatever t is.
template <bool kAcc>
__device__ __forceinline__ uint32_t qg_word(uint32_t x, uint32_t a1, uint32_t b1, uint32_t a2,
                                            uint32_t b2, uint32_t a3, uint32_t b3, uint32_t j1,
                                            uint32_t j2, uint32_t j3, uint32_t accept,
                                            uint32_t &acc) {
    const uint32_t p1 = lop3<kXor3>(a1, b1, j1);
    const uint32_t p2 = lop3<kXor3>(a2, b2, j2);
    const uint32_t p3 = lop3<kXor3>(a3, b3, j3);
    const uint32_t m = lop3<kMaj3>(p1, p2, p3);     // new spin unless k == 1
    const uint32_t par = lop3<kXor3>(p1, p2, p3);
    if (kAcc) acc |= lop3<kAnyDiff>(x, m, par);      // k >= 1
    const uint32_t t = lop3<kXorAnd2>(x, par, accept);
    return lop3<kFlipIfEq>(m, x, t);
}

// The same word with w0 > 0 (Section "The quasi-greedy algorithm": w0 = w1^3 gives the
// detailed-balance Metropolis rule at the pseudo-temperature of w1): a k = 0 spin flips when the
// group's w0 bit is set. When k <= 1 (dmaj = 0), k = 1 iff x differs from p1 ^ p2 ^ p3, which
// selects acc1 over acc0; nine three-input operations.
__device__ __forceinline__ uint32_t met_word(uint32_t x, uint32_t a1, uint32_t b1, uint32_t a2,
                                             uint32_t b2, uint32_t a3, uint32_t b3, uint32_t j1,
                                             uint32_t j2, uint32_t j3, uint32_t acc1,
                                             uint32_t acc0) {
    const uint32_t p1 = lop3<kXor3>(a1, b1, j1);
    const uint32_t p2 = lop3<kXor3>(a2, b2, j2);
    const uint32_t p3 = lop3<kXor3>(a3, b3, j3);
    const uint32_t m = lop3<kMaj3>(p1, p2, p3);
    const uint32_t par = lop3<kXor3>(p1, p2, p3);
    const uint32_t e = x ^ par;      // k odd
    const uint32_t dmaj = x ^ m;     // k >= 2
    return lop3<kXorAndN>(m, lop3<kMux>(e, acc1, acc0), dmaj);
}


constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

__host__ __device__ constexpr size_t lds_rec_bytes(uint32_t n) { return size_t(16) * n; }
// Acceptance-bit buffers of a tile: sweeps alternate between two, and tiles with records in
// global memory and w0 = 0 keep a third for the cross-sweep body, whose iterations draw into
// a buffer two iterations after its last reads.
__host__ __device__ constexpr uint32_t accept_buffers(bool rec_global, bool met) {
    return rec_global && !met ? 3u : 2u;
}

// ------------------------------------------------------------------------------ init

// Start configuration: the 32 clones of group g of spin i take the bits of
// philox(i, 0xFFFFFFFF, g >> 2, id)[g & 3]. One thread per (spin, pair of words).
__global__ __launch_bounds__(256) void qg_init(InstDev *I) {
    const uint32_t n = I->n, W = I->n_words;
    const uint32_t pairs = W >> 1;
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = (uint64_t)n * (pairs + 1);  // + first_hit clearing share
    if (q >= total) return;
    const bool init_state = !(I->flags & XS_RESUME);
    if (q < (uint64_t)n * pairs) {
        if (init_state) {
            const uint32_t i = (uint32_t)(q / pairs), w2 = (uint32_t)(q % pairs);
            const uint4 o = philox10(make_uint4(i, kInitSweep, w2, I->inst_id), I->seed_lo,
                                     I->seed_hi);
            uint64_t *row = I->state + (size_t)i * W + 2 * w2;
            row[0] = (uint64_t)o.x | ((uint64_t)o.y << 32);
            row[1] = (uint64_t)o.z | ((uint64_t)o.w << 32);
        }
    }
    // first_hit = -1 for every clone (grid-stride over the clones).
    const uint64_t n_clones = (uint64_t)W * 64;
    for (uint64_t c = q; c < n_clones; c += total) I->first_hit[c] = -1;
}

// ------------------------------------------------------------------------------ chunk

// The workgroup's dynamic LDS. Every LDS access below indexes this array, so the compiler
// keeps them all as ds_* instructions.
extern __shared__ __align__(16) uint8_t xs_lds[];

// Global address space: loads through it are global_load (vector memory counter only), not
// flat loads, which also count against the LDS counter and so make every LDS wait -- the one
// before a step's barrier among them -- wait for them too.
#define GLOBAL_AS __attribute__((address_space(1)))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// 16-byte global load / store of element idx of a device array (global_load/store_dwordx4).
__device__ __forceinline__ uint4 gload16(const void *base, size_t idx) {
    const u32x4 v = ((const GLOBAL_AS u32x4 *)base)[idx];
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore16(void *base, size_t idx, uint4 v) {
    ((GLOBAL_AS u32x4 *)base)[idx] = u32x4{v.x, v.y, v.z, v.w};
}
// LDS address space: an integer LDS address used as a pointer, so that a uniform base folds
// into scalar arithmetic.
#define LDS_AS __attribute__((address_space(3)))
__device__ __forceinline__ uint32_t lds_base() {
    return (uint32_t)(uintptr_t)(LDS_AS uint8_t *)xs_lds;
}

// Per-workgroup view of one tile. LDS locations are byte offsets into xs_lds. A task is one
// spin of the current step and one column of CW bytes of the tile's rows (CW / 4 groups of 32
// clones); `col` is this thread's column, fixed because the workgroup size is a multiple of the
// column count.
struct Tile {
    InstDev *I;
    const uint4 *grec;   // records in global memory (GR kernels), offsets for this tile's rows
    uint32_t n, W, B, lB, rowb, ncol, lcol, n16, l16, ngrp, blk0, tid, col;
    uint32_t st;         // state rows (records start at 0)
    uint32_t rb0, rb1;   // acceptance bytes, double-buffered by sweep parity
    uint32_t acc;        // per-group accumulators [8*B] (uint32)
    uint32_t flag;       // workgroup flag (uint32)
    uint32_t stp;        // step bounds (u16, n_steps + 1 of them and the last again), staged
                         // from the step table
    uint32_t meta;       // spin index of each position (u16): the low 13 bits of the record's
                         // meta half-word in LDS, or an array of the indices alone (GR)
    uint32_t colbase;    // st + this thread's column
    uint32_t rb_sel, rb_shift;
    uint32_t thr, thr0, key0, key1, iid, nsteps;
    uint32_t tpos;       // this thread's first task position in a step (tid >> lcol)
    uint32_t rbo;        // its acceptance entry index relative to the step start
    const int32_t *step_off;
    uint32_t lds0;       // absolute LDS address of xs_lds
};

__device__ __forceinline__ uint4 &lds_rec(uint32_t p) {
    return reinterpret_cast<uint4 *>(xs_lds)[p];
}
__device__ __forceinline__ uint32_t &lds_u32(uint32_t off) {
    return *reinterpret_cast<uint32_t *>(xs_lds + off);
}
// The record of position p: in LDS, or in global memory (read through the caches) when the
// tile keeps its LDS for clone state (GR).
template <bool GR>
__device__ __forceinline__ uint4 rec_at(const Tile &T, uint32_t p) {
    if (GR) return gload16(T.grec, p);
    return lds_rec(p);
}

// Column access: CW = 16, 8 or 4 bytes as one ds_read_b128 / b64 / b32.
template <int CW> struct ColVec;
template <> struct ColVec<16> { using T = uint4; };
template <> struct ColVec<8> { using T = uint2; };
template <> struct ColVec<4> { using T = uint32_t; };

template <int CW>
__device__ __forceinline__ void col_load(uint32_t addr, uint32_t (&w)[CW / 4]) {
    const typename ColVec<CW>::T v = *reinterpret_cast<const typename ColVec<CW>::T *>(xs_lds + addr);
    __builtin_memcpy(w, &v, CW);
}
template <int CW>
__device__ __forceinline__ void col_store(uint32_t addr, const uint32_t (&w)[CW / 4]) {
    typename ColVec<CW>::T v;
    __builtin_memcpy(&v, w, CW);
    *reinterpret_cast<typename ColVec<CW>::T *>(xs_lds + addr) = v;
}

// Bit g of the result: draw g of the eight 16-bit draws in o is below thr.
// 1 in each 16-bit half of w that is at most the same half of lim (saturating 16-bit
// subtractions: w - lim is 0 exactly then, and 1 - (w - lim) is 1 exactly then).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t halves_at_most(uint32_t w, uint32_t lim) {
    const u16x2 one = {1, 1};
    const u16x2 d = __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, w),
                                                  __builtin_bit_cast(u16x2, lim));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(one, d));
}

// Bit g (g = 0..7) set iff the g-th 16-bit draw of o (half g & 1 of word g >> 1) is below thr,
// 0 <= thr <= 65536: for thr >= 1, d < thr <=> d <= thr - 1. The low halves' bits land on even
// positions, the high halves' on 16 + even positions, folded down by 15.
__device__ __forceinline__ uint32_t draws_below(uint4 o, uint32_t thr) {
    const uint32_t lim = (thr - 1u) * 0x00010001u;
    const uint32_t x = halves_at_most(o.x, lim) | halves_at_most(o.y, lim) << 2 |
                       halves_at_most(o.z, lim) << 4 | halves_at_most(o.w, lim) << 6;
    return (x | x >> 15) & (thr ? 0xFFu : 0u);
}

// Acceptance bits of sweep t: one Philox call per (position, block) gives the eight 16-bit draws
// of the block's eight groups. MET: a 16-bit entry, the w1 byte and above it the w0 byte of the
// same draws. A thread keeps one block (NT is a multiple of B) and strides over positions.
// BODY (the cross-sweep body): a spin marked late (bit 12 of its staged meta) is updated in the
// iteration after its sweep's, so its bits go to buffer rb_late, the one that iteration reads.
template <int NT, bool GR, bool MET, bool BODY = false>
__device__ __forceinline__ void accept_bits(const Tile &T, uint32_t t, uint32_t rb,
                                            uint32_t rb_late = 0) {
    const uint32_t b = T.tid & (T.B - 1);
    const uint64_t pz = (uint64_t)0xCD9E8D57u * (T.blk0 + b);
    const uint32_t t_k0 = t ^ T.key0, id_k1 = T.iid ^ T.key1;
    const uint32_t base = T.lds0 + rb, dlate = rb_late - rb;  // absolute LDS addresses
    constexpr uint32_t MS = GR ? 2 : 16, E = MET ? 2 : 1;  // bytes per meta, per entry
    // position p: its meta at mp, its entry at ea (base + E * q, q = (p << lB) + b)
    auto one = [&](uint32_t mp, uint32_t ea) {
        const uint32_t v = *(const LDS_AS uint16_t *)(uintptr_t)mp;
        const uint32_t i = GR ? v & 0x7FFu : v & 0x1FFFu;  // spins < 2048 with records in global memory
        const uint4 o = philox10_draw(i, pz, t_k0, id_k1, T.key0, T.key1);
        // a late spin's bits go dlate = rb_late - rb further: bit 12 sign-extracted as a mask
        if constexpr (BODY) ea += (uint32_t)__builtin_amdgcn_sbfe((int)v, 12, 1) & dlate;
        if constexpr (MET)
            *(LDS_AS uint16_t *)(uintptr_t)ea =
                (uint16_t)(draws_below(o, T.thr) | draws_below(o, T.thr0) << 8);
        else
            *(LDS_AS uint8_t *)(uintptr_t)ea = (uint8_t)draws_below(o, T.thr);
    };
    const uint32_t ps = NT >> T.lB, p0 = T.tid >> T.lB;  // positions per pass, the first
    const uint32_t m0 = T.lds0 + T.meta + MS * p0, e0 = base + E * ((p0 << T.lB) + b);
    if ((T.n & (ps - 1)) == 0) {
        // every thread has n / ps positions: a uniform count and running addresses
        const uint32_t k1 = (uint32_t)__builtin_amdgcn_readfirstlane(T.n >> (__builtin_ctz(NT) - T.lB));
        for (uint32_t k = 0; k < k1; ++k) one(m0 + k * (MS * ps), e0 + k * (E * NT));
    } else {
        for (uint32_t p = p0, k = 0; p < T.n; p += ps, ++k) one(m0 + k * (MS * ps), e0 + k * (E * NT));
    }
}

// One task: the spin whose record is r, this thread's column; ra is the absolute LDS address of
// the acceptance entry of the spin's position and the column's block.
template <int CW, bool kAcc, bool MET, bool J0>
__device__ __forceinline__ void update_task(const Tile &T, uint4 r, uint32_t ra,
                                            uint32_t (&acc)[CW / 4]) {
    constexpr int G = CW / 4;
    const uint32_t self = T.colbase + (r.x & 0xFFFFu);
    uint32_t x[G], a1[G], b1[G], a2[G], b2[G], a3[G], b3[G], y[G];
    col_load<CW>(self, x);
    col_load<CW>(T.colbase + (r.x >> 16), a1);
    col_load<CW>(T.colbase + (r.y & 0xFFFFu), b1);
    col_load<CW>(T.colbase + (r.y >> 16), a2);
    col_load<CW>(T.colbase + (r.z & 0xFFFFu), b2);
    col_load<CW>(T.colbase + (r.z >> 16), a3);
    col_load<CW>(T.colbase + (r.w & 0xFFFFu), b3);
    // J0: every coupling is +1 in the tile's gauge, so the records carry no coupling bits
    const uint32_t meta = r.w >> 16;
    const uint32_t j1 = J0 ? 0u : 0u - ((meta >> 13) & 1u);
    const uint32_t j2 = J0 ? 0u : 0u - ((meta >> 14) & 1u);
    const uint32_t j3 = J0 ? 0u : 0u - (meta >> 15);
    // rb_shift is a multiple of G, so the column's G bits stay inside their byte
    if constexpr (MET) {
        const uint32_t v = *(const LDS_AS uint16_t *)(uintptr_t)ra;
        const uint32_t bits = v >> T.rb_shift, bits0 = v >> (8 + T.rb_shift);
#pragma unroll
        for (int g = 0; g < G; ++g)
            y[g] = met_word(x[g], a1[g], b1[g], a2[g], b2[g], a3[g], b3[g], j1, j2, j3,
                            0u - ((bits >> g) & 1u), 0u - ((bits0 >> g) & 1u));
    } else {
        const int bits = *(const LDS_AS uint8_t *)(uintptr_t)ra;
#pragma unroll
        for (int g = 0; g < G; ++g)  // sign-extended bit rb_shift + g: the group's mask
            y[g] = qg_word<kAcc>(x[g], a1[g], b1[g], a2[g], b2[g], a3[g], b3[g], j1, j2, j3,
                                 (uint32_t)__builtin_amdgcn_sbfe(bits, T.rb_shift + g, 1),
                                 acc[g]);
    }
    col_store<CW>(self, y);
}

// This thread's records as a raw buffer over the tile's n records (global memory): a scalar
// resource, and this thread's position offset (tpos records) in a vector register that never
// changes, so a step's fetch needs only a scalar offset and no vector instruction. Resource
// word 3 = 0x00020000 (32-bit data format, no swizzle, as raw loads on this architecture family
// take it); a fetch past the n records reads zeros, never faults.
struct RecBuf {
    __amdgpu_buffer_rsrc_t rs;
    int voff;
};
__device__ __forceinline__ RecBuf rec_buf(const Tile &T) {
    const uint64_t gp = (uint64_t)(uintptr_t)T.grec;
    // (readfirstlane returns a signed int: each half is taken as unsigned before widening, or a
    // low half with bit 31 set would fill the high half with ones)
    const uint32_t g_hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(gp >> 32));
    const uint32_t g_lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)gp);
    const uint32_t nb = (uint32_t)__builtin_amdgcn_readfirstlane(T.n) * (uint32_t)sizeof(u32x4);
    return RecBuf{__builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)((uint64_t)g_hi << 32 | g_lo),
                                                    (short)0, (int)nb, 0x00020000),
                  (int)(T.tpos * (uint32_t)sizeof(u32x4))};
}
// The record of position p0 + tpos (p0 uniform).
__device__ __forceinline__ u32x4 rec_fetch(const RecBuf &R, uint32_t p0) {
    return __builtin_amdgcn_raw_buffer_load_b128(R.rs, R.voff, (int)(p0 * (uint32_t)sizeof(u32x4)), 0);
}

// The steps of one sweep when every step holds exactly P = NT >> lcol positions (n = steps x
// P, as the cross-sweep body at its width bound gives): each thread has one task per step, at
// position c * P + tpos, so no step bound is read and no thread is idle; the step's records
// start at a uniform address.
template <int NT, int CW, bool GR, bool kAcc, bool MET, bool J0>
__device__ __forceinline__ void sweep_full(const Tile &T, uint32_t rb, uint32_t (&acc)[CW / 4]) {
    constexpr uint32_t E = MET ? 2 : 1;
    const uint32_t P = NT >> T.lcol;
    const uint32_t ra0 = T.lds0 + rb + E * T.rbo;
    if constexpr (GR) {
        // This thread's record of each step, fetched one step ahead into two registers used in
        // turn (no copy at the loop's back edge); a fetch beyond the last step reads the last
        // step's record again. With 8-byte columns through the raw buffer (rec_buf); with
        // 16-byte columns the plain load measured faster.
        const RecBuf R = rec_buf(T);
        const uint32_t last = (uint32_t)__builtin_amdgcn_readfirstlane(T.nsteps) - 1;
        const uint32_t Pu = (uint32_t)__builtin_amdgcn_readfirstlane(P);
        const GLOBAL_AS u32x4 *rp = (const GLOBAL_AS u32x4 *)T.grec + T.tpos;
        auto fetch = [&](uint32_t c) -> u32x4 {
            const uint32_t cc = c < last ? c : last;
            if constexpr (CW == 8)
                return rec_fetch(R, cc * Pu);
            else
                return rp[cc * P];
        };
        u32x4 a = fetch(0);
        for (uint32_t c = 0; c < T.nsteps; c += 2) {
            const u32x4 b = fetch(c + 1);
            __syncthreads();
            update_task<CW, kAcc, MET, J0>(T, make_uint4(a.x, a.y, a.z, a.w),
                                           ra0 + E * ((c * P) << T.lB), acc);
            if (c + 1 >= T.nsteps) break;
            a = fetch(c + 2);
            __syncthreads();
            update_task<CW, kAcc, MET, J0>(T, make_uint4(b.x, b.y, b.z, b.w),
                                           ra0 + E * (((c + 1) * P) << T.lB), acc);
        }
    } else {
        for (uint32_t c = 0; c < T.nsteps; ++c) {
            const uint4 r0 = lds_rec(c * P + T.tpos);
            __syncthreads();
            update_task<CW, kAcc, MET, J0>(T, r0, ra0 + E * ((c * P) << T.lB), acc);
        }
    }
}

// The steps of one sweep, a barrier before each (the first one also publishes the sweep's
// acceptance bits and the previous sweep's last writes). Records and step bounds are
// read-only, so each thread fetches its first record of a step before that step's barrier.
template <int NT, int CW, bool GR, bool kAcc, bool MET, bool J0>
__device__ __forceinline__ void sweep(const Tile &T, uint32_t rb, uint32_t (&acc)[CW / 4]) {
    if (T.n == T.nsteps * (NT >> T.lcol)) {  // every step full
        sweep_full<NT, CW, GR, kAcc, MET, J0>(T, rb, acc);
        return;
    }
    constexpr uint32_t E = MET ? 2 : 1;  // bytes per acceptance entry
    // Step bounds come from the tile's LDS copy of the step table, read (the same address in
    // every lane) right after each barrier: an LDS read returns in order with the task's reads,
    // where a scalar load would have to complete before the barrier.
    const LDS_AS uint16_t *so = (const LDS_AS uint16_t *)(uintptr_t)(T.lds0 + T.stp);
    const uint32_t stride = NT >> T.lcol;  // positions between a thread's tasks of one step
    uint32_t cs = 0, ce = so[1];
    if constexpr (GR && CW == 8) {
        // The first round's record of a step is fetched through the raw buffer (rec_buf) at the
        // end of the step before, by every thread (past the tile's records it reads zeros; such
        // a record is unused): no vector instruction forms its address.
        const RecBuf R = rec_buf(T);
        u32x4 rn = rec_fetch(R, 0);
        for (uint32_t c = 0; c < T.nsteps; ++c) {
            const uint32_t ntask = (ce - cs) << T.lcol;
            const u32x4 r0 = rn;
            __syncthreads();
            const uint32_t ce_next = so[c + 2];
            const uint32_t ra = (T.lds0 + rb + E * (cs << T.lB)) + E * T.rbo;
            if (T.tid < ntask)
                update_task<CW, kAcc, MET, J0>(T, make_uint4(r0.x, r0.y, r0.z, r0.w), ra, acc);
            const uint32_t rounds = (ntask - 1) / NT;
            for (uint32_t k = 1; k <= rounds; ++k)
                if (T.tid + k * NT < ntask)
                    update_task<CW, kAcc, MET, J0>(T, rec_at<GR>(T, cs + T.tpos + k * stride),
                                                   ra + E * ((k * stride) << T.lB), acc);
            rn = rec_fetch(R, ce);
            cs = ce;
            ce = __builtin_amdgcn_readfirstlane(ce_next);
        }
        return;
    }
    for (uint32_t c = 0; c < T.nsteps; ++c) {
        const uint32_t ntask = (ce - cs) << T.lcol;
        uint4 r0;  // read only by threads with a task
        if (T.tid < ntask) r0 = rec_at<GR>(T, cs + T.tpos);
        __syncthreads();
        const uint32_t ce_next = so[c + 2];  // the table repeats its last bound once
        const uint32_t ra = (T.lds0 + rb + E * (cs << T.lB)) + E * T.rbo;
        if (T.tid < ntask) update_task<CW, kAcc, MET, J0>(T, r0, ra, acc);
        // further rounds of the step (more tasks than threads): a uniform trip count
        const uint32_t rounds = (ntask - 1) / NT;
        for (uint32_t k = 1; k <= rounds; ++k)
            if (T.tid + k * NT < ntask)
                update_task<CW, kAcc, MET, J0>(T, rec_at<GR>(T, cs + T.tpos + k * stride),
                                           ra + E * ((k * stride) << T.lB), acc);
        cs = ce;
        ce = __builtin_amdgcn_readfirstlane(ce_next);  // uniform: taken where first needed
    }
}

// The first or last iteration of a chunk run on the cross-sweep body (records in global memory,
// w0 = 0): the body's steps, a barrier before each, as in sweep(), but the first iteration
// (first = true) runs only the spins that are not late (record meta bit 12), for the chunk's
// first sweep, and the last only the late ones, for its last sweep. Every task reads the
// acceptance bits of its position in buffer rb (the acceptance pass puts a late spin's bits
// where the iteration after its sweep's reads them).
template <int NT, int CW, bool J0>
__device__ __forceinline__ void body_edge(const Tile &T, uint32_t rb, bool first) {
    const LDS_AS uint16_t *so = (const LDS_AS uint16_t *)(uintptr_t)(T.lds0 + T.stp);
    uint32_t none[CW / 4] = {};
    uint32_t cs = 0, ce = __builtin_amdgcn_readfirstlane(so[1]);
    for (uint32_t c = 0; c < T.nsteps; ++c) {
        const uint32_t ntask = (ce - cs) << T.lcol;  // at most NT: body steps hold one round
        uint4 r0;
        if (T.tid < ntask) r0 = rec_at<true>(T, cs + T.tpos);
        __syncthreads();
        const uint32_t ce_next = so[c + 2];
        const uint32_t ra = (T.lds0 + rb + (cs << T.lB)) + T.rbo;
        if (T.tid < ntask && ((r0.w >> 28) & 1u) != (first ? 1u : 0u))
            update_task<CW, false, false, J0>(T, r0, ra, none);
        cs = ce;
        ce = __builtin_amdgcn_readfirstlane(ce_next);
    }
}

// k >= 1 for any visited spin, over every spin of the current LDS state (no update): a zero
// bit marks a clone whose configuration is a ground state.
template <int NT, int CW, bool GR, bool J0>
__device__ __forceinline__ void unsat_any(const Tile &T, uint32_t (&acc)[CW / 4]) {
    constexpr int G = CW / 4;
    for (uint32_t q = T.tid; q < T.n << T.lcol; q += NT) {
        const uint4 r = rec_at<GR>(T, q >> T.lcol);
        uint32_t x[G], a1[G], b1[G], a2[G], b2[G], a3[G], b3[G];
        col_load<CW>(T.colbase + (r.x & 0xFFFFu), x);
        col_load<CW>(T.colbase + (r.x >> 16), a1);
        col_load<CW>(T.colbase + (r.y & 0xFFFFu), b1);
        col_load<CW>(T.colbase + (r.y >> 16), a2);
        col_load<CW>(T.colbase + (r.z & 0xFFFFu), b2);
        col_load<CW>(T.colbase + (r.z >> 16), a3);
        col_load<CW>(T.colbase + (r.w & 0xFFFFu), b3);
        const uint32_t meta = r.w >> 16;
        const uint32_t j1 = J0 ? 0u : 0u - ((meta >> 13) & 1u);
        const uint32_t j2 = J0 ? 0u : 0u - ((meta >> 14) & 1u);
        const uint32_t j3 = J0 ? 0u : 0u - (meta >> 15);
#pragma unroll
        for (int g = 0; g < G; ++g)
            qg_word<true>(x[g], a1[g], b1[g], a2[g], b2[g], a3[g], b3[g], j1, j2, j3, 0u, acc[g]);
    }
}

// OR the threads' accumulators into the per-group LDS words (threads owning the same column
// first combine within the wave). Caller synchronises before reading T.acc.
template <int CW>
__device__ __forceinline__ void reduce_acc(const Tile &T, uint32_t (&acc)[CW / 4]) {
    constexpr int G = CW / 4;
    for (uint32_t m = T.ncol; m < 64; m <<= 1)
        for (int g = 0; g < G; ++g) acc[g] |= __shfl_xor(acc[g], (int)m);
    if ((T.tid & 63) < T.ncol)
        for (int g = 0; g < G; ++g) atomicOr(&lds_u32(T.acc + 4 * (G * T.col + g)), acc[g]);
}

// Record first hits at sweep t for the clones of group T.tid (threads below ngrp) whose bit
// in the group's accumulator is zero and that had no hit yet, and flag the instance. Returns
// the new hits.
__device__ __forceinline__ uint32_t record_hits(const Tile &T, uint32_t t, uint32_t &hm) {
    const uint32_t v = lds_u32(T.acc + 4 * T.tid);
    lds_u32(T.acc + 4 * T.tid) = 0;
    uint32_t fresh = ~v & ~hm;
    const uint32_t out = fresh;
    if (fresh) {
        int32_t *fh = T.I->first_hit + ((size_t)(T.blk0 * 8 + T.tid) << 5);
        hm |= fresh;
        while (fresh) {
            fh[__builtin_ctz(fresh)] = (int32_t)t;
            fresh &= fresh - 1;
        }
        atomicOr(&T.I->hit, 1u);
    }
    return out;
}

// Ground-state check of the current LDS state, recording hits at sweep t. Returns nonzero in
// every thread if some clone of the tile got a new hit. Ends synchronised.
template <int NT, int CW, bool GR, bool J0>
__device__ __forceinline__ uint32_t check_state(const Tile &T, uint32_t t, uint32_t &hm) {
    uint32_t acc[CW / 4] = {};
    __syncthreads();  // state final, accumulators clear
    unsat_any<NT, CW, GR, J0>(T, acc);
    reduce_acc<CW>(T, acc);
    if (T.tid == 0) lds_u32(T.flag) = 0;
    __syncthreads();
    if (T.tid < T.ngrp && record_hits(T, t, hm)) atomicOr(&lds_u32(T.flag), 1u);
    __syncthreads();
    return lds_u32(T.flag);
}

// LDS row of spin i: the instance's row map, or i itself.
__device__ __forceinline__ uint32_t lds_row(const Tile &T, uint32_t i) {
    const GLOBAL_AS uint16_t *rm = (const GLOBAL_AS uint16_t *)T.I->rowmap;
    return rm ? rm[i] : i;
}

// Stage the tile's rows global -> LDS in 16-byte pieces.
template <int NT>
__device__ __forceinline__ void load_state(const Tile &T) {
    const uint64_t *src0 = T.I->state + 4 * (size_t)T.blk0;
    for (uint32_t q = T.tid; q < T.n * T.n16; q += NT) {
        const uint32_t i = q >> T.l16, k = q & (T.n16 - 1);
        *reinterpret_cast<uint4 *>(xs_lds + T.st + lds_row(T, i) * T.rowb + 16 * k) =
            gload16(src0 + (size_t)i * T.W, k);
    }
}

// Write the tile's rows back LDS -> global (caller synchronises first).
template <int NT>
__device__ __forceinline__ void store_state(const Tile &T) {
    uint64_t *dst0 = T.I->state + 4 * (size_t)T.blk0;
    for (uint32_t q = T.tid; q < T.n * T.n16; q += NT) {
        const uint32_t i = q >> T.l16, k = q & (T.n16 - 1);
        gstore16(dst0 + (size_t)i * T.W, k,
                 *reinterpret_cast<const uint4 *>(xs_lds + T.st + lds_row(T, i) * T.rowb + 16 * k));
    }
}

// Control fields of a descriptor that kernels change while others run (t_cur, done, track,
// hit, arrived): read with vector loads at device scope, never through the scalar cache.
__device__ __forceinline__ uint32_t ld_dev(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Make the tile run a step table: its records, step bounds (staged into LDS, at most n + 1 of
// them, the last one repeated once) and, with records in global memory, the spin index of every
// position (for the acceptance pass) in its own LDS array. The caller synchronises before the
// staged arrays are read.
template <int NT, bool GR>
__device__ __forceinline__ void stage_table(Tile &T, const uint4 *grec, const int32_t *off,
                                            uint32_t nsteps) {
    T.grec = grec;
    T.step_off = off;
    T.nsteps = nsteps;
    for (uint32_t c = T.tid; c <= nsteps + 1; c += NT)
        *reinterpret_cast<uint16_t *>(xs_lds + T.stp + 2 * c) =
            (uint16_t)((const GLOBAL_AS int32_t *)off)[min(c, nsteps)];
    for (uint32_t p = T.tid; GR && p < T.n; p += NT)  // spin (bits 0-10) and late bit (12)
        *reinterpret_cast<uint16_t *>(xs_lds + T.meta + 2 * p) =
            (uint16_t)((((const GLOBAL_AS uint32_t *)grec)[4 * p + 3] >> 16) & 0x1FFFu);
}

// Sweeps [t0, t1) (one chunk) of one workgroup tile: the tile of blocks blk0 .. blk0 + B - 1
// of instance I, its rows staged in LDS and written back at the end. The caller passes
// t0 < t1.
//
// The hot loop does not track ground states. After the chunk every clone is tested once; with
// w0 = 0 a ground state is never left, so a clone in a ground state now that had no hit before
// reached it during this chunk. Only then the chunk is replayed from its start state (still
// unchanged in global memory: the tile is written back at the end) with a per-sweep test, which
// gives the exact first sweep; the replay draws the same random numbers, so it reproduces the
// same trajectory.
//
// MET (w0 > 0): a ground state can be left again, so no sweep is tested; the final pass tests
// the end configuration only.
template <int NT, int CW, bool GR, bool MET, bool J0>
__device__ __forceinline__ void tile_chunk(InstDev *I, uint32_t blk0, uint32_t t0, uint32_t t1) {
    constexpr int G = CW / 4;        // groups per column
    constexpr int LG = G == 4 ? 2 : G == 2 ? 1 : 0;
    Tile T;
    T.I = I;
    T.n = I->n;
    T.W = I->n_words;
    T.B = I->tile_blocks;
    T.lB = I->log2_tile_blocks;
    T.rowb = T.B << 5;
    T.ncol = T.B << (3 - LG);
    T.lcol = T.lB + 3 - LG;
    T.n16 = T.B << 1;
    T.l16 = T.lB + 1;
    T.ngrp = T.B << 3;
    T.blk0 = blk0;
    T.tid = threadIdx.x;
    T.col = T.tid & (T.ncol - 1);  // fixed per thread: NT is a multiple of ncol
    T.grec = I->grec;
    T.st = GR ? 0u : (uint32_t)lds_rec_bytes(T.n);
    const uint32_t rbb = (uint32_t)align16((size_t)T.n * T.B * (MET ? 2 : 1));
    T.rb0 = T.st + T.n * T.rowb;
    T.rb1 = T.rb0 + rbb;
    T.acc = T.rb0 + accept_buffers(GR, MET) * rbb;
    T.flag = T.acc + 4 * T.ngrp;
    T.meta = GR ? T.flag + 16 : 14u;  // GR: after the flag; else the top half of each record's w
    T.stp = T.flag + 16 + (GR ? (uint32_t)align16(2 * (size_t)T.n) : 0u);
    T.colbase = T.st + T.col * CW;
    T.rb_sel = (T.col << LG) >> 3;
    T.rb_shift = (T.col << LG) & 7;
    T.tpos = T.tid >> T.lcol;
    T.rbo = (T.tpos << T.lB) + T.rb_sel;
    T.step_off = I->step_off;
    T.lds0 = lds_base();
    T.thr = I->thr;
    T.thr0 = I->thr0;
    T.key0 = I->seed_lo;
    T.key1 = I->seed_hi;
    T.iid = I->inst_id;
    T.nsteps = I->n_steps;

    // Untracked chunks of an instance with a cross-sweep body run the body's iterations;
    // chunks that test every sweep and replays run the plain steps. The track flag can be set
    // by another tile of the instance meanwhile, so one thread reads it for the workgroup
    // (check_state's first barrier comes before the flag word is reused).
    if (T.tid == 0) lds_u32(T.flag) = MET ? 0u : ld_dev(&I->track);
    __syncthreads();
    const bool track = lds_u32(T.flag) != 0;
    const bool body = GR && !MET && I->bgrec != nullptr && !track;
    if (body)
        stage_table<NT, GR>(T, I->bgrec, I->bstep_off, I->n_bsteps);
    else
        stage_table<NT, GR>(T, T.grec, T.step_off, T.nsteps);
    // Records: LDS rows -> byte offsets of the rows in this tile (GR: done by the host).
    for (uint32_t p = T.tid; !GR && p < T.n; p += NT) {
        const uint4 r = gload16(I->rec, p);
        const uint32_t rowb = T.rowb;
        uint4 o;
        o.x = ((r.x & 0xFFFFu) * rowb) | (((r.x >> 16) * rowb) << 16);
        o.y = ((r.y & 0xFFFFu) * rowb) | (((r.y >> 16) * rowb) << 16);
        o.z = ((r.z & 0xFFFFu) * rowb) | (((r.z >> 16) * rowb) << 16);
        o.w = ((r.w & 0xFFFFu) * rowb) | (r.w & 0xFFFF0000u);
        lds_rec(p) = o;
    }
    load_state<NT>(T);
    if constexpr (MET) {
        uint32_t none[G] = {};
        __syncthreads();  // records and state visible to every thread
        accept_bits<NT, GR, true>(T, t0, (t0 & 1) ? T.rb1 : T.rb0);
        for (uint32_t t = t0; t < t1; ++t) {
            sweep<NT, CW, GR, false, true, J0>(T, (t & 1) ? T.rb1 : T.rb0, none);
            if (t + 1 < t1) accept_bits<NT, GR, true>(T, t + 1, (t & 1) ? T.rb0 : T.rb1);
        }
        __syncthreads();
        store_state<NT>(T);
        return;
    }
    // Groups of the tile already in a ground state keep their recorded first hit.
    uint32_t hm = 0;
    if (T.tid < T.ngrp) {
        const int32_t *fh = I->first_hit + ((size_t)(T.blk0 * 8 + T.tid) << 5);
        for (int b = 0; b < 32; ++b) hm |= (fh[b] >= 0 ? 1u : 0u) << b;
        lds_u32(T.acc + 4 * T.tid) = 0;
    }
    __syncthreads();  // records, state and accumulators visible to every thread
    if (t0 == I->t_start) check_state<NT, CW, GR, J0>(T, t0, hm);  // the run's start configuration

    if (track) {
        // This instance keeps producing new ground-state clones: test every sweep.
        uint32_t hm_t = hm;
        accept_bits<NT, GR, false>(T, t0, (t0 & 1) ? T.rb1 : T.rb0);
        for (uint32_t t = t0; t < t1; ++t) {
            uint32_t acc[G] = {};
            sweep<NT, CW, GR, true, false, J0>(T, (t & 1) ? T.rb1 : T.rb0, acc);
            reduce_acc<CW>(T, acc);
            __syncthreads();
            if (T.tid < T.ngrp) record_hits(T, t, hm_t);
            if (t + 1 < t1) accept_bits<NT, GR, false>(T, t + 1, (t & 1) ? T.rb0 : T.rb1);
        }
        hm = hm_t;
        check_state<NT, CW, GR, J0>(T, t1, hm);
    } else {
        uint32_t none[G] = {};  // unused: this loop tracks no ground states
        if constexpr (GR && !MET) {
            if (body) {
                // Iterations t0 .. t1 of the body: iteration k draws the bits of sweep k (those
                // of early spins into buffer k mod 3, of late ones into buffer k + 1 mod 3) and
                // runs sweep k's early spins with sweep k - 1's late ones, all reading buffer
                // k mod 3; the first runs sweep t0's early spins alone, the last sweep t1 - 1's
                // late spins alone, so the chunk ends with the state at exactly t1. A buffer is
                // drawn into two iterations after its last reads.
                const uint32_t rbb = T.rb1 - T.rb0;
                auto rbuf = [&](uint32_t k) { return T.rb0 + (k % 3u) * rbb; };
                accept_bits<NT, GR, false, true>(T, t0, rbuf(t0), rbuf(t0 + 1));
                body_edge<NT, CW, J0>(T, rbuf(t0), true);
                for (uint32_t k = t0 + 1; k < t1; ++k) {
                    accept_bits<NT, GR, false, true>(T, k, rbuf(k), rbuf(k + 1));
                    sweep<NT, CW, GR, false, false, J0>(T, rbuf(k), none);
                }
                body_edge<NT, CW, J0>(T, rbuf(t1), false);
            }
        }
        if (!body) {
            accept_bits<NT, GR, false>(T, t0, (t0 & 1) ? T.rb1 : T.rb0);
            for (uint32_t t = t0; t < t1; ++t) {
                sweep<NT, CW, GR, false, false, J0>(T, (t & 1) ? T.rb1 : T.rb0, none);
                if (t + 1 < t1) accept_bits<NT, GR, false>(T, t + 1, (t & 1) ? T.rb0 : T.rb1);
            }
        }
        if (check_state<NT, CW, GR, J0>(T, t1, hm)) {
            // Replay from the chunk's start state with a per-sweep ground-state test, on the
            // plain steps (check_state ends synchronised, so the tables can be restaged).
            if (body) stage_table<NT, GR>(T, I->grec, I->step_off, I->n_steps);
            uint32_t hm_replay = 0;  // hits before this chunk; the end check's are redone
            if (T.tid < T.ngrp) {
                const int32_t *fh = I->first_hit + ((size_t)(T.blk0 * 8 + T.tid) << 5);
                for (int b = 0; b < 32; ++b)
                    hm_replay |= (fh[b] >= 0 && fh[b] < (int32_t)t1 ? 1u : 0u) << b;
            }
            __syncthreads();
            load_state<NT>(T);
            accept_bits<NT, GR, false>(T, t0, (t0 & 1) ? T.rb1 : T.rb0);
            for (uint32_t t = t0; t < t1; ++t) {
                uint32_t acc[G] = {};
                sweep<NT, CW, GR, true, false, J0>(T, (t & 1) ? T.rb1 : T.rb0, acc);
                reduce_acc<CW>(T, acc);
                __syncthreads();
                if (T.tid < T.ngrp) record_hits(T, t, hm_replay);
                if (t + 1 < t1) accept_bits<NT, GR, false>(T, t + 1, (t & 1) ? T.rb0 : T.rb1);
            }
            if (T.tid == 0) atomicOr(&I->track, 1u);
        }
    }
    __syncthreads();
    store_state<NT>(T);
}

// One chunk (K sweeps, or fewer at the budget end) of every tile in `tiles`, one workgroup per
// tile. The grid holds every tile of every instance of the batch with this launch shape; tiles
// of finished instances return at once.
template <int NT, int CW, bool GR, bool MET>
__global__ __launch_bounds__(NT) void qg_chunk(InstDev *__restrict__ insts,
                                               const uint2 *__restrict__ tiles) {
    const uint2 tile = tiles[blockIdx.x];
    InstDev *I = insts + tile.x;
    if (ld_dev(&I->done)) return;
    const uint32_t t0 = ld_dev(&I->t_cur);
    const uint32_t t1 = min(t0 + I->chunk, I->t_stop);
    if (t0 >= t1) return;
    // the gauge is used with records in global memory only (the host sets it so)
    if (GR && I->gauge)
        tile_chunk<NT, CW, GR, MET, true>(I, tile.y, t0, t1);
    else
        tile_chunk<NT, CW, GR, MET, false>(I, tile.y, t0, t1);
}

// ------------------------------------------------------------------------------ control

// After a chunk: advance every unfinished instance, end it at the budget or (stop-on-first)
// once a ground state was seen, and count the ones still running. One workgroup.
__global__ __launch_bounds__(256) void qg_decide(InstDev *insts, int count, uint32_t *active) {
    __shared__ uint32_t total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    uint32_t mine = 0;
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        InstDev *I = insts + k;
        if (I->done) continue;
        const uint32_t t = min(I->t_cur + I->chunk, I->t_stop);
        I->t_cur = t;
        const bool stop = t >= I->t_stop || ((I->flags & XS_STOP_ON_FIRST) && I->hit);
        if (stop)
            I->done = 1;
        else
            ++mine;
    }
    atomicAdd(&total, mine);
    __syncthreads();
    if (threadIdx.x == 0) *active = total;
}

// ------------------------------------------------------------------------------ work queue

// A persistent launch runs the chunks of many instances without a launch per chunk. Tickets
// (Q->head) are taken in order; ticket q is served by slot q of the ring, which a push fills
// with (launch tag << 32) | tile index. A set-up kernel fills the first slots with every tile
// of every unfinished instance (largest tiles first: the host orders the tile list). The last
// tile of an instance to finish a chunk decides for the instance, as qg_decide does for the
// launch-per-chunk loop, and while the instance may run more chunks in this launch it reserves
// slots for all its tiles and publishes them. Every published slot is served: a ticket below
// the reserved count is held by a workgroup that takes it and waits for its slot, and slots
// are published by workgroups that are running. Once no instance of the launch can push any
// more (Q->live = 0), every reserved slot has been served, so the workgroups still waiting hold
// tickets that no push will reach; Q->finished releases them.

constexpr uint32_t kNoItem = 0xFFFFFFFFu;

__global__ __launch_bounds__(256) void qg_queue_clear(uint64_t *ring, uint32_t cap) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < cap; i += (size_t)gridDim.x * 256)
        ring[i] = 0;
}

// One workgroup: every unfinished instance (in tile-list order) gets a place in the ring for
// its tiles and a budget of epoch_chunks chunks; the tiles are written in tile-list order.
__global__ __launch_bounds__(1024) void qg_queue_setup(InstDev *insts, int count,
                                                       const uint32_t *order, const uint2 *tiles,
                                                       uint32_t n_tiles, QueueDev *Q, uint32_t gen,
                                                       uint32_t epoch_chunks) {
    __shared__ uint32_t scan[1024];
    __shared__ uint32_t s_base, s_live;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        s_base = 0;
        s_live = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < count; c0 += 1024) {
        const int j = c0 + (int)tid;
        InstDev *I = j < count ? insts + order[j] : nullptr;
        const bool run = I && !ld_dev(&I->done);
        const uint32_t v = run ? I->ntiles : 0u;
        scan[tid] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {  // inclusive prefix sum
            const uint32_t add = tid >= d ? scan[tid - d] : 0u;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        if (run) {
            I->ring_off = s_base + scan[tid] - v;
            st_dev(&I->arrived, 0u);
            st_dev(&I->epoch_left, epoch_chunks);
        }
        const int nrun = __syncthreads_count(run);
        if (tid == 0) {
            s_base += scan[1023];
            s_live += (uint32_t)nrun;
        }
        __syncthreads();
    }
    for (uint32_t t = tid; t < n_tiles; t += 1024) {
        const InstDev *I = insts + tiles[t].x;
        if (!ld_dev(&I->done)) Q->ring[I->ring_off + (t - I->tile0)] = (uint64_t)gen << 32 | t;
    }
    if (tid == 0) {
        st_dev(&Q->head, 0u);
        st_dev(&Q->tail, s_base);
        st_dev(&Q->live, s_live);
        st_dev(&Q->active, s_live);
        st_dev(&Q->error, 0u);
        st_dev(&Q->finished, s_live == 0 ? 1u : 0u);
    }
}

// Take the next ticket and wait for its slot: the tile index, or kNoItem once no push can reach
// the ticket any more. A wait longer than Q->wait_limit wall-clock ticks (the host sets a
// minute; a launch's chunks take seconds at most) can only come from a broken queue: the
// workgroup then sets Q->error, which the host reports, and ends the launch.
__device__ uint32_t queue_pop(QueueDev *Q, uint32_t gen) {
    const uint32_t q = atomicAdd(&Q->head, 1u);
    if (q >= Q->cap) return kNoItem;
    const uint64_t t_start = wall_clock64();
    for (;;) {
        const uint64_t v =
            __hip_atomic_load(&Q->ring[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == gen) return (uint32_t)v;
        if (ld_dev(&Q->finished)) return kNoItem;
        if (wall_clock64() - t_start > Q->wait_limit) {
            st_dev(&Q->error, 1u);
            st_dev(&Q->finished, 1u);
            return kNoItem;
        }
        __builtin_amdgcn_s_sleep(32);  // about 2,000 clocks between polls
    }
}

// The last tile of an instance's item (nrun chunks ending at t1) to arrive: advance the
// instance, end it at its budget or (stop-on-first) once a ground state was seen, and reserve
// slots for its next item while it may run more chunks in this launch. Returns the first
// reserved slot, or kNoItem.
__device__ uint32_t queue_decide(InstDev *I, QueueDev *Q, uint32_t t1, uint32_t nrun) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every tile's hits
    st_dev(&I->arrived, 0u);
    st_dev(&I->t_cur, t1);
    const bool stop = t1 >= I->t_stop || ((I->flags & XS_STOP_ON_FIRST) && ld_dev(&I->hit));
    const uint32_t el = ld_dev(&I->epoch_left);
    const uint32_t left = el > nrun ? el - nrun : 0u;
    st_dev(&I->epoch_left, left);
    if (stop) {
        st_dev(&I->done, 1u);
        atomicSub(&Q->active, 1u);
    }
    uint32_t base = kNoItem;
    if (!stop && left > 0) {
        base = atomicAdd(&Q->tail, I->ntiles);
        if (base + I->ntiles > Q->cap) {  // cannot happen with cap >= tiles x epoch_chunks
            st_dev(&Q->error, 1u);
            st_dev(&Q->finished, 1u);
            base = kNoItem;
        }
    } else if (atomicSub(&Q->live, 1u) == 1u) {
        st_dev(&Q->finished, 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // control fields before the slots
    return base;
}

// The persistent kernel: `grid` workgroups serve tickets until the queue is finished. Each tile
// runs with its instance's column width and record placement.
template <int NT, bool MET>
__global__ __launch_bounds__(NT) void qg_queue_run(InstDev *__restrict__ insts,
                                                   const uint2 *__restrict__ tiles, QueueDev *Q,
                                                   uint32_t gen) {
    __shared__ uint32_t s_item, s_push;
    for (;;) {
        if (threadIdx.x == 0) s_item = queue_pop(Q, gen);
        __syncthreads();
        const uint32_t item = s_item;
        if (item == kNoItem) return;
        // acquire, in every wave: the pusher's control fields and the tile's state and first
        // hits from its last chunk (written by other workgroups, possibly on other XCDs)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint2 tile = tiles[item];
        InstDev *I = insts + tile.x;
        const uint32_t t0 = ld_dev(&I->t_cur);
        // An instance that does not stop at its first ground state runs to its budget whatever
        // its tiles find, and its tiles never wait for each other: a tile runs all the chunks
        // the instance may still run in this launch back to back, as one item with one
        // arrival. With stop-on-first every tile must end at the same chunk, so an item is one
        // chunk and the last arrival decides.
        const uint32_t nrun =
            (I->flags & XS_STOP_ON_FIRST) ? 1u : max(ld_dev(&I->epoch_left), 1u);
        const uint32_t t1 = (uint32_t)min((uint64_t)t0 + (uint64_t)nrun * I->chunk,
                                          (uint64_t)I->t_stop);
        // the gauge is used with records in global memory only (the host sets it so)
        const bool gr = I->grec != nullptr, j0 = I->gauge != nullptr;
        for (uint32_t tc = t0; tc < t1; tc += I->chunk) {
            const uint32_t te = min(tc + I->chunk, t1);
            // (the previous chunk's write-back read the LDS, so wait for it before the next
            // chunk stages its tables; each chunk stages the rows again: keeping them in LDS
            // measured 1.3 % slower)
            if (tc != t0) __syncthreads();
            if (I->col_bytes == 16) {
                if (gr) {
                    if (j0) tile_chunk<NT, 16, true, MET, true>(I, tile.y, tc, te);
                    else tile_chunk<NT, 16, true, MET, false>(I, tile.y, tc, te);
                } else {
                    tile_chunk<NT, 16, false, MET, false>(I, tile.y, tc, te);
                }
            } else {
                if (gr) {
                    if (j0) tile_chunk<NT, 8, true, MET, true>(I, tile.y, tc, te);
                    else tile_chunk<NT, 8, true, MET, false>(I, tile.y, tc, te);
                } else {
                    tile_chunk<NT, 8, false, MET, false>(I, tile.y, tc, te);
                }
            }
        }
        // Release this tile's state and first hits to the device before its arrival. Every
        // wave fences its own stores: a wave's fence waits only for that wave's stores, and a
        // workgroup barrier does not make other waves' stores complete.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t push = kNoItem;
            if (atomicAdd(&I->arrived, 1u) + 1u == I->ntiles) push = queue_decide(I, Q, t1, nrun);
            s_push = push;
        }
        __syncthreads();
        const uint32_t base = s_push;
        if (base != kNoItem) {
            const uint32_t n = I->ntiles, first = I->tile0;
            for (uint32_t j = threadIdx.x; j < n; j += NT)
                __hip_atomic_store(&Q->ring[base + j], (uint64_t)gen << 32 | (first + j),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // s_item and s_push are rewritten for the next ticket
    }
}

// ------------------------------------------------------------------------------ gauge

// The state of instance I + blockIdx.y, if it runs in its gauge, flipped row by row where
// g_i = 1: into the gauge before its chunks, back after them. One thread per 16 bytes.
__global__ __launch_bounds__(256) void qg_gauge_flip(InstDev *I) {
    I += blockIdx.y;
    if (!I->gauge) return;
    const uint32_t per_row = I->n_words >> 1;  // 16-byte pieces per row
    const uint64_t total = (uint64_t)I->n * per_row;
    const uint8_t *g = I->gauge;
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * 256) {
        const uint32_t i = (uint32_t)(q / per_row);
        if (!g[i]) continue;
        uint64_t *w = I->state + (size_t)i * I->n_words + 2 * (q % per_row);
        const uint4 v = gload16(w, 0);
        gstore16(w, 0, make_uint4(~v.x, ~v.y, ~v.z, ~v.w));
    }
}

// ------------------------------------------------------------------------------ final pass

// Final pass. Each kernel serves instance I + blockIdx.y, so one launch covers a whole batch
// (grids sized for the batch's largest instance; threads beyond an instance's range return).
//
// Energies at the end sweep, E = 2U - N, from bit-sliced counters of unsatisfied triplets (one
// thread per 64-clone word). A clone whose end configuration is a ground state and has no
// recorded hit gets first_hit = end sweep.
__global__ __launch_bounds__(256) void qg_energy(InstDev *I) {
    I += blockIdx.y;
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t W = I->n_words, n = I->n;
    if (w >= W) return;
    const uint64_t *st = I->state;
    uint64_t cnt[12];  // U <= n <= 2048 < 2^12
#pragma unroll
    for (int k = 0; k < 12; ++k) cnt[k] = 0;
    for (uint32_t t = 0; t < n; ++t) {
        const uint2 tr = I->tri[t];
        uint64_t u = st[(size_t)(tr.x & 0xFFFFu) * W + w] ^ st[(size_t)(tr.x >> 16) * W + w] ^
                     st[(size_t)(tr.y & 0xFFFFu) * W + w];
        if (tr.y >> 16) u = ~u;
        // add u (one bit per clone) to the vertical counter
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const uint64_t carry = cnt[k] & u;
            cnt[k] ^= u;
            u = carry;
        }
    }
    const int32_t tend = (int32_t)I->t_cur;
    for (int b = 0; b < 64; ++b) {
        uint32_t U = 0;
#pragma unroll
        for (int k = 0; k < 12; ++k) U |= (uint32_t)((cnt[k] >> b) & 1u) << k;
        const size_t c = (size_t)w * 64 + b;
        if (I->energy) I->energy[c] = 2 * (int32_t)U - (int32_t)n;
        if (U == 0 && I->first_hit[c] < 0) I->first_hit[c] = tend;
    }
}

__global__ __launch_bounds__(256) void qg_tts(InstDev *I) {
    I += blockIdx.y;
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (size_t)I->n_words * 64) return;
    const int32_t f = I->first_hit[c];
    if (f >= 0) atomicMin(&I->tts, f);
}

__global__ __launch_bounds__(256) void qg_winner(InstDev *I) {
    I += blockIdx.y;
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (size_t)I->n_words * 64) return;
    if (I->tts != INT32_MAX && I->first_hit[c] == I->tts) atomicMin(&I->winner, (int32_t)c);
}

__global__ __launch_bounds__(256) void qg_gather(InstDev *I) {
    I += blockIdx.y;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I->n || I->winner == INT32_MAX) return;
    const uint32_t c = (uint32_t)I->winner;
    const uint64_t wv = I->state[(size_t)i * I->n_words + (c >> 6)];
    I->solved[i] = ((wv >> (c & 63)) & 1u) ? (int8_t)-1 : (int8_t)1;
}

}  // namespace

size_t chunk_lds_bytes(uint32_t n, uint32_t B, bool rec_global, bool met) {
    return (rec_global ? align16(2 * (size_t)n) : lds_rec_bytes(n)) + (size_t)n * B * 32 +
           accept_buffers(rec_global, met) * align16((size_t)n * B * (met ? 2 : 1)) +
           (size_t)B * 8 * 4 + 16 + align16(2 * ((size_t)n + 2));
}

hipError_t launch_init(InstDev *d_inst, const InstDev &h, hipStream_t s) {
    const uint64_t total = (uint64_t)h.n * ((h.n_words >> 1) + 1);
    const uint32_t blocks = (uint32_t)((total + 255) / 256);
    hipLaunchKernelGGL(qg_init, dim3(blocks), dim3(256), 0, s, d_inst);
    return hipGetLastError();
}

template <int NT, int CW, bool GR, bool MET>
hipError_t launch_chunk_nt(InstDev *d_insts, const uint2 *d_tiles, int n_tiles,
                           size_t lds_bytes, hipStream_t s) {
    // The 160 KB dynamic-LDS limit is set once per device (bit d of the mask; setting it twice
    // from racing threads is harmless).
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = uint64_t(1) << (dev & 63);
    if (!(attr_set.load(std::memory_order_acquire) & bit)) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(qg_chunk<NT, CW, GR, MET>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit, std::memory_order_release);
    }
    hipLaunchKernelGGL((qg_chunk<NT, CW, GR, MET>), dim3(n_tiles), dim3(NT), lds_bytes, s,
                       d_insts, d_tiles);
    return hipGetLastError();
}

template <int CW, bool GR, bool MET>
hipError_t launch_chunk_cw(InstDev *d_insts, const uint2 *d_tiles, int n_tiles,
                           int threads, size_t lds_bytes, hipStream_t s) {
    switch (threads) {
        case 64: return launch_chunk_nt<64, CW, GR, MET>(d_insts, d_tiles, n_tiles, lds_bytes, s);
        case 128: return launch_chunk_nt<128, CW, GR, MET>(d_insts, d_tiles, n_tiles, lds_bytes, s);
        case 256: return launch_chunk_nt<256, CW, GR, MET>(d_insts, d_tiles, n_tiles, lds_bytes, s);
        case 512: return launch_chunk_nt<512, CW, GR, MET>(d_insts, d_tiles, n_tiles, lds_bytes, s);
        case 1024:
            return launch_chunk_nt<1024, CW, GR, MET>(d_insts, d_tiles, n_tiles, lds_bytes, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool GR, bool MET>
hipError_t launch_chunk_gr(InstDev *d_insts, const uint2 *d_tiles, int n_tiles,
                           int threads, int col_bytes, size_t lds_bytes, hipStream_t s) {
    switch (col_bytes) {
        case 4:
            return launch_chunk_cw<4, GR, MET>(d_insts, d_tiles, n_tiles, threads, lds_bytes, s);
        case 8:
            return launch_chunk_cw<8, GR, MET>(d_insts, d_tiles, n_tiles, threads, lds_bytes, s);
        case 16:
            return launch_chunk_cw<16, GR, MET>(d_insts, d_tiles, n_tiles, threads, lds_bytes, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chunk(InstDev *d_insts, const uint2 *d_tiles, int n_tiles, int threads,
                        int col_bytes, bool rec_global, bool met, size_t lds_bytes,
                        hipStream_t s) {
    if (met)
        return rec_global ? launch_chunk_gr<true, true>(d_insts, d_tiles, n_tiles, threads,
                                                        col_bytes, lds_bytes, s)
                          : launch_chunk_gr<false, true>(d_insts, d_tiles, n_tiles, threads,
                                                         col_bytes, lds_bytes, s);
    return rec_global ? launch_chunk_gr<true, false>(d_insts, d_tiles, n_tiles, threads,
                                                     col_bytes, lds_bytes, s)
                      : launch_chunk_gr<false, false>(d_insts, d_tiles, n_tiles, threads,
                                                      col_bytes, lds_bytes, s);
}

hipError_t launch_decide(InstDev *d_insts, int count, uint32_t *d_active, hipStream_t s) {
    hipLaunchKernelGGL(qg_decide, dim3(1), dim3(256), 0, s, d_insts, count, d_active);
    return hipGetLastError();
}

hipError_t launch_final(InstDev *d_insts, int count, uint32_t max_words, uint32_t max_n,
                        hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const uint64_t max_clones = (uint64_t)max_words * 64;
    const dim3 g_words((max_words + 255) / 256, (uint32_t)count);
    const dim3 g_clones((uint32_t)((max_clones + 255) / 256), (uint32_t)count);
    const dim3 g_spins((max_n + 255) / 256, (uint32_t)count);
    hipLaunchKernelGGL(qg_energy, g_words, dim3(256), 0, s, d_insts);
    hipLaunchKernelGGL(qg_tts, g_clones, dim3(256), 0, s, d_insts);
    hipLaunchKernelGGL(qg_winner, g_clones, dim3(256), 0, s, d_insts);
    hipLaunchKernelGGL(qg_gather, g_spins, dim3(256), 0, s, d_insts);
    return hipGetLastError();
}

hipError_t launch_gauge_flip(InstDev *d_insts, int count, uint64_t max_pieces, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const uint32_t bx =
        (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(2048, (max_pieces + 255) / 256));
    hipLaunchKernelGGL(qg_gauge_flip, dim3(bx, (uint32_t)count), dim3(256), 0, s, d_insts);
    return hipGetLastError();
}

hipError_t launch_queue_clear(uint64_t *ring, uint32_t cap, hipStream_t s) {
    const uint32_t blocks = std::max(1u, std::min(1024u, (cap + 255) / 256));
    hipLaunchKernelGGL(qg_queue_clear, dim3(blocks), dim3(256), 0, s, ring, cap);
    return hipGetLastError();
}

hipError_t launch_queue_setup(InstDev *d_insts, int count, const uint32_t *d_order,
                              const uint2 *d_tiles, uint32_t n_tiles, QueueDev *d_q,
                              uint32_t gen, uint32_t epoch_chunks, hipStream_t s) {
    hipLaunchKernelGGL(qg_queue_setup, dim3(1), dim3(1024), 0, s, d_insts, count, d_order,
                       d_tiles, n_tiles, d_q, gen, epoch_chunks);
    return hipGetLastError();
}

template <int NT, bool MET>
hipError_t set_queue_lds_limit() {
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = uint64_t(1) << (dev & 63);
    if (!(attr_set.load(std::memory_order_acquire) & bit)) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(qg_queue_run<NT, MET>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 64);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit, std::memory_order_release);
    }
    return hipSuccess;
}

template <int NT, bool MET>
hipError_t launch_queue_nt(InstDev *d_insts, const uint2 *d_tiles, QueueDev *d_q, uint32_t gen,
                           size_t lds_bytes, int grid, hipStream_t s) {
    hipError_t e = set_queue_lds_limit<NT, MET>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((qg_queue_run<NT, MET>), dim3(grid), dim3(NT), lds_bytes, s, d_insts,
                       d_tiles, d_q, gen);
    return hipGetLastError();
}

hipError_t launch_queue_run(InstDev *d_insts, const uint2 *d_tiles, QueueDev *d_q, uint32_t gen,
                            int threads, bool met, size_t lds_bytes, int grid, hipStream_t s) {
    if (threads == 256)
        return met ? launch_queue_nt<256, true>(d_insts, d_tiles, d_q, gen, lds_bytes, grid, s)
                   : launch_queue_nt<256, false>(d_insts, d_tiles, d_q, gen, lds_bytes, grid, s);
    if (threads == 512)
        return met ? launch_queue_nt<512, true>(d_insts, d_tiles, d_q, gen, lds_bytes, grid, s)
                   : launch_queue_nt<512, false>(d_insts, d_tiles, d_q, gen, lds_bytes, grid, s);
    return hipErrorInvalidValue;
}

template <int NT, bool MET>
hipError_t queue_blocks_nt(size_t lds_bytes, int *blocks) {
    hipError_t e = set_queue_lds_limit<NT, MET>();
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, reinterpret_cast<const void *>(qg_queue_run<NT, MET>), NT, lds_bytes);
}

hipError_t queue_blocks_per_cu(int threads, bool met, size_t lds_bytes, int *blocks) {
    if (threads == 256)
        return met ? queue_blocks_nt<256, true>(lds_bytes, blocks)
                   : queue_blocks_nt<256, false>(lds_bytes, blocks);
    if (threads == 512)
        return met ? queue_blocks_nt<512, true>(lds_bytes, blocks)
                   : queue_blocks_nt<512, false>(lds_bytes, blocks);
    return hipErrorInvalidValue;
}

// Device scratch of xs_run_batch_noalloc: one array per device, held until the process ends,
// shared by every such call on that device (calls that overlap on one device race). In host
// code its name is not a device address; noalloc_scratch looks the address up.
static __device__ __align__(256) uint8_t scratch[XS_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(uint8_t **ptr, size_t *bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static uint8_t *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<uint8_t *>(p);
    }
    *ptr = addr[dev];
    *bytes = sizeof scratch;
    return hipSuccess;
}

}  // namespace xs
