// Device-side helpers shared by the HIP translation units: LDS staging of
// the lookup tables, the sublattice-coding representative search, index
// lookups and small reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ed_internal.hpp"

namespace ed {

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return set_error(ED_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxBondWords = 4;   // up to 256 bonds
constexpr int kWave = 64;
constexpr uint64_t kEmpty = ~0ull;  // empty slot key (norm index 255 never occurs)

enum { IDX_HASH = 0, IDX_LIMITS = 1 };

struct BondLds {
    uint64_t mask;     // both sites of the bond
    double jhalf;      // J_b / 2: exchange amplitude of the flip term
    double jzhalf;     // Jz_b / 2: an antiparallel bond lowers the diagonal by this
};

// ---------------------------------------------------------------------------
// LDS staging
// ---------------------------------------------------------------------------
template <typename AT>
struct Ctx {
    int N, ns, m, cb, nc;
    uint32_t mmask, cmask;
    uint64_t low_mask;           // state bits below the top block
    const uint32_t *rep;
    const uint32_t *sym;         // [count, e_1, ...], e = g | u << 16 | flip << 31
    const AT *act;
    const uint8_t *shift;
    const double *chi;           // [ng] real, or [ng][2] complex
    const double *div_sqrt;
    const double *div_rsqrt;
    const uint32_t *div_val;
    const BondLds *bonds;
    const uint16_t *rank;
    const uint16_t *pos1;        // two-stage search: source block at position 1 | its state bit offset << 8
    int staged;                  // pos1 is staged
    const uint64_t *between;     // fermions: orbitals strictly between the two of each bond
    const uint16_t *g_u;         // fermions: distinct permutation of every group element
};

__device__ __forceinline__ void lds_copy(char *dst, const void *src, uint32_t bytes)
{
    const uint4 *s = (const uint4 *)src;
    uint4 *d = (uint4 *)dst;
    for (uint32_t k = threadIdx.x; k < bytes / 16; k += blockDim.x) d[k] = s[k];
}

template <typename AT>
__device__ __forceinline__ Ctx<AT> stage(const DevModel &dm, char *lds)
{
    lds_copy(lds, dm.blob, dm.lds_total);
    __syncthreads();
    Ctx<AT> c;
    c.N = dm.N;
    c.ns = dm.ns;
    c.m = dm.m;
    c.cb = dm.chunk_bits;
    c.nc = dm.n_chunks;
    c.mmask = dm.P - 1;
    c.cmask = (1u << dm.chunk_bits) - 1u;
    c.low_mask = (dm.N - dm.m >= 64) ? ~0ull : ((1ull << (dm.N - dm.m)) - 1ull);
    c.rep = (const uint32_t *)(lds + dm.off_rep);
    c.sym = (const uint32_t *)(lds + dm.off_sym);
    c.act = (const AT *)(lds + dm.off_act);
    c.shift = (const uint8_t *)(lds + dm.off_shift);
    c.chi = (const double *)(lds + dm.off_chi);
    c.div_sqrt = (const double *)(lds + dm.off_div);
    c.div_rsqrt = c.div_sqrt + dm.n_div;
    c.div_val = (const uint32_t *)(lds + dm.off_divval);
    c.bonds = (const BondLds *)(lds + dm.off_bonds);
    c.rank = (const uint16_t *)(lds + dm.off_rank);
    c.pos1 = (const uint16_t *)(lds + dm.off_pos1);
    c.staged = dm.staged;
    c.between = (const uint64_t *)(lds + dm.off_between);
    c.g_u = (const uint16_t *)(lds + dm.off_gu);
    return c;
}

// 2-byte action-table entry of a fermionic basis: the image in bits 0-11,
// the target block index in bits 12-14 (chunk 0), and the parity of the
// orbital pairs inside the chunk whose order the element reverses in bit 15.
// A type of its own, so that the spin tables' 2-byte entries (block index in
// bits 12-15) keep their layout and their kernels' code.
struct FermiU16 {
    uint16_t v;
    __device__ __forceinline__ operator uint32_t() const { return v; }
};

// Action-table entries: uint8 holds the image pattern only (its block
// position comes from the shift table); uint16 / uint32 entries of chunk 0
// also carry the target block index above bit 12 / 16, which saves that
// lookup.  kParity: the bit of fermionic entries holding the chunk's parity.
template <typename AT>
struct ActTraits {
    static constexpr bool kPos = sizeof(AT) > 1;
    static constexpr int kPosShift = sizeof(AT) == 2 ? 12 : 16;
    static constexpr uint32_t kPosMask = sizeof(AT) == 4 ? 0xFFu : 0u;   // 0: every bit above the image
    static constexpr int kParity = 31;
};
template <>
struct ActTraits<FermiU16> {
    static constexpr bool kPos = true;
    static constexpr int kPosShift = 12;
    static constexpr uint32_t kPosMask = 0x7u;
    static constexpr int kParity = 15;
};

template <typename AT>
__device__ __forceinline__ uint64_t place_block(const Ctx<AT> &c, uint32_t u, int ns, int X, uint32_t e)
{
    if (ActTraits<AT>::kPos) {
        const uint32_t img = e & ((1u << ActTraits<AT>::kPosShift) - 1u);
        // fermionic entries keep their top bit for the sign parity
        const uint32_t pos = ActTraits<AT>::kPosMask ? (e >> ActTraits<AT>::kPosShift) & ActTraits<AT>::kPosMask
                                                     : e >> ActTraits<AT>::kPosShift;
        // position and block width are below 2^24: full-rate 24-bit multiply
        return (uint64_t)img << ((uint32_t)(c.N - c.m) - __umul24(pos, (uint32_t)c.m));
    }
    return (uint64_t)e << c.shift[u * ns + X];
}

// image of block X of s under the permutation u (chunked action table)
template <typename AT>
__device__ __forceinline__ uint32_t block_image(const Ctx<AT> &c, uint32_t u, int X, uint32_t sx)
{
    const AT *t = c.act + ((size_t)(u * c.ns + X) * c.nc << c.cb);
    uint32_t v = 0;
    for (int k = 0; k < c.nc; ++k) v |= t[(k << c.cb) | ((sx >> (k * c.cb)) & c.cmask)];
    return v;
}

// all blocks except Y of g s, placed at their target positions, flip applied
template <typename AT>
__device__ __forceinline__ uint64_t image_below_top(const Ctx<AT> &c, uint32_t u, uint32_t fl, int Y, uint64_t s)
{
    uint64_t v = 0;
    for (int X = 0; X < c.ns; ++X) {
        if (X == Y) continue;
        const uint32_t sx = (uint32_t)(s >> (c.N - (X + 1) * c.m)) & c.mmask;
        v |= place_block(c, u, c.ns, X, block_image(c, u, X, sx));
    }
    if (fl) v ^= c.low_mask;
    return v;
}

// ---------------------------------------------------------------------------
// Alg. "Sublattice coding algorithm for finding the representative":
//   MinRep = min_X Rep_X(s_X); for every block Y attaining it and every g in
//   Sym_Y(s_Y), assemble g s from the per-block action table and keep the
//   strict minimum.  The top block of every candidate is MinRep itself, so
//   only the other blocks are assembled.
// ---------------------------------------------------------------------------
template <typename AT>
__device__ __forceinline__ uint64_t find_rep(const Ctx<AT> &c, uint64_t s, uint32_t &g_best, uint32_t &min_val)
{
    const int N = c.N, m = c.m, ns = c.ns;
    const uint32_t P = c.mmask + 1;
    uint32_t minr = 0xFFFFFFFFu, tie = 0;
    for (int X = 0; X < ns; ++X) {
        const uint32_t sx = (uint32_t)(s >> (N - (X + 1) * m)) & c.mmask;
        const uint32_t r = c.rep[X * P + sx] & 0xFFFFu;
        if (r < minr) {
            minr = r;
            tie = 1u << X;
        } else if (r == minr) {
            tie |= 1u << X;
        }
    }
    const uint64_t top = (uint64_t)minr << (N - m);
    uint64_t best = ~0ull;
    uint32_t bg = 0;
    while (tie) {
        const int Y = __builtin_ctz(tie);
        tie &= tie - 1;
        const uint32_t sy = (uint32_t)(s >> (N - (Y + 1) * m)) & c.mmask;
        const uint32_t off = c.rep[Y * P + sy] >> 16;
        const uint32_t cnt = c.sym[off];
        for (uint32_t k = 1; k <= cnt; ++k) {
            const uint32_t ent = c.sym[off + k];
            const uint32_t g = ent & 0xFFFFu;
            const uint64_t v = image_below_top(c, (ent >> 16) & 0x7FFFu, ent >> 31, Y, s) | top;
            if (v < best) {
                best = v;
                bg = g;
            }
        }
    }
    g_best = bg;
    min_val = minr;
    return best;
}

// The same search with the number of sublattices (and, if NC > 0, the number
// of action-table chunks) fixed at compile time: the substate blocks stay in
// registers and the block and chunk loops unroll.  Every block of a candidate
// is assembled, the one landing on top included, so that the table reads of
// a candidate are independent and issue together; the top block is then
// replaced by MinRep, and the flip applied to the rest.
template <typename AT, int NS, int NC>
__device__ __forceinline__ uint64_t find_rep_ns(const Ctx<AT> &c, uint64_t s, uint32_t &g_best)
{
    const int N = c.N, m = c.m, cb = c.cb;
    const int nc = NC > 0 ? NC : c.nc;
    const uint32_t P = c.mmask + 1;
    uint32_t sx[NS];
    uint32_t minr = 0xFFFFFFFFu;
#pragma unroll
    for (int X = 0; X < NS; ++X) {
        sx[X] = (uint32_t)(s >> (N - (X + 1) * m)) & c.mmask;
        minr = min(minr, c.rep[X * P + sx[X]] & 0xFFFFu);
    }
    uint32_t tie = 0;
#pragma unroll
    for (int X = 0; X < NS; ++X) tie |= (uint32_t)((c.rep[X * P + sx[X]] & 0xFFFFu) == minr) << X;
    const uint64_t top = (uint64_t)minr << (N - m);
    uint64_t best = ~0ull;
    uint32_t bg = 0;
    while (tie) {
        const int Y = __builtin_ctz(tie);
        tie &= tie - 1;
        const uint32_t sy = (uint32_t)(s >> (N - (Y + 1) * m)) & c.mmask;
        const uint32_t off = c.rep[Y * P + sy] >> 16;
        const uint32_t cnt = c.sym[off];
        for (uint32_t k = 1; k <= cnt; ++k) {
            const uint32_t ent = c.sym[off + k];
            const uint32_t u = (ent >> 16) & 0x7FFFu;
            const AT *tu = c.act + ((u * (uint32_t)(NS * nc)) << cb);
            uint64_t v = 0;
#pragma unroll
            for (int X = 0; X < NS; ++X) {
                const AT *t = tu + ((X * nc) << cb);
                uint32_t blk = 0;
                if (NC > 0) {
#pragma unroll
                    for (int k2 = 0; k2 < (NC > 0 ? NC : 1); ++k2)
                        blk |= t[(k2 << cb) | ((sx[X] >> (k2 * cb)) & c.cmask)];
                } else {
                    for (int k2 = 0; k2 < nc; ++k2) blk |= t[(k2 << cb) | ((sx[X] >> (k2 * cb)) & c.cmask)];
                }
                v |= place_block(c, u, NS, X, blk);
            }
            v = ((v ^ ((ent >> 31) ? ~0ull : 0ull)) & c.low_mask) | top;
            if (v < best) {
                best = v;
                bg = ent & 0xFFFFu;
            }
        }
    }
    g_best = bg;
    return best;
}

// The same search in two stages, for groups with many candidates per search.
// Every candidate's top block is MinRep, so the image order is decided first
// by the block landing at position 1.  Stage 1 images only that block for
// every candidate of a Sym list (the per-permutation table pos1 names its
// source block and that block's bit offset in the state) and keeps the
// candidates attaining its minimum in a bit mask; stage 2 assembles the full
// image of those few.  The minimum and the minimiser chosen (the first in
// list order) are those of find_rep_ns.  Lists longer than 32 candidates take
// the one-stage loop.
template <typename AT, int NS, int NC>
__device__ __forceinline__ uint64_t find_rep_staged(const Ctx<AT> &c, uint64_t s, uint32_t &g_best)
{
    static_assert(NS >= 2, "a position-1 block needs two sublattices");
    const int N = c.N, m = c.m, cb = c.cb;
    const int nc = NC > 0 ? NC : c.nc;
    const uint32_t P = c.mmask + 1;
    uint32_t sx[NS];
    uint32_t minr = 0xFFFFFFFFu;
#pragma unroll
    for (int X = 0; X < NS; ++X) {
        sx[X] = (uint32_t)(s >> (N - (X + 1) * m)) & c.mmask;
        minr = min(minr, c.rep[X * P + sx[X]] & 0xFFFFu);
    }
    uint32_t tie = 0;
#pragma unroll
    for (int X = 0; X < NS; ++X) tie |= (uint32_t)((c.rep[X * P + sx[X]] & 0xFFFFu) == minr) << X;
    const uint64_t top = (uint64_t)minr << (N - m);
    constexpr uint32_t kImgMask = ActTraits<AT>::kPos ? (1u << ActTraits<AT>::kPosShift) - 1u : 0xFFFFFFFFu;
    uint64_t best = ~0ull;
    uint32_t bg = 0;
    // full image of candidate entry ent
    auto full_image = [&](uint32_t ent) -> uint64_t {
        const uint32_t u = (ent >> 16) & 0x7FFFu;
        const AT *tu = c.act + ((u * (uint32_t)(NS * nc)) << cb);
        uint64_t v = 0;
#pragma unroll
        for (int X = 0; X < NS; ++X) {
            const AT *t = tu + ((X * nc) << cb);
            uint32_t blk = 0;
            if (NC > 0) {
#pragma unroll
                for (int k2 = 0; k2 < (NC > 0 ? NC : 1); ++k2) blk |= t[(k2 << cb) | ((sx[X] >> (k2 * cb)) & c.cmask)];
            } else {
                for (int k2 = 0; k2 < nc; ++k2) blk |= t[(k2 << cb) | ((sx[X] >> (k2 * cb)) & c.cmask)];
            }
            v |= place_block(c, u, NS, X, blk);
        }
        return ((v ^ ((ent >> 31) ? ~0ull : 0ull)) & c.low_mask) | top;
    };
    while (tie) {
        const int Y = __builtin_ctz(tie);
        tie &= tie - 1;
        const uint32_t sy = (uint32_t)(s >> (N - (Y + 1) * m)) & c.mmask;
        const uint32_t off = c.rep[Y * P + sy] >> 16;
        const uint32_t cnt = c.sym[off];
        if (cnt > 32) {
            for (uint32_t k = 1; k <= cnt; ++k) {
                const uint32_t ent = c.sym[off + k];
                const uint64_t v = full_image(ent);
                if (v < best) {
                    best = v;
                    bg = ent & 0xFFFFu;
                }
            }
            continue;
        }
        // stage 1: the position-1 block of every candidate (two candidates
        // per iteration, so that their dependent LDS reads overlap)
        uint32_t min1 = 0xFFFFFFFFu, keep = 0;
#pragma unroll 2
        for (uint32_t k = 0; k < cnt; ++k) {
            const uint32_t ent = c.sym[off + 1 + k];
            const uint32_t u = (ent >> 16) & 0x7FFFu;
            const uint32_t pw = c.pos1[u];
            const uint32_t sxs = (uint32_t)(s >> (pw >> 8)) & c.mmask;
            const AT *t = c.act + (((u * (uint32_t)NS + (pw & 0xFFu)) * (uint32_t)nc) << cb);
            uint32_t blk = 0;
            if (NC > 0) {
#pragma unroll
                for (int k2 = 0; k2 < (NC > 0 ? NC : 1); ++k2)
                    blk |= t[(k2 << cb) | __builtin_amdgcn_ubfe(sxs, k2 * cb, cb)];
            } else {
                for (int k2 = 0; k2 < nc; ++k2) blk |= t[(k2 << cb) | __builtin_amdgcn_ubfe(sxs, k2 * cb, cb)];
            }
            blk = (blk & kImgMask) ^ ((ent >> 31) ? c.mmask : 0u);
            const uint32_t bit = 1u << k;
            const bool lt = blk < min1, eq = blk == min1;
            keep = lt ? bit : (eq ? (keep | bit) : keep);
            min1 = lt ? blk : min1;
        }
        // stage 2: full images of the survivors, in list order
        while (keep) {
            const int k = __builtin_ctz(keep);
            keep &= keep - 1;
            const uint32_t ent = c.sym[off + 1 + k];
            const uint64_t v = full_image(ent);
            if (v < best) {
                best = v;
                bg = ent & 0xFFFFu;
            }
        }
    }
    g_best = bg;
    return best;
}

// Fermi sign of a group element on an occupation pattern (sec. "Discussion":
// fermions in the occupation-number basis need a sign besides the
// representative).  The element permutes orbitals; the sign is (-1) to the
// number of occupied orbital pairs whose order it reverses.  Sublattice
// stability splits that count: pairs in different source blocks are reversed
// iff their target blocks are (all occupied pairs of the two blocks at once),
// pairs in one chunk come from the parity bit of the chunk's table entry, and
// pairs in two chunks of one block from the chunk images: for the chunks in
// source order, the pairs an image forms with the images of the earlier
// chunks that land below it.  Returns the parity (0 or 1); 4-byte entries
// or the 2-byte fermionic ones.
template <typename AT, int NSC = 0>
__device__ __forceinline__ uint32_t fermi_parity(const Ctx<AT> &c, uint32_t u, uint64_t s)
{
    using Tr = ActTraits<AT>;
    static_assert(sizeof(AT) == 4 || Tr::kParity == 15, "fermionic tables use 4-byte or FermiU16 entries");
    constexpr uint32_t kImg = (1u << Tr::kPosShift) - 1u;
    // sublattice and chunk counts fixed at compile time when NSC gives them
    constexpr int NS_ = (NSC & 127) / 8, NC_ = NSC % 8;
    const int ns = NS_ > 0 ? NS_ : c.ns, nc = NC_ > 0 ? NC_ : c.nc;
    uint32_t par = 0;
    uint64_t seen = 0;   // target blocks of the earlier source blocks with odd occupation
#pragma unroll
    for (int X = 0; X < ns; ++X) {
        const uint32_t sx = (uint32_t)(s >> (c.N - (X + 1) * c.m)) & c.mmask;
        const AT *t = c.act + ((size_t)(u * ns + X) * nc << c.cb);
        uint32_t earlier = 0, pos = 0;
#pragma unroll
        for (int k = nc - 1; k >= 0; --k) {   // chunk nc-1 holds the block's first orbitals
            const uint32_t e = t[(k << c.cb) | ((sx >> (k * c.cb)) & c.cmask)];
            const uint32_t img = e & kImg;
            uint32_t px = earlier;               // px bit j: parity of earlier image bits at or below j
            px ^= px << 1;
            px ^= px << 2;
            px ^= px << 4;
            px ^= px << 8;
            par ^= ((e >> Tr::kParity) & 1u) ^ ((uint32_t)__popc(img & (px << 1)) & 1u);
            earlier |= img;
            if (k == 0) pos = (e >> Tr::kPosShift) & Tr::kPosMask;
        }
        const uint32_t odd = (uint32_t)__popc(sx) & 1u;
        par ^= odd & ((uint32_t)__popcll(seen >> (pos + 1)) & 1u);
        seen |= (uint64_t)odd << pos;
    }
    return par;
}

constexpr int kStagedFlag = 128;   // NSC bit selecting the two-stage search

// NSC = NS * 8 + NC: sublattices and chunks fixed at compile time (0 = read
// them at run time; NC = 0 with NS > 0 fixes only the sublattice count);
// NSC + kStagedFlag selects the two-stage search (2 to 4 sublattices)
// The same choice made at run time (a uniform branch on the staged flag),
// for kernels that would otherwise need twice the template instances;
// STAGED = false leaves the two-stage code out (same results, fewer
// registers).
template <typename AT, int NSC, bool STAGED>
__device__ __forceinline__ uint64_t rep_search_rt(const Ctx<AT> &c, uint64_t s, uint32_t &g)
{
    constexpr int NS = (NSC & 127) / 8, NC = NSC % 8;
    if constexpr (STAGED && NS >= 2 && NS <= 4) {
        if (c.staged) return find_rep_staged<AT, NS, NC>(c, s, g);
    }
    if (NS > 0) return find_rep_ns<AT, (NS > 0 ? NS : 1), NC>(c, s, g);
    uint32_t mv;
    return find_rep(c, s, g, mv);
}

template <typename AT, int NSC>
__device__ __forceinline__ uint64_t rep_search(const Ctx<AT> &c, uint64_t s, uint32_t &g)
{
    constexpr int NS = (NSC & 127) / 8, NC = NSC % 8;
    constexpr bool STAGED = (NSC & kStagedFlag) != 0;
    if constexpr (STAGED) return find_rep_staged<AT, (NS >= 2 && NS <= 4 ? NS : 4), NC>(c, s, g);
    if (NS > 0) return find_rep_ns<AT, (NS > 0 ? NS : 1), NC>(c, s, g);
    uint32_t mv;
    return find_rep(c, s, g, mv);
}

// ---------------------------------------------------------------------------
// index lookups
// ---------------------------------------------------------------------------
// home slot of a state: multiplicative (Fibonacci) hashing, the top log2n
// bits of s * floor(2^64 / golden ratio) (Knuth, TAOCP vol. 3, sec. 6.4).
// One 64-bit multiply; a bit of s changes the product at its position and
// above, so the top bits depend on every state bit.
__device__ __forceinline__ uint64_t slot_of_state(uint64_t s, int log2n)
{
    s *= 0x9e3779b97f4a7c15ull;
    return log2n ? (s >> (64 - log2n)) : 0ull;
}

// Probe sequence of the slot table, the same for every insertion and every
// lookup.  Slots are visited a 128-byte line at a time: from the home slot
// round its own line (8 slots of 16 bytes, or 4 of 32: GLOG2 = 3 or 2), then
// round the next line from the same offset, and so on; every slot comes once
// in 2^slot_log2 steps.  A key whose home slot is taken stays in the home
// line unless that line is full, so a lookup reads one line however far it
// probes inside it (plain linear probing leaves the line whenever the home
// slot is near its end).  Tables hold at least 16 slots.
__device__ __forceinline__ uint64_t next_slot(uint64_t sl, uint64_t home, uint64_t smask, int glog2)
{
    const uint64_t gm = (1ull << glog2) - 1ull;
    uint64_t nx = (sl & ~gm) | ((sl + 1ull) & gm);
    if (((nx ^ home) & gm) == 0) nx = (nx + gm + 1ull) & smask;
    return nx;
}

// first 16 bytes of a slot: {key, x} (real) or {key, -} (complex).  Slot
// reads are random and rarely reused, yet ordinary loads measure faster than
// non-temporal ones: 2.4 % on the 40-site J1-J2 Gamma sector with real
// slots.  A complex slot is two 16-byte reads of one line, and with a
// non-temporal first read the line is often gone when the second arrives
// (1.20 lines per term on the 36-site momentum sector, against 1.08).
template <bool CPLX>
__device__ __forceinline__ ulonglong2 load_slot(const char *slots, uint64_t sl)
{
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2 v = *(const u64x2 *)(slots + (sl << (CPLX ? 5 : 4)));
    return make_ulonglong2(v.x, v.y);
}

// second 16 bytes of a complex slot: the amplitude (re, im)
__device__ __forceinline__ double2 load_slot_value(const char *slots, uint64_t sl)
{
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const f64x2 v = *(const f64x2 *)(slots + (sl << 5) + 16);
    return make_double2(v.x, v.y);
}

// Probe from the home slot (whose first 16 bytes are q) until the target or
// an empty slot; returns 1 and the packed key and amplitude if found.  For
// complex slots v_home is the home slot's amplitude, read together with q
// (HAVE_V) so that a hit on the home slot needs no second, dependent read.
template <bool CPLX, bool HAVE_V = false>
__device__ __forceinline__ int resolve_slot(const DevBasis &db, ulonglong2 q, uint64_t sl, uint64_t target,
                                            uint64_t &key, double &vr, double &vi,
                                            double2 v_home = make_double2(0.0, 0.0))
{
    const uint64_t smask = (1ull << db.slot_log2) - 1ull;
    const uint64_t home_sl = sl;
    bool home = true;
    while (true) {
        if (q.x == kEmpty) return 0;
        if ((q.x & kStateMask) == target) {
            key = q.x;
            if (CPLX) {
                const double2 v = (HAVE_V && home) ? v_home : load_slot_value(db.slots, sl);
                vr = v.x;
                vi = v.y;
            } else {
                vr = __longlong_as_double((long long)q.y);
                vi = 0.0;
            }
            return 1;
        }
        home = false;
        sl = next_slot(sl, home_sl, smask, CPLX ? 2 : 3);
        q = load_slot<CPLX>(db.slots, sl);
    }
}

// the paper's index: Limits(key) -> [begin, end), binary search of the states
template <typename AT>
__device__ __forceinline__ int64_t lookup_limits(const Ctx<AT> &c, const DevBasis &db, uint64_t rep, uint32_t min_val,
                                                 uint64_t &entry)
{
    const uint64_t key = ((uint64_t)c.rank[min_val] << db.key_bits) |
                         ((rep >> db.key_shift) & ((1ull << db.key_bits) - 1ull));
    uint32_t lo = db.limits[key], hi = db.limits[key + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t e = db.states[mid];
        const uint64_t sv = e & kStateMask;
        if (sv == rep) {
            entry = e;
            return (int64_t)mid;
        }
        if (sv < rep) lo = mid + 1; else hi = mid;
    }
    return -1;
}

template <bool CPLX>
struct Scalar;
template <>
struct Scalar<false> {
    using T = double;
};
template <>
struct Scalar<true> {
    using T = double2;
};

struct LzState {
    int j;              // step index
    int done;           // breakdown or finished
    double scale;       // running max(|alpha_k|, beta_k)
    double alpha_cur, beta_cur, beta_prev;
};

template <bool CPLX, typename AT>
__device__ __forceinline__ void chi_of(const Ctx<AT> &c, uint32_t g, double &cr, double &ci)
{
    if (CPLX) {
        cr = c.chi[2 * g];
        ci = c.chi[2 * g + 1];
    } else {
        cr = c.chi[g];
        ci = 0.0;
    }
}


// antiparallel bonds of a row, one bit per bond, in four named words so that
// they stay in registers
struct BondMask {
    uint64_t w0, w1, w2, w3;
};

template <typename AT>
__device__ __forceinline__ uint64_t bond_word(const Ctx<AT> &c, uint64_t s, int w, int nb)
{
    uint64_t am = 0;
    const int bend = min(64, nb - 64 * w);
    for (int k = 0; k < bend; ++k) {
        const uint64_t bm = c.bonds[64 * w + k].mask;
        const uint64_t t = s & bm;
        am |= (uint64_t)((t != 0) & (t != bm)) << k;
    }
    return am;
}

__device__ __forceinline__ int pop_bond(BondMask &m)
{
    if (m.w0) {
        const int k = __builtin_ctzll(m.w0);
        m.w0 &= m.w0 - 1;
        return k;
    }
    if (m.w1) {
        const int k = __builtin_ctzll(m.w1);
        m.w1 &= m.w1 - 1;
        return 64 + k;
    }
    if (m.w2) {
        const int k = __builtin_ctzll(m.w2);
        m.w2 &= m.w2 - 1;
        return 128 + k;
    }
    const int k = __builtin_ctzll(m.w3);
    m.w3 &= m.w3 - 1;
    return 192 + k;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

inline int num_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

inline int lds_limit()
{
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 65536;
    return v;
}

int upload_couplings(const ed_basis *bc, const double *J, const double *Jz, hipStream_t st, double *jsum_quarter);

}  // namespace ed
