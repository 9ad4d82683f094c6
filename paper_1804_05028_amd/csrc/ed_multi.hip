// Batched sectors: several 1-D irreps of one group in one launch.
//
// Every sector's representatives are orbit minima of the same group, so the
// representatives of all sectors together are the trivial-irrep basis; sector
// k keeps the rows whose stabiliser carries the trivial value of chi_k (a
// representative with a non-trivial character on its stabiliser has zero
// norm, sec. "Symmetry adapted basis states").  One launch therefore runs the
// representative search (Alg. "Sublattice coding algorithm for finding the
// representative") and the index lookup once per term for all sectors, and
// applies the K characters to the K amplitudes of the target row:
//   y[i][k] = d_i x[i][k] + sum_terms (J_b/2) sqrt(n_j/n_i) chi_k(g) x[j][k]
// for rows i and targets j compatible with sector k; rows incompatible with k
// are written as zero and incompatible entries of x are never read.
//
// Layout: vectors are complex128 [dim][K], sector index fastest, so the K
// amplitudes of a target are one contiguous read.  The slot table's value
// field holds the row index (low 32 bits) and the row's sector mask (high 32
// bits), so one 16-byte probe returns index, norm and compatibility; with
// more than 32 sectors the target's mask is read from the per-row mask array.
#include "ed_device.hpp"

namespace ed {

constexpr int kMaxSectors = 64;
constexpr int kMlzThreads = 256;

struct MultiDev {
    int K;
    const uint64_t *masks;    // [dim]
    const double2 *chi;       // [ng][K] in HBM
    const void *lds_src;      // what is staged at chi_off: chi, or the sign bytes
    uint32_t chi_off;         // LDS byte offset of the staged copy
    uint32_t chi_bytes;       // bytes staged in LDS (0: read chi from HBM)
    int chi_signs;            // staged: [ng] bytes, bit k set iff chi_k(g) = -1
};

// per-sector Lanczos state
struct MlzSector {
    double alpha, beta, beta_prev, scale, inv_beta;
    int done, n_done;
};

struct MlzState {
    int j;          // steps taken
    int n_active;   // sectors still iterating
};

// ---------------------------------------------------------------------------
// Sector masks: bit k of row i is set iff chi_k(g) = 1 for every g in
// Stab(sigma_i).  A representative's stabiliser elements are among the
// candidates of the rep search (each maps a block whose Rep equals the top
// block onto it), so the search loop enumerates them.
// ---------------------------------------------------------------------------
template <typename AT>
__global__ void __launch_bounds__(256) k_multi_masks(DevModel dm, DevBasis db, const uint64_t *triv, uint64_t all,
                                                     int K, uint64_t *masks, unsigned long long *counts)
{
    extern __shared__ __align__(16) char lds[];
    const Ctx<AT> c = stage<AT>(dm, lds);
    unsigned int *cnt = (unsigned int *)(lds + dm.lds_total);
    for (int k = threadIdx.x; k < K; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    const int N = c.N, m = c.m, ns = c.ns;
    const uint32_t P = c.mmask + 1;
    const int64_t D = db.dim;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < D; i0 += stride) {
        const int64_t i = i0 + lane;
        uint64_t mk = 0;
        if (i < D) {
            const uint64_t s = db.states[i] & kStateMask;
            const uint32_t t = (uint32_t)(s >> (N - m));
            const uint64_t top = (uint64_t)t << (N - m);
            mk = all;
            for (int Y = 0; Y < ns; ++Y) {
                const uint32_t sy = (uint32_t)(s >> (N - (Y + 1) * m)) & c.mmask;
                const uint32_t rv = c.rep[Y * P + sy];
                if ((rv & 0xFFFFu) != t) continue;
                const uint32_t off = rv >> 16;
                const uint32_t n_g = c.sym[off];
                for (uint32_t k = 1; k <= n_g; ++k) {
                    const uint32_t ent = c.sym[off + k];
                    const uint64_t img = image_below_top(c, (ent >> 16) & 0x7FFFu, ent >> 31, Y, s) | top;
                    if (img == s) mk &= triv[ent & 0xFFFFu];
                }
            }
            masks[i] = mk;
        }
        for (int k = 0; k < K; ++k) {
            const uint64_t bal = __ballot((mk >> k) & 1ull);
            if (lane == 0) atomicAdd(&cnt[k], (unsigned int)__popcll(bal));
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) atomicAdd(&counts[k], (unsigned long long)cnt[k]);
}

// value field of every slot: row index | sector mask << 32
__global__ void k_multi_pack_index(const uint32_t *slot_of, const uint64_t *masks, char *slots, int64_t D)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x)
        *(uint64_t *)(slots + (size_t)slot_of[j] * 16 + 8) = (uint64_t)j | (masks[j] << 32);
}

// (ar, ai) += amp * chi * xv with the fused multiply-adds written out, so
// that every kernel instance rounds the same way whatever the compiler would
// contract on its own
__device__ __forceinline__ void cmac(double &ar, double &ai, double amp, double2 chi, double2 xv)
{
    ar = fma(amp, fma(chi.x, xv.x, -(chi.y * xv.y)), ar);
    ai = fma(amp, fma(chi.x, xv.y, chi.y * xv.x), ai);
}

// ---------------------------------------------------------------------------
// Batched H.v.  KB is the compile-time bound of the sector loop.  SPLIT lanes
// share a row: each runs the row's searches and probes (same addresses, so
// the requests of a load instruction merge) and owns every SPLIT-th sector
// (lane r: r, r + SPLIT, ...), which divides the per-lane accumulator and
// amplitude registers by SPLIT and raises the number of waves a compute unit
// holds; the lanes of a row read adjacent amplitudes in each instruction.
// MODE 0: y = H x, or w = H v - beta_prev[k] vprev when vprev is given
// (Lanczos; y may be vprev itself: each element is read and then written by
// the same thread).  MODE 1 (SPLIT 1): per-sector term counts (D_k + kept_k)
// in stats[0..K), shared kept terms in stats[K], dropped lookups in
// stats[K+1].
// ---------------------------------------------------------------------------
// threads per block: 512 where a lane holds more than 4 sectors, so that the
// registers of one wave may exceed 128 without spilling
template <int KB, int SPLIT>
constexpr int multi_block_bound()
{
    return KB >= 8 ? 512 : 1024;
}

template <typename AT, int NS, int KB, int MODE, int SPLIT>
__global__ void __launch_bounds__((multi_block_bound<KB, SPLIT>()))
    k_apply_multi(DevModel dm, DevBasis db, MultiDev md, const double2 *__restrict__ x, double2 *y,
                  const double2 *vprev, const MlzSector *__restrict__ sec, double *stats, double jsq)
{
    static_assert(MODE == 0 || SPLIT == 1, "term counting runs one lane per row");
    static_assert(kWave % SPLIT == 0, "lanes per row must divide the wave");
    extern __shared__ __align__(16) char lds[];
    const Ctx<AT> c = stage<AT>(dm, lds);
    double2 *chik = (double2 *)(lds + md.chi_off);
    lds_copy((char *)chik, md.lds_src, md.chi_bytes);
    __syncthreads();
    const int K = md.K;
    const int nb = dm.nb;
    const int64_t D = db.dim;
    const uint64_t smask = (1ull << db.slot_log2) - 1ull;
    const int lane = threadIdx.x & (kWave - 1);
    // the two-stage search is compiled in where registers allow it without
    // spilling; elsewhere the one-stage search gives the same results
    constexpr bool kStagedFits = KB <= 8;
    // the same instances can read a character table kept in HBM
    constexpr bool kChiHbm = kStagedFits;
    // this lane's row within the wave's group of rows, and its sectors
    constexpr int kRows = kWave / SPLIT;
    const int rl = lane / SPLIT;
    // sectors of this lane: koff, koff + SPLIT, ... (KL of them), so that the
    // lanes of a row read neighbouring amplitudes in each load instruction
    const int koff = lane % SPLIT;
    const int KL = koff < K ? (K - koff + SPLIT - 1) / SPLIT : 0;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t n_waves = (int64_t)gridDim.x * blockDim.x / kWave;
    double shared = 0.0, dropped = 0.0;
    double ar[KB], ai[KB];
    if (MODE == 1) {
#pragma unroll
        for (int k = 0; k < KB; ++k) ar[k] = 0.0;
    }
    for (int64_t i0 = wave * kRows; i0 < D; i0 += n_waves * kRows) {
        const int64_t i = i0 + rl;
        const bool row_ok = i < D;
        const uint64_t e = row_ok ? db.states[i] : 0ull;
        const uint64_t mi = row_ok ? md.masks[i] : 0ull;
        const uint64_t s = e & kStateMask;
        const double rs_i = c.div_rsqrt[e >> kNormShift];
        if (MODE == 0) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                ar[k] = 0.0;
                ai[k] = 0.0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < KB; ++k) ar[k] += (double)((mi >> k) & 1ull);
        }
        double anti_sum = 0.0;
        BondMask am;
        am.w0 = bond_word(c, s, 0, nb);
        am.w1 = nb > 64 ? bond_word(c, s, 1, nb) : 0ull;
        am.w2 = nb > 128 ? bond_word(c, s, 2, nb) : 0ull;
        am.w3 = nb > 192 ? bond_word(c, s, 3, nb) : 0ull;
        const int n_terms = row_ok ? __popcll(am.w0) + __popcll(am.w1) + __popcll(am.w2) + __popcll(am.w3) : 0;
        // software pipeline: the slot of the next term is requested before
        // the current term is resolved
        uint64_t r_nx = 0, sl_nx = 0;
        uint32_t g_nx = 0;
        double jh_nx = 0.0;
        ulonglong2 q_nx = make_ulonglong2(0ull, 0ull);
        if (n_terms > 0) {
            const BondLds bd = c.bonds[pop_bond(am)];
            anti_sum += bd.jzhalf;
            jh_nx = bd.jhalf;
            r_nx = rep_search_rt<AT, NS, kStagedFits>(c, s ^ bd.mask, g_nx);
            sl_nx = slot_of_state(r_nx, db.slot_log2);
            q_nx = load_slot<false>(db.slots, sl_nx);
        }
        for (int term = 0; term < n_terms; ++term) {
            const uint64_t r = r_nx;
            uint64_t sl = sl_nx;
            const uint64_t sl_home = sl_nx;
            const uint32_t g = g_nx;
            const double jh = jh_nx;
            ulonglong2 q = q_nx;
            while (q.x != kEmpty && (q.x & kStateMask) != r) {
                sl = next_slot(sl, sl_home, smask, 3);
                q = load_slot<false>(db.slots, sl);
            }
            const bool found = q.x != kEmpty;
            // bit koff + SPLIT k: local sector k
            const uint64_t mj = K > 32 ? (found ? md.masks[q.y & 0xFFFFFFFFull] : 0ull) : (q.y >> 32);
            const uint64_t mij = found ? (mi & mj) : 0ull;
            // the target's amplitudes are requested before the next term's
            // search, which hides their latency
            // registers allow holding the next row's amplitudes (split rows
            // trade the prefetch for more resident waves, except for 4 sectors)
            constexpr bool kPre = KB <= 16 && (SPLIT == 1 || KB <= 4);
            double2 xv[kPre ? KB : 1];
            if (MODE == 0 && kPre) {
                const double2 *xj = x + (size_t)(q.y & 0xFFFFFFFFull) * K + koff;
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    xv[k] = (k < KL && ((mij >> (koff + SPLIT * k)) & 1ull)) ? xj[SPLIT * k] : make_double2(0.0, 0.0);
            }
            if (term + 1 < n_terms) {
                const BondLds bd = c.bonds[pop_bond(am)];
                anti_sum += bd.jzhalf;
                jh_nx = bd.jhalf;
                r_nx = rep_search_rt<AT, NS, kStagedFits>(c, s ^ bd.mask, g_nx);
                sl_nx = slot_of_state(r_nx, db.slot_log2);
                q_nx = load_slot<false>(db.slots, sl_nx);
            }
            if (!found) {
                dropped += 1.0;
                continue;
            }
            if (MODE == 1) {
                shared += 1.0;
#pragma unroll
                for (int k = 0; k < KB; ++k) ar[k] += (double)((mij >> k) & 1ull);
                continue;
            }
            const double amp = jh * rs_i * c.div_sqrt[q.x >> kNormShift];
            auto accumulate = [&](const double2 *ch) {
                if (kPre) {
#pragma unroll
                    for (int k = 0; k < (kPre ? KB : 1); ++k) {
                        if (k < KL) cmac(ar[k], ai[k], amp, ch[SPLIT * k], xv[k]);
                    }
                } else {
                    const double2 *xj = x + (size_t)(q.y & 0xFFFFFFFFull) * K + koff;
#pragma unroll
                    for (int k = 0; k < KB; ++k) {
                        if (k < KL && ((mij >> (koff + SPLIT * k)) & 1ull)) cmac(ar[k], ai[k], amp, ch[SPLIT * k], xj[SPLIT * k]);
                    }
                }
            };
            // characters +-1: (ar, ai) += (+-amp) x, the value the complex
            // product gives for chi = (+-1, 0)
            auto accumulate_signs = [&](uint32_t sg) {
                if (kPre) {
#pragma unroll
                    for (int k = 0; k < (kPre ? KB : 1); ++k) {
                        if (k < KL) {
                            const double a = ((sg >> (koff + SPLIT * k)) & 1u) ? -amp : amp;
                            ar[k] = fma(a, xv[k].x, ar[k]);
                            ai[k] = fma(a, xv[k].y, ai[k]);
                        }
                    }
                } else {
                    const double2 *xj = x + (size_t)(q.y & 0xFFFFFFFFull) * K + koff;
#pragma unroll
                    for (int k = 0; k < KB; ++k) {
                        if (k < KL && ((mij >> (koff + SPLIT * k)) & 1ull)) {
                            const double a = ((sg >> (koff + SPLIT * k)) & 1u) ? -amp : amp;
                            const double2 xx = xj[SPLIT * k];
                            ar[k] = fma(a, xx.x, ar[k]);
                            ai[k] = fma(a, xx.y, ai[k]);
                        }
                    }
                }
            };
            // characters chi_k(g) of this lane's sectors: the LDS copy, their
            // sign bits in LDS, or HBM; the last two in the instances with
            // registers for a second accumulate path
            if (kChiHbm && md.chi_signs)
                accumulate_signs(((const uint8_t *)chik)[g]);
            else if (kChiHbm && md.chi_bytes == 0)
                accumulate(md.chi + (size_t)g * K + koff);
            else
                accumulate(chik + (size_t)g * K + koff);
        }
        if (MODE == 1 || !row_ok) continue;
        const double d = jsq - anti_sum;
        double2 *yi = y + (size_t)i * K + koff;
        const double2 *xi = x + (size_t)i * K + koff;
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if (k < KL) {
                double2 out = make_double2(0.0, 0.0);
                if ((mi >> (koff + SPLIT * k)) & 1ull) {
                    const double2 xv = xi[SPLIT * k];
                    out.x = d * xv.x + ar[k];
                    out.y = d * xv.y + ai[k];
                    if (vprev) {
                        const double bp = sec[koff + SPLIT * k].beta_prev;
                        const double2 vp = vprev[(size_t)i * K + koff + SPLIT * k];
                        out.x -= bp * vp.x;
                        out.y -= bp * vp.y;
                    }
                }
                yi[SPLIT * k] = out;
            }
        }
    }
    if (MODE == 1) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const double v = wave_sum(ar[k]);
            if (k < K && lane == 0) atomicAdd(&stats[k], v);
        }
        const double sh = wave_sum(shared), dr = wave_sum(dropped);
        if (lane == 0) {
            atomicAdd(&stats[K], sh);
            atomicAdd(&stats[K + 1], dr);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched Lanczos vector kernels.  Thread t of a block handles sector
// t % K of rows t / K of each group of R = blockDim / K rows, so it always
// sees one sector; per-(block, sector) sums are formed in a fixed order.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void sector_partials(int64_t D, int K, F f, double *partials)
{
    __shared__ double sh[kMlzThreads];
    const int R = kMlzThreads / K;
    const int t = threadIdx.x;
    const int r = t / K, k = t - r * K;
    double acc = 0.0;
    if (r < R)
        for (int64_t i = (int64_t)blockIdx.x * R + r; i < D; i += (int64_t)gridDim.x * R) acc += f(i, k);
    sh[t] = acc;
    __syncthreads();
    if (t < K) {
        double s = 0.0;
        for (int rr = 0; rr < R; ++rr) s += sh[rr * K + t];
        partials[(size_t)blockIdx.x * K + t] = s;
    }
}

template <typename F>
__device__ __forceinline__ void sector_foreach(int64_t D, int K, F f)
{
    const int R = kMlzThreads / K;
    const int t = threadIdx.x;
    const int r = t / K, k = t - r * K;
    if (r < R)
        for (int64_t i = (int64_t)blockIdx.x * R + r; i < D; i += (int64_t)gridDim.x * R) f(i, k);
}

// |masked v0|^2 per sector
__global__ void __launch_bounds__(kMlzThreads) k_mlz_init_norm(const double2 *v0, const uint64_t *masks, int64_t D,
                                                               int K, double *partials)
{
    sector_partials(
        D, K,
        [&](int64_t i, int k) {
            if (!((masks[i] >> k) & 1ull)) return 0.0;
            const double2 a = v0[(size_t)i * K + k];
            return a.x * a.x + a.y * a.y;
        },
        partials);
}

// Per-sector totals of the per-block partials, by every thread of a block
// of kTotThreads: the G = kTotThreads / K threads of sector k each add the
// blocks r, r + G, ... in order, and thread k then adds their G sums in
// order, so the result is deterministic.  Every thread must call it; the
// totals are valid in threads k < K.
constexpr int kTotThreads = 1024;
__device__ __forceinline__ double sector_total(const double *partials, int nblk, int K)
{
    __shared__ double red[kTotThreads];
    const int t = threadIdx.x;
    const int G = kTotThreads / K;
    const int k = t % K, r = t / K;
    double s = 0.0;
    if (r < G)
        for (int b = r; b < nblk; b += G) s += partials[(size_t)b * K + k];
    red[t] = s;
    __syncthreads();
    double tot = 0.0;
    if (t < K)
        for (int q = 0; q < G; ++q) tot += red[q * K + t];
    __syncthreads();
    return tot;
}

__global__ void __launch_bounds__(kTotThreads) k_mlz_init_finish(const double *partials, int nblk, int K, MlzSector *sec,
                                                                  MlzState *st)
{
    const int k = threadIdx.x;
    int active = 0;
    const double n2 = sector_total(partials, nblk, K);
    if (k < K) {
        MlzSector s{};
        s.done = n2 > 0.0 ? 0 : 1;   // empty sector or zero start vector: nothing to iterate
        s.inv_beta = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
        sec[k] = s;
        active = !s.done;
    }
    const uint64_t bal = __ballot(active);
    if (threadIdx.x == 0) {
        st->j = 0;
        st->n_active = __popcll(bal);
    }
}

// v = masked v0 / |masked v0|, vprev = 0
__global__ void __launch_bounds__(kMlzThreads) k_mlz_init_vec(const double2 *v0, const uint64_t *masks, int64_t D,
                                                              int K, const MlzSector *sec, double2 *v, double2 *vprev)
{
    sector_foreach(D, K, [&](int64_t i, int k) {
        const size_t e = (size_t)i * K + k;
        const double sc = ((masks[i] >> k) & 1ull) ? sec[k].inv_beta : 0.0;
        const double2 a = v0[e];
        v[e] = make_double2(a.x * sc, a.y * sc);
        vprev[e] = make_double2(0.0, 0.0);
    });
}

// alpha_k partials: Re <v_k, w_k>
__global__ void __launch_bounds__(kMlzThreads) k_mlz_dot(const double2 *v, const double2 *w, int64_t D, int K,
                                                         double *partials)
{
    sector_partials(
        D, K,
        [&](int64_t i, int k) {
            const size_t e = (size_t)i * K + k;
            const double2 a = v[e], b = w[e];
            return a.x * b.x + a.y * b.y;
        },
        partials);
}

__global__ void __launch_bounds__(kTotThreads) k_mlz_alpha(const double *partials, int nblk, int K, MlzSector *sec,
                                                            const MlzState *st, double *ahist, int n_steps)
{
    const int k = threadIdx.x;
    const double a = sector_total(partials, nblk, K);
    if (k >= K) return;
    sec[k].alpha = a;
    if (!sec[k].done) ahist[(size_t)k * n_steps + st->j] = a;
}

// w -= alpha_k v_k, and |w_k|^2 partials
__global__ void __launch_bounds__(kMlzThreads) k_mlz_update(double2 *w, const double2 *v, int64_t D, int K,
                                                            const MlzSector *sec, double *partials)
{
    sector_partials(
        D, K,
        [&](int64_t i, int k) {
            const size_t e = (size_t)i * K + k;
            const double a = sec[k].alpha;
            const double2 vv = v[e];
            double2 ww = w[e];
            ww.x -= a * vv.x;
            ww.y -= a * vv.y;
            w[e] = ww;
            return ww.x * ww.x + ww.y * ww.y;
        },
        partials);
}

__global__ void __launch_bounds__(kTotThreads) k_mlz_beta(const double *partials, int nblk, int K, MlzSector *sec,
                                                           MlzState *st, double *bhist, int n_steps, double tol)
{
    const int k = threadIdx.x;
    const int j = st->j;
    int active = 0;
    const double n2 = sector_total(partials, nblk, K);
    if (k < K) {
        MlzSector s = sec[k];
        const double b = sqrt(n2);
        if (!s.done) {
            s.scale = fmax(s.scale, fmax(fabs(s.alpha), b));
            bhist[(size_t)k * n_steps + j] = b;
            s.n_done = j + 1;
            s.beta = b;
            if (b <= tol * s.scale || j + 1 >= n_steps) s.done = 1;
            s.inv_beta = s.done ? 0.0 : 1.0 / b;
            s.beta_prev = b;
        } else {
            s.inv_beta = 0.0;
            s.beta_prev = 0.0;
        }
        sec[k] = s;
        active = !s.done;
    }
    const uint64_t bal = __ballot(active);
    if (threadIdx.x == 0) {
        st->j = j + 1;
        st->n_active = __popcll(bal);
    }
}

// v_next = w / beta_k in place (zero for finished sectors)
__global__ void __launch_bounds__(kMlzThreads) k_mlz_normalize(double2 *w, int64_t D, int K, const MlzSector *sec)
{
    sector_foreach(D, K, [&](int64_t i, int k) {
        const size_t e = (size_t)i * K + k;
        const double sc = sec[k].inv_beta;
        const double2 a = w[e];
        w[e] = make_double2(a.x * sc, a.y * sc);
    });
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int table_width(const ed_basis *b) { return b->dm.act_bytes; }

template <int MODE, typename AT, int NS, int KB, int SPLIT>
static int multi_launch_impl(const ed_multi *mb, const void *x, void *y, const void *vprev, const void *sec,
                             double *stats, double jsq, hipStream_t st)
{
    const ed_basis *b = mb->base;
    auto kern = k_apply_multi<AT, NS, KB, MODE, SPLIT>;
    const int bound = multi_block_bound<KB, SPLIT>();
    int threads = b->tuning.block_threads > 0 ? std::min(b->tuning.block_threads, bound) : bound;
    MultiDev md;
    md.K = mb->K;
    md.masks = mb->masks;
    md.chi = (const double2 *)mb->chi_dev;
    md.chi_off = mb->lds_chi_off;
    md.chi_bytes = mb->chi_in_lds ? (uint32_t)((size_t)b->t.ng * mb->K * 16)
                                  : (mb->chi_signs ? ((uint32_t)b->t.ng + 15u) & ~15u : 0u);
    md.chi_signs = mb->chi_signs ? 1 : 0;
    md.lds_src = mb->chi_signs ? mb->sgn_dev : mb->chi_dev;
    const size_t lds = (size_t)md.chi_off + md.chi_bytes;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (b->tuning.blocks_per_cu > 0) per_cu = std::min(per_cu, b->tuning.blocks_per_cu);
    const int64_t need = (b->db.dim * SPLIT + threads - 1) / threads;
    int64_t grid = std::min<int64_t>((int64_t)per_cu * num_cus(), need);
    grid = std::max<int64_t>(grid, 1);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, st, b->dm, b->db, md, (const double2 *)x,
                       (double2 *)y, (const double2 *)vprev, (const MlzSector *)sec, stats, jsq);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "batched H.v launch failed: %s", hipGetErrorString(e));
    return ED_OK;
}

// lanes per row of the batched H.v: the caller's choice, else 1 lane for up
// to 2 sectors, 2 lanes for up to 8 and 4 lanes above (measured on the
// 36-site triangular momentum sectors: each lane then holds at most 4
// sectors for K <= 16 and prefetches their next amplitudes).  With the
// character table in HBM, 1 lane for up to 8 sectors (measured on the 8
// Gamma irreps of the 36-site triangular group, whose search dominates:
// 47.2 ms against 51.6 ms with 2 lanes); such a table needs an instance
// with the HBM path (see kChiHbm), at most 8 sectors per lane.
int multi_lanes_per_row(const ed_multi *mb)
{
    const int K = mb->K;
    int t = mb->base->tuning.lanes_per_row;
    if (t <= 0) t = (K <= 2 || (!mb->chi_in_lds && K <= 8)) ? 1 : (K <= 8 ? 2 : 4);
    // a character table read from HBM needs an instance with at most 8
    // sectors per lane
    if (!mb->chi_in_lds) t = std::max(t, K <= 8 ? 1 : (K <= 16 ? 2 : 4));
    // more than 32 sectors: 4 lanes of at most 16 sectors each
    if (K > 32) t = 4;
    return t;
}

template <int MODE, typename AT, int NS>
static int multi_launch_kb(const ed_multi *mb, const void *x, void *y, const void *vprev, const void *sec,
                           double *stats, double jsq, hipStream_t st)
{
    const int K = mb->K;
    const int split = MODE == 0 ? multi_lanes_per_row(mb) : 1;
    const int kh = (K + split - 1) / split;   // sectors per lane
#define ED_KB(KB, S) return multi_launch_impl<MODE, AT, NS, KB, (MODE == 0 ? S : 1)>(mb, x, y, vprev, sec, stats, jsq, st)
    if (MODE == 0 && split == 2) {
        if (kh <= 4) ED_KB(4, 2);
        if (kh <= 8) ED_KB(8, 2);
        ED_KB(16, 2);
    }
    if (MODE == 0 && split == 4) {
        if (kh <= 4) ED_KB(4, 4);
        if (kh <= 8) ED_KB(8, 4);
        ED_KB(16, 4);
    }
    if (kh <= 4) ED_KB(4, 1);
    if (kh <= 8) ED_KB(8, 1);
    if (kh <= 16) ED_KB(16, 1);
    if constexpr (MODE == 1) {   // term counts of more than 32 sectors (lanes of 4 run the H.v)
        if (kh > 32) ED_KB(64, 1);
    }
    ED_KB(32, 1);
#undef ED_KB
}

template <int MODE>
static int multi_launch(const ed_multi *mb, const void *x, void *y, const void *vprev, const void *sec, double *stats,
                        double jsq, hipStream_t st)
{
    const ed_basis *b = mb->base;
    // four sublattices with one to three chunks: search loops fixed at compile
    // time (three chunks for 2-byte entries only)
    const int nsc = (MODE == 0 && b->dm.ns == 4 && b->dm.n_chunks <= 3) ? 32 + b->dm.n_chunks : 0;
    if (table_width(b) == 2) {
        if (nsc == 33) return multi_launch_kb<MODE, uint16_t, 33>(mb, x, y, vprev, sec, stats, jsq, st);
        if (nsc == 34) return multi_launch_kb<MODE, uint16_t, 34>(mb, x, y, vprev, sec, stats, jsq, st);
        if (nsc == 35) return multi_launch_kb<MODE, uint16_t, 35>(mb, x, y, vprev, sec, stats, jsq, st);
        return multi_launch_kb<MODE, uint16_t, 0>(mb, x, y, vprev, sec, stats, jsq, st);
    }
    if (table_width(b) == 4) {
        if (nsc == 33) return multi_launch_kb<MODE, uint32_t, 33>(mb, x, y, vprev, sec, stats, jsq, st);
        if (nsc == 34) return multi_launch_kb<MODE, uint32_t, 34>(mb, x, y, vprev, sec, stats, jsq, st);
        return multi_launch_kb<MODE, uint32_t, 0>(mb, x, y, vprev, sec, stats, jsq, st);
    }
    return set_error(ED_ERR_UNSUPPORTED, "batched sectors need 2- or 4-byte action-table entries");
}

template <typename AT>
static void launch_masks(const ed_multi *mb, const uint64_t *triv, uint64_t all, unsigned long long *counts,
                         hipStream_t st)
{
    const ed_basis *b = mb->base;
    const int threads = 256;
    const size_t lds = (size_t)b->dm.lds_total + (size_t)mb->K * 4;
    int per_cu = 1;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_multi_masks<AT>, threads, lds);
    per_cu = std::max(per_cu, 1);
    const int64_t grid =
        std::max<int64_t>(std::min<int64_t>((b->db.dim + threads - 1) / threads, (int64_t)per_cu * num_cus() * 4), 1);
    hipLaunchKernelGGL(k_multi_masks<AT>, dim3((unsigned)grid), dim3(threads), lds, st, b->dm, b->db, triv, all,
                       mb->K, mb->masks, counts);
}

int multi_setup(ed_multi *mb, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    ed_basis *b = mb->base;
    const int K = mb->K, ng = b->t.ng;
    const int64_t D = b->db.dim;
    if (K < 1 || K > kMaxSectors) return set_error(ED_ERR_UNSUPPORTED, "%d sectors (1..%d supported)", K, kMaxSectors);
    if (K > 32 && !mb->chi_in_lds)
        return set_error(ED_ERR_UNSUPPORTED, "more than 32 sectors need their character table (%zu bytes) in LDS",
                         (size_t)ng * K * 16);
    if (b->db.index_mode != 0) return set_error(ED_ERR_ARG, "batched sectors use the hash-slot index");
    // trivial-character masks per element and the character table [ng][K]
    std::vector<uint64_t> triv(ng, 0);
    std::vector<double> chi((size_t)ng * K * 2);
    for (int k = 0; k < K; ++k)
        for (int g = 0; g < ng; ++g) {
            const double re = mb->chi_host[((size_t)k * ng + g) * 2], im = mb->chi_host[((size_t)k * ng + g) * 2 + 1];
            if (std::fabs(re - 1.0) <= 1e-9 && std::fabs(im) <= 1e-9) triv[g] |= 1ull << k;
            chi[((size_t)g * K + k) * 2] = re;
            chi[((size_t)g * K + k) * 2 + 1] = im;
        }
    void *d_triv = nullptr, *d_chi = nullptr, *d_masks = nullptr, *d_cnt = nullptr;
    int rc = device_alloc(b, &d_triv, (size_t)ng * 8);
    if (!rc) rc = device_alloc(b, &d_chi, chi.size() * 8);
    if (!rc) rc = device_alloc(b, &d_masks, (size_t)std::max<int64_t>(D, 1) * 8);
    if (!rc) rc = device_alloc(b, &d_cnt, (size_t)K * 8);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(d_triv, triv.data(), (size_t)ng * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_chi, chi.data(), chi.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(d_cnt, 0, (size_t)K * 8, st));
    mb->chi_dev = d_chi;
    mb->masks = (uint64_t *)d_masks;
    if (mb->chi_signs) {
        // one byte per element: bit k set iff chi_k(g) = -1 (every character is +-1)
        std::vector<uint8_t> sgn(((size_t)ng + 15) & ~(size_t)15, 0);
        for (int g = 0; g < ng; ++g)
            for (int k = 0; k < K; ++k)
                if (chi[((size_t)g * K + k) * 2] < 0.0) sgn[g] |= (uint8_t)(1u << k);
        void *d_sgn = nullptr;
        rc = device_alloc(b, &d_sgn, sgn.size());
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(d_sgn, sgn.data(), sgn.size(), hipMemcpyHostToDevice, st));
        mb->sgn_dev = d_sgn;
    }
    mb->lds_chi_off = (b->dm.lds_total + 15u) & ~15u;
    const uint64_t all = K == 64 ? ~0ull : ((1ull << K) - 1ull);
    if (D > 0) {
        if (b->dm.act_bytes == 2)
            launch_masks<uint16_t>(mb, (const uint64_t *)d_triv, all, (unsigned long long *)d_cnt, st);
        else if (b->dm.act_bytes == 4)
            launch_masks<uint32_t>(mb, (const uint64_t *)d_triv, all, (unsigned long long *)d_cnt, st);
        else
            return set_error(ED_ERR_UNSUPPORTED, "batched sectors need 2- or 4-byte action-table entries");
        HIP_TRY(hipGetLastError());
        const unsigned g = (unsigned)std::min<int64_t>((D + 255) / 256, (int64_t)num_cus() * 16);
        hipLaunchKernelGGL(k_multi_pack_index, dim3(g), dim3(256), 0, st, b->db.slot_of, (const uint64_t *)d_masks,
                           b->db.slots, D);
        HIP_TRY(hipGetLastError());
    }
    std::vector<unsigned long long> cnt(K, 0);
    HIP_TRY(hipMemcpyAsync(cnt.data(), d_cnt, (size_t)K * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    mb->dims.assign(cnt.begin(), cnt.end());
    return ED_OK;
}

int multi_apply(const ed_multi *mb, const double *J, const void *x, void *y, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const ed_basis *b = mb->base;
    int rc = check_couplings(b, J);
    if (rc) return rc;
    double jsq = 0.0;
    rc = upload_couplings(b, J, nullptr, st, &jsq);
    if (rc) return rc;
    if (b->db.dim == 0) return ED_OK;
    return multi_launch<0>(mb, x, y, nullptr, nullptr, nullptr, jsq, st);
}

int multi_stats(const ed_multi *mb, int64_t *terms, int64_t *shared_terms, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const int K = mb->K;
    std::vector<double> h(K + 2, 0.0);
    if (mb->base->db.dim > 0) {
        double *d = nullptr;
        if (hipMalloc((void **)&d, (K + 2) * 8) != hipSuccess) return set_error(ED_ERR_OOM, "stats buffer");
        hipError_t e = hipMemcpyAsync(d, h.data(), (K + 2) * 8, hipMemcpyHostToDevice, st);
        int rc = ED_OK;
        if (e == hipSuccess) rc = multi_launch<1>(mb, nullptr, nullptr, nullptr, nullptr, d, 0.0, st);
        if (e == hipSuccess && rc == ED_OK) e = hipMemcpyAsync(h.data(), d, (K + 2) * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && rc == ED_OK) e = hipStreamSynchronize(st);
        (void)hipFree(d);
        if (rc) return rc;
        if (e != hipSuccess) return set_error(ED_ERR_HIP, "batched stats: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < K; ++k) terms[k] = (int64_t)h[k];
    *shared_terms = (int64_t)h[K];
    if (h[K + 1] != 0.0) return set_error(ED_ERR_HIP, "%.0f targets missing from the shared index", h[K + 1]);
    return ED_OK;
}

void multi_free_workspace(ed_multi *mb)
{
    auto &W = mb->lzw;
    for (auto &p : W.vec) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    for (double **p : {&W.partials, &W.ahist, &W.bhist, &W.sector}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    if (W.state) (void)hipFree(W.state);
    W.state = nullptr;
    W.cap_steps = 0;
    W.cap_partials = 0;
}

// One Lanczos step for all sectors on two vectors: w = H v - beta vprev is
// written over vprev, then alpha, w -= alpha v, beta, and w / beta in place
// becomes the next v (v becomes the next vprev).  Only kernel launches, so
// the sequence can be captured in a graph.
static int mlz_step(const ed_multi *mb, double jsq, const double2 *v, double2 *w, int vgrid, int n_steps,
                    hipStream_t st)
{
    const int K = mb->K;
    const int64_t D = mb->base->db.dim;
    auto &W = mb->lzw;
    MlzSector *sec = (MlzSector *)W.sector;
    MlzState *state = (MlzState *)W.state;
    int rc = multi_launch<0>(mb, v, w, w, sec, nullptr, jsq, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlz_dot, dim3(vgrid), dim3(kMlzThreads), 0, st, v, (const double2 *)w, D, K, W.partials);
    hipLaunchKernelGGL(k_mlz_alpha, dim3(1), dim3(kTotThreads), 0, st, (const double *)W.partials, vgrid, K, sec,
                       (const MlzState *)state, W.ahist, n_steps);
    hipLaunchKernelGGL(k_mlz_update, dim3(vgrid), dim3(kMlzThreads), 0, st, w, v, D, K, (const MlzSector *)sec,
                       W.partials);
    hipLaunchKernelGGL(k_mlz_beta, dim3(1), dim3(kTotThreads), 0, st, (const double *)W.partials, vgrid, K, sec, state, W.bhist,
                       n_steps, 1e-12);
    hipLaunchKernelGGL(k_mlz_normalize, dim3(vgrid), dim3(kMlzThreads), 0, st, w, D, K, (const MlzSector *)sec);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "batched Lanczos launch: %s", hipGetErrorString(e));
    return ED_OK;
}

int multi_lanczos(ed_multi *mb, const double *J, const void *v0, int n_steps, double *alpha, double *beta,
                  int *n_done, int use_graph, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const ed_basis *b = mb->base;
    const int K = mb->K;
    const int64_t D = b->db.dim;
    for (int k = 0; k < K; ++k) n_done[k] = 0;
    int rc = check_couplings(b, J);
    if (rc) return rc;
    double jsq = 0.0;
    rc = upload_couplings(b, J, nullptr, st, &jsq);
    if (rc) return rc;
    if (D == 0 || n_steps <= 0) return ED_OK;
    const int R = kMlzThreads / K;
    const int vgrid = (int)std::max<int64_t>(std::min<int64_t>((D + R - 1) / R, (int64_t)num_cus() * 8), 1);
    auto &W = mb->lzw;
    const size_t vb = (size_t)D * K * 16;
    const size_t npart = (size_t)vgrid * K;
    // vectors are sized by the basis and kept between calls; only the
    // coefficient histories grow with n_steps
    if (!W.vec[0] || W.cap_partials < npart) {
        multi_free_workspace(mb);
        bool ok = true;
        for (int k = 0; k < 2; ++k) ok = ok && hipMalloc(&W.vec[k], vb) == hipSuccess;
        ok = ok && hipMalloc((void **)&W.partials, npart * 8) == hipSuccess;
        ok = ok && hipMalloc((void **)&W.sector, (size_t)K * sizeof(MlzSector)) == hipSuccess;
        ok = ok && hipMalloc(&W.state, sizeof(MlzState)) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            multi_free_workspace(mb);
            return set_error(ED_ERR_OOM, "batched Lanczos vectors (2 x %zu bytes)", vb);
        }
        W.cap_partials = npart;
    }
    if (W.cap_steps < n_steps) {
        for (double **p : {&W.ahist, &W.bhist}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        bool ok = true;
        for (double **p : {&W.ahist, &W.bhist}) ok = ok && hipMalloc((void **)p, (size_t)K * n_steps * 8) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            multi_free_workspace(mb);
            return set_error(ED_ERR_OOM, "batched Lanczos coefficient history");
        }
        W.cap_steps = n_steps;
    }
    double2 *A = (double2 *)W.vec[0], *B = (double2 *)W.vec[1];
    MlzSector *sec = (MlzSector *)W.sector;
    MlzState *state = (MlzState *)W.state;
    HIP_TRY(hipMemsetAsync(W.ahist, 0, (size_t)K * n_steps * 8, st));
    HIP_TRY(hipMemsetAsync(W.bhist, 0, (size_t)K * n_steps * 8, st));
    hipLaunchKernelGGL(k_mlz_init_norm, dim3(vgrid), dim3(kMlzThreads), 0, st, (const double2 *)v0,
                       (const uint64_t *)mb->masks, D, K, W.partials);
    hipLaunchKernelGGL(k_mlz_init_finish, dim3(1), dim3(kTotThreads), 0, st, (const double *)W.partials, vgrid, K, sec, state);
    hipLaunchKernelGGL(k_mlz_init_vec, dim3(vgrid), dim3(kMlzThreads), 0, st, (const double2 *)v0,
                       (const uint64_t *)mb->masks, D, K, (const MlzSector *)sec, B, A);
    HIP_TRY(hipGetLastError());

    // the step alternates between two buffer assignments: (vprev, v) = (A, B)
    // then (B, A)
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipStream_t cap = nullptr;
    auto release = [&]() {
        for (auto &x : exec)
            if (x) (void)hipGraphExecDestroy(x);
        if (cap) (void)hipStreamDestroy(cap);
    };
    if (use_graph) {
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ED_ERR_HIP, "capture stream");
        }
        for (int p = 0; p < 2; ++p) {
            double2 *vp = p == 0 ? A : B, *vv = p == 0 ? B : A;
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                (void)hipGetLastError();
                release();
                return set_error(ED_ERR_HIP, "begin capture");
            }
            rc = mlz_step(mb, jsq, vv, vp, vgrid, n_steps, cap);
            const hipError_t e = hipStreamEndCapture(cap, &graph);
            if (rc || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                release();
                return rc ? rc : set_error(ED_ERR_HIP, "end capture: %s", hipGetErrorString(e));
            }
            const hipError_t ei = hipGraphInstantiate(&exec[p], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                release();
                return set_error(ED_ERR_HIP, "graph instantiate: %s", hipGetErrorString(ei));
            }
        }
    }
    for (int step = 0; step < n_steps; ++step) {
        const int p = step & 1;
        if (use_graph) {
            const hipError_t e = hipGraphLaunch(exec[p], st);
            if (e != hipSuccess) {
                release();
                return set_error(ED_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
            }
        } else {
            double2 *vp = p == 0 ? A : B, *vv = p == 0 ? B : A;
            rc = mlz_step(mb, jsq, vv, vp, vgrid, n_steps, st);
            if (rc) return rc;
        }
        if ((step & 15) == 15) {
            MlzState hs;
            const hipError_t e = hipMemcpyAsync(&hs, state, sizeof hs, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
                release();
                return set_error(ED_ERR_HIP, "batched Lanczos state readback");
            }
            if (hs.n_active == 0) break;
        }
    }
    std::vector<MlzSector> hsec(K);
    hipError_t e = hipMemcpyAsync(hsec.data(), sec, (size_t)K * sizeof(MlzSector), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(alpha, W.ahist, (size_t)K * n_steps * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(beta, W.bhist, (size_t)K * n_steps * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    release();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "batched Lanczos failed: %s", hipGetErrorString(e));
    for (int k = 0; k < K; ++k) n_done[k] = hsec[k].n_done;
    return ED_OK;
}

}  // namespace ed
