// HIP kernels for gfx950 (CDNA4): sector basis build, fused H.v, adjoint and
// Lanczos vector operations.
//
// Data layout in HBM
//   states[D]   uint64: bits [0,56) representative, bits [56,64) index of its
//               stabiliser size among the divisors of |G|.
//   slots       hash-slot index (default): open addressing, line-local probing
//               over 16-byte slots {packed state, x} (complex: 32-byte slots
//               {packed state, -, re, im}) at a low load factor; the input
//               vector is scattered into the slots before each H.v, so that one
//               16-byte read usually returns the index check, the norm and the
//               amplitude of a target together.
//   limits[K+1] uint32: the paper's Limits ranges (index mode 1): begin offset
//               of every key (top-block rank, next q bits), then binary search.
//   x, y[D]     double (or double2), ascending-representative order.
// All lookup tables are staged once per persistent block in LDS.
#include "ed_device.hpp"

#include <mutex>

namespace ed {

// ---------------------------------------------------------------------------
// H.v, gather form of the parallel matrix-vector multiply:
//   y_i = d_i x_i + sum_{b antiparallel} (J_b/2) chi(g) sqrt(n_j/n_i) x_j
// One thread per row, persistent blocks, every y_i written once.  NS encodes
// sublattices * 8 + chunks fixed at compile time (0: read at run time).
// MODE 0: y = H x.  MODE 1: count kept/dropped terms.  MODE 2: Lanczos
// w = H v - beta_prev v_prev with per-block <v, w> partial sums.
// ---------------------------------------------------------------------------

// FERMI: fermions in the occupation-number basis (4-byte or FermiU16 tables, hash
// index): a flip of bond b is the hop -t_b (c+_p c_q + h.c.) with sign
// (-1)^(occupied orbitals between p and q) times the Fermi sign of the
// element mapping the hopped configuration to its representative, and the
// diagonal is sum_b V_b n_p n_q (jhalf = -t_b, jzhalf = V_b).
template <bool CPLX, typename AT, int INDEX, int MODE, int NS, bool FERMI = false>
__global__ void __launch_bounds__(1024) k_apply(DevModel dm, DevBasis db, const typename Scalar<CPLX>::T *__restrict__ x,
                                                typename Scalar<CPLX>::T *__restrict__ y,
                                                const typename Scalar<CPLX>::T *__restrict__ vprev, double *partials,
                                                unsigned long long *stats, const LzState *lz, double jsum_quarter)
{
    extern __shared__ __align__(16) char lds[];
    if (MODE == 2 && lz->done) return;
    const Ctx<AT> c = stage<AT>(dm, lds);
    const int nb = dm.nb;
    const int64_t D = db.dim;
    double acc_part = 0.0;
    unsigned long long kept = 0, dropped = 0;
    const double beta_prev = (MODE == 2) ? lz->beta_prev : 0.0;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // wave-uniform row loop: every lane of a wave runs the same iterations
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < D; i0 += stride) {
        const int64_t i = i0 + lane;
        const bool row_ok = i < D;
        const uint64_t e = row_ok ? db.states[i] : 0ull;
        const uint64_t s = e & kStateMask;
        const double rs_i = c.div_rsqrt[e >> kNormShift];
        // Lanczos step: the row's own v_i and v_prev,i requested before the
        // term loop (in the plain H.v, loading x_i there measured slower)
        typename Scalar<CPLX>::T xi_pf{}, vp_pf{};
        if (MODE == 2 && row_ok) {
            xi_pf = x[i];
            vp_pf = vprev[i];
        }
        double anti_sum = 0.0, ar = 0.0, ai = 0.0;
        // antiparallel bonds of this row
        BondMask am;
        am.w0 = bond_word(c, s, 0, nb);
        am.w1 = nb > 64 ? bond_word(c, s, 1, nb) : 0ull;
        am.w2 = nb > 128 ? bond_word(c, s, 2, nb) : 0ull;
        am.w3 = nb > 192 ? bond_word(c, s, 3, nb) : 0ull;
        const int n_terms = row_ok ? __popcll(am.w0) + __popcll(am.w1) + __popcll(am.w2) + __popcll(am.w3) : 0;
        double fdiag = 0.0;   // fermions: sum_b V_b n_p n_q
        if constexpr (FERMI) {
            for (int k = 0; k < nb; ++k) {
                const uint64_t bm = c.bonds[k].mask;
                if ((s & bm) == bm) fdiag += c.bonds[k].jzhalf;
            }
        }
        if (INDEX == IDX_HASH && MODE != 1) {
            // software pipeline: the slot of the next term is requested before
            // the current term is resolved, so the random read overlaps the
            // next representative search
            uint64_t r_nx = 0, sl_nx = 0;
            uint32_t g_nx = 0;
            double jh_nx = 0.0;
            ulonglong2 q_nx = make_ulonglong2(0ull, 0ull);
            double2 v_nx = make_double2(0.0, 0.0);   // complex: home slot's amplitude
            // fermions: hop sign times the Fermi sign of the element found
            auto fermi_amp = [&](int bi, uint64_t sp, uint32_t g, double jh) -> double {
                if constexpr (FERMI) {
                    const uint32_t par = ((uint32_t)__popcll(s & c.between[bi]) & 1u) ^ fermi_parity<AT, NS>(c, c.g_u[g], sp);
                    return par ? -jh : jh;
                }
                return jh;
            };
            if (n_terms > 0) {
                const int bi = pop_bond(am);
                const BondLds bd = c.bonds[bi];
                anti_sum += bd.jzhalf;
                r_nx = rep_search<AT, NS>(c, s ^ bd.mask, g_nx);
                jh_nx = fermi_amp(bi, s ^ bd.mask, g_nx, bd.jhalf);
                sl_nx = slot_of_state(r_nx, db.slot_log2);
                q_nx = load_slot<CPLX>(db.slots, sl_nx);
                if (CPLX) v_nx = load_slot_value(db.slots, sl_nx);
            }
            for (int term = 0; term < n_terms; ++term) {
                const uint64_t r = r_nx, sl = sl_nx;
                const uint32_t g = g_nx;
                const double jh = jh_nx;
                const ulonglong2 q = q_nx;
                const double2 v = v_nx;
                if (term + 1 < n_terms) {
                    const int bi = pop_bond(am);
                    const BondLds bd = c.bonds[bi];
                    anti_sum += bd.jzhalf;
                    r_nx = rep_search<AT, NS>(c, s ^ bd.mask, g_nx);
                    jh_nx = fermi_amp(bi, s ^ bd.mask, g_nx, bd.jhalf);
                    sl_nx = slot_of_state(r_nx, db.slot_log2);
                    q_nx = load_slot<CPLX>(db.slots, sl_nx);
                    if (CPLX) v_nx = load_slot_value(db.slots, sl_nx);
                }
                uint64_t key;
                double vr, vi;
                if (!resolve_slot<CPLX, true>(db, q, sl, r, key, vr, vi, v)) {
                    ++dropped;
                    continue;
                }
                ++kept;
                double cr, ci;
                chi_of<CPLX>(c, g, cr, ci);
                const double amp = jh * rs_i * c.div_sqrt[key >> kNormShift];
                ar += amp * (cr * vr - ci * vi);
                if (CPLX) ai += amp * (cr * vi + ci * vr);
            }
        } else if (INDEX == IDX_HASH) {
            // term counting
            for (int term = 0; term < n_terms; ++term) {
                const BondLds bd = c.bonds[pop_bond(am)];
                uint32_t g;
                const uint64_t r = rep_search<AT, NS>(c, s ^ bd.mask, g);
                const uint64_t sl = slot_of_state(r, db.slot_log2);
                uint64_t key;
                double vr, vi;
                if (resolve_slot<CPLX>(db, load_slot<CPLX>(db.slots, sl), sl, r, key, vr, vi))
                    ++kept;
                else
                    ++dropped;
            }
        } else {
            for (int term = 0; term < n_terms; ++term) {
                const BondLds bd = c.bonds[pop_bond(am)];
                anti_sum += bd.jzhalf;
                uint32_t g, mval;
                const uint64_t r = find_rep(c, s ^ bd.mask, g, mval);
                uint64_t ej = 0;
                const int64_t j = lookup_limits(c, db, r, mval, ej);
                if (j < 0) {
                    ++dropped;
                    continue;
                }
                ++kept;
                if (MODE == 1) continue;
                double cr, ci;
                chi_of<CPLX>(c, g, cr, ci);
                const double amp = bd.jhalf * rs_i * c.div_sqrt[ej >> kNormShift];
                if (CPLX) {
                    const double2 xv = *(const double2 *)&x[j];
                    ar += amp * (cr * xv.x - ci * xv.y);
                    ai += amp * (cr * xv.y + ci * xv.x);
                } else {
                    ar += amp * cr * *(const double *)&x[j];
                }
            }
        }
        if (MODE == 1 || !row_ok) continue;
        const double d = FERMI ? fdiag : jsum_quarter - anti_sum;
        if (CPLX) {
            const double2 xi = MODE == 2 ? *(const double2 *)&xi_pf : *(const double2 *)&x[i];
            double2 out;
            out.x = d * xi.x + ar;
            out.y = d * xi.y + ai;
            if (MODE == 2) {
                const double2 vp = *(const double2 *)&vp_pf;
                out.x -= beta_prev * vp.x;
                out.y -= beta_prev * vp.y;
                acc_part += xi.x * out.x + xi.y * out.y;   // Re(conj(v) w)
            }
            *(double2 *)&y[i] = out;
        } else {
            const double xi = MODE == 2 ? *(const double *)&xi_pf : *(const double *)&x[i];
            double out = d * xi + ar;
            if (MODE == 2) {
                out -= beta_prev * *(const double *)&vp_pf;
                acc_part += xi * out;
            }
            *(double *)&y[i] = out;
        }
    }
    if (MODE == 1) {
        atomicAdd(&stats[0], kept);
        atomicAdd(&stats[1], dropped);
    }
    if (MODE == 2) {
        // deterministic block reduction in LDS (the tables are no longer needed)
        __syncthreads();
        double *red = (double *)lds;
        red[threadIdx.x] = acc_part;
        __syncthreads();
        for (int o = blockDim.x >> 1; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
    }
}

// x -> value fields of the slot table (hash index); slot_of gives each
// representative's slot
__global__ void k_pack_real(const double *x, const uint32_t *slot_of, char *slots, int64_t D)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x)
        *(double *)(slots + (size_t)slot_of[j] * 16 + 8) = x[j];
}

__global__ void k_pack_cplx(const double2 *x, const uint32_t *slot_of, char *slots, int64_t D)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x)
        *(double2 *)(slots + (size_t)slot_of[j] * 32 + 16) = x[j];
}

// ---------------------------------------------------------------------------
// Adjoint slots at the positions of the H.v slots (same keys, same probe
// sequences): 32 bytes {key, x, gy, -} for a real sector, 64 bytes
// {key, -, x, gy, -} for a complex one (one 128-byte line either way).
// ---------------------------------------------------------------------------

template <bool CPLX>
__global__ void k_adj_slots_keys(const char *slots, char *adj, uint64_t n_slots)
{
    constexpr int kIn = CPLX ? 5 : 4, kOut = CPLX ? 6 : 5;
    for (uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < n_slots;
         sl += (uint64_t)gridDim.x * blockDim.x)
        *(uint64_t *)(adj + (sl << kOut)) = *(const uint64_t *)(slots + (sl << kIn));
}

template <bool CPLX>
__global__ void k_pack_adj(const typename Scalar<CPLX>::T *x, const typename Scalar<CPLX>::T *gy,
                           const uint32_t *slot_of, char *adj, int64_t D)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x) {
        if (CPLX) {
            char *p = adj + ((size_t)slot_of[j] << 6);
            *(double2 *)(p + 16) = *(const double2 *)&x[j];
            *(double2 *)(p + 32) = *(const double2 *)&gy[j];
        } else {
            char *p = adj + ((size_t)slot_of[j] << 5);
            *(double *)(p + 8) = *(const double *)&x[j];
            *(double *)(p + 16) = *(const double *)&gy[j];
        }
    }
}

// probe the adjoint slots from the home slot of target; returns 1 with the
// packed key, x_j and gy_j.  A real slot is one 32-byte vector load, so its
// two 16-byte halves are requested together (loaded as two 16-byte values,
// the compiler waits for the key half before it issues the other).  Complex
// slots read the key first and the amplitudes of the matching slot only.
template <bool CPLX>
__device__ __forceinline__ int resolve_adj(const DevBasis &db, const char *adj, uint64_t sl, uint64_t target,
                                           uint64_t &key, double2 &xv, double2 &gv)
{
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    typedef unsigned long long u64x4 __attribute__((ext_vector_type(4)));
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const uint64_t smask = (1ull << db.slot_log2) - 1ull;
    const uint64_t home = sl;
    while (true) {
        if (CPLX) {
            const char *p = adj + (sl << 6);   // {key, -, x.re, x.im, gy.re, gy.im, -, -}
            const u64x2 q = *(const u64x2 *)p;
            const f64x2 a = *(const f64x2 *)(p + 16);
            const f64x2 b = *(const f64x2 *)(p + 32);
            if (q.x == kEmpty) return 0;
            if ((q.x & kStateMask) == target) {
                key = q.x;
                xv = make_double2(a.x, a.y);
                gv = make_double2(b.x, b.y);
                return 1;
            }
        } else {
            const u64x4 q = *(const u64x4 *)(adj + (sl << 5));   // {key, x, gy, -}
            if (q[0] == kEmpty) return 0;
            if ((q[0] & kStateMask) == target) {
                key = q[0];
                xv = make_double2(__longlong_as_double((long long)q[1]), 0.0);
                gv = make_double2(__longlong_as_double((long long)q[2]), 0.0);
                return 1;
            }
        }
        sl = next_slot(sl, home, smask, CPLX ? 2 : 3);   // the H.v slots' sequence
    }
}

// ---------------------------------------------------------------------------
// Adjoint, bond part: A_b = Re sum_i conj(gy_i) (dH/dJ_b x)_i.  Bonds are
// visited in the same order by every lane so that each bond's contributions
// are summed across the wave in a fixed tree order, then across waves and
// blocks in fixed order: the result is deterministic.
// ---------------------------------------------------------------------------

// FUSED (hash-slot index): the same pass also computes gx = H gy.  Each
// target's x_j and gy_j come from one adjoint slot of adj, so one search and
// one line serve both products; gx_i sums its terms in the order and form of
// k_apply, so it equals ed_apply_H's H gy bit for bit.
template <bool CPLX, typename AT, int INDEX, int NSC, bool FUSED = false>
__global__ void __launch_bounds__(1024) k_backward_J(DevModel dm, DevBasis db, const typename Scalar<CPLX>::T *__restrict__ x,
                                                     const typename Scalar<CPLX>::T *__restrict__ gy,
                                                     double *partials /* [grid][nb + 1] */,
                                                     const char *__restrict__ adj = nullptr, double *__restrict__ gx = nullptr,
                                                     double jsum_quarter = 0.0)
{
    static_assert(!FUSED || INDEX == IDX_HASH, "the fused adjoint reads hash slots");
    // A_b = 1/4 sum_i Re(conj(gy_i) x_i)                      (every bond parallel)
    //     + sum_{i: b antiparallel} [ -1/2 Re(conj(gy_i) x_i) + Re(conj(gy_i) t_b(i)) ]
    // where t_b(i) is the flip term of bond b in row i.  Column nb of the
    // partials carries the bond-independent sum, added on the host.  Wave
    // sums are held by lane b % 64 in registers; blocks reduce in fixed order.
    extern __shared__ __align__(16) char lds[];
    const Ctx<AT> c = stage<AT>(dm, lds);
    const int nb = dm.nb;
    const int nwaves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, tot = 0.0;
    const int64_t D = db.dim;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t wave_first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane;
    for (int64_t i0 = wave_first; i0 < D; i0 += stride) {
        const int64_t i = i0 + lane;
        const bool valid = i < D;
        uint64_t s = 0;
        double rs_i = 0.0, gx_r = 0.0, g_r = 0.0, g_i = 0.0;   // gx_r = Re(conj(gy_i) x_i)
        if (valid) {
            const uint64_t e = db.states[i];
            s = e & kStateMask;
            rs_i = c.div_rsqrt[e >> kNormShift];
            if (CPLX) {
                const double2 gv = *(const double2 *)&gy[i];
                const double2 xv = *(const double2 *)&x[i];
                g_r = gv.x;
                g_i = gv.y;
                gx_r = gv.x * xv.x + gv.y * xv.y;
            } else {
                g_r = *(const double *)&gy[i];
                gx_r = g_r * *(const double *)&x[i];
            }
        }
        tot += wave_sum(gx_r);
        double anti_sum = 0.0, ar = 0.0, ai = 0.0;   // FUSED: diagonal and off-diagonal parts of (H gy)_i
        for (int b = 0; b < nb; ++b) {
            const BondLds bd = c.bonds[b];
            const uint64_t t = s & bd.mask;
            const bool anti = valid && (t != 0) && (t != bd.mask);
            if (!__ballot(anti)) continue;   // no row of this wave flips bond b
            double contrib = 0.0;
            if (anti && FUSED) {
                contrib = -0.5 * gx_r;
                anti_sum += bd.jzhalf;
                uint32_t g;
                const uint64_t r = rep_search<AT, NSC>(c, s ^ bd.mask, g);
                uint64_t key;
                double2 xj, gj;
                if (resolve_adj<CPLX>(db, adj, slot_of_state(r, db.slot_log2), r, key, xj, gj)) {
                    double cr, ci;
                    chi_of<CPLX>(c, g, cr, ci);
                    const double sq = c.div_sqrt[key >> kNormShift];
                    // the per-bond term exactly as the unfused branch forms it
                    const double vr = xj.x, vi = CPLX ? xj.y : 0.0;
                    const double amp = 0.5 * sq * rs_i;
                    const double tr = amp * (cr * vr - ci * vi), ti = amp * (cr * vi + ci * vr);
                    contrib += g_r * tr + g_i * ti;
                    // and the H gy term exactly as k_apply forms it
                    const double wr = gj.x, wi = CPLX ? gj.y : 0.0;
                    const double ampg = bd.jhalf * rs_i * c.div_sqrt[key >> kNormShift];
                    ar += ampg * (cr * wr - ci * wi);
                    if (CPLX) ai += ampg * (cr * wi + ci * wr);
                }
            } else if (anti) {
                contrib = -0.5 * gx_r;
                uint32_t g, mval = 0;
                uint64_t r;
                if (INDEX == IDX_HASH)
                    r = rep_search<AT, NSC>(c, s ^ bd.mask, g);
                else
                    r = find_rep(c, s ^ bd.mask, g, mval);
                double cr, ci;
                chi_of<CPLX>(c, g, cr, ci);
                bool found = false;
                double sq = 0.0, vr = 0.0, vi = 0.0;
                if (INDEX == IDX_HASH) {
                    const uint64_t sl = slot_of_state(r, db.slot_log2);
                    uint64_t key;
                    if (resolve_slot<CPLX>(db, load_slot<CPLX>(db.slots, sl), sl, r, key, vr, vi)) {
                        found = true;
                        sq = c.div_sqrt[key >> kNormShift];
                    }
                } else {
                    uint64_t ej = 0;
                    const int64_t j = lookup_limits(c, db, r, mval, ej);
                    if (j >= 0) {
                        found = true;
                        sq = c.div_sqrt[ej >> kNormShift];
                        if (CPLX) {
                            const double2 xv = *(const double2 *)&x[j];
                            vr = xv.x;
                            vi = xv.y;
                        } else {
                            vr = *(const double *)&x[j];
                        }
                    }
                }
                if (found) {
                    const double amp = 0.5 * sq * rs_i;
                    const double tr = amp * (cr * vr - ci * vi), ti = amp * (cr * vi + ci * vr);
                    contrib += g_r * tr + g_i * ti;   // Re(conj(gy) t)
                }
            }
            const double wsum = wave_sum(contrib);
            if (lane == (b & (kWave - 1))) {
                const int q = b >> 6;
                if (q == 0) a0 += wsum;
                else if (q == 1) a1 += wsum;
                else if (q == 2) a2 += wsum;
                else a3 += wsum;
            }
        }
        if (FUSED && valid) {
            const double d = jsum_quarter - anti_sum;
            if (CPLX) {
                double2 out;
                out.x = d * g_r + ar;
                out.y = d * g_i + ai;
                *(double2 *)&gx[2 * i] = out;
            } else {
                gx[i] = d * g_r + ar;
            }
        }
    }
    // block reduction in fixed order (the tables are no longer needed)
    __syncthreads();
    double *red = (double *)lds;   // [nwaves][nb + 1]
    const int w1 = nb + 1;
    for (int b = lane; b < nb; b += kWave) {
        const int q = b >> 6;
        red[wave * w1 + b] = q == 0 ? a0 : q == 1 ? a1 : q == 2 ? a2 : a3;
    }
    if (lane == 0) red[wave * w1 + nb] = tot;
    __syncthreads();
    for (int b = threadIdx.x; b < w1; b += blockDim.x) {
        double sum = 0.0;
        for (int w = 0; w < nwaves; ++w) sum += red[w * w1 + b];
        partials[(size_t)blockIdx.x * w1 + b] = sum;
    }
}

__global__ void k_sum_partials_cols(const double *partials, int nrows, int ncols, double *out)
{
    for (int col = blockIdx.x * blockDim.x + threadIdx.x; col < ncols; col += gridDim.x * blockDim.x) {
        double t = 0.0;
        for (int r = 0; r < nrows; ++r) t += partials[(size_t)r * ncols + col];
        out[col] = t;
    }
}

// ---------------------------------------------------------------------------
// Basis build: Alg. "Preparation of the distributed and symmetrized Hilbert
// space" on one device.  Prefixes are the top Pb bits; each thread
// enumerates the postfixes of one prefix with the right popcount in
// ascending order and keeps the representatives compatible with chi.
// Pass 0 counts per prefix, pass 1 writes at the scanned offsets.
// ---------------------------------------------------------------------------
struct BuildParams {
    int Pb, R, n_up;
    uint64_t n_prefix;
};

template <typename AT, bool EMIT>
__global__ void __launch_bounds__(256) k_basis_enum(DevModel dm, BuildParams bp, uint32_t *counts,
                                                    const uint64_t *offsets, uint64_t *out)
{
    extern __shared__ __align__(16) char lds[];
    const Ctx<AT> c = stage<AT>(dm, lds);
    const int N = c.N, m = c.m, ns = c.ns;
    const uint32_t P = c.mmask + 1;
    const int R = bp.R;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < bp.n_prefix;
         p += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t cnt = 0;
        const uint32_t t = (uint32_t)(p >> (bp.Pb - m));
        const int pc = __popcll(p);
        const int r = bp.n_up - pc;
        bool ok = ((c.rep[t] & 0xFFFFu) == t) && r >= 0 && r <= R;
        // blocks entirely inside the prefix must not beat the top block
        for (int X = 1; ok && (X + 1) * m <= bp.Pb; ++X) {
            const uint32_t sx = (uint32_t)(p >> (bp.Pb - (X + 1) * m)) & c.mmask;
            ok = (c.rep[X * P + sx] & 0xFFFFu) >= t;
        }
        uint64_t wpos = EMIT ? offsets[p] : 0;
        if (ok) {
            uint64_t v = (r == 0) ? 0ull : ((1ull << r) - 1ull);
            const uint64_t vend = 1ull << R;
            const uint64_t top = (uint64_t)t << (N - m);
            while (v < vend) {
                const uint64_t sgm = (p << R) | v;
                // quick reject: every block's Rep must be >= the top block
                uint32_t tie = 0;
                bool pass = true;
                for (int X = 0; X < ns; ++X) {
                    const uint32_t sx = (uint32_t)(sgm >> (N - (X + 1) * m)) & c.mmask;
                    const uint32_t rv = c.rep[X * P + sx] & 0xFFFFu;
                    if (rv < t) {
                        pass = false;
                        break;
                    }
                    if (rv == t) tie |= 1u << X;
                }
                if (pass) {
                    bool is_rep = true, compat = true;
                    uint32_t nstab = 0;
                    while (tie && is_rep) {
                        const int Y = __builtin_ctz(tie);
                        tie &= tie - 1;
                        const uint32_t sy = (uint32_t)(sgm >> (N - (Y + 1) * m)) & c.mmask;
                        const uint32_t off = c.rep[Y * P + sy] >> 16;
                        const uint32_t n_g = c.sym[off];
                        for (uint32_t k = 1; k <= n_g; ++k) {
                            const uint32_t ent = c.sym[off + k];
                            const uint32_t g = ent & 0xFFFFu;
                            const uint64_t img = image_below_top(c, (ent >> 16) & 0x7FFFu, ent >> 31, Y, sgm) | top;
                            if (img < sgm) {
                                is_rep = false;
                                break;
                            }
                            if (img == sgm) {
                                ++nstab;
                                // the symmetrised state survives iff chi(g) equals the action's
                                // sign on the stabiliser: 1 for spins, the Fermi sign for fermions
                                double sign = 1.0;
                                if constexpr (sizeof(AT) == 4 || ActTraits<AT>::kParity == 15) {
                                    if (dm.fermion && fermi_parity(c, (ent >> 16) & 0x7FFFu, sgm)) sign = -1.0;
                                }
                                if (!dm.trivial_irrep || sign < 0.0) {
                                    double cr, ci;
                                    if (dm.is_complex) {
                                        cr = c.chi[2 * g];
                                        ci = c.chi[2 * g + 1];
                                    } else {
                                        cr = c.chi[g];
                                        ci = 0.0;
                                    }
                                    if (fabs(cr - sign) > 1e-9 || fabs(ci) > 1e-9) compat = false;
                                }
                            }
                        }
                    }
                    if (is_rep && compat) {
                        if (EMIT) {
                            int lo = 0, hi = dm.n_div - 1;
                            while (lo < hi) {
                                const int mid = (lo + hi) >> 1;
                                if (c.div_val[mid] < nstab) lo = mid + 1; else hi = mid;
                            }
                            out[wpos++] = ((uint64_t)lo << kNormShift) | sgm;
                        }
                        ++cnt;
                    }
                }
                if (v == 0) break;
                // next larger integer with the same popcount
                const uint64_t tt = v | (v - 1);
                v = (tt + 1) | (((~tt & (0ull - ~tt)) - 1) >> (__builtin_ctzll(v) + 1));
            }
        }
        if (!EMIT) counts[p] = cnt;
    }
}

// Multi-level exclusive scan of uint32 counts into uint64 offsets.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename TIn>
__global__ void __launch_bounds__(kScanThreads) k_scan_tile(const TIn *in, uint64_t *out, uint64_t n, uint64_t *tile_sums)
{
    __shared__ uint64_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t loc[kScanItems];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint64_t idx = base + k;
        const uint64_t v = idx < n ? (uint64_t)in[idx] : 0ull;
        loc[k] = run;
        run += v;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t excl = sh[threadIdx.x] - run;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint64_t idx = base + k;
        if (idx < n) out[idx] = loc[k] + excl;
    }
    if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void k_scan_add(uint64_t *out, uint64_t n, const uint64_t *tile_offsets)
{
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (uint64_t)gridDim.x * blockDim.x)
        out[idx] += tile_offsets[idx / kScanTile];
}

// Limits: begin offset of every key = lower bound of its smallest state.
__global__ void k_limits(const uint64_t *states, int64_t D, const uint16_t *top_vals, int N, int m, int q,
                         int key_shift, uint64_t n_keys, uint32_t *limits)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= n_keys;
         k += (uint64_t)gridDim.x * blockDim.x) {
        if (k == n_keys) {
            limits[k] = (uint32_t)D;
            continue;
        }
        const uint64_t rank = k >> q, low = k & ((1ull << q) - 1ull);
        const uint64_t lb = ((uint64_t)top_vals[rank] << (N - m)) | (low << key_shift);
        int64_t lo = 0, hi = D;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((states[mid] & kStateMask) < lb) lo = mid + 1; else hi = mid;
        }
        limits[k] = (uint32_t)lo;
    }
}

// slot table: clear, then insert every representative along its probe sequence
__global__ void k_slots_clear(uint64_t *slots_u64, uint64_t n_u64)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_u64; k += (uint64_t)gridDim.x * blockDim.x)
        slots_u64[k] = kEmpty;
}

__global__ void k_slots_insert(const uint64_t *states, int64_t D, char *slots, int log2n, int slot_bytes,
                               uint32_t *slot_of, unsigned int *overflow)
{
    const uint64_t smask = (1ull << log2n) - 1ull;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = states[j];
        const uint64_t home = slot_of_state(key & kStateMask, log2n);
        const int glog2 = slot_bytes == 32 ? 2 : 3;   // slots per 128-byte line
        uint64_t sl = home;
        bool done = false;
        for (uint64_t probe = 0; probe <= smask; ++probe) {
            unsigned long long *kp = (unsigned long long *)(slots + sl * (uint64_t)slot_bytes);
            const unsigned long long old = atomicCAS(kp, (unsigned long long)kEmpty, (unsigned long long)key);
            if (old == kEmpty) {
                slot_of[j] = (uint32_t)sl;
                done = true;
                break;
            }
            sl = next_slot(sl, home, smask, glog2);
        }
        if (!done) atomicAdd(overflow, 1u);
    }
}

__global__ void k_unpack_states(const uint64_t *packed, uint64_t *out, int64_t D)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = packed[i] & kStateMask;
}

// ---------------------------------------------------------------------------
// Lanczos vector kernels (FP64, deterministic two-stage reductions)
// ---------------------------------------------------------------------------
constexpr int kVecThreads = 256;

__device__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += sh[w];
    return t;   // valid in thread 0
}

__global__ void __launch_bounds__(kVecThreads) k_norm2_partial(const double *v, int64_t n, double *partials)
{
    __shared__ double sh[kVecThreads / kWave];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a += v[i] * v[i];
    const double t = block_sum(a, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// v_out = v_in / sqrt(sum of partials), the sum recomputed in fixed order per block
__global__ void __launch_bounds__(kVecThreads) k_scale_by_norm(const double *vin, double *vout, int64_t n,
                                                                  const double *partials, int np)
{
    __shared__ double inv;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < np; ++k) t += partials[k];
        inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        vout[i] = vin[i] * inv;
}

__global__ void k_lz_alpha(LzState *lz, const double *partials, int np, double *alpha_hist)
{
    if (lz->done) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < np; ++k) t += partials[k];
        lz->alpha_cur = t;
        alpha_hist[lz->j] = t;
    }
}

// w -= alpha v ; partial |w|^2 ; psi += s_j v (second pass).  n counts
// doubles: complex vectors are handled by the same loop since alpha is real.
__global__ void __launch_bounds__(kVecThreads) k_lz_update(double *w, const double *v, int64_t n, double *partials,
                                                              const LzState *lz, double *psi, const double *svec)
{
    __shared__ double sh[kVecThreads / kWave];
    if (lz->done) return;
    const double a = lz->alpha_cur;
    const double sj = psi ? svec[lz->j] : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double vi = v[i];
        const double wi = w[i] - a * vi;
        w[i] = wi;
        acc += wi * wi;
        if (psi) psi[i] += sj * vi;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void k_lz_beta(LzState *lz, const double *partials, int np, double *beta_hist, int n_steps, double tol)
{
    if (lz->done) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < np; ++k) t += partials[k];
        const double b = sqrt(t);
        beta_hist[lz->j] = b;
        lz->beta_cur = b;
        lz->scale = fmax(lz->scale, fmax(fabs(lz->alpha_cur), b));
        lz->j += 1;
        if (b <= tol * lz->scale || lz->j >= n_steps) lz->done = 1;
    }
}

// v_new = w / beta_j, written over the oldest vector
__global__ void __launch_bounds__(kVecThreads) k_lz_normalize(const double *w, double *vnew, int64_t n, const LzState *lz)
{
    if (lz->done) return;
    const double inv = 1.0 / lz->beta_cur;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        vnew[i] = w[i] * inv;
}

__global__ void k_lz_shift_beta(LzState *lz)
{
    if (lz->done) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) lz->beta_prev = lz->beta_cur;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int device_alloc(ed_basis *b, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ED_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    b->allocs.push_back(*p);
    b->device_bytes += (int64_t)bytes;
    return ED_OK;
}


// Pack every table into one blob laid out as the LDS image.
static int upload_tables(ed_basis *b, hipStream_t st)
{
    const Tables &t = b->t;
    DevModel &dm = b->dm;
    const uint32_t P = t.P;
    const int m = t.m, ns = t.ns;
    // Sym lists with a count header; rep entries carry the list offset; each
    // entry carries g, its distinct-permutation index and its flip bit
    if (t.nu > 0x7FFF) return set_error(ED_ERR_UNSUPPORTED, "%d distinct permutations exceed 32767", t.nu);
    std::vector<uint32_t> sym;
    std::vector<uint32_t> rep((size_t)ns * P);
    for (int X = 0; X < ns; ++X) {
        for (uint32_t s = 0; s < P; ++s) {
            const uint32_t k0 = t.sym_off[(size_t)X * (P + 1) + s], k1 = t.sym_off[(size_t)X * (P + 1) + s + 1];
            const size_t off = sym.size();
            if (off > 0xFFFFu) return set_error(ED_ERR_UNSUPPORTED, "Sym_X lists exceed 65535 entries");
            sym.push_back(k1 - k0);
            for (uint32_t k = k0; k < k1; ++k) {
                const uint32_t g = t.sym_list[k];
                sym.push_back(g | ((uint32_t)t.g_u[g] << 16) | (t.flip[g] ? 0x80000000u : 0u));
            }
            rep[(size_t)X * P + s] = (t.rep[(size_t)X * P + s] & 0xFFFFu) | ((uint32_t)off << 16);
        }
    }
    std::vector<uint8_t> shift((size_t)t.nu * ns);
    for (size_t k = 0; k < shift.size(); ++k) shift[k] = (uint8_t)(t.N - (t.u_tgt[k] + 1) * m);
    std::vector<double> chi;
    if (dm.is_complex) {
        chi = b->chi_host;
    } else {
        chi.resize(t.ng);
        for (int g = 0; g < t.ng; ++g) chi[g] = b->chi_host[2 * g];
    }
    std::vector<double> dv;
    for (uint32_t d : b->divs) dv.push_back(std::sqrt((double)d));
    for (uint32_t d : b->divs) dv.push_back(1.0 / std::sqrt((double)d));
    std::vector<uint32_t> dvals(b->divs.begin(), b->divs.end());
    std::vector<BondLds> bz((size_t)std::max(t.nb, 1));
    for (int k = 0; k < t.nb; ++k) {
        const int p = t.bonds[2 * k], q = t.bonds[2 * k + 1];
        bz[k].mask = (1ull << (t.N - 1 - p)) | (1ull << (t.N - 1 - q));
        bz[k].jhalf = 0.0;
        bz[k].jzhalf = 0.0;
    }
    // two-stage search: for every permutation u, the source block landing at
    // position 1 and that block's bit offset in the state
    std::vector<uint16_t> pos1(b->staged ? t.nu : 0, 0);
    for (int u = 0; u < (int)pos1.size(); ++u)
        for (int X = 0; X < ns; ++X)
            if (t.u_tgt[(size_t)u * ns + X] == 1) pos1[u] = (uint16_t)(X | (t.N - (X + 1) * m) << 8);
    // fermions: the orbitals strictly between the two of each bond, and the
    // distinct permutation of every group element
    std::vector<uint64_t> between(b->fermion ? std::max(t.nb, 1) : 0, 0ull);
    for (int k = 0; k < (int)between.size() && k < t.nb; ++k) {
        const int lo = std::min(t.bonds[2 * k], t.bonds[2 * k + 1]), hi = std::max(t.bonds[2 * k], t.bonds[2 * k + 1]);
        for (int i = lo + 1; i < hi; ++i) between[k] |= 1ull << (t.N - 1 - i);
    }
    std::vector<uint16_t> gu(b->fermion ? t.ng : 0);
    for (size_t g = 0; g < gu.size(); ++g) gu[g] = t.g_u[g];
    // fermions: image bit of every single orbital of a block, per permutation
    std::vector<uint8_t> img_bit(b->fermion ? (size_t)t.nu * ns * m : 0);
    for (size_t ux = 0; ux < (b->fermion ? (size_t)t.nu * ns : 0); ++ux)
        for (int j = 0; j < m; ++j) img_bit[ux * m + j] = (uint8_t)__builtin_ctz(t.act[ux * P + (1u << j)]);
    // rank of every top-block value, staged only for the Limits index
    std::vector<uint16_t> rank(b->db.index_mode == IDX_LIMITS ? P : 1, 0);
    if (b->db.index_mode == IDX_LIMITS)
        for (size_t r = 0; r < t.top_vals.size(); ++r) rank[t.top_vals[r]] = (uint16_t)r;

    const int lmax = lds_limit();
    const uint32_t budget = (uint32_t)std::max<int64_t>((int64_t)lmax - 8192 - b->lds_reserve, 0);
    auto layout = [&](int cb, int esz, std::vector<char> *blob) -> uint32_t {
        const int nc = (m + cb - 1) / cb;
        size_t pos = 0;
        auto put = [&](const void *src, size_t bytes) -> uint32_t {
            pos = (pos + 15) & ~(size_t)15;
            const uint32_t off = (uint32_t)pos;
            if (blob) {
                blob->resize(pos + bytes);
                if (bytes && src) memcpy(blob->data() + pos, src, bytes);
            }
            pos += bytes;
            return off;
        };
        dm.off_rep = put(rep.data(), rep.size() * 4);
        dm.off_sym = put(sym.data(), sym.size() * 4);
        dm.off_shift = put(shift.data(), shift.size());
        dm.off_chi = put(chi.data(), chi.size() * 8);
        dm.off_div = put(dv.data(), dv.size() * 8);
        dm.off_divval = put(dvals.data(), dvals.size() * 4);
        dm.off_bonds = put(bz.data(), bz.size() * sizeof(BondLds));
        dm.off_rank = put(rank.data(), rank.size() * 2);
        dm.off_pos1 = put(pos1.data(), pos1.size() * 2);
        dm.off_between = put(between.data(), between.size() * 8);
        dm.off_gu = put(gu.data(), gu.size() * 2);
        // chunked action table [nu][ns][nc][2^cb]; wide entries of chunk 0
        // also carry the target block index
        const size_t ent = (size_t)t.nu * ns * nc << cb;
        const int pos_shift = esz == 2 ? 12 : 16;
        if (blob) {
            std::vector<char> act(ent * esz, 0);
            for (int u = 0; u < t.nu; ++u)
                for (int X = 0; X < ns; ++X)
                    for (int k = 0; k < nc; ++k) {
                        const int width = std::min(cb, m - k * cb);
                        for (uint32_t v = 0; v < (1u << width); ++v) {
                            uint32_t img = t.act[((size_t)u * ns + X) * P + (v << (k * cb))];
                            if (esz > 1 && k == 0) img |= (uint32_t)t.u_tgt[(size_t)u * ns + X] << pos_shift;
                            if (b->fermion) {
                                // orbital pairs of the chunk whose order u reverses: bit a above
                                // bit c of the substate (a is the earlier orbital) landing below
                                const uint8_t *ib = &img_bit[((size_t)u * ns + X) * m + k * cb];
                                uint32_t par = 0;
                                for (int a = 0; a < width; ++a)
                                    for (int c2 = 0; c2 < a; ++c2)
                                        if ((v >> a & 1u) && (v >> c2 & 1u) && ib[a] < ib[c2]) par ^= 1u;
                                img |= par << (esz == 2 ? 15 : 31);
                            }
                            const size_t idx = ((((size_t)u * ns + X) * nc + k) << cb) | v;
                            memcpy(&act[idx * esz], &img, esz);   // little endian: low bytes
                        }
                    }
            dm.off_act = put(act.data(), act.size());
        } else {
            dm.off_act = put(nullptr, ent * esz);
        }
        pos = (pos + 15) & ~(size_t)15;
        if (blob) blob->resize(pos);
        return (uint32_t)pos;
    };
    // Entry widths that can hold an image: 1 byte (m <= 8, no position),
    // 2 bytes (m <= 12) or 4 bytes, the wide ones with the block position.
    // Automatic choice: fewest chunks (fewest lookups per block) that fit the
    // LDS budget, a wide entry if it fits at that chunk count; for a given
    // chunk count the narrowest equal split is the smallest table.
    const int wide = m <= 12 ? 2 : 4;
    // fermionic sign parities live in bit 15 of 2-byte entries (images of up
    // to 12 orbitals, block index below 8 in bits 12-14) or in bit 31 of
    // 4-byte ones; automatic choice: 2 bytes where they fit
    const bool fermi16 = m <= 12 && ns <= 8;
    int want_esz = b->fermion ? (b->tuning.table_entry_bytes == 4 || !fermi16 ? 4 : 2) : b->tuning.table_entry_bytes;
    if (want_esz == 1 && m > 8) want_esz = wide;
    if (want_esz == 2 && m > 12) want_esz = 4;
    int cb = m, esz = want_esz ? want_esz : wide;
    if (b->tuning.chunk_bits > 0) {
        cb = std::min(b->tuning.chunk_bits, m);
        if (!want_esz && layout(cb, esz, nullptr) > budget && m <= 8) esz = 1;
    } else {
        bool found = false;
        for (int nc = 1; nc <= m && !found; ++nc) {
            cb = (m + nc - 1) / nc;
            if (want_esz) {
                esz = want_esz;
                found = layout(cb, esz, nullptr) <= budget;
            } else {
                for (int e : {wide, 1}) {
                    if (e == 1 && m > 8) continue;
                    esz = e;
                    if (layout(cb, esz, nullptr) <= budget) {
                        found = true;
                        break;
                    }
                }
            }
        }
    }
    uint32_t total = layout(cb, esz, nullptr);
    if (total > budget)
        return set_error(ED_ERR_UNSUPPORTED, "lookup tables need %u bytes of LDS (limit %u)", total, budget);
    dm.act_bytes = esz;
    std::vector<char> blob;
    total = layout(cb, esz, &blob);
    dm.chunk_bits = cb;
    dm.n_chunks = (m + cb - 1) / cb;
    dm.lds_total = total;
    void *d = nullptr;
    int rc = device_alloc(b, &d, blob.size());
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(d, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    dm.blob = (const char *)d;
    return ED_OK;
}

// bonds' J/2 and Jz/2 live inside the blob; rewrite them when they change.
// Jz == nullptr means Jz = J (Heisenberg).  *jsum_quarter = sum_b Jz_b / 4,
// the diagonal of a row whose bonds are all parallel.
int upload_couplings(const ed_basis *bc, const double *J, const double *Jz, hipStream_t st, double *jsum_quarter)
{
    ed_basis *b = const_cast<ed_basis *>(bc);
    const Tables &t = b->t;
    if (b->fermion) {
        // fermions: J holds the hoppings t_b, Jz the density couplings V_b
        // (nullptr: 0); the flip term of bond b carries -t_b, the diagonal
        // sum_b V_b n_p n_q
        std::vector<double> key(J, J + t.nb);
        for (int k = 0; k < t.nb; ++k) key.push_back(Jz ? Jz[k] : 0.0);
        *jsum_quarter = 0.0;
        if (b->J_cache == key) return ED_OK;
        std::vector<BondLds> bz((size_t)std::max(t.nb, 1));
        for (int k = 0; k < t.nb; ++k) {
            const int p = t.bonds[2 * k], q = t.bonds[2 * k + 1];
            bz[k].mask = (1ull << (t.N - 1 - p)) | (1ull << (t.N - 1 - q));
            bz[k].jhalf = -J[k];
            bz[k].jzhalf = Jz ? Jz[k] : 0.0;
        }
        char *dst = (char *)b->dm.blob + b->dm.off_bonds;
        HIP_TRY(hipMemcpyAsync(dst, bz.data(), (size_t)t.nb * sizeof(BondLds), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        b->J_cache = key;
        return ED_OK;
    }
    if (!Jz) Jz = J;
    double js = 0.0;
    for (int k = 0; k < t.nb; ++k) js += Jz[k];
    *jsum_quarter = 0.25 * js;
    std::vector<double> key(J, J + t.nb);
    key.insert(key.end(), Jz, Jz + t.nb);
    if (b->J_cache == key) return ED_OK;
    std::vector<BondLds> bz((size_t)std::max(t.nb, 1));
    for (int k = 0; k < t.nb; ++k) {
        const int p = t.bonds[2 * k], q = t.bonds[2 * k + 1];
        bz[k].mask = (1ull << (t.N - 1 - p)) | (1ull << (t.N - 1 - q));
        bz[k].jhalf = 0.5 * J[k];
        bz[k].jzhalf = 0.5 * Jz[k];
    }
    char *dst = (char *)b->dm.blob + b->dm.off_bonds;
    HIP_TRY(hipMemcpyAsync(dst, bz.data(), (size_t)t.nb * sizeof(BondLds), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    b->J_cache = key;
    return ED_OK;
}

int check_couplings(const ed_basis *b, const double *J)
{
    const Tables &t = b->t;
    if (t.nb > 0 && !J) return set_error(ED_ERR_ARG, "null couplings");
    std::vector<double> first(t.nb, 0.0);
    std::vector<int> seen(t.nb, 0);
    for (int k = 0; k < t.nb; ++k) {
        if (!std::isfinite(J[k])) return set_error(ED_ERR_ARG, "J[%d] is not finite", k);
        const int o = t.bond_orbit[k];
        if (!seen[o]) {
            seen[o] = 1;
            first[o] = J[k];
        } else if (std::fabs(J[k] - first[o]) > 1e-12 * std::max(1.0, std::fabs(first[o]))) {
            return set_error(ED_ERR_NONINVARIANT_H,
                             "J is not constant on the orbit of bond %d (%.17g vs %.17g); "
                             "average it over the orbit first",
                             k, J[k], first[o]);
        }
    }
    return ED_OK;
}

template <typename Kern>
static void launch_cfg(const ed_basis *b, Kern kern, size_t lds, int *grid, int *threads)
{
    // one 1024-thread block per CU when the tables take most of the LDS
    const int th = b->tuning.block_threads > 0 ? b->tuning.block_threads
                                               : ((int)b->dm.lds_total * 2 > lds_limit() ? 1024 : 512);
    *threads = th;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, th, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    if (b->tuning.blocks_per_cu > 0) per_cu = std::min(per_cu, b->tuning.blocks_per_cu);
    const int64_t need = (b->db.dim + th - 1) / th;
    int64_t g = (int64_t)per_cu * num_cus();
    if (g > need) g = need;
    if (g < 1) g = 1;
    *grid = (int)g;
}

// ---- basis build ---------------------------------------------------------

template <typename AT>
static int build_impl(ed_basis *b, hipStream_t st)
{
    Tables &t = b->t;
    DevModel &dm = b->dm;
    const int N = t.N, m = t.m;
    BuildParams bp{};
    int R = std::min(std::max(N - 20, 8), 16);
    R = std::max(R, N - 28);
    if (R > N - m) R = N - m;
    if (R < 0) R = 0;
    bp.R = R;
    bp.Pb = N - R;
    bp.n_up = b->n_up;
    bp.n_prefix = 1ull << bp.Pb;
    const uint64_t np = bp.n_prefix;
    uint32_t *counts = nullptr;
    uint64_t *offsets = nullptr;
    if (hipMalloc((void **)&counts, np * 4) != hipSuccess || hipMalloc((void **)&offsets, np * 8) != hipSuccess) {
        (void)hipGetLastError();
        if (counts) (void)hipFree(counts);
        return set_error(ED_ERR_OOM, "prefix arrays of %llu entries", (unsigned long long)np);
    }
    auto cleanup = [&]() {
        (void)hipFree(counts);
        (void)hipFree(offsets);
    };
    const int threads = 256;
    const size_t lds = dm.lds_total;
    int per_cu = 1;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_basis_enum<AT, false>, threads, lds);
    per_cu = std::max(per_cu, 1);
    const uint64_t grid = std::min<uint64_t>((np + threads - 1) / threads, (uint64_t)per_cu * num_cus() * 8);
    hipLaunchKernelGGL((k_basis_enum<AT, false>), dim3((unsigned)grid), dim3(threads), lds, st, dm, bp, counts,
                       (const uint64_t *)nullptr, (uint64_t *)nullptr);
    if (hipGetLastError() != hipSuccess) {
        cleanup();
        return set_error(ED_ERR_HIP, "basis count launch failed");
    }
    {
        std::vector<std::pair<uint64_t *, uint64_t>> levels;
        uint64_t n = np;
        const void *in = counts;
        bool in32 = true;
        uint64_t *outp = offsets;
        std::vector<void *> tmp;
        int rc = ED_OK;
        while (true) {
            const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
            uint64_t *sums = nullptr;
            if (hipMalloc((void **)&sums, std::max<uint64_t>(tiles, 1) * 8) != hipSuccess) {
                rc = set_error(ED_ERR_OOM, "scan scratch");
                break;
            }
            tmp.push_back(sums);
            if (in32)
                hipLaunchKernelGGL(k_scan_tile<uint32_t>, dim3((unsigned)tiles), dim3(kScanThreads), 0, st,
                                   (const uint32_t *)in, outp, n, sums);
            else
                hipLaunchKernelGGL(k_scan_tile<uint64_t>, dim3((unsigned)tiles), dim3(kScanThreads), 0, st,
                                   (const uint64_t *)in, outp, n, sums);
            levels.push_back({outp, n});
            if (tiles == 1) break;
            uint64_t *next_out = nullptr;
            if (hipMalloc((void **)&next_out, tiles * 8) != hipSuccess) {
                rc = set_error(ED_ERR_OOM, "scan scratch");
                break;
            }
            tmp.push_back(next_out);
            in = sums;
            in32 = false;
            outp = next_out;
            n = tiles;
        }
        for (int lv = (int)levels.size() - 2; rc == ED_OK && lv >= 0; --lv) {
            const uint64_t nn = levels[lv].second;
            const unsigned g = (unsigned)std::min<uint64_t>((nn + 255) / 256, 65536);
            hipLaunchKernelGGL(k_scan_add, dim3(g), dim3(256), 0, st, levels[lv].first, nn,
                               (const uint64_t *)levels[lv + 1].first);
        }
        uint64_t last_off = 0;
        uint32_t last_cnt = 0;
        if (rc == ED_OK) {
            if (hipMemcpyAsync(&last_off, offsets + np - 1, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(&last_cnt, counts + np - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = set_error(ED_ERR_HIP, "basis count readback failed");
        }
        for (void *p : tmp) (void)hipFree(p);
        if (rc) {
            cleanup();
            return rc;
        }
        b->db.dim = (int64_t)(last_off + last_cnt);
    }
    const int64_t D = b->db.dim;
    if (D >= (int64_t)0xFFFFFFFFll) {
        cleanup();
        return set_error(ED_ERR_UNSUPPORTED, "sector dimension %lld exceeds 32-bit indices", (long long)D);
    }
    void *states = nullptr;
    int rc = device_alloc(b, &states, (size_t)std::max<int64_t>(D, 1) * 8);
    if (rc) {
        cleanup();
        return rc;
    }
    hipLaunchKernelGGL((k_basis_enum<AT, true>), dim3((unsigned)grid), dim3(threads), lds, st, dm, bp,
                       (uint32_t *)nullptr, (const uint64_t *)offsets, (uint64_t *)states);
    if (hipGetLastError() != hipSuccess) {
        cleanup();
        return set_error(ED_ERR_HIP, "basis emit launch failed");
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        cleanup();
        return set_error(ED_ERR_HIP, "basis emit failed: %s", hipGetErrorString(hipGetLastError()));
    }
    cleanup();
    b->db.states = (const uint64_t *)states;

    if (b->db.index_mode == IDX_LIMITS) {
        // Limits over (top-block rank, next q bits)
        const int n_top = (int)t.top_vals.size();
        int q = b->tuning.limits_bits;
        const int avail = N - m;
        if (q <= 0) {
            const double target = std::max(1.0, (double)D / 4.0 / std::max(1, n_top));
            q = std::max((int)std::ceil(std::log2(target)), 0);
            while (q > 0 && ((uint64_t)n_top << q) > (1ull << 28)) --q;
        }
        q = std::min(q, avail);
        b->db.key_bits = q;
        b->db.key_shift = N - m - q;
        b->db.n_keys = (int64_t)n_top << q;
        void *tv = nullptr, *lim = nullptr;
        rc = device_alloc(b, &tv, t.top_vals.size() * 2);
        if (!rc) rc = device_alloc(b, &lim, ((size_t)b->db.n_keys + 1) * 4);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(tv, t.top_vals.data(), t.top_vals.size() * 2, hipMemcpyHostToDevice, st));
        const unsigned g = (unsigned)std::min<uint64_t>(((uint64_t)b->db.n_keys + 256) / 256, 1u << 20);
        hipLaunchKernelGGL(k_limits, dim3(g), dim3(256), 0, st, (const uint64_t *)states, D, (const uint16_t *)tv, N, m,
                           q, b->db.key_shift, (uint64_t)b->db.n_keys, (uint32_t *)lim);
        b->db.limits = (const uint32_t *)lim;
    } else {
        // slot table: power-of-two slots, load factor at most hash_load_pct
        const int slot_bytes = dm.is_complex ? 32 : 16;
        const int pct = b->tuning.hash_load_pct > 0 ? std::min(std::max(b->tuning.hash_load_pct, 10), 90) : 30;
        const double need = std::max(2.0, (double)D * 100.0 / pct);
        const int lg = std::max((int)std::ceil(std::log2(need)), 4);   // whole lines of slots
        if (lg > 32) return set_error(ED_ERR_UNSUPPORTED, "slot table exceeds 32-bit slot indices");
        b->db.slot_log2 = lg;
        b->n_slots = (int64_t)1 << lg;
        void *slots = nullptr, *slot_of = nullptr, *ovf = nullptr;
        const size_t sbytes = (size_t)slot_bytes << lg;
        rc = device_alloc(b, &slots, sbytes);
        if (!rc) rc = device_alloc(b, &slot_of, (size_t)std::max<int64_t>(D, 1) * 4);
        if (!rc) rc = device_alloc(b, &ovf, 16);
        if (rc) return rc;
        HIP_TRY(hipMemsetAsync(ovf, 0, 16, st));
        const uint64_t nu64 = sbytes / 8;
        hipLaunchKernelGGL(k_slots_clear, dim3((unsigned)std::min<uint64_t>((nu64 + 255) / 256, 1u << 20)), dim3(256), 0,
                           st, (uint64_t *)slots, nu64);
        if (D > 0)
            hipLaunchKernelGGL(k_slots_insert, dim3((unsigned)std::min<int64_t>((D + 255) / 256, 1 << 20)), dim3(256), 0,
                               st, (const uint64_t *)states, D, (char *)slots, lg, slot_bytes, (uint32_t *)slot_of,
                               (unsigned int *)ovf);
        unsigned int h_ovf = 0;
        HIP_TRY(hipMemcpyAsync(&h_ovf, ovf, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h_ovf) return set_error(ED_ERR_HIP, "slot table insertion failed for %u states", h_ovf);
        b->db.slots = (char *)slots;
        b->db.slot_of = (const uint32_t *)slot_of;
    }
    if (hipStreamSynchronize(st) != hipSuccess)
        return set_error(ED_ERR_HIP, "basis build failed: %s", hipGetErrorString(hipGetLastError()));
    return ED_OK;
}

int launch_basis_build(ed_basis *b, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    b->db.index_mode = b->tuning.index_mode == 1 ? IDX_LIMITS : IDX_HASH;
    int rc = upload_tables(b, st);
    if (rc) return rc;
    if (b->dm.act_bytes == 1) return build_impl<uint8_t>(b, st);
    if (b->dm.act_bytes == 2) return b->fermion ? build_impl<FermiU16>(b, st) : build_impl<uint16_t>(b, st);
    return build_impl<uint32_t>(b, st);
}

// ---- H.v -----------------------------------------------------------------

static int pack_input(const ed_basis *b, const void *x, hipStream_t st)
{
    if (b->db.index_mode != IDX_HASH || b->db.dim == 0) return ED_OK;
    const int64_t D = b->db.dim;
    const unsigned g = (unsigned)std::min<int64_t>((D + 255) / 256, (int64_t)num_cus() * 16);
    if (b->dm.is_complex)
        hipLaunchKernelGGL(k_pack_cplx, dim3(g), dim3(256), 0, st, (const double2 *)x, b->db.slot_of, b->db.slots, D);
    else
        hipLaunchKernelGGL(k_pack_real, dim3(g), dim3(256), 0, st, (const double *)x, b->db.slot_of, b->db.slots, D);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "pack launch failed: %s", hipGetErrorString(e));
    return ED_OK;
}

template <bool CPLX, typename AT, int INDEX, int MODE, int NS, bool FERMI = false>
static int apply_impl(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                      unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st)
{
    using T = typename Scalar<CPLX>::T;
    auto kern = k_apply<CPLX, AT, INDEX, MODE, NS, FERMI>;
    int grid, threads;
    size_t lds = b->dm.lds_total;
    launch_cfg(b, kern, lds, &grid, &threads);
    if (MODE == 2) {
        lds = std::max(lds, (size_t)threads * 8);
        grid = b->grid_blocks;   // fixed grid so the reductions are deterministic
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, b->dm, b->db, (const T *)x, (T *)y, (const T *)vprev,
                       partials, stats, lz, jsq);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "H.v launch failed: %s", hipGetErrorString(e));
    return ED_OK;
}

template <int MODE, bool CPLX, typename AT>
static int apply_ns(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                    unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st)
{
#define ED_NS(K) \
    case K: return apply_impl<CPLX, AT, IDX_HASH, MODE, K * 8>(b, x, y, vprev, partials, stats, lz, jsq, st);
    if (b->staged) {
        constexpr int F = kStagedFlag;
        if (b->dm.ns == 4 && b->dm.n_chunks == 1)
            return apply_impl<CPLX, AT, IDX_HASH, MODE, 33 + F>(b, x, y, vprev, partials, stats, lz, jsq, st);
        if (b->dm.ns == 4 && b->dm.n_chunks == 2)
            return apply_impl<CPLX, AT, IDX_HASH, MODE, 34 + F>(b, x, y, vprev, partials, stats, lz, jsq, st);
        if (b->dm.ns == 4 && b->dm.n_chunks == 3)
            return apply_impl<CPLX, AT, IDX_HASH, MODE, 35 + F>(b, x, y, vprev, partials, stats, lz, jsq, st);
        if (MODE != 1) {
            if (b->dm.ns == 2) return apply_impl<CPLX, AT, IDX_HASH, MODE, 16 + F>(b, x, y, vprev, partials, stats, lz, jsq, st);
            if (b->dm.ns == 3) return apply_impl<CPLX, AT, IDX_HASH, MODE, 24 + F>(b, x, y, vprev, partials, stats, lz, jsq, st);
            if (b->dm.ns == 4) return apply_impl<CPLX, AT, IDX_HASH, MODE, 32 + F>(b, x, y, vprev, partials, stats, lz, jsq, st);
        }
    }
    // four sublattices with one to three chunks: chunk count fixed too
    if (b->dm.ns == 4 && b->dm.n_chunks == 1)
        return apply_impl<CPLX, AT, IDX_HASH, MODE, 33>(b, x, y, vprev, partials, stats, lz, jsq, st);
    if (b->dm.ns == 4 && b->dm.n_chunks == 2)
        return apply_impl<CPLX, AT, IDX_HASH, MODE, 34>(b, x, y, vprev, partials, stats, lz, jsq, st);
    if (b->dm.ns == 4 && b->dm.n_chunks == 3)
        return apply_impl<CPLX, AT, IDX_HASH, MODE, 35>(b, x, y, vprev, partials, stats, lz, jsq, st);
    if (MODE != 1) {
        switch (b->dm.ns) {
            ED_NS(2) ED_NS(3) ED_NS(4) ED_NS(5) ED_NS(6) ED_NS(8) ED_NS(9) ED_NS(10)
        default: break;
        }
    }
#undef ED_NS
    return apply_impl<CPLX, AT, IDX_HASH, MODE, 0>(b, x, y, vprev, partials, stats, lz, jsq, st);
}

template <int MODE, typename AT>
static int apply_dispatch_t(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                            unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st)
{
    const bool c = b->dm.is_complex;
    if (b->db.index_mode == IDX_LIMITS) {
        if (c) return apply_impl<true, AT, IDX_LIMITS, MODE, 0>(b, x, y, vprev, partials, stats, lz, jsq, st);
        return apply_impl<false, AT, IDX_LIMITS, MODE, 0>(b, x, y, vprev, partials, stats, lz, jsq, st);
    }
    if (c) return apply_ns<MODE, true, AT>(b, x, y, vprev, partials, stats, lz, jsq, st);
    return apply_ns<MODE, false, AT>(b, x, y, vprev, partials, stats, lz, jsq, st);
}

// fermions: four sublattices with two or three chunks fix both counts at
// compile time; other shapes read them at run time
template <int MODE, typename AT>
static int apply_fermi(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                       unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st)
{
    const bool c = b->dm.is_complex;
    if (b->dm.ns == 4 && b->dm.n_chunks == 3)
        return c ? apply_impl<true, AT, IDX_HASH, MODE, 35, true>(b, x, y, vprev, partials, stats, lz, jsq, st)
                 : apply_impl<false, AT, IDX_HASH, MODE, 35, true>(b, x, y, vprev, partials, stats, lz, jsq, st);
    if (b->dm.ns == 4 && b->dm.n_chunks == 2)
        return c ? apply_impl<true, AT, IDX_HASH, MODE, 34, true>(b, x, y, vprev, partials, stats, lz, jsq, st)
                 : apply_impl<false, AT, IDX_HASH, MODE, 34, true>(b, x, y, vprev, partials, stats, lz, jsq, st);
    return c ? apply_impl<true, AT, IDX_HASH, MODE, 0, true>(b, x, y, vprev, partials, stats, lz, jsq, st)
             : apply_impl<false, AT, IDX_HASH, MODE, 0, true>(b, x, y, vprev, partials, stats, lz, jsq, st);
}

template <int MODE>
static int apply_dispatch(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                          unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st)
{
    if (b->fermion) {   // 2- or 4-byte tables, hash index, one-stage search
        if (b->dm.act_bytes == 2) return apply_fermi<MODE, FermiU16>(b, x, y, vprev, partials, stats, lz, jsq, st);
        return apply_fermi<MODE, uint32_t>(b, x, y, vprev, partials, stats, lz, jsq, st);
    }
    if (b->dm.act_bytes == 1) return apply_dispatch_t<MODE, uint8_t>(b, x, y, vprev, partials, stats, lz, jsq, st);
    if (b->dm.act_bytes == 2) return apply_dispatch_t<MODE, uint16_t>(b, x, y, vprev, partials, stats, lz, jsq, st);
    return apply_dispatch_t<MODE, uint32_t>(b, x, y, vprev, partials, stats, lz, jsq, st);
}

int launch_apply(const ed_basis *b, const double *J, const double *Jz, const void *x, void *y, void *stream,
                 int stats_mode, unsigned long long *stats_dev)
{
    hipStream_t st = (hipStream_t)stream;
    if (stats_mode) {
        if (b->db.dim == 0) return ED_OK;
        return apply_dispatch<1>(b, nullptr, nullptr, nullptr, nullptr, stats_dev, nullptr, 0.0, st);
    }
    int rc = check_couplings(b, J);
    if (!rc && Jz) rc = check_couplings(b, Jz);
    if (rc) return rc;
    double jsq = 0.0;
    rc = upload_couplings(b, J, Jz, st, &jsq);
    if (rc) return rc;
    if (b->db.dim == 0) return ED_OK;
    rc = pack_input(b, x, st);
    if (rc) return rc;
    return apply_dispatch<0>(b, x, y, nullptr, nullptr, nullptr, nullptr, jsq, st);
}

// ed_apply_H repeated reps times, with HIP events on the stream around the
// amplitude scatter and around the H.v kernel of every launch
int launch_apply_timed(const ed_basis *b, const double *J, const double *Jz, const void *x, void *y, int reps,
                       double *pack_ms, double *kernel_ms, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = check_couplings(b, J);
    if (!rc && Jz) rc = check_couplings(b, Jz);
    if (rc) return rc;
    double jsq = 0.0;
    rc = upload_couplings(b, J, Jz, st, &jsq);
    if (rc) return rc;
    *pack_ms = 0.0;
    *kernel_ms = 0.0;
    if (b->db.dim == 0) return ED_OK;
    std::vector<hipEvent_t> ev((size_t)reps * 3, nullptr);
    auto destroy = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            destroy();
            return set_error(ED_ERR_HIP, "event creation failed");
        }
    for (int r = 0; r < reps && rc == ED_OK; ++r) {
        if (hipEventRecord(ev[3 * r], st) != hipSuccess) rc = set_error(ED_ERR_HIP, "event record failed");
        if (!rc) rc = pack_input(b, x, st);
        if (!rc && hipEventRecord(ev[3 * r + 1], st) != hipSuccess) rc = set_error(ED_ERR_HIP, "event record failed");
        if (!rc) rc = apply_dispatch<0>(b, x, y, nullptr, nullptr, nullptr, nullptr, jsq, st);
        if (!rc && hipEventRecord(ev[3 * r + 2], st) != hipSuccess) rc = set_error(ED_ERR_HIP, "event record failed");
    }
    if (!rc && hipStreamSynchronize(st) != hipSuccess)
        rc = set_error(ED_ERR_HIP, "timed H.v failed: %s", hipGetErrorString(hipGetLastError()));
    for (int r = 0; r < reps && rc == ED_OK; ++r) {
        float a = 0.f, k = 0.f;
        if (hipEventElapsedTime(&a, ev[3 * r], ev[3 * r + 1]) != hipSuccess ||
            hipEventElapsedTime(&k, ev[3 * r + 1], ev[3 * r + 2]) != hipSuccess)
            rc = set_error(ED_ERR_HIP, "event timing failed");
        *pack_ms += a;
        *kernel_ms += k;
    }
    destroy();
    if (rc) return rc;
    *pack_ms /= reps;
    *kernel_ms /= reps;
    return ED_OK;
}

// ---- adjoint ---------------------------------------------------------------

// Scratch of the allocation-free adjoint entry point: the per-block partial
// sums [grid][nb + 1] of the per-bond adjoint and their column sums [nb + 1].
// Each device holds its own copy; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (scratch_on_device).
constexpr size_t kScratchDoubles = (size_t)1 << 19;   // 4 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices];

// device address of the current device's scratch array, resolved once per
// device with that device current
static int scratch_on_device(double **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(ED_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(ED_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return ED_OK;
}

// per-bond adjoint sums; the partial sums live in scratch_dev when it is
// given (at most kScratchDoubles doubles), else in buffers allocated here
template <bool CPLX, typename AT, int INDEX, int NSC, bool FUSED = false>
static int backward_impl(const ed_basis *b, const void *x, const void *gy, double *gJ_host, double *scratch_dev,
                         hipStream_t st, void *gx = nullptr, double jsq = 0.0)
{
    using T = typename Scalar<CPLX>::T;
    auto kern = k_backward_J<CPLX, AT, INDEX, NSC, FUSED>;
    const int nb = b->t.nb;
    int grid, threads;
    launch_cfg(b, kern, b->dm.lds_total, &grid, &threads);
    // the block reduction reuses the table area: [waves][nb + 1] doubles
    const size_t lds = std::max((size_t)b->dm.lds_total, (size_t)(threads / kWave) * (nb + 1) * 8);
    const size_t n_part = (size_t)grid * (nb + 1);
    double *partials = nullptr, *out = nullptr;
    if (scratch_dev) {
        if (n_part + (size_t)(nb + 1) > kScratchDoubles)
            return set_error(ED_ERR_UNSUPPORTED, "adjoint partials of %zu doubles exceed the %zu-double scratch array",
                             n_part + (size_t)(nb + 1), kScratchDoubles);
        partials = scratch_dev;
        out = scratch_dev + n_part;
    } else if (hipMalloc((void **)&partials, n_part * 8) != hipSuccess ||
               hipMalloc((void **)&out, (size_t)(nb + 1) * 8) != hipSuccess) {
        (void)hipGetLastError();
        if (partials) (void)hipFree(partials);
        return set_error(ED_ERR_OOM, "adjoint partials");
    }
    // every block writes its whole row of partials and every column sum is
    // written, so nothing has to start at zero
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, b->dm, b->db, (const T *)x, (const T *)gy, partials,
                       (const char *)b->adj_slots, (double *)gx, jsq);
    hipLaunchKernelGGL(k_sum_partials_cols, dim3((nb + 256) / 256), dim3(256), 0, st, (const double *)partials, grid,
                       nb + 1, out);
    double h[kMaxBondWords * 64 + 1];
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, out, (size_t)(nb + 1) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (!scratch_dev) {
        (void)hipFree(partials);
        (void)hipFree(out);
    }
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "adjoint failed: %s", hipGetErrorString(e));
    for (int k = 0; k < nb; ++k) gJ_host[k] = h[k] + 0.25 * h[nb];
    return ED_OK;
}

bool backward_fusable(const ed_basis *b)
{
    return b->db.index_mode == IDX_HASH && !b->fermion;
}

// adjoint slots, made once per basis: keys copied from the H.v slots
static int ensure_adj_slots(const ed_basis *bc, hipStream_t st)
{
    ed_basis *b = const_cast<ed_basis *>(bc);
    if (b->adj_slots) return ED_OK;
    const bool c = b->dm.is_complex;
    void *p = nullptr;
    int rc = device_alloc(b, &p, (size_t)b->n_slots * (c ? 64 : 32));
    if (rc) return rc;
    const uint64_t n = (uint64_t)b->n_slots;
    const dim3 grid((unsigned)std::min<uint64_t>((n + 255) / 256, 1u << 20));
    if (c)
        hipLaunchKernelGGL(k_adj_slots_keys<true>, grid, dim3(256), 0, st, (const char *)b->db.slots, (char *)p, n);
    else
        hipLaunchKernelGGL(k_adj_slots_keys<false>, grid, dim3(256), 0, st, (const char *)b->db.slots, (char *)p, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "adjoint slot setup failed: %s", hipGetErrorString(e));
    b->adj_slots = (char *)p;
    return ED_OK;
}

int launch_backward_J(const ed_basis *b, const double *J, const void *x, const void *gy, double *gJ_host, void *stream,
                      bool static_scratch, void *gx)
{
    hipStream_t st = (hipStream_t)stream;
    if (gx && (static_scratch || !backward_fusable(b))) return set_error(ED_ERR_ARG, "no fused adjoint for this basis");
    int rc = check_couplings(b, J);
    if (rc) return rc;
    double jsq;
    rc = upload_couplings(b, J, nullptr, st, &jsq);
    if (rc) return rc;
    if (b->db.dim == 0) {
        for (int k = 0; k < b->t.nb; ++k) gJ_host[k] = 0.0;
        return ED_OK;
    }
    if (b->t.nb == 0) {
        for (int k = 0; k < b->t.nb; ++k) gJ_host[k] = 0.0;
        // no bonds: H gy is the constant diagonal
        if (gx) return launch_apply(b, J, nullptr, gy, gx, stream, 0, nullptr);
        return ED_OK;
    }
    double *scratch_dev = nullptr;
    if (static_scratch) {
        rc = scratch_on_device(&scratch_dev);
        if (rc) return rc;
    }
    const bool c = b->dm.is_complex;
    const int ix = b->db.index_mode, w = b->dm.act_bytes;
    // four sublattices with one to three chunks: search loops fixed at compile time
    const int nsc = (ix == IDX_HASH && b->dm.ns == 4 && b->dm.n_chunks <= 3) ? 32 + b->dm.n_chunks : 0;
    if (gx) {
        // x and gy scattered into the 32-byte adjoint slots; one pass for gJ and gx
        rc = ensure_adj_slots(b, st);
        if (rc) return rc;
        const int64_t D = b->db.dim;
        const dim3 pgrid((unsigned)std::min<int64_t>((D + 255) / 256, 1 << 20));
        if (c)
            hipLaunchKernelGGL(k_pack_adj<true>, pgrid, dim3(256), 0, st, (const double2 *)x, (const double2 *)gy,
                               b->db.slot_of, b->adj_slots, D);
        else
            hipLaunchKernelGGL(k_pack_adj<false>, pgrid, dim3(256), 0, st, (const double *)x, (const double *)gy,
                               b->db.slot_of, b->adj_slots, D);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return set_error(ED_ERR_HIP, "adjoint pack failed: %s", hipGetErrorString(e));
#define ED_FCASE(C, A, K) \
    if (c == C && w == (int)sizeof(A) && nsc == K) \
        return backward_impl<C, A, IDX_HASH, K, true>(b, x, gy, gJ_host, nullptr, st, gx, jsq);
#define ED_FCASES(C, A) ED_FCASE(C, A, 0) ED_FCASE(C, A, 33) ED_FCASE(C, A, 34) ED_FCASE(C, A, 35)
        ED_FCASES(false, uint8_t)
        ED_FCASES(false, uint16_t)
        ED_FCASES(false, uint32_t)
        ED_FCASES(true, uint8_t)
        ED_FCASES(true, uint16_t)
        ED_FCASES(true, uint32_t)
#undef ED_FCASES
#undef ED_FCASE
        return set_error(ED_ERR_ARG, "no kernel variant");
    }
    rc = pack_input(b, x, st);
    if (rc) return rc;
#define ED_CASE(C, A, I, K) \
    if (c == C && w == (int)sizeof(A) && ix == I && nsc == K) \
        return backward_impl<C, A, I, K>(b, x, gy, gJ_host, scratch_dev, st);
#define ED_CASES(C, A) \
    ED_CASE(C, A, IDX_HASH, 0) ED_CASE(C, A, IDX_HASH, 33) ED_CASE(C, A, IDX_HASH, 34) ED_CASE(C, A, IDX_HASH, 35) \
    ED_CASE(C, A, IDX_LIMITS, 0)
    ED_CASES(false, uint8_t)
    ED_CASES(false, uint16_t)
    ED_CASES(false, uint32_t)
    ED_CASES(true, uint8_t)
    ED_CASES(true, uint16_t)
    ED_CASES(true, uint32_t)
#undef ED_CASES
#undef ED_CASE
    return set_error(ED_ERR_ARG, "no kernel variant");
}

// ---- Lanczos ---------------------------------------------------------------

void free_lanczos_workspace(ed_basis *b)
{
    auto &W = b->lzw;
    for (auto &p : W.vec) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    for (double **p : {&W.partials, &W.ahist, &W.bhist, &W.svec}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    if (W.state) (void)hipFree(W.state);
    W.state = nullptr;
    W.cap_steps = 0;
    W.cap_partials = 0;
}

int run_lanczos(const ed_basis *bc, const double *J, const double *Jz, const void *v0, int n_steps, double *alpha,
                double *beta, int *n_done, void *psi0, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(bc);
    hipStream_t st = (hipStream_t)stream;
    int rc = check_couplings(b, J);
    if (!rc && Jz) rc = check_couplings(b, Jz);
    if (rc) return rc;
    double jsq;
    rc = upload_couplings(b, J, Jz, st, &jsq);
    if (rc) return rc;
    const int64_t D = b->db.dim;
    *n_done = 0;
    if (D == 0 || n_steps <= 0) return ED_OK;
    const bool cplx = b->dm.is_complex;
    const int64_t nd = cplx ? 2 * D : D;   // doubles per vector
    {
        int grid, threads;
        launch_cfg(b, k_apply<false, uint8_t, IDX_HASH, 2, 0>, b->dm.lds_total, &grid, &threads);
        b->grid_blocks = grid;   // fixed launch geometry -> deterministic reductions
    }
    const int vgrid = (int)std::min<int64_t>((nd + kVecThreads - 1) / kVecThreads, (int64_t)num_cus() * 8);
    const int np_apply = b->grid_blocks;
    const size_t vb = (size_t)nd * 8;
    auto &W = b->lzw;
    const size_t npart = (size_t)std::max(np_apply, vgrid);
    // the vectors are sized by the basis and kept between calls; only the
    // coefficient histories grow with n_steps
    if (!W.vec[0] || W.cap_partials < npart) {
        free_lanczos_workspace(b);
        bool ok = true;
        for (int k = 0; k < 3; ++k) ok = ok && hipMalloc((void **)&W.vec[k], vb) == hipSuccess;
        ok = ok && hipMalloc((void **)&W.partials, npart * 8) == hipSuccess;
        ok = ok && hipMalloc(&W.state, sizeof(LzState)) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            free_lanczos_workspace(b);
            return set_error(ED_ERR_OOM, "Lanczos vectors (3 x %zu bytes)", vb);
        }
        W.cap_partials = npart;
    }
    if (W.cap_steps < n_steps) {
        for (double **p : {&W.ahist, &W.bhist, &W.svec}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        bool ok = true;
        for (double **p : {&W.ahist, &W.bhist, &W.svec}) ok = ok && hipMalloc((void **)p, (size_t)n_steps * 8) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            free_lanczos_workspace(b);
            return set_error(ED_ERR_OOM, "Lanczos coefficient history");
        }
        W.cap_steps = n_steps;
    }
    double *A = W.vec[0], *B = W.vec[1], *C = W.vec[2], *partials = W.partials, *ahist = W.ahist, *bhist = W.bhist,
           *svec = W.svec;
    LzState *lz = (LzState *)W.state;
    std::vector<double> svec_host(n_steps, 0.0);
    const int passes = psi0 ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
        double *psi = pass == 1 ? (double *)psi0 : nullptr;
        LzState init{};
        HIP_TRY(hipMemcpyAsync(lz, &init, sizeof init, hipMemcpyHostToDevice, st));
        if (psi) {
            HIP_TRY(hipMemsetAsync(psi, 0, vb, st));
            HIP_TRY(hipMemcpyAsync(svec, svec_host.data(), (size_t)n_steps * 8, hipMemcpyHostToDevice, st));
        }
        // v (B) = v0 / |v0| ; v_prev (A) = 0
        HIP_TRY(hipMemsetAsync(A, 0, vb, st));
        hipLaunchKernelGGL(k_norm2_partial, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)v0, nd, partials);
        hipLaunchKernelGGL(k_scale_by_norm, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)v0, B, nd,
                           (const double *)partials, vgrid);
        // one step: pack v into the slots, w = H v - beta v_prev with <v, w>
        // partials, alpha, w -= alpha v (and psi += s_j v), beta, v_prev <-
        // w / beta.  Every quantity that changes between steps lives on the
        // device (the step index in lz), so the step can be captured once per
        // buffer assignment and replayed.
        auto step_kernels = [&](double *vprev_, double *v_, hipStream_t s_) -> int {
            int r = pack_input(b, v_, s_);
            if (r) return r;
            r = apply_dispatch<2>(b, v_, C, vprev_, partials, nullptr, lz, jsq, s_);
            if (r) return r;
            hipLaunchKernelGGL(k_lz_alpha, dim3(1), dim3(64), 0, s_, lz, (const double *)partials, np_apply, ahist);
            hipLaunchKernelGGL(k_lz_update, dim3(vgrid), dim3(kVecThreads), 0, s_, C, (const double *)v_, nd, partials,
                               (const LzState *)lz, psi, (const double *)svec);
            hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(64), 0, s_, lz, (const double *)partials, vgrid, bhist,
                               n_steps, 1e-12);
            hipLaunchKernelGGL(k_lz_normalize, dim3(vgrid), dim3(kVecThreads), 0, s_, (const double *)C, vprev_, nd,
                               (const LzState *)lz);
            hipLaunchKernelGGL(k_lz_shift_beta, dim3(1), dim3(64), 0, s_, lz);
            const hipError_t e = hipGetLastError();
            return e == hipSuccess ? ED_OK : set_error(ED_ERR_HIP, "Lanczos step launch: %s", hipGetErrorString(e));
        };
        // the buffer roles alternate: (v_prev, v) = (A, B), then (B, A)
        const bool use_graph = !b->tuning.lanczos_direct;
        hipGraphExec_t exec[2] = {nullptr, nullptr};
        hipStream_t cap = nullptr;
        auto release = [&]() {
            for (auto &x : exec)
                if (x) (void)hipGraphExecDestroy(x);
            if (cap) (void)hipStreamDestroy(cap);
            exec[0] = exec[1] = nullptr;
            cap = nullptr;
        };
        if (use_graph) {
            if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                return set_error(ED_ERR_HIP, "capture stream");
            }
            for (int p = 0; p < 2; ++p) {
                hipGraph_t graph = nullptr;
                if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    (void)hipGetLastError();
                    release();
                    return set_error(ED_ERR_HIP, "begin capture");
                }
                rc = step_kernels(p == 0 ? A : B, p == 0 ? B : A, cap);
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
                rc = step_kernels(p == 0 ? A : B, p == 0 ? B : A, st);
                if (rc) return rc;
            }
            if ((step & 15) == 15) {
                LzState hs;
                if (hipMemcpyAsync(&hs, lz, sizeof hs, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess) {
                    release();
                    return set_error(ED_ERR_HIP, "Lanczos state readback");
                }
                if (hs.done) break;
            }
        }
        if (use_graph) {
            // the replays are ordered on st; the executables may go once they finish
            if (hipStreamSynchronize(st) != hipSuccess) {
                release();
                return set_error(ED_ERR_HIP, "Lanczos replay");
            }
            release();
        }
        LzState hs;
        HIP_TRY(hipMemcpyAsync(&hs, lz, sizeof hs, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(alpha, ahist, (size_t)n_steps * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(beta, bhist, (size_t)n_steps * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *n_done = hs.j;
        if (pass == 0 && psi0) {
            std::vector<double> ev(hs.j), z(hs.j);
            rc = ed_tridiag_eigh(hs.j, alpha, beta, ev.data(), z.data());
            if (rc) return rc;
            for (int k = 0; k < hs.j; ++k) svec_host[k] = z[k];
        }
        if (pass == 1) {
            hipLaunchKernelGGL(k_norm2_partial, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)psi, nd, partials);
            hipLaunchKernelGGL(k_scale_by_norm, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)psi, psi, nd,
                               (const double *)partials, vgrid);
        }
    }
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "Lanczos failed: %s", hipGetErrorString(e));
    return ED_OK;
}

}  // namespace ed

extern "C" int ed_internal_unpack_states(const ed_basis *b, uint64_t *dev_out, void *stream)
{
    const int64_t D = b->db.dim;
    if (D == 0) return ED_OK;
    const unsigned g = (unsigned)std::min<int64_t>((D + 255) / 256, 65536);
    hipLaunchKernelGGL(ed::k_unpack_states, dim3(g), dim3(256), 0, (hipStream_t)stream, b->db.states, dev_out, D);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ed::set_error(ED_ERR_HIP, "unpack launch: %s", hipGetErrorString(e));
    return ED_OK;
}

extern "C" int ed_internal_apply_stats(const ed_basis *b, int64_t *kept, int64_t *dropped, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *d = nullptr;
    if (hipMalloc((void **)&d, 16) != hipSuccess) return ed::set_error(ED_ERR_OOM, "stats buffer");
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(d, h, 16, hipMemcpyHostToDevice, st);
    int rc = ED_OK;
    if (e == hipSuccess && b->db.dim > 0) rc = ed::launch_apply(b, nullptr, nullptr, nullptr, nullptr, stream, 1, d);
    if (e == hipSuccess && rc == ED_OK) e = hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && rc == ED_OK) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (rc) return rc;
    if (e != hipSuccess) return ed::set_error(ED_ERR_HIP, "stats: %s", hipGetErrorString(e));
    *kept = (int64_t)h[0];
    *dropped = (int64_t)h[1];
    return ED_OK;
}
