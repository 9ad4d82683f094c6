// HIP kernels for gfx950 (CDNA4): sector basis build, fused H.v, adjoint and
// Lanczos vector operations.
//
// Data layout in HBM
//   states[D]   uint64: bits [0,56) representative, bits [56,64) index of its
//               stabiliser size among the divisors of |G| (the norm is read
//               in the same load that confirms the index lookup).
//   limits[K+1] uint32: begin offset of every key (top-block rank, next q bits).
//   x, y[D]     double (or double2 for complex sectors), ascending-rep order.
// Small lookup tables (Rep_X, Sym_X, the symmetry action when it fits, the
// group-element descriptors, characters, bonds) are staged once per
// persistent block in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
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

// ---------------------------------------------------------------------------
// LDS staging
// ---------------------------------------------------------------------------

struct BondLds {
    uint64_t mask;     // both sites of the bond
    double jhalf;      // J_b / 2
};

// Pointers into LDS (or global memory for a table that does not fit).
template <typename AT>
struct Ctx {
    int N, ns, m;
    uint32_t mmask;
    uint64_t low_mask;           // state bits below the top block
    const uint32_t *rep;         // [ns][P]
    const uint32_t *sym_off;     // [ns][P+1]
    const uint16_t *sym_list;
    const AT *act;               // [nu][ns][P]
    const uint8_t *u_shift;      // [nu][ns]
    const uint16_t *g_u;         // [ng]
    const uint8_t *g_flip;       // [ng]
    const double *chi;           // [ng][2]
    const double *div_sqrt;      // [n_div]
    const double *div_rsqrt;     // [n_div]
    const BondLds *bonds;        // [nb]
};

__device__ __forceinline__ void lds_copy(char *dst, const void *src, uint32_t bytes)
{
    const uint32_t *s = (const uint32_t *)src;
    uint32_t *d = (uint32_t *)dst;
    for (uint32_t k = threadIdx.x; k < bytes / 4; k += blockDim.x) d[k] = s[k];
}

// The host packs every table into one device blob with the same layout as the
// LDS image, so staging is one contiguous copy.
template <typename AT, bool ACT_LDS>
__device__ __forceinline__ Ctx<AT> stage(const DevModel &dm, const char *blob, char *lds)
{
    lds_copy(lds, blob, dm.lds_total);
    __syncthreads();
    Ctx<AT> c;
    c.N = dm.N;
    c.ns = dm.ns;
    c.m = dm.m;
    c.mmask = dm.P - 1;
    c.low_mask = (dm.N - dm.m >= 64) ? ~0ull : ((1ull << (dm.N - dm.m)) - 1ull);
    c.rep = (const uint32_t *)(lds + dm.lds_rep);
    c.sym_off = (const uint32_t *)(lds + dm.lds_sym_off);
    c.sym_list = (const uint16_t *)(lds + dm.lds_sym_list);
    c.act = ACT_LDS ? (const AT *)(lds + dm.lds_act) : (const AT *)(dm.blob + dm.lds_act);
    c.u_shift = (const uint8_t *)(lds + dm.lds_u_shift);
    c.g_u = (const uint16_t *)(lds + dm.lds_g_u);
    c.g_flip = (const uint8_t *)(lds + dm.lds_g_flip);
    c.chi = (const double *)(lds + dm.lds_chi);
    c.div_sqrt = (const double *)(lds + dm.lds_div);
    c.div_rsqrt = c.div_sqrt + dm.n_div;
    c.bonds = (const BondLds *)(lds + dm.lds_bonds);
    return c;
}

// ---------------------------------------------------------------------------
// Alg. "Sublattice coding algorithm for finding the representative"
//   MinRep = min_X Rep_X(s_X); for every block Y attaining it and every
//   g in Sym_Y(s_Y), assemble g s from the per-block action table and keep
//   the strict minimum.  The top block of every candidate equals MinRep, so
//   only the other blocks are assembled.  Returns the representative, the
//   first minimising group element, and the packed rep-table entry of MinRep
//   (rank << 16 | value) used for the index key.
// ---------------------------------------------------------------------------
template <typename AT>
__device__ __forceinline__ uint64_t find_rep(const Ctx<AT> &c, uint64_t s, uint32_t &g_best, uint32_t &min_ent)
{
    const int N = c.N, m = c.m, ns = c.ns;
    const uint32_t P = c.mmask + 1;
    uint32_t minr = 0xFFFFFFFFu, tie = 0;
    for (int X = 0; X < ns; ++X) {
        uint32_t sx = (uint32_t)(s >> (N - (X + 1) * m)) & c.mmask;
        uint32_t r = c.rep[X * P + sx];
        if (r < minr) {
            minr = r;
            tie = 1u << X;
        } else if (r == minr) {
            tie |= 1u << X;
        }
    }
    const uint64_t top = (uint64_t)(minr & 0xFFFFu) << (N - m);
    uint64_t best = ~0ull;
    uint32_t bg = 0;
    while (tie) {
        const int Y = __builtin_ctz(tie);
        tie &= tie - 1;
        const uint32_t sy = (uint32_t)(s >> (N - (Y + 1) * m)) & c.mmask;
        const uint32_t k0 = c.sym_off[Y * (P + 1) + sy], k1 = c.sym_off[Y * (P + 1) + sy + 1];
        for (uint32_t k = k0; k < k1; ++k) {
            const uint32_t g = c.sym_list[k];
            const uint32_t u = c.g_u[g];
            const AT *au = c.act + (size_t)u * ns * P;
            const uint8_t *sh = c.u_shift + u * ns;
            uint64_t v = 0;
            for (int X = 0; X < ns; ++X) {
                if (X == Y) continue;
                uint32_t sx = (uint32_t)(s >> (N - (X + 1) * m)) & c.mmask;
                v |= (uint64_t)au[X * P + sx] << sh[X];
            }
            if (c.g_flip[g]) v ^= c.low_mask;
            v |= top;
            if (v < best) {
                best = v;
                bg = g;
            }
        }
    }
    g_best = bg;
    min_ent = minr;
    return best;
}

// Index lookup (Alg. "Parallel matrix-vector multiply", receiving step):
// Limits(key) -> [begin, end), then binary search of the ascending states.
// Returns the position or -1; *entry receives the packed entry found.
__device__ __forceinline__ int64_t lookup(const DevBasis &b, uint64_t rep, uint32_t min_ent, uint64_t &entry)
{
    const uint64_t key = ((uint64_t)(min_ent >> 16) << b.key_bits) |
                         ((rep >> b.key_shift) & ((1ull << b.key_bits) - 1ull));
    uint32_t lo = b.limits[key], hi = b.limits[key + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t e = b.states[mid];
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

__device__ __forceinline__ double load_x(const double *x, int64_t j) { return x[j]; }
__device__ __forceinline__ double2 load_x(const double2 *x, int64_t j) { return x[j]; }

// ---------------------------------------------------------------------------
// Row kernel of H.v (gather form of the parallel matrix-vector multiply):
//   y_i = d_i x_i + sum_{b antiparallel} (J_b/2) chi(g) sqrt(n_j/n_i) x_j
// one thread per row, persistent blocks, every y_i written once.
// MODE 0: y = H x.   MODE 1: count kept/dropped terms.
// MODE 2: Lanczos w = H v - beta_prev v_prev, with per-block <v, w> partials.
// ---------------------------------------------------------------------------
struct LzState {
    int j;              // step index
    int done;           // breakdown or finished
    double scale;       // running max(|alpha_k|, beta_k)
    double alpha_cur, beta_cur, beta_prev;
};

template <bool CPLX, typename AT, bool ACT_LDS, int MODE>
__global__ void __launch_bounds__(1024) k_apply(DevModel dm, DevBasis db, const char *blob,
                                                const typename Scalar<CPLX>::T *__restrict__ x,
                                                typename Scalar<CPLX>::T *__restrict__ y,
                                                const typename Scalar<CPLX>::T *__restrict__ vprev,
                                                double *partials, unsigned long long *stats,
                                                const LzState *lz, double jsum_quarter)
{
    using T = typename Scalar<CPLX>::T;
    extern __shared__ __align__(16) char lds[];
    if (MODE == 2 && lz->done) return;
    const Ctx<AT> c = stage<AT, ACT_LDS>(dm, blob, lds);
    const int nb = dm.nb;
    const int nw = (nb + 63) >> 6;
    const int64_t D = db.dim;
    double acc_part = 0.0;
    unsigned long long kept = 0, dropped = 0;
    const double beta_prev = (MODE == 2) ? lz->beta_prev : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t e = db.states[i];
        const uint64_t s = e & kStateMask;
        const double rs_i = c.div_rsqrt[e >> kNormShift];
        double anti_sum = 0.0;
        double ar = 0.0, ai = 0.0;
        for (int w = 0; w < kMaxBondWords; ++w) {
            if (w >= nw) break;
            // antiparallel bonds of this word
            uint64_t am = 0;
            const int bend = min(64, nb - 64 * w);
            for (int k = 0; k < bend; ++k) {
                const uint64_t bm = c.bonds[64 * w + k].mask;
                const uint64_t t = s & bm;
                am |= (uint64_t)((t != 0) & (t != bm)) << k;
            }
            while (am) {
                const int k = __builtin_ctzll(am);
                am &= am - 1;
                const BondLds bd = c.bonds[64 * w + k];
                anti_sum += bd.jhalf;
                const uint64_t sp = s ^ bd.mask;
                uint32_t g, ment;
                const uint64_t r = find_rep(c, sp, g, ment);
                uint64_t ej = 0;
                const int64_t j = lookup(db, r, ment, ej);
                if (MODE == 1) {
                    if (j >= 0) ++kept; else ++dropped;
                    continue;
                }
                if (j < 0) continue;
                const double amp = bd.jhalf * c.div_sqrt[ej >> kNormShift] * rs_i;
                if (CPLX) {
                    const T xj = load_x(x, j);
                    const double cr = amp * c.chi[2 * g], ci = amp * c.chi[2 * g + 1];
                    const double2 xv = *(const double2 *)&xj;
                    ar += cr * xv.x - ci * xv.y;
                    ai += cr * xv.y + ci * xv.x;
                } else {
                    const double xj = *(const double *)&x[j];
                    ar += amp * c.chi[2 * g] * xj;
                }
            }
        }
        if (MODE == 1) continue;
        const double d = jsum_quarter - anti_sum;
        if (CPLX) {
            const double2 xi = *(const double2 *)&x[i];
            double2 out;
            out.x = d * xi.x + ar;
            out.y = d * xi.y + ai;
            if (MODE == 2) {
                const double2 vp = *(const double2 *)&vprev[i];
                out.x -= beta_prev * vp.x;
                out.y -= beta_prev * vp.y;
                acc_part += xi.x * out.x + xi.y * out.y;   // Re(conj(v) w)
            }
            *(double2 *)&y[i] = out;
        } else {
            const double xi = *(const double *)&x[i];
            double out = d * xi + ar;
            if (MODE == 2) {
                out -= beta_prev * *(const double *)&vprev[i];
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
        // deterministic block reduction in LDS (tables are no longer needed)
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

// ---------------------------------------------------------------------------
// Adjoint, bond part: A_b = Re sum_i conj(gy_i) (dH/dJ_b x)_i.  Bonds are
// visited in the same order by every lane so that each bond's contributions
// can be summed across the wave (fixed tree order), then across waves and
// blocks in fixed order: the result is deterministic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool CPLX, typename AT, bool ACT_LDS>
__global__ void __launch_bounds__(1024) k_backward_J(DevModel dm, DevBasis db, const char *blob,
                                                     const typename Scalar<CPLX>::T *__restrict__ x,
                                                     const typename Scalar<CPLX>::T *__restrict__ gy,
                                                     double *partials /* [grid][nb] */)
{
    extern __shared__ __align__(16) char lds[];
    const Ctx<AT> c = stage<AT, ACT_LDS>(dm, blob, lds);
    const int nb = dm.nb;
    const int nwaves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double *acc = (double *)(lds + dm.lds_total);   // [nwaves][nb]
    for (int k = threadIdx.x; k < nwaves * nb; k += blockDim.x) acc[k] = 0.0;
    __syncthreads();
    const int64_t D = db.dim;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // every lane of a wave runs the same number of iterations
    const int64_t wave_first = base - lane;
    for (int64_t i0 = wave_first; i0 < D; i0 += stride) {
        const int64_t i = i0 + lane;
        const bool valid = i < D;
        uint64_t s = 0;
        double rs_i = 0.0, gx_r = 0.0, gx_i = 0.0;   // conj(gy_i) * x_i
        double g_r = 0.0, g_i = 0.0;
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
        (void)gx_i;
        for (int b = 0; b < nb; ++b) {
            const BondLds bd = c.bonds[b];
            const uint64_t t = s & bd.mask;
            const bool anti = valid && (t != 0) && (t != bd.mask);
            double contrib = valid ? (anti ? -0.25 : 0.25) * gx_r : 0.0;
            if (anti) {
                uint32_t g, ment;
                const uint64_t r = find_rep(c, s ^ bd.mask, g, ment);
                uint64_t ej = 0;
                const int64_t j = lookup(db, r, ment, ej);
                if (j >= 0) {
                    const double amp = 0.5 * c.div_sqrt[ej >> kNormShift] * rs_i;
                    const double cr = amp * c.chi[2 * g], ci = amp * c.chi[2 * g + 1];
                    if (CPLX) {
                        const double2 xv = *(const double2 *)&x[j];
                        const double tr = cr * xv.x - ci * xv.y, ti = cr * xv.y + ci * xv.x;
                        contrib += g_r * tr + g_i * ti;   // Re(conj(gy) t)
                    } else {
                        contrib += g_r * cr * *(const double *)&x[j];
                    }
                }
            }
            const double wsum = wave_sum(contrib);
            if (lane == 0) acc[wave * nb + b] += wsum;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double tot = 0.0;
        for (int w = 0; w < nwaves; ++w) tot += acc[w * nb + b];
        partials[(size_t)blockIdx.x * nb + b] = tot;
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

template <typename AT, bool ACT_LDS, bool EMIT>
__global__ void __launch_bounds__(256) k_basis_enum(DevModel dm, BuildParams bp, const char *blob,
                                                    uint32_t *counts, const uint64_t *offsets, uint64_t *out)
{
    extern __shared__ __align__(16) char lds[];
    const Ctx<AT> c = stage<AT, ACT_LDS>(dm, blob, lds);
    const uint32_t *div_val = (const uint32_t *)(c.div_rsqrt + dm.n_div);
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
            uint32_t sx = (uint32_t)(p >> (bp.Pb - (X + 1) * m)) & c.mmask;
            ok = (c.rep[X * P + sx] & 0xFFFFu) >= t;
        }
        uint64_t w = EMIT ? offsets[p] : 0;
        if (ok) {
            uint64_t v = (r == 0) ? 0ull : ((1ull << r) - 1ull);
            const uint64_t vend = 1ull << R;
            while (v < vend) {
                const uint64_t sgm = (p << R) | v;
                // quick reject: every block's Rep must be >= the top block
                uint32_t tie = 0;
                bool pass = true;
                for (int X = 0; X < ns; ++X) {
                    uint32_t sx = (uint32_t)(sgm >> (N - (X + 1) * m)) & c.mmask;
                    uint32_t rv = c.rep[X * P + sx] & 0xFFFFu;
                    if (rv < t) { pass = false; break; }
                    if (rv == t) tie |= 1u << X;
                }
                if (pass) {
                    bool is_rep = true, compat = true;
                    uint32_t nstab = 0;
                    while (tie && is_rep) {
                        const int Y = __builtin_ctz(tie);
                        tie &= tie - 1;
                        const uint32_t sy = (uint32_t)(sgm >> (N - (Y + 1) * m)) & c.mmask;
                        for (uint32_t k = c.sym_off[Y * (P + 1) + sy]; k < c.sym_off[Y * (P + 1) + sy + 1]; ++k) {
                            const uint32_t g = c.sym_list[k];
                            const uint32_t u = c.g_u[g];
                            const AT *au = c.act + (size_t)u * ns * P;
                            const uint8_t *sh = c.u_shift + u * ns;
                            uint64_t img = 0;
                            for (int X = 0; X < ns; ++X) {
                                uint32_t sx = (uint32_t)(sgm >> (N - (X + 1) * m)) & c.mmask;
                                img |= (uint64_t)au[X * P + sx] << sh[X];
                            }
                            if (c.g_flip[g]) img ^= (c.low_mask | ((uint64_t)c.mmask << (N - m)));
                            if (img < sgm) { is_rep = false; break; }
                            if (img == sgm) {
                                ++nstab;
                                if (!dm.trivial_irrep &&
                                    (fabs(c.chi[2 * g] - 1.0) > 1e-9 || fabs(c.chi[2 * g + 1]) > 1e-9))
                                    compat = false;
                            }
                        }
                    }
                    if (is_rep && compat) {
                        if (EMIT) {
                            // index of nstab among the divisors of |G|
                            int lo = 0, hi = dm.n_div - 1;
                            while (lo < hi) {
                                int mid = (lo + hi) >> 1;
                                if (div_val[mid] < nstab) lo = mid + 1; else hi = mid;
                            }
                            out[w++] = ((uint64_t)lo << kNormShift) | sgm;
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
        uint64_t idx = base + k;
        uint64_t v = idx < n ? (uint64_t)in[idx] : 0ull;
        loc[k] = run;
        run += v;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals
    for (int o = 1; o < kScanThreads; o <<= 1) {
        uint64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t excl = sh[threadIdx.x] - run;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t idx = base + k;
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
            int64_t mid = (lo + hi) >> 1;
            if ((states[mid] & kStateMask) < lb) lo = mid + 1; else hi = mid;
        }
        limits[k] = (uint32_t)lo;
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

// partial sums of |v|^2 (n doubles = D or 2D)
__global__ void __launch_bounds__(kVecThreads) k_norm2_partial(const double *v, int64_t n, double *partials,
                                                                  const LzState *lz)
{
    __shared__ double sh[kVecThreads / kWave];
    if (lz && lz->done) return;
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a += v[i] * v[i];
    double t = block_sum(a, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// v_out = v_in * (1 / sqrt(sum of partials)), recomputing the sum per block
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

// alpha_j = sum of partials; record it
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

// w -= alpha v ; partial |w|^2 ; psi += s_j v (second pass)
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
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// complex variant: alpha is real, w and v interleaved
__global__ void __launch_bounds__(kVecThreads) k_lz_update_c(double *w, const double *v, int64_t nc, double *partials,
                                                                const LzState *lz, double *psi, const double *svec)
{
    __shared__ double sh[kVecThreads / kWave];
    if (lz->done) return;
    const double a = lz->alpha_cur;
    const double sj = psi ? svec[lz->j] : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
        double2 vi = ((const double2 *)v)[i];
        double2 wi = ((double2 *)w)[i];
        wi.x -= a * vi.x;
        wi.y -= a * vi.y;
        ((double2 *)w)[i] = wi;
        acc += wi.x * wi.x + wi.y * wi.y;
        if (psi) {
            double2 pv = ((double2 *)psi)[i];
            pv.x += sj * vi.x;
            pv.y += sj * vi.y;
            ((double2 *)psi)[i] = pv;
        }
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// beta_j = sqrt(sum of partials); breakdown test; advance j
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

// v_new = w / beta_j (written over the oldest vector); beta_prev <- beta_j
__global__ void __launch_bounds__(kVecThreads) k_lz_normalize(const double *w, double *vnew, int64_t n, LzState *lz)
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
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ED_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    b->allocs.push_back(*p);
    b->device_bytes += (int64_t)bytes;
    return ED_OK;
}

static int num_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

// All tables in one blob whose layout equals the LDS image (the action table
// sits at the end so that it can be left out of LDS).
static int upload_tables(ed_basis *b, hipStream_t st, bool act_u8)
{
    const Tables &t = b->t;
    DevModel &dm = b->dm;
    auto align16 = [](uint32_t v) { return (v + 15u) & ~15u; };
    const uint32_t P = t.P;
    std::vector<char> blob;
    auto put = [&](const void *src, size_t bytes) -> uint32_t {
        uint32_t off = align16((uint32_t)blob.size());
        blob.resize(off + bytes);
        if (bytes) memcpy(blob.data() + off, src, bytes);
        return off;
    };
    dm.lds_rep = put(t.rep.data(), t.rep.size() * 4);
    dm.lds_sym_off = put(t.sym_off.data(), t.sym_off.size() * 4);
    dm.lds_sym_list = put(t.sym_list.data(), t.sym_list.size() * 2);
    std::vector<uint8_t> ush((size_t)t.nu * t.ns);
    for (size_t k = 0; k < ush.size(); ++k) ush[k] = (uint8_t)(t.N - (t.u_tgt[k] + 1) * t.m);
    dm.lds_u_shift = put(ush.data(), ush.size());
    dm.lds_g_u = put(t.g_u.data(), t.g_u.size() * 2);
    dm.lds_g_flip = put(t.flip.data(), t.flip.size());
    dm.lds_chi = put(b->chi_host.data(), b->chi_host.size() * 8);
    std::vector<double> dv;
    for (uint32_t d : b->divs) dv.push_back(std::sqrt((double)d));
    for (uint32_t d : b->divs) dv.push_back(1.0 / std::sqrt((double)d));
    std::vector<uint32_t> dvals(b->divs.begin(), b->divs.end());
    dm.lds_div = put(dv.data(), dv.size() * 8);
    put(dvals.data(), dvals.size() * 4);   // div_val right after the sqrt tables (same 16B alignment chain)
    // bonds: masks and J/2 are written per call; reserve space
    std::vector<BondLds> bz((size_t)std::max(t.nb, 1));
    for (int k = 0; k < t.nb; ++k) {
        int p = t.bonds[2 * k], q = t.bonds[2 * k + 1];
        bz[k].mask = (1ull << (t.N - 1 - p)) | (1ull << (t.N - 1 - q));
        bz[k].jhalf = 0.0;
    }
    dm.lds_bonds = put(bz.data(), bz.size() * sizeof(BondLds));
    const uint32_t small_end = align16((uint32_t)blob.size());
    // action table
    std::vector<uint8_t> act8;
    if (act_u8) {
        act8.resize(t.act.size());
        for (size_t k = 0; k < t.act.size(); ++k) act8[k] = (uint8_t)t.act[k];
        dm.lds_act = put(act8.data(), act8.size());
    } else {
        dm.lds_act = put(t.act.data(), t.act.size() * 2);
    }
    const uint32_t full_end = align16((uint32_t)blob.size());
    blob.resize(full_end);
    (void)P;
    // decide LDS placement of the action table; keep 8 KB of the per-block
    // LDS limit for reductions and the adjoint's per-wave accumulators
    int dev = 0, lds_max = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds_max <= 0)
        lds_max = 65536;
    const uint32_t lds_cap = (uint32_t)lds_max - 8192u;
    bool fits = full_end <= std::min<uint32_t>(lds_cap, 56u * 1024u);
    if (b->tuning.table_lds == 1) fits = full_end <= lds_cap;
    if (b->tuning.table_lds == 2) fits = false;
    dm.act_in_lds = fits ? 1 : 0;
    dm.lds_total = fits ? full_end : small_end;
    if (small_end > lds_cap)
        return set_error(ED_ERR_UNSUPPORTED, "lookup tables (%u bytes) exceed the LDS budget (%u)", small_end, lds_cap);
    void *d = nullptr;
    int rc = device_alloc(b, &d, blob.size());
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(d, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    dm.blob = (const char *)d;
    return ED_OK;
}

static inline const char *blob_ptr(const ed_basis *b) { return b->dm.blob; }
static inline bool act_is_u8(const ed_basis *b) { return b->t.m <= 8; }

// bonds' J/2 live inside the blob; rewrite them when J changes
static int upload_couplings(const ed_basis *bc, const double *J, hipStream_t st, double *jsum_quarter)
{
    ed_basis *b = const_cast<ed_basis *>(bc);
    const Tables &t = b->t;
    double js0 = 0.0;
    for (int k = 0; k < t.nb; ++k) js0 += J[k];
    *jsum_quarter = 0.25 * js0;
    if ((int)b->J_cache.size() == t.nb && std::equal(b->J_cache.begin(), b->J_cache.end(), J)) return ED_OK;
    std::vector<BondLds> bz((size_t)std::max(t.nb, 1));
    double js = 0.0;
    for (int k = 0; k < t.nb; ++k) {
        int p = t.bonds[2 * k], q = t.bonds[2 * k + 1];
        bz[k].mask = (1ull << (t.N - 1 - p)) | (1ull << (t.N - 1 - q));
        bz[k].jhalf = 0.5 * J[k];
        js += J[k];
    }
    *jsum_quarter = 0.25 * js;
    char *dst = (char *)blob_ptr(b) + b->dm.lds_bonds;
    HIP_TRY(hipMemcpyAsync(dst, bz.data(), (size_t)t.nb * sizeof(BondLds), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    b->J_cache.assign(J, J + t.nb);
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
        int o = t.bond_orbit[k];
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
static int launch_cfg(const ed_basis *b, Kern kern, int lds_extra, int *grid, int *threads, size_t *lds)
{
    int th = b->tuning.block_threads > 0 ? b->tuning.block_threads : 256;
    *threads = th;
    *lds = (size_t)b->dm.lds_total + (size_t)lds_extra;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, th, *lds) != hipSuccess || per_cu < 1) per_cu = 1;
    if (b->tuning.blocks_per_cu > 0) per_cu = std::min(per_cu, b->tuning.blocks_per_cu);
    const int64_t need = (b->db.dim + th - 1) / th;
    int64_t g = (int64_t)per_cu * num_cus();
    if (g > need) g = need;
    if (g < 1) g = 1;
    *grid = (int)g;
    return ED_OK;
}

// ---- basis build ---------------------------------------------------------

template <typename AT, bool ACT_LDS>
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
    const char *blob = blob_ptr(b);
    const int threads = 256;
    const size_t lds = dm.lds_total;
    int per_cu = 1;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_basis_enum<AT, ACT_LDS, false>, threads, lds);
    per_cu = std::max(per_cu, 1);
    uint64_t grid = std::min<uint64_t>((np + threads - 1) / threads, (uint64_t)per_cu * num_cus() * 8);
    hipLaunchKernelGGL((k_basis_enum<AT, ACT_LDS, false>), dim3((unsigned)grid), dim3(threads), lds, st, dm, bp, blob,
                       counts, (const uint64_t *)nullptr, (uint64_t *)nullptr);
    if (hipGetLastError() != hipSuccess) {
        cleanup();
        return set_error(ED_ERR_HIP, "basis count launch failed");
    }
    // exclusive scan counts -> offsets (multi-level)
    {
        std::vector<std::pair<uint64_t *, uint64_t>> levels;   // (array, n) to be fixed up
        uint64_t n = np;
        const void *in = counts;
        bool in32 = true;
        uint64_t *outp = offsets;
        std::vector<void *> tmp;
        int rc = ED_OK;
        while (true) {
            uint64_t tiles = (n + kScanTile - 1) / kScanTile;
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
        // fix up from the coarsest level down
        for (int lv = (int)levels.size() - 2; rc == ED_OK && lv >= 0; --lv) {
            uint64_t nn = levels[lv].second;
            unsigned g = (unsigned)std::min<uint64_t>((nn + 255) / 256, 65536);
            hipLaunchKernelGGL(k_scan_add, dim3(g), dim3(256), 0, st, levels[lv].first, nn,
                               (const uint64_t *)levels[lv + 1].first);
        }
        // total = offsets[np-1] + counts[np-1]
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
        return set_error(ED_ERR_UNSUPPORTED, "sector dimension %lld needs 64-bit Limits", (long long)D);
    }
    void *states = nullptr;
    int rc = device_alloc(b, &states, (size_t)std::max<int64_t>(D, 1) * 8);
    if (rc) {
        cleanup();
        return rc;
    }
    hipLaunchKernelGGL((k_basis_enum<AT, ACT_LDS, true>), dim3((unsigned)grid), dim3(threads), lds, st, dm, bp, blob,
                       (uint32_t *)nullptr, (const uint64_t *)offsets, (uint64_t *)states);
    if (hipGetLastError() != hipSuccess) {
        cleanup();
        return set_error(ED_ERR_HIP, "basis emit launch failed");
    }
    // Limits over (top-block rank, next q bits)
    const int n_top = (int)t.top_vals.size();
    int q = b->tuning.limits_bits;
    const int avail = N - m;
    if (q <= 0) {
        // about 4 states per key, at most 2^28 keys
        double target = std::max(1.0, (double)D / 4.0 / std::max(1, n_top));
        q = (int)std::ceil(std::log2(target));
        q = std::max(q, 0);
        while (q > 0 && ((uint64_t)n_top << q) > (1ull << 28)) --q;
    }
    q = std::min(q, avail);
    b->db.key_bits = q;
    b->db.key_shift = N - m - q;
    b->db.n_keys = (int64_t)n_top << q;
    void *tv = nullptr, *lim = nullptr;
    rc = device_alloc(b, &tv, t.top_vals.size() * 2);
    if (!rc) rc = device_alloc(b, &lim, ((size_t)b->db.n_keys + 1) * 4);
    if (rc) {
        cleanup();
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(tv, t.top_vals.data(), t.top_vals.size() * 2, hipMemcpyHostToDevice, st));
    {
        unsigned g = (unsigned)std::min<uint64_t>(((uint64_t)b->db.n_keys + 256) / 256, 1u << 20);
        hipLaunchKernelGGL(k_limits, dim3(g), dim3(256), 0, st, (const uint64_t *)states, D, (const uint16_t *)tv, N, m, q,
                           b->db.key_shift, (uint64_t)b->db.n_keys, (uint32_t *)lim);
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        cleanup();
        return set_error(ED_ERR_HIP, "basis build failed: %s", hipGetErrorString(hipGetLastError()));
    }
    cleanup();
    b->db.states = (const uint64_t *)states;
    b->db.limits = (const uint32_t *)lim;
    return ED_OK;
}

int launch_basis_build(ed_basis *b, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const bool u8 = act_is_u8(b);
    int rc = upload_tables(b, st, u8);
    if (rc) return rc;
    if (u8) return b->dm.act_in_lds ? build_impl<uint8_t, true>(b, st) : build_impl<uint8_t, false>(b, st);
    return b->dm.act_in_lds ? build_impl<uint16_t, true>(b, st) : build_impl<uint16_t, false>(b, st);
}

// ---- H.v -----------------------------------------------------------------

template <bool CPLX, typename AT, bool ACT_LDS, int MODE>
static int apply_impl(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                      unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st, int *grid_out)
{
    using T = typename Scalar<CPLX>::T;
    auto kern = k_apply<CPLX, AT, ACT_LDS, MODE>;
    int grid, threads;
    size_t lds;
    launch_cfg(b, kern, 0, &grid, &threads, &lds);
    if (MODE == 2) {
        lds = std::max(lds, (size_t)threads * 8);
        grid = b->grid_blocks;   // fixed grid so the reductions are deterministic
    }
    if (grid_out) *grid_out = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, b->dm, b->db, blob_ptr(b), (const T *)x, (T *)y,
                       (const T *)vprev, partials, stats, lz, jsq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "H.v launch failed: %s", hipGetErrorString(e));
    return ED_OK;
}

template <int MODE>
static int apply_dispatch(const ed_basis *b, const void *x, void *y, const void *vprev, double *partials,
                          unsigned long long *stats, const LzState *lz, double jsq, hipStream_t st)
{
    const bool c = b->dm.is_complex, u8 = act_is_u8(b), l = b->dm.act_in_lds;
#define ED_CASE(C, A, L)                                                                             \
    if (c == C && u8 == (sizeof(A) == 1) && l == L)                                                  \
        return apply_impl<C, A, L, MODE>(b, x, y, vprev, partials, stats, lz, jsq, st, nullptr);
    ED_CASE(false, uint8_t, true)
    ED_CASE(false, uint8_t, false)
    ED_CASE(false, uint16_t, true)
    ED_CASE(false, uint16_t, false)
    ED_CASE(true, uint8_t, true)
    ED_CASE(true, uint8_t, false)
    ED_CASE(true, uint16_t, true)
    ED_CASE(true, uint16_t, false)
#undef ED_CASE
    return set_error(ED_ERR_ARG, "no kernel variant");
}

int launch_apply(const ed_basis *b, const double *J, const void *x, void *y, void *stream, int stats_mode,
                 unsigned long long *stats_dev)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = check_couplings(b, J);
    if (rc) return rc;
    double jsq = 0.0;
    if (!stats_mode) {
        rc = upload_couplings(b, J, st, &jsq);
        if (rc) return rc;
    }
    if (b->db.dim == 0) return ED_OK;
    if (stats_mode) return apply_dispatch<1>(b, x, y, nullptr, nullptr, stats_dev, nullptr, 0.0, st);
    return apply_dispatch<0>(b, x, y, nullptr, nullptr, nullptr, nullptr, jsq, st);
}

// ---- adjoint ---------------------------------------------------------------

template <bool CPLX, typename AT, bool ACT_LDS>
static int backward_impl(const ed_basis *b, const void *x, const void *gy, double *gJ_host, hipStream_t st)
{
    using T = typename Scalar<CPLX>::T;
    auto kern = k_backward_J<CPLX, AT, ACT_LDS>;
    const int nb = b->t.nb;
    int grid, threads;
    size_t lds;
    const int threads_req = 256;
    int per_cu = 1;
    lds = (size_t)b->dm.lds_total + (size_t)(threads_req / kWave) * nb * 8;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads_req, lds);
    per_cu = std::max(per_cu, 1);
    threads = threads_req;
    grid = (int)std::min<int64_t>((b->db.dim + threads - 1) / threads, (int64_t)per_cu * num_cus());
    grid = std::max(grid, 1);
    double *partials = nullptr, *out = nullptr;
    if (hipMalloc((void **)&partials, (size_t)grid * nb * 8) != hipSuccess ||
        hipMalloc((void **)&out, (size_t)nb * 8) != hipSuccess) {
        (void)hipGetLastError();
        if (partials) (void)hipFree(partials);
        return set_error(ED_ERR_OOM, "adjoint partials");
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, b->dm, b->db, blob_ptr(b), (const T *)x, (const T *)gy,
                       partials);
    hipLaunchKernelGGL(k_sum_partials_cols, dim3((nb + 255) / 256), dim3(256), 0, st, (const double *)partials, grid, nb,
                       out);
    hipError_t e = hipMemcpyAsync(gJ_host, out, (size_t)nb * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(partials);
    (void)hipFree(out);
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "adjoint failed: %s", hipGetErrorString(e));
    return ED_OK;
}

int launch_backward_J(const ed_basis *b, const double *J, const void *x, const void *gy, double *gJ_host, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    int rc = check_couplings(b, J);
    if (rc) return rc;
    double jsq;
    rc = upload_couplings(b, J, st, &jsq);
    if (rc) return rc;
    if (b->db.dim == 0 || b->t.nb == 0) {
        for (int k = 0; k < b->t.nb; ++k) gJ_host[k] = 0.0;
        return ED_OK;
    }
    const bool c = b->dm.is_complex, u8 = act_is_u8(b), l = b->dm.act_in_lds;
#define ED_CASE(C, A, L) \
    if (c == C && u8 == (sizeof(A) == 1) && l == L) return backward_impl<C, A, L>(b, x, gy, gJ_host, st);
    ED_CASE(false, uint8_t, true)
    ED_CASE(false, uint8_t, false)
    ED_CASE(false, uint16_t, true)
    ED_CASE(false, uint16_t, false)
    ED_CASE(true, uint8_t, true)
    ED_CASE(true, uint8_t, false)
    ED_CASE(true, uint16_t, true)
    ED_CASE(true, uint16_t, false)
#undef ED_CASE
    return set_error(ED_ERR_ARG, "no kernel variant");
}

// ---- Lanczos ---------------------------------------------------------------

int run_lanczos(const ed_basis *bc, const double *J, const void *v0, int n_steps, double *alpha, double *beta,
                int *n_done, void *psi0, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(bc);
    hipStream_t st = (hipStream_t)stream;
    int rc = check_couplings(b, J);
    if (rc) return rc;
    double jsq;
    rc = upload_couplings(b, J, st, &jsq);
    if (rc) return rc;
    const int64_t D = b->db.dim;
    *n_done = 0;
    if (D == 0 || n_steps <= 0) return ED_OK;
    const bool cplx = b->dm.is_complex;
    const int64_t nd = cplx ? 2 * D : D;   // doubles per vector
    // fixed launch geometry -> deterministic reductions, identical passes
    {
        int grid, threads;
        size_t lds;
        launch_cfg(b, k_apply<false, uint8_t, true, 2>, 0, &grid, &threads, &lds);
        b->grid_blocks = grid;
    }
    const int vgrid = (int)std::min<int64_t>((nd + kVecThreads - 1) / kVecThreads, (int64_t)num_cus() * 8);
    const int np_apply = b->grid_blocks;
    double *A = nullptr, *B = nullptr, *C = nullptr, *partials = nullptr, *ahist = nullptr, *bhist = nullptr,
           *svec = nullptr;
    LzState *lz = nullptr;
    auto freeall = [&]() {
        for (void *p : {(void *)A, (void *)B, (void *)C, (void *)partials, (void *)ahist, (void *)bhist, (void *)svec,
                        (void *)lz})
            if (p) (void)hipFree(p);
    };
    const size_t vb = (size_t)nd * 8;
    if (hipMalloc((void **)&A, vb) != hipSuccess || hipMalloc((void **)&B, vb) != hipSuccess ||
        hipMalloc((void **)&C, vb) != hipSuccess ||
        hipMalloc((void **)&partials, (size_t)std::max(np_apply, vgrid) * 8) != hipSuccess ||
        hipMalloc((void **)&ahist, (size_t)n_steps * 8) != hipSuccess ||
        hipMalloc((void **)&bhist, (size_t)n_steps * 8) != hipSuccess ||
        hipMalloc((void **)&svec, (size_t)n_steps * 8) != hipSuccess || hipMalloc((void **)&lz, sizeof(LzState)) != hipSuccess) {
        (void)hipGetLastError();
        freeall();
        return set_error(ED_ERR_OOM, "Lanczos vectors (3 x %zu bytes)", vb);
    }
    std::vector<double> svec_host(n_steps, 0.0);
    int passes = psi0 ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
        double *psi = pass == 1 ? (double *)psi0 : nullptr;
        LzState init{};
        init.j = 0;
        init.done = 0;
        init.scale = 0.0;
        init.beta_prev = 0.0;
        HIP_TRY(hipMemcpyAsync(lz, &init, sizeof init, hipMemcpyHostToDevice, st));
        if (psi) {
            HIP_TRY(hipMemsetAsync(psi, 0, vb, st));
            HIP_TRY(hipMemcpyAsync(svec, svec_host.data(), (size_t)n_steps * 8, hipMemcpyHostToDevice, st));
        }
        // v (B) = v0 / |v0| ; v_prev (A) = 0
        HIP_TRY(hipMemsetAsync(A, 0, vb, st));
        hipLaunchKernelGGL(k_norm2_partial, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)v0, nd, partials,
                           (const LzState *)nullptr);
        hipLaunchKernelGGL(k_scale_by_norm, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)v0, B, nd,
                           (const double *)partials, vgrid);
        double *vprev = A, *v = B, *w = C;
        for (int step = 0; step < n_steps; ++step) {
            rc = apply_dispatch<2>(b, v, w, vprev, partials, nullptr, lz, jsq, st);
            if (rc) {
                freeall();
                return rc;
            }
            hipLaunchKernelGGL(k_lz_alpha, dim3(1), dim3(64), 0, st, lz, (const double *)partials, np_apply, ahist);
            if (cplx)
                hipLaunchKernelGGL(k_lz_update_c, dim3(vgrid), dim3(kVecThreads), 0, st, w, (const double *)v, D, partials,
                                   (const LzState *)lz, psi, (const double *)svec);
            else
                hipLaunchKernelGGL(k_lz_update, dim3(vgrid), dim3(kVecThreads), 0, st, w, (const double *)v, D, partials,
                                   (const LzState *)lz, psi, (const double *)svec);
            hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(64), 0, st, lz, (const double *)partials, vgrid, bhist, n_steps,
                               1e-12);
            hipLaunchKernelGGL(k_lz_normalize, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)w, vprev, nd, lz);
            hipLaunchKernelGGL(k_lz_shift_beta, dim3(1), dim3(64), 0, st, lz);
            // rotate: new v was written over vprev
            std::swap(vprev, v);
            if ((step & 15) == 15) {
                LzState hs;
                HIP_TRY(hipMemcpyAsync(&hs, lz, sizeof hs, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (hs.done) break;
            }
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
            if (rc) {
                freeall();
                return rc;
            }
            for (int k = 0; k < hs.j; ++k) svec_host[k] = z[k];
        }
        if (pass == 1) {
            hipLaunchKernelGGL(k_norm2_partial, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)psi, nd, partials,
                               (const LzState *)nullptr);
            hipLaunchKernelGGL(k_scale_by_norm, dim3(vgrid), dim3(kVecThreads), 0, st, (const double *)psi, psi, nd,
                               (const double *)partials, vgrid);
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    freeall();
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "Lanczos failed: %s", hipGetErrorString(e));
    return ED_OK;
}

}  // namespace ed

extern "C" int ed_internal_unpack_states(const ed_basis *b, uint64_t *dev_out, void *stream)
{
    const int64_t D = b->db.dim;
    if (D == 0) return ED_OK;
    unsigned g = (unsigned)std::min<int64_t>((D + 255) / 256, 65536);
    hipLaunchKernelGGL(ed::k_unpack_states, dim3(g), dim3(256), 0, (hipStream_t)stream, b->db.states, dev_out, D);
    hipError_t e = hipGetLastError();
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
    if (e == hipSuccess && b->db.dim > 0)
        rc = ed::apply_dispatch<1>(b, nullptr, nullptr, nullptr, nullptr, d, nullptr, 0.0, st);
    if (e == hipSuccess && rc == ED_OK) e = hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && rc == ED_OK) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (rc) return rc;
    if (e != hipSuccess) return ed::set_error(ED_ERR_HIP, "stats: %s", hipGetErrorString(e));
    *kept = (int64_t)h[0];
    *dropped = (int64_t)h[1];
    return ED_OK;
}
