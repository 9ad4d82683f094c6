/*
 * Brute-force CPU oracle for the symmetry-sector Hamiltonian-vector product.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code; the product library never
 * does, and this file shares nothing with it.
 *
 * Everything here is the plain definition, applied literally:
 *   - the group acts on a configuration by moving the spin on site i to site
 *     perm[g][i] and, for flip elements, inverting every spin
 *     (sec. "Symmetry adapted basis states"; site 1 is the most significant
 *     bit, up = 1, as the worked examples' integers (011)_2 = 3 fix);
 *   - the representative of a configuration is the smallest integer in its
 *     orbit, found by applying every group element (the first, memory-free
 *     option listed in sec. "Sublattice coding algorithm"), and g_sigma is
 *     the first minimiser in group order;
 *   - a representative belongs to the sector of the 1-D irrep chi iff chi is
 *     1 on its stabiliser (otherwise its symmetrised state has zero norm);
 *     the norm ratio N_sigma'/N_sigma is sqrt(|Stab sigma'| / |Stab sigma|);
 *   - the matrix element between symmetrised states is
 *     (J_b/2) * conj(chi(g_sigma')) * sqrt(n_i/n_j)  (Eq. for matrix elements
 *     between representatives, with the conjugate that the state definition
 *     implies), applied in the scatter order of the parallel matrix-vector
 *     algorithm: every source state sends its terms to the target's index,
 *     found by binary search in the ascending list of representatives;
 *   - the S.S diagonal is +J/4 for parallel and -J/4 for antiparallel pairs.
 * The Hamiltonian is a sum of non-branching two-site terms (sec. "Parallel
 * matrix-vector multiply"): per bond an exchange J_b/2 (S+S- + S-S+) and an
 * Ising part Jz_b Sz Sz; Jz = J (passed as NULL) is the Heisenberg model,
 * Jz != J the XXZ model.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static uint64_t full_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

static int get_bit(uint64_t s, int n, int site) { return (int)((s >> (n - 1 - site)) & 1ull); }

/* g applied to s: the spin on site i moves to site perm[i]; flip inverts all. */
uint64_t orc_act(int n, const int32_t *perm, int flip, uint64_t s)
{
    uint64_t r = 0;
    for (int i = 0; i < n; ++i)
        r |= (uint64_t)get_bit(s, n, i) << (n - 1 - perm[i]);
    if (flip) r ^= full_mask(n);
    return r;
}

/* Smallest orbit element and the first group element reaching it. */
uint64_t orc_rep(int n, int ng, const int32_t *perm, const uint8_t *flip, uint64_t s, int32_t *g_out)
{
    uint64_t best = ~0ull;
    int32_t bg = -1;
    for (int g = 0; g < ng; ++g) {
        uint64_t t = orc_act(n, perm + (size_t)g * n, flip[g], s);
        if (t < best) { best = t; bg = g; }
    }
    if (g_out) *g_out = bg;
    return best;
}

/* Stabiliser size and whether chi is identically 1 on the stabiliser. */
static int stabiliser(int n, int ng, const int32_t *perm, const uint8_t *flip, const double *chi,
                      uint64_t s, int *compatible)
{
    int cnt = 0;
    double re = 0.0, im = 0.0;
    for (int g = 0; g < ng; ++g) {
        if (orc_act(n, perm + (size_t)g * n, flip[g], s) == s) {
            ++cnt;
            re += chi[2 * g];
            im += chi[2 * g + 1];
        }
    }
    *compatible = fabs(re - cnt) < 1e-9 && fabs(im) < 1e-9;
    return cnt;
}

void orc_rep_many(int n, int ng, const int32_t *perm, const uint8_t *flip, const double *chi,
                  int64_t m, const uint64_t *in, uint64_t *rep_out, int32_t *g_out,
                  int32_t *stab_out, uint8_t *compat_out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < m; ++k) {
        int32_t g;
        uint64_t r = orc_rep(n, ng, perm, flip, in[k], &g);
        int comp;
        int st = stabiliser(n, ng, perm, flip, chi, r, &comp);
        rep_out[k] = r;
        if (g_out) g_out[k] = g;
        if (stab_out) stab_out[k] = st;
        if (compat_out) compat_out[k] = (uint8_t)comp;
    }
}

/* ---- enumeration of fixed-popcount states in ascending order ---------- */

/* exact binomial: C(a-b+i, i) = C(a-b+i-1, i-1) * (a-b+i) / i at every step */
static uint64_t binom_u(int a, int b)
{
    if (b < 0 || b > a) return 0;
    unsigned __int128 r = 1;
    for (int i = 1; i <= b; ++i) r = r * (unsigned)(a - b + i) / (unsigned)i;
    return (uint64_t)r;
}

/* r-th (0-based) n-bit integer with k set bits, ascending order. */
static uint64_t unrank(int n, int k, uint64_t r)
{
    uint64_t s = 0;
    for (int i = n - 1; i >= 0 && k > 0; --i) {
        uint64_t zeros = binom_u(i, k); /* numbers with bit i clear */
        if (r >= zeros) {
            r -= zeros;
            s |= 1ull << i;
            --k;
        }
    }
    return s;
}

/* next larger integer with the same popcount */
static uint64_t next_comb(uint64_t v)
{
    uint64_t t = v | (v - 1);
    return (t + 1) | (((~t & -~t) - 1) >> (__builtin_ctzll(v) + 1));
}

/* r-th (0-based) state of the ascending enumeration, for callers that split it */
uint64_t orc_unrank(int n, int k, uint64_t r) { return unrank(n, k, r); }

/*
 * Enumerate the sector basis restricted to ranks [rank_lo, rank_hi) of the
 * ascending list of popcount-n_up configurations: every configuration there
 * that equals its representative and is compatible with chi.  If states_out
 * is NULL only the count is returned.  Otherwise at most cap entries are
 * written, in ascending order, together with the stabiliser sizes.  Returns
 * the number of sector states in the range.
 */
int64_t orc_basis_range(int n, int n_up, int ng, const int32_t *perm, const uint8_t *flip,
                        const double *chi, uint64_t rank_lo, uint64_t rank_hi,
                        uint64_t *states_out, int32_t *stab_out, int64_t cap)
{
    uint64_t total = binom_u(n, n_up);
    if (rank_hi > total) rank_hi = total;
    if (rank_lo >= rank_hi) return 0;
    uint64_t span = rank_hi - rank_lo;
    int nchunk = 256;
    if ((uint64_t)nchunk > span) nchunk = (int)span;
    int64_t *counts = (int64_t *)calloc((size_t)nchunk + 1, sizeof(int64_t));
    uint64_t **lists = (uint64_t **)calloc((size_t)nchunk, sizeof(uint64_t *));
    int32_t **stabs = (int32_t **)calloc((size_t)nchunk, sizeof(int32_t *));
    int want = states_out != NULL;

#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nchunk; ++c) {
        uint64_t lo = rank_lo + (uint64_t)((unsigned __int128)span * (unsigned)c / (unsigned)nchunk);
        uint64_t hi = rank_lo + (uint64_t)((unsigned __int128)span * (unsigned)(c + 1) / (unsigned)nchunk);
        int64_t capl = 0, cnt = 0;
        uint64_t *lst = NULL;
        int32_t *stb = NULL;
        uint64_t s = unrank(n, n_up, lo);
        for (uint64_t r = lo; r < hi; ++r) {
            /* s is a representative iff no image is smaller; the images equal
               to s form its stabiliser, whose characters decide compatibility */
            int is_rep = 1, st = 0;
            double re = 0.0, im = 0.0;
            for (int g = 0; g < ng; ++g) {
                uint64_t t = orc_act(n, perm + (size_t)g * n, flip[g], s);
                if (t < s) { is_rep = 0; break; }
                if (t == s) {
                    ++st;
                    re += chi[2 * g];
                    im += chi[2 * g + 1];
                }
            }
            if (is_rep) {
                int comp = fabs(re - st) < 1e-9 && fabs(im) < 1e-9;
                if (comp) {
                    if (want) {
                        if (cnt == capl) {
                            capl = capl ? 2 * capl : 1024;
                            lst = (uint64_t *)realloc(lst, (size_t)capl * sizeof(uint64_t));
                            stb = (int32_t *)realloc(stb, (size_t)capl * sizeof(int32_t));
                        }
                        lst[cnt] = s;
                        stb[cnt] = st;
                    }
                    ++cnt;
                }
            }
            if (r + 1 < hi) s = next_comb(s);
        }
        counts[c] = cnt;
        lists[c] = lst;
        stabs[c] = stb;
    }
    int64_t dim = 0;
    for (int c = 0; c < nchunk; ++c) {
        if (want) {
            for (int64_t k = 0; k < counts[c] && dim + k < cap; ++k) {
                states_out[dim + k] = lists[c][k];
                stab_out[dim + k] = stabs[c][k];
            }
        }
        dim += counts[c];
        free(lists[c]);
        free(stabs[c]);
    }
    free(counts);
    free(lists);
    free(stabs);
    return dim;
}

/* The whole sector basis: orc_basis_range over every rank. */
int64_t orc_basis(int n, int n_up, int ng, const int32_t *perm, const uint8_t *flip,
                  const double *chi, uint64_t *states_out, int32_t *stab_out, int64_t cap)
{
    return orc_basis_range(n, n_up, ng, perm, flip, chi, 0, binom_u(n, n_up), states_out, stab_out, cap);
}

static int64_t find_state(int64_t dim, const uint64_t *basis, uint64_t s)
{
    int64_t lo = 0, hi = dim;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (basis[mid] < s) lo = mid + 1; else hi = mid;
    }
    return (lo < dim && basis[lo] == s) ? lo : -1;
}

/*
 * y = H x in the sector (scatter order).  x, y are complex interleaved
 * (re, im) of length dim.  Returns the number of kept off-diagonal terms in
 * *kept and of dropped ones (target representative not in the sector) in
 * *dropped.  Each thread accumulates into its own copy of y; the copies are
 * summed in thread order.
 */
void orc_apply(int n, int ng, const int32_t *perm, const uint8_t *flip, const double *chi,
               int nb, const int32_t *bonds, const double *J, const double *Jz, int64_t dim,
               const uint64_t *basis, const int32_t *stab, const double *x, double *y, int nthreads,
               int64_t *kept, int64_t *dropped)
{
    if (!Jz) Jz = J; /* isotropic S.S */
    if (nthreads < 1) nthreads = 1;
    double *acc = (double *)calloc((size_t)nthreads * (size_t)dim * 2, sizeof(double));
    int64_t *kc = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
    int64_t *dc = (int64_t *)calloc((size_t)nthreads, sizeof(int64_t));
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t j = 0; j < dim; ++j) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *yt = acc + (size_t)tid * (size_t)dim * 2;
        uint64_t s = basis[j];
        double xr = x[2 * j], xi = x[2 * j + 1];
        double d = 0.0;
        for (int b = 0; b < nb; ++b) {
            int p = bonds[2 * b], q = bonds[2 * b + 1];
            int same = get_bit(s, n, p) == get_bit(s, n, q);
            d += same ? 0.25 * Jz[b] : -0.25 * Jz[b];
        }
        yt[2 * j] += d * xr;
        yt[2 * j + 1] += d * xi;
        for (int b = 0; b < nb; ++b) {
            int p = bonds[2 * b], q = bonds[2 * b + 1];
            if (get_bit(s, n, p) == get_bit(s, n, q)) continue;
            uint64_t sp = s ^ (1ull << (n - 1 - p)) ^ (1ull << (n - 1 - q));
            int32_t h;
            uint64_t r = orc_rep(n, ng, perm, flip, sp, &h);
            int64_t i = find_state(dim, basis, r);
            if (i < 0) { ++dc[tid]; continue; }
            ++kc[tid];
            double amp = 0.5 * J[b] * sqrt((double)stab[i] / (double)stab[j]);
            double cr = amp * chi[2 * h], ci = -amp * chi[2 * h + 1]; /* conj(chi(h)) */
            yt[2 * i] += cr * xr - ci * xi;
            yt[2 * i + 1] += cr * xi + ci * xr;
        }
    }
    memset(y, 0, sizeof(double) * (size_t)dim * 2);
    int64_t k = 0, dd = 0;
    for (int t = 0; t < nthreads; ++t) {
        const double *yt = acc + (size_t)t * (size_t)dim * 2;
        for (int64_t e = 0; e < 2 * dim; ++e) y[e] += yt[e];
        k += kc[t];
        dd += dc[t];
    }
    if (kept) *kept = k;
    if (dropped) *dropped = dd;
    free(acc);
    free(kc);
    free(dc);
}

/*
 * Terms of selected rows, for checks of H x row by row when the full basis
 * is too large to enumerate.  For each row state (a representative) this
 * returns its stabiliser size and compatibility, its S.S diagonal, and for
 * every bond b the representative of the flipped configuration (or 0 with
 * flag 0 for parallel bonds), the target's stabiliser size and
 * compatibility, and the element H_{row, target} of the Hermitian matrix,
 * i.e. the complex conjugate of the scatter element that the row sends to
 * the target: (J_b/2) * chi(g) * sqrt(n_target / n_row).
 */
void orc_row_terms(int n, int ng, const int32_t *perm, const uint8_t *flip, const double *chi,
                   int nb, const int32_t *bonds, const double *J, const double *Jz, int64_t nrows,
                   const uint64_t *rows, int32_t *row_stab, uint8_t *row_compat, double *row_diag,
                   uint64_t *tgt, int32_t *tgt_stab, uint8_t *tgt_flag, double *coef)
{
    if (!Jz) Jz = J;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        uint64_t s = rows[r];
        int comp;
        int ns = stabiliser(n, ng, perm, flip, chi, s, &comp);
        row_stab[r] = ns;
        row_compat[r] = (uint8_t)comp;
        double d = 0.0;
        for (int b = 0; b < nb; ++b) {
            int p = bonds[2 * b], q = bonds[2 * b + 1];
            size_t o = (size_t)r * nb + b;
            int same = get_bit(s, n, p) == get_bit(s, n, q);
            d += same ? 0.25 * Jz[b] : -0.25 * Jz[b];
            tgt[o] = 0;
            tgt_stab[o] = 0;
            tgt_flag[o] = 0;
            coef[2 * o] = 0.0;
            coef[2 * o + 1] = 0.0;
            if (same) continue;
            uint64_t sp = s ^ (1ull << (n - 1 - p)) ^ (1ull << (n - 1 - q));
            int32_t h;
            uint64_t rp = orc_rep(n, ng, perm, flip, sp, &h);
            int tc;
            int nt = stabiliser(n, ng, perm, flip, chi, rp, &tc);
            tgt[o] = rp;
            tgt_stab[o] = nt;
            tgt_flag[o] = tc ? 1 : 2; /* 1 = kept, 2 = dropped (target not in sector) */
            double amp = 0.5 * J[b] * sqrt((double)nt / (double)ns);
            coef[2 * o] = amp * chi[2 * h];
            coef[2 * o + 1] = amp * chi[2 * h + 1];
        }
        row_diag[r] = d;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================
 * Fermions in the occupation-number basis (sec. "Discussion": the method
 * carries over to fermionic Hamiltonians written in occupation numbers,
 * where a Fermi sign joins the representative and its symmetry).
 *
 * A configuration lists which orbitals are occupied, orbital i <-> bit
 * N-1-i, and stands for the ordered product of creation operators
 * c+_{i1} c+_{i2} ... c+_{ik} |0> with i1 < i2 < ... < ik.  A group element
 * moves orbital i to perm[i]; as an operator it maps c+_i to c+_{perm[i]},
 * so the image of a configuration is its permuted occupation pattern times
 * the sign of the permutation that sorts (perm[i1], ..., perm[ik]), i.e.
 * (-1)^(number of occupied pairs i < j with perm[i] > perm[j]).  Spin flip
 * is not part of a fermionic group here.
 *
 * Hamiltonian: every bond b = (p, q) carries a hopping -t_b (c+_p c_q +
 * c+_q c_p) and a density interaction V_b n_p n_q.  c+_p c_q on a
 * configuration with q occupied and p empty gives the configuration with
 * the two swapped, times (-1)^(occupied orbitals strictly between p and q).
 * ====================================================================== */

/* parity of the Fermi sign of the group element perm on configuration s */
int orc_fsign(int n, const int32_t *perm, uint64_t s)
{
    int inv = 0;
    for (int a = 0; a < n; ++a) {
        if (!get_bit(s, n, a)) continue;
        for (int b = a + 1; b < n; ++b)
            if (get_bit(s, n, b) && perm[a] > perm[b]) ++inv;
    }
    return inv & 1;
}

/* parity of the number of occupied orbitals strictly between p and q */
static int hop_parity(uint64_t s, int n, int p, int q)
{
    int lo = p < q ? p : q, hi = p < q ? q : p, c = 0;
    for (int i = lo + 1; i < hi; ++i) c += get_bit(s, n, i);
    return c & 1;
}

/* stabiliser size of s and whether chi(g) equals the Fermi sign of g on s for
   every g of the stabiliser (otherwise the symmetrised state vanishes) */
static int fstabiliser(int n, int ng, const int32_t *perm, const double *chi, uint64_t s, int *compatible)
{
    int cnt = 0;
    double re = 0.0, im = 0.0;
    for (int g = 0; g < ng; ++g) {
        const int32_t *pg = perm + (size_t)g * n;
        if (orc_act(n, pg, 0, s) == s) {
            const double sg = orc_fsign(n, pg, s) ? -1.0 : 1.0;
            ++cnt;
            re += sg * chi[2 * g];
            im += sg * chi[2 * g + 1];
        }
    }
    *compatible = fabs(re - cnt) < 1e-9 && fabs(im) < 1e-9;
    return cnt;
}

/* representative, first minimiser, stabiliser size and compatibility */
void orc_frep_many(int n, int ng, const int32_t *perm, const double *chi, int64_t m, const uint64_t *in,
                   uint64_t *rep_out, int32_t *g_out, int32_t *sign_out, int32_t *stab_out, uint8_t *compat_out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < m; ++k) {
        uint64_t best = ~0ull;
        int32_t bg = -1;
        for (int g = 0; g < ng; ++g) {
            uint64_t t = orc_act(n, perm + (size_t)g * n, 0, in[k]);
            if (t < best) { best = t; bg = g; }
        }
        int comp;
        int st = fstabiliser(n, ng, perm, chi, best, &comp);
        rep_out[k] = best;
        if (g_out) g_out[k] = bg;
        if (sign_out) sign_out[k] = orc_fsign(n, perm + (size_t)bg * n, in[k]);
        if (stab_out) stab_out[k] = st;
        if (compat_out) compat_out[k] = (uint8_t)comp;
    }
}

/* sector basis of n_part fermions: the orbit minima whose symmetrised state
   does not vanish, ascending, with their stabiliser sizes */
int64_t orc_fbasis(int n, int n_part, int ng, const int32_t *perm, const double *chi, uint64_t *states_out,
                   int32_t *stab_out, int64_t cap)
{
    uint64_t total = binom_u(n, n_part);
    int64_t dim = 0;
    if (total == 0) return 0;
    uint64_t s = unrank(n, n_part, 0);
    for (uint64_t r = 0; r < total; ++r) {
        int is_rep = 1;
        for (int g = 0; g < ng && is_rep; ++g)
            if (orc_act(n, perm + (size_t)g * n, 0, s) < s) is_rep = 0;
        if (is_rep) {
            int comp;
            int st = fstabiliser(n, ng, perm, chi, s, &comp);
            if (comp) {
                if (states_out && dim < cap) {
                    states_out[dim] = s;
                    stab_out[dim] = st;
                }
                ++dim;
            }
        }
        if (r + 1 < total) s = next_comb(s);
    }
    return dim;
}

/*
 * y = H x in the fermionic sector, scatter order: every source state sends
 * each hop to its target representative sigma~' = h sigma' (h the first
 * minimiser) with the element
 *   -t_b (-1)^hop (-1)^fsign(h, sigma') conj(chi(h)) sqrt(n_i / n_j),
 * the projection of the hopped configuration onto the target's symmetrised
 * state; the diagonal is sum_b V_b n_p n_q.  x, y complex interleaved.
 */
void orc_fapply(int n, int ng, const int32_t *perm, const double *chi, int nb, const int32_t *bonds,
                const double *t, const double *V, int64_t dim, const uint64_t *basis, const int32_t *stab,
                const double *x, double *y, int64_t *kept, int64_t *dropped)
{
    int64_t k = 0, dd = 0;
    memset(y, 0, sizeof(double) * (size_t)dim * 2);
    for (int64_t j = 0; j < dim; ++j) {
        uint64_t s = basis[j];
        double xr = x[2 * j], xi = x[2 * j + 1];
        double d = 0.0;
        for (int b = 0; b < nb; ++b) {
            int p = bonds[2 * b], q = bonds[2 * b + 1];
            if (get_bit(s, n, p) && get_bit(s, n, q)) d += V ? V[b] : 0.0;
        }
        y[2 * j] += d * xr;
        y[2 * j + 1] += d * xi;
        for (int b = 0; b < nb; ++b) {
            int p = bonds[2 * b], q = bonds[2 * b + 1];
            if (get_bit(s, n, p) == get_bit(s, n, q)) continue;
            uint64_t sp = s ^ (1ull << (n - 1 - p)) ^ (1ull << (n - 1 - q));
            uint64_t best = ~0ull;
            int32_t h = -1;
            for (int g = 0; g < ng; ++g) {
                uint64_t tt = orc_act(n, perm + (size_t)g * n, 0, sp);
                if (tt < best) { best = tt; h = g; }
            }
            int64_t i = find_state(dim, basis, best);
            if (i < 0) { ++dd; continue; }
            ++k;
            int par = hop_parity(s, n, p, q) ^ orc_fsign(n, perm + (size_t)h * n, sp);
            double amp = -t[b] * (par ? -1.0 : 1.0) * sqrt((double)stab[i] / (double)stab[j]);
            double cr = amp * chi[2 * h], ci = -amp * chi[2 * h + 1]; /* conj(chi(h)) */
            y[2 * i] += cr * xr - ci * xi;
            y[2 * i + 1] += cr * xi + ci * xr;
        }
    }
    if (kept) *kept = k;
    if (dropped) *dropped = dd;
}

/*
 * Rows of the Hermitian fermionic sector matrix for sampled representatives
 * (the conjugate of what each row sends in orc_fapply): row stabiliser and
 * compatibility, diagonal, and per bond the target representative, its
 * stabiliser size, flag (0 no hop, 1 kept, 2 target not in the sector) and
 * element -t_b (-1)^(hop + fsign) chi(h) sqrt(n_target / n_row).
 */
void orc_frow_terms(int n, int ng, const int32_t *perm, const double *chi, int nb, const int32_t *bonds,
                    const double *t, const double *V, int64_t nrows, const uint64_t *rows, int32_t *row_stab,
                    uint8_t *row_compat, double *row_diag, uint64_t *tgt, int32_t *tgt_stab, uint8_t *tgt_flag,
                    double *coef)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        uint64_t s = rows[r];
        int comp;
        int ns_ = fstabiliser(n, ng, perm, chi, s, &comp);
        row_stab[r] = ns_;
        row_compat[r] = (uint8_t)comp;
        double d = 0.0;
        for (int b = 0; b < nb; ++b) {
            int p = bonds[2 * b], q = bonds[2 * b + 1];
            size_t o = (size_t)r * nb + b;
            if (get_bit(s, n, p) && get_bit(s, n, q)) d += V ? V[b] : 0.0;
            tgt[o] = 0;
            tgt_stab[o] = 0;
            tgt_flag[o] = 0;
            coef[2 * o] = 0.0;
            coef[2 * o + 1] = 0.0;
            if (get_bit(s, n, p) == get_bit(s, n, q)) continue;
            uint64_t sp = s ^ (1ull << (n - 1 - p)) ^ (1ull << (n - 1 - q));
            uint64_t best = ~0ull;
            int32_t h = -1;
            for (int g = 0; g < ng; ++g) {
                uint64_t tt = orc_act(n, perm + (size_t)g * n, 0, sp);
                if (tt < best) { best = tt; h = g; }
            }
            int tc;
            int nt = fstabiliser(n, ng, perm, chi, best, &tc);
            tgt[o] = best;
            tgt_stab[o] = nt;
            tgt_flag[o] = tc ? 1 : 2;
            int par = hop_parity(s, n, p, q) ^ orc_fsign(n, perm + (size_t)h * n, sp);
            double amp = -t[b] * (par ? -1.0 : 1.0) * sqrt((double)nt / (double)ns_);
            coef[2 * o] = amp * chi[2 * h];
            coef[2 * o + 1] = amp * chi[2 * h + 1];
        }
        row_diag[r] = d;
    }
}
