// C ABI entry points (see include/ed.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "ed_internal.hpp"

extern "C" int ed_internal_unpack_states(const ed_basis *b, uint64_t *dev_out, void *stream);
extern "C" int ed_internal_apply_stats(const ed_basis *b, int64_t *kept, int64_t *dropped, void *stream);

using ed::set_error;

namespace {

int check_lattice(const ed_lattice_t *lat)
{
    if (!lat) return set_error(ED_ERR_ARG, "null lattice");
    if (lat->n_bonds > 256) return set_error(ED_ERR_UNSUPPORTED, "%d bonds exceed the 256-bond limit", lat->n_bonds);
    return ED_OK;
}

}  // namespace

extern "C" {

const char *ed_version(void) { return "ed-mi355x 0.1 (gfx950)"; }

const char *ed_last_error(void) { return ed::last_error(); }

int ed_validate(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep, int32_t n_up)
{
    int rc = check_lattice(lat);
    if (rc) return rc;
    return ed::validate_model(lat, grp, irrep, n_up, nullptr);
}

int ed_tables_create(const ed_lattice_t *lat, const ed_group_t *grp, ed_tables_t **out)
{
    if (!out) return set_error(ED_ERR_ARG, "null output handle");
    *out = nullptr;
    int rc = check_lattice(lat);
    if (rc) return rc;
    ed_tables *t = new (std::nothrow) ed_tables();
    if (!t) return set_error(ED_ERR_OOM, "host allocation");
    rc = ed::validate_model(lat, grp, nullptr, -1, &t->t);
    if (!rc) rc = ed::build_tables(lat, grp, t->t);
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    return ED_OK;
}

void ed_tables_free(ed_tables_t *t) { delete t; }

int ed_tables_info(const ed_tables_t *tt, ed_tables_info_t *info)
{
    if (!tt || !info) return set_error(ED_ERR_ARG, "null argument");
    const ed::Tables &t = tt->t;
    info->n_sites = t.N;
    info->n_sublat = t.ns;
    info->sub_bits = t.m;
    info->n_elems = t.ng;
    info->n_perms = t.nu;
    info->rep_entries = (int64_t)t.rep.size();
    info->sym_entries = (int64_t)t.sym_list.size();
    info->action_bytes = (int64_t)t.act.size() * (t.m <= 8 ? 1 : 2);   /* unchunked, one entry per substate */
    info->max_sym_len = t.max_sym;
    info->n_top = (int32_t)t.top_vals.size();
    return ED_OK;
}

int ed_tables_sublattice(const ed_tables_t *tt, int32_t X, uint32_t substate, uint32_t *rep_out, int32_t *sym_out,
                         int32_t cap, int32_t *n_sym)
{
    if (!tt || !rep_out || !n_sym) return set_error(ED_ERR_ARG, "null argument");
    const ed::Tables &t = tt->t;
    if (X < 0 || X >= t.ns || substate >= t.P) return set_error(ED_ERR_ARG, "sublattice or substate out of range");
    *rep_out = t.rep[(size_t)X * t.P + substate] & 0xFFFFu;
    uint32_t k0 = t.sym_off[(size_t)X * (t.P + 1) + substate], k1 = t.sym_off[(size_t)X * (t.P + 1) + substate + 1];
    *n_sym = (int32_t)(k1 - k0);
    for (uint32_t k = k0; k < k1 && (int32_t)(k - k0) < cap && sym_out; ++k) sym_out[k - k0] = t.sym_list[k];
    return ED_OK;
}

int ed_tables_find_rep(const ed_tables_t *tt, int64_t n, const uint64_t *states, uint64_t *rep_out, int32_t *g_out,
                       int32_t *n_cand_out)
{
    if (!tt || (n > 0 && !states) || n < 0) return set_error(ED_ERR_ARG, "bad arguments");
    const ed::Tables &t = tt->t;
    for (int64_t k = 0; k < n; ++k) {
        if (states[k] & ~t.full_mask()) return set_error(ED_ERR_ARG, "state %lld has bits above N", (long long)k);
        int g, nc;
        uint64_t r = t.find_rep(states[k], &g, &nc);
        if (rep_out) rep_out[k] = r;
        if (g_out) g_out[k] = g;
        if (n_cand_out) n_cand_out[k] = nc;
    }
    return ED_OK;
}

// Mean number of candidate symmetries of the host search (Alg. "Sublattice
// coding algorithm for finding the representative") over 2048 configurations
// with n_up up spins, drawn from a fixed splitmix64 stream.
static double sample_mean_candidates(const ed::Tables &t, int n_up)
{
    if (n_up <= 0 || n_up >= t.N) return 1.0;
    uint64_t z = 0x2545F4914F6CDD1Dull;
    auto next = [&z]() {
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        return x ^ (x >> 31);
    };
    const int n_samples = 2048;
    std::vector<int> sites(t.N);
    double total = 0.0;
    for (int k = 0; k < n_samples; ++k) {
        for (int i = 0; i < t.N; ++i) sites[i] = i;
        uint64_t s = 0;
        for (int i = 0; i < n_up; ++i) {   // partial Fisher-Yates: n_up distinct sites
            const int j = i + (int)(next() % (uint64_t)(t.N - i));
            std::swap(sites[i], sites[j]);
            s |= 1ull << (t.N - 1 - sites[i]);
        }
        int g = 0, nc = 0;
        (void)t.find_rep(s, &g, &nc);
        total += nc;
    }
    return total / n_samples;
}

// two-stage search by default from this mean candidate count on
static constexpr double kTwoStageMinCandidates = 3.0;

static int build_basis_common(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep, int32_t n_up,
                              const ed_tuning_t *tuning, uint32_t lds_reserve, void *stream, ed_basis_t **out,
                              bool fermion = false)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!out) return set_error(ED_ERR_ARG, "null output handle");
    *out = nullptr;
    int rc = check_lattice(lat);
    if (rc) return rc;
    if (!irrep || !irrep->chi) return set_error(ED_ERR_ARG, "null irrep");
    if (n_up < 0) return set_error(ED_ERR_ARG, "n_up=%d < 0", n_up);
    ed_basis *b = new (std::nothrow) ed_basis();
    if (!b) return set_error(ED_ERR_OOM, "host allocation");
    rc = ed::validate_model(lat, grp, irrep, n_up, &b->t);
    if (!rc) rc = ed::build_tables(lat, grp, b->t);
    if (rc) {
        delete b;
        return rc;
    }
    if (tuning) b->tuning = *tuning;
    b->lds_reserve = lds_reserve;
    if (fermion) {
        for (int g = 0; g < b->t.ng; ++g)
            if (b->t.flip[g]) {
                delete b;
                return set_error(ED_ERR_UNSUPPORTED, "element %d of a fermionic group carries a spin flip", g);
            }
        const int eb = b->tuning.table_entry_bytes;
        if (b->tuning.index_mode != 0 || (eb != 0 && eb != 2 && eb != 4)) {
            delete b;
            return set_error(ED_ERR_UNSUPPORTED, "fermionic bases use the hash-slot index and 2- or 4-byte table entries");
        }
        const int m = b->t.m, ns = b->t.ns;   // read before any delete of b
        if (eb == 2 && (m > 12 || ns > 8)) {
            delete b;
            return set_error(ED_ERR_UNSUPPORTED,
                             "2-byte fermionic table entries need blocks of at most 12 orbitals and at most 8 "
                             "sublattices (%d, %d)", m, ns);
        }
        if (m > 16) {
            delete b;
            return set_error(ED_ERR_UNSUPPORTED, "fermionic blocks hold at most 16 orbitals (%d)", m);
        }
        b->fermion = 1;
    }
    if (b->tuning.block_threads && (b->tuning.block_threads < 64 || b->tuning.block_threads > 1024 ||
                                    b->tuning.block_threads % 64)) {
        delete b;
        return set_error(ED_ERR_ARG, "block_threads must be a multiple of 64 in [64, 1024]");
    }
    if (b->tuning.index_mode < 0 || b->tuning.index_mode > 1 || b->tuning.chunk_bits < 0 ||
        b->tuning.chunk_bits > 16 || b->tuning.hash_load_pct < 0 || b->tuning.hash_load_pct > 90 ||
        (b->tuning.table_entry_bytes != 0 && b->tuning.table_entry_bytes != 1 && b->tuning.table_entry_bytes != 2 &&
         b->tuning.table_entry_bytes != 4) ||
        b->tuning.search_mode < 0 || b->tuning.search_mode > ED_SEARCH_TWO_STAGE ||
        (b->tuning.lanes_per_row != 0 && b->tuning.lanes_per_row != 1 && b->tuning.lanes_per_row != 2 &&
         b->tuning.lanes_per_row != 4) ||
        (b->tuning.lanczos_direct != 0 && b->tuning.lanczos_direct != 1)) {
        delete b;
        return set_error(ED_ERR_ARG, "tuning fields out of range");
    }
    const ed::Tables &t = b->t;
    b->n_up = n_up;
    (void)hipGetDevice(&b->device);
    b->chi_host.assign(irrep->chi, irrep->chi + 2 * (size_t)t.ng);
    bool cplx = false, trivial = true;
    for (int g = 0; g < t.ng; ++g) {
        if (std::fabs(b->chi_host[2 * g + 1]) > 1e-14) cplx = true;
        if (std::fabs(b->chi_host[2 * g] - 1.0) > 1e-12 || std::fabs(b->chi_host[2 * g + 1]) > 1e-12) trivial = false;
    }
    b->divs = ed::divisors_of((uint32_t)t.ng);
    if (b->divs.size() > 255) {
        const int ng = t.ng;   // t lives in *b
        delete b;
        return set_error(ED_ERR_UNSUPPORTED, "|G|=%d has more than 255 divisors", ng);
    }
    ed::DevModel &dm = b->dm;
    dm.N = t.N;
    dm.ns = t.ns;
    dm.m = t.m;
    dm.ng = t.ng;
    dm.nu = t.nu;
    dm.nb = t.nb;
    dm.P = t.P;
    dm.is_complex = cplx ? 1 : 0;
    dm.trivial_irrep = trivial ? 1 : 0;
    dm.fermion = b->fermion;
    dm.n_div = (int)b->divs.size();
    b->mean_candidates = sample_mean_candidates(t, n_up);
    const bool two_stage_ok = t.ns >= 2 && t.ns <= 4;
    if (b->tuning.search_mode == ED_SEARCH_TWO_STAGE && !two_stage_ok) {
        const int ns = t.ns;   // t lives in *b
        delete b;
        return set_error(ED_ERR_UNSUPPORTED, "the two-stage search needs 2 to 4 sublattices (%d)", ns);
    }
    b->staged = two_stage_ok && (b->tuning.search_mode == ED_SEARCH_TWO_STAGE ||
                                 (b->tuning.search_mode == 0 && b->mean_candidates >= kTwoStageMinCandidates));
    dm.staged = b->staged;
    rc = ed::launch_basis_build(b, stream);
    if (rc) {
        ed_free_basis(b);
        return rc;
    }
    b->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = b;
    return ED_OK;
}

int ed_build_basis(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep, int32_t n_up,
                   const ed_tuning_t *tuning, void *stream, ed_basis_t **out)
{
    return build_basis_common(lat, grp, irrep, n_up, tuning, 0, stream, out);
}

int ed_build_basis_fermions(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep,
                            int32_t n_particles, const ed_tuning_t *tuning, void *stream, ed_basis_t **out)
{
    return build_basis_common(lat, grp, irrep, n_particles, tuning, 0, stream, out, true);
}

void ed_free_basis(ed_basis_t *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    ed::free_lanczos_workspace(b);
    for (void *p : b->allocs) (void)hipFree(p);
    delete b;
}

int64_t ed_basis_dim(const ed_basis_t *b) { return b ? b->db.dim : -1; }

int ed_basis_is_complex(const ed_basis_t *b) { return b ? b->dm.is_complex : 0; }

int ed_basis_info(const ed_basis_t *b, ed_basis_info_t *info)
{
    if (!b || !info) return set_error(ED_ERR_ARG, "null argument");
    memset(info, 0, sizeof *info);
    info->dim = b->db.dim;
    info->is_complex = b->dm.is_complex;
    info->n_sites = b->t.N;
    info->n_up = b->n_up;
    info->n_sublat = b->t.ns;
    info->sub_bits = b->t.m;
    info->n_elems = b->t.ng;
    info->n_bonds = b->t.nb;
    info->index_mode = b->db.index_mode;
    info->limits_bits = b->db.key_bits;
    info->n_keys = b->db.n_keys;
    info->n_slots = b->n_slots;
    info->chunk_bits = b->dm.chunk_bits;
    info->table_entry_bytes = b->dm.act_bytes;
    info->lds_bytes = (int32_t)b->dm.lds_total;
    info->device_bytes = b->device_bytes;
    info->build_ms = b->build_ms;
    info->search_mode = b->staged ? ED_SEARCH_TWO_STAGE : ED_SEARCH_ONE_STAGE;
    info->mean_candidates = b->mean_candidates;
    info->is_fermion = b->fermion;
    return ED_OK;
}

int ed_basis_copy_states(const ed_basis_t *b, uint64_t *host_out, void *stream)
{
    if (!b || (!host_out && b->db.dim > 0)) return set_error(ED_ERR_ARG, "null argument");
    if (b->db.dim == 0) return ED_OK;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(host_out, b->db.states, (size_t)b->db.dim * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "copy states: %s", hipGetErrorString(e));
    for (int64_t i = 0; i < b->db.dim; ++i) host_out[i] &= ed::kStateMask;
    return ED_OK;
}

int ed_basis_copy_states_device(const ed_basis_t *b, uint64_t *dev_out, void *stream)
{
    if (!b || (!dev_out && b->db.dim > 0)) return set_error(ED_ERR_ARG, "null argument");
    return ed_internal_unpack_states(b, dev_out, stream);
}

int ed_basis_copy_norms(const ed_basis_t *b, uint16_t *host_out, void *stream)
{
    if (!b || (!host_out && b->db.dim > 0)) return set_error(ED_ERR_ARG, "null argument");
    const int64_t D = b->db.dim;
    if (D == 0) return ED_OK;
    uint64_t *tmp = new (std::nothrow) uint64_t[(size_t)D];
    if (!tmp) return set_error(ED_ERR_OOM, "host buffer");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(tmp, b->db.states, (size_t)D * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete[] tmp;
        return set_error(ED_ERR_HIP, "copy norms: %s", hipGetErrorString(e));
    }
    for (int64_t i = 0; i < D; ++i) host_out[i] = (uint16_t)b->divs[tmp[i] >> ed::kNormShift];
    delete[] tmp;
    return ED_OK;
}

int ed_apply_H(const ed_basis_t *b, const double *J, const void *x_dev, void *y_dev, void *stream)
{
    return ed_apply_H_xxz(b, J, nullptr, x_dev, y_dev, stream);
}

int ed_apply_H_timed(const ed_basis_t *b, const double *J, const double *Jz, const void *x_dev, void *y_dev,
                     int32_t reps, double *pack_ms, double *kernel_ms, void *stream)
{
    if (!b || !J || !pack_ms || !kernel_ms || (b->db.dim > 0 && (!x_dev || !y_dev)))
        return set_error(ED_ERR_ARG, "null argument");
    if (x_dev == y_dev && b->db.dim > 0) return set_error(ED_ERR_ARG, "x and y must be distinct");
    if (reps < 1 || reps > 1000) return set_error(ED_ERR_ARG, "reps = %d (1..1000)", reps);
    return ed::launch_apply_timed(b, J, Jz, x_dev, y_dev, reps, pack_ms, kernel_ms, stream);
}

static int no_fermions(const ed_basis_t *b)
{
    if (b && b->fermion) return set_error(ED_ERR_ARG, "the basis holds fermions: use the *_fermions entry points");
    return ED_OK;
}

int ed_apply_H_xxz(const ed_basis_t *b, const double *Jxy, const double *Jz, const void *x_dev, void *y_dev,
                   void *stream)
{
    if (!b) return set_error(ED_ERR_ARG, "null basis");
    if (no_fermions(b)) return ED_ERR_ARG;
    if (b->db.dim > 0 && (!x_dev || !y_dev)) return set_error(ED_ERR_ARG, "null vector");
    if (b->db.dim > 0 && x_dev == y_dev) return set_error(ED_ERR_ARG, "x and y must be distinct");
    return ed::launch_apply(b, Jxy, Jz, x_dev, y_dev, stream, 0, nullptr);
}

int ed_apply_H_stats(const ed_basis_t *bc, int64_t *n_diag, int64_t *n_kept, int64_t *n_dropped, void *stream)
{
    if (!bc) return set_error(ED_ERR_ARG, "null basis");
    ed_basis *b = const_cast<ed_basis *>(bc);
    if (!b->stats_valid) {
        int rc = ed_internal_apply_stats(b, &b->n_kept, &b->n_dropped, stream);
        if (rc) return rc;
        b->stats_valid = 1;
    }
    if (n_diag) *n_diag = b->db.dim;
    if (n_kept) *n_kept = b->n_kept;
    if (n_dropped) *n_dropped = b->n_dropped;
    return ED_OK;
}

int ed_lanczos(const ed_basis_t *b, const double *J, const void *v0_dev, int32_t n_steps, double *alpha_host,
               double *beta_host, int32_t *n_done, void *psi0_dev, void *stream)
{
    return ed_lanczos_xxz(b, J, nullptr, v0_dev, n_steps, alpha_host, beta_host, n_done, psi0_dev, stream);
}

int ed_apply_H_fermions(const ed_basis_t *b, const double *t, const double *V, const void *x_dev, void *y_dev,
                        void *stream)
{
    if (!b) return set_error(ED_ERR_ARG, "null basis");
    if (!b->fermion) return set_error(ED_ERR_ARG, "the basis holds spins: use ed_apply_H");
    if (b->db.dim > 0 && (!x_dev || !y_dev)) return set_error(ED_ERR_ARG, "null vector");
    if (b->db.dim > 0 && x_dev == y_dev) return set_error(ED_ERR_ARG, "x and y must be distinct");
    return ed::launch_apply(b, t, V, x_dev, y_dev, stream, 0, nullptr);
}

static int lanczos_common(const ed_basis_t *b, const double *J, const double *Jz, const void *v0_dev,
                          int32_t n_steps, double *alpha_host, double *beta_host, int32_t *n_done, void *psi0_dev,
                          void *stream)
{
    if (!b || !n_done) return set_error(ED_ERR_ARG, "null argument");
    if (n_steps < 0) return set_error(ED_ERR_ARG, "n_steps < 0");
    if (n_steps > 0 && (!alpha_host || !beta_host)) return set_error(ED_ERR_ARG, "null alpha/beta");
    if (b->db.dim > 0 && !v0_dev) return set_error(ED_ERR_ARG, "null start vector");
    int nd = 0;
    int rc = ed::run_lanczos(b, J, Jz, v0_dev, n_steps, alpha_host, beta_host, &nd, psi0_dev, stream);
    *n_done = nd;
    return rc;
}

int ed_lanczos_fermions(const ed_basis_t *b, const double *t, const double *V, const void *v0_dev, int32_t n_steps,
                        double *alpha_host, double *beta_host, int32_t *n_done, void *psi0_dev, void *stream)
{
    if (b && !b->fermion) return set_error(ED_ERR_ARG, "the basis holds spins: use ed_lanczos");
    return lanczos_common(b, t, V, v0_dev, n_steps, alpha_host, beta_host, n_done, psi0_dev, stream);
}

int ed_lanczos_xxz(const ed_basis_t *b, const double *Jxy, const double *Jz, const void *v0_dev, int32_t n_steps,
                   double *alpha_host, double *beta_host, int32_t *n_done, void *psi0_dev, void *stream)
{
    if (no_fermions(b)) return ED_ERR_ARG;
    return lanczos_common(b, Jxy, Jz, v0_dev, n_steps, alpha_host, beta_host, n_done, psi0_dev, stream);
}

static int backward_common(const ed_basis_t *b, const double *J, const void *x_dev, const void *gy_dev, void *gx_dev,
                           double *gJ_host, void *stream, bool static_scratch)
{
    if (!b) return set_error(ED_ERR_ARG, "null basis");
    if (b->fermion) return set_error(ED_ERR_UNSUPPORTED, "the adjoint covers spin bases");
    if (b->db.dim > 0 && !gy_dev) return set_error(ED_ERR_ARG, "null gy");
    if (gx_dev && gx_dev == gy_dev) return set_error(ED_ERR_ARG, "gx and gy must be distinct");
    if (gJ_host && b->db.dim > 0 && !x_dev) return set_error(ED_ERR_ARG, "null x");
    if (gx_dev && gJ_host && gx_dev == x_dev) return set_error(ED_ERR_ARG, "gx and x must be distinct");
    // both products of a real sector in one pass (one search and one slot line per term)
    if (gx_dev && gJ_host && !static_scratch && ed::backward_fusable(b))
        return ed::launch_backward_J(b, J, x_dev, gy_dev, gJ_host, stream, false, gx_dev);
    if (gx_dev) {
        int rc = ed::launch_apply(b, J, nullptr, gy_dev, gx_dev, stream, 0, nullptr);
        if (rc) return rc;
    }
    if (gJ_host) {
        int rc = ed::launch_backward_J(b, J, x_dev, gy_dev, gJ_host, stream, static_scratch);
        if (rc) return rc;
    }
    return ED_OK;
}

int ed_apply_H_backward(const ed_basis_t *b, const double *J, const void *x_dev, const void *gy_dev, void *gx_dev,
                        double *gJ_host, void *stream)
{
    return backward_common(b, J, x_dev, gy_dev, gx_dev, gJ_host, stream, false);
}

int ed_apply_H_backward_noalloc(const ed_basis_t *b, const double *J, const void *x_dev, const void *gy_dev,
                                void *gx_dev, double *gJ_host, void *stream)
{
    return backward_common(b, J, x_dev, gy_dev, gx_dev, gJ_host, stream, true);
}

// Symmetric tridiagonal eigenproblem: eigenvalues by Sturm-sequence
// bisection (the count of negative pivots of T - x I equals the number of
// eigenvalues below x), the lowest eigenvector by inverse iteration.
static int sturm_count(int m, const double *a, const double *b2, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (int k = 0; k < m; ++k) {
        double off = k > 0 ? b2[k - 1] / q : 0.0;
        q = a[k] - x - off;
        if (q == 0.0) q = -DBL_MIN * 16;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

/* ---- batched sectors ---------------------------------------------------- */

static constexpr size_t kChiLdsMaxBytes = 32768;   // largest character table staged in LDS

int ed_build_multi(const ed_lattice_t *lat, const ed_group_t *grp, int32_t n_sectors, const ed_irrep_t *irreps,
                   int32_t n_up, const ed_tuning_t *tuning, void *stream, ed_multi_t **out)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!out) return set_error(ED_ERR_ARG, "null output handle");
    *out = nullptr;
    if (!grp || !irreps) return set_error(ED_ERR_ARG, "null argument");
    if (n_sectors < 1 || n_sectors > 64) return set_error(ED_ERR_UNSUPPORTED, "%d sectors (1..64 supported)", n_sectors);
    int rc = check_lattice(lat);
    if (rc) return rc;
    for (int k = 0; k < n_sectors; ++k) {
        if (!irreps[k].chi) return set_error(ED_ERR_ARG, "null character table of sector %d", k);
        rc = ed::validate_model(lat, grp, &irreps[k], n_up, nullptr);
        if (rc) return rc;
    }
    const int ng = grp->n_elems;
    std::vector<double> ones((size_t)ng * 2, 0.0);
    for (int g = 0; g < ng; ++g) ones[2 * g] = 1.0;
    ed_irrep_t trivial{ones.data()};
    ed_tuning_t tn{};
    if (tuning) tn = *tuning;
    tn.index_mode = 0;                          // shared hash-slot index (row index | mask in the value)
    if (tn.table_entry_bytes == 1) tn.table_entry_bytes = 0;
    if (tn.table_entry_bytes == 0) tn.table_entry_bytes = lat->n_sublat > 0 && lat->n_sites / lat->n_sublat <= 12 ? 2 : 4;
    ed_multi *mb = new (std::nothrow) ed_multi();
    if (!mb) return set_error(ED_ERR_OOM, "host allocation");
    mb->K = n_sectors;
    // the character table [ng][K] is staged in LDS beside the lookup tables
    // when it is small; a large one (big groups, many sectors) is read from
    // HBM through the caches instead
    const size_t chi_bytes = (size_t)ng * n_sectors * 16;
    mb->chi_in_lds = chi_bytes <= kChiLdsMaxBytes;
    if (n_sectors > 32 && !mb->chi_in_lds) {
        delete mb;
        return set_error(ED_ERR_UNSUPPORTED, "more than 32 sectors need their character table (%zu bytes) in LDS",
                         chi_bytes);
    }
    // a table too large for LDS whose characters are all +1 or -1 (the real
    // one-dimensional irreps) is staged as one sign bit per sector instead
    if (!mb->chi_in_lds && n_sectors <= 8) {
        bool signs = true;
        for (int k = 0; k < n_sectors && signs; ++k)
            for (int g = 0; g < ng && signs; ++g) {
                const double re = irreps[k].chi[2 * g], im = irreps[k].chi[2 * g + 1];
                signs = (re == 1.0 || re == -1.0) && im == 0.0;
            }
        mb->chi_signs = signs;
    }
    const uint32_t reserve = mb->chi_in_lds ? (uint32_t)((chi_bytes + 15) & ~(size_t)15)
                                            : (mb->chi_signs ? (uint32_t)((ng + 15) & ~15) : 0u);
    rc = build_basis_common(lat, grp, &trivial, n_up, &tn, reserve, stream, &mb->base);
    if (rc) {
        delete mb;
        return rc;
    }
    mb->chi_host.resize((size_t)n_sectors * ng * 2);
    for (int k = 0; k < n_sectors; ++k)
        std::copy(irreps[k].chi, irreps[k].chi + 2 * (size_t)ng, mb->chi_host.begin() + (size_t)k * ng * 2);
    rc = ed::multi_setup(mb, stream);
    if (rc) {
        ed_free_multi(mb);
        return rc;
    }
    mb->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = mb;
    return ED_OK;
}

void ed_free_multi(ed_multi_t *mb)
{
    if (!mb) return;
    (void)hipDeviceSynchronize();
    ed::multi_free_workspace(mb);
    ed_free_basis(mb->base);
    delete mb;
}

int ed_multi_info(const ed_multi_t *mb, ed_multi_info_t *info)
{
    if (!mb || !info) return set_error(ED_ERR_ARG, "null argument");
    memset(info, 0, sizeof *info);
    const ed_basis *b = mb->base;
    info->dim = b->db.dim;
    info->n_sectors = mb->K;
    info->n_sites = b->t.N;
    info->n_up = b->n_up;
    info->n_sublat = b->t.ns;
    info->n_elems = b->t.ng;
    info->n_bonds = b->t.nb;
    info->chunk_bits = b->dm.chunk_bits;
    info->table_entry_bytes = b->dm.act_bytes;
    info->lds_bytes = (int32_t)(mb->lds_chi_off + (mb->chi_in_lds ? (uint32_t)b->t.ng * mb->K * 16
                                                                   : (mb->chi_signs ? ((uint32_t)b->t.ng + 15u) & ~15u : 0u)));
    info->chi_in_lds = mb->chi_in_lds ? 1 : 0;
    info->chi_signs = mb->chi_signs ? 1 : 0;
    info->n_slots = b->n_slots;
    info->device_bytes = b->device_bytes;
    info->build_ms = mb->build_ms;
    info->lanes_per_row = ed::multi_lanes_per_row(mb);
    return ED_OK;
}

int ed_multi_sector_dims(const ed_multi_t *mb, int64_t *dims_host)
{
    if (!mb || !dims_host) return set_error(ED_ERR_ARG, "null argument");
    for (int k = 0; k < mb->K; ++k) dims_host[k] = mb->dims[k];
    return ED_OK;
}

int ed_multi_copy_states(const ed_multi_t *mb, uint64_t *host_out, void *stream)
{
    if (!mb) return set_error(ED_ERR_ARG, "null argument");
    return ed_basis_copy_states(mb->base, host_out, stream);
}

int ed_multi_copy_masks(const ed_multi_t *mb, uint64_t *host_out, void *stream)
{
    if (!mb || (!host_out && mb->base->db.dim > 0)) return set_error(ED_ERR_ARG, "null argument");
    const int64_t D = mb->base->db.dim;
    if (D == 0) return ED_OK;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(host_out, mb->masks, (size_t)D * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_error(ED_ERR_HIP, "copy masks: %s", hipGetErrorString(e));
    return ED_OK;
}

int ed_apply_H_batched(const ed_multi_t *mb, const double *J, const void *x_dev, void *y_dev, void *stream)
{
    if (!mb) return set_error(ED_ERR_ARG, "null basis");
    if (mb->base->db.dim > 0 && (!x_dev || !y_dev)) return set_error(ED_ERR_ARG, "null vector");
    if (mb->base->db.dim > 0 && x_dev == y_dev) return set_error(ED_ERR_ARG, "x and y must be distinct");
    return ed::multi_apply(mb, J, x_dev, y_dev, stream);
}

int ed_apply_H_batched_stats(const ed_multi_t *mb, int64_t *n_terms, int64_t *n_shared_terms, void *stream)
{
    if (!mb || !n_terms || !n_shared_terms) return set_error(ED_ERR_ARG, "null argument");
    return ed::multi_stats(mb, n_terms, n_shared_terms, stream);
}

int ed_lanczos_batched(const ed_multi_t *mbc, const double *J, const void *v0_dev, int32_t n_steps,
                       double *alpha_host, double *beta_host, int32_t *n_done, int32_t flags, void *stream)
{
    if (!mbc || !n_done || (n_steps > 0 && (!alpha_host || !beta_host)))
        return set_error(ED_ERR_ARG, "null argument");
    if (n_steps < 0) return set_error(ED_ERR_ARG, "n_steps < 0");
    if (mbc->base->db.dim > 0 && !v0_dev) return set_error(ED_ERR_ARG, "null start vector");
    if (flags & ~ED_LANCZOS_NO_GRAPH) return set_error(ED_ERR_ARG, "unknown flags 0x%x", flags);
    ed_multi *mb = const_cast<ed_multi *>(mbc);
    std::vector<int> nd(mb->K, 0);
    const int rc = ed::multi_lanczos(mb, J, v0_dev, n_steps, alpha_host, beta_host, nd.data(),
                                     (flags & ED_LANCZOS_NO_GRAPH) ? 0 : 1, stream);
    for (int k = 0; k < mb->K; ++k) n_done[k] = nd[k];
    return rc;
}

int ed_tridiag_eigh(int32_t m, const double *alpha, const double *beta, double *evals, double *evec0)
{
    if (m < 0 || (m > 0 && (!alpha || !evals))) return set_error(ED_ERR_ARG, "bad arguments");
    if (m > 1 && !beta) return set_error(ED_ERR_ARG, "null beta");
    if (m == 0) return ED_OK;
    std::vector<double> b2(std::max(m - 1, 1), 0.0);
    double lo = alpha[0], hi = alpha[0];
    for (int k = 0; k < m; ++k) {
        double r = (k > 0 ? std::fabs(beta[k - 1]) : 0.0) + (k < m - 1 ? std::fabs(beta[k]) : 0.0);
        lo = std::min(lo, alpha[k] - r);
        hi = std::max(hi, alpha[k] + r);
        if (k < m - 1) b2[k] = beta[k] * beta[k];
    }
    const double span = std::max(hi - lo, std::max(std::fabs(hi), std::fabs(lo)) * DBL_EPSILON) + DBL_MIN;
    lo -= 1e-12 * span;
    hi += 1e-12 * span;
    for (int k = 0; k < m; ++k) {
        double a = lo, c = hi;   // count(a) <= k < count(c)
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (a + c);
            if (mid <= a || mid >= c) break;
            if (sturm_count(m, alpha, b2.data(), mid) > k) c = mid; else a = mid;
        }
        evals[k] = 0.5 * (a + c);
    }
    if (evec0) {
        // inverse iteration on (T - lambda0 I) with a pivoting tridiagonal solve
        const double lam = evals[0];
        std::vector<double> v(m), rhs(m);
        uint64_t seed = 0x9E3779B97F4A7C15ull;
        for (int k = 0; k < m; ++k) {
            seed = seed * 6364136223846793005ull + 1442695040888963407ull;
            v[k] = 0.5 + (double)(seed >> 11) * (1.0 / 9007199254740992.0);
        }
        const double pert = DBL_EPSILON * span;
        for (int iter = 0; iter < 4; ++iter) {
            rhs = v;
            // Gaussian elimination with partial pivoting on the tridiagonal
            // matrix (sub = super = beta, diag = alpha - lam); row k may pick up
            // a second super-diagonal after a swap.
            std::vector<double> d(m), du(m, 0.0), du2(m, 0.0), dl(m, 0.0);
            for (int k = 0; k < m; ++k) d[k] = alpha[k] - lam;
            for (int k = 0; k < m - 1; ++k) {
                du[k] = beta[k];
                dl[k] = beta[k];
            }
            for (int k = 0; k < m - 1; ++k) {
                if (std::fabs(d[k]) >= std::fabs(dl[k])) {
                    if (d[k] == 0.0) d[k] = pert;
                    double f = dl[k] / d[k];
                    d[k + 1] -= f * du[k];
                    rhs[k + 1] -= f * rhs[k];
                    dl[k] = 0.0;
                } else {
                    double f = d[k] / dl[k];
                    std::swap(rhs[k], rhs[k + 1]);
                    rhs[k + 1] -= f * rhs[k];
                    d[k] = dl[k];
                    double t = du[k];
                    du[k] = d[k + 1];
                    d[k + 1] = t - f * d[k + 1];
                    if (k < m - 2) {
                        du2[k] = du[k + 1];
                        du[k + 1] = -f * du[k + 1];
                    }
                }
            }
            if (d[m - 1] == 0.0) d[m - 1] = pert;
            for (int k = m - 1; k >= 0; --k) {
                double s = rhs[k];
                if (k + 1 < m) s -= du[k] * v[k + 1];
                if (k + 2 < m) s -= du2[k] * v[k + 2];
                v[k] = s / d[k];
            }
            double nrm = 0.0;
            for (double x : v) nrm += x * x;
            nrm = std::sqrt(nrm);
            if (!(nrm > 0.0) || !std::isfinite(nrm)) return set_error(ED_ERR_ARG, "inverse iteration failed");
            for (double &x : v) x /= nrm;
        }
        for (int k = 0; k < m; ++k) evec0[k] = v[k];
    }
    return ED_OK;
}

}  // extern "C"
