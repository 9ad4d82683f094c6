// Internal declarations shared by the host code and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ed.h"

namespace ed {

// Packed basis entry: bits [0, 56) hold the state, bits [56, 64) the index of
// |Stab sigma| in the sorted list of divisors of |G|.
constexpr int kNormShift = 56;
constexpr uint64_t kStateMask = (1ull << kNormShift) - 1ull;
constexpr int kMaxSites = 56;
constexpr int kMaxSubBits = 16;

int set_error(int code, const char *fmt, ...);

// Host-side model and sublattice-coding tables (Alg. "Preparation of lookup
// tables for sublattice coding algorithm").
struct Tables {
    int N = 0;           // sites
    int ns = 0;          // sublattices
    int m = 0;           // sites per sublattice
    int ng = 0;          // group elements
    int nu = 0;          // distinct site permutations
    uint32_t P = 0;      // 2^m substates
    std::vector<int32_t> perm;      // [ng][N]
    std::vector<uint8_t> flip;      // [ng]
    std::vector<uint16_t> g_u;      // [ng] -> distinct permutation
    std::vector<int32_t> u_perm;    // [nu][N]
    std::vector<uint8_t> u_tgt;     // [nu][ns]: block that block X is mapped onto
    // rep[X][s] = (rank of Rep_X(s) among top-block values) << 16 | Rep_X(s)
    std::vector<uint32_t> rep;      // [ns][P]
    std::vector<uint32_t> sym_off;  // [ns][P + 1] offsets into sym_list
    std::vector<uint16_t> sym_list; // group indices, ascending within a list
    std::vector<uint16_t> act;      // [nu][ns][P]: image pattern on block u_tgt[u][X]
    std::vector<uint16_t> top_vals; // ascending values t with Rep_0(t) == t
    int max_sym = 0;
    // bonds (validated separately when present)
    std::vector<int32_t> bonds;     // [nb][2]
    std::vector<int32_t> bond_orbit;// [nb]
    int nb = 0;

    uint64_t full_mask() const { return N >= 64 ? ~0ull : ((1ull << N) - 1ull); }
    int block_shift(int X) const { return N - (X + 1) * m; }
    uint64_t apply(int g, uint64_t s) const;       // group element via tables
    uint64_t find_rep(uint64_t s, int *g_out, int *n_cand) const;  // host Alg. 2
};

// Validation and table construction (ed_tables.cpp).
int validate_model(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep, int n_up,
                   Tables *tab_or_null);
int build_tables(const ed_lattice_t *lat, const ed_group_t *grp, Tables &t);
std::vector<uint32_t> divisors_of(uint32_t n);

// Device-side description of the tables handed to kernels.  All tables live
// in one device blob whose layout is the LDS image (byte offsets below); the
// symmetry-action table is last so that it can stay in global memory when it
// does not fit the LDS budget.
struct DevModel {
    int N, ns, m, ng, nu, nb;
    uint32_t P;
    int is_complex;
    int trivial_irrep;
    int n_div;
    const char *blob;          // device blob
    uint32_t lds_rep, lds_sym_off, lds_sym_list, lds_act, lds_u_shift, lds_g_u, lds_g_flip, lds_chi,
        lds_div, lds_bonds, lds_total;
    int act_in_lds;
};

struct DevBasis {
    int64_t dim;
    const uint64_t *states;    // packed entries [dim]
    const uint32_t *limits;    // [n_keys + 1]
    int64_t n_keys;
    int key_bits;              // q
    int key_shift;             // N - m - q
};

}  // namespace ed

struct ed_tables {
    ed::Tables t;
};

struct ed_basis {
    ed::Tables t;
    ed::DevModel dm{};
    ed::DevBasis db{};
    int n_up = 0;
    int device = 0;
    int64_t device_bytes = 0;
    double build_ms = 0.0;
    ed_tuning_t tuning{};
    std::vector<void *> allocs;
    std::vector<double> chi_host;  // [ng][2]
    std::vector<uint32_t> divs;
    int stats_valid = 0;
    int64_t n_kept = 0, n_dropped = 0;
    int grid_blocks = 0;
    std::vector<double> J_cache;   // couplings currently written into the blob
};

namespace ed {
// Kernel launchers (ed_kernels.hip)
int launch_basis_build(ed_basis *b, void *stream);
int launch_apply(const ed_basis *b, const double *J, const void *x, void *y, void *stream, int stats_mode,
                 unsigned long long *stats_dev);
int launch_backward_J(const ed_basis *b, const double *J, const void *x, const void *gy, double *gJ_host,
                      void *stream);
int run_lanczos(const ed_basis *b, const double *J, const void *v0, int n_steps, double *alpha, double *beta,
                int *n_done, void *psi0, void *stream);
int device_alloc(ed_basis *b, void **p, size_t bytes);
const char *last_error();
}  // namespace ed
