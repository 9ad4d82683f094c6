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
// in one device blob whose layout is the LDS image (byte offsets below); every
// block of the H.v and basis kernels stages the whole image in LDS.
//   rep  : uint32 [ns][P]  low 16 bits Rep_X(s), high 16 bits offset of Sym_X(s)
//   sym  : uint32 lists [count, e_1, ..., e_count], ascending g, with
//          e = g | distinct-permutation index << 16 | flip << 31
//   act  : AT [nu][ns][nc][2^c]  image pattern of one c-bit chunk of a substate;
//          2- and 4-byte entries of chunk 0 also hold the target block index
//   shift: uint8 [nu][ns]  bit position of the image block
//   chi  : double [ng] (real sectors) or double2 [ng] (complex sectors)
//   div  : double [n_div] sqrt of the divisors of |G|, then their inverses
//   bonds: {uint64 mask, double J/2} [nb]
//   rank : uint16 [P]      rank of a top-block value (Limits index only)
// Fermionic bases (orbital occupations) also stage
//   between: uint64 [nb]   orbitals strictly between the two of each bond
//   g_u    : uint16 [ng]   distinct-permutation index of every element
// and their 4-byte action entries carry, in bit 31, the parity of the
// orbital pairs of the chunk whose order the permutation reverses.
struct DevModel {
    int N, ns, m, ng, nu, nb;
    uint32_t P;
    int is_complex;
    int trivial_irrep;
    int n_div;
    int chunk_bits, n_chunks;
    int act_bytes;             // 1, 2 or 4 bytes per action-table entry
    int staged;                // the pos1 table is staged: two-stage search available
    int fermion;               // occupation-number basis of fermions
    const char *blob;
    uint32_t off_rep, off_sym, off_act, off_shift, off_chi, off_div, off_divval, off_bonds, off_rank,
        off_pos1, off_between, off_gu, lds_total;
};

struct DevBasis {
    int64_t dim;
    const uint64_t *states;    // packed entries [dim]
    int index_mode;            // 0 hash slots, 1 Limits + binary search
    // Limits index (Alg. "Parallel matrix-vector multiply", receiving step)
    const uint32_t *limits;    // [n_keys + 1]
    int64_t n_keys;
    int key_bits;              // q
    int key_shift;             // N - m - q
    // hash-slot index: 16-byte (real) or 32-byte (complex) slots
    // {packed state, amplitude}; open addressing, line-local probe sequence
    char *slots;
    int slot_log2;             // number of slots = 2^slot_log2
    const uint32_t *slot_of;   // [dim] slot index of every representative
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
    int64_t n_slots = 0;
    std::vector<double> J_cache;   // couplings currently written into the blob
    uint32_t lds_reserve = 0;      // LDS bytes kept free for kernels that stage more
    double mean_candidates = 0.0;  // host Alg. 2 on random configurations
    int staged = 0;                // the H.v kernels run the two-stage search
    int fermion = 0;               // fermions in the occupation-number basis
    // fused adjoint: slots {key, x, gy} at the positions of the H.v slots
    // (32 bytes real, 64 bytes complex), allocated by the first fused call
    // and freed with the handle
    char *adj_slots = nullptr;
    // Lanczos workspace, kept between calls and freed with the handle
    struct {
        double *vec[3] = {nullptr, nullptr, nullptr};
        double *partials = nullptr, *ahist = nullptr, *bhist = nullptr, *svec = nullptr;
        void *state = nullptr;
        int cap_steps = 0;
        size_t cap_partials = 0;
    } lzw;
};

// Several sectors (1-D irreps of one group) over one shared set of orbit
// representatives: the union basis is the trivial-irrep basis, each row
// carries a mask of the sectors its stabiliser is compatible with, and the
// slot table's value field holds the row index and that mask.
struct ed_multi {
    ed_basis *base = nullptr;      // representatives of every orbit, hash-slot index
    int K = 0;                     // sectors
    std::vector<double> chi_host;  // [K][ng][2]
    uint64_t *masks = nullptr;     // [dim] bit k: compatible with sector k (owned by base)
    void *chi_dev = nullptr;       // [ng][K] double2 (owned by base)
    std::vector<int64_t> dims;     // [K]
    uint32_t lds_chi_off = 0;      // LDS byte offset of the staged character table
    bool chi_in_lds = true;        // else the kernel reads chi_dev through the caches
    bool chi_signs = false;        // all characters +-1, table not in LDS: stage sign bits
    void *sgn_dev = nullptr;       // [ng] bytes (padded to 16): bit k set iff chi_k(g) = -1
    double build_ms = 0.0;
    int grid_blocks = 0;
    // Lanczos workspace, kept between calls
    struct {
        void *vec[3] = {nullptr, nullptr, nullptr};
        double *partials = nullptr, *ahist = nullptr, *bhist = nullptr, *sector = nullptr;
        void *state = nullptr;
        int cap_steps = 0;
        size_t cap_partials = 0;
    } lzw;
};

namespace ed {
// Kernel launchers (ed_kernels.hip)
int launch_basis_build(ed_basis *b, void *stream);
int multi_lanes_per_row(const ed_multi *mb);
int launch_apply(const ed_basis *b, const double *J, const double *Jz, const void *x, void *y, void *stream, int stats_mode,
                 unsigned long long *stats_dev);
int launch_apply_timed(const ed_basis *b, const double *J, const double *Jz, const void *x, void *y, int reps,
                       double *pack_ms, double *kernel_ms, void *stream);
// gx (may be NULL): also gx = H gy in the same pass, for bases with the
// hash-slot index (the caller checks backward_fusable) and no static scratch
int launch_backward_J(const ed_basis *b, const double *J, const void *x, const void *gy, double *gJ_host, void *stream,
                      bool static_scratch, void *gx = nullptr);
bool backward_fusable(const ed_basis *b);
int run_lanczos(const ed_basis *b, const double *J, const double *Jz, const void *v0, int n_steps, double *alpha, double *beta,
                int *n_done, void *psi0, void *stream);
int check_couplings(const ed_basis *b, const double *J);
// Batched sectors (ed_multi.hip)
int multi_setup(ed_multi *mb, void *stream);
int multi_apply(const ed_multi *mb, const double *J, const void *x, void *y, void *stream);
int multi_stats(const ed_multi *mb, int64_t *terms, int64_t *shared_terms, void *stream);
int multi_lanczos(ed_multi *mb, const double *J, const void *v0, int n_steps, double *alpha, double *beta,
                  int *n_done, int use_graph, void *stream);
void multi_free_workspace(ed_multi *mb);
int device_alloc(ed_basis *b, void **p, size_t bytes);
void free_lanczos_workspace(ed_basis *b);
const char *last_error();
}  // namespace ed
