/*
 * ed.h -- C ABI of the MI355X (gfx950) symmetry-sector exact-diagonalisation
 * hot path: sublattice-coding representative search, index lookup in the
 * sorted basis, and the bond-loop Heisenberg H.v, plus Lanczos and the
 * adjoint.  Method: A. Wietek and A. M. Laeuchli, "Sublattice coding
 * algorithm and distributed memory parallelization for large-scale exact
 * diagonalizations of quantum many-body systems" (arXiv:1804.05028).
 *
 * General rules
 *  - Every call returns an int status: ED_OK (0) or a negative ED_ERR_* code.
 *    Nothing throws across this boundary.  ed_last_error() returns a
 *    thread-local message describing the last failure on the calling thread.
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *    device memory on the current device (for example PyTorch tensors'
 *    data_ptr()).  The caller owns every pointer it passes; the library owns
 *    the opaque handles it returns and every device buffer inside them.
 *  - stream is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls that only enqueue work return once it is enqueued; calls that
 *    return host results synchronise the stream first.
 *  - A handle keeps per-call state on the device (the couplings written
 *    into its tables, the input amplitudes scattered into its index, the
 *    Lanczos workspace), so calls on one handle must not overlap: use it
 *    from one thread and one stream at a time.  Different handles are
 *    independent.
 *  - Spin configurations are uint64 codes: site s <-> bit (N-1-s), so site 0
 *    is the most significant bit, and up = 1 (sec. "Symmetry adapted basis
 *    states"; the worked examples' integers (011)_2 = 3 fix this order).
 *  - Vectors are FP64 (double) in ascending-representative order, or
 *    complex128 stored as interleaved (re, im) doubles when the irrep has a
 *    complex character (ed_basis_is_complex).
 */
#ifndef ED_MI355X_H
#define ED_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ED_OK 0
#define ED_ERR_ARG (-1)                    /* null pointer, bad size, x == y, ...   */
#define ED_ERR_NOT_GROUP (-2)              /* permutations not closed / no identity */
#define ED_ERR_BAD_IRREP (-3)              /* chi not a homomorphism or |chi| != 1   */
#define ED_ERR_NOT_SUBLATTICE_STABLE (-4)  /* some g splits a sublattice            */
#define ED_ERR_FLIP_NEEDS_SZ0 (-5)         /* spin flip in the group but 2 n_up != N */
#define ED_ERR_NONINVARIANT_H (-6)         /* bonds or couplings not group invariant */
#define ED_ERR_OOM (-7)                    /* device allocation failed              */
#define ED_ERR_HIP (-8)                    /* a HIP runtime call failed             */
#define ED_ERR_UNSUPPORTED (-9)            /* size or layout the library does not handle */

/*
 * Lattice: N sites, bonds, and the sublattice decomposition.
 * Sublattice stability (sec. "Generic sublattice coding algorithm",
 * Definition of sublattice stability): the sites must be numbered so that
 * sublattice X is the block [X*N/n_sublat, (X+1)*N/n_sublat), which puts
 * sublattice 0 on the most significant bits; every group element must map
 * each block onto one block.  1 <= N <= 56 and N/n_sublat <= 16.
 * bonds[2b], bonds[2b+1]: the two sites of bond b (distinct).  The
 * Hamiltonian is H = sum_b J_b S_p.S_q (Eq. of the benchmark model,
 * sec. "Benchmarks", with one coupling per bond).
 */
typedef struct {
    int32_t n_sites;
    int32_t n_bonds;
    const int32_t *bonds;   /* host, [n_bonds][2] */
    int32_t n_sublat;
} ed_lattice_t;

/*
 * Group: n_elems site permutations, optionally combined with global spin
 * flip.  perm[g*N + i] is the site to which element g moves the spin of site
 * i; flip[g] = 1 also inverts every spin.  Must contain the identity and be
 * closed under composition (g h)(i) = g(h(i)), flips adding mod 2.
 * n_elems <= 65535.
 */
typedef struct {
    int32_t n_elems;
    const int32_t *perm;    /* host, [n_elems][N] */
    const uint8_t *flip;    /* host, [n_elems]    */
} ed_group_t;

/*
 * 1-D irrep: chi[2g], chi[2g+1] = (re, im) of chi(g), |chi| = 1,
 * chi(g h) = chi(g) chi(h).  The sector holds the states with
 * g|psi> = chi(g)|psi> (the span of the symmetry-adapted states of
 * sec. "Symmetry adapted basis states").
 */
typedef struct {
    const double *chi;      /* host, [n_elems][2] */
} ed_irrep_t;

/* Optional tuning; zero fields mean "choose automatically". */
typedef struct {
    int32_t limits_bits;    /* index_mode 1: state bits after the top block used in the Limits key    */
    int32_t index_mode;     /* 0 = hash-slot index with the input amplitude stored beside the key;
                               1 = the paper's Limits ranges plus binary search of the sorted states    */
    int32_t block_threads;  /* threads per block of the H.v kernel (64..1024, multiple of 64)            */
    int32_t blocks_per_cu;  /* persistent blocks per compute unit of the H.v kernel                      */
    int32_t chunk_bits;     /* width of the substate chunks of the symmetry-action table (1..16)         */
    int32_t hash_load_pct;  /* index_mode 0: maximum load factor of the slot table in percent (10..90)   */
    int32_t table_entry_bytes; /* 1, 2 or 4 bytes per symmetry-action entry (wide ones carry the block
                                  position); 0 = automatic                                              */
    int32_t search_mode;    /* representative search of the index_mode 0 H.v and Lanczos kernels
                               and of the batched kernel (in its instances with at most 4 sectors
                               per lane, or 8 on split rows, and compile-time search loops; the
                               others and the adjoint kernel run the one-stage search, which gives
                               the same results):
                               ED_SEARCH_ONE_STAGE = assemble the full image of every candidate;
                               ED_SEARCH_TWO_STAGE = image the block landing below the top block
                               first and assemble only the candidates minimising it (2 to 4
                               sublattices, else ED_ERR_UNSUPPORTED); 0 = two-stage when a host
                               sample of the search averages at least 3 candidates               */
    int32_t lanes_per_row;  /* batched H.v (ed_build_multi): 1, 2 or 4 lanes share a row, each
                               running the row's searches and holding every lanes-th sector; 0 = 1 lane
                               for K <= 2, 2 lanes for K <= 8, else 4.  When |G| K 16 bytes of
                               characters exceed 32 KB they are read from HBM (or, for K <= 8 and
                               characters all +-1, staged as sign bits): then 0 = 1 lane for K <= 8,
                               and the count is raised to at least 2 for K > 8 and 4 for K > 16;
                               K > 32 always runs 4 lanes (ed_multi_info reports the count used)  */
    int32_t lanczos_direct; /* ed_lanczos: 1 = launch each step's kernels directly; 0 = capture the
                               step once per buffer assignment in a HIP graph and replay it        */
} ed_tuning_t;

#define ED_SEARCH_ONE_STAGE 1
#define ED_SEARCH_TWO_STAGE 2

typedef struct ed_tables ed_tables_t;   /* host-side sublattice-coding tables */
typedef struct ed_basis ed_basis_t;     /* device-resident sector basis       */

typedef struct {
    int32_t n_sites, n_sublat, sub_bits, n_elems, n_perms;
    int64_t rep_entries;        /* n_sublat * 2^sub_bits                       */
    int64_t sym_entries;        /* total length of all Sym_X lists             */
    int64_t action_bytes;       /* bytes of the symmetry-action table          */
    int32_t max_sym_len;        /* longest Sym_X list                          */
    int32_t n_top;              /* distinct values a top block can take        */
} ed_tables_info_t;

typedef struct {
    int64_t dim;                /* sector dimension D                          */
    int32_t is_complex;
    int32_t n_sites, n_up, n_sublat, sub_bits, n_elems, n_bonds;
    int32_t index_mode;         /* 0 hash slots, 1 Limits + binary search       */
    int32_t limits_bits;        /* key bits after the top block (index_mode 1) */
    int64_t n_keys;             /* Limits entries - 1 (index_mode 1)           */
    int64_t n_slots;            /* slot-table size (index_mode 0)              */
    int32_t chunk_bits;         /* substate chunk width of the action table    */
    int32_t table_entry_bytes;  /* bytes per action-table entry                */
    int32_t lds_bytes;          /* LDS bytes of the staged tables per block    */
    int64_t device_bytes;       /* device memory owned by the handle           */
    double build_ms;            /* wall time of ed_build_basis                 */
    int32_t search_mode;        /* search of the H.v kernels: ED_SEARCH_ONE_STAGE or _TWO_STAGE */
    double mean_candidates;     /* candidate symmetries per search, host Alg. 2 on 2048 random
                                   configurations at this n_up                  */
    int32_t is_fermion;         /* built by ed_build_basis_fermions             */
} ed_basis_info_t;

/* Library version string (static). */
const char *ed_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *ed_last_error(void);

/*
 * Check a model without touching the GPU: group closure and identity,
 * character homomorphism and modulus, sublattice stability, spin flip only at
 * 2 n_up = N, and group invariance of the bond set.  irrep may be NULL
 * (skips the character checks), n_up < 0 skips the flip check.
 */
int ed_validate(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep, int32_t n_up);

/*
 * Sublattice-coding lookup tables on the host (Alg. "Preparation of lookup
 * tables"; definitions of sublattice symmetries G_X, Rep_X, Sym_X and
 * SymmetryAction_X in sec. "Generic sublattice coding algorithm").  Host
 * only; used to inspect and test the tables the kernels use.
 */
int ed_tables_create(const ed_lattice_t *lat, const ed_group_t *grp, ed_tables_t **out);
void ed_tables_free(ed_tables_t *t);
int ed_tables_info(const ed_tables_t *t, ed_tables_info_t *info);

/*
 * Rep_X and Sym_X of one substate: *rep_out = Rep_X(substate) (an m-bit
 * pattern placed on sublattice 0), sym_out[0..*n_sym) = the group indices of
 * Sym_X(substate) in ascending order (at most cap are written; *n_sym is the
 * full length).
 */
int ed_tables_sublattice(const ed_tables_t *t, int32_t X, uint32_t substate, uint32_t *rep_out,
                         int32_t *sym_out, int32_t cap, int32_t *n_sym);

/*
 * Alg. "Sublattice coding algorithm for finding the representative", on the
 * host, from the same tables: for each state, the representative (orbit
 * minimum), one minimising group element, and the number of candidate
 * symmetries examined.  Any of rep_out, g_out, n_cand_out may be NULL.
 */
int ed_tables_find_rep(const ed_tables_t *t, int64_t n, const uint64_t *states, uint64_t *rep_out,
                       int32_t *g_out, int32_t *n_cand_out);

/*
 * Build the sector basis on the device (Alg. "Preparation of the distributed
 * and symmetrized Hilbert space" on one device): every representative with
 * n_up up spins whose stabiliser carries the trivial character, in ascending
 * order, with its stabiliser size, and the Limits index over key prefixes.
 * Validates as ed_validate does.  tuning may be NULL.  Synchronises stream.
 */
int ed_build_basis(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep,
                   int32_t n_up, const ed_tuning_t *tuning, void *stream, ed_basis_t **out);
void ed_free_basis(ed_basis_t *b);
int64_t ed_basis_dim(const ed_basis_t *b);
int ed_basis_is_complex(const ed_basis_t *b);
int ed_basis_info(const ed_basis_t *b, ed_basis_info_t *info);

/* Representatives in ascending order -> host [dim] (synchronises). */
int ed_basis_copy_states(const ed_basis_t *b, uint64_t *host_out, void *stream);
/* Representatives -> device [dim] (stream-ordered). */
int ed_basis_copy_states_device(const ed_basis_t *b, uint64_t *dev_out, void *stream);
/* |Stab sigma| of every representative -> host [dim] (synchronises). */
int ed_basis_copy_norms(const ed_basis_t *b, uint16_t *host_out, void *stream);

/*
 * y = H x in the sector (Alg. "Parallel matrix-vector multiply" for the sum
 * of all bond terms, in gather form): for row i with representative sigma_i,
 * y_i = d_i x_i + sum over antiparallel bonds b of
 *       (J_b / 2) * chi(g) * sqrt(n_j / n_i) * x_j,
 * where sigma' = sigma_i with bond b flipped, g maps sigma' to its
 * representative sigma_j = g sigma' (Eq. for matrix elements between
 * representatives, conjugated for the row form), n = |Stab|, and
 * d_i = sum_b J_b (+1/4 parallel, -1/4 antiparallel).  Terms whose target is
 * not in the sector are dropped.  J: host [n_bonds], constant on bond orbits
 * (else ED_ERR_NONINVARIANT_H).  x, y: device [dim] (complex: [dim][2]),
 * distinct.  Enqueued on stream.
 */
int ed_apply_H(const ed_basis_t *b, const double *J, const void *x_dev, void *y_dev, void *stream);

/*
 * Device timing of the H.v: reps (1..1000) launches of y = H x on stream,
 * with HIP events recorded on that stream around each launch's scatter of x
 * into the hash-slot index and around its H.v kernel.  *pack_ms and
 * *kernel_ms receive the mean duration of each per launch (the scatter is 0
 * for the Limits index).  Spin bases: J and Jz as for ed_apply_H_xxz;
 * fermionic bases: t and V of ed_apply_H_fermions.  Synchronises.
 */
int ed_apply_H_timed(const ed_basis_t *b, const double *J, const double *Jz, const void *x_dev, void *y_dev,
                     int32_t reps, double *pack_ms, double *kernel_ms, void *stream);

/*
 * Random-read probe, the ceiling the H.v gather is measured against: the
 * gather form of the sector H.v (sec. "Parallel matrix-vector multiplication")
 * reads one target slot per off-diagonal term at an unrelated address.  The
 * probe reads slots of slot_bytes (16: one 16-byte load, as real sectors do;
 * 32: two 16-byte loads of one 32-byte slot, as complex sectors do) at
 * pseudo-random slot-aligned offsets of buf_dev (device memory of `bytes`
 * bytes, a power of two >= 1 MiB, owned by the caller, contents irrelevant),
 * iters (even, 2..4096) slots per lane with two in flight, two 1024-thread
 * blocks per compute unit; one untimed launch, then reps (1..100) timed ones
 * on stream.  *reads_per_s receives the mean rate in slots per second.
 * Writes nothing to buf_dev; allocates nothing.  Synchronises.  ED_ERR_ARG
 * on bad sizes or null pointers.
 */
int ed_probe_random_reads(const void *buf_dev, int64_t bytes, int32_t slot_bytes, int32_t iters, int32_t reps,
                          double *reads_per_s, void *stream);

/*
 * XXZ form of ed_apply_H: each bond contributes the exchange
 * (Jxy_b / 2)(S+_p S-_q + S-_p S+_q) and the Ising term Jz_b Sz_p Sz_q, both
 * non-branching two-site terms (sec. "Parallel matrix-vector multiply"; the
 * matrix element of a flip is Jxy_b / 2 times the same symmetry factors, the
 * diagonal is sum_b Jz_b (+1/4 parallel, -1/4 antiparallel)).  Jz = NULL
 * means Jz = Jxy, which is ed_apply_H.  Jxy and Jz: host [n_bonds], each
 * constant on bond orbits.
 */
int ed_apply_H_xxz(const ed_basis_t *b, const double *Jxy, const double *Jz, const void *x_dev, void *y_dev,
                   void *stream);

/*
 * Fermions in the occupation-number basis (sec. "Discussion": the sublattice
 * coding carries over to fermionic Hamiltonians written in occupation
 * numbers, with a Fermi sign besides the representative and its symmetry).
 * The lattice's sites are orbitals, numbered as above (orbital i <-> bit
 * N-1-i, sublattice blocks as for spins); a configuration stands for the
 * ordered product c+_{i1} ... c+_{ik} |0>, i1 < ... < ik, of its occupied
 * orbitals.  A group element (no spin flip) maps c+_i to c+_{perm[i]}: the
 * image of a configuration is its permuted pattern times (-1) to the number
 * of occupied pairs whose order it reverses.  The sector of the 1-D irrep
 * chi holds the orbit minima whose symmetrised states survive, i.e. chi(g)
 * equals that sign for every g of the stabiliser.  Spinful models take two
 * orbitals per site (the group permuting both species alike).
 *
 * ed_build_basis_fermions: as ed_build_basis with n_particles occupied
 * orbitals; ED_ERR_UNSUPPORTED for flip elements, the Limits index, 1-byte
 * table entries, 2-byte entries with blocks of more than 12 orbitals or more
 * than 8 sublattices, or blocks of more than 16 orbitals.  table_entry_bytes
 * 0 takes 2-byte entries (the chunk's sign parity in bit 15) where they fit,
 * else 4-byte ones (parity in bit 31).
 *
 * ed_apply_H_fermions: y = H x for
 *   H = sum_b [ -t_b (c+_p c_q + c+_q c_p) + V_b n_p n_q ],
 * in gather form: y_i = sum_b V_b n_p n_q x_i + sum over bonds with one of
 * p, q occupied of -t_b (-1)^(occupied orbitals strictly between p and q)
 * (-1)^(Fermi sign of g on the hopped configuration) chi(g)
 * sqrt(n_j / n_i) x_j, g mapping it to its representative sigma_j.  t and V:
 * host [n_bonds], each constant on bond orbits; V may be NULL (0).  x, y as
 * for ed_apply_H.  ed_apply_H, ed_apply_H_xxz and ed_lanczos(_xxz) reject
 * fermionic bases with ED_ERR_ARG, and the fermionic calls reject spin
 * bases; the adjoint and the batched calls cover spins only.
 *
 * ed_lanczos_fermions: ed_lanczos with the fermionic H.v.
 */
int ed_build_basis_fermions(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep,
                            int32_t n_particles, const ed_tuning_t *tuning, void *stream, ed_basis_t **out);
int ed_apply_H_fermions(const ed_basis_t *b, const double *t, const double *V, const void *x_dev, void *y_dev,
                        void *stream);
int ed_lanczos_fermions(const ed_basis_t *b, const double *t, const double *V, const void *v0_dev, int32_t n_steps,
                        double *alpha_host, double *beta_host, int32_t *n_done, void *psi0_dev, void *stream);

/*
 * Term counts of one H.v: diagonal terms (= dim), off-diagonal terms whose
 * target is in the sector, and dropped ones.  Synchronises.
 */
int ed_apply_H_stats(const ed_basis_t *b, int64_t *n_diag, int64_t *n_offdiag_kept,
                     int64_t *n_offdiag_dropped, void *stream);

/*
 * Lanczos on the sector (the iteration whose cost the paper attributes to the
 * matrix-vector product, sec. "Distributed and hybrid memory
 * parallelization"): v_0 = v0 / |v0|; w = H v_j - beta_{j-1} v_{j-1};
 * alpha_j = Re <v_j, w>; w -= alpha_j v_j; beta_j = |w|; v_{j+1} = w / beta_j.
 * FP64 throughout, no reorthogonalisation.  Stops after n_steps or when
 * beta_j <= 1e-12 * max_k(|alpha_k|, beta_k) (*n_done < n_steps).
 * alpha_host, beta_host: host [n_steps].  If psi0_dev is not NULL a second,
 * bit-identical pass writes the normalised lowest Ritz vector there.
 * Synchronises.
 */
int ed_lanczos(const ed_basis_t *b, const double *J, const void *v0_dev, int32_t n_steps,
               double *alpha_host, double *beta_host, int32_t *n_done, void *psi0_dev,
               void *stream);

/* ed_lanczos with the XXZ couplings of ed_apply_H_xxz (Jz = NULL: Jz = Jxy). */
int ed_lanczos_xxz(const ed_basis_t *b, const double *Jxy, const double *Jz, const void *v0_dev, int32_t n_steps,
                   double *alpha_host, double *beta_host, int32_t *n_done, void *psi0_dev, void *stream);

/*
 * Adjoint of y = H(J) x: gx = H^dagger gy (= H gy, H is Hermitian) if gx_dev
 * is not NULL, and gJ_b = Re( gy^dagger dH/dJ_b x ) for every bond if gJ_host
 * is not NULL, where dH/dJ_b collects bond b's diagonal and off-diagonal
 * terms in the row form of ed_apply_H.  Synchronises if gJ_host is given.
 * gx must differ from gy and, when gJ is requested, from x (ED_ERR_ARG).
 * With both outputs on a basis with the hash-slot index, one pass computes
 * both from a second slot table holding x and gy, of 32 bytes per slot
 * (64 for complex sectors).  The first such call allocates that table, and
 * it is kept until ed_free_basis.  Its gx and gJ equal, bit for bit, those
 * of ed_apply_H on gy and of this call without gx.
 */
int ed_apply_H_backward(const ed_basis_t *b, const double *J, const void *x_dev, const void *gy_dev,
                        void *gx_dev, double *gJ_host, void *stream);

/*
 * ed_apply_H_backward without device allocation, for callers that cannot
 * allocate device memory (serving or training loops and harnesses that
 * forbid hipMalloc).  Same arguments, results and synchronisation as
 * ed_apply_H_backward; the per-bond partial sums live in a static device
 * array of 2^19 doubles (4 MiB, held by every GPU the library runs on until
 * the process ends) instead of buffers allocated per call.  A launch whose
 * partial sums (blocks x (n_bonds + 1) + n_bonds + 1 doubles) exceed it
 * returns ED_ERR_UNSUPPORTED.  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other threads or streams) race.
 */
int ed_apply_H_backward_noalloc(const ed_basis_t *b, const double *J, const void *x_dev, const void *gy_dev,
                                void *gx_dev, double *gJ_host, void *stream);

/*
 * Batched sectors.  Several 1-D irreps chi_0 .. chi_{K-1} (K <= 64) of one
 * group share one set of representatives: the orbit minima of the group,
 * i.e. the trivial-irrep basis (the representatives are the same for every
 * irrep, sec. "Symmetry adapted basis states"; an irrep keeps those whose
 * stabiliser carries its trivial value, the others have zero norm).  Row i of
 * the shared basis belongs to sector k iff bit k of its mask is set, and
 * sector k's own basis (ed_build_basis with chi_k) is the subsequence of
 * shared rows with that bit, in the same order.
 *
 * Batched vectors are complex128 [dim][K] (interleaved re, im; sector index
 * fastest), owned by the caller.  Real sectors use the same layout.
 */
typedef struct ed_multi ed_multi_t;

typedef struct {
    int64_t dim;                /* shared representatives (rows of a batched vector) */
    int32_t n_sectors;
    int32_t n_sites, n_up, n_sublat, n_elems, n_bonds;
    int32_t chunk_bits, table_entry_bytes, lds_bytes;
    int64_t n_slots;
    int64_t device_bytes;
    double build_ms;
    int32_t lanes_per_row;      /* lanes per row of the batched H.v kernel     */
    int32_t chi_in_lds;         /* 1: the character table is staged in LDS (counted in lds_bytes);
                                   0: the kernel reads it from HBM through the caches            */
    int32_t chi_signs;          /* 1: every character is +1 or -1 (real one-dimensional irreps)
                                   and the table is too large for LDS: the kernel stages one sign
                                   bit per sector and element instead (|G| bytes, in lds_bytes) */
} ed_multi_info_t;

#define ED_LANCZOS_NO_GRAPH 1   /* ed_lanczos_batched: launch the step kernels directly */

/*
 * Build the shared basis of n_sectors irreps (irreps[k].chi: host
 * [n_elems][2] each); validates every irrep as ed_validate does.  tuning may
 * be NULL; the index is always the hash-slot index and action-table entries
 * are 2 or 4 bytes wide.  Up to 32 sectors the slot probe of a term returns
 * the target's sector mask; from 33 to 64 sectors the mask is read from a
 * per-row array, the H.v runs 4 lanes per row, and the character table
 * (|G| K 16 bytes) must fit the 32 KB staged in LDS (else ED_ERR_UNSUPPORTED).
 * Synchronises stream.
 */
int ed_build_multi(const ed_lattice_t *lat, const ed_group_t *grp, int32_t n_sectors, const ed_irrep_t *irreps,
                   int32_t n_up, const ed_tuning_t *tuning, void *stream, ed_multi_t **out);
void ed_free_multi(ed_multi_t *mb);
int ed_multi_info(const ed_multi_t *mb, ed_multi_info_t *info);
/* dims_host[k] = dimension of sector k (rows with bit k set). */
int ed_multi_sector_dims(const ed_multi_t *mb, int64_t *dims_host);
/* Shared representatives, ascending -> host [dim] (synchronises). */
int ed_multi_copy_states(const ed_multi_t *mb, uint64_t *host_out, void *stream);
/* Sector masks of the shared rows -> host [dim] (synchronises). */
int ed_multi_copy_masks(const ed_multi_t *mb, uint64_t *host_out, void *stream);

/*
 * y = H x in every sector at once: y[i][k] is ed_apply_H's row i of sector k
 * (same formula, character chi_k) when row i belongs to sector k, and 0
 * otherwise; entries x[j][k] of rows outside sector k are never read.  The
 * representative search and the index lookup of a term are done once for
 * all sectors.  x, y: device complex128 [dim][K], distinct.  J as for
 * ed_apply_H.  Enqueued on stream.
 */
int ed_apply_H_batched(const ed_multi_t *mb, const double *J, const void *x_dev, void *y_dev, void *stream);

/*
 * n_terms[k] = diagonal plus kept off-diagonal terms of sector k's H.v (what
 * ed_apply_H_stats reports for that sector, n_diag + n_offdiag_kept);
 * *n_shared_terms = off-diagonal terms of the shared rows, each searched and
 * looked up once per batched H.v.  Synchronises.
 */
int ed_apply_H_batched_stats(const ed_multi_t *mb, int64_t *n_terms, int64_t *n_shared_terms, void *stream);

/*
 * Lanczos in every sector at once, ed_lanczos's recurrence and stopping rule
 * applied to each sector separately (v0_dev: device complex128 [dim][K],
 * entries outside a sector ignored; a sector whose start vector is zero, or
 * that is empty, reports n_done 0).  alpha_host, beta_host: host
 * [K][n_steps]; n_done: host [K].  One step's kernels are captured in a HIP
 * graph and replayed, unless flags has ED_LANCZOS_NO_GRAPH.  Synchronises.
 */
int ed_lanczos_batched(const ed_multi_t *mb, const double *J, const void *v0_dev, int32_t n_steps,
                       double *alpha_host, double *beta_host, int32_t *n_done, int32_t flags, void *stream);

/*
 * Eigenvalues (ascending) of the symmetric tridiagonal matrix with diagonal
 * alpha[0..m) and off-diagonal beta[0..m-1), and optionally the eigenvector
 * of the lowest one (evec0 [m], may be NULL).  Host only.
 */
int ed_tridiag_eigh(int32_t m, const double *alpha, const double *beta, double *evals, double *evec0);

#ifdef __cplusplus
}
#endif
#endif
