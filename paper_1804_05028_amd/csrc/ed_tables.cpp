// Model validation and the sublattice-coding lookup tables, on the host.
//
// Definitions (sec. "Generic sublattice coding algorithm"):
//   G_X  = { g : g maps sublattice X onto sublattice 1 (block 0 here) }
//   Rep_X(s) = min over g in G_X of g s          (an m-bit pattern on block 0)
//   Sym_X(s) = { g in G_X : g s = Rep_X(s) }
//   SymmetryAction_X(g, s) = g s                 (an m-bit pattern on block g(X))
// Spin flip (a group element (pi, f)) is read as: G_X is defined by pi alone
// and the action includes the complement when f = 1; the flip is applied to
// the assembled state by an XOR, so the action table is stored once per
// distinct permutation pi.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>

#include "ed_internal.hpp"

namespace ed {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

std::vector<uint32_t> divisors_of(uint32_t n)
{
    std::vector<uint32_t> d;
    for (uint32_t k = 1; k <= n; ++k)
        if (n % k == 0) d.push_back(k);
    return d;
}

namespace {

struct PermKey {
    const int32_t *p;
    int n;
    uint8_t f;
};

struct VecHash {
    size_t operator()(const std::vector<int32_t> &v) const
    {
        uint64_t h = 1469598103934665603ull;
        for (int32_t x : v) {
            h ^= (uint64_t)(uint32_t)x;
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};

}  // namespace

int validate_model(const ed_lattice_t *lat, const ed_group_t *grp, const ed_irrep_t *irrep, int n_up,
                   Tables *tab)
{
    if (!lat || !grp) return set_error(ED_ERR_ARG, "null lattice or group");
    const int N = lat->n_sites;
    if (N < 1 || N > kMaxSites) return set_error(ED_ERR_UNSUPPORTED, "n_sites=%d outside [1, %d]", N, kMaxSites);
    const int ns = lat->n_sublat;
    if (ns < 1 || N % ns != 0)
        return set_error(ED_ERR_NOT_SUBLATTICE_STABLE, "n_sites=%d is not divisible by n_sublat=%d", N, ns);
    const int m = N / ns;
    if (m > kMaxSubBits)
        return set_error(ED_ERR_UNSUPPORTED, "sublattice of %d sites exceeds the %d-bit table limit", m, kMaxSubBits);
    const int ng = grp->n_elems;
    if (ng < 1 || ng > 65535 || !grp->perm || !grp->flip)
        return set_error(ED_ERR_ARG, "group must have 1..65535 elements with perm and flip arrays");
    if (n_up > N) return set_error(ED_ERR_ARG, "n_up=%d > n_sites=%d", n_up, N);
    // each row a permutation
    std::vector<int> seen(N);
    for (int g = 0; g < ng; ++g) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int i = 0; i < N; ++i) {
            int p = grp->perm[(size_t)g * N + i];
            if (p < 0 || p >= N || seen[p]++) return set_error(ED_ERR_NOT_GROUP, "element %d is not a permutation", g);
        }
        if (grp->flip[g] > 1) return set_error(ED_ERR_ARG, "flip[%d] must be 0 or 1", g);
    }
    // identity and closure; key = permutation with the flip bit appended
    std::unordered_map<std::vector<int32_t>, int, VecHash> index;
    index.reserve((size_t)ng * 2);
    int ident = -1;
    bool any_flip = false;
    for (int g = 0; g < ng; ++g) {
        std::vector<int32_t> k(grp->perm + (size_t)g * N, grp->perm + (size_t)(g + 1) * N);
        k.push_back(grp->flip[g]);
        if (!index.emplace(k, g).second) return set_error(ED_ERR_NOT_GROUP, "element %d is repeated", g);
        bool id = grp->flip[g] == 0;
        for (int i = 0; i < N && id; ++i) id = grp->perm[(size_t)g * N + i] == i;
        if (id) ident = g;
        any_flip |= grp->flip[g] != 0;
    }
    if (ident < 0) return set_error(ED_ERR_NOT_GROUP, "the identity is missing");
    std::vector<int32_t> comp(N + 1);
    const double *chi = irrep ? irrep->chi : nullptr;
    if (irrep && !chi) return set_error(ED_ERR_ARG, "irrep without characters");
    for (int g = 0; g < ng; ++g) {
        if (chi) {
            double mod = std::hypot(chi[2 * g], chi[2 * g + 1]);
            if (std::fabs(mod - 1.0) > 1e-9) return set_error(ED_ERR_BAD_IRREP, "|chi(%d)| = %.17g != 1", g, mod);
        }
        const int32_t *pg = grp->perm + (size_t)g * N;
        for (int h = 0; h < ng; ++h) {
            const int32_t *ph = grp->perm + (size_t)h * N;
            for (int i = 0; i < N; ++i) comp[i] = pg[ph[i]];
            comp[N] = grp->flip[g] ^ grp->flip[h];
            auto it = index.find(comp);
            if (it == index.end()) return set_error(ED_ERR_NOT_GROUP, "elements %d*%d not in the group", g, h);
            if (chi) {
                int k = it->second;
                double re = chi[2 * g] * chi[2 * h] - chi[2 * g + 1] * chi[2 * h + 1];
                double im = chi[2 * g] * chi[2 * h + 1] + chi[2 * g + 1] * chi[2 * h];
                if (std::fabs(re - chi[2 * k]) > 1e-9 || std::fabs(im - chi[2 * k + 1]) > 1e-9)
                    return set_error(ED_ERR_BAD_IRREP, "chi(%d)chi(%d) != chi(%d*%d)", g, h, g, h);
            }
        }
    }
    if (any_flip && n_up >= 0 && 2 * n_up != N)
        return set_error(ED_ERR_FLIP_NEEDS_SZ0, "spin flip needs 2*n_up == n_sites (n_up=%d, N=%d)", n_up, N);
    // sublattice stability: every element maps each block onto one block
    for (int g = 0; g < ng; ++g) {
        const int32_t *pg = grp->perm + (size_t)g * N;
        for (int X = 0; X < ns; ++X) {
            int Y = pg[X * m] / m;
            for (int k = 1; k < m; ++k)
                if (pg[X * m + k] / m != Y)
                    return set_error(ED_ERR_NOT_SUBLATTICE_STABLE,
                                     "element %d splits sublattice %d (sites %d..%d)", g, X, X * m, X * m + m - 1);
        }
    }
    // bonds: sites valid and the bond multiset invariant under every element
    const int nb = lat->n_bonds;
    if (nb < 0 || (nb > 0 && !lat->bonds)) return set_error(ED_ERR_ARG, "bad bond array");
    std::map<std::pair<int, int>, int> bset;
    for (int b = 0; b < nb; ++b) {
        int p = lat->bonds[2 * b], q = lat->bonds[2 * b + 1];
        if (p < 0 || q < 0 || p >= N || q >= N || p == q) return set_error(ED_ERR_ARG, "bond %d = (%d,%d) invalid", b, p, q);
        bset[{std::min(p, q), std::max(p, q)}]++;
    }
    std::vector<int32_t> orbit(nb, -1);
    for (int g = 0; g < ng; ++g) {
        const int32_t *pg = grp->perm + (size_t)g * N;
        std::map<std::pair<int, int>, int> img;
        for (int b = 0; b < nb; ++b) {
            int p = pg[lat->bonds[2 * b]], q = pg[lat->bonds[2 * b + 1]];
            img[{std::min(p, q), std::max(p, q)}]++;
        }
        if (img != bset) return set_error(ED_ERR_NONINVARIANT_H, "bond set is not invariant under element %d", g);
    }
    if (tab) {
        // bond orbits (union over images), used to check couplings per call
        std::map<std::pair<int, int>, std::vector<int>> where;
        for (int b = 0; b < nb; ++b) {
            int p = lat->bonds[2 * b], q = lat->bonds[2 * b + 1];
            where[{std::min(p, q), std::max(p, q)}].push_back(b);
        }
        int next = 0;
        for (int b = 0; b < nb; ++b) {
            if (orbit[b] >= 0) continue;
            for (int g = 0; g < ng; ++g) {
                const int32_t *pg = grp->perm + (size_t)g * N;
                int p = pg[lat->bonds[2 * b]], q = pg[lat->bonds[2 * b + 1]];
                for (int c : where[{std::min(p, q), std::max(p, q)}]) orbit[c] = next;
            }
            ++next;
        }
        tab->bonds.assign(lat->bonds, lat->bonds + 2 * (size_t)nb);
        tab->bond_orbit = orbit;
        tab->nb = nb;
    }
    return ED_OK;
}

int build_tables(const ed_lattice_t *lat, const ed_group_t *grp, Tables &t)
{
    const int N = lat->n_sites, ns = lat->n_sublat, m = N / ns, ng = grp->n_elems;
    t.N = N;
    t.ns = ns;
    t.m = m;
    t.ng = ng;
    t.P = 1u << m;
    const uint32_t P = t.P, mmask = P - 1;
    t.perm.assign(grp->perm, grp->perm + (size_t)ng * N);
    t.flip.assign(grp->flip, grp->flip + ng);
    // distinct permutations
    std::unordered_map<std::vector<int32_t>, int, VecHash> uidx;
    t.g_u.resize(ng);
    t.u_perm.clear();
    for (int g = 0; g < ng; ++g) {
        std::vector<int32_t> k(grp->perm + (size_t)g * N, grp->perm + (size_t)(g + 1) * N);
        auto it = uidx.find(k);
        if (it == uidx.end()) {
            int u = (int)uidx.size();
            uidx.emplace(k, u);
            t.u_perm.insert(t.u_perm.end(), k.begin(), k.end());
            t.g_u[g] = (uint16_t)u;
        } else {
            t.g_u[g] = (uint16_t)it->second;
        }
    }
    t.nu = (int)uidx.size();
    const int nu = t.nu;
    // block images and the SymmetryAction table
    t.u_tgt.resize((size_t)nu * ns);
    t.act.assign((size_t)nu * ns * P, 0);
    for (int u = 0; u < nu; ++u) {
        const int32_t *pu = &t.u_perm[(size_t)u * N];
        for (int X = 0; X < ns; ++X) {
            int Y = pu[X * m] / m;
            t.u_tgt[(size_t)u * ns + X] = (uint8_t)Y;
            uint16_t *row = &t.act[((size_t)u * ns + X) * P];
            for (uint32_t s = 0; s < P; ++s) {
                uint32_t img = 0;
                for (int k = 0; k < m; ++k) {
                    if ((s >> (m - 1 - k)) & 1u) {
                        int tgt = pu[X * m + k] - Y * m;   // position inside block Y
                        img |= 1u << (m - 1 - tgt);
                    }
                }
                row[s] = (uint16_t)img;
            }
        }
    }
    // Rep_X and Sym_X
    std::vector<uint16_t> repv((size_t)ns * P);
    t.sym_off.assign((size_t)ns * (P + 1), 0);
    t.sym_list.clear();
    t.max_sym = 0;
    // blocks that no element maps onto block 0 (e.g. the spin species of a
    // Hubbard model as two orbitals per site) can never hold the top block:
    // their Rep_X is "infinite", stored as 0xFFFF with an empty Sym list
    std::vector<char> no_top(ns, 0);
    for (int X = 0; X < ns; ++X) {
        std::vector<int> GX;
        for (int g = 0; g < ng; ++g)
            if (t.u_tgt[(size_t)t.g_u[g] * ns + X] == 0) GX.push_back(g);
        no_top[X] = GX.empty();
        for (uint32_t s = 0; s < P; ++s) {
            uint32_t best = 0xFFFFFFFFu;
            for (int g : GX) {
                uint32_t v = t.act[((size_t)t.g_u[g] * ns + X) * P + s] ^ (t.flip[g] ? mmask : 0u);
                best = std::min(best, v);
            }
            repv[(size_t)X * P + s] = (uint16_t)best;
            t.sym_off[(size_t)X * (P + 1) + s] = (uint32_t)t.sym_list.size();
            int cnt = 0;
            for (int g : GX) {
                uint32_t v = t.act[((size_t)t.g_u[g] * ns + X) * P + s] ^ (t.flip[g] ? mmask : 0u);
                if (v == best) {
                    t.sym_list.push_back((uint16_t)g);
                    ++cnt;
                }
            }
            t.max_sym = std::max(t.max_sym, cnt);
        }
        t.sym_off[(size_t)X * (P + 1) + P] = (uint32_t)t.sym_list.size();
    }
    // top-block values: every Rep_X value is a fixed point of Rep_0
    t.top_vals.clear();
    for (uint32_t s = 0; s < P; ++s)
        if (repv[s] == s) t.top_vals.push_back((uint16_t)s);
    std::vector<int32_t> rank(P, -1);
    for (size_t r = 0; r < t.top_vals.size(); ++r) rank[t.top_vals[r]] = (int32_t)r;
    t.rep.resize((size_t)ns * P);
    for (size_t k = 0; k < repv.size(); ++k) {
        if (no_top[k / P]) {
            t.rep[k] = 0xFFFFu;
            continue;
        }
        int32_t r = rank[repv[k]];
        if (r < 0) return set_error(ED_ERR_NOT_SUBLATTICE_STABLE, "internal: Rep_X value is not a block-0 representative");
        t.rep[k] = ((uint32_t)r << 16) | repv[k];
    }
    return ED_OK;
}

uint64_t Tables::apply(int g, uint64_t s) const
{
    const uint32_t mmask = P - 1;
    const int u = g_u[g];
    uint64_t v = 0;
    for (int X = 0; X < ns; ++X) {
        uint32_t sx = (uint32_t)(s >> block_shift(X)) & mmask;
        int Y = u_tgt[(size_t)u * ns + X];
        v |= (uint64_t)act[((size_t)u * ns + X) * P + sx] << block_shift(Y);
    }
    if (flip[g]) v ^= full_mask();
    return v;
}

// Alg. "Sublattice coding algorithm for finding the representative".
uint64_t Tables::find_rep(uint64_t s, int *g_out, int *n_cand) const
{
    const uint32_t mmask = P - 1;
    uint32_t minrep = 0xFFFFFFFFu;
    for (int X = 0; X < ns; ++X) {
        uint32_t sx = (uint32_t)(s >> block_shift(X)) & mmask;
        minrep = std::min(minrep, rep[(size_t)X * P + sx] & 0xFFFFu);
    }
    uint64_t best = ~0ull;
    int bg = -1, cand = 0;
    for (int Y = 0; Y < ns; ++Y) {
        uint32_t sy = (uint32_t)(s >> block_shift(Y)) & mmask;
        if ((rep[(size_t)Y * P + sy] & 0xFFFFu) != minrep) continue;
        for (uint32_t k = sym_off[(size_t)Y * (P + 1) + sy]; k < sym_off[(size_t)Y * (P + 1) + sy + 1]; ++k) {
            int g = sym_list[k];
            uint64_t v = apply(g, s);
            ++cand;
            if (v < best) {
                best = v;
                bg = g;
            }
        }
    }
    if (g_out) *g_out = bg;
    if (n_cand) *n_cand = cand;
    return best;
}

}  // namespace ed
