"""Choice of the sublattice decomposition.

A cluster usually admits several sublattice-stable decompositions. Fewer
sublattices mean larger lookup tables; more sublattices mean more blocks to
assemble and more candidate symmetries per representative search
(sec. "Generic sublattice coding algorithm", the discussion of the number of
sublattices). This module ranks the decompositions that fit the LDS of one
compute unit by an estimate of the search cost. The estimate uses:
  * the sizes of the tables the library builds on the host;
  * the mean number of candidate symmetries of the library's host search
    (Alg. "Sublattice coding algorithm for finding the representative") on
    random configurations.
The GPU autotuner then times the best few.
"""
from __future__ import annotations

import math

import numpy as np

from . import _lib as L

LDS_BUDGET = 160 * 1024 - 8192
TWO_STAGE_MIN_CANDIDATES = 3.0   # the library's automatic search choice


def _divisors(n):
    return [d for d in range(1, n + 1) if n % d == 0]


def table_layout(n_sub, sub_bits, n_perms, sym_entries, n_elems, n_bonds, complex_chi=False, budget=LDS_BUDGET,
                 two_stage=False):
    """Fewest action-table chunks whose LDS image fits the budget, as the
    library lays it out.  Returns (chunks, lds_bytes) or None.

    The image holds, each part padded to 16 B:
      * Rep|Sym offset (4 B per substate and sublattice);
      * the Sym lists (a 4 B count per list plus 4 B per entry);
      * block shifts;
      * the characters (8 B real or 16 B complex per element);
      * square roots of the stabiliser sizes and their inverses, and the divisors;
      * the bonds (24 B each);
      * for the two-stage search, 2 B per permutation (the source block at
        position 1 and its bit offset);
      * the chunked action table, with 2-byte entries for blocks of up to 12 sites and
        4-byte entries above.
    """
    pad = lambda n: (n + 15) // 16 * 16
    P = 1 << sub_bits
    n_div = len(_divisors(n_elems))
    fixed = (pad(4 * n_sub * P) + pad(4 * (n_sub * P + sym_entries)) + pad(n_perms * n_sub)
             + pad((16 if complex_chi else 8) * n_elems) + pad(16 * n_div) + pad(4 * n_div)
             + pad(24 * max(n_bonds, 1)) + pad(2) + (pad(2 * n_perms) if two_stage else 0))
    esz = 2 if sub_bits <= 12 else 4
    for nc in range(1, sub_bits + 1):
        cb = math.ceil(sub_bits / nc)
        total = fixed + pad(n_perms * n_sub * nc * (1 << cb) * esz)
        if total <= budget:
            return nc, total
    return None


def _random_configs(n_sites, n_up, count, seed):
    rng = np.random.default_rng(seed)
    keys = rng.random((count, n_sites)).argsort(axis=1)[:, :n_up]
    s = np.zeros(count, np.uint64)
    for k in range(n_up):
        s |= np.left_shift(np.uint64(1), (n_sites - 1 - keys[:, k]).astype(np.uint64))
    return s


def rank_decompositions(make_cluster, decompositions, n_up, samples=4000, seed=7):
    """Rank (n_sub, superlattice) choices by estimated search cost.

    make_cluster(superlattice) -> cluster with that sublattice numbering.
    Returns a list of dicts (fastest estimate first) with n_sub, superlattice,
    sub_bits, chunks, lds_bytes, mean/p99 candidate counts and the estimated
    LDS table reads per search; decompositions whose tables do not fit LDS
    are returned last with fits=False.
    """
    out = []
    for n_sub, M in decompositions:
        cl = make_cluster(M)
        arrays = L.ModelArrays(cl.n_sites, cl.bonds, cl.n_sublat, cl.perm, cl.flip)
        try:
            h = L.ed_tables_create(arrays)
        except L.EDError as e:
            out.append(dict(n_sub=n_sub, superlattice=M, fits=False, error=e.name))
            continue
        try:
            info = L.ed_tables_info(h)
            cfg = _random_configs(cl.n_sites, n_up, samples, seed)
            _, _, cand = L.ed_tables_find_rep(h, cfg)
            # the library's automatic choice of the two-stage search
            two_stage = 2 <= n_sub <= 4 and float(cand.mean()) >= TWO_STAGE_MIN_CANDIDATES
            lay = table_layout(n_sub, info["sub_bits"], info["n_perms"], info["sym_entries"], info["n_elems"],
                               cl.n_bonds, two_stage=two_stage)
        finally:
            L.ed_tables_free(h)
        rec = dict(n_sub=n_sub, superlattice=M, sub_bits=info["sub_bits"], fits=lay is not None,
                   mean_candidates=float(cand.mean()), p99_candidates=float(np.percentile(cand, 99)))
        if lay is not None:
            nc, lds = lay
            rec.update(chunks=nc, lds_bytes=lds,
                       reads_per_search=n_sub + rec["mean_candidates"] * (1 + n_sub * nc))
        out.append(rec)
    return sorted(out, key=lambda r: (not r["fits"], r.get("reads_per_search", math.inf)))
