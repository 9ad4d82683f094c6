"""Launch-configuration search for the sector H.v on the current GPU.

For each sublattice decomposition offered by the caller and each candidate
tuning (action-table chunk width and entry width, threads per block, blocks
per compute unit, one- or two-stage representative search), build the basis, time a few H.v launches with HIP events
on the current stream, and keep the fastest.  Configurations the library
rejects (tables that do not fit in LDS, unsupported entry widths) are
recorded and skipped.  Every candidate computes the same H.v; only its speed
differs.  For batched sectors, autotune_batched picks the group size and
the lanes per row of each group.
"""
from __future__ import annotations

import time

import torch

from . import _lib as L
from . import ed


def default_candidates(sub_bits):
    """Tunings worth trying for sublattice blocks of sub_bits sites."""
    out = [{}]   # the library's automatic choice
    for cb in sorted({(sub_bits + 1) // 2, (sub_bits + 2) // 3}):
        if 1 <= cb < sub_bits:
            for th in (512, 1024):
                out.append({"chunk_bits": cb, "block_threads": th})
    out.append({"block_threads": 512})
    if sub_bits <= 8:
        out.append({"table_entry_bytes": 1})
    # both representative searches (the automatic choice is one of them)
    out.append({"search_mode": L.ED_SEARCH_ONE_STAGE})
    out.append({"search_mode": L.ED_SEARCH_TWO_STAGE})
    return out


def _time_apply(basis, J, reps):
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    x = torch.randn(basis.dim, dtype=basis.dtype, device="cuda", generator=gen)
    y = basis.empty()
    basis.apply(J, x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        basis.apply(J, x, out=y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(make_workload, n_subs, candidates=None, reps=2, time_limit_s=None, log=None):
    """Return (best, results).

    make_workload(key) -> workload for one sublattice decomposition (key is
    n_sub, or any label such as an (n_sub, superlattice) pair);
    candidates(sub_bits) -> list of tuning dicts (default_candidates if None).
    best = {"n_sub", "tuning", "hv_ms", "info"}; results lists every trial.
    """
    candidates = candidates or default_candidates
    results = []
    t_start = time.perf_counter()
    for ns in n_subs:
        w = make_workload(ns)
        sub_bits = w.cluster.n_sites // w.cluster.n_sublat
        for tn in candidates(sub_bits):
            if time_limit_s is not None and time.perf_counter() - t_start > time_limit_s:
                break
            rec = {"n_sub": ns, "tuning": dict(tn)}
            try:
                b = ed.Basis.from_workload(w, tn)
            except L.EDError as e:
                rec["error"] = e.name
                results.append(rec)
                if log:
                    log(f"[autotune] n_sub={ns} {tn}: {e.name}")
                continue
            try:
                rec["hv_ms"] = _time_apply(b, w.J, reps)
                rec["info"] = b.info()
            finally:
                b.close()
                torch.cuda.empty_cache()
            results.append(rec)
            if log:
                log(f"[autotune] n_sub={ns} {tn}: {rec['hv_ms']:.2f} ms")
    timed = [r for r in results if "hv_ms" in r]
    if not timed:
        raise RuntimeError("no candidate configuration could be built")
    best = min(timed, key=lambda r: r["hv_ms"])
    return best, results


def autotune_decompositions(make_workload_for, decompositions, n_up, top=3, **kw):
    """Rank sublattice decompositions on the host (decompose.rank_decompositions),
    then time the best `top` of them with every candidate tuning.

    make_workload_for(superlattice) -> workload whose cluster uses that
    superlattice; decompositions: (n_sub, superlattice) pairs, e.g. from
    ed_inputs.lattice.sublattice_decompositions.  Returns (best, results,
    ranking); best["n_sub"] is the (n_sub, superlattice) pair.
    """
    from . import decompose
    ranked = decompose.rank_decompositions(lambda M: make_workload_for(M).cluster, decompositions, n_up)
    keys = [(r["n_sub"], r["superlattice"]) for r in ranked if r["fits"]][:top]
    best, results = autotune(lambda key: make_workload_for(key[1]), keys, **kw)
    return best, results, ranked


def _time_batched(mb, J, reps):
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    x = torch.randn((mb.dim, mb.K), dtype=torch.complex128, device="cuda", generator=gen)
    y = mb.empty()
    mb.apply(J, x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mb.apply(J, x, out=y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune_batched(workloads, batches=(4, 8, 12, 16), lanes=(1, 2, 4), reps=1, log=None):
    """Schedule of batched launches for the sectors `workloads` (one group,
    shared cluster, n_up and couplings).

    The sectors run in consecutive groups of B (the last group holds the
    remainder).  For every B in `batches` and every group size that schedule
    needs, each lanes-per-row value is timed on the first sectors of that
    size; the schedule with the smallest summed time wins.  Returns
    {"batch", "groups": [(first, size, lanes_per_row)], "est_ms", "trials"}.
    """
    n = len(workloads)
    J = workloads[0].J
    best_of = {}   # group size -> (ms, lanes)
    trials = []
    for K in schedule_sizes(n, batches):
        for L in lanes:
            mb = ed.MultiBasis.from_workloads(workloads[:K], {"lanes_per_row": L})
            try:
                ms = _time_batched(mb, J, reps)
            finally:
                mb.close()
                torch.cuda.empty_cache()
            trials.append({"K": K, "lanes_per_row": L, "hv_ms": ms})
            if log:
                log(f"[autotune] K={K} lanes_per_row={L}: {ms:.1f} ms")
            if K not in best_of or ms < best_of[K][0]:
                best_of[K] = (ms, L)
    return dict(plan_schedule(n, batches, best_of), trials=trials)


def schedule_sizes(n, batches):
    """Group sizes the schedules with these batch sizes need for n sectors
    (full groups and remainders)."""
    return sorted({min(b, n) for b in batches} | {n % b for b in batches if n % b and b < n})


def plan_schedule(n, batches, best_of):
    """Cheapest schedule of consecutive groups for n sectors.

    best_of[size] = (ms, lanes_per_row) for every size in schedule_sizes.
    Returns {"batch", "groups": [(first, size, lanes_per_row)], "est_ms"};
    ties go to the smaller batch size.
    """
    plans = []
    for b in batches:
        b = min(b, n)
        groups = [(i, min(b, n - i)) for i in range(0, n, b)]
        plans.append((sum(best_of[k][0] for _, k in groups), b, groups))
    est, b, groups = min(plans)
    return {"batch": b, "groups": [(i, k, best_of[k][1]) for i, k in groups], "est_ms": est}


def speedup_table(results):
    """(n_sub, tuning, ms, ms / best ms) rows, fastest first."""
    timed = sorted((r for r in results if "hv_ms" in r), key=lambda r: r["hv_ms"])
    b = timed[0]["hv_ms"]
    return [(r["n_sub"], r["tuning"], r["hv_ms"], r["hv_ms"] / b) for r in timed]


__all__ = ["autotune", "autotune_batched", "autotune_decompositions", "default_candidates", "plan_schedule",
           "schedule_sizes", "speedup_table"]
