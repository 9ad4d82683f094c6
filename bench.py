"""Benchmark: symmetry-sector H.v throughput inside FP64 Lanczos on one MI355X.

A step is one Lanczos iteration of the sector Hamiltonian: one fused H.v
(representative search, index lookup, bond-loop gather) plus the FP64 vector
updates, all in the library's HIP kernels.  value = H.v terms per second =
(D + kept off-diagonal terms) per H.v x steps / elapsed seconds, with every
input already resident in HBM.  The basis build is timed and reported
separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload: J1-J2 Heisenberg (J2/J1 = 0.5) on the 40-site tilted square
cluster, 40 translations x C4 x spin flip, Gamma sector at Sz = 0
(D = 430,909,650).  Inputs are synthetic and seeded.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H·v nonzero terms/sec + achieved HBM GB/s fraction, N=36/40 sector Lanczos"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes (FP64 real, gather form): per row the state, x_i and y_i
# (the stabiliser size travels inside the state word) -- counted as 25 B with
# a separate 1-byte norm; per kept off-diagonal term x_j (8 B), n_j (1 B) and
# one 8 B index probe.  Complex sectors add 8 B to x_i, x_j and y_i.
BYTES_ROW_REAL, BYTES_TERM_REAL = 25.0, 17.0
BYTES_ROW_CPLX, BYTES_TERM_CPLX = 41.0, 25.0

# Measured HBM bytes per H.v launch: FETCH_SIZE and WRITE_SIZE runs of
# rocprofv3, scaled by what the same counters read for a plain device copy of
# known size (x2.0 and x1.0).  A figure is valid only for the kernel sources it
# was taken on (sha256 of ed_kernels.hip + ed_device.hpp + ed_internal.hpp,
# concatenated) and the same configuration; otherwise traffic is reported as
# null.
KERNEL_SRCS = [os.path.join(ROOT, "paper_1804_05028_amd", "csrc", f)
               for f in ("ed_kernels.hip", "ed_device.hpp", "ed_internal.hpp")]
MEASURED_TRAFFIC = {
    # (workload, n_sublat, index, chunk_bits): (kernel sha256, fetch bytes, write bytes, profile)
    ("square40_j1j2", 4, "hash-slot", 5): (
        "65f865045fddf0948f6d1fd330e70d6f17e56c8eb5eeaf09e04b20826133bfd4", 4.69342e+12, 3.44728e+09,
        "profiles/k_apply_square40_j1j2_ns4.md"),
    ("triangular36_k1", 4, "hash-slot", 5): (
        "65f865045fddf0948f6d1fd330e70d6f17e56c8eb5eeaf09e04b20826133bfd4", 1.92584e+12, 4.03337e+09,
        "profiles/k_apply_triangular36_k1_complex.md"),
    ("triangular36_tV", 4, "hash-slot", 5): (
        "65f865045fddf0948f6d1fd330e70d6f17e56c8eb5eeaf09e04b20826133bfd4", 3.03372e+11, 3.36083e+08,
        "profiles/k_apply_fermions_triangular36_tV.md"),
}


# Integer-op rate of the representative search, from the SQ_INSTS_VALU_INT32 /
# _INT64 counters of the same profile (wave instructions x 64 lanes / kernel
# time); not measured by this script.
MEASURED_INT_OPS = {
    ("square40_j1j2", 4, "hash-slot", 5): {
        "rate": 9.53e12, "unit": "lane-ops/s", "valu_issue_floor_frac": 0.58,
        "source": "profiles/k_apply_square40_j1j2_ns4.md (rocprofv3 --pmc SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64), "
                  "not measured in this run"},
}


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key):
    """(fetch bytes, write bytes, profile) of the current kernel sources, or None."""
    rec = MEASURED_TRAFFIC.get(key)
    if rec is None or kernel_digest() != rec[0]:
        return None
    return rec[1], rec[2], rec[3]


AUTOTUNE_NSUB = {"square40_j1j2": [4, 5], "square40_j1j2j3": [4, 5], "triangular36": [3, 4], "triangular36_k1": [4],
                 "square32_disorder": [4, 8], "square16": [2, 4]}


def _workload(name, n_sub):
    from ed_inputs import workloads as wl
    if name == "square40_j1j2":
        return wl.square_40_j1j2(n_sub=n_sub or 4), "J1-J2 square 40 (6,2)x(-2,6), 40T x C4 x flip, Gamma.A.even, Sz=0"
    if name == "square40_j1j2j3":
        return (wl.square_40_j1j2j3(n_sub=n_sub or 4),
                "J1-J2-J3 square 40 (6,2)x(-2,6), J2=0.5 J3=0.25, 40T x C4 x flip, Gamma.A.even, Sz=0")
    if name == "triangular36":
        return wl.triangular_36(n_sub=n_sub or 4), "Heisenberg triangular 36 (6,0)x(0,6), 36T x C6v x flip, Gamma.A1.even, Sz=0"
    if name == "square32_disorder":
        from ed_inputs import lattice as lat
        w = wl.square_32_disorder(n_sub=n_sub or 4)
        # the translation sector of a disordered H is that of its orbit-averaged couplings
        w = wl.Workload(w.name, w.cluster, w.chi, w.n_up, lat.orbit_mean(w.J, lat.bond_orbits(w.cluster)),
                        w.description)
        return w, "Heisenberg square 32 (4,4)x(-4,4), 32T, k=0, orbit-averaged J_b ~ U(0.8,1.2)"
    if name == "triangular36_k1":
        return (wl.triangular_36_momentum(1, n_sub=n_sub or 4),
                "Heisenberg triangular 36 (6,0)x(0,6), 36 T, momentum sector k=1 (complex), Sz=0")
    if name == "square16":
        return wl.square_4x4(n_sub=n_sub or 4), "Heisenberg square 16 (4x4), 16T, k=0, Sz=0"
    if name == "triangular36_tV":
        return (wl.triangular_36_tV(n_sub=n_sub or 4, V=1.0),
                "spinless fermions t=1 V=1, triangular 36 (6,0)x(0,6), 18 particles, 36T x C6, Gamma.A")
    raise SystemExit(f"unknown workload {name}")


def _allk_workloads(n_sub, which="all"):
    from ed_inputs import workloads as wl
    return wl.triangular_36_all_momenta(n_sub or 4, which)


def _gamma_workloads(n_sub):
    from ed_inputs import workloads as wl
    return wl.triangular_36_gamma(n_sub or 4)


BATCHED_WORKLOADS = {
    "triangular36_allk": "36 T, {n} momentum sectors ({which})",
    "triangular36_gamma": "36 T x C6v x flip, the {n} one-dimensional irreps at Gamma",
}


def bench_allk(args):
    """Batched all-sector H.v and Lanczos against one launch per sector."""
    import torch
    from paper_1804_05028_amd import ed
    if args.workload == "triangular36_gamma":
        ws = _gamma_workloads(args.n_sub)
    else:
        ws = _allk_workloads(args.n_sub, args.sectors)
    J = ws[0].J
    reps = max(args.hv_reps, 1)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    if args.profile_only:
        # the first group only: build, one untimed and --hv-reps timed batched
        # launches, then one plain copy of the vector (byte-counter calibration)
        mb = ed.MultiBasis.from_workloads(ws[:args.batch])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        x = torch.randn((mb.dim, mb.K), dtype=torch.complex128, device="cuda", generator=gen)
        y = mb.empty()
        mb.apply(J, x, out=y)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            mb.apply(J, x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        _, sh = mb.stats()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"hv_ms": ev0.elapsed_time(ev1) / reps, "K": mb.K, "shared_terms": int(sh),
                          "lanes_per_row": mb.info()["lanes_per_row"], "copy_bytes_each_way": x.numel() * 16}))
        mb.close()
        return

    # one launch per sector, sector by sector (each with its own basis and index)
    per_ms, per_terms = 0.0, 0
    for w in ws:
        b = ed.Basis.from_workload(w)
        n_diag, kept, _ = b.stats()
        per_terms += n_diag + kept
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        x = torch.randn(b.dim, dtype=b.dtype, device="cuda", generator=gen)
        y = b.empty()
        b.apply(J, x, out=y)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            b.apply(J, x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        per_ms += ev0.elapsed_time(ev1) / reps
        print(f"[bench] sector {w.name}: D={b.dim} {ev0.elapsed_time(ev1) / reps:.1f} ms", file=sys.stderr, flush=True)
        del x, y
        b.close()
        torch.cuda.empty_cache()

    # batched: sectors in groups of --batch (or the autotuned schedule), search
    # and lookup shared per group
    tuned = None
    if args.autotune:
        from paper_1804_05028_amd import autotune as at
        tuned = at.autotune_batched(ws, log=lambda m: print(m, file=sys.stderr, flush=True))
        groups = [(ws[i:i + k], lanes) for i, k, lanes in tuned["groups"]]
    else:
        groups = [(ws[i:i + args.batch], 0) for i in range(0, len(ws), args.batch)]
    hv_ms, terms, shared_terms, lz_s, lz_steps, build_s, e0 = 0.0, 0, 0, 0.0, 0, 0.0, []
    info = None
    for grp, lanes in groups:
        t0 = time.perf_counter()
        mb = ed.MultiBasis.from_workloads(grp, {"lanes_per_row": lanes} if lanes else None)
        torch.cuda.synchronize()
        build_s += time.perf_counter() - t0
        info = mb.info()
        t, sh = mb.stats()
        terms += int(t.sum())
        shared_terms += sh
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        x = torch.randn((mb.dim, mb.K), dtype=torch.complex128, device="cuda", generator=gen)
        y = mb.empty()
        mb.apply(J, x, out=y)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            mb.apply(J, x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        hv_ms += ev0.elapsed_time(ev1) / reps
        del y
        torch.cuda.empty_cache()
        if args.warmup > 0:
            mb.lanczos(J, x, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = mb.lanczos(J, x, args.steps)
        torch.cuda.synchronize()
        lz_s += time.perf_counter() - t0
        lz_steps = max(lz_steps, int(res["n_done"].max()))
        e0 += [float(e[0]) for e in res["eigenvalues"] if len(e)]
        del x
        mb.close()
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC,
        "value": terms * lz_steps / lz_s,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": lz_steps,
        "warmup": args.warmup,
        "ms_per_step": lz_s * 1e3 / max(lz_steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_sectors": len(ws),
                   "batch": tuned["batch"] if tuned else args.batch,
                   "description": "Heisenberg triangular 36 (6,0)x(0,6), "
                                  + BATCHED_WORKLOADS[args.workload].format(n=len(ws), which=args.sectors)
                                  + ", Sz=0",
                   "shared_rows": info["dim"] if info else 0, "n_sublat": info["n_sublat"] if info else 0,
                   "parallelism": "1 GPU"},
        "batched_hv_ms": hv_ms,
        "per_sector_hv_ms": per_ms,
        "batched_speedup": per_ms / hv_ms if hv_ms else None,
        "terms_per_hv": terms,
        "per_sector_terms_per_hv": per_terms,
        "shared_terms_per_hv": shared_terms,
        "batched_hv_terms_per_s": terms / (hv_ms * 1e-3) if hv_ms else None,
        "per_sector_hv_terms_per_s": per_terms / (per_ms * 1e-3) if per_ms else None,
        "basis_build_s": build_s,
        "lowest_e0": min(e0) if e0 else None,
    }
    if tuned is not None:
        out["autotune"] = {"groups": tuned["groups"], "est_ms": tuned["est_ms"], "trials": len(tuned["trials"])}
    print(json.dumps(out))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_square16(steps=200):
    """The oracle on the 16-site square (4x4, k = 0, D = 822): basis, one full
    H.v and a 200-step Lanczos, timed on the host cores."""
    from ed_inputs import vectors as vec
    from ed_inputs import workloads as wl
    from oracle import bruteforce as bf
    from oracle import lanczos as olz
    w = wl.square_4x4()
    m = bf.Model.from_workload(w)
    t0 = time.perf_counter()
    st, stab = bf.basis(m, w.n_up)
    t_basis = time.perf_counter() - t0
    x = vec.normal_vector(len(st))
    t0 = time.perf_counter()
    _, kept, _ = bf.apply(m, st, stab, x)
    t_hv = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = olz.lanczos(lambda v: bf.apply(m, st, stab, v)[0], x, steps)
    t_lz = time.perf_counter() - t0
    return {"workload": "square16 (4x4, 16 T, k=0, Sz=0)", "dim": int(len(st)), "terms_per_hv": int(len(st) + kept),
            "basis_s": t_basis, "hv_s": t_hv, "lanczos_steps": int(res["n_done"]), "lanczos_s": t_lz,
            "e0": float(res["eigenvalues"][0]), "cores": int(bf.lib().orc_max_threads()), "kind": "oracle"}


def time_adjoint(basis, J, x, reps, hv_ms):
    """gx = H gy plus the per-bond sums, and the per-bond sums alone (both
    synchronise, so wall time on the host is the device time)."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(vec_seed_target())
    gy = torch.randn(basis.dim, dtype=basis.dtype, device="cuda", generator=gen)
    basis.backward(J, x, gy)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        basis.backward(J, x, gy)          # gx = H gy and gJ_b (synchronises)
    full_ms = (time.perf_counter() - t0) * 1e3 / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        basis.backward(J, x, gy, want_gx=False)
    gj_ms = (time.perf_counter() - t0) * 1e3 / reps
    print(f"[bench] adjoint {full_ms:.2f} ms (per-bond sums {gj_ms:.2f} ms, H.v {hv_ms:.2f} ms)", file=sys.stderr,
          flush=True)
    return {"backward_ms": full_ms, "per_bond_sums_ms": gj_ms, "hv_ms": hv_ms, "backward_over_hv": full_ms / hv_ms,
            "n_bonds": int(basis.n_bonds),
            "path": ("one fused pass for gx and the per-bond sums (real sector, hash slots; its 32-byte adjoint "
                     "slot table allocated by the untimed first call)") if not basis.is_complex
            else "H gy and the per-bond sums as two passes"}


def vec_seed_target():
    from ed_inputs import vectors as vec
    return vec.SEED_TARGET


def bench_adjoint_c5(reps):
    """Adjoint on the 32-site disorder workload (orbit-averaged couplings,
    translation sector k = 0): backward time against one H.v."""
    import torch
    from paper_1804_05028_amd import ed
    w, desc = _workload("square32_disorder", 0)
    b = ed.Basis.from_workload(w)
    try:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        x = torch.randn(b.dim, dtype=b.dtype, device="cuda", generator=gen)
        y = b.empty()
        b.apply(w.J, x, out=y)
        _, pack_ms, kernel_ms = b.apply_timed(w.J, x, out=y, reps=reps)
        out = time_adjoint(b, w.J, x, reps, pack_ms + kernel_ms)
        out.update(workload="square32_disorder", description=desc, dim=int(b.dim))
        return out
    finally:
        b.close()
        torch.cuda.empty_cache()


def bench_gamma_batched(reps):
    """The eight Gamma irreps of the 36-site triangular full group: one
    batched H.v over shared representatives against one launch per sector."""
    import torch
    from paper_1804_05028_amd import ed
    ws = _gamma_workloads(4)
    J = ws[0].J
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per_ms, per = 0.0, []
    for w in ws:
        b = ed.Basis.from_workload(w)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        x = torch.randn(b.dim, dtype=b.dtype, device="cuda", generator=gen)
        y = b.empty()
        b.apply(J, x, out=y)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            b.apply(J, x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        per.append(round(ms, 3))
        per_ms += ms
        del x, y
        b.close()
    mb = ed.MultiBasis.from_workloads(ws)
    try:
        info = mb.info()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(0)
        x = torch.randn((mb.dim, mb.K), dtype=torch.complex128, device="cuda", generator=gen)
        y = mb.empty()
        mb.apply(J, x, out=y)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            mb.apply(J, x, out=y)
        ev1.record()
        torch.cuda.synchronize()
        bat_ms = ev0.elapsed_time(ev1) / reps
        t, shared = mb.stats()
        del x, y
    finally:
        mb.close()
        torch.cuda.empty_cache()
    print(f"[bench] Gamma irreps: per-sector {per_ms:.1f} ms, batched {bat_ms:.1f} ms ({per_ms / bat_ms:.2f}x)",
          file=sys.stderr, flush=True)
    return {"workload": "triangular36_gamma", "description": "36 T x C6v x flip, the 8 one-dimensional irreps at "
                                                              "Gamma, Sz=0", "n_sectors": len(ws),
            "per_sector_ms": per, "per_sector_total_ms": per_ms, "batched_ms": bat_ms, "speedup": per_ms / bat_ms,
            "terms_per_hv": int(t.sum()), "shared_terms_per_hv": int(shared), "lanes_per_row": info["lanes_per_row"],
            "chi_in_lds": info["chi_in_lds"], "chi_signs": info["chi_signs"],
            "timing": f"torch.cuda events on the launch stream, mean of {reps}"}


def wl_mod():
    from ed_inputs import workloads as wl
    return wl


def cpu_baseline(w, rows, seed):
    """Oracle (brute-force C) on a bounded sample of rows of the same H.v."""
    import numpy as np
    from ed_inputs import vectors as vec
    from oracle import bruteforce as bf
    amp = lambda s: vec.hashed_amplitudes(s, salt=1, complex_=w.is_complex)  # noqa: E731
    if isinstance(w, wl_mod().FermionWorkload):
        c = w.cluster
        m = bf.FermionModel(c.n_sites, c.perm, w.chi, c.bonds, w.t, w.V)
        sample = bf.random_representatives(bf.Model(c.n_sites, c.perm, c.flip, np.ones(c.n_elems)), w.n_up,
                                           2 * rows, seed)
        _, _, _, _, comp = bf.frep_many(m, sample)
        sample = sample[comp][:rows]
        t0 = time.perf_counter()
        _, kept, _, _ = bf.frows_apply(m, sample, amp)
    else:
        m = bf.Model.from_workload(w)
        sample = bf.random_representatives(m, w.n_up, rows, seed)
        t0 = time.perf_counter()
        _, kept, _, _ = bf.rows_apply(m, sample, amp)
    dt = time.perf_counter() - t0
    return dict(value=(kept + len(sample)) / dt, unit="terms/s", cores=int(bf.lib().orc_max_threads()),
                kind="oracle", cpu_model=cpu_model(),
                sample=f"{len(sample)} seeded random representatives (seed {seed}), all their H.v terms "
                       f"({kept + len(sample)} terms) by brute-force group application, {dt:.1f} s")


PROBE_BYTES = 1 << 32       # 4 GiB: far beyond the 4 MB L2 of an XCD and the 256 MB MALL


def random_read_probe(reps=5, iters=512, slot_bytes=16):
    """Independent random slot reads per second over a 4 GiB device buffer
    (ed_probe_random_reads): 16-byte slots as real sectors read them, or
    32-byte slots read as two 16-byte loads as complex sectors do.  One 128 B
    line request per slot: the rate that bounds the H.v gather's one slot
    read per term."""
    import torch
    from paper_1804_05028_amd import _lib as L
    buf = torch.zeros(PROBE_BYTES, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rate = L.ed_probe_random_reads(buf, PROBE_BYTES, iters, reps, torch.cuda.current_stream().cuda_stream,
                                   slot_bytes=slot_bytes)
    del buf
    torch.cuda.empty_cache()
    return {"reads_per_s": rate, "slot_bytes": slot_bytes, "buffer_bytes": PROBE_BYTES, "reps": reps,
            "kernel": "ed_probe_random_reads (two 1024-thread blocks per CU, two slots in flight per lane)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="square40_j1j2")
    ap.add_argument("--n-sub", type=int, default=0)
    ap.add_argument("--limits-bits", type=int, default=0)
    ap.add_argument("--index-mode", type=int, default=0, help="0 hash slots, 1 the paper's Limits + binary search")
    ap.add_argument("--chunk-bits", type=int, default=0)
    ap.add_argument("--hash-load-pct", type=int, default=0)
    ap.add_argument("--table-entry-bytes", type=int, default=0)
    ap.add_argument("--search-mode", type=int, default=0, help="1 one-stage, 2 two-stage representative search")
    ap.add_argument("--lanczos-direct", action="store_true",
                    help="launch the Lanczos step kernels directly instead of replaying a HIP graph")
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--hv-reps", type=int, default=5, help="extra timed H.v launches for the roofline")
    ap.add_argument("--cpu-rows", type=int, default=40000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true", help="build, then run --hv-reps H.v launches only")
    ap.add_argument("--batch", type=int, default=16, help="sectors per batched launch (triangular36_allk)")
    ap.add_argument("--sectors", default="all", choices=["all", "inequivalent"],
                    help="triangular36_allk: all 36 momenta, or the 20 inequivalent ones")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the adjoint (dL/dx = H gy and the per-bond sums) on the same basis")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the batched Gamma-irrep, adjoint and small-oracle measurements")
    ap.add_argument("--probe-only", action="store_true",
                    help="run only the random-read probe (the ceiling of the H.v gather) and print its rate")
    ap.add_argument("--autotune", action="store_true",
                    help="search sublattice decompositions and launch tunings first, then bench the fastest")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the H.v path runs on one GPU; sharding a sector over several GPUs "
                                   "is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1804_05028_amd import ed

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs an MI355X GPU")
    torch.cuda.set_device(0)
    if args.probe_only:
        print(json.dumps([random_read_probe(slot_bytes=16), random_read_probe(slot_bytes=32)]))
        return
    if args.workload in BATCHED_WORKLOADS:
        return bench_allk(args)
    w, desc = _workload(args.workload, args.n_sub)
    tuning = dict(limits_bits=args.limits_bits, index_mode=args.index_mode, block_threads=args.block_threads,
                  blocks_per_cu=args.blocks_per_cu, chunk_bits=args.chunk_bits, hash_load_pct=args.hash_load_pct,
                  table_entry_bytes=args.table_entry_bytes, search_mode=args.search_mode,
                  lanczos_direct=int(args.lanczos_direct))
    tuned = None
    if args.autotune:
        from paper_1804_05028_amd import autotune as at
        best, results = at.autotune(lambda ns: _workload(args.workload, ns)[0], AUTOTUNE_NSUB[args.workload],
                                    reps=2, log=lambda m: print(m, file=sys.stderr, flush=True))
        w, desc = _workload(args.workload, best["n_sub"])
        tuning = dict(best["tuning"], lanczos_direct=int(args.lanczos_direct))
        tuned = {"n_sub": best["n_sub"], "tuning": tuning, "hv_ms": best["hv_ms"],
                 "trials": [(r["n_sub"], r["tuning"], r.get("hv_ms"), r.get("error")) for r in results]}
    print(f"[bench] building basis: {desc}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    fermions = isinstance(w, wl_mod().FermionWorkload)
    basis = (ed.FermionBasis if fermions else ed.Basis).from_workload(w, tuning)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = basis.info()
    D = basis.dim
    _, kept, dropped = basis.stats()
    terms = D + kept
    print(f"[bench] D={D} kept={kept} dropped={dropped} build={build_s:.2f}s info={info}", file=sys.stderr,
          flush=True)

    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    dt = basis.dtype
    x = torch.randn(D, dtype=dt, device="cuda", generator=gen)
    x /= torch.linalg.norm(x)
    J, Jz = (w.t, w.V) if fermions else (w.J, None)

    # ---- H.v kernel timing: HIP events recorded by the library on the launch
    # stream around the scatter of x into the index and around the kernel ------
    y = basis.empty()
    if fermions:
        basis.apply(J, x, out=y, V=Jz)
    else:
        basis.apply(J, x, out=y)
    torch.cuda.synchronize()
    _, pack_ms, kernel_ms = basis.apply_timed(J, x, out=y, reps=args.hv_reps, Jz=Jz)
    hv_ms = pack_ms + kernel_ms
    print(f"[bench] H.v kernel {kernel_ms:.2f} ms + scatter {pack_ms:.2f} ms  ({terms / hv_ms * 1e3:.3e} terms/s)",
          file=sys.stderr, flush=True)
    if args.profile_only:
        # calibration for the HBM byte counters: one plain copy of D values
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"hv_ms": hv_ms, "terms": terms, "D": D, "copy_bytes_each_way": D * x.element_size()}))
        return

    adjoint = None
    if args.adjoint:
        adjoint = time_adjoint(basis, J, x, args.hv_reps, hv_ms)

    # ---- Lanczos steps ----------------------------------------------------------
    if args.warmup > 0:
        basis.lanczos(J, x, args.warmup, **({"V": Jz} if fermions else {}))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = basis.lanczos(J, x, args.steps, **({"V": Jz} if fermions else {}))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_done = int(res["n_done"])
    e0_after = float(res["eigenvalues"][0]) if len(res["eigenvalues"]) else None
    ms_per_step = elapsed * 1e3 / max(steps_done, 1)
    value = terms * steps_done / elapsed

    cplx = basis.is_complex
    br, bt = (BYTES_ROW_CPLX, BYTES_TERM_CPLX) if cplx else (BYTES_ROW_REAL, BYTES_TERM_REAL)
    alg_bytes = D * br + kept * bt
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    index_name = ["hash-slot", "limits"][info["index_mode"]]
    key = (args.workload, info["n_sublat"], index_name, info["chunk_bits"])
    meas = measured_traffic(key)
    traffic = meas[0] + meas[1] if meas else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "traffic_source": (f"{meas[2]} (rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE, scaled by a plain copy), "
                                   "not measured in this run") if meas else None,
                "traffic_gbs": round(traffic / (kernel_ms * 1e-3) / 1e9, 1) if traffic else None,
                "lines_per_term": round(meas[0] / 128.0 / kept, 3) if meas and kept else None,
                "kernel": "k_apply (fused H.v)", "alg_bytes_per_launch": alg_bytes,
                "alg_bytes_per_unit": {"row": br, "kept_term": bt},
                "launch_ms": round(kernel_ms, 3), "scatter_ms": round(pack_ms, 3),
                "timing": "HIP events recorded on the launch stream around the k_apply kernel, mean of "
                          f"{args.hv_reps} launches"}

    int_ops = MEASURED_INT_OPS.get(key) if traffic else None
    del x, y, res
    probe = random_read_probe(slot_bytes=32 if cplx else 16)
    if meas:
        # line requests the H.v kernel issues per second, against the probe's rate
        kernel_lines = meas[0] / 128.0 / (kernel_ms * 1e-3)
        probe["kernel_line_requests_per_s"] = round(kernel_lines, 1)
        probe["kernel_frac_of_probe"] = round(kernel_lines / probe["reads_per_s"], 4)
    roofline["random_read_ceiling"] = probe
    basis.close()
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] CPU oracle baseline on {args.cpu_rows} rows", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, args.cpu_rows, 2)

    extras = {}
    if args.workload == "square40_j1j2" and not args.no_extras:
        extras["batched"] = bench_gamma_batched(args.hv_reps)
        extras["adjoint"] = bench_adjoint_c5(args.hv_reps)
        if not args.no_cpu_baseline:
            extras["oracle_square16"] = oracle_square16()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cplx else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n_sites": w.cluster.n_sites,
                   "n_up": w.n_up, "group_order": int(w.cluster.n_elems), "dim": D,
                   "terms_per_hv": terms, "offdiag_kept": kept, "offdiag_dropped": dropped,
                   "n_sublat": info["n_sublat"], "index_mode": index_name,
                   "chunk_bits": info["chunk_bits"], "lds_bytes": info["lds_bytes"], "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "int_ops": int_ops,
        "hv_terms_per_s": terms / (hv_ms * 1e-3),
        "hv_ms": round(hv_ms, 3),
        "basis_build_s": build_s,
        "lanczos_e0_after_steps": e0_after,
    }
    if tuned is not None:
        out["autotune"] = tuned
    if adjoint is not None:
        out["adjoint"] = adjoint
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
