"""Write SHA-256 digests of full sector bases, enumerated by the CPU oracle.

    python tests/golden/make_basis_digests.py [--only NAME] [--out PATH]

For each configuration the oracle enumerates every popcount-n_up
configuration in ascending order and keeps those that are their own orbit
minimum and are compatible with the irrep (Alg. "Preparation of the
distributed and symmetrized Hilbert space" on one process, with the
brute-force representative test of sec. "Sublattice coding algorithm").
Only ``oracle/`` computes anything here; ``ed_inputs`` supplies the lattice,
group and characters.

The enumeration is split into pieces of equal rank span.  Piece p holds the
sector states s with first_state[p] <= s < first_state[p+1], where
first_state[p] is the configuration of rank rank_lo[p].  Each piece records
its count and two digests:
  * sha256_states: SHA-256 of the states as little-endian uint64, ascending;
  * sha256_stab:   SHA-256 of the stabiliser sizes |Stab s| as little-endian
                   uint16, in the same order.
The output file is rewritten after every piece, so an interrupted run
resumes where it stopped.  A configuration is complete when it holds
n_pieces pieces.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from ed_inputs import workloads as wl  # noqa: E402
from oracle import bruteforce as bf  # noqa: E402

OUT = os.path.join(HERE, "basis_digests.json")
FORMAT = ("piece p holds the sector states s with first_state[p] <= s < first_state[p+1] (the last piece "
          "runs to the end); sha256_states = SHA-256 of those states as little-endian uint64 in ascending "
          "order; sha256_stab = SHA-256 of their stabiliser sizes as little-endian uint16; written by "
          "make_basis_digests.py from the CPU oracle's brute-force enumeration")

# name -> (workload factory, pieces); the site numbering is that of the
# 4-sublattice decomposition each workload uses by default
CONFIGS = {
    "square32_disorder": (lambda: wl.square_32_disorder(n_sub=4), 64),
    "triangular36": (lambda: wl.triangular_36(n_sub=4), 256),
    "square40_j1j2": (lambda: wl.square_40_j1j2(n_sub=4), 512),
}


def piece_ranks(total, n_pieces, p):
    return total * p // n_pieces, total * (p + 1) // n_pieces


def digests(states, stab):
    hs = hashlib.sha256(np.ascontiguousarray(states, dtype="<u8").tobytes()).hexdigest()
    ht = hashlib.sha256(np.ascontiguousarray(stab, dtype="<u2").tobytes()).hexdigest()
    return hs, ht


def load(path):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {"format": FORMAT, "configs": {}}


def save(path, data):
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")
    os.replace(tmp, path)


def run(name, path):
    make, n_pieces = CONFIGS[name]
    w = make()
    c = w.cluster
    m = bf.Model.from_workload(w)
    total = math.comb(c.n_sites, w.n_up)
    data = load(path)
    cfg = data["configs"].setdefault(name, {
        "workload": w.name, "n_sites": c.n_sites, "n_up": w.n_up, "group_order": int(c.n_elems),
        "n_configurations": total, "n_pieces": n_pieces, "pieces": [], "dim": None})
    done = len(cfg["pieces"])
    t_start = time.time()
    for p in range(done, n_pieces):
        lo, hi = piece_ranks(total, n_pieces, p)
        t0 = time.time()
        states, stab = bf.basis_range(m, w.n_up, lo, hi)
        assert np.all(states[1:] > states[:-1])
        hs, ht = digests(states, stab)
        cfg["pieces"].append({"rank_lo": lo, "first_state": bf.unrank(c.n_sites, w.n_up, lo),
                              "count": int(len(states)), "sha256_states": hs, "sha256_stab": ht})
        if p + 1 == n_pieces:
            cfg["dim"] = int(sum(q["count"] for q in cfg["pieces"]))
        save(path, data)
        print(f"[digest] {name} piece {p + 1}/{n_pieces}: {len(states)} states, {time.time() - t0:.1f} s "
              f"(elapsed {time.time() - t_start:.0f} s)", flush=True)
    print(f"[digest] {name} complete: D = {cfg['dim']}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=sorted(CONFIGS), action="append")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    for name in args.only or list(CONFIGS):
        run(name, args.out)


if __name__ == "__main__":
    main()
