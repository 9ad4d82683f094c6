"""Planted mistakes in a copy of the oracle must fail at least one pin.

Each mutant is a textual edit of orc.c compiled into a temporary library; the
pins (worked examples, closed-form energies, definition-level matrix,
character-formula dimensions) are then run against it.  This runs on the CPU
only and never touches the product library.
"""
import math
import os
import subprocess

import numpy as np
import pytest

from ed_inputs import lattice as lat
from oracle import bruteforce as bf
from oracle import definition as de
from oracle import dimension as dm

SRC = os.path.join(os.path.dirname(bf.__file__), "orc.c")

MUTANTS = {
    "no_conjugate": ("ci = -amp * chi[2 * h + 1];", "ci = amp * chi[2 * h + 1];"),
    "inverted_norm_ratio": ("sqrt((double)stab[i] / (double)stab[j])",
                            "sqrt((double)stab[j] / (double)stab[i])"),
    "lsb_site_order": ("return (int)((s >> (n - 1 - site)) & 1ull);", "return (int)((s >> site) & 1ull);"),
    "diagonal_sign": ("d += same ? 0.25 * Jz[b] : -0.25 * Jz[b];\n        }\n        yt",
                      "d += same ? -0.25 * Jz[b] : 0.25 * Jz[b];\n        }\n        yt"),
    "ising_uses_exchange": ("d += same ? 0.25 * Jz[b] : -0.25 * Jz[b];\n        }\n        yt",
                            "d += same ? 0.25 * J[b] : -0.25 * J[b];\n        }\n        yt"),
    "ignore_compatibility": ("                if (comp) {\n                    if (want)",
                             "                if (1) {\n                    if (want)"),
    "action_inverse": ("r |= (uint64_t)get_bit(s, n, i) << (n - 1 - perm[i]);",
                       "r |= (uint64_t)get_bit(s, n, perm[i]) << (n - 1 - i);"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    src = src.replace(old, new)
    if name == "lsb_site_order":
        src = src.replace("<< (n - 1 - perm[i]);", "<< perm[i];")
        src = src.replace("(1ull << (n - 1 - p)) ^ (1ull << (n - 1 - q))", "(1ull << p) ^ (1ull << q)")
    path = os.path.join(str(tmp_path), f"liborc_{name}.so")
    csrc = os.path.join(str(tmp_path), f"orc_{name}.c")
    with open(csrc, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", path, csrc])
    return path


def xx_ring_ground_energy(n, n_up, jxy=1.0):
    """XX ring by the Jordan-Wigner map: free fermions with hopping jxy/2,
    periodic for an odd particle number and antiperiodic for an even one."""
    shift = 0.0 if n_up % 2 == 1 else 0.5
    eps = sorted(jxy * math.cos(2 * math.pi * (m + shift) / n) for m in range(n))
    return sum(eps[:n_up])


def _pins_pass():
    """The oracle pins in compact form; True if all of them hold."""
    ok = True
    # worked example, three sublattices: rep 7 via T2; T5 image 11
    c = lat.chain(6, superlattice_period=3)
    m = bf.Model(6, c.perm, c.flip, np.ones(6))
    ok &= bf.rep(m, 50) == (7, 2) and bf.act(m, 5, 50) == 11
    # 6-ring ground energy over all momenta
    c = lat.chain(6)
    best = 1e9
    for k in range(6):
        chi = lat.characters(c, k)
        m = bf.Model(6, c.perm, c.flip, chi, c.bonds, np.ones(6))
        st, stab = bf.basis(m, 3)
        if len(st):
            H = np.stack([bf.apply(m, st, stab, e.astype(complex))[0] for e in np.eye(len(st))], 1)
            best = min(best, np.linalg.eigvalsh((H + H.conj().T) / 2)[0])
    ok &= abs(best - (-1 - math.sqrt(13) / 2)) < 1e-10
    # XX ring (Jz = 0): free-fermion ground energy over all momenta
    c = lat.chain(8)
    best = 1e9
    for k in range(8):
        m = bf.Model(8, c.perm, c.flip, lat.characters(c, k), c.bonds, np.ones(8), np.zeros(8))
        st, stab = bf.basis(m, 4)
        if len(st):
            H = np.stack([bf.apply(m, st, stab, e.astype(complex))[0] for e in np.eye(len(st))], 1)
            best = min(best, np.linalg.eigvalsh((H + H.conj().T) / 2)[0])
    ok &= abs(best - xx_ring_ground_energy(8, 4)) < 1e-10
    # definition-level matrices: complex momentum on the 8-ring, full group on 12-site triangular
    cases = []
    c8 = lat.chain(8)
    cases.append((c8, lat.characters(c8, 1), 4))
    cases.append((c8, lat.characters(c8, 0), 4))
    ct = lat.triangular((2, 2), (-2, 4), spin_flip=True)
    cases.append((ct, lat.characters(ct, 0), 6))
    for cl, chi, n_up in cases:
        J = np.ones(cl.n_bonds)
        reps, Md = de.sector_matrix(cl.n_sites, n_up, cl.perm, cl.flip, chi, cl.bonds, J)
        m = bf.Model(cl.n_sites, cl.perm, cl.flip, chi, cl.bonds, J)
        st, stab = bf.basis(m, n_up)
        if len(st) != dm.sector_dimension(cl.perm, cl.flip, chi, n_up) or not np.array_equal(st, reps):
            ok = False
            continue
        Mf = np.stack([bf.apply(m, st, stab, e.astype(complex))[0] for e in np.eye(len(st))], 1)
        ok &= np.abs(Mf - Md).max() < 1e-12
    return bool(ok)


def test_pins_hold_for_real_oracle():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name, monkeypatch):
    path = _build_mutant(tmp_path, name)
    saved = bf._lib
    try:
        bf._lib = None
        monkeypatch.setattr(bf, "_LIB", path)
        monkeypatch.setattr(bf, "build", lambda force=False: path)
        assert not _pins_pass(), f"planted mistake '{name}' passed every pin"
    finally:
        bf._lib = saved
