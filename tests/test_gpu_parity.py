"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact for the basis (representatives, stabiliser sizes) and term counts;
FP64 H.v within 1e-12 relative (norm-wise, and element-wise with an absolute
floor of 1e-12 * max|y|, since gather and scatter orders round differently);
Lanczos eigenvalues within 1e-10 for converged Ritz values.
"""
import math

import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import dimension as dm
from oracle import lanczos as olz

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _small_workloads():
    out = [
        ("square16_k0", wl.square_4x4()),
        ("square16_k5", wl.square_4x4(momentum_index=5)),
        ("square16_full_n2", wl.square_4x4(n_sub=2, group="full")),
        ("tri12_A1_even", wl.triangular_12()),
        ("sq20_j1j2_n5", wl.square_20_j1j2(n_sub=5)),
        ("sq20_j1j2_n10", wl.square_20_j1j2(n_sub=10)),
        ("tri12_n1_k1", wl.triangular_12(n_sub=1, spin_flip=False, momentum_index=1, rotations=False,
                                         mirrors=False)),
    ]
    c = lat.chain(12, superlattice_period=3, reflection=True, spin_flip=True)
    chars = lat.point_group_chars_1d(c.point_group)
    out.append(("chain12_odd", wl.Workload("chain12", c, lat.characters(c, 0, chars[-1], -1), 6, np.ones(12))))
    c = lat.chain(14, superlattice_period=7)
    out.append(("chain14_k3_nup5", wl.Workload("chain14", c, lat.characters(c, 3), 5, np.ones(14))))
    c = lat.square((3, 1), (-1, 3), rotations=True)
    pc = lat.point_group_chars_1d(c.point_group)
    cplx = [p for p in pc if np.abs(p.imag).max() > 0.5][0]
    out.append(("sq10_C4_complex", wl.Workload("sq10", c, lat.characters(c, 0, cplx), 5, np.ones(c.n_bonds))))
    return out


SMALL = _small_workloads()


# the paper's Limits + binary-search index, and a narrow action-table split
LIMITS = {"index_mode": 1}
VARIANTS = [("square16_k0", LIMITS), ("sq20_j1j2_n5", LIMITS), ("sq10_C4_complex", LIMITS),
            ("chain14_k3_nup5", LIMITS), ("sq20_j1j2_n5", {"chunk_bits": 2, "block_threads": 256}),
            ("tri12_A1_even", {"chunk_bits": 3, "hash_load_pct": 85}),
            ("sq10_C4_complex", {"hash_load_pct": 90, "table_entry_bytes": 4}),
            ("chain12_odd", {"hash_load_pct": 80, "block_threads": 1024}),
            ("sq20_j1j2_n10", {"table_entry_bytes": 1}), ("sq20_j1j2_n5", {"table_entry_bytes": 4, "index_mode": 1}),
            ("tri12_n1_k1", {"table_entry_bytes": 1, "chunk_bits": 5})]


@pytest.fixture(scope="module")
def built():
    ed = _ed()
    cache = {}
    for name, w in SMALL:
        print(f"[build] {name}", flush=True)
        cache[name] = (w, ed.Basis.from_workload(w))
    yield cache
    for _, (_, b) in cache.items():
        b.close()


@pytest.mark.parametrize("name,tuning", VARIANTS, ids=[f"{n}-{sorted(t.items())}" for n, t in VARIANTS])
def test_index_and_table_variants(name, tuning):
    ed = _ed()
    w = dict(SMALL)[name]
    b = ed.Basis.from_workload(w, tuning)
    try:
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        assert np.array_equal(b.states(), st)
        x = vec.normal_vector(len(st), seed=4, complex_=w.is_complex)
        y_ref, kept, dropped = bf.apply(m, st, stab, x)
        y = b.apply(w.J, torch.as_tensor(x).cuda()).cpu().numpy()
        assert np.linalg.norm(y - y_ref) <= RTOL * np.linalg.norm(y_ref)
        assert b.stats() == (len(st), kept, dropped)
        info = b.info()
        assert info["index_mode"] == tuning.get("index_mode", 0)
        if "chunk_bits" in tuning:
            assert info["chunk_bits"] == tuning["chunk_bits"]
    finally:
        b.close()


WAVES = [(th, sm) for th in (512, 1024) for sm in (1, 2)]


@pytest.mark.parametrize("threads,search", WAVES, ids=[f"t{t}_s{s}" for t, s in WAVES])
def test_every_wave_of_a_block_with_one_byte_single_chunk_tables(threads, search):
    """Blocks of 8 and 16 waves over a 1321-row sector with 1-byte,
    single-chunk action tables (the smallest LDS footprint): every row, on
    repeated launches, against the oracle.  Rows 256 onwards are computed by
    the second and later waves of each SIMD."""
    ed = _ed()
    w = wl.square_20_j1j2(n_sub=4)
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    x = vec.normal_vector(len(st), seed=9)
    y_ref, _, _ = bf.apply(m, st, stab, x)
    b = ed.Basis.from_workload(w, {"table_entry_bytes": 1, "search_mode": search, "block_threads": threads})
    try:
        info = b.info()
        assert (info["table_entry_bytes"], info["chunk_bits"], info["search_mode"]) == (1, 5, search)
        xd = torch.as_tensor(x).cuda()
        for _ in range(3):
            y = b.apply(w.J, xd).cpu().numpy()
            assert np.abs(y - y_ref).max() <= RTOL * np.abs(y_ref).max()
    finally:
        b.close()


@pytest.mark.parametrize("threads", [512, 1024])
@pytest.mark.parametrize("case", ["square16_k3", "square16_k5_u8", "sq16T_k1_fermions"])
def test_every_wave_of_a_block_complex_and_fermionic(threads, case):
    """The same for complex sectors (32-byte slots, two loads per slot) with 2-
    and 1-byte tables, and for a fermionic complex momentum sector (2-byte
    fermionic entries): every row of 8 and 16 waves per block, three launches,
    against the oracle."""
    ed = _ed()
    x = None
    if case.endswith("fermions"):
        c = lat.square((4, 0), (0, 4), rotations=False, mirrors=False, superlattice=wl.SQ_2X2, name="sq16T_4sub")
        w = wl.FermionWorkload("sq16T_k1", c, lat.characters(c, 1), 7, np.full(c.n_bonds, 1.0), np.full(c.n_bonds, 0.4))
        m = bf.FermionModel(c.n_sites, c.perm, w.chi, c.bonds, w.t, w.V)
        st, stab = bf.fbasis(m, w.n_part)
        x = vec.normal_vector(len(st), seed=9, complex_=True)
        y_ref, _, _ = bf.fapply(m, st, stab, x)
        b = ed.FermionBasis.from_workload(w, {"block_threads": threads})
        run = lambda xd: b.apply(w.t, xd, V=w.V)
    else:
        w = wl.square_4x4(momentum_index=3 if case == "square16_k3" else 5)
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, w.n_up)
        x = vec.normal_vector(len(st), seed=9, complex_=True)
        y_ref, _, _ = bf.apply(m, st, stab, x)
        b = ed.Basis.from_workload(w, {"block_threads": threads, **({"table_entry_bytes": 1} if case.endswith("u8") else {})})
        run = lambda xd: b.apply(w.J, xd)
    try:
        assert b.is_complex and b.dim > 256
        xd = torch.as_tensor(x).cuda()
        for _ in range(3):
            y = run(xd).cpu().numpy()
            assert np.abs(y - y_ref).max() <= RTOL * np.abs(y_ref).max()
    finally:
        b.close()


@pytest.mark.parametrize("name", [n for n, _ in SMALL])
def test_basis_bit_exact(built, name):
    w, b = built[name]
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    assert b.dim == len(st) == dm.sector_dimension(w.cluster.perm, w.cluster.flip, w.chi, w.n_up)
    assert np.array_equal(b.states(), st)
    assert np.array_equal(b.norms().astype(np.int32), stab)


@pytest.mark.parametrize("name", [n for n, _ in SMALL])
def test_apply_parity(built, name):
    w, b = built[name]
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    x = vec.normal_vector(len(st), seed=vec.SEED_VECTOR, complex_=w.is_complex)
    y_ref, kept, dropped = bf.apply(m, st, stab, x)
    xt = torch.as_tensor(x).cuda()
    y = b.apply(w.J, xt).cpu().numpy()
    err = np.linalg.norm(y - y_ref) / max(np.linalg.norm(y_ref), 1e-300)
    assert err <= RTOL, err
    assert np.abs(y - y_ref).max() <= RTOL * max(np.abs(y_ref).max(), 1e-300) * 10
    nd, nk, ndrop = b.stats()
    assert (nd, nk, ndrop) == (len(st), kept, dropped)


def test_square16_counts_and_energy(built):
    w, b = built["square16_k0"]
    assert b.dim == 822
    assert b.stats() == (822, 14048, 0)
    v0 = torch.as_tensor(vec.normal_vector(822)).cuda()
    res = b.lanczos(w.J, v0, 200)
    assert abs(res["eigenvalues"][0] - (-11.2284832084)) < 1e-9
    assert abs(res["eigenvalues"][0] / 16 - (-0.701780)) < 5e-7


@pytest.mark.parametrize("name", ["square16_k0", "tri12_A1_even", "sq20_j1j2_n5", "chain14_k3_nup5",
                                  "sq10_C4_complex"])
def test_lanczos_eigenvalues(built, name):
    w, b = built[name]
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    v0 = vec.normal_vector(len(st), complex_=w.is_complex)
    n_steps = min(200, len(st) + 5)
    # the oracle's sector matrix (row form, equal to its scatter H.v) drives
    # the oracle recurrence and gives the dense spectrum
    H = bf.dense_matrix(m, st)
    ref = olz.lanczos(lambda v: H @ v, v0, n_steps)
    res = b.lanczos(w.J, torch.as_tensor(v0).cuda(), n_steps)
    exact = np.linalg.eigvalsh((H + H.conj().T) / 2)
    conv = olz.converged_ritz(res["alpha"], res["beta"])
    assert len(conv) >= 1
    assert abs(res["eigenvalues"][0] - exact[0]) < 1e-10
    assert abs(ref["eigenvalues"][0] - exact[0]) < 1e-10
    for e in conv:
        assert np.abs(exact - e).min() < 1e-10
    # the early steps agree with the oracle recurrence step by step
    k = min(10, res["n_done"], ref["n_done"])
    assert np.abs(res["alpha"][:k] - ref["alpha"][:k]).max() < 1e-11
    assert np.abs(res["beta"][:k] - ref["beta"][:k]).max() < 1e-11


def test_lanczos_breakdown_small_sector():
    # In a one-state sector (all spins down) H v0 = alpha v0 exactly, so
    # beta_0 = 0 and the recurrence stops after one step.  In a 13-state
    # sector plain FP64 Lanczos does not reach the 1e-12 breakdown rule (the
    # oracle's recurrence behaves the same), but its lowest value is exact.
    ed = _ed()
    c = lat.chain(6)
    w = wl.Workload("ring6_empty", c, lat.characters(c, 0), 0, np.ones(6))
    b = ed.Basis.from_workload(w)
    try:
        assert b.dim == 1
        res = b.lanczos(w.J, torch.ones(1, dtype=torch.float64, device="cuda"), 50)
        assert res["n_done"] == 1 and res["beta"][0] == 0.0
        assert res["eigenvalues"][0] == 1.5
    finally:
        b.close()
    c = lat.chain(10, reflection=True, spin_flip=True)
    w = wl.Workload("ring10", c, lat.characters(c, 0), 5, np.ones(10))
    b = ed.Basis.from_workload(w)
    try:
        D = b.dim
        assert D == 13
        res = b.lanczos(w.J, torch.as_tensor(vec.normal_vector(D)).cuda(), 100)
        m = bf.Model.from_workload(w)
        st, stab = bf.basis(m, 5)
        H = bf.dense_matrix(m, st).real
        assert abs(res["eigenvalues"][0] - np.linalg.eigvalsh(H)[0]) < 1e-10
        ref = olz.lanczos(lambda v: bf.apply(m, st, stab, v)[0], vec.normal_vector(D), 100)
        assert res["n_done"] == ref["n_done"]
    finally:
        b.close()


def test_lanczos_ground_state_vector(built):
    w, b = built["sq20_j1j2_n5"]
    v0 = torch.as_tensor(vec.normal_vector(b.dim)).cuda()
    res = b.lanczos(w.J, v0, 150, want_psi0=True)
    psi = res["psi0"]
    hpsi = b.apply(w.J, psi)
    e0 = res["eigenvalues"][0]
    resid = torch.linalg.norm(hpsi - e0 * psi).item()
    assert abs(torch.linalg.norm(psi).item() - 1) < 1e-12
    assert resid < 1e-6
    # two passes are bit-identical: a second call reproduces alpha exactly
    res2 = b.lanczos(w.J, v0, 150)
    assert np.array_equal(res["alpha"], res2["alpha"])


def test_apply_rejects_noninvariant_couplings(built):
    from paper_1804_05028_amd import EDError
    w, b = built["square16_k0"]
    J = np.ones(w.cluster.n_bonds)
    J[0] = 1.5
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(EDError) as ei:
        b.apply(J, x)
    assert ei.value.name == "ED_ERR_NONINVARIANT_H"


def test_empty_sector():
    ed = _ed()
    # momentum pi on a 4-site ring with n_up = 0 has no states
    c = lat.chain(4)
    w = wl.Workload("ring4", c, lat.characters(c, 2), 0, np.ones(4))
    b = ed.Basis.from_workload(w)
    try:
        assert b.dim == 0
        y = b.apply(w.J, torch.zeros(0, dtype=torch.float64, device="cuda"))
        assert y.numel() == 0
        assert b.stats() == (0, 0, 0)
    finally:
        b.close()
    _ = math


NEAR_BREAKDOWN = [
    # (cluster, momentum, n_up): sectors of two and three states, where the
    # Krylov space is exhausted and beta falls to rounding level, ~1e-16 of
    # the scale, before orthogonality can be lost
    ("ring4_k0", 4, 0, 2), ("ring4_k2", 4, 2, 2), ("ring6_k0_n2", 6, 0, 2), ("ring6_k3_n3", 6, 3, 3),
]


@pytest.mark.parametrize("name,n,k,n_up", NEAR_BREAKDOWN, ids=[c[0] for c in NEAR_BREAKDOWN])
def test_lanczos_near_breakdown_matches_oracle_step_count(name, n, k, n_up):
    ed = _ed()
    c = lat.chain(n, superlattice_period=2)
    w = wl.Workload(name, c, lat.characters(c, k), n_up, np.ones(c.n_bonds))
    b = ed.Basis.from_workload(w)
    try:
        D = b.dim
        assert 2 <= D <= 4, D
        m = bf.Model.from_workload(w)
        st, _ = bf.basis(m, n_up)
        H = bf.dense_matrix(m, st)
        v0 = vec.normal_vector(D, seed=9, complex_=b.is_complex)
        ref = olz.lanczos(lambda v: H @ v, v0, 20)
        res = b.lanczos(w.J, torch.as_tensor(v0).cuda(), 20)
        print(f"[breakdown] {name}: D={D} n_done={res['n_done']} oracle {ref['n_done']} "
              f"last beta {res['beta'][res['n_done'] - 1]:.2e}", flush=True)
        assert res["n_done"] == ref["n_done"] <= D
        assert res["beta"][res["n_done"] - 1] <= 1e-12 * max(np.abs(res["alpha"]).max(), res["beta"].max())
        exact = np.linalg.eigvalsh((H + H.conj().T) / 2)
        assert np.abs(np.sort(res["eigenvalues"]) - exact[:len(res["eigenvalues"])]).max() < 1e-12
    finally:
        b.close()
