"""Fermions in the occupation-number basis on the GPU against the oracle.

The fermionic path (ed_build_basis_fermions, ed_apply_H_fermions,
ed_lanczos_fermions) carries the Fermi sign of every group element and of
every hop (sec. "Discussion").  Small sectors are compared with the oracle's
brute-force fermionic basis and scatter H.v (tests/test_oracle_fermions.py
pins it): the basis and stabilisers bit for bit, H.v within 1e-12, term
counts exactly, and the lowest Lanczos value against the dense sector
spectrum to 1e-10.  The cases cover real and complex momenta, point-group
irreps, interactions, the Hubbard ring as two orbitals per site, one to four
sublattices and several table chunk widths.  36-site triangular t-V
sectors check the character-formula dimension and sampled rows at full
size.
"""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf
from oracle import dimension as odim

pytestmark = pytest.mark.gpu


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _fw(name, c, chi, n, t=1.0, V=0.0):
    return wl.FermionWorkload(name, c, chi, n, np.full(c.n_bonds, t), np.full(c.n_bonds, V))


def _cases():
    out = []
    c = lat.chain(8, superlattice_period=2)
    out += [(_fw("ring8_k0", c, lat.characters(c, 0), 4, V=0.7), None),
            (_fw("ring8_k3", c, lat.characters(c, 3), 3, V=-0.4), None),
            (_fw("ring8_k4", c, lat.characters(c, 4), 4), None)]
    c = lat.triangular((2, 2), (-2, 4), superlattice=wl.TRI_4, name="tri12_4sub")
    for p, pc in enumerate(lat.point_group_chars_1d(c.point_group)):
        out.append((_fw(f"tri12_G{p}", c, lat.characters(c, 0, pc), 5, V=0.5), None))
    out.append((_fw("tri12_G0_c1", c, lat.characters(c, 0), 6, V=1.0), {"chunk_bits": 1}))
    c = lat.triangular((2, 2), (-2, 4), rotations=False, mirrors=False, superlattice=wl.TRI_3, name="tri12T_3sub")
    out += [(_fw(f"tri12T_k{k}", c, lat.characters(c, k), 5, V=0.3), None) for k in (0, 1, 5)]
    c = lat.square((4, 0), (0, 4), superlattice=wl.SQ_2X2, name="sq16C4")
    U, det = lat.momenta(c)
    km = U.index((det // 2, det // 2))
    out += [(_fw("sq16_G", c, lat.characters(c, 0), 6, V=0.5), None),
            (_fw("sq16_M", c, lat.characters(c, km), 7, V=0.5), {"chunk_bits": 2})]
    c = lat.square((4, 0), (0, 4), rotations=False, superlattice=wl.SQ_CHECKER, name="sq16T_2sub")
    out.append((_fw("sq16T_k1_2sub", c, lat.characters(c, 1), 5, V=0.2), None))
    c = lat.chain(8, superlattice_period=None)
    out.append((_fw("ring8_k2_1sub", c, lat.characters(c, 2), 3, V=0.4), None))
    for k in (0, 1, 2):
        out.append((wl.hubbard_ring(4, 1.0, 2.5, momentum_index=k, n_sub=2), None))
    out.append((wl.hubbard_ring(6, 1.0, 4.0, momentum_index=1, n_sub=4), None))
    # 4-byte entries (sign parity in bit 31) beside the automatic 2-byte ones
    # (bit 15); one to three chunks
    c = lat.triangular((2, 2), (-2, 4), superlattice=wl.TRI_4, name="tri12_4sub")
    out.append((_fw("tri12_G0_e4", c, lat.characters(c, 0), 5, V=0.5), {"table_entry_bytes": 4}))
    out.append((_fw("tri12_G0_e4_c1", c, lat.characters(c, 0), 6, V=1.0), {"table_entry_bytes": 4, "chunk_bits": 1}))
    c = lat.square((4, 0), (0, 4), superlattice=wl.SQ_2X2, name="sq16C4")
    U, det = lat.momenta(c)
    km = U.index((det // 2, det // 2))
    out.append((_fw("sq16_M_e4", c, lat.characters(c, km), 7, V=0.5), {"table_entry_bytes": 4, "chunk_bits": 2}))
    out.append((_fw("sq16_M_e2", c, lat.characters(c, km), 7, V=0.5), {"table_entry_bytes": 2, "chunk_bits": 3}))
    out.append((wl.hubbard_ring(6, 1.0, 4.0, momentum_index=1, n_sub=4), {"table_entry_bytes": 4}))
    return out


CASES = _cases()
IDS = [w.name + ("_" + "_".join(f"{k}{v}" for k, v in t.items()) if t else "") for w, t in CASES]


def _oracle(w):
    c = w.cluster
    m = bf.FermionModel(c.n_sites, c.perm, w.chi, c.bonds, w.t, w.V)
    st, stab = bf.fbasis(m, w.n_part)
    return m, st, stab


@pytest.mark.parametrize("w,tune", CASES, ids=IDS)
def test_fermion_basis_hv_and_lanczos(w, tune):
    ed = _ed()
    print(f"[fermions] {w.name} {tune}", flush=True)
    m, st, stab = _oracle(w)
    c = w.cluster
    assert len(st) == odim.fermion_sector_dimension(c.perm, w.chi, w.n_part)
    b = ed.FermionBasis.from_workload(w, tune)
    try:
        info = b.info()
        assert info["is_fermion"] == 1
        # 2-byte entries wherever a block has at most 12 orbitals, unless 4 are asked for
        want = (tune or {}).get("table_entry_bytes", 0) or (2 if info["sub_bits"] <= 12 else 4)
        assert info["table_entry_bytes"] == want
        assert b.dim == len(st)
        if b.dim == 0:
            return
        assert np.array_equal(b.states(), st)
        assert np.array_equal(b.norms().astype(np.int64), stab.astype(np.int64))
        x = vec.normal_vector(b.dim, seed=3, complex_=b.is_complex)
        y = b.apply(w.t, torch.as_tensor(x).cuda(), V=w.V).cpu().numpy()
        ref, kept, dropped = bf.fapply(m, st, stab, x)
        assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max()
        n_diag, k2, d2 = b.stats()
        assert (n_diag, k2, d2) == (b.dim, kept, dropped)
        # Lanczos: the lowest Ritz value is the lowest eigenvalue of the sector
        M = bf.fdense_matrix(m, st) if len(st) <= 2000 else None
        if M is not None:
            dense = np.linalg.eigvalsh((M + M.conj().T) / 2)
            res = b.lanczos(w.t, torch.as_tensor(x).cuda(), min(150, 4 * len(st) + 5), V=w.V)
            assert abs(res["eigenvalues"][0] - dense[0]) <= 1e-10 * max(1.0, abs(dense[0])), (res["eigenvalues"][0],
                                                                                             dense[0])
    finally:
        b.close()


def test_fermion_entry_points_reject_the_other_kind():
    ed = _ed()
    from paper_1804_05028_amd import _lib as L
    c = lat.chain(8, superlattice_period=2)
    w = _fw("ring8", c, lat.characters(c, 0), 4)
    fb = ed.FermionBasis.from_workload(w)
    sb = ed.Basis(c.n_sites, c.bonds, c.n_sublat, c.perm, c.flip, lat.characters(c, 0), 4)
    try:
        x = fb.empty().normal_()
        y = fb.empty()
        with pytest.raises(L.EDError) as e:
            L.ed_apply_H(fb.handle, w.t, x, y)
        assert e.value.name == "ED_ERR_ARG"
        with pytest.raises(L.EDError) as e:
            L.ed_apply_H_fermions(sb.handle, w.t, None, x, y)
        assert e.value.name == "ED_ERR_ARG"
        with pytest.raises(L.EDError) as e:
            L.ed_apply_H_backward(fb.handle, w.t, x, x, y, True)
        assert e.value.name == "ED_ERR_UNSUPPORTED"
        # 1-byte entries, and 2-byte ones for blocks of more than 12 orbitals
        c16 = lat.chain(16, superlattice_period=None)
        w16 = _fw("ring16_1sub", c16, lat.characters(c16, 0), 3)
        for eb in (1, 2):
            with pytest.raises(L.EDError) as e:
                ed.FermionBasis.from_workload(w16, {"table_entry_bytes": eb})
            assert e.value.name == "ED_ERR_UNSUPPORTED"
        # couplings that break the group
        t = w.t.copy()
        t[0] = 2.0
        with pytest.raises(L.EDError) as e:
            fb.apply(t, x, out=y)
        assert e.value.name == "ED_ERR_NONINVARIANT_H"
    finally:
        fb.close()
        sb.close()
    # a fermionic group with spin flip
    cf = lat.chain(8, superlattice_period=2, spin_flip=True)
    with pytest.raises(L.EDError) as e:
        L.ed_build_basis_fermions(L.ModelArrays(cf.n_sites, cf.bonds, cf.n_sublat, cf.perm, cf.flip,
                                                lat.characters(cf, 0)), 4)
    assert e.value.name == "ED_ERR_UNSUPPORTED"


def test_fermion_fullsize_sampled_rows():
    """36-site triangular t-V at half filling, 36 T x C6 (216 elements), the
    trivial and a complex Gamma irrep: dimension from the character formula
    and sampled rows of H.v against the oracle's row evaluation."""
    ed = _ed()
    for pg in (0, 2):
        w = wl.triangular_36_tV(n_sub=4, V=1.0, pg_irrep=pg)
        c = w.cluster
        print(f"[fermions] {w.name}: building", flush=True)
        b = ed.FermionBasis.from_workload(w)
        try:
            D = b.dim
            info = b.info()
            print(f"[fermions] {w.name}: {info['table_entry_bytes']}-byte entries, {info['chunk_bits']}-bit chunks, "
                  f"{info['lds_bytes']} B of LDS", flush=True)
            assert D == odim.fermion_sector_dimension(c.perm, w.chi, w.n_part)
            st = b.states_device()
            assert bool((st[1:] > st[:-1]).all())
            x = vec.hashed_amplitudes_torch(st, salt=4, complex_=b.is_complex)
            y = b.apply(w.t, x, V=w.V)
            rng = np.random.default_rng(vec.SEED_ROWS)
            rows = np.unique(np.concatenate([np.arange(500), np.arange(D - 500, D), rng.choice(D, 4000, replace=False)]))
            rows_t = torch.as_tensor(rows).cuda()
            s_rows = st[rows_t].cpu().numpy().astype(np.uint64)
            y_rows = y[rows_t].cpu().numpy()
            del x, y, st
            m = bf.FermionModel(c.n_sites, c.perm, w.chi, c.bonds, w.t, w.V)
            r, _, _, stab, comp = bf.frep_many(m, s_rows)
            assert np.array_equal(r, s_rows) and comp.all()
            assert np.array_equal(b.norms()[rows].astype(np.int64), stab.astype(np.int64))
            ref, kept, _, rc = bf.frows_apply(m, s_rows, lambda s: vec.hashed_amplitudes(s, 4, b.is_complex))
            assert rc.all()
            err = np.abs(y_rows - ref).max()
            print(f"[fermions] {w.name}: D={D} rows={len(rows)} terms={kept} max error {err:.2e}", flush=True)
            assert err <= 1e-11 * np.abs(ref).max()
            assert np.linalg.norm(y_rows - ref) <= 1e-12 * np.linalg.norm(ref)
        finally:
            b.close()
