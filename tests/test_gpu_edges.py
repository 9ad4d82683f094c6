"""Edge cases of the GPU path at the limits of what it supports: the largest
site count (56, the width of the state field of a basis word), many small
sublattice blocks, large blocks (11 sites), sector dimensions that are not
multiples of the wave size, and tables too large for LDS, which must be
rejected with ED_ERR_UNSUPPORTED before any kernel runs.  Each buildable case
against the oracle: basis bit-exact, H.v to 1e-12, exact term counts."""
import numpy as np
import pytest
import torch

from ed_inputs import lattice as lat
from ed_inputs import vectors as vec
from ed_inputs import workloads as wl
from oracle import bruteforce as bf

pytestmark = pytest.mark.gpu


def _ed():
    from paper_1804_05028_amd import ed
    return ed


def _cases():
    out = []
    c = lat.chain(56, superlattice_period=8)            # 8 sublattices of 7 sites
    out.append(("ring56_k5_nup3", wl.Workload("ring56", c, lat.characters(c, 5), 3, np.ones(56))))
    out.append(("ring56_k0_nup2", wl.Workload("ring56", c, lat.characters(c, 0), 2, np.ones(56))))
    c = lat.chain(48, superlattice_period=6)            # 6 sublattices of 8 sites
    out.append(("ring48_k7_nup3", wl.Workload("ring48", c, lat.characters(c, 7), 3, np.ones(48))))
    c = lat.chain(22, superlattice_period=2)            # 2 sublattices of 11 sites
    out.append(("ring22_k3_nup4", wl.Workload("ring22", c, lat.characters(c, 3), 4, np.ones(22))))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,w", CASES, ids=[c[0] for c in CASES])
def test_edge_sizes_match_oracle(name, w):
    ed = _ed()
    m = bf.Model.from_workload(w)
    st, stab = bf.basis(m, w.n_up)
    print(f"[edges] {name}: D={len(st)}", flush=True)
    b = ed.Basis.from_workload(w)
    try:
        assert b.dim == len(st)
        assert np.array_equal(b.states(), st)
        assert np.array_equal(b.norms().astype(np.int64), stab.astype(np.int64))
        x = vec.normal_vector(len(st), seed=8, complex_=b.is_complex)
        y = b.apply(w.J, torch.as_tensor(x).cuda()).cpu().numpy()
        ref, kept, _ = bf.apply(m, st, stab, x)
        assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
        assert b.stats()[1] == kept
    finally:
        b.close()


def test_tables_too_large_for_lds_are_rejected():
    from paper_1804_05028_amd import _lib as L
    ed = _ed()
    c = lat.chain(48, superlattice_period=4)            # 4 sublattices of 12 sites
    w = wl.Workload("ring48", c, lat.characters(c, 0), 3, np.ones(48))
    with pytest.raises(L.EDError) as e:
        ed.Basis.from_workload(w)
    assert e.value.name == "ED_ERR_UNSUPPORTED"
