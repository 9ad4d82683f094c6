"""bench.py without a GPU: workload table, refusal of several GPUs, traffic
lookup keyed by the kernel sources."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from ed_inputs import lattice as lat  # noqa: E402


@pytest.mark.parametrize("name", sorted(bench.AUTOTUNE_NSUB))
def test_workloads_have_orbit_invariant_couplings(name):
    for n_sub in bench.AUTOTUNE_NSUB[name]:
        w, desc = bench._workload(name, n_sub)
        orbit = lat.bond_orbits(w.cluster)
        for o in np.unique(orbit):
            assert np.ptp(w.J[orbit == o]) < 1e-12, (name, n_sub, o)
        assert w.cluster.n_sublat == n_sub and desc


def test_allk_sector_sets():
    assert len(bench._allk_workloads(4, "all")) == 36
    ws = bench._allk_workloads(4, "inequivalent")
    assert len(ws) == 20 and sum(w.is_complex for w in ws) == 16


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_is_reported_only_for_the_profiled_kernel():
    assert bench.measured_traffic(("no-such-workload", 4, "hash-slot", 5)) is None
    for key, (digest, fetch, write, profile) in bench.MEASURED_TRAFFIC.items():
        t = bench.measured_traffic(key)
        assert t is None or (bench.kernel_digest() == digest and t == (fetch, write, profile))
        # every figure names a committed profile summary
        assert os.path.exists(os.path.join(ROOT, profile)), profile


def test_gamma_irreps_workload():
    import bench
    from paper_1804_05028_amd import _lib as L
    ws = bench._gamma_workloads(4)
    assert len(ws) == 8 and len({w.name for w in ws}) == 8
    chis = [tuple(np.round(w.chi.real, 6)) for w in ws]
    assert len(set(chis)) == 8
    for w in ws:
        c = w.cluster
        L.ed_validate(L.ModelArrays(c.n_sites, c.bonds, c.n_sublat, c.perm, c.flip, w.chi), w.n_up)
    assert set(bench.BATCHED_WORKLOADS) == {"triangular36_allk", "triangular36_gamma"}
