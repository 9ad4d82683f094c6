"""Seeded input generators: the torch state hash equals the NumPy one bit for bit."""
import numpy as np
import torch

from ed_inputs import vectors as vec


def test_hashed_amplitudes_torch_matches_numpy():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 2 ** 56, 100_000, dtype=np.uint64)
    s[:4] = [0, 1, 2 ** 56 - 1, 12345]
    for salt in (0, 1, 7):
        for cplx in (False, True):
            a = vec.hashed_amplitudes(s, salt, cplx)
            b = vec.hashed_amplitudes_torch(torch.from_numpy(s.astype(np.int64)), salt, cplx).numpy()
            assert np.array_equal(a, b)
            assert np.all(np.abs(np.real(a)) <= 1.0)


def test_normal_vector_is_seeded_and_normalised():
    a = vec.normal_vector(1000, seed=3)
    b = vec.normal_vector(1000, seed=3)
    assert np.array_equal(a, b)
    assert abs(np.linalg.norm(a) - 1.0) < 1e-14
    c = vec.normal_vector(1000, seed=3, complex_=True)
    assert np.iscomplexobj(c) and abs(np.linalg.norm(c) - 1.0) < 1e-14
