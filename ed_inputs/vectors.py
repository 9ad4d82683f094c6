"""Seeded synthetic inputs: start vectors, couplings and state-hashed vectors.

Nothing here computes any part of the exact-diagonalisation method.  The
state-hashed vector assigns every spin configuration a fixed pseudo-random
amplitude, so that one side can fill a vector in its own basis order and the
other side can evaluate the amplitude of any configuration it meets without
knowing an index.  The hash is the SplitMix64 output function (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SEED_VECTOR = 0      # start vectors / x
SEED_COUPLING = 1    # random bond couplings
SEED_ROWS = 2        # sampled rows
SEED_TARGET = 3      # random fit target


def splitmix64(z):
    """SplitMix64 output function applied element-wise to uint64 values."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def hashed_amplitudes(states, salt=0, complex_=False):
    """Amplitude in [-1, 1) (or complex with both parts so) for each state."""
    s = np.asarray(states, dtype=np.uint64)
    salt = np.uint64(salt)
    with np.errstate(over="ignore"):
        re = splitmix64(s ^ (salt * _M2))
        re = (re >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
        if not complex_:
            return re
        im = splitmix64(s ^ ((salt + np.uint64(1)) * _M2) ^ _GOLDEN)
        im = (im >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
    return re + 1j * im


def _signed(u):
    return u - (1 << 64) if u >= (1 << 63) else u


def _srl(z, k):
    """Logical right shift of int64 tensors holding uint64 bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _splitmix64_torch(z):
    z = z + _signed(int(_GOLDEN))
    z = (z ^ _srl(z, 30)) * _signed(int(_M1))
    z = (z ^ _srl(z, 27)) * _signed(int(_M2))
    return z ^ _srl(z, 31)


def hashed_amplitudes_torch(states, salt=0, complex_=False):
    """hashed_amplitudes for an int64 torch tensor of states, on its device.

    Integer arithmetic wraps modulo 2^64 as in the NumPy version, so the two
    agree bit for bit (checked by the tests).
    """
    import torch
    s = states.to(torch.int64)
    k1 = _signed((int(salt) * int(_M2)) % (1 << 64))
    re = _splitmix64_torch(s ^ k1)
    re = _srl(re, 11).to(torch.float64) * (2.0 ** -52) - 1.0
    if not complex_:
        return re
    k2 = _signed((((int(salt) + 1) * int(_M2)) % (1 << 64)) ^ int(_GOLDEN))
    im = _splitmix64_torch(s ^ k2)
    im = _srl(im, 11).to(torch.float64) * (2.0 ** -52) - 1.0
    return torch.complex(re, im)


def normal_vector(dim, seed=SEED_VECTOR, complex_=False, normalise=True):
    """N(0,1) entries from numpy's default_rng(seed); complex: independent parts."""
    rng = np.random.default_rng(seed)
    if complex_:
        v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    else:
        v = rng.standard_normal(dim)
    if normalise and dim > 0:
        v = v / np.linalg.norm(v)
    return v


def random_couplings(n_bonds, seed=SEED_COUPLING, low=0.8, high=1.2):
    return np.random.default_rng(seed).uniform(low, high, size=n_bonds)


def couplings_by_kind(bond_kind, values):
    """J_b = values[kind_b] (e.g. J1 for nearest, J2 for next-nearest bonds)."""
    return np.asarray(values, dtype=np.float64)[np.asarray(bond_kind)]
