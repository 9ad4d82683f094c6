"""The slot table's probe sequence, restated on the CPU.

Insertion and every lookup walk the same sequence: from the home slot round
its own 128-byte line (8 slots of 16 bytes or 4 of 32), then round the next
line from the same offset, and so on (next_slot in csrc/ed_device.hpp).  A
lookup stops at the first empty slot, which is only correct if the sequence
from any home slot visits every slot exactly once; and the point of the
order is that the first line-full of probes stays in the home line.
"""
import pytest


def next_slot(sl, home, smask, glog2):
    gm = (1 << glog2) - 1
    nx = (sl & ~gm) | ((sl + 1) & gm)
    if ((nx ^ home) & gm) == 0:
        nx = (nx + gm + 1) & smask
    return nx


@pytest.mark.parametrize("log2n", [4, 5, 7])
@pytest.mark.parametrize("glog2", [2, 3])
def test_sequence_is_a_permutation_and_line_first(log2n, glog2):
    n = 1 << log2n
    g = 1 << glog2
    for home in range(n):
        seq = [home]
        for _ in range(n - 1):
            seq.append(next_slot(seq[-1], home, n - 1, glog2))
        assert sorted(seq) == list(range(n))
        # the first g probes are the home line, the next g the following one
        assert all(s // g == home // g for s in seq[:g])
        assert all(s // g == (home // g + 1) % (n // g) for s in seq[g:2 * g])
        # and every line is entered at the home offset
        assert all(seq[k * g] % g == home % g for k in range(n // g))
