"""Pins of the oracle's Philox4x32-10 against the published known-answer
vectors (Salmon et al., SC'11; Random123 known-answer tests)."""
import os

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert O.philox(ctr, key) == want


def test_counter_sensitivity():
    # every counter word and key word changes the output (no dropped operand)
    base = O.philox([1, 2, 3, 4], [5, 6])
    for q in range(4):
        c = [1, 2, 3, 4]
        c[q] ^= 1
        assert O.philox(c, [5, 6]) != base
    for q in range(2):
        k = [5, 6]
        k[q] ^= 1
        assert O.philox([1, 2, 3, 4], k) != base
