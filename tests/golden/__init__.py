"""Readers of the stored expected values under tests/golden/ (each file
states where its values come from)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def philox_kat():
    """(width, counter, key, output) of every published Philox known-answer
    vector in philox_kat.txt (ten rounds)."""
    rows = []
    with open(os.path.join(HERE, "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            width, rounds = int(v[0]), int(v[1])
            assert rounds == 10
            h = [int(x, 16) for x in v[2:]]
            rows.append((width, h[0:4], h[4:6], h[6:10]))
    return rows
