"""Writes tests/golden/window_hashes.txt using the oracle only.

Each line: <window bytes as hex> <d> <q> <hash>.  The windows cover the cases
the hash tests care about: lengths 1..64, bytes 0x00 and 0xFF, the constructed
equal-hash pair for d=256 (a change of +1 at byte i and -8 at byte i+8 keeps
the hash, since 2^64 = 8 mod 2^61-1) and the shift-and-add example pair of the
paper's own hash (d=2: "ac" and "ba" both give 293, Sec. 3.1).
Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import rkgen  # noqa: E402

Q = (1 << 61) - 1


def main():
    g = rkgen.rng(99, 0)
    wins = [(b"abcdefghi", 256, Q), (b"bbcdefgha", 256, Q), (b"ac", 2, Q), (b"ba", 2, Q),
            (b"\x00", 256, Q), (b"\xff" * 8, 256, Q), (b"\xff" * 9, 256, Q), (b"\xff" * 64, 256, Q),
            (b"\x00" * 63 + b"\x01", 256, Q)]
    for m in range(1, 65):
        wins.append((np.frombuffer(g.bytes(m), np.uint8).tobytes(), 256, Q))
    for m in (1, 2, 7, 8, 9, 16, 31, 32, 33, 64):
        wins.append((rkgen.ACGT[g.integers(0, 4, size=m)].tobytes(), 256, Q))
    with open(os.path.join(HERE, "window_hashes.txt"), "w") as f:
        f.write("# window_hex d q hash   (written by make_golden.py from the oracle)\n")
        for w, d, q in wins:
            f.write("%s %d %d %d\n" % (w.hex(), d, q, oracle.hash(w, d, q)))


if __name__ == "__main__":
    main()
