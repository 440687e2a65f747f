"""Writes the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.points import leja_points  # noqa: E402


def main():
    xi = leja_points(101)
    with open(os.path.join(HERE, "leja_points_101.txt"), "w") as fh:
        fh.write("# Leja points xi_0..xi_100 on [-2, 2], xi_0 = +2, ties to the leftmost point\n")
        fh.write("# (Sec. 2.2: the spectrum is mapped onto pre-computed Leja points in [-2, 2]).\n")
        fh.write("# Written by tests/golden/make_golden.py from oracle.points; one hex float per line.\n")
        for x in xi:
            fh.write(float(x).hex() + "\n")


if __name__ == "__main__":
    main()
