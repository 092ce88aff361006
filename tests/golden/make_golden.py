"""Writes the regression fixtures of this folder.  Calls only the oracle.

bank_tiny.txt -- Eq. (1) by direct summation (FP64) for a 6 x 7 image with
pixels (3 y + 5 x) mod 11 / 10, omega = pi/3 and 1.2, sigma = 1.1 and 0.9,
theta_k = k pi / 3, radius 3 sigma, mirror boundary.  One line per output:
i k y x re im.
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def tiny_image():
    y, x = np.mgrid[0:6, 0:7]
    return (((3 * y + 5 * x) % 11) / 10.0).astype(np.float32)


TINY_ARGS = dict(omegas=[math.pi / 3, 1.2], sigmas=[1.1, 0.9],
                 thetas=[0.0, math.pi / 3, 2 * math.pi / 3], radius_sigmas=3.0,
                 boundary="mirror")


def main():
    F = oracle.gabor_bank(tiny_image(), **TINY_ARGS)
    with open(os.path.join(HERE, "bank_tiny.txt"), "w") as fh:
        fh.write("# i k y x re im  (Eq. (1), FP64 direct sum; see make_golden.py)\n")
        for (i, k, y, x), v in np.ndenumerate(F):
            fh.write(f"{i} {k} {y} {x} {v.real:.17e} {v.imag:.17e}\n")


if __name__ == "__main__":
    main()
