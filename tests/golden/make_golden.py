"""Writes the stored expected values under tests/golden/.

Calls only the oracle package (its exact, symbolic-differentiation module),
never the HIP library. Run from the repository root:

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import multi_indices          # noqa: E402
from oracle.exact import dtensor_exact, numerator_at   # noqa: E402

# integer points: stencil offsets of several shapes (axis, face diagonal,
# body diagonal, generic, the |d|^2 = 5 and |d|^2 = 36 shell boundaries)
POINTS = [(1, 2, 0), (0, 0, 3), (2, 2, 1), (-3, 1, 2), (6, 0, 0), (-4, -4, 2),
          (1, -5, 3), (2, 3, -5), (-2, -1, 0)]
ORDER = 8


def main():
    path = os.path.join(HERE, "dtensor_integer_points.txt")
    with open(path, "w") as f:
        f.write("# Derivatives of 1/r at integer points: D_m(d) = P_m(d) / (|d|^2)^|m| / sqrt(|d|^2)\n")
        f.write("# The potential of a point mass and its Cartesian derivatives are what the\n")
        f.write("# cell-to-cell multipole interactions of the gravity solver evaluate\n")
        f.write("# (Sec. IV-C, Octo-Tiger: FMM gravity on the 8^3 sub-grids).\n")
        f.write("# Exact integer numerator P_m(d) by symbolic differentiation; value rounded once.\n")
        f.write("# columns: dx dy dz mx my mz numerator value\n")
        for d in POINTS:
            for m in multi_indices(ORDER):
                f.write("%d %d %d %d %d %d %d %.17e\n" % (d + m + (numerator_at(m, d), dtensor_exact(m, d))))
    print("wrote", path)


if __name__ == "__main__":
    main()
