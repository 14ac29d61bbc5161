"""Writes the stored expected values under tests/golden/.

Calls only the oracle package (exact rational Gauss-Jordan) and the seeded
input generators; nothing here comes from the GPU library.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle.exact import exact_inverse, to_float  # noqa: E402


def main():
    # Exact integer inverse of a unimodular matrix (all leading minors 1):
    # Strassen's scheme never breaks down on it and every rounding-free
    # implementation must reproduce it bit for bit.
    for n, seed in [(16, 16), (64, 64)]:
        a = W.unimodular_bidiag(n, seed)
        x = to_float(exact_inverse(a))
        np.savetxt(os.path.join(HERE, f"unimodular{n}_A.txt"), a, fmt="%d")
        np.savetxt(os.path.join(HERE, f"unimodular{n}_Ainv.txt"), x, fmt="%d")
    # Structural counts stated by the paper for one internal node of the
    # recursion and for the leaf level.
    counts = {
        "source": "Alg. 2 (Sec. 3.3) lists per internal node: 6 multiply, 2 subtract, "
                  "1 scalarMul, 2 recursive Inverse calls; Sec. 4 (leafNode cost) gives "
                  "2^(p-q) leaves, i.e. n / blockSize, and 2^i nodes at level i (Fig. 1)",
        "multiply_per_internal_node": 6,
        "subtract_per_internal_node": 2,
        "scalar_mul_per_internal_node": 1,
        "inverse_calls_per_internal_node": 2,
    }
    with open(os.path.join(HERE, "paper_counts.json"), "w") as f:
        json.dump(counts, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
