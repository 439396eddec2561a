"""Write the oracle's result for the 512 x 512 plain workload (seed 0).

Calls only the oracle and the seeded input generator; the GPU tests compare
against the stored file.  Usage: python tests/golden/make_oracle_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1902_08250_amd import workloads  # noqa: E402


def main():
    w = workloads.make(0)
    u = oracle.apply(w["src"], w["q"], w["tgt"], w["k"], w["d"])
    np.save(os.path.join(HERE, "oracle_plain512_u.npy"), u)
    print("wrote", u.shape)


if __name__ == "__main__":
    main()
