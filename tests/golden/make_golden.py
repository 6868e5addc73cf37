"""Writes the stored expected values under tests/golden/ (calls only oracle/).

  counts_k2_d2_nb10.txt : triangle counts N_tri(b1,b2,b3) for bins of width
      2 k_f with centres 2, 4, ..., 20 k_f (the 64^3 monopole workload),
      by direct enumeration of closed integer triangles.
  counts_c5_k11_d11_first.txt : the counts of the triangles (0,0,0) and
      (1,0,0) of the 1024^3 binning (shells of width 11 k_f centred on 11,
      22, ... k_f), by the same enumeration restricted to the two shells.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def counts_table(k0, dk, nb, path, tris=None, chunk=2048):
    tris = O.triangle_list(nb) if tris is None else tris
    cnt = O.triangle_counts_brute(k0, dk, nb, tris, chunk=chunk)
    with open(path, "w") as f:
        f.write(f"# closed-triangle counts by enumeration: k0={k0} dk={dk} nbins={nb}\n")
        f.write("# b1 b2 b3 count\n")
        for (a, b, c), n in zip(tris, cnt):
            f.write(f"{a} {b} {c} {n}\n")


if __name__ == "__main__":
    counts_table(2.0, 2.0, 10, os.path.join(HERE, "counts_k2_d2_nb10.txt"))
    counts_table(11.0, 11.0, 2, os.path.join(HERE, "counts_c5_k11_d11_first.txt"), [(0, 0, 0), (1, 0, 0)], 256)
