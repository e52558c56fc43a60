"""Writes box_partition_counts.txt from closed forms (no library, no oracle).

For the 7-point stencil on N^3 nodes split into P^3 equal boxes (P divides N)
with the interface on the lower faces of every box (the nodes adjacent to a
lower-numbered box):
  interface nodes   N^3 - (N - P + 1)^3
  faces             3 (P-1) P^2     (pieces shared by 2 boxes)
  edges             3 P (P-1)^2     (shared by 3 boxes)
  vertices          (P-1)^3         (shared by 4 boxes)
  sum of overlapping subdomain sizes with one layer of overlap
                    N^3 + 2 * 3 (P-1) P^2 * (N/P)^2
                    (every internal box face adds a face layer of (N/P)^2 nodes
                    to each of the two boxes sharing it)
These are the pieces of the paper's Sec. III decomposition (interface,
components, overlapping subdomains) for a structured box partition.
"""
import os

CASES = [(20, 2), (12, 3), (24, 4), (30, 5), (128, 8)]


def counts(N, P):
    assert N % P == 0
    return (N, P, N ** 3 - (N - P + 1) ** 3, 3 * (P - 1) * P * P, 3 * P * (P - 1) ** 2,
            (P - 1) ** 3, N ** 3 + 2 * 3 * (P - 1) * P * P * (N // P) ** 2)


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "box_partition_counts.txt")
    with open(out, "w") as f:
        f.write("# N P n_gamma faces edges vertices sum_overlap  (closed forms; "
                "make_box_partition_counts.py)\n")
        for N, P in CASES:
            f.write(" ".join(str(v) for v in counts(N, P)) + "\n")
