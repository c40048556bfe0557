"""Writes refine_golden.txt: the refinement oracle's result on fixed seeded inputs (final point
count, steps as candidates/kept, and SHA-256 of the canonical tetrahedra and of the final
coordinates).  Calls only the oracle package and the input generators.

Run from the repository root: python tests/golden/make_refine_golden.py
With --fullsize it writes refine_fullsize_golden.txt instead: the same for the benchmark's
refinement workload (2.5e5 points, h = 0.0064; about five minutes on one core).
"""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

CASES = [("uniform", 600, 7, 0.08), ("uniform", 2000, 11, 0.05), ("clusters", 800, 8, 0.03),
         ("uniform", 20000, 5, 0.03),
         # deep refinement: h n^(1/3) about 0.4, as in the benchmark workload (about six times
         # the input points)
         ("uniform", 10000, 13, 0.0185),
         # near-cospherical input: the interior tetrahedra's circumcentres crowd the centre, so
         # most candidates of the first steps have more than eight close earlier ones
         ("shell", 300, 21, 0.15)]

# the benchmark's refinement workload (bench.py --workload refine)
FULLSIZE_CASES = [("uniform", 250000, 4007, 0.0064)]


def run_case(kind, n, seed, h):
    import oracle
    from oracle import refine
    from synth import cluster_points, shell_points, uniform_points
    xyz = (uniform_points(n, seed) if kind == "uniform" else shell_points(n, seed) if kind == "shell"
           else cluster_points(n, seed, clusters=4))
    pts, tets, nbrs, steps = refine.refine(xyz, h)
    canon = oracle.canonical(tets).astype(np.int64)
    return (len(pts), ";".join(f"{a}/{b}" for a, b in steps),
            hashlib.sha256(canon.tobytes()).hexdigest(),
            hashlib.sha256(np.ascontiguousarray(pts, dtype=np.float64).tobytes()).hexdigest())


def main():
    full = "--fullsize" in sys.argv[1:]
    name = "refine_fullsize_golden.txt" if full else "refine_golden.txt"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with open(out, "w") as fh:
        fh.write("# refinement oracle results (written by make_refine_golden.py%s)\n" % (" --fullsize" if full else ""))
        fh.write("# kind n seed h | points steps(candidates/kept) sha256(canonical tets) sha256(points)\n")
        for kind, n, seed, h in (FULLSIZE_CASES if full else CASES):
            npts, steps, ht, hp = run_case(kind, n, seed, h)
            fh.write(f"{kind} {n} {seed} {h} | {npts} {steps} {ht} {hp}\n")
    print(out)


if __name__ == "__main__":
    main()
