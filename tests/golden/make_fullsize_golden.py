"""Writes fullsize_golden.txt: count and SHA-256 of the oracle's canonical tetrahedra for the
benchmark-size workloads (the canonical form is defined in tests/canon.py).  Calls only the
oracle package, the input generators and numpy.

Run from the repository root: python tests/golden/make_fullsize_golden.py [names...]
(uniform_1e7 and mix_1e7 take minutes and about 10 GB of memory each, on one core).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

# name: (generator, n, seed)
CASES = {
    "uniform_1e6": ("uniform", 1_000_000, 1006),
    "uniform_1e7": ("uniform", 10_000_000, 1007),
    "mix_1e7": ("mix", 10_000_000, 2007),
}


def points(kind, n, seed):
    """uniform: n points in [0, 1)^3; mix: the MIX recipe (lattice 40 %, clusters 30 %,
    shell 30 %) with n points in all."""
    from synth import mix_points, uniform_points
    if kind == "uniform":
        return uniform_points(n, seed)
    return mix_points(seed, int(0.4 * n), int(0.3 * n), n - int(0.4 * n) - int(0.3 * n))


def main(names):
    import oracle
    from canon import canonical_hash
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_golden.txt")
    rows = {}
    if os.path.exists(path):
        for line in open(path):
            if line.strip() and not line.startswith("#"):
                rows[line.split()[0]] = line.rstrip("\n")
    for name in names or list(CASES):
        kind, n, seed = CASES[name]
        xyz = points(kind, n, seed)
        t0 = time.time()
        rc, tets, _, st = oracle.delaunay(xyz)
        assert rc == 0, rc
        t1 = time.time()
        count, digest = canonical_hash(tets)
        del tets
        rows[name] = f"{name} kind={kind} n={n} seed={seed} tets={count} sha256={digest}"
        print(f"{name}: {count} tetrahedra, oracle {t1 - t0:.1f} s, canonical hash "
              f"{time.time() - t1:.1f} s", flush=True)
    with open(path, "w") as fh:
        fh.write("# oracle results at benchmark sizes (written by make_fullsize_golden.py):\n")
        fh.write("# name kind n seed tets sha256(canonical tetrahedra, tests/canon.py)\n")
        for name in CASES:
            if name in rows:
                fh.write(rows[name] + "\n")
    print(path)


if __name__ == "__main__":
    main(sys.argv[1:])
