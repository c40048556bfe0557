"""Checks at the benchmark's full sizes, in the launch configuration bench.py times (default
options, device input and device outputs on torch's stream).

* whole-output equality with the oracle where the oracle's result is stored: uniform 1e6 and
  1e7 and MIX 1e7 (tests/golden/fullsize_golden.txt holds the count and SHA-256 of the
  oracle's canonical tetrahedra, written by make_fullsize_golden.py from the oracle alone);
  the GPU output is canonicalized on the device and hashed;
* at 1e8 (no stored oracle result: the serial oracle needs about 100 GB and most of an hour),
  a complete certificate: every tetrahedron positive, every neighbour link mirrored on the
  same facet, no two neighbours overlapping, every interior facet locally Delaunay under the
  perturbation (fullcheck.c, the oracle's exact predicates), the hull facets one closed
  locally convex surface and every point a vertex.  By Delaunay's lemma this is the unique
  perturbed Delaunay tetrahedralization, the oracle's result.  A sub-box is also compared
  with the oracle directly: a tetrahedron whose circumball lies inside a box B belongs to the
  tetrahedralization of all points iff it belongs to that of the points in B;
* the adjacency, hull and volume checks on the device at 1e7.
"""
from __future__ import annotations

import numpy as np
import pytest

import os

from canon import canonical_hash_torch, read_golden
from synth import uniform_points
from test_gpu import dtlib, say  # noqa: F401  (fixture)

GOLDEN = read_golden(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_golden.txt"))

pytestmark = pytest.mark.gpu


def _triangulate(dtlib, xyz):
    """Bench configuration: device input, default options, device outputs."""
    import torch
    d = torch.from_numpy(xyz).cuda()
    stream = torch.cuda.current_stream()
    tri = dtlib.Triangulation(device=0, stream=stream.cuda_stream, timing=True)
    tri.insert(d)
    T = dtlib.dt_get_tets(tri.ctx)
    t = torch.empty((T, 4), dtype=torch.int32, device="cuda")
    nb = torch.empty((T, 4), dtype=torch.int64, device="cuda")
    assert dtlib.dt_get_tets(tri.ctx, t, nb, T) == T
    torch.cuda.synchronize()
    tri.close()
    return t, nb


def _circumballs(xyz, q):
    a = xyz[q[:, 0]]
    m = np.stack([xyz[q[:, k]] - a for k in (1, 2, 3)], axis=1)  # [k, 3, 3]
    rhs = 0.5 * np.einsum("kij,kij->ki", m, m)
    c = np.linalg.solve(m, rhs[:, :, None])[:, :, 0]
    return a + c, np.sqrt(np.einsum("ki,ki->k", c, c))


def _in_box(xyz, q, lo, hi, margin=1e-9):
    cen, r = _circumballs(xyz, q)
    return np.all(cen - r[:, None] > lo + margin, axis=1) & np.all(cen + r[:, None] < hi - margin, axis=1)


def _subbox_check(oracle_mod, xyz, t_dev, lo, side, min_tets=None):
    import torch
    hi = lo + side
    inb = np.all((xyz >= lo) & (xyz < hi), axis=1)
    sub_idx = np.nonzero(inb)[0]
    say(f"sub-box [{lo}, {hi})^3: {len(sub_idx)} points")
    # GPU tetrahedra with all four vertices in the box, then the circumball classifier
    m = torch.from_numpy(inb).cuda()
    keep = m[t_dev.long()].all(dim=1)
    g = t_dev[keep].cpu().numpy().astype(np.int64)
    g = g[_in_box(xyz, g, lo, hi)]
    # the oracle on the points of the box (their input order kept: same perturbation order)
    rc, ot, _, _ = oracle_mod.delaunay(xyz[sub_idx])
    assert rc == 0
    o = sub_idx[ot.astype(np.int64)]
    o = o[_in_box(xyz, o, lo, hi)]
    a, b = oracle_mod.canonical(g), oracle_mod.canonical(o)
    say(f"sub-box: {len(a)} GPU and {len(b)} oracle tetrahedra with the ball inside")
    assert len(a) > (0.5 * 6.5 * len(sub_idx) if min_tets is None else min_tets)
    assert a.shape == b.shape and np.array_equal(a, b)


def _adjacency_and_hull_check(t, nb):
    """On the device (torch): mirrored links sharing a facet; V - E + F = 2 on the hull."""
    import torch
    T = t.shape[0]
    chunk = 1 << 22
    for s in range(0, T, chunk):
        e = min(T, s + chunk)
        ti = torch.arange(s, e, device="cuda").repeat_interleave(4)
        nf = nb[s:e].reshape(-1)
        ok = nf >= 0
        back = nb[nf[ok]]
        assert bool((back == ti[ok][:, None]).any(dim=1).all()), "neighbour link not mirrored"
        va = t[ti[ok]]
        vb = t[nf[ok]]
        shared = (va[:, :, None] == vb[:, None, :]).any(dim=2).sum(dim=1)
        assert bool((shared == 3).all()), "neighbours do not share a facet"
    # hull faces: facet j of t without neighbour; V - E + F = 2 (a closed triangulated sphere)
    hf = torch.nonzero(nb < 0)
    F = hf.shape[0]
    faces = torch.stack([t[hf[:, 0], (hf[:, 1] + k) % 4] for k in (1, 2, 3)], dim=1)
    V = torch.unique(faces).numel()
    assert F % 2 == 0 and V - (3 * F) // 2 + F == 2


def _volume_check(xyz, t):
    """Sum of the tetrahedra's volumes (fp64, on the device) against Qhull's hull volume."""
    import torch
    from scipy.spatial import ConvexHull
    X = torch.from_numpy(xyz).cuda()
    vol = 0.0
    chunk = 1 << 22
    for s in range(0, t.shape[0], chunk):
        q = t[s:s + chunk].long()
        a = X[q[:, 0]]
        u, v, w = X[q[:, 1]] - a, X[q[:, 2]] - a, X[q[:, 3]] - a
        vol += float((u * torch.cross(v, w, dim=1)).sum()) / 6.0
    hull = ConvexHull(xyz).volume
    say(f"volume: tetrahedra {vol:.12f}, hull {hull:.12f}")
    assert abs(vol - hull) <= 1e-8 * hull


def _hash_check(t_dev, name):
    g = GOLDEN[name]
    count, digest = canonical_hash_torch(t_dev)
    say(f"{name}: GPU {count} tetrahedra sha256 {digest[:16]}..; oracle {g['tets']} {g['sha256'][:16]}..")
    assert count == int(g["tets"]) and digest == g["sha256"], f"{name}: output differs from the oracle's"


def _full_certificate(oracle_mod, xyz, t_dev, nb_dev):
    import fullcheck
    t = t_dev.cpu().numpy().view(np.uint32)
    nb = nb_dev.cpu().numpy()
    say("every tetrahedron and facet (I1, I2, folds, I7)")
    T, interior, hull = fullcheck.check_all_facets(xyz, t, nb)
    say(f"{T} tetrahedra, {interior} interior facets locally Delaunay, {hull} hull facets")
    assert 2 * interior + hull == 4 * T
    assert fullcheck.check_hull_and_vertices(xyz, t, nb, oracle_mod, n_expect=len(xyz)) == hull


def test_uniform_1e6_whole_output(dtlib):
    """1e6 uniform points (seed 1006): the whole output equals the oracle's."""
    say("full size: uniform 1e6 (seed 1006)")
    t_dev, _ = _triangulate(dtlib, uniform_points(1_000_000, 1006))
    _hash_check(t_dev, "uniform_1e6")


def test_uniform_1e7_bench_config(dtlib, oracle_mod):
    """The benchmark workload: 1e7 uniform points, seed 1007.  The whole output equals the
    oracle's; the certificate and the device-side checks run on it too."""
    n = 10_000_000
    say("full size: uniform 1e7 (seed 1007), bench configuration")
    xyz = uniform_points(n, 1007)
    t_dev, nb_dev = _triangulate(dtlib, xyz)
    say(f"{len(t_dev)} tetrahedra")
    _hash_check(t_dev, "uniform_1e7")
    say("adjacency and hull")
    _adjacency_and_hull_check(t_dev, nb_dev)
    say("volume")
    _volume_check(xyz, t_dev)
    _full_certificate(oracle_mod, xyz, t_dev, nb_dev)


def test_uniform_1e8_certificate(dtlib, oracle_mod):
    """1e8 uniform points (seed 1008): the complete certificate on every facet, and a sub-box
    against the oracle."""
    import torch
    n = 100_000_000
    say("full size: uniform 1e8 (seed 1008), bench configuration")
    xyz = uniform_points(n, 1008)
    t_dev, nb_dev = _triangulate(dtlib, xyz)
    say(f"{len(t_dev)} tetrahedra")
    _subbox_check(oracle_mod, xyz, t_dev, 0.61, 0.126)
    _full_certificate(oracle_mod, xyz, t_dev, nb_dev)
    del t_dev, nb_dev
    torch.cuda.empty_cache()


def test_mix_1e7_whole_output(dtlib, oracle_mod):
    """MIX 1e7 (seed 2007, the benchmark's MIX input): the whole output equals the oracle's,
    and sub-boxes in the lattice and in the clusters against the oracle directly."""
    from synth import mix_points
    say("full size: MIX 1e7 (seed 2007), bench configuration")
    xyz = mix_points(2007)
    t_dev, nb_dev = _triangulate(dtlib, xyz)
    say(f"{len(t_dev)} tetrahedra")
    del nb_dev
    _hash_check(t_dev, "mix_1e7")
    # lattice nodes are odd multiples of 1/512; the box edges avoid them
    _subbox_check(oracle_mod, xyz, t_dev, -0.0996, 0.06, min_tets=1000)
    # a box around a cluster point (outside the lattice cube, inside r < 0.9)
    r = np.linalg.norm(xyz, axis=1)
    c = xyz[np.nonzero((r < 0.9) & (np.abs(xyz).max(axis=1) > 0.35))[0][0]]
    _subbox_check(oracle_mod, xyz, t_dev, c - 0.015, 0.03, min_tets=1000)


def test_batch_bench_config(dtlib, oracle_mod):
    """The benchmark's batch configuration: all 4096 clouds of the recipe (1.58e8 points, about
    1.05e9 tetrahedra) in one dt_insert_batch call, which takes 64-bit adjacency codes; a
    sample of clouds (the smallest, the largest, and every 256th) against the oracle run on
    that cloud alone."""
    import torch
    from synth import batch_clouds
    say("full size: batch of 4096 clouds (seeds 3000..7095), one call")
    xyz, off = batch_clouds(4096, seed_base=3000)
    off = off.astype(np.int64)
    stream = torch.cuda.current_stream()
    with dtlib.Triangulation(device=0, stream=stream.cuda_stream, timing=True) as tri:
        tri.insert_batch(torch.from_numpy(xyz).cuda(), off.astype(np.uint64))
        st = tri.stats()
        say(f"{st['rounds']} rounds, index_bits {st['index_bits']}")
        assert st["index_bits"] == 64
        sizes = np.diff(off)
        pick = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes))] + list(range(0, 4096, 256))))
        for k in pick:
            pts = xyz[off[k]:off[k + 1]]
            t, nb = tri.tets_batch(k)
            rc, ot, _, _ = oracle_mod.delaunay(pts)
            assert rc == 0
            a, b = oracle_mod.canonical(t.astype(np.int64)), oracle_mod.canonical(ot)
            assert a.shape == b.shape and np.array_equal(a, b), f"cloud {k}"
        say(f"{len(pick)} clouds match, largest {int(sizes.max())} points")
