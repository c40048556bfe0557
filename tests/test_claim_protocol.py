"""The round rule of the concurrent insertion, checked on the CPU with the oracle's exact
predicates (no GPU code involved).

One round on an existing triangulation: every attempt p with rank r has the cavity C(p) (the
tetrahedra whose perturbed circumsphere holds p) and the outer tetrahedra O(p) (neighbours of
C(p) outside it).  Each tetrahedron keeps the lowest claim of the round: 2 r from an attempt
with it in its cavity, 2 r + 1 from one with it outside.  p wins iff every tetrahedron of
C(p) holds 2 r and every tetrahedron of O(p) holds an odd claim.  These are the conflict rules
of Sec. 3.2 as claims.  The checks: the lowest rank wins; winners' cavities are disjoint and
no winner's cavity meets another winner's outer tetrahedra; and applying all winners at once
(remove every cavity, add every ball: the cavity's boundary facets joined to p, Sec. 2.5)
gives exactly the Delaunay tetrahedralization of the old points plus the winners.  Without
the claims on outer tetrahedra, adjacent cavities both win and that last equality breaks.
"""
import numpy as np
import pytest

from synth import uniform_points


def _cavities(oracle_mod, xyz, tets, nbrs, new_idx):
    """C(p) and O(p) for every new point, or None when the cavity reaches the hull."""
    from oracle.refine import circumcentres
    cc, r2 = circumcentres(xyz, tets)
    out = []
    for p in new_idx:
        d2 = ((cc - xyz[p]) ** 2).sum(axis=1)
        near = np.nonzero(d2 <= r2 * (1 + 1e-6) + 1e-12)[0]  # float prefilter, generous
        pts = np.concatenate([xyz[tets[near]], np.broadcast_to(xyz[p], (len(near), 1, 3))], axis=1)
        idx = np.concatenate([tets[near], np.full((len(near), 1), p)], axis=1)
        inside = near[oracle_mod.insphere_sos(pts, idx) < 0]
        cav = set(inside.tolist())
        nb = nbrs[inside]
        if np.any(nb < 0):
            out.append(None)
            continue
        outer = set(nb.reshape(-1).tolist()) - cav
        out.append((cav, outer))
    return out


def _round(oracle_mod, seed, claim_outer=True):
    """One round on the triangulation of 2500 points, attempted by the next 500 points that lie
    in [0.15, 0.85]^3 (about 170): returns (attempts, ranks, winners, number of winner pairs
    whose cavities meet, whether all winners applied at once give the oracle's
    triangulation)."""
    xyz = uniform_points(3000, 900 + seed)
    n0 = 2500
    # the new points away from the hull, so that no cavity reaches a ghost
    new = [i for i in range(n0, 3000) if np.all((xyz[i] > 0.15) & (xyz[i] < 0.85))]
    rc, tets, nbrs, _ = oracle_mod.delaunay(xyz[:n0])
    assert rc == 0
    tets, nbrs = tets.astype(np.int64), nbrs.astype(np.int64)
    att = [(p, c) for p, c in zip(new, _cavities(oracle_mod, xyz, tets, nbrs, new)) if c is not None]
    assert len(att) > 0.9 * len(new)
    rank = {p: r for r, p in enumerate(np.random.default_rng(seed).permutation([p for p, _ in att]))}
    claim = {}
    for p, (cav, outer) in att:
        S = 2 * rank[p]
        for t in cav:
            claim[t] = min(claim.get(t, S), S)
        if claim_outer:
            for t in outer:
                claim[t] = min(claim.get(t, S + 1), S + 1)
    winners = [(p, cav, outer) for p, (cav, outer) in att
               if all(claim[t] == 2 * rank[p] for t in cav)
               and (not claim_outer or all(claim[t] % 2 == 1 for t in outer))]
    touching = sum(1 for i, (p, cav, outer) in enumerate(winners) for q, cav2, outer2 in winners[i + 1:]
                   if (cav & cav2) or (cav & outer2) or (cav2 & outer))
    # all winners at once against the oracle on the old points and the winners (relative
    # index order kept, so the perturbation is the same); winners renumbered to their positions
    keep = np.ones(len(tets), dtype=bool)
    balls = []
    for p, cav, _ in winners:
        keep[list(cav)] = False
        for t in cav:
            for j in range(4):
                if nbrs[t, j] not in cav:
                    balls.append([v for k, v in enumerate(tets[t]) if k != j] + [p])
    built = np.vstack([tets[keep], np.array(balls, dtype=np.int64)])
    sub = np.concatenate([np.arange(n0), sorted(p for p, _, _ in winners)])
    pos = {int(g): k for k, g in enumerate(sub)}
    rc, ref, _, _ = oracle_mod.delaunay(xyz[sub])
    assert rc == 0
    a, b = oracle_mod.canonical(np.vectorize(pos.get)(built)), oracle_mod.canonical(ref)
    same = a.shape == b.shape and np.array_equal(a, b)
    return att, rank, winners, touching, same


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_one_round_of_claims(oracle_mod, seed):
    att, rank, winners, touching, same = _round(oracle_mod, seed)
    low = min(att, key=lambda a: rank[a[0]])[0]
    assert low in {p for p, _, _ in winners}  # progress: the lowest rank always wins
    assert 1 < len(winners) < len(att)
    assert touching == 0  # disjoint cavities, none meeting another winner's outer tetrahedra
    # winners may share an outer tetrahedron (each rewrites a different facet of it); such
    # pairs occur in every seed, so the equality below covers them
    assert any(o & o2 for i, (_, _, o) in enumerate(winners) for _, _, o2 in winners[i + 1:])
    assert same  # all winners at once = the triangulation of the old points plus the winners


def test_unclaimed_outer_tetrahedra_break_the_round(oracle_mod):
    """The same round with claims on cavity tetrahedra only: adjacent cavities both win, and
    their balls built at once are not the Delaunay tetrahedralization."""
    att, rank, winners, touching, same = _round(oracle_mod, 1, claim_outer=False)
    assert touching > 0 and not same


def test_rounds_until_every_point_is_in(oracle_mod):
    """Losers retry in the next round with their rank until none is left: every round inserts
    its lowest remaining rank (so the rounds end), and every round's winners applied at once
    give the oracle's triangulation of the points inserted so far."""
    xyz = uniform_points(2400, 907)
    n0 = 2000
    pending = [i for i in range(n0, 2400) if np.all((xyz[i] > 0.15) & (xyz[i] < 0.85))]
    rank = {p: r for r, p in enumerate(np.random.default_rng(7).permutation(pending))}
    done = list(range(n0))
    rounds = 0
    while pending:
        rounds += 1
        sub = np.array(sorted(done))
        rc, tets, nbrs, _ = oracle_mod.delaunay(xyz[sub])
        assert rc == 0
        tets, nbrs = sub[tets.astype(np.int64)], nbrs.astype(np.int64)  # global point indices
        cavs = _cavities(oracle_mod, xyz, tets, nbrs, pending)
        assert all(c is not None for c in cavs)
        claim = {}
        for p, (cav, outer) in zip(pending, cavs):
            S = 2 * rank[p]
            for t in cav:
                claim[t] = min(claim.get(t, S), S)
            for t in outer:
                claim[t] = min(claim.get(t, S + 1), S + 1)
        won = [(p, cav) for p, (cav, outer) in zip(pending, cavs)
               if all(claim[t] == 2 * rank[p] for t in cav) and all(claim[t] % 2 == 1 for t in outer)]
        assert min(pending, key=rank.get) in {p for p, _ in won}
        keep = np.ones(len(tets), dtype=bool)
        balls = []
        for p, cav in won:
            keep[list(cav)] = False
            balls += [[v for k, v in enumerate(tets[t]) if k != j] + [p]
                      for t in cav for j in range(4) if nbrs[t, j] not in cav]
        built = np.vstack([tets[keep], np.array(balls, dtype=np.int64)])
        done += [p for p, _ in won]
        pending = [p for p in pending if p not in {q for q, _ in won}]
        sub = np.array(sorted(done))
        pos = {int(g): k for k, g in enumerate(sub)}
        rc, ref, _, _ = oracle_mod.delaunay(xyz[sub])
        assert np.array_equal(oracle_mod.canonical(np.vectorize(pos.get)(built)), oracle_mod.canonical(ref))
    assert 2 < rounds < 60
