"""Canonical form and hash of a tetrahedralization, for whole-output comparisons at sizes
where the arrays are too large to store.  Test infrastructure: plain numpy, no part of the
method.

Canonical form: each tetrahedron's four vertex indices sorted ascending; the rows sorted
lexicographically.  The hash is SHA-256 over the canonical array as little-endian uint32
(16 bytes per tetrahedron).  The triangulation is unique under the perturbation, so two
correct outputs have equal hashes whatever their order.
"""
from __future__ import annotations

import hashlib

import numpy as np


def canonical_u32(tets) -> np.ndarray:
    """(T, 4) uint32 canonical array.  Indices must be below 2^31."""
    q = np.sort(np.asarray(tets).reshape(-1, 4).astype(np.int64), axis=1)
    if len(q) == 0:
        return np.zeros((0, 4), dtype=np.uint32)
    assert q.min() >= 0 and q.max() < (1 << 31)
    hi = (q[:, 0] << 32) | q[:, 1]
    lo = (q[:, 2] << 32) | q[:, 3]
    order = np.lexsort((lo, hi))
    return np.ascontiguousarray(q[order].astype("<u4"))


def digest_u32(canon: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(canon, dtype="<u4").tobytes()).hexdigest()


def canonical_hash(tets) -> tuple[int, str]:
    """(number of tetrahedra, SHA-256 of the canonical array)."""
    c = canonical_u32(tets)
    return len(c), digest_u32(c)


def canonical_hash_torch(t) -> tuple[int, str]:
    """The same hash of a (T, 4) int32 torch tensor, canonicalized on its device (stable
    sorts), then hashed on the host."""
    import torch
    q = torch.sort(t.long(), dim=1).values
    if q.shape[0] == 0:
        return 0, digest_u32(np.zeros((0, 4), dtype=np.uint32))
    hi = (q[:, 0] << 32) | q[:, 1]
    lo = (q[:, 2] << 32) | q[:, 3]
    o1 = torch.sort(lo, stable=True).indices
    o2 = torch.sort(hi[o1], stable=True).indices
    order = o1[o2]
    del hi, lo, o1, o2
    c = q[order].to(torch.int32).cpu().numpy().astype("<u4")
    return len(c), digest_u32(c)


def read_golden(path: str) -> dict:
    """Lines `name key=value ...` -> {name: {key: value}} (comments start with #)."""
    out = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, *kv = line.split()
        out[name] = dict(x.split("=", 1) for x in kv)
    return out
