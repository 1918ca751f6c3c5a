"""Independent helpers for pinning the oracle (plain Python, tiny inputs).

These restate the definitions in the paper's words (forward joins, connected
components) rather than re-running the oracle's own tables.
"""
from __future__ import annotations

import itertools

import numpy as np

# The paper's forward joins of p(theta_i, phi_j): (i+1, j), (i+1, j+1), (i, j+1)
# (Section 2, Mesh Construction).  Everything else is a reverse of these.
FORWARD = ((1, 0), (1, 1), (0, 1))


def joins(H, Wp, wrap, valid):
    """Undirected join set built from the forward rule only."""
    E = set()
    for k in range(Wp):
        for i in range(H):
            for di, dk in FORWARD:
                ii, kk = i + di, k + dk
                if ii >= H:
                    continue
                if kk >= Wp:
                    if not wrap:
                        continue
                    kk -= Wp
                a, b = k * H + i, kk * H + ii
                if valid[a] and valid[b] and a != b:
                    E.add(frozenset((a, b)))
    return E


def cliques3(E):
    adj = {}
    for e in E:
        a, b = tuple(e)
        adj.setdefault(a, set()).add(b)
        adj.setdefault(b, set()).add(a)
    out = set()
    for a in adj:
        for b, c in itertools.combinations(sorted(adj[a]), 2):
            if c in adj.get(b, ()):
                out.add(frozenset((a, b, c)))
    return out


def mask_edges(H, Wp, mask):
    """Undirected edges implied by an oracle neighbour mask, using the opposite-slot
    symmetry only: bit t of p pairs with bit (t+3)%6 of the neighbour."""
    n = 0
    for m in mask:
        n += bin(int(m)).count("1")
    assert n % 2 == 0
    return n // 2


def closure_components(n, edges):
    """Connected components by transitive closure of the adjacency matrix (brute force)."""
    R = np.eye(n, dtype=bool)
    for a, b in edges:
        R[a, b] = R[b, a] = True
    while True:
        R2 = (R.astype(np.int64) @ R.astype(np.int64)) > 0
        if np.array_equal(R2, R):
            break
        R = R2
    return R


def union_find_labels(n, nodes, edges):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    # numbering: first appearance in cell (firing) order
    lab = np.zeros(n, dtype=np.int32)
    nxt = 1
    seen = {}
    for c in sorted(nodes):
        r = find(c)
        if r not in seen:
            seen[r] = nxt
            nxt += 1
        lab[c] = seen[r]
    return lab, nxt - 1


def canonical(labels):
    """Relabel a partition by first appearance (0 stays 0)."""
    out = np.zeros_like(labels)
    m = {}
    for i, l in enumerate(labels):
        if l == 0:
            continue
        if l not in m:
            m[l] = len(m) + 1
        out[i] = m[l]
    return out
