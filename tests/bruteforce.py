"""Pure-Python brute force by definition, for tiny inputs only.

Independent of the C oracle: used to pin it.  Nothing here is fast.
"""
from __future__ import annotations

import itertools


def sqdist_pairs(points):
    """{(i, j): sum of squared coordinate differences} for i < j."""
    pts = [[int(v) for v in row] for row in points]
    n = len(pts)
    return {(i, j): sum((a - b) ** 2 for a, b in zip(pts[i], pts[j]))
            for i in range(n) for j in range(i + 1, n)}


def filtration(points, K_of):
    """Definition-level filtration.

    Edges are ordered by (squared distance, i, j); K_of(list_of_q) gives the
    number kept.  Returns (edges, rank, triangles) with triangles as sorted
    tuples (value, i, j, k), value = the largest rank among the three edges.
    """
    q = sqdist_pairs(points)
    n = len(points)
    edges = sorted(q, key=lambda e: (q[e], e[0], e[1]))
    K = K_of([q[e] for e in sorted(q)])
    kept = edges[:K]
    rank = {e: r for r, e in enumerate(kept)}
    tris = []
    for i, j, k in itertools.combinations(range(n), 3):
        if (i, j) in rank and (i, k) in rank and (j, k) in rank:
            tris.append((max(rank[(i, j)], rank[(i, k)], rank[(j, k)]), i, j, k))
    tris.sort()
    return kept, rank, tris, q


def total_order(n, kept, tris, tets=()):
    """Simplices in filtration order (value, dim, lex): vertices (value -1),
    then for each rank r the edge r followed by the triangles of value r and
    the tetrahedra of value r (rows (value, a, b, c, d))."""
    by_value, tet_by_value = {}, {}
    for t in sorted(tris):
        by_value.setdefault(t[0], []).append(t)
    for q in sorted(tuple(x) for x in tets):
        tet_by_value.setdefault(q[0], []).append(q)
    order = [("v", (i,)) for i in range(n)]
    for r, e in enumerate(kept):
        order.append(("e", e))
        for t in by_value.get(r, []):
            order.append(("t", t[1:]))
        for q in tet_by_value.get(r, []):
            order.append(("q", q[1:]))
    return order


def _f2_rank(vectors):
    basis = {}
    rank = 0
    for v in vectors:
        while v:
            h = v.bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                rank += 1
                break
    return rank


def persistent_betti(n, kept, tris, tets=()):
    """beta[k][(s, t)] for all s <= t indices into the total order: the rank of
    H_k(X_s) -> H_k(X_t), from F2 ranks of boundary matrices.

    beta_k^{s,t} = dim Z_k(X_s) - dim(B_k(X_t) cap C_k(X_s)),
    dim(B_k(X_t) cap C_k(X_s)) = rank d_{k+1}(X_t) - rank(P d_{k+1}(X_t)),
    with P the projection onto the k-simplices of X_t that are not in X_s.
    """
    order = total_order(n, kept, tris, tets)
    N = len(order)
    pos = {s: p for p, s in enumerate(order)}
    dim = [{"v": 0, "e": 1, "t": 2, "q": 3}[s[0]] for s in order]
    top = max(dim) if dim else 0

    def boundary(p):
        kind, verts = order[p]
        if kind == "v":
            return 0
        if kind == "e":
            return (1 << pos[("v", (verts[0],))]) | (1 << pos[("v", (verts[1],))])
        if kind == "t":
            i, j, k = verts
            return (1 << pos[("e", (i, j))]) | (1 << pos[("e", (i, k))]) | (1 << pos[("e", (j, k))])
        out = 0
        for f in itertools.combinations(verts, 3):
            out |= 1 << pos[("t", f)]
        return out

    bnd = [boundary(p) for p in range(N)]
    dims = tuple(range(max(3, top + 1)))
    beta = {k: {} for k in dims}
    for s in range(N):
        for k in dims:
            nk = sum(1 for p in range(s + 1) if dim[p] == k)
            rk = _f2_rank([bnd[p] for p in range(s + 1) if dim[p] == k])
            zk = nk - rk
            for t in range(s, N):
                cols = [bnd[p] for p in range(t + 1) if dim[p] == k + 1]
                if not cols:
                    beta[k][(s, t)] = zk
                    continue
                mask_out = 0
                for p in range(s + 1, t + 1):
                    if dim[p] == k:
                        mask_out |= 1 << p
                r_full = _f2_rank(cols)
                r_proj = _f2_rank([c & mask_out for c in cols])
                beta[k][(s, t)] = zk - (r_full - r_proj)
    return order, beta


def betti_from_pairs(N, pairs_by_dim, essential_by_dim, dims=(0, 1, 2)):
    """Same quantity from a pairing: bars (b, d) in total-order indices with
    b <= s and d > t, plus essential births b <= s."""
    beta = {k: {} for k in dims}
    for k in dims:
        for s in range(N):
            for t in range(s, N):
                c = sum(1 for b, d in pairs_by_dim.get(k, []) if b <= s and d > t)
                c += sum(1 for b in essential_by_dim.get(k, []) if b <= s)
                beta[k][(s, t)] = c
    return beta


def kruskal_deaths(n, kept):
    """Ranks of the edges that join two components, scanning edges in rank
    order with union-find (Kruskal's minimum spanning forest)."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    deaths = []
    for r, (i, j) in enumerate(kept):
        a, b = find(i), find(j)
        if a != b:
            parent[max(a, b)] = min(a, b)
            deaths.append(r)
    return deaths


def column_order(colptr, v):
    """z[i] = first slot of i's column + the entries of the column with a
    smaller value + the earlier entries of the column with the same value."""
    z = []
    for j in range(len(colptr) - 1):
        a, b = int(colptr[j]), int(colptr[j + 1])
        for i in range(a, b):
            z.append(a + sum(1 for t in range(a, b) if v[t] < v[i] or (v[t] == v[i] and t < i)))
    return z


def tetra_counts(points, K_of):
    """Per kept edge rank, the tetrahedra {a<b<c<d} with all six edges kept
    whose largest edge rank is that edge's (by definition, itertools)."""
    kept, rank, _, _ = filtration(points, K_of)
    out = [0] * len(kept)
    n = len(points)
    for quad in itertools.combinations(range(n), 4):
        rs = [rank.get(e) for e in itertools.combinations(quad, 2)]
        if all(x is not None for x in rs):
            out[max(rs)] += 1
    return out
