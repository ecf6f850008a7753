"""Closed triangulated surfaces and their RWG edge tables.

Seeded synthetic scatterers shaped like the paper's experiments (Section VI:
a sphere, a torus, a non-smooth body): geodesic icospheres, a torus on a
major x minor grid and the surface of an axis-aligned box.  Every mesh is
returned with counter-clockwise triangles with respect to the outward normal.

The edge table follows the RWG and incidence-matrix definitions of
Section II and Section IV-B:

* edge m is oriented from v_minus to v_plus (the vertex-edge matrix Lambda
  has +1 at v_plus and -1 at v_minus);
* the RWG function f_m flows from triangle c_plus to triangle c_minus (the
  face-edge matrix Sigma has +1 at c_plus and -1 at c_minus).

The paper does not tie the two orientations together; here c_plus is the
triangle whose counter-clockwise boundary runs v_minus -> v_plus.  With that
tie Sigma^T Lambda = 0 holds exactly.  Edges are enumerated in lexicographic
order of (min vertex, max vertex) and v_minus is the smaller index.

Nothing in this module computes any part of the marching-on-in-time method.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "icosphere", "torus", "box", "edge_table", "incidence", "incidence_sparse", "euler_genus",
    "check_mesh", "diameter", "mesh_size",
]


def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v / np.linalg.norm(v, axis=1, keepdims=True), f


def _dedupe(points, tris, tol=1e-9):
    key = np.round(points / tol).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    # keep the original order of first appearance for a stable numbering
    order = np.argsort(first)
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    verts = points[first[order]]
    return verts, rank[inv][tris]


def icosphere(nu: int, radius: float = 1.0):
    """Class-I geodesic sphere: each icosahedron face split into nu^2 triangles.

    20 nu^2 triangles, 30 nu^2 edges, 10 nu^2 + 2 vertices, projected onto the
    sphere of the given radius.
    """
    if nu < 1:
        raise ValueError("nu >= 1")
    v0, f0 = _icosahedron()
    pts, tris = [], []
    base = 0
    for a, b, c in f0:
        A, B, C = v0[a], v0[b], v0[c]
        idx = {}
        local = []
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                k = nu - i - j
                idx[(i, j)] = len(local)
                local.append((k * A + i * B + j * C) / nu)
        for i in range(nu):
            for j in range(nu - i):
                tris.append((base + idx[(i, j)], base + idx[(i + 1, j)], base + idx[(i, j + 1)]))
                if i + j < nu - 1:
                    tris.append((base + idx[(i + 1, j)], base + idx[(i + 1, j + 1)], base + idx[(i, j + 1)]))
        pts.extend(local)
        base += len(local)
    pts = np.asarray(pts)
    pts = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    verts, tris = _dedupe(pts, np.asarray(tris, dtype=np.int64))
    verts = verts * radius
    return verts, _orient_outward(verts, tris)


def torus(R: float = 1.0, r: float = 0.4, n_major: int = 64, n_minor: int = 16):
    """Torus with a n_major x n_minor vertex grid, quads split on a fixed diagonal."""
    th = 2.0 * np.pi * np.arange(n_major) / n_major
    ph = 2.0 * np.pi * np.arange(n_minor) / n_minor
    T, P = np.meshgrid(th, ph, indexing="ij")
    verts = np.stack([(R + r * np.cos(P)) * np.cos(T),
                      (R + r * np.cos(P)) * np.sin(T),
                      r * np.sin(P)], axis=-1).reshape(-1, 3)

    def vid(i, j):
        return (i % n_major) * n_minor + (j % n_minor)

    tris = []
    for i in range(n_major):
        for j in range(n_minor):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    tris = np.asarray(tris, dtype=np.int64)
    return verts, _orient_outward(verts, tris)


def box(nx: int, ny: int, nz: int, lengths=(1.0, 1.0, 1.0)):
    """Surface of [0,Lx]x[0,Ly]x[0,Lz] with an nx x ny x nz cell grid.

    4 (nx ny + ny nz + nx nz) triangles; sharp edges and corners.
    """
    Lx, Ly, Lz = lengths
    pts, tris = [], []

    def add_face(origin, du, dv, nu_, nv_):
        base = len(pts)
        for i in range(nu_ + 1):
            for j in range(nv_ + 1):
                pts.append(origin + du * (i / nu_) + dv * (j / nv_))
        for i in range(nu_):
            for j in range(nv_):
                a = base + i * (nv_ + 1) + j
                b = base + (i + 1) * (nv_ + 1) + j
                c = base + (i + 1) * (nv_ + 1) + j + 1
                d = base + i * (nv_ + 1) + j + 1
                tris.append((a, b, c))
                tris.append((a, c, d))

    o = np.zeros(3)
    ex, ey, ez = np.array([Lx, 0, 0.]), np.array([0, Ly, 0.]), np.array([0, 0, Lz])
    add_face(o, ex, ey, nx, ny)            # z = 0
    add_face(o + ez, ex, ey, nx, ny)       # z = Lz
    add_face(o, ey, ez, ny, nz)            # x = 0
    add_face(o + ex, ey, ez, ny, nz)       # x = Lx
    add_face(o, ex, ez, nx, nz)            # y = 0
    add_face(o + ey, ex, ez, nx, nz)       # y = Ly
    scale = max(Lx, Ly, Lz)
    verts, tris = _dedupe(np.asarray(pts) / scale, np.asarray(tris, dtype=np.int64))
    verts = verts * scale
    return verts, _orient_outward(verts, tris)


def star_pyramid(n_tips: int = 12, r_out: float = 1.0, r_in: float = 0.3, height: float = 0.5, nu: int = 1):
    """Pyramid over a star polygon (the paper's third, highly non-smooth
    scatterer, Section VI): the base has 2 n_tips vertices in the plane z = 0,
    alternately on circles of radius r_out (tips) and r_in (notches); the
    apex is at (0, 0, height).  Coarse facets: a fan of the base around its
    centre (the star is star-shaped about it) and one flat side triangle per
    base edge; each facet is split into nu^2 triangles.

    8 n_tips nu^2 triangles, 12 n_tips nu^2 edges, 4 n_tips nu^2 + 2 vertices.
    """
    if nu < 1 or n_tips < 3:
        raise ValueError("nu >= 1 and n_tips >= 3")
    nb = 2 * n_tips
    ang = 2.0 * np.pi * np.arange(nb) / nb
    rad = np.where(np.arange(nb) % 2 == 0, r_out, r_in)
    base = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.zeros(nb)], axis=1)
    centre = np.zeros(3)
    apex = np.array([0.0, 0.0, height])
    facets = []
    for i in range(nb):
        a, b = base[i], base[(i + 1) % nb]
        facets.append((centre, b, a))
        facets.append((a, b, apex))
    pts, tris = [], []
    for A, B, C in facets:
        idx = {}
        first = len(pts)
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                idx[(i, j)] = first + len(idx)
                pts.append(((nu - i - j) * A + i * B + j * C) / nu)
        for i in range(nu):
            for j in range(nu - i):
                tris.append((idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]))
                if i + j < nu - 1:
                    tris.append((idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]))
    verts, tris = _dedupe(np.asarray(pts), np.asarray(tris, dtype=np.int64))
    return verts, _orient_outward(verts, tris)


def _orient_outward(verts, tris):
    """Make every triangle counter-clockwise w.r.t. the outward normal.

    Orientation is first made consistent across edges by a breadth-first walk
    of the face graph, then flipped globally if the enclosed signed volume is
    negative.
    """
    tris = tris.copy()
    nf = tris.shape[0]
    # directed-edge -> face map for consistency propagation
    emap = {}
    for f in range(nf):
        for k in range(3):
            a, b = tris[f, k], tris[f, (k + 1) % 3]
            emap.setdefault((min(a, b), max(a, b)), []).append(f)
    done = np.zeros(nf, dtype=bool)
    done[0] = True
    stack = [0]
    while stack:
        f = stack.pop()
        for k in range(3):
            a, b = tris[f, k], tris[f, (k + 1) % 3]
            for g in emap[(min(a, b), max(a, b))]:
                if g == f or done[g]:
                    continue
                # consistent orientation: neighbour traverses the edge b -> a
                ok = False
                for kk in range(3):
                    if tris[g, kk] == b and tris[g, (kk + 1) % 3] == a:
                        ok = True
                if not ok:
                    tris[g] = tris[g, ::-1]
                done[g] = True
                stack.append(g)
    p0, p1, p2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    vol = np.einsum("ij,ij->i", p0, np.cross(p1, p2)).sum() / 6.0
    if vol < 0:
        tris = tris[:, ::-1].copy()
    return np.ascontiguousarray(tris.astype(np.int32))


def edge_table(tris):
    """Edge table E[ne][4] = (v_minus, v_plus, c_plus, c_minus), int32."""
    tris = np.asarray(tris)
    nf = tris.shape[0]
    a = tris.reshape(-1)
    b = np.roll(tris, -1, axis=1).reshape(-1)
    face = np.repeat(np.arange(nf), 3)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo.astype(np.int64) * (1 << 32) + hi
    order = np.lexsort((hi, lo))
    key_s = key[order]
    if key_s.size % 2 or not np.all(key_s[0::2] == key_s[1::2]):
        raise ValueError("surface is not closed and 2-manifold")
    if key_s.size > 2 and np.any(key_s[2::2] == key_s[1:-1:2]):
        raise ValueError("an edge is shared by more than two triangles")
    i0, i1 = order[0::2], order[1::2]
    ne = i0.size
    E = np.empty((ne, 4), dtype=np.int32)
    E[:, 0] = lo[i0]
    E[:, 1] = hi[i0]
    # the face that traverses lo -> hi (counter-clockwise) is c_plus
    fwd0 = a[i0] == lo[i0]
    E[:, 2] = np.where(fwd0, face[i0], face[i1])
    E[:, 3] = np.where(fwd0, face[i1], face[i0])
    fwd1 = a[i1] == lo[i1]
    if np.any(fwd0 == fwd1):
        raise ValueError("inconsistent triangle orientation")
    return E


def incidence(E, nv, nf):
    """Dense integer Lambda (ne x nv) and Sigma (ne x nf) of Section IV-B."""
    ne = E.shape[0]
    Lam = np.zeros((ne, nv), dtype=np.int64)
    Sig = np.zeros((ne, nf), dtype=np.int64)
    r = np.arange(ne)
    Lam[r, E[:, 1]] = 1
    Lam[r, E[:, 0]] = -1
    Sig[r, E[:, 2]] = 1
    Sig[r, E[:, 3]] = -1
    return Lam, Sig


def euler_genus(nv, ne, nf):
    chi = nv - ne + nf
    if chi % 2:
        raise ValueError("odd Euler characteristic")
    return (2 - chi) // 2


def incidence_sparse(E, nv, nf):
    """Lambda and Sigma as scipy.sparse CSR int64 matrices."""
    import scipy.sparse as sp
    ne = E.shape[0]
    r = np.repeat(np.arange(ne), 2)
    one = np.tile(np.array([1, -1], dtype=np.int64), ne)
    Lam = sp.csr_matrix((one, (r, E[:, [1, 0]].reshape(-1))), shape=(ne, nv))
    Sig = sp.csr_matrix((one, (r, E[:, [2, 3]].reshape(-1))), shape=(ne, nf))
    return Lam, Sig


def check_mesh(V, F, E):
    """Validate a closed orientable mesh; return its genus."""
    nv, nf, ne = V.shape[0], F.shape[0], E.shape[0]
    if 2 * ne != 3 * nf:
        raise ValueError("2 ne != 3 nf")
    Lam, Sig = incidence_sparse(E, nv, nf)
    if (Sig.T @ Lam).count_nonzero():
        raise ValueError("Sigma^T Lambda != 0")
    return euler_genus(nv, ne, nf)


def diameter(V):
    """Largest vertex-to-vertex distance."""
    V = np.asarray(V, dtype=np.float64)
    best = 0.0
    for s in range(0, V.shape[0], 512):
        d = np.linalg.norm(V[s:s + 512, None, :] - V[None, :, :], axis=-1)
        best = max(best, float(d.max()))
    return best


def mesh_size(V, F):
    """Mean edge length."""
    V, F = np.asarray(V), np.asarray(F)
    e = np.concatenate([V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 1]], V[F[:, 0]] - V[F[:, 2]]])
    return float(np.linalg.norm(e, axis=1).mean())
