"""Barycentric refinement, RWG and Buffa-Christiansen (BC) functions.

Section III of the paper discretises the static preconditioner on the BC
dual basis g_n: for every primal edge e_n = [v_minus, v_plus] a div-conforming
field on the barycentric refinement, built from fine RWG functions.  The
paper does not print the coefficients (it cites Buffa and Christiansen's
construction); this module derives them from the construction's defining
properties, with the paper's RWG normalisation (unit flux, no edge-length
factor):

* g_n is supported on the dual cells C(v_minus) and C(v_plus); the dual
  cell C(v) is the union of the 2 deg(v) fine triangles that touch v;
* g_n carries unit flux across the dual edge e_n* = [b(c_plus), m_n] U
  [m_n, b(c_minus)] (1/2 through each half), from C(v_minus) to C(v_plus),
  which makes it roughly n x f_n;
* inside a cell every fine triangle has the same net outflow,
  +1/(2 deg v_minus) in the source cell and -1/(2 deg v_plus) in the sink
  cell, so the BC loops (Sigma-combinations) are exactly div-free;
* the circulation left free by those conditions is fixed by mirror symmetry
  about e_n (no flux along the half of e_n itself).

On a fine triangle a lowest-order Raviart-Thomas field with outward edge
fluxes F_k (edge opposite vertex P_k) is sum_k F_k (x - P_k) / (2 A), so
every restriction has the form g_n|_t(x) = a x - b with a scalar a and a
vector b.  The same form holds for primal RWG functions on primal triangles.

This module is an input generator: it builds discretisation data only.
"""
from __future__ import annotations

import numpy as np

__all__ = ["Refinement", "refine", "rwg_local", "gram_bc"]


class Refinement:
    """Barycentric refinement plus BC restrictions.

    Attributes
    ----------
    fverts : (6 nf, 3, 3) fine triangle vertex coordinates, counter-clockwise
    fparent : (6 nf,) primal parent triangle
    fowner : (6 nf,) primal vertex whose dual cell contains the fine triangle
    bc_t, bc_n : (nnz,) fine triangle and BC index of each restriction
    bc_a : (nnz,) scalar a;  bc_b : (nnz, 3) vector b  (g_n|_t = a x - b)
    """


def _tri_area_normal(P):
    c = np.cross(P[..., 1, :] - P[..., 0, :], P[..., 2, :] - P[..., 0, :])
    A = 0.5 * np.linalg.norm(c, axis=-1)
    return A, c / (2.0 * A[..., None])


def refine(V, F, E):
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    E = np.asarray(E, dtype=np.int64)
    nv, nf, ne = V.shape[0], F.shape[0], E.shape[0]
    edge_of = {}
    for m in range(ne):
        edge_of[(int(E[m, 0]), int(E[m, 1]))] = m
    def eid(a, b):
        return edge_of[(a, b) if a < b else (b, a)]

    mid = 0.5 * (V[E[:, 0]] + V[E[:, 1]])
    bar = V[F].mean(axis=1)

    # fine triangles (f, k), k = 0..5:
    #  (a,M_ab,B) (M_ab,b,B) (b,M_bc,B) (M_bc,c,B) (c,M_ca,B) (M_ca,a,B)
    fverts = np.empty((nf, 6, 3, 3))
    fowner = np.empty((nf, 6), dtype=np.int64)
    for k in range(3):
        a, b = F[:, k], F[:, (k + 1) % 3]
        Mab = mid[[eid(int(x), int(y)) for x, y in zip(a, b)]]
        fverts[:, 2 * k, 0] = V[a]
        fverts[:, 2 * k, 1] = Mab
        fverts[:, 2 * k, 2] = bar
        fverts[:, 2 * k + 1, 0] = Mab
        fverts[:, 2 * k + 1, 1] = V[b]
        fverts[:, 2 * k + 1, 2] = bar
        fowner[:, 2 * k] = a
        fowner[:, 2 * k + 1] = b
    fverts = fverts.reshape(nf * 6, 3, 3)
    fowner = fowner.reshape(-1)
    fparent = np.repeat(np.arange(nf), 6)
    fA, _ = _tri_area_normal(fverts)

    # directed edge -> (face, local index of its start vertex)
    dir_face = {}
    for f in range(nf):
        for k in range(3):
            dir_face[(int(F[f, k]), int(F[f, (k + 1) % 3]))] = (f, k)

    # fine triangle index of the triangle in face f owned by vertex F[f,k],
    # adjacent to the edge leaving (k) or entering (k-1) that vertex
    def fine_out(f, k):      # (v, M_{v,next}, B)  -> k-th "even" triangle
        return f * 6 + 2 * k

    # ring around each vertex: sequence of (spoke vertex p, face after it)
    start = {}
    for (a, b), (f, k) in dir_face.items():
        start.setdefault(a, (f, k))
    rings = []
    for v in range(nv):
        f, k = start[v]
        seq = []
        f0 = f
        while True:
            p = int(F[f, (k + 1) % 3])       # spoke [v, p] precedes face f
            q = int(F[f, (k + 2) % 3])
            seq.append((p, f, k))
            f, k = dir_face[(v, q)]
            if f == f0:
                break
            if len(seq) > 64:
                raise ValueError("vertex ring did not close")
        rings.append(seq)

    rows_t, rows_n, rows_a, rows_b = [], [], [], []
    for n in range(ne):
        vm, vp = int(E[n, 0]), int(E[n, 1])
        for v, other, sgn in ((vm, vp, 1.0), (vp, vm, -1.0)):
            seq = rings[v]
            N = len(seq)
            j0 = [i for i, (p, _, _) in enumerate(seq) if p == other]
            if len(j0) != 1:
                raise ValueError("edge not found in vertex ring")
            j0 = j0[0]
            seq = seq[j0:] + seq[:j0]
            # internal fine edges e_0..e_{2N-1}: [v,M(spoke_0)], [v,B(face_0)], ...
            # fine triangles t_k between e_k and e_{k+1}
            # face f around v contributes (v, M_vp, B_f) then (M_qv, v, B_f)
            pts, tris = [], []
            for (p, f, k) in seq:
                pts.append(mid[eid(v, p)])
                pts.append(bar[f])
                tris.append(fine_out(f, k))
                tris.append(f * 6 + 2 * ((k + 2) % 3) + 1)
            Fk = np.array([0.0] + [(kk - N) / (2.0 * N) for kk in range(1, 2 * N)] + [0.0]) * sgn
            out = np.zeros(2 * N)
            out[0] = out[2 * N - 1] = 0.5 * sgn
            vpos = V[v]
            for kk in range(2 * N):
                t = tris[kk]
                P0 = pts[kk]                  # endpoint of e_k
                P1 = pts[(kk + 1) % (2 * N)]  # endpoint of e_{k+1}
                # outward fluxes: edge opposite v -> out_k; opposite P0 -> F_{k+1};
                # opposite P1 -> -F_k
                A2 = 2.0 * fA[t]
                a = (out[kk] + Fk[kk + 1] - Fk[kk]) / A2
                b = (out[kk] * vpos + Fk[kk + 1] * P0 - Fk[kk] * P1) / A2
                rows_t.append(t)
                rows_n.append(n)
                rows_a.append(a)
                rows_b.append(b)
    R = Refinement()
    R.nv, R.nf, R.ne = nv, nf, ne
    R.fverts = fverts
    R.fparent = fparent
    R.fowner = fowner
    R.farea = fA
    R.bc_t = np.asarray(rows_t, dtype=np.int64)
    R.bc_n = np.asarray(rows_n, dtype=np.int64)
    R.bc_a = np.asarray(rows_a)
    R.bc_b = np.asarray(rows_b)
    _check_fine_vertices(R, V, F)
    return R


def _check_fine_vertices(R, V, F):
    # each fine triangle owned by v must contain v as a vertex
    ok = np.any(np.all(np.isclose(R.fverts, V[R.fowner][:, None, :]), axis=-1), axis=-1)
    if not np.all(ok):
        raise ValueError("fine triangle ownership is inconsistent")


def rwg_local(V, F, E):
    """Primal RWG restrictions: f_m|_c(x) = a x - b on c in {c_plus, c_minus}.

    Returns arrays (tri, edge, a, b) with one row per (edge, side).
    """
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    E = np.asarray(E, dtype=np.int64)
    ne = E.shape[0]
    A, _ = _tri_area_normal(V[F])
    tri, edge, aa, bb = [], [], [], []
    for side, sgn in ((2, 1.0), (3, -1.0)):
        c = E[:, side]
        fv = F[c]
        opp = np.where((fv != E[:, [0]]) & (fv != E[:, [1]]), fv, -1).max(axis=1)
        # c_plus: (x - x_plus)/(2A);  c_minus: (x_minus - x)/(2A)
        a = sgn / (2.0 * A[c])
        b = sgn * V[opp] / (2.0 * A[c])[:, None]
        tri.append(c)
        edge.append(np.arange(ne))
        aa.append(a)
        bb.append(b)
    return (np.concatenate(tri), np.concatenate(edge), np.concatenate(aa),
            np.concatenate(bb))


def _rule3():
    # degree-2 rule: barycentric (2/3,1/6,1/6) permutations, weights 1/3
    L = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    return L, np.full(3, 1.0 / 3.0)


def gram_bc(V, F, E, R):
    """Dense Gram matrix G_mn = <n x f_m, g_n> (Section III).

    The integrand is quadratic on every fine triangle, so a degree-2 rule
    per fine triangle is exact.  Every BC restriction (fine triangle t, BC
    function n) meets the three RWG restrictions of t's primal parent; the
    products are formed for all of them at once and added in restriction
    order.
    """
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    ne, nf = E.shape[0], F.shape[0]
    _, nrm = _tri_area_normal(V[F])
    rt, re_, ra, rb = rwg_local(V, F, E)
    # the three RWG restrictions of every primal triangle, in restriction order
    order = np.argsort(rt, kind="stable")
    counts = np.bincount(rt, minlength=nf)
    if not np.all(counts == 3):
        raise ValueError("every primal triangle must carry three RWG restrictions")
    by_tri = order.reshape(nf, 3)
    Lq, wq = _rule3()
    xq = np.einsum("qk,tkd->tqd", Lq, R.fverts)          # (nft, 3, 3)
    T = R.bc_t
    C = R.fparent[T]
    I3 = by_tri[C]                                        # (nres, 3)
    X = xq[T]                                             # (nres, 3 pts, 3)
    g = R.bc_a[:, None, None] * X - R.bc_b[:, None, :]    # (nres, 3 pts, 3)
    f = ra[I3][:, :, None, None] * X[:, None] - rb[I3][:, :, None, :]   # (nres, 3, 3 pts, 3)
    nxf = np.cross(nrm[C][:, None, None, :], f)
    val = R.farea[T][:, None] * np.einsum("q,rkq->rk", wq, np.einsum("rkqd,rqd->rkq", nxf, g))
    G = np.zeros((ne, ne))
    np.add.at(G, (re_[I3].ravel(), np.repeat(R.bc_n, 3)), val.ravel())
    return G
