"""Input generators: meshes, edge tables, BC basis, quadrature, temporal basis."""
import math

import numpy as np
import pytest

import fixture as fx
from fixture import geometry as geo
from fixture.bc import refine, gram_bc


@pytest.mark.parametrize("spec,counts,genus", [
    (("icosphere", 1), (12, 20, 30), 0),
    (("icosphere", 4), (162, 320, 480), 0),
    (("torus", 1.0, 0.4, 64, 16), (1024, 2048, 3072), 1),
    (("box", 32, 32, 24), (5122, 10240, 15360), 0),
    (("star_pyramid", 12, 1.0, 0.3, 0.5, 1), (26, 48, 72), 0),
    (("star_pyramid", 12, 1.0, 0.3, 0.5, 7), (1178, 2352, 3528), 0),
])
def test_mesh_counts_and_topology(spec, counts, genus):
    from fixture.problem import make_mesh
    V, F, E = make_mesh(spec)
    assert (V.shape[0], F.shape[0], E.shape[0]) == counts
    assert geo.euler_genus(counts[0], counts[2], counts[1]) == genus
    Lam, Sig = geo.incidence_sparse(E, V.shape[0], F.shape[0])
    assert (Sig.T @ Lam).count_nonzero() == 0            # Sigma^T Lambda = 0 exactly
    # every triangle counter-clockwise w.r.t. the outward normal: positive volume
    p0, p1, p2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    assert np.einsum("ij,ij->i", p0, np.cross(p1, p2)).sum() > 0


def test_edge_table_convention():
    V, F = geo.icosphere(2)
    E = geo.edge_table(F)
    assert np.all(E[:, 0] < E[:, 1])
    for m in range(E.shape[0]):
        vm, vp, cp, cm = E[m]
        f = list(F[cp])
        k = f.index(vm)
        assert f[(k + 1) % 3] == vp                      # c_plus runs v_minus -> v_plus
        g = list(F[cm])
        k = g.index(vp)
        assert g[(k + 1) % 3] == vm


def test_triangle_rules_exact_on_monomials():
    # int over the reference triangle of x^a y^b = a! b! / (a+b+2)!
    for nq, deg in ((3, 2), (6, 4), (7, 5), (12, 6)):
        L, W = fx.triangle_rule(nq)
        assert abs(W.sum() - 1) < 1e-12
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                val = 0.5 * np.sum(W * L[:, 1] ** a * L[:, 2] ** b)
                ex = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
                assert abs(val - ex) < 1e-12, (nq, a, b)


def test_inner_quadrature_closed_forms():
    """Source-triangle point sets: area and solid angle (Van Oosterom-Strackee)."""
    tri = np.array([[0, 0, 0], [1, 0, 0], [0.2, 0.9, 0.]])
    area = 0.45
    rng = np.random.default_rng(1)
    for _ in range(60):
        x = np.array([rng.uniform(-0.5, 1.5), rng.uniform(-0.5, 1.4),
                      10 ** rng.uniform(-5, 0.3) * rng.choice([-1, 1])])
        bps = np.sort(rng.uniform(0, 2, size=rng.integers(0, 4)))
        s0, _, s3, _ = fx.inner_test(x, tri, bps, near=1, nth=6, nrh=6)
        a, b, c = tri - x
        la, lb, lc = map(np.linalg.norm, (a, b, c))
        om = abs(2 * np.arctan2(np.dot(a, np.cross(b, c)),
                                la * lb * lc + a @ b * lc + a @ c * lb + b @ c * la))
        assert abs(s0 - area) < 1e-8
        assert abs(s3 * abs(x[2]) - om) < 2e-5


def test_temporal_basis_identities():
    """Section V: q0 = (1/dt) int p0(xi) h0(t + xi) dxi (closed form), eq. (ph),
    eq. (hq), and d/dt^-1 p0."""
    dt = 0.7
    xs = np.linspace(-1.0, 0.0, 20001)
    for u in np.linspace(-1.5, 2.5, 41):
        vals = fx.temporal(u, dt)
        h = np.array([fx.temporal(u + x, dt)[0] for x in xs])      # h0(t + xi) on xi in (-dt,0)
        q_num = np.trapezoid(h, xs)                                 # (1/dt) int ... dxi, xi = x dt
        assert abs(vals[2] - q_num) < 1e-6
        # derivatives by central differences
        e = 1e-6
        hp, hm = fx.temporal(u + e, dt), fx.temporal(u - e, dt)
        if min(abs(u - k) for k in (-1, 0, 1, 2)) > 1e-3:
            assert abs((hp[0] - hm[0]) / (2 * e * dt) - vals[1]) < 1e-6
            assert abs((hp[2] - hm[2]) / (2 * e * dt) - vals[3]) < 1e-6
            assert abs((hp[3] - hm[3]) / (2 * e * dt) - vals[4]) < 1e-5
            assert abs((hp[6] - hm[6]) / (2 * e * dt) - vals[5]) < 1e-6
    # eq. (hq) with i = 0: (1/dt) int p0(t) h0(t + xi) dt = q0(xi)
    # eq. (ph): (1/dt) int p_i p0(t + xi) dt = h0(i dt + xi)
    for xi in np.linspace(-2.2, 2.2, 23):
        ts = np.linspace(-1.0, 0.0, 20001)
        lhs = np.trapezoid([fx.temporal(t + xi, dt)[5] for t in ts], ts)
        assert abs(lhs - fx.temporal(xi, dt)[0]) < 1e-3


def test_bc_basis_properties():
    for spec in (("icosphere", 2), ("torus", 1.0, 0.4, 12, 6), ("box", 2, 2, 2)):
        from fixture.problem import make_mesh
        V, F, E = make_mesh(spec)
        nv, nf, ne = V.shape[0], F.shape[0], E.shape[0]
        R = refine(V, F, E)
        G = gram_bc(V, F, E, R)
        Lam, Sig = geo.incidence(E, nv, nf)
        divg = np.zeros((ne, 6 * nf))
        divg[R.bc_n, R.bc_t] += 2 * R.bc_a
        assert abs(Sig.T @ divg).max() < 1e-12            # BC loops are div-free
        assert abs((divg * R.farea).sum(1)).max() < 1e-12  # zero net divergence
        assert abs(Lam.T @ G @ Sig).max() < 1e-12         # Lambda^T G Sigma = 0
        assert G.diagonal().min() > 0
        assert np.linalg.cond(G) < 10                      # well-conditioned Gram matrix


def test_static_blocks():
    from fixture.problem import make_mesh
    V, F, E = make_mesh(("icosphere", 2))
    R = refine(V, F, E)
    T0s, T0h = fx.static_blocks(R, geo.diameter(V))
    Lam, Sig = geo.incidence(E, V.shape[0], F.shape[0])
    assert np.linalg.eigvalsh(T0s).min() > 0                             # SPD
    assert np.linalg.eigvalsh(T0h).min() > -1e-12 * abs(T0h).max()        # PSD
    assert abs(T0h @ Sig).max() < 1e-12 * abs(T0h).max()                  # BC loops in its kernel


def test_retarded_blocks_structure():
    from fixture.problem import make_mesh
    V, F, E = make_mesh(("icosphere", 1))
    dt = 0.5
    B = fx.retarded_blocks(V, F, E, dt, 1.0, 6, 7, 5)
    Lam, Sig = geo.incidence(E, V.shape[0], F.shape[0])
    for k, X in B.items():
        assert np.allclose(X, np.transpose(X, (0, 2, 1)))                # Galerkin symmetry
    # asking for one family alone gives the same blocks
    D = B["T_hat"]
    Bs = fx.retarded_blocks(V, F, E, dt, 1.0, 6, 7, 5, which=("T_hat",))
    assert np.allclose(D, Bs["T_hat"])
    # causality: the diameter is 2, so nothing reaches beyond lag ceil(2/dt)+2
    assert abs(B["T_h"][5]).max() == 0.0


def test_star_pyramid_shape():
    """Base vertices alternate between the two circles in z = 0, one apex at
    the height; every vertex lies on a facet of the coarse pyramid."""
    from fixture.problem import make_mesh
    V, F, E = make_mesh(("star_pyramid", 12, 1.0, 0.3, 0.5, 2))
    assert np.isclose(V[:, 2].max(), 0.5) and np.isclose(V[:, 2].min(), 0.0)
    apex = V[np.argmax(V[:, 2])]
    assert np.allclose(apex, [0, 0, 0.5])
    r = np.hypot(V[:, 0], V[:, 1])
    assert np.isclose(r.max(), 1.0)
    base = V[np.isclose(V[:, 2], 0.0)]
    ang = np.degrees(np.arctan2(base[:, 1], base[:, 0])) % 360
    tips = np.isclose(np.hypot(base[:, 0], base[:, 1]), 1.0)
    notches = np.isclose(np.hypot(base[:, 0], base[:, 1]), 0.3)
    assert tips.sum() == 12 and notches.sum() == 12
    assert np.allclose(np.sort(ang[tips]), np.arange(0, 360, 30))
    assert np.allclose(np.sort(ang[notches]), np.arange(15, 360, 30))
    # closed, outward: positive enclosed volume equal to the pyramid's
    p0, p1, p2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    vol = np.einsum("ij,ij->i", p0, np.cross(p1, p2)).sum() / 6.0
    star_area = 12 * 2 * 0.5 * 1.0 * 0.3 * np.sin(np.radians(15))
    assert np.isclose(vol, star_area * 0.5 / 3)


def test_tilde_family_tail():
    """Section V-B, tilde family: once i dt exceeds the diameter (c = 1), the
    retarded time of every pair is past the pulse, so T~_i = 0 (p0 is zero
    there) and K~_i is one constant matrix (the integrated pulse has reached
    dt): the reason the tilde family is truncated at k_max - 1."""
    from fixture.problem import make_mesh
    V, F, E = make_mesh(("icosphere", 1))
    dt = 0.5
    B = fx.retarded_blocks(V, F, E, dt, 1.0, 6, 7, 9)
    first = int(np.ceil(geo.diameter(V) / dt))
    Kt, Tt = B["K_tilde"], B["T_tilde"]
    assert abs(Kt[first]).max() > 0
    for i in range(first, Kt.shape[0]):
        assert abs(Tt[i]).max() == 0.0
        assert np.allclose(Kt[i], Kt[first], rtol=0, atol=1e-15 * abs(Kt[first]).max())
    assert abs(Kt[first - 1] - Kt[first]).max() > 1e-3 * abs(Kt[first]).max()    # still varying before
