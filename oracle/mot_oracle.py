"""Plain FP64 CPU oracle of the qHP TD-PMCHWT marching-on-in-time scheme.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the solver library
never does, and this module imports nothing from it.

Every function follows one passage of the paper (Le, Muenger, Andriulli,
Cools, "A Stable, Accurate, and Well-Conditioned Time-Domain PMCHWT
Formulation"):

* incidence matrices Lambda, Sigma ......... Section IV (opening)
* quasi-Helmholtz projectors ............... Section IV-B (projector defs)
* static preconditioner, loop-star form .... Section III, eq. (CP)
* media sum of the PMCHWT blocks ........... Section II, eq. (PMCHWT)
* lag matrices Q_i = Q^ll + Q^ls + Q^sl + Q^ss and the truncations,
  eq. (spec_prop); their inner sums block by block from one lag's raw
  blocks (lag_products) ........................ Section V-B
* right-hand side, loop and star parts ..... Section V-C, eq. (rhs), (hin)
* marching-on-in-time recurrence ........... Section V-A, eq. (MOT)
* current recovery, loop/star kept apart ... Section V-A, eq. (dis_jm)
* spectra of the loop and star currents at one frequency and the scattered
  far field they radiate ...................... Section VI (far-field
  computation) with eq. (dis_jm); the radiation integral itself is the
  textbook one, which the paper does not print

Dense linear algebra throughout: pseudo-inverses by numpy.linalg.pinv (of the
symmetric Gram matrices Sigma^T Sigma and Lambda^T Lambda, through their
symmetric eigendecomposition), G^-1 and Q_0^-1 by LU (scipy.linalg), no
blocking or fusion.

Readings where the paper is silent (also listed in the design notes):
* exterior c = eta = 1; interior c' = 1/sqrt(eps_r mu_r), eta' = sqrt(mu_r/eps_r);
* D = largest vertex distance, T_max = D / min(c, c'), k_max = ceil(T_max/dt);
* the raw hat and tilde blocks arrive without their T_max, 1/T_max factors;
* when k_max = 1 the lag-0 tilde K block is exactly dt K_0 (every pair inside
  the first shell) and is dropped like the tilde tail beyond k_max - 1, by
  eq. (spec_prop), so that its quadrature error does not grow with dt;
* RWG testing of the incident field uses the 7-point degree-5 triangle rule;
* the star part of the RHS is set to zero once the pulse has passed every
  point of the surface: t > t0 + (max_x k.x + 1.6 w)/c (erfc(6.4) ~ 1e-19);
* far field: exp(+i omega t) time convention, spectrum
  J(f) = int j(t) exp(-i 2 pi f t) dt of j(t) = sum_i j_i p_i(t) with p_i the
  unit pulse on ((i-1) dt, i dt); E_inf(rhat) = (i k / 4 pi)
  [rhat x L + eta rhat x (rhat x N)] (the exp(-i k r)/r factor dropped),
  N = int J exp(i k rhat.x) dS, L the same with M, eta = 1: the relative sign
  is the one for which a scatterer with the exterior's own medium radiates no
  scattered field.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.linalg as sla
from scipy.special import erf, erfc

__all__ = [
    "medium", "time_constants", "incidence", "projectors", "preconditioner",
    "media_sum", "lag_blocks", "lag_matrices", "LagOperator", "lag_products", "tri_rule7", "tested_fields", "rhs",
    "march", "recover", "Oracle", "block_toeplitz_solve", "star_cut",
    "rwg_at_rule_points", "current_spectrum", "radiation_vectors", "far_field",
]


# ------------------------------------------------------------------ media ---
def medium(eps_r, mu_r):
    """Section II: eta = sqrt(mu/eps), c = 1/sqrt(mu eps) per medium."""
    return 1.0, 1.0, 1.0 / math.sqrt(eps_r * mu_r), math.sqrt(mu_r / eps_r)


def time_constants(V, dt, eps_r, mu_r):
    """Section IV-C eq. (alpha): T_max = D / c_min; Section V-B: k_max = ceil(T_max/dt)."""
    V = np.asarray(V, dtype=np.float64)
    diff = V[:, None, :] - V[None, :, :]
    D = float(np.sqrt((diff ** 2).sum(-1)).max())
    _, _, cp, _ = medium(eps_r, mu_r)
    Tmax = D / min(1.0, cp)
    kmax = int(math.ceil(Tmax / dt - 1e-12))
    return D, Tmax, kmax


# ------------------------------------------------------------- incidence ---
def incidence(E, nv, nf):
    """Section IV: Lambda[m, v] = +1 at v_plus, -1 at v_minus;
    Sigma[m, f] = +1 at c_plus, -1 at c_minus."""
    E = np.asarray(E)
    ne = E.shape[0]
    Lam = np.zeros((ne, nv))
    Sig = np.zeros((ne, nf))
    for m in range(ne):
        Lam[m, E[m, 1]] += 1.0
        Lam[m, E[m, 0]] -= 1.0
        Sig[m, E[m, 2]] += 1.0
        Sig[m, E[m, 3]] -= 1.0
    return Lam, Sig


def projectors(Lam, Sig):
    """Section IV-B: P^Sigma = Sigma (Sigma^T Sigma)^+ Sigma^T, P^{Lambda H} = I - P^Sigma
    (RWG space); PP^Lambda = Lambda (Lambda^T Lambda)^+ Lambda^T, PP^{Sigma H} = I - PP^Lambda
    (BC space)."""
    ne = Lam.shape[0]
    I = np.eye(ne)
    PS = Sig @ np.linalg.pinv(Sig.T @ Sig, hermitian=True) @ Sig.T
    BL = Lam @ np.linalg.pinv(Lam.T @ Lam, hermitian=True) @ Lam.T
    return dict(PS=PS, PL=I - PS, BL=BL, BSH=I - BL)


def preconditioner(T0s, T0h, G, P):
    """Section III eq. (CP): T^{Sigma H} = PP^{Sigma H} T0s PP^{Sigma H},
    T^Lambda = PP^Lambda T0h PP^Lambda.  The left factors of the lag matrices
    (Section V-B) and of the RHS (Section V-C):
        C1 = T^{Sigma H} G^-1,   C2 = T^Lambda G^-1 P^{Lambda H}."""
    Tsh = P["BSH"] @ T0s @ P["BSH"]
    Tl = P["BL"] @ T0h @ P["BL"]
    lu = sla.lu_factor(G)
    Ginv = sla.lu_solve(lu, np.eye(G.shape[0]))
    C1 = Tsh @ Ginv
    C2 = Tl @ Ginv @ P["PL"]
    return dict(Tsh=Tsh, Tl=Tl, Ginv=Ginv, C1=C1, C2=C2)


def media_sum(T_ext, T_int, K_ext, K_int, eta, etap):
    """Section II eq. (PMCHWT) block pattern with both media:
    [[eta T + eta' T', -(K + K')], [K + K', T/eta + T'/eta']]."""
    M1 = eta * T_ext + etap * T_int
    M2 = T_ext / eta + T_int / etap
    Ks = K_ext + K_int
    return np.block([[M1, -Ks], [Ks, M2]])


def blk(X):
    """Block-wise action on the (j; m) halves: diag(X, X)."""
    Z = np.zeros_like(X)
    return np.block([[X, Z], [Z, X]])


def lag_blocks(raw, eps_r, mu_r, Tmax, kmax, i):
    """Section V-B: the media-summed raw blocks of lag i with their time
    scalings, each zero beyond its family's truncation:
        Z_i^h (i <= k_max),  T_max Z_i^hat (i <= k_max + 1),
        Z_i^tilde / T_max (i <= k_max - 1).
    The K part of Z_i^tilde is the time integral of the double layer; where it
    equals its constant tail (dt/T_max) K_0, eq. (spec_prop) makes its
    contribution to Q_i^sl vanish, and the paper sets it to zero (i > k_max - 1,
    where the whole tilde family is truncated).  The same holds at lag 0 when
    k_max = 1 (c_min dt >= D): every pair lies in the first shell, where the
    integral of p_0 is dt - R/c and its constant part has no gradient, so the
    lag-0 tilde K block is exactly dt K_0 and is set to zero as well.
    raw[medium][name] has shape (nlags, ne, ne), name in T_h, K_h, T_hat,
    K_hat, T_tilde, K_tilde; medium in ext, int; lags past the stored ones
    are zero."""
    _, eta, _, etap = medium(eps_r, mu_r)
    ne = raw["ext"]["T_h"].shape[1]
    n = 2 * ne

    def Z(fam, limit, scale, static_k=False):
        if i > limit or i >= raw["ext"]["T_" + fam].shape[0]:
            return np.zeros((n, n))
        Ke, Ki = raw["ext"]["K_" + fam][i], raw["int"]["K_" + fam][i]
        if static_k:
            Ke, Ki = np.zeros_like(Ke), np.zeros_like(Ki)
        return scale * media_sum(raw["ext"]["T_" + fam][i], raw["int"]["T_" + fam][i], Ke, Ki, eta, etap)

    return (Z("h", kmax, 1.0), Z("hat", kmax + 1, Tmax),
            Z("tilde", kmax - 1, 1.0 / Tmax, static_k=(i == 0 and kmax <= 1)))


def lag_matrices(raw, pre, P, eps_r, mu_r, Tmax, kmax, nlag=None):
    """Section V-B: Q_i for i = 0 .. k_max + 1 (only the first nlag of them
    when nlag is given, enough for the first nlag steps of the march),

        Q_i^ll = C1 Z_i^h  P^{Lambda H}      (h family, i <= k_max)
        Q_i^ls = C1 Z_i^hat P^Sigma          (hat family times T_max, i <= k_max + 1)
        Q_i^ss = C2 Z_i^h  P^Sigma           (h family, i <= k_max)
        Q_i^sl = C2 Z_i^til P^{Lambda H}     (tilde family over T_max, i <= k_max - 1,
                                              truncated beyond as the paper enforces)
    each acting block-wise on the (u; v) halves (lag_blocks for the Z's).
    """
    C1b, C2b = blk(pre["C1"]), blk(pre["C2"])
    PLb, PSb = blk(P["PL"]), blk(P["PS"])
    Q = []
    for i in range(kmax + 2 if nlag is None else min(kmax + 2, nlag)):
        Zh, Zhat, Ztil = lag_blocks(raw, eps_r, mu_r, Tmax, kmax, i)
        Q.append(C1b @ (Zh @ PLb + Zhat @ PSb) + C2b @ (Zh @ PSb + Ztil @ PLb))
    return Q


class LagOperator:
    """Q_i of Section V-B as an operator, for meshes on which forming every
    dense Q_i costs too much: the products of lag_matrices taken right to left,
        Q_i X = C1 (Z_i^h P^{Lambda H} X + Z_i^hat P^Sigma X)
              + C2 (Z_i^h P^Sigma X + Z_i^til P^{Lambda H} X)   (block-wise C, P),
    equal to lag_matrices(...)[i] @ X up to the order of the roundings.
    Q_i @ X works as with the dense matrix (march accepts either)."""

    def __init__(self, raw, pre, P, eps_r, mu_r, Tmax, kmax, i, blocks=None):
        self.Zh, self.Zhat, self.Ztil = lag_blocks(raw, eps_r, mu_r, Tmax, kmax, i)
        self.blocks = blocks if blocks is not None else dict(
            C1b=blk(pre["C1"]), C2b=blk(pre["C2"]), PLb=blk(P["PL"]), PSb=blk(P["PS"]))

    def __matmul__(self, X):
        b = self.blocks
        xl = b["PLb"] @ X
        xs = b["PSb"] @ X
        return b["C1b"] @ (self.Zh @ xl + self.Zhat @ xs) + b["C2b"] @ (self.Zh @ xs + self.Ztil @ xl)


def lag_products(raw_i, eps_r, mu_r, Tmax, kmax, i, XL, XS):
    """Section V-B, the inner sums of Q_i X from the raw blocks of lag i alone,
    block by block, without forming the media sums:
        Y1 = Z_i^h XL + Z_i^hat XS,    Y2 = Z_i^h XS + Z_i^til XL,
    each Z with the block pattern of eq. (PMCHWT) (media_sum) and its family's
    time scaling and truncation (lag_blocks); so that Q_i X = C1b Y1 + C2b Y2
    for XL = P^{Lambda H} X, XS = P^Sigma X block-wise (LagOperator).
    raw_i[medium][name]: the (ne, ne) blocks of lag i (a family whose blocks
    are absent counts as zero); XL, XS: (2 ne, c), halves (u; v)."""
    _, eta, _, etap = medium(eps_r, mu_r)
    ne = XL.shape[0] // 2
    Y1 = np.zeros(XL.shape)
    Y2 = np.zeros(XL.shape)

    def apply(fam, limit, scale, static_k, X, Y):
        if i > limit or ("T_" + fam) not in raw_i["ext"]:
            return
        a, b = X[:ne], X[ne:]
        Te, Ti = raw_i["ext"]["T_" + fam], raw_i["int"]["T_" + fam]
        Y[:ne] += scale * (eta * (Te @ a) + etap * (Ti @ a))          # eta T + eta' T'
        Y[ne:] += scale * ((Te @ b) / eta + (Ti @ b) / etap)          # T/eta + T'/eta'
        if not static_k:
            Ke, Ki = raw_i["ext"]["K_" + fam], raw_i["int"]["K_" + fam]
            Y[:ne] -= scale * (Ke @ b + Ki @ b)                       # -(K + K')
            Y[ne:] += scale * (Ke @ a + Ki @ a)                       # K + K'

    apply("h", kmax, 1.0, False, XL, Y1)
    apply("hat", kmax + 1, Tmax, False, XS, Y1)
    apply("h", kmax, 1.0, False, XS, Y2)
    apply("tilde", kmax - 1, 1.0 / Tmax, i == 0 and kmax <= 1, XL, Y2)
    return Y1, Y2


# ------------------------------------------------------------------- RHS ---
def tri_rule7():
    """Radon's 7-point degree-5 rule on a triangle (barycentric, weights sum 1)."""
    s = math.sqrt(15.0)
    a, b = (6 - s) / 21, (6 + s) / 21
    wa, wb = (155 - s) / 1200, (155 + s) / 1200
    L = [(1 / 3, 1 / 3, 1 / 3)]
    W = [9 / 40]
    for x, w in ((a, wa), (b, wb)):
        L += [(1 - 2 * x, x, x), (x, 1 - 2 * x, x), (x, x, 1 - 2 * x)]
        W += [w, w, w]
    return np.array(L), np.array(W)


def _erf_diff(s1, s0):
    """erf(s1) - erf(s0) without cancellation in the tails."""
    out = np.empty_like(s1)
    pos = s0 >= 0
    neg = s1 <= 0
    mid = ~(pos | neg)
    out[pos] = erfc(s0[pos]) - erfc(s1[pos])
    out[neg] = erfc(-s1[neg]) - erfc(-s0[neg])
    out[mid] = erf(s1[mid]) - erf(s0[mid])
    return out


def star_cut(V, wave):
    """Time after which the star RHS is truncated (Section V-C)."""
    kx = np.asarray(V) @ wave.dir
    return wave.t0 + (kx.max() + 1.6 * wave.width) / 1.0


def tested_fields(V, F, E, waves, dt, k):
    """Section II (RHS vectors) and Section V-C (eq. rhs, hin), at step k:

        ebar_k = (1/dt) int_{(k-1)dt}^{k dt} (e; h)(t) dt     (loop part, p_k testing)
        Ebar_k = int_{-inf}^{k dt} (e; h)(t) dt                 (star part, delta_k testing)

    with [e(t)]_m = <n x f_m, e_in x n> = -<f_m, e_in> and likewise h with
    h_in = k x e_in / eta.  The Gaussian time integral is closed-form:
    int_{-inf}^t e_in = A/(2c) p (1 + erf s),  s = (4/w)(c (t - t0) - k.x).
    The spatial integral over the two triangles of each RWG uses the 7-point
    rule; all edges are evaluated at once (numpy), one wave at a time.
    Returns ebar, Ebar of shape (2 ne, R); Ebar is zeroed after star_cut.
    """
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F)
    E = np.asarray(E)
    ne = E.shape[0]
    L, W = tri_rule7()
    R = len(waves)
    ebar = np.zeros((2 * ne, R))
    Ebar = np.zeros((2 * ne, R))
    c = 1.0
    for side, sgn in ((2, 1.0), (3, -1.0)):
        f = E[:, side]
        tv = V[F[f]]                                        # (ne, 3, 3)
        area = 0.5 * np.linalg.norm(np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0]), axis=1)
        fv = F[f]
        opp = np.where((fv != E[:, [0]]) & (fv != E[:, [1]]), fv, -1).max(axis=1)
        X = np.einsum("qk,mkd->mqd", L, tv)                 # (ne, 7, 3) quadrature points
        fm = sgn * (X - V[opp][:, None, :]) / (2 * area)[:, None, None]   # RWG values (Section II)
        wq = W[None, :] * area[:, None]
        for r, wv in enumerate(waves):
            s1 = (4 / wv.width) * (c * (k * dt - wv.t0) - X @ wv.dir)
            s0 = (4 / wv.width) * (c * ((k - 1) * dt - wv.t0) - X @ wv.dir)
            amp = wv.amp / (2 * c)
            hp = np.cross(wv.dir, wv.pol)                   # eta = 1
            te = amp * _erf_diff(s1.ravel(), s0.ravel()).reshape(s1.shape) / dt
            tE = amp * erfc(-s1)
            if k * dt > star_cut(V, wv):
                tE = np.zeros_like(tE)
            fp = fm @ wv.pol
            fh = fm @ hp
            ebar[:ne, r] += -np.sum(wq * te * fp, axis=1)
            ebar[ne:, r] += -np.sum(wq * te * fh, axis=1)
            Ebar[:ne, r] += -np.sum(wq * tE * fp, axis=1)
            Ebar[ne:, r] += -np.sum(wq * tE * fh, axis=1)
    return ebar, Ebar


def rhs(pre, Tmax, ebar, Ebar):
    """Section V-C eq. (rhs): r = C1 ebar + (1/T_max) C2 Ebar, block-wise."""
    return blk(pre["C1"]) @ ebar + blk(pre["C2"]) @ Ebar / Tmax


# ------------------------------------------------------------------ march ---
def march(Q, rhs_vectors, lu=None, W0=None):
    """Section V-A eq. (MOT): Q_0 w_i = r_i - sum_{k=1}^{i-1} Q_k w_{i-k},
    with Q_k = 0 beyond the last stored lag.  rhs_vectors: (N_t, n, R).
    lu: the LU factorization of Q_0 (scipy.linalg.lu_factor), formed here if
    None.  W0: (M, n, R) unknowns of the M steps that precede the first of
    rhs_vectors (none if None), so that a march can be resumed."""
    Nt = rhs_vectors.shape[0]
    if lu is None:
        lu = sla.lu_factor(Q[0])
    M = 0 if W0 is None else W0.shape[0]
    W = np.zeros((M + Nt,) + rhs_vectors.shape[1:], dtype=rhs_vectors.dtype)
    if M:
        W[:M] = W0
    for i in range(M, M + Nt):               # step i+1 in the paper's numbering
        b = rhs_vectors[i - M].copy()
        for k in range(1, min(i, len(Q) - 1) + 1):
            b -= Q[k] @ W[i - k]
        W[i] = sla.lu_solve(lu, b)
    return W[M:]


def block_toeplitz_solve(Q, rhs_vectors):
    """The whole lower block-triangular Toeplitz system eq. (fulldis_PMCHWT)
    assembled and solved at once (tiny problems only)."""
    Nt, n, R = rhs_vectors.shape
    A = np.zeros((Nt * n, Nt * n))
    for i in range(Nt):
        for j in range(i + 1):
            k = i - j
            if k < len(Q):
                A[i * n:(i + 1) * n, j * n:(j + 1) * n] = Q[k]
    x = np.linalg.solve(A, rhs_vectors.reshape(Nt * n, R))
    return x.reshape(Nt, n, R)


def recover(P, Tmax, dt, W):
    """Section V-A eq. (dis_jm), loop and star parts kept apart:
    j_i^loop = P^{Lambda H} u_i,  j_i^star = (T_max/dt) P^Sigma (u_i - u_{i-1}),
    u_0 = 0; the same for m from v.  W: (N_t, 2 ne, R)."""
    ne = P["PS"].shape[0]
    Nt = W.shape[0]
    prev = np.zeros_like(W[0])
    loop = np.zeros_like(W)
    star = np.zeros_like(W)
    for i in range(Nt):
        for h in (slice(0, ne), slice(ne, 2 * ne)):
            loop[i, h] = P["PL"] @ W[i, h]
            star[i, h] = (Tmax / dt) * (P["PS"] @ (W[i, h] - prev[h]))
        prev = W[i]
    return loop, star


# -------------------------------------------------------------- far field ---
def rwg_at_rule_points(V, F, E):
    """Section II (RWG definition): the 7-point rule points of both triangles
    of every edge, the RWG value there and the weight times area.
    Returns X (ne, 2, 7, 3), f (ne, 2, 7, 3), w (ne, 2, 7)."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F)
    E = np.asarray(E)
    L, W = tri_rule7()
    Xs, fs, ws = [], [], []
    for side, sgn in ((2, 1.0), (3, -1.0)):
        f = E[:, side]
        tv = V[F[f]]
        area = 0.5 * np.linalg.norm(np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0]), axis=1)
        fv = F[f]
        opp = np.where((fv != E[:, [0]]) & (fv != E[:, [1]]), fv, -1).max(axis=1)
        X = np.einsum("qk,mkd->mqd", L, tv)
        Xs.append(X)
        fs.append(sgn * (X - V[opp][:, None, :]) / (2 * area)[:, None, None])
        ws.append(W[None, :] * area[:, None])
    return np.stack(Xs, 1), np.stack(fs, 1), np.stack(ws, 1)


def current_spectrum(X, dt, freq, first=0):
    """Section VI (far-field computation) on eq. (dis_jm): the Fourier
    transform at freq of the current sum_i X_i p_i(t), where row s of X is
    the coefficient of step first+s+1, whose pulse covers
    ((first+s) dt, (first+s+1) dt):  sum_s X_s int_pulse exp(-i 2 pi f t) dt.
    X: (count, n, R) real.  Returns (n, R) complex."""
    s = first + np.arange(X.shape[0])
    if freq == 0:
        w = np.full(s.shape, dt, dtype=complex)
    else:
        om = 2 * np.pi * freq
        w = (np.exp(-1j * om * s * dt) - np.exp(-1j * om * (s + 1) * dt)) / (1j * om)
    return np.einsum("s,snr->nr", w, X)


def radiation_vectors(V, F, E, k, dirs):
    """int f_n(x) exp(i k rhat.x) dS for every RWG f_n and direction rhat
    (7-point rule on both triangles).  dirs: (ndir, 3).  Returns
    (ndir, ne, 3) complex."""
    X, f, w = rwg_at_rule_points(V, F, E)
    dirs = np.asarray(dirs, dtype=np.float64)
    out = np.zeros((dirs.shape[0], E.shape[0], 3), complex)
    for a, rh in enumerate(dirs):
        ph = np.exp(1j * k * (X @ rh))                        # (ne, 2, 7)
        out[a] = np.einsum("mtq,mtqd->md", w * ph, f)
    return out


def far_field(V, F, E, spec, freq, dirs, eta=1.0, c=1.0):
    """Far field radiated by the spectra spec (2 ne, R) = (J; M) at freq:
    E_inf(rhat) = (i k / 4 pi) [rhat x L + eta rhat x (rhat x N)],
    N = sum_n J_n F_n(rhat), L = sum_n M_n F_n(rhat), k = 2 pi f / c.
    Returns (ndir, R, 3) complex."""
    ne = E.shape[0]
    k = 2 * np.pi * freq / c
    Fv = radiation_vectors(V, F, E, k, dirs)                  # (ndir, ne, 3)
    dirs = np.asarray(dirs, dtype=np.float64)
    out = np.zeros((dirs.shape[0], spec.shape[1], 3), complex)
    for a, rh in enumerate(dirs):
        Nv = np.einsum("nd,nr->rd", Fv[a], spec[:ne])
        Lv = np.einsum("nd,nr->rd", Fv[a], spec[ne:])
        rr = np.broadcast_to(rh, Nv.shape)
        out[a] = (1j * k / (4 * np.pi)) * (np.cross(rr, Lv) + eta * np.cross(rr, np.cross(rr, Nv)))
    return out


# ------------------------------------------------------------ convenience ---
class Oracle:
    """All oracle stages for one problem dict (see fixture.problem)."""

    def __init__(self, prob, nlag=None, operators=False, log=None):
        """nlag: build Q_0 .. Q_{nlag-1} only; run() is then exact for the
        first nlag steps (eq. (MOT) uses Q_1 .. Q_{i-1} at step i).
        operators: Q_0 dense (its LU solves each step), Q_1 .. as LagOperator.
        log: called with the name of each stage as it completes."""
        self.prob = prob
        self.nlag = nlag
        self.log = log if log is not None else (lambda stage: None)
        V, F, E = prob["V"], prob["F"], prob["E"]
        self.D, self.Tmax, self.kmax = time_constants(V, prob["dt"], prob["eps_r"], prob["mu_r"])
        Lam, Sig = incidence(E, V.shape[0], F.shape[0])
        self.Lam, self.Sig = Lam, Sig
        self.P = projectors(Lam, Sig)
        self.log("projectors")
        self.pre = preconditioner(prob["T0s"], prob["T0h"], prob["G"], self.P)
        self.log("preconditioner")
        if not operators:
            self.Q = lag_matrices(prob["raw"], self.pre, self.P, prob["eps_r"], prob["mu_r"],
                                  self.Tmax, self.kmax, nlag)
        else:
            self.Q = lag_matrices(prob["raw"], self.pre, self.P, prob["eps_r"], prob["mu_r"],
                                  self.Tmax, self.kmax, 1)
            blocks = dict(C1b=blk(self.pre["C1"]), C2b=blk(self.pre["C2"]), PLb=blk(self.P["PL"]),
                          PSb=blk(self.P["PS"]))
            last = self.kmax + 2 if nlag is None else min(self.kmax + 2, nlag)
            self.Q += [LagOperator(prob["raw"], self.pre, self.P, prob["eps_r"], prob["mu_r"], self.Tmax,
                                   self.kmax, i, blocks) for i in range(1, last)]
        self.log("lag matrices")

    def rhs_all(self, nsteps):
        p = self.prob
        out = []
        for k in range(1, nsteps + 1):
            eb, Eb = tested_fields(p["V"], p["F"], p["E"], p["waves"], p["dt"], k)
            out.append(rhs(self.pre, self.Tmax, eb, Eb))
        return np.array(out)

    def run(self, nsteps=None):
        nsteps = self.prob["nsteps"] if nsteps is None else nsteps
        if self.nlag is not None and nsteps > self.nlag:
            raise ValueError("only the first %d steps are exact with %d lag matrices" % (self.nlag, self.nlag))
        r = self.rhs_all(nsteps)
        self.log("right-hand sides")
        W = march(self.Q, r)
        self.log("march")
        loop, star = recover(self.P, self.Tmax, self.prob["dt"], W)
        return dict(r=r, W=W, loop=loop, star=star)

    def far_field(self, res, freq, dirs, first=0, count=None):
        """Spectra at freq of the loop and star currents of steps
        first+1 .. first+count (res from run) and the far field each radiates,
        kept apart (eq. (dis_jm) remark).  Returns dict(spec (2, n, R) complex:
        loop, star; field (ndir, R, 2, 3) complex)."""
        count = res["W"].shape[0] - first if count is None else count
        p = self.prob
        spec = np.stack([current_spectrum(res[part][first:first + count], p["dt"], freq, first)
                         for part in ("loop", "star")])
        field = np.stack([far_field(p["V"], p["F"], p["E"], spec[i], freq, dirs) for i in range(2)], axis=2)
        return dict(spec=spec, field=field)
