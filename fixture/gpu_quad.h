/*
 * Quadrature core of the device assembler (gpu_assemble.hip), written once
 * for the device and the host: the host build is how the point sets and the
 * per-test-point moments are checked against assemble.c without a GPU.
 *
 * Source points of a test point x on a source triangle: the far 7-point rule
 * when x is far and its distance range meets no retarded shell, else a polar
 * rule about the projection of x, split at every shell radius c dt k, in the
 * host assembler's order (see assemble.c).  Tables (Gauss-Legendre on [0, 1]
 * as [MAXGL + 1][MAXGL], the test rule and the far rule as rows of (l0, l1,
 * l2, w)) are read through a Tab.
 */
#ifndef FIXTURE_GPU_QUAD_H
#define FIXTURE_GPU_QUAD_H

#include <math.h>
#include <stddef.h>

#if defined(__HIPCC__)
#define QD __host__ __device__ __forceinline__
#define QM __host__ __device__ __forceinline__
#else
#define QD static inline
#define QM inline
#endif

#define FOUR_PI 12.566370614359172953850573533118
#define MAXGL 12

struct Tab { const double* glx; const double* glw; const double* rule; const double* far; };

struct V3 { double x, y, z; };
QD V3 mk(double x, double y, double z) { V3 r; r.x = x; r.y = y; r.z = z; return r; }
QD V3 add(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
QD V3 sub(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
QD V3 scl(V3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
QD double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
QD V3 crs(V3 a, V3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
QD double nrm(V3 a) { return sqrt(dot(a, a)); }

/* Triangle record, 16 doubles: vertices a0 a1 a2 (0-8), unit normal (9-11),
 * area (12), radius about the centroid (13); the centroid follows from the
 * vertices as in the host assembler, ((a0 + a1) + a2) (1/3). */
struct Tri { V3 a[3]; V3 n; double area; V3 c; double rad; };
QD Tri load_tri(const double* T, int t) {
    const double* p = T + (size_t)t * 16;
    Tri r;
    r.a[0] = mk(p[0], p[1], p[2]); r.a[1] = mk(p[3], p[4], p[5]); r.a[2] = mk(p[6], p[7], p[8]);
    r.n = mk(p[9], p[10], p[11]); r.area = p[12];
    const double third = 1.0 / 3;   /* a sum, then one product: nothing to contract */
    r.c = mk(((p[0] + p[3]) + p[6]) * third, ((p[1] + p[4]) + p[7]) * third, ((p[2] + p[5]) + p[8]) * third);
    r.rad = p[13];
    return r;
}

/* Polar rule over the sub-triangle (p, A, B) in the source plane, test point
 * at height d: emits sgn-weighted points (y, R, w) in the host assembler's
 * order.  Shell radii bps[k] = k cdt, k < nbp. */
template <class F>
QD void polar_subtri(const Tab& T, F& emit, V3 p, V3 nrml, double d, V3 A, V3 B, double sgn, double cdt, int nbp,
                             int nth, int nrh, double Rlo, double Rhi, int rstride, int roff, int& ray,
                             int kb) {
    V3 ua = sub(A, p), ub = sub(B, p);
    V3 eAB = sub(B, A);
    double lab = nrm(eAB);
    if (lab <= 0) return;
    double cr = dot(crs(ua, ub), nrml);
    double h = fabs(cr) / lab;
    if (h < 1e-14 * lab) return;
    double s = -dot(ua, eAB) / (lab * lab);
    V3 foot = add(ua, scl(eAB, s));
    V3 e1 = scl(foot, 1.0 / nrm(foot));
    V3 e2 = crs(nrml, e1);
    /* angular variable v = asinh(tan theta), theta measured from e1 (towards
     * the foot of the perpendicular, so the e1 components equal h > 0):
     * tan(theta) = (u . e2) / (u . e1) */
    double va = asinh(dot(ua, e2) / dot(ua, e1)), vb = asinh(dot(ub, e2) / dot(ub, e1));
    double lo = fmin(va, vb), hi = fmax(va, vb);
    double sg = (cr >= 0 ? 1.0 : -1.0) * sgn;
    /* Angular cuts in increasing order: lo, -vv_k (k descending), +vv_k (k
     * ascending), hi, where rho_edge(v) = h cosh v meets the shell radius. */
    /* stage 0: negatives, k from nbp-1 down; stage 1: positives, k up; stage 2: hi.
     * vv grows with k, so stage 0 can start below the first shell whose vv
     * reaches -lo (rb < h cosh(-lo), i.e. k c dt < sqrt((h cosh(-lo))^2 + d^2)),
     * and stage 1 can stop at the first vv >= hi; the cuts are the same. */
    int stage = 0, k = nbp - 1;
    if (lo >= 0) {
        stage = 1; k = 0;                        /* no negative cut: -vv < 0 <= lo */
    } else {
        double ch = h * cosh(-lo);
        double kb = floor(sqrt(ch * ch + d * d) / cdt) + 1;
        if (kb < k) k = (int)kb;
    }
    double prev = lo;
    for (;;) {
        double next;
        bool have = false;
        while (!have) {
            if (stage == 0) {
                if (k < 0) { stage = 1; k = 0; continue; }
                double Rb = cdt * k;
                --k;
                if (Rb <= d) continue;
                double rb = sqrt(Rb * Rb - d * d);
                if (rb <= h) continue;
                double vv = acosh(rb / h);
                if (-vv > lo && -vv < hi) { next = -vv; have = true; }
            } else if (stage == 1) {
                if (k >= nbp) { stage = 2; continue; }
                double Rb = cdt * k;
                ++k;
                if (Rb <= d) continue;
                double rb = sqrt(Rb * Rb - d * d);
                if (rb <= h) continue;
                double vv = acosh(rb / h);
                if (vv >= hi) { stage = 2; continue; }
                if (vv > lo) { next = vv; have = true; }
            } else if (stage == 2) {
                next = hi; have = true; stage = 3;
            } else {
                break;
            }
        }
        if (!have) break;
        /* piece [prev, next] split into ceil(L) equal parts */
        double L = next - prev;
        int np = (int)ceil(L / 1.0);
        if (np < 1) np = 1;
#pragma nounroll
        for (int j = 0; j < np; ++j) {
            double t0 = j == 0 ? prev : prev + L * j / np;
            double t1 = j == np - 1 ? next : prev + L * (j + 1) / np;
            if (t1 - t0 < 1e-15) continue;
#pragma nounroll
            for (int ia = 0; ia < nth; ++ia) {
                const int r = ray++;                      /* rays shared among rstride lanes */
                if (r % rstride != roff) continue;
                double v = t0 + (t1 - t0) * T.glx[nth * MAXGL + ia];
                /* theta = atan(sinh v): cos theta = 1 / cosh v, sin theta = tanh v */
                double chv = cosh(v);
                double wth = (t1 - t0) * T.glw[nth * MAXGL + ia] * sg / chv;
                double ct = 1.0 / chv, st = sinh(v) / chv;
                double re = h * chv;
                V3 dir = add(scl(e1, ct), scl(e2, st));
                /* the ray's points have R in [d, sqrt(re^2 + d^2)]: none in the band range */
                if (sqrt(re * re + d * d) < Rlo * (1 - 1e-12)) continue;
                /* radial breakpoints: 0, shell radii below re (ascending), grading
                 * points 2d 6d 18d ... below re (ascending), re; merged in order */
                double r0 = 0;
                int ks = (int)(d / cdt);                  /* shells up to d lie below the ray */
                if (ks > nbp) ks = nbp;
                double gnext = d > 0 ? 2 * d : 1e300;
                double rstop = 1e300;
                if (kb >= 0) {
                    /* only band kb: start at its lower shell (a breakpoint of the
                     * merged list), stop at its upper one; the pieces between
                     * are those of the full list */
                    const double Rb = cdt * kb, Rb1 = cdt * (kb + 1);
                    if (Rb1 <= d) continue;               /* every point lies above the band */
                    if (Rb > d) {
                        const double rb = sqrt(Rb * Rb - d * d);
                        if (!(rb > 0 && rb < re)) continue;   /* the ray ends below the band */
                        r0 = rb;
                        if (ks < kb + 1) ks = kb + 1;
                        while (gnext < r0) gnext *= 3;
                    }
                    rstop = sqrt(Rb1 * Rb1 - d * d);
                }
                for (;;) {
                    /* next shell radius rb in (0, re) */
                    double rs = 1e300;
                    while (ks < nbp) {
                        double Rb = cdt * ks;
                        if (Rb <= d) { ++ks; continue; }
                        double rb = sqrt(Rb * Rb - d * d);
                        if (rb > 0 && rb < re) { rs = rb; break; }
                        ++ks;
                        if (rb >= re) { ks = nbp; break; }
                    }
                    double rg = gnext < re ? gnext : 1e300;
                    double r1;
                    if (rs <= rg && rs < 1e300) { r1 = rs; ++ks; }
                    else if (rg < 1e300) { r1 = rg; gnext *= 3; }
                    else r1 = re;
                    /* R of the piece runs from sqrt(r0^2 + d^2) to sqrt(r1^2 + d^2) */
                    const bool inband = sqrt(r1 * r1 + d * d) >= Rlo * (1 - 1e-12) &&
                                        sqrt(r0 * r0 + d * d) <= Rhi * (1 + 1e-12);
                    if (inband && r1 - r0 > 1e-15 * re) {
                        if (d > 0) {
                            double u0 = asinh(r0 / d), u1 = asinh(r1 / d);
#pragma nounroll
                            for (int ir = 0; ir < nrh; ++ir) {
                                double u = u0 + (u1 - u0) * T.glx[nrh * MAXGL + ir];
                                double rho = d * sinh(u), R = sqrt(d * d + rho * rho);   /* d cosh u */
                                double w = wth * (u1 - u0) * T.glw[nrh * MAXGL + ir] * rho * R;
                                emit(add(p, scl(dir, rho)), R, w);
                            }
                        } else {
#pragma nounroll
                            for (int ir = 0; ir < nrh; ++ir) {
                                double rho = r0 + (r1 - r0) * T.glx[nrh * MAXGL + ir];
                                double w = wth * (r1 - r0) * T.glw[nrh * MAXGL + ir] * rho;
                                emit(add(p, scl(dir, rho)), rho, w);
                            }
                        }
                    }
                    if (r1 == re || r1 >= rstop) break;
                    r0 = r1;
                }
            }
        }
        prev = next;
        if (stage == 3) break;
    }
}

/* Source points of test point x on triangle t (shell spacing cdt, nbp radii;
 * nbp = 0: no shells).  far_n: points of the far rule.  Rlo, Rhi: polar
 * pieces (split at the shells) whose distance range misses [Rlo, Rhi] are not
 * emitted; the caller's callback must give such points zero weight anyway.
 * stride, off: this caller emits far points off, off + stride, ... and the
 * polar rays (sub-triangle, angular piece, node, counted in order) of the
 * same residue, so that stride lanes share one test point.  kb >= 0: only
 * shell band kb is wanted ([Rlo, Rhi] = [kb, kb + 1] c dt); each ray's radial
 * pieces are then walked from the band's lower shell to its upper one. */
template <class F>
QD void inner_points(const Tab& T, F& emit, V3 x, const Tri& t, double cdt, int nbp, int near, int far_n, int nth,
                             int nrh, double Rlo = 0.0, double Rhi = 1e300, int stride = 1, int off = 0,
                             int kb = -1) {
    double dc = nrm(sub(x, t.c));
    double Rmin = dc - t.rad, Rmax = dc + t.rad;
    int crosses = 0;
    for (int k = 0; k < nbp; ++k) {
        double b = cdt * k;
        if (b > Rmin && b < Rmax) { crosses = 1; break; }
    }
    if (!near && !crosses) {
#pragma nounroll
        for (int q = off; q < far_n; q += stride) {
            V3 y = add(add(scl(t.a[0], T.far[4 * q]), scl(t.a[1], T.far[4 * q + 1])), scl(t.a[2], T.far[4 * q + 2]));
            emit(y, nrm(sub(x, y)), T.far[4 * q + 3] * t.area);
        }
        return;
    }
    double d = dot(sub(x, t.a[0]), t.n);
    V3 p = sub(x, scl(t.n, d));
    d = fabs(d);
    if (d < 1e-12 * t.rad) d = 0;
    if (d > Rhi * (1 + 1e-12)) return;      /* every polar point has R >= d */
    int ray = 0;
    /* sub-triangles (p, a0, a1), (p, a1, a2), (p, a2, a0): the vertices are
     * rotated through registers (an indexed pick would put t in memory) */
    V3 A = t.a[0], B = t.a[1], C = t.a[2];
#pragma nounroll
    for (int k = 0; k < 3; ++k) {
        polar_subtri(T, emit, p, t.n, d, A, B, 1.0, cdt, nbp, nth, nrh, Rlo, Rhi, stride, off, ray, kb);
        const V3 tmp = A;
        A = B; B = C; C = tmp;
    }
}

/* temporal basis at u = tau/dt (Section V-A) */
QD double h0(double u) { double a = fabs(u); return a < 1 ? 1 - a : 0; }
QD double hd0(double u, double idt) {
    return (u > -1 && u < 0) ? idt : ((u >= 0 && u < 1) ? -idt : 0);
}
QD double q0f(double u) {
    if (u < -1 || u > 2) return 0;
    if (u < 0) return 0.5 * (u + 1) * (u + 1);
    if (u < 1) return 0.5 - u * u + u;
    return 0.5 * (u - 2) * (u - 2);
}
QD double qd0(double u, double idt) {
    if (u < -1 || u > 2) return 0;
    if (u < 0) return (u + 1) * idt;
    if (u < 1) return (1 - 2 * u) * idt;
    return (u - 2) * idt;
}
QD double qdd0(double u, double idt2) {
    if (u < -1 || u > 2) return 0;
    if (u < 0) return idt2;
    if (u < 1) return -2 * idt2;
    return idt2;
}
QD double p0f(double u) { return (u > -1 && u < 0) ? 1 : 0; }

/* Moments of one shell band k at one test point.  A point with
 * floor(R / (c dt)) = k adds window terms to lags k, k + 1, k + 2 (at u = i -
 * R/(c dt) in (-1, 0], (0, 1], (1, 2]) and its tilde-K tail (P = dt behind the
 * wavefront) to every lag from k + 1 on.  The host keeps a window term of lag
 * i only when i lies in the test point's window [ilo, ihi] (inwin[d] for i =
 * k + d), the tail always.  Slots hold (sum v, sum v y); the temporal factors
 * that vanish on a band's range are not stored (p0 and the P = tau + dt part
 * beyond lag k, h0 and hdot0 at lag k + 2). */
enum {
    BM_TH0 = 0, BM_KH0 = 4, BM_TFF0 = 8, BM_KHT0 = 12, BM_TT0 = 16, BM_KTW0 = 20, BM_TDD0 = 24,
    BM_TH1 = 25, BM_KH1 = 29, BM_TFF1 = 33, BM_KHT1 = 37, BM_TDD1 = 41,
    BM_TFF2 = 42, BM_KHT2 = 46, BM_TDD2 = 50,
    BM_KTT = 51, BM_N = 55
};
struct BandMoments {
    double m[BM_N];
    int band, nlag;
    int inwin[3];
    double ic, idt, idt2, dt, c;
    QM void clear() {
        for (int j = 0; j < BM_N; ++j) m[j] = 0;
    }
    QM void add4(int o, double v, V3 y) { m[o] += v; m[o + 1] += v * y.x; m[o + 2] += v * y.y; m[o + 3] += v * y.z; }
    QM void operator()(V3 y, double R, double w) {
        const double xi = R * ic * idt;
        const int i0 = (int)floor(xi);
        if (i0 != band) return;                 /* other bands have passes of their own */
        const double iR = 1.0 / R, gR = iR / FOUR_PI;
        const int k = band;
        /* lag k: u in (-1, 0] */
        if (inwin[0] && k <= nlag - 1) {
            const double u = k - xi;
            const double a_hd = hd0(u, idt), a_h0 = h0(u), a_q0 = q0f(u), a_qd = qd0(u, idt), a_qdd = qdd0(u, idt2);
            add4(BM_TH0, -ic * a_hd * gR * w, y);
            add4(BM_KH0, -(a_hd * ic * iR + a_h0 * iR * iR) * gR * w, y);
            add4(BM_TFF0, -ic * a_qdd * gR * w, y);
            m[BM_TDD0] += -c * a_q0 * gR * w;
            add4(BM_KHT0, -(a_qdd * ic * iR + a_qd * iR * iR) * gR * w, y);
            add4(BM_TT0, -ic * p0f(u) * gR * w, y);
            if (u > -1 && u <= 0) add4(BM_KTW0, -(ic * iR + (u + 1) * dt * iR * iR) * gR * w, y);
        }
        /* lag k + 1: u in (0, 1] */
        if (inwin[1] && k + 1 <= nlag - 1) {
            const double u = (k + 1) - xi;
            const double a_hd = hd0(u, idt), a_h0 = h0(u), a_q0 = q0f(u), a_qd = qd0(u, idt), a_qdd = qdd0(u, idt2);
            add4(BM_TH1, -ic * a_hd * gR * w, y);
            add4(BM_KH1, -(a_hd * ic * iR + a_h0 * iR * iR) * gR * w, y);
            add4(BM_TFF1, -ic * a_qdd * gR * w, y);
            m[BM_TDD1] += -c * a_q0 * gR * w;
            add4(BM_KHT1, -(a_qdd * ic * iR + a_qd * iR * iR) * gR * w, y);
        }
        /* lag k + 2: u in (1, 2] */
        if (inwin[2] && k + 2 <= nlag - 1) {
            const double u = (k + 2) - xi;
            const double a_q0 = q0f(u), a_qd = qd0(u, idt), a_qdd = qdd0(u, idt2);
            add4(BM_TFF2, -ic * a_qdd * gR * w, y);
            m[BM_TDD2] += -c * a_q0 * gR * w;
            add4(BM_KHT2, -(a_qdd * ic * iR + a_qd * iR * iR) * gR * w, y);
        }
        add4(BM_KTT, -(dt * iR * iR) * gR * w, y);
    }
};

/* Moments of one fine-triangle pair (s test, t source):
 *   M[i][j] = sum_x w_x X_i sum_y w_y Y_j / (4 pi R),  X = (x, 1), Y = (y, 1). */
struct StatMoments {
    double m0, m1x, m1y, m1z;
    QM void operator()(V3 y, double R, double w) {
        double v = w / (FOUR_PI * R);
        m0 += v; m1x += v * y.x; m1y += v * y.y; m1z += v * y.z;
    }
};


/* Shell bands a pair's source points can fall in.  Generated points have R
 * <= Rmax = |cs - ct| + rs + rt.  A far-rule point has R >= Rmin = |cs - ct|
 * - rs - rt; the polar rule (near pairs, or a test point whose distance range
 * meets a shell) walks signed sub-triangles about the projection of x on the
 * source plane, whose points only satisfy R >= the distance of x to that
 * plane, bounded below over the test triangle by its vertices' distances (0
 * if the plane cuts it).  cull: the host's pair cull (no contribution). */
struct PairBands { int cull, near, blo, bhi; };
QD PairBands pair_bands(const Tri& S, const Tri& Tt, const int* tris, int s, int t, double c, double dt, int nlag) {
    PairBands r;
    const double ic = 1.0 / c, idt = 1.0 / dt, cdt = c * dt;
    const double dcc = nrm(sub(S.c, Tt.c));
    const double Rpmin = dcc - S.rad - Tt.rad, Rpmax = dcc + S.rad + Tt.rad;
    int near = (s == t);
    if (!near) {
        for (int a = 0; a < 3 && !near; ++a)
            for (int b = 0; b < 3; ++b)
                if (tris[3 * s + a] == tris[3 * t + b]) { near = 1; break; }
        if (dcc < 2.0 * (S.rad + Tt.rad)) near = 1;
    }
    r.near = near;
    int polar = near;
    if (!polar) {
        /* is some shell radius k c dt, 0 <= k < nlag + 3, inside [Rmin, Rmax]? */
        double kmin = ceil(Rpmin * ic * idt - 1e-9);
        if (kmin < 0) kmin = 0;
        polar = kmin <= Rpmax * ic * idt + 1e-9 && kmin < nlag + 3;
    }
    double Rlow = Rpmin;
    if (polar) {
        double d0 = dot(sub(S.a[0], Tt.a[0]), Tt.n), d1 = dot(sub(S.a[1], Tt.a[0]), Tt.n),
               d2 = dot(sub(S.a[2], Tt.a[0]), Tt.n);
        double lb = 0;
        if (d0 > 0 && d1 > 0 && d2 > 0) lb = fmin(d0, fmin(d1, d2));
        else if (d0 < 0 && d1 < 0 && d2 < 0) lb = fmin(-d0, fmin(-d1, -d2));
        Rlow = fmin(Rlow, lb);
    }
    if (Rlow < 0) Rlow = 0;
    r.blo = (int)floor(Rlow * ic * idt * (1 - 1e-12) - 1e-12);
    r.bhi = (int)floor(Rpmax * ic * idt * (1 + 1e-12) + 1e-12);
    r.cull = Rpmin > cdt * (nlag + 1);
    return r;
}

/* Moments of band k at test point q of S against source triangle Tt; false
 * when the point lies beyond every stored lag (the host skips it). */
QD bool test_point_band(const Tab& T, const Tri& S, const Tri& Tt, int q, int near, double c, double dt, int nlag,
                        int k, int nth, int nrh, BandMoments& M) {
    const double ic = 1.0 / c, idt = 1.0 / dt;
    M.clear();
    M.band = k; M.nlag = nlag; M.ic = ic; M.idt = idt; M.idt2 = idt * idt; M.dt = dt; M.c = c;
    const V3 x = add(add(scl(S.a[0], T.rule[4 * q]), scl(S.a[1], T.rule[4 * q + 1])), scl(S.a[2], T.rule[4 * q + 2]));
    double dc = nrm(sub(x, Tt.c));
    double Rmin = fmax(0.0, dc - Tt.rad), Rmax = dc + Tt.rad;
    int ilo = (int)floor(Rmin * ic * idt) - 1;
    if (ilo < 0) ilo = 0;
    int ihi = (int)ceil(Rmax * ic * idt) + 2;
    if (ihi > nlag + 2) ihi = nlag + 2;
    if (ilo > nlag - 1) return false;
    for (int d = 0; d < 3; ++d) M.inwin[d] = k + d >= ilo && k + d <= ihi;
    const double cdt = c * dt;
    inner_points(T, M, x, Tt, cdt, nlag + 3, near, 7, nth, nrh, k * cdt, (k + 1) * cdt, 1, 0, k);
    return true;
}

/* Which rule test point q of the pair takes at lag i: 0 none (beyond every
 * stored lag, as the host skips it), 1 the far 7-point rule, 2 the polar rule
 * (near pair, or its distance range meets a shell). */
QD int test_point_class(const Tab& T, const Tri& S, const Tri& Tt, int q, int near, double c, double dt, int nlag) {
    const double ic = 1.0 / c, idt = 1.0 / dt, cdt = c * dt;
    V3 x = add(add(scl(S.a[0], T.rule[4 * q]), scl(S.a[1], T.rule[4 * q + 1])), scl(S.a[2], T.rule[4 * q + 2]));
    double dc = nrm(sub(x, Tt.c));
    int ilo = (int)floor(fmax(0.0, dc - Tt.rad) * ic * idt) - 1;
    if (ilo < 0) ilo = 0;
    if (ilo > nlag - 1) return 0;
    if (near) return 2;
    double Rmin = dc - Tt.rad, Rmax = dc + Tt.rad;
    for (int k = 0; k < nlag + 3; ++k) {
        double b = cdt * k;
        if (b > Rmin && b < Rmax) return 2;
    }
    return 1;
}

/* Output channels of a band pass: (lag offset d, block b: 0 Th 1 Kh 2 That 3 Khat
 * 4 Ttil 5 Ktil, K-type, moment slot, div-div slot or -1).  Channel 12 is the
 * tilde-K tail of the band, added to Ktil of lags k + 1 and k + 2 and to the
 * running accumulator that seeds later lags. */
struct Channel { int d, blk, isK, mom, dd; };
QD Channel band_channel(int ch) {
    Channel r;
    switch (ch) {
    case 0: r = Channel{0, 0, 0, BM_TH0, -1}; break;
    case 1: r = Channel{0, 1, 1, BM_KH0, -1}; break;
    case 2: r = Channel{0, 2, 0, BM_TFF0, BM_TDD0}; break;
    case 3: r = Channel{0, 3, 1, BM_KHT0, -1}; break;
    case 4: r = Channel{0, 4, 0, BM_TT0, -1}; break;
    case 5: r = Channel{0, 5, 1, BM_KTW0, -1}; break;
    case 6: r = Channel{1, 0, 0, BM_TH1, -1}; break;
    case 7: r = Channel{1, 1, 1, BM_KH1, -1}; break;
    case 8: r = Channel{1, 2, 0, BM_TFF1, BM_TDD1}; break;
    case 9: r = Channel{1, 3, 1, BM_KHT1, -1}; break;
    case 10: r = Channel{2, 2, 0, BM_TFF2, BM_TDD2}; break;
    case 11: r = Channel{2, 3, 1, BM_KHT2, -1}; break;
    default: r = Channel{1, 5, 1, BM_KTT, -1}; break;
    }
    return r;
}

/* RWG data of a pair at test point x: f_m = cm (x - Pm) on s, f_n = cn (y - Pn) on t. */
struct PairRWG { double cm[3], cn[3]; V3 xm[3], Pn[3], xn[3], Pm_[3]; };
QD PairRWG pair_rwg(const double* fcoef, const double* fopp, int s, int t, V3 x) {
    PairRWG r;
    for (int a = 0; a < 3; ++a) {
        r.cm[a] = fcoef[3 * s + a];
        const double* pa = fopp + 9 * s + 3 * a;
        r.Pm_[a] = mk(pa[0], pa[1], pa[2]);
        r.xm[a] = sub(x, r.Pm_[a]);
        r.cn[a] = fcoef[3 * t + a];
        const double* pb = fopp + 9 * t + 3 * a;
        r.Pn[a] = mk(pb[0], pb[1], pb[2]);
        r.xn[a] = sub(x, r.Pn[a]);
    }
    return r;
}

/* The RWG product of one block at one test point x of weight wx, for
 * f_m = cm (x - Pm) on the test triangle and f_n = cn (y - Pn) on the source:
 * T-type <f_m, sum v f_n> (+ the div-div term 4 dd of That), K-type
 * <f_m, (x - y) x f_n sum v>, with (x - y) x (y - Pn) = (x - Pn) x (y - Pn). */
QD double block_product(int isK, double m0, V3 m1, double dd, double cm, double cn, double wx, V3 xm, V3 Pn,
                        V3 x) {
    const double cc = cm * cn * wx;
    const V3 mm = sub(m1, scl(Pn, m0));
    if (isK) return cc * dot(xm, crs(sub(x, Pn), mm));
    return cc * (dot(xm, mm) + 4.0 * dd);
}

#endif
