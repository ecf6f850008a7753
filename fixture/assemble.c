/*
 * Galerkin assembly of the retarded and static boundary-integral blocks
 * that the qHP TD-PMCHWT marching scheme consumes (input generator).
 *
 * Retarded blocks, per medium of wave speed c, lag i, with g = 1/(4 pi R)
 * and tau_i = i dt - R/c (Section V-B):
 *   h family     T_i  = -(1/c) <f_m, f_n hdot0(tau) g>
 *                K_i  = <f_m, grad_x[h0(tau) g] x f_n>
 *   hat family   That_i = -(1/c) <f_m, f_n qddot0(tau) g> - c <div f_m, div f_n q0(tau) g>
 *                Khat_i = <f_m, grad_x[qdot0(tau) g] x f_n>
 *   tilde family Ttil_i = -(1/c) <f_m, f_n p0(tau) g>
 *                Ktil_i = <f_m, grad_x[P(tau) g] x f_n>,  P = integral of p0
 * i.e. the collocated-in-time operators T^s(h0 f), d/dt T(q0 f) and
 * d/dt^{-1} T^s(p0 f) (and the K analogues) without the T_max factors,
 * which the solver applies.  <n x f_m, n x X> = <f_m, X> for tangential f_m.
 *
 * grad_x[phi(tau) g(R)] = -(x - y)/(4 pi R) [phi'(tau)/(c R) + phi(tau)/R^2],
 * and (x - y) x (y - P) = (x - P) x (y - P) for an RWG f_n = s (y - P).
 *
 * Static blocks on the BC basis (Section III, eq. static_EFIE):
 *   T0s_mn = (1/D) <g_m, g_n g>,   T0h_mn = D <div g_m, div g_n g>.
 *
 * Quadrature: an N_q-point symmetric rule on the test triangle; the source
 * integral is done in polar coordinates about the projection of the test
 * point on the source plane, split at every retarded-shell radius
 * R = c dt k, with Gauss-Legendre nodes in each angular / radial piece
 * (a radial asinh substitution removes the near-singular behaviour of
 * 1/R and 1/R^3 near the projection point).  Far pairs whose distance range
 * meets no shell radius use a plain product rule.
 *
 * Rows m of an output block are written only by the triangles that carry
 * RWG m; the caller passes a face order grouped by a colouring of the face
 * graph so that one colour can be processed in parallel without races.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FOUR_PI 12.566370614359172953850573533118
#define MAXGL 12

typedef struct { double x, y, z; } v3;
static inline v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 crs(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static inline double nrm(v3 a) { return sqrt(dot(a, a)); }
static inline v3 ld(const double* p) { return mk(p[0], p[1], p[2]); }

/* ---------------- Gauss-Legendre on [0,1] ---------------- */
static double gl_x[MAXGL + 1][MAXGL], gl_w[MAXGL + 1][MAXGL];
static int gl_ready = 0;
static void gl_init(void) {
    if (gl_ready) return;
    for (int n = 1; n <= MAXGL; ++n) {
        for (int i = 0; i < n; ++i) {
            double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0;
            for (int it = 0; it < 100; ++it) {
                double p1 = 1, p2 = 0;
                for (int j = 1; j <= n; ++j) { double p3 = p2; p2 = p1; p1 = ((2.0 * j - 1) * z * p2 - (j - 1.0) * p3) / j; }
                pp = n * (z * p1 - p2) / (z * z - 1);
                double dz = p1 / pp; z -= dz;
                if (fabs(dz) < 1e-16) break;
            }
            gl_x[n][i] = 0.5 * (1 - z);
            gl_w[n][i] = 1.0 / ((1 - z * z) * pp * pp);
        }
    }
    gl_ready = 1;
}

/* ---------------- triangle rules (barycentric, weights sum 1) ---------------- */
typedef struct { int n; double l[16][3]; double w[16]; } trule;
static void perm3(trule* r, double a, double b, double w) {
    r->l[r->n][0] = a; r->l[r->n][1] = b; r->l[r->n][2] = b; r->w[r->n++] = w;
    r->l[r->n][0] = b; r->l[r->n][1] = a; r->l[r->n][2] = b; r->w[r->n++] = w;
    r->l[r->n][0] = b; r->l[r->n][1] = b; r->l[r->n][2] = a; r->w[r->n++] = w;
}
static void perm6(trule* r, double a, double b, double c, double w) {
    double p[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
    for (int k = 0; k < 6; ++k) { for (int d = 0; d < 3; ++d) r->l[r->n][d] = p[k][d]; r->w[r->n++] = w; }
}
static int make_rule(int nq, trule* r) {
    r->n = 0;
    if (nq == 1) { r->l[0][0] = r->l[0][1] = r->l[0][2] = 1.0 / 3; r->w[0] = 1; r->n = 1; return 0; }
    if (nq == 3) { perm3(r, 2.0 / 3, 1.0 / 6, 1.0 / 3); return 0; }
    if (nq == 6) {
        perm3(r, 0.108103018168070, 0.445948490915965, 0.223381589678011);
        perm3(r, 0.816847572980459, 0.091576213509771, 0.109951743655322);
        return 0;
    }
    if (nq == 7) {
        double s15 = sqrt(15.0), a = (6 - s15) / 21, b = (6 + s15) / 21;
        r->l[0][0] = r->l[0][1] = r->l[0][2] = 1.0 / 3; r->w[0] = 9.0 / 40; r->n = 1;
        perm3(r, 1 - 2 * a, a, (155 - s15) / 1200);
        perm3(r, 1 - 2 * b, b, (155 + s15) / 1200);
        return 0;
    }
    if (nq == 12) {
        perm3(r, 0.501426509658179, 0.249286745170910, 0.116786275726379);
        perm3(r, 0.873821971016996, 0.063089014491502, 0.050844906370207);
        perm6(r, 0.053145049844817, 0.310352451033784, 0.636502499121399, 0.082851075618374);
        return 0;
    }
    return -1;
}

/* ---------------- inner (source) quadrature point sets ---------------- */
typedef struct { int n, cap; double* y; double* R; double* w; } ipts;
static void ip_push(ipts* p, v3 y, double R, double w) {
    if (p->n == p->cap) {
        p->cap = p->cap ? 2 * p->cap : 4096;
        p->y = (double*)realloc(p->y, sizeof(double) * 3 * p->cap);
        p->R = (double*)realloc(p->R, sizeof(double) * p->cap);
        p->w = (double*)realloc(p->w, sizeof(double) * p->cap);
    }
    p->y[3 * p->n] = y.x; p->y[3 * p->n + 1] = y.y; p->y[3 * p->n + 2] = y.z;
    p->R[p->n] = R; p->w[p->n] = w; p->n++;
}

typedef struct { v3 a[3]; v3 n; double area; v3 c; double rad; } tri_t;
static void tri_make(tri_t* t, v3 a, v3 b, v3 c) {
    t->a[0] = a; t->a[1] = b; t->a[2] = c;
    v3 cr = crs(sub(b, a), sub(c, a));
    double l = nrm(cr);
    t->area = 0.5 * l; t->n = scl(cr, 1.0 / l);
    t->c = scl(add(add(a, b), c), 1.0 / 3);
    double r0 = nrm(sub(a, t->c)), r1 = nrm(sub(b, t->c)), r2 = nrm(sub(c, t->c));
    t->rad = fmax(r0, fmax(r1, r2));
}

static int cmp_d(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Sub-triangle (p, A, B) in the source plane, with test point at height d.
 * Adds points for sgn * integral over the sub-triangle.  Radial variable
 * u = asinh(rho/d) (d > 0) or rho (d == 0), split at the shell radii and at
 * geometric grading points 2d, 8d, 32d, ... */
static void polar_subtri(ipts* P, v3 p, v3 nrml, double d, v3 A, v3 B, double sgn,
                         const double* bps, int nbp, int nth, int nrh) {
    v3 ua = sub(A, p), ub = sub(B, p);
    v3 eAB = sub(B, A);
    double lab = nrm(eAB);
    if (lab <= 0) return;
    double cr = dot(crs(ua, ub), nrml);
    double h = fabs(cr) / lab;                     /* distance p -> line AB */
    if (h < 1e-14 * lab) return;
    /* in-plane frame: e1 towards the foot of the perpendicular */
    double s = -dot(ua, eAB) / (lab * lab);
    v3 foot = add(ua, scl(eAB, s));
    v3 e1 = scl(foot, 1.0 / nrm(foot));
    v3 e2 = crs(nrml, e1);
    double tha = atan2(dot(ua, e2), dot(ua, e1)), thb = atan2(dot(ub, e2), dot(ub, e1));
    /* angular variable v = asinh(tan theta): rho_edge = h cosh v, dtheta = dv / cosh v */
    double va = asinh(tan(tha)), vb = asinh(tan(thb));
    double lo = fmin(va, vb), hi = fmax(va, vb);
    double sg = (cr >= 0 ? 1.0 : -1.0) * sgn;
    /* split points: where rho_edge = rho_b (v = +-acosh(rho_b/h)) and pieces of length <= 1 */
    double cut[512]; int nc = 0;
    cut[nc++] = lo;
    for (int k = 0; k < nbp; ++k) {
        double Rb = bps[k];
        if (Rb <= d) continue;
        double rb = sqrt(Rb * Rb - d * d);
        if (rb <= h) continue;
        double vv = acosh(rb / h);
        if (vv > lo && vv < hi && nc < 200) cut[nc++] = vv;
        if (-vv > lo && -vv < hi && nc < 200) cut[nc++] = -vv;
    }
    cut[nc++] = hi;
    qsort(cut, nc, sizeof(double), cmp_d);
    int nc2 = nc;
    for (int a = 0; a + 1 < nc; ++a) {
        double L = cut[a + 1] - cut[a];
        int np = (int)ceil(L / 1.0);
        for (int j = 1; j < np && nc2 < 500; ++j) cut[nc2++] = cut[a] + L * j / np;
    }
    nc = nc2;
    qsort(cut, nc, sizeof(double), cmp_d);
    for (int a = 0; a + 1 < nc; ++a) {
        double t0 = cut[a], t1 = cut[a + 1];
        if (t1 - t0 < 1e-15) continue;
        for (int ia = 0; ia < nth; ++ia) {
            double v = t0 + (t1 - t0) * gl_x[nth][ia];
            double chv = cosh(v);
            double wth = (t1 - t0) * gl_w[nth][ia] * sg / chv;
            double th = atan(sinh(v));
            double ct = cos(th), st = sin(th);
            double re = h * chv;
            v3 dir = add(scl(e1, ct), scl(e2, st));
            /* radial breakpoints in rho */
            double rk[160]; int nr = 0;
            rk[nr++] = 0;
            for (int k = 0; k < nbp; ++k) {
                double Rb = bps[k];
                if (Rb <= d) continue;
                double rb = sqrt(Rb * Rb - d * d);
                if (rb > 0 && rb < re && nr < 100) rk[nr++] = rb;
            }
            if (d > 0) for (double g = 2 * d; g < re && nr < 150; g *= 3) rk[nr++] = g;
            rk[nr++] = re;
            qsort(rk, nr, sizeof(double), cmp_d);
            for (int b = 0; b + 1 < nr; ++b) {
                double r0 = rk[b], r1 = rk[b + 1];
                if (r1 - r0 <= 1e-15 * re) continue;
                if (d > 0) {
                    double u0 = asinh(r0 / d), u1 = asinh(r1 / d);
                    for (int ir = 0; ir < nrh; ++ir) {
                        double u = u0 + (u1 - u0) * gl_x[nrh][ir];
                        double rho = d * sinh(u), R = d * cosh(u);
                        double w = wth * (u1 - u0) * gl_w[nrh][ir] * rho * R;   /* rho drho = rho R du */
                        ip_push(P, add(p, scl(dir, rho)), R, w);
                    }
                } else {
                    for (int ir = 0; ir < nrh; ++ir) {
                        double rho = r0 + (r1 - r0) * gl_x[nrh][ir];
                        double w = wth * (r1 - r0) * gl_w[nrh][ir] * rho;
                        ip_push(P, add(p, scl(dir, rho)), rho, w);
                    }
                }
            }
        }
    }
}

/* Source points for test point x over triangle t.  bps: shell radii. */
static void inner_points(ipts* P, v3 x, const tri_t* t, const double* bps, int nbp,
                         int near, const trule* far_rule, int nth, int nrh) {
    P->n = 0;
    double dc = nrm(sub(x, t->c));
    double Rmin = dc - t->rad, Rmax = dc + t->rad;
    int crosses = 0;
    for (int k = 0; k < nbp; ++k) if (bps[k] > Rmin && bps[k] < Rmax) { crosses = 1; break; }
    if (!near && !crosses) {
        for (int q = 0; q < far_rule->n; ++q) {
            v3 y = add(add(scl(t->a[0], far_rule->l[q][0]), scl(t->a[1], far_rule->l[q][1])), scl(t->a[2], far_rule->l[q][2]));
            ip_push(P, y, nrm(sub(x, y)), far_rule->w[q] * t->area);
        }
        return;
    }
    double d = dot(sub(x, t->a[0]), t->n);
    v3 p = sub(x, scl(t->n, d));
    d = fabs(d);
    if (d < 1e-12 * t->rad) d = 0;
    for (int k = 0; k < 3; ++k)
        polar_subtri(P, p, t->n, d, t->a[k], t->a[(k + 1) % 3], 1.0, bps, nbp, nth, nrh);
}

/* ---------------- temporal basis functions (Section V-A/B) ---------------- */
/* u = tau / dt.  Values are returned already divided by dt powers as noted. */
static inline double h0(double u) { double a = fabs(u); return a < 1 ? 1 - a : 0; }
static inline double hd0(double u, double idt) { return (u > -1 && u < 0) ? idt : ((u >= 0 && u < 1) ? -idt : 0); }
static inline double q0(double u) {
    if (u < -1 || u > 2) return 0;
    if (u < 0) return 0.5 * (u + 1) * (u + 1);
    if (u < 1) return 0.5 - u * u + u;
    return 0.5 * (u - 2) * (u - 2);
}
static inline double qd0(double u, double idt) {
    if (u < -1 || u > 2) return 0;
    if (u < 0) return (u + 1) * idt;
    if (u < 1) return (1 - 2 * u) * idt;
    return (u - 2) * idt;
}
static inline double qdd0(double u, double idt2) {
    if (u < -1 || u > 2) return 0;
    if (u < 0) return idt2;
    if (u < 1) return -2 * idt2;
    return idt2;
}
static inline double p0f(double u) { return (u > -1 && u < 0) ? 1 : 0; }

/* ---------------- retarded assembly ---------------- */
typedef struct {
    int nh, nhat, ntil;        /* number of lags per family (max lag + 1) */
    double* Th; double* Kh; double* That; double* Khat; double* Ttil; double* Ktil;
} outblk;

/* moment slots per lag: 0 Th, 1 Kh, 2 That(ff), 3 That(dd), 4 Khat, 5 Ttil, 6 Ktil
   each slot holds M0 and M1[3] */
#define NSLOT 7

int fx_retarded(int nv, const double* verts, int nf, const int32_t* tris, int ne,
                const int32_t* edges, const int32_t* face_order, const int32_t* color_ptr, int ncolor,
                double dt, double c, int nh, int nhat, int ntil, int nq, int nth, int nrh,
                double* Th, double* Kh, double* That, double* Khat, double* Ttil, double* Ktil) {
    (void)nv;
    gl_init();
    trule rule, far_rule;
    if (make_rule(nq, &rule) || make_rule(7, &far_rule)) return -1;
    if (nth < 1 || nth > MAXGL || nrh < 1 || nrh > MAXGL) return -2;
    int nlag = nh; if (nhat > nlag) nlag = nhat; if (ntil > nlag) nlag = ntil;
    /* shell radii c dt k for k = 0 .. nlag + 2 */
    int nbp = nlag + 3;
    double* bps = (double*)malloc(sizeof(double) * nbp);
    for (int k = 0; k < nbp; ++k) bps[k] = c * dt * k;
    tri_t* T = (tri_t*)malloc(sizeof(tri_t) * nf);
    for (int f = 0; f < nf; ++f)
        tri_make(&T[f], ld(verts + 3 * tris[3 * f]), ld(verts + 3 * tris[3 * f + 1]), ld(verts + 3 * tris[3 * f + 2]));
    /* RWG restrictions per face: edge index, coefficient s/(2A), free vertex */
    int* fe = (int*)malloc(sizeof(int) * 3 * nf);
    double* fcoef = (double*)malloc(sizeof(double) * 3 * nf);
    double* fopp = (double*)malloc(sizeof(double) * 9 * nf);
    int* cnt = (int*)calloc(nf, sizeof(int));
    for (int m = 0; m < ne; ++m) {
        for (int side = 0; side < 2; ++side) {
            int f = edges[4 * m + 2 + side];
            int k = cnt[f]++;
            if (k >= 3) { free(cnt); return -3; }
            int opp = -1;
            for (int j = 0; j < 3; ++j) { int v = tris[3 * f + j]; if (v != edges[4 * m] && v != edges[4 * m + 1]) opp = v; }
            fe[3 * f + k] = m;
            fcoef[3 * f + k] = (side == 0 ? 1.0 : -1.0) / (2 * T[f].area);
            for (int dd = 0; dd < 3; ++dd) fopp[9 * f + 3 * k + dd] = verts[3 * opp + dd];
        }
    }
    free(cnt);
    const double idt = 1.0 / dt, idt2 = idt * idt, ic = 1.0 / c;
    const size_t NN = (size_t)ne * ne;
    double* outs[6] = {Th, Kh, That, Khat, Ttil, Ktil};
    int nls[6] = {nh, nh, nhat, nhat, ntil, ntil};
    for (int b = 0; b < 6; ++b) if (outs[b]) memset(outs[b], 0, sizeof(double) * NN * nls[b]);

    for (int col = 0; col < ncolor; ++col) {
#pragma omp parallel
        {
            ipts P = {0, 0, 0, 0, 0};
            double* acc = (double*)malloc(sizeof(double) * (nlag + 4) * NSLOT * 4);
            double* tail = (double*)malloc(sizeof(double) * (nlag + 4) * 4);
            /* per-pair local blocks loc[blk][lag][3][3] */
            double* loc = (double*)malloc(sizeof(double) * 6 * nlag * 9);
#pragma omp for schedule(dynamic, 1)
            for (int ii = color_ptr[col]; ii < color_ptr[col + 1]; ++ii) {
                int s = face_order[ii];
                const tri_t* S = &T[s];
                for (int t = 0; t < nf; ++t) {
                    const tri_t* Tt = &T[t];
                    int near = (s == t);
                    if (!near) {
                        for (int a = 0; a < 3 && !near; ++a)
                            for (int b = 0; b < 3; ++b) if (tris[3 * s + a] == tris[3 * t + b]) { near = 1; break; }
                        if (nrm(sub(S->c, Tt->c)) < 2.0 * (S->rad + Tt->rad)) near = 1;
                    }
                    /* causality: the pair interacts at lag i only if R_min < c dt (i+1) */
                    double Rpair = nrm(sub(S->c, Tt->c)) - S->rad - Tt->rad;
                    if (Rpair > c * dt * (nlag + 1)) continue;
                    memset(loc, 0, sizeof(double) * 6 * nlag * 9);
                    int lag_hi = -1;
                    for (int q = 0; q < rule.n; ++q) {
                        v3 x = add(add(scl(S->a[0], rule.l[q][0]), scl(S->a[1], rule.l[q][1])), scl(S->a[2], rule.l[q][2]));
                        double wx = rule.w[q] * S->area;
                        double dc = nrm(sub(x, Tt->c));
                        double Rmin = fmax(0, dc - Tt->rad), Rmax = dc + Tt->rad;
                        int ilo = (int)floor(Rmin * ic * idt) - 1; if (ilo < 0) ilo = 0;
                        int ihi = (int)ceil(Rmax * ic * idt) + 2; if (ihi > nlag + 2) ihi = nlag + 2;
                        if (ilo > nlag - 1) continue;
                        inner_points(&P, x, Tt, bps, nbp, near, &far_rule, nth, nrh);
                        memset(acc + (size_t)ilo * NSLOT * 4, 0, sizeof(double) * (ihi - ilo + 1) * NSLOT * 4);
                        memset(tail, 0, sizeof(double) * (nlag + 4) * 4);
                        for (int k = 0; k < P.n; ++k) {
                            double R = P.R[k], w = P.w[k];
                            const double* y = P.y + 3 * k;
                            double xi = R * ic * idt;     /* R / (c dt) */
                            double iR = 1.0 / R, gR = iR / FOUR_PI;
                            int i0 = (int)floor(xi);
                            int ia = i0 - 1 < 0 ? 0 : i0 - 1, ib = i0 + 2 > nlag - 1 ? nlag - 1 : i0 + 2;
                            for (int i = ia; i <= ib; ++i) {
                                double u = i - xi;
                                double* A = acc + (size_t)i * NSLOT * 4;
                                double v;
                                /* 0: Th */
                                v = -ic * hd0(u, idt) * gR * w;
                                A[0] += v; A[1] += v * y[0]; A[2] += v * y[1]; A[3] += v * y[2];
                                /* 1: Kh, Psi = -[hdot/(cR) + h/R^2] g */
                                v = -(hd0(u, idt) * ic * iR + h0(u) * iR * iR) * gR * w;
                                A[4] += v; A[5] += v * y[0]; A[6] += v * y[1]; A[7] += v * y[2];
                                /* 2: That ff */
                                v = -ic * qdd0(u, idt2) * gR * w;
                                A[8] += v; A[9] += v * y[0]; A[10] += v * y[1]; A[11] += v * y[2];
                                /* 3: That dd (scalar only) */
                                A[12] += -c * q0(u) * gR * w;
                                /* 4: Khat */
                                v = -(qdd0(u, idt2) * ic * iR + qd0(u, idt) * iR * iR) * gR * w;
                                A[16] += v; A[17] += v * y[0]; A[18] += v * y[1]; A[19] += v * y[2];
                                /* 5: Ttil */
                                v = -ic * p0f(u) * gR * w;
                                A[20] += v; A[21] += v * y[0]; A[22] += v * y[1]; A[23] += v * y[2];
                                /* 6: Ktil, part with tau in (-dt, 0]: p0 = 1, P = tau + dt */
                                if (u > -1 && u <= 0) {
                                    v = -(ic * iR + (u + 1) * dt * iR * iR) * gR * w;
                                    A[24] += v; A[25] += v * y[0]; A[26] += v * y[1]; A[27] += v * y[2];
                                }
                            }
                            /* Ktil constant tail: P = dt, p0 = 0 for every lag i > xi */
                            int it = i0 + 1;
                            if (it < nlag + 3) {
                                double v = -(dt * iR * iR) * gR * w;
                                double* tl = tail + 4 * it;
                                tl[0] += v; tl[1] += v * y[0]; tl[2] += v * y[1]; tl[3] += v * y[2];
                            }
                        }
                        int imax = ihi > nlag - 1 ? nlag - 1 : ihi;
                        if (ntil - 1 > imax) imax = ntil - 1;
                        if (imax > lag_hi) lag_hi = imax;
                        for (int a = 0; a < 3; ++a) {
                            double cm = fcoef[3 * s + a];
                            v3 xm = sub(x, ld(fopp + 9 * s + 3 * a));
                            for (int b = 0; b < 3; ++b) {
                                double cn = fcoef[3 * t + b];
                                v3 Pn = ld(fopp + 9 * t + 3 * b);
                                v3 xn = sub(x, Pn);
                                double cc = cm * cn * wx;
                                int ab = 3 * a + b;
                                double run0 = 0; v3 run1 = mk(0, 0, 0);
                                for (int i = 0; i <= imax; ++i) {
                                    const double* tl = tail + 4 * i;
                                    run0 += tl[0]; run1 = add(run1, mk(tl[1], tl[2], tl[3]));
                                    int inwin = (i >= ilo && i <= ihi);
                                    const double* A = acc + (size_t)i * NSLOT * 4;
                                    double* L = loc + (size_t)i * 9 + ab;
                                    const size_t BS = (size_t)nlag * 9;
                                    if (inwin && i < nh) {
                                        L[0 * BS] += cc * dot(xm, sub(mk(A[1], A[2], A[3]), scl(Pn, A[0])));
                                        L[1 * BS] += cc * dot(xm, crs(xn, sub(mk(A[5], A[6], A[7]), scl(Pn, A[4]))));
                                    }
                                    if (inwin && i < nhat) {
                                        double vff = dot(xm, sub(mk(A[9], A[10], A[11]), scl(Pn, A[8])));
                                        L[2 * BS] += cc * (vff + 4.0 * A[12]);
                                        L[3 * BS] += cc * dot(xm, crs(xn, sub(mk(A[17], A[18], A[19]), scl(Pn, A[16]))));
                                    }
                                    if (i < ntil) {
                                        double m0 = run0; v3 m1 = run1;
                                        if (inwin) {
                                            L[4 * BS] += cc * dot(xm, sub(mk(A[21], A[22], A[23]), scl(Pn, A[20])));
                                            m0 += A[24]; m1 = add(m1, mk(A[25], A[26], A[27]));
                                        }
                                        L[5 * BS] += cc * dot(xm, crs(xn, sub(m1, scl(Pn, m0))));
                                    }
                                }
                            }
                        }
                    }
                    /* write the pair's local blocks: rows are RWGs of s */
                    for (int blk = 0; blk < 6; ++blk) {
                        double* O = outs[blk];
                        if (!O) continue;
                        int nl = nls[blk] - 1 < lag_hi ? nls[blk] - 1 : lag_hi;
                        for (int i = 0; i <= nl; ++i) {
                            const double* L = loc + ((size_t)blk * nlag + i) * 9;
                            for (int a = 0; a < 3; ++a) {
                                double* row = O + (size_t)i * NN + (size_t)fe[3 * s + a] * ne;
                                for (int b = 0; b < 3; ++b) row[fe[3 * t + b]] += L[3 * a + b];
                            }
                        }
                    }
                }
            }
            free(P.y); free(P.R); free(P.w); free(acc); free(tail); free(loc);
        }
    }
    free(bps); free(T); free(fe); free(fcoef); free(fopp);
    return 0;
}

/* ---------------- static BC blocks ---------------- */
/* fine mesh: nft triangles fv[nft][3][3];  BC restrictions in CSR by fine
 * triangle: rowptr[nft+1], bcn[], bca[], bcb[][3] (g_n|_t = a x - b).
 * T0s (ne x ne) and T0h (ne x ne) are written; order = fine triangles
 * grouped by BC support for stage 2: by_n_ptr[ne+1], by_n_t[], by_n_k[]
 * (index into the restriction arrays). */
int fx_static_bc(int nft, const double* fv, const int32_t* rowptr, const int32_t* bcn,
                 const double* bca, const double* bcb, int ne, const int32_t* by_n_ptr,
                 const int32_t* by_n_k, double D, int nq, int nth, int nrh, int chunk,
                 double* T0s, double* T0h) {
    gl_init();
    trule rule, far_rule;
    if (make_rule(nq, &rule) || make_rule(3, &far_rule)) return -1;
    tri_t* T = (tri_t*)malloc(sizeof(tri_t) * nft);
    for (int t = 0; t < nft; ++t) tri_make(&T[t], ld(fv + 9 * t), ld(fv + 9 * t + 3), ld(fv + 9 * t + 6));
    memset(T0s, 0, sizeof(double) * (size_t)ne * ne);
    memset(T0h, 0, sizeof(double) * (size_t)ne * ne);
    if (chunk <= 0) chunk = 1024;
    /* stage-1 buffer W[s - s0][n][13]: 12 for T0s (3 comps x 4), 1 for T0h */
    double* W = (double*)malloc(sizeof(double) * (size_t)chunk * ne * 13);
    int* srow = (int*)malloc(sizeof(int) * nft);   /* position of s inside the chunk or -1 */
    for (int s0 = 0; s0 < nft; s0 += chunk) {
        int s1 = s0 + chunk < nft ? s0 + chunk : nft;
        memset(W, 0, sizeof(double) * (size_t)(s1 - s0) * ne * 13);
#pragma omp parallel
        {
            ipts P = {0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 4)
            for (int s = s0; s < s1; ++s) {
                const tri_t* S = &T[s];
                double* Ws = W + (size_t)(s - s0) * ne * 13;
                for (int t = 0; t < nft; ++t) {
                    const tri_t* Tt = &T[t];
                    int near = (s == t) || nrm(sub(S->c, Tt->c)) < 3.0 * (S->rad + Tt->rad);
                    /* M[i][j] = int_s int_t X_i Y_j / (4 pi R), X = (x,1), Y = (y,1) */
                    double M[4][4];
                    memset(M, 0, sizeof(M));
                    const trule* ro = near ? &rule : &far_rule;
                    for (int q = 0; q < ro->n; ++q) {
                        v3 x = add(add(scl(S->a[0], ro->l[q][0]), scl(S->a[1], ro->l[q][1])), scl(S->a[2], ro->l[q][2]));
                        double wx = ro->w[q] * S->area;
                        double m0 = 0, m1x = 0, m1y = 0, m1z = 0;
                        if (near) {
                            inner_points(&P, x, Tt, NULL, 0, 1, &far_rule, nth, nrh);
                        } else {
                            P.n = 0;
                            for (int k = 0; k < far_rule.n; ++k) {
                                v3 y = add(add(scl(Tt->a[0], far_rule.l[k][0]), scl(Tt->a[1], far_rule.l[k][1])), scl(Tt->a[2], far_rule.l[k][2]));
                                ip_push(&P, y, nrm(sub(x, y)), far_rule.w[k] * Tt->area);
                            }
                        }
                        for (int k = 0; k < P.n; ++k) {
                            double v = P.w[k] / (FOUR_PI * P.R[k]);
                            m0 += v; m1x += v * P.y[3 * k]; m1y += v * P.y[3 * k + 1]; m1z += v * P.y[3 * k + 2];
                        }
                        double X[4] = {x.x, x.y, x.z, 1};
                        double Y[4] = {m1x, m1y, m1z, m0};
                        for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) M[i][j] += wx * X[i] * Y[j];
                    }
                    /* W[s][n] += M c_{n,d}(t) for each BC n with t in its support */
                    for (int k = rowptr[t]; k < rowptr[t + 1]; ++k) {
                        int n = bcn[k];
                        double a = bca[k];
                        const double* b = bcb + 3 * k;
                        double* w = Ws + (size_t)n * 13;
                        for (int dd = 0; dd < 3; ++dd) {
                            /* c_{n,d} = (a e_d, -b_d) */
                            for (int i = 0; i < 4; ++i) w[4 * dd + i] += a * M[i][dd] - b[dd] * M[i][3];
                        }
                        w[12] += 2.0 * a * M[3][3];
                    }
                }
            }
            free(P.y); free(P.R); free(P.w);
        }
        for (int s = 0; s < nft; ++s) srow[s] = (s >= s0 && s < s1) ? s - s0 : -1;
#pragma omp parallel for schedule(dynamic, 8)
        for (int m = 0; m < ne; ++m) {
            for (int kk = by_n_ptr[m]; kk < by_n_ptr[m + 1]; ++kk) {
                int k = by_n_k[kk];
                /* find the fine triangle of restriction k */
                int t = -1;
                { int lo = 0, hi = nft; while (hi - lo > 1) { int mid = (lo + hi) / 2; if (rowptr[mid] <= k) lo = mid; else hi = mid; } t = lo; }
                if (srow[t] < 0) continue;
                double a = bca[k];
                const double* b = bcb + 3 * k;
                const double* Wt = W + (size_t)srow[t] * ne * 13;
                double* rs = T0s + (size_t)m * ne;
                double* rh = T0h + (size_t)m * ne;
                for (int n = 0; n < ne; ++n) {
                    const double* w = Wt + (size_t)n * 13;
                    double v = 0;
                    for (int dd = 0; dd < 3; ++dd) {
                        const double* wd = w + 4 * dd;
                        v += a * wd[dd] - b[dd] * wd[3];
                    }
                    rs[n] += v / D;
                    rh[n] += D * 2.0 * a * w[12];
                }
            }
        }
    }
    free(W); free(srow); free(T);
    return 0;
}

/* plain rule export for tests of the quadrature tables */
int fx_rule(int nq, double* l, double* w) {
    trule r;
    if (make_rule(nq, &r)) return -1;
    for (int i = 0; i < r.n; ++i) { l[3 * i] = r.l[i][0]; l[3 * i + 1] = r.l[i][1]; l[3 * i + 2] = r.l[i][2]; w[i] = r.w[i]; }
    return r.n;
}

/* generic inner integral for tests: int_t y^k F(R) dy via the same point sets,
 * returns sum w, sum w/R, sum w/R^3 moments at x */
int fx_inner_test(const double* x, const double* tv, const double* bps, int nbp, int near,
                  int nth, int nrh, double* out) {
    gl_init();
    trule far_rule; make_rule(7, &far_rule);
    tri_t t; tri_make(&t, ld(tv), ld(tv + 3), ld(tv + 6));
    ipts P = {0, 0, 0, 0, 0};
    inner_points(&P, ld(x), &t, bps, nbp, near, &far_rule, nth, nrh);
    double s0 = 0, s1 = 0, s3 = 0;
    for (int k = 0; k < P.n; ++k) { s0 += P.w[k]; s1 += P.w[k] / P.R[k]; s3 += P.w[k] / (P.R[k] * P.R[k] * P.R[k]); }
    out[0] = s0; out[1] = s1; out[2] = s3; out[3] = P.n;
    free(P.y); free(P.R); free(P.w);
    return 0;
}

/* temporal basis values at u = tau/dt: h0, hdot0, q0, qdot0, qddot0, p0, P (test hook) */
int fx_temporal(double u, double dt, double* out) {
    double idt = 1.0 / dt;
    out[0] = h0(u); out[1] = hd0(u, idt); out[2] = q0(u); out[3] = qd0(u, idt);
    out[4] = qdd0(u, idt * idt); out[5] = p0f(u);
    out[6] = u <= -1 ? 0 : (u <= 0 ? (u + 1) * dt : dt);
    return 0;
}

/* Gauss-Legendre tables on [0, 1] (nodes, weights) as [MAXGL + 1][MAXGL], row n
 * holding the n-point rule: shared with the device assembler so that both
 * build the same point sets. */
int fx_gl_tables(double* x, double* w) {
    gl_init();
    for (int n = 0; n <= MAXGL; ++n)
        for (int i = 0; i < MAXGL; ++i) {
            x[n * MAXGL + i] = gl_x[n][i];
            w[n * MAXGL + i] = gl_w[n][i];
        }
    return MAXGL;
}
