/*
 * Device-side Galerkin assembly of the inputs of the qHP TD-PMCHWT marching
 * scheme (input generator, not part of the solver): the retarded h / hat /
 * tilde families of Section V-B for one medium, one lag at a time, and the
 * static blocks T0s, T0h of Section III on the Buffa-Christiansen basis.
 *
 * The quadrature is the one of the host assembler in assemble.c, point for
 * point: an N_q-point rule on the test triangle; on the source triangle a
 * polar rule about the projection of the test point, split at every retarded
 * shell radius c dt k (angular variable asinh(tan theta), radial variable
 * asinh(rho/d)), or the 7-point rule when the test point is far and its
 * distance range meets no shell.  The Gauss-Legendre and triangle-rule tables
 * come from the host assembler, so both produce the same point sets; only the
 * order of the sums differs.
 *
 * Kernels per lag i and medium (wave speed c, tau = i dt - R/c, g = 1/(4 pi R)):
 *   T_i  = -(1/c) <f_m, f_n hdot0(tau) g>       K_i  = <f_m, grad_x[h0 g] x f_n>
 *   That = -(1/c) <f_m, f_n qddot0 g> - c <div f_m, div f_n q0 g>
 *   Khat = <f_m, grad_x[qdot0 g] x f_n>
 *   Ttil = -(1/c) <f_m, f_n p0 g>                Ktil = <f_m, grad_x[P g] x f_n>, P = int p0
 * without the T_max factors (the solver applies them), symmetrised as
 * (X + X^T)/2 like the host blocks.
 *
 * Work layout.  One launch per lag, per pair of face colours (faces of one
 * colour share no edge), so that within a launch every entry (m, n) of a
 * block receives at most one triangle-pair contribution: plain read-add-write,
 * and a fixed summation order.  Work goes by shell band: band k holds the
 * source points with k c dt <= R < (k + 1) c dt, which add to lags k, k + 1,
 * k + 2 (the temporal basis spans two steps) and to the tilde-K tail of every
 * later lag, so each point is evaluated once.  A compaction pass lists the
 * pairs with points in the band; their (pair, test point) items are sorted
 * into far-rule and polar lists, so that the lanes of a walk launch do work
 * of one kind; one lane walks one item's points of the band (whole polar
 * pieces outside it are passed over: the rule is split at the shells) and
 * stores its moments; a last pass, one thread per (pair, output channel, RWG
 * pair), sums the products over the pair's test points in order and adds the
 * entry.
 *
 * Lags are produced in increasing order into a ring of three: after band k,
 * lag k is complete.  The tilde-K tail of band k goes to the lags in flight
 * (k + 1, k + 2) and to a running accumulator that seeds the tilde K block of
 * every lag started later.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gpu_quad.h"

namespace {

/* Quadrature tables of one assembler (or one static-block build), in device
 * memory of its own: concurrent builds with different rules (the static blocks
 * use a 6-point test rule and a 3-point far rule, the retarded blocks 7 and 7)
 * never see each other's tables. */
struct QTables {
    double glx[(MAXGL + 1) * MAXGL];
    double glw[(MAXGL + 1) * MAXGL];
    double rule[16 * 4];             /* test rule: l0 l1 l2 w */
    double far[16 * 4];              /* far source rule */
};

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

struct RetParams {
    const double* tri;      /* [nf][16] */
    const int* fe;          /* [nf][3] edge index of the RWG on each face side */
    const double* fcoef;    /* [nf][3] +-1/(2A) */
    const double* fopp;     /* [nf][3][3] free vertex */
    const int32_t* tris;    /* [nf][3] vertex indices (adjacency test) */
    const int* slist;       /* test faces of the colour */
    const int* tlist;       /* source faces of the colour */
    int ns, ntl;
    int ne, nlag, nh, nhat, ntil, nq, nth, nrh;
    int band;
    double dt, c;
    double* ring[18];       /* [slot = lag % 3][Th Kh That Khat Ttil Ktil], [ne][ne] each */
    double* acc_tail;       /* running tilde-K tail, [ne][ne] */
    int2* plist;            /* active pairs of this colour pair (s, t) */
    int* pcount;
    int p0, nb;             /* batch: pairs p0 .. p0 + nb - 1 of the list */
    double* mom;            /* [nb * nq][MOMW] band moments of each (pair, test point) */
    int* items;             /* [2][nb * nq] far-rule items, then polar items */
    int* icount;            /* [2] */
    const QTables* qt;      /* quadrature tables */
};

constexpr int MOMW = 56;    /* doubles per item: the BM_N band moments and padding */
constexpr int NCH = 13;     /* output channels of a band pass (band_channel) */

__device__ __forceinline__ Tab dev_tab(const QTables* q) {
    Tab T;
    T.glx = q->glx; T.glw = q->glw; T.rule = q->rule; T.far = q->far;
    return T;
}

__device__ __forceinline__ int family_limit(const RetParams& P, int blk) {
    return blk < 2 ? P.nh : (blk < 4 ? P.nhat : P.ntil);
}

/* Pairs of one colour pair with source points in band k, appended in any
 * order: each pair writes entries no other pair of the launch writes, so the
 * order of the list does not change any sum. */
__global__ void k_pairs(RetParams P) {
    const long pair = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= (long)P.ns * P.ntl) return;
    const int s = P.slist[pair / P.ntl], t = P.tlist[pair % P.ntl];
    const Tri S = load_tri(P.tri, s), Tt = load_tri(P.tri, t);
    const PairBands pb = pair_bands(S, Tt, P.tris, s, t, P.c, P.dt, P.nlag);
    if (pb.cull || P.band < pb.blo || P.band > pb.bhi) return;
    const int slot = atomicAdd(P.pcount, 1);
    P.plist[slot] = make_int2(s, t);
}

/* Items (pair, test point) of a batch sorted into a far-rule list and a
 * polar list, so that the lanes of one walk launch do work of one kind; items
 * with no rule, or far-rule items none of whose seven points lies in the
 * band, get zero moments. */
__global__ void k_classify(RetParams P) {
    const long it = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= (long)P.nb * P.nq) return;
    const int pi = (int)(it / P.nq), q = (int)(it % P.nq);
    const int2 st = P.plist[P.p0 + pi];
    const Tri S = load_tri(P.tri, st.x), Tt = load_tri(P.tri, st.y);
    const PairBands pb = pair_bands(S, Tt, P.tris, st.x, st.y, P.c, P.dt, P.nlag);
    const Tab T = dev_tab(P.qt);
    int cls = test_point_class(T, S, Tt, q, pb.near, P.c, P.dt, P.nlag);
    if (cls == 1) {
        const V3 x = add(add(scl(S.a[0], T.rule[4 * q]), scl(S.a[1], T.rule[4 * q + 1])), scl(S.a[2], T.rule[4 * q + 2]));
        const double ic = 1.0 / P.c, idt = 1.0 / P.dt;
        bool any = false;
        for (int k = 0; k < 7; ++k) {
            V3 y = add(add(scl(Tt.a[0], T.far[4 * k]), scl(Tt.a[1], T.far[4 * k + 1])), scl(Tt.a[2], T.far[4 * k + 2]));
            if ((int)floor(nrm(sub(x, y)) * ic * idt) == P.band) any = true;
        }
        if (!any) cls = 0;
    }
    if (cls == 0) {
        double* m = P.mom + it * MOMW;
        for (int j = 0; j < BM_N; ++j) m[j] = 0;
        return;
    }
    const int slot = atomicAdd(P.icount + (cls - 1), 1);
    P.items[(size_t)(cls - 1) * P.nb * P.nq + slot] = (int)it;
}

/* One lane per listed item: the band moments of its test point. */
__global__ void __launch_bounds__(256) k_walk(RetParams P, int cls) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.icount[cls]) return;
    const int it = P.items[(size_t)cls * P.nb * P.nq + k];
    const int pi = it / P.nq, q = it % P.nq;
    const int2 st = P.plist[P.p0 + pi];
    const Tri S = load_tri(P.tri, st.x), Tt = load_tri(P.tri, st.y);
    const PairBands pb = pair_bands(S, Tt, P.tris, st.x, st.y, P.c, P.dt, P.nlag);
    BandMoments M;
    const bool act = test_point_band(dev_tab(P.qt), S, Tt, q, pb.near, P.c, P.dt, P.nlag, P.band, P.nth, P.nrh, M);
    double* m = P.mom + (size_t)it * MOMW;
    if (!act) M.clear();
#pragma unroll
    for (int j = 0; j < BM_N; ++j) m[j] = M.m[j];
}

/* One thread per (pair, channel, RWG pair (a, b)): the sum over the pair's
 * test points, in order, added to the block entry of its lag (and, for the
 * tail channel, to Ktil of lags k + 1, k + 2 and the running accumulator). */
__global__ void k_products(RetParams P) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)P.nb * NCH * 9) return;
    const int pi = (int)(idx / (NCH * 9)), r = (int)(idx % (NCH * 9));
    const int ch = r / 9, ab = r % 9, a = ab / 3, b = ab % 3;
    const Channel C = band_channel(ch);
    const int k = P.band;
    const int lag = k + C.d;
    const bool tail = ch == NCH - 1;
    if (!tail && (lag > P.nlag - 1 || lag >= family_limit(P, C.blk))) return;
    const int2 st = P.plist[P.p0 + pi];
    const int s = st.x, t = st.y;
    const Tri S = load_tri(P.tri, s);
    const Tab T = dev_tab(P.qt);
    const double cm = P.fcoef[3 * s + a], cn = P.fcoef[3 * t + b];
    const double* pa = P.fopp + 9 * s + 3 * a;
    const double* pb = P.fopp + 9 * t + 3 * b;
    const V3 Pm = mk(pa[0], pa[1], pa[2]), Pn = mk(pb[0], pb[1], pb[2]);
    double acc = 0;
    for (int q = 0; q < P.nq; ++q) {
        const double* m = P.mom + ((size_t)pi * P.nq + q) * MOMW;
        const V3 x = add(add(scl(S.a[0], T.rule[4 * q]), scl(S.a[1], T.rule[4 * q + 1])), scl(S.a[2], T.rule[4 * q + 2]));
        const double wx = T.rule[4 * q + 3] * S.area;
        const double dd = C.dd >= 0 ? m[C.dd] : 0.0;
        acc += block_product(C.isK, m[C.mom], mk(m[C.mom + 1], m[C.mom + 2], m[C.mom + 3]), dd, cm, cn, wx,
                             sub(x, Pm), Pn, x);
    }
    const size_t o = (size_t)P.fe[3 * s + a] * P.ne + P.fe[3 * t + b];
    if (!tail) {
        P.ring[(lag % 3) * 6 + C.blk][o] += acc;
        return;
    }
    for (int d = 1; d <= 2; ++d)
        if (k + d <= P.nlag - 1 && k + d < P.ntil) P.ring[((k + d) % 3) * 6 + 5][o] += acc;
    P.acc_tail[o] += acc;
}

/* X <- (X + X^T) / 2, in place, upper-triangle threads */
__global__ void k_symmetrise(double* X, int n) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nn = (long)n * n;
    if (idx >= nn) return;
    int i = (int)(idx / n), j = (int)(idx % n);
    if (j <= i) return;
    double a = X[(size_t)i * n + j], b = X[(size_t)j * n + i];
    double v = 0.5 * (a + b);
    X[(size_t)i * n + j] = v;
    X[(size_t)j * n + i] = v;
}

struct StatParams {
    const double* tri;     /* fine triangles [nft][16] */
    int nft, s0, s1;       /* test chunk [s0, s1) */
    int nq, far_n, nth, nrh;
    double* MB;            /* [s1 - s0][nft][16] */
    int* near_list;        /* [cap][2] */
    int* near_count;
    int near_cap;
    const QTables* qt;     /* quadrature tables */
};

/* far pairs: one lane per pair; near pairs are listed for k_static_near */
__global__ void __launch_bounds__(256) k_static_far(StatParams P) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long np = (long)(P.s1 - P.s0) * P.nft;
    if (idx >= np) return;
    int s = P.s0 + (int)(idx / P.nft), t = (int)(idx % P.nft);
    Tri S = load_tri(P.tri, s), T = load_tri(P.tri, t);
    int near = (s == t) || nrm(sub(S.c, T.c)) < 3.0 * (S.rad + T.rad);
    double* M = P.MB + (size_t)idx * 16;
    if (near) {
        int slot = atomicAdd(P.near_count, 1);
        if (slot < P.near_cap) { P.near_list[2 * slot] = s; P.near_list[2 * slot + 1] = t; }
        return;
    }
    double m[16];
    for (int j = 0; j < 16; ++j) m[j] = 0;
    for (int q = 0; q < P.far_n; ++q) {
        const double* fq = P.qt->far + 4 * q;
        V3 x = add(add(scl(S.a[0], fq[0]), scl(S.a[1], fq[1])), scl(S.a[2], fq[2]));
        double wx = fq[3] * S.area;
        StatMoments A = {0, 0, 0, 0};
        for (int k = 0; k < P.far_n; ++k) {
            const double* fk = P.qt->far + 4 * k;
            V3 y = add(add(scl(T.a[0], fk[0]), scl(T.a[1], fk[1])), scl(T.a[2], fk[2]));
            A(y, nrm(sub(x, y)), fk[3] * T.area);
        }
        double X[4] = {x.x, x.y, x.z, 1};
        double Y[4] = {A.m1x, A.m1y, A.m1z, A.m0};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) m[4 * i + j] += wx * X[i] * Y[j];
    }
    for (int j = 0; j < 16; ++j) M[j] = m[j];
}

/* near pairs: a group of 8 lanes per pair, one lane per test point */
__global__ void __launch_bounds__(256) k_static_near(StatParams P, int count) {
    const int lane = threadIdx.x % 8;
    const long pi = ((long)blockIdx.x * blockDim.x + threadIdx.x) / 8;
    if (pi >= count) return;
    int s = P.near_list[2 * pi], t = P.near_list[2 * pi + 1];
    Tri S = load_tri(P.tri, s), T = load_tri(P.tri, t);
    double m[16];
    for (int j = 0; j < 16; ++j) m[j] = 0;
    if (lane < P.nq) {
        const double* rl = P.qt->rule + 4 * lane;
        V3 x = add(add(scl(S.a[0], rl[0]), scl(S.a[1], rl[1])), scl(S.a[2], rl[2]));
        double wx = rl[3] * S.area;
        StatMoments A = {0, 0, 0, 0};
        const Tab TB = dev_tab(P.qt);
        inner_points(TB, A, x, T, 0.0, 0, 1, P.far_n, P.nth, P.nrh);
        double X[4] = {x.x, x.y, x.z, 1};
        double Y[4] = {A.m1x, A.m1y, A.m1z, A.m0};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) m[4 * i + j] = wx * X[i] * Y[j];
    }
    for (int j = 0; j < 16; ++j) m[j] = group_sum<8>(m[j]);
    if (lane == 0) {
        double* M = P.MB + ((size_t)(s - P.s0) * P.nft + t) * 16;
        for (int j = 0; j < 16; ++j) M[j] = m[j];
    }
}

/* W[s][n][13] = sum over the restrictions k of BC n (on fine triangle t_k):
 *   W[4d + i] = a M[i][d] - b_d M[i][3] (d < 3),  W[12] = 2 a M[3][3]. */
__global__ void k_static_w(const double* MB, int nft, int s0, int s1, int ne, const int* byn_ptr,
                           const int* byn_k, const int* res_t, const double* res_a, const double* res_b,
                           double* W) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)(s1 - s0) * ne) return;
    int sl = (int)(idx / ne), n = (int)(idx % ne);
    double w[13];
    for (int j = 0; j < 13; ++j) w[j] = 0;
    for (int kk = byn_ptr[n]; kk < byn_ptr[n + 1]; ++kk) {
        int k = byn_k[kk];
        int t = res_t[k];
        const double* M = MB + ((size_t)sl * nft + t) * 16;
        double a = res_a[k];
        const double* b = res_b + 3 * k;
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < 4; ++i) w[4 * d + i] += a * M[4 * i + d] - b[d] * M[4 * i + 3];
        w[12] += 2.0 * a * M[15];
    }
    double* o = W + idx * 13;
    for (int j = 0; j < 13; ++j) o[j] = w[j];
}

/* T0s[m][n] += sum over restrictions k of m on test triangles of the chunk:
 *   (a W[4d + d] - b_d W[4d + 3]) / D;   T0h[m][n] += D 2 a W[12]. */
__global__ void k_static_t(const double* W, int s0, int ne, const int* rows, const int* row_ptr,
                           const int* row_k, int nrows, const int* res_t, const double* res_a,
                           const double* res_b, double D, double* T0s, double* T0h) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nrows * ne) return;
    int r = (int)(idx / ne), n = (int)(idx % ne);
    int m = rows[r];
    double vs = 0, vh = 0;
    for (int kk = row_ptr[r]; kk < row_ptr[r + 1]; ++kk) {
        int k = row_k[kk];
        int t = res_t[k];
        double a = res_a[k];
        const double* b = res_b + 3 * k;
        const double* w = W + ((size_t)(t - s0) * ne + n) * 13;
        double v = 0;
        for (int d = 0; d < 3; ++d) v += a * w[4 * d + d] - b[d] * w[4 * d + 3];
        vs += v / D;
        vh += D * 2.0 * a * w[12];
    }
    T0s[(size_t)m * ne + n] += vs;
    T0h[(size_t)m * ne + n] += vh;
}

}  // namespace

/* ================================================================ C ABI === */
extern "C" {

typedef struct gfx_ret {
    int nf, ne, nlag, nh, nhat, ntil, nq, nth, nrh, ncolor;
    double dt, c;
    double* tri; int* fe; double* fcoef; double* fopp; int32_t* tris;
    int* order; int* cptr_h;     /* colour lists: device order, host pointers */
    double* acc_tail;
    int2* plist;                 /* active pairs of one colour pair, [max ns * nt] */
    int* pcount;
    int batch;                   /* pairs per batch of the item buffers */
    double* mom;                 /* [batch * nq][MOMW] */
    int* items;                  /* [2][batch * nq] */
    int* icount;                 /* [2] */
    QTables* qt;                 /* quadrature tables of this assembler */
    int next_lag;
    hipStream_t stream;
} gfx_ret;

/* A device copy of the tables (allocated here, freed by the caller). */
static int make_tables(const double* glx, const double* glw, const double* rule, int nrule, const double* far,
                       int nfar, QTables** out) {
    *out = nullptr;
    if (nrule > 16 || nfar > 16) return -1;
    QTables h;
    memset(&h, 0, sizeof(h));
    memcpy(h.glx, glx, sizeof(h.glx));
    memcpy(h.glw, glw, sizeof(h.glw));
    for (int i = 0; i < 4 * nrule; ++i) h.rule[i] = rule[i];
    for (int i = 0; i < 4 * nfar; ++i) h.far[i] = far[i];
    QTables* d = nullptr;
    if (hipMalloc(&d, sizeof(QTables)) != hipSuccess) return -2;
    if (hipMemcpy(d, &h, sizeof(QTables), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(d);
        return -2;
    }
    *out = d;
    return 0;
}

static void tri_record(const double* a, const double* b, const double* c, double* o) {
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double l = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double il = 1.0 / l;
    for (int k = 0; k < 3; ++k) { o[k] = a[k]; o[3 + k] = b[k]; o[6 + k] = c[k]; o[9 + k] = cr[k] * il; }
    o[12] = 0.5 * l;
    double cen[3];
    for (int k = 0; k < 3; ++k) cen[k] = ((a[k] + b[k]) + c[k]) * (1.0 / 3);
    double r = 0;
    const double* P[3] = {a, b, c};
    for (int j = 0; j < 3; ++j) {
        double dx = P[j][0] - cen[0], dy = P[j][1] - cen[1], dz = P[j][2] - cen[2];
        double dd = sqrt(dx * dx + dy * dy + dz * dz);
        if (dd > r) r = dd;
    }
    o[13] = r;
    o[14] = o[15] = 0;
}

#define GCHK(x) do { if ((x) != hipSuccess) { rc = -2; goto fail; } } while (0)

/* Context for the retarded blocks of one medium (wave speed c): mesh, RWG
 * data and face colouring are copied to the device.  glx/glw: Gauss-Legendre
 * tables [13][12]; rule: test rule [nq][4] (barycentric, weight); far: the
 * 7-point source rule [7][4].  face_order / color_ptr: faces grouped by a
 * colouring of the face graph.  Returns 0 or a negative code. */
int gfx_ret_create(int nv, const double* verts, int nf, const int32_t* tris, int ne, const int32_t* edges,
                   const int32_t* face_order, const int32_t* color_ptr, int ncolor, double dt, double c, int nh,
                   int nhat, int ntil, int nq, int nth, int nrh, const double* glx, const double* glw,
                   const double* rule, const double* far, void* stream, gfx_ret** out) {
    (void)nv;
    int rc = 0;
    if (!out || nq < 1 || nq > 16 || nth < 1 || nth > MAXGL || nrh < 1 || nrh > MAXGL) return -1;
    int nlag = nh > nhat ? nh : nhat;
    if (ntil > nlag) nlag = ntil;
    if (nlag + 3 > 90) return -1;   /* the cut lists of the host rule stay within their caps */
    gfx_ret* g = (gfx_ret*)calloc(1, sizeof(gfx_ret));
    g->nf = nf; g->ne = ne; g->nlag = nlag; g->nh = nh; g->nhat = nhat; g->ntil = ntil;
    g->nq = nq; g->nth = nth; g->nrh = nrh; g->ncolor = ncolor; g->dt = dt; g->c = c;
    g->stream = (hipStream_t)stream;
    double* T = (double*)malloc(sizeof(double) * 16 * (size_t)nf);
    int* fe = (int*)malloc(sizeof(int) * 3 * (size_t)nf);
    double* fcoef = (double*)malloc(sizeof(double) * 3 * (size_t)nf);
    double* fopp = (double*)malloc(sizeof(double) * 9 * (size_t)nf);
    int* cnt = (int*)calloc(nf, sizeof(int));
    for (int f = 0; f < nf; ++f)
        tri_record(verts + 3 * tris[3 * f], verts + 3 * tris[3 * f + 1], verts + 3 * tris[3 * f + 2], T + 16 * f);
    for (int m = 0; m < ne && rc == 0; ++m) {
        for (int side = 0; side < 2; ++side) {
            int f = edges[4 * m + 2 + side];
            int k = cnt[f]++;
            if (k >= 3) { rc = -3; break; }
            int opp = -1;
            for (int j = 0; j < 3; ++j) {
                int v = tris[3 * f + j];
                if (v != edges[4 * m] && v != edges[4 * m + 1]) opp = v;
            }
            fe[3 * f + k] = m;
            fcoef[3 * f + k] = (side == 0 ? 1.0 : -1.0) / (2 * T[16 * f + 12]);
            for (int dd = 0; dd < 3; ++dd) fopp[9 * f + 3 * k + dd] = verts[3 * opp + dd];
        }
    }
    /* every face must carry exactly three RWG sides (closed mesh): the write
     * indices of the kernels come from fe */
    for (int f = 0; f < nf && rc == 0; ++f)
        if (cnt[f] != 3) rc = -3;
    for (int f = 0; f < nf && rc == 0; ++f)
        for (int k = 0; k < 3; ++k)
            if (fe[3 * f + k] < 0 || fe[3 * f + k] >= ne) rc = -3;
    if (ncolor < 1 || color_ptr[0] != 0 || color_ptr[ncolor] != nf) rc = -1;
    for (int cix = 0; cix < ncolor && rc == 0; ++cix)
        if (color_ptr[cix + 1] < color_ptr[cix]) rc = -1;
    for (int f = 0; f < nf && rc == 0; ++f)
        if (face_order[f] < 0 || face_order[f] >= nf) rc = -1;
    free(cnt);
    if (rc == 0) rc = make_tables(glx, glw, rule, nq, far, 7, &g->qt);
    if (rc == 0) {
        GCHK(hipMalloc(&g->tri, sizeof(double) * 16 * (size_t)nf));
        GCHK(hipMalloc(&g->fe, sizeof(int) * 3 * (size_t)nf));
        GCHK(hipMalloc(&g->fcoef, sizeof(double) * 3 * (size_t)nf));
        GCHK(hipMalloc(&g->fopp, sizeof(double) * 9 * (size_t)nf));
        GCHK(hipMalloc(&g->tris, sizeof(int32_t) * 3 * (size_t)nf));
        GCHK(hipMalloc(&g->order, sizeof(int) * (size_t)nf));
        GCHK(hipMalloc(&g->acc_tail, sizeof(double) * (size_t)ne * ne));
        {
            long mx = 0;
            for (int a = 0; a < ncolor; ++a)
                for (int b = 0; b < ncolor; ++b) {
                    long np = (long)(color_ptr[a + 1] - color_ptr[a]) * (color_ptr[b + 1] - color_ptr[b]);
                    if (np > mx) mx = np;
                }
            GCHK(hipMalloc(&g->plist, sizeof(int2) * (size_t)(mx > 0 ? mx : 1)));
            GCHK(hipMalloc(&g->pcount, sizeof(int)));
            /* item buffers of about 1 GiB of moments */
            long b = (1L << 30) / ((long)nq * MOMW * sizeof(double));
            if (b > mx) b = mx > 0 ? mx : 1;
            g->batch = (int)b;
            GCHK(hipMalloc(&g->mom, sizeof(double) * MOMW * (size_t)b * nq));
            GCHK(hipMalloc(&g->items, sizeof(int) * 2 * (size_t)b * nq));
            GCHK(hipMalloc(&g->icount, 2 * sizeof(int)));
        }
        GCHK(hipMemcpy(g->tri, T, sizeof(double) * 16 * (size_t)nf, hipMemcpyHostToDevice));
        GCHK(hipMemcpy(g->fe, fe, sizeof(int) * 3 * (size_t)nf, hipMemcpyHostToDevice));
        GCHK(hipMemcpy(g->fcoef, fcoef, sizeof(double) * 3 * (size_t)nf, hipMemcpyHostToDevice));
        GCHK(hipMemcpy(g->fopp, fopp, sizeof(double) * 9 * (size_t)nf, hipMemcpyHostToDevice));
        GCHK(hipMemcpy(g->tris, tris, sizeof(int32_t) * 3 * (size_t)nf, hipMemcpyHostToDevice));
        GCHK(hipMemcpy(g->order, face_order, sizeof(int) * (size_t)nf, hipMemcpyHostToDevice));
        GCHK(hipMemset(g->acc_tail, 0, sizeof(double) * (size_t)ne * ne));
        g->cptr_h = (int*)malloc(sizeof(int) * (ncolor + 1));
        memcpy(g->cptr_h, color_ptr, sizeof(int) * (ncolor + 1));
    }
fail:
    free(T); free(fe); free(fcoef); free(fopp);
    if (rc) {
        hipFree(g->tri); hipFree(g->fe); hipFree(g->fcoef); hipFree(g->fopp); hipFree(g->tris);
        hipFree(g->order); hipFree(g->acc_tail); hipFree(g->plist); hipFree(g->pcount);
        hipFree(g->mom); hipFree(g->items); hipFree(g->icount); hipFree(g->qt); free(g->cptr_h); free(g);
        return rc;
    }
    *out = g;
    return 0;
}

/* Blocks of lag 'lag', the next in order (0, 1, 2, ...), in a ring of three
 * lags the caller owns: ring[slot * 6 + b], slot = lag % 3, b = Th, Kh, That,
 * Khat, Ttil, Ktil, each a device [ne][ne] row-major array (all 18 given on
 * every call).  The call processes shell band 'lag', whose points add to lags
 * lag .. lag + 2; on return lag 'lag' is complete and symmetrised in its slot
 * (blocks outside their family's range: Th, Kh for lag >= nh, That, Khat for
 * lag >= nhat, Ttil, Ktil for lag >= ntil, are left unwritten), and stays
 * valid until the next call, which starts lag + 3 in the same slot.
 * Enqueued on the context's stream; returns 0, -1 for a lag out of order or
 * a null pointer, -2 on a HIP error. */
int gfx_ret_lag(gfx_ret* g, int lag, double* const* ring) {
    if (!g || !ring || lag != g->next_lag || lag >= g->nlag) return -1;
    for (int j = 0; j < 18; ++j)
        if (!ring[j]) return -1;
    const int lim[6] = {g->nh, g->nh, g->nhat, g->nhat, g->ntil, g->ntil};
    const size_t nn = (size_t)g->ne * g->ne;
    /* start the lags this band adds to but none before it did: 0, 1, 2 at
     * band 0, else lag + 2; Ktil starts from the tail of the bands below */
    for (int l = lag == 0 ? 0 : lag + 2; l <= lag + 2 && l < g->nlag; ++l) {
        const int slot = l % 3;
        for (int b = 0; b < 6; ++b) {
            if (l >= lim[b]) continue;
            hipError_t e = b == 5 ? hipMemcpyAsync(ring[slot * 6 + b], g->acc_tail, nn * sizeof(double),
                                                   hipMemcpyDeviceToDevice, g->stream)
                                  : hipMemsetAsync(ring[slot * 6 + b], 0, nn * sizeof(double), g->stream);
            if (e != hipSuccess) return -2;
        }
    }
    RetParams P;
    P.tri = g->tri; P.fe = g->fe; P.fcoef = g->fcoef; P.fopp = g->fopp; P.tris = g->tris;
    P.ne = g->ne; P.nlag = g->nlag; P.nh = g->nh; P.nhat = g->nhat; P.ntil = g->ntil;
    P.nq = g->nq; P.nth = g->nth; P.nrh = g->nrh; P.band = lag; P.dt = g->dt; P.c = g->c;
    for (int j = 0; j < 18; ++j) P.ring[j] = ring[j];
    P.acc_tail = g->acc_tail;
    P.plist = g->plist;
    P.pcount = g->pcount;
    P.mom = g->mom;
    P.items = g->items;
    P.icount = g->icount;
    P.qt = g->qt;
    for (int cs = 0; cs < g->ncolor; ++cs) {
        for (int ct = 0; ct < g->ncolor; ++ct) {
            P.slist = g->order + g->cptr_h[cs];
            P.ns = g->cptr_h[cs + 1] - g->cptr_h[cs];
            P.tlist = g->order + g->cptr_h[ct];
            P.ntl = g->cptr_h[ct + 1] - g->cptr_h[ct];
            long npairs = (long)P.ns * P.ntl;
            if (npairs == 0) continue;
            if (hipMemsetAsync(g->pcount, 0, sizeof(int), g->stream) != hipSuccess) return -2;
            hipLaunchKernelGGL(k_pairs, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, g->stream, P);
            int nact = 0;
            if (hipMemcpyAsync(&nact, g->pcount, sizeof(int), hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
                hipStreamSynchronize(g->stream) != hipSuccess)
                return -2;
            /* batches of active pairs: classify their (pair, test point) items,
             * walk the far-rule and the polar items in launches of their own,
             * then form and add the products */
            for (int p0 = 0; p0 < nact; p0 += g->batch) {
                P.p0 = p0;
                P.nb = nact - p0 < g->batch ? nact - p0 : g->batch;
                const long nit = (long)P.nb * P.nq;
                if (hipMemsetAsync(g->icount, 0, 2 * sizeof(int), g->stream) != hipSuccess) return -2;
                hipLaunchKernelGGL(k_classify, dim3((unsigned)((nit + 255) / 256)), dim3(256), 0, g->stream, P);
                for (int cls = 0; cls < 2; ++cls)
                    hipLaunchKernelGGL(k_walk, dim3((unsigned)((nit + 255) / 256)), dim3(256), 0, g->stream, P, cls);
                const long npr = (long)P.nb * NCH * 9;
                hipLaunchKernelGGL(k_products, dim3((unsigned)((npr + 255) / 256)), dim3(256), 0, g->stream, P);
                if (hipGetLastError() != hipSuccess) return -2;
            }
        }
    }
    const int slot = lag % 3;
    for (int b = 0; b < 6; ++b) {
        if (lag >= lim[b]) continue;
        long nn2 = (long)nn;
        hipLaunchKernelGGL(k_symmetrise, dim3((unsigned)((nn2 + 255) / 256)), dim3(256), 0, g->stream,
                           ring[slot * 6 + b], g->ne);
    }
    if (hipGetLastError() != hipSuccess) return -2;
    g->next_lag = lag + 1;
    return 0;
}

void gfx_ret_destroy(gfx_ret* g) {
    if (!g) return;
    hipStreamSynchronize(g->stream);
    hipFree(g->tri); hipFree(g->fe); hipFree(g->fcoef); hipFree(g->fopp); hipFree(g->tris);
    hipFree(g->order); hipFree(g->acc_tail); hipFree(g->plist); hipFree(g->pcount);
    hipFree(g->mom); hipFree(g->items); hipFree(g->icount); hipFree(g->qt);
    free(g->cptr_h);
    free(g);
}

/* Static blocks on the BC basis (Section III):  T0s = (1/D) <g_m, g_n g>,
 * T0h = D <div g_m, div g_n g>, dense [ne][ne] device outputs (overwritten,
 * then symmetrised).  fv: fine triangles [nft][3][3]; BC restrictions
 * g_n|_t = a x - b sorted by fine triangle: res_t, res_n, res_a, res_b
 * [nres][3]; rule: the nq-point test rule of near pairs; far: the 3-point
 * rule (test and source of far pairs, source rule of the polar walk's far
 * case).  chunk: test triangles per pass.  Synchronous.  Returns 0 or a
 * negative code. */
int gfx_static_bc(int nft, const double* fv, int nres, const int32_t* res_t, const int32_t* res_n,
                  const double* res_a, const double* res_b, int ne, double D, int nq, int nth, int nrh,
                  const double* glx, const double* glw, const double* rule, const double* far, int chunk,
                  void* stream, double* T0s, double* T0h) {
    for (int k = 0; k < nres; ++k) {
        if (res_t[k] < 0 || res_t[k] >= nft || res_n[k] < 0 || res_n[k] >= ne) return -1;
        if (k > 0 && res_t[k] < res_t[k - 1]) return -1;   /* sorted by fine triangle */
    }
    QTables* qt = nullptr;
    int rc = make_tables(glx, glw, rule, nq, far, 3, &qt);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (chunk <= 0) chunk = 512;
    double* T = (double*)malloc(sizeof(double) * 16 * (size_t)nft);
    for (int t = 0; t < nft; ++t) tri_record(fv + 9 * t, fv + 9 * t + 3, fv + 9 * t + 6, T + 16 * t);
    /* restrictions grouped by BC function n, and per chunk by row m */
    int* byn_ptr = (int*)calloc(ne + 1, sizeof(int));
    int* byn_k = (int*)malloc(sizeof(int) * (size_t)nres);
    for (int k = 0; k < nres; ++k) byn_ptr[res_n[k] + 1]++;
    for (int n = 0; n < ne; ++n) byn_ptr[n + 1] += byn_ptr[n];
    {
        int* fill = (int*)malloc(sizeof(int) * (ne + 1));
        memcpy(fill, byn_ptr, sizeof(int) * (ne + 1));
        for (int k = 0; k < nres; ++k) byn_k[fill[res_n[k]]++] = k;
        free(fill);
    }
    double *dT = 0, *dMB = 0, *dW = 0, *da = 0, *db = 0;
    int *dbp = 0, *dbk = 0, *drt = 0, *dnl = 0, *dnc = 0, *drows = 0, *drp = 0, *drk = 0;
    int near_cap = 0;
    int* rows = (int*)malloc(sizeof(int) * (size_t)ne);
    int* rptr = (int*)malloc(sizeof(int) * ((size_t)ne + 1));
    int* rk = (int*)malloc(sizeof(int) * (size_t)nres);
    int* mark = (int*)malloc(sizeof(int) * (size_t)ne);
    for (int m = 0; m < ne; ++m) mark[m] = -1;
    const size_t nn = (size_t)ne * ne;
    GCHK(hipMalloc(&dT, sizeof(double) * 16 * (size_t)nft));
    GCHK(hipMalloc(&dMB, sizeof(double) * 16 * (size_t)chunk * nft));
    GCHK(hipMalloc(&dW, sizeof(double) * 13 * (size_t)chunk * ne));
    GCHK(hipMalloc(&da, sizeof(double) * (size_t)nres));
    GCHK(hipMalloc(&db, sizeof(double) * 3 * (size_t)nres));
    GCHK(hipMalloc(&drt, sizeof(int) * (size_t)nres));
    GCHK(hipMalloc(&dbp, sizeof(int) * (size_t)(ne + 1)));
    GCHK(hipMalloc(&dbk, sizeof(int) * (size_t)nres));
    GCHK(hipMalloc(&drows, sizeof(int) * (size_t)ne));
    GCHK(hipMalloc(&drp, sizeof(int) * ((size_t)ne + 1)));
    GCHK(hipMalloc(&drk, sizeof(int) * (size_t)nres));
    near_cap = chunk * 2048;
    GCHK(hipMalloc(&dnl, sizeof(int) * 2 * (size_t)near_cap));
    GCHK(hipMalloc(&dnc, sizeof(int)));
    GCHK(hipMemcpy(dT, T, sizeof(double) * 16 * (size_t)nft, hipMemcpyHostToDevice));
    GCHK(hipMemcpy(da, res_a, sizeof(double) * (size_t)nres, hipMemcpyHostToDevice));
    GCHK(hipMemcpy(db, res_b, sizeof(double) * 3 * (size_t)nres, hipMemcpyHostToDevice));
    GCHK(hipMemcpy(drt, res_t, sizeof(int) * (size_t)nres, hipMemcpyHostToDevice));
    GCHK(hipMemcpy(dbp, byn_ptr, sizeof(int) * (size_t)(ne + 1), hipMemcpyHostToDevice));
    GCHK(hipMemcpy(dbk, byn_k, sizeof(int) * (size_t)nres, hipMemcpyHostToDevice));
    GCHK(hipMemsetAsync(T0s, 0, nn * sizeof(double), st));
    GCHK(hipMemsetAsync(T0h, 0, nn * sizeof(double), st));
    for (int s0 = 0; s0 < nft; s0 += chunk) {
        int s1 = s0 + chunk < nft ? s0 + chunk : nft;
        StatParams P;
        P.tri = dT; P.nft = nft; P.s0 = s0; P.s1 = s1; P.nq = nq; P.far_n = 3; P.nth = nth; P.nrh = nrh;
        P.MB = dMB; P.near_list = dnl; P.near_count = dnc; P.near_cap = near_cap;
        P.qt = qt;
        GCHK(hipMemsetAsync(dnc, 0, sizeof(int), st));
        long np = (long)(s1 - s0) * nft;
        hipLaunchKernelGGL(k_static_far, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, P);
        GCHK(hipGetLastError());
        int cnt = 0;
        GCHK(hipMemcpyAsync(&cnt, dnc, sizeof(int), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        if (cnt > near_cap) { rc = -4; goto fail; }
        if (cnt > 0) {
            hipLaunchKernelGGL(k_static_near, dim3((unsigned)(((long)cnt * 8 + 255) / 256)), dim3(256), 0, st, P,
                               cnt);
            GCHK(hipGetLastError());
        }
        long nw = (long)(s1 - s0) * ne;
        hipLaunchKernelGGL(k_static_w, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, (const double*)dMB,
                           nft, s0, s1, ne, (const int*)dbp, (const int*)dbk, (const int*)drt, (const double*)da,
                           (const double*)db, dW);
        GCHK(hipGetLastError());
        /* rows m with a restriction on a test triangle of the chunk (res_t sorted) */
        int nrows = 0;
        {
            int klo = 0;
            while (klo < nres && res_t[klo] < s0) ++klo;
            int khi = klo;
            while (khi < nres && res_t[khi] < s1) ++khi;
            for (int k = klo; k < khi; ++k) {
                int m = res_n[k];
                if (mark[m] < 0) { mark[m] = nrows; rows[nrows++] = m; }
            }
            for (int r = 0; r <= nrows; ++r) rptr[r] = 0;
            for (int k = klo; k < khi; ++k) rptr[mark[res_n[k]] + 1]++;
            for (int r = 0; r < nrows; ++r) rptr[r + 1] += rptr[r];
            int* fill = (int*)malloc(sizeof(int) * (nrows + 1));
            memcpy(fill, rptr, sizeof(int) * (nrows + 1));
            for (int k = klo; k < khi; ++k) rk[fill[mark[res_n[k]]]++] = k;
            free(fill);
            for (int r = 0; r < nrows; ++r) mark[rows[r]] = -1;
        }
        if (nrows > 0) {
            GCHK(hipMemcpyAsync(drows, rows, sizeof(int) * nrows, hipMemcpyHostToDevice, st));
            GCHK(hipMemcpyAsync(drp, rptr, sizeof(int) * (nrows + 1), hipMemcpyHostToDevice, st));
            GCHK(hipMemcpyAsync(drk, rk, sizeof(int) * rptr[nrows], hipMemcpyHostToDevice, st));
            long nt = (long)nrows * ne;
            hipLaunchKernelGGL(k_static_t, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, (const double*)dW, s0,
                               ne, (const int*)drows, (const int*)drp, (const int*)drk, nrows, (const int*)drt,
                               (const double*)da, (const double*)db, D, T0s, T0h);
            GCHK(hipGetLastError());
            GCHK(hipStreamSynchronize(st));   /* host row lists are reused by the next chunk */
        }
    }
    {
        long nn2 = (long)nn;
        hipLaunchKernelGGL(k_symmetrise, dim3((unsigned)((nn2 + 255) / 256)), dim3(256), 0, st, T0s, ne);
        hipLaunchKernelGGL(k_symmetrise, dim3((unsigned)((nn2 + 255) / 256)), dim3(256), 0, st, T0h, ne);
        GCHK(hipGetLastError());
        GCHK(hipStreamSynchronize(st));
    }
fail:
    hipStreamSynchronize(st);
    free(T); free(byn_ptr); free(byn_k); free(rows); free(rptr); free(rk); free(mark);
    hipFree(dT); hipFree(dMB); hipFree(dW); hipFree(da); hipFree(db); hipFree(drt); hipFree(dbp); hipFree(dbk);
    hipFree(dnl); hipFree(dnc); hipFree(drows); hipFree(drp); hipFree(drk); hipFree(qt);
    return rc;
}

}  /* extern "C" */
