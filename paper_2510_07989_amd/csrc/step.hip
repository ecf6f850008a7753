// Per-step kernels of the marching-on-in-time loop (single right-hand side).
#include "mot_internal.h"

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------ tested incident ---
// Section V-C: ebar_k = (1/dt) int_{(k-1)dt}^{k dt} (e; h) dt and
// Ebar_k = int_{-inf}^{k dt} (e; h) dt, tested with n x f_m (= -<f_m, .>).
// Gaussian time integral: A/(2c) p (1 + erf s), s = (4/w)(c(t - t0) - k.x).
__device__ __forceinline__ double erf_diff(double s1, double s0) {
    if (s0 >= 0.0) return erfc(s0) - erfc(s1);
    if (s1 <= 0.0) return erfc(-s1) - erfc(-s0);
    return erf(s1) - erf(s0);
}

__global__ void k_rhs_fields(int ne, int hs, int k0, const int* __restrict__ kbase, int B, int R, int Rp,
                             double dt, const double* __restrict__ X, const double* __restrict__ Fw,
                             const double* __restrict__ waves, const double* __restrict__ tcut,
                             double* __restrict__ ebar, double* __restrict__ Ebar,
                             const GmState* __restrict__ gm) {
    // thread per (edge m, batch column sc, wave r); step k = k0 + sc, with k0
    // read from the device (kbase, graph replay) or passed by the host
    // outputs [half][hs][B * Rp], column sc * Rp + r (zero for padding waves r >= R)
    if (gm->halt) return;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * B * Rp) return;
    const int r = t % Rp, sc = (t / Rp) % B, m = t / (Rp * B);
    const size_t ld = (size_t)B * Rp;
    const size_t hb = (size_t)hs * ld;
    const size_t o = (size_t)m * ld + (size_t)sc * Rp + r;
    if (r >= R) {
        ebar[o] = 0; ebar[hb + o] = 0; Ebar[o] = 0; Ebar[hb + o] = 0;
        return;
    }
    const int k = (kbase ? *kbase : k0) + sc;
    const double* wv = waves + 9 * r;
    const double amp = wv[0], w = wv[7], t0 = wv[8];
    const double px = wv[1], py = wv[2], pz = wv[3];
    const double kx = wv[4], ky = wv[5], kz = wv[6];
    // h polarisation k x p (eta = 1)
    const double hx = ky * pz - kz * py, hy = kz * px - kx * pz, hz = kx * py - ky * px;
    const double c4 = 4.0 / w;
    const double tk = k * dt, tk1 = (k - 1) * dt;
    const bool star_on = tk <= tcut[r];
    double ee = 0, eh = 0, Ee = 0, Eh = 0;
    for (int q = 0; q < 14; ++q) {
        const double* x = X + ((size_t)m * 14 + q) * 3;
        const double* f = Fw + ((size_t)m * 14 + q) * 3;
        double kdx = kx * x[0] + ky * x[1] + kz * x[2];
        double s1 = c4 * ((tk - t0) - kdx), s0 = c4 * ((tk1 - t0) - kdx);
        double te = erf_diff(s1, s0) / dt;
        double tE = star_on ? erfc(-s1) : 0.0;
        double fp = f[0] * px + f[1] * py + f[2] * pz;
        double fh = f[0] * hx + f[1] * hy + f[2] * hz;
        ee += te * fp; eh += te * fh;
        Ee += tE * fp; Eh += tE * fh;
    }
    const double a = -0.5 * amp;   // -(A / (2c)), the minus from n x f testing
    ebar[o] = a * ee;
    ebar[hb + o] = a * eh;
    Ebar[o] = a * Ee;
    Ebar[hb + o] = a * Eh;
}

// ------------------------------------------------ streamed row products ---
// One wavefront per output row; 16-byte loads, eight in flight per lane.
__device__ __forceinline__ void row2(const double* __restrict__ A, const double* __restrict__ xa,
                                     const double* __restrict__ xb, int len, int lane, double& sa,
                                     double& sb) {
    const d2v* a2 = reinterpret_cast<const d2v*>(A);
    const d2v* x2 = reinterpret_cast<const d2v*>(xa);
    const d2v* y2 = reinterpret_cast<const d2v*>(xb);
    const int n2 = len >> 1;
    int c = lane;
    for (; c + 448 < n2; c += 512) {
        d2v a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(a2 + c + 64 * u);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            d2v xu = x2[c + 64 * u], yv = y2[c + 64 * u];
            sa = fma(a[u].x, xu.x, sa); sa = fma(a[u].y, xu.y, sa);
            sb = fma(a[u].x, yv.x, sb); sb = fma(a[u].y, yv.y, sb);
        }
    }
    for (; c < n2; c += 64) {
        d2v a0 = __builtin_nontemporal_load(a2 + c);
        d2v u0 = x2[c], v0 = y2[c];
        sa = fma(a0.x, u0.x, sa); sa = fma(a0.y, u0.y, sa);
        sb = fma(a0.x, v0.x, sb); sb = fma(a0.y, v0.y, sb);
    }
}

__device__ __forceinline__ void row1(const double* __restrict__ A, const double* __restrict__ xa,
                                     int len, int lane, double& sa) {
    const d2v* a2 = reinterpret_cast<const d2v*>(A);
    const d2v* x2 = reinterpret_cast<const d2v*>(xa);
    const int n2 = len >> 1;
    int c = lane;
    for (; c + 448 < n2; c += 512) {
        d2v a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(a2 + c + 64 * u);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            d2v xu = x2[c + 64 * u];
            sa = fma(a[u].x, xu.x, sa); sa = fma(a[u].y, xu.y, sa);
        }
    }
    for (; c < n2; c += 64) {
        d2v a0 = __builtin_nontemporal_load(a2 + c);
        d2v u0 = x2[c];
        sa = fma(a0.x, u0.x, sa); sa = fma(a0.y, u0.y, sa);
    }
}

// row1 that also adds the squares of the vector entries it reads into sq,
// and their squares scaled by 2^600 into ss (open_norm)
__device__ __forceinline__ void row1sq(const double* __restrict__ A, const double* __restrict__ xa,
                                       int len, int lane, double& sa, double& sq, double& ss) {
    const d2v* a2 = reinterpret_cast<const d2v*>(A);
    const d2v* x2 = reinterpret_cast<const d2v*>(xa);
    const int n2 = len >> 1;
    int c = lane;
    for (; c + 448 < n2; c += 512) {
        d2v a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = __builtin_nontemporal_load(a2 + c + 64 * u);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            d2v xu = x2[c + 64 * u];
            sa = fma(a[u].x, xu.x, sa); sa = fma(a[u].y, xu.y, sa);
            sq = fma(xu.x, xu.x, sq); sq = fma(xu.y, xu.y, sq);
            ss += sq_scaled(xu.x); ss += sq_scaled(xu.y);
        }
    }
    for (; c < n2; c += 64) {
        d2v a0 = __builtin_nontemporal_load(a2 + c);
        d2v u0 = x2[c];
        sa = fma(a0.x, u0.x, sa); sa = fma(a0.y, u0.y, sa);
        sq = fma(u0.x, u0.x, sq); sq = fma(u0.y, u0.y, sq);
        ss += sq_scaled(u0.x); ss += sq_scaled(u0.y);
    }
}

// Opening of a cold GMRES cycle (x0 = 0, r = b, ||b|| = beta), as k_gm_start1
// with first = 1 leaves the state (written by one thread).
__device__ __forceinline__ void open_cycle(GmState* gm, double beta, double tol) {
    gm->bnorm = beta;
    gm->total = 0;
    gm->beta = beta;
    gm->g[0] = beta;
    gm->j = 0;
    gm->cycle_iters = 0;
    gm->breakdown = 0;
    gm->relres = beta > 0 ? beta / beta : 0.0;
    const int conv = (beta <= MOT_ZERO_NORM) || (beta <= tol * beta);
    gm->converged = conv;
    gm->done = conv;
    gm->inv_h = beta > MOT_ZERO_NORM ? 1.0 / beta : 0.0;
    gm->seq = 1;
}

// y = r_k - sum_{j=1}^{min(k-1, nh)} Q_j w_{k-j}   (eq. MOT right-hand side).
// r_k comes from the batched RHS [half][ne][B] (column (k-1) mod B).
// Q_j = [[q1, -qk], [qk, q2]] in three [ne][hs] blocks; ring slot of w_{k-j}
// is (k-j) mod nh.
__global__ __launch_bounds__(256) void k_history(int ne, int hs, const int* __restrict__ dk, int nh,
                                                 const double* __restrict__ Q,
                                                 const double* __restrict__ ring,
                                                 const double* __restrict__ rb, int B,
                                                 double* __restrict__ y, int wpr,
                                                 const GmState* __restrict__ gm) {
    if (gm->halt) return;
    // wpr wavefronts share one row, each streaming a contiguous 1/wpr of it
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = blockIdx.x * (4 / wpr) + wv / wpr;
    const int part = wv % wpr;
    const int plen = hs / wpr, off = part * plen;
    __shared__ double red[4][2];
    const int k = *dk;
    double hu = 0, hv = 0;
    if (m < ne) {
        const size_t blk = (size_t)ne * hs;
        const int n2 = 2 * hs;
        int nact = k - 1 < nh ? k - 1 : nh;
        for (int j = 1; j <= nact; ++j) {
            int slot = (k - j) % nh;
            const double* wu = ring + (size_t)slot * n2 + off;
            const double* wvv = ring + (size_t)slot * n2 + hs + off;
            const double* Qj = Q + (size_t)j * 3 * blk + (size_t)m * hs + off;
            double a = 0, b = 0, cc = 0, d = 0;
            row1(Qj, wu, plen, lane, a);                     // q1 u
            row2(Qj + blk, wvv, wu, plen, lane, b, cc);      // qk v, qk u
            row1(Qj + 2 * blk, wvv, plen, lane, d);          // q2 v
            hu += a - b;
            hv += cc + d;
        }
    }
    hu = wave_sum(hu);
    hv = wave_sum(hv);
    if (lane == 0) { red[wv][0] = hu; red[wv][1] = hv; }
    __syncthreads();
    if (lane == 0 && part == 0 && m < ne) {
        double su = 0, sv = 0;
        for (int p = 0; p < wpr; ++p) { su += red[wv + p][0]; sv += red[wv + p][1]; }
        const int sc = (k - 1) % B;
        const double* r = rb + (size_t)(((k - 1) / B) & 1) * 2 * ne * B;   // double-buffered batches
        y[m] = r[(size_t)m * B + sc] - su;
        y[hs + m] = r[(size_t)ne * B + (size_t)m * B + sc] - sv;
    }
}

// Variant with the columns outermost: every lane walks the same column slice of
// all 3 (L-1) row blocks, so each iteration has several independent 16-byte
// loads from different blocks in flight.
__global__ __launch_bounds__(256) void k_history_co(int ne, int hs, const int* __restrict__ dk, int nh,
                                                    const double* __restrict__ Q,
                                                    const double* __restrict__ ring,
                                                    const double* __restrict__ rb, int B,
                                                    double* __restrict__ y, const GmState* __restrict__ gm,
                                                    int wpr) {
    // wpr wavefronts share one row, each taking a contiguous 1/wpr of its
    // column slices (across all lag blocks)
    if (gm->halt) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = blockIdx.x * (4 / wpr) + wv / wpr;
    const int part = wv % wpr;
    const int k = *dk;
    const size_t blk = (size_t)ne * hs;
    const int n2 = 2 * hs;
    const int nact = k - 1 < nh ? k - 1 : nh;
    const int np = hs >> 1;
    const int cpart = np / wpr;                 // hs is a multiple of 8: np of 4
    const int cb = part * cpart, ce = cb + cpart;
    __shared__ double red[4][2];
    double hu = 0, hv = 0;
    if (m < ne) {
        for (int c = cb + lane; c < ce; c += 64) {
            int j = 1;
            for (; j + 1 <= nact; j += 2) {
                const d2v* A0 = reinterpret_cast<const d2v*>(Q + (size_t)j * 3 * blk + (size_t)m * hs);
                const d2v* A1 = reinterpret_cast<const d2v*>(Q + (size_t)(j + 1) * 3 * blk + (size_t)m * hs);
                const size_t b2 = blk >> 1;
                d2v a0 = __builtin_nontemporal_load(A0 + c), k0 = __builtin_nontemporal_load(A0 + b2 + c),
                    q0 = __builtin_nontemporal_load(A0 + 2 * b2 + c);
                d2v a1 = __builtin_nontemporal_load(A1 + c), k1 = __builtin_nontemporal_load(A1 + b2 + c),
                    q1 = __builtin_nontemporal_load(A1 + 2 * b2 + c);
                const d2v* w0 = reinterpret_cast<const d2v*>(ring + (size_t)((k - j) % nh) * n2);
                const d2v* w1 = reinterpret_cast<const d2v*>(ring + (size_t)((k - j - 1) % nh) * n2);
                d2v u0 = w0[c], v0 = w0[(hs >> 1) + c], u1 = w1[c], v1 = w1[(hs >> 1) + c];
                hu = fma(a0.x, u0.x, hu); hu = fma(a0.y, u0.y, hu);
                hu = fma(-k0.x, v0.x, hu); hu = fma(-k0.y, v0.y, hu);
                hv = fma(k0.x, u0.x, hv); hv = fma(k0.y, u0.y, hv);
                hv = fma(q0.x, v0.x, hv); hv = fma(q0.y, v0.y, hv);
                hu = fma(a1.x, u1.x, hu); hu = fma(a1.y, u1.y, hu);
                hu = fma(-k1.x, v1.x, hu); hu = fma(-k1.y, v1.y, hu);
                hv = fma(k1.x, u1.x, hv); hv = fma(k1.y, u1.y, hv);
                hv = fma(q1.x, v1.x, hv); hv = fma(q1.y, v1.y, hv);
            }
            for (; j <= nact; ++j) {
                const d2v* A0 = reinterpret_cast<const d2v*>(Q + (size_t)j * 3 * blk + (size_t)m * hs);
                const size_t b2 = blk >> 1;
                d2v a0 = __builtin_nontemporal_load(A0 + c), k0 = __builtin_nontemporal_load(A0 + b2 + c),
                    q0 = __builtin_nontemporal_load(A0 + 2 * b2 + c);
                const d2v* w0 = reinterpret_cast<const d2v*>(ring + (size_t)((k - j) % nh) * n2);
                d2v u0 = w0[c], v0 = w0[(hs >> 1) + c];
                hu = fma(a0.x, u0.x, hu); hu = fma(a0.y, u0.y, hu);
                hu = fma(-k0.x, v0.x, hu); hu = fma(-k0.y, v0.y, hu);
                hv = fma(k0.x, u0.x, hv); hv = fma(k0.y, u0.y, hv);
                hv = fma(q0.x, v0.x, hv); hv = fma(q0.y, v0.y, hv);
            }
        }
    }
    hu = wave_sum(hu);
    hv = wave_sum(hv);
    if (lane == 0) { red[wv][0] = hu; red[wv][1] = hv; }
    __syncthreads();
    if (lane == 0 && part == 0 && m < ne) {
        double su = 0, sv = 0;
        for (int p = 0; p < wpr; ++p) { su += red[wv + p][0]; sv += red[wv + p][1]; }
        const int sc = (k - 1) % B;
        const double* r = rb + (size_t)(((k - 1) / B) & 1) * 2 * ne * B;   // double-buffered batches
        y[m] = r[(size_t)m * B + sc] - su;
        y[hs + m] = r[(size_t)ne * B + (size_t)m * B + sc] - sv;
    }
}

// ------------------------------------------------------------------ GMRES ---
// Arnoldi with classical Gram-Schmidt and one re-orthogonalisation, Givens
// rotations and the triangular solve on the device.  Reductions use per-block
// partials and a last-block-done finish (fixed summation order).

__device__ __forceinline__ bool last_block(unsigned int* counter) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

// y = Q0 * (scale * src); when vout != nullptr also write vout = scale * src
// (rows this wave owns).  scale is read from gm->inv_h when use_inv.
__global__ __launch_bounds__(256) void k_q0_matvec(int ne, int hs, const double* __restrict__ Q0,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ vout, double* __restrict__ y,
                                                   const GmState* __restrict__ gm, int check_done,
                                                   int use_inv, int wpr) {
    if (gm->halt || (check_done && gm->done)) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = blockIdx.x * (4 / wpr) + wv / wpr;
    const int part = wv % wpr;
    const int plen = hs / wpr, off = part * plen;
    __shared__ double red[4][2];
    double a = 0, b = 0, cc = 0, d = 0;
    if (m < ne) {
        const size_t blk = (size_t)ne * hs;
        const double* xu = src + off;
        const double* xv = src + hs + off;
        row1(Q0 + (size_t)m * hs + off, xu, plen, lane, a);
        row2(Q0 + blk + (size_t)m * hs + off, xv, xu, plen, lane, b, cc);
        row1(Q0 + 2 * blk + (size_t)m * hs + off, xv, plen, lane, d);
    }
    a = wave_sum(a - b);
    cc = wave_sum(cc + d);
    if (lane == 0) { red[wv][0] = a; red[wv][1] = cc; }
    __syncthreads();
    if (lane == 0 && part == 0 && m < ne) {
        double su = 0, sv = 0;
        for (int p = 0; p < wpr; ++p) { su += red[wv + p][0]; sv += red[wv + p][1]; }
        const double sc = use_inv ? gm->inv_h : 1.0;
        y[m] = sc * su;
        y[hs + m] = sc * sv;
        if (vout) {
            vout[m] = sc * src[m];
            vout[hs + m] = sc * src[hs + m];
        }
    }
}

// z = M (inv_h src), V_j = inv_h src : the right preconditioner of the Q_0 solve,
// an approximate inverse of Q_0 stored dense [n2][n2] in FP32 or FP64.
// start (FP64, cold start): src is the step's right-hand side r = y and this
// launch also opens the GMRES cycle: every row group forms ||src|| from the
// entries it streams anyway (same order in every group, so the same bits),
// scales by its inverse, zeroes x, and row 0 writes the cycle state.
template <typename T>
__global__ __launch_bounds__(256) void k_precond(int n2, const T* __restrict__ M,
                                                 const double* __restrict__ src, double* __restrict__ vj,
                                                 double* __restrict__ z, GmState* __restrict__ gm,
                                                 int wpr, int start, double tol, double* __restrict__ x) {
    if (gm->halt || (!start && gm->done)) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = blockIdx.x * (4 / wpr) + wv / wpr;
    const int part = wv % wpr;
    const int plen = n2 / wpr, off = part * plen;
    __shared__ double red[4], rq[4], rs[4];
    double s0 = 0, s1 = 0, sq = 0, ss = 0;
    if (m < n2) {
        const T* row = M + (size_t)m * n2 + off;
        const double* xs = src + off;
        if constexpr (sizeof(T) == 4) {
            typedef float f4v __attribute__((ext_vector_type(4)));
            typedef double d4v __attribute__((ext_vector_type(4)));
            const f4v* a4 = reinterpret_cast<const f4v*>(row);
            const d4v* x4 = reinterpret_cast<const d4v*>(xs);
            const int n4 = plen >> 2;
            int c = lane;
            for (; c + 192 < n4; c += 256) {
                f4v a[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = __builtin_nontemporal_load(a4 + c + 64 * u);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    d4v xu = x4[c + 64 * u];
                    s0 = fma((double)a[u].x, xu.x, s0); s0 = fma((double)a[u].y, xu.y, s0);
                    s1 = fma((double)a[u].z, xu.z, s1); s1 = fma((double)a[u].w, xu.w, s1);
                }
            }
            for (; c < n4; c += 64) {
                f4v a0 = __builtin_nontemporal_load(a4 + c);
                d4v u0 = x4[c];
                s0 = fma((double)a0.x, u0.x, s0); s0 = fma((double)a0.y, u0.y, s0);
                s1 = fma((double)a0.z, u0.z, s1); s1 = fma((double)a0.w, u0.w, s1);
            }
        } else if (start) {
            row1sq(reinterpret_cast<const double*>(row), xs, plen, lane, s0, sq, ss);
        } else {
            row1(reinterpret_cast<const double*>(row), xs, plen, lane, s0);
        }
    }
    double s = wave_sum(s0 + s1);
    if (start) { sq = wave_sum(sq); ss = wave_sum(ss); }
    if (lane == 0) { red[wv] = s; rq[wv] = sq; rs[wv] = ss; }
    __syncthreads();
    if (lane == 0 && part == 0 && m < n2) {
        double t = 0;
        for (int p = 0; p < wpr; ++p) t += red[wv + p];
        double sc = start ? 0.0 : gm->inv_h;
        if (start) {
            double q = 0, qs = 0;
            for (int p = 0; p < wpr; ++p) { q += rq[wv + p]; qs += rs[wv + p]; }
            const double beta = open_norm(q, qs);
            sc = beta > MOT_ZERO_NORM ? 1.0 / beta : 0.0;
            x[m] = 0.0;
            if (m == 0) open_cycle(gm, beta, tol);
        }
        z[m] = sc * t;
        vj[m] = sc * src[m];
    }
}

// ------------------------------------- several rows per wavefront (RPW) ---
// Workgroups of cs wavefronts, each owning RPW consecutive output rows, every
// wavefront on 1/cs of the columns: every vector slice loaded from L2 serves
// RPW matrix rows, so a larger share of the load instructions stream matrix
// entries from HBM (cs = RPW keeps one wavefront per row).  Rows past the end are
// clamped to the last row for loading (same addresses, results dropped).

// history: column slices across all lag blocks, as k_history_co.  cs
// wavefronts (the workgroup) share the RPW rows, each taking a contiguous
// 1/cs of the column slices: the ring slices a wavefront loads then serve RPW
// rows while the launch keeps as many wavefronts as one row per wavefront.
template <int RPW>
__global__ __launch_bounds__(256) void k_history_rows(int ne, int hs, const int* __restrict__ dk, int nh,
                                                       const double* __restrict__ Q,
                                                       const double* __restrict__ ring,
                                                       const double* __restrict__ rb, int B,
                                                       double* __restrict__ y, const GmState* __restrict__ gm,
                                                       int cs) {
    if (gm->halt) return;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int m0 = blockIdx.x * RPW;             // < ne: the grid has ceil(ne / RPW) workgroups
    const int k = *dk;
    const size_t blk = (size_t)ne * hs;
    const size_t b2 = blk >> 1;                  // one block in 16-byte units
    const int n2 = 2 * hs;
    const int nact = k - 1 < nh ? k - 1 : nh;
    const int np = hs >> 1;
    size_t ro[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) ro[r] = (size_t)min(m0 + r, ne - 1) * np;
    double hu[RPW], hv[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) hu[r] = hv[r] = 0.0;
    const int cpart = np / cs;                   // hs is a multiple of 8: np of 4
    for (int c = part * cpart + lane; c < (part + 1) * cpart; c += 64) {
        int j = 1;
        for (; j + 1 <= nact; j += 2) {
            const d2v* A0 = reinterpret_cast<const d2v*>(Q + (size_t)j * 3 * blk) + c;
            const d2v* A1 = reinterpret_cast<const d2v*>(Q + (size_t)(j + 1) * 3 * blk) + c;
            d2v a0[RPW], k0[RPW], q0[RPW], a1[RPW], k1[RPW], q1[RPW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                a0[r] = __builtin_nontemporal_load(A0 + ro[r]);
                k0[r] = __builtin_nontemporal_load(A0 + b2 + ro[r]);
                q0[r] = __builtin_nontemporal_load(A0 + 2 * b2 + ro[r]);
                a1[r] = __builtin_nontemporal_load(A1 + ro[r]);
                k1[r] = __builtin_nontemporal_load(A1 + b2 + ro[r]);
                q1[r] = __builtin_nontemporal_load(A1 + 2 * b2 + ro[r]);
            }
            const d2v* w0 = reinterpret_cast<const d2v*>(ring + (size_t)((k - j) % nh) * n2);
            const d2v* w1 = reinterpret_cast<const d2v*>(ring + (size_t)((k - j - 1) % nh) * n2);
            const d2v u0 = w0[c], v0 = w0[np + c], u1 = w1[c], v1 = w1[np + c];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                double su = hu[r], sv = hv[r];
                su = fma(a0[r].x, u0.x, su); su = fma(a0[r].y, u0.y, su);
                su = fma(-k0[r].x, v0.x, su); su = fma(-k0[r].y, v0.y, su);
                sv = fma(k0[r].x, u0.x, sv); sv = fma(k0[r].y, u0.y, sv);
                sv = fma(q0[r].x, v0.x, sv); sv = fma(q0[r].y, v0.y, sv);
                su = fma(a1[r].x, u1.x, su); su = fma(a1[r].y, u1.y, su);
                su = fma(-k1[r].x, v1.x, su); su = fma(-k1[r].y, v1.y, su);
                sv = fma(k1[r].x, u1.x, sv); sv = fma(k1[r].y, u1.y, sv);
                sv = fma(q1[r].x, v1.x, sv); sv = fma(q1[r].y, v1.y, sv);
                hu[r] = su; hv[r] = sv;
            }
        }
        for (; j <= nact; ++j) {
            const d2v* A0 = reinterpret_cast<const d2v*>(Q + (size_t)j * 3 * blk) + c;
            d2v a0[RPW], k0[RPW], q0[RPW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                a0[r] = __builtin_nontemporal_load(A0 + ro[r]);
                k0[r] = __builtin_nontemporal_load(A0 + b2 + ro[r]);
                q0[r] = __builtin_nontemporal_load(A0 + 2 * b2 + ro[r]);
            }
            const d2v* w0 = reinterpret_cast<const d2v*>(ring + (size_t)((k - j) % nh) * n2);
            const d2v u0 = w0[c], v0 = w0[np + c];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                double su = hu[r], sv = hv[r];
                su = fma(a0[r].x, u0.x, su); su = fma(a0[r].y, u0.y, su);
                su = fma(-k0[r].x, v0.x, su); su = fma(-k0[r].y, v0.y, su);
                sv = fma(k0[r].x, u0.x, sv); sv = fma(k0[r].y, u0.y, sv);
                sv = fma(q0[r].x, v0.x, sv); sv = fma(q0[r].y, v0.y, sv);
                hu[r] = su; hv[r] = sv;
            }
        }
    }
    __shared__ double red[4][RPW][2];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        hu[r] = wave_sum(hu[r]);
        hv[r] = wave_sum(hv[r]);
        if (lane == 0) { red[part][r][0] = hu[r]; red[part][r][1] = hv[r]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int sc = (k - 1) % B;
        const double* rr = rb + (size_t)(((k - 1) / B) & 1) * 2 * ne * B;   // double-buffered batches
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int m = m0 + r;
            if (m < ne) {
                double su = 0, sv = 0;
                for (int p = 0; p < cs; ++p) { su += red[p][r][0]; sv += red[p][r][1]; }
                y[m] = rr[(size_t)m * B + sc] - su;
                y[hs + m] = rr[(size_t)ne * B + (size_t)m * B + sc] - sv;
            }
        }
    }
}

// y = Q0 (scale src), vout = scale src (when given), as k_q0_matvec; cs
// wavefronts (the workgroup) share the RPW rows, each on 1/cs of the columns
template <int RPW>
__global__ __launch_bounds__(256) void k_q0_rows(int ne, int hs, const double* __restrict__ Q0,
                                                  const double* __restrict__ src, double* __restrict__ vout,
                                                  double* __restrict__ y, const GmState* __restrict__ gm,
                                                  int check_done, int use_inv, int cs) {
    if (gm->halt || (check_done && gm->done)) return;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int m0 = blockIdx.x * RPW;             // < ne: the grid has ceil(ne / RPW) workgroups
    const int np = hs >> 1;
    const int cpart = np / cs, c1 = (part + 1) * cpart;
    const size_t b2 = ((size_t)ne * hs) >> 1;
    const d2v* A = reinterpret_cast<const d2v*>(Q0);
    const d2v* xu = reinterpret_cast<const d2v*>(src);
    const d2v* xv = reinterpret_cast<const d2v*>(src + hs);
    size_t ro[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) ro[r] = (size_t)min(m0 + r, ne - 1) * np;
    double su[RPW], sv[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) su[r] = sv[r] = 0.0;
    int c = part * cpart + lane;
    for (; c + 64 < c1; c += 128) {
        d2v a[2][RPW], kk[2][RPW], q[2][RPW];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const size_t o = ro[r] + c + 64 * u;
                a[u][r] = __builtin_nontemporal_load(A + o);
                kk[u][r] = __builtin_nontemporal_load(A + b2 + o);
                q[u][r] = __builtin_nontemporal_load(A + 2 * b2 + o);
            }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const d2v uu = xu[c + 64 * u], vv = xv[c + 64 * u];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                double s1 = su[r], s2 = sv[r];
                s1 = fma(a[u][r].x, uu.x, s1); s1 = fma(a[u][r].y, uu.y, s1);
                s1 = fma(-kk[u][r].x, vv.x, s1); s1 = fma(-kk[u][r].y, vv.y, s1);
                s2 = fma(kk[u][r].x, uu.x, s2); s2 = fma(kk[u][r].y, uu.y, s2);
                s2 = fma(q[u][r].x, vv.x, s2); s2 = fma(q[u][r].y, vv.y, s2);
                su[r] = s1; sv[r] = s2;
            }
        }
    }
    for (; c < c1; c += 64) {
        const d2v uu = xu[c], vv = xv[c];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const d2v a = __builtin_nontemporal_load(A + ro[r] + c);
            const d2v kk = __builtin_nontemporal_load(A + b2 + ro[r] + c);
            const d2v q = __builtin_nontemporal_load(A + 2 * b2 + ro[r] + c);
            double s1 = su[r], s2 = sv[r];
            s1 = fma(a.x, uu.x, s1); s1 = fma(a.y, uu.y, s1);
            s1 = fma(-kk.x, vv.x, s1); s1 = fma(-kk.y, vv.y, s1);
            s2 = fma(kk.x, uu.x, s2); s2 = fma(kk.y, uu.y, s2);
            s2 = fma(q.x, vv.x, s2); s2 = fma(q.y, vv.y, s2);
            su[r] = s1; sv[r] = s2;
        }
    }
    __shared__ double red[4][RPW][2];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        su[r] = wave_sum(su[r]);
        sv[r] = wave_sum(sv[r]);
        if (lane == 0) { red[part][r][0] = su[r]; red[part][r][1] = sv[r]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sc = use_inv ? gm->inv_h : 1.0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int m = m0 + r;
            if (m < ne) {
                double a = 0, b = 0;
                for (int p = 0; p < cs; ++p) { a += red[p][r][0]; b += red[p][r][1]; }
                y[m] = sc * a;
                y[hs + m] = sc * b;
                if (vout) {
                    vout[m] = sc * src[m];
                    vout[hs + m] = sc * src[hs + m];
                }
            }
        }
    }
}

// z = M (inv_h src), V_j = inv_h src, as k_precond (start likewise, FP64); cs
// wavefronts (the workgroup) share the RPW rows, each on 1/cs of the columns
template <typename T, int RPW>
__global__ __launch_bounds__(256) void k_precond_rows(int n2, const T* __restrict__ M,
                                                       const double* __restrict__ src, double* __restrict__ vj,
                                                       double* __restrict__ z, GmState* __restrict__ gm,
                                                       int start, double tol, double* __restrict__ x, int cs) {
    if (gm->halt || (!start && gm->done)) return;
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int m0 = blockIdx.x * RPW;             // < n2: the grid has ceil(n2 / RPW) workgroups
    double s[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) s[r] = 0.0;
    double sq = 0.0, ss = 0.0;
    if constexpr (sizeof(T) == 8) {
        const int np = n2 >> 1;
        const d2v* A = reinterpret_cast<const d2v*>(M);
        const d2v* x2 = reinterpret_cast<const d2v*>(src);
        size_t ro[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) ro[r] = (size_t)min(m0 + r, n2 - 1) * np;
        const int cpart = np / cs, c1 = (part + 1) * cpart;
        int c = part * cpart + lane;
        for (; c + 192 < c1; c += 256) {
            d2v a[4][RPW];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < RPW; ++r) a[u][r] = __builtin_nontemporal_load(A + ro[r] + c + 64 * u);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const d2v xx = x2[c + 64 * u];
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    s[r] = fma(a[u][r].x, xx.x, s[r]);
                    s[r] = fma(a[u][r].y, xx.y, s[r]);
                }
                if (start) {
                    sq = fma(xx.x, xx.x, sq); sq = fma(xx.y, xx.y, sq);
                    ss += sq_scaled(xx.x); ss += sq_scaled(xx.y);
                }
            }
        }
        for (; c < c1; c += 64) {
            const d2v xx = x2[c];
            if (start) {
                sq = fma(xx.x, xx.x, sq); sq = fma(xx.y, xx.y, sq);
                ss += sq_scaled(xx.x); ss += sq_scaled(xx.y);
            }
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const d2v a = __builtin_nontemporal_load(A + ro[r] + c);
                s[r] = fma(a.x, xx.x, s[r]);
                s[r] = fma(a.y, xx.y, s[r]);
            }
        }
    } else {
        typedef float f4v __attribute__((ext_vector_type(4)));
        typedef double d4v __attribute__((ext_vector_type(4)));
        const int nq = n2 >> 2;
        const f4v* A = reinterpret_cast<const f4v*>(M);
        const d4v* x4 = reinterpret_cast<const d4v*>(src);
        size_t ro[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) ro[r] = (size_t)min(m0 + r, n2 - 1) * nq;
        const int cpart = nq / cs, c1 = (part + 1) * cpart;
        int c = part * cpart + lane;
        for (; c + 64 < c1; c += 128) {
            f4v a[2][RPW];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < RPW; ++r) a[u][r] = __builtin_nontemporal_load(A + ro[r] + c + 64 * u);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const d4v xx = x4[c + 64 * u];
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    s[r] = fma((double)a[u][r].x, xx.x, s[r]); s[r] = fma((double)a[u][r].y, xx.y, s[r]);
                    s[r] = fma((double)a[u][r].z, xx.z, s[r]); s[r] = fma((double)a[u][r].w, xx.w, s[r]);
                }
            }
        }
        for (; c < c1; c += 64) {
            const d4v xx = x4[c];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const f4v a = __builtin_nontemporal_load(A + ro[r] + c);
                s[r] = fma((double)a.x, xx.x, s[r]); s[r] = fma((double)a.y, xx.y, s[r]);
                s[r] = fma((double)a.z, xx.z, s[r]); s[r] = fma((double)a.w, xx.w, s[r]);
            }
        }
    }
    __shared__ double red[4][RPW + 2];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        s[r] = wave_sum(s[r]);
        if (lane == 0) red[part][r] = s[r];
    }
    if (start) {
        sq = wave_sum(sq);
        ss = wave_sum(ss);
        if (lane == 0) { red[part][RPW] = sq; red[part][RPW + 1] = ss; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sc = start ? 0.0 : gm->inv_h;
        if (start) {
            double q = 0, qs = 0;
            for (int p = 0; p < cs; ++p) { q += red[p][RPW]; qs += red[p][RPW + 1]; }
            const double beta = open_norm(q, qs);
            sc = beta > MOT_ZERO_NORM ? 1.0 / beta : 0.0;
            if (m0 == 0) open_cycle(gm, beta, tol);
        }
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int m = m0 + r;
            if (m < n2) {
                double t = 0;
                for (int p = 0; p < cs; ++p) t += red[p][r];
                z[m] = sc * t;
                vj[m] = sc * src[m];
                if (start) x[m] = 0.0;
            }
        }
    }
}

// Dense padded Q_0 = [[q1, -qk], [qk, q2]] on the index space [0, 2 hs), identity on padding.
__global__ void k_dense_q0(int ne, int hs, const double* __restrict__ Q, double* __restrict__ D) {
    const int n2 = 2 * hs;
    const size_t blk = (size_t)ne * hs;
    size_t total = (size_t)n2 * n2;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(t / n2), j = (int)(t % n2);
        int hi = i >= hs, hj = j >= hs;
        int ii = i - hi * hs, jj = j - hj * hs;
        double v;
        if (ii >= ne || jj >= ne) v = (i == j) ? 1.0 : 0.0;
        else if (!hi && !hj) v = Q[(size_t)ii * hs + jj];
        else if (!hi && hj) v = -Q[blk + (size_t)ii * hs + jj];
        else if (hi && !hj) v = Q[blk + (size_t)ii * hs + jj];
        else v = Q[2 * blk + (size_t)ii * hs + jj];
        D[t] = v;
    }
}

// X = alpha A^T (square n)
__global__ void k_transpose_scale(int n, double alpha, const double* __restrict__ A, double* __restrict__ X) {
    __shared__ double tile[32][33];
    int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    int tx = threadIdx.x, ty = threadIdx.y;
    for (int k = ty; k < 32; k += 8) {
        int r = by + k, c = bx + tx;
        tile[k][tx] = (r < n && c < n) ? A[(size_t)r * n + c] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        int r = bx + k, c = by + tx;
        if (r < n && c < n) X[(size_t)r * n + c] = alpha * tile[tx][k];
    }
}

// out[0] += sum |row sums| max ... : per-row abs sums -> rs[i], per-column abs sums -> cs[j]
__global__ void k_abs_sums(int n, const double* __restrict__ A, double* __restrict__ rs, double* __restrict__ cs) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = 0, c = 0;
    for (int j = 0; j < n; ++j) { r += fabs(A[(size_t)i * n + j]); c += fabs(A[(size_t)j * n + i]); }
    rs[i] = r;
    cs[i] = c;
}

// out += sum_{ij} (delta_ij - T_ij)^2   (atomic; setup only)
__global__ void k_eye_residual(int n, const double* __restrict__ T, double* __restrict__ out) {
    __shared__ double sh[8];
    double s = 0;
    size_t total = (size_t)n * n;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(t / n), j = (int)(t % n);
        double d = (i == j ? 1.0 : 0.0) - T[t];
        s = fma(d, d, s);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += sh[w];
        atomicAdd(out, a);
    }
}

__global__ void k_to_f32(size_t n, const double* __restrict__ X, float* __restrict__ Y) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        Y[t] = (float)X[t];
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

// r = b - r ; beta = ||r||, bnorm = ||b|| ; start a cycle.
__global__ __launch_bounds__(256) void k_gm_residual(int n2, const double* __restrict__ b,
                                                     double* __restrict__ r, GmState* gm,
                                                     GmFlag* flag, double tol, int first) {
    __shared__ double sh[8];
    double s1 = 0, s2 = 0, t1 = 0, t2 = 0;      // plain and scaled sums of squares
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
        double bi = b[i];
        double ri = bi - r[i];
        r[i] = ri;
        s1 = fma(ri, ri, s1);
        s2 = fma(bi, bi, s2);
        t1 += sq_scaled(ri);
        t2 += sq_scaled(bi);
    }
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    t1 = block_sum(t1, sh);
    t2 = block_sum(t2, sh);
    if (threadIdx.x == 0) {
        gm->partial[blockIdx.x] = s1;
        gm->partial[MOT_GM_BLOCKS + blockIdx.x] = s2;
        gm->partial[2 * MOT_GM_BLOCKS + blockIdx.x] = t1;
        gm->partial[3 * MOT_GM_BLOCKS + blockIdx.x] = t2;
    }
    if (!last_block(&gm->counter)) return;
    if (threadIdx.x == 0) {
        double rr = 0, bb = 0, rs = 0, bs = 0;
        for (int i = 0; i < (int)gridDim.x; ++i) {
            rr += gm->partial[i];
            bb += gm->partial[MOT_GM_BLOCKS + i];
            rs += gm->partial[2 * MOT_GM_BLOCKS + i];
            bs += gm->partial[3 * MOT_GM_BLOCKS + i];
        }
        double beta = open_norm(rr, rs);
        if (first) { gm->bnorm = open_norm(bb, bs); gm->total = 0; }
        gm->beta = beta;
        gm->g[0] = beta;
        gm->j = 0;
        gm->cycle_iters = 0;
        gm->breakdown = 0;
        double bn = gm->bnorm;
        gm->relres = bn > 0 ? beta / bn : 0.0;
        int conv = (bn <= MOT_ZERO_NORM) || (beta <= MOT_ZERO_NORM) || (beta <= tol * bn);
        gm->converged = conv;
        gm->done = conv;
        gm->inv_h = beta > MOT_ZERO_NORM ? 1.0 / beta : 0.0;
        gm->counter = 0;
        flag->relres = gm->relres;
        flag->converged = conv;
        flag->done = conv;
        flag->total = gm->total;
        __threadfence_system();
        flag->seq = ++gm->seq;
    }
}

// h1[l] = V[l] . w  for l <= j
__global__ __launch_bounds__(256) void k_gm_dots(int n2, const double* __restrict__ V,
                                                 const double* __restrict__ w, GmState* gm) {
    if (gm->done) return;
    const int j = gm->j;
    const int nb = gridDim.x;
    const int i0 = (int)((int64_t)n2 * blockIdx.x / nb), i1 = (int)((int64_t)n2 * (blockIdx.x + 1) / nb);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int l = wv; l <= j; l += nw) {
        const double* v = V + (size_t)l * n2;
        double s = 0;
        for (int i = i0 + lane; i < i1; i += 64) s = fma(v[i], w[i], s);
        s = wave_sum(s);
        if (lane == 0) gm->partial[(size_t)l * MOT_GM_BLOCKS + blockIdx.x] = s;
    }
    if (!last_block(&gm->counter)) return;
    for (int l = threadIdx.x; l <= j; l += blockDim.x) {
        double s = 0;
        for (int b = 0; b < nb; ++b) s += gm->partial[(size_t)l * MOT_GM_BLOCKS + b];
        gm->h1[l] = s;
    }
    if (threadIdx.x == 0) gm->counter = 0;
}

// w -= V h1 ; then h2 = V . w (stored into H column j), or ||w||^2 for the final pass
__global__ __launch_bounds__(256) void k_gm_orth(int n2, const double* __restrict__ V,
                                                 double* __restrict__ w, GmState* gm, GmFlag* flag,
                                                 double tol, int M, int final_pass) {
    if (gm->done) return;
    const int j = gm->j;
    const int nb = gridDim.x;
    const int i0 = (int)((int64_t)n2 * blockIdx.x / nb), i1 = (int)((int64_t)n2 * (blockIdx.x + 1) / nb);
    __shared__ double hl[MOT_MAXM + 1];
    for (int l = threadIdx.x; l <= j; l += blockDim.x) hl[l] = gm->h1[l];
    __syncthreads();
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double s = w[i];
        for (int l = 0; l <= j; ++l) s = fma(-hl[l], V[(size_t)l * n2 + i], s);
        w[i] = s;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (!final_pass) {
        for (int l = wv; l <= j; l += nw) {
            const double* v = V + (size_t)l * n2;
            double s = 0;
            for (int i = i0 + lane; i < i1; i += 64) s = fma(v[i], w[i], s);
            s = wave_sum(s);
            if (lane == 0) gm->partial[(size_t)l * MOT_GM_BLOCKS + blockIdx.x] = s;
        }
    } else {
        __shared__ double sh[8];
        double s = 0;
        for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) s = fma(w[i], w[i], s);
        s = block_sum(s, sh);
        if (threadIdx.x == 0) gm->partial[blockIdx.x] = s;
    }
    if (!last_block(&gm->counter)) return;
    if (!final_pass) {
        // H[:, j] = h1 (first pass) ; keep h1 <- h2 for the second update
        for (int l = threadIdx.x; l <= j; l += blockDim.x) {
            double s = 0;
            for (int b = 0; b < nb; ++b) s += gm->partial[(size_t)l * MOT_GM_BLOCKS + b];
            gm->H[(size_t)j * (M + 1) + l] = hl[l];
            gm->h1[l] = s;
        }
        if (threadIdx.x == 0) gm->counter = 0;
        return;
    }
    if (threadIdx.x != 0) return;
    double nn = 0;
    for (int b = 0; b < nb; ++b) nn += gm->partial[b];
    double hn = sqrt(nn);
    double* col = gm->H + (size_t)j * (M + 1);
    for (int l = 0; l <= j; ++l) col[l] += hl[l];      // h1 + h2
    col[j + 1] = hn;
    // apply previous rotations
    for (int l = 0; l < j; ++l) {
        double a = col[l], b = col[l + 1];
        col[l] = gm->cs[l] * a + gm->sn[l] * b;
        col[l + 1] = -gm->sn[l] * a + gm->cs[l] * b;
    }
    double a = col[j], b = col[j + 1];
    double r = hypot(a, b);
    double cs = r > 0 ? a / r : 1.0, sn = r > 0 ? b / r : 0.0;
    gm->cs[j] = cs;
    gm->sn[j] = sn;
    col[j] = r;
    col[j + 1] = 0.0;
    double gj = gm->g[j];
    gm->g[j] = cs * gj;
    gm->g[j + 1] = -sn * gj;
    int jj = j + 1;
    gm->j = jj;
    gm->cycle_iters = jj;
    gm->total += 1;
    double rel = gm->bnorm > 0 ? fabs(gm->g[jj]) / gm->bnorm : 0.0;
    gm->relres = rel;
    int conv = rel <= tol;
    int brk = !(hn > 1e-300 * (gm->beta + 1e-300));
    gm->breakdown = brk;
    gm->converged = conv || brk;
    gm->done = conv || brk || jj >= M;
    gm->inv_h = hn > 0 ? 1.0 / hn : 0.0;
    // triangular solve for the cycle so far (cheap; used when done)
    if (gm->done) {
        for (int i = jj - 1; i >= 0; --i) {
            double s = gm->g[i];
            for (int l = i + 1; l < jj; ++l) s -= gm->H[(size_t)l * (M + 1) + i] * gm->y[l];
            double d = gm->H[(size_t)i * (M + 1) + i];
            gm->y[i] = d != 0 ? s / d : 0.0;
        }
    }
    gm->counter = 0;
    flag->relres = rel;
    flag->converged = gm->converged;
    flag->done = gm->done;
    flag->total = gm->total;
    __threadfence_system();
    flag->seq = ++gm->seq;
}

// Single-workgroup variants used when a good preconditioner keeps the Krylov
// space small: the whole classical Gram-Schmidt pass with re-orthogonalisation,
// the norm and the Givens update run in one 1024-thread workgroup.
constexpr int kSW = 1024;
constexpr int kSWE = 32;     // elements per thread: n2 <= 32768

__device__ __forceinline__ double block_sum_sw(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
#pragma unroll
    for (int i = 0; i < kSW / 64; ++i) s += sh[i];
    return s;
}

// r = y - t (t = Q0 x0, or nothing for x0 = 0); beta, bnorm; start a cycle.
__global__ __launch_bounds__(kSW) void k_gm_start1(int n2, const double* __restrict__ b,
                                                    double* __restrict__ r, int have_t, GmState* gm,
                                                    GmFlag* flag, double tol, int first,
                                                    double* __restrict__ xzero) {
    if (gm->halt) return;
    __shared__ double sh[kSW / 64];
    double s1 = 0, s2 = 0, t1 = 0, t2 = 0;      // plain and scaled sums of squares
    for (int i = threadIdx.x; i < n2; i += kSW) {
        if (xzero) xzero[i] = 0.0;      // cold start x0 = 0
        double bi = b[i];
        double ri = have_t ? bi - r[i] : bi;
        r[i] = ri;
        s1 = fma(ri, ri, s1);
        s2 = fma(bi, bi, s2);
        t1 += sq_scaled(ri);
        t2 += sq_scaled(bi);
    }
    s1 = block_sum_sw(s1, sh);
    s2 = block_sum_sw(s2, sh);
    t1 = block_sum_sw(t1, sh);
    t2 = block_sum_sw(t2, sh);
    if (threadIdx.x == 0) {
        double beta = open_norm(s1, t1);
        if (first) { gm->bnorm = open_norm(s2, t2); gm->total = 0; gm->seq = 0; }
        gm->beta = beta;
        gm->g[0] = beta;
        gm->j = 0;
        gm->cycle_iters = 0;
        gm->breakdown = 0;
        double bn = gm->bnorm;
        gm->relres = bn > 0 ? beta / bn : 0.0;
        int conv = (bn <= MOT_ZERO_NORM) || (beta <= MOT_ZERO_NORM) || (beta <= tol * bn);
        gm->converged = conv;
        gm->done = conv;
        gm->inv_h = beta > MOT_ZERO_NORM ? 1.0 / beta : 0.0;
        ++gm->seq;
        if (flag) {               // null: queued steps, nobody waits on the host
            flag->relres = gm->relres;
            flag->converged = conv;
            flag->done = conv;
            flag->total = gm->total;
            __threadfence_system();
            flag->seq = gm->seq;
        }
    }
}

__device__ void givens_finish(GmState* gm, GmFlag* flag, const double* hvals, double* col, double hn, int j,
                              int M, double tol) {
    // the earlier rotations sweep the new column from the top: rotation l
    // touches entries l and l + 1 only, so entry l is final after it and is
    // stored at once, and entry l + 1 is carried in a register (no local array,
    // which would live in scratch memory)
    double carry = hvals[0];
    for (int l = 0; l < j; ++l) {
        const double cs = gm->cs[l], sn = gm->sn[l];
        const double a = carry, b = hvals[l + 1];
        col[l] = cs * a + sn * b;
        carry = -sn * a + cs * b;
    }
    double a = carry, b = hn;
    double r = hypot(a, b);
    double cs = r > 0 ? a / r : 1.0, sn = r > 0 ? b / r : 0.0;
    const double gj = gm->g[j], bnorm = gm->bnorm, beta = gm->beta;
    const int total = gm->total + 1;
    const double gnew = -sn * gj;
    const int jj = j + 1;
    const double rel = bnorm > 0 ? fabs(gnew) / bnorm : 0.0;
    const int conv = rel <= tol;
    const int brk = !(hn > 1e-300 * (beta + 1e-300));
    const int done = conv || brk || jj >= M;
    const int seq = gm->seq + 1;
    // publish the progress word first (host-visible), then the device state
    if (flag) {
        flag->relres = rel;
        flag->converged = conv || brk;
        flag->done = done;
        flag->total = total;
    }
    col[j] = r;
    col[j + 1] = 0.0;
    gm->cs[j] = cs;
    gm->sn[j] = sn;
    gm->g[j] = cs * gj;
    gm->g[jj] = gnew;
    gm->j = jj;
    gm->cycle_iters = jj;
    gm->total = total;
    gm->iters_all += 1;
    gm->relres = rel;
    gm->breakdown = brk;
    gm->converged = conv || brk;
    gm->done = done;
    gm->inv_h = hn > 0 ? 1.0 / hn : 0.0;
    gm->seq = seq;
    if (done) {
        for (int i = jj - 1; i >= 0; --i) {
            double s = gm->g[i];
            for (int l = i + 1; l < jj; ++l) s -= gm->H[(size_t)l * (M + 1) + i] * gm->y[l];
            double d = (i == j) ? r : gm->H[(size_t)i * (M + 1) + i];
            gm->y[i] = d != 0 ? s / d : 0.0;
        }
    }
    if (flag) {
        __threadfence_system();
        flag->seq = seq;
    }
}

// When the cycle is done: x += sum_l y_l Z_l ; when converged (or forced) also
// push x into the ring and the kept history.
// spec = 1 (speculative stepping): a solve that has not converged pushes
// nothing and raises the halt word instead, so that the later queued steps do
// nothing until the host has finished this one.
// kq > 0 (queued steps): the step index comes from the host; kq < 0 (steps
// replayed from a captured graph): it is the window's first step dk[1] plus
// -kq - 1.  In both cases the device step counter dk[0] is set to k + 1 after
// a push, for the next queued step (no thread of the launch reads it, so the
// write does not race).
struct FinArgs {
    const double* Zb;
    double* x;
    int* dk;
    int nh;
    double* ring;
    double* hist;
    int hist_cap;
    int kq;
};

// t0, nt: this thread's first element and the element stride of the launch;
// lead: the one thread that writes the scalars
__device__ __forceinline__ void finish_body(int n2, GmState* __restrict__ gm, const FinArgs& f, int force, int spec,
                                            int t0, int nt, bool lead) {
    const int k = f.kq > 0 ? f.kq : (f.kq < 0 ? f.dk[1] - f.kq - 1 : f.dk[0]);
    if (spec && !(gm->done && gm->converged)) {
        if (lead) {
            gm->halt_k = k;
            gm->halt = 1;
        }
        return;
    }
    if (!gm->done && !force) return;
    const int jj = gm->done ? gm->cycle_iters : 0;
    const int push = gm->converged || force;
    if (f.kq != 0 && push && lead) f.dk[0] = k + 1;
    double* slot = f.ring + (size_t)(k % f.nh) * n2;
    double* hs = (f.hist && k - 1 < f.hist_cap) ? f.hist + (size_t)(k - 1) * n2 : nullptr;
    for (int i = t0; i < n2; i += nt) {
        double s = f.x[i];
        for (int l = 0; l < jj; ++l) s = fma(gm->y[l], f.Zb[(size_t)l * n2 + i], s);
        f.x[i] = s;
        if (push) {
            slot[i] = s;
            if (hs) hs[i] = s;
        }
    }
}

__global__ void k_gm_finish(int n2, GmState* __restrict__ gm, FinArgs f, int force, int spec) {
    if (gm->halt) return;
    finish_body(n2, gm, f, force, spec, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x,
                blockIdx.x == 0 && threadIdx.x == 0);
}

// CGS2 of w against V[0..j], norm, Givens: one workgroup; EPT elements of w
// per thread stay in registers (EPT * 1024 >= n2).  fin: the queued step's
// speculative finisher (spec = 1) runs in the same workgroup afterwards.
template <int EPT>
__global__ __launch_bounds__(kSW) void k_gm_orth1(int n2, const double* __restrict__ V,
                                                   double* __restrict__ w, GmState* gm, GmFlag* flag,
                                                   double tol, int M, int fin, FinArgs fa) {
    if (gm->halt) return;
    if (gm->done) {
        // nothing to do, but every launch publishes one progress word
        if (threadIdx.x == 0) {
            ++gm->seq;
            if (flag) {
                flag->relres = gm->relres;
                flag->converged = gm->converged;
                flag->done = 1;
                flag->total = gm->total;
                __threadfence_system();
                flag->seq = gm->seq;
            }
        }
        if (fin) finish_body(n2, gm, fa, 0, 1, threadIdx.x, kSW, threadIdx.x == 0);
        return;
    }
    __shared__ double sh[kSW / 64];
    __shared__ double hc[MOT_MAXM + 1];
    const int j = gm->j;
    double wv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = threadIdx.x + e * kSW;
        wv[e] = i < n2 ? w[i] : 0.0;
    }
    if ((int)threadIdx.x <= j) hc[threadIdx.x] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int l = 0; l <= j; ++l) {
            const double* v = V + (size_t)l * n2;
            double vl[EPT];
            double s = 0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = threadIdx.x + e * kSW;
                vl[e] = i < n2 ? v[i] : 0.0;
                s = fma(vl[e], wv[e], s);
            }
            s = block_sum_sw(s, sh);
#pragma unroll
            for (int e = 0; e < EPT; ++e) wv[e] = fma(-s, vl[e], wv[e]);
            if (threadIdx.x == 0) hc[l] += s;
        }
    }
    double nn = 0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) nn = fma(wv[e], wv[e], nn);
    nn = block_sum_sw(nn, sh);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = threadIdx.x + e * kSW;
        if (i < n2) w[i] = wv[e];
    }
    __syncthreads();
    if (threadIdx.x == 0) givens_finish(gm, flag, hc, gm->H + (size_t)j * (M + 1), sqrt(nn), j, M, tol);
    if (fin) {
        __syncthreads();                  // the cycle state written by thread 0
        finish_body(n2, gm, fa, 0, 1, threadIdx.x, kSW, threadIdx.x == 0);
    }
}

// x += sum_l y[l] V[l]   (l < cycle length)
__global__ void k_gm_update_x(int n2, const double* __restrict__ V, const GmState* __restrict__ gm,
                              double* __restrict__ x) {   // V: the stored M v_l (or v_l)
    const int jj = gm->cycle_iters;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
        double s = x[i];
        for (int l = 0; l < jj; ++l) s = fma(gm->y[l], V[(size_t)l * n2 + i], s);
        x[i] = s;
    }
}

// ------------------------------------------------------------ ring / misc ---
// x0 = 2 w_{k-1} - w_{k-2} (or w_{k-1}, or 0) from the ring
__global__ void k_warm_start(int n2, const int* __restrict__ dk, int nh,
                             const double* __restrict__ ring, double* __restrict__ x,
                             const GmState* __restrict__ gm) {
    if (gm->halt) return;
    const int k = *dk;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (k >= 3 && nh >= 2) {
            v = 2.0 * ring[(size_t)((k - 1) % nh) * n2 + i] - ring[(size_t)((k - 2) % nh) * n2 + i];
        } else if (k >= 2) {
            v = ring[(size_t)((k - 1) % nh) * n2 + i];
        }
        x[i] = v;
    }
}

// ring[k mod nh] = x ; hist[k-1] = x (if hist)
__global__ void k_push(int n2, const int* __restrict__ dk, int nh, const double* __restrict__ x,
                       double* __restrict__ ring, double* __restrict__ hist, int hist_cap) {
    const int k = *dk;
    double* slot = ring + (size_t)(k % nh) * n2;
    double* hs = (hist && k - 1 < hist_cap) ? hist + (size_t)(k - 1) * n2 : nullptr;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
        double v = x[i];
        slot[i] = v;
        if (hs) hs[i] = v;
    }
}

__global__ void k_inc_step(int* dk, const GmState* __restrict__ gm) {
    if (!gm->halt) *dk += 1;
}

__global__ void k_clear_halt(GmState* gm) { gm->halt = 0; }

__global__ void k_set_step(int* dk, int k) { *dk = k; }

// recovery gather: columns (step s in [s0, s1), half h, kind t, rhs r) of
// X[ne][ncol], kind 0 = u_k, kind 1 = u_k - u_{k-1} (u_0 = 0)
__global__ void k_rec_gather(int ne, int hs, int n2, int R, int Rp, int s0, int ns,
                             const double* __restrict__ hist, double* __restrict__ X) {
    const int ncol = ns * 4 * R;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int m = blockIdx.y;
    if (c >= ncol) return;
    int r = c % R, t = (c / R) % 2, hh = (c / (2 * R)) % 2, s = c / (4 * R);
    int step = s0 + s;     // 0-based index into hist
    size_t off = (size_t)(hh * hs + m) * Rp + r;
    double v = hist[(size_t)step * n2 * Rp + off];
    if (t == 1 && step > 0) v -= hist[(size_t)(step - 1) * n2 * Rp + off];
    X[(size_t)m * ncol + c] = v;
}

// loop = u - P^Sigma u ; star = (Tmax/dt) P^Sigma (u_k - u_{k-1}); outputs [ns][n][R] packed (n = 2 ne)
__global__ void k_rec_scatter(int ne, int R, int ns, const double* __restrict__ X,
                              const double* __restrict__ PX, double scale, double* __restrict__ loop,
                              double* __restrict__ star) {
    const int ncol = ns * 4 * R;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int m = blockIdx.y;
    if (c >= ncol) return;
    int r = c % R, t = (c / R) % 2, hh = (c / (2 * R)) % 2, s = c / (4 * R);
    size_t o = ((size_t)s * 2 * ne + (size_t)hh * ne + m) * R + r;
    double px = PX[(size_t)m * ncol + c];
    if (t == 0) {
        if (loop) loop[o] = X[(size_t)m * ncol + c] - px;
    } else {
        if (star) star[o] = scale * px;
    }
}

// pack w from the internal padded layout [n2][R] to [n][R]
__global__ void k_pack(int ne, int hs, int R, int Rp, int ns, const double* __restrict__ src,
                       double* __restrict__ dst) {
    size_t total = (size_t)ns * 2 * ne * R;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int r = (int)(t % R);
        size_t q = t / R;
        int i = (int)(q % (2 * ne));
        size_t s = q / (2 * ne);
        int row = i < ne ? i : hs + (i - ne);
        dst[t] = src[(s * 2 * hs + row) * Rp + r];
    }
}

}  // namespace

// ------------------------------------------------------------ launchers ---
namespace motk_step {

// RHS of steps k0 .. k0+B-1: fields, then r = C1 ebar + C2 Ebar / T_max per half.
// kbase: read k0 from the device when the launches are replayed from a graph
// (k0 then only selects the half of rb, by its batch parity).
void rhs_batch(mot_handle* h, int k0, double* rb, const int* kbase) {
    const int ne = h->ne, hs = h->hs, B = h->B, Rp = h->Rp;
    const int N = B * Rp;
    size_t tot = (size_t)ne * N;
    hipLaunchKernelGGL(k_rhs_fields, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream, ne, hs, k0, kbase,
                       B, h->R, Rp, h->dt, h->rq_x, h->rq_f, h->waves, h->tcut, h->ebar, h->Ebar, h->gm);
    // consecutive batches alternate between the two halves of rb, so a batch
    // queued ahead of a halted step never overwrites the one it still needs
    double* rbk = rb + (size_t)(((k0 - 1) / B) & 1) * 2 * ne * N;
    // both halves (u and v) in one launch per factor
    motk::gemm(h->stream, ne, N, ne, 1.0, h->C1, hs, h->ebar, N, 0.0, rbk, N, 2, (size_t)hs * N, (size_t)ne * N);
    motk::gemm(h->stream, ne, N, ne, 1.0 / h->Tmax, h->C2, hs, h->Ebar, N, 1.0, rbk, N, 2, (size_t)hs * N,
               (size_t)ne * N);
}

void history(mot_handle* h) {
    const int sc = h->sch_hist;
    if (sc == 11 || sc == 22 || sc == 24) {
        const int w = sc == 11 ? 1 : sc - 20, rpb = 4 / w;
        hipLaunchKernelGGL(k_history_co, dim3((h->ne + rpb - 1) / rpb), dim3(256), 0, h->stream, h->ne, h->hs,
                           h->d_k, h->nh, h->Q, h->ring, h->rb, h->B, h->y, h->gm, w);
        return;
    }
    if (sc > 10) {
        // 12, 14: one wavefront per r rows; 32, 34: r wavefronts share r rows
        const int r = sc % 10, cs = sc > 30 ? r : 1;
#define L_(R_) hipLaunchKernelGGL(k_history_rows<R_>, dim3((h->ne + R_ - 1) / R_), dim3(64 * cs), 0, h->stream, \
                                  h->ne, h->hs, h->d_k, h->nh, h->Q, h->ring, h->rb, h->B, h->y, h->gm, cs)
        if (r == 4) L_(4); else L_(2);
#undef L_
        return;
    }
    const int rpb = 4 / sc;
    hipLaunchKernelGGL(k_history, dim3((h->ne + rpb - 1) / rpb), dim3(256), 0, h->stream, h->ne, h->hs, h->d_k,
                       h->nh, h->Q, h->ring, h->rb, h->B, h->y, sc, h->gm);
}

void gm_start1(mot_handle* h, const double* b, double* r, int have_t, int first, double* xzero, int publish) {
    hipLaunchKernelGGL(k_gm_start1, dim3(1), dim3(kSW), 0, h->stream, h->n2, b, r, have_t, h->gm,
                       publish ? h->dflag : nullptr, h->opt.gmres_tol, first, xzero);
}

static FinArgs fin_args(mot_handle* h, const double* basis, int kq) {
    return FinArgs{basis, h->x, h->d_k, h->nh, h->ring, h->hist, h->hist_cap, kq};
}

// fin_kq != 0: also the speculative finisher of queued step fin_kq (as gm_finish
// with spec = 1), in the same workgroup
void gm_orth1(mot_handle* h, double* w, int publish, int fin_kq) {
    const int ept = (h->n2 + kSW - 1) / kSW;
    const FinArgs fa = fin_args(h, h->Z, fin_kq);
    const int fin = fin_kq != 0;
#define L_(E_) hipLaunchKernelGGL(k_gm_orth1<E_>, dim3(1), dim3(kSW), 0, h->stream, h->n2, h->V, w, h->gm, \
                                  publish ? h->dflag : nullptr, h->opt.gmres_tol, h->M, fin, fa)
    if (ept <= 2) L_(2);
    else if (ept <= 4) L_(4);
    else if (ept <= 8) L_(8);
    else if (ept <= 16) L_(16);
    else L_(32);
#undef L_
}

void gm_finish(mot_handle* h, const double* basis, int force, int spec, int kq) {
    hipLaunchKernelGGL(k_gm_finish, dim3((h->n2 + 255) / 256), dim3(256), 0, h->stream, h->n2, h->gm,
                       fin_args(h, basis, kq), force, spec);
}

void q0_matvec(mot_handle* h, const double* src, double* vout, double* y, int check_done, int use_inv) {
    const int sc = h->sch_q0;
    if (sc > 10) {
        // 12, 14, 18: one wavefront per r rows; 32, 34: r wavefronts share r rows
        const int r = sc % 10, cs = sc > 30 ? r : 1;
#define L_(R_) hipLaunchKernelGGL(k_q0_rows<R_>, dim3((h->ne + R_ - 1) / R_), dim3(64 * cs), 0, h->stream, h->ne, \
                                  h->hs, h->Q, src, vout, y, h->gm, check_done, use_inv, cs)
        if (r == 8) L_(8); else if (r == 4) L_(4); else if (r == 2) L_(2); else L_(1);
#undef L_
        return;
    }
    const int rpb = 4 / sc;
    hipLaunchKernelGGL(k_q0_matvec, dim3((h->ne + rpb - 1) / rpb), dim3(256), 0, h->stream, h->ne, h->hs, h->Q,
                       src, vout, y, h->gm, check_done, use_inv, sc);
}

// start: src is the step's right-hand side and the launch opens the cold
// GMRES cycle (FP64 approximate inverse only)
void precond(mot_handle* h, const double* src, double* vj, double* z, bool start) {
    const int sc = h->sch_pc;
    const int st = start && !h->M32;
    const double tol = h->opt.gmres_tol;
    if (sc > 10) {
        const int r = sc % 10, cs = sc > 30 ? r : 1;
#define L_(T_, R_, M_) hipLaunchKernelGGL((k_precond_rows<T_, R_>), dim3((h->n2 + R_ - 1) / R_), dim3(64 * cs), 0, \
                                          h->stream, h->n2, M_, src, vj, z, h->gm, st, tol, h->x, cs)
#define P_(R_) do { if (h->M32) L_(float, R_, h->M32); else L_(double, R_, h->M64); } while (0)
        if (r == 8) P_(8); else if (r == 4) P_(4); else if (r == 2) P_(2); else P_(1);
#undef P_
#undef L_
        return;
    }
    const int rpb = 4 / sc;
    dim3 grid((h->n2 + rpb - 1) / rpb);
    if (h->M32)
        hipLaunchKernelGGL(k_precond<float>, grid, dim3(256), 0, h->stream, h->n2, h->M32, src, vj, z, h->gm, sc, 0,
                           tol, h->x);
    else
        hipLaunchKernelGGL(k_precond<double>, grid, dim3(256), 0, h->stream, h->n2, h->M64, src, vj, z, h->gm, sc, st,
                           tol, h->x);
}

void dense_q0(mot_handle* h, double* D) {
    hipLaunchKernelGGL(k_dense_q0, dim3(4096), dim3(256), 0, h->stream, h->ne, h->hs, h->Q, D);
}

void transpose_scale(mot_handle* h, int n, double alpha, const double* A, double* X) {
    hipLaunchKernelGGL(k_transpose_scale, dim3((n + 31) / 32, (n + 31) / 32), dim3(32, 8), 0, h->stream, n, alpha, A, X);
}

void abs_sums(mot_handle* h, int n, const double* A, double* rs, double* cs) {
    hipLaunchKernelGGL(k_abs_sums, dim3((n + 255) / 256), dim3(256), 0, h->stream, n, A, rs, cs);
}

void eye_residual(mot_handle* h, int n, const double* T, double* out) {
    hipLaunchKernelGGL(k_eye_residual, dim3(2048), dim3(256), 0, h->stream, n, T, out);
}

void to_f32(mot_handle* h, size_t n, const double* X, float* Y) {
    hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(256), 0, h->stream, n, X, Y);
}

void gm_residual(mot_handle* h, const double* b, double* r, int first) {
    hipLaunchKernelGGL(k_gm_residual, dim3(MOT_GM_BLOCKS), dim3(256), 0, h->stream, h->n2, b, r, h->gm,
                       h->dflag, h->opt.gmres_tol, first);
}

void gm_dots(mot_handle* h, const double* w) {
    hipLaunchKernelGGL(k_gm_dots, dim3(MOT_GM_BLOCKS), dim3(256), 0, h->stream, h->n2, h->V, w, h->gm);
}

void gm_orth(mot_handle* h, double* w, int final_pass) {
    hipLaunchKernelGGL(k_gm_orth, dim3(MOT_GM_BLOCKS), dim3(256), 0, h->stream, h->n2, h->V, w, h->gm,
                       h->dflag, h->opt.gmres_tol, h->M, final_pass);
}

void gm_update_x(mot_handle* h, const double* basis, double* x) {
    hipLaunchKernelGGL(k_gm_update_x, dim3((h->n2 + 255) / 256), dim3(256), 0, h->stream, h->n2, basis,
                       h->gm, x);
}

void warm_start(mot_handle* h) {
    hipLaunchKernelGGL(k_warm_start, dim3((h->n2 + 255) / 256), dim3(256), 0, h->stream, h->n2, h->d_k,
                       h->nh, h->ring, h->x, h->gm);
}

void push(mot_handle* h) {
    hipLaunchKernelGGL(k_push, dim3((h->n2 + 255) / 256), dim3(256), 0, h->stream, h->n2, h->d_k, h->nh,
                       h->x, h->ring, h->hist, h->hist_cap);
}

void inc_step(mot_handle* h) { hipLaunchKernelGGL(k_inc_step, dim3(1), dim3(1), 0, h->stream, h->d_k, h->gm); }

void clear_halt(mot_handle* h) { hipLaunchKernelGGL(k_clear_halt, dim3(1), dim3(1), 0, h->stream, h->gm); }

void set_step(mot_handle* h, int k) { hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, h->stream, h->d_k, k); }

// first step of a window replayed from a graph
void set_base(mot_handle* h, int k) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, h->stream, h->d_k + 1, k);
}

void rec_gather(mot_handle* h, int s0, int ns, double* X) {
    int ncol = ns * 4 * h->R;
    dim3 grid((ncol + 255) / 256, h->ne);
    hipLaunchKernelGGL(k_rec_gather, grid, dim3(256), 0, h->stream, h->ne, h->hs, h->n2, h->R, h->Rp, s0, ns,
                       h->hist, X);
}

void rec_scatter(mot_handle* h, int ns, const double* X, const double* PX, double* loop, double* star) {
    int ncol = ns * 4 * h->R;
    dim3 grid((ncol + 255) / 256, h->ne);
    hipLaunchKernelGGL(k_rec_scatter, grid, dim3(256), 0, h->stream, h->ne, h->R, ns, X, PX,
                       h->Tmax / h->dt, loop, star);
}

void pack(mot_handle* h, int ns, const double* src, double* dst) {
    size_t total = (size_t)ns * 2 * h->ne * h->R;
    int nb = (int)((total + 255) / 256);
    if (nb > 65535 * 8) nb = 65535 * 8;
    hipLaunchKernelGGL(k_pack, dim3(nb), dim3(256), 0, h->stream, h->ne, h->hs, h->R, h->Rp, ns, src, dst);
}

}  // namespace motk_step
