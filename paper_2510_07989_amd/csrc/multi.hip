// Multi-right-hand-side march: the R plane waves of one scatterer share every
// lag matrix, so the history convolution and the Q_0 products become
// tall-skinny GEMMs [ne x hs] x [hs x RP] (RP = R rounded up to a power of two).
// Vectors are [n2][RP] (column index fastest).
//
// Tile-major lag storage.  Each ne x hs block of Q_j (q1, qk, q2, with
// Q_j = [[q1, -qk], [qk, q2]]) is cut into 16 x 16 tiles; tile (g, c) holds rows
// 16g..16g+15 and summation indices 16c..16c+15, tiles stored g-major
// (index g * KT + c), 256 entries each, zero beyond ne.  Inside a tile, lane l
// of a wavefront owns row 16g + l%16 and indices 16c + 4(l/16) + e, e = 0..3:
//   FP32 entry (l, e) at l*4 + e                 (one 16-byte load per lane)
//   FP64 entry (l, e) at (e/2)*128 + l*2 + e%2   (two 16-byte loads per lane)
// so one wavefront reads each tile as contiguous 1 KB pieces.  The 16x16x4
// MFMAs take A as lane l = row l%16, summation slot l/16; slot l/16 of MFMA e is
// index 4(l/16) + e here, and the B operand (the history vector, from LDS) is
// read with the same permutation, so the product is unchanged.
// Operand layout, measured on gfx950: B lane l = column l%16, slot l/16 for
// both MFMAs; result register r of lane l holds column l%16 and row
//   4(l/16) + r   for v_mfma_f32_16x16x4f32,
//   l/16 + 4r     for v_mfma_f64_16x16x4f64.
#include "mot_internal.h"

#include <algorithm>

namespace {


__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// y = rb(step) - sum of history partials     (hist = 1)
// y = sum of partials                         (hist = 0, Q_0 product)
template <int RP>
__global__ void k_struct_reduce(int ne, int hs, const int* __restrict__ dk, int nh, int q0_mode, int KC,
                                const double* __restrict__ part, const double* __restrict__ rb, int B,
                                double* __restrict__ y, const GmState* __restrict__ agg) {
    if (agg->halt) return;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * RP) return;
    const int m = t / RP, c = t % RP;
    const int k = *dk;
    const int nact = q0_mode ? 1 : (k - 1 < nh ? k - 1 : nh);
    // four interleaved partial sums keep several loads in flight
    double su4[4] = {0, 0, 0, 0}, sv4[4] = {0, 0, 0, 0};
    const int np = nact * KC;
    const size_t stride = (size_t)2 * ne * RP;
    const double* Pu = part + (size_t)m * RP + c;
    const double* Pv = part + (size_t)(ne + m) * RP + c;
#pragma unroll 4
    for (int p = 0; p < np; ++p) {
        su4[p & 3] += Pu[(size_t)p * stride];
        sv4[p & 3] += Pv[(size_t)p * stride];
    }
    const double su = (su4[0] + su4[1]) + (su4[2] + su4[3]);
    const double sv = (sv4[0] + sv4[1]) + (sv4[2] + sv4[3]);
    if (q0_mode) {
        y[(size_t)m * RP + c] = su;
        y[(size_t)(hs + m) * RP + c] = sv;
    } else {
        const int sc = (k - 1) % B;
        const size_t ld = (size_t)B * RP;
        rb += (size_t)(((k - 1) / B) & 1) * 2 * ne * ld;   // double-buffered batches
        y[(size_t)m * RP + c] = rb[(size_t)m * ld + (size_t)sc * RP + c] - su;
        y[(size_t)(hs + m) * RP + c] = rb[(size_t)ne * ld + (size_t)m * ld + (size_t)sc * RP + c] - sv;
    }
}

template <int RP>
__global__ void k_plain_reduce(int n, int KC, const double* __restrict__ part, const double* __restrict__ src,
                               const GmState* __restrict__ gms, const GmState* __restrict__ agg,
                               double* __restrict__ z, double* __restrict__ vj) {
    if (agg->done || agg->halt) return;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * RP) return;
    const int m = t / RP, c = t % RP;
    double s = 0;
    for (int p = 0; p < KC; ++p) s += part[(size_t)p * n * RP + (size_t)m * RP + c];
    const double sc = gms[c].inv_h;
    z[t] = sc * s;
    vj[t] = sc * src[t];
}

__device__ __forceinline__ double bsum(double v, double* sh) {
    v = wsum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    __syncthreads();
    return s;
}

// Combine the column states into the aggregate state and publish one word.
// Called by every thread of one workgroup: threads c < RP read column c (the
// states are far apart in memory, so the reads go out together), thread 0
// combines them from LDS.
__device__ void aggregate(int RP, int R, GmState* gms, GmState* agg, GmFlag* flag, int arnoldi) {
    __shared__ int s_done[64], s_conv[64], s_total[64];
    __shared__ double s_rel[64];
    const int c = threadIdx.x;
    if (c < RP) {
        const GmState* g = gms + c;
        s_done[c] = g->done;
        s_conv[c] = g->converged;
        s_total[c] = g->total;
        s_rel[c] = g->relres;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int done = 1, conv = 1, total = 0;
        double rel = 0;
        for (int q = 0; q < RP; ++q) {
            done &= s_done[q];
            conv &= s_conv[q];
            if (q < R) { total = max(total, s_total[q]); rel = fmax(rel, s_rel[q]); }
        }
        if (arnoldi) agg->iters_all += 1;
        agg->done = done;
        agg->converged = done && conv;
        agg->total = total;
        agg->relres = rel;
        agg->counter = 0;
        const int seq = agg->seq + 1;
        agg->seq = seq;
        if (flag) {               // null: queued steps, nobody waits on the host
            flag->relres = rel;
            flag->converged = done && conv;
            flag->done = done;
            flag->total = total;
            __threadfence_system();
            flag->seq = seq;
        }
    }
}

__device__ __forceinline__ bool last_of_grid(unsigned int* counter) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

// one workgroup per column: r = y - t (or y), beta, bnorm; x = 0 when cold
// Start and Arnoldi steps for all columns at once.  Workgroups own ranges of
// RB rows and all RP columns (thread t: column t % RP, rows t / RP, t / RP +
// 256 / RP, ...: consecutive threads read consecutive addresses); each sweep
// writes per-workgroup column sums to part[block][l][c], and the last
// workgroup of the grid adds them in block order (deterministic) and carries
// the per-column state.
__device__ __forceinline__ void col_sums(double s, int RP, double* red, double* out) {
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < RP) {
        double a = 0.0;
        for (int k = threadIdx.x; k < 256; k += RP) a += red[k];
        out[threadIdx.x] = a;
    }
    __syncthreads();
}

// In the last workgroup: the sum over workgroups b of part[b][l][c] for one l
// and every column, spread over all 256 threads (256 / RP per column, then a
// fixed-order sum in LDS); threads c < RP get column c's value.
__device__ __forceinline__ double grid_col_sum(const double* __restrict__ part, int nb, int RP, int l,
                                               double* red) {
    const int c = threadIdx.x % RP, q = threadIdx.x / RP, nq = 256 / RP;
    double a = 0.0;
    for (int b = q; b < nb; b += nq) a += part[((size_t)b * (MOT_MAXM + 1) + l) * RP + c];
    red[threadIdx.x] = a;
    __syncthreads();
    double s = 0.0;
    if ((int)threadIdx.x < RP)
        for (int k = 0; k < nq; ++k) s += red[threadIdx.x + k * RP];
    __syncthreads();
    return s;
}

// r = y - t (have_t) or y; x = 0 (xzero); beta = ||r||, ||y|| per column.
__global__ __launch_bounds__(256) void k_gmb_start(int n2, int RP, int R, int RB, const double* __restrict__ y,
                                                   double* __restrict__ r, int have_t, GmState* gms,
                                                   GmState* agg, GmFlag* flag, double tol, int first,
                                                   double* __restrict__ xzero, double* __restrict__ part) {
    if (agg->halt) return;
    __shared__ double red[256];
    const int c = threadIdx.x % RP, r0 = threadIdx.x / RP, stride = 256 / RP;
    const int i0 = blockIdx.x * RB, i1 = min(n2, i0 + RB);
    double s1 = 0, s2 = 0, t1 = 0, t2 = 0;      // plain and scaled sums of squares
    for (int i = i0 + r0; i < i1; i += stride) {
        const size_t o = (size_t)i * RP + c;
        if (xzero) xzero[o] = 0.0;
        const double bi = y[o];
        const double ri = have_t ? bi - r[o] : bi;
        r[o] = ri;
        s1 = fma(ri, ri, s1);
        s2 = fma(bi, bi, s2);
        t1 += sq_scaled(ri);
        t2 += sq_scaled(bi);
    }
    double* P = part + (size_t)blockIdx.x * (MOT_MAXM + 1) * RP;
    col_sums(s1, RP, red, P);
    col_sums(s2, RP, red, P + RP);
    col_sums(t1, RP, red, P + 2 * RP);
    col_sums(t2, RP, red, P + 3 * RP);
    if (!last_of_grid(&agg->counter)) return;
    // part[b][l][c], l = 0, 1: plain sums of r and y; 2, 3: scaled sums
    const double a1 = grid_col_sum(part, gridDim.x, RP, 0, red);
    const double a2 = grid_col_sum(part, gridDim.x, RP, 1, red);
    const double b1 = grid_col_sum(part, gridDim.x, RP, 2, red);
    const double b2 = grid_col_sum(part, gridDim.x, RP, 3, red);
    if ((int)threadIdx.x < RP) {
        GmState* g = gms + c;
        const double beta = open_norm(a1, b1);
        if (first) { g->bnorm = open_norm(a2, b2); g->total = 0; }
        g->beta = beta;
        g->g[0] = beta;
        g->j = 0;
        g->cycle_iters = 0;
        const double bn = g->bnorm;
        g->relres = bn > 0 ? beta / bn : 0.0;
        const int conv = (bn <= MOT_ZERO_NORM) || (beta <= MOT_ZERO_NORM) || (beta <= tol * bn);
        g->converged = conv;
        g->done = conv;
        g->inv_h = beta > MOT_ZERO_NORM ? 1.0 / beta : 0.0;
    }
    __syncthreads();
    if (first && threadIdx.x == 0) agg->seq = 0;
    __syncthreads();
    aggregate(RP, R, gms, agg, flag, 0);
}

// Arnoldi step, classical Gram-Schmidt with one re-orthogonalisation, in three
// sweeps over w (the new Krylov vector, in place) and the basis V_0..V_j:
//   1: h1_l = <V_l, w>
//   2: w -= sum_l h1_l V_l;  h2_l = <V_l, w>
//   3: w -= sum_l h2_l V_l;  ||w||, then H column, Givens, residual estimate.
// Columns whose cycle is done are left as they are.
__global__ __launch_bounds__(256) void k_gmb_orth(int n2, int RP, int R, int RB, int sweep,
                                                  const double* __restrict__ V, double* __restrict__ w,
                                                  GmState* gms, GmState* agg, GmFlag* flag, double tol, int M,
                                                  double* __restrict__ part) {
    // once every column is done the sweeps do no arithmetic, but the third
    // still publishes a progress word (the host-driven solve waits for one
    // word per Arnoldi step)
    if (agg->halt) return;
    __shared__ double red[256];
    __shared__ int jmax_s;
    const int c = threadIdx.x % RP, r0 = threadIdx.x / RP, stride = 256 / RP;
    GmState* g = gms + c;
    const bool active = !agg->done && !g->done;
    const int jc = active ? g->j : -1;
    __shared__ int s_j[64];
    if ((int)threadIdx.x < RP) s_j[threadIdx.x] = active ? jc : -1;
    __syncthreads();
    if (threadIdx.x == 0) {
        int jm = -1;
        for (int q = 0; q < RP; ++q) jm = max(jm, s_j[q]);
        jmax_s = jm;
    }
    __syncthreads();
    const int J = jmax_s;
    const int i0 = blockIdx.x * RB, i1 = min(n2, i0 + RB);
    const size_t vs = (size_t)n2 * RP;
    double* P = part + (size_t)blockIdx.x * (MOT_MAXM + 1) * RP;
    if (sweep > 1 && active) {
        const double* h = sweep == 2 ? g->h1 : g->h2;
        for (int i = i0 + r0; i < i1; i += stride) {
            const size_t o = (size_t)i * RP + c;
            double x = w[o];
            for (int l = 0; l <= jc; ++l) x = fma(-h[l], V[l * vs + o], x);
            w[o] = x;
        }
    }
    if (sweep < 3) {
        for (int l = 0; l <= J; ++l) {
            double s = 0;
            if (active && l <= jc)
                for (int i = i0 + r0; i < i1; i += stride) {
                    const size_t o = (size_t)i * RP + c;
                    s = fma(V[l * vs + o], w[o], s);
                }
            col_sums(s, RP, red, P + (size_t)l * RP);
        }
    } else {
        double s = 0;
        if (active)
            for (int i = i0 + r0; i < i1; i += stride) {
                const double x = w[(size_t)i * RP + c];
                s = fma(x, x, s);
            }
        col_sums(s, RP, red, P);
    }
    if (!last_of_grid(&agg->counter)) return;
    if (sweep < 3) {
        for (int l = 0; l <= J; ++l) {
            const double a = grid_col_sum(part, gridDim.x, RP, l, red);
            if ((int)threadIdx.x < RP && active && l <= jc) (sweep == 1 ? g->h1 : g->h2)[l] = a;
        }
    }
    const double nn = sweep == 3 ? grid_col_sum(part, gridDim.x, RP, 0, red) : 0.0;
    if ((int)threadIdx.x < RP && active) {
        if (sweep == 3) {
            const int j = jc;
            const double hn = sqrt(nn);
            double* col = g->H + (size_t)j * (M + 1);
            // rotation l touches entries l and l + 1: entry l is final after
            // it, entry l + 1 is carried (no local array in scratch memory)
            double carry = g->h1[0] + g->h2[0];
            for (int l = 0; l < j; ++l) {
                const double a = carry, b = g->h1[l + 1] + g->h2[l + 1];
                col[l] = g->cs[l] * a + g->sn[l] * b;
                carry = -g->sn[l] * a + g->cs[l] * b;
            }
            double a = carry, b = hn;
            double rr = hypot(a, b);
            double cs = rr > 0 ? a / rr : 1.0, sn = rr > 0 ? b / rr : 0.0;
            col[j] = rr;
            col[j + 1] = 0.0;
            g->cs[j] = cs;
            g->sn[j] = sn;
            double gj = g->g[j];
            g->g[j] = cs * gj;
            g->g[j + 1] = -sn * gj;
            const int jn = j + 1;
            g->j = jn;
            g->cycle_iters = jn;
            g->total += 1;
            double rel = g->bnorm > 0 ? fabs(g->g[jn]) / g->bnorm : 0.0;
            g->relres = rel;
            int conv = rel <= tol;
            int brk = !(hn > 1e-300 * (g->beta + 1e-300));
            g->converged = conv || brk;
            g->done = conv || brk || jn >= M;
            g->inv_h = hn > 0 ? 1.0 / hn : 0.0;
            if (g->done) {
                for (int i = jn - 1; i >= 0; --i) {
                    double s2 = g->g[i];
                    for (int l = i + 1; l < jn; ++l) s2 -= g->H[(size_t)l * (M + 1) + i] * g->y[l];
                    double d = g->H[(size_t)i * (M + 1) + i];
                    g->y[i] = d != 0 ? s2 / d : 0.0;
                }
            }
        }
    }
    __syncthreads();
    if (sweep == 3) aggregate(RP, R, gms, agg, flag, 1);
    else if (threadIdx.x == 0) agg->counter = 0;
}

// x[:, c] += sum_l y_l(c) Z_l[:, c] for columns whose cycle is done (once per
// cycle: cycle_iters is consumed); push x into the ring and history when every
// column converged, or when forced.
// spec = 1 (speculative stepping): unless every column has converged, push
// nothing and raise the halt word, so that later queued steps do nothing.
__global__ void k_gmb_finish(int n2, int RP, const double* __restrict__ Z, GmState* gms,
                             GmState* __restrict__ agg, double* __restrict__ x,
                             int* __restrict__ dk, int nh, double* __restrict__ ring,
                             double* __restrict__ hist, int hist_cap, int force, int spec, int kq) {
    if (agg->halt) return;
    // kq > 0 (queued steps): host step index; kq < 0 (graph replay): the
    // window's first step dk[1] plus -kq - 1; the counter dk[0] is set to k + 1
    // after a push (no block of this launch reads it)
    const int k = kq > 0 ? kq : (kq < 0 ? dk[1] - kq - 1 : dk[0]);
    if (spec && !agg->converged) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            agg->halt_k = k;
            agg->halt = 1;
        }
        return;
    }
    const int push = agg->converged || force;
    if (kq != 0 && push && blockIdx.x == 0 && threadIdx.x == 0) dk[0] = k + 1;
    double* slot = ring + (size_t)(k % nh) * n2 * RP;
    double* hs = (hist && k - 1 < hist_cap) ? hist + (size_t)(k - 1) * n2 * RP : nullptr;
    const size_t total = (size_t)n2 * RP;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(t % RP);
        const GmState* g = gms + c;
        double s = x[t];
        if (g->done)
            for (int l = 0; l < g->cycle_iters; ++l) s = fma(g->y[l], Z[(size_t)l * total + t], s);
        x[t] = s;
        if (push) {
            slot[t] = s;
            if (hs) hs[t] = s;
        }
    }
}

// after a finish: mark consumed cycles (so a restart does not add them twice)
__global__ void k_gmb_consume(int RP, GmState* gms, const GmState* __restrict__ agg) {
    if (agg->halt) return;
    int c = threadIdx.x;
    if (c < RP && gms[c].done) gms[c].cycle_iters = 0;
}

// ---------------------------------------------------------------- tiles ---
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

__host__ __device__ inline size_t tile_pos64(int lane, int e) { return (size_t)(e >> 1) * 128 + lane * 2 + (e & 1); }
__host__ __device__ inline size_t tile_pos32(int lane, int e) { return (size_t)lane * 4 + e; }

// Pack one ne x hs row-major block into tiles: FP64 (hi64), or FP32 hi = fl(v)
// and, when lo is given, lo = fl(v - hi).
__global__ void k_pack_tiles(int ne, int hs, int G16, int KT, const double* __restrict__ src,
                             double* __restrict__ hi64, float* __restrict__ hi32, float* __restrict__ lo32) {
    const size_t total = (size_t)G16 * KT * 256;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
        const size_t tile = p / 256;
        const int in = (int)(p % 256);
        const int g = (int)(tile / KT), c = (int)(tile % KT);
        int lane, e;
        if (hi64) { lane = (in & 127) >> 1; e = ((in >> 7) << 1) | (in & 1); }
        else { lane = in >> 2; e = in & 3; }
        const int row = g * 16 + (lane & 15), kk = c * 16 + 4 * (lane >> 4) + e;
        const double v = (row < ne && kk < ne) ? src[(size_t)row * hs + kk] : 0.0;
        if (hi64) {
            hi64[p] = v;
        } else {
            const float h = (float)v;
            hi32[p] = h;
            if (lo32) lo32[p] = (float)(v - (double)h);
        }
    }
}

__device__ __forceinline__ void load_tile(const double* __restrict__ t, int lane, double a[4]) {
    const v2d x = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(t) + lane);
    const v2d y = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(t + 128) + lane);
    a[0] = x[0]; a[1] = x[1]; a[2] = y[0]; a[3] = y[1];
}
__device__ __forceinline__ void load_tile(const float* __restrict__ t, int lane, double a[4]) {
    const v4f x = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(t) + lane);
    a[0] = x[0]; a[1] = x[1]; a[2] = x[2]; a[3] = x[3];
}

// A tile triple (q1, qk, q2) as loaded, before any conversion: a prefetch into
// these registers stays in flight until its tile is unpacked.
template <typename T> struct RawTiles;
template <> struct RawTiles<double> {
    v2d x1, y1, xk, yk, x2, y2;
};
template <> struct RawTiles<float> {
    v4f t1, tk, t2;                    // FP32 entries
    v4f l1, lk, l2;                    // their FP32 low parts (lags with a low part)
};

__device__ __forceinline__ void fetch_raw(const double* __restrict__ a1, const double* __restrict__ ak,
                                          const double* __restrict__ a2, const float*, size_t, bool, int lane,
                                          RawTiles<double>& r) {
    r.x1 = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(a1) + lane);
    r.y1 = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(a1 + 128) + lane);
    r.xk = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(ak) + lane);
    r.yk = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(ak + 128) + lane);
    r.x2 = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(a2) + lane);
    r.y2 = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(a2 + 128) + lane);
}

// lo: the low-part tile of q1 (those of qk and q2 follow at +tsz, +2 tsz)
__device__ __forceinline__ void fetch_raw(const float* __restrict__ a1, const float* __restrict__ ak,
                                          const float* __restrict__ a2, const float* __restrict__ lo, size_t tsz,
                                          bool hl, int lane, RawTiles<float>& r) {
    r.t1 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(a1) + lane);
    r.tk = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(ak) + lane);
    r.t2 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(a2) + lane);
    if (hl) {
        r.l1 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(lo) + lane);
        r.lk = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(lo + tsz) + lane);
        r.l2 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(lo + 2 * tsz) + lane);
    }
}

__device__ __forceinline__ void unpack(const RawTiles<double>& r, bool, double a1[4], double ak[4], double a2[4]) {
    a1[0] = r.x1[0]; a1[1] = r.x1[1]; a1[2] = r.y1[0]; a1[3] = r.y1[1];
    ak[0] = r.xk[0]; ak[1] = r.xk[1]; ak[2] = r.yk[0]; ak[3] = r.yk[1];
    a2[0] = r.x2[0]; a2[1] = r.x2[1]; a2[2] = r.y2[0]; a2[3] = r.y2[1];
}

// entry = FP64(hi) + FP64(lo) on lags with a low part
__device__ __forceinline__ void unpack(const RawTiles<float>& r, bool hl, double a1[4], double ak[4], double a2[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        a1[e] = r.t1[e];
        ak[e] = r.tk[e];
        a2[e] = r.t2[e];
        if (hl) {
            a1[e] += (double)r.l1[e];
            ak[e] += (double)r.lk[e];
            a2[e] += (double)r.l2[e];
        }
    }
}

// Structured product on FP64 MFMA for one 64-row block (4 wavefronts x 16
// rows), one lag and one K chunk:
//   Yu = q1 Wu - qk Wv,   Yv = qk Wu + q2 Wv
// Tiles in FP64 (plain path) or FP32 (mixed path, with an FP32 low part added
// in registers on lags 1..hilo); every product and sum in FP64, so the mixed
// path differs from FP64 only by the rounding of the stored entries.
// History (q0_mode 0): lag j = blockIdx.y + 1, At = tiles of lag 1, W = ring
// slot of w_{k-j}.  Q_0 (q0_mode 1): At = tiles of lag 0, W = X.
// Partial results part[(blockIdx.y * KC + kc)][2][ne][Rp].
// WG wavefronts per workgroup (4 or 8: 64 or 128 rows) share each staged slice
// of the history vectors: with 8, every slice read from L2 serves twice the
// rows.  The rows' sums are the same either way.
//
// One column block is bound by HBM, not by the matrix cores: there the
// compiler is held to three wavefronts per SIMD (accumulators in VGPRs, no
// AGPRs), so that more tile loads are in flight per CU than at the two its
// register-hungry schedule would allow.
template <typename T, int CB, int WG>
__global__ __launch_bounds__(64 * WG) __attribute__((amdgpu_waves_per_eu(CB == 1 ? 3 : 1)))
void k_tile_gemm(int ne, int hs, int G16, int KT, int Rp,
                                                   const int* __restrict__ dk, int nh, int q0_mode,
                                                   const T* __restrict__ At, const float* __restrict__ Alo,
                                                   int hilo, const double* __restrict__ ring,
                                                   const double* __restrict__ X, int KC,
                                                   double* __restrict__ part, const GmState* __restrict__ agg) {
    if (agg->halt) return;
    const int k = *dk;
    const int jj = blockIdx.y;
    const int nact = q0_mode ? 1 : (k - 1 < nh ? k - 1 : nh);
    if (jj >= nact) return;
    const int j = q0_mode ? 0 : jj + 1;
    const size_t tsz = (size_t)G16 * KT * 256;
    const T* a1p = At + (size_t)(q0_mode ? 0 : j - 1) * 3 * tsz;
    const T* akp = a1p + tsz;
    const T* a2p = a1p + 2 * tsz;
    const bool hl = Alo != nullptr && !q0_mode && j <= hilo;
    const float* l1p = hl ? Alo + (size_t)(j - 1) * 3 * tsz : nullptr;
    const double* W = q0_mode ? X : ring + (size_t)((k - j) % nh) * 2 * hs * Rp;
    const int kc = blockIdx.z;
    const int CT = (KT + KC - 1) / KC;
    const int c0 = kc * CT, c1 = min(KT, c0 + CT);

    constexpr int NC = CB * 16;                // columns staged
    constexpr int ST = CB >= 4 ? 2 : 4;        // tiles per staged slice
    constexpr int NT = 64 * WG;                // threads
    __shared__ double Ws[2][ST * 16][NC + 2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int g = blockIdx.x * WG + wv;
    const bool gok = g < G16;
    const int kq = 4 * (lane >> 4), cl = lane & 15;

    // two accumulator sets (even / odd e) give a single column block independent
    // MFMA chains; several column blocks already do
    constexpr int NS = CB == 1 ? 2 : 1;
    v4d Cu[CB][NS], Cv[CB][NS];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) Cu[cb][s2] = Cv[cb][s2] = (v4d){0.0, 0.0, 0.0, 0.0};

    // two tile triples in flight: tile t of the chunk sits in raw set t % 2 and
    // is converted only when it is multiplied, so its loads overlap the MFMAs
    // of the tile before (ST is even, so the set of a tile is ci % 2)
    RawTiles<T> rs[2];
    auto fetch = [&](int c, RawTiles<T>& r) {
        const size_t o = ((size_t)g * KT + c) * 256;
        fetch_raw(a1p + o, akp + o, a2p + o, hl ? l1p + o : nullptr, tsz, hl, lane, r);
    };
    if (gok && c0 < c1) fetch(c0, rs[0]);
    if (gok && c0 + 1 < c1) fetch(c0 + 1, rs[1]);

    // With one or two column blocks, or eight wavefronts, the history slice of
    // the next K step is loaded into registers while the current one is
    // multiplied, and stored to LDS after the barrier.  With four column
    // blocks in a four-wavefront workgroup those registers would halve the
    // occupancy (two workgroups per CU, whose barriers cover each other), so
    // the slice is loaded between the barriers; an eight-wavefront workgroup
    // fills a CU alone, and only the prefetch hides its slice loads.
    constexpr bool WPF = CB < 4 || WG == 8;
    constexpr int WE = ST * 16 * NC / NT;      // staged (u, v) pairs per thread
    double pu[WPF ? WE : 1], pv[WPF ? WE : 1];
    auto wfetch = [&](int cs) {
        const int nst = min(ST, c1 - cs);
#pragma unroll
        for (int q = 0; q < WE; ++q) {
            const int e = t + NT * q;
            const int col = e % NC, kk = e / NC;
            const int gk = cs * 16 + kk;
            pu[q] = pv[q] = 0.0;
            if (col < Rp && kk < nst * 16 && gk < hs) {
                pu[q] = W[(size_t)gk * Rp + col];
                pv[q] = W[(size_t)(hs + gk) * Rp + col];
            }
        }
    };
    if constexpr (WPF) {
        if (c0 < c1) wfetch(c0);
    }

    for (int cs = c0; cs < c1; cs += ST) {
        const int nst = min(ST, c1 - cs);
        if constexpr (WPF) {
#pragma unroll
            for (int q = 0; q < WE; ++q) {
                const int e = t + NT * q;
                Ws[0][e / NC][e % NC] = pu[q];
                Ws[1][e / NC][e % NC] = pv[q];
            }
        } else {
            for (int e = t; e < ST * 16 * NC; e += NT) {
                const int col = e % NC, kk = e / NC;
                const int gk = cs * 16 + kk;
                double wu = 0.0, wvv = 0.0;
                if (col < Rp && kk < nst * 16 && gk < hs) {
                    wu = W[(size_t)gk * Rp + col];
                    wvv = W[(size_t)(hs + gk) * Rp + col];
                }
                Ws[0][kk][col] = wu;
                Ws[1][kk][col] = wvv;
            }
        }
        __syncthreads();
        if constexpr (WPF) {
            if (cs + ST < c1) wfetch(cs + ST);
        }
#pragma unroll
        for (int ci = 0; ci < ST; ++ci) {
            if (ci >= nst) break;
            double a1[4], ak[4], a2[4];
            unpack(rs[ci & 1], hl, a1, ak, a2);
            if (gok && cs + ci + 2 < c1) fetch(cs + ci + 2, rs[ci & 1]);
            if (gok) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kk = ci * 16 + kq + e;
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const double wu = Ws[0][kk][cb * 16 + cl];
                        const double wvv = Ws[1][kk][cb * 16 + cl];
                        v4d& u = Cu[cb][e % NS];
                        v4d& v = Cv[cb][e % NS];
                        // u and v chains alternate (each keeps its own summation order)
                        u = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], wu, u, 0, 0, 0);
                        v = __builtin_amdgcn_mfma_f64_16x16x4f64(ak[e], wu, v, 0, 0, 0);
                        u = __builtin_amdgcn_mfma_f64_16x16x4f64(-ak[e], wvv, u, 0, 0, 0);
                        v = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[e], wvv, v, 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!gok) return;
    double* P = part + ((size_t)jj * KC + kc) * 2 * ne * Rp;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = cb * 16 + cl;
        if (col >= Rp) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = g * 16 + (lane >> 4) + 4 * r;
            if (row < ne) {
                double su = 0.0, sv = 0.0;
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2) { su += Cu[cb][s2][r]; sv += Cv[cb][s2][r]; }
                P[(size_t)row * Rp + col] = su;
                P[(size_t)(ne + row) * Rp + col] = sv;
            }
        }
    }
}

// Plain product z = M x with the approximate inverse of Q_0 stored in tiles
// (n x n, FP64 or FP32 entries, FP64 MFMA): one 64-row block and one K chunk
// per workgroup, partial results part[kc][n][Rp] (summed and scaled by
// k_plain_reduce).  Skipped once every column's GMRES is done.
template <typename T, int CB>
__global__ __launch_bounds__(256) void k_tile_plain(int n, int G16, int KT, int Rp, const T* __restrict__ At,
                                                    const double* __restrict__ X, int KC,
                                                    double* __restrict__ part, const GmState* __restrict__ agg) {
    if (agg->done || agg->halt) return;
    const int kc = blockIdx.z;
    const int CT = (KT + KC - 1) / KC;
    const int c0 = kc * CT, c1 = min(KT, c0 + CT);
    constexpr int NC = CB * 16;
    constexpr int ST = CB >= 4 ? 2 : 4;
    __shared__ double Ws[ST * 16][NC + 2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int g = blockIdx.x * 4 + wv;
    const bool gok = g < G16;
    const int kq = 4 * (lane >> 4), cl = lane & 15;
    constexpr int NS = CB == 1 ? 2 : 1;
    v4d C[CB][NS];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) C[cb][s2] = (v4d){0.0, 0.0, 0.0, 0.0};
    double nx[4];
    if (gok && c0 < c1) load_tile(At + ((size_t)g * KT + c0) * 256, lane, nx);
    for (int cs = c0; cs < c1; cs += ST) {
        const int nst = min(ST, c1 - cs);
        for (int e = t; e < ST * 16 * NC; e += 256) {
            const int col = e % NC, kk = e / NC;
            const int gk = cs * 16 + kk;
            Ws[kk][col] = (col < Rp && kk < nst * 16 && gk < n) ? X[(size_t)gk * Rp + col] : 0.0;
        }
        __syncthreads();
        for (int ci = 0; ci < nst; ++ci) {
            double a[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = nx[e];
            if (gok && cs + ci + 1 < c1) load_tile(At + ((size_t)g * KT + cs + ci + 1) * 256, lane, nx);
            if (gok) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kk = ci * 16 + kq + e;
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        C[cb][e % NS] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], Ws[kk][cb * 16 + cl], C[cb][e % NS],
                                                                             0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    if (!gok) return;
    double* P = part + (size_t)kc * n * Rp;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = cb * 16 + cl;
        if (col >= Rp) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = g * 16 + (lane >> 4) + 4 * r;
            if (row < n) {
                double sum = 0.0;
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2) sum += C[cb][s2][r];
                P[(size_t)row * Rp + col] = sum;
            }
        }
    }
}

// ------------------------------------------------------ FP32 MFMA history ---
// History with FP32 products (v_mfma_f32_16x16x4f32) on the FP32 tiles:
//   Q W ~ Q_hi W_hi + Q_hi W_lo + Q_lo W_hi   on lags 1..hilo, Q_hi W_hi beyond.
// One FP32 accumulator sums 4*FL summation indices of each half (u and v), then
// is added into the FP64 total: the history sums cancel strongly (row sums are
// 10-100x below the sums of magnitudes), so FP32 partial sums are kept short.
// Slices of MTK indices are staged per block; FP64 across slices, K chunks and
// lags.
constexpr int MTK = 64;       // K slice staged in LDS (4 tiles)

template <int CB, int FL>
__global__ __launch_bounds__(256) void k_hist_mfma(int ne, int hs, int G16, int KT, int Rp,
                                                   const int* __restrict__ dk, int nh, int hilo,
                                                   const float* __restrict__ Qf, const float* __restrict__ Qlo,
                                                   const double* __restrict__ ring, int KC,
                                                   double* __restrict__ part, const GmState* __restrict__ agg) {
    if (agg->halt) return;
    const int k = *dk;
    const int jj = blockIdx.y;
    const int nact = k - 1 < nh ? k - 1 : nh;
    if (jj >= nact) return;
    const int j = jj + 1;
    const bool hl = Qlo != nullptr && j <= hilo;
    const int n2 = 2 * hs;
    const size_t tsz = (size_t)G16 * KT * 256;
    const float* a1p = Qf + (size_t)(j - 1) * 3 * tsz;
    const float* akp = a1p + tsz;
    const float* a2p = a1p + 2 * tsz;
    const float* l1p = hl ? Qlo + (size_t)(j - 1) * 3 * tsz : nullptr;
    const float* lkp = hl ? l1p + tsz : nullptr;
    const float* l2p = hl ? l1p + 2 * tsz : nullptr;
    const double* W = ring + (size_t)((k - j) % nh) * n2 * Rp;
    const int kc = blockIdx.z;
    const int KL = ((hs + KC - 1) / KC + MTK - 1) / MTK * MTK;
    const int kb = kc * KL, ke = min(hs, kb + KL);

    // staged history vectors, transposed: [u/v][hi/lo][column][k]
    __shared__ float Wt[2][2][CB * 16][MTK + 4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int g = blockIdx.x * 4 + wv;
    const bool gok = g < G16;
    const int kq = 4 * (lane >> 4);
    double Du[CB][4], Dv[CB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) Du[c][r] = Dv[c][r] = 0.0;

    for (int s0 = kb; s0 < ke; s0 += MTK) {
        // stage the slice of W (FP64) as hi/lo FP32
        for (int e = t; e < CB * 16 * MTK; e += 256) {
            const int col = e % (CB * 16), kk = e / (CB * 16);
            const int gk = s0 + kk;
            double wu = 0.0, wvv = 0.0;
            if (col < Rp && gk < ke) {
                wu = W[(size_t)gk * Rp + col];
                wvv = W[(size_t)(hs + gk) * Rp + col];
            }
            const float uh = (float)wu, vh = (float)wvv;
            Wt[0][0][col][kk] = uh;
            Wt[0][1][col][kk] = (float)(wu - (double)uh);
            Wt[1][0][col][kk] = vh;
            Wt[1][1][col][kk] = (float)(wvv - (double)vh);
        }
        __syncthreads();
        v4f Cu[CB], Cv[CB];
        // unrolling the quarters lets the compiler keep more loads in flight,
        // but with one-step groups it keeps every group's accumulator alive
        constexpr int QUN = (FL == 1 && CB > 1) ? 1 : MTK / 16;
#pragma unroll QUN
        for (int ss = 0; ss < MTK / 16; ++ss) {
            const int kl = ss * 16 + kq;          // k within the slice
            const int c = (s0 >> 4) + ss;         // tile column
            v4f a1 = {0.f, 0.f, 0.f, 0.f}, ak = a1, a2 = a1, b1 = a1, bk = a1, b2 = a1;
            if (gok && s0 + ss * 16 < ke) {
                const size_t o = ((size_t)g * KT + c) * 256;
                a1 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(a1p + o) + lane);
                ak = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(akp + o) + lane);
                a2 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(a2p + o) + lane);
                if (hl) {
                    b1 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(l1p + o) + lane);
                    bk = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(lkp + o) + lane);
                    b2 = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(l2p + o) + lane);
                }
            }
            v4f UH[CB], VH[CB], UL[CB], VL[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int col = cb * 16 + (lane & 15);
                UH[cb] = *reinterpret_cast<const v4f*>(&Wt[0][0][col][kl]);
                VH[cb] = *reinterpret_cast<const v4f*>(&Wt[1][0][col][kl]);
                if (hl) {
                    UL[cb] = *reinterpret_cast<const v4f*>(&Wt[0][1][col][kl]);
                    VL[cb] = *reinterpret_cast<const v4f*>(&Wt[1][1][col][kl]);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = ss * 4 + e;         // 4-index step within the slice
                if (q % FL == 0) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) Cu[cb] = Cv[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const float uh = UH[cb][e], vh = VH[cb][e];
                    Cu[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[e], uh, Cu[cb], 0, 0, 0);
                    Cv[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ak[e], uh, Cv[cb], 0, 0, 0);
                    Cu[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ak[e], vh, Cu[cb], 0, 0, 0);
                    Cv[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[e], vh, Cv[cb], 0, 0, 0);
                    if (hl) {
                        const float ul = UL[cb][e], vl = VL[cb][e];
                        // Q_hi W_lo
                        Cu[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[e], ul, Cu[cb], 0, 0, 0);
                        Cu[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ak[e], vl, Cu[cb], 0, 0, 0);
                        Cv[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ak[e], ul, Cv[cb], 0, 0, 0);
                        Cv[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[e], vl, Cv[cb], 0, 0, 0);
                        // Q_lo W_hi
                        Cu[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[e], uh, Cu[cb], 0, 0, 0);
                        Cu[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-bk[e], vh, Cu[cb], 0, 0, 0);
                        Cv[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bk[e], uh, Cv[cb], 0, 0, 0);
                        Cv[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b2[e], vh, Cv[cb], 0, 0, 0);
                    }
                }
                if (q % FL == FL - 1) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            Du[cb][r] += (double)Cu[cb][r];
                            Dv[cb][r] += (double)Cv[cb][r];
                        }
                }
            }
        }
        __syncthreads();
    }
    if (!gok) return;
    double* P = part + ((size_t)jj * KC + kc) * 2 * ne * Rp;
    const int rbase = g * 16 + kq;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = cb * 16 + (lane & 15);
        if (col >= Rp) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = rbase + r;
            if (rr < ne) {
                P[(size_t)rr * Rp + col] = Du[cb][r];
                P[(size_t)(ne + rr) * Rp + col] = Dv[cb][r];
            }
        }
    }
}


template <int RP>
void plain_product(mot_handle* h, const double* src, double* vj, double* z) {
    const int n = h->n2;
    const int KC = h->plain_kc;
    const int G16 = n / 16, KT = n / 16;
    dim3 grid((G16 + 3) / 4, 1, KC);
    constexpr int CB = RP >= 64 ? 4 : (RP >= 32 ? 2 : 1);
    if (h->M32)
        hipLaunchKernelGGL((k_tile_plain<float, CB>), grid, dim3(256), 0, h->stream, n, G16, KT, RP, h->M32, src, KC,
                           h->mr_part, h->gm);
    else
        hipLaunchKernelGGL((k_tile_plain<double, CB>), grid, dim3(256), 0, h->stream, n, G16, KT, RP, h->M64, src, KC,
                           h->mr_part, h->gm);
    hipLaunchKernelGGL(k_plain_reduce<RP>, dim3((n * RP + 255) / 256), dim3(256), 0, h->stream, n, KC, h->mr_part, src,
                       h->gms, h->gm, z, vj);
}

template <typename T>
void tile_launch(mot_handle* h, int q0_mode, const T* At, const float* Alo, const double* X, int KC, int groups) {
    const int WG = (q0_mode ? h->q0_wg : h->hist_wg) == 8 ? 8 : 4;
    dim3 grid((h->G16 + WG - 1) / WG, groups, KC);
    const int CB = (h->Rp + 15) / 16;
#define L_(CB_, WG_) hipLaunchKernelGGL((k_tile_gemm<T, CB_, WG_>), grid, dim3(64 * WG_), 0, h->stream, h->ne, h->hs, \
                                        h->G16, h->KT, h->Rp, h->d_k, h->nh, q0_mode, At, Alo, h->hilo, h->ring, X, \
                                        KC, h->mr_part, h->gm)
#define W_(CB_) do { if (WG == 8) L_(CB_, 8); else L_(CB_, 4); } while (0)
    if (CB == 1)
        W_(1);
    else if (CB == 2)
        W_(2);
    else
        W_(4);
#undef W_
#undef L_
}

}  // namespace

namespace motk_multi {

#define MOT_RP_SWITCH(RPV, CALL)                                         \
    switch (RPV) {                                                       \
        case 4: CALL(4); break;                                          \
        case 8: CALL(8); break;                                          \
        case 16: CALL(16); break;                                        \
        case 32: CALL(32); break;                                        \
        case 64: CALL(64); break;                                        \
        default: break;                                                  \
    }

// K chunks so that one launch has about 2048 workgroups, each chunk at least
// `unit` tiles long.
static int tile_kc(int blocks, int KT, int unit) {
    int want = (2048 + blocks - 1) / blocks;
    int maxkc = KT / unit;
    if (maxkc < 1) maxkc = 1;
    return want < 1 ? 1 : (want > maxkc ? maxkc : want);
}

// Autotuner candidates around the size rule's choice: base/4 .. 4 base, within
// 1..maxkc (the partial buffer is sized for the largest).
static std::vector<int> kc_candidates(int base, int maxkc) {
    std::vector<int> c;
    for (int v : {base / 4, base / 2, base, base * 2, base * 4}) {
        v = std::max(1, std::min(v, maxkc));
        if (std::find(c.begin(), c.end(), v) == c.end()) c.push_back(v);
    }
    return c;
}

void plan_tiles(mot_handle* h) {
    h->G16 = (h->ne + 15) / 16;
    h->KT = (h->hs + 15) / 16;
    const int gx = (h->G16 + 3) / 4;
    h->hist_kc = tile_kc(gx * h->nh, h->KT, MTK / 16);
    h->q0_kc = tile_kc(gx, h->KT, 4);
    // the approximate inverse (n2 x n2 tiles): about 1024 workgroups
    const int gp = (h->n2 / 16 + 3) / 4;
    int want = (1024 + gp - 1) / gp, maxkc = std::max(1, h->n2 / 64);
    h->plain_kc = std::max(1, std::min(want, maxkc));
    h->hist_kc_c.clear();
    h->q0_kc_c.clear();
    h->plain_kc_c.clear();
    if (h->opt.autotune) {
        h->hist_kc_c = kc_candidates(h->hist_kc, std::max(1, h->KT / (MTK / 16)));
        h->q0_kc_c = kc_candidates(h->q0_kc, std::max(1, h->KT / 4));
        if (h->opt.precond) h->plain_kc_c = kc_candidates(h->plain_kc, maxkc);
    }
    // Krylov sweeps: about 1024 (row, column) entries per workgroup, at most
    // 120 workgroups: every workgroup ends with a device-scope release before
    // the grid counter, and that write-back costs more than the rows it saves
    // (three sweeps at 30,720 x 16: 160 us with 480 workgroups, 79 with 120)
    h->orth_nb = std::max(1, std::min(120, (int)(((size_t)h->n2 * h->Rp + 1023) / 1024)));
    h->orth_rb = (h->n2 + h->orth_nb - 1) / h->orth_nb;
    h->orth_nb = (h->n2 + h->orth_rb - 1) / h->orth_rb;
}

size_t orth_part_doubles(const mot_handle* h) { return (size_t)h->orth_nb * (MOT_MAXM + 1) * h->Rp; }

size_t tile_elems(const mot_handle* h) { return (size_t)h->G16 * h->KT * 256; }

size_t part_doubles(const mot_handle* h) {
    auto top = [](int v, const std::vector<int>& c) {
        for (int x : c) v = std::max(v, x);
        return (size_t)v;
    };
    size_t a = (size_t)h->nh * top(h->hist_kc, h->hist_kc_c) * 2 * h->ne * h->Rp;
    size_t b = top(h->q0_kc, h->q0_kc_c) * 2 * h->ne * h->Rp;
    size_t c = top(h->plain_kc, h->plain_kc_c) * h->n2 * h->Rp;
    return std::max(a, std::max(b, c));
}

static void reduce(mot_handle* h, int q0_mode, int KC, double* out) {
    const int n = h->ne * h->Rp;
#define C_(R_) hipLaunchKernelGGL(k_struct_reduce<R_>, dim3((n + 255) / 256), dim3(256), 0, h->stream, h->ne, h->hs, \
                                  h->d_k, h->nh, q0_mode, KC, h->mr_part, h->rb, h->B, out, h->gm)
    MOT_RP_SWITCH(h->Rp, C_)
#undef C_
}

void history_gemm(mot_handle* h) {
    const int KC = h->hist_kc;
    if (h->opt.precision == MOT_MIXED32) {
        dim3 grid((h->G16 + 3) / 4, h->nh, KC);
        const int CB = (h->Rp + 15) / 16;
        const int FL = h->opt.mix_group == 64 ? 16 : (h->opt.mix_group == 16 ? 4 : 1);
#define L_(CB_, FL_) hipLaunchKernelGGL((k_hist_mfma<CB_, FL_>), grid, dim3(256), 0, h->stream, h->ne, h->hs, h->G16, \
                                        h->KT, h->Rp, h->d_k, h->nh, h->hilo, h->QtF, h->QtL, h->ring, KC, h->mr_part, \
                                        h->gm)
#define F_(CB_)              \
    do {                     \
        if (FL == 16)        \
            L_(CB_, 16);     \
        else if (FL == 4)    \
            L_(CB_, 4);      \
        else                 \
            L_(CB_, 1);      \
    } while (0)
        if (CB == 1)
            F_(1);
        else if (CB == 2)
            F_(2);
        else
            F_(4);
#undef F_
#undef L_
    } else if (h->QtF) {
        tile_launch<float>(h, 0, h->QtF, h->QtL, nullptr, KC, h->nh);
    } else {
        tile_launch<double>(h, 0, h->Qt + 3 * tile_elems(h), nullptr, nullptr, KC, h->nh);
    }
}

void history_reduce(mot_handle* h) { reduce(h, 0, h->hist_kc, h->y); }

// After the fold of one lag: its tiles (FP64 for lag 0 and the plain path,
// FP32 hi and, on lags 1..hilo, lo for the mixed paths).
void pack_lag(mot_handle* h, int lag) {
    const size_t blk = (size_t)h->ne * h->hs;
    const size_t tsz = tile_elems(h);
    for (int x = 0; x < 3; ++x) {
        const double* src = h->Q + ((size_t)lag * 3 + x) * blk;
        double* t64 = nullptr;
        float *t32 = nullptr, *lo = nullptr;
        if (lag == 0 || !h->QtF) {
            t64 = h->Qt + ((size_t)lag * 3 + x) * tsz;
        } else {
            t32 = h->QtF + ((size_t)(lag - 1) * 3 + x) * tsz;
            if (lag <= h->hilo) lo = h->QtL + ((size_t)(lag - 1) * 3 + x) * tsz;
        }
        hipLaunchKernelGGL(k_pack_tiles, dim3(4096), dim3(256), 0, h->stream, h->ne, h->hs, h->G16, h->KT, src, t64, t32,
                           lo);
    }
}

// The approximate inverse (n2 x n2, row-major X) into tiles, FP64 or FP32.
void pack_square(mot_handle* h, const double* X, double* t64, float* t32) {
    const int n = h->n2;
    hipLaunchKernelGGL(k_pack_tiles, dim3(4096), dim3(256), 0, h->stream, n, n, n / 16, n / 16, X, t64, t32,
                       (float*)nullptr);
}

void q0_gemm(mot_handle* h, const double* X) { tile_launch<double>(h, 1, h->Qt, nullptr, X, h->q0_kc, 1); }

void q0_reduce(mot_handle* h, double* out) { reduce(h, 1, h->q0_kc, out); }

void precond(mot_handle* h, const double* src, double* vj, double* z) {
#define C_(R_) plain_product<R_>(h, src, vj, z)
    MOT_RP_SWITCH(h->Rp, C_)
#undef C_
}

void start(mot_handle* h, const double* y, double* r, int have_t, int first, double* xzero, int publish) {
    hipLaunchKernelGGL(k_gmb_start, dim3(h->orth_nb), dim3(256), 0, h->stream, h->n2, h->Rp, h->R, h->orth_rb, y, r,
                       have_t, h->gms, h->gm, publish ? h->dflag : nullptr, h->opt.gmres_tol, first, xzero,
                       h->orth_part);
}

void orth(mot_handle* h, double* w, int publish) {
    for (int sweep = 1; sweep <= 3; ++sweep)
        hipLaunchKernelGGL(k_gmb_orth, dim3(h->orth_nb), dim3(256), 0, h->stream, h->n2, h->Rp, h->R, h->orth_rb,
                           sweep, h->V, w, h->gms, h->gm, publish ? h->dflag : nullptr, h->opt.gmres_tol, h->M,
                           h->orth_part);
}

// spec: a queued step; the next step's start resets every column's cycle, so
// consumed cycles need no marking
void finish(mot_handle* h, int force, int spec, int kq) {
    size_t total = (size_t)h->n2 * h->Rp;
    int nb = (int)std::min<size_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gmb_finish, dim3(nb), dim3(256), 0, h->stream, h->n2, h->Rp, h->Z, h->gms, h->gm, h->x,
                       h->d_k, h->nh, h->ring, h->hist, h->hist_cap, force, spec, kq);
    if (!spec) hipLaunchKernelGGL(k_gmb_consume, dim3(1), dim3(64), 0, h->stream, h->Rp, h->gms, h->gm);
}

}  // namespace motk_multi
