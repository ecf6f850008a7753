// History convolution of the marching-on-in-time loop from the raw families
// of each lag (mot_options.history_form = 1; single right-hand side).
#include "mot_internal.h"

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One workgroup of four wavefronts per row m: the 256 threads stride the row's
// columns together (2 KiB of each block per pass), then the four wavefronts'
// partial sums meet in LDS.  N sums; every thread receives the totals.
template <int N>
__device__ __forceinline__ void wg_sum(double (&v)[N]) {
    __shared__ double red[4][N];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) red[wv][i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
}

// History convolution from the raw families (history_form 1; Sec. V-B): per
// row m,
//   y1 = sum_j (Z^h_j XL_{k-j} + Z^hat_j XS_{k-j}),
//   y2 = sum_j (Z^h_j XS_{k-j} + Z^til_j XL_{k-j}),
// each Z = [[M1, -Ks], [Ks, M2]] on the (u; v) halves (blocks [3][ne][hs] as
// staged: media summed, time-scaled), XL = P^{Lambda H} w and XS = P^Sigma w
// in rings of nh slots [2 hs].  Z[3 j + f] null: family f absent at lag j.
__global__ __launch_bounds__(256) void k_raw_lags(int ne, int hs, int k, int nh, double* const* __restrict__ Z,
                                                  const double* __restrict__ RL, const double* __restrict__ RS,
                                                  double* __restrict__ y1, double* __restrict__ y2) {
    const int m = blockIdx.x;
    if (m >= ne) return;                         // the whole workgroup
    const size_t blk = (size_t)ne * hs, row = (size_t)m * hs;
    const int n2 = 2 * hs;
    const int nact = k - 1 < nh ? k - 1 : nh;
    double p[4] = {0, 0, 0, 0};                  // y1 (u, v), y2 (u, v)
    for (int j = 1; j <= nact; ++j) {
        const double* L = RL + (size_t)((k - j) % nh) * n2;
        const double* S = RS + (size_t)((k - j) % nh) * n2;
        const double* zh = Z[3 * j];
        const double* zt = Z[3 * j + 1];
        const double* zl = Z[3 * j + 2];
        for (int n = threadIdx.x; n < ne; n += 256) {
            const double lu = L[n], lv = L[hs + n], su = S[n], sv = S[hs + n];
            if (zh) {                            // h: XL into y1, XS into y2
                const double a = zh[row + n], kk = zh[blk + row + n], q = zh[2 * blk + row + n];
                p[0] = fma(a, lu, p[0]); p[0] = fma(-kk, lv, p[0]);
                p[1] = fma(kk, lu, p[1]); p[1] = fma(q, lv, p[1]);
                p[2] = fma(a, su, p[2]); p[2] = fma(-kk, sv, p[2]);
                p[3] = fma(kk, su, p[3]); p[3] = fma(q, sv, p[3]);
            }
            if (zt) {                            // hat: XS into y1
                const double a = zt[row + n], kk = zt[blk + row + n], q = zt[2 * blk + row + n];
                p[0] = fma(a, su, p[0]); p[0] = fma(-kk, sv, p[0]);
                p[1] = fma(kk, su, p[1]); p[1] = fma(q, sv, p[1]);
            }
            if (zl) {                            // tilde: XL into y2
                const double a = zl[row + n], kk = zl[blk + row + n], q = zl[2 * blk + row + n];
                p[2] = fma(a, lu, p[2]); p[2] = fma(-kk, lv, p[2]);
                p[3] = fma(kk, lu, p[3]); p[3] = fma(q, lv, p[3]);
            }
        }
    }
    wg_sum(p);
    if (threadIdx.x == 0) {
        y1[m] = p[0];
        y1[hs + m] = p[1];
        y2[m] = p[2];
        y2[hs + m] = p[3];
    }
}

// P^Sigma applied to both halves of w, a workgroup per row m: XS = P^Sigma w
// and XL = w - XS (the padding rows are never read)
__global__ __launch_bounds__(256) void k_raw_project(int ne, int hs, const double* __restrict__ PS,
                                                     const double* __restrict__ w, double* __restrict__ xs,
                                                     double* __restrict__ xl) {
    const int m = blockIdx.x;
    if (m >= ne) return;
    const double* a = PS + (size_t)m * hs;
    double p[2] = {0, 0};
    for (int n = threadIdx.x; n < ne; n += 256) {
        const double c = a[n];
        p[0] = fma(c, w[n], p[0]);
        p[1] = fma(c, w[hs + n], p[1]);
    }
    wg_sum(p);
    if (threadIdx.x == 0) {
        xs[m] = p[0];
        xs[hs + m] = p[1];
        xl[m] = w[m] - p[0];
        xl[hs + m] = w[hs + m] - p[1];
    }
}

// y = r_k - (C1b y1 + C2b y2) for step k, a workgroup per row; r_k from the
// double-buffered RHS batch [half][ne][B] (column (k-1) mod B)
__global__ __launch_bounds__(256) void k_raw_combine(int ne, int hs, int k, int B, const double* __restrict__ rb,
                                                     const double* __restrict__ C1, const double* __restrict__ C2,
                                                     const double* __restrict__ y1, const double* __restrict__ y2,
                                                     double* __restrict__ y) {
    const int m = blockIdx.x;
    if (m >= ne) return;
    const double* a = C1 + (size_t)m * hs;
    const double* c = C2 + (size_t)m * hs;
    double p[2] = {0, 0};
    for (int n = threadIdx.x; n < ne; n += 256) {
        const double e = a[n], f = c[n];
        p[0] = fma(e, y1[n], p[0]);
        p[0] = fma(f, y2[n], p[0]);
        p[1] = fma(e, y1[hs + n], p[1]);
        p[1] = fma(f, y2[hs + n], p[1]);
    }
    wg_sum(p);
    if (threadIdx.x == 0) {
        const int sc = (k - 1) % B;
        const double* rr = rb + (size_t)(((k - 1) / B) & 1) * 2 * ne * B;
        y[m] = rr[(size_t)m * B + sc] - p[0];
        y[hs + m] = rr[(size_t)ne * B + (size_t)m * B + sc] - p[1];
    }
}

}  // namespace

namespace motk_step {

// history_form 1, step h->k: project w_{k-1} into the rings, the raw-family
// sums y1, y2, then y = r_k - (C1b y1 + C2b y2)
void raw_history(mot_handle* h) {
    const int k = h->k, nh = h->nh, ne = h->ne, hs = h->hs, n2 = h->n2;
    hipStream_t s = h->stream;
    const dim3 grid(ne);
    if (k >= 2) {
        const size_t off = (size_t)((k - 1) % nh) * n2;
        hipLaunchKernelGGL(k_raw_project, grid, dim3(256), 0, s, ne, hs, h->PS, h->ring + off, h->rawS + off,
                           h->rawL + off);
    }
    hipLaunchKernelGGL(k_raw_lags, grid, dim3(256), 0, s, ne, hs, k, nh, h->rawZtab, h->rawL, h->rawS, h->ry1,
                       h->ry2);
    hipLaunchKernelGGL(k_raw_combine, grid, dim3(256), 0, s, ne, hs, k, h->B, h->rb, h->C1, h->C2, h->ry1, h->ry2,
                       h->y);
}

// history_form 1 after a restore: the projections of every ring slot
void raw_reproject(mot_handle* h) {
    const size_t n2 = h->n2;
    for (int j = 0; j < h->nh; ++j)
        hipLaunchKernelGGL(k_raw_project, dim3(h->ne), dim3(256), 0, h->stream, h->ne, h->hs, h->PS,
                           h->ring + j * n2, h->rawS + j * n2, h->rawL + j * n2);
}

}  // namespace motk_step
