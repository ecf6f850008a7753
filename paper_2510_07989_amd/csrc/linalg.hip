// Dense and sparse FP64 building blocks for setup, lag fold and recovery.
#include "mot_internal.h"

namespace {

// ------------------------------------------------------------------ GEMM ---
// C = alpha A B + beta C, row-major, FP64, on v_mfma_f64_16x16x4f64.
// A workgroup of four wavefronts computes a (2 WT) x (2 WT) tile of C, each
// wavefront a WT x WT quarter as (WT/16)^2 MFMA tiles of 16 x 16.  K advances
// in slices of 16: A is staged transposed (As[k][m]) and B as is (Bs[k][n]) in
// LDS, and the next slice's global loads are issued before the current
// slice's MFMAs.  Operand layout: A lane l = row l%16, summation slot l/16; B
// lane l = column l%16, slot l/16; result register r of lane l = row
// l/16 + 4r, column l%16.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int GK = 16;

// blockIdx.z selects one of several products with the same A: B and C are
// offset by z * sB and z * sC elements.
// The 128 x 128 tile is held to two wavefronts per SIMD: left to itself the
// compiler takes 240 VGPRs and 128 AGPRs (one wavefront per SIMD, whose
// barriers and LDS reads then stall the matrix core); with the hint the
// accumulators live in 246 VGPRs without spills, 46 -> 61 TFLOP/s on
// 7680 x 8192 x 7680 and 15360^3.
template <int WT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WT == 64 ? 2 : 1)))
void k_gemm(int M, int N, int K, double alpha,
                                              const double* __restrict__ A, int lda,
                                              const double* __restrict__ B, int ldb, double beta,
                                              double* __restrict__ C, int ldc, size_t sB, size_t sC) {
    B += blockIdx.z * sB;
    C += blockIdx.z * sC;
    constexpr int BT = 2 * WT;               // block tile edge
    constexpr int NT = WT / 16;              // MFMA tiles per wavefront edge
    constexpr int PE = BT * GK / 256;        // staged elements per thread, per operand
    __shared__ double As[GK][BT + 2];
    __shared__ double Bs[GK][BT + 2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
    const int wm = (wv >> 1) * WT, wn = (wv & 1) * WT;
    v4d acc[NT][NT];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

    double ra[PE], rb[PE];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < PE; ++r) {
            const int e = tid + 256 * r;
            const int am = e / GK, ak = e % GK;            // A: 16 consecutive k per row
            const int gm = m0 + am, gk = k0 + ak;
            ra[r] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.0;
            const int bk = e / BT, bn = e % BT;            // B: BT consecutive columns per k
            const int gk2 = k0 + bk, gn = n0 + bn;
            rb[r] = (gk2 < K && gn < N) ? B[(size_t)gk2 * ldb + gn] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int r = 0; r < PE; ++r) {
            const int e = tid + 256 * r;
            As[e % GK][e / GK] = ra[r];
            Bs[e / BT][e % BT] = rb[r];
        }
        __syncthreads();
        if (k0 + GK < K) fetch(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[NT], b[NT];
#pragma unroll
            for (int i = 0; i < NT; ++i) a[i] = As[kr][wm + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NT; ++j) b[j] = Bs[kr][wn + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < NT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + (lane >> 4) + 4 * r;
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm < M && gn < N) {
                    double* c = C + (size_t)gm * ldc + gn;
                    *c = beta == 0.0 ? alpha * acc[i][j][r] : alpha * acc[i][j][r] + beta * *c;
                }
            }
}

__global__ void k_axpby2d(int rows, int cols, double a, const double* __restrict__ X, int ldx,
                          double b, double* __restrict__ Y, int ldy) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)rows * cols;
    for (; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int r = (int)(t / cols), c = (int)(t % cols);
        double* y = Y + (size_t)r * ldy + c;
        *y = (b == 0.0 ? 0.0 : b * *y) + a * X[(size_t)r * ldx + c];
    }
}

__global__ void k_fill2d(int rows, int cols, double v, double* __restrict__ Y, int ldy) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)rows * cols;
    for (; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int r = (int)(t / cols), c = (int)(t % cols);
        Y[(size_t)r * ldy + c] = v;
    }
}

__global__ void k_identity(int n, double* __restrict__ Y, int ldy) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Y[(size_t)i * ldy + i] = 1.0;
}

__global__ void k_scatter_csr_add(int n, const int64_t* __restrict__ ptr, const int* __restrict__ col,
                                  const double* __restrict__ val, double a, double* __restrict__ Y,
                                  int ldy) {
    int r = blockIdx.x;
    for (int64_t k = ptr[r] + threadIdx.x; k < ptr[r + 1]; k += blockDim.x)
        Y[(size_t)r * ldy + col[k]] += a * val[k];
}

// count of non-finite entries of a rows x cols block (leading dimension ldx)
__global__ void k_count_nonfinite(int rows, int cols, const double* __restrict__ X, int64_t ldx,
                                  int* __restrict__ count) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)rows * cols;
    int bad = 0;
    for (; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int r = (int)(t / cols), c = (int)(t % cols);
        if (!isfinite(X[(size_t)r * ldx + c])) ++bad;
    }
    if (bad) atomicAdd(count, bad);
}

// ------------------------------------------------- column-batched sparse ---
__global__ void k_spmm_csr(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                           const double* __restrict__ val, int ncol, const double* __restrict__ X,
                           double* __restrict__ Y) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (c >= ncol) return;
    double acc = 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) acc = fma(val[k], X[(size_t)col[k] * ncol + c], acc);
    Y[(size_t)r * ncol + c] = acc;
}

// graph Laplacian Inc^T Inc: (L z)_i = deg_i z_i - sum_{j in adj(i)} z_j
__global__ void k_spmm_lap(int n, const int* __restrict__ ptr, const int* __restrict__ adj, int ncol,
                           const double* __restrict__ X, double* __restrict__ Y) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (c >= ncol) return;
    int p0 = ptr[r], p1 = ptr[r + 1];
    double acc = (double)(p1 - p0) * X[(size_t)r * ncol + c];
    for (int k = p0; k < p1; ++k) acc -= X[(size_t)adj[k] * ncol + c];
    Y[(size_t)r * ncol + c] = acc;
}

// S = Inc^T X : S[node][c] = sum_{m in inc(node)} sign * X[m][c]
__global__ void k_inc_T(int nnode, const int* __restrict__ ptr, const int* __restrict__ edge,
                        const double* __restrict__ sign, int ncol, const double* __restrict__ X,
                        int ldx, double* __restrict__ S) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (c >= ncol) return;
    double acc = 0.0;
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) acc = fma(sign[k], X[(size_t)edge[k] * ldx + c], acc);
    S[(size_t)r * ncol + c] = acc;
}

// Y = Inc Z : Y[m][c] = Z[plus(m)][c] - Z[minus(m)][c]
__global__ void k_inc_apply(int ne, const int* __restrict__ plus, const int* __restrict__ minus,
                            int ncol, const double* __restrict__ Z, double* __restrict__ Y, int ldy) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int m = blockIdx.y;
    if (c >= ncol) return;
    Y[(size_t)m * ldy + c] = Z[(size_t)plus[m] * ncol + c] - Z[(size_t)minus[m] * ncol + c];
}

// partial column dots over row chunk blockIdx.y
__global__ void k_coldot_part(int rows, int ncol, const double* __restrict__ A,
                              const double* __restrict__ B, double* __restrict__ part) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    int nch = gridDim.y;
    int r0 = (int)((int64_t)rows * blockIdx.y / nch), r1 = (int)((int64_t)rows * (blockIdx.y + 1) / nch);
    double acc = 0.0;
    for (int r = r0; r < r1; ++r) acc = fma(A[(size_t)r * ncol + c], B[(size_t)r * ncol + c], acc);
    part[(size_t)blockIdx.y * ncol + c] = acc;
}

__global__ void k_colsum(int ncol, int nch, const double* __restrict__ part, double* __restrict__ out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    double acc = 0.0;
    for (int k = 0; k < nch; ++k) acc += part[(size_t)k * ncol + c];
    out[c] = acc;
}

// X += alpha P ; R -= alpha Q ; partial rr over row chunk blockIdx.y
__global__ void k_cg_update(int rows, int ncol, const double* __restrict__ alpha,
                            const double* __restrict__ P, const double* __restrict__ Q,
                            double* __restrict__ X, double* __restrict__ R, double* __restrict__ part) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    int nch = gridDim.y;
    int r0 = (int)((int64_t)rows * blockIdx.y / nch), r1 = (int)((int64_t)rows * (blockIdx.y + 1) / nch);
    double a = alpha[c], acc = 0.0;
    for (int r = r0; r < r1; ++r) {
        size_t i = (size_t)r * ncol + c;
        X[i] = fma(a, P[i], X[i]);
        double rv = fma(-a, Q[i], R[i]);
        R[i] = rv;
        acc = fma(rv, rv, acc);
    }
    part[(size_t)blockIdx.y * ncol + c] = acc;
}

// phase 0: after pq: alpha = rr/pq (0 when inactive)
// phase 1: after rr_new: beta = rr_new/rr, rr = rr_new, deactivate converged
// phase 2: initial: rr0 = rr = sum(part)
__global__ void k_cg_scalars(int ncol, const double* __restrict__ pq, const double* __restrict__ part,
                             int nch, double* __restrict__ rr, double* __restrict__ rr0,
                             double* __restrict__ alpha, double* __restrict__ beta,
                             int* __restrict__ active, double tol, int phase) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    if (phase == 0) {
        double d = pq[c];
        alpha[c] = (active[c] && d > 0.0) ? rr[c] / d : 0.0;
        return;
    }
    double s = 0.0;
    for (int k = 0; k < nch; ++k) s += part[(size_t)k * ncol + c];
    if (phase == 2) {
        rr[c] = s;
        rr0[c] = s;
        active[c] = s > 0.0 ? 1 : 0;
        beta[c] = 0.0;
        return;
    }
    if (!active[c]) { beta[c] = 0.0; return; }
    double old = rr[c];
    beta[c] = old > 0.0 ? s / old : 0.0;
    rr[c] = s;
    if (s <= tol * tol * rr0[c]) active[c] = 0;
}

__global__ void k_cg_pupdate(int rows, int ncol, const double* __restrict__ beta,
                             const double* __restrict__ R, double* __restrict__ P) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)rows * ncol;
    for (; t < total; t += (size_t)gridDim.x * blockDim.x) {
        int c = (int)(t % ncol);
        P[t] = fma(beta[c], P[t], R[t]);
    }
}

// subtract each column's mean: the RHS of a graph-Laplacian pseudo-inverse solve
// is projected onto the complement of the constant null vector
__global__ void k_col_center(int rows, int ncol, double* __restrict__ X) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += X[(size_t)r * ncol + c];
    s /= rows;
    for (int r = 0; r < rows; ++r) X[(size_t)r * ncol + c] -= s;
}

__global__ void k_count(int ncol, const int* __restrict__ active, int* __restrict__ out) {
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    int loc = 0;
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) loc += active[c];
    atomicAdd(&s, loc);
    __syncthreads();
    if (threadIdx.x == 0) *out = s;
}

inline int nblk(size_t total, int bs = 256) {
    size_t b = (total + bs - 1) / bs;
    return (int)(b > 65535 * 4 ? 65535 * 4 : (b ? b : 1));
}

}  // namespace

namespace motk {

void gemm(hipStream_t s, int M, int N, int K, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc, int batch, size_t sB, size_t sC) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    // 128 x 128 tiles when they still give about four workgroups per CU
    const long big = (long)((N + 127) / 128) * ((M + 127) / 128) * batch;
    if (big >= 1024) {
        dim3 grid((N + 127) / 128, (M + 127) / 128, batch);
        hipLaunchKernelGGL(k_gemm<64>, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, sB,
                           sC);
    } else {
        dim3 grid((N + 63) / 64, (M + 63) / 64, batch);
        hipLaunchKernelGGL(k_gemm<32>, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, sB,
                           sC);
    }
}

void axpby2d(hipStream_t s, int rows, int cols, double a, const double* X, int ldx, double b,
             double* Y, int ldy) {
    hipLaunchKernelGGL(k_axpby2d, dim3(nblk((size_t)rows * cols)), dim3(256), 0, s, rows, cols, a, X,
                       ldx, b, Y, ldy);
}

int count_nonfinite(hipStream_t s, int rows, int cols, const double* X, int64_t ldx, int* d_count) {
    int h = 0;
    if (hipMemsetAsync(d_count, 0, sizeof(int), s) != hipSuccess) return -1;
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nblk((size_t)rows * cols)), dim3(256), 0, s, rows, cols, X, ldx,
                       d_count);
    if (hipMemcpyAsync(&h, d_count, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    return h;
}

void fill2d(hipStream_t s, int rows, int cols, double v, double* Y, int ldy) {
    hipLaunchKernelGGL(k_fill2d, dim3(nblk((size_t)rows * cols)), dim3(256), 0, s, rows, cols, v, Y, ldy);
}

void set_identity(hipStream_t s, int n, double* Y, int ldy) {
    hipLaunchKernelGGL(k_identity, dim3((n + 255) / 256), dim3(256), 0, s, n, Y, ldy);
}

void scatter_csr_add(hipStream_t s, int n, const int64_t* ptr, const int* col, const double* val,
                     double a, double* Y, int ldy) {
    hipLaunchKernelGGL(k_scatter_csr_add, dim3(n), dim3(64), 0, s, n, ptr, col, val, a, Y, ldy);
}

void spmm_csr(hipStream_t s, const DevCSR& A, int ncol, const double* X, double* Y) {
    dim3 grid((ncol + 255) / 256, A.n);
    hipLaunchKernelGGL(k_spmm_csr, grid, dim3(256), 0, s, A.n, A.ptr, A.col, A.val, ncol, X, Y);
}

void spmm_lap(hipStream_t s, const DevGraph& g, int ncol, const double* X, double* Y) {
    dim3 grid((ncol + 255) / 256, g.nnode);
    hipLaunchKernelGGL(k_spmm_lap, grid, dim3(256), 0, s, g.nnode, g.adj_ptr, g.adj, ncol, X, Y);
}

void inc_T(hipStream_t s, const DevGraph& g, int ncol, const double* X, int ldx, double* S) {
    dim3 grid((ncol + 255) / 256, g.nnode);
    hipLaunchKernelGGL(k_inc_T, grid, dim3(256), 0, s, g.nnode, g.inc_ptr, g.inc_edge, g.inc_sign,
                       ncol, X, ldx, S);
}

void inc_apply(hipStream_t s, const DevGraph& g, int ncol, const double* Z, double* Y, int ldy) {
    dim3 grid((ncol + 255) / 256, g.ne);
    hipLaunchKernelGGL(k_inc_apply, grid, dim3(256), 0, s, g.ne, g.plus, g.minus, ncol, Z, Y, ldy);
}

void coldot(hipStream_t s, int rows, int ncol, const double* A, const double* B, double* part,
            double* out) {
    dim3 grid((ncol + 255) / 256, MOT_CG_CHUNKS);
    hipLaunchKernelGGL(k_coldot_part, grid, dim3(256), 0, s, rows, ncol, A, B, part);
    hipLaunchKernelGGL(k_colsum, dim3((ncol + 255) / 256), dim3(256), 0, s, ncol, MOT_CG_CHUNKS, part, out);
}

void cg_update(hipStream_t s, int rows, int ncol, const double* alpha, const double* P,
               const double* Q, double* X, double* R, double* part) {
    dim3 grid((ncol + 255) / 256, MOT_CG_CHUNKS);
    hipLaunchKernelGGL(k_cg_update, grid, dim3(256), 0, s, rows, ncol, alpha, P, Q, X, R, part);
}

void cg_scalars(hipStream_t s, int ncol, const double* pq, const double* part, int nchunk,
                double* rr, double* rr0, double* alpha, double* beta, int* active, double tol,
                int phase) {
    hipLaunchKernelGGL(k_cg_scalars, dim3((ncol + 255) / 256), dim3(256), 0, s, ncol, pq, part, nchunk,
                       rr, rr0, alpha, beta, active, tol, phase);
}

void cg_pupdate(hipStream_t s, int rows, int ncol, const double* beta, const double* R, double* P) {
    hipLaunchKernelGGL(k_cg_pupdate, dim3(nblk((size_t)rows * ncol)), dim3(256), 0, s, rows, ncol, beta,
                       R, P);
}

void col_center(hipStream_t s, int rows, int ncol, double* X) {
    hipLaunchKernelGGL(k_col_center, dim3((ncol + 255) / 256), dim3(256), 0, s, rows, ncol, X);
}

int count_active(hipStream_t s, int ncol, const int* active, int* d_count, int* h_count) {
    hipLaunchKernelGGL(k_count, dim3(1), dim3(1024), 0, s, ncol, active, d_count);
    if (hipMemcpyAsync(h_count, d_count, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    return 0;
}

}  // namespace motk
