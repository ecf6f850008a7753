// Far field of the computed currents (Section VI, far-field computation, on
// eq. (dis_jm)): the spectrum at one frequency of the loop and star currents of
// a range of kept steps, kept apart, and the scattered far field each radiates.
//
// The currents are j(t) = sum_i j_i p_i(t) with p_i the unit pulse on
// ((i-1) dt, i dt), so with the exp(+i omega t) convention
//   J(f) = sum_i j_i phi_i,  phi_i = dt sinc(omega dt / 2) exp(-i omega (i - 1/2) dt).
// eq. (dis_jm) is linear in the unknowns, so the transform is taken of the
// kept unknowns first (one streaming pass over the history: S = sum w_i phi_i
// and D = sum (w_i - w_{i-1}) phi_i) and the projectors are applied once to
// the result: loop = P^{Lambda H} S = S - P^Sigma S, star = (T_max/dt) P^Sigma D.
// The far field is E(rhat) = (i k / 4 pi) [rhat x L + eta rhat x (rhat x N)]
// with N = sum_n J_n F_n(rhat), L = sum_n M_n F_n(rhat),
// F_n(rhat) = int f_n exp(i k rhat.x) dS on the RHS quadrature points, eta = 1.
#include <algorithm>

#include "mot_internal.h"

namespace {

// phase table phi_s of kept steps first .. first+count-1 (step s covers
// (s dt, (s+1) dt)): [count][2] (re, im)
__global__ void k_ff_phase(int first, int count, double omega, double dt, double* __restrict__ phi) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const double hw = 0.5 * omega * dt;
    const double amp = hw == 0.0 ? dt : dt * sin(hw) / hw;
    double sn, cs;
    sincos(omega * ((first + s) + 0.5) * dt, &sn, &cs);
    phi[2 * s] = amp * cs;
    phi[2 * s + 1] = -amp * sn;
}

// One element e = (half hh, edge m, wave r) of the kept unknowns per thread,
// one chunk of steps per blockIdx.y: partial sums of S and D (re, im) to
// part[chunk][E][4].  The step loop reads one double per thread per step
// (consecutive threads, consecutive addresses) and keeps w_{s-1} in a
// register, so the history is read once.
__global__ __launch_bounds__(256) void k_ff_spectrum(int ne, int hs, int n2, int R, int Rp, int first, int count,
                                                     int chunk, const double* __restrict__ hist,
                                                     const double* __restrict__ phi, double* __restrict__ part) {
    const int E = 2 * ne * R;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int r = e % R, m = (e / R) % ne, hh = e / (R * ne);
    const size_t off = (size_t)(hh * hs + m) * Rp + r;
    const size_t ld = (size_t)n2 * Rp;
    const int s0 = blockIdx.y * chunk, s1 = min(count, s0 + chunk);
    const double* w = hist + (size_t)first * ld + off;
    double prev = (first + s0 > 0) ? w[((ptrdiff_t)s0 - 1) * (ptrdiff_t)ld] : 0.0;
    double sr = 0, si = 0, dr = 0, di = 0;
    int s = s0;
    for (; s + 4 <= s1; s += 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(w + (size_t)(s + u) * ld);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double pr = phi[2 * (s + u)], pi = phi[2 * (s + u) + 1];
            const double d = v[u] - prev;
            sr += v[u] * pr; si += v[u] * pi;
            dr += d * pr; di += d * pi;
            prev = v[u];
        }
    }
    for (; s < s1; ++s) {
        const double v = w[(size_t)s * ld];
        const double pr = phi[2 * s], pi = phi[2 * s + 1];
        const double d = v - prev;
        sr += v * pr; si += v * pi;
        dr += d * pr; di += d * pi;
        prev = v;
    }
    double* o = part + ((size_t)blockIdx.y * E + e) * 4;
    o[0] = sr; o[1] = si; o[2] = dr; o[3] = di;
}

// sum the chunks; X is [ne][8R], column ((p * 2 + hh) * 2 + c) * R + r with
// p 0 for S, 1 for D and c 0 re, 1 im
__global__ void k_ff_reduce(int ne, int R, int nchunk, const double* __restrict__ part, double* __restrict__ X) {
    const int E = 2 * ne * R;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double a[4] = {0, 0, 0, 0};
    for (int c = 0; c < nchunk; ++c) {
        const double* p = part + ((size_t)c * E + e) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] += p[q];
    }
    const int r = e % R, m = (e / R) % ne, hh = e / (R * ne);
    const size_t row = (size_t)m * 8 * R;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int p = q >> 1, c = q & 1;
        X[row + ((p * 2 + hh) * 2 + c) * R + r] = a[q];
    }
}

// spec [2 parts][2 ne][R][2]: loop = S - P^Sigma S, star = scale P^Sigma D
__global__ void k_ff_parts(int ne, int R, double scale, const double* __restrict__ X, const double* __restrict__ PX,
                           double* __restrict__ spec) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = 2 * ne * R * 2;                     // one part
    if (t >= 2 * per) return;
    const int c = t % 2, r = (t / 2) % R, i = (t / (2 * R)) % (2 * ne), part = t / per;
    const int hh = i / ne, m = i % ne;
    const size_t row = (size_t)m * 8 * R;
    const int colS = ((0 * 2 + hh) * 2 + c) * R + r, colD = ((1 * 2 + hh) * 2 + c) * R + r;
    spec[t] = part == 0 ? X[row + colS] - PX[row + colS] : scale * PX[row + colD];
}

__device__ __forceinline__ double ff_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// one workgroup per (direction a, wave r): radiation vectors F_n(rhat) on the
// 14 quadrature points of each edge, N and L of both parts, then the field;
// out [ndir][R][2 parts][3][2]
__global__ __launch_bounds__(256) void k_ff_field(int ne, int R, double k, const double* __restrict__ dirs,
                                                  const double* __restrict__ qx, const double* __restrict__ qf,
                                                  const double* __restrict__ spec, double* __restrict__ out) {
    const int a = blockIdx.x, r = blockIdx.y;
    const double dx = dirs[3 * a], dy = dirs[3 * a + 1], dz = dirs[3 * a + 2];
    // acc[part][N or L][xyz][re, im]
    double acc[2][2][3][2] = {};
    const size_t per = (size_t)2 * ne * R * 2;
    for (int n = threadIdx.x; n < ne; n += blockDim.x) {
        double F[3][2] = {};
        for (int q = 0; q < 14; ++q) {
            const double* x = qx + ((size_t)n * 14 + q) * 3;
            const double* f = qf + ((size_t)n * 14 + q) * 3;
            double sn, cs;
            sincos(k * (dx * x[0] + dy * x[1] + dz * x[2]), &sn, &cs);
#pragma unroll
            for (int d = 0; d < 3; ++d) { F[d][0] += f[d] * cs; F[d][1] += f[d] * sn; }
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const double* sp = spec + p * per + (((size_t)hh * ne + n) * R + r) * 2;
                const double cr = sp[0], ci = sp[1];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    acc[p][hh][d][0] += cr * F[d][0] - ci * F[d][1];
                    acc[p][hh][d][1] += cr * F[d][1] + ci * F[d][0];
                }
            }
    }
    __shared__ double red[4][24];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double* flat = &acc[0][0][0][0];
#pragma unroll
    for (int q = 0; q < 24; ++q) {
        double v = ff_wave_sum(flat[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x >= 2) return;
    const int p = threadIdx.x;
    double NL[2][3][2];
    for (int hh = 0; hh < 2; ++hh)
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 2; ++c) {
                double v = 0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][((p * 2 + hh) * 3 + d) * 2 + c];
                NL[hh][d][c] = v;
            }
    const double rh[3] = {dx, dy, dz};
    double res[3][2];
    for (int c = 0; c < 2; ++c) {
        double Nv[3] = {NL[0][0][c], NL[0][1][c], NL[0][2][c]}, Lv[3] = {NL[1][0][c], NL[1][1][c], NL[1][2][c]};
        // rhat x L
        double a1[3] = {rh[1] * Lv[2] - rh[2] * Lv[1], rh[2] * Lv[0] - rh[0] * Lv[2], rh[0] * Lv[1] - rh[1] * Lv[0]};
        // rhat x (rhat x N) = rhat (rhat.N) - N
        const double rn = rh[0] * Nv[0] + rh[1] * Nv[1] + rh[2] * Nv[2];
        for (int d = 0; d < 3; ++d) res[d][c] = a1[d] + (rh[d] * rn - Nv[d]);   // eta = 1
    }
    // times i k / (4 pi)
    const double g = k / (4.0 * M_PI);
    double* o = out + (((size_t)a * R + r) * 2 + p) * 6;
    for (int d = 0; d < 3; ++d) {
        o[2 * d] = -g * res[d][1];
        o[2 * d + 1] = g * res[d][0];
    }
}

}  // namespace

namespace motk_ff {

void phase(mot_handle* h, int first, int count, double omega, double* phi) {
    hipLaunchKernelGGL(k_ff_phase, dim3((count + 255) / 256), dim3(256), 0, h->stream, first, count, omega, h->dt,
                       phi);
}

int chunks(const mot_handle* h, int count, int* chunk) {
    const int E = 2 * h->ne * h->R;
    const int bx = (E + 255) / 256;
    int nch = std::max(1, std::min(count / 16, (2048 + bx - 1) / bx));
    nch = std::max(1, std::min(nch, count));
    *chunk = (count + nch - 1) / nch;
    return (count + *chunk - 1) / *chunk;
}

void spectrum(mot_handle* h, int first, int count, int chunk, int nchunk, const double* phi, double* part) {
    const int E = 2 * h->ne * h->R;
    hipLaunchKernelGGL(k_ff_spectrum, dim3((E + 255) / 256, nchunk), dim3(256), 0, h->stream, h->ne, h->hs, h->n2,
                       h->R, h->Rp, first, count, chunk, h->hist, phi, part);
}

void reduce(mot_handle* h, int nchunk, const double* part, double* X) {
    const int E = 2 * h->ne * h->R;
    hipLaunchKernelGGL(k_ff_reduce, dim3((E + 255) / 256), dim3(256), 0, h->stream, h->ne, h->R, nchunk, part, X);
}

void parts(mot_handle* h, const double* X, const double* PX, double* spec) {
    const int tot = 2 * 2 * h->ne * h->R * 2;
    hipLaunchKernelGGL(k_ff_parts, dim3((tot + 255) / 256), dim3(256), 0, h->stream, h->ne, h->R, h->Tmax / h->dt,
                       X, PX, spec);
}

void field(mot_handle* h, double k, int ndir, const double* dirs, const double* spec, double* out) {
    hipLaunchKernelGGL(k_ff_field, dim3(ndir, h->R), dim3(256), 0, h->stream, h->ne, h->R, k, dirs, h->rq_x,
                       h->rq_f, spec, out);
}

}  // namespace motk_ff
