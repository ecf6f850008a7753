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

// sum the chunks in order, one thread per (element, quantity); X is [ne][8R],
// column ((p * 2 + hh) * 2 + c) * R + r with p 0 for S, 1 for D and c 0 re, 1 im
__global__ void k_ff_reduce(int ne, int R, int nchunk, const double* __restrict__ part, double* __restrict__ X) {
    const int E = 2 * ne * R;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * E) return;
    const size_t ld = (size_t)4 * E;
    double a = 0;
    int c = 0;
    for (; c + 8 <= nchunk; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(c + u) * ld + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; c < nchunk; ++c) a += part[(size_t)c * ld + t];
    const int e = t >> 2, q = t & 3;
    const int r = e % R, m = (e / R) % ne, hh = e / (R * ne);
    const int p = q >> 1, ri = q & 1;
    X[(size_t)m * 8 * R + ((p * 2 + hh) * 2 + ri) * R + r] = a;
}

__device__ __forceinline__ double ff_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// PX = P^Sigma X for the 8R transformed columns, a tall-skinny product: one
// wavefront per two rows of P^Sigma (read once per group of 8 columns), each
// lane striding the row and reading its 8 columns of X (64 contiguous bytes,
// L2-resident), then a wavefront sum.  grid (ceil(ne / 8), 8R / 8).
__global__ __launch_bounds__(256) void k_ff_project(int ne, int hs, int nc, const double* __restrict__ PS,
                                                    const double* __restrict__ X, double* __restrict__ PX) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = (blockIdx.x * 4 + wv) * 2;
    if (m0 >= ne) return;
    const bool two = m0 + 1 < ne;
    const int cg = blockIdx.y * 8;
    const double* a0 = PS + (size_t)m0 * hs;
    const double* a1 = PS + (size_t)(two ? m0 + 1 : m0) * hs;
    double c0[8] = {}, c1[8] = {};
    for (int j = lane; j < ne; j += 64) {
        const double p0 = __builtin_nontemporal_load(a0 + j), p1 = __builtin_nontemporal_load(a1 + j);
        const d2* xr = reinterpret_cast<const d2*>(X + (size_t)j * nc + cg);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const d2 x = xr[u];
            c0[2 * u] += p0 * x.x; c0[2 * u + 1] += p0 * x.y;
            c1[2 * u] += p1 * x.x; c1[2 * u + 1] += p1 * x.y;
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        c0[c] = ff_wave_sum(c0[c]);
        c1[c] = ff_wave_sum(c1[c]);
    }
    if (lane < 8) {
        double v0 = c0[0], v1 = c1[0];
#pragma unroll
        for (int c = 1; c < 8; ++c)
            if (lane == c) { v0 = c0[c]; v1 = c1[c]; }
        PX[(size_t)m0 * nc + cg + lane] = v0;
        if (two) PX[(size_t)(m0 + 1) * nc + cg + lane] = v1;
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

// workgroup (direction a, wave r, edge slice z): radiation vectors F_n(rhat)
// on the 14 quadrature points of each edge of the slice, and the slice's sums
// N and L of both parts to part [ndir][R][nz][24] (part, N or L, xyz, re/im)
__global__ __launch_bounds__(256) void k_ff_radiate(int ne, int R, int per_z, double k,
                                                    const double* __restrict__ dirs, const double* __restrict__ qx,
                                                    const double* __restrict__ qf, const double* __restrict__ spec,
                                                    double* __restrict__ part) {
    const int a = blockIdx.x, r = blockIdx.y, z = blockIdx.z;
    const double dx = dirs[3 * a], dy = dirs[3 * a + 1], dz = dirs[3 * a + 2];
    double acc[2][2][3][2] = {};
    const size_t per = (size_t)2 * ne * R * 2;
    const int n0 = z * per_z, n1 = min(ne, n0 + per_z);
    for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
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
    if (threadIdx.x < 24) {
        double v = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
        part[(((size_t)a * R + r) * gridDim.z + z) * 24 + threadIdx.x] = v;
    }
}

// one thread per (direction, wave, part): the slices summed in order, then
// E = (i k / 4 pi) [rhat x L + eta rhat x (rhat x N)], eta = 1;
// out [ndir][R][2 parts][3][2]
__global__ void k_ff_field(int ndir, int R, int nz, double k, const double* __restrict__ dirs,
                           const double* __restrict__ part, double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ndir * R * 2) return;
    const int p = t % 2, r = (t / 2) % R, a = t / (2 * R);
    double NL[2][3][2] = {};
    const double* src = part + ((size_t)a * R + r) * nz * 24;
    for (int z = 0; z < nz; ++z)
        for (int hh = 0; hh < 2; ++hh)
            for (int d = 0; d < 3; ++d)
                for (int c = 0; c < 2; ++c) NL[hh][d][c] += src[(size_t)z * 24 + ((p * 2 + hh) * 3 + d) * 2 + c];
    const double rh[3] = {dirs[3 * a], dirs[3 * a + 1], dirs[3 * a + 2]};
    const double g = k / (4.0 * M_PI);
    double* o = out + (size_t)t * 6;
    double res[3][2];
    for (int c = 0; c < 2; ++c) {
        double N[3] = {NL[0][0][c], NL[0][1][c], NL[0][2][c]}, L[3] = {NL[1][0][c], NL[1][1][c], NL[1][2][c]};
        // rhat x L, and rhat x (rhat x N) = rhat (rhat.N) - N
        const double rn = rh[0] * N[0] + rh[1] * N[1] + rh[2] * N[2];
        res[0][c] = rh[1] * L[2] - rh[2] * L[1] + rh[0] * rn - N[0];
        res[1][c] = rh[2] * L[0] - rh[0] * L[2] + rh[1] * rn - N[1];
        res[2][c] = rh[0] * L[1] - rh[1] * L[0] + rh[2] * rn - N[2];
    }
    for (int d = 0; d < 3; ++d) {      // times i k / (4 pi)
        o[2 * d] = -g * res[d][1];
        o[2 * d + 1] = g * res[d][0];
    }
}

// ||w_s|| over the unknowns of each kept step s and wave r (the late-time
// behaviour of eq. (MOT)): one workgroup per step, norms [count][R]
__global__ __launch_bounds__(256) void k_step_norms(int ne, int hs, int n2, int R, int Rp, int first,
                                                    const double* __restrict__ hist, double* __restrict__ norms) {
    const int s = blockIdx.x;
    const double* w = hist + (size_t)(first + s) * n2 * Rp;
    __shared__ double red[4];
    for (int r = 0; r < R; ++r) {
        double a = 0;
        for (int i = threadIdx.x; i < 2 * ne; i += blockDim.x) {
            const int row = i < ne ? i : hs + (i - ne);
            const double v = w[(size_t)row * Rp + r];
            a = fma(v, v, a);
        }
        a = ff_wave_sum(a);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
            norms[(size_t)s * R + r] = sqrt(t);
        }
        __syncthreads();
    }
}

}  // namespace

namespace motk_ff {

void step_norms(mot_handle* h, int first, int count, double* norms) {
    hipLaunchKernelGGL(k_step_norms, dim3(count), dim3(256), 0, h->stream, h->ne, h->hs, h->n2, h->R, h->Rp, first,
                       h->hist, norms);
}


void phase(mot_handle* h, int first, int count, double omega, double* phi) {
    hipLaunchKernelGGL(k_ff_phase, dim3((count + 255) / 256), dim3(256), 0, h->stream, first, count, omega, h->dt,
                       phi);
}

int chunks(const mot_handle* h, int count, int* chunk) {
    // at least 64 steps per thread, and about 4096 workgroups at most
    const int E = 2 * h->ne * h->R;
    const int bx = (E + 255) / 256;
    int nch = std::max(1, std::min(count / 64, (4096 + bx - 1) / bx));
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
    hipLaunchKernelGGL(k_ff_reduce, dim3((4 * E + 255) / 256), dim3(256), 0, h->stream, h->ne, h->R, nchunk, part, X);
}

void project(mot_handle* h, const double* X, double* PX) {
    const int nc = 8 * h->R;
    hipLaunchKernelGGL(k_ff_project, dim3((h->ne + 7) / 8, nc / 8), dim3(256), 0, h->stream, h->ne, h->hs, nc, h->PS,
                       X, PX);
}

void parts(mot_handle* h, const double* X, const double* PX, double* spec) {
    const int tot = 2 * 2 * h->ne * h->R * 2;
    hipLaunchKernelGGL(k_ff_parts, dim3((tot + 255) / 256), dim3(256), 0, h->stream, h->ne, h->R, h->Tmax / h->dt,
                       X, PX, spec);
}

int field_slices(const mot_handle* h) { return std::max(1, std::min(64, (h->ne + 255) / 256)); }

void field(mot_handle* h, double k, int ndir, const double* dirs, const double* spec, double* part, double* out) {
    const int nz = field_slices(h);
    const int per_z = (h->ne + nz - 1) / nz;
    hipLaunchKernelGGL(k_ff_radiate, dim3(ndir, h->R, nz), dim3(256), 0, h->stream, h->ne, h->R, per_z, k, dirs,
                       h->rq_x, h->rq_f, spec, part);
    const int tot = ndir * h->R * 2;
    hipLaunchKernelGGL(k_ff_field, dim3((tot + 255) / 256), dim3(256), 0, h->stream, ndir, h->R, nz, k, dirs, part,
                       out);
}

}  // namespace motk_ff
