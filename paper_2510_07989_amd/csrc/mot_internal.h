// Internal declarations of the MOT library (device kernels and host glue).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <atomic>
#include <string>
#include <vector>

#include "../../include/mot.h"

#define MOT_MAXM 64          // largest GMRES restart length
#define MOT_GM_BLOCKS 64     // blocks of the GMRES reduction kernels
#define MOT_CG_CHUNKS 32     // row chunks of column-batched reductions

// ---------------------------------------------------------------- graphs ---
// Incidence of one family of nodes (faces for Sigma, vertices for Lambda):
// edge m joins node plus[m] (+1) and minus[m] (-1).  inc_*: node -> incident
// edges (CSR) with signs; adj_*: node -> neighbour nodes (CSR, one per edge).
struct DevGraph {
    int nnode = 0, ne = 0;
    int* plus = nullptr;
    int* minus = nullptr;
    int* inc_ptr = nullptr;
    int* inc_edge = nullptr;
    double* inc_sign = nullptr;
    int* adj_ptr = nullptr;
    int* adj = nullptr;
};

struct DevCSR {
    int n = 0, nnz = 0;
    int* ptr = nullptr;
    int* col = nullptr;
    double* val = nullptr;
};

// GMRES state in device memory (one right-hand side).
struct GmState {
    double H[(MOT_MAXM + 1) * MOT_MAXM];   // column j at H[j*(M+1) + i]
    double h1[MOT_MAXM + 1];
    double h2[MOT_MAXM + 1];                // re-orthogonalisation coefficients
    double cs[MOT_MAXM], sn[MOT_MAXM], g[MOT_MAXM + 1], y[MOT_MAXM];
    double beta, bnorm, relres, inv_h;
    int j, done, converged, total, cycle_iters, breakdown;
    unsigned int counter;
    int seq;                                // progress words published so far
    // speculative stepping: a finisher whose solve did not converge sets halt
    // (and the step in halt_k); every step kernel returns at entry while it is
    // set.  iters_all counts Arnoldi steps over the whole run.
    int halt, halt_k, iters_all;
    double partial[(MOT_MAXM + 1) * MOT_GM_BLOCKS];
};

// Host-visible progress word written by the device after each Arnoldi step.
struct GmFlag {
    volatile int seq;
    volatile int done;
    volatile int converged;
    volatile int total;
    volatile double relres;
};

// Norm of a GMRES opening (||y||, ||r||) from two sums of squares of its
// entries: the plain one, and one of the entries scaled by 2^600.  The plain
// sum is used while it is at least 2^-960; below that every entry is under
// 2^-480, its scaled square cannot overflow, and the scaled sum keeps the
// digits that the plain one loses once the squares fall below the normal
// range (entries under ~1.5e-154, which late steps of a decaying march reach).
// An inaccurate norm would leave the first Krylov vector off unit length,
// after which the Gram-Schmidt steps cannot bring the residual to tolerance.
// Norms at or below MOT_ZERO_NORM count as a zero right-hand side (x = 0):
// their reciprocal would overflow.
#define MOT_NORM_SCALE 0x1p600
#define MOT_ZERO_NORM 0x1p-1000
__device__ __forceinline__ double sq_scaled(double v) {
    const double t = v * MOT_NORM_SCALE;
    return t * t;
}
__device__ __forceinline__ double open_norm(double plain, double scaled) {
    return plain >= 0x1p-960 ? sqrt(plain) : sqrt(scaled) * 0x1p-600;
}

// --------------------------------------------------------- kernel entry ---
namespace motk {
// dense
// C_z = alpha A B_z + beta C_z for z < batch, B_z = B + z sB, C_z = C + z sC
void gemm(hipStream_t s, int M, int N, int K, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc, int batch = 1, size_t sB = 0,
          size_t sC = 0);
void axpby2d(hipStream_t s, int rows, int cols, double a, const double* X, int ldx, double b,
             double* Y, int ldy);                       // Y = a X + b Y
void fill2d(hipStream_t s, int rows, int cols, double v, double* Y, int ldy);
// number of non-finite entries of X (synchronises s); -1 on a HIP error
int count_nonfinite(hipStream_t s, int rows, int cols, const double* X, int64_t ldx, int* d_count);
void set_identity(hipStream_t s, int n, double* Y, int ldy);
void scatter_csr_add(hipStream_t s, int n, const int64_t* ptr, const int* col, const double* val,
                     double a, double* Y, int ldy);     // Y += a * CSR
// column-batched ops on [rows][ncol] row-major arrays (ld = ncol)
void spmm_csr(hipStream_t s, const DevCSR& A, int ncol, const double* X, double* Y);
void spmm_lap(hipStream_t s, const DevGraph& g, int ncol, const double* X, double* Y);
void inc_T(hipStream_t s, const DevGraph& g, int ncol, const double* X, int ldx, double* S);
void inc_apply(hipStream_t s, const DevGraph& g, int ncol, const double* Z, double* Y, int ldy);
void coldot(hipStream_t s, int rows, int ncol, const double* A, const double* B, double* part,
            double* out);                               // out[c] = sum_i A[i,c] B[i,c]
void cg_update(hipStream_t s, int rows, int ncol, const double* alpha, const double* P,
               const double* Q, double* X, double* R, double* part);
void cg_scalars(hipStream_t s, int ncol, const double* pq, const double* rr_new_part, int nchunk,
                double* rr, double* rr0, double* alpha, double* beta, int* active, double tol,
                int phase);
void cg_pupdate(hipStream_t s, int rows, int ncol, const double* beta, const double* R, double* P);
int count_active(hipStream_t s, int ncol, const int* active, int* d_count, int* h_count);
void col_center(hipStream_t s, int rows, int ncol, double* X);
}  // namespace motk

// Event pairs bracketing one kernel's launches (profile mode).
struct EvPool {
    std::vector<hipEvent_t> a, b;
    int used = 0;
    double ms = 0;
    long long n = 0;
    long long seen = 0;              // launches offered for timing (sampling)
    bool open = false;               // the current launch is bracketed
};

// ------------------------------------------------------------ the handle ---
struct mot_handle {
    hipStream_t stream = nullptr;
    std::string err;
    mot_options opt;
    int nv = 0, nf = 0, ne = 0, hs = 0, n2 = 0, R = 1;
    int Rp = 1;                      // internal column count (R rounded up to a power of two >= 4, or 1)
    double eps_r = 1, mu_r = 1, dt = 1, D = 0, Tmax = 0;
    double c = 1, eta = 1, cp = 1, etap = 1;
    int kmax = 0, nlags = 0, nh = 0, genus = 0;
    double setup_ms = 0, fold_ms = 0;
    uint64_t bytes = 0;
    uint64_t peak_bytes = 0;         // high-water mark of bytes
    std::atomic<int> cancel{0};      // mot_cancel: stop the run at its next window boundary
    int device = -1;                 // HIP device current at create
    double* scratch = nullptr;       // this device's static scratch array (mot_step_norms_noalloc)
    std::vector<void*> allocs;
    std::vector<size_t> sizes;

    DevGraph gf, gv;                 // faces (Sigma), vertices (Lambda)
    DevCSR G, GT;
    // RHS quadrature geometry: per (edge, side, point)
    double* rq_x = nullptr;          // [ne][2][7][3]
    double* rq_f = nullptr;          // [ne][2][7][3]   weight * RWG value
    double* waves = nullptr;         // [R][9]: amp, pol(3), dir(3), width, t0
    double* tcut = nullptr;          // [R]

    double *PS = nullptr, *BL = nullptr, *Ginv = nullptr, *C1 = nullptr, *C2 = nullptr;
    double* Q = nullptr;             // [nlags][3][ne][hs]: q1, qk, q2 per lag

    // lag staging: per lag, per family, 3 media-summed blocks [3][ne][hs]
    std::vector<double*> stage;      // index lag*3 + family
    std::vector<uint32_t> got;       // arrival bits per lag: family*4 + medium*2 + op
    std::vector<char> lag_done;
    // history_form 1: the staged families of lags >= 1 kept (rawZ[lag*3 + f],
    // a device copy of the table in rawZtab), the projected unknowns in rings,
    // and the two family sums
    std::vector<double*> rawZ;
    double** rawZtab = nullptr;
    double *rawL = nullptr, *rawS = nullptr;   // [nh][n2]: P^{Lambda H} w, P^Sigma w
    double *ry1 = nullptr, *ry2 = nullptr;     // [n2]
    int rawtab_ok = 0;
    double* tmp = nullptr;           // [3][ne][hs] fold temporaries
    double* raw = nullptr;           // [ne][hs] upload buffer

    // march state
    int* d_k = nullptr;              // [0] current step, [1] first step of a graph-replayed window (device)
    int k = 0;
    double* ring = nullptr;          // [nh][n2][R]
    double* hist = nullptr;          // [max_steps][n2][R]
    int hist_cap = 0;
    int hist_first = 0;              // first kept step that holds data (after a restore without history)
    int B = 128;                     // steps per RHS batch
    // launch schedules of the one-RHS streaming products (fixed by options or
    // picked by the autotuner):  1, 2, 4: that many wavefronts share one
    // matrix row (history: whole rows of one lag block at a time);  10 + r:
    // one wavefront owns r rows (history: column slices across all lag blocks;
    // 11 is the four-wavefront workgroup form);  history 22, 24: 2 or 4
    // wavefronts share a row's column slices across all lag blocks; 32, 34:
    // 2 or 4 wavefronts share as many rows
    int sch_hist = 11;
    int sch_q0 = 1;
    int sch_pc = 1;
    int tune_hist = 0, tune_mv = 0;  // 1: that part of the schedule is tuned
    int tuned = 0;
    double tune_ms = 0;
    // speculative windows captured as HIP graphs, one per batch parity of the
    // window's RHS half; captured with spec_iters Arnoldi steps per step
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int g_iters[2] = {0, 0};
    int graph_off = 0;               // capture failed (e.g. the legacy default stream): stream launches
    long long graph_windows = 0;
    double* ebar = nullptr;          // [2][hs][B] tested fields of a batch
    double* Ebar = nullptr;
    double* rb = nullptr;            // [2][ne][B] r_k = C1 ebar + C2 Ebar / T_max
    double* y = nullptr;             // rhs - history
    double* x = nullptr;             // solution of the step
    // GMRES workspace (R = 1 path)
    double* V = nullptr;             // [M+1][n2]
    double* Z = nullptr;             // [M+1][n2]  preconditioned basis M v_j
    float* M32 = nullptr;            // [n2][n2]   approximate Q_0^-1 (FP32); 16x16 tiles when Rp > 1
    double* M64 = nullptr;           // [n2][n2]   approximate Q_0^-1 (FP64); 16x16 tiles when Rp > 1
    int ns_iters = 0;                // Newton-Schulz iterations used
    double ns_resid = 0;             // ||I - M Q_0||_F reached
    double* wA = nullptr;
    double* wB = nullptr;
    GmState* gm = nullptr;           // single-RHS state, aggregate state when R > 1
    GmState* gms = nullptr;          // [Rp] per-column states (R > 1)
    double* mr_part = nullptr;       // split-K partial products (R > 1)
    // multi-RHS tile-major lag storage (16 x 16 tiles, see multi.hip)
    int G16 = 0, KT = 0;             // row groups and summation tiles per block
    double* Qt = nullptr;            // FP64 tiles: lags 0..nh (FP64 path) or lag 0 (mixed)
    float* QtF = nullptr;            // FP32 tiles of lags 1..nh (mixed paths)
    float* QtL = nullptr;            // FP32 low parts fl(Q - fl(Q)) of lags 1..hilo
    int hilo = 0;                    // lags with a low part
    int spec_iters = 1;              // Arnoldi steps queued per speculative step
    int hist_kc = 1, q0_kc = 1;      // K chunks of the tile products
    int hist_wg = 4, q0_wg = 4;      // wavefronts per workgroup of the tile products (4 or 8)
    int plain_kc = 1;                // K chunks of the preconditioner product (Rp > 1)
    std::vector<int> hist_kc_c, q0_kc_c, plain_kc_c;   // autotuner candidates (Rp > 1)
    int orth_nb = 1, orth_rb = 1;    // workgroups and rows of the multi-RHS Krylov sweeps
    double* orth_part = nullptr;     // [orth_nb][MOT_MAXM + 1][Rp] per-workgroup column sums
    GmFlag* hflag = nullptr;         // pinned, device-mapped
    GmFlag* dflag = nullptr;
    int M = 40;
    long long iters_total = 0;
    double recover_ms = 0;
    EvPool ev_hist, ev_q0;
    int last_iters = 0;
    double last_relres = 0;
    int last_conv = 1;
};

// host glue implemented in mot_api.hip
int mot_fail(mot_handle* h, int code, const std::string& msg);

// return MOT_EHIP (with the call's text) from the enclosing function on a HIP error
#define HIPCHK(h, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return mot_fail(h, MOT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

// launch-schedule autotuner (tune.hip): times the candidates of every tuned
// product on the handle's stream once all lags are folded; returns MOT_OK or
// MOT_EHIP
int mot_autotune(mot_handle* h);

// far field of the kept currents (farfield.hip); every launcher queues on the
// handle's stream.  X and PX are [ne][8R]; spec is [2 parts][2 ne][R][2].
namespace motk_ff {
void phase(mot_handle* h, int first, int count, double omega, double* phi);     // phi [count][2]
int chunks(const mot_handle* h, int count, int* chunk);                         // step chunks of the pass
void spectrum(mot_handle* h, int first, int count, int chunk, int nchunk, const double* phi, double* part);
void reduce(mot_handle* h, int nchunk, const double* part, double* X);
void project(mot_handle* h, const double* X, double* PX);                      // PX = P^Sigma X (dense P^Sigma)
void parts(mot_handle* h, const double* X, const double* PX, double* spec);
void step_norms(mot_handle* h, int first, int count, double* norms);          // norms [count][R]
int field_slices(const mot_handle* h);                                          // edge slices of the field pass
void field(mot_handle* h, double k, int ndir, const double* dirs, const double* spec, double* part, double* out);
}  // namespace motk_ff
