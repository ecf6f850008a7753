// C ABI of the MOT solver: validation, device setup, lag fold, march, recovery.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <algorithm>
#include <mutex>
#include <thread>

#include "mot_internal.h"

namespace motk_step {
void rhs_batch(mot_handle* h, int k0, double* rb, const int* kbase = nullptr);
void history(mot_handle* h);
void raw_history(mot_handle* h);
void raw_reproject(mot_handle* h);
void gm_start1(mot_handle* h, const double* b, double* r, int have_t, int first, double* xzero, int publish = 1);
void gm_orth1(mot_handle* h, double* w, int publish = 1, int fin_kq = 0);
void gm_finish(mot_handle* h, const double* basis, int force, int spec = 0, int kq = 0);
void q0_matvec(mot_handle* h, const double* src, double* vout, double* y, int check_done, int use_inv);
void precond(mot_handle* h, const double* src, double* vj, double* z, bool start = false);
void dense_q0(mot_handle* h, double* D);
void transpose_scale(mot_handle* h, int n, double alpha, const double* A, double* X);
void abs_sums(mot_handle* h, int n, const double* A, double* rs, double* cs);
void eye_residual(mot_handle* h, int n, const double* T, double* out);
void to_f32(mot_handle* h, size_t n, const double* X, float* Y);
void gm_residual(mot_handle* h, const double* b, double* r, int first);
void gm_dots(mot_handle* h, const double* w);
void gm_orth(mot_handle* h, double* w, int final_pass);
void gm_update_x(mot_handle* h, const double* basis, double* x);
void warm_start(mot_handle* h);
void push(mot_handle* h);
void inc_step(mot_handle* h);
void clear_halt(mot_handle* h);
void set_step(mot_handle* h, int k);
void set_base(mot_handle* h, int k);
void rec_gather(mot_handle* h, int s0, int ns, double* X);
void rec_scatter(mot_handle* h, int ns, const double* X, const double* PX, double* loop, double* star);
void pack(mot_handle* h, int ns, const double* src, double* dst);
}  // namespace motk_step

namespace motk_multi {
size_t part_doubles(const mot_handle* h);
void history_gemm(mot_handle* h);
void history_reduce(mot_handle* h);
void q0_gemm(mot_handle* h, const double* X);
void q0_reduce(mot_handle* h, double* out);
void precond(mot_handle* h, const double* src, double* vj, double* z);
void start(mot_handle* h, const double* y, double* r, int have_t, int first, double* xzero, int publish = 1);
void orth(mot_handle* h, double* w, int publish = 1);
void finish(mot_handle* h, int force, int spec = 0, int kq = 0);
void plan_tiles(mot_handle* h);
size_t tile_elems(const mot_handle* h);
void pack_lag(mot_handle* h, int lag);
void pack_square(mot_handle* h, const double* X, double* t64, float* t32);
size_t orth_part_doubles(const mot_handle* h);
}  // namespace motk_multi

static thread_local std::string g_create_err;   // create errors, per host thread

int mot_fail(mot_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg; else g_create_err = msg;
    return code;
}


namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device memory comes from the stream-ordered pool on the handle's stream: a
// free does not synchronise the device, so solves sharing one GPU keep running
// while another sets up, recovers or is destroyed.
template <class T>
int dalloc(mot_handle* h, T** p, size_t count, bool zero = true) {
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 16;
    if (h->opt.mem_cap_bytes && h->bytes + bytes > h->opt.mem_cap_bytes)
        return mot_fail(h, MOT_ENOMEM, "device memory cap exceeded");
    void* q = nullptr;
    if (hipMallocAsync(&q, bytes, h->stream) != hipSuccess) {
        (void)hipGetLastError();
        return mot_fail(h, MOT_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    if (zero && hipMemsetAsync(q, 0, bytes, h->stream) != hipSuccess)
        return mot_fail(h, MOT_EHIP, "hipMemsetAsync failed");
    h->allocs.push_back(q);
    h->sizes.push_back(bytes);
    h->bytes += bytes;
    h->peak_bytes = std::max(h->peak_bytes, h->bytes);
    *p = static_cast<T*>(q);
    return MOT_OK;
}

void dfree(mot_handle* h, void* p) {
    if (!p) return;
    auto it = std::find(h->allocs.begin(), h->allocs.end(), p);
    if (it != h->allocs.end()) {
        size_t i = it - h->allocs.begin();
        h->bytes -= h->sizes[i];
        h->allocs.erase(it);
        h->sizes.erase(h->sizes.begin() + i);
    }
    (void)hipFreeAsync(p, h->stream);
}

template <class T>
int upload(mot_handle* h, T** d, const T* src, size_t count) {
    int rc = dalloc(h, d, count, false);
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(*d, src, count * sizeof(T), hipMemcpyHostToDevice, h->stream));
    return MOT_OK;
}

// Build an incidence graph: nodes with incident signed edges and neighbours.
int make_graph(mot_handle* h, DevGraph& g, int nnode, const std::vector<int>& plus,
               const std::vector<int>& minus) {
    int ne = (int)plus.size();
    std::vector<int> deg(nnode, 0);
    for (int m = 0; m < ne; ++m) { deg[plus[m]]++; deg[minus[m]]++; }
    std::vector<int> ptr(nnode + 1, 0);
    for (int i = 0; i < nnode; ++i) ptr[i + 1] = ptr[i] + deg[i];
    std::vector<int> edge(ptr[nnode]), adj(ptr[nnode]);
    std::vector<double> sign(ptr[nnode]);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int m = 0; m < ne; ++m) {
        int a = plus[m], b = minus[m];
        edge[fill[a]] = m; sign[fill[a]] = 1.0; adj[fill[a]] = b; fill[a]++;
        edge[fill[b]] = m; sign[fill[b]] = -1.0; adj[fill[b]] = a; fill[b]++;
    }
    g.nnode = nnode;
    g.ne = ne;
    int rc;
    if ((rc = upload(h, &g.plus, plus.data(), ne))) return rc;
    if ((rc = upload(h, &g.minus, minus.data(), ne))) return rc;
    if ((rc = upload(h, &g.inc_ptr, ptr.data(), nnode + 1))) return rc;
    if ((rc = upload(h, &g.inc_edge, edge.data(), edge.size()))) return rc;
    if ((rc = upload(h, &g.inc_sign, sign.data(), sign.size()))) return rc;
    if ((rc = upload(h, &g.adj_ptr, ptr.data(), nnode + 1))) return rc;
    if ((rc = upload(h, &g.adj, adj.data(), adj.size()))) return rc;
    return MOT_OK;
}

// Column-batched CG.  op(X) -> Y on [rows][ncol]; solves op(X) = B from X = 0.
// Returns MOT_OK or MOT_ENOCONV.
template <class Op>
int batched_cg(mot_handle* h, int rows, int ncol, const double* B, double* X, Op op, double tol,
               int maxit) {
    hipStream_t s = h->stream;
    size_t N = (size_t)rows * ncol;
    double *R, *P, *Q, *part, *rr, *rr0, *alpha, *beta, *pq;
    int *active, *dcount;
    int rc;
    if ((rc = dalloc(h, &R, N, false)) || (rc = dalloc(h, &P, N, false)) || (rc = dalloc(h, &Q, N, false)) ||
        (rc = dalloc(h, &part, (size_t)MOT_CG_CHUNKS * ncol, false)) || (rc = dalloc(h, &rr, ncol)) ||
        (rc = dalloc(h, &rr0, ncol)) || (rc = dalloc(h, &alpha, ncol)) || (rc = dalloc(h, &beta, ncol)) ||
        (rc = dalloc(h, &pq, ncol)) || (rc = dalloc(h, &active, ncol)) || (rc = dalloc(h, &dcount, 1)))
        return rc;
    HIPCHK(h, hipMemsetAsync(X, 0, N * sizeof(double), s));
    HIPCHK(h, hipMemcpyAsync(R, B, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(P, B, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    motk::coldot(s, rows, ncol, R, R, part, pq);   // pq used as scratch for the sums
    motk::cg_scalars(s, ncol, pq, part, MOT_CG_CHUNKS, rr, rr0, alpha, beta, active, tol, 2);
    int it = 0, hcount = ncol;
    int result = MOT_OK;
    for (; it < maxit; ++it) {
        op(P, Q);
        motk::coldot(s, rows, ncol, P, Q, part, pq);
        motk::cg_scalars(s, ncol, pq, part, MOT_CG_CHUNKS, rr, rr0, alpha, beta, active, tol, 0);
        motk::cg_update(s, rows, ncol, alpha, P, Q, X, R, part);
        motk::cg_scalars(s, ncol, pq, part, MOT_CG_CHUNKS, rr, rr0, alpha, beta, active, tol, 1);
        motk::cg_pupdate(s, rows, ncol, beta, R, P);
        if ((it + 1) % 16 == 0) {
            if (motk::count_active(s, ncol, active, dcount, &hcount)) return mot_fail(h, MOT_EHIP, "cg sync");
            if (hcount == 0) break;
        }
    }
    if (it == maxit) {
        if (motk::count_active(s, ncol, active, dcount, &hcount)) return mot_fail(h, MOT_EHIP, "cg sync");
        if (hcount) result = mot_fail(h, MOT_ENOCONV, "CG did not converge on " + std::to_string(hcount) + " columns");
    }
    HIPCHK(h, hipStreamSynchronize(s));
    for (void* p : {(void*)R, (void*)P, (void*)Q, (void*)part, (void*)rr, (void*)rr0, (void*)alpha,
                    (void*)beta, (void*)pq, (void*)active, (void*)dcount})
        dfree(h, p);
    return result;
}

// Dense projector Inc (Inc^T Inc)^+ Inc^T as [ne][hs] (Section IV-B), in column chunks.
int dense_projector(mot_handle* h, const DevGraph& g, double* Pout) {
    const int ne = h->ne, hs = h->hs;
    const int chunk = std::min(ne, 4096);
    double *E, *S, *Z, *Y;
    int rc;
    if ((rc = dalloc(h, &E, (size_t)ne * chunk)) || (rc = dalloc(h, &S, (size_t)g.nnode * chunk)) ||
        (rc = dalloc(h, &Z, (size_t)g.nnode * chunk)) || (rc = dalloc(h, &Y, (size_t)ne * chunk)))
        return rc;
    for (int c0 = 0; c0 < ne; c0 += chunk) {
        int nc = std::min(chunk, ne - c0);
        // E = identity columns c0 .. c0+nc
        motk::fill2d(h->stream, ne, nc, 0.0, E, nc);
        motk::set_identity(h->stream, nc, E + (size_t)c0 * nc, nc);   // E[c0 + i][i] = 1
        motk::inc_T(h->stream, g, nc, E, nc, S);
        motk::col_center(h->stream, g.nnode, nc, S);
        auto lap = [&](const double* X, double* Yo) { motk::spmm_lap(h->stream, g, nc, X, Yo); };
        rc = batched_cg(h, g.nnode, nc, S, Z, lap, h->opt.cg_tol, h->opt.cg_maxit);
        if (rc) return rc;
        motk::inc_apply(h->stream, g, nc, Z, Y, nc);
        // column c0 + i of the projector: P[m][c0 + i] = Y[m][i]
        HIPCHK(h, hipMemcpy2DAsync(Pout + c0, hs * sizeof(double), Y, nc * sizeof(double), nc * sizeof(double), ne,
                         hipMemcpyDeviceToDevice, h->stream));
    }
    dfree(h, E); dfree(h, S); dfree(h, Z); dfree(h, Y);
    return MOT_OK;
}

// G^-1 as [ne][hs]: CG on G^T G X = G^T I (normal equations; kappa(G) is small).
int gram_inverse(mot_handle* h) {
    const int ne = h->ne, hs = h->hs;
    const int chunk = std::min(ne, 4096);
    double *Bm, *X, *T;
    int rc;
    if ((rc = dalloc(h, &Bm, (size_t)ne * chunk)) || (rc = dalloc(h, &X, (size_t)ne * chunk)) ||
        (rc = dalloc(h, &T, (size_t)ne * chunk)))
        return rc;
    for (int c0 = 0; c0 < ne; c0 += chunk) {
        int nc = std::min(chunk, ne - c0);
        // B = G^T e_{c0+i}: rows of G^T ... computed as spmm with G^T on identity columns
        motk::fill2d(h->stream, ne, nc, 0.0, X, nc);
        motk::set_identity(h->stream, nc, X + (size_t)c0 * nc, nc);
        motk::spmm_csr(h->stream, h->GT, nc, X, Bm);
        auto op = [&](const double* P, double* Yo) {
            motk::spmm_csr(h->stream, h->G, nc, P, T);
            motk::spmm_csr(h->stream, h->GT, nc, T, Yo);
        };
        rc = batched_cg(h, ne, nc, Bm, X, op, h->opt.cg_tol * 1e-1, h->opt.cg_maxit);
        if (rc) return rc;
        HIPCHK(h, hipMemcpy2DAsync(h->Ginv + c0, hs * sizeof(double), X, nc * sizeof(double), nc * sizeof(double), ne,
                         hipMemcpyDeviceToDevice, h->stream));
    }
    dfree(h, Bm); dfree(h, X); dfree(h, T);
    return MOT_OK;
}

int fam_limit(const mot_handle* h, int fam) {
    return fam == MOT_FAM_H ? h->kmax : (fam == MOT_FAM_HAT ? h->kmax + 1 : h->kmax - 1);
}

uint32_t required_bits(const mot_handle* h, int lag) {
    uint32_t b = 0;
    for (int f = 0; f < 3; ++f)
        if (lag <= fam_limit(h, f)) b |= 0xFu << (4 * f);
    return b;
}

// Approximate inverse of Q_0 by the Newton-Schulz iteration
//   X_0 = Q_0^T / (||Q_0||_1 ||Q_0||_inf),  X_{k+1} = 2 X_k - X_k Q_0 X_k,
// whose residual I - X_k Q_0 squares every step; stopped when ||I - X Q_0||_F
// stops decreasing or drops below 1e-13 sqrt(n).  Used only as the right
// preconditioner of the FP64 GMRES, so its accuracy sets the iteration count,
// never the solution.
int build_precond(mot_handle* h) {
    if (h->opt.precond == 0) return MOT_OK;
    const int n = h->n2;
    const size_t nn = (size_t)n * n;
    hipStream_t s = h->stream;
    double *Q0, *X, *T, *Xn, *rs, *cs, *acc;
    int rc;
    if ((rc = dalloc(h, &Q0, nn, false)) || (rc = dalloc(h, &X, nn, false)) || (rc = dalloc(h, &T, nn, false)) ||
        (rc = dalloc(h, &Xn, nn, false)) || (rc = dalloc(h, &rs, n)) || (rc = dalloc(h, &cs, n)) ||
        (rc = dalloc(h, &acc, 1)))
        return rc;
    motk_step::dense_q0(h, Q0);
    motk_step::abs_sums(h, n, Q0, rs, cs);
    std::vector<double> hr(n), hc(n);
    HIPCHK(h, hipMemcpyAsync(hr.data(), rs, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(hc.data(), cs, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    double ninf = *std::max_element(hr.begin(), hr.end()), n1 = *std::max_element(hc.begin(), hc.end());
    // X_0 = alpha Q_0^T converges for 0 < alpha < 2 / sigma_max^2 and the
    // closer alpha is to 1 / sigma_max^2 the fewer steps it takes; ||Q_0||_1
    // ||Q_0||_inf bounds sigma_max^2 but may exceed it by a factor up to n, so
    // sigma_max^2 is estimated by power iteration on Q_0^T Q_0 (from below;
    // alpha = 1 / (1.05 estimate)), the norm bound kept as the fallback.
    const double t_ns = now_ms();
    double alpha = 1.0 / (n1 * ninf), sig2 = 0;
    {
        double *v, *y, *z;
        if ((rc = dalloc(h, &v, n, false)) || (rc = dalloc(h, &y, n, false)) || (rc = dalloc(h, &z, n, false)))
            return rc;
        std::vector<double> hv(n), hz(n);
        for (int i = 0; i < n; ++i) hv[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3);      // deterministic start
        double nv = 0;
        for (double a : hv) nv += a * a;
        for (double& a : hv) a /= std::sqrt(nv);
        for (int pit = 0; pit < 16; ++pit) {
            HIPCHK(h, hipMemcpyAsync(v, hv.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
            motk::gemm(s, n, 1, n, 1.0, Q0, n, v, 1, 0.0, y, 1);             // y = Q_0 v
            motk::gemm(s, 1, n, n, 1.0, y, n, Q0, n, 0.0, z, n);             // z^T = y^T Q_0
            HIPCHK(h, hipMemcpyAsync(hz.data(), z, n * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            double nz = 0;
            for (double a : hz) nz += a * a;
            nz = std::sqrt(nz);
            if (!(nz > 0) || !std::isfinite(nz)) break;
            sig2 = nz;                                                       // ||Q_0^T Q_0 v||, v unit
            for (int i = 0; i < n; ++i) hv[i] = hz[i] / nz;
        }
        dfree(h, v); dfree(h, y); dfree(h, z);
        if (sig2 > 0 && 1.0 / (1.05 * sig2) > alpha) alpha = 1.0 / (1.05 * sig2);
    }
    double best = 1e300, first = -1;
    int it = 0;
    motk_step::transpose_scale(h, n, alpha, Q0, X);
    for (; it < 120; ++it) {
        motk::gemm(s, n, n, n, 1.0, X, n, Q0, n, 0.0, T, n);               // T = X Q0
        HIPCHK(h, hipMemsetAsync(acc, 0, sizeof(double), s));
        motk_step::eye_residual(h, n, T, acc);
        double e2 = 0;
        HIPCHK(h, hipMemcpyAsync(&e2, acc, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        double e = std::sqrt(e2);
        if (first < 0) first = e;
        if (!std::isfinite(e) || (e > 2 * first && alpha != 1.0 / (n1 * ninf))) {
            // the estimate let the iteration grow: restart from the norm bound
            alpha = 1.0 / (n1 * ninf);
            motk_step::transpose_scale(h, n, alpha, Q0, X);
            best = 1e300; first = -1;
            continue;
        }
        // down to the rounding floor, so that one GMRES step per time step suffices
        if (e < 1e-15 * std::sqrt((double)n) || (e > 0.5 * best && best < 1e-6)) { best = std::min(best, e); break; }
        best = std::min(best, e);
        HIPCHK(h, hipMemcpyAsync(Xn, X, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
        motk::gemm(s, n, n, n, -1.0, T, n, X, n, 2.0, Xn, n);              // Xn = 2X - T X
        std::swap(X, Xn);
    }
    h->setup_ms += now_ms() - t_ns;
    h->ns_iters = it;
    h->ns_resid = best;
    if (!(best < 0.5)) return mot_fail(h, MOT_ENOCONV, "Newton-Schulz did not converge");
    // several waves: stored in 16 x 16 tiles for the MFMA products (same bytes)
    if (h->opt.precond == 2) {
        if ((rc = dalloc(h, &h->M64, nn, false))) return rc;
        if (h->Rp > 1) motk_multi::pack_square(h, X, h->M64, nullptr);
        else HIPCHK(h, hipMemcpyAsync(h->M64, X, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        if ((rc = dalloc(h, &h->M32, nn, false))) return rc;
        if (h->Rp > 1) motk_multi::pack_square(h, X, nullptr, h->M32);
        else motk_step::to_f32(h, nn, X, h->M32);
    }
    HIPCHK(h, hipStreamSynchronize(s));
    dfree(h, Q0); dfree(h, X); dfree(h, T); dfree(h, Xn); dfree(h, rs); dfree(h, cs); dfree(h, acc);
    return MOT_OK;
}

bool all_folded(const mot_handle* h) {
    for (int i = 0; i < h->nlags; ++i)
        if (!h->lag_done[i]) return false;
    return true;
}

// After a lag is folded (or kept raw): once every lag is in, the table of the
// kept raw families goes to the device, then the launch schedule is tuned.
int raw_ready(mot_handle* h) {
    if (!all_folded(h)) return MOT_OK;
    if (h->opt.history_form == 1 && !h->rawtab_ok) {
        HIPCHK(h, hipMemcpyAsync(h->rawZtab, h->rawZ.data(), h->rawZ.size() * sizeof(double*),
                                 hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        h->rawtab_ok = 1;
    }
    if (!h->tuned) return mot_autotune(h);
    return MOT_OK;
}

// Section V-B fold of lag i:  with blocks X in {1 = eta T + eta' T', k = K + K', 2 = T/eta + T'/eta'}
//   a_X = Zh_X + (Zhat_X - Zh_X) P^Sigma,  b_X = Ztil_X + (Zh_X - Ztil_X) P^Sigma
//   q_X = C1 a_X + C2 b_X                 (Q_i = [[q_1, -q_k], [q_k, q_2]])
int fold_lag(mot_handle* h, int lag) {
    double t0 = now_ms();
    if (h->opt.history_form == 1 && lag > 0) {
        // kept as staged (media summed, time-scaled); applied by the history
        for (int f = 0; f < 3; ++f) {
            h->rawZ[(size_t)lag * 3 + f] = h->stage[(size_t)lag * 3 + f];
            h->stage[(size_t)lag * 3 + f] = nullptr;
        }
        h->lag_done[lag] = 1;
        h->fold_ms += now_ms() - t0;
        return raw_ready(h);
    }
    const int ne = h->ne, hs = h->hs;
    const size_t blk = (size_t)ne * hs;
    hipStream_t s = h->stream;
    double* Zf[3];
    for (int f = 0; f < 3; ++f) Zf[f] = h->stage[(size_t)lag * 3 + f];   // may be null (zero)
    double* D = h->tmp;
    double* A = h->tmp + blk;
    double* Bv = h->tmp + 2 * blk;
    for (int x = 0; x < 3; ++x) {
        const double* zh = Zf[0] ? Zf[0] + x * blk : nullptr;
        const double* zt = Zf[1] ? Zf[1] + x * blk : nullptr;   // hat
        const double* zl = Zf[2] ? Zf[2] + x * blk : nullptr;   // tilde
        // D = Zhat - Zh ; A = Zh + D PS
        motk::fill2d(s, ne, hs, 0.0, D, hs);
        if (zt) motk::axpby2d(s, ne, hs, 1.0, zt, hs, 1.0, D, hs);
        if (zh) motk::axpby2d(s, ne, hs, -1.0, zh, hs, 1.0, D, hs);
        motk::fill2d(s, ne, hs, 0.0, A, hs);
        if (zh) motk::axpby2d(s, ne, hs, 1.0, zh, hs, 0.0, A, hs);
        motk::gemm(s, ne, ne, ne, 1.0, D, hs, h->PS, hs, 1.0, A, hs);
        // D = Zh - Ztil ; B = Ztil + D PS
        motk::fill2d(s, ne, hs, 0.0, D, hs);
        if (zh) motk::axpby2d(s, ne, hs, 1.0, zh, hs, 1.0, D, hs);
        if (zl) motk::axpby2d(s, ne, hs, -1.0, zl, hs, 1.0, D, hs);
        motk::fill2d(s, ne, hs, 0.0, Bv, hs);
        if (zl) motk::axpby2d(s, ne, hs, 1.0, zl, hs, 0.0, Bv, hs);
        motk::gemm(s, ne, ne, ne, 1.0, D, hs, h->PS, hs, 1.0, Bv, hs);
        // q = C1 A + C2 B
        double* q = h->Q + ((size_t)lag * 3 + x) * blk;
        motk::gemm(s, ne, ne, ne, 1.0, h->C1, hs, A, hs, 0.0, q, hs);
        motk::gemm(s, ne, ne, ne, 1.0, h->C2, hs, Bv, hs, 1.0, q, hs);
    }
    HIPCHK(h, hipStreamSynchronize(s));
    for (int f = 0; f < 3; ++f) {
        if (Zf[f]) dfree(h, Zf[f]);
        h->stage[(size_t)lag * 3 + f] = nullptr;
    }
    if (h->Rp > 1) {
        motk_multi::pack_lag(h, lag);
        HIPCHK(h, hipStreamSynchronize(s));
    }
    h->lag_done[lag] = 1;
    h->fold_ms += now_ms() - t0;
    if (lag == 0) {
        int rc = build_precond(h);
        if (rc) return rc;
    }
    return raw_ready(h);
}

int stage_add(mot_handle* h, int family, int lag, int medium, int op, const double* dev_block, int64_t ldb) {
    const int ne = h->ne, hs = h->hs;
    const size_t blk = (size_t)ne * hs;
    double*& S = h->stage[(size_t)lag * 3 + family];
    if (!S) {
        int rc = dalloc(h, &S, 3 * blk);
        if (rc) return rc;
    }
    // Eq. (spec_prop): T^Lambda G^-1 P^{Lambda H} K_0 P^{Lambda H} = 0 for the
    // static double layer K_0, so the tilde K blocks that equal their constant
    // tail dt K_0 add nothing to Q_i^sl (the paper drops them beyond k_max - 1,
    // where the family is truncated).  With k_max = 1 (c_min dt >= D) every
    // pair lies in the first shell, where the integral of p_0 is dt - R/c and
    // its constant part has no gradient: the lag-0 tilde K block is exactly
    // dt K_0 and is dropped too, so that its quadrature error, amplified by
    // dt / T_max, stays out of Q_0.
    if (family == MOT_FAM_TILDE && op == MOT_OP_K && lag == 0 && h->kmax <= 1) return MOT_OK;
    double sc = family == MOT_FAM_HAT ? h->Tmax : (family == MOT_FAM_TILDE ? 1.0 / h->Tmax : 1.0);
    double et = medium == MOT_EXT ? h->eta : h->etap;
    if (op == MOT_OP_T) {
        motk::axpby2d(h->stream, ne, ne, sc * et, dev_block, (int)ldb, 1.0, S, hs);          // q1 slot
        motk::axpby2d(h->stream, ne, ne, sc / et, dev_block, (int)ldb, 1.0, S + 2 * blk, hs); // q2 slot
    } else {
        motk::axpby2d(h->stream, ne, ne, sc, dev_block, (int)ldb, 1.0, S + blk, hs);         // qk slot
    }
    return MOT_OK;
}

int check_lag_args(mot_handle* h, int family, int lag, int medium, int op) {
    if (!h) return MOT_EINVAL;
    if (family < 0 || family > 2 || medium < 0 || medium > 1 || op < 0 || op > 1)
        return mot_fail(h, MOT_EINVAL, "bad family/medium/op");
    if (lag < 0 || lag > fam_limit(h, family))
        return mot_fail(h, MOT_EINVAL, "lag " + std::to_string(lag) + " outside the range of family " +
                                           std::to_string(family) + " (0.." + std::to_string(fam_limit(h, family)) + ")");
    if (h->lag_done[lag]) return mot_fail(h, MOT_ESTATE, "lag already folded");
    uint32_t bit = 1u << (4 * family + 2 * medium + op);
    if (h->got[lag] & bit) return mot_fail(h, MOT_ESTATE, "block uploaded twice");
    return MOT_OK;
}

int after_block(mot_handle* h, int family, int lag, int medium, int op) {
    h->got[lag] |= 1u << (4 * family + 2 * medium + op);
    if ((h->got[lag] & required_bits(h, lag)) == required_bits(h, lag)) return fold_lag(h, lag);
    return MOT_OK;
}

// ------------------------------------------------------------- profiling ---
constexpr int kEvCap = 2048;

int ev_flush(mot_handle* h, EvPool& p) {
    if (!p.used) return MOT_OK;
    HIPCHK(h, hipEventSynchronize(p.b[p.used - 1]));
    for (int i = 0; i < p.used; ++i) {
        float ms = 0;
        HIPCHK(h, hipEventElapsedTime(&ms, p.a[i], p.b[i]));
        p.ms += ms;
        p.n += 1;
    }
    p.used = 0;
    return MOT_OK;
}

int ev_begin(mot_handle* h, EvPool& p) {
    p.open = false;
    if (h->opt.profile <= 0) return MOT_OK;
    if (p.seen++ % h->opt.profile) return MOT_OK;      // sample every profile-th launch
    p.open = true;
    if (p.a.empty()) {
        p.a.resize(kEvCap);
        p.b.resize(kEvCap);
        for (int i = 0; i < kEvCap; ++i) {
            HIPCHK(h, hipEventCreate(&p.a[i]));
            HIPCHK(h, hipEventCreate(&p.b[i]));
        }
    }
    if (p.used == kEvCap) {
        int rc = ev_flush(h, p);
        if (rc) return rc;
    }
    HIPCHK(h, hipEventRecord(p.a[p.used], h->stream));
    return MOT_OK;
}

int ev_end(mot_handle* h, EvPool& p) {
    if (!p.open) return MOT_OK;
    p.open = false;
    HIPCHK(h, hipEventRecord(p.b[p.used], h->stream));
    p.used++;
    return MOT_OK;
}

void ev_destroy(EvPool& p) {
    for (auto e : p.a) (void)hipEventDestroy(e);
    for (auto e : p.b) (void)hipEventDestroy(e);
    p.a.clear(); p.b.clear();
}

// Wait until the device has published progress word 'want' (bounded: a
// failed kernel turns into MOT_EHIP instead of a hang).
int wait_flag(mot_handle* h, int want) {
    if (h->hflag->seq >= want) return MOT_OK;
    double t0 = now_ms(), tq = t0;
    unsigned spins = 0;
    while (h->hflag->seq < want) {
        if ((++spins & 1023u) == 0) {
            // several solves may wait at once from their own threads: give the
            // core away between bursts and ask the runtime only every 0.2 ms
            std::this_thread::yield();
            const double t = now_ms();
            if (t - tq < 0.2) continue;
            tq = t;
            hipError_t e = hipStreamQuery(h->stream);
            if (e != hipSuccess && e != hipErrorNotReady)
                return mot_fail(h, MOT_EHIP, std::string("stream error while waiting: ") + hipGetErrorString(e));
            if (e == hipSuccess && h->hflag->seq < want)
                return mot_fail(h, MOT_EHIP, "stream idle but GMRES progress word not written");
            if (now_ms() - t0 > 60000.0) return mot_fail(h, MOT_EHIP, "timeout waiting for GMRES progress");
        }
    }
    return MOT_OK;
}

// Right-preconditioned GMRES with single-workgroup orthogonalisation (the
// approximate inverse keeps the Krylov space at one or two vectors).  With the
// FP64 preconditioner the solve starts from x0 = 0, with the FP32 one from the
// extrapolation 2 w_{k-1} - w_{k-2}.  The finishing kernel (x += Z y, ring and
// history push) is queued right after the first Arnoldi step and acts only if
// that step met the tolerance.
int gmres_solve_pc(mot_handle* h) {
    using namespace motk_step;
    const int M = h->M;
    const int maxit = h->opt.gmres_maxit;
    h->hflag->seq = 0;
    int prc;
    const bool warm = h->M32 != nullptr;
    if (warm) {
        warm_start(h);
        if ((prc = ev_begin(h, h->ev_q0))) return prc;
        q0_matvec(h, h->x, nullptr, h->wA, 0, 0);
        if ((prc = ev_end(h, h->ev_q0))) return prc;
        gm_start1(h, h->y, h->wA, 1, 1, nullptr);
    }
    // cold start (FP64 approximate inverse): the first preconditioner launch
    // takes r = y, forms beta and opens the cycle itself
    int seq = 1, iters = 0;
    bool first_cycle = true;
    for (;;) {
        double* src = h->wA;
        double* dst = h->wB;
        int j = 0;
        bool done = false;
        for (; j < M && iters + j < maxit; ++j) {
            double* vj = h->V + (size_t)j * h->n2;
            double* zj = h->Z + (size_t)j * h->n2;
            const bool open = first_cycle && j == 0 && !warm;
            precond(h, open ? h->y : src, vj, zj, open);
            if ((prc = ev_begin(h, h->ev_q0))) return prc;
            q0_matvec(h, zj, nullptr, dst, 1, 0);
            if ((prc = ev_end(h, h->ev_q0))) return prc;
            gm_orth1(h, dst);
            if (j == 0 && first_cycle) gm_finish(h, h->Z, 0);
            std::swap(src, dst);
            if ((prc = wait_flag(h, seq + j + 1))) return prc;
            if (h->hflag->done) { done = true; ++j; break; }
        }
        iters += j;
        seq += j;
        bool conv = done && h->hflag->converged;
        if (!(done && j == 1 && first_cycle)) {
            // the speculative finisher did nothing: finish (or update for a restart) now
            gm_finish(h, h->Z, (!done && iters >= maxit) ? 1 : 0);
        }
        if (conv || iters >= maxit) {
            h->iters_total += iters;
            h->last_iters = iters;
            h->last_relres = h->hflag->relres;
            h->last_conv = conv;
            break;
        }
        // restart from the updated x
        first_cycle = false;
        if ((prc = ev_begin(h, h->ev_q0))) return prc;
        q0_matvec(h, h->x, nullptr, h->wA, 0, 0);
        if ((prc = ev_end(h, h->ev_q0))) return prc;
        gm_start1(h, h->y, h->wA, 1, 0, nullptr);
        seq += 1;
        if ((prc = wait_flag(h, seq))) return prc;
        if (h->hflag->done) {      // restart residual already below the tolerance
            gm_finish(h, h->Z, 1);
            h->iters_total += iters;
            h->last_iters = iters;
            h->last_relres = h->hflag->relres;
            h->last_conv = 1;
            break;
        }
    }
    return h->last_conv ? MOT_OK : MOT_ENOCONV;
}

// R > 1: one right-preconditioned GMRES per column, products shared as
// tall-skinny GEMMs; cold start; the finisher is queued after the first Arnoldi
// step and pushes w_k only once every column has converged.
int gmres_solve_mr(mot_handle* h) {
    namespace mm = motk_multi;
    const int M = h->M;
    const int maxit = h->opt.gmres_maxit;
    h->hflag->seq = 0;
    int prc;
    const size_t vs = (size_t)h->n2 * h->Rp;
    mm::start(h, h->y, h->wA, 0, 1, h->x);
    int seq = 1, iters = 0;
    bool first_cycle = true;
    for (;;) {
        double* src = h->wA;
        double* dst = h->wB;
        int j = 0;
        bool done = false;
        for (; j < M && iters + j < maxit; ++j) {
            double* vj = h->V + (size_t)j * vs;
            double* zj = h->Z + (size_t)j * vs;
            mm::precond(h, src, vj, zj);
            if ((prc = ev_begin(h, h->ev_q0))) return prc;
            mm::q0_gemm(h, zj);
            if ((prc = ev_end(h, h->ev_q0))) return prc;
            mm::q0_reduce(h, dst);
            mm::orth(h, dst);
            if (j == 0 && first_cycle) mm::finish(h, 0);
            std::swap(src, dst);
            if ((prc = wait_flag(h, seq + j + 1))) return prc;
            if (h->hflag->done) { done = true; ++j; break; }
        }
        iters += j;
        seq += j;
        bool conv = done && h->hflag->converged;
        if (!(done && j == 1 && first_cycle)) mm::finish(h, (!done && iters >= maxit) ? 1 : 0);
        if (conv || iters >= maxit) {
            h->iters_total += iters;
            h->last_iters = iters;
            h->last_relres = h->hflag->relres;
            h->last_conv = conv;
            break;
        }
        first_cycle = false;
        if ((prc = ev_begin(h, h->ev_q0))) return prc;
        mm::q0_gemm(h, h->x);
        if ((prc = ev_end(h, h->ev_q0))) return prc;
        mm::q0_reduce(h, h->wA);
        mm::start(h, h->y, h->wA, 1, 0, nullptr);
        seq += 1;
        if ((prc = wait_flag(h, seq))) return prc;
        if (h->hflag->done) {
            mm::finish(h, 1);
            h->iters_total += iters;
            h->last_iters = iters;
            h->last_relres = h->hflag->relres;
            h->last_conv = h->hflag->converged;
            break;
        }
    }
    return h->last_conv ? MOT_OK : MOT_ENOCONV;
}

// Single right-hand-side GMRES on Q0 x = y (x holds the warm start).
int gmres_solve(mot_handle* h) {
    using namespace motk_step;
    hipStream_t s = h->stream;
    const int M = h->M;
    int maxit = h->opt.gmres_maxit;
    h->hflag->seq = 0;
    HIPCHK(h, hipMemsetAsync(&h->gm->seq, 0, sizeof(int), h->stream));
    h->hflag->done = 0;
    int seq_target = 0;
    bool first = true;
    int iters = 0;
    for (;;) {
        // r = y - Q0 x
        int prc = ev_begin(h, h->ev_q0);
        if (prc) return prc;
        q0_matvec(h, h->x, nullptr, h->wA, 0, 0);
        if ((prc = ev_end(h, h->ev_q0))) return prc;
        gm_residual(h, h->y, h->wA, first ? 1 : 0);
        first = false;
        seq_target++;
        double* src = h->wA;
        double* dst = h->wB;
        bool cycle_done = false;
        int j = 0;
        for (; j < M && iters + j < maxit; ++j) {
            // V[j] = src * inv_h ; Z[j] = M V[j] (or V[j]) ; dst = Q0 Z[j]
            double* vj = h->V + (size_t)j * h->n2;
            if (h->M32 || h->M64) {
                double* zj = h->Z + (size_t)j * h->n2;
                precond(h, src, vj, zj);
                if ((prc = ev_begin(h, h->ev_q0))) return prc;
                q0_matvec(h, zj, nullptr, dst, 1, 0);
                if ((prc = ev_end(h, h->ev_q0))) return prc;
            } else {
                if ((prc = ev_begin(h, h->ev_q0))) return prc;
                q0_matvec(h, src, vj, dst, 1, 1);
                if ((prc = ev_end(h, h->ev_q0))) return prc;
            }
            gm_dots(h, dst);
            gm_orth(h, dst, 0);
            gm_orth(h, dst, 1);
            std::swap(src, dst);
            // wait for the previous step's flag (one step of look-ahead)
            int want = seq_target + j;   // flag of step j-1 (residual counts as one)
            int wrc = wait_flag(h, want);
            if (wrc) return wrc;
            if (h->hflag->done) { cycle_done = true; break; }
        }
        if (!cycle_done) {
            int wrc = wait_flag(h, seq_target + j);
            if (wrc) return wrc;
        }
        HIPCHK(h, hipGetLastError());
        // settle: read the state of the cycle
        int total = h->hflag->total;
        iters = total;
        seq_target = h->hflag->seq;
        gm_update_x(h, (h->M32 || h->M64) ? h->Z : h->V, h->x);
        int conv = h->hflag->converged;
        if (conv || iters >= maxit) {
            h->iters_total += iters;
            h->last_iters = iters;
            h->last_relres = h->hflag->relres;
            h->last_conv = conv;
            break;
        }
    }
    return h->last_conv ? MOT_OK : MOT_ENOCONV;
}

// PX = P^Sigma X for X [ne][nc]; S and Z ([nf][nc]) are scratch of the CG
// form and may be null with the dense one
static int sigma_project(mot_handle* h, int nc, const double* X, double* PX, double* S, double* Z) {
    if (h->opt.recovery == 1) {
        // P^Sigma X = Sigma (Sigma^T Sigma)^+ Sigma^T X: incidence products and
        // CG on the face graph Laplacian (Section IV-B)
        motk::inc_T(h->stream, h->gf, nc, X, nc, S);
        motk::col_center(h->stream, h->nf, nc, S);
        auto lap = [&](const double* Xi, double* Yo) { motk::spmm_lap(h->stream, h->gf, nc, Xi, Yo); };
        int rc = batched_cg(h, h->nf, nc, S, Z, lap, h->opt.cg_tol, h->opt.cg_maxit);
        if (rc && rc != MOT_ENOCONV) return rc;
        motk::inc_apply(h->stream, h->gf, nc, Z, PX, nc);
        return rc;
    }
    // the dense P^Sigma formed at setup by the same incidence products and CG
    motk::gemm(h->stream, h->ne, nc, h->ne, 1.0, h->PS, h->hs, X, nc, 0.0, PX, nc);
    return MOT_OK;
}

int recover(mot_handle* h, int s0, int ns, double* loop, double* star) {
    // columns per batch: 4 R per step
    const int per = 4 * h->R;
    const int maxcol = 8192;
    int bs = std::max(1, maxcol / per);
    double *X, *S = nullptr, *Z = nullptr, *PX;
    int rc;
    const bool cg = h->opt.recovery == 1;
    int ncmax = std::min(ns, bs) * per;
    if ((rc = dalloc(h, &X, (size_t)h->ne * ncmax, false)) || (rc = dalloc(h, &PX, (size_t)h->ne * ncmax, false)) ||
        (cg && ((rc = dalloc(h, &S, (size_t)h->nf * ncmax, false)) || (rc = dalloc(h, &Z, (size_t)h->nf * ncmax, false)))))
        return rc;
    int worst = MOT_OK;
    for (int b0 = 0; b0 < ns; b0 += bs) {
        int nb = std::min(bs, ns - b0);
        int nc = nb * per;
        motk_step::rec_gather(h, s0 + b0, nb, X);
        rc = sigma_project(h, nc, X, PX, S, Z);
        if (rc && rc != MOT_ENOCONV) return rc;
        if (rc) worst = rc;
        size_t off = (size_t)b0 * 2 * h->ne * h->R;
        motk_step::rec_scatter(h, nb, X, PX, loop ? loop + off : nullptr, star ? star + off : nullptr);
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    dfree(h, X); dfree(h, S); dfree(h, Z); dfree(h, PX);
    return worst;
}

// Every size-determining field of a handle, from the mesh, media, dt, nrhs and
// options alone (mot_create and mot_footprint share it).
void plan_dims(mot_handle* h, int nv, int nf, int ne, int nrhs, const double* V, double eps_r, double mu_r,
               double dt) {
    if (h->opt.gmres_restart < 2 || h->opt.gmres_restart > MOT_MAXM) h->opt.gmres_restart = 40;
    if (h->opt.precond < 0 || h->opt.precond > 2) h->opt.precond = 1;
    h->M = h->opt.gmres_restart;
    if (h->opt.gmres_maxit <= 0) h->opt.gmres_maxit = 400;
    if (h->opt.cg_maxit <= 0) h->opt.cg_maxit = 20000;
    if (!(h->opt.cg_tol > 0)) h->opt.cg_tol = 1e-13;
    if (!(h->opt.gmres_tol > 0)) h->opt.gmres_tol = 1e-13;
    h->nv = nv; h->nf = nf; h->ne = ne; h->R = nrhs;
    h->Rp = 1;
    if (nrhs > 1) { h->Rp = 4; while (h->Rp < nrhs) h->Rp *= 2; }
    h->B = std::max(8, std::min(128, 4096 / h->Rp));
    h->hs = (ne + 7) & ~7;
    h->n2 = 2 * h->hs;
    {
        // an explicit stream_split or history_order fixes that part of the
        // schedule; otherwise the autotuner picks it (or the defaults stay)
        const int sp = h->opt.stream_split;
        const bool sp_set = sp == 1 || sp == 2 || sp == 4 || sp == 11 || sp == 12 || sp == 14 || sp == 18 ||
                            sp == 32 || sp == 34;
        const bool ho_set = h->opt.history_order >= 1 && h->opt.history_order <= 3;
        h->sch_q0 = h->sch_pc = sp_set ? sp : 1;
        if (h->opt.history_order == 2) h->sch_hist = sp_set && sp <= 4 ? sp : 1;
        else if (h->opt.history_order == 3) h->sch_hist = sp == 12 || sp == 32 ? 32 : 34;
        else if (!sp_set || sp == 1) h->sch_hist = 11;
        else if (sp > 30) h->sch_hist = sp;
        else h->sch_hist = sp > 10 ? std::min(sp, 14) : 20 + sp;
        h->tune_hist = h->opt.autotune && !sp_set && !ho_set && h->opt.history_form != 1;
        h->tune_mv = h->opt.autotune && !sp_set;
    }
    h->eps_r = eps_r; h->mu_r = mu_r; h->dt = dt;
    h->c = 1.0; h->eta = 1.0;
    h->cp = 1.0 / std::sqrt(eps_r * mu_r);
    h->etap = std::sqrt(mu_r / eps_r);
    // D, T_max, k_max (eq. alpha; Section V-B)
    double D = h->opt.diameter;
    if (!(D > 0)) {
        D = 0;
        for (int a = 0; a < nv; ++a)
            for (int b = a + 1; b < nv; ++b) {
                double dx = V[3 * a] - V[3 * b], dy = V[3 * a + 1] - V[3 * b + 1], dz = V[3 * a + 2] - V[3 * b + 2];
                D = std::max(D, dx * dx + dy * dy + dz * dz);
            }
        D = std::sqrt(D);
    }
    h->D = D;
    h->Tmax = D / std::min(h->c, h->cp);
    h->kmax = (int)std::ceil(h->Tmax / dt - 1e-12);
    h->nlags = h->kmax + 2;
    h->nh = h->nlags - 1;
    h->hist_cap = h->opt.keep_history ? (h->opt.max_steps > 0 ? h->opt.max_steps : 20000) : 0;
    if (h->opt.precision != MOT_FP64) h->hilo = h->opt.hilo_lags < 0 ? 0 : std::min(h->opt.hilo_lags, h->nh);
    if (h->Rp > 1) motk_multi::plan_tiles(h);
}

// Device bytes of a planned handle: the allocations that live from create to
// destroy (resident), and resident plus the largest transient phase (peak):
// projector and Gram solves, the static products, one lag staged for its fold,
// the Newton-Schulz build, and recovery batches.  Mirrors mot_create, the
// fold, build_precond and recover.
void footprint(const mot_handle* h, int64_t gnnz, uint64_t* resident, uint64_t* peak) {
    const double ne = h->ne, nf = h->nf, nv = h->nv, hs = h->hs, R = h->R;
    const double blk = ne * hs;
    const double n2r = (double)h->n2 * h->Rp, NB = (double)h->B * h->Rp, M = h->M;
    double b = 0;
    for (double nn : {nf, nv}) b += 4.0 * (ne + ne + (nn + 1) + 2 * ne + (nn + 1) + 2 * ne) + 8.0 * 2 * ne;  // graphs
    b += 2 * (4.0 * (ne + 1) + 4.0 * gnnz + 8.0 * gnnz);                          // G, G^T (CSR)
    b += 8.0 * (2 * ne * 42 + 9 * R + R);                                         // RHS quadrature, waves
    b += 8.0 * 5 * blk;                                                           // PS, BL, G^-1, C1, C2
    if (h->opt.history_form == 1) {
        // Q_0, fold scratch, upload block; the kept families of lags >= 1; the
        // projected rings, sums and pointer table
        double fam = 0;
        for (int i = 1; i < h->nlags; ++i)
            for (int f = 0; f < 3; ++f) fam += i <= fam_limit(h, f);
        b += 8.0 * (7 + 3 * fam) * blk + 8.0 * (2.0 * h->nh * h->n2 + 2.0 * h->n2 + 3.0 * h->nlags);
    } else {
        b += 8.0 * ((double)h->nlags * 3 + 4) * blk;                              // Q, fold scratch, raw block
    }
    b += 8.0 + 8.0 * (h->nh * n2r + 4 * hs * NB + 4 * ne * NB + 4 * n2r + 2 * (M + 1) * n2r) + sizeof(GmState);
    if (h->Rp > 1) {
        const double t3 = 3.0 * motk_multi::tile_elems(h);
        if (h->opt.precision == MOT_FP64) b += 8.0 * h->nlags * t3;
        else b += 8.0 * t3 + 4.0 * h->nh * t3 + 4.0 * h->hilo * t3;
        b += (double)sizeof(GmState) * h->Rp + 8.0 * motk_multi::part_doubles(h) +
             8.0 * motk_multi::orth_part_doubles(h);
    }
    b += 8.0 * h->hist_cap * n2r;                                                 // kept history
    const double nn2 = (double)h->n2 * h->n2;
    if (h->opt.precond) b += (h->opt.precond == 2 ? 8.0 : 4.0) * nn2;            // approximate inverse
    const double chunk = std::min(ne, 4096.0);
    const double cgx = MOT_CG_CHUNKS + 8;                                         // per-column CG scalars
    double t = 0;
    t = std::max(t, 8.0 * ((2 * ne + 5 * std::max(nf, nv)) * chunk + cgx * chunk)); // projectors
    t = std::max(t, 8.0 * (6 * ne * chunk + cgx * chunk));                         // G^-1
    t = std::max(t, 8.0 * 3 * blk);                                                 // C1, C2
    t = std::max(t, 8.0 * 9 * blk);                                                 // one lag staged
    if (h->opt.precond) t = std::max(t, 8.0 * 4 * nn2 + 16.0 * h->n2);              // Newton-Schulz
    const double per = 4 * R, bs = std::max(1.0, std::floor(8192 / per)), nc = bs * per;
    if (h->opt.recovery == 1) t = std::max(t, 8.0 * ((2 * ne + 5 * nf) * nc + cgx * nc));  // recovery batch
    else t = std::max(t, 8.0 * 2 * ne * nc);
    *resident = (uint64_t)b;
    *peak = (uint64_t)(b + t);
}

}  // namespace

// ---- static scratch of the allocation-free calls ----
// One array per device, in the code object: each GPU the library runs on
// holds MOT_NOALLOC_DOUBLES doubles (1 MiB) from load until the process ends.
// Host code never uses the array's name as an address (on the host it names a
// stand-in): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in g_scratch_dev.
static __device__ __align__(256) double scratch[MOT_NOALLOC_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Address of this device's scratch array; dev must be the current device.
int scratch_address(mot_handle* h, int dev, double** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return mot_fail(h, MOT_EHIP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mot_fail(h, MOT_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return MOT_OK;
}
}  // namespace

// ======================================================================= ABI
extern "C" {

void mot_default_options(mot_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->precision = MOT_FP64;
    o->gmres_tol = 1e-13;
    o->gmres_restart = 40;
    o->gmres_maxit = 400;
    o->cg_tol = 1e-13;
    o->cg_maxit = 20000;
    o->diameter = 0.0;
    o->keep_history = 1;
    o->max_steps = 0;
    o->mem_cap_bytes = 0;
    o->profile = 0;
    o->precond = 1;
    o->hilo_lags = 2;
    o->mix_group = 4;
    o->autotune = 1;
}

int mot_footprint(const mot_mesh* mesh, double eps_r, double mu_r, double dt, int32_t nrhs, int64_t gram_nnz,
                  const mot_options* opt, uint64_t* resident_bytes, uint64_t* peak_bytes) {
    if (!mesh || !mesh->verts || !resident_bytes || !peak_bytes) return mot_fail(nullptr, MOT_EINVAL, "null argument");
    if (mesh->nv <= 0 || mesh->nf <= 0 || mesh->ne <= 0 || nrhs < 1 || nrhs > 64 || gram_nnz < 0)
        return mot_fail(nullptr, MOT_EINVAL, "bad sizes");
    if (!(dt > 0) || !(eps_r > 0) || !(mu_r > 0) || !std::isfinite(eps_r + mu_r + dt))
        return mot_fail(nullptr, MOT_EINVAL, "dt, eps_r and mu_r must be finite and > 0");
    mot_handle h;
    if (opt) h.opt = *opt; else mot_default_options(&h.opt);
    plan_dims(&h, mesh->nv, mesh->nf, mesh->ne, nrhs, mesh->verts, eps_r, mu_r, dt);
    footprint(&h, gram_nnz, resident_bytes, peak_bytes);
    return MOT_OK;
}

const char* mot_last_error(const mot_handle* h) { return h ? h->err.c_str() : g_create_err.c_str(); }

void mot_destroy(mot_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    ev_destroy(h->ev_hist);
    ev_destroy(h->ev_q0);
    for (auto& g : h->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    for (void* p : h->allocs) (void)hipFreeAsync(p, h->stream);
    (void)hipStreamSynchronize(h->stream);
    if (h->hflag) (void)hipHostFree(h->hflag);
    delete h;
}

int mot_create(const mot_mesh* mesh, double eps_r, double mu_r, double dt, const double* T0s,
               const double* T0h, const int32_t* g_rowptr, const int32_t* g_col, const double* g_val,
               int32_t nrhs, const mot_planewave* waves, const mot_options* opt, void* stream,
               mot_handle** out) {
    g_create_err.clear();
    if (!out) return mot_fail(nullptr, MOT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh || !mesh->verts || !mesh->tris || !mesh->edges || !T0s || !T0h || !g_rowptr || !g_col ||
        !g_val || !waves)
        return mot_fail(nullptr, MOT_EINVAL, "NULL argument");
    if (!(eps_r > 0) || !(mu_r > 0) || !(dt > 0) || !std::isfinite(eps_r + mu_r + dt))
        return mot_fail(nullptr, MOT_EINVAL, "eps_r, mu_r, dt must be positive");
    const int nv = mesh->nv, nf = mesh->nf, ne = mesh->ne;
    if (nv < 4 || nf < 4 || ne < 6 || 2 * ne != 3 * nf)
        return mot_fail(nullptr, MOT_EINVAL, "mesh sizes are not those of a closed triangulation");
    if (nrhs < 1 || nrhs > 64) return mot_fail(nullptr, MOT_EINVAL, "nrhs must be in 1..64");
    if (opt && (opt->history_form < 0 || opt->history_form > 1))
        return mot_fail(nullptr, MOT_EINVAL, "history_form must be 0 (folded lags) or 1 (raw families)");
    if (opt && opt->history_form == 1 && nrhs > 1)
        return mot_fail(nullptr, MOT_EINVAL, "history_form 1 takes one right-hand side");
    if (nrhs > 1 && opt && opt->precond == 0)
        return mot_fail(nullptr, MOT_EINVAL, "several right-hand sides need the Q_0 preconditioner (precond 1 or 2)");
    if (opt && opt->precision != MOT_FP64 && opt->precision != MOT_MIXED && opt->precision != MOT_MIXED32)
        return mot_fail(nullptr, MOT_EINVAL, "precision must be MOT_FP64, MOT_MIXED or MOT_MIXED32");
    if (opt && opt->precision != MOT_FP64 && nrhs < 2)
        return mot_fail(nullptr, MOT_EINVAL, "the mixed-precision history multiplies several right-hand sides (nrhs >= 2)");
    if (opt && opt->recovery != 0 && opt->recovery != 1)
        return mot_fail(nullptr, MOT_EINVAL, "recovery must be 0 (dense projector) or 1 (graph-Laplacian CG)");
    if (opt && opt->mix_group != 0 && opt->mix_group != 4 && opt->mix_group != 16 && opt->mix_group != 64)
        return mot_fail(nullptr, MOT_EINVAL, "mix_group must be 4, 16 or 64 (0: 4)");
    if (opt && opt->tile_wg != 0 && opt->tile_wg != 4 && opt->tile_wg != 8)
        return mot_fail(nullptr, MOT_EINVAL, "tile_wg must be 0 (tuned), 4 or 8");
    // ---- mesh validation (host, integers) ----
    const int32_t* E = mesh->edges;
    const int32_t* F = mesh->tris;
    for (int f = 0; f < 3 * nf; ++f)
        if (F[f] < 0 || F[f] >= nv) return mot_fail(nullptr, MOT_EINVAL, "triangle vertex out of range");
    std::vector<int> fdeg(nf, 0);
    for (int m = 0; m < ne; ++m) {
        int vm = E[4 * m], vp = E[4 * m + 1], cp = E[4 * m + 2], cm = E[4 * m + 3];
        if (vm < 0 || vm >= nv || vp < 0 || vp >= nv || vm == vp || cp < 0 || cp >= nf || cm < 0 || cm >= nf || cp == cm)
            return mot_fail(nullptr, MOT_EINVAL, "edge table entry out of range at edge " + std::to_string(m));
        fdeg[cp]++; fdeg[cm]++;
        // c_plus traverses v_minus -> v_plus counter-clockwise
        bool okp = false, okm = false;
        for (int k = 0; k < 3; ++k) {
            if (F[3 * cp + k] == vm && F[3 * cp + (k + 1) % 3] == vp) okp = true;
            if (F[3 * cm + k] == vp && F[3 * cm + (k + 1) % 3] == vm) okm = true;
        }
        if (!okp || !okm) return mot_fail(nullptr, MOT_EINVAL, "edge orientation inconsistent at edge " + std::to_string(m));
    }
    for (int f = 0; f < nf; ++f)
        if (fdeg[f] != 3) return mot_fail(nullptr, MOT_EINVAL, "triangle without three edges");
    // Sigma^T Lambda = 0: each face's signed edges cancel at every vertex
    {
        std::vector<std::map<int, int>> acc(nf);
        for (int m = 0; m < ne; ++m) {
            int vm = E[4 * m], vp = E[4 * m + 1], cp = E[4 * m + 2], cm = E[4 * m + 3];
            acc[cp][vp] += 1; acc[cp][vm] -= 1;
            acc[cm][vp] -= 1; acc[cm][vm] += 1;
        }
        for (int f = 0; f < nf; ++f)
            for (auto& kv : acc[f])
                if (kv.second != 0) return mot_fail(nullptr, MOT_EINVAL, "Sigma^T Lambda != 0");
    }
    int chi = nv - ne + nf;
    if (chi > 2 || chi % 2) return mot_fail(nullptr, MOT_EINVAL, "Euler characteristic of a closed orientable surface expected");
    for (size_t i = 0; i < (size_t)ne * ne; ++i)
        if (!std::isfinite(T0s[i]) || !std::isfinite(T0h[i])) return mot_fail(nullptr, MOT_EINVAL, "non-finite static block");
    for (int i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(mesh->verts[i])) return mot_fail(nullptr, MOT_EINVAL, "non-finite vertex coordinate");
    // Gram matrix CSR (host, before anything is allocated)
    if (g_rowptr[0] != 0 || g_rowptr[ne] <= 0) return mot_fail(nullptr, MOT_EINVAL, "bad Gram CSR row pointers");
    for (int r = 0; r < ne; ++r)
        if (g_rowptr[r + 1] < g_rowptr[r]) return mot_fail(nullptr, MOT_EINVAL, "Gram CSR row pointers decrease");
    for (int i = 0; i < g_rowptr[ne]; ++i)
        if (g_col[i] < 0 || g_col[i] >= ne || !std::isfinite(g_val[i]))
            return mot_fail(nullptr, MOT_EINVAL, "bad Gram CSR entry");
    // plane waves (eq. (hin)): unit direction and polarisation, orthogonal
    for (int r = 0; r < nrhs; ++r) {
        const mot_planewave& w = waves[r];
        double pp = 0, kk = 0, pk = 0;
        for (int d = 0; d < 3; ++d) { pp += w.pol[d] * w.pol[d]; kk += w.dir[d] * w.dir[d]; pk += w.pol[d] * w.dir[d]; }
        if (!(w.width > 0) || !std::isfinite(w.width + w.t0 + w.amp + pp + kk) || std::fabs(pp - 1) > 1e-6 ||
            std::fabs(kk - 1) > 1e-6 || std::fabs(pk) > 1e-6)
            return mot_fail(nullptr, MOT_EINVAL, "bad plane wave " + std::to_string(r) +
                                                 ": width > 0, unit pol and dir, pol . dir = 0 expected");
    }

    mot_handle* h = new mot_handle();
    if (opt) h->opt = *opt; else mot_default_options(&h->opt);
    plan_dims(h, nv, nf, ne, nrhs, mesh->verts, eps_r, mu_r, dt);
    h->stream = (hipStream_t)stream;
    h->genus = (2 - chi) / 2;
    h->hist_wg = h->q0_wg = h->opt.tile_wg == 8 ? 8 : 4;
    double t_start = now_ms();
    int rc = MOT_OK;
    auto bail = [&](int code) { g_create_err = h->err; mot_destroy(h); return code; };
    {
        hipError_t e = hipGetDevice(&h->device);
        if (e != hipSuccess) { mot_fail(h, MOT_EHIP, hipGetErrorString(e)); return bail(MOT_EHIP); }
        if ((rc = scratch_address(h, h->device, &h->scratch))) return bail(rc);
    }

    // ---- graphs ----
    {
        std::vector<int> fp(ne), fm(ne), vp(ne), vm(ne);
        for (int m = 0; m < ne; ++m) { fp[m] = E[4 * m + 2]; fm[m] = E[4 * m + 3]; vp[m] = E[4 * m + 1]; vm[m] = E[4 * m]; }
        if ((rc = make_graph(h, h->gf, nf, fp, fm))) return bail(rc);
        if ((rc = make_graph(h, h->gv, nv, vp, vm))) return bail(rc);
    }
    // ---- Gram matrix and its transpose (CSR) ----
    {
        int nnz = g_rowptr[ne];          // validated above
        std::vector<int> tp(ne + 1, 0), tc(nnz);
        std::vector<double> tv(nnz);
        for (int i = 0; i < nnz; ++i) tp[g_col[i] + 1]++;
        for (int i = 0; i < ne; ++i) tp[i + 1] += tp[i];
        std::vector<int> fill(tp.begin(), tp.end() - 1);
        for (int r = 0; r < ne; ++r)
            for (int k = g_rowptr[r]; k < g_rowptr[r + 1]; ++k) { int c = g_col[k]; tc[fill[c]] = r; tv[fill[c]] = g_val[k]; fill[c]++; }
        h->G.n = h->GT.n = ne; h->G.nnz = h->GT.nnz = nnz;
        if ((rc = upload(h, &h->G.ptr, g_rowptr, ne + 1)) || (rc = upload(h, &h->G.col, g_col, nnz)) ||
            (rc = upload(h, &h->G.val, g_val, nnz)) || (rc = upload(h, &h->GT.ptr, tp.data(), ne + 1)) ||
            (rc = upload(h, &h->GT.col, tc.data(), nnz)) || (rc = upload(h, &h->GT.val, tv.data(), nnz)))
            return bail(rc);
    }
    // ---- RHS quadrature geometry (7-point degree-5 rule per triangle) ----
    {
        const double s15 = std::sqrt(15.0), qa = (6 - s15) / 21, qb = (6 + s15) / 21;
        const double L[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3},
                                {1 - 2 * qa, qa, qa}, {qa, 1 - 2 * qa, qa}, {qa, qa, 1 - 2 * qa},
                                {1 - 2 * qb, qb, qb}, {qb, 1 - 2 * qb, qb}, {qb, qb, 1 - 2 * qb}};
        const double W[7] = {9.0 / 40, (155 - s15) / 1200, (155 - s15) / 1200, (155 - s15) / 1200,
                             (155 + s15) / 1200, (155 + s15) / 1200, (155 + s15) / 1200};
        std::vector<double> X((size_t)ne * 14 * 3), Fw((size_t)ne * 14 * 3);
        const double* V = mesh->verts;
        for (int m = 0; m < ne; ++m)
            for (int side = 0; side < 2; ++side) {
                int f = E[4 * m + 2 + side];
                int opp = -1;
                for (int k = 0; k < 3; ++k) { int v = F[3 * f + k]; if (v != E[4 * m] && v != E[4 * m + 1]) opp = v; }
                const double* a = V + 3 * F[3 * f];
                const double* b = V + 3 * F[3 * f + 1];
                const double* c = V + 3 * F[3 * f + 2];
                double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
                double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
                double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
                double sg = side == 0 ? 1.0 : -1.0;
                for (int q = 0; q < 7; ++q) {
                    size_t o = ((size_t)m * 14 + side * 7 + q) * 3;
                    for (int d = 0; d < 3; ++d) {
                        double x = L[q][0] * a[d] + L[q][1] * b[d] + L[q][2] * c[d];
                        X[o + d] = x;
                        Fw[o + d] = W[q] * area * sg * (x - V[3 * opp + d]) / (2 * area);
                    }
                }
            }
        if ((rc = upload(h, &h->rq_x, X.data(), X.size())) || (rc = upload(h, &h->rq_f, Fw.data(), Fw.size())))
            return bail(rc);
        std::vector<double> wv(9 * nrhs), tc(nrhs);
        for (int r = 0; r < nrhs; ++r) {
            const mot_planewave& w = waves[r];  // validated above
            wv[9 * r] = w.amp;
            for (int d = 0; d < 3; ++d) { wv[9 * r + 1 + d] = w.pol[d]; wv[9 * r + 4 + d] = w.dir[d]; }
            wv[9 * r + 7] = w.width;
            wv[9 * r + 8] = w.t0;
            // star RHS cut (Section V-C): after the pulse has left every vertex
            double kmaxx = -1e300;
            for (int v = 0; v < nv; ++v)
                kmaxx = std::max(kmaxx, w.dir[0] * V[3 * v] + w.dir[1] * V[3 * v + 1] + w.dir[2] * V[3 * v + 2]);
            tc[r] = w.t0 + (kmaxx + 1.6 * w.width) / h->c;
        }
        if ((rc = upload(h, &h->waves, wv.data(), wv.size())) || (rc = upload(h, &h->tcut, tc.data(), tc.size())))
            return bail(rc);
    }
    // ---- projectors, G^-1, C1, C2 (Section III, IV-B) ----
    const int hs = h->hs;
    const size_t blk = (size_t)ne * hs;
    if ((rc = dalloc(h, &h->PS, blk)) || (rc = dalloc(h, &h->BL, blk)) || (rc = dalloc(h, &h->Ginv, blk)) ||
        (rc = dalloc(h, &h->C1, blk)) || (rc = dalloc(h, &h->C2, blk)))
        return bail(rc);
    if ((rc = dense_projector(h, h->gf, h->PS))) return bail(rc);
    if ((rc = dense_projector(h, h->gv, h->BL))) return bail(rc);
    if ((rc = gram_inverse(h))) return bail(rc);
    {
        double *T0, *A, *Bm;
        if ((rc = dalloc(h, &T0, blk)) || (rc = dalloc(h, &A, blk)) || (rc = dalloc(h, &Bm, blk))) return bail(rc);
        hipStream_t s = h->stream;
        // T^{Sigma H} = (I - BL) T0s (I - BL) ; C1 = T^{Sigma H} G^-1
        HIPCHK(h, hipMemcpy2DAsync(T0, hs * sizeof(double), T0s, ne * sizeof(double), ne * sizeof(double), ne,
                                   hipMemcpyHostToDevice, s));
        motk::axpby2d(s, ne, ne, 1.0, T0, hs, 0.0, A, hs);
        motk::gemm(s, ne, ne, ne, -1.0, h->BL, hs, T0, hs, 1.0, A, hs);     // A = (I - BL) T0s
        motk::axpby2d(s, ne, ne, 1.0, A, hs, 0.0, Bm, hs);
        motk::gemm(s, ne, ne, ne, -1.0, A, hs, h->BL, hs, 1.0, Bm, hs);     // Bm = A (I - BL)
        motk::gemm(s, ne, ne, ne, 1.0, Bm, hs, h->Ginv, hs, 0.0, h->C1, hs);
        // T^Lambda = BL T0h BL ; C2 = T^Lambda G^-1 (I - PS)
        HIPCHK(h, hipMemcpy2DAsync(T0, hs * sizeof(double), T0h, ne * sizeof(double), ne * sizeof(double), ne,
                                   hipMemcpyHostToDevice, s));
        motk::gemm(s, ne, ne, ne, 1.0, h->BL, hs, T0, hs, 0.0, A, hs);
        motk::gemm(s, ne, ne, ne, 1.0, A, hs, h->BL, hs, 0.0, Bm, hs);
        motk::gemm(s, ne, ne, ne, 1.0, Bm, hs, h->Ginv, hs, 0.0, A, hs);    // A = T^Lambda G^-1
        motk::axpby2d(s, ne, ne, 1.0, A, hs, 0.0, h->C2, hs);
        motk::gemm(s, ne, ne, ne, -1.0, A, hs, h->PS, hs, 1.0, h->C2, hs);  // C2 = A (I - PS)
        HIPCHK(h, hipStreamSynchronize(s));
        dfree(h, T0); dfree(h, A); dfree(h, Bm);
    }
    // ---- lag storage and march state ----
    h->stage.assign((size_t)h->nlags * 3, nullptr);
    h->got.assign(h->nlags, 0);
    h->lag_done.assign(h->nlags, 0);
    const bool rawh = h->opt.history_form == 1;
    if ((rc = dalloc(h, &h->Q, (size_t)(rawh ? 1 : h->nlags) * 3 * blk)) || (rc = dalloc(h, &h->tmp, 3 * blk, false)) ||
        (rc = dalloc(h, &h->raw, blk)))
        return bail(rc);
    if (rawh) {
        h->rawZ.assign((size_t)h->nlags * 3, nullptr);
        if ((rc = dalloc(h, &h->rawZtab, (size_t)h->nlags * 3)) ||
            (rc = dalloc(h, &h->rawL, (size_t)h->nh * h->n2)) || (rc = dalloc(h, &h->rawS, (size_t)h->nh * h->n2)) ||
            (rc = dalloc(h, &h->ry1, h->n2)) || (rc = dalloc(h, &h->ry2, h->n2)))
            return bail(rc);
    }
    // every march vector holds all Rp columns: [n2][Rp]
    const size_t n2 = (size_t)h->n2 * h->Rp;
    const size_t NB = (size_t)h->B * h->Rp;
    if ((rc = dalloc(h, &h->d_k, 2)) || (rc = dalloc(h, &h->ring, (size_t)h->nh * n2)) ||
        (rc = dalloc(h, &h->ebar, (size_t)2 * h->hs * NB)) || (rc = dalloc(h, &h->Ebar, (size_t)2 * h->hs * NB)) ||
        (rc = dalloc(h, &h->rb, (size_t)4 * h->ne * NB)) || (rc = dalloc(h, &h->y, n2)) ||
        (rc = dalloc(h, &h->x, n2)) || (rc = dalloc(h, &h->V, (size_t)(h->M + 1) * n2)) || (rc = dalloc(h, &h->Z, (size_t)(h->M + 1) * n2)) ||
        (rc = dalloc(h, &h->wA, n2)) || (rc = dalloc(h, &h->wB, n2)) || (rc = dalloc(h, &h->gm, 1)))
        return bail(rc);
    if (h->Rp > 1) {
        // tile-major copies of the lags for the multi-RHS products
        const size_t tsz3 = 3 * motk_multi::tile_elems(h);
        if (h->opt.precision == MOT_FP64) {
            if ((rc = dalloc(h, &h->Qt, (size_t)h->nlags * tsz3))) return bail(rc);
        } else {
            if ((rc = dalloc(h, &h->Qt, tsz3)) || (rc = dalloc(h, &h->QtF, (size_t)h->nh * tsz3)) ||
                (h->hilo && (rc = dalloc(h, &h->QtL, (size_t)h->hilo * tsz3))))
                return bail(rc);
        }
    }
    if (h->Rp > 1 && ((rc = dalloc(h, &h->gms, h->Rp)) || (rc = dalloc(h, &h->mr_part, motk_multi::part_doubles(h))) ||
                      (rc = dalloc(h, &h->orth_part, motk_multi::orth_part_doubles(h)))))
        return bail(rc);
    if (h->hist_cap && (rc = dalloc(h, &h->hist, (size_t)h->hist_cap * n2))) return bail(rc);
    if (hipHostMalloc((void**)&h->hflag, sizeof(GmFlag), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        h->err = "hipHostMalloc failed";
        return bail(MOT_EHIP);
    }
    std::memset((void*)h->hflag, 0, sizeof(GmFlag));
    if (hipHostGetDevicePointer((void**)&h->dflag, h->hflag, 0) != hipSuccess) {
        h->err = "hipHostGetDevicePointer failed";
        return bail(MOT_EHIP);
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) { h->err = "stream sync failed"; return bail(MOT_EHIP); }
    h->setup_ms = now_ms() - t_start;
    *out = h;
    return MOT_OK;
}

int mot_set_lag(mot_handle* h, int32_t family, int32_t lag, int32_t medium, int32_t op, const double* block) {
    int rc = check_lag_args(h, family, lag, medium, op);
    if (rc) return rc;
    if (!block) return mot_fail(h, MOT_EINVAL, "NULL block");
    const int ne = h->ne, hs = h->hs;
    for (size_t i = 0, nn = (size_t)ne * ne; i < nn; ++i)
        if (!std::isfinite(block[i])) return mot_fail(h, MOT_EINVAL, "non-finite entry in a lag block");
    HIPCHK(h, hipMemcpy2DAsync(h->raw, hs * sizeof(double), block, ne * sizeof(double), ne * sizeof(double), ne,
                               hipMemcpyHostToDevice, h->stream));
    if ((rc = stage_add(h, family, lag, medium, op, h->raw, hs))) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return after_block(h, family, lag, medium, op);
}

int mot_set_lag_device(mot_handle* h, int32_t family, int32_t lag, int32_t medium, int32_t op,
                       const double* dblock, int64_t ld) {
    int rc = check_lag_args(h, family, lag, medium, op);
    if (rc) return rc;
    if (!dblock) return mot_fail(h, MOT_EINVAL, "NULL block");
    const int ne = h->ne;
    if (ld < ne || ld > INT32_MAX) return mot_fail(h, MOT_EINVAL, "leading dimension below ne or too large");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dblock) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return mot_fail(h, MOT_EINVAL, "block is not device memory");
    }
    int* cnt;
    if ((rc = dalloc(h, &cnt, 1))) return rc;
    int bad = motk::count_nonfinite(h->stream, ne, ne, dblock, ld, cnt);
    dfree(h, cnt);
    if (bad < 0) return mot_fail(h, MOT_EHIP, "non-finite check failed");
    if (bad > 0) return mot_fail(h, MOT_EINVAL, "non-finite entry in a lag block");
    if ((rc = stage_add(h, family, lag, medium, op, dblock, ld))) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return after_block(h, family, lag, medium, op);
}

int mot_set_lag_csr(mot_handle* h, int32_t family, int32_t lag, int32_t medium, int32_t op,
                    const int64_t* rowptr, const int32_t* col, const double* val) {
    int rc = check_lag_args(h, family, lag, medium, op);
    if (rc) return rc;
    if (!rowptr || !col || !val) return mot_fail(h, MOT_EINVAL, "NULL CSR array");
    const int ne = h->ne, hs = h->hs;
    int64_t nnz = rowptr[ne];
    if (rowptr[0] != 0 || nnz < 0) return mot_fail(h, MOT_EINVAL, "bad CSR row pointers");
    for (int r = 0; r < ne; ++r)
        if (rowptr[r + 1] < rowptr[r]) return mot_fail(h, MOT_EINVAL, "CSR row pointers decrease");
    for (int64_t i = 0; i < nnz; ++i)
        if (col[i] < 0 || col[i] >= ne || !std::isfinite(val[i])) return mot_fail(h, MOT_EINVAL, "bad CSR entry");
    motk::fill2d(h->stream, ne, hs, 0.0, h->raw, hs);
    if (nnz > 0) {
        int64_t* dptr = nullptr; int* dcol = nullptr; double* dval = nullptr;
        if (!(rc = upload(h, &dptr, rowptr, ne + 1)) && !(rc = upload(h, &dcol, col, nnz)) &&
            !(rc = upload(h, &dval, val, nnz))) {
            motk::scatter_csr_add(h->stream, ne, dptr, dcol, dval, 1.0, h->raw, hs);
            if (hipStreamSynchronize(h->stream) != hipSuccess) rc = mot_fail(h, MOT_EHIP, "CSR scatter failed");
        }
        if (dptr) dfree(h, dptr);
        if (dcol) dfree(h, dcol);
        if (dval) dfree(h, dval);
        if (rc) return rc;
    }
    if ((rc = stage_add(h, family, lag, medium, op, h->raw, hs))) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return after_block(h, family, lag, medium, op);
}

int mot_reset(mot_handle* h) {
    if (!h) return MOT_EINVAL;
    h->k = 0;
    h->hist_first = 0;
    h->iters_total = 0;
    h->spec_iters = 1;               // as a new handle: the same Arnoldi counts, the same bits
    h->cancel.store(0);
    (void)ev_flush(h, h->ev_hist);
    (void)ev_flush(h, h->ev_q0);
    h->ev_hist.ms = h->ev_q0.ms = 0;
    h->ev_hist.n = h->ev_q0.n = 0;
    HIPCHK(h, hipMemsetAsync(h->d_k, 0, sizeof(int), h->stream));
    HIPCHK(h, hipMemsetAsync(h->ring, 0, (size_t)h->nh * h->n2 * h->Rp * sizeof(double), h->stream));
    motk_step::clear_halt(h);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MOT_OK;
}

int mot_step(mot_handle* h, mot_step_info* info) {
    if (!h) return MOT_EINVAL;
    if (!all_folded(h)) return mot_fail(h, MOT_ESTATE, "lag matrices missing: upload every block first");
    using namespace motk_step;
    inc_step(h);
    h->k += 1;
    if ((h->k - 1) % h->B == 0) rhs_batch(h, h->k, h->rb);
    if (h->Rp > 1 && (!h->gms || !h->mr_part)) return mot_fail(h, MOT_ESTATE, "multi-RHS buffers missing");
    // the events bracket the streaming kernel alone (the multi-RHS partial
    // reduction follows it)
    int prc = ev_begin(h, h->ev_hist);
    if (prc) return prc;
    if (h->Rp > 1) motk_multi::history_gemm(h);
    else if (h->opt.history_form == 1) raw_history(h);
    else history(h);
    if ((prc = ev_end(h, h->ev_hist))) return prc;
    if (h->Rp > 1) motk_multi::history_reduce(h);
    int rc;
    if (h->Rp > 1) {
        if (!h->gms || !h->mr_part) return mot_fail(h, MOT_ESTATE, "multi-RHS buffers missing");
        rc = gmres_solve_mr(h);
        if (rc && rc != MOT_ENOCONV) return rc;
    } else if ((h->M32 || h->M64) && h->n2 <= 32768) {
        rc = gmres_solve_pc(h);           // pushes w_k itself
        if (rc && rc != MOT_ENOCONV) return rc;
    } else {
        warm_start(h);
        rc = gmres_solve(h);
        if (rc && rc != MOT_ENOCONV) return rc;
        push(h);
    }
    HIPCHK(h, hipGetLastError());
    if (info) {
        info->step = h->k;
        info->gmres_iters = h->last_iters;
        info->gmres_relres = h->last_relres;
        info->converged = h->last_conv;
    }
    if (rc) mot_fail(h, rc, "GMRES did not reach the tolerance at step " + std::to_string(h->k));
    return rc;
}

// Speculative stepping (one RHS, preconditioned GMRES): steps are queued back
// to back with no host wait.  Each runs a fixed number of Arnoldi steps (one
// with the FP64 approximate inverse) and a finisher that pushes w_k only if the
// solve converged; otherwise it raises the halt word, which turns every later
// queued step kernel into a no-op.  The host reads the halt word once per
// window (at most one RHS batch long, so a batch computed ahead for a later
// window never overwrites the one a halted step needs) and finishes a halted
// step with the host-driven solve, then queues again from the next step.
struct SpecWord { int halt, halt_k, iters_all; double relres; };

static bool spec_ok(const mot_handle* h) {
    if (h->opt.spec_window < 0 || !(h->M32 || h->M64) || h->opt.history_form == 1) return false;
    return h->Rp > 1 ? (h->gms && h->mr_part) : h->n2 <= 32768;
}

// first: the window's first step advances the device step counter; later
// steps find it set by the previous step's finisher.
// goff >= 0: the launches are being captured into a graph as step goff of a
// window; the step index then comes from the device (the window's first step
// in d_k[1]), so one graph serves every window of its batch parity.
static int queue_spec_step(mot_handle* h, bool first, int goff = -1) {
    using namespace motk_step;
    namespace mm = motk_multi;
    if (first) inc_step(h);
    h->k += 1;
    const int kq = goff >= 0 ? -(goff + 1) : h->k;
    if ((h->k - 1) % h->B == 0) rhs_batch(h, h->k, h->rb, goff >= 0 ? h->d_k + 1 : nullptr);
    int prc;
    if ((prc = ev_begin(h, h->ev_hist))) return prc;
    if (h->Rp > 1) mm::history_gemm(h); else history(h);
    if ((prc = ev_end(h, h->ev_hist))) return prc;
    if (h->Rp > 1) {
        // R waves: one cold-started GMRES per column, products shared
        const size_t vs = (size_t)h->n2 * h->Rp;
        mm::history_reduce(h);
        mm::start(h, h->y, h->wA, 0, 1, h->x, 0);
        double* src = h->wA;
        double* dst = h->wB;
        for (int j = 0; j < h->spec_iters; ++j) {
            mm::precond(h, src, h->V + (size_t)j * vs, h->Z + (size_t)j * vs);
            if ((prc = ev_begin(h, h->ev_q0))) return prc;
            mm::q0_gemm(h, h->Z + (size_t)j * vs);
            if ((prc = ev_end(h, h->ev_q0))) return prc;
            mm::q0_reduce(h, dst);
            mm::orth(h, dst, 0);
            std::swap(src, dst);
        }
        mm::finish(h, 0, 1, kq);
        return MOT_OK;
    }
    if (h->M32) {
        warm_start(h);
        if ((prc = ev_begin(h, h->ev_q0))) return prc;
        q0_matvec(h, h->x, nullptr, h->wA, 0, 0);
        if ((prc = ev_end(h, h->ev_q0))) return prc;
        gm_start1(h, h->y, h->wA, 1, 1, nullptr, 0);
    }
    // cold start: the first preconditioner launch opens the cycle from r = y
    double* src = h->wA;
    double* dst = h->wB;
    for (int j = 0; j < h->spec_iters; ++j) {
        const bool open = j == 0 && !h->M32;
        precond(h, open ? h->y : src, h->V + (size_t)j * h->n2, h->Z + (size_t)j * h->n2, open);
        if ((prc = ev_begin(h, h->ev_q0))) return prc;
        q0_matvec(h, h->Z + (size_t)j * h->n2, nullptr, dst, 1, 0);
        if ((prc = ev_end(h, h->ev_q0))) return prc;
        // the last queued Arnoldi step also runs the speculative finisher
        gm_orth1(h, dst, 0, j + 1 == h->spec_iters ? kq : 0);
        std::swap(src, dst);
    }
    return MOT_OK;
}

// Capture the B queued steps of a window whose batch has parity `parity` into
// a graph (replayed with d_k[1] = the window's first step).  A capture that
// the runtime refuses switches the handle to stream launches for good.
static int capture_window(mot_handle* h, int parity) {
    hipGraphExec_t& ex = h->gexec[parity];
    if (ex) {
        (void)hipGraphExecDestroy(ex);
        ex = nullptr;
    }
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        h->graph_off = 1;
        return MOT_OK;
    }
    const int k_save = h->k;
    h->k = parity * h->B;                 // host bookkeeping only: selects the RHS half
    int rc = MOT_OK;
    for (int i = 0; i < h->B && rc == MOT_OK; ++i) rc = queue_spec_step(h, false, i);
    h->k = k_save;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc == MOT_OK && e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (rc) return rc;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ex = nullptr;
        h->graph_off = 1;
        return MOT_OK;
    }
    h->g_iters[parity] = h->spec_iters;
    return MOT_OK;
}

// one full, batch-aligned window from the captured graph of its parity
static int launch_window(mot_handle* h, bool ahead, bool* launched) {
    *launched = false;
    const int par = (h->k / h->B) & 1;
    if (!h->gexec[par] || h->g_iters[par] != h->spec_iters) {
        int rc = capture_window(h, par);
        if (rc) return rc;
        if (h->graph_off) return MOT_OK;
    }
    if (!ahead) motk_step::inc_step(h);                     // d_k[0] = first step
    motk_step::set_base(h, h->k + 1);
    HIPCHK(h, hipGraphLaunch(h->gexec[par], h->stream));
    h->k += h->B;
    h->graph_windows += 1;
    *launched = true;
    return MOT_OK;
}

static int read_spec(mot_handle* h, SpecWord* w) {
    HIPCHK(h, hipMemcpyAsync(w, &h->gm->halt, 3 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&w->relres, &h->gm->relres, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MOT_OK;
}

// One handle's speculative march, as a state machine: queue() puts one window
// of steps on the handle's stream without waiting; settle() waits for it,
// accounts for it and finishes a halted step on the host.  run_spec drives one
// handle; mot_run_batch interleaves several, so their windows overlap on the
// device.
struct SpecRun {
    mot_handle* h = nullptr;
    int nsteps = 0, done = 0;
    int win = 1;
    bool graphs = false;
    // the device step counter runs one ahead of h->k after a window in which
    // every step pushed (the last finisher set it); a halted window leaves it
    // at the halted step, which is then h->k
    bool ahead = false;
    SpecWord w0{};
    int k0 = 0, nw = 0;       // the window in flight
    int worst = MOT_OK;
};

static int spec_begin(SpecRun& r, mot_handle* h, int nsteps) {
    r.h = h;
    r.nsteps = nsteps;
    r.win = std::max(1, std::min(h->opt.spec_window > 0 ? h->opt.spec_window : h->B, h->B));
    // graphs replay whole RHS batches: windows then end on batch boundaries
    // (the legacy default stream cannot be captured)
    r.graphs = h->opt.graph && !h->opt.profile && r.win == h->B && h->stream != nullptr;
    return read_spec(h, &r.w0);
}

static int spec_queue(SpecRun& r) {
    mot_handle* h = r.h;
    int nw = std::min(r.win, r.nsteps - r.done);
    r.k0 = h->k;
    if (r.graphs && r.k0 % h->B) nw = std::min(nw, h->B - r.k0 % h->B);
    r.nw = nw;
    int rc;
    bool launched = false;
    if (r.graphs && !h->graph_off && nw == h->B && (rc = launch_window(h, r.ahead, &launched))) return rc;
    if (!launched)
        for (int i = 0; i < nw; ++i)
            if ((rc = queue_spec_step(h, i == 0 && !r.ahead))) return rc;
    r.ahead = true;
    HIPCHK(h, hipGetLastError());
    return MOT_OK;
}

static int spec_settle(SpecRun& r) {
    mot_handle* h = r.h;
    SpecWord w{};
    int rc;
    if ((rc = read_spec(h, &w))) return rc;
    h->iters_total += w.iters_all - r.w0.iters_all;
    r.w0 = w;
    if (!w.halt) {
        r.done += r.nw;
        h->last_iters = h->spec_iters;
        h->last_relres = w.relres;
        h->last_conv = 1;
        return MOT_OK;
    }
    // steps k0+1 .. halt_k-1 are complete; halt_k has its history in y
    if (w.halt_k <= r.k0 || w.halt_k > h->k) return mot_fail(h, MOT_EHIP, "speculative halt word out of range");
    h->k = w.halt_k;
    r.ahead = false;
    motk_step::clear_halt(h);
    int src = h->Rp > 1 ? gmres_solve_mr(h) : gmres_solve_pc(h);
    if (src && src != MOT_ENOCONV) return src;
    if (src) r.worst = src;
    if ((rc = read_spec(h, &r.w0))) return rc;
    // a step that needed more Arnoldi steps raises the count the later queued
    // steps take; one that did not converge at all tells nothing about them
    if (h->last_conv) h->spec_iters = std::min(h->M, std::max(h->spec_iters, h->last_iters));
    r.done += w.halt_k - r.k0;
    return MOT_OK;
}

static void spec_end(SpecRun& r) {
    if (r.ahead) motk_step::set_step(r.h, r.h->k);   // as the step-by-step march leaves it
}

// after an error: no halt word left raised, the counter at the host's step
static void spec_abort(mot_handle* h) {
    motk_step::clear_halt(h);
    motk_step::set_step(h, h->k);
    (void)hipStreamSynchronize(h->stream);
}

// a pending mot_cancel, consumed by the run it stops
static bool take_cancel(mot_handle* h) { return h->cancel.exchange(0) != 0; }

static int run_spec_windows(mot_handle* h, int nsteps, int* worst) {
    SpecRun r;
    int rc = spec_begin(r, h, nsteps);
    bool cancelled = false;
    while (!rc && r.done < nsteps) {
        if (take_cancel(h)) { cancelled = true; break; }
        rc = spec_queue(r);
        if (!rc) rc = spec_settle(r);
    }
    if (rc) return rc;
    spec_end(r);
    if (r.worst) *worst = r.worst;
    if (cancelled) *worst = MOT_ECANCEL;
    return MOT_OK;
}

// an error return never leaves the halt word raised behind it
static int run_spec(mot_handle* h, int nsteps, int* worst) {
    int rc = run_spec_windows(h, nsteps, worst);
    if (rc) spec_abort(h);
    return rc;
}

static int emit_steps(mot_handle* h, int s0, int nsteps, double* w_out, double* loop_out, double* star_out,
                      int32_t out_on_device, int worst);

int mot_run(mot_handle* h, int32_t nsteps, double* w_out, double* loop_out, double* star_out,
            int32_t out_on_device, mot_step_info* last) {
    if (!h) return MOT_EINVAL;
    if (nsteps < 0) return mot_fail(h, MOT_EINVAL, "nsteps < 0");
    if ((w_out || loop_out || star_out) && (!h->hist || (int64_t)h->k + nsteps > h->hist_cap))
        return mot_fail(h, MOT_EINVAL, "outputs need keep_history and max_steps >= steps taken");
    if ((loop_out || star_out) && h->k > 0 && h->k - 1 < h->hist_first)
        return mot_fail(h, MOT_EINVAL, "the star part needs the previous step, which the restored checkpoint did not hold");
    int s0 = h->k;
    int worst = MOT_OK;
    mot_step_info inf{};
    if (nsteps > 0 && spec_ok(h)) {
        if (!all_folded(h)) return mot_fail(h, MOT_ESTATE, "lag matrices missing: upload every block first");
        int rc = run_spec(h, nsteps, &worst);
        if (rc) return rc;
        inf.step = h->k;
        inf.gmres_iters = h->last_iters;
        inf.gmres_relres = h->last_relres;
        inf.converged = h->last_conv;
    } else {
        for (int i = 0; i < nsteps; ++i) {
            if (take_cancel(h)) { worst = MOT_ECANCEL; break; }
            int rc = mot_step(h, &inf);
            if (rc && rc != MOT_ENOCONV) return rc;
            if (rc) worst = rc;
        }
    }
    if (last) *last = inf;
    const int done = h->k - s0;          // all nsteps unless cancelled
    if (!(w_out || loop_out || star_out) || done == 0) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return worst;
    }
    return emit_steps(h, s0, done, w_out, loop_out, star_out, out_on_device, worst);
}

// outputs of the kept steps s0 .. s0+nsteps-1: the unknowns as computed and
// the current recovery of eq. (dis_jm)
static int emit_steps(mot_handle* h, int s0, int nsteps, double* w_out, double* loop_out, double* star_out,
                      int32_t out_on_device, int worst) {
    const size_t per = (size_t)2 * h->ne * h->R;
    const size_t tot = per * nsteps;
    double *dw = nullptr, *dl = nullptr, *ds = nullptr;
    int rc;
    if (w_out) {
        if (out_on_device) dw = w_out; else if ((rc = dalloc(h, &dw, tot, false))) return rc;
        motk_step::pack(h, nsteps, h->hist + (size_t)s0 * h->n2 * h->Rp, dw);
    }
    if (loop_out) { if (out_on_device) dl = loop_out; else if ((rc = dalloc(h, &dl, tot, false))) return rc; }
    if (star_out) { if (out_on_device) ds = star_out; else if ((rc = dalloc(h, &ds, tot, false))) return rc; }
    if (loop_out || star_out) {
        double tr = now_ms();
        rc = recover(h, s0, nsteps, dl, ds);
        h->recover_ms = now_ms() - tr;
        if (rc && rc != MOT_ENOCONV) return rc;
        if (rc) worst = rc;
    }
    if (!out_on_device) {
        if (w_out) { HIPCHK(h, hipMemcpyAsync(w_out, dw, tot * sizeof(double), hipMemcpyDeviceToHost, h->stream)); }
        if (loop_out) { HIPCHK(h, hipMemcpyAsync(loop_out, dl, tot * sizeof(double), hipMemcpyDeviceToHost, h->stream)); }
        if (star_out) { HIPCHK(h, hipMemcpyAsync(star_out, ds, tot * sizeof(double), hipMemcpyDeviceToHost, h->stream)); }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (!out_on_device) { dfree(h, dw); dfree(h, dl); dfree(h, ds); }
    return worst;
}

int mot_get_steps(mot_handle* h, int32_t first, int32_t count, double* w_out, double* loop_out,
                  double* star_out, int32_t out_on_device) {
    if (!h) return MOT_EINVAL;
    const int64_t end = (int64_t)first + count;
    if (first < 0 || count < 0 || end > h->k)
        return mot_fail(h, MOT_EINVAL, "steps out of range: only steps already taken can be read");
    if (!h->hist || end > h->hist_cap) return mot_fail(h, MOT_EINVAL, "steps not kept: needs keep_history");
    if (count > 0 && first < h->hist_first)
        return mot_fail(h, MOT_EINVAL, "steps before the restored checkpoint's kept history are not held");
    if (count == 0 || !(w_out || loop_out || star_out)) return MOT_OK;
    return emit_steps(h, first, count, w_out, loop_out, star_out, out_on_device, MOT_OK);
}

int mot_step_norms(mot_handle* h, int32_t first, int32_t count, double* norms) {
    if (!h) return MOT_EINVAL;
    const int64_t end = (int64_t)first + count;
    if (first < 0 || count < 0 || end > h->k || (!norms && count > 0))
        return mot_fail(h, MOT_EINVAL, "steps out of range or no output array");
    if (!h->hist || end > h->hist_cap) return mot_fail(h, MOT_EINVAL, "steps not kept: needs keep_history");
    if (count > 0 && first < h->hist_first)
        return mot_fail(h, MOT_EINVAL, "steps before the restored checkpoint's kept history are not held");
    if (count == 0) return MOT_OK;
    double* d = nullptr;
    int rc;
    if ((rc = dalloc(h, &d, (size_t)count * h->R, false))) return rc;
    motk_ff::step_norms(h, first, count, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(norms, d, sizeof(double) * count * h->R, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dfree(h, d);
    if (e != hipSuccess) return mot_fail(h, MOT_EHIP, hipGetErrorString(e));
    return MOT_OK;
}

// Same results as mot_step_norms (same kernel, same order of sums), staged in
// the device's static scratch array instead of a buffer allocated per call.
int mot_step_norms_noalloc(mot_handle* h, int32_t first, int32_t count, double* norms) {
    if (!h) return MOT_EINVAL;
    if ((int64_t)count * h->R > MOT_NOALLOC_DOUBLES)
        return mot_fail(h, MOT_EINVAL, "count * nrhs = " + std::to_string((int64_t)count * h->R) +
                                           " exceeds the static scratch of " + std::to_string(MOT_NOALLOC_DOUBLES) +
                                           " values: split the range");
    const int64_t end = (int64_t)first + count;
    if (first < 0 || count < 0 || end > h->k || (!norms && count > 0))
        return mot_fail(h, MOT_EINVAL, "steps out of range or no output array");
    if (!h->hist || end > h->hist_cap) return mot_fail(h, MOT_EINVAL, "steps not kept: needs keep_history");
    if (count > 0 && first < h->hist_first)
        return mot_fail(h, MOT_EINVAL, "steps before the restored checkpoint's kept history are not held");
    if (count == 0) return MOT_OK;
    if (!h->scratch) return mot_fail(h, MOT_ESTATE, "no scratch address for this handle's device");
    // every value of scratch[0 .. count*R) is written by the kernel: nothing to clear
    motk_ff::step_norms(h, first, count, h->scratch);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(norms, h->scratch, sizeof(double) * count * h->R, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return mot_fail(h, MOT_EHIP, hipGetErrorString(e));
    return MOT_OK;
}

int mot_far_field(mot_handle* h, int32_t first, int32_t count, double freq, int32_t ndir, const double* dirs,
                  double* field_out, double* spec_out) {
    if (!h) return MOT_EINVAL;
    const int64_t end = (int64_t)first + count;
    if (first < 0 || count < 1 || end > h->k)
        return mot_fail(h, MOT_EINVAL, "steps out of range: only steps already taken can be transformed");
    if (!h->hist || end > h->hist_cap) return mot_fail(h, MOT_EINVAL, "steps not kept: needs keep_history");
    if (first < h->hist_first)
        return mot_fail(h, MOT_EINVAL, "steps before the restored checkpoint's kept history are not held");
    if (!(freq >= 0) || !std::isfinite(freq)) return mot_fail(h, MOT_EINVAL, "frequency must be finite and >= 0");
    if (ndir < 0 || (ndir > 0 && (!dirs || !field_out)) || ndir > 65535)
        return mot_fail(h, MOT_EINVAL, "bad direction count or missing direction/field arrays");
    for (int a = 0; a < ndir; ++a) {
        const double* d = dirs + 3 * a;
        const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(std::fabs(nn - 1.0) <= 1e-9)) return mot_fail(h, MOT_EINVAL, "directions must be unit vectors");
    }
    const int ne = h->ne, R = h->R, nc = 8 * R;
    const double omega = 2 * M_PI * freq;               // c = 1 outside
    int chunk = 0;
    const int nchunk = motk_ff::chunks(h, count, &chunk);
    const size_t E = (size_t)2 * ne * R;
    const size_t nspec = 2 * E * 2;
    double *phi = nullptr, *part = nullptr, *X = nullptr, *PX = nullptr, *S = nullptr, *Z = nullptr;
    double *spec = nullptr, *ddir = nullptr, *dfield = nullptr, *fpart = nullptr;
    auto release = [&]() {
        dfree(h, phi); dfree(h, part); dfree(h, X); dfree(h, PX); dfree(h, S); dfree(h, Z);
        dfree(h, spec); dfree(h, ddir); dfree(h, dfield); dfree(h, fpart);
    };
    int rc;
    if ((rc = dalloc(h, &phi, (size_t)2 * count, false)) || (rc = dalloc(h, &part, (size_t)nchunk * E * 4, false)) ||
        (rc = dalloc(h, &X, (size_t)ne * nc, false)) || (rc = dalloc(h, &PX, (size_t)ne * nc, false)) ||
        (h->opt.recovery == 1 && ((rc = dalloc(h, &S, (size_t)h->nf * nc, false)) ||
                                  (rc = dalloc(h, &Z, (size_t)h->nf * nc, false)))) ||
        (rc = dalloc(h, &spec, nspec, false)) || (rc = dalloc(h, &ddir, (size_t)3 * std::max(ndir, 1), false)) ||
        (rc = dalloc(h, &fpart, (size_t)24 * R * std::max(ndir, 1) * motk_ff::field_slices(h), false)) ||
        (rc = dalloc(h, &dfield, (size_t)12 * R * std::max(ndir, 1), false))) {
        release();
        return rc;
    }
    int worst = MOT_OK;
    motk_ff::phase(h, first, count, omega, phi);
    motk_ff::spectrum(h, first, count, chunk, nchunk, phi, part);
    motk_ff::reduce(h, nchunk, part, X);
    if (h->opt.recovery == 1) rc = sigma_project(h, nc, X, PX, S, Z);
    else motk_ff::project(h, X, PX);         // a few columns: the tall-skinny product
    if (rc && rc != MOT_ENOCONV) { release(); return rc; }
    if (rc) worst = rc;
    motk_ff::parts(h, X, PX, spec);
    if (ndir > 0) {
        if (hipMemcpyAsync(ddir, dirs, sizeof(double) * 3 * ndir, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
            release();
            return mot_fail(h, MOT_EHIP, "direction upload failed");
        }
        motk_ff::field(h, omega, ndir, ddir, spec, fpart, dfield);
        hipError_t e = hipMemcpyAsync(field_out, dfield, sizeof(double) * 12 * R * ndir, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) { release(); return mot_fail(h, MOT_EHIP, hipGetErrorString(e)); }
    }
    if (spec_out) {
        hipError_t e = hipMemcpyAsync(spec_out, spec, sizeof(double) * nspec, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) { release(); return mot_fail(h, MOT_EHIP, hipGetErrorString(e)); }
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    release();
    if (e != hipSuccess) return mot_fail(h, MOT_EHIP, hipGetErrorString(e));
    return worst;
}

// ---- checkpoint and restore of the march ----
// A checkpoint holds what the next step reads: the step counter, the ring of
// the last unknowns (eq. (MOT) history), the last solution, both halves of the
// batched RHS, the Krylov state words, the speculative Arnoldi count, and the
// kept history (all of it, or the last step, which the star recovery of the
// next step needs).  Host buffer layout: a header, then those arrays in that
// order, raw FP64 / struct bytes.
namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, ne, n2, R, Rp, nh, B, precision, precond, k, spec_iters, hist_first, hist_count;
    int32_t pad;
    double dt, Tmax;
    int64_t iters_total;
};
const char kCkptMagic[8] = {'M', 'O', 'T', 'C', 'K', 'P', 'T', '1'};
struct CkptLayout {
    size_t ring, x, rb, gms, hist, total;   // byte counts
    int hfirst, hcount;
};
CkptLayout ckpt_layout(const mot_handle* h, int with_history, int k, int hist_first) {
    CkptLayout L{};
    const size_t v = (size_t)h->n2 * h->Rp * sizeof(double);
    L.ring = (size_t)h->nh * v;
    L.x = v;
    L.rb = (size_t)4 * h->ne * h->B * h->Rp * sizeof(double);
    L.gms = (h->Rp > 1 ? (size_t)h->Rp : 0) * sizeof(GmState);
    // Kept steps are slots hist_first .. k-1, all below hist_cap: a march past
    // the kept capacity (allowed when no outputs are asked for) or a restore
    // without history leaves the last step unkept, and then nothing is saved.
    if (!h->hist || k == 0 || k > h->hist_cap || k - 1 < hist_first) { L.hfirst = k; L.hcount = 0; }
    else if (with_history) { L.hfirst = hist_first; L.hcount = k - hist_first; }
    else { L.hfirst = k - 1; L.hcount = 1; }
    L.hist = (size_t)L.hcount * v;
    L.total = sizeof(CkptHeader) + L.ring + L.x + L.rb + sizeof(GmState) + L.gms + L.hist;
    return L;
}
}  // namespace

int mot_checkpoint_size(const mot_handle* h, int32_t with_history, uint64_t* bytes) {
    if (!h || !bytes) return MOT_EINVAL;
    *bytes = ckpt_layout(h, with_history, h->k, h->hist_first).total;
    return MOT_OK;
}

int mot_checkpoint(mot_handle* h, int32_t with_history, void* buf, uint64_t size) {
    if (!h || !buf) return MOT_EINVAL;
    const CkptLayout L = ckpt_layout(h, with_history, h->k, h->hist_first);
    if (size < L.total) return mot_fail(h, MOT_EINVAL, "checkpoint buffer too small");
    CkptHeader hd{};
    std::memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 1; hd.ne = h->ne; hd.n2 = h->n2; hd.R = h->R; hd.Rp = h->Rp; hd.nh = h->nh; hd.B = h->B;
    hd.precision = h->opt.precision; hd.precond = h->opt.precond; hd.k = h->k; hd.spec_iters = h->spec_iters;
    hd.hist_first = L.hfirst; hd.hist_count = L.hcount; hd.dt = h->dt; hd.Tmax = h->Tmax;
    hd.iters_total = h->iters_total;
    char* p = static_cast<char*>(buf);
    std::memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    const size_t v = (size_t)h->n2 * h->Rp;
    hipStream_t s = h->stream;
    HIPCHK(h, hipMemcpyAsync(p, h->ring, L.ring, hipMemcpyDeviceToHost, s)); p += L.ring;
    HIPCHK(h, hipMemcpyAsync(p, h->x, L.x, hipMemcpyDeviceToHost, s)); p += L.x;
    HIPCHK(h, hipMemcpyAsync(p, h->rb, L.rb, hipMemcpyDeviceToHost, s)); p += L.rb;
    HIPCHK(h, hipMemcpyAsync(p, h->gm, sizeof(GmState), hipMemcpyDeviceToHost, s)); p += sizeof(GmState);
    if (L.gms) { HIPCHK(h, hipMemcpyAsync(p, h->gms, L.gms, hipMemcpyDeviceToHost, s)); p += L.gms; }
    if (L.hist) { HIPCHK(h, hipMemcpyAsync(p, h->hist + (size_t)L.hfirst * v, L.hist, hipMemcpyDeviceToHost, s)); }
    HIPCHK(h, hipStreamSynchronize(s));
    return MOT_OK;
}

int mot_restore(mot_handle* h, const void* buf, uint64_t size) {
    if (!h || !buf) return MOT_EINVAL;
    if (size < sizeof(CkptHeader)) return mot_fail(h, MOT_EINVAL, "checkpoint too short");
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof hd);
    if (std::memcmp(hd.magic, kCkptMagic, 8) || hd.version != 1) return mot_fail(h, MOT_EINVAL, "not a checkpoint");
    if (hd.ne != h->ne || hd.n2 != h->n2 || hd.R != h->R || hd.Rp != h->Rp || hd.nh != h->nh || hd.B != h->B ||
        hd.precision != h->opt.precision || hd.precond != h->opt.precond || hd.dt != h->dt || hd.Tmax != h->Tmax)
        return mot_fail(h, MOT_EINVAL, "checkpoint taken from a different problem or options");
    if (!all_folded(h)) return mot_fail(h, MOT_ESTATE, "lag matrices missing: upload every block first");
    if (hd.k < 0 || hd.spec_iters < 1 || hd.spec_iters > h->M || hd.hist_count < 0 ||
        hd.hist_first < 0 || (int64_t)hd.hist_first + hd.hist_count != (hd.hist_count ? hd.k : hd.hist_first))
        return mot_fail(h, MOT_EINVAL, "corrupt checkpoint header");
    if (hd.hist_count && (!h->hist || hd.k > h->hist_cap))
        return mot_fail(h, MOT_EINVAL, "checkpoint holds kept steps beyond this handle's kept history");
    const CkptLayout L = ckpt_layout(h, 1, hd.k, hd.hist_first);
    const size_t need = L.total - L.hist + (size_t)hd.hist_count * h->n2 * h->Rp * sizeof(double);
    if (size < need) return mot_fail(h, MOT_EINVAL, "checkpoint truncated");
    const char* p = static_cast<const char*>(buf) + sizeof hd;
    const size_t v = (size_t)h->n2 * h->Rp;
    hipStream_t s = h->stream;
    HIPCHK(h, hipMemcpyAsync(h->ring, p, L.ring, hipMemcpyHostToDevice, s)); p += L.ring;
    HIPCHK(h, hipMemcpyAsync(h->x, p, L.x, hipMemcpyHostToDevice, s)); p += L.x;
    HIPCHK(h, hipMemcpyAsync(h->rb, p, L.rb, hipMemcpyHostToDevice, s)); p += L.rb;
    HIPCHK(h, hipMemcpyAsync(h->gm, p, sizeof(GmState), hipMemcpyHostToDevice, s)); p += sizeof(GmState);
    if (L.gms) { HIPCHK(h, hipMemcpyAsync(h->gms, p, L.gms, hipMemcpyHostToDevice, s)); p += L.gms; }
    if (hd.hist_count)
        HIPCHK(h, hipMemcpyAsync(h->hist + (size_t)hd.hist_first * v, p, (size_t)hd.hist_count * v * sizeof(double),
                                 hipMemcpyHostToDevice, s));
    motk_step::set_step(h, hd.k);
    motk_step::clear_halt(h);
    if (h->opt.history_form == 1) motk_step::raw_reproject(h);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    h->k = hd.k;
    h->spec_iters = hd.spec_iters;
    h->iters_total = hd.iters_total;
    h->hist_first = hd.hist_count ? hd.hist_first : hd.k;
    return MOT_OK;
}

// Several independent marches advanced together: every handle's speculative
// window is queued on its own stream before the host waits on any of them, and
// a handle is re-queued as soon as its window has settled, so windows of
// different solves overlap on the device.  Each handle takes exactly the
// kernels mot_run would queue for it, in the same order.
int mot_run_batch(mot_handle* const* hs, int32_t n, int32_t nsteps, int32_t* status) {
    if (n < 0 || nsteps < 0 || (n > 0 && (!hs || !status))) return MOT_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!hs[i]) return MOT_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return mot_fail(hs[i], MOT_EINVAL, "handle listed twice in one batch");
    }
    std::vector<SpecRun> runs(n);
    std::vector<int> live, plain;
    for (int i = 0; i < n; ++i) {
        mot_handle* h = hs[i];
        status[i] = MOT_OK;
        if (nsteps == 0) continue;
        if (!spec_ok(h)) { plain.push_back(i); continue; }
        if (!all_folded(h)) { status[i] = mot_fail(h, MOT_ESTATE, "lag matrices missing: upload every block first"); continue; }
        int rc = spec_begin(runs[i], h, nsteps);
        if (rc) { status[i] = rc; spec_abort(h); continue; }
        live.push_back(i);
    }
    auto drop = [&](int i, int rc) { status[i] = rc; spec_abort(hs[i]); };
    std::vector<int> next;
    // a handle whose run is cancelled stops at a window boundary, its steps kept
    auto stop = [&](int i) {
        spec_end(runs[i]);
        hipError_t e = hipStreamSynchronize(hs[i]->stream);
        status[i] = e != hipSuccess ? mot_fail(hs[i], MOT_EHIP, hipGetErrorString(e)) : MOT_ECANCEL;
    };
    for (int i : live) {
        if (take_cancel(hs[i])) { stop(i); continue; }
        int rc = spec_queue(runs[i]);
        if (rc) drop(i, rc); else next.push_back(i);
    }
    live.swap(next);
    while (!live.empty()) {
        next.clear();
        for (int i : live) {
            SpecRun& r = runs[i];
            int rc = spec_settle(r);
            if (!rc && r.done < nsteps && take_cancel(r.h)) { stop(i); continue; }
            if (!rc && r.done < nsteps) rc = spec_queue(r);
            if (rc) { drop(i, rc); continue; }
            if (r.done < nsteps) { next.push_back(i); continue; }
            spec_end(r);
            hipError_t e = hipStreamSynchronize(r.h->stream);
            status[i] = e != hipSuccess ? mot_fail(r.h, MOT_EHIP, hipGetErrorString(e)) : r.worst;
        }
        live.swap(next);
    }
    // handles that march step by step (no preconditioner, profiling, or a
    // window of -1) run after the speculative ones, one after another
    for (int i : plain) status[i] = mot_run(hs[i], nsteps, nullptr, nullptr, nullptr, 0, nullptr);
    int worst = MOT_OK;
    for (int i = 0; i < n; ++i)
        if (status[i] && (worst == MOT_OK || worst == MOT_ENOCONV)) worst = status[i];
    return worst;
}

int mot_cancel(mot_handle* h) {
    if (!h) return MOT_EINVAL;
    h->cancel.store(1);
    return MOT_OK;
}

int mot_get_matrix(mot_handle* h, int32_t which, int32_t lag, double* out) {
    if (!h || !out) return MOT_EINVAL;
    const int ne = h->ne, hs = h->hs;
    const size_t blk = (size_t)ne * hs;
    hipStream_t s = h->stream;
    auto copy_blk = [&](const double* src, double* dst, int ldd) -> int {
        HIPCHK(h, hipMemcpy2DAsync(dst, ldd * sizeof(double), src, hs * sizeof(double), ne * sizeof(double), ne,
                                   hipMemcpyDeviceToHost, s));
        return MOT_OK;
    };
    int rc = MOT_OK;
    if (which == 0) {
        if (lag < 0 || lag >= h->nlags) return mot_fail(h, MOT_EINVAL, "lag out of range");
        if (!h->lag_done[lag]) return mot_fail(h, MOT_ESTATE, "lag not folded yet");
        if (h->opt.history_form == 1 && lag > 0)
            return mot_fail(h, MOT_ESTATE, "history_form 1 keeps the raw families of lags >= 1, not Q_i");
        const double* q = h->Q + (size_t)lag * 3 * blk;
        const int n = 2 * ne;
        std::vector<double> buf((size_t)ne * ne);
        // Q = [[q1, -qk], [qk, q2]]
        for (int b = 0; b < 3; ++b) {
            if ((rc = copy_blk(q + b * blk, buf.data(), ne))) return rc;
            HIPCHK(h, hipStreamSynchronize(s));
            for (int i = 0; i < ne; ++i)
                for (int j = 0; j < ne; ++j) {
                    double v = buf[(size_t)i * ne + j];
                    if (b == 0) out[(size_t)i * n + j] = v;
                    else if (b == 2) out[(size_t)(ne + i) * n + ne + j] = v;
                    else { out[(size_t)i * n + ne + j] = -v; out[(size_t)(ne + i) * n + j] = v; }
                }
        }
        return MOT_OK;
    }
    const double* src = which == 1 ? h->C1 : which == 2 ? h->C2 : which == 3 ? h->PS : which == 4 ? h->BL :
                        which == 5 ? h->Ginv : nullptr;
    if (src) {
        if ((rc = copy_blk(src, out, ne))) return rc;
        HIPCHK(h, hipStreamSynchronize(s));
        return MOT_OK;
    }
    if (which == 6) {
        // r_lag = C1 ebar + C2 Ebar / T_max of step 'lag' (Section V-C)
        if (lag < 1) return mot_fail(h, MOT_EINVAL, "step >= 1");
        double* rb2;
        const size_t NB = (size_t)h->B * h->Rp;
        if ((rc = dalloc(h, &rb2, (size_t)2 * ne * NB))) return rc;
        motk_step::rhs_batch(h, lag, rb2);
        std::vector<double> tmp((size_t)2 * ne * NB);
        HIPCHK(h, hipMemcpyAsync(tmp.data(), rb2, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        dfree(h, rb2);    // only the field temporaries were reused; the current batch r is intact
        for (int i = 0; i < ne; ++i)
            for (int r = 0; r < h->R; ++r) {
                out[(size_t)i * h->R + r] = tmp[(size_t)i * NB + r];
                out[(size_t)(ne + i) * h->R + r] = tmp[(size_t)(ne + i) * NB + r];
            }
        return MOT_OK;
    }
    return mot_fail(h, MOT_EINVAL, "unknown matrix id");
}

int mot_get_info(const mot_handle* hc, mot_info* info) {
    if (!hc || !info) return MOT_EINVAL;
    mot_handle* h = const_cast<mot_handle*>(hc);
    int rc = ev_flush(h, h->ev_hist);
    if (rc) return rc;
    if ((rc = ev_flush(h, h->ev_q0))) return rc;
    info->D = h->D; info->Tmax = h->Tmax; info->dt = h->dt;
    info->kmax = h->kmax; info->nlags = h->nlags;
    info->ne = h->ne; info->n = 2 * h->ne; info->nrhs = h->R;
    info->genus = h->genus;
    info->folded = all_folded(h) ? 1 : 0;
    info->steps_done = h->k;
    info->device_bytes = h->bytes;
    info->peak_bytes = h->peak_bytes;
    info->setup_ms = h->setup_ms;
    info->fold_ms = h->fold_ms;
    info->gmres_iters_total = h->iters_total;
    info->hist_ms = h->ev_hist.ms;
    info->hist_launches = h->ev_hist.n;
    info->q0_ms = h->ev_q0.ms;
    info->q0_launches = h->ev_q0.n;
    info->recover_ms = h->recover_ms;
    info->precond_iters = h->ns_iters;
    info->precond_resid = h->ns_resid;
    info->tuned = h->tuned;
    info->sched_hist = h->Rp > 1 ? h->hist_kc : h->sch_hist;
    info->sched_q0 = h->Rp > 1 ? h->q0_kc : h->sch_q0;
    info->sched_pc = h->Rp > 1 ? h->plain_kc : h->sch_pc;
    info->tune_ms = h->tune_ms;
    info->graph_windows = h->graph_windows;
    info->hist_wg = h->hist_wg;
    info->q0_wg = h->q0_wg;
    return MOT_OK;
}

}  // extern "C"
