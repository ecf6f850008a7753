// Launch-schedule autotuner for the per-step products of the march.
//
// Every MOT step streams the lag matrices once (history convolution), and each
// Arnoldi step applies the approximate inverse and Q_0 once.  How a launch cuts
// that work into workgroups is a schedule:
//   one RHS:      wavefronts per matrix row (1, 2 or 4), or matrix rows per
//                 wavefront (2, 4, 8), of the streaming products, and for the
//                 history the loop order (column slices across all lag blocks,
//                 or whole rows of one block);
//   several RHS:  the number of K chunks of the tile products on MFMA (more
//                 chunks: more workgroups in flight, more partial sums to add),
//                 and their workgroup shape: 4 or 8 wavefronts (64 or 128
//                 rows) sharing each staged slice of the history vectors.
// The fastest schedule depends on the sizes, the lag count and the chip, so it
// is measured: once all lags are folded, each candidate runs on the real
// operands a few times on the handle's stream, timed with HIP events, and the
// fastest (smallest of its repetitions) is kept.  Choices are cached for the
// process under a key of every size and option that shapes the launches, so
// solves of the same shape (a serving stream) time nothing.  A schedule only
// changes the order of summation, never what is summed.
#include "mot_internal.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

namespace motk_step {
void history(mot_handle* h);
void q0_matvec(mot_handle* h, const double* src, double* vout, double* y, int check_done, int use_inv);
void precond(mot_handle* h, const double* src, double* vj, double* z, bool start = false);
}  // namespace motk_step

namespace motk_multi {
void history_gemm(mot_handle* h);
void q0_gemm(mot_handle* h, const double* X);
void precond(mot_handle* h, const double* src, double* vj, double* z);
}  // namespace motk_multi

namespace {

struct Schedule {
    int sch_hist, sch_q0, sch_pc;
    int hist_kc, q0_kc, plain_kc;
    int hist_wg, q0_wg;
};

typedef std::tuple<int, int, int, int, int, int, int, int, int, int> Key;

std::mutex g_mu;
std::map<Key, Schedule> g_cache;

Key key_of(const mot_handle* h, int dev) {
    return Key(dev, h->ne, h->nh, h->Rp, h->opt.precision, h->hilo, h->opt.precond,
               h->opt.precision == MOT_MIXED32 ? h->opt.mix_group : 0, 2 * h->tune_hist + h->tune_mv,
               (h->tune_hist ? 0 : h->sch_hist) + 100000 * h->opt.tile_wg);
}

Schedule current(const mot_handle* h) {
    return Schedule{h->sch_hist, h->sch_q0, h->sch_pc, h->hist_kc, h->q0_kc, h->plain_kc, h->hist_wg, h->q0_wg};
}

void apply(mot_handle* h, const Schedule& s) {
    h->sch_hist = s.sch_hist;
    h->sch_q0 = s.sch_q0;
    h->sch_pc = s.sch_pc;
    h->hist_kc = s.hist_kc;
    h->q0_kc = s.q0_kc;
    h->plain_kc = s.plain_kc;
    h->hist_wg = s.hist_wg;
    h->q0_wg = s.q0_wg;
}

// Smallest time (ms) of `reps` launches of f, after one untimed launch.
template <class F>
int best_time(mot_handle* h, F f, int reps, float* out) {
    hipEvent_t a, b;
    HIPCHK(h, hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return mot_fail(h, MOT_EHIP, "hipEventCreate failed");
    }
    float best = 3.4e38f;
    int rc = MOT_OK;
    f();
    for (int r = 0; r < reps && rc == MOT_OK; ++r) {
        float ms = 0;
        if (hipEventRecord(a, h->stream) != hipSuccess) { rc = MOT_EHIP; break; }
        f();
        if (hipEventRecord(b, h->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess)
            rc = MOT_EHIP;
        best = std::min(best, ms);
    }
    if (rc == MOT_OK && hipGetLastError() != hipSuccess) rc = MOT_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return mot_fail(h, rc, "autotune: a timed launch failed");
    *out = best;
    return MOT_OK;
}

// Pick the fastest value of one schedule field among cands.  With MOT_TUNE_LOG
// set in the environment every measurement is written to stderr.
template <class Set, class F>
int pick(mot_handle* h, const char* what, const std::vector<int>& cands, Set set, F launch, int reps) {
    if (cands.size() < 2) return MOT_OK;
    static const bool log = std::getenv("MOT_TUNE_LOG") != nullptr;
    int best_v = cands[0];
    float best_t = 3.4e38f;
    for (int v : cands) {
        set(v);
        float t;
        int rc = best_time(h, launch, reps, &t);
        if (rc) return rc;
        if (log) std::fprintf(stderr, "[mot autotune] ne %d R %d %s schedule %d: %.2f us\n", h->ne, h->R, what, v,
                              1e3 * t);
        if (t < best_t) { best_t = t; best_v = v; }
    }
    set(best_v);
    return MOT_OK;
}

int tune(mot_handle* h) {
    const int reps = 5;
    // every lag active: the timed history launches stream all of Q_1..Q_{L-1}
    const int kfull = h->nh + 1;
    HIPCHK(h, hipMemcpyAsync(h->d_k, &kfull, sizeof(int), hipMemcpyHostToDevice, h->stream));
    int rc = MOT_OK;
    if (h->Rp == 1) {
        // codes: 1, 2, 4 wavefronts per row; 10 + r rows per wavefront
        if (h->tune_hist) {
            const std::vector<int> c = {11, 22, 24, 12, 14, 32, 34, 1, 2, 4};
            rc = pick(h, "history", c, [&](int v) { h->sch_hist = v; }, [&] { motk_step::history(h); }, reps);
        }
        if (!rc && h->tune_mv) {
            const std::vector<int> c = {1, 2, 4, 11, 12, 14, 18, 32, 34};
            rc = pick(h, "Q_0 product", c, [&](int v) { h->sch_q0 = v; },
                      [&] { motk_step::q0_matvec(h, h->x, nullptr, h->wA, 0, 0); }, reps);
            if (!rc && (h->M32 || h->M64))
                rc = pick(h, "approximate inverse", c, [&](int v) { h->sch_pc = v; },
                          [&] { motk_step::precond(h, h->wA, h->V, h->Z); }, reps);
        }
    } else {
        // workgroup shape at the sized K chunks, then the K chunks at that shape
        const std::vector<int> wg = {4, 8};
        // the FP32-product kernel has one shape; tile_wg fixes it
        const bool tiles = h->opt.precision != MOT_MIXED32 && h->opt.tile_wg == 0;
        if (tiles)
            rc = pick(h, "history workgroup wavefronts", wg, [&](int v) { h->hist_wg = v; },
                      [&] { motk_multi::history_gemm(h); }, reps);
        if (!rc) rc = pick(h, "history K chunks", h->hist_kc_c, [&](int v) { h->hist_kc = v; }, [&] { motk_multi::history_gemm(h); }, reps);
        if (!rc && h->opt.tile_wg == 0)
            rc = pick(h, "Q_0 workgroup wavefronts", wg, [&](int v) { h->q0_wg = v; },
                      [&] { motk_multi::q0_gemm(h, h->x); }, reps);
        if (!rc) rc = pick(h, "Q_0 K chunks", h->q0_kc_c, [&](int v) { h->q0_kc = v; }, [&] { motk_multi::q0_gemm(h, h->x); }, reps);
        if (!rc && (h->M32 || h->M64))
            rc = pick(h, "approximate inverse K chunks", h->plain_kc_c, [&](int v) { h->plain_kc = v; },
                      [&] { motk_multi::precond(h, h->wA, h->V, h->Z); }, reps);
    }
    // the march starts from step 0 with clean scratch
    const int zero = 0;
    HIPCHK(h, hipMemcpyAsync(h->d_k, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return rc;
}

}  // namespace

int mot_autotune(mot_handle* h) {
    h->tuned = 1;
    const bool any = h->Rp > 1 ? !h->hist_kc_c.empty() : (h->tune_hist || h->tune_mv);
    if (!h->opt.autotune || !any) return MOT_OK;
    int dev = 0;
    HIPCHK(h, hipGetDevice(&dev));
    const Key key = key_of(h, dev);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            apply(h, it->second);
            return MOT_OK;
        }
    }
    const auto t0 = std::chrono::steady_clock::now();
    int rc = tune(h);
    if (rc) return rc;
    h->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // a concurrent tuner of the same key may have stored its choice first:
    // every handle of one shape then runs the stored one
    std::lock_guard<std::mutex> lk(g_mu);
    apply(h, g_cache.emplace(key, current(h)).first->second);
    return MOT_OK;
}
