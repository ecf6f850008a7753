/*
 * mot.h - C ABI of the MI355X marching-on-in-time (MOT) solver for the
 * quasi-Helmholtz-projected, Calderon-preconditioned TD-PMCHWT equation
 * (Le, Muenger, Andriulli, Cools, "A Stable, Accurate, and Well-Conditioned
 * Time-Domain PMCHWT Formulation").
 *
 * The library solves, for one closed surface and R incident plane waves,
 * the lower block-triangular Toeplitz system of eq. (fulldis_PMCHWT) by the
 * recurrence of eq. (MOT):  Q_0 w_i = r_i - sum_{k>=1} Q_k w_{i-k},
 * and recovers the physical currents of eq. (dis_jm) with loop and star
 * parts kept apart.  All arithmetic runs in HIP kernels on the current
 * device; the host only validates, copies and launches.
 *
 * Conventions shared by every call
 *  - Units: exterior eps = mu = 1 (c = eta = 1); interior eps_r, mu_r.
 *  - Unknown vector w = (u; v) of length n = 2 ne, u first (Section IV-B:
 *    u = R^-1 j, v = R^-1 m).  Multi-RHS arrays are [n][nrhs] row-major
 *    (the RHS index fastest) unless stated otherwise.
 *  - Dense matrices are row-major float64.
 *  - Host pointers are owned by the caller and may be freed when the call
 *    returns; the library copies what it needs.
 *  - Return codes: MOT_OK (0) or a negative MOT_E* value; mot_last_error()
 *    then describes the failure.  A failed call leaves the handle usable
 *    unless the code is MOT_EHIP.
 *  - A handle is bound to one HIP stream and is not thread-safe.
 */
#ifndef MOT_H
#define MOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MOT_OK = 0,
    MOT_EINVAL = -1,   /* bad argument, bad mesh, lag out of range          */
    MOT_ENOMEM = -2,   /* device allocation failed or over mem_cap_bytes    */
    MOT_ENOCONV = -3,  /* GMRES hit its iteration cap; the step is kept     */
    MOT_EHIP = -4,     /* a HIP runtime call failed                         */
    MOT_ESTATE = -5,   /* call out of order (e.g. a required lag missing)   */
    MOT_ECANCEL = -6   /* the run was stopped by mot_cancel; steps kept    */
};

enum { MOT_FP64 = 0, MOT_MIXED = 1, MOT_MIXED32 = 2 }; /* history precision     */
enum { MOT_FAM_H = 0, MOT_FAM_HAT = 1, MOT_FAM_TILDE = 2 };
enum { MOT_EXT = 0, MOT_INT = 1 };
enum { MOT_OP_T = 0, MOT_OP_K = 1 };

/* Surface mesh (Section II).  Triangles counter-clockwise w.r.t. the outward
 * normal.  edges[m] = (v_minus, v_plus, c_plus, c_minus): edge m runs
 * v_minus -> v_plus (Lambda: +1 at v_plus, -1 at v_minus) and RWG f_m flows
 * from c_plus to c_minus (Sigma: +1 at c_plus, -1 at c_minus); c_plus must
 * traverse v_minus -> v_plus counter-clockwise.  f_m carries unit flux
 * (no edge-length factor): f_m = (x - x_plus)/(2 A_plus) on c_plus. */
typedef struct {
    int32_t nv, nf, ne;
    const double* verts;     /* [nv][3]  host */
    const int32_t* tris;     /* [nf][3]  host */
    const int32_t* edges;    /* [ne][4]  host */
} mot_mesh;

/* Gaussian plane wave of eq. (hin): e_in = 4A/(w sqrt(pi)) p exp(-((4/w)(c(t - t0) - k.x))^2),
 * h_in = k x e_in / eta.  pol and dir are unit vectors, pol . dir = 0. */
typedef struct {
    double amp;
    double pol[3];
    double dir[3];
    double width;            /* w  */
    double t0;
} mot_planewave;

typedef struct {
    int32_t precision;       /* history precision (Q_0, GMRES, projectors and
                                recovery are FP64 in every mode):
                                MOT_FP64 (default);
                                MOT_MIXED: Q_1..Q_{L-1} stored in FP32 (plus an
                                FP32 low part on lags 1..hilo_lags), every
                                product and sum on FP64 MFMA;
                                MOT_MIXED32: the same storage multiplied on
                                FP32 MFMA, short FP32 sums added in FP64.
                                Both mixed modes need nrhs > 1.               */
    double gmres_tol;        /* relative residual of each Q_0 solve (1e-13)  */
    int32_t gmres_restart;   /* Krylov dimension m (40)                      */
    int32_t gmres_maxit;     /* total iterations per step (400)              */
    double cg_tol;           /* graph-Laplacian and Gram solves (1e-13)      */
    int32_t cg_maxit;        /* (20000)                                      */
    double diameter;         /* D; <= 0: largest vertex distance             */
    int32_t keep_history;    /* keep every w_k on the device (1)             */
    int32_t max_steps;       /* capacity of the kept history (0: 20000)      */
    uint64_t mem_cap_bytes;  /* 0: no cap                                     */
    int32_t profile;         /* N >= 1: time every N-th launch of the history
                                kernel and of the Q_0 product with HIP events
                                on the handle's stream (results in mot_info;
                                each bracketed launch costs two event markers,
                                so N > 1 keeps the march near its unprofiled
                                rate); 0: off                                  */
    int32_t precond;         /* right preconditioner of the Q_0 GMRES: an
                                approximate inverse of Q_0 built once on the
                                device by Newton-Schulz iteration;
                                0 none, 1 stored FP32 (default), 2 FP64       */
    int32_t stream_split;    /* schedule of the one-RHS streaming products:
                                1, 2 or 4 wavefronts share one matrix row, or
                                11, 12, 14, 18: one wavefront owns 1, 2, 4 or 8
                                rows, column slices outermost
                                (the history at most 4); 32, 34: 2 or 4
                                wavefronts share as many rows; 0: chosen by
                                the autotuner (or 1).  The history follows
                                it in the loop order of history_order.        */
    int32_t history_order;   /* history kernel loop order: 1 (or 0) column
                                slices across all blocks, 2 whole rows of one
                                block at a time, 3 column slices with 2 (with
                                stream_split 12) or 4 (otherwise) wavefronts
                                sharing as many rows                          */
    int32_t hilo_lags;       /* mixed modes: lags 1..hilo_lags keep the FP32
                                low part fl(Q - fl(Q)) (default 2, -1: none);
                                MOT_MIXED32 multiplies it as split hi/lo
                                products                                      */
    int32_t mix_group;       /* MOT_MIXED32: summation indices per half that one
                                FP32 MFMA accumulator sums before it is added
                                into the FP64 total: 4 (default), 16 or 64    */
    int32_t spec_window;     /* mot_run with one RHS and a preconditioner:
                                steps queued per host check of the device halt
                                word (0: one RHS batch, 128; -1: wait for every
                                step's GMRES on the host)                     */
    int32_t recovery;        /* P^Sigma in the current recovery of eq.
                                (dis_jm): 0 (default) the dense projector
                                formed at setup, one GEMM per batch of steps;
                                1 incidence products and graph-Laplacian CG
                                per batch (no dense ne^2 product)             */
    int32_t autotune;        /* launch schedules of the per-step products
                                (history convolution, Q_0 product, approximate
                                inverse): 1 (default) time each candidate once
                                on the device when the last lag is folded and
                                keep the fastest (choices cached per process
                                for the same sizes and options); 0 fixed size
                                rules.  stream_split and history_order, when
                                set, fix their part of the choice.  Schedules
                                change only the order of summation.           */
    int32_t graph;           /* mot_run with speculative stepping: 1 replays
                                every full window of one RHS batch (B steps,
                                B = max(8, min(128, 4096 / Rp)), Rp = nrhs
                                rounded up to a power of two), aligned to a
                                batch and spec_window 0, from a
                                HIP graph captured once per batch parity (and
                                again when the Arnoldi count per queued step
                                grows); other windows, and handles on the
                                legacy default stream, queue their launches
                                one by one.  Ignored with profile = 1.
                                Results are identical to graph = 0.           */
    int32_t tile_wg;         /* several RHS: wavefronts per workgroup of the
                                history and Q_0 tile products, 4 (64 rows) or
                                8 (128 rows sharing each staged slice of the
                                history vectors); 0 (default): the autotuner
                                picks (4 without it).  Results do not depend
                                on it.                                         */
    int32_t history_form;    /* history convolution of eq. (MOT) (Sec. V-B):
                                0 (default) the folded lags
                                Q_i = C1 (Z^h_i P^{Lambda H} + Z^hat_i P^Sigma)
                                + C2 (Z^h_i P^Sigma + Z^til_i P^{Lambda H});
                                1 the raw media-summed families Z^h_i, Z^hat_i,
                                Z^til_i of lags i >= 1 kept as uploaded and
                                applied to the projected unknowns
                                P^{Lambda H} w, P^Sigma w of every step, with
                                C1 and C2 applied once per step (Q_0 stays
                                folded).  Form 1: one right-hand side,
                                host-driven steps (no speculative windows or
                                graphs); mot_get_matrix(0, i >= 1) fails with
                                MOT_ESTATE; the same results up to the order
                                of the sums.  Other values: MOT_EINVAL.        */
} mot_options;

typedef struct {
    int32_t step;            /* index k of the step just taken (1-based)     */
    int32_t gmres_iters;     /* iterations of the Q_0 solve                  */
    double gmres_relres;     /* final relative residual estimate             */
    int32_t converged;       /* 1 if the tolerance was met                   */
} mot_step_info;

typedef struct {
    double D, Tmax, dt;      /* diameter, T_max = D / c_min (eq. alpha)      */
    int32_t kmax;            /* ceil(T_max / dt)                              */
    int32_t nlags;           /* k_max + 2: Q_0 .. Q_{k_max+1}                 */
    int32_t ne, n, nrhs;
    int32_t genus;
    int32_t folded;          /* 1 once every lag matrix is formed            */
    int32_t steps_done;
    uint64_t device_bytes;   /* device memory held by the handle             */
    double setup_ms;         /* setup time: projectors, Gram inverse and the
                                C1 / C2 factors at create, plus the approximate
                                inverse of Q_0 built once lag 0 is folded     */
    double fold_ms;          /* lag-matrix fold time (sum over lags)         */
    int64_t gmres_iters_total;  /* Arnoldi steps over all steps taken        */
    double hist_ms;          /* profile: summed history-kernel time          */
    int64_t hist_launches;
    double q0_ms;            /* profile: summed Q_0 product time (GMRES)     */
    int64_t q0_launches;
    double recover_ms;       /* wall time of the last recovery (host clock)  */
    int32_t precond_iters;   /* Newton-Schulz iterations of the preconditioner */
    double precond_resid;    /* ||I - M Q_0||_F of the stored preconditioner  */
    uint64_t peak_bytes;     /* high-water mark of device_bytes so far        */
    int32_t tuned;           /* 1 once the schedules were timed (autotune)    */
    int32_t sched_hist;      /* history schedule.  One RHS: 1, 2, 4 wavefronts
                                share a matrix row (whole rows of one lag
                                block at a time); 10 + r: one wavefront owns
                                r rows (column slices across all lag blocks;
                                11 in four-wavefront workgroups); 20 + w: w
                                wavefronts share those slices of one row;
                                30 + r: r wavefronts share r rows.  Several
                                RHS: K chunks of the tile product              */
    int32_t sched_q0;        /* Q_0 product: 1, 2, 4 wavefronts per row,
                                10 + r rows per wavefront, or 30 + r: r
                                wavefronts share r rows / K chunks            */
    int32_t sched_pc;        /* approximate inverse: as sched_q0 / K chunks   */
    double tune_ms;          /* time spent timing candidates (0 on a cache hit) */
    int64_t graph_windows;   /* windows replayed from captured graphs          */
    int32_t hist_wg, q0_wg;  /* several RHS: wavefronts per workgroup of the
                                history and Q_0 tile products (4 or 8)        */
} mot_info;

typedef struct mot_handle mot_handle;

/* Fill *opt with the defaults listed above. */
void mot_default_options(mot_options* opt);

/* Create a solver (Section III-V).  Validates the mesh (Sigma^T Lambda = 0,
 * closed 2-manifold), derives D, T_max and k_max, and on the device builds
 * the projectors of Section IV-B (graph-Laplacian CG), G^-1 (CG on the normal
 * equations of the Gram matrix), and the factors
 *     C1 = PP^{Sigma H} T0s PP^{Sigma H} G^-1,
 *     C2 = PP^Lambda T0h PP^Lambda G^-1 P^{Lambda H}
 * of the lag matrices and RHS.
 *   T0s, T0h: dense [ne][ne] host, the static EFIO blocks of Section III on the
 *             BC basis (T0s SPD, T0h PSD).
 *   G: CSR [ne][ne] host, G_mn = <n x f_m, g_n>; g_rowptr has ne+1 entries.
 *   waves: nrhs plane waves (host).   stream: hipStream_t or NULL.
 * Every host input is checked before anything is allocated (mesh integers
 * and orientation, finite vertices and static blocks, Gram CSR row pointers
 * non-decreasing and columns in range, each wave with width > 0 and unit,
 * orthogonal pol and dir within 1e-6).
 * Returns MOT_EINVAL on a bad mesh or argument, MOT_ENOMEM, MOT_ENOCONV if a
 * setup solve fails to converge, MOT_EHIP. */
int mot_create(const mot_mesh* mesh, double eps_r, double mu_r, double dt,
               const double* T0s, const double* T0h,
               const int32_t* g_rowptr, const int32_t* g_col, const double* g_val,
               int32_t nrhs, const mot_planewave* waves, const mot_options* opt,
               void* stream, mot_handle** out);

/* Upload one raw retarded block of Section V-B (host, dense [ne][ne]):
 *   family MOT_FAM_H:     T_i  = <n x f_m, T^s(h0 f_n)>|_{i dt},       K_i  likewise,  lags 0..k_max
 *   family MOT_FAM_HAT:   <n x f_m, d/dt T(q0 f_n)>|_{i dt} (no T_max factor), lags 0..k_max+1
 *   family MOT_FAM_TILDE: <n x f_m, d/dt^-1 T^s(p0 f_n)>|_{i dt} (no 1/T_max factor), lags 0..k_max-1
 * medium MOT_EXT / MOT_INT, op MOT_OP_T / MOT_OP_K.  The library applies the
 * T_max scalings and the media sum of eq. (PMCHWT).  Once the twelve blocks
 * of lag i (or the subset its range requires) have arrived, Q_i is folded on
 * the device and the raw blocks are dropped.  A lag outside its family's
 * range is MOT_EINVAL (the truncation is part of the method), so is a block
 * with a non-finite entry (nothing is staged; the block may be sent again);
 * uploading a block twice is MOT_ESTATE.  With k_max = 1 the lag-0 tilde K
 * block (exactly dt times the static double layer, every pair lying inside
 * the first shell) is accepted and not used: by eq. (spec_prop) it adds
 * nothing to Q_0, as the tilde K tail adds nothing beyond k_max - 1. */
int mot_set_lag(mot_handle* h, int32_t family, int32_t lag, int32_t medium, int32_t op,
                const double* block);

/* The same with a CSR block (row pointers ne+1, int32 columns, float64 values;
 * nnz = rowptr[ne] may be 0, an all-zero block).  Row pointers must start at 0
 * and not decrease, columns lie in 0..ne-1 and values are finite, else
 * MOT_EINVAL and nothing is staged. */
int mot_set_lag_csr(mot_handle* h, int32_t family, int32_t lag, int32_t medium, int32_t op,
                    const int64_t* rowptr, const int32_t* col, const double* val);

/* The same with a dense block already in device memory (Section V-B blocks
 * assembled on the GPU, so that large problems never stage their lags on the
 * host): dblock [ne] rows of ld >= ne float64, row-major, on the handle's
 * device.  The library reads it on the handle's stream during the call and
 * keeps no reference; the caller owns it and may free or reuse it when the
 * call returns.  Work that writes dblock must be complete, or ordered before
 * the handle's stream, when the call is made.  Same checks and codes as
 * mot_set_lag; MOT_EINVAL also when dblock is not device memory or ld < ne. */
int mot_set_lag_device(mot_handle* h, int32_t family, int32_t lag, int32_t medium, int32_t op,
                       const double* dblock, int64_t ld);

/* One MOT step (eq. MOT): tested incident fields, RHS, history convolution,
 * GMRES on Q_0 (warm start 2 w_{k-1} - w_{k-2}), ring update.  MOT_ESTATE if
 * a lag is missing.  info may be NULL. */
int mot_step(mot_handle* h, mot_step_info* info);

/* nsteps MOT steps followed by the current recovery of eq. (dis_jm) for
 * those steps.  Output arrays are [nsteps][n][nrhs]; any may be NULL:
 *   w_out     the auxiliary unknowns (u; v) per step,
 *   loop_out  (P^{Lambda H} u_k; P^{Lambda H} v_k),
 *   star_out  (T_max/dt) (P^Sigma (u_k - u_{k-1}); P^Sigma (v_k - v_{k-1})).
 * out_on_device: 1 if the output pointers are device memory.  Steps continue
 * from the handle's current time.  Returns the worst step's code. */
int mot_run(mot_handle* h, int32_t nsteps, double* w_out, double* loop_out,
            double* star_out, int32_t out_on_device, mot_step_info* last);

/* Outputs of steps already taken, as mot_run returns them for its own steps
 * (same layouts, [count][n][nrhs]; any pointer may be NULL): steps are counted
 * from 0 since create or reset, and first .. first+count-1 must all be taken
 * and kept (keep_history, max_steps).  The loop and star parts are the
 * current recovery of eq. (dis_jm), recomputed on each call.  out_on_device:
 * 1 if the pointers are device memory.  MOT_EINVAL for a range not taken or
 * not kept. */
int mot_get_steps(mot_handle* h, int32_t first, int32_t count, double* w_out, double* loop_out,
                  double* star_out, int32_t out_on_device);

/* Euclidean norm of the unknowns w_s = (u_s; v_s) of each kept step s = first
 * .. first+count-1 and wave: the late-time behaviour of the march of eq. (MOT)
 * (Sec. VI-A), without copying the history out.  norms: host [count][nrhs].
 * MOT_EINVAL for a range not taken or not kept. */
int mot_step_norms(mot_handle* h, int32_t first, int32_t count, double* norms);

/* mot_step_norms for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops that poll the late-time behaviour
 * between windows, harnesses that forbid hipMalloc.  Same arguments and the
 * same results, bit for bit; the call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine): the per-step norms are staged in a
 * static device array of MOT_NOALLOC_DOUBLES doubles (1 MiB), one per GPU,
 * which the library holds from its first mot_create on that GPU until the
 * process ends.  count * nrhs must not exceed MOT_NOALLOC_DOUBLES (else
 * MOT_EINVAL; split the range).  Every handle on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (handles on different streams
 * or host threads) race and must be serialised by the caller.  The array
 * keeps the last call's contents; nothing in it needs clearing, as each call
 * writes every value it reads back. */
#define MOT_NOALLOC_DOUBLES 131072
int mot_step_norms_noalloc(mot_handle* h, int32_t first, int32_t count, double* norms);

/* Spectra and far fields of the currents of kept steps (Section VI, far-field
 * computation, on eq. (dis_jm)), the loop and star parts kept apart so that
 * neither is lost in the other at low frequency.  Steps first ..
 * first+count-1 (counted from 0, as in mot_get_steps) must be taken and kept;
 * step s carries the unit pulse on (s dt, (s+1) dt).  With the exp(+i omega t)
 * convention, omega = 2 pi freq, the spectrum of each part is
 *   X(f) = sum_s x_s int_{s dt}^{(s+1) dt} exp(-i omega t) dt,
 * x_s the loop or star coefficients of mot_run, and the far field of each
 * part in the unit direction rhat (the exp(-i k r)/r factor dropped, k =
 * omega, exterior c = eta = 1) is
 *   E(rhat) = (i k / 4 pi) [rhat x L + rhat x (rhat x N)],
 *   N = sum_n J_n int f_n exp(i k rhat.x) dS,  L likewise with M,
 * the integrals on the 7-point rule of the incident-field testing.
 *   dirs       host [ndir][3] unit vectors (|d|^2 within 1e-9 of 1);
 *   field_out  host [ndir][nrhs][2 parts: loop, star][3][2: re, im];
 *   spec_out   host [2 parts][n][nrhs][2: re, im], or NULL.
 * ndir may be 0 (spectra only).  Scratch device memory is taken from the
 * handle's pool for the call and released before it returns.  MOT_EINVAL for
 * a range not taken or not kept, a negative or non-finite frequency, or a
 * direction that is not a unit vector; MOT_ENOCONV if the CG form of
 * P^Sigma (recovery = 1) hit its cap (outputs still written). */
int mot_far_field(mot_handle* h, int32_t first, int32_t count, double freq, int32_t ndir,
                  const double* dirs, double* field_out, double* spec_out);

/* Checkpoint of the march of eq. (MOT) after the steps taken so far, to
 * resume it later in a handle built from the same inputs: the step counter,
 * the ring of the last unknowns, the last solution, the batched RHS, the
 * Krylov state and, with with_history = 1, every kept step (with 0, the last
 * kept step only, which the star recovery of the next step needs).
 * mot_checkpoint_size gives the bytes; mot_checkpoint writes them to host
 * memory buf (size at least that).  Call between marches, with nothing queued
 * on the handle.  MOT_EINVAL for a null handle or a short buffer. */
int mot_checkpoint_size(const mot_handle* h, int32_t with_history, uint64_t* bytes);
int mot_checkpoint(mot_handle* h, int32_t with_history, void* buf, uint64_t size);

/* Resume a march from a checkpoint (host memory): h must be created with the
 * same mesh, media, dt, waves and options and hold every lag block.  The next
 * steps then compute exactly what the checkpointed handle would have (the
 * same launch schedules, fixed by options or chosen by the autotuner in the
 * same process, give bit-identical results; others differ by summation
 * order).  Kept steps before the checkpoint's are not held: mot_get_steps and
 * mot_far_field refuse them.  MOT_EINVAL if buf is not a checkpoint of a
 * matching problem, is truncated, or holds more kept steps than max_steps;
 * MOT_ESTATE if a lag block is missing. */
int mot_restore(mot_handle* h, const void* buf, uint64_t size);

/* nsteps MOT steps (eq. MOT) on each of n independent handles, for serving
 * several scattering problems at once: the handles' windows of queued steps
 * are interleaved across their streams, so small solves share the device
 * instead of taking turns.  Every handle computes exactly what mot_run(h,
 * nsteps, NULL, NULL, NULL, 0, NULL) would; mot_get_steps reads the outputs
 * afterwards (keep_history).  Handles on distinct non-default streams
 * overlap; handles sharing a stream run in turn.  The call drives every
 * handle from the calling thread: no other thread may use them meanwhile.
 * hs: n distinct handles (host array); status: n codes out,
 * each handle's worst step code (MOT_OK, MOT_ENOCONV) or its error, after
 * which that handle stops at its last completed step while the others go on.
 * Returns MOT_EINVAL for a bad argument or a repeated handle (nothing run),
 * else the first error among the handles, else MOT_ENOCONV if any step hit
 * its iteration cap, else MOT_OK. */
int mot_run_batch(mot_handle* const* hs, int32_t n, int32_t nsteps, int32_t* status);

/* Stop a mot_run or mot_run_batch in progress on h, for a server whose
 * request outlives its time limit: safe to call from any host thread.  The
 * run stops at its next window boundary (at most spec_window steps of the
 * speculative march, or the next step when it steps one at a time) and
 * returns MOT_ECANCEL (in h's status slot for mot_run_batch, the other
 * handles going on); every completed step is kept and the handle stays
 * usable, a later mot_run continuing from there.  mot_run's outputs then
 * hold the completed steps (mot_get_info: steps_done), the rest of its
 * output arrays untouched.  A request made while no run is in progress stops
 * the next run before its first window; mot_reset clears it.  Returns MOT_OK,
 * or MOT_EINVAL for a NULL handle. */
int mot_cancel(mot_handle* h);

/* Copy internal operators to host memory (diagnostics and parity checks):
 *   which 0: Q_lag as dense [n][n]; 1: C1 [ne][ne]; 2: C2 [ne][ne];
 *   3: P^Sigma [ne][ne]; 4: PP^Lambda [ne][ne]; 5: G^-1 [ne][ne];
 *   6: RHS r_lag of step 'lag' as [n][nrhs] (computed, not stored state). */
int mot_get_matrix(mot_handle* h, int32_t which, int32_t lag, double* out);

int mot_get_info(const mot_handle* h, mot_info* info);

/* Device memory a solve will need, before creating it: for admission by memory
 * footprint when several solves share one GPU.  The arguments are those of
 * mot_create (gram_nnz: nonzeros of G); nothing is allocated.
 *   resident_bytes: held from the end of setup until mot_destroy (lag
 *                   matrices Q_0..Q_{k_max+1} of Section V-B, projectors and
 *                   factors of Sections III-IV, ring and kept history of the
 *                   march of eq. (MOT), Krylov space, preconditioner);
 *   peak_bytes:     resident plus the largest transient phase (setup solves,
 *                   one lag staged for its fold, recovery batches).
 * Both match what mot_create and mot_run allocate under the same options.
 * MOT_EINVAL on a bad argument. */
int mot_footprint(const mot_mesh* mesh, double eps_r, double mu_r, double dt, int32_t nrhs,
                  int64_t gram_nnz, const mot_options* opt, uint64_t* resident_bytes,
                  uint64_t* peak_bytes);

/* Restart the march at step 0 (keeps every operator); the march that follows
 * is the one a new handle would compute. */
int mot_reset(mot_handle* h);

void mot_destroy(mot_handle* h);

/* Text of the last error on this handle, or of the last failed create when h is NULL. */
const char* mot_last_error(const mot_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* MOT_H */
