/*
 * fcas.h -- C ABI of the MI355X coherent-fitness library.
 *
 * The library evaluates the coherent fitness Gamma^2(theta) of a fully
 * coherent all-sky search for compact-binary inspirals (Normandin & Mohanty,
 * arXiv:2002.02150, Sec. II.C eqs. FCASdetStat / gammaSqd) for whole batches
 * of parameter points theta = (alpha, delta, tau0, tau1.5) at once, its
 * gradient at the maximising time sample, and the lbest particle-swarm update
 * that drives the search (Sec. III).
 *
 * Conventions shared by every entry point
 *   - Every pointer named d_* is a DEVICE pointer owned by the caller,
 *     contiguous, with the element type and shape stated.  The library never
 *     frees caller memory.  It allocates device memory only in fcas_create()
 *     (context tables and workspace) and fcas_set_segment() (per-segment data).
 *   - fitness_eval_batch, fitness_grad_batch, pso_init, pso_step and pso_best
 *     are asynchronous on `hip_stream` (a hipStream_t, NULL = the null
 *     stream): no allocation, no host synchronisation, no device-to-host copy.
 *     They may be captured into a HIP graph.  One context must not be used by
 *     two streams at once (calls on one context share its workspace).
 *   - Return value: FCAS_OK (0) or a negative FCAS_E* code; the message of the
 *     last failure on the calling thread is returned by fcas_last_error().
 *     Arguments are validated on the host before anything is enqueued.
 *   - A parameter point outside the search rectangle, or with a non-finite
 *     coordinate, is not an error: its fitness is -inf and its argmax -1
 *     (particles may leave the rectangle and are then not evaluated).
 *   - A segment id that is out of range or not registered is detected on the
 *     device: fitness NaN, argmax -2, and the context's device error flag is
 *     set (read it with fcas_device_error(), which synchronises).
 *   - Results are bitwise repeatable: a point's fitness and argmax do not depend
 *     on the batch, the order, the grid sizes, the workspace chunking or the
 *     schedule it is evaluated with.
 */
#ifndef FCAS_H
#define FCAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCAS_MAX_DET 8

/* return codes */
#define FCAS_OK 0
#define FCAS_EINVAL (-1)          /* bad pointer, size, shape or parameter          */
#define FCAS_ENOSEG (-2)          /* segment id out of range                         */
#define FCAS_EUNSUPPORTED_N (-3)  /* segment length has no FFT plan                  */
#define FCAS_EHIP (-4)            /* a HIP runtime call failed (no device, launch)   */
#define FCAS_ENOMEM (-5)          /* device allocation failed                        */
#define FCAS_ECAPACITY (-6)       /* batch larger than the context was created for  */

/* arithmetic of the fitness path */
#define FCAS_MIXED 0  /* template phase in FP64, reduced mod 1 cycle; data, FFT,
                         projection and maximum in FP32                           */
#define FCAS_FP64 1   /* everything in FP64 (the plain reference path)            */

/* launch schedule of the FFT passes (FUSED: FCAS_MIXED only; an FCAS_FP64
 * context runs TWO_PASS, and so do, under FUSED, the three-pass plans and the
 * plans whose two passes use work-groups of different sizes) */
#define FCAS_SCHEDULE_FUSED 0     /* one persistent launch per plan, passes pipelined  */
#define FCAS_SCHEDULE_TWO_PASS 1  /* a pass-1 and a pass-2 launch per workspace chunk
                                     (the faster one on MI355X: recommended)          */

typedef struct fcas_ctx fcas_ctx;

/* Detector network (Sec. II eq. detresponse).  pos_m: vertex of detector i in
 * the Earth-centred Earth-fixed frame (metres); tensor: its response tensor
 * D^i = (a a^T - b b^T) / 2 for unit arm vectors a, b.  Only the first n_det
 * rows are read. */
typedef struct {
  int32_t n_det;                       /* 1..FCAS_MAX_DET */
  double pos_m[FCAS_MAX_DET][3];
  double tensor[FCAS_MAX_DET][3][3];
} fcas_network;

/* Search configuration.  f_low_hz is both the high-pass cutoff f_* below
 * which templates vanish and the reference frequency of the chirp times
 * (Sec. II.B); f_high_hz is the generic upper cutoff.  In-band bins are
 * f_* < k/T <= min(f_high, fs/2), 1 <= k < N/2.  box_lo/box_hi bound
 * (alpha [rad], delta [rad], tau0 [s], tau1.5 [s]). */
typedef struct {
  double fs_hz, f_low_hz, f_high_hz;
  int32_t precision;      /* FCAS_MIXED or FCAS_FP64 */
  int32_t max_batch;      /* largest n accepted by fitness_eval/grad_batch */
  int32_t max_segments;   /* segment ids are 0..max_segments-1 */
  int32_t schedule;       /* FCAS_SCHEDULE_TWO_PASS or FCAS_SCHEDULE_FUSED */
  int64_t max_samples;    /* largest segment length N that will be registered */
  int64_t workspace_bytes;/* FFT workspace; 0 = enough for max_batch evaluations
                             of max_samples (batches beyond it run in chunks) */
  double box_lo[4], box_hi[4];
} fcas_config;

/* Creates a context on HIP device `device` (its tables and workspace live in
 * that device's memory).  Fails with FCAS_EINVAL on a bad network/config,
 * FCAS_EUNSUPPORTED_N if max_samples has no plan, FCAS_EHIP if the device is
 * not usable, FCAS_ENOMEM if allocation fails.  *out is NULL on failure. */
int fcas_create(const fcas_network* net, const fcas_config* cfg, int device, fcas_ctx** out);

/* Frees the context and all library-owned device memory (synchronises the device). */
int fcas_destroy(fcas_ctx* ctx);

/* Bytes of FFT workspace owned by the context. */
size_t fcas_workspace_bytes(const fcas_ctx* ctx);

/* 1 if a segment of n samples has an FFT plan, else 0 (host only, no device).
 * Supported: 2^k for 2^11 <= n <= 2^18, 3 * 2^k for 2^13 <= n / 3 <= 2^16, and
 * 2^k * 225 for k = 11, 14, 15 (225 s, 30 min and one hour at 2048 Hz). */
int fcas_supported_n(int64_t n_samples);

/* FFT plans.  A plan splits N = N1 N2 into N1-point column transforms (pass 1,
 * E1 elements per thread, `cols` columns per work-group) and N2-point row
 * transforms (pass 2, E2 elements per thread, `rows` rows per work-group);
 * several plans may serve one length.  The 2^k * 225 lengths run three
 * passes, N = N1 * 225 * N2', with 225-point transforms between the two: for
 * them `n2` reports the 225 N2' columns of pass 1 and `e2`, `rows` describe
 * the N2'-point last pass.  fcas_plan_info reports plan `plan` (float
 * figures; host only, any output may be NULL). */
int fcas_plan_count(void);
int fcas_plan_info(int32_t plan, int64_t* n_samples, int32_t* n1, int32_t* n2, int32_t* e1, int32_t* e2,
                   int32_t* cols, int32_t* rows);

/* Use plan `plan` for segments of its length registered after this call, with
 * grid1 / grid2 persistent work-groups for its first and last passes (grid2
 * also sizes a three-pass plan's middle pass; 0 = default).
 * This is how the autotuner's choice is applied.  FCAS_EINVAL for a plan out
 * of range or grid sizes outside [0, 2^20]. */
int fcas_select_plan(fcas_ctx* ctx, int32_t plan, int32_t grid1, int32_t grid2);

/* Registers (or replaces) segment `seg_id` of n_samples samples per detector
 * (Sec. II.D: the template norms are precomputed and the data over-whitened
 * once).  d_xf: one-sided Fourier data of each detector in continuum units
 * (dt times the DFT), complex128 interleaved (re, im), shape
 * [n_det][n_samples/2 + 1].  d_psd: one-sided PSD, float64, same shape.
 * The library stores sigma_i^2 = 4 df sum_B f^-7/3 / S^i and
 * y^i_k = 4 df x^i_k f_k^-7/6 / (S^i_k sigma_i) for the in-band bins.  The
 * inputs may be freed once the call returns; it synchronises `hip_stream`.
 * Not capturable.  Errors: FCAS_ENOSEG (id out of range),
 * FCAS_EUNSUPPORTED_N / FCAS_EINVAL (length, NULL pointer, empty band, a
 * template norm sigma_i^2 that is not positive and finite, e.g. a zero or
 * non-finite PSD value in band), FCAS_ENOMEM, FCAS_EHIP.  A call that fails
 * after its arguments were validated leaves seg_id unregistered, also when
 * it was registered before (evaluations of it then give NaN, -2). */
int fcas_set_segment(fcas_ctx* ctx, int32_t seg_id, int64_t n_samples,
                     const double* d_xf, const double* d_psd, void* hip_stream);

/* Restricts the maximisation over the coalescence time (Sec. II.C) for
 * segment seg_id to samples j_lo <= j < j_hi (default: all N samples, right
 * for cyclic data).  For a segment cut from a longer stream, searching only its
 * central part keeps the matched filter away from the wrap-around at the
 * edges, and overlapping segments cover every coalescence time once.
 * Synchronous; not capturable; applies to later evaluations. */
int fcas_set_segment_range(fcas_ctx* ctx, int32_t seg_id, int64_t j_lo, int64_t j_hi);

/* Coherent fitness of n parameter points (Sec. II.C eqs. FCASdetStat,
 * gammaSqd; Sec. II.D).  For each point:
 *   Gamma^2 = max_j max_{A_1..A_4} 2 lambda(theta, A, t_c = j / fs),
 * evaluated as max_j z_j^H P z_j with z^i_j the matched-filter output of
 * detector i at coalescence sample j (data shifted by the detector delay
 * Delta^i, eq. data_template_innprod) and P the projector onto the span of
 * diag(sigma) F(alpha, delta, 0).  With this scale Gamma^2 = SNR^2 for a
 * noiseless signal at its true parameters.
 *   d_theta   float64 [n][4]  (alpha, delta, tau0, tau1.5)
 *   d_seg     int32   [n]     segment of each point
 *   d_fitness float64 [n]     Gamma^2 (-inf outside the rectangle)
 *   d_argmax  int32   [n]     j*, smallest maximising sample (-1 outside);
 *                             j* times 1/fs is the coalescence time at the Earth's
 *                             centre modulo the segment length
 * 0 <= n <= max_batch (n = 0 does nothing). */
int fitness_eval_batch(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg,
                       double* d_fitness, int32_t* d_argmax, void* hip_stream);

/* For callers that cannot allocate device memory at call time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, arguments, results and errors as fitness_eval_batch (the
 * same kernels; results bitwise equal), with the call's scratch memory (point
 * descriptors, work lists, pass-2 partials, FFT workspace) taken from a static
 * array of 64 MiB that the library holds on each GPU it runs on until the
 * process ends, instead of the context's buffers.  The call allocates nothing.
 * Limit: the tables take about 0.75 KB + 8 S bytes per point (S = pass-2
 * partials per point: at most 512 for contexts whose max_samples is at most
 * 262144) and the rest is FFT workspace, which must hold at least one point of
 * the longest registered segment (2 N 8 bytes mixed, 2 N 16 bytes FP64: an
 * hour-long segment does not fit); more points than it holds run in chunks.  A call
 * beyond the limit fails with FCAS_ECAPACITY before anything is enqueued.
 * Every call on one GPU, from any context, uses that GPU's one array: calls
 * whose executions overlap on a GPU race (serialise them on one stream).
 * Always the two-pass schedule; no per-kernel timing is recorded. */
int fitness_eval_batch_static(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg,
                              double* d_fitness, int32_t* d_argmax, void* hip_stream);

/* As fitness_eval_batch, plus d_grad float64 [n][4] = dGamma^2/dtheta with the
 * maximising sample j* held fixed (zero outside the rectangle).  Supports
 * networks whose antenna matrix has rank two, or a single detector. */
int fitness_grad_batch(fcas_ctx* ctx, int32_t n, const double* d_theta, const int32_t* d_seg,
                       double* d_fitness, int32_t* d_argmax, double* d_grad, void* hip_stream);

/* Gradient ascent ("polish") of n points, typically the best particles of a
 * search: step s computes dGamma^2/dtheta at fixed j* (as fitness_grad_batch),
 * evaluates the n_trials points theta + step_frac 2^-t w^2 g / |w g|,
 * t = 0..n_trials-1 (w = widths of the search rectangle, g the gradient) in
 * one fitness batch, and moves each point to its best trial if that raises
 * Gamma^2.  d_theta float64 [n][4] is read and updated in place; d_fitness
 * float64 [n] and d_argmax int32 [n] receive Gamma^2 and j* at the final
 * points.  Needs n * n_trials <= max_batch, 1 <= n_trials <= 32. */
int fitness_polish(fcas_ctx* ctx, int32_t n, double* d_theta, const int32_t* d_seg, int32_t n_steps,
                   double step_frac, int32_t n_trials, double* d_fitness, int32_t* d_argmax, void* hip_stream);

/* lbest particle swarm (Sec. III).  Positions and velocities live in the unit
 * hypercube of the search rectangle, theta = lo + x (hi - lo).  Random numbers
 * are Philox4x32-10 keyed by the seed, counter (iteration, particle, run,
 * stream).  Update: v <- w v + c1 r1 (pbest - x) + c2 r2 (lbest - x), w falls
 * linearly from w0 to w1 over n_iter, |v| <= vmax per coordinate, x <- x + v;
 * lbest is the best personal best among ring neighbours (i-1, i, i+1). */
typedef struct {
  int32_t n_runs, n_particles, n_iter, reserved;
  double w0, w1, c1, c2, vmax;
  uint64_t seed;
} fcas_pso_params;

/* Caller-owned device arrays of a swarm (R = n_runs, P = n_particles). */
typedef struct {
  double* x;        /* [R][P][4] position (unit-cube coordinates) */
  double* v;        /* [R][P][4] velocity */
  double* pbest_x;  /* [R][P][4] personal best position */
  double* pbest_f;  /* [R][P]    personal best fitness */
  int32_t* pbest_j; /* [R][P]    argmax sample at the personal best */
  double* best_x;   /* [R][4]    best position of each run */
  double* best_f;   /* [R]       best fitness of each run */
  int32_t* best_j;  /* [R]       argmax sample at the run's best */
  int32_t* iteration; /* [2]     [0]: iterations taken (pso_init sets 0, pso_step adds 1);
                                [1]: pso_step's tally of finished runs (pso_init sets 0) */
} fcas_pso_state;

/* Random initial positions / velocities; pbest_f = best_f = -inf.
 * d_theta_out float64 [R*P][4]: the first points to evaluate. */
int pso_init(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s,
             double* d_theta_out, void* hip_stream);

/* One iteration given d_fitness / d_argmax [R*P] of the current positions
 * (from fitness_eval_batch on the points pso_init or the previous pso_step
 * wrote): updates personal, local and run bests, moves the swarm (inertia of
 * iteration *s->iteration, read on the device, which is then incremented), and
 * writes the next points to d_theta_next float64 [R*P][4].  Because the
 * iteration count lives on the device, one captured iteration can be replayed. */
int pso_step(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s,
             const double* d_fitness, const int32_t* d_argmax, double* d_theta_next, void* hip_stream);

/* n_iter iterations of the swarm (Sec. III), each the fitness of the current
 * points followed by the swarm update: the same results, bit for bit, as
 * n_iter alternations of fitness_eval_batch and pso_step on these arrays.
 * d_theta float64 [R*P][4] holds the current points on entry (those pso_init
 * or the previous pso_step / pso_run wrote) and the next points on return;
 * d_seg int32 [R*P] the segment of every particle; d_fitness float64 [R*P]
 * and d_argmax int32 [R*P] receive the last iteration's fitness and samples.
 * An iteration takes the FFT passes and one more launch, which finalizes the
 * fitness of every run's points, moves the swarm and sets up the next
 * points (one work-group per run, for n_particles <= 128; larger runs take
 * the separate kernels).  FCAS_ECAPACITY if R*P > max_batch.  Asynchronous;
 * capturable (the iteration count lives on the device); no timing events. */
int pso_run(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, int32_t n_iter, double* d_theta,
            const int32_t* d_seg, double* d_fitness, int32_t* d_argmax, void* hip_stream);

/* Best of the M independent runs (Sec. III): d_out_f float64 [1] (the
 * coherent search statistic squared), d_out_theta float64 [4], d_out_j int32
 * [1] (coalescence sample), d_out_run int32 [1] (lowest run on ties). */
int pso_best(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s,
             double* d_out_f, double* d_out_theta, int32_t* d_out_j, int32_t* d_out_run,
             void* hip_stream);

/* Best of the runs of each segment (Sec. III) when one swarm searches several
 * segments: runs g*runs_per_segment .. (g+1)*runs_per_segment - 1 belong to
 * segment g, for g = 0 .. n_runs/runs_per_segment - 1, and the best is taken
 * over the first runs_used of them (runs_used = runs_per_segment: all; fewer
 * give the statistic of a search with fewer runs, as the tuning metric of
 * Sec. III compares).  Per segment g: d_out_f[g] float64 (its coherent search
 * statistic squared), d_out_theta[g] float64 [4] (rectangle coordinates),
 * d_out_j[g] int32 (coalescence sample), d_out_run[g] int32 (index of the best
 * run in the swarm, the lowest on ties).  FCAS_EINVAL unless
 * runs_per_segment >= 1 divides n_runs and 1 <= runs_used <= runs_per_segment.
 * Asynchronous; capturable. */
int pso_best_segments(fcas_ctx* ctx, const fcas_pso_params* p, const fcas_pso_state* s, int32_t runs_per_segment,
                      int32_t runs_used, double* d_out_f, double* d_out_theta, int32_t* d_out_j, int32_t* d_out_run,
                      void* hip_stream);

/* Synthetic input (the signal model of Sec. II eq. detresponse with the SPA
 * polarisations of Sec. II.B): adds to d_xf (complex128 [n_det][N/2+1], raw
 * one-sided Fourier data in continuum units, read and written) the response
 *   h^i_k = [F+^i A+ - i Fx^i Ax] f_k^-7/6 exp(-2 pi i [Phi_k + f_k (t_c + Delta^i)]) e^{i (phi_c + pi/4)}
 * on the in-band bins, with A+ = (1 + cos^2 iota)/2, Ax = cos iota, and the
 * whole response scaled so that the network SNR (eq. optimalSNR, PSD d_psd
 * float64 [n_det][N/2+1]) equals `snr` (snr = 0: unit amplitudes).
 * params float64 [8] (host): alpha, delta, tau0, tau1.5, psi, phi_c, cos_iota,
 * t_c in seconds (coalescence at the Earth's centre).  Asynchronous. */
int fcas_inject(fcas_ctx* ctx, int64_t n_samples, const double* params, double snr, const double* d_psd,
                double* d_xf, void* hip_stream);

/* Synchronises the device and returns the context's device error flags
 * (bit 0: an unregistered segment id was evaluated; bit 1: a wait of the fused
 * schedule exceeded its bound, results of that call are not valid), then
 * clears them. */
int fcas_device_error(fcas_ctx* ctx, int32_t* flags_out);

/* Synchronises and returns the number of parameter points evaluated by
 * this context since its creation (points inside the search rectangle with a
 * registered segment; points that left the rectangle are not evaluated). */
int fcas_evaluated(fcas_ctx* ctx, uint64_t* count_out);

/* Enables (1) or disables (0) per-kernel timing with HIP events recorded on
 * the caller's stream around the FFT kernels of fitness_eval_batch. */
int fcas_set_timing(fcas_ctx* ctx, int enable);

/* Synchronises and returns the summed duration (ms) and launch count of the
 * FFT kernel named `which` ("pass1", "pass2" of the two-pass schedule,
 * "passm" for the middle pass of three-pass plans, "fused" of the fused
 * schedule) since timing was enabled; resets the counters. */
int fcas_read_timing(fcas_ctx* ctx, const char* which, double* total_ms, int64_t* launches);

/* Message of the last failure on the calling thread ("" if none). */
const char* fcas_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FCAS_H */
