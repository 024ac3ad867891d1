/*
 * enuf.h -- C ABI of the MI355X (gfx950) ENUF electrostatics library.
 *
 * ENUF (Ewald summation with the non-uniform FFT, Wang, Laaksonen & Lu,
 * Sec. 3) evaluates the electrostatic energy and per-particle forces of N
 * point or Slater-smeared charges in a periodic cubic box of edge L:
 *
 *   E = E_real + E_recip + E_self                                   (eq. 16)
 *   E_real  = sum_{i<j, r<r_cut} q_i q_j [erfc(alpha r) - (1 + r/lambda) e^{-2r/lambda}] / r
 *             (eq. 31 plus the Slater correction of eq. 27, additive reading)
 *   E_recip = 1/(2 pi L) sum_{0<|k|<Kc} exp(-pi^2 k^2/(alpha L)^2)/k^2 |S(k)|^2   (eq. 18)
 *   S(k)    = sum_j q_j exp(-2 pi i k . r_j / L)                    (eq. 19)
 *   E_self  = -(alpha/sqrt(pi)) sum_j q_j^2                        (eq. 16)
 *
 * S(k) is approximated by the transposed NFFT (eq. 14): the charges are
 * spread onto an M^3 mesh with a window of half-width p mesh cells, the mesh
 * is Fourier transformed and deconvolved.  Forces are the exact gradient of
 * that approximate energy through the window (an inverse FFT of the
 * influence-weighted spectrum, gathered with the window gradient) plus the
 * exact gradient of E_real.  The Coulomb prefactor 1/(4 pi eps0 epsr) is 1.
 *
 * Conventions shared by every entry point below:
 *  - Pointers named pos, q, forces, energy are DEVICE pointers on the device
 *    that was current when the plan was created.  Work is only enqueued on
 *    the plan's stream (default: the null stream); the call returns before
 *    it completes, and the caller keeps the buffers alive until then.
 *  - Return values are ENUF_* status codes; a NULL plan from a *_create call
 *    means failure.  enuf_last_error() then holds a message (per thread).
 *  - A plan is not thread safe.  Different plans may be used concurrently.
 */
#ifndef ENUF_H
#define ENUF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define ENUF_OK            0
#define ENUF_EINVAL       -1   /* invalid argument (detected on the host, synchronously) */
#define ENUF_ENOMEM       -2   /* device allocation failed */
#define ENUF_EDEVICE      -3   /* a HIP runtime call failed */
#define ENUF_ENONNEUTRAL  -4   /* |sum q| > 1e-10 sum |q| (the method assumes neutrality, Sec. 3.1) */
#define ENUF_ENONFINITE   -5   /* a position or charge is NaN or infinite */
#define ENUF_EBUSY        -6   /* resource limit reached (serving / batching) */
#define ENUF_ECOINCIDENT  -7   /* two point charges (lambda = 0) at the same position */
#define ENUF_EOVERFLOW    -8   /* a cell held more charges than its capacity, or a
                                  fixed-point accumulator left its range */

/* Precision modes. */
#define ENUF_FP64   0   /* every stage in FP64 */
#define ENUF_MIXED  1   /* spread, FFT and gather in FP32; influence coefficients,
                           energy reduction and the real-space term in FP64 */

/* Window functions of the NFFT. */
#define ENUF_WINDOW_KB     0   /* Kaiser-Bessel (default) */
#define ENUF_WINDOW_GAUSS  1   /* Gaussian, the window named in Sec. 4 */

typedef struct enuf_plan enuf_plan;

/*
 * Create a plan for N particles (charged or not) in a cubic box of edge `box`.
 *   alpha  : Ewald splitting parameter (> 0), eq. 16.
 *   p      : window half-width in mesh cells; 2p points per axis (1 <= p <= 15, 2p <= M/2).
 *   sigma  : oversampling factor sigma_s >= 1 (Sec. 3.3); enters the Kaiser-Bessel
 *            shape b = pi (2 - 1/sigma) and the Gaussian width.
 *   M      : FFT mesh points per side; even and of the form 2^a 3^b 5^c.
 *   Kc     : reciprocal cutoff; integer wave vectors with 0 < |k| < Kc are summed
 *            (1 <= Kc <= M/(2 sigma)).
 *   r_cut  : real-space cutoff, 0 < r_cut <= box/2 (minimum image).
 *   lambda : Slater decay length lambda_e of eq. 26 (>= 0); 0 means point charges.
 * Allocates all device scratch on the current device.  Returns NULL on error.
 * The mesh passes keep one x-plane in LDS; a plane too large for it (FP64 beyond
 * M = 96 with Kc = M/4) is processed in chunks of mesh rows.  The environment
 * variable ENUF_MAX_LDS_BYTES, read here, lowers the LDS budget per block below
 * the device's (tuning and testing of the chunked passes).
 */
enuf_plan *enuf_plan_create(int64_t N, double box, double alpha, int p, double sigma,
                            int M, int Kc, double r_cut, double lambda);

/*
 * Work-groups per mesh plane in the spread and gather passes (1 .. the value
 * the plan was created with).  Each work-group takes the plane's charges with
 * compact index j = part (mod parts), spreads them into its own plane and
 * transforms it; the partial spectra are rounded to fixed point and summed
 * exactly, so results are reproducible for a given number of parts (and
 * differ between part counts only in the last bits).  The default spreads
 * one system's mesh passes over about half the device, leaving the rest to
 * the pair and real-space kernels that run beside them: parts = min(8, 128 / M)
 * (ENUF_MESH_PARTS, read at plan creation, overrides it).  The gather pass
 * takes as many work-groups per plane (ENUF_BWD_PARTS overrides it at plan
 * creation; this call sets both).  The x pass takes min(Kc, 64 / (2 Kc - 1))
 * work-groups per ky row (ENUF_X_SPLIT overrides it).  Systems stepped
 * together in a batch already fill the device: 1 part per plane avoids the
 * repeated transforms there.
 * A batch reads the value when its membership changes.  Synchronises the
 * plan's stream.  ENUF_EINVAL outside the allowed range.
 */
int enuf_plan_set_parts(enuf_plan *plan, int parts);

/* Overlap the real-space term (Sec. 4, eq. 31-32, on an internal stream)
 * with the mesh passes of the reciprocal sum (Sec. 3.3, eq. 14-25) in
 * enuf_compute and enuf_compute_components (enable = 1, the default), or run
 * the whole evaluation on the plan's stream (0).  The evaluation is serial
 * anyway while the plan's stream is being captured into a graph or a kernel
 * is being timed.  Results are the same either way.  Synchronises the plan's
 * stream; ENUF_EINVAL for a NULL plan. */
int enuf_plan_set_concurrency(enuf_plan *plan, int enable);

/* Release the plan and its device memory.  Synchronises the plan's stream.  NULL is a no-op. */
void enuf_destroy(enuf_plan *plan);

/* Message describing the last failure on the calling thread ("" if none). */
const char *enuf_last_error(void);

/* Bind the plan to a HIP stream (a hipStream_t passed as void*; NULL = null stream). */
int enuf_plan_set_stream(enuf_plan *plan, void *hip_stream);

/* Choose the precision mode (ENUF_FP64 / ENUF_MIXED) and window (ENUF_WINDOW_*). */
int enuf_plan_set_options(enuf_plan *plan, int precision, int window);

/* Forces of the reciprocal sum.
 *   ENUF_FORCE_GRADIENT (default): the exact gradient of the NFFT energy -- one
 *     inverse transform, gathered with the window's gradient.
 *   ENUF_FORCE_IK: ik-differentiation (eq. 24-25) -- the three fields i k_t h
 *     transformed back and gathered with the window; conserves total momentum
 *     to rounding.  energy5[4] (the gathered-potential check) is 0 in this mode.
 * Returns ENUF_EINVAL if the mesh does not fit the LDS in this mode. */
#define ENUF_FORCE_GRADIENT 0
#define ENUF_FORCE_IK       1
int enuf_plan_set_force_mode(enuf_plan *plan, int mode);

/*
 * Energy and forces (eq. 16, 18, 22-25, 27, 31).
 *   pos    : N x 3 row-major FP64 positions; any real values, wrapped into [0, box)
 *            internally and never modified.
 *   q      : N FP64 charges; zero marks a neutral particle.
 *   forces : N x 3 FP64, OVERWRITTEN with the force on each particle (0 for neutral ones).
 *   energy : one FP64, overwritten with the total energy.
 * Data-dependent failures (non-neutral charges, non-finite input, coincident point
 * charges, cell overflow) are recorded in the plan's sticky status word; read it
 * with enuf_plan_status.
 */
int enuf_compute(enuf_plan *plan, const double *pos, const double *q,
                 double *forces, double *energy);

/*
 * As enuf_compute, with the energy split into five FP64 values:
 *   energy5[0] = E_real   (whole short-range sum: erfc term + Slater correction)
 *   energy5[1] = E_slater (the Slater part of E_real; diagnostic)
 *   energy5[2] = E_recip  (k-space sum of the NFFT approximation)
 *   energy5[3] = E_self
 *   energy5[4] = E_recip recomputed from the gathered potential (Parseval check)
 * and the total E = energy5[0] + energy5[2] + energy5[3].
 */
int enuf_compute_components(enuf_plan *plan, const double *pos, const double *q,
                            double *forces, double *energy5);

/*
 * enuf_compute_components without a plan and without allocating device memory,
 * for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The arguments are those of
 * enuf_plan_create (Kaiser-Bessel window, window-gradient forces, the default
 * work-groups per plane) plus:
 *   precision : ENUF_FP64 or ENUF_MIXED.
 *   pos, q, forces, energy5 : as for enuf_compute_components (DEVICE pointers on
 *            the current device).
 *   status   : DEVICE pointer to one int, or NULL; receives the evaluation's
 *            data-dependent status (ENUF_OK, ENUF_ENONNEUTRAL, ...).
 *   hip_stream : stream the work is enqueued on (NULL = null stream).
 * The buffers of the evaluation live in one fixed device array of
 * ENUF_NOALLOC_SCRATCH_BYTES per device, held from the library's first use of
 * a device until the process ends; tables reach the device as kernel
 * arguments.  Sizes whose buffers exceed that array, or M > 256, return
 * ENUF_EINVAL (the message gives the bytes needed).  The call issues no
 * hipMalloc, hipFree or hipMemset: every launch is a kernel.  All calls on one
 * device share the array, and each call starts by clearing what it needs, so
 * calls that overlap on one device (two streams, or two threads) race: order
 * them on one stream.  Enqueue-only; the results equal enuf_compute_components
 * on a plan of the same parameters and precision.
 */
#define ENUF_NOALLOC_SCRATCH_BYTES (64u << 20)
int enuf_compute_noalloc(int64_t N, double box, double alpha, int p, double sigma, int M, int Kc,
                         double r_cut, double lambda, int precision, const double *pos, const double *q,
                         double *forces, double *energy5, int *status, void *hip_stream);

/* Synchronise the plan's stream and return the sticky status word in *status
 * (ENUF_OK or the first data-dependent error since the last call); clears it. */
int enuf_plan_status(enuf_plan *plan, int *status);

/* Device bytes held by the plan (for admission control). 0 for NULL. */
size_t enuf_plan_footprint_bytes(const enuf_plan *plan);

/* ------------------------------------------------------------------------
 * DPD trajectories with ENUF electrostatics (Sec. 2 and Table 2).
 *
 * Reduced units R_c = m = k_B T = 1.  Pair forces act for r < 1 (eq. 2-7):
 *   F^C = a (1 - r) rhat,  F^D = -gamma (1 - r)^2 (v_ij . rhat) rhat,
 *   F^R = sigma (1 - r) theta_ij rhat / sqrt(dt),
 * theta_ij uniform on [-sqrt 3, sqrt 3) from Philox4x32-10 with counter
 * (min(i,j), max(i,j), step low word, step high word) and key (seed low word,
 * seed high word), 53 bits from the first two output words; harmonic bonds
 * F = -K (r - r_eq) rhat; electrostatics kappa times the ENUF force.
 * One step is Table 2: v0 = v + lam dt F; v += dt F/2; r += dt v (wrapped
 * into [0, box)); F = F(r, v0); v += dt F/2.
 * ------------------------------------------------------------------------ */
typedef struct enuf_dpd enuf_dpd;

typedef struct {
  double a;        /* conservative amplitude a_ij (one species), eq. 3 */
  double gamma;    /* dissipation strength, eq. 4 */
  double sigma;    /* noise amplitude, eq. 5 (sigma^2 = 2 gamma k_B T, eq. 6) */
  double dt;       /* time step (> 0) */
  double lam;      /* velocity prediction parameter of the modified velocity Verlet */
  double k_bond;   /* spring constant K^S */
  double r0_bond;  /* bond rest length r_eq */
  double kappa;    /* coupling that multiplies the ENUF energy and forces */
  uint64_t seed;   /* random-force stream */
} enuf_dpd_params;

/*
 * Create a DPD integrator for N particles in a cubic box (box >= 2).
 *   plan   : ENUF plan for the same N and box, or NULL for no electrostatics.
 *            Not owned; it must outlive the integrator.
 *   q      : DEVICE pointer to N charges, copied at creation (charges are fixed).
 *   bonds  : HOST pointer to nbonds (i, j) index pairs (int64), copied.
 * The cell grid has floor(box) cells per side and
 * ceil(m + 6 sqrt(m) + 16) slots per cell (m = N / cells); creation fails if
 * that exceeds 128 (about 70 particles per unit volume).
 * Returns NULL on error (enuf_last_error).  Allocates device scratch.
 */
enuf_dpd *enuf_dpd_create(int64_t N, double box, const enuf_dpd_params *params, enuf_plan *plan,
                          const double *q, int64_t nbonds, const int64_t *bonds);

/* Bind the integrator (and its ENUF plan) to a HIP stream; NULL = null stream. */
int enuf_dpd_set_stream(enuf_dpd *dpd, void *hip_stream);

/* Total force at pos with the velocities vel standing in for the predicted
 * ones and the random numbers of `step` (device pointers, N x 3 FP64).
 * force is overwritten.  pos is wrapped into the box in place. */
int enuf_dpd_forces(enuf_dpd *dpd, double *pos, const double *vel, double *force, uint64_t step);

/* Advance nsteps steps in place.  On entry force holds the force of the last
 * step (from enuf_dpd_forces or a previous run); step s uses the random
 * numbers of step s, s = first_step .. first_step + nsteps - 1.  Within a
 * run, each step's closing kernel also starts the next step (one launch), and
 * all but the last step are replayed from graphs of 8 and of 2 steps
 * (enuf_dpd_set_graphs; at most one of them is launched eagerly); the ENUF
 * energies are reduced on the last step only.  Enqueue-only, except that a
 * graph missing for these buffers is first captured, which synchronises the
 * integrator's stream (enuf_dpd_prepare_graphs captures them ahead). */
int enuf_dpd_run(enuf_dpd *dpd, double *pos, double *vel, double *force, uint64_t first_step,
                 int nsteps);

/* Capture, for these state buffers, every graph enuf_dpd_run replays (8- and
 * 2-step graphs, for runs starting on even and on odd steps), so that later
 * runs on these buffers launch without capturing.  Launches no step.
 * Synchronises the integrator's stream.  ENUF_OK without doing anything when
 * graphs are disabled; ENUF_EDEVICE if capture fails. */
int enuf_dpd_prepare_graphs(enuf_dpd *dpd, double *pos, double *vel, double *force);

/* Species-dependent conservative amplitudes (eq. 3; Sec. 2 sets
 * a_ij = a_ii + 2.05 chi_ij between species).
 *   nspecies : 1..4.  With 1, a_table[0] replaces params->a for every pair.
 *   species  : HOST pointer to N ints in [0, nspecies), copied (ignored when
 *              nspecies = 1).
 *   a_table  : HOST pointer to the nspecies x nspecies row-major amplitudes;
 *              must be symmetric (a_ij = a_ji keeps the pair force antisymmetric).
 * The dissipative and random forces keep one gamma and sigma.  Synchronises
 * the integrator's stream.  ENUF_EINVAL if the integrator is a member of a
 * batch (set the species before enuf_batch_add), or on a bad argument. */
int enuf_dpd_set_species(enuf_dpd *dpd, int nspecies, const int *species, const double *a_table);

/* Overlap the pair forces and the real-space term (one after the other, on an
 * internal stream) with the mesh passes on the integrator's stream
 * (enable = 1, the default), or run the whole step on the integrator's
 * stream (0).  Results are the same either way. */
int enuf_dpd_set_concurrency(enuf_dpd *dpd, int enable);

/* Launch the steps of enuf_dpd_run (all but its last) as HIP graphs of 8
 * and 2 steps (enable = 1, the default), captured on the first run with given
 * pos / vel / force buffers and captured again when they or the parameters
 * change; the fork and join of the concurrent schedule are graph edges.  With
 * 0, or while a kernel is being timed, every step is launched eagerly.
 * Results are the same either way (the step index of a replayed step is read
 * from device memory).  Synchronises the integrator's stream. */
int enuf_dpd_set_graphs(enuf_dpd *dpd, int enable);

/* Copy (on the stream) the ENUF energy components of the last force
 * evaluation, unscaled by kappa, into the device array energy5 (as in
 * enuf_compute_components).  Without a plan all five are 0. */
int enuf_dpd_energy(enuf_dpd *dpd, double *energy5);

/* Synchronise and return (and clear) the sticky status of the integrator and
 * of its plan (ENUF_EOVERFLOW if a DPD cell overflowed). */
int enuf_dpd_status(enuf_dpd *dpd, int *status);

/* Release the integrator (not its plan).  NULL is a no-op. */
void enuf_dpd_destroy(enuf_dpd *dpd);

/* Device bytes held by the integrator and its plan (admission control). */
size_t enuf_dpd_footprint_bytes(const enuf_dpd *dpd);

/* Device bytes enuf_plan_create (on the current device) and enuf_dpd_create
 * would allocate for these sizes, without allocating: admission control
 * before a system is created.  0 for invalid sizes. */
size_t enuf_plan_footprint_estimate(int64_t N, double box, int p, int M, int Kc, double r_cut);
size_t enuf_dpd_footprint_estimate(int64_t N, double box, int64_t nbonds);

/* ------------------------------------------------------------------------
 * Batched DPD steps: many independent systems (each an integrator with its
 * own plan, N, box, M, Kc, charges and parameters) advanced together, one
 * kernel launch per stage of the step for all members, the step captured
 * once in a HIP graph and replayed.  A member's trajectory is bitwise the one
 * enuf_dpd_run gives it alone (same kernels, same per-system arithmetic, and
 * the same enuf_plan_set_parts setting).
 * ------------------------------------------------------------------------ */
typedef struct enuf_batch enuf_batch;

/* Create an empty batch on the current device for members of one precision
 * (ENUF_FP64 / ENUF_MIXED).  NULL on error. */
enuf_batch *enuf_batch_create(int precision);

/* Release the batch (synchronises; members are not destroyed).  NULL is a no-op. */
void enuf_batch_destroy(enuf_batch *batch);

/* The caller's stream (NULL = null stream): a run is ordered after the work
 * already queued on it and before work queued on it later.  Members use it as
 * their stream while they belong to the batch.  Binding the stream the batch
 * already uses does nothing; another stream first synchronises the batch's
 * work and drops its captured graph. */
int enuf_batch_set_stream(enuf_batch *batch, void *hip_stream);

/* use_graph: replay one captured step (1, default), launch eagerly (0), or
 * ENUF_GRAPH_AUTO: capture only for a run of at least ENUF_GRAPH_AUTO_STEPS
 * steps and replay the graph while the membership stays the same, launching
 * shorter runs of a new membership eagerly (a capture costs milliseconds,
 * more than the few steps between membership changes of a serving stream).
 * concurrent: in eager launches, fork the pair forces and real space onto
 * side streams (1, default) or keep the step on one stream (0).  The captured
 * step always uses the single-stream schedule.  Results do not depend on
 * either option.  Other values of use_graph return ENUF_EINVAL. */
#define ENUF_GRAPH_AUTO        2
#define ENUF_GRAPH_AUTO_STEPS 16
int enuf_batch_set_options(enuf_batch *batch, int use_graph, int concurrent);

/* Launch parameters of the batched step; none of them changes any result bit
 * (fixed-point sums, per-line k-space energies), only the time a step takes.
 *   pass_threads: work-group size of the spread and gather passes, 256
 *                 (default) or 512;
 *   x_threads:    of the x pass, 128 (default), 256 or 512 (both are raised
 *                 when a member's FFT has more butterflies per line);
 *   stage:        most charges a mesh work-group stages in LDS at a time,
 *                 32..512 (default 256; never more than the member's plan
 *                 chose for its LDS budget);
 *   pair_steps:   candidate steps in flight per lane of the pair kernel, 4
 *                 (default) or 8;
 *   x_split_mul:  x-pass work-groups per ky row, the plan's times this, 1..8
 *                 (default 1; at most Kc);
 *   pair_seg:     cells per column segment of the pair kernel, about, 1..26
 *                 (default 26; a system stepped alone uses 10).
 * 0 keeps a value.  Takes effect at the next run (the graph is re-captured).
 * ENUF_EINVAL (nothing changed) for values out of range. */
int enuf_batch_set_tuning(enuf_batch *batch, int pass_threads, int x_threads, int stage, int pair_steps,
                          int x_split_mul, int pair_seg);

/*
 * Add an integrator (with a plan of the batch's precision) and its state:
 * device arrays pos, vel, force of N x 3 FP64, owned by the caller and kept
 * alive while the member belongs to the batch.  force must hold the force of
 * the current state (enuf_dpd_forces or an earlier run); the member's next
 * step uses the random numbers of step first_step.  Returns a member id >= 0,
 * or a negative ENUF_* code.
 */
int enuf_batch_add(enuf_batch *batch, enuf_dpd *dpd, double *pos, double *vel, double *force,
                   uint64_t first_step);

/* Remove a member (synchronises the batch's work first). */
int enuf_batch_remove(enuf_batch *batch, int member_id);

/* Number of members. */
int enuf_batch_size(const enuf_batch *batch);

/* Advance every member nsteps steps (enqueue-only).  Replayed runs (graphs)
 * fuse each step's combine with the next step's pre kernel and reduce the
 * energies (enuf_dpd_energy) of the last step only; results are bitwise those
 * of eager runs. */
int enuf_batch_run(enuf_batch *batch, int nsteps);

/* Device bytes of the batch's tables and of all members (with their plans). */
size_t enuf_batch_footprint_bytes(const enuf_batch *batch);



/* ------------------------------------------------------------------------
 * Kernel timing (measurement support).  While enabled, an integrator records
 * a pair of HIP events on its stream around each launch of one kernel of the
 * step, for at most max_launches launches; enuf_dpd_kernel_time synchronises
 * and returns the summed milliseconds and the number of timed launches.
 * ------------------------------------------------------------------------ */
#define ENUF_K_DPD_PRE       0
#define ENUF_K_DPD_PAIR      1
#define ENUF_K_PREP_COUNT    2
#define ENUF_K_PREP_COMPACT  3
#define ENUF_K_REAL          4
#define ENUF_K_MESH_FWD      5   /* spread + z/y FFT per x-plane */
#define ENUF_K_MESH_X        6   /* x FFT + influence multiply + inverse x FFT */
#define ENUF_K_MESH_BWD      7   /* inverse y/z FFT + gather per x-plane */
#define ENUF_K_COMBINE       8
#define ENUF_K_DPD_POST      9

/* kernel = ENUF_K_* to start timing it (resets the totals), -1 to stop. */
int enuf_dpd_time_kernel(enuf_dpd *dpd, int kernel, int max_launches);
int enuf_dpd_kernel_time(enuf_dpd *dpd, double *total_ms, int *launches);

/* The same for the kernels of enuf_compute / enuf_compute_components on a
 * plan (ENUF_K_PREP_COUNT ... ENUF_K_COMBINE). */
int enuf_plan_time_kernel(enuf_plan *plan, int kernel, int max_launches);
int enuf_plan_kernel_time(enuf_plan *plan, double *total_ms, int *launches);

/* The same for one stage of a batch's step (ENUF_K_DPD_PRE, _DPD_PAIR, _REAL,
 * _MESH_FWD, _MESH_X, _MESH_BWD, _COMBINE; each is one launch for all members).
 * While timing is on, enuf_batch_run launches every step eagerly on one
 * stream, without its graph. */
int enuf_batch_time_kernel(enuf_batch *batch, int kernel, int max_launches);
int enuf_batch_kernel_time(enuf_batch *batch, double *total_ms, int *launches);

/* ------------------------------------------------------------------------
 * Structure observables, sampled on the device between steps (enqueued on
 * hip_stream; NULL = null stream).  All pointers are DEVICE pointers.
 * ------------------------------------------------------------------------ */

/*
 * Pair-distance histogram by class, the counts behind the radial distribution
 * functions g_ab(r) of Sec. 5.  Every unordered pair {sel[a], sel[b]}, a < b,
 * of the nsel selected particles is counted once, at its minimum-image distance
 * r in the cubic box, into
 *     hist[(c_lo * ncls + c_hi) * nbins + k],  c_lo = min(cls[a], cls[b]), c_hi = max,
 * for the bin k with (k w)^2 <= r^2 < ((k + 1) w)^2, w = r_max / nbins; pairs
 * beyond the last edge are not counted.  hist (ncls * ncls * nbins uint64) is
 * accumulated, not cleared, so that successive samples add up.  The bin is
 * decided in FP64 on r^2 against the squared edges, without fused
 * multiply-adds, so the counts are those of a plain IEEE evaluation.
 *   pos  : N x 3 FP64 positions; sel: nsel int64 indices; cls: nsel int32 classes.
 * Entries with an index outside [0, n) or a class outside [0, ncls) are skipped.
 * ENUF_EINVAL: ncls * ncls * nbins > 12288, nsel > 65535 * 256, box or r_max
 * not finite and positive, NULL buffers.  Normalisation to g(r) is the
 * caller's: g_ab = counts / (pairs_ab * shell volume / box^3 * samples).
 */
int enuf_pair_histogram(const double *pos, int64_t n, int64_t nsel, const int64_t *sel, const int *cls, int ncls,
                        double box, double r_max, int nbins, unsigned long long *hist, void *hip_stream);

/*
 * Squared radius of gyration of nchains chains of len beads (Sec. 6).  Chain c
 * is beads[c * len .. c * len + len - 1] (int64) in bond order; it is unwrapped
 * by the minimum image of each bond vector (bonds shorter than box / 2), and
 * out[c] = (1/len) sum_k |u_k - u_cm|^2 with u_cm the mean unwrapped position.
 * A chain with a bead index outside [0, n) gets NaN.  Write to out + s * nchains
 * to keep sample s of a trajectory on the device.
 */
int enuf_chain_rg2(const double *pos, int64_t n, int nchains, int len, const int64_t *beads, double box, double *out,
                   void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ENUF_H */
