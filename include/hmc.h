/*
 * libhmc -- HMC density sampler of Jasche & Wandelt (2013), "Methods for
 * Bayesian power spectrum inference with galaxy surveys", on AMD MI355X.
 *
 * The library samples the joint posterior P(delta, S, {Nbar^l}, {b^l} | {N^l_i})
 * of Sec. "The joint posterior distribution" with the block scheme of
 * eq. multiblock: an HMC step for the density field (Sec. "The HMC algorithm",
 * Sec. "Equations of motion for the Wiener Posterior"), the inverse-Gamma
 * power-spectrum draw (eq. INVERSE_GAMMA via eq. XI_SQUARE), the GIG draw for
 * Nbar (eq. GIG_post), the normal draw for the biases (Appendix B) and the
 * joint (P, delta) move of Appendix C (eq. det_trans, eq.
 * spec_posterior_MIXING_1).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Grid: N^3 voxels, N in {8, 16, 32, 64, 128, 192, 256}; real fields are
 *    float32 row-major [x][y][z] (z fastest).
 *  - Fourier fields are complex64 (interleaved re, im floats), layout
 *    [kx][ky][kz] with kz in [0, N/2]: N * N * (N/2+1) complex values.  The DFT
 *    is the Appendix "Discrete Fourier transformation" convention with the
 *    unitary normalisation C = C_hat = N^(-3/2); kx, ky map to signed
 *    frequencies -(N/2-1)..N/2.
 *  - k-shells: n_bins linear shells over (0, sqrt(3) (N/2) 2 pi / L]; with
 *    q = kx^2 + ky^2 + kz^2 (signed integer frequencies) and q_max = 3 (N/2)^2,
 *    mode q >= 1 is in the shell m with m^2 q_max < n_bins^2 q <= (m+1)^2 q_max.
 *    The mean mode k = 0 is in no shell and is held at zero.
 *  - Power spectrum values P_m are in (Mpc/h)^3; the prior eigenvalue is
 *    lambda_m = P_m N^3 / L^3.
 *  - Ownership: the caller owns every device buffer (inputs, state, the
 *    workspace); the library owns only host-side objects inside hmc_ctx and a
 *    few small device tables it allocates at init (freed by hmc_destroy).
 *    Device pointers are plain HIP device addresses; `stream` is a hipStream_t
 *    (void* here so that the header needs no HIP include).  All device work is
 *    stream-ordered on that stream.  Calls that return host scalars
 *    synchronise the stream before returning.
 *  - Errors: every call returns hmc_status.  HMC_EINVAL: bad shape, size or
 *    null pointer; HMC_ENOMEM: workspace too small; HMC_EDEVICE: a HIP call
 *    failed; HMC_EUNSUPPORTED: a valid request the library does not implement;
 *    HMC_ENUMERIC: non-finite energy (the trajectory is rejected and the state
 *    restored).  hmc_last_error() returns a static description.  A context is
 *    not thread-safe; use one per stream.
 *  - Random numbers: Philox4x32-10 keyed by `seed`; counter =
 *    (block, draw index, chain_id << 8 | stream, sub index).  Streams: 3 HMC
 *    momenta, 4 HMC accept, 5 chi^2, 6 GIG, 7 bias, 8 joint-move momenta,
 *    9 joint-move accept.
 */
#ifndef LIBHMC_HMC_H
#define LIBHMC_HMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hmc_status;
#define HMC_OK 0
#define HMC_EINVAL (-1)
#define HMC_ENOMEM (-2)
#define HMC_EDEVICE (-3)
#define HMC_EUNSUPPORTED (-4)
#define HMC_ENUMERIC (-5)

typedef struct hmc_ctx hmc_ctx;

/* Sampler settings for one chain. */
typedef struct hmc_config {
  int32_t n;                 /* grid side N */
  double box;                /* box side L [Mpc/h] */
  int32_t n_sub;             /* number of galaxy subsamples c (1..32) */
  int32_t n_bins;            /* number of k-shells (1..128) */
  double alpha_prior;        /* power-law prior index: P^-alpha (1 = Jeffreys) */
  uint64_t seed;             /* Philox key */
  uint32_t chain_id;         /* Philox chain field (< 2^24) */
  int32_t n_leapfrog;        /* leapfrog steps per trajectory (>= 1) */
  double eps;                /* leapfrog step size */
  uint32_t fixed_bias_mask;  /* bit l set: b_l is held at its current value */
  int32_t rj_move;           /* 1: run the joint (P, delta) move in gibbs_sweep */
  double rj_log_bound;       /* joint move keeps ln lambda within +-bound of its
                                value at init (reflecting walls); 0 -> 10 */
  int32_t tau_mode;          /* 0: every trajectory runs n_leapfrog steps; 1: the
                                pseudo-time is drawn uniformly (Sec. "The HMC
                                algorithm"): n ~ U{1..n_leapfrog} per trajectory /
                                sweep from Philox stream 10 of the first chain at
                                the trajectory / sweep index, shared by all chains
                                of a context and by the joint move of that sweep */
} hmc_config;

/* Caller-owned device buffers of one chain.  R and counts are read at init (the
   survey support, i.e. the voxels with some R^l > 0, and the static sums of the
   Nbar conditional) and by every sweep: their contents must not change after
   hmc_init. */
typedef struct hmc_buffers {
  const float* R;       /* [c][N][N][N] survey response R^l_i >= 0 */
  const float* counts;  /* [c][N][N][N] galaxy counts N^l_i (0 where R = 0) */
  float* delta_k;       /* [N][N][N/2+1] complex64: density state delta_hat */
  float* mom_k;         /* [N][N][N/2+1] complex64: momentum of the last trajectory */
  float* grad_k;        /* [N][N][N/2+1] complex64: F(alpha delta - beta) at delta_hat */
  float* delta_r;       /* [N][N][N] real-space density of the state */
  float* alpha;         /* [N][N][N] sum_l b_l^2 Nbar_l R^l (library writes) */
  float* beta;          /* [N][N][N] sum_l b_l (N^l - Nbar_l R^l) (library writes) */
  void* work;           /* workspace, at least hmc_workspace_bytes(cfg) bytes */
  size_t work_bytes;
  const float* growth;  /* [N][N][N] linear growth factor D+ > 0 per voxel of the data model
                           (eq. data_model: mean counts Nbar R (1 + b D+ delta)), or NULL
                           for D+ = 1 (the paper's experiments) */
} hmc_buffers;

/* Per-sweep results; the arrays are library-owned views valid until the next
 * call on the same context. */
typedef struct hmc_sweep_stats {
  double dH;             /* energy error of the density trajectory */
  int32_t accepted;      /* 1 if the density trajectory was accepted */
  double rj_dH;          /* energy error of the joint move (0 if off) */
  int32_t rj_accepted;   /* 1 if the joint move was accepted */
  int32_t rj_wall_hits;  /* reflections of ln lambda off the joint move's walls
                            (rj_log_bound) during the move; 0 when the walls were
                            never reached */
  const double* pk;      /* [n_bins] P_m after the sweep, (Mpc/h)^3 */
  const double* bias;    /* [c] */
  const double* nbar;    /* [c] */
} hmc_sweep_stats;

/* Workspace bytes one chain needs (0 on invalid config). */
size_t hmc_workspace_bytes(const hmc_config* cfg);

/* Create a context for one chain.  Validates the configuration, binds the
 * buffers, computes the data model's static sums and alpha, beta (Sec. "The
 * density likelihood and the data model"), the shell tables and the mass of
 * the text after eq. Mass_matrix (diagonal of S^-1 + diag(alpha) in Fourier
 * space), and the real field and gradient of the initial delta_hat (which the
 * caller has written to delta_k; zeros are fine).  bias, nbar: [c] host
 * float64; pk: [n_bins] host float64 (Mpc/h)^3.  HMC_EINVAL (after the device
 * sums) if a k-shell has no modes or a subsample has no voxel with R > 0. */
hmc_status hmc_init(const hmc_config* cfg, const hmc_buffers* buf, const double* bias,
                    const double* nbar, const double* pk, void* stream, hmc_ctx** out);

/* Same for `n_chains` independent chains that advance together: every stage of
 * a trajectory or sweep is one launch over all chains.  All chains must use
 * the same n_leapfrog.  cfg, buf: [n_chains]; bias, nbar: concatenated [sum c];
 * pk: concatenated [sum n_bins]. */
hmc_status hmc_init_batch(const hmc_config* cfg, const hmc_buffers* buf, int32_t n_chains,
                          const double* bias, const double* nbar, const double* pk, void* stream,
                          hmc_ctx** out);

/* One HMC trajectory for the density (Sec. "The HMC algorithm"): momenta
 * p ~ N(0, M) drawn as p_hat = sqrt(m_k) F w, KDK leapfrog of eqs. HAMILTON1_a /
 * HAMILTON2_a with n_leapfrog steps of size eps, Metropolis test of eq.
 * acceptance_rule (accept iff ln u < -dH).  On reject delta_k, grad_k and
 * delta_r are restored; mom_k holds the final momentum of the proposal.
 * traj_index (low 32 bits) selects the Philox draws (momenta, u): a chain must
 * not repeat an index (nor use one that a gibbs_sweep used), since the same
 * momenta from a nearby state retrace part of the earlier move.
 * dH, accepted: host pointers with one entry per chain. */
hmc_status leapfrog_trajectory(hmc_ctx* ctx, uint64_t traj_index, double* dH, int32_t* accepted);

/* leapfrog_trajectory without a host round trip: dH_dev (device [n_chains]
 * float64) and accepted_dev (device [n_chains] int32) receive the results in
 * stream order; nothing is synchronised, so calls can be queued back to back or
 * captured by the caller.  A non-finite dH is rejected on the device (no
 * HMC_ENUMERIC report). */
hmc_status leapfrog_trajectory_async(hmc_ctx* ctx, uint64_t traj_index, double* dH_dev,
                                     int32_t* accepted_dev);

/* Energies of eq. Hamiltonian for chain `chain` on the current buffers
 * (float64 accumulation): out[0] kinetic 1/2 sum_k |p_hat|^2/m_k from mom_k,
 * out[1] prior 1/2 sum_k |delta_hat|^2/lambda_k from delta_k, out[2] data
 * sum_i (1/2 alpha_i delta_i^2 - beta_i delta_i) from delta_r (eq.
 * Wiener_Posterior_psi without constants).  out: host, 3 doubles. */
hmc_status hamiltonian(hmc_ctx* ctx, int32_t chain, double* out);

/* Shell power of chain `chain`: sigma_m = sum_{k in m} |delta_hat_k|^2 over the
 * full grid (the sigma_m that follows eq. INVERSE_GAMMA) and mode counts n_m.
 * sigma: host [n_bins] float64; n_modes: host [n_bins] int64 (may be NULL). */
hmc_status shell_power(hmc_ctx* ctx, int32_t chain, double* sigma, int64_t* n_modes);

/* shell_power for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sigma_m and n_m, bit for bit, of a caller's half-complex field, with no
 * context and no allocation.  delta_k: device [N][N][N/2+1] complex64 with
 * N in {8, 16, 32, 64, 128, 192, 256}; n_bins in 1..128 (shells as above);
 * sigma: device [n_bins] float64; n_modes: device [n_bins] int64 or NULL.
 * Stream-ordered on `stream`, no synchronisation.  Its per-tile partial sums
 * live in a library-owned device array of 1.06 MB (2 x 128 shells x 516 tiles
 * of float64, enough for 256^3) that each GPU holds until the process ends and
 * every call on that GPU shares: calls that overlap on one GPU (other streams,
 * other threads) race on it.  Nothing needs clearing between calls (every
 * partial the sums read is rewritten).  HMC_EINVAL on a null pointer or a size
 * beyond these limits, HMC_EDEVICE on a HIP error; hmc_last_error(NULL)
 * describes it. */
hmc_status shell_power_noalloc(int32_t n, int32_t n_bins, const float* delta_k, double* sigma,
                               int64_t* n_modes, void* stream);

/* One block sweep (eq. multiblock): density HMC, P | delta, the joint move (if
 * rj_move), Nbar | delta, b, b | delta, Nbar, then alpha, beta, mass and
 * gradient are refreshed.  sweep_index (low 32 bits) selects every Philox
 * draw of the sweep; as for trajectories, a chain must not repeat an index.
 * out: host [n_chains]. */
hmc_status gibbs_sweep(hmc_ctx* ctx, uint64_t sweep_index, hmc_sweep_stats* out);

/* Doubles of the per-sweep record gibbs_sweep_async writes, summed over chains:
 * for each chain, in order, [dH, accepted (0/1), rj_dH, rj_accepted, status
 * (0 ok, nonzero: a draw or energy was not finite), rj_wall_hits, P_m (n_bins
 * values, (Mpc/h)^3), b_l (c values), Nbar_l (c values)]. */
size_t hmc_sweep_record_doubles(const hmc_ctx* ctx);

/* gibbs_sweep without a host round trip: stats_dev (device float64,
 * hmc_sweep_record_doubles values) receives the records in stream order. */
hmc_status gibbs_sweep_async(hmc_ctx* ctx, uint64_t sweep_index, double* stats_dev);

/* Replace the density state of chain `chain` with a real field (device
 * [N][N][N] float32), e.g. a warm start; the mean is removed. */
hmc_status hmc_set_state(hmc_ctx* ctx, int32_t chain, const float* delta_r_dev);

/* Warm start from a predicted posterior mean mu and log-variance s (device
 * [N][N][N] float32 each, e.g. from cnn_forward): the state becomes
 *   delta = mu + sqrt(exp(s) / sigma^2) xi,   xi = F^-1(sqrt(lambda_k) F w),
 * w white noise from Philox stream 11 at draw index `draw_index` (low 32 bits),
 * lambda_k the chain's current prior eigenvalues (k = 0 excluded) and
 * sigma^2 = N^-3 sum_{k != 0} lambda_k the prior variance per voxel, i.e. a prior
 * draw rescaled to the predicted variance and shifted to the predicted mean.
 * Unlike the mean alone (whose power is far below P(k)), such a start keeps the
 * first P draws of a sweep near their stationary values.  Gradient, real field
 * and data energy are refreshed as by hmc_set_state.  The mass only affects
 * efficiency (text after eq. Mass_matrix) and a start near the posterior only
 * the burn-in (Sec. "Testing burn-in and statistical efficiency"). */
hmc_status hmc_warm_start(hmc_ctx* ctx, int32_t chain, const float* mu_dev,
                          const float* logvar_dev, uint64_t draw_index);

/* Launch shape of a pass class (0: k-space x passes, 1: y passes, 2: real-space
 * z passes): grid = number of persistent workgroups that walk the tiles (a
 * multiple of 8 keeps each XCD on a contiguous run of tiles), 0 for one
 * workgroup per tile (the default), or -1 for one single-size launch per grid
 * size of a mixed-size batch (one workgroup per tile each; the same as 0 when
 * every chain has one size).  Results do not depend on it. */
hmc_status hmc_set_launch(hmc_ctx* ctx, int32_t pass_class, int32_t grid);

/* Radix plan of the transforms of a pass class (0 the k-space step pass, 1 the
 * y passes, 2 the real-space force pass) in single-size launches of grids of
 * 64^3, 128^3, 192^3 and 256^3: plan 0 (default), one of two alternative
 * factorisations of the same pencil shape (plans 1, 2: same tiles, LDS and memory
 * access; different stage counts and LDS exchanges), or, at 64^3, 128^3 and
 * 256^3, another tile shape for the step and y passes (plan 3: twice the threads
 * per pencil and 512-thread workgroups at the same pencils per workgroup, so the
 * same tiles; plan 3 is plan 0 elsewhere), 0 <= plan < 4.  Other grid sizes and
 * mixed-size launches use plan 0.  The fused plane pass has one plan.  A plan changes the rounding of the
 * transforms (results agree with plan 0 to float32 rounding, not bitwise);
 * results are reproducible for a fixed plan.  Captured graphs are dropped.
 * HMC_EINVAL on a bad class or plan. */
hmc_status hmc_set_plan(hmc_ctx* ctx, int32_t pass_class, int32_t plan);

/* Fused y-z plane pass (enable = 1, the default) or separate passes (0) for
 * the gradient evaluations of grid sizes that have one (64^3 to 256^3):
 * contexts whose chains all have that size, and the size groups of a batch whose
 * y and real-space passes run one launch per size group (hmc_set_launch with
 * grid -1, the autotuner's usual choice).  The fused pass runs, per real-space x plane, the
 * inverse y transforms, the C2R z transforms, the data force of eq.
 * Wiener_Posterior_force, the R2C z transforms and the forward y transforms
 * with the plane on chip, so a leapfrog step moves 40 N^3 instead of 56 N^3
 * bytes.  Results agree with the separate passes to float32 rounding, not
 * bitwise.  Captured graphs are dropped.  HMC_EINVAL unless enable is 0 or 1. */
hmc_status hmc_set_plane_pass(hmc_ctx* ctx, int32_t enable);

/* The launch configuration in force: grid[3] in the form hmc_set_launch takes,
 * plan[3] as hmc_set_plan (host arrays, either may be NULL). */
hmc_status hmc_get_launch(hmc_ctx* ctx, int32_t* grid, int32_t* plan);

/* Autotuner of the launch shapes: for each pass class, times `reps` launches of
 * each candidate (for mixed-size batches one launch per size group, then one
 * launch over the batch with one workgroup per tile or 2, 3, 4, 5, 6, 8, 12
 * workgroups per compute unit) on the context's chains with HIP events and keeps
 * the fastest (in a batch with a size group that has a fused plane pass, the y
 * and real-space classes keep one launch per size group, which the plane pass
 * needs), then, when the chosen launches are single-size and a grid size has
 * alternative plans, times plans 1 to 3 at that grid and keeps the fastest of
 * the four (hmc_set_plan: a plan other than 0 changes rounding); chosen
 * (host [3], may be NULL) receives the grids in the form hmc_set_launch takes
 * (hmc_get_launch also returns the plans).  The state (delta_hat, p_hat, the
 * parameters) is unchanged; captured graphs are dropped. */
hmc_status hmc_autotune(hmc_ctx* ctx, int32_t reps, int32_t* chosen);

/* Change the leapfrog step size eps of chain `chain` (the same eps also steps
 * the joint (P, delta) move).  Takes effect from the next trajectory or sweep,
 * also for captured graphs.  HMC_EINVAL unless eps is positive and finite. */
hmc_status hmc_set_step(hmc_ctx* ctx, int32_t chain, double eps);

/* Replace P (host [n_bins], (Mpc/h)^3), biases and Nbar (host [c]) of a chain;
 * NULL leaves a block unchanged.  Refreshes alpha, beta, mass and gradient. */
hmc_status hmc_set_params(hmc_ctx* ctx, int32_t chain, const double* pk, const double* bias,
                          const double* nbar);

/* Install caller-computed coefficients alpha, beta (device [N][N][N] float32,
 * the two real fields of eq. Wiener_Posterior_force) for chain `chain`, in
 * place of the ones the library derives from R, counts, b and Nbar; the mean
 * of alpha, the mass and the gradient are refreshed from them.  They stay in
 * force until the next gibbs_sweep or hmc_set_params recomputes them. */
hmc_status hmc_set_coefficients(hmc_ctx* ctx, int32_t chain, const float* alpha_dev,
                                const float* beta_dev);

/* Current P, b, Nbar of a chain (host arrays; NULL skips). */
hmc_status hmc_get_params(hmc_ctx* ctx, int32_t chain, double* pk, double* bias, double* nbar);

/* Shell index of every stored mode of chain `chain` (device [N][N][N/2+1]
 * int16, -1 for k = 0), as the kernels compute it. */
hmc_status hmc_shell_index(hmc_ctx* ctx, int32_t chain, int16_t* out_dev);

/* Learned mass (the mass affects only efficiency, text after eq. Mass_matrix):
 * with logvar_dev a device [N][N][N] float32 log-variance s and
 * D = exp(s) / mean(exp(s)), the inverse mass on the zero-mean field becomes
 * T T^T with T = P D^(1/2) F^-1 diag(m_k^-1/2), P the mean projector, i.e.
 * P D^(1/2) F^-1 diag(1/m_k) F D^(1/2) P; D = 1 is the paper's Fourier-diagonal
 * mass.  A step then costs two more real transforms.  NULL restores the plain
 * mass.  chain = -1 applies the field to every chain (all of one grid size).
 * Every chain of a context must use the same kind of mass: while only some
 * have a learned one, leapfrog_trajectory and gibbs_sweep return
 * HMC_EUNSUPPORTED and do nothing. */
hmc_status hmc_set_mass(hmc_ctx* ctx, int32_t chain, const float* logvar_dev);

/* Posterior field moments (streaming): fold the chain's current real-space
 * state delta_r into per-voxel running moments with Welford's update in float64:
 * mean_dev, m2_dev (device [N][N][N] float64, caller-owned) hold the mean and the
 * sum of squared deviations of the first count - 1 states; count >= 1 is the
 * number of states including this one (count = 1 starts them: mean = delta,
 * m2 = 0).  The variance is m2 / (count - 1).  Stream-ordered, no
 * synchronisation; call after a sweep or trajectory.  HMC_EINVAL on a bad
 * argument. */
hmc_status hmc_field_moments(hmc_ctx* ctx, int32_t chain, double* mean_dev, double* m2_dev,
                             int64_t count);

/* The real-space diagonal variant of the mass from the same field: the learned
 * form above with the Fourier diagonal replaced by the constant m_k = 1/mean(v)
 * (v = exp(logvar_dev)), so no Fourier preconditioning; its inverse mass is
 * P diag(v) P less one rank-one term (the mean of the whitened momentum stays
 * frozen), positive definite on the zero-mean fields.  It runs on the same passes as hmc_set_mass (the
 * same cost per step).  NULL restores the plain mass; chain = -1 and the rule
 * on mixed kinds are as for hmc_set_mass (the two learned kinds may be mixed). */
hmc_status hmc_set_mass_diagonal(hmc_ctx* ctx, int32_t chain, const float* logvar_dev);

/* Graph replay: with enable = 1, leapfrog_trajectory and gibbs_sweep record
 * their device work once into a HIP graph on a library-owned stream (default
 * priority, ordered after and before the caller's stream by events) and replay
 * it on later calls; the trajectory or sweep index is passed through device
 * memory, so one graph serves every index.  enable = 0 returns to direct
 * launches.  Pass timing (hmc_timing) does not see graph replays. */
hmc_status hmc_use_graph(hmc_ctx* ctx, int32_t enable);

/* Device timing of the leapfrog passes (tracing).  enable = 1 starts
 * recording HIP events on the context's stream around every launch of the
 * step passes and clears the totals; enable = 0x10 | mask | (s << 8) does the
 * same for the classes whose bits (1 << class) are set in mask, around every
 * (s + 1)-th launch of each class only (s < 256; fewer events, less
 * perturbation); enable = 0 stops recording; enable = -1 only reads.  Other
 * values leave the state unchanged.  ms[4] / launches[4] (host, may be NULL)
 * receive the summed
 * durations and launch counts of: [0] k-space passes of interior leapfrog
 * steps (kick, drift and both x transforms), [1] y passes, [2] real-space
 * passes (z transforms and the data force), [3] every other pass kernel, over
 * the timed launches.  Reading synchronises the stream. */
hmc_status hmc_timing(hmc_ctx* ctx, int32_t enable, double* ms, int64_t* launches);

/* Static description of the last error on this context (or of the last
 * context-free failure when ctx is NULL). */
const char* hmc_last_error(const hmc_ctx* ctx);

void hmc_destroy(hmc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
