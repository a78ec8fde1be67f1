/*
 * glmb.h -- C ABI of the MI355X (gfx950) multi-detection GLMB hot path.
 *
 * The library implements one time step of the labeled multi-object filter of
 * arXiv 2512.06230 (Sec. 3): prediction (survival + LMB birth), the update with a
 * measurement set in which one object may produce several detections (Eq. 2 entries,
 * factorised hypothesis weights, Kalman update of every (track, detection set)), the
 * truncation to the H_max best hypotheses with tau pruning, and the state estimate.
 * All arithmetic runs in hand-written HIP kernels on the stream given at creation.
 *
 * Conventions for every entry point:
 *   - Return value: a glmb_status; nothing crosses the ABI as an exception.
 *   - Argument errors (GLMB_E_ARG) and capacity errors (GLMB_E_CAPACITY) detected before
 *     any device work leave the filter state unchanged.  A capacity overflow detected
 *     during a step (GLMB_E_CAPACITY) and device failures (GLMB_E_DEVICE) leave the
 *     state undefined: re-import a state before the next step.
 *   - "device pointer" arguments must point to memory of the context's device and stay
 *     valid until the context's stream has executed the call; "host pointer" arguments
 *     are read or written before the call returns.  The caller owns all its buffers.
 *   - One context per stream; a context must not be used from two threads at once.
 *   - glmb_last_error() returns a human-readable message for the last failure.
 */
#ifndef GLMB_H
#define GLMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GLMB_OK = 0,
  GLMB_E_ARG = -1,       /* invalid argument (null pointer, negative size, NaN, bad label order) */
  GLMB_E_CAPACITY = -2,  /* a configured capacity would be exceeded                              */
  GLMB_E_NOMEM = -3,     /* device allocation failed                                             */
  GLMB_E_DEVICE = -4,    /* a HIP call failed                                                    */
  GLMB_E_STATE = -5      /* call not valid in the current state (e.g. destroyed context)         */
} glmb_status;

/* Model and filter parameters (Sec. 3; constant-velocity state [px, py, vx, vy]). */
typedef struct {
  float dt;               /* scan interval (s)                                                */
  float q;                /* white-noise acceleration intensity of the motion model           */
  float sigma_z;          /* detection noise std (m), R = sigma_z^2 I                         */
  float p_survive;        /* per-scan survival probability of a track                         */
  float det_rate;         /* gamma: expected detections per object (Poisson); plays P_D's role */
  float clutter_density;  /* kappa: clutter intensity per unit area (> 0)                     */
  float gate_d2;          /* Mahalanobis gate: a pair is compatible iff d^2 <= gate_d2        */
  float birth_r_max;      /* cap of a birth component's existence probability                 */
  float birth_rate;       /* expected births per scan, shared over the birth clusters         */
  float birth_sigma_v;    /* velocity std of a new track (m/s)                                */
  float birth_ru_max;     /* a detection seeds a birth if P(not clutter) < birth_ru_max       */
  float birth_cluster_d;  /* seeds within this distance of a cluster's first seed join it     */
  int32_t h_max;          /* hypotheses kept by predict and by update                         */
  float tau;              /* weight threshold applied after normalising over the kept set     */
  int32_t cap_nodes;      /* selection search nodes (0: 1<<22)                                */
  int32_t cap_labels;     /* distinct labels alive at once (0: 8192)                          */
} glmb_params;

typedef struct glmb_ctx glmb_ctx;

/* Host-side description of a GLMB (used by import, export and warm start).
 * Instances: n_inst Gaussian track densities, inst_lab[2*u] = birth scan, inst_lab[2*u+1] =
 * index within that scan; inst_m[4*u], inst_P[16*u] row-major.  Hypotheses: hyp_logw[h]
 * (need not be normalised; the state keeps its hypotheses in rank order, weight descending,
 * so import ranks them by weight, stably: equal weights keep the input order; export lists
 * them in that order and hyp_parent names the input position), the instances of hypothesis h are
 * hyp_idx[hyp_off[h] .. hyp_off[h+1]) (distinct labels).  Pending births for the next
 * predict: birth_lab/m/P as above and existence probability birth_r.  On export the library
 * also fills inst_src (the input index the instance derives from), inst_nz and
 * inst_z (number and indices of the detections of the last update, at most 8 per
 * instance are listed), hyp_parent (input index of the hypothesis it derives from). */
typedef struct {
  int32_t n_inst, n_hyp, n_idx, n_birth;
  int32_t* inst_lab;
  float* inst_m;
  float* inst_P;
  int32_t* inst_src;   /* export only (may be NULL) */
  int32_t* inst_nz;    /* export only (may be NULL) */
  int32_t* inst_z;     /* export only, 8 per instance (may be NULL) */
  float* hyp_logw;
  int32_t* hyp_off;
  int32_t* hyp_idx;
  int32_t* hyp_parent; /* export only (may be NULL) */
  int32_t* birth_lab;
  float* birth_m;
  float* birth_P;
  float* birth_r;
} glmb_state_host;

/* Per-step statistics of the last update (filled by glmb_stats, which synchronises). */
typedef struct {
  int32_t n_hyp_in, n_hyp_out, n_meas, n_inst_in, n_inst_out, n_labels;
  int64_t gated_pairs;      /* (instance, measurement) pairs inside the gate              */
  int64_t option_terms;     /* sum over (hypothesis, measurement) cells of options        */
  int64_t dense_triples;    /* sum_h |J_h| * M                                           */
  int32_t search_nodes, search_levels, n_births;
  double retained_mass;     /* posterior mass of the kept hypotheses                     */
  double lost_mass;         /* posterior mass removed by the learned proposal (measured only
                               when enabled by glmb_set_proposal; 0 otherwise)           */
  int32_t pairs_removed;    /* gated pairs the learned proposal removed                   */
  /* stage durations of the last update from HIP events on the context's stream (ms):
   * [0] gate + score (through the per-label lists and hypothesis 0's cells), [1] the
   * per-(hypothesis, detection) association kernel of hypotheses 1..H-1 alone, [2] cut bound + deviation items + selection, [3] materialise + Kalman,
   * [4] births (with the side stream, the clutter probabilities run beside [2] and [3], and
   * [4] is the wait for them and the clustering), [5] whole update */
  float stage_ms[6];
  /* (instance, detection set) records whose 16-bit fingerprint equalled that of a different
   * set of the same instance; such runs are resolved by full comparison (results unchanged).
   * The environment variable GLMB_REC_HASH_BITS (1..15, read by glmb_create) narrows the
   * fingerprint so that this path can be exercised. */
  int32_t rec_collisions;
  int32_t host_syncs;       /* host round trips (waits for the device) made by the update  */
  int32_t search_form;      /* selection search of the update: 0 one workgroup, 1 one cooperative
                               whole-GPU launch, 2 host-driven levels of whole-GPU kernels,
                               3 sampled maps (glmb_set_sampling).  Diagnostic environment
                               variables read by glmb_create: GLMB_SEARCH_FORM=multi|coop starts
                               every search on form 2 or 1; GLMB_SEARCH_GROUP_BITS=0|1|2 limits
                               how form 0 rejects a second pick in one group (0 item tables in
                               global memory, 1 in LDS with hashed group bits, 2 exact bits when
                               the items carry at most 64 groups: the default);
                               GLMB_DP_BOUND_INFLATE=x (0 < x < 1) raises the update's counting
                               bound that part of the way to the best value, so that the search
                               again from the caller's bound runs.  Results do not depend on
                               any of them.                                                 */
} glmb_step_stats;

/* Library / status utilities */
const char* glmb_status_string(glmb_status s);
const char* glmb_last_error(const glmb_ctx* ctx);

/* Create a filter on HIP device `device` using `hip_stream` (a hipStream_t, or NULL for the
 * null stream) for every launch.  The context holds one hypothesis with no tracks.  The update
 * also uses a second stream of its own (created on first use, default priority) for work that
 * overlaps the main chain (the births' clutter probabilities, the learned proposal's label
 * inputs), joined by events before its results are read; the environment variable
 * GLMB_SIDE_STREAM=0 (read here) keeps every stage on `hip_stream`.  Host round trips wait
 * for a word the device writes to pinned host memory, spinning briefly before a stream
 * wait. */
glmb_status glmb_create(const glmb_params* params, int device, void* hip_stream, glmb_ctx** out);
glmb_status glmb_destroy(glmb_ctx* ctx);

/* Replace the filter state by a host description (labels of hypotheses must be distinct;
 * birth labels must sort after every instance label). Synchronises. */
glmb_status glmb_import_state(glmb_ctx* ctx, const glmb_state_host* s);
/* Sizes of the current state, for allocating an export: n_inst, n_hyp, n_idx, n_birth. */
glmb_status glmb_state_sizes(glmb_ctx* ctx, int32_t* n_inst, int32_t* n_hyp, int32_t* n_idx, int32_t* n_birth);
/* Copy the state to caller-allocated host arrays sized by glmb_state_sizes. Synchronises. */
glmb_status glmb_export_state(glmb_ctx* ctx, glmb_state_host* s);

/* Prediction to scan k (Sec. 3, prediction): Kalman prediction of every track, the pending
 * birth components join, and the h_max most likely survive/die x include/exclude children of
 * every hypothesis are kept; identical track sets are merged. */
glmb_status glmb_predict(glmb_ctx* ctx, int32_t k);

/* Update with the M detections of scan k (Sec. 3, Eq. 2 to the end of Sec. 3).
 * z_dev: device pointer, float32 [M][2] (x, y), caller-owned, stream-ordered.
 * Computes every gated (track, detection) entry of Eq. 2, the factorised weight of every
 * association map of every hypothesis, keeps the exact h_max best maps (log-weight
 * descending, canonical key ascending), applies tau, runs the Kalman update of every
 * distinct (track, detection set), and derives the birth components for scan k+1. */
glmb_status glmb_update(glmb_ctx* ctx, int32_t k, const float* z_dev, int32_t M);

/* The paper's own hypothesis generator (Sec. 3, hypothesis generation) in place of the exact
 * h_max best maps, for the following glmb_update calls: every predicted hypothesis h draws
 * h_up association maps, each detection independently from the normalised row of the
 * compatibility matrix (Eq. 2) over clutter and h's gated tracks (options in order: clutter,
 * then tracks by label; inverse distribution function of a uniform number); only distinct
 * maps are kept, each with its exact weight (parent weight times association likelihood);
 * then the h_max best (weight descending, then parent rank, then first draw) and tau.  The
 * uniform numbers are Philox4x32-10 (Salmon et al., SC'11) under key `seed` at counter
 * (detection, draw, hypothesis rank, 16 x k + 1), 24-bit.  h_up = 0 restores the exact
 * update; 1 <= h_up <= 65536 and at most 2^30 draws (h_up x hypotheses) per update, else
 * GLMB_E_ARG / GLMB_E_CAPACITY.  glmb_stats reports search_form 3 and the distinct maps in
 * search_nodes. */
glmb_status glmb_set_sampling(glmb_ctx* ctx, int32_t h_up, uint64_t seed);

/* Exact-joint reweighting of the kept hypotheses (Sec. 3 end: a new hypothesis' weight is its
 * parent's times the joint likelihood of its associations), for the following glmb_update
 * calls when on != 0: after the selection (which ranks by the factorised weights, i.e. the
 * product of per-detection likelihoods), every track with a detection set S of two or more
 * detections has that product replaced by the joint likelihood
 *   J(S) = integral N(x; m, P) prod_{i in S} N(z_i; H x, R) dx
 *        = (2 pi sigma^2)^-(|S|-1) |S|^-1 exp(-sum_i |z_i - zbar|^2 / (2 sigma^2)) N(zbar; H m, H P H^T + R/|S|);
 * the hypotheses are re-ranked by the new weight (ties keep the selection's order), tau is
 * applied to the renormalised weights (the best is kept) and the kept ones renormalised.
 * glmb_update_theta lists the maps in the re-ranked order.  on = 0 restores the factorised
 * weights. */
glmb_status glmb_set_joint_reweighting(glmb_ctx* ctx, int32_t on);

/* Keep the h_max first hypotheses in rank order, renormalise over them, drop the hypotheses
 * from the first weight below tau on (the first is always kept), renormalise again (Sec. 3
 * end). Idempotent. */
glmb_status glmb_truncate(glmb_ctx* ctx, int32_t h_max, float tau);

/* State estimate: maximum a posteriori cardinality n, then the most likely hypothesis with
 * n tracks.  Host buffers: labels_out[2*cap], means_out[4*cap]; *n_out receives n.
 * Returns GLMB_E_CAPACITY if n > cap. Synchronises. */
glmb_status glmb_estimate(glmb_ctx* ctx, int32_t cap, int32_t* n_out, int32_t* labels_out, float* means_out);

/* Statistics of the last update. Synchronises. */
glmb_status glmb_stats(glmb_ctx* ctx, glmb_step_stats* out);

/* Diagnostics of the last update, for parity checks (host buffers, sized by the predicted
 * hypothesis count H and the detection count M of that update):
 * best[h] = log weight of hypothesis h's best child minus the log normaliser of every child
 * of every hypothesis; logpi[h] = log posterior mass of h's children; ru[i] = posterior
 * probability that detection i is not clutter. Synchronises. */
glmb_status glmb_update_diag(glmb_ctx* ctx, int32_t H, int32_t M, float* best, float* logpi, float* ru);

/* Association maps of the hypotheses produced by the last update: theta[h*M + i] is the
 * input index of the predicted instance that detection i is assigned to, -1 for clutter.
 * Host buffer of n_hyp*M int32. Synchronises. */
glmb_status glmb_update_theta(glmb_ctx* ctx, int32_t n_hyp, int32_t M, int32_t* theta);

/* ---- Learned pair proposal ------------------------------------------------------------
 * An addition to the update of Sec. 3: a small network scores every gated (track instance,
 * detection) pair of the predicted GLMB from six features, and pairs scoring below a
 * threshold are removed from the option sets of the update (Eq. 2 entries to which the
 * posterior gives negligible mass).  Without parameters the update is the plain method.
 *
 * Network: features -> standardise -> 64 ReLU -> 64 ReLU -> logit.  Parameters: float32
 * vector of GLMB_MLP_NPARAM values W1[64][6] | b1[64] | W2[64][64] | b2[64] | w3[64] | b3,
 * W[j][k] the weight from input k to output j.  Arithmetic: weights, standardised inputs
 * and both hidden activations are rounded to bfloat16 (nearest, ties to even); every sum is
 * accumulated in float32.
 * Features of pair (u, i), from predicted instance u (mean m, covariance P) and detection
 * z_i, in this order: d2 = nu^T (H P H^T + sigma_z^2 I)^-1 nu with nu = z_i - H m; nu_x;
 * nu_y; r_label = existence probability of u's label (total weight of the hypotheses that
 * hold it); age = k - birth scan of the label; n_gate = detections gated with u.
 * norm: host float[12], per-feature mean[6] then standard deviation[6]. */
#define GLMB_MLP_NPARAM 4673
#define GLMB_MLP_NFEAT 6

/* Load the proposal's parameters (params_dev: device float32 [GLMB_MLP_NPARAM], copied
 * before the call returns; NULL unloads them and makes every update plain).  flags:
 * GLMB_PROPOSAL_APPLY: the following updates remove every pair with
 *   sigmoid(logit) < threshold (0 < threshold < 1);
 * GLMB_PROPOSAL_MEASURE: each such update first measures, on the full association space,
 *   the posterior mass the removal loses (stats.lost_mass; one extra pass over the
 *   hypotheses).
 * With flags = 0 the parameters serve glmb_proposal_lost only. Synchronises. */
#define GLMB_PROPOSAL_APPLY 1
#define GLMB_PROPOSAL_MEASURE 2
glmb_status glmb_set_proposal(glmb_ctx* ctx, const float* params_dev, const float* norm, float threshold,
                              int32_t flags);

/* Training data from the current (predicted) state and the M detections of scan k
 * (z_dev as in glmb_update); the state is unchanged.  For every gated pair:
 * feat_dev[cap][6] the features above, pair_dev[cap][2] (input index of the instance as
 * exported, detection index), target_dev[cap] = m_ui / e_u and weight_dev[cap] = e_u, where
 * over the full posterior of the plain update m_ui = sum of pi_h q_hi(u) over the
 * hypotheses h holding u (pi_h: posterior mass of h's children; q_hi(u): probability that
 * detection i belongs to u given h) and e_u = sum of those pi_h.  Pairs are listed by
 * instance (state order), then detection.  *n_pairs (host) receives the pair count;
 * GLMB_E_CAPACITY when it exceeds cap (nothing written). Synchronises. */
glmb_status glmb_pair_features(glmb_ctx* ctx, int32_t k, const float* z_dev, int32_t M, int32_t cap,
                               float* feat_dev, int32_t* pair_dev, float* target_dev, float* weight_dev,
                               int32_t* n_pairs);

/* Posterior mass the proposal with the loaded parameters (glmb_set_proposal) would remove, for
 * each of T thresholds (host thresholds[T], 1 <= T <= 16, each in (0, 1); host lost[T]),
 * on the current predicted state and the detections of scan k; the state is unchanged.
 * lost = 1 - Z_kept / Z_full with Z the total weight of every association map of every
 * hypothesis (with the kept options only, resp. with all). Synchronises. */
glmb_status glmb_proposal_lost(glmb_ctx* ctx, int32_t k, const float* z_dev, int32_t M, int32_t T,
                               const float* thresholds, double* lost);

/* Network kernels on the context's stream (device arrays; n >= 0 samples; feat_dev[n][6]
 * raw features; norm host float[12]).
 * glmb_mlp_forward: logit_dev[n].
 * glmb_mlp_grad: weighted binary cross-entropy L = sum_p w_p (softplus(s_p) - y_p s_p) /
 *   sum_p w_p (s: logit, y: target in [0, 1], w >= 0 with a positive sum) into loss_dev[1],
 *   its gradient into grad_dev[GLMB_MLP_NPARAM]; the bfloat16 roundings pass the gradient
 *   unchanged.  Deterministic: fixed reduction order.
 * glmb_mlp_adam: one Adam step (Kingma & Ba, 2015, with bias correction) at step number
 *   t >= 1: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *   params -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); m_dev, v_dev start at zero. */
glmb_status glmb_mlp_forward(glmb_ctx* ctx, const float* params_dev, const float* norm, const float* feat_dev,
                             int32_t n, float* logit_dev);
glmb_status glmb_mlp_grad(glmb_ctx* ctx, const float* params_dev, const float* norm, const float* feat_dev,
                          const float* target_dev, const float* weight_dev, int32_t n, float* grad_dev,
                          float* loss_dev);
glmb_status glmb_mlp_adam(glmb_ctx* ctx, float* params_dev, float* m_dev, float* v_dev, const float* grad_dev,
                          int32_t t, float lr, float beta1, float beta2, float eps);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * training or serving loops, harnesses that forbid hipMalloc): glmb_mlp_grad without any
 * allocation.  Same arguments and the same results, bit for bit.  Its per-workgroup partial
 * sums (one row of GLMB_MLP_NPARAM + 2 floats per 64 samples) live in a fixed device array of
 * (GLMB_MLP_NOALLOC_MAX / 64) rows, 9.6 MB, that each GPU holds from the first glmb_create on
 * it until the process ends.  n > GLMB_MLP_NOALLOC_MAX returns GLMB_E_CAPACITY before any
 * device work.  Every call on one GPU shares that array, so calls that overlap on one GPU (from
 * several streams, contexts or threads) race: the caller serialises them. */
#define GLMB_MLP_NOALLOC_MAX 32768
glmb_status glmb_mlp_grad_noalloc(glmb_ctx* ctx, const float* params_dev, const float* norm, const float* feat_dev,
                                  const float* target_dev, const float* weight_dev, int32_t n, float* grad_dev,
                                  float* loss_dev);

/* ---- Particle form of the track densities --------------------------------------------
 * Sec. 3 represents every track by P weighted particles, propagated with constant turn rate and
 * velocity (CTRV) kinematics and weighted by the measurement likelihood, with resampling to
 * prevent degeneracy.  These three calls are stateless and stream-ordered on hip_stream (NULL:
 * the default stream); every pointer is a device pointer owned by the caller.  Particle states
 * are component-major float32 [5][n] (x, y, v, psi, omega; n = U P, track u holds particles
 * u P .. u P + P - 1) with normalised natural-log weights float32 [n].  Uniform numbers are
 * Philox4x32-10 (Salmon et al., SC'11) under key `seed`, 24-bit.  Errors: GLMB_E_ARG for a null
 * pointer or a value out of range (nothing launched), GLMB_E_CAPACITY for P > 4096,
 * GLMB_E_DEVICE when a launch fails.
 *
 * glmb_pf_predict: in place, every particle over dt with white accelerations
 *   a_v = sigma_a n1, a_w = sigma_w n2 held over the step (n1, n2 standard normal by the
 *   Box-Muller transform of the first two Philox words at counter (q, 0, 16 k + 2, 0), q the
 *   particle index < 2^32):  x += v/w (sin(psi + w dt) - sin psi) + dt^2/2 a_v cos psi,
 *   y += v/w (cos psi - cos(psi + w dt)) + dt^2/2 a_v sin psi (the straight-line limit as
 *   w -> 0), v += dt a_v, psi += w dt + dt^2/2 a_w, w += dt a_w.
 * glmb_pf_loglik: phi float32 [U][M], the Eq. 2 entry of every (track, detection) pair:
 *   log gamma + log sum_p w_p N(z_i; (x_p, y_p), sigma^2 I) when the detection passes the gate
 *   d^2 <= gate on the particles' weighted mean and covariance plus sigma^2 I, else -inf.
 *   z: float32 [M][2].
 * glmb_pf_update: R records (track rec_u[r], detections rec_z[rec_off[r] .. rec_off[r+1]) of
 *   z [M][2]): log w'_p = log w_p + sum_{i in S} log N(z_i; (x_p, y_p), sigma^2 I), normalised;
 *   when the effective sample size 1 / sum w'^2 < ess_frac P, systematic resampling (output
 *   particle j copies the first particle whose cumulative weight exceeds (j + u0) / P, u0 the
 *   Philox uniform at counter (r, 0, 16 k + 3, 0); weights 1 / P).  Outputs out_state [5][R P],
 *   out_logw [R P], resampled[r] = 1 (resampled), 0 (reweighted) or -1 (the record names a
 *   track or detection out of range: its outputs are left unwritten). */
glmb_status glmb_pf_predict(void* hip_stream, float* state_dev, int64_t n, float dt, float sigma_a, float sigma_w,
                            uint64_t seed, int32_t k);
glmb_status glmb_pf_loglik(void* hip_stream, const float* state_dev, const float* logw_dev, int32_t U, int32_t P,
                           const float* z_dev, int32_t M, float sigma, float gamma, float gate, float* phi_dev);
glmb_status glmb_pf_update(void* hip_stream, const float* state_dev, const float* logw_dev, int32_t U, int32_t P,
                           int32_t R, const int32_t* rec_u_dev, const int32_t* rec_off_dev, const int32_t* rec_z_dev,
                           const float* z_dev, int32_t M, float sigma, float ess_frac, uint64_t seed, int32_t k,
                           float* out_state_dev, float* out_logw_dev, int32_t* resampled_dev);

/* ---- Batched scenes -------------------------------------------------------------------
 * An addition to the method (the paper filters one scene): many independent scenes of uneven
 * size advance one time step in one call.  Each scene is a context of its own (its state,
 * parameters and statistics); host worker threads, each driving its own HIP stream, pull the
 * scenes in longest-job-first order of the cost estimate H * M * (1 + gated tracks per
 * detection) of the previous step (H * M on the first) and run glmb_predict, glmb_update and
 * glmb_truncate(h_max, tau) on them.  A scene's result equals that of its own single-scene
 * calls bit for bit, whatever the number of workers or the order. */
#define GLMB_BATCH_MAX_WORKERS 16
typedef struct glmb_batch glmb_batch;

typedef struct {
  int32_t n_scenes, workers, longest_first;
  float step_ms;               /* wall time of the last glmb_batch_step (host clock)          */
  double scene_updates_per_s;  /* n_scenes / step time                                        */
  int32_t first_error_scene;   /* -1 if every scene succeeded                                  */
} glmb_batch_stats;

/* n scenes with parameters params[n] on HIP device `device`; 1 <= workers <= 16 worker
 * streams (created by the batch, default priority).  Every scene starts as glmb_create's. */
glmb_status glmb_batch_create(int32_t n, const glmb_params* params, int device, int32_t workers,
                              glmb_batch** out);
glmb_status glmb_batch_destroy(glmb_batch* b);
/* Schedule of the following steps: number of workers, longest-job-first (1) or index order (0). */
glmb_status glmb_batch_set_schedule(glmb_batch* b, int32_t workers, int32_t longest_first);
/* The context of scene `scene` (owned by the batch: valid until glmb_batch_destroy, not to be
 * destroyed by the caller) for import, export, estimate and statistics. */
glmb_status glmb_batch_scene(glmb_batch* b, int32_t scene, glmb_ctx** out);
/* One time step k of every scene.  z_dev: device float32 [z_off[n]][2], the detections of
 * scene s are rows z_off[s] .. z_off[s+1]); z_off: host int32 [n+1], z_off[0] = 0,
 * non-decreasing.  caller_stream: the hipStream_t on which z_dev was written (NULL: the null
 * stream); the worker streams wait for the work queued there before reading it.
 * Synchronises.  On failure the status of the first failing scene is returned
 * (glmb_batch_last_error names it) and the other scenes have still been stepped. */
glmb_status glmb_batch_step(glmb_batch* b, int32_t k, const float* z_dev, const int32_t* z_off,
                            void* caller_stream);
glmb_status glmb_batch_stats_get(glmb_batch* b, glmb_batch_stats* out);
const char* glmb_batch_last_error(const glmb_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* GLMB_H */
