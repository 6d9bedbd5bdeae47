/*
 * pyfpt.h -- C ABI of the MI355X (gfx950) importance-sampled first-passage
 * engine for stochastic inflation.
 *
 * Method: Jackson, Assadullahi, Koyama, Vennin, Wands, "Numerical simulations
 * of stochastic inflation using importance sampling" (arXiv:2206.11234).
 *
 *   - Each run integrates the slow-roll Langevin equation with the
 *     Euler-Maruyama step of the BIASED equation (Sec. 2.2,
 *     eq. eq_euler_maruyam_modified):
 *         phi_{k+1} = phi_k + [D(phi_k) + B(phi_k)] dN + S(phi_k) sqrt(dN) xi_k,
 *     D = -V'/V and S = sqrt(V/3)/(2 pi) in Planck units (Sec. 2.3,
 *     eq. eq_sr_diffusion with H^2 = V/3).
 *   - The importance weight w = p_T/p_S of the path (Sec. 2.2,
 *     eqs. eq_importance_sampling_bias ... eq_importance_sampling_bias_w) is
 *     carried as ln w = -sum_k r_k (r_k dN/2 + sqrt(dN) xi_k), r = B/S: the
 *     likelihood ratio of the two Gaussian path densities (the exponent as
 *     printed in eq_importance_sampling_bias_w lacks this minus sign).
 *   - A run stops at first passage phi <= phi_end and records N = k dN
 *     (Sec. 2.1); phi > phi_UV is reflected (Sec. 2.3, Sec. 3).
 *   - Runs are binned in N (right-closed bins, Sec. 2.1
 *     eq. eq_bin_pdf_reconstrcuted) and each bin accumulates the weighted
 *     estimator's sums (Sec. 2.2 eq. eq_bin_pdf_reconstrcuted_weighted_naive),
 *     the jackknife subsets (Sec. 2.1) and moments of ln w (Sec. 2.4).
 *
 * Step arithmetic is IEEE binary32; ln w and all per-bin sums are binary64
 * with log-sum-exp merges (weights span far more than the binary32 range).
 * Noise: Philox4x32-10 (Salmon et al., SC'11) with counter
 * (k/4, t_lo, t_hi, stream) and key (seed_lo, seed_hi); each 32-bit word x
 * gives u = (2 (x >> 9) + 1) 2^-24 and Box-Muller maps (u0,u1), (u2,u3) to
 * the normals of steps 4j..4j+3: rho = sqrt(-2 ln u_a), (rho cos 2 pi u_b,
 * rho sin 2 pi u_b).  A trajectory's result depends only on
 * (seed, stream, t) and the instance: it is the same for every launch
 * configuration.
 *
 * Conventions for every entry point:
 *   - returns PYFPT_OK (0) or a negative PYFPT_E* code; never aborts, never
 *     throws across the ABI; pyfpt_last_error() gives a message (per thread);
 *   - host-side structs and arrays passed in are read during the call only;
 *   - output buffers are owned by the caller; the library never frees them;
 *   - device pointers refer to memory of the current HIP device;
 *   - work is enqueued on opt->stream (a hipStream_t; NULL = null stream).
 *     With host outputs the call returns after the stream has finished; with
 *     device outputs it returns once the work is enqueued.
 */
#ifndef PYFPT_H
#define PYFPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PYFPT_OK 0
#define PYFPT_EINVAL (-1)      /* invalid argument (message says which) */
#define PYFPT_ENOMEM (-2)      /* device or host allocation failed, or workspace too small */
#define PYFPT_EDEVICE (-3)     /* HIP runtime error (message carries hipGetErrorString) */
#define PYFPT_EUNSUPPORTED (-4)

/* ---- potentials V(phi), Planck units (Sec. 2.3, Sec. 3) ---- */
#define PYFPT_POT_QUADRATIC 0        /* V = m^2 phi^2 / 2 (eq. eq_quadratic_inflation_potential) */
#define PYFPT_POT_QUADRATIC_BUMP 1   /* V = m^2 phi^2/2 [1 + a exp(-(phi-phi0)^2/(2 w^2))] */
#define PYFPT_POT_FLAT 2             /* V = V0: the quantum well of Sec. 3 (D = 0, S const) */

/* ---- bias B(phi) (Sec. 2.3 eq. eq_importance_sampling_amplitude_general) ---- */
#define PYFPT_BIAS_NONE 0            /* B = 0: direct sampling, w = 1 */
#define PYFPT_BIAS_NOISE_SCALED 1    /* B = A S(phi): f = S, the paper's default */
#define PYFPT_BIAS_POWER 2           /* B = A phi^p (eq. eq_importance_sampling_amplitude_power_law), p >= 0 integer */
#define PYFPT_BIAS_MLP 3             /* B = r_theta(phi, k dN, N*) S: learned proposal, see pyfpt_mlp */

/* ---- run status (dump) ---- */
#define PYFPT_ST_ENDED 1             /* phi <= phi_end reached: N = k dN */
#define PYFPT_ST_CENSORED 2          /* k reached k_max */
#define PYFPT_ST_ESCAPED 3           /* no wall and phi > phi_esc */

typedef struct pyfpt_potential {
    int32_t kind;                    /* PYFPT_POT_* */
    double m, a, phi0, w;            /* quadratic (m) and bump (a, phi0, w) parameters */
    double V0;                       /* flat potential */
} pyfpt_potential;

/* Learned proposal: a 3 -> 64 -> 64 -> 1 tanh network giving the bias in noise units,
 * r = B/S = out_scale * (w3 . h2 + b3), h2 = tanh(W2 h1 + b2), h1 = tanh(W1 x + b1), from
 * x_i = (in_i - in_mean_i) * in_inv_scale_i with in = (phi, k dN, N*).  Any such bias leaves
 * the weighted estimator unbiased (the weight of Sec. 2.2 holds for any adapted drift).
 * `params` (device memory) holds the 4481 parameters as bfloat16, in this order:
 *   W1[64][3], b1[64], W2[64][64], b2[64], w3[64], b3        (row-major, W[out][in]).
 * The network is evaluated on the matrix cores with binary32 accumulation and bfloat16
 * activations, every step (eval_every = 1) or once per group of 4, 8 or 16 steps at the
 * group's first step (eval_every = 4, 8 or 16; the bias is then held for the group).  The
 * sampler's tanh is accurate to the bfloat16 its result is rounded to (a clamped polynomial,
 * within a third of a bfloat16 ulp of tanh); pyfpt_train_proposal's gradients use tanh. */
typedef struct pyfpt_mlp {
    const void *params;              /* device pointer, 4481 bfloat16 */
    int32_t hidden;                  /* must be 64 */
    float in_mean[3], in_inv_scale[3];
    float out_scale;
    int32_t eval_every;              /* 1, 4, 8 or 16 */
} pyfpt_mlp;

typedef struct pyfpt_bias {
    int32_t kind;                    /* PYFPT_BIAS_* */
    int32_t p;                       /* power-law exponent */
    double A;                        /* amplitude (A or A_p) */
    double target_N;                 /* N* for the learned proposal */
    pyfpt_mlp mlp;                   /* used when kind == PYFPT_BIAS_MLP */
} pyfpt_bias;

/* Bins: n_bins right-closed bins (e_j, e_{j+1}] over strictly ascending
 * binary64 edges (host array of n_bins + 1).  n_sub jackknife subsets:
 * trajectory t belongs to subset t mod n_sub (Sec. 2.1; >= 2; 16 if 0). */
typedef struct pyfpt_bins {
    int32_t n_bins;
    int32_t n_sub;
    const double *edges;
} pyfpt_bins;

/* One instance of a batched run. */
typedef struct pyfpt_instance {
    pyfpt_potential pot;
    pyfpt_bias bias;
    double phi_in, phi_end;          /* phi_in > phi_end */
    double phi_uv;                   /* reflecting wall; +INFINITY = none; phi_uv >= phi_in */
    double phi_esc;                  /* escape level without a wall; 0 -> 100 phi_in */
    double dN;                       /* step, > 0 */
    uint64_t n_traj;                 /* runs t = t_first .. t_first + n_traj - 1 */
    uint64_t t_first;                /* first run id (0 usually).  Runs are addressed by their id
                                        alone, so id ranges split one instance into shards (other
                                        launches or devices) whose counts and jackknife tables add
                                        and whose log-sum-exp sums combine; t_first + n_traj must
                                        not exceed 2^64 - 1 */
    uint64_t k_max;                  /* step cap, 1 .. 2^32-1; 0 -> 2^20 */
    uint32_t stream;                 /* noise stream id (Philox counter word 3) */
    uint32_t reserved;
    double cost_hint;                /* expected steps per run, for the queue order (longest
                                        first) and as the centre of the step-count sums; 0 -> the
                                        noise-free run length under the applied drift for the
                                        quadratic potentials with no or noise-scaled bias (k_max
                                        where that drift does not lead to phi_end), the unbiased
                                        one for the other biases, k_max for other potentials */
    pyfpt_bins bins;
} pyfpt_instance;

/*
 * Result of one instance: two caller-owned flat buffers (host memory, or
 * device memory when on_device != 0), sized by pyfpt_result_layout.
 * R = n_bins + 4 rows: rows 0..n_bins-1 are the bins, then underflow
 * (N <= e_0), overflow (N > e_B), censored, escaped.  J = n_sub.
 *
 * counts (uint64):
 *   count[R]           runs per row
 *   jk_count[J][R]     runs per (subset, row)
 *   n_traj, total_steps (sum of k over every run, censored included)
 * values (double):
 *   lse_w[R]           log sum w per row (-inf when empty)
 *   lse_w2[R]          log sum w^2 per row
 *   jk_lse_w[J][R]     log sum w per (subset, row)
 *   mean_lnw[R], m2_lnw[R], m3_lnw[R], m4_lnw[R]
 *                      mean and central moments (1/n) sum (ln w - mean)^j (NaN when empty)
 *   log_p[B]           log P_hat_j = lse_w - log(e_{j+1} - e_j) - log n_traj
 *   rel_err_jk[B]      jackknife relative error of P_hat_j (sd over subsets / sqrt J)
 *   rel_err_kish[B]    sqrt(sum w^2/(sum w)^2 - 1/n_traj): delta-method relative error
 *   log_p_ln[B]        lognormal estimator (Sec. 2.4, eqs. eq_lognormal_mean_maximum_likelihood and
 *                      eq_lognormal_bin_pdf_reconstrcuted_weighted_maximum_likelihood):
 *                      log( n_j exp(<ln w>_j + s_j^2/2) / (n_traj (e_{j+1} - e_j)) ), s_j^2 the
 *                      unbiased sample variance of ln w in the bin (NaN for n_j < 2)
 *   rel_err_ln_lo[B], rel_err_ln_hi[B]
 *                      its error (eq. eq_log_normal_bin_pdf_reconstrcuted_error_maximum_likelihood,
 *                      the Cox interval): P_hat (1 - rel_lo) .. P_hat (1 + rel_hi), rel = |exp(-+u) - 1|,
 *                      u = sqrt(s^2/n_j + s^4/(2 n_j - 2))
 *   normal_p[B]        p-value of D'Agostino and Pearson's K^2 normality test of ln w in the bin
 *                      (skewness test of D'Agostino 1970, kurtosis test of Anscombe and Glynn 1983,
 *                      K^2 ~ chi^2 with 2 degrees of freedom; NaN for n_j < 8).  The paper accepts
 *                      the lognormal estimator when every bin's p-value is at least 0.005.
 *   lse_w_all, lse_w2_all, lse_wk, lse_wk2   log sum over all runs of w, w^2, w k, w k^2
 *   sum_k2             sum of k^2 over all runs
 *   pearson_r          Pearson's correlation coefficient of ln w (equivalently log10 w) with N over
 *                      the runs that ended (Sec. 3.4: |r| near 1 means a squeezed (N, w) scatter, the
 *                      criterion for tuning the power p of the bias A_p phi^p); NaN if undefined
 *   ess[B]             Kish's effective sample size of the bin, (sum w)^2 / sum w^2 = exp(2 lse_w - lse_w2)
 *                      (0 for an empty bin)
 *   lognormal_gate     1 when every bin with n_j >= 8 (a defined normality p-value) has p >= 0.005, the
 *                      paper's condition for using the lognormal estimator on the result (Sec. 2.4),
 *                      else 0
 */
typedef struct pyfpt_result {
    uint64_t *counts;
    double *values;
    int32_t on_device;
} pyfpt_result;

typedef struct pyfpt_layout {
    uint64_t n_counts, n_values;     /* buffer lengths in elements */
    uint64_t count, jk_count, n_traj, total_steps;
    uint64_t lse_w, lse_w2, jk_lse_w, mean_lnw, m2_lnw, m3_lnw, m4_lnw;
    uint64_t log_p, rel_err_jk, rel_err_kish;
    uint64_t log_p_ln, rel_err_ln_lo, rel_err_ln_hi, normal_p;
    uint64_t lse_w_all, lse_w2_all, lse_wk, lse_wk2, sum_k2;
    uint64_t pearson_r;
    uint64_t ess, lognormal_gate;
} pyfpt_layout;

/* Per-trajectory record of runs t with t % stride == 0 and t / stride < n
 * (device arrays of n entries per instance, instance i at offset i*n). */
typedef struct pyfpt_dump {
    uint64_t n, stride;              /* n = 0: no dump */
    uint32_t *k;
    double *lw;
    float *phi;
    int32_t *status;
} pyfpt_dump;

typedef struct pyfpt_options {
    void *stream;                    /* hipStream_t; NULL = null stream */
    int32_t block;                   /* threads per workgroup (64..1024, multiple of 64; <= 256 for the
                                        learned bias); 0 = autotune */
    int32_t chunk;                   /* queue claim multiplier per wave (>= 1); 0 = autotune */
    int32_t wg_per_cu;               /* persistent workgroups per CU; 0 = autotune */
    int32_t use_graph;               /* capture the launch sequence in a hipGraph and replay it */
    void *workspace;                 /* device scratch; NULL = library-managed */
    size_t workspace_bytes;
    pyfpt_dump dump;
    uint64_t k_max;                  /* pyfpt_run only: step cap (0 -> 2^20) */
    double phi_esc;                  /* pyfpt_run only: escape level (0 -> 100 phi_in) */
    uint32_t stream_id;              /* pyfpt_run only: noise stream */
    uint32_t reserved;
    uint64_t t_first;                /* pyfpt_run only: first run id (see pyfpt_instance) */
    float *timing_ms;                /* if not NULL: [0] step kernel, [1] merge kernel (synchronises) */
} pyfpt_options;

/*
 * Buffer lengths and element offsets of one instance's result for n_bins bins and n_sub
 * jackknife subsets (0 -> 16): per bin the counts and log-sums of w and w^2 (Sec. 2.1, 2.2), the
 * jackknife tables, the moments of ln w and the lognormal estimate with its normality p-value
 * (Sec. 2.4), the estimates log P and their errors; per instance the whole-run sums and
 * Pearson's r (Sec. 3.4).  The caller allocates counts (u64) and values (f64) of these lengths
 * and passes them in a pyfpt_result.  Host arithmetic; EINVAL for a NULL out, n_bins < 1, or
 * n_sub other than 0 or 2 .. 64.
 */
int pyfpt_result_layout(int32_t n_bins, int32_t n_sub, pyfpt_layout *out);

/*
 * The integer step thresholds the kernels bin by (Sec. 2.1: a run that ends after k steps has
 * N = k dN, and bins are right-closed, N in (e_j, e_{j+1}]): out[j] = max{k >= 0 : fl(k dN) <= e_j}
 * in binary64, clamped to [0, 2^32 - 1].  A run of k steps falls in bin j exactly when
 * out[j] < k <= out[j+1], below the range when k <= out[0], above it when k > out[n_edges-1].
 * edges: n_edges host values; out: n_edges host values.  Host arithmetic; EINVAL for NULL
 * pointers, n_edges < 1, or dN not finite and > 0.
 */
int pyfpt_bin_thresholds(const double *edges, int32_t n_edges, double dN, uint32_t *out);

/*
 * Single instance (the paper's inputs: V via pot, phi_in, phi_end, phi_UV,
 * dN, bias, number of runs; Sec. 2.3 and Sec. 3).
 * EINVAL: NaN/Inf in finite fields; phi_in <= phi_end; phi_uv < phi_in;
 * dN <= 0; edges not strictly ascending or not finite; n_bins < 1;
 * n_sub == 1 or n_sub > 64; k_max >= 2^32; a zero or negative V on
 * [phi_end, phi_uv].  n_traj = 0 returns OK with empty rows.  Censored or
 * escaped runs are not errors.
 */
int pyfpt_run(const pyfpt_potential *pot, double phi_in, double phi_end, double phi_uv, double dN,
              const pyfpt_bias *bias, uint64_t n_traj, uint64_t seed, const pyfpt_bins *bins,
              pyfpt_result *out, const pyfpt_options *opt);

/*
 * Batch: n_inst instances (1..1024) in one persistent launch over a shared
 * work queue ordered longest-expected-run first; out is an array of n_inst
 * results.  All instances must share the potential kind and bias kind
 * (otherwise EUNSUPPORTED; learned-bias instances must also share the network
 * parameters and eval_every), except that PYFPT_BIAS_NONE and
 * PYFPT_BIAS_NOISE_SCALED mix (no bias is the noise-scaled bias with A = 0,
 * with identical results).  Same validation as pyfpt_run per instance.
 */
int pyfpt_run_batch(const pyfpt_instance *inst, int32_t n_inst, uint64_t seed,
                    pyfpt_result *out, const pyfpt_options *opt);

/*
 * For callers that cannot allocate (code under HIP stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): pyfpt_run_batch without any allocation.  Same instances, seed, results
 * and errors as pyfpt_run_batch, with the same kernels; its device scratch (queue counter,
 * instance records, thresholds, staging results, per-workgroup tables) is a static device array
 * of PYFPT_NOALLOC_SCRATCH_BYTES that each device the library runs on holds from its first use
 * until the process ends, and its host bookkeeping comes from a static host arena of 8 MiB.  The
 * call makes no hipMalloc, hipFree, hipHostMalloc or heap allocation.
 *   - The caller still owns inst, out (host or device buffers) and the dump arrays.
 *   - opt->block, opt->chunk and opt->wg_per_cu as given, 0 = the defaults (no autotuning, which
 *     would allocate); opt->workspace must be NULL and opt->use_graph 0 (EINVAL otherwise).
 *   - PYFPT_ENOMEM, with the bytes needed, when the batch's tables do not fit the scratch (the
 *     tables take about n_workgroups x (n_rows x (24 + 12 n_sub) + 128 n_inst) bytes with
 *     n_rows = sum of (n_bins + 4)); fewer workgroups per CU or fewer bins make them fit.
 *   - Every call on a device shares that device's scratch and the process's host arena: the call
 *     holds the library's lock until its work is enqueued, but work enqueued on two streams that
 *     overlap on one device races on the scratch.  Serialise such calls (one stream, or an event
 *     between them).  The scratch keeps the last call's contents; the kernels clear what they use.
 */
#define PYFPT_NOALLOC_SCRATCH_BYTES (64u << 20)
int pyfpt_run_batch_noalloc(const pyfpt_instance *inst, int32_t n_inst, uint64_t seed,
                            pyfpt_result *out, const pyfpt_options *opt);

/* Device workspace in bytes that pyfpt_run_batch needs for these instances and options
 * (block/wg_per_cu as resolved; 0 fields take the defaults): the per-workgroup tables, the
 * queue counter, the instance records and the staging results.  A caller that supplies
 * opt->workspace must give at least this many bytes (ENOMEM otherwise).  Host arithmetic;
 * EINVAL as pyfpt_run_batch for invalid instances. */
int pyfpt_workspace_size(const pyfpt_instance *inst, int32_t n_inst, const pyfpt_options *opt,
                         size_t *bytes);

/*
 * The learned bias on its own (for checks and for tools): r[i] = r_theta(phi[i], N[i], N*)
 * for i < n, with the same matrix-core evaluation as inside the step loop.  phi, N and r are
 * device arrays of n binary32 values; work is enqueued on `stream` (a hipStream_t, NULL =
 * null stream) and the call returns once it is enqueued.  EINVAL for a NULL pointer with
 * n > 0 or hidden != 64.
 */
int pyfpt_mlp_forward(const pyfpt_mlp *mlp, double target_N, const float *phi, const float *N, float *r,
                      uint64_t n, void *stream);

/*
 * Multi-bias reconstruction.  Runs with different bias amplitudes probe different regions of
 * one P(N) and agree where they overlap (Sec. 3.2 and 3.3); this combines, bin by bin, the
 * estimates of n_res results that share the same n_bins bins and n_sub.  A result contributes
 * to a bin only where its estimate is trusted, and contributions are weighted by the inverse
 * variance of log P_hat:
 *   estimator 0: naive P_hat (log_p) with the jackknife error rel_err_jk as the error of
 *                log P; trusted when n_j > 400 (Sec. 2.1) and n_j > exp(sigma^2_lnw) (Sec. 2.4);
 *   estimator 1: lognormal P_hat (log_p_ln) with u = log(1 + rel_err_ln_hi) as the error of
 *                log P; trusted when n_j >= 8 and the bin's normality p-value >= 0.005;
 *   estimator 2: per result, estimator 1 when the result passes the lognormal gate (no bin with
 *                a defined p-value below 0.005, Sec. 2.4), else estimator 0;
 *   estimator 3: per bin, estimator 1 where the bin passes the gate (n_j >= 8, p >= 0.005),
 *                else estimator 0 with its own trust rule (the fallback of Sec. 2.4 taken bin
 *                by bin: with many runs per bin the test resolves the departure from a
 *                lognormal of wide bins and a whole-result gate rejects nearly every result).
 * Adding PYFPT_COMBINE_NO_EXTRAPOLATION to the estimator also requires n_j >= exp(s_j^2/2) of a
 * lognormal estimate (s_j^2 the unbiased variance of ln w in the bin): its value
 * exp(<ln w> + s^2/2) comes from ln w about s standard deviations above the mean, which n draws
 * reach only if s <= sqrt(2 ln n); beyond that the estimate extrapolates the normal law of
 * ln w into a range no run has sampled (an addition to the paper's gate, which cannot test
 * that range).
 * Where several results contribute to a bin and scatter more than their errors allow
 * (chi^2 = sum_i (y_i - y_bar)^2 / e_i^2 > n_used - 1), err_log is scaled by Birge's ratio
 * sqrt(chi^2 / (n_used - 1)).
 * res: n_res results (host or device buffers, as each one's on_device says).  Outputs (host,
 * n_bins each): log_p (NaN where nothing contributes), err_log (standard error of log P),
 * n_used (contributing results).  Host arithmetic; EINVAL for bad arguments.
 */
#define PYFPT_COMBINE_NO_EXTRAPOLATION 16
int pyfpt_combine(const pyfpt_result *res, int32_t n_res, int32_t n_bins, int32_t n_sub, int32_t estimator,
                  double *log_p, double *err_log, int32_t *n_used);

/* ---- training of the learned proposal ----
 *
 * The paper leaves the choice of the best bias open (Sec. 3.4).  The learned proposal is
 * tuned to minimise the second moment of the weights of the runs that end in a target window
 * B* = (lo, hi] of N:
 *     log M2(theta) = log( sum_{i in B*} w_0,i w_theta,i / n_total ),
 * over runs i drawn once from the current proposal theta_0 (weights w_0, Sec. 2.2), where
 * w_theta,i is the weight the same path would have under the candidate network theta.  With
 * eta_k = r_0,k dN + sqrt(dN) xi_k, the noise increment of step k under the target process,
 * ln w_theta = sum_k [ -r_theta,k eta_k + r_theta,k^2 dN/2 ].  The candidate is held over
 * groups of `group` (1, 4, 8 or 16) steps, so each path reduces to one record per group.
 */
typedef struct pyfpt_record {
    float phi;                       /* field before the group's first step */
    uint32_t k;                      /* step index of the group's first step */
    float H;                         /* sum over the group of fma(r_0, dN, sqrt(dN) xi), binary32 in step order */
    uint32_t path_n;                 /* path index << 5 | number of steps in the group (1..16) */
} pyfpt_record;

/*
 * Replay the runs t_ids[0..n_paths) of a sampling run (same instance, same seed) under the
 * instance's proposal, with the sampler's own arithmetic, and cut them into records: path i
 * writes rec[rec_off[i] .. rec_off[i+1]), which must be its records: with stride s >= 1 only the
 * groups g = 0, s, 2s, ... are kept, ceil(ceil(k_i / group) / s) records.  All
 * arrays are host memory; k_out, lw_out and status_out receive the replayed run (identical to
 * the sampled one), so a caller can check the slots.  EINVAL: group not 1, 4, 8 or 16,
 * n_paths >= 2^27, rec_off not ascending, stride < 1, or the instance as in pyfpt_run.  The
 * call synchronises.
 */
int pyfpt_proposal_records(const pyfpt_instance *inst, uint64_t seed, const uint64_t *t_ids, int32_t n_paths,
                           int32_t group, int32_t stride, const uint64_t *rec_off, pyfpt_record *rec,
                           uint32_t *k_out, double *lw_out, int32_t *status_out, const pyfpt_options *opt);

/*
 * The objective and its gradient from records (host arrays).  objective 0: log M2(theta) as
 * above; objective 1: the cross entropy sum_i c_i ln w_theta,i with c_i = w_0,i / sum_j w_0,j,
 * i.e. the Kullback-Leibler divergence of the proposal from the target restricted to the
 * window, up to a theta-independent constant (its minimiser is the same zero-variance
 * proposal, and its path weights do not depend on theta).  temper = beta in (0, 1]: w_0 enters
 * the path weights as w_0^beta (1 = the objectives as written; a smaller beta gives a gradient
 * less dominated by the few heaviest runs while the proposal is poor; the estimates of any run
 * stay unbiased whatever proposal results).  rec_weight = the record stride s: each record
 * stands for s groups (1 for complete records; s > 1 only with objective 1, whose path
 * weights do not depend on the sums being estimated).  theta holds the 4481 binary32
 * master parameters in the order of pyfpt_mlp; net supplies the input normalisation and
 * out_scale (its params are not read); dN as in the sampling run; lw0[i] = ln w_0 of path i;
 * n_total = number of runs drawn.  Outputs: *loss, grad[4481] (binary64), lw_theta[n_paths].
 * The network is evaluated in binary32 without roundings (the training copy); the gradient is
 * summed in a fixed order.  EINVAL: n_paths < 1 or >= 2^27, rec_off not ascending to n_rec, a
 * record's path index >= n_paths or its step count outside 1..16.  The call synchronises.
 */
int pyfpt_proposal_loss_grad(const pyfpt_mlp *net, double target_N, double dN, const float *theta,
                             const pyfpt_record *rec, uint64_t n_rec, const uint64_t *rec_off, int32_t n_paths,
                             const double *lw0, double n_total, int32_t objective, double temper,
                             double rec_weight, double *loss, double *grad, double *lw_theta,
                             const pyfpt_options *opt);

typedef struct pyfpt_train_config {
    double window_lo, window_hi;     /* target window B* = (lo, hi] in N */
    uint64_t n_sample;               /* runs drawn per round from the current proposal */
    int32_t max_paths;               /* window runs kept per round (0 = all, up to 2^27 - 1) */
    int32_t rounds;                  /* sampling rounds */
    int32_t steps;                   /* Adam steps per round */
    int32_t group;                   /* 1, 4, 8 or 16: the network's evaluation interval */
    float lr, beta1, beta2, eps;     /* Adam */
    int32_t objective;               /* 0: log M2; 1: cross entropy (see pyfpt_proposal_loss_grad) */
    float temper;                    /* beta in (0, 1] of pyfpt_proposal_loss_grad */
    int32_t stride;                  /* record stride (>= 1; > 1 needs objective 1) */
    int32_t select;                  /* 0, or a pilot size: after the rounds, the starting network and
                                        each round's end network each draw `select` runs (seeds apart
                                        from the rounds'), and the one whose window runs have the largest
                                        Kish ESS is returned */
} pyfpt_train_config;

typedef struct pyfpt_train_report {
    int32_t n_window;                /* runs of the round that ended in the window */
    int32_t n_used;                  /* of which used for training */
    uint64_t n_records;
    double loss_first, loss_last;    /* objective before the round's first and after its last Adam step */
    double kish_window;              /* sum w_0 over the used window runs squared / sum w_0^2 */
    float ms_sample, ms_records, ms_optimise;
    int32_t selected;                /* 1 for the round whose end network was returned (select mode;
                                        0 in every round if the starting network was kept) */
    double pilot_ess;                /* select mode: Kish ESS of the window runs of the pilot of the
                                        network this round ended with; NaN otherwise */
} pyfpt_train_report;

/*
 * Train the learned proposal of `inst` (bias.kind = PYFPT_BIAS_MLP; its normalisation,
 * out_scale, eval_every and target_N are used, its params are not): each round draws
 * cfg->n_sample runs from the current network (seed + round), keeps the runs that ended in the
 * window, replays them into records and takes cfg->steps Adam steps on the objective.  theta (host,
 * 4481 binary32) is the starting master copy on entry and the trained one on return (in select
 * mode, the best-scoring of the starting network and the round ends; the pilots use seeds
 * seed + 2^30 + c, c = 0 for the starting network and r + 1 for round r's, so an evaluation on
 * another seed stays unbiased);
 * params_bf16 (host, 4481) receives the bfloat16 copy for pyfpt_run.  report has cfg->rounds
 * entries.  EINVAL for a bad configuration.  The call synchronises.
 */
int pyfpt_train_proposal(const pyfpt_instance *inst, uint64_t seed, const pyfpt_train_config *cfg, float *theta,
                         uint16_t *params_bf16, pyfpt_train_report *report, const pyfpt_options *opt);

/* Number of compute units of the current device, which sets the default grid (0 and
 * EDEVICE if there is none).  EINVAL for a NULL cus. */
int pyfpt_device_cus(int32_t *cus);

/* Message of the calling thread's last failed call (thread-local; owned by the library, valid
 * until that thread's next call). */
const char *pyfpt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PYFPT_H */
