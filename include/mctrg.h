/*
 * mctrg.h - C ABI of the MI355X (gfx950) Monte Carlo TRG library.
 *
 * Problem (Huggins, Freeman, Stoudenmire, Tubman, Whaley, "Monte Carlo
 * Tensor Network Renormalization", Sections II-III): the trace of a square
 * tensor network is Z.  Each sample coarse-grains the network with TRG
 * (Levin-Nave) where every SVD keeps a random subset of k singular values,
 * drawn with probability p(e) proportional to the product of the squared
 * kept values (Section II, w(e) and p(e)), and divides each kept value by
 * its inclusion rate r(S_ii) (Section II), so that every truncated tensor
 * averages to the exact one (Eqs. Tsum, Ssum) and the mean of the sample
 * traces estimates Z without bias (Section III, Eqs. infiniteSum and
 * infiniteEnsemble).  The error of the mean falls as 1/sqrt(samples)
 * (Section V, Eq. shrunkDev).
 *
 * Conventions shared by every call
 *   - Every function returns an int status: MCTRG_OK (0) or a negative
 *     MCTRG_E* code.  No C++ exception crosses the ABI.
 *   - Argument errors are detected before any work is enqueued; the call
 *     then returns MCTRG_EINVAL and leaves every output untouched.
 *   - "device" pointers are HIP device allocations (for example from
 *     torch tensors on cuda:0); "host" pointers are ordinary host memory.
 *     The caller owns every pointer it passes; the library owns its tensor
 *     sets and their workspace.
 *   - hip_stream is a hipStream_t (NULL = default stream).  Calls block
 *     until their results are written unless a flag says otherwise.
 *   - Tensors are FP64, row-major with legs ordered [l][u][r][d].
 *   - Decompositions, sampling probabilities, inclusion rates and the
 *     running log-normalisation are always FP64; only the large coarse-
 *     graining GEMM takes the contraction dtype.
 *   - A tensor set is not thread-safe; use one per host thread / stream.
 */
#ifndef MCTRG_H
#define MCTRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mctrg_status {
  MCTRG_OK = 0,
  MCTRG_EINVAL = -1,       /* invalid argument; nothing was enqueued          */
  MCTRG_ENOMEM = -2,       /* device workspace could not be allocated         */
  MCTRG_EDEVICE = -3,      /* HIP runtime or kernel launch error              */
  MCTRG_ENUMERIC = -4,     /* some samples failed numerically (see outputs)   */
  MCTRG_EUNSUPPORTED = -5  /* valid but not implemented combination           */
};

/* Initial tensor constructions (all with legs l,u,r,d and bond dimension 2,
 * leg index 0 <-> spin +1 where a leg carries a spin):
 *   MCTRG_ISING_SITE      one tensor per spin of the square-lattice Ising
 *                         model (Section IV, Eq. ising_model): every bond
 *                         weight exp(beta s s') is split symmetrically into
 *                         two half-bonds W = [[sqrt cosh b, sqrt sinh b],
 *                         [sqrt cosh b, -sqrt sinh b]], and the field factor
 *                         exp(beta h s) sits on the spin.  An L x L torus of
 *                         these tensors traces to Z of the L x L Ising torus.
 *   MCTRG_ISING_PLAQUETTE spins on the network bonds; every tensor holds the
 *                         four interactions between cyclically adjacent leg
 *                         spins (Section III, Fig. 1), field split in half.
 *   MCTRG_USER            caller-provided tensors.                           */
enum mctrg_model { MCTRG_ISING_SITE = 0, MCTRG_ISING_PLAQUETTE = 1, MCTRG_USER = 2 };

/* Estimator forms:
 *   MCTRG_SHARED       one random tensor per level per sample: every tensor
 *                      of a level equals the same sampled tensor (a
 *                      translation-invariant chain whose cost is logarithmic
 *                      in the number of sites).  Biased for Z in general,
 *                      because the paper requires independent samples per
 *                      tensor (Section III, the paragraph after
 *                      Eq. infiniteEnsemble); provided because it is the
 *                      only form feasible on 2^20..2^30 sites.
 *   MCTRG_INDEPENDENT  the paper's estimator: every tensor of every level on
 *                      an L x L torus (L = 2^(n_steps/2)) gets its own
 *                      independent truncation; unbiased.
 *   MCTRG_TOPK         deterministic TRG keeping the k largest singular
 *                      values (Section II, Eq. approxSVD), shared form.      */
enum mctrg_mode { MCTRG_SHARED = 0, MCTRG_INDEPENDENT = 1, MCTRG_TOPK = 2 };

/* dtype of the coarse-graining GEMM (FP32 accumulation for the narrow ones,
 * with one power-of-two scale per operand tensor and sample). */
enum mctrg_dtype { MCTRG_F64 = 0, MCTRG_F32 = 1, MCTRG_BF16 = 2, MCTRG_FP8_E4M3 = 3 };

/* Decomposition of each unfolding M:
 *   MCTRG_DEC_SVD  the exact FP64 SVD (Section II, Eq. exactSVD; default);
 *   MCTRG_DEC_QR3, MCTRG_DEC_QR5  a cheaper decomposition that keeps the
 *                  estimator unbiased: an orthonormal basis V from three
 *                  (five) steps of QR iteration (M P = Q1 R1 with column
 *                  re-ordering, R_i^T = Q_{i+1} R_{i+1}, V = P Q2 (Q4)) and
 *                  the exact expansion M = sum_j (M v_j) v_j^T, whose terms
 *                  are drawn and reweighted as the SVD terms are (Section II
 *                  needs only inclusion rates r > 0 for Eqs. Tsum, Ssum), with
 *                  weights |M v_j| = the column norms of the last R.  No
 *                  Jacobi; the variance of the samples grows where V is
 *                  far from the singular vectors.  k <= 32 (unfoldings of at
 *                  most 1024 rows). */
enum mctrg_decomposition { MCTRG_DEC_SVD = 0, MCTRG_DEC_QR3 = 1, MCTRG_DEC_QR5 = 2 };

/* flags */
#define MCTRG_RECORD 1u   /* write per-step selection records to record_buf   */
                          /* (bit 2u is not used)                              */
#define MCTRG_PROFILE 4u  /* chains: time the decomposition and GEMM kernels  */
                          /* with HIP events (see mctrg_chain_get_profile)     */
#define MCTRG_ONE_STREAM 8u  /* run every wave as one part on hip_stream (see */
                             /* "Parts" below)                                  */

typedef struct mctrg_tensor_set mctrg_tensor_set;  /* opaque, library-owned */

/* Build the initial tensors of n_groups (beta, h) groups on the current HIP
 * device.  beta, h: host arrays of n_groups values (beta >= 0).
 * For MCTRG_USER, d_user is the bond dimension (2..4) and user_T a host
 * array of n_groups * d_user^4 FP64 values (row-major [g][l][u][r][d]),
 * copied; beta and h may then be NULL.  *out receives the new set.
 * Errors: EINVAL (bad model, n_groups < 1, beta < 0 or non-finite, missing
 * arrays), ENOMEM, EDEVICE. */
int mctrg_init_tensor(int model, int32_t n_groups, const double* beta, const double* h,
                      int32_t d_user, const double* user_T, mctrg_tensor_set** out);

/* Number of groups and bond dimension of a set; 0 on success. */
int mctrg_tensor_set_info(const mctrg_tensor_set* ts, int32_t* n_groups, int32_t* d0);

typedef struct {
  uint64_t seed;           /* Philox4x64-10 key word 0                               */
  int64_t sample_offset;   /* global sample id of output i = sample_offset + i        */
  int32_t n_steps;         /* N = 2^n_steps sites, 1..40; independent mode: even, <= 12 */
  int32_t k;               /* kept count per decomposition, 1..64                     */
  int32_t mode;            /* enum mctrg_mode                                         */
  int32_t contract_dtype;  /* enum mctrg_dtype                                        */
  double tau_null;         /* singular values <= tau_null * s_1 count as zero (1e-11) */
                           /*   and are never drawn; rows of the decomposition below */
                           /*   max(2^-48, tau_null / 10) of the largest row are not */
                           /*   rotated (their values stay below the cut).  With a  */
                           /*   narrow contraction dtype the rounding of T' gives    */
                           /*   singular values near its unit roundoff times s_1     */
                           /*   (1e-8..1e-7 for F32) that carry no signal: a cut     */
                           /*   above them (1e-6 for F32) drops them from both the   */
                           /*   candidates and the rotations.                        */
  uint32_t flags;          /* MCTRG_RECORD | MCTRG_PROFILE | MCTRG_ONE_STREAM         */
  int32_t* record_buf;     /* device int32, or NULL; with MCTRG_RECORD the kept sets: */
                           /*   shared / top-k: n_samples * n_steps * (4 + 2k):       */
                           /*   per step cA, cB (candidates), kA, kB (kept), selA[k], */
                           /*   selB[k] (kept indices into the descending spectrum,   */
                           /*   -1 padded);                                           */
                           /*   independent: n_samples * sum_s 2^(n_steps-s) * (2+k): */
                           /*   per step s, per position p of its level (in position  */
                           /*   order: the rank of the originating A-site id), c,     */
                           /*   kept, sel[k] of that tensor's one decomposition.      */
  double* out_tensor;      /* device or NULL: final normalised tensor of every sample */
                           /*   (shared/top-k), n_samples * Dc^4 with Dc the capacity */
                           /*   bond dimension after n_steps (mctrg_capacity_dim)     */
  size_t max_workspace_bytes; /* device workspace the library may hold at once:      */
                           /*   0 = 70% of the free device memory; waves of samples   */
                           /*   are sized to fit; ENOMEM (outputs untouched) when one */
                           /*   sample does not fit                                   */
  int32_t n_det;           /* 0..n_steps: the first n_det steps are deterministic     */
                           /*   (top-k: the first min(k, c) values, r = 1), the rest  */
                           /*   stochastic (Section V, Discussion: deterministic       */
                           /*   coarse-graining steps before switching to Monte Carlo */
                           /*   for translation-invariant systems).  Independent mode:*/
                           /*   the prefix coarse-grains one tensor per sample, whose */
                           /*   result starts every position of level n_det, from     */
                           /*   where each tensor is sampled on its own; out_ln_c of a*/
                           /*   prefix step is the sum over the level's equal tensors.*/
                           /*   Unbiased for Z when every prefix step keeps all its   */
                           /*   candidates (c <= k); otherwise for the network left  */
                           /*   by the deterministic truncation.  Default 0.          */
  int32_t decomposition;   /* enum mctrg_decomposition (default MCTRG_DEC_SVD)         */
} mctrg_run_config;

/* Fill *cfg with the defaults (seed 0, offset 0, tau_null 1e-11, F64, shared). */
void mctrg_default_config(mctrg_run_config* cfg);

/* Bond dimension of the stored tensors after n_steps steps at kept count k,
 * starting from bond dimension d0: D_0 = d0, D_{s+1} = min(k, D_s^2).
 * Kept counts below the capacity are zero-padded. */
int32_t mctrg_capacity_dim(int32_t d0, int32_t k, int32_t n_steps);

/* Parts: a wave of n samples runs as min(3, n) parts of consecutive samples
 * (as equal as possible), each with its own device workspace and stream (the
 * first on hip_stream, the others on non-blocking streams of default
 * priority that the library creates and destroys), advanced concurrently by
 * one host thread each, so that the kernels of some parts fill the GPU while
 * another waits on a convergence count or runs latency-bound QR panels.
 * hip_stream waits for all parts before a call returns or completes.
 * Results do not depend on the split (bit for bit, see below);
 * MCTRG_ONE_STREAM keeps one part.
 *
 * Run n_samples independent Monte Carlo samples (Section III).
 *   group_of_sample: host, n_samples group indices, or NULL (all group 0)
 *   k_of_sample:     host, n_samples kept counts, or NULL (all cfg->k);
 *                    samples are bucketed by k internally
 *   out_sign:        device int8, n_samples: sign of Z~ (0 = failed sample)
 *   out_ln_abs_Z:    device FP64, n_samples: ln|Z~| (NaN for failed)
 *   out_ln_c:        device FP64 or NULL, n_samples * n_steps: per-step
 *                    ln of the normalisation (shared: max|T'| of the one
 *                    tensor; independent: sum over the level's tensors)
 * Per-sample results depend only on (seed, global sample id, group, k,
 * n_steps, mode, dtype, tau_null, n_det, decomposition), bit for bit: every
 * random draw is addressed by the global sample id, and the decomposition's
 * early QR stop, rank limit, number of QR steps and deflation are decided
 * per decomposition (a batch runs its kernels to the largest extent, where
 * the parts a decomposition has dropped are exact zeros), so neither the
 * other samples of the batch, nor the waves, parts or buckets change a
 * sample.  Samples of different k run as concurrent buckets.
 * Returns ENUMERIC if any sample failed (its sign is 0, its ln|Z~| NaN: a
 * non-finite normalisation, a zero trace or a decomposition that did not
 * converge); the other samples are valid.  Blocks until the outputs are
 * written.  Errors: EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED.
 * Test hook (here and in mctrg_chain_create): when the environment variable
 * MCTRG_TEST_FAIL_SAMPLE holds a global sample id, that sample's
 * normalisation at the last step is made non-finite (the failure path above, without feeding a non-finite value
 * through the decomposition kernels). */
int mctrg_run_samples(mctrg_tensor_set* ts, const mctrg_run_config* cfg, int64_t n_samples,
                      const int32_t* group_of_sample, const int32_t* k_of_sample,
                      int8_t* out_sign, double* out_ln_abs_Z, double* out_ln_c,
                      void* hip_stream);

typedef struct {
  double ln_meanZ_per_site;  /* ln(mean of signed Z~) / n_sites (NaN if mean <= 0)   */
  double rel_stderr_Z;       /* stderr of the mean of Z~ over |mean|                 */
  double mean_lnZ_per_site;  /* mean of ln|Z~| / n_sites                             */
  double stderr_mean_lnZ;    /* its standard error                                   */
  int64_t n_used, n_negative, n_failed;
} mctrg_estimate;

/* Monte Carlo estimate from per-sample results (Section III
 * Eq. infiniteEnsemble; error bars per Section V Eq. shrunkDev), computed on
 * the device with a signed log-sum-exp.  sign, ln_abs_Z: device arrays of
 * n_samples (samples with sign 0 or non-finite ln are excluded and
 * counted as failed).  *out is written on the host.  Blocks on hip_stream. */
int mctrg_estimate_lnZ(int64_t n_samples, const int8_t* sign, const double* ln_abs_Z,
                       double n_sites, mctrg_estimate* out, void* hip_stream);

/* ---- Stepping interface (one wave of samples, one kept count) ----------
 * The same per-sample chain as mctrg_run_samples, advanced step by step:
 * create gathers the starting tensors of n_samples samples (ids
 * cfg->sample_offset + i, groups from the host array group_of_sample or 0)
 * and allocates the device workspace; step applies n TRG steps (at most
 * cfg->n_steps in total); finish traces the current tensor - after s
 * steps this is the sample of Z for the 2^s-site lattice - and writes
 * sign / ln|Z~| / ln c (device arrays, n_samples and n_samples *
 * cfg->n_steps; out_ln_c may be NULL).  Errors as mctrg_run_samples (finish
 * returns ENUMERIC when some sample failed, its sign 0 and ln|Z~| NaN);
 * MCTRG_RECORD writes cfg->record_buf as mctrg_run_samples does (sample i
 * of the chain at index i); out_tensor is ignored here. */
typedef struct mctrg_chain mctrg_chain;
int mctrg_chain_create(mctrg_tensor_set* ts, const mctrg_run_config* cfg, int64_t n_samples,
                       const int32_t* group_of_sample, void* hip_stream, mctrg_chain** out);
int mctrg_chain_step(mctrg_chain* ch, int32_t n);
int mctrg_chain_finish(mctrg_chain* ch, int8_t* out_sign, double* out_ln_abs_Z, double* out_ln_c);
/* The current normalised tensor T-hat of every sample after the steps done
 * so far (Section III: the coarse tensor of the last step, divided by its
 * largest |entry|): out (device FP64, caller-owned) receives n_samples * D^4
 * values, sample i at offset i * D^4, legs [l][u][r][d] row-major, with D =
 * mctrg_capacity_dim(d0, k, steps done).  Shared and top-k chains only
 * (EUNSUPPORTED in independent mode).  Blocks until the copy is done. */
int mctrg_chain_tensor(const mctrg_chain* ch, double* out);

typedef struct {
  double jacobi_ms;         /* summed duration of the Jacobi rotation kernels    */
  int64_t jacobi_launches;  /* number of those launches                          */
  double gemm_ms;           /* summed duration of the coarse-graining GEMMs      */
  int64_t gemm_launches;
  int32_t steps_done;
  int32_t last_sweeps;      /* Jacobi sweeps used by the last step               */
  int32_t last_pairs[64];   /* last step, per sweep: block pairs that rotated,
                               summed over all decompositions of the step       */
  int32_t last_active[64];  /* last step, per sweep: decompositions still
                               rotating after that sweep                        */
  double jacobi_busy_ms;    /* union of the Jacobi launch intervals over all
                               parts (launches of the parts overlap in time)     */
  double gemm_busy_ms;      /* the same for the GEMMs                            */
  int32_t parts;            /* parts of the chain (1 to 3)                       */
  int32_t step_sweeps[64];  /* Jacobi sweeps of every step done (the most over
                               the step's decompositions), steps 0..63          */
  double qr128_ms;          /* summed duration of the 128-column trailing updates
                               of the second to fifth QR (qr_trailing128)        */
  int64_t qr128_launches;   /* number of those launches                          */
  double qr128_busy_ms;     /* union of their intervals over all parts           */
  double qr128_flops;       /* their algorithmic flops: per job and launch
                               4 m 128 c + 128^2 c (m rows, c columns updated)  */
  int64_t jacobi_rotated_pairs; /* block pairs (2 x 32 rows) rotated by the
                               Jacobi, summed over all steps and sweeps         */
  double jacobi_flops;      /* their algorithmic flops: per rotated pair of
                               r = 64 rows the Gram r^2 len and the update
                               2 r^2 len, len = the row length rotated (the
                               columns up to the rank limit of the QRs)        */
} mctrg_chain_profile;
/* Timings are collected only when cfg->flags has MCTRG_PROFILE. */
int mctrg_chain_get_profile(const mctrg_chain* ch, mctrg_chain_profile* out);
void mctrg_chain_destroy(mctrg_chain* ch);

void mctrg_destroy(mctrg_tensor_set* ts);
const char* mctrg_status_string(int status);

/* ---- Step-level entry points (the individual steps of one TRG step) ----
 * An empty batch (n_mats or n_jobs = 0) with otherwise valid sizes returns
 * MCTRG_OK without reading or writing anything (its pointers may be NULL). */

/* Decomposition step (Section II, Eq. exactSVD): FP64 SVD of n_mats square
 * n x n matrices (device, row-major, n_mats * n * n), n = d1 * d2 <= 4096 with
 * the column index j = i1 * d2 + i2, by the same route and with the same
 * approximations as every chain step: a column-re-ordered QR that stops at
 * the numerical rank, two or four more QRs over the leading columns, the
 * deflation of rows below the budget, block one-sided Jacobi on the rest.
 * tau_null (0 <= tau_null < 1) is the candidate cut of the sampler: the parts
 * of M the approximations drop total at most max(2^-48, tau_null / 10) * s_1
 * in Frobenius norm, which bounds the error of every singular value (Weyl's
 * inequality); tau_null = 0 keeps M to the rounding floor.
 * sigma_out: device, n_mats * n, descending (values beyond the numerical
 * rank are 0).
 * V_out: device or NULL, n_mats * n * n, row i = the i-th right singular
 * vector, signed so that sum_j V[i][j] / (1 + i1 + phi*i2) > 0 (phi = golden
 * ratio); rows of zero values are zero, and rows of values below the budget
 * are accurate only to budget / (their distance to the other values).
 * sweeps_out: device or NULL, n_mats int32 Jacobi sweeps used (-1 = no
 * convergence).  Allocates its workspace (about 4 n_pad^2 doubles per
 * matrix, n_pad = n rounded up to 32, plus n^2 with V_out).  Blocks on
 * hip_stream.  Errors: EINVAL, ENOMEM, EDEVICE. */
int mctrg_svd_batched(int64_t n_mats, int32_t d1, int32_t d2, const double* M, double tau_null,
                      double* sigma_out, double* V_out, int32_t* sweeps_out, void* hip_stream);

/* Sampling and reweighting step (Section II): for each of n_jobs descending
 * spectra sigma (device, n_jobs * n) choose the kept subset: mode
 * MCTRG_TOPK keeps the first min(k, c); otherwise a subset drawn from
 * p(e) ~ prod s^2 when c > k (c = #{s > tau_null * s_1}), else all c.
 * rng: device, n_jobs * 3 uint64 (sample id, position id, step) naming the
 * Philox counters; split: device int32 per job (0 = A, 1 = B).
 * Outputs (device): kept[n_jobs], cand[n_jobs], sel[n_jobs*k] (ascending
 * indices, -1 padded), log_r[n_jobs*k] (ln inclusion rate), weight
 * [n_jobs*k] (sqrt(s/r)).  Blocks on hip_stream. */
int mctrg_sample_batched(int64_t n_jobs, int32_t n, int32_t k, int32_t mode, uint64_t seed,
                         double tau_null, const double* sigma, const uint64_t* rng,
                         const int32_t* split, int32_t* kept, int32_t* cand, int32_t* sel,
                         double* log_r, double* weight, void* hip_stream);

/* mctrg_sample_batched without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, kernel and results.
 * The draw's tables live in a fixed per-device scratch array of 64 MiB
 * (8,388,608 doubles), which each device holds until the process ends; a
 * call needs n_jobs * (2 (k+1) (n+1) + n + 8) doubles of it (e.g. 122 jobs at
 * n = 1024, k = 32) and returns ENOMEM, with nothing enqueued, beyond that.
 * Nothing in the scratch must start at zero (every table entry is written
 * before it is read).  Calls on one device share its scratch: calls that
 * overlap in time on one device (several host threads or streams) race.
 * Blocks on hip_stream.  Errors: EINVAL, ENOMEM, EDEVICE. */
int mctrg_sample_batched_noalloc(int64_t n_jobs, int32_t n, int32_t k, int32_t mode, uint64_t seed,
                                 double tau_null, const double* sigma, const uint64_t* rng,
                                 const int32_t* split, int32_t* kept, int32_t* cand, int32_t* sel,
                                 double* log_r, double* weight, void* hip_stream);

/* Contraction step (Section III, Levin-Nave TRG): for each job,
 *   T'[a,b,c,e] = sum_{p,q,s,t} GA[a,p,t] GB[b,q,p] FA[s,q,c] FB[t,s,e]
 * with GA, GB: kk x D x D, FA, FB: D x D x kk (device, FP64, per job
 * contiguous).  T_out: device FP64, n_jobs * kk^4.  dtype selects the
 * precision of the kk^2 x kk^2 x D^2 GEMM.  Blocks on hip_stream.
 * The GEMM's tile shape (64 x 64 or 128 x 128 per workgroup) is chosen by
 * timing both on the first GEMM of each (dtype, shape, batch) on a device
 * (also inside the chains); the environment variable MCTRG_GEMM_TILE = 64
 * or 128 forces one (a test hook). */
int mctrg_contract_batched(int64_t n_jobs, int32_t D, int32_t kk, int32_t dtype,
                           const double* GA, const double* GB, const double* FA,
                           const double* FB, double* T_out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MCTRG_H */
