// Internal declarations of the MI355X Monte Carlo TRG library: device
// helpers shared by the HIP kernels and the launchers called by the host
// runtime.  Not part of the public C ABI (see include/mctrg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <utility>
#include <vector>

namespace mctrg {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double kGolden = 1.6180339887498948482;   // gauge weight ratio

// Accumulator layouts of the 16x16 MFMAs (measured on gfx950): lane l,
// register i of the result holds C[row][l % 16] with
//   v_mfma_f64_16x16x4_f64:            row = l/16 + 4*i
//   f32-accumulating 16x16 variants:   row = 4*(l/16) + i
__device__ __forceinline__ int acc_row_f64(int lg, int i) { return lg + 4 * i; }
__device__ __forceinline__ int acc_row_f32(int lg, int i) { return 4 * lg + i; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): four 64-bit counter
// words, two key words, ten rounds of two 64x64->128 multiplies, Weyl key
// schedule.  Counter map of one selection uniform:
//   key = (seed, 0); counter = (sample, position, purpose<<32 | step<<1 |
//   split, m >> 2); word m & 3; u = (word >> 11) * 2^-53.
// ---------------------------------------------------------------------------
struct u64x4 { uint64_t v[4]; };

__device__ __forceinline__ u64x4 philox4x64_10(u64x4 x, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, x.v[0]), lo0 = M0 * x.v[0];
    uint64_t hi1 = __umul64hi(M1, x.v[2]), lo1 = M1 * x.v[2];
    u64x4 y;
    y.v[0] = hi1 ^ x.v[1] ^ k0;
    y.v[1] = lo1;
    y.v[2] = hi0 ^ x.v[3] ^ k1;
    y.v[3] = lo0;
    x = y;
    k0 += W0;
    k1 += W1;
  }
  return x;
}

__device__ __forceinline__ double word_to_uniform(uint64_t w) {
  return (double)(w >> 11) * 0x1.0p-53;
}

// ln(e^a + e^b) with -inf handled exactly.
__device__ __forceinline__ double logaddexp(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  double m = fmax(a, b), d = -fabs(a - b);
  return m + log1p(exp(d));
}

// Order-preserving atomic max of non-negative doubles via their bit pattern.
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline int round_up32(int n) { return ((n + 31) / 32) * 32; }

// ---------------------------------------------------------------------------
// Launchers (host functions, each enqueues on `stream`, returns hipError_t).
// ---------------------------------------------------------------------------

// Initial tensors.
hipError_t launch_init_tensors(int model, int ngroups, const double* beta, const double* h,
                               double* out, hipStream_t stream);
// Gather per-sample starting tensors: T[s] = T0[group[s]] (d0^4 each).
hipError_t launch_gather_tensors(int64_t nsamp, int d0, const double* T0, const int32_t* group,
                                 double* T, hipStream_t stream);

// Unfold: W[j] (n_pad x n_pad, zero padded) = M_split(T[src[j]]), n = D^2.
hipError_t launch_unfold(int64_t njobs, int D, int n_pad, const double* T, const int32_t* src,
                         const int32_t* split, double* W, hipStream_t stream);

// Optional per-kernel timing with HIP events (profiling runs only): each
// timed launch is bracketed by an event pair on its stream; elapsed times
// are collected after the next host synchronisation.
struct KernelTimer {
  double ms = 0.0;
  int64_t launches = 0;
  hipEvent_t ev[2 * 256] = {};
  int used = 0;
  bool enabled = false;
  // optional common origin (not owned): when set, every launch's interval
  // after it is kept, so that launches on several streams can be merged
  hipEvent_t ref = nullptr;
  std::vector<std::pair<float, float>> spans;
  ~KernelTimer() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t begin(hipStream_t s);
  hipError_t end(hipStream_t s);
  hipError_t collect();   // call after the stream has been synchronised
};

// One-sided block Jacobi SVD of W[j] (rows are rotated).  Host-driven sweeps.
// Rows per block of the block Jacobi rotations: 32 (pairs of 64 rows) when
// n_pad is a multiple of 64, else 16.
inline int jacobi_block_rows(int n_pad) { return n_pad % 64 == 0 ? 32 : 16; }
struct JacobiWork {
  int* active;      // njobs
  int* rotated;     // njobs
  int* sweeps;      // njobs (-1 until converged)
  int* counter;      // device 2 ints per slot: jobs still rotating, block pairs rotated in the sweep
  int* counter_host; // pinned host, as many ints as counter
  // optional (64-row pairs): per job and 32-row block, the round stamp of its
  // last rotation (kJacobiMaxBlocks ints), and per block pair the stamp at
  // which it was last found orthogonal (kJacobiMaxBlocks^2 ints); a pair
  // whose blocks have not changed since then is skipped without reading it
  int* lastmod = nullptr;
  int* lastchk = nullptr;
  int hist_len = 1;   // counter slots (pairs of ints) in counter / counter_host
};
constexpr int kJacobiMaxBlocks = 128;   // n_pad / 32 for n_pad <= 4096
// Three approximations of the decomposition drop parts of the matrix below
// the candidate cut: the early stop of the first QR, the rank limit of the
// later QRs and the row deflation before the Jacobi.  Each may drop at most
// approx_budget(tau_null) times s_1 in Frobenius norm (relative to the
// largest column or row norm of its matrix, which is at most s_1), so
// together they move every singular value by at most max(2^-48, tau_null /
// 10) times s_1 (Weyl's inequality; all three perturb M by orthogonal
// transforms of the dropped parts), a tenth of the cut.
inline double approx_budget(double tau_null) { return fmax(0x1.0p-48, 0.1 * tau_null) / 3.0; }
// history (optional, host, max_sweeps x 2): per sweep, the block pairs that
// rotated (summed over jobs) and the jobs still rotating after it.  blind:
// sweeps launched before the first host round trip (needs wk.hist_len >=
// max_sweeps; a sweep after convergence is a launch of idle workgroups).  ncol
// (0: n_pad; a multiple of 64 for the 64-row pairs): the rows are zero from
// column ncol on, so the Gram and the update stop there (rotations keep those
// columns zero).
// tabs / abs_from (abs_from 0: off): from sweep abs_from on, an entry g_ij
// of a pair's Gram no longer counts as unconverged once |g_ij| <= tabs
// max(g_ii, g_jj).  Rows far below the largest ones can stall above the
// relative tolerance: the rounding of the larger rows (about eps times
// their norm) keeps their cosines from falling.  With tabs =
// approx_budget(tau_null) / sqrt(n_pad) the entries left move every
// singular value by at most approx_budget(tau_null) s_1 in all.
hipError_t run_jacobi(int64_t njobs, int n_pad, double* W, const JacobiWork& wk, int max_sweeps,
                      hipStream_t stream, KernelTimer* timer = nullptr, int* sweeps_done = nullptr,
                      const int* nb_job = nullptr, int nb_max = 0, int* history = nullptr, int ncol = 0,
                      int blind = 0, double tabs = 0.0, int abs_from = 0);
// Rank of the rows of W (n_pad x n_pad per job, row-major): *rows_max = the
// largest over the jobs of the smallest L such that the rows from L on hold
// at most approx_budget(tau_null)^2 times the largest squared row norm of
// their job in total (setting them to zero moves no singular value by more
// than approx_budget times s_1).  nrm: n_pad doubles per job, last: one int per job, of
// scratch; synchronises the stream.
hipError_t run_rank_rows(int64_t njobs, int n_pad, double tau_null, const double* W, double* nrm, int* last,
                         int* scratch_dev, int* scratch_host, int* rows_max, hipStream_t stream);
// Per job after the first deflation of the five-QR route: three[j] = 1 when
// its active rows are at most half of n_pad (it stops after three QRs),
// nb_first[j] = its active blocks; *n_five = the jobs that take five
// (synchronises the stream).  launch_keep_three: for those three[j] jobs,
// Wdst <- Wsrc (their deflated rows of R3) and nb_job <- nb_first.
hipError_t run_choose_qr_count(int64_t njobs, int n_pad, const int* nb_job, int* three, int* nb_first,
                               int* scratch_dev, int* scratch_host, int* n_five, hipStream_t stream);
hipError_t launch_keep_three(int64_t njobs, int n_pad, const int* three, const double* Wsrc, double* Wdst,
                             const int* nb_first, int* nb_job, hipStream_t stream);
// Noise-floor deflation: Wout = rows of Win with the active rows (norm >
// approx_budget(tau_null) / sqrt(n_pad) times the largest, so that the rows
// left out hold at most approx_budget^2 times the largest squared norm in
// total) first, in order, the others after them; nb_job = the even number of Jacobi row blocks covering the
// active rows; the maximum over jobs is returned in *nb_max (synchronises the
// stream).  nrm / newpos: n_pad doubles / int32 per job of scratch;
// n_pad <= 4096.
hipError_t run_deflate(int64_t njobs, int n_pad, double tau_null, const double* Win, double* Wout, int* nb_job,
                       double* nrm, int32_t* newpos, int* scratch_dev, int* scratch_host, int* nb_max,
                       hipStream_t stream);
// QR-iteration basis instead of the Jacobi: nrm (n_pad per job) receives the
// squared column norms of the row-major triangular factors R (rows from nrows
// on are zero), W the diagonal matrix of the norms, sigma / order (n per job)
// the norms in descending order and their columns, as after the Jacobi.
hipError_t launch_qr_basis(int64_t njobs, int n, int n_pad, int nrows, const double* R, double* nrm, double* W,
                           double* sigma, int32_t* order, hipStream_t stream);
// QR preconditioning (k_qr.hip): perm[j] (n_pad) orders the columns of the
// unfolding by decreasing norm, the QRs factor M P column-wise.  split 0 / 1:
// the A / B unfolding of a D^4 tensor; split 2: a plain row-major n x n
// matrix.
constexpr int kQrMaxN = 4096;
// Scratch of the blocked QR path per job: two 64 x 64 T factors and the
// 128 x 128 T as 144 MFMA fragments of 64 doubles.
constexpr int64_t kQrBlockScratch = 8192 + 144 * 64;
// Tscr of the five-QR preconditioning per job: two 32 x 32 panel T slots and
// the blocked-path scratch.
constexpr int64_t kQrTscr = 2048 + kQrBlockScratch;
hipError_t launch_iota(int64_t njobs, int n_pad, int32_t* perm, hipStream_t stream);
// Three-QR preconditioning (see k_qr.hip): *rows receives the buffer with
// the rows of R3 (S1); W1 keeps Q2 (V) and Tws2 its panel T factors
// (n_pad * 32 doubles per job).  Tws1 (n_pad * 32 doubles per job) is
// scratch for the panel T factors of the first and third QR.  colmap / colnorm: n_pad int32 / doubles
// per job (the column re-ordering of the first QR, n_pad <= 1024; NULL:
// static order only).
hipError_t run_qr3_precondition(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src,
                                const int32_t* split, int32_t* perm, int32_t* iperm, double* S1, double* Tws1, double* W1,
                                double* Tws2, double* W2, int32_t* colmap, double* colnorm, double** rows,
                                hipStream_t stream);
// Five-QR preconditioning (see k_qr.hip; n_pad <= 1024): the rows of R5 in
// W3; Q2 in W1 / Tws2, Q4 in S1 / Tws4 (n_pad * 32 doubles per job each);
// Tscr: kQrTscr doubles per job of scratch; W2 is free afterwards.  nqr = 3
// stops after the third QR: the rows of R3 in W3 (then v = P Q2 y), W2 still
// holding the factored third QR, so that run_qr45 can continue with the
// fourth and fifth (S1 / Tws4 are not written before).  tq /
// tq_flops (optional, both or neither): a HIP-event timer around every
// 128-column trailing update of the second to fifth QR, and the running sum
// of their algorithmic flops (4 m 128 c + 128^2 c per job for m rows and c
// updated columns).
hipError_t run_qr5_precondition(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src,
                                const int32_t* split, int32_t* perm, int32_t* iperm, double* S1, double* W1, double* Tws2,
                                double* W2, double* Tws4, double* W3, double* Tscr, int32_t* colmap, double* colnorm,
                                hipStream_t stream, KernelTimer* tq = nullptr, double* tq_flops = nullptr,
                                int nqr = 5);
// The same in parts.  run_qr1: the unfolding and the first (re-ordered) QR,
// the rows of R1 in W1.  run_qr23: the second and third QR over the first
// ncols columns (a multiple of 128, or n_pad; the rows of R1 from ncols on
// are set to zero first, so that R2 and R3 are zero outside their leading
// ncols x ncols block; rows_job (or NULL): per job the rank rows of
// run_rank_rows, whose rows from that count rounded up to 128 (the ncols of
// a batch of that job alone) are set to zero instead - ncols is then their
// largest): Q2 in W1 / Tws2 (the T of the panels from column
// ncols on set to zero), the rows of R3 in W3, W2 holding the factored third
// QR.  run_qr45: the fourth and fifth after it, the rows of R5 in W3, Q4 in
// S1 / Tws4.
// stop (or NULL): after every 64 columns of the first QR, a job whose
// columns not yet factored hold (summed squares below the factored rows) at
// most budget^2 times the squared leading diagonal entry of R stops there
// (rows_job[job]: its later rows of R1 are written as zero and its column
// order is frozen; the batch goes on factoring, which leaves its earlier
// rows as they are); the QR ends once every job has stopped, rows = the
// rows factored by then (n_pad if it ran to the end).  dev / host: one int
// of device and pinned host scratch; each check synchronises the stream.
struct QrStop {
  double budget = 0.0;   // approx_budget(tau_null)
  int* dev = nullptr;
  int* host = nullptr;
  int* rows_job = nullptr;   // device, one int per job: the row at which that job stopped (n_pad: none)
  int rows = 0;              // the batch stopped after this many rows (every job stopped at or before)
};
hipError_t run_qr1(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src, const int32_t* split,
                   int32_t* perm, int32_t* iperm, double* S1, double* W1, double* Tscr, int32_t* colmap,
                   double* colnorm, hipStream_t stream, QrStop* stop = nullptr);
hipError_t run_qr23(int64_t njobs, int n_pad, int ncols, double* W1, double* Tws2, double* W2, double* W3,
                    double* Tscr, hipStream_t stream, KernelTimer* tq = nullptr, double* tq_flops = nullptr,
                    const int* rows_job = nullptr);
hipError_t run_qr45(int64_t njobs, int n_pad, int ncols, double* S1, double* W2, double* Tws4, double* W3,
                    double* Tscr, hipStream_t stream, KernelTimer* tq = nullptr, double* tq_flops = nullptr);
// X[:, a] = w_a Q Qb (W[order[sel[a]]] / s) with Q the orthogonal factor
// kept in S1 (V, stored columns via colmap, NULL: identity) and Tws1 (panel
// T), and Qb (optional: S1b / Tws1b, no column map, applied first; n_pad <=
// 1024) a second factor in the same format; nob (or NULL): per job, nonzero
// where Qb is not applied (a job whose decomposition stopped after three QRs)
hipError_t launch_apply_q1(int64_t njobs, int n, int n_pad, int kcap, const double* S1, const int32_t* colmap,
                           const double* Tws1, const double* S1b, const double* Tws1b, const double* W2,
                           const double* sigma, const int32_t* order, const int32_t* kept, const int32_t* sel,
                           const double* weight, double* F, hipStream_t stream, const int* nob = nullptr);
// G[a][perm[colmap[c]]] = X[c][a] (c < n; colmap NULL: identity), signed
// with the gauge of the factor kernels; zero rows for a >= kept.
hipError_t launch_scatter_G(int64_t njobs, int D, int n_pad, int kcap, const double* X, const int32_t* perm,
                            const int32_t* colmap, const int32_t* kept, double* G, hipStream_t stream);
// The same for the step-level SVD: V[a][perm[colmap[c]]] = X[c][a] for n x n
// matrices with columns (i1, i2), gauge over 1 + i1 + phi i2, kcap = n.
hipError_t launch_scatter_V(int64_t nmats, int n, int d2, int n_pad, const double* X, const int32_t* perm,
                            const int32_t* colmap, const int32_t* kept, double* V, hipStream_t stream);
// kept[j] = #{a : sigma[j][a] > 0}, sel[j][a] = a, weight[j][a] = 1 (n per matrix).
hipError_t launch_select_all(int64_t nmats, int n, const double* sigma, int32_t* kept, int32_t* sel, double* weight,
                             hipStream_t stream);

// Norms of the rotated rows, sorted descending: sigma[j][0..n), order[j][0..n).
// nrm (n_pad doubles per job, or NULL): scratch for the squared row norms,
// which are then summed by a grid of one wavefront per row first.
hipError_t launch_jacobi_finalize(int64_t njobs, int n, int n_pad, const double* W, double* sigma,
                                  int32_t* order, hipStream_t stream, double* nrm = nullptr);

// Sampler: chooses kept subsets, inclusion rates and weights.
struct SampleArgs {
  int64_t njobs;
  int n;            // spectrum length per job (sigma stride)
  int k;            // kept count capacity (sel/log_r/weight stride)
  int mode;         // MCTRG_* mode (TOPK => top-k)
  uint64_t seed;
  double tau;
  const double* sigma;
  const uint64_t* rng;     // 3 words per job: sample, position, step
  const int32_t* split;    // per job
  int32_t* kept;
  int32_t* cand;
  int32_t* sel;
  double* log_r;
  double* weight;
  double* scratch;         // njobs * (k+1) * (n+1) * 2 + njobs * n doubles
};
hipError_t launch_sample(const SampleArgs& a, hipStream_t stream);
// The fixed per-device scratch of the allocation-free sampler (k_noalloc.hip):
// its size in doubles, and its device address on the current device (looked
// up once per device with hipGetSymbolAddress).
size_t noalloc_scratch_doubles();
hipError_t noalloc_scratch(double** out);
size_t sample_scratch_doubles(int64_t njobs, int n, int k);

// Factors.  G[j]: kcap x n (row a = w_a v_a), F[j]: kcap x n (row a = w_a u_a,
// stored by kept index so that the contraction reads each u_a contiguously).
hipError_t launch_factor_G(int64_t njobs, int D, int n_pad, int kcap, const double* W,
                           const double* sigma, const int32_t* order, const int32_t* kept,
                           const int32_t* sel, const double* weight, const int32_t* perm, double* G,
                           hipStream_t stream);
hipError_t launch_factor_F(int64_t njobs, int D, int kcap, const double* T, const int32_t* src,
                           const int32_t* split, const double* sigma, const int32_t* kept,
                           const int32_t* sel, const double* G, double* Gt, double* F, hipStream_t stream);

// Contraction of four factors per output tensor.
struct ContractArgs {
  int64_t nout;            // number of output tensors
  int D, kk, dtype;
  const double* GA; const double* GB;   // factor pools indexed by decomposition job
  const double* FA; const double* FB;   // F by kept index: [a][s D + q] per job
  int64_t g_stride, f_stride;           // doubles per job in the G and F pools
  const int32_t* jobs;     // nout x 4: (job of GA, job of GB, job of FA, job of FB)
  double* X; double* Y;    // workspace: nout * kk^2 * D^2 each
  void* Xlp; void* Ylp;    // low-precision copies (bytes: nout * kk^2 * D^2 * elt)
  double* scales;          // nout * 2
  void* Tout;              // nout * kk^4, FP64 (dtype F64) or FP32 (others)
};
hipError_t launch_contract(const ContractArgs& a, hipStream_t stream, KernelTimer* gemm_timer = nullptr);
// out[j][c][e] = in[j][e][c] for e < D^2, c < kk: the F factors of the
// step-level contraction entry ([s][q][c] per job) into the kept-index order.
hipError_t launch_f_by_kept(int64_t njobs, int D, int kk, const double* in, double* out, hipStream_t stream);
// The GEMM tile shape (64 or 128) the autotuner chose for this shape on the
// current device, 0 if none yet.
int gemm_tile_chosen(int dt, int M, int N, int K, int64_t nout);

// T_out = C / (scale_X * scale_Y) in FP64 (C FP64 or FP32).
hipError_t launch_unscale(int64_t nout, int64_t elems, int src_is_f32, const void* C, const double* scales,
                          double* T_out, hipStream_t stream);

// Normalisation: c = max|T'|, T = T'/c, ln c - ln(scales) written to lnc[j].
hipError_t launch_normalize(int64_t nout, int64_t elems, int src_is_f32, const void* Tp,
                            const double* scales, double* cbuf, double* T, double* lnc,
                            hipStream_t stream);

// Final trace and per-sample ln|Z~|.
hipError_t launch_trace(int64_t nsamp, int D, const double* T, const double* lnc_steps, int lnc_stride,
                        int n_steps, int shared_weights, const int* failed, int8_t* sign, double* ln_abs_Z,
                        hipStream_t stream);

// Estimator (single workgroup, deterministic order).
hipError_t launch_estimate(int64_t n, const int8_t* sign, const double* ln_abs, double n_sites,
                           double* out8, hipStream_t stream);

// Chain bookkeeping (k_chain.hip).
hipError_t launch_set_double(double* p, double v, hipStream_t stream);
hipError_t launch_record_positions(int64_t nsamp, int npos, int64_t per_sample, int64_t base, int kmax, int kcap,
                                   const int64_t* idx, const int32_t* cand, const int32_t* kept, const int32_t* sel,
                                   int32_t* rec, hipStream_t stream);
hipError_t launch_record(int64_t nsamp, int step, int n_steps, int kmax, int kcap, const int64_t* idx,
                         const int32_t* cand, const int32_t* kept, const int32_t* sel, int32_t* rec,
                         hipStream_t stream);
hipError_t launch_lnc_accum(int64_t nsamp, int out_per_sample, int step, int n_steps, double mult, const double* lnc,
                            double* lnc_steps, int* failed, hipStream_t stream);
hipError_t launch_jacobi_fail(int64_t njobs, int jobs_per_sample, const int* sweeps, int* failed,
                              hipStream_t stream);
hipError_t launch_izero(int64_t n, int* p, hipStream_t stream);
hipError_t launch_scatter(int64_t nsamp, int n_steps, const int64_t* idx, const int8_t* sign, const double* ln,
                          const double* lnc_steps, int8_t* out_sign, double* out_ln, double* out_lnc,
                          hipStream_t stream);

}  // namespace mctrg
