// Sampling and reweighting step (paper Section II): choose the kept subset
// e of the nonzero singular values with p(e) = w(e)/sum w, w(e) = prod s^2,
// and reweight every kept value by 1/r(S_ii), r(S_ii) = sum_{e containing i}
// p(e).  The paper defers the sampler to Ferris (2015) and states an
// O(chi * chi-tilde) cost; this kernel uses the elementary-symmetric-
// polynomial (ESP) sequential draw, which has that cost and samples p(e)
// exactly:
//   lambda_m = (s_m / s_1)^2 over the c candidates s_m > tau * s_1,
//   LS[m][j] = ln e_j(lambda_m .. lambda_{c-1})  (suffix table, m = c..0),
//   walk m = 0, 1, ...: with rem values still to choose, keep m with
//   probability exp(ln lambda_m + LS[m+1][rem-1] - LS[m][rem]) (forced when
//   rem = c - m), one Philox uniform per candidate index;
//   ln r_i = ln lambda_i + ln sum_a e_a(prefix before i) e_{k-1-a}(suffix
//   after i) - LS[0][k]  (prefix table LP built up to the last kept index).
// One wavefront per decomposition: lane j-1 owns column j of the tables
// (k <= 64), the rows advance sequentially over m; tables live in global
// scratch ((c+1) x (k+1) doubles each, row-major over j for coalescing).
#include "mctrg_internal.h"
#include "../../include/mctrg.h"

namespace mctrg {

size_t sample_scratch_doubles(int64_t njobs, int n, int k) {
  return (size_t)njobs * (2 * (size_t)(k + 1) * (n + 1) + (size_t)n + 8);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__global__ __launch_bounds__(64) void sample_kernel(SampleArgs a) {
  const int64_t job = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = a.n, k = a.k;
  const double* sig = a.sigma + job * n;
  int32_t* sel = a.sel + job * k;
  double* log_r = a.log_r + job * k;
  double* wt = a.weight + job * k;

  const double s0 = sig[0];
  int cl = 0;
  if (s0 > 0.0 && isfinite(s0)) {
    const double thr = a.tau * s0;
    for (int i = lane; i < n; i += 64) cl += (sig[i] > thr) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) cl += __shfl_xor(cl, o);
  const int c = cl;
  if (lane == 0) a.cand[job] = c;

  if (c <= k || a.mode == MCTRG_TOPK) {
    const int kk = c < k ? c : k;
    for (int j = lane; j < k; j += 64) {
      if (j < kk) { sel[j] = j; log_r[j] = 0.0; wt[j] = sqrt(sig[j]); }
      else { sel[j] = -1; log_r[j] = 0.0; wt[j] = 0.0; }
    }
    if (lane == 0) a.kept[job] = kk;
    return;
  }

  const size_t stride = 2 * (size_t)(k + 1) * (n + 1) + (size_t)n + 8;
  double* LS = a.scratch + job * stride;            // (c+1) x (k+1)
  double* LP = LS + (size_t)(k + 1) * (n + 1);       // (c+1) x (k+1)
  double* U = LP + (size_t)(k + 1) * (n + 1);        // c uniforms
  const int K1 = k + 1;

  // ---- uniforms: counter (sample, position, step<<1 | split, m>>2) ------
  const uint64_t sid = a.rng[3 * job + 0], pos = a.rng[3 * job + 1], stp = a.rng[3 * job + 2];
  const uint64_t w2 = (stp << 1) | (uint64_t)(a.split[job] & 1);   // purpose 0
  for (int blk = lane; blk < (c + 3) / 4; blk += 64) {
    u64x4 x;
    x.v[0] = sid; x.v[1] = pos; x.v[2] = w2; x.v[3] = (uint64_t)blk;
    u64x4 y = philox4x64_10(x, a.seed, 0ull);
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (4 * blk + w < c) U[4 * blk + w] = word_to_uniform(y.v[w]);
  }

  // The sequential loops below take ln lambda_m (and the uniforms) from
  // registers: 64 consecutive indices at a time, one per lane, read back by
  // shuffles, so that no global load or logarithm sits on their critical path.
  auto ln_lambda = [&](int m) { return m >= 0 && m < c ? 2.0 * log(sig[m] / s0) : 0.0; };

  // ---- suffix table ------------------------------------------------------
  const int j = lane + 1;                 // column owned by this lane
  double prev = -INFINITY;                // LS[c][j], j >= 1
  if (lane == 0) LS[(size_t)c * K1] = 0.0;
  if (j <= k) LS[(size_t)c * K1 + j] = -INFINITY;
  for (int m1 = c - 1; m1 >= 0; m1 -= 64) {    // indices m1, m1 - 1, ..., m1 - 63
    const double lmc = ln_lambda(m1 - lane);
    for (int d = 0; d < 64 && m1 - d >= 0; ++d) {
      const int m = m1 - d;
      const double lm = __shfl(lmc, d);
      double left = __shfl_up(prev, 1);   // LS[m+1][j-1]
      if (lane == 0) left = 0.0;
      const double cur = logaddexp(prev, lm + left);
      prev = cur;
      if (j <= k) LS[(size_t)m * K1 + j] = cur;
      if (lane == 0) LS[(size_t)m * K1] = 0.0;
    }
  }
  __threadfence_block();
  __syncthreads();

  // ---- sequential draw (wave-uniform walk) --------------------------------
  // rows m and m + 1 of LS sit in the lanes (lane j: column j), loaded one
  // row ahead; column 64 (k = 64 only) has no lane and is loaded when needed
  int rem = k, nsel = 0, last = -1;
  auto ls_row = [&](int m) { return (m <= c && lane < K1) ? LS[(size_t)m * K1 + lane] : 0.0; };
  double row0 = ls_row(0), row1 = ls_row(1);
  for (int m0 = 0; m0 < c && rem > 0; m0 += 64) {
    const double lmc = ln_lambda(m0 + lane);
    const double uc = m0 + lane < c ? U[m0 + lane] : 0.0;
    for (int d = 0; d < 64 && m0 + d < c && rem > 0; ++d) {
      const int m = m0 + d;
      const double row2 = ls_row(m + 2);
      bool take;
      if (rem == c - m) {
        take = true;
      } else {
        const double lm = __shfl(lmc, d);
        const double a1 = __shfl(row1, rem - 1);                                     // LS[m+1][rem-1]
        const double a0 = rem < 64 ? __shfl(row0, rem) : LS[(size_t)m * K1 + rem];   // LS[m][rem]
        const double q = exp(lm + a1 - a0);
        take = __shfl(uc, d) < q;
      }
      if (take) {
        if (lane == 0) sel[nsel] = m;
        ++nsel;
        --rem;
        last = m;
      }
      row0 = row1;
      row1 = row2;
    }
  }
  for (int t = nsel + lane; t < k; t += 64) sel[t] = -1;   // (nsel == k always)
  if (lane == 0) a.kept[job] = nsel;

  // ---- prefix table up to the last kept index -----------------------------
  prev = -INFINITY;                       // LP[0][j], j >= 1
  if (lane == 0) LP[0] = 0.0;
  if (j <= k) LP[j] = -INFINITY;
  for (int m0 = 0; m0 < last; m0 += 64) {
    const double lmc = ln_lambda(m0 + lane);
    for (int d = 0; d < 64 && m0 + d < last; ++d) {
      const int m = m0 + d;
      const double lm = __shfl(lmc, d);
      double left = __shfl_up(prev, 1);   // LP[m][j-1]
      if (lane == 0) left = 0.0;
      const double cur = logaddexp(prev, lm + left);
      prev = cur;
      if (j <= k) LP[(size_t)(m + 1) * K1 + j] = cur;
      if (lane == 0) LP[(size_t)(m + 1) * K1] = 0.0;
    }
  }
  __threadfence_block();
  __syncthreads();

  // ---- inclusion rates and weights of the kept values ----------------------
  const double lek = LS[k];               // LS[0][k] = ln e_k(all)
  for (int t = 0; t < nsel; ++t) {
    const int i = sel[t];
    double term = -INFINITY;
    if (lane < k) term = LP[(size_t)i * K1 + lane] + LS[(size_t)(i + 1) * K1 + (k - 1 - lane)];
    const double mx = wave_max(term);
    double e = (lane < k && mx > -INFINITY) ? exp(term - mx) : 0.0;
    e = wave_sum(e);
    const double lr = 2.0 * log(sig[i] / s0) + (mx + log(e)) - lek;
    if (lane == 0) {
      log_r[t] = lr;
      wt[t] = sqrt(sig[i] * exp(-lr));
    }
  }
  for (int t = nsel + lane; t < k; t += 64) { log_r[t] = 0.0; wt[t] = 0.0; }
}

hipError_t launch_sample(const SampleArgs& a, hipStream_t stream) {
  if (a.njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)a.njobs), dim3(64), 0, stream, a);
  return hipGetLastError();
}

}  // namespace mctrg
