// Per-chain bookkeeping kernels: selection records, per-sample sums of the
// normalisation logs, failure flags and scatter of results to the caller's
// sample order.
#include "mctrg_internal.h"

namespace mctrg {

// record[(idx[s] * n_steps + step) * (4 + 2*kmax) + ...] = cA, cB, kA, kB, selA[kmax], selB[kmax]
__global__ void record_kernel(int64_t nsamp, int step, int n_steps, int kmax, int kcap,
                              const int64_t* __restrict__ idx, const int32_t* __restrict__ cand,
                              const int32_t* __restrict__ kept, const int32_t* __restrict__ sel,
                              int32_t* __restrict__ rec) {
  const int64_t s = blockIdx.x;
  const int stride = 4 + 2 * kmax;
  int32_t* r = rec + ((size_t)idx[s] * n_steps + step) * stride;
  const int64_t jA = 2 * s, jB = 2 * s + 1;
  for (int t = threadIdx.x; t < stride; t += blockDim.x) {
    int32_t v;
    if (t == 0) v = cand[jA];
    else if (t == 1) v = cand[jB];
    else if (t == 2) v = kept[jA];
    else if (t == 3) v = kept[jB];
    else {
      const int q = t - 4;
      const int64_t j = q < kmax ? jA : jB;
      const int a = q < kmax ? q : q - kmax;
      v = a < kcap ? sel[j * kcap + a] : -1;
    }
    r[t] = v;
  }
}

hipError_t launch_record(int64_t nsamp, int step, int n_steps, int kmax, int kcap, const int64_t* idx,
                         const int32_t* cand, const int32_t* kept, const int32_t* sel, int32_t* rec,
                         hipStream_t stream) {
  if (nsamp == 0) return hipSuccess;
  hipLaunchKernelGGL(record_kernel, dim3((unsigned)nsamp), dim3(64), 0, stream, nsamp, step, n_steps, kmax, kcap,
                     idx, cand, kept, sel, rec);
  return hipGetLastError();
}

// Independent mode: rec[idx[s] * per_sample + base + p * (2 + kmax) + ...] =
// c, kept, sel[kmax] of the decomposition at position p of this step's level
// (jobs s * npos + p), -1 padded.
__global__ void record_positions_kernel(int npos, int64_t per_sample, int64_t base, int kmax, int kcap,
                                        const int64_t* __restrict__ idx, const int32_t* __restrict__ cand,
                                        const int32_t* __restrict__ kept, const int32_t* __restrict__ sel,
                                        int32_t* __restrict__ rec) {
  const int64_t s = blockIdx.y;
  const int p = blockIdx.x;
  const int stride = 2 + kmax;
  const int64_t j = s * npos + p;
  int32_t* r = rec + (size_t)idx[s] * per_sample + base + (int64_t)p * stride;
  for (int t = threadIdx.x; t < stride; t += blockDim.x) {
    int32_t v;
    if (t == 0) v = cand[j];
    else if (t == 1) v = kept[j];
    else v = (t - 2) < kcap ? sel[j * kcap + (t - 2)] : -1;
    r[t] = v;
  }
}

hipError_t launch_record_positions(int64_t nsamp, int npos, int64_t per_sample, int64_t base, int kmax, int kcap,
                                   const int64_t* idx, const int32_t* cand, const int32_t* kept, const int32_t* sel,
                                   int32_t* rec, hipStream_t stream) {
  if (nsamp == 0 || npos == 0) return hipSuccess;
  hipLaunchKernelGGL(record_positions_kernel, dim3((unsigned)npos, (unsigned)nsamp), dim3(64), 0, stream, npos,
                     per_sample, base, kmax, kcap, idx, cand, kept, sel, rec);
  return hipGetLastError();
}

// lnc_steps[s * n_steps + step] = mult * sum over the sample's outputs (fixed
// order); failed[s] |= any non-finite.
__global__ void lnc_accum_kernel(int64_t nsamp, int out_per_sample, int step, int n_steps, double mult,
                                 const double* __restrict__ lnc, double* __restrict__ lnc_steps,
                                 int* __restrict__ failed) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nsamp) return;
  double acc = 0.0;
  for (int P = 0; P < out_per_sample; ++P) acc += lnc[s * out_per_sample + P];
  acc *= mult;
  lnc_steps[s * n_steps + step] = acc;
  if (!isfinite(acc)) failed[s] = 1;
}

hipError_t launch_lnc_accum(int64_t nsamp, int out_per_sample, int step, int n_steps, double mult, const double* lnc,
                            double* lnc_steps, int* failed, hipStream_t stream) {
  if (nsamp == 0) return hipSuccess;
  hipLaunchKernelGGL(lnc_accum_kernel, dim3(ceil_div(nsamp, 128)), dim3(128), 0, stream, nsamp, out_per_sample,
                     step, n_steps, mult, lnc, lnc_steps, failed);
  return hipGetLastError();
}

__global__ void jacobi_fail_kernel(int64_t njobs, int jobs_per_sample, const int* __restrict__ sweeps,
                                   int* __restrict__ failed) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < njobs && sweeps[j] < 0) failed[j / jobs_per_sample] = 1;
}

hipError_t launch_jacobi_fail(int64_t njobs, int jobs_per_sample, const int* sweeps, int* failed,
                              hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_fail_kernel, dim3(ceil_div(njobs, 256)), dim3(256), 0, stream, njobs, jobs_per_sample,
                     sweeps, failed);
  return hipGetLastError();
}

__global__ void set_double_kernel(double* p, double v) { *p = v; }

hipError_t launch_set_double(double* p, double v, hipStream_t stream) {
  hipLaunchKernelGGL(set_double_kernel, dim3(1), dim3(1), 0, stream, p, v);
  return hipGetLastError();
}

__global__ void izero_kernel(int64_t n, int* p) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_izero(int64_t n, int* p, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(izero_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, stream, n, p);
  return hipGetLastError();
}

__global__ void scatter_kernel(int64_t nsamp, int n_steps, const int64_t* __restrict__ idx,
                               const int8_t* __restrict__ sign, const double* __restrict__ ln,
                               const double* __restrict__ lnc_steps, int8_t* __restrict__ out_sign,
                               double* __restrict__ out_ln, double* __restrict__ out_lnc) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nsamp) return;
  const int64_t d = idx[s];
  out_sign[d] = sign[s];
  out_ln[d] = ln[s];
  if (out_lnc)
    for (int t = 0; t < n_steps; ++t) out_lnc[d * n_steps + t] = lnc_steps[s * n_steps + t];
}

hipError_t launch_scatter(int64_t nsamp, int n_steps, const int64_t* idx, const int8_t* sign, const double* ln,
                          const double* lnc_steps, int8_t* out_sign, double* out_ln, double* out_lnc,
                          hipStream_t stream) {
  if (nsamp == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(ceil_div(nsamp, 128)), dim3(128), 0, stream, nsamp, n_steps, idx, sign,
                     ln, lnc_steps, out_sign, out_ln, out_lnc);
  return hipGetLastError();
}

}  // namespace mctrg
