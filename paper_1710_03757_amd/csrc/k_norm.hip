// Initial tensors, normalisation, final trace and the estimator.
//
// Normalisation (a reading: the paper does not normalise, but a chain over
// 2^30 sites needs it): every coarse tensor T' is stored as c * T_hat with
// c = max|T'|; ln c is kept in FP64 and, in the shared chain, enters ln Z
// with the number of tensors of that level (2^(n_steps - step - 1)).
// Final trace: the last tensor is traced over its periodic legs,
// Tr = sum_{a,b} T_hat[a,b,a,b] (the explicit trace of the final small
// network, paper Section III after Eq. infiniteSum).
// Estimator: mean of the signed samples (Section III Eq. infiniteEnsemble)
// in the log domain, error of the mean per Section V Eq. shrunkDev.
#include "mctrg_internal.h"
#include "../../include/mctrg.h"

namespace mctrg {

// ---- initial tensors --------------------------------------------------------
__global__ void init_tensors_kernel(int model, int ngroups, const double* __restrict__ beta,
                                    const double* __restrict__ h, double* __restrict__ out) {
  const int g = blockIdx.x;
  const int e = threadIdx.x;   // 16 entries (l,u,r,d) in {0,1}^4
  if (g >= ngroups || e >= 16) return;
  const int l = (e >> 3) & 1, u = (e >> 2) & 1, r = (e >> 1) & 1, d = e & 1;
  const double b = beta[g], hh = h[g];
  double v;
  if (model == MCTRG_ISING_SITE) {
    // sum over the spin s of exp(b h s) * prod over legs of W[s][leg]
    const double c = sqrt(cosh(b)), s = sqrt(sinh(b));
    v = 0.0;
    for (int si = 0; si < 2; ++si) {
      const double spin = si == 0 ? 1.0 : -1.0;
      double p = exp(b * hh * spin);
      const int legs[4] = {l, u, r, d};
      for (int t = 0; t < 4; ++t) p *= (legs[t] == 0) ? c : (si == 0 ? s : -s);
      v += p;
    }
  } else {
    const double sl = l ? -1.0 : 1.0, su = u ? -1.0 : 1.0, sr = r ? -1.0 : 1.0, sd = d ? -1.0 : 1.0;
    v = exp(b * (sl * su + su * sr + sr * sd + sd * sl) + 0.5 * b * hh * (sl + su + sr + sd));
  }
  out[(size_t)g * 16 + e] = v;
}

hipError_t launch_init_tensors(int model, int ngroups, const double* beta, const double* h, double* out,
                               hipStream_t stream) {
  hipLaunchKernelGGL(init_tensors_kernel, dim3(ngroups), dim3(16), 0, stream, model, ngroups, beta, h, out);
  return hipGetLastError();
}

__global__ void gather_tensors_kernel(int64_t nsamp, int per, const double* __restrict__ T0,
                                      const int32_t* __restrict__ group, double* __restrict__ T) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nsamp * per) return;
  const int64_t s = i / per;
  const int e = (int)(i % per);
  T[i] = T0[(size_t)group[s] * per + e];
}

hipError_t launch_gather_tensors(int64_t nsamp, int d0, const double* T0, const int32_t* group, double* T,
                                 hipStream_t stream) {
  const int per = d0 * d0 * d0 * d0;
  const int64_t tot = nsamp * per;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_tensors_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, stream, nsamp, per, T0, group, T);
  return hipGetLastError();
}

// ---- normalisation ------------------------------------------------------------
__global__ void zero_kernel(int64_t n, double* p) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

template <typename T>
__global__ void absmax_out_kernel(int64_t elems, const T* __restrict__ A, double* __restrict__ cbuf) {
  const int64_t o = blockIdx.y;
  const T* Ao = A + o * elems;
  double m = 0.0;
  bool bad = false;
#pragma unroll 4
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < elems; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)Ao[e];
    if (!isfinite(v)) bad = true;
    m = fmax(m, fabs(v));
  }
  if (bad) m = INFINITY;
  for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(&cbuf[o], m);
}

template <typename T>
__global__ void scale_out_kernel(int64_t elems, const T* __restrict__ A, const double* __restrict__ cbuf,
                                 double* __restrict__ out) {
  const int64_t o = blockIdx.y;
  const double c = cbuf[o];
  const double inv = (c > 0.0 && isfinite(c)) ? 1.0 / c : 0.0;
#pragma unroll 4
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < elems; e += (int64_t)gridDim.x * blockDim.x)
    out[o * elems + e] = (double)A[o * elems + e] * inv;
}

__global__ void lnc_kernel(int64_t nout, const double* __restrict__ cbuf, const double* __restrict__ scales,
                           double* __restrict__ lnc) {
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o >= nout) return;
  const double c = cbuf[o];
  if (c > 0.0 && isfinite(c)) lnc[o] = log(c) - log(scales[o]) - log(scales[nout + o]);
  else lnc[o] = NAN;
}

hipError_t launch_normalize(int64_t nout, int64_t elems, int src_is_f32, const void* Tp, const double* scales,
                            double* cbuf, double* T, double* lnc, hipStream_t stream) {
  if (nout == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(ceil_div(nout, 256)), dim3(256), 0, stream, nout, cbuf);
  int gx = (int)((elems + 255) / 256);
  if (gx > 256) gx = 256;
  if (src_is_f32) {
    hipLaunchKernelGGL(absmax_out_kernel<float>, dim3(gx, (unsigned)nout), dim3(256), 0, stream, elems,
                       (const float*)Tp, cbuf);
    hipLaunchKernelGGL(scale_out_kernel<float>, dim3(gx, (unsigned)nout), dim3(256), 0, stream, elems,
                       (const float*)Tp, cbuf, T);
  } else {
    hipLaunchKernelGGL(absmax_out_kernel<double>, dim3(gx, (unsigned)nout), dim3(256), 0, stream, elems,
                       (const double*)Tp, cbuf);
    hipLaunchKernelGGL(scale_out_kernel<double>, dim3(gx, (unsigned)nout), dim3(256), 0, stream, elems,
                       (const double*)Tp, cbuf, T);
  }
  hipLaunchKernelGGL(lnc_kernel, dim3(ceil_div(nout, 256)), dim3(256), 0, stream, nout, cbuf, scales, lnc);
  return hipGetLastError();
}

// ---- final trace ---------------------------------------------------------------
// shared_weights: ln|Z| = sum_s 2^(n_steps-s-1) lnc[s] + ln|tr|; otherwise the
// per-step values are already summed over the level's tensors.
__global__ void trace_kernel(int64_t nsamp, int D, const double* __restrict__ T, const double* __restrict__ lnc,
                             int lnc_stride, int n_steps, int shared_weights, const int* __restrict__ failed,
                             int8_t* __restrict__ sign, double* __restrict__ ln_abs) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nsamp) return;
  const size_t D2 = (size_t)D * D;
  const double* Ts = T + (size_t)s * D2 * D2;
  double tr = 0.0;
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) tr += Ts[((size_t)a * D + b) * D2 + (size_t)a * D + b];
  double acc = 0.0;
  for (int st = 0; st < n_steps; ++st) {
    const double w = shared_weights ? ldexp(1.0, n_steps - st - 1) : 1.0;
    acc += w * lnc[(size_t)s * lnc_stride + st];
  }
  const bool bad = failed[s] || !isfinite(acc) || !(tr != 0.0) || !isfinite(tr);
  if (bad) {
    sign[s] = 0;
    ln_abs[s] = NAN;
  } else {
    sign[s] = tr > 0.0 ? 1 : -1;
    ln_abs[s] = acc + log(fabs(tr));
  }
}

hipError_t launch_trace(int64_t nsamp, int D, const double* T, const double* lnc_steps, int lnc_stride,
                        int n_steps, int shared_weights, const int* failed, int8_t* sign, double* ln_abs_Z,
                        hipStream_t stream) {
  if (nsamp == 0) return hipSuccess;
  hipLaunchKernelGGL(trace_kernel, dim3(ceil_div(nsamp, 128)), dim3(128), 0, stream, nsamp, D, T, lnc_steps,
                     lnc_stride, n_steps, shared_weights, failed, sign, ln_abs_Z);
  return hipGetLastError();
}

// ---- estimator -------------------------------------------------------------------
// out8: ln_meanZ_per_site, rel_stderr_Z, mean_lnZ_per_site, stderr_mean_lnZ,
//       n_used, n_negative, n_failed (as doubles).  One workgroup of 256
//       threads; fixed reduction order so the result is reproducible.
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}
__device__ double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void estimate_kernel(int64_t n, const int8_t* __restrict__ sign,
                                                       const double* __restrict__ ln_abs, double n_sites,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  double mx = -INFINITY, cnt = 0.0, neg = 0.0, sl = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double l = ln_abs[i];
    if (sign[i] != 0 && isfinite(l)) {
      mx = fmax(mx, l);
      cnt += 1.0;
      neg += sign[i] < 0 ? 1.0 : 0.0;
      sl += l;
    }
  }
  mx = block_max(mx, red);
  cnt = block_sum(cnt, red);
  neg = block_sum(neg, red);
  sl = block_sum(sl, red);
  double sz = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double l = ln_abs[i];
    if (sign[i] != 0 && isfinite(l)) sz += (double)sign[i] * exp(l - mx);
  }
  sz = block_sum(sz, red);
  const double meanz = sz / cnt, meanl = sl / cnt;
  double vz = 0.0, vl = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double l = ln_abs[i];
    if (sign[i] != 0 && isfinite(l)) {
      const double z = (double)sign[i] * exp(l - mx) - meanz;
      vz += z * z;
      vl += (l - meanl) * (l - meanl);
    }
  }
  vz = block_sum(vz, red);
  vl = block_sum(vl, red);
  if (threadIdx.x == 0) {
    const double nu = cnt;
    out[0] = (nu > 0 && meanz > 0) ? (mx + log(meanz)) / n_sites : NAN;
    out[1] = (nu > 1 && meanz != 0) ? sqrt(vz / (nu - 1) / nu) / fabs(meanz) : NAN;
    out[2] = nu > 0 ? meanl / n_sites : NAN;
    out[3] = nu > 1 ? sqrt(vl / (nu - 1) / nu) / n_sites : NAN;
    out[4] = nu;
    out[5] = neg;
    out[6] = (double)n - nu;
  }
}

hipError_t launch_estimate(int64_t n, const int8_t* sign, const double* ln_abs, double n_sites, double* out8,
                           hipStream_t stream) {
  hipLaunchKernelGGL(estimate_kernel, dim3(1), dim3(256), 0, stream, n, sign, ln_abs, n_sites, out8);
  return hipGetLastError();
}

}  // namespace mctrg
