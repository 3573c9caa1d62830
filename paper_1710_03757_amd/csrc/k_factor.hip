// Unfolding and factor construction.
//
// Unfold (paper Section II, the index grouping before Eq. exactSVD): a
// tensor T[l][u][r][d] with all legs of (capacity) dimension D is viewed
// as an n x n matrix, n = D^2:
//   A split  M_A[(l,u)][(r,d)] = T[l][u][r][d]  (T itself, row-major);
//   B split  M_B[(u,r)][(d,l)] = T[l][u][r][d].
// The Jacobi workspace W receives a zero-padded copy (n_pad x n_pad).
//
// Factors (Section II: T~ = U S^(e) V restricted to the kept set, with
// S^(e)_ii = S_ii / r(S_ii); the reweighted value is split symmetrically):
//   G[a][:] = w_a v_{i_a}^T,          v = normalised Jacobi row, signed so
//                                     that sum_j v_j / (1 + i1 + phi i2) > 0
//   F[a][:] = w_a u_{i_a}^T = (M G[a]^T)^T / s_{i_a}  (stored by kept index)
// with w_a = sqrt(s_{i_a} / r_{i_a}); entries a >= kept are zero
// (capacity padding).
#include "mctrg_internal.h"

namespace mctrg {

__device__ __forceinline__ size_t unfold_index(int split, int D, int row, int col) {
  if (split == 0) return (size_t)row * (D * D) + col;
  const int u = row / D, r = row % D, d = col / D, l = col % D;
  return (((size_t)l * D + u) * D + r) * D + d;
}

__global__ void unfold_kernel(int64_t njobs, int D, int n_pad, const double* __restrict__ T,
                              const int32_t* __restrict__ src, const int32_t* __restrict__ split,
                              double* __restrict__ W) {
  const int64_t job = blockIdx.y;
  const int n = D * D;
  const size_t per = (size_t)n_pad * n_pad;
  const double* Ts = T + (size_t)src[job] * n * n;
  const int sp = split[job];
  double* Wj = W + job * per;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < per; e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / n_pad), col = (int)(e % n_pad);
    double v = 0.0;
    if (row < n && col < n) v = Ts[unfold_index(sp, D, row, col)];
    Wj[e] = v;
  }
}

hipError_t launch_unfold(int64_t njobs, int D, int n_pad, const double* T, const int32_t* src,
                         const int32_t* split, double* W, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  const size_t per = (size_t)n_pad * n_pad;
  int gx = (int)((per + 255) / 256);
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(unfold_kernel, dim3(gx, (unsigned)njobs), dim3(256), 0, stream, njobs, D, n_pad, T, src,
                     split, W);
  return hipGetLastError();
}

// One workgroup per (kept index a, job).
__global__ __launch_bounds__(256) void factor_G_kernel(int D, int n_pad, int kcap, const double* __restrict__ W,
                                                       const double* __restrict__ sigma,
                                                       const int32_t* __restrict__ order,
                                                       const int32_t* __restrict__ kept,
                                                       const int32_t* __restrict__ sel,
                                                       const double* __restrict__ weight,
                                                       const int32_t* __restrict__ perm,
                                                       double* __restrict__ G) {
  const int a = blockIdx.x;
  const int64_t job = blockIdx.y;
  const int n = D * D;
  double* Ga = G + (size_t)job * kcap * n + (size_t)a * n;
  if (a >= kept[job]) {
    for (int e = threadIdx.x; e < n; e += 256) Ga[e] = 0.0;
    return;
  }
  const int i = sel[job * kcap + a];
  const int row = order[(size_t)job * n + i];
  const double s = sigma[(size_t)job * n + i];
  const double w = weight[job * kcap + a];
  const double* v = W + (size_t)job * n_pad * n_pad + (size_t)row * n_pad;
  const int32_t* pj = perm + job * n_pad;
  __shared__ double red[4];
  double g = 0.0;
  // entry c of the Jacobi row belongs to column perm[c] of the unfolding
  for (int c = threadIdx.x; c < n_pad; c += 256) {
    const int e = pj[c];
    if (e < n) g += v[c] / (1.0 + (double)(e / D) + kGolden * (double)(e % D));
  }
  for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g;
  __syncthreads();
  g = (red[0] + red[1]) + (red[2] + red[3]);
  const double f = (g < 0.0 ? -w : w) / s;
  for (int c = threadIdx.x; c < n_pad; c += 256) {
    const int e = pj[c];
    if (e < n) Ga[e] = f * v[c];
  }
}

hipError_t launch_factor_G(int64_t njobs, int D, int n_pad, int kcap, const double* W, const double* sigma,
                           const int32_t* order, const int32_t* kept, const int32_t* sel, const double* weight,
                           const int32_t* perm, double* G, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(factor_G_kernel, dim3(kcap, (unsigned)njobs), dim3(256), 0, stream, D, n_pad, kcap, W, sigma,
                     order, kept, sel, weight, perm, G);
  return hipGetLastError();
}

// Gt[job][a][l D + d] = G[job][a][d D + l] for the B-split jobs: the columns
// (d, l) of M_B in the order in which T stores them.
__global__ void transpose_G_kernel(int D, int kcap, const int32_t* __restrict__ split, const double* __restrict__ G,
                                   double* __restrict__ Gt) {
  const int64_t job = blockIdx.z;
  const int a = blockIdx.y, n = D * D;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;   // l D + d
  if (split[job] != 1 || e >= n) return;
  const int l = e / D, d = e - l * D;
  const size_t base = ((size_t)job * kcap + a) * n;
  Gt[base + e] = G[base + (size_t)d * D + l];
}

// F[job][a][row] = (1/s_a) sum_col M[row][col] G[job][a][col].  One
// workgroup per (64-row tile, job); column chunks of 32 staged in LDS.  For
// the B split M_B[(u,r)][(d,l)] = T[l][u][r][d], so the columns are taken in
// T's order (l, d), contiguous per row, with G from its transposed copy Gt.
__global__ __launch_bounds__(256) void factor_F_kernel(int D, int kcap, const double* __restrict__ T,
                                                       const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ split,
                                                       const double* __restrict__ sigma,
                                                       const int32_t* __restrict__ kept,
                                                       const int32_t* __restrict__ sel,
                                                       const double* __restrict__ G, const double* __restrict__ Gt,
                                                       double* __restrict__ F) {
  const int64_t job = blockIdx.y;
  const int n = D * D;
  const int row0 = blockIdx.x * 64;
  const int sp = split[job];
  const double* Ts = T + (size_t)src[job] * n * n;
  const double* Gj = (sp == 1 ? Gt : G) + (size_t)job * kcap * n;
  const size_t D3 = (size_t)D * D * D;
  const int kk = kept[job];
  __shared__ double Ms[64][33];
  __shared__ double Gs[64][33];
  const int tid = threadIdx.x;
  const int rloc = tid & 63, agrp = tid >> 6;   // a = agrp + 4*q
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int c0 = 0; c0 < n; c0 += 32) {
    for (int e = tid; e < 64 * 32; e += 256) {
      const int rr = e >> 5, cc = e & 31;
      const int row = row0 + rr, col = c0 + cc;
      double v = 0.0;
      if (row < n && col < n) {
        if (sp == 1) {   // col = l D + d
          const int l = col / D, d = col - l * D;
          v = Ts[(size_t)l * D3 + (size_t)row * D + d];
        } else {
          v = Ts[(size_t)row * n + col];
        }
      }
      Ms[rr][cc] = v;
    }
    for (int e = tid; e < 64 * 32; e += 256) {
      const int aa = e >> 5, cc = e & 31;
      const int col = c0 + cc;
      Gs[aa][cc] = (aa < kk && col < n) ? Gj[(size_t)aa * n + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int aa = agrp + 4 * q;
      if (aa < kcap) {
        double s = acc[q];
#pragma unroll 8
        for (int cc = 0; cc < 32; ++cc) s += Ms[rloc][cc] * Gs[aa][cc];
        acc[q] = s;
      }
    }
    __syncthreads();
  }
  const int row = row0 + rloc;
  if (row < n) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int aa = agrp + 4 * q;
      if (aa < kcap) {
        double v = 0.0;
        if (aa < kk) v = acc[q] / sigma[(size_t)job * n + sel[job * kcap + aa]];
        F[(size_t)job * n * kcap + (size_t)aa * n + row] = v;   // by kept index: rows contiguous
      }
    }
  }
}

hipError_t launch_factor_F(int64_t njobs, int D, int kcap, const double* T, const int32_t* src,
                           const int32_t* split, const double* sigma, const int32_t* kept,
                           const int32_t* sel, const double* G, double* Gt, double* F, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  const int n = D * D;
  hipLaunchKernelGGL(transpose_G_kernel, dim3(ceil_div(n, 256), kcap, (unsigned)njobs), dim3(256), 0, stream, D, kcap,
                     split, G, Gt);
  hipLaunchKernelGGL(factor_F_kernel, dim3(ceil_div(n, 64), (unsigned)njobs), dim3(256), 0, stream, D, kcap, T,
                     src, split, sigma, kept, sel, G, (const double*)Gt, F);
  return hipGetLastError();
}

// Right factors from the QR routes (an odd number of QR steps): X[c][a] =
// w_a z_a[c] is the kept
// right singular vector of M P (logical column c, c < n: the padding columns
// sort last), so G[a][perm[colmap[c]]] = X[c][a] (= w_a v_a^T), signed so
// that sum_e G[a][e] / (1 + e/d2 + phi (e % d2)) > 0 (the chains: n = D^2,
// d2 = D).  One workgroup per (a, job).
__global__ __launch_bounds__(256) void scatter_G_kernel(int n, int d2, int n_pad, int kcap,
                                                        const double* __restrict__ X,
                                                        const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ colmap,
                                                        const int32_t* __restrict__ kept, double* __restrict__ G) {
  const int a = blockIdx.x;
  const int64_t job = blockIdx.y;
  double* Ga = G + (size_t)job * kcap * n + (size_t)a * n;
  if (a >= kept[job]) {
    for (int e = threadIdx.x; e < n; e += 256) Ga[e] = 0.0;
    return;
  }
  const double* Xj = X + (size_t)job * n * kcap;
  const int32_t* pj = perm + job * n_pad;
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;
  __shared__ double red[4];
  double g = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) {
    const int e = pj[cm ? cm[c] : c];
    g += Xj[(size_t)c * kcap + a] / (1.0 + (double)(e / d2) + kGolden * (double)(e % d2));
  }
  for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g;
  __syncthreads();
  g = (red[0] + red[1]) + (red[2] + red[3]);
  const double sg = g < 0.0 ? -1.0 : 1.0;
  for (int c = threadIdx.x; c < n; c += 256) Ga[pj[cm ? cm[c] : c]] = sg * Xj[(size_t)c * kcap + a];
}

hipError_t launch_scatter_G(int64_t njobs, int D, int n_pad, int kcap, const double* X, const int32_t* perm,
                            const int32_t* colmap, const int32_t* kept, double* G, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_G_kernel, dim3(kcap, (unsigned)njobs), dim3(256), 0, stream, D * D, D, n_pad, kcap, X,
                     perm, colmap, kept, G);
  return hipGetLastError();
}

hipError_t launch_scatter_V(int64_t nmats, int n, int d2, int n_pad, const double* X, const int32_t* perm,
                            const int32_t* colmap, const int32_t* kept, double* V, hipStream_t stream) {
  if (nmats == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_G_kernel, dim3(n, (unsigned)nmats), dim3(256), 0, stream, n, d2, n_pad, n, X, perm,
                     colmap, kept, V);
  return hipGetLastError();
}

// All right vectors of a step-level SVD: kept[j] = the number of positive
// values in sigma[j] (n, descending), sel[j][a] = a, weight[j][a] = 1.  One
// workgroup per matrix.
__global__ __launch_bounds__(256) void select_all_kernel(int n, const double* __restrict__ sigma,
                                                         int32_t* __restrict__ kept, int32_t* __restrict__ sel,
                                                         double* __restrict__ weight) {
  const int64_t j = blockIdx.x;
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int a = threadIdx.x; a < n; a += 256) {
    sel[j * n + a] = a;
    weight[j * n + a] = 1.0;
    mine += sigma[j * n + a] > 0.0 ? 1 : 0;
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) kept[j] = cnt;
}

hipError_t launch_select_all(int64_t nmats, int n, const double* sigma, int32_t* kept, int32_t* sel, double* weight,
                             hipStream_t stream) {
  if (nmats == 0) return hipSuccess;
  hipLaunchKernelGGL(select_all_kernel, dim3((unsigned)nmats), dim3(256), 0, stream, n, sigma, kept, sel, weight);
  return hipGetLastError();
}

}  // namespace mctrg
