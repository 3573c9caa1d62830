// QR preconditioning of the decomposition step.
//
// One-sided Jacobi converges slowly on the strongly graded TRG unfoldings
// (tens of sweeps).  Rotating the rows of the triangular factor R of
// M P = Q R instead (P orders the columns of M by decreasing norm) leaves
// the right singular vectors unchanged up to P (R = Q^T M P) and cuts the
// number of sweeps several-fold (preconditioned Jacobi in the sense of
// Drmac and Veselic).  Only R and P are needed, never Q.
//
// Storage: S (n_pad x n_pad per job) holds M P column by column: S[c][r] =
// M[r][P[c]], so every column is contiguous.  The factorisation is the
// blocked Householder QR with 32-column panels (8-column panels for
// n_pad > 1024):
//   panel kernel     one workgroup per job factors the panel in registers
//                    (each thread owns up to four (eight) rows of the panel;
//                    qr_panel32_kernel for the 32-column panels),
//                    leaves the Householder vectors below the diagonal and
//                    R on and above it, and forms the 32 x 32 triangular T of
//                    the compact WY form I - V T V^T;
//   trailing kernel  (job, 64-column tile) workgroups apply
//                    C <- C - V (T^T (V^T C)) with v_mfma_f64_16x16x4.
// Finally the rows of R are copied into the Jacobi workspace.
#include "mctrg_internal.h"

namespace mctrg {


// ---------------------------------------------------------------------------
// Column norms of M and their descending order (ties by index): P.
// ---------------------------------------------------------------------------
// split 0: M_A of a D^4 tensor, M_A[(l,u)][(r,d)] = T[l][u][r][d]; 1: M_B,
// M_B[(u,r)][(d,l)] = T[l][u][r][d]; 2: a plain row-major n x n matrix.
// perm = the columns of M by decreasing norm (ties by index, padding
// columns last), iperm its inverse.  The threads take the columns in the
// order T stores them (for M_B, column (d, l) as l D + d), so that the loads
// of a row are contiguous.
__global__ __launch_bounds__(256) void colnorm_order_kernel(int n, int D, int n_pad, const double* __restrict__ T,
                                                            const int32_t* __restrict__ src,
                                                            const int32_t* __restrict__ split,
                                                            int32_t* __restrict__ perm, int32_t* __restrict__ iperm) {
  extern __shared__ unsigned char smem[];
  int P = 1;
  while (P < n_pad) P <<= 1;
  double* key = reinterpret_cast<double*>(smem);
  int* idx = reinterpret_cast<int*>(key + P);
  const int64_t job = blockIdx.x;
  const double* Ts = T + (size_t)src[job] * n * n;
  const int sp = split[job];
  for (int t = threadIdx.x; t < P; t += 256) {
    double s = -1.0;
    int c = t;
    if (t < n) {
      s = 0.0;
      if (sp == 1) {   // t = l D + d, column (d, l) of M_B: T[l][.][.][d]
        const int l = t / D, d = t - l * D;
        c = d * D + l;
        const double* base = Ts + (size_t)l * D * D * D + d;
        for (int r = 0; r < n; ++r) {
          const double v = base[(size_t)r * D];
          s += v * v;
        }
      } else {
        for (int r = 0; r < n; ++r) {
          const double v = Ts[(size_t)r * n + t];
          s += v * v;
        }
      }
    } else if (t < n_pad) {
      s = -0.5;
    }
    key[c] = s;
    idx[c] = c;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += 256) {
        const int i = 2 * stride * (t / stride) + (t % stride), j = i + stride;
        const bool up = (i & size) == 0;
        const double ki = key[i], kj = key[j];
        const int ii = idx[i], ij = idx[j];
        const bool i_first = (ki > kj) || (ki == kj && ii < ij);
        if (up ? !i_first : i_first) { key[i] = kj; key[j] = ki; idx[i] = ij; idx[j] = ii; }
      }
      __syncthreads();
    }
  }
  for (int c = threadIdx.x; c < n_pad; c += 256) {
    perm[job * n_pad + c] = idx[c];
    iperm[job * n_pad + idx[c]] = c;
  }
}

// S[c][r] = M[r][perm[c]] (zero outside n x n).  Tiles of 64 rows x 32
// columns of M, the columns taken in the order T stores them (as in
// colnorm_order_kernel), are read row by row, transposed through LDS, and
// each column written contiguously to its place S[iperm[col]].
__global__ __launch_bounds__(256) void unfold_cols_kernel(int n, int D, int n_pad, const double* __restrict__ T,
                                                          const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ split,
                                                          const int32_t* __restrict__ iperm, double* __restrict__ S) {
  const int64_t job = blockIdx.z;
  const int r0 = 64 * blockIdx.x, t0 = 32 * blockIdx.y, tid = threadIdx.x;
  const double* Ts = T + (size_t)src[job] * n * n;
  const int sp = split[job];
  __shared__ double tile[32][65];   // [column][row]
  {
    const int tc = tid & 31, tr = tid >> 5, t = t0 + tc;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = r0 + tr + 8 * q;
      double v = 0.0;
      if (r < n && t < n) {
        if (sp == 1) {
          const int l = t / D, d = t - l * D;
          v = Ts[(size_t)l * D * D * D + (size_t)r * D + d];
        } else {
          v = Ts[(size_t)r * n + t];
        }
      }
      tile[tc][tr + 8 * q] = v;
    }
  }
  __syncthreads();
  double* Sj = S + (size_t)job * n_pad * n_pad;
  const int32_t* ip = iperm + job * n_pad;
  for (int e = tid; e < 32 * 64; e += 256) {
    const int tc = e >> 6, rr = e & 63, t = t0 + tc, r = r0 + rr;
    if (t >= n_pad || r >= n_pad) continue;
    int col = t;
    if (sp == 1 && t < n) {
      const int l = t / D;
      col = (t - l * D) * D + l;
    }
    Sj[(size_t)ip[col] * n_pad + r] = tile[tc][rr];
  }
}

// ---------------------------------------------------------------------------
// Panel factorisation (columns j..j+31, rows j..n_pad-1), one workgroup/job.
// Thread t owns rows j + t + 256 q, q < QR_MAXQ.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void block_reduce_vec(double* v, int cnt, double (*red)[33], int tid) {
  // v[0..cnt) per thread -> summed over the NT threads, result in red[0][..]
  const int lane = tid & 63, wave = tid >> 6;
  for (int x = 0; x < cnt; ++x) {
    double s = v[x];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wave + 1][x] = s;
  }
  __syncthreads();
  if (tid < cnt) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w + 1][tid];
    red[0][tid] = s;
  }
  __syncthreads();
}

// Panel kernel: NT threads, MAXQ rows per thread, PW-column panels.
template <int NT, int MAXQ, int PW>
__global__ __launch_bounds__(NT) void qr_panel_kernel(int n_pad, int j, double* __restrict__ S,
                                                      double* __restrict__ Tws, int64_t t_stride, int64_t t_off) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x;
  double* Sj = S + job * (size_t)n_pad * n_pad;
  __shared__ double red[NT / 64 + 1][33];
  __shared__ double Tm[PW][PW + 1];
  __shared__ double sh_alpha;

  double A[MAXQ][PW];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) {
    const int r = j + tid + NT * q;
#pragma unroll
    for (int c = 0; c < PW; ++c) A[q][c] = (r < n_pad) ? Sj[(size_t)(j + c) * n_pad + r] : 0.0;
  }
  for (int e = tid; e < PW * (PW + 1); e += NT) Tm[e / (PW + 1)][e % (PW + 1)] = 0.0;

  double part[PW];
#pragma unroll
  for (int i = 0; i < PW; ++i) {
    const int cj = j + i;
    // --- Householder vector of column i --------------------------------------
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int r = j + tid + NT * q;
      if (r > cj && r < n_pad) sq += A[q][i] * A[q][i];
      if (r == cj) sh_alpha = A[q][i];
    }
    part[0] = sq;
    block_reduce_vec<NT>(part, 1, red, tid);
    const double xn2 = red[0][0];
    const double alpha = sh_alpha;
    double beta, tau, scale;
    if (xn2 == 0.0) {
      beta = alpha; tau = 0.0; scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v: 1 at r == cj, A * scale below, 0 above; stored in column i
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int r = j + tid + NT * q;
      if (r > cj) A[q][i] *= scale;
      else if (r == cj) A[q][i] = beta;   // R diagonal; the implicit 1 is used below
    }
    // --- dots: w_c = v^T col_c (c > i), z_m = v_m^T v (m < i) ------------------
#pragma unroll
    for (int x = 0; x < PW; ++x) part[x] = 0.0;
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int r = j + tid + NT * q;
      if (r >= cj && r < n_pad) {
        const double vr = (r == cj) ? 1.0 : A[q][i];
#pragma unroll
        for (int c = 0; c < PW; ++c) {
          if (c > i) part[c] += vr * A[q][c];
          else if (c < i) {
            // v_c at row r: below its diagonal j+c it is stored, at j+c it is 1
            const double vc = (r > j + c) ? A[q][c] : (r == j + c ? 1.0 : 0.0);
            part[c] += vr * vc;
          }
        }
      }
    }
    block_reduce_vec<NT>(part, PW, red, tid);
    // --- apply H_i to the remaining panel columns ----------------------------
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int r = j + tid + NT * q;
      if (r >= cj && r < n_pad) {
        const double vr = (r == cj) ? 1.0 : A[q][i];
#pragma unroll
        for (int c = 0; c < PW; ++c)
          if (c > i) A[q][c] -= tau * red[0][c] * vr;
      }
    }
    // --- T column i: T[0:i, i] = -tau T[0:i, 0:i] z[0:i], T[i][i] = tau --------
    if (tid < PW) {
      const int m = tid;
      if (m < i) {
        double s2 = 0.0;
        for (int p = m; p < i; ++p) s2 += Tm[m][p] * red[0][p];
        part[0] = -tau * s2;
      }
    }
    __syncthreads();
    if (tid < i) Tm[tid][i] = part[0];
    if (tid == 0) Tm[i][i] = tau;
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) {
    const int r = j + tid + NT * q;
    if (r < n_pad) {
#pragma unroll
      for (int c = 0; c < PW; ++c) Sj[(size_t)(j + c) * n_pad + r] = A[q][c];
    }
  }
  double* Tj = Tws + job * t_stride + t_off;
  for (int e = tid; e < PW * PW; e += NT) Tj[e] = Tm[e / PW][e % PW];
}

// Panel factorisation for n_pad <= 1024 with 32-column panels: 256 threads,
// thread t owns rows j + t + 256 q (q < 4) of the 32 panel columns in
// registers.  The register slots rotate by one column per step so that the
// pivot column is always slot 0 (no dynamic register indexing): at step i,
// slots 1 .. 31 - i hold columns i + 1 .. 31 and slots 32 - i .. 31 the
// finished Householder vectors v_0 .. v_{i-1}.  One reduction per column
// gives, with x = the pivot column below the diagonal row cj = j + i,
//   x^T x (slot 0), x^T col_c (slots of later columns), x^T v_m (finished);
// with the row-cj entries this yields the Householder reflector (LAPACK
// dlarfg convention), w_c = v^T col_c and z_m = v_m^T v.  The 64 lanes of a
// wave reduce their 32 partial sums by halving exchanges (16 + 8 + 4 + 2 + 1
// + 1 shuffles).  T of the compact WY form follows at the end, row m by
// thread m: T[m][m] = tau_m, T[m][i] = -tau_i sum_{p=m}^{i-1} T[m][p] z_p^(i).
template <int NQ>
__global__ __launch_bounds__(256) void qr_panel32_kernel(int n_pad, int j, double* __restrict__ S,
                                                         double* __restrict__ Tws, int64_t t_stride, int64_t t_off,
                                                         const int32_t* __restrict__ colmap) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Sj = S + job * (size_t)n_pad * n_pad;
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;   // logical -> stored column
  __shared__ double red[4][32];
  __shared__ double rowcj[32];
  __shared__ double wz[32];
  __shared__ double Zs[32][33];
  __shared__ double taus[32];
  __shared__ double prm[3];   // tau, scale, beta of the current column

  double A[NQ][32];   // rows j + tid + 256 q, q < NQ (n_pad - j <= 256 NQ)
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = j + tid + 256 * q;
#pragma unroll
    for (int c = 0; c < 32; ++c) A[q][c] = (r < n_pad) ? Sj[(size_t)(cm ? cm[j + c] : j + c) * n_pad + r] : 0.0;
  }
  // lane l holds, after the halving exchanges, the sum of slot sidx
  const int sidx = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 + ((lane >> 2) & 1) * 2 +
                   ((lane >> 1) & 1);
  for (int i = 0; i < 32; ++i) {
    const int cj = j + i;
    double p[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) p[c] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = j + tid + 256 * q;
      const double x = (r > cj && r < n_pad) ? A[q][0] : 0.0;
#pragma unroll
      for (int c = 0; c < 32; ++c) p[c] = fma(A[q][c], x, p[c]);
    }
    if (tid == i) {
#pragma unroll
      for (int c = 0; c < 32; ++c) rowcj[c] = A[0][c];
    }
    // halving exchanges: 32 -> 16 -> 8 -> 4 -> 2 -> 1 values per lane
#pragma unroll
    for (int h = 0; h < 16; ++h) {
      const bool up = lane & 32;
      const double keep = up ? p[16 + h] : p[h], send = up ? p[h] : p[16 + h];
      p[h] = keep + __shfl_xor(send, 32);
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const bool up = lane & 16;
      const double keep = up ? p[8 + h] : p[h], send = up ? p[h] : p[8 + h];
      p[h] = keep + __shfl_xor(send, 16);
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const bool up = lane & 8;
      const double keep = up ? p[4 + h] : p[h], send = up ? p[h] : p[4 + h];
      p[h] = keep + __shfl_xor(send, 8);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool up = lane & 4;
      const double keep = up ? p[2 + h] : p[h], send = up ? p[h] : p[2 + h];
      p[h] = keep + __shfl_xor(send, 4);
    }
    {
      const bool up = lane & 2;
      const double keep = up ? p[1] : p[0], send = up ? p[0] : p[1];
      p[0] = keep + __shfl_xor(send, 2);
    }
    p[0] += __shfl_xor(p[0], 1);
    if ((lane & 1) == 0) red[wave][sidx] = p[0];
    __syncthreads();
    if (tid < 32) {
      const int c = tid;
      const double xn2 = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
      const double sc = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      const double alpha = rowcj[0];
      double tau, scale, beta;
      if (xn2 == 0.0) {
        tau = 0.0; scale = 0.0; beta = alpha;
      } else {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      const double v = rowcj[c] + scale * sc;   // w_c (later columns) or z_m (finished v_m)
      wz[c] = v;
      if (c >= 32 - i) Zs[c + i - 32][i] = v;
      if (c == 0) { prm[0] = tau; prm[1] = scale; prm[2] = beta; taus[i] = tau; }
    }
    __syncthreads();
    const double tau = prm[0], scale = prm[1], beta = prm[2];
    double wv[32];
#pragma unroll
    for (int c = 1; c < 32; ++c) wv[c] = (c <= 31 - i) ? tau * wz[c] : 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = j + tid + 256 * q;
      const bool below = r > cj && r < n_pad, at = r == cj;
      const double vr = at ? 1.0 : (below ? scale * A[q][0] : 0.0);
#pragma unroll
      for (int c = 1; c < 32; ++c) A[q][c] = fma(-wv[c], vr, A[q][c]);
      // the pivot column keeps v below the diagonal and beta on it
      A[q][0] = below ? vr : (at ? beta : A[q][0]);
    }
    // rotate the slots: the finished column goes to slot 31
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double f = A[q][0];
#pragma unroll
      for (int c = 0; c < 31; ++c) A[q][c] = A[q][c + 1];
      A[q][31] = f;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = j + tid + 256 * q;
    if (r < n_pad) {
#pragma unroll
      for (int c = 0; c < 32; ++c) Sj[(size_t)(cm ? cm[j + c] : j + c) * n_pad + r] = A[q][c];
    }
  }
  if (tid < 32) {
    const int m = tid;
    double Tr[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      double t = 0.0;
      if (i == m) t = taus[i];
      else if (i > m) {
        double acc = 0.0;
#pragma unroll
        for (int p2 = 0; p2 < i; ++p2)
          if (p2 >= m) acc = fma(Tr[p2], Zs[p2][i], acc);
        t = -taus[i] * acc;
      }
      Tr[i] = t;
    }
    double* Tj = Tws + job * t_stride + t_off;
#pragma unroll
    for (int i = 0; i < 32; ++i) Tj[m * 32 + i] = Tr[i];
  }
}

// The panel at column j spans n_pad - j rows: NQ = ceil((n_pad - j) / 256)
// row slots per thread, so that the later panels hold fewer registers and
// fit more workgroups per CU.
static void launch_panel32(dim3 grid, dim3 block, size_t shm, hipStream_t stream, int n_pad, int j, double* S,
                           double* Tws, int64_t t_stride, int64_t t_off, const int32_t* colmap) {
  const int nq = (n_pad - j + 255) / 256;
  if (nq >= 4)
    hipLaunchKernelGGL(qr_panel32_kernel<4>, grid, block, shm, stream, n_pad, j, S, Tws, t_stride, t_off, colmap);
  else if (nq == 3)
    hipLaunchKernelGGL(qr_panel32_kernel<3>, grid, block, shm, stream, n_pad, j, S, Tws, t_stride, t_off, colmap);
  else if (nq == 2)
    hipLaunchKernelGGL(qr_panel32_kernel<2>, grid, block, shm, stream, n_pad, j, S, Tws, t_stride, t_off, colmap);
  else
    hipLaunchKernelGGL(qr_panel32_kernel<1>, grid, block, shm, stream, n_pad, j, S, Tws, t_stride, t_off, colmap);
}

// ---------------------------------------------------------------------------
// Trailing update of the columns right of the panel: C <- C - V T^T... in the
// compact WY form H_0 H_1 ... H_31 = I - V T V^T, so Q^T C = C - V T^T V^T C.
// One workgroup per (job, 64-column tile); wave w owns 16 columns.
// ---------------------------------------------------------------------------
template <int PW>
__global__ __launch_bounds__(256) void qr_trailing_kernel(int n_pad, int j, double* __restrict__ S,
                                                          const double* __restrict__ Tws, int64_t t_stride,
                                                          int64_t t_off, const int32_t* __restrict__ colmap,
                                                          double* __restrict__ colnorm) {
  constexpr int NI = (PW + 15) / 16;     // 16-row MFMA tiles of V^T C
  const int64_t job = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  double* Sj = S + job * (size_t)n_pad * n_pad;
  const int c0w = j + PW + 64 * blockIdx.x + 16 * wave;   // first column of this wave
  __shared__ double W1[32][65];
  __shared__ double Tm[PW][PW + 1];
  for (int e = tid; e < PW * PW; e += 256) Tm[e / PW][e % PW] = Tws[job * t_stride + t_off + e];
  const bool active = c0w < n_pad;
  const bool col_ok = (c0w + lr) < n_pad;
  // logical column -> stored column (identity without a column map); V
  // column j + i is stored at vcol(j + i)
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;
  auto scol = [&](int c) { return cm ? cm[c] : c; };

  // ---- phase 1: W1 = V^T C (PW x 16 per wave) ------------------------------
  f64x4 acc[NI];
#pragma unroll
  for (int t = 0; t < NI; ++t) acc[t] = f64x4{0, 0, 0, 0};
  if (active) {
    // rows in chunks of 16; lane (lr, lg) takes rows rb .. rb + 3 of its
    // column (C) and of V column 16 t + lr, as 16-byte loads
    const double* cbase = Sj + (size_t)scol(col_ok ? c0w + lr : c0w) * n_pad;
    for (int r0 = j; r0 < n_pad; r0 += 16) {
      const int rb = r0 + 4 * lg;
      // n_pad and rb are multiples of 4: rows rb .. rb + 3 exist iff rb < n_pad
      const bool row_ok = rb < n_pad;
      double2 c01 = {0.0, 0.0}, c23 = {0.0, 0.0};
      if (row_ok) {
        c01 = *reinterpret_cast<const double2*>(cbase + rb);
        c23 = *reinterpret_cast<const double2*>(cbase + rb + 2);
      }
      const double cv[4] = {col_ok ? c01.x : 0.0, col_ok ? c01.y : 0.0, col_ok ? c23.x : 0.0, col_ok ? c23.y : 0.0};
#pragma unroll
      for (int t = 0; t < NI; ++t) {
        const int i = 16 * t + lr, d = j + i;
        double v[4];
        if (i < PW && row_ok) {
          const double* vp = Sj + (size_t)scol(d) * n_pad + rb;
          const double2 v01 = *reinterpret_cast<const double2*>(vp);
          const double2 v23 = *reinterpret_cast<const double2*>(vp + 2);
          v[0] = v01.x; v[1] = v01.y; v[2] = v23.x; v[3] = v23.y;
          if (r0 < j + PW) {   // V is stored below the diagonal, 1 on it, 0 above
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) v[jj] = rb + jj > d ? v[jj] : (rb + jj == d ? 1.0 : 0.0);
          }
        } else {
          v[0] = v[1] = v[2] = v[3] = 0.0;
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[jj], cv[jj], acc[t], 0, 0, 0);
      }
    }
  }
  // acc[t][x]: row i = 16*t + acc_row_f64(lg, x), column lr of the wave
#pragma unroll
  for (int t = 0; t < NI; ++t)
#pragma unroll
    for (int x = 0; x < 4; ++x) W1[16 * t + acc_row_f64(lg, x)][16 * wave + lr] = acc[t][x];
  __syncthreads();
  // ---- phase 2: W2 = T^T W1 (in place, column by column) -------------------
  {
    const int col = tid & 63, i0 = (tid >> 6) * 8;
    double w2[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      const int i = i0 + ii;
      double s2 = 0.0;
      if (i < PW)
        for (int m = 0; m <= i; ++m) s2 += Tm[m][i] * W1[m][col];
      w2[ii] = s2;
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) W1[i0 + ii][col] = w2[ii];
  }
  __syncthreads();
  if (!active) return;
  // ---- phase 3: C <- C - V W2 ------------------------------------------------
  // output tile C^T[c (16)][r (16)] = sum_i W2^T[c][i] V^T[i][r]
  constexpr int KSTEPS = (PW + 3) / 4;
  double aw[KSTEPS];
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks) aw[ks] = W1[4 * ks + lg][16 * wave + lr];
  int vcols[KSTEPS], ccols[4];
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks) vcols[ks] = (4 * ks + lg < PW) ? scol(j + 4 * ks + lg) : 0;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int c = c0w + acc_row_f64(lg, x);
    ccols[x] = c < n_pad ? scol(c) : -1;
  }
  // with colnorm: squared norms of the updated columns over rows >= j + PW
  // (what remains for the next panels), for the column re-ordering
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = j; r0 < n_pad; r0 += 16) {
    f64x4 a = {0, 0, 0, 0};
    const int rr = r0 + lr;
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int i = 4 * ks + lg, d = j + i;
      double bv = 0.0;
      if (i < PW && rr < n_pad) {
        bv = Sj[(size_t)vcols[ks] * n_pad + rr];
        if (r0 < j + PW) bv = rr > d ? bv : (rr == d ? 1.0 : 0.0);
      }
      a = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[ks], bv, a, 0, 0, 0);
    }
    const int r = r0 + lr;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if (ccols[x] >= 0 && r < n_pad) {
        double* cp = Sj + (size_t)ccols[x] * n_pad + r;
        const double v = *cp - a[x];
        *cp = v;
        if (r >= j + PW) sq[x] = fma(v, v, sq[x]);
      }
    }
  }
  if (colnorm) {
    // lanes with equal lg share the four columns: sum over lr (xor 1..8)
#pragma unroll
    for (int x = 0; x < 4; ++x)
      for (int o = 1; o < 16; o <<= 1) sq[x] += __shfl_xor(sq[x], o);
    if (lr == 0) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (ccols[x] >= 0) colnorm[job * n_pad + ccols[x]] = sq[x];
    }
  }
}

// The trailing update for 32-column panels (n_pad <= 1024; columns j + 32 ..
// cend - 1) with the V
// Workgroups reach the eight XCDs round-robin by linear index, and each XCD
// has its own L2.  The trailing updates launch (tile, job) grids with the
// job count rounded up to a multiple of 8 and take their (job, tile) from
// this map, which puts every tile of a job on one XCD: the V chunks, which
// all tiles of a job read, are then fetched from HBM about once per job
// instead of once per XCD.  False for the padding workgroups (uniform).
__device__ __forceinline__ bool xcd_job_tile(int64_t njobs, int64_t& job, int& tile) {
  const unsigned L = blockIdx.x + gridDim.x * blockIdx.y;
  const unsigned q = L >> 3;
  job = (int64_t)(q / gridDim.x) * 8 + (L & 7);
  tile = (int)(q % gridDim.x);
  return job < njobs;
}
static inline dim3 xcd_tile_grid(int ntiles, int64_t njobs) {
  return dim3((unsigned)ntiles, (unsigned)((njobs + 7) / 8 * 8));
}

// panel staged through LDS: every 16-row chunk of V (16 x 32) is loaded once
// per workgroup, coalesced, masked to the unit lower trapezoid, and shared
// by the four waves (instead of each wave fetching it), double-buffered with
// one barrier per chunk.  Same arithmetic as qr_trailing_kernel<32>.
// probe (colnorm required): C is not written; instead every column c gets
// colnorm = |c[j:]|^2 - |(Q^T c)[j : j + 32]|^2, its squared norm below the
// panel's rows after the panel's reflectors, by downdating (for the column
// re-ordering only, so the rounding of the difference is harmless).
__global__ __launch_bounds__(256) void qr_trailing32_kernel(int64_t njobs, int n_pad, int j, int cend,
                                                            double* __restrict__ S, const double* __restrict__ Tws,
                                                            int64_t t_stride, int64_t t_off,
                                                            const int32_t* __restrict__ colmap,
                                                            double* __restrict__ colnorm, int probe) {
  int64_t job;
  int tile;
  if (!xcd_job_tile(njobs, job, tile)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  double* Sj = S + job * (size_t)n_pad * n_pad;
  const int c0w = j + 32 + 64 * tile + 16 * wave;   // first column of this wave
  __shared__ double Vs[2][16][33];
  __shared__ double W1[32][65];
  __shared__ double Tm[32][33];
  for (int e = tid; e < 1024; e += 256) Tm[e >> 5][e & 31] = Tws[job * t_stride + t_off + e];
  const bool active = c0w < cend;   // columns j + 32 .. cend - 1 are updated
  const bool col_ok = (c0w + lr) < cend;
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;
  auto scol = [&](int c) { return cm ? cm[c] : c; };
  // V staging: thread t takes V column vd = t / 8, rows 2 (t % 8) and +1 of
  // a chunk; the next chunk's loads are issued before the products of the
  // current one, the masking is done when they are stored
  const int vd = tid >> 3, vr = 2 * (tid & 7);
  const double* vbase = Sj + (size_t)scol(j + vd) * n_pad + vr;
  auto store_v = [&](int r0, int buf, double2 v) {
    double a = v.x, b = v.y;
    if (r0 < j + 32) {   // V is stored below the diagonal, 1 on it, 0 above
      const int d = j + vd, ra = r0 + vr, rb = ra + 1;
      a = ra > d ? a : (ra == d ? 1.0 : 0.0);
      b = rb > d ? b : (rb == d ? 1.0 : 0.0);
    }
    Vs[buf][vr][vd] = a;
    Vs[buf][vr + 1][vd] = b;
  };
  const int nch = (n_pad - j) / 16;   // n_pad - j is a multiple of 32

  // ---- phase 1: W1 = V^T C (32 x 16 per wave) ------------------------------
  f64x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  const double* cbase = Sj + (size_t)scol(col_ok ? c0w + lr : (active ? c0w : j + 32)) * n_pad + 4 * lg;
  double2 vn = *reinterpret_cast<const double2*>(vbase + j);
  double2 cn0 = *reinterpret_cast<const double2*>(cbase + j), cn1 = *reinterpret_cast<const double2*>(cbase + j + 2);
  double sqn = 0.0;   // probe: |c[j:]|^2, this lane's rows
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = j + 16 * ch, buf = ch & 1;
    store_v(r0, buf, vn);
    const double cv[4] = {col_ok ? cn0.x : 0.0, col_ok ? cn0.y : 0.0, col_ok ? cn1.x : 0.0, col_ok ? cn1.y : 0.0};
    if (probe) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) sqn = fma(cv[jj], cv[jj], sqn);
    }
    if (ch + 1 < nch) {
      vn = *reinterpret_cast<const double2*>(vbase + r0 + 16);
      cn0 = *reinterpret_cast<const double2*>(cbase + r0 + 16);
      cn1 = *reinterpret_cast<const double2*>(cbase + r0 + 18);
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[buf][4 * lg + jj][lr], cv[jj], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[buf][4 * lg + jj][16 + lr], cv[jj], acc1, 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    W1[acc_row_f64(lg, x)][16 * wave + lr] = acc0[x];
    W1[16 + acc_row_f64(lg, x)][16 * wave + lr] = acc1[x];
  }
  __syncthreads();
  // ---- phase 2: W2 = T^T W1 (in place, column by column) -------------------
  {
    const int col = tid & 63, i0 = (tid >> 6) * 8;
    double w2[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      const int i = i0 + ii;
      double s2 = 0.0;
      for (int m = 0; m <= i; ++m) s2 += Tm[m][i] * W1[m][col];
      w2[ii] = s2;
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) W1[i0 + ii][col] = w2[ii];
  }
  __syncthreads();
  if (probe) {
    // top 32 rows of Q^T c = c[j + i] - sum_{m <= i} V[j + i][m] W2[m][c]
    // (the panel's top V block is unit lower triangular, staged in Tm); lane
    // (lr, lg) takes rows 8 lg .. 8 lg + 7 of column c0w + lr
    for (int e = tid; e < 1024; e += 256) {
      const int i = e >> 5, m = e & 31;
      Tm[i][m] = i == m ? 1.0 : (i > m ? Sj[(size_t)scol(j + m) * n_pad + j + i] : 0.0);
    }
    __syncthreads();
    const int wc = 16 * wave + lr;
    const double* ctop = Sj + (size_t)scol(col_ok ? c0w + lr : j) * n_pad + j + 8 * lg;
    double tsq = 0.0;
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      const int i = 8 * lg + ii;
      double t = ctop[ii];
      for (int m = 0; m <= i; ++m) t = fma(-Tm[i][m], W1[m][wc], t);
      tsq = fma(t, t, tsq);
    }
    // sum over the four lane groups of the column
    sqn += __shfl_xor(sqn, 16);
    sqn += __shfl_xor(sqn, 32);
    tsq += __shfl_xor(tsq, 16);
    tsq += __shfl_xor(tsq, 32);
    if (lg == 0 && col_ok) colnorm[job * n_pad + scol(c0w + lr)] = fmax(sqn - tsq, 0.0);
    return;
  }
  // ---- phase 3: C <- C - V W2 ------------------------------------------------
  // output tile C^T[c (16)][r (16)] = sum_i W2^T[c][i] V^T[i][r]
  double aw[8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) aw[ks] = W1[4 * ks + lg][16 * wave + lr];
  int ccols[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int c = c0w + acc_row_f64(lg, x);
    ccols[x] = (active && c < cend) ? scol(c) : -1;
  }
  // columns not updated read a V column instead (always there, never stored)
  const double* cp[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) cp[x] = Sj + (size_t)(ccols[x] >= 0 ? ccols[x] : scol(j)) * n_pad + lr;
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
  double cold[4];
  vn = *reinterpret_cast<const double2*>(vbase + j);
#pragma unroll
  for (int x = 0; x < 4; ++x) cold[x] = cp[x][j];
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = j + 16 * ch, buf = ch & 1;
    store_v(r0, buf, vn);
    const int r = r0 + lr;
    double cc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) cc[x] = cold[x];
    if (ch + 1 < nch) {
      vn = *reinterpret_cast<const double2*>(vbase + r0 + 16);
#pragma unroll
      for (int x = 0; x < 4; ++x) cold[x] = cp[x][r0 + 16];
    }
    __syncthreads();
    f64x4 a = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[ks], Vs[buf][lr][4 * ks + lg], a, 0, 0, 0);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if (ccols[x] >= 0) {
        const double v = cc[x] - a[x];
        Sj[(size_t)ccols[x] * n_pad + r] = v;
        if (r >= j + 32) sq[x] = fma(v, v, sq[x]);
      }
    }
  }
  if (colnorm) {
    // lanes with equal lg share the four columns: sum over lr (xor 1..8)
#pragma unroll
    for (int x = 0; x < 4; ++x)
      for (int o = 1; o < 16; o <<= 1) sq[x] += __shfl_xor(sq[x], o);
    if (lr == 0) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (ccols[x] >= 0) colnorm[job * n_pad + ccols[x]] = sq[x];
    }
  }
}

// ---------------------------------------------------------------------------
// 64-column blocks (factorisations without column re-ordering): the block's
// two 32-column panels are factored one after the other (the second after the
// first has been applied to it), then Q = (I - V1 T1 V1^T)(I - V2 T2 V2^T) =
// I - V T V^T with V = [V1 V2] and T = [[T1, -T1 (V1^T V2) T2], [0, T2]] is
// applied to the rest in one pass, half the passes over the trailing matrix
// of 32-column blocks.
//
// Per-job scratch of the blocked path (kQrBlockScratch doubles): the T of
// the first 64-column block of a 128-column step (row-major) at 0, of the
// second at 4096, and the T of both, as MFMA A fragments of its transpose,
// at 8192 (t128_frag).
constexpr int64_t kT64Stride = kQrBlockScratch;
constexpr int kT128Off = 8192;
// Fragment (g, ks) of T^T (128 x 128, T upper triangular): rows 16 g .. 16 g
// + 15, columns 4 ks .. 4 ks + 3, only ks <= 4 g + 3 (the rest is zero);
// lane (lr, lg) holds T[4 ks + lg][16 g + lr].  144 fragments of 64 doubles.
__device__ __forceinline__ int t128_frag(int g, int ks) { return 2 * g * (g + 1) + ks; }

// qr_t64_kernel: T (64 x 64, row-major) of the block at column j into T64
// (+ job * kT64Stride), one workgroup per job.  V1^T V2 only involves rows >= j + 32 (V2 vanishes
// above); each wave forms one 16 x 16 tile of it with MFMA, a lane taking
// two consecutive rows per step (16-byte loads; V is stored column-major).
__global__ __launch_bounds__(256) void qr_t64_kernel(int n_pad, int j, const double* __restrict__ S,
                                                     const double* __restrict__ Tws, int64_t t_stride, int64_t t_off1,
                                                     int64_t t_off2, double* __restrict__ T64,
                                                     const int32_t* __restrict__ colmap) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const double* Sj = S + job * (size_t)n_pad * n_pad;
  __shared__ double X[32][33], T1[32][33], T2[32][33], Y[32][33];
  for (int e = tid; e < 1024; e += 256) {
    T1[e >> 5][e & 31] = Tws[job * t_stride + t_off1 + e];
    T2[e >> 5][e & 31] = Tws[job * t_stride + t_off2 + e];
  }
  const int ta = wave >> 1, tb = wave & 1;
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;
  auto scol = [&](int c) { return cm ? cm[c] : c; };                  // logical -> stored column
  const double* c1 = Sj + (size_t)scol(j + 16 * ta + lr) * n_pad;    // column of V1 (all rows >= j + 32 below its diagonal)
  const int d2 = j + 32 + 16 * tb + lr;                                // diagonal row of this V2 column
  const double* c2 = Sj + (size_t)scol(d2) * n_pad;
  // four independent accumulators over interleaved 8-row chunks, so that
  // the loads of four chunks are in flight at once (n_pad - j - 32 is a
  // multiple of 32)
  f64x4 acc4[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc4[u] = f64x4{0, 0, 0, 0};
  for (int r0 = j + 32; r0 < n_pad; r0 += 32) {
    double2 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 8 * u + 2 * lg;
      a[u] = *reinterpret_cast<const double2*>(c1 + r);
      b[u] = *reinterpret_cast<const double2*>(c2 + r);
      b[u].x = r > d2 ? b[u].x : (r == d2 ? 1.0 : 0.0);
      b[u].y = r + 1 > d2 ? b[u].y : (r + 1 == d2 ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc4[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].x, acc4[u], 0, 0, 0);
      acc4[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[u].y, acc4[u], 0, 0, 0);
    }
  }
  f64x4 acc;
#pragma unroll
  for (int x = 0; x < 4; ++x) acc[x] = ((acc4[0][x] + acc4[1][x]) + acc4[2][x]) + acc4[3][x];
#pragma unroll
  for (int x = 0; x < 4; ++x) X[16 * ta + acc_row_f64(lg, x)][16 * tb + lr] = acc[x];
  __syncthreads();
  for (int e = tid; e < 1024; e += 256) {   // Y = X T2
    const int a = e >> 5, b = e & 31;
    double v = 0.0;
    for (int m = 0; m <= b; ++m) v = fma(X[a][m], T2[m][b], v);
    Y[a][b] = v;
  }
  __syncthreads();
  double* Tj = T64 + job * kT64Stride;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, k = e & 63;
    double v;
    if (i < 32 && k < 32) v = T1[i][k];
    else if (i >= 32 && k >= 32) v = T2[i - 32][k - 32];
    else if (i >= 32) v = 0.0;
    else {   // T12 = -T1 Y
      v = 0.0;
      for (int m = i; m < 32; ++m) v = fma(T1[i][m], Y[m][k - 32], v);
      v = -v;
    }
    Tj[e] = v;
  }
}

// C <- C - V T^T V^T C for the 64-column block at column j (columns j + 64 ..
// n_pad - 1, (job, 64-column tile) workgroups): phase 1 W = V^T C with the V
// chunks staged through LDS as in qr_trailing32_kernel; phase 2 W <- T^T W
// with MFMA (T packed upper in the staging buffer); phase 3 C <- C - V W.
__global__ __launch_bounds__(256) void qr_trailing64_kernel(int64_t njobs, int n_pad, int j, int cend,
                                                            double* __restrict__ S, const double* __restrict__ T64,
                                                            const int32_t* __restrict__ colmap,
                                                            double* __restrict__ colnorm) {
  int64_t job;
  int tile;
  if (!xcd_job_tile(njobs, job, tile)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  double* Sj = S + job * (size_t)n_pad * n_pad;
  const int c0w = j + 64 + 64 * tile + 16 * wave;   // first (logical) column of this wave
  __shared__ double Vs[2][16][65];   // V chunks; T (packed upper, 2080 entries) in phase 2
  __shared__ double W1[64][65];
  const bool active = c0w < cend;   // columns j + 64 .. cend - 1 are updated
  const bool col_ok = (c0w + lr) < cend;
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;
  auto scol = [&](int c) { return cm ? cm[c] : c; };   // logical -> stored column
  // V staging: thread t takes V column vd = t / 4, rows 4 (t % 4) .. + 3 of a
  // chunk; the next chunk's loads are issued before the products of the
  // current one, the masking is done when they are stored
  const int vd = tid >> 2, vr = 4 * (tid & 3);
  const double* vbase = Sj + (size_t)scol(j + vd) * n_pad + vr;
  auto load_v = [&](int r0, double2 (&v)[2]) {
    v[0] = *reinterpret_cast<const double2*>(vbase + r0);
    v[1] = *reinterpret_cast<const double2*>(vbase + r0 + 2);
  };
  auto store_v = [&](int r0, int buf, const double2 (&v)[2]) {
    double a[4] = {v[0].x, v[0].y, v[1].x, v[1].y};
    if (r0 < j + 64) {   // V is stored below the diagonal, 1 on it, 0 above
      const int d = j + vd;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = r0 + vr + q;
        a[q] = rr > d ? a[q] : (rr == d ? 1.0 : 0.0);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Vs[buf][vr + q][vd] = a[q];
  };
  const int nch = (n_pad - j) / 16;   // n_pad - j is a multiple of 32

  // ---- phase 1: W1 = V^T C (64 x 16 per wave) ------------------------------
  f64x4 acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = f64x4{0, 0, 0, 0};
  const double* cbase = Sj + (size_t)scol(col_ok ? c0w + lr : (active ? c0w : j + 64)) * n_pad + 4 * lg;
  double2 vn[2], cn[2];
  load_v(j, vn);
  cn[0] = *reinterpret_cast<const double2*>(cbase + j);
  cn[1] = *reinterpret_cast<const double2*>(cbase + j + 2);
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = j + 16 * ch, buf = ch & 1;
    store_v(r0, buf, vn);
    const double cv[4] = {col_ok ? cn[0].x : 0.0, col_ok ? cn[0].y : 0.0, col_ok ? cn[1].x : 0.0,
                          col_ok ? cn[1].y : 0.0};
    if (ch + 1 < nch) {
      load_v(r0 + 16, vn);
      cn[0] = *reinterpret_cast<const double2*>(cbase + r0 + 16);
      cn[1] = *reinterpret_cast<const double2*>(cbase + r0 + 18);
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[buf][4 * lg + jj][16 * g + lr], cv[jj], acc[g], 0, 0, 0);
  }
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int x = 0; x < 4; ++x) W1[16 * g + acc_row_f64(lg, x)][16 * wave + lr] = acc[g][x];
  __syncthreads();
  // ---- phase 2: W2 = T^T W1, each wave on its own 16 columns --------------
  double* Tp = &Vs[0][0][0];   // T[m][i], m <= i, at i (i + 1) / 2 + m
  const double* Tj = T64 + job * kT64Stride;
  for (int e = tid; e < 4096; e += 256) {
    const int m = e >> 6, i = e & 63;
    if (m <= i) Tp[((i * (i + 1)) >> 1) + m] = Tj[e];
  }
  __syncthreads();
  {
    f64x4 w2[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) w2[g] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const double b = W1[4 * ks + lg][16 * wave + lr];
      const int m = 4 * ks + lg;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i = 16 * g + lr;   // A = T^T: A[i][m] = T[m][i]
        const double a = m <= i ? Tp[((i * (i + 1)) >> 1) + m] : 0.0;
        w2[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, w2[g], 0, 0, 0);
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int x = 0; x < 4; ++x) W1[16 * g + acc_row_f64(lg, x)][16 * wave + lr] = w2[g][x];
  }
  __syncthreads();
  // ---- phase 3: C <- C - V W2 (and, with colnorm, the squared norms of the
  // updated columns below the block's rows for the re-ordering) -------------
  // output tile C^T[c (16)][r (16)] = sum_i W2^T[c][i] V^T[i][r]
  double aw[16];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) aw[ks] = W1[4 * ks + lg][16 * wave + lr];
  int ccols[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int c = c0w + acc_row_f64(lg, x);
    ccols[x] = (active && c < cend) ? scol(c) : -1;
  }
  // columns not updated read a V column instead (always there, never stored)
  const double* cp[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) cp[x] = Sj + (size_t)(ccols[x] >= 0 ? ccols[x] : scol(j)) * n_pad + lr;
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
  double cold[4];
  load_v(j, vn);
#pragma unroll
  for (int x = 0; x < 4; ++x) cold[x] = cp[x][j];
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = j + 16 * ch, buf = ch & 1;
    store_v(r0, buf, vn);
    const int r = r0 + lr;
    double cc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) cc[x] = cold[x];
    if (ch + 1 < nch) {
      load_v(r0 + 16, vn);
#pragma unroll
      for (int x = 0; x < 4; ++x) cold[x] = cp[x][r0 + 16];
    }
    __syncthreads();
    f64x4 a = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) a = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[ks], Vs[buf][lr][4 * ks + lg], a, 0, 0, 0);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if (ccols[x] >= 0) {
        const double v = cc[x] - a[x];
        Sj[(size_t)ccols[x] * n_pad + r] = v;
        if (r >= j + 64) sq[x] = fma(v, v, sq[x]);
      }
    }
  }
  if (colnorm) {
    // lanes with equal lg share the four columns: sum over lr (xor 1..8)
#pragma unroll
    for (int x = 0; x < 4; ++x)
      for (int o = 1; o < 16; o <<= 1) sq[x] += __shfl_xor(sq[x], o);
    if (lr == 0) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (ccols[x] >= 0) colnorm[job * n_pad + ccols[x]] = sq[x];
    }
  }
}

// qr_t128_kernel: T of the 128 columns j .. j + 127 (blocks A and B, their
// 64 x 64 T factors at 0 and 4096 of the job's scratch) as
// [[T_A, -T_A (V_A^T V_B) T_B], [0, T_B]], written as A fragments of its
// transpose (t128_frag).  One workgroup per job.  X = V_A^T V_B only
// involves rows >= j + 64 (V_B vanishes above), where every V_A entry lies
// strictly below its diagonal; wave w forms the four 16 x 16 tiles of row
// block w, a lane taking two consecutive rows per step.  The two 64 x 64
// triangular products run on MFMA as well (only the upper triangles of T_A
// and T_B are read); the tiles of T_AB end in the accumulator layout, which
// is the fragment layout, and are stored from the registers.
__global__ __launch_bounds__(256) void qr_t128_kernel(int n_pad, int j, const double* __restrict__ S,
                                                      double* __restrict__ T64) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int ws = __builtin_amdgcn_readfirstlane(wave);
  const double* Sj = S + job * (size_t)n_pad * n_pad;
  double* Tb = T64 + job * kT64Stride;
  const double* TA = Tb;
  const double* TB = Tb + 4096;
  __shared__ double L[64][65];   // X, then X T_B
  const double* ca = Sj + (size_t)(j + 16 * ws + lr) * n_pad;
  const double* cb[4];
  int d2[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) {
    d2[tb] = j + 64 + 16 * tb + lr;   // diagonal row of this V_B column
    cb[tb] = Sj + (size_t)d2[tb] * n_pad;
  }
  f64x4 acc[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) acc[tb] = f64x4{0, 0, 0, 0};
  for (int r0 = j + 64; r0 < n_pad; r0 += 16) {   // n_pad - j - 64 is a multiple of 32
    double2 a[2], b[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = r0 + 8 * u + 2 * lg;
      a[u] = *reinterpret_cast<const double2*>(ca + r);
#pragma unroll
      for (int tb = 0; tb < 4; ++tb) {
        double2 v = *reinterpret_cast<const double2*>(cb[tb] + r);
        v.x = r > d2[tb] ? v.x : (r == d2[tb] ? 1.0 : 0.0);
        v.y = r + 1 > d2[tb] ? v.y : (r + 1 == d2[tb] ? 1.0 : 0.0);
        b[u][tb] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int tb = 0; tb < 4; ++tb) acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u][tb].x, acc[tb], 0, 0, 0);
#pragma unroll
      for (int tb = 0; tb < 4; ++tb) acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[u][tb].y, acc[tb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int x = 0; x < 4; ++x) L[16 * ws + acc_row_f64(lg, x)][16 * tb + lr] = acc[tb][x];
  __syncthreads();
  // Y = X T_B: tile (w, tb) over k-steps ks <= 4 tb + 3 (T_B upper)
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) {
    f64x4 y = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks <= 4 * tb + 3; ++ks) {
      const int k = 4 * ks + lg, c = 16 * tb + lr;
      const double bv = k <= c ? TB[k * 64 + c] : 0.0;
      y = __builtin_amdgcn_mfma_f64_16x16x4f64(L[16 * ws + lr][k], bv, y, 0, 0, 0);
    }
    acc[tb] = y;
  }
  __syncthreads();
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int x = 0; x < 4; ++x) L[16 * ws + acc_row_f64(lg, x)][16 * tb + lr] = acc[tb][x];
  __syncthreads();
  // T_AB = -T_A Y: tile (w, tb) over k-steps ks >= 4 w (T_A upper)
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) acc[tb] = f64x4{0, 0, 0, 0};
  for (int ks = 4 * ws; ks < 16; ++ks) {
    const int i = 16 * ws + lr, m = 4 * ks + lg;
    const double av = m >= i ? TA[i * 64 + m] : 0.0;
#pragma unroll
    for (int tb = 0; tb < 4; ++tb)
      acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, L[m][16 * tb + lr], acc[tb], 0, 0, 0);
  }
  // fragments (g, ks) of T^T: T_AB for g >= 4, ks < 16 from the registers
  // (tile (ks / 4, g - 4), register ks % 4); T_A and T_B from the scratch
  double* F = Tb + kT128Off + lane;
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int x = 0; x < 4; ++x) F[(size_t)t128_frag(4 + tb, 4 * ws + x) * 64] = -acc[tb][x];
  for (int g = 0; g < 8; ++g)
    for (int ks = g < 4 ? 0 : 16; ks <= 4 * g + 3; ++ks) {
      const int f = t128_frag(g, ks);
      if ((f & 3) != ws) continue;
      const int m = 4 * ks + lg, i = 16 * g + lr;   // T[m][i]
      double v = 0.0;
      if (m <= i) v = g < 4 ? TA[m * 64 + i] : TB[(m - 64) * 64 + (i - 64)];
      F[(size_t)f * 64] = v;
    }
}

// C <- C - V T^T V^T C for the 128 columns j .. j + 127 (V = [V_A V_B], T
// from qr_t128_kernel) on columns j + 128 .. n_pad - 1, one pass over C
// for two 64-column blocks.  (job, 64-column tile) workgroups, wave w owning
// 16 columns.  W = V^T C (128 x 16 per wave) stays in registers: the MFMA
// accumulator of v_mfma_f64_16x16x4 holds row lg + 4 i of its tile in
// register i, which is also where the B operand of the k-step over rows 4 i
// .. 4 i + 3 and the A operand of the transposed product expect it, so W is
// multiplied by T^T in place (tiles from the last to the first, each new
// tile only reading the old ones at or above it) and used directly as the
// left factor of C - V W.  The 16-row V chunks are staged through LDS,
// double-buffered; V_B (zero above row j + 64) is skipped where it vanishes.
// lower_zero: every column c of C is still zero above row c (the first step
// on a lower triangular matrix); chunks of V^T C above a wave's columns are
// then skipped.
__global__ __launch_bounds__(256, 3) void qr_trailing128_kernel(int64_t njobs, int n_pad, int j,
                                                                double* __restrict__ S,
                                                                const double* __restrict__ T64, int lower_zero) {
  int64_t job;
  int tile;
  if (!xcd_job_tile(njobs, job, tile)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  double* Sj = S + job * (size_t)n_pad * n_pad;
  const int c0w = j + 128 + 64 * tile + 16 * wave;   // first column of this wave
  __shared__ double Vs[2][16][129];
  const bool active = c0w < n_pad;
  const bool col_ok = (c0w + lr) < n_pad;
  // V staging: thread t takes V column vd = t / 2, rows 8 (t % 2) .. + 7 of
  // a chunk; the loads of the next chunk are issued before the products of
  // the current one, the masking is done when they are stored
  const int vd = tid >> 1, vr = 8 * (tid & 1);
  const double* vbase = Sj + (size_t)(j + vd) * n_pad;
  auto load_v = [&](int r0, double2 (&a)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = *reinterpret_cast<const double2*>(vbase + r0 + vr + 2 * q);
  };
  auto store_v = [&](int r0, int buf, const double2 (&a)[4]) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = a[q].x;
      v[2 * q + 1] = a[q].y;
    }
    if (r0 < j + 128) {   // V is stored below the diagonal, 1 on it, 0 above
      const int d = j + vd;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int rr = r0 + vr + q;
        v[q] = rr > d ? v[q] : (rr == d ? 1.0 : 0.0);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) Vs[buf][vr + q][vd] = v[q];
  };
  const int nch = (n_pad - j) / 16;   // n_pad - j is a multiple of 32

  // ---- phase 1: W = V^T C --------------------------------------------------
  f64x4 w[8];
#pragma unroll
  for (int g = 0; g < 8; ++g) w[g] = f64x4{0, 0, 0, 0};
  const double* cbase = Sj + (size_t)(col_ok ? c0w + lr : (active ? c0w : j + 128)) * n_pad + 4 * lg;
  double2 va[4], cn[2];
  load_v(j, va);
  cn[0] = *reinterpret_cast<const double2*>(cbase + j);
  cn[1] = *reinterpret_cast<const double2*>(cbase + j + 2);
  const int zero_below = lower_zero ? c0w : 0;   // rows < zero_below of this wave's columns are zero
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = j + 16 * ch, buf = ch & 1;
    store_v(r0, buf, va);
    const double cv[4] = {col_ok ? cn[0].x : 0.0, col_ok ? cn[0].y : 0.0, col_ok ? cn[1].x : 0.0,
                          col_ok ? cn[1].y : 0.0};
    if (ch + 1 < nch) {
      load_v(r0 + 16, va);
      if (r0 + 32 > zero_below) {
        cn[0] = *reinterpret_cast<const double2*>(cbase + r0 + 16);
        cn[1] = *reinterpret_cast<const double2*>(cbase + r0 + 18);
      }
    }
    __syncthreads();
    if (r0 + 16 <= zero_below) continue;   // C vanishes in this chunk (uniform per wave)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        w[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[buf][4 * lg + jj][16 * g + lr], cv[jj], w[g], 0, 0, 0);
    if (r0 + 16 > j + 64) {   // V_B has entries in this chunk (uniform)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int g = 4; g < 8; ++g)
          w[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[buf][4 * lg + jj][16 * g + lr], cv[jj], w[g], 0, 0, 0);
    }
  }
  // ---- phase 2: W <- T^T W in registers ------------------------------------
  {
    const double* Tf = T64 + job * kT64Stride + kT128Off + lane;
#pragma unroll
    for (int g = 7; g >= 0; --g) {
      f64x4 e0 = {0, 0, 0, 0}, e1 = {0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks <= 4 * g + 3; ks += 2) {
        e0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Tf[t128_frag(g, ks) * 64], w[ks >> 2][ks & 3], e0, 0, 0, 0);
        e1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Tf[t128_frag(g, ks + 1) * 64], w[(ks + 1) >> 2][(ks + 1) & 3],
                                                  e1, 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) w[g][x] = e0[x] + e1[x];
      __builtin_amdgcn_sched_barrier(0);   // keep each tile's fragment loads with its products
    }
  }
  // ---- phase 3: C <- C - V W -----------------------------------------------
  // output tile C^T[c (16)][r (16)] = sum_i W^T[c][i] V^T[i][r]
  int ccols[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int c = c0w + acc_row_f64(lg, x);
    ccols[x] = (active && c < n_pad) ? c : -1;
  }
  double* cp[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) cp[x] = Sj + (size_t)(ccols[x] >= 0 ? ccols[x] : j + 128) * n_pad + lr;
  double cold[4];
  load_v(j, va);
#pragma unroll
  for (int x = 0; x < 4; ++x) cold[x] = cp[x][j];
  __syncthreads();   // every wave is done with the phase-1 V chunks
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = j + 16 * ch, buf = ch & 1;
    store_v(r0, buf, va);
    double cc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) cc[x] = cold[x];
    if (ch + 1 < nch) {
      load_v(r0 + 16, va);
#pragma unroll
      for (int x = 0; x < 4; ++x) cold[x] = cp[x][r0 + 16];
    }
    __syncthreads();
    f64x4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 16; ks += 2) {
      a = __builtin_amdgcn_mfma_f64_16x16x4f64(w[ks >> 2][ks & 3], Vs[buf][lr][4 * ks + lg], a, 0, 0, 0);
      b = __builtin_amdgcn_mfma_f64_16x16x4f64(w[(ks + 1) >> 2][(ks + 1) & 3], Vs[buf][lr][4 * ks + 4 + lg], b, 0,
                                               0, 0);
    }
    if (r0 + 16 > j + 64) {
#pragma unroll
      for (int ks = 16; ks < 32; ks += 2) {
        a = __builtin_amdgcn_mfma_f64_16x16x4f64(w[ks >> 2][ks & 3], Vs[buf][lr][4 * ks + lg], a, 0, 0, 0);
        b = __builtin_amdgcn_mfma_f64_16x16x4f64(w[(ks + 1) >> 2][(ks + 1) & 3], Vs[buf][lr][4 * ks + 4 + lg], b, 0,
                                                 0, 0);
      }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
      if (ccols[x] >= 0) cp[x][r0] = cc[x] - (a[x] + b[x]);
  }
}

// Column re-ordering between panels: the not yet factored logical columns
// j0 .. n_pad - 1 are put in decreasing order of their remaining squared
// norms (ties by position), by permuting the column map.  One workgroup per
// job, bitonic sort in LDS.
__global__ __launch_bounds__(256) void resort_cols_kernel(int n_pad, int j0, const double* __restrict__ colnorm,
                                                          int32_t* __restrict__ colmap,
                                                          const int* __restrict__ stopped) {
  __shared__ double key[1024];
  __shared__ int idx[1024];
  __shared__ int32_t old[1024];
  const int64_t job = blockIdx.x;
  // a job whose first QR has stopped keeps its column order (the columns it
  // did not factor are dropped, whatever the other jobs of the batch do)
  if (stopped && stopped[job] < n_pad) return;
  const int m = n_pad - j0;
  int P = 1;
  while (P < m) P <<= 1;
  int32_t* cm = colmap + job * n_pad;
  for (int t = threadIdx.x; t < P; t += 256) {
    if (t < m) {
      old[t] = cm[j0 + t];
      const double v = colnorm[job * n_pad + old[t]];
      key[t] = v == v ? v : 0.0;   // a NaN (failed job) must not break the order
    } else {
      key[t] = -1.0;   // padding sorts last
    }
    idx[t] = t;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += 256) {
        const int i = 2 * stride * (t / stride) + (t % stride), k = i + stride;
        const bool up = (i & size) == 0;
        const double ki = key[i], kk = key[k];
        const int ii = idx[i], ik = idx[k];
        const bool i_first = (ki > kk) || (ki == kk && ii < ik);
        if (up ? !i_first : i_first) { key[i] = kk; key[k] = ki; idx[i] = ik; idx[k] = ii; }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < m; t += 256) cm[j0 + t] = old[idx[t] < m ? idx[t] : t];
}

// W[r][c] = R[r][c] = S[colmap[c]][r] for r <= c, r < rlim and c < clim,
// else 0 (rows of R for the Jacobi or the next QR; colmap NULL: identity;
// rlim / clim multiples of 32: the rows and columns of R known to be zero;
// rlim_job (or NULL): a lower row limit per job, a multiple of 32).
// One 32 x 32 tile per workgroup, transposed through LDS; tiles wholly below
// the diagonal or beyond the limits are written as zeros without reading S.
__global__ void r_rows_kernel(int n_pad, const double* __restrict__ S, double* __restrict__ W,
                              const int32_t* __restrict__ colmap, int rlim, int clim,
                              const int* __restrict__ rlim_job = nullptr) {
  const int64_t job = blockIdx.z;
  if (rlim_job) rlim = min(rlim, rlim_job[job]);
  __shared__ double tile[32][33];
  const size_t per = (size_t)n_pad * n_pad;
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;   // bx: column c block, by: row r block
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  double* Wj = W + job * per;
  if (by > bx + 31 || by >= rlim || bx >= clim) {   // zero everywhere (uniform)
    for (int yy = ty; yy < 32; yy += 8) Wj[(size_t)(by + yy) * n_pad + bx + tx] = 0.0;
    return;
  }
  const int32_t* cm = colmap ? colmap + job * n_pad : nullptr;
  for (int yy = ty; yy < 32; yy += 8)
    tile[yy][tx] = S[job * per + (size_t)(cm ? cm[bx + yy] : bx + yy) * n_pad + by + tx];  // [c][r]
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int r = by + yy, c = bx + tx;
    Wj[(size_t)r * n_pad + c] = (r <= c) ? tile[tx][yy] : 0.0;
  }
}

// Blocked Householder QR of the column-stored matrices S (in place: V below
// the diagonal, R on and above).  Panels of PW columns: 32 for n_pad <= 1024
// (4 rows per thread in 256 threads), 8 for n_pad <= 4096 (8 rows per thread
// in 512 threads).  keep_T: the T factor of panel p is kept at
// Tws[job * n_pad * PW + p * PW^2], otherwise every panel reuses
// Tws[job * PW^2].
// colmap / colnorm (n_pad entries per job, 32-column panels only): before
// every panel after the first, the remaining columns are re-ordered by their
// current norms below the factored rows (a blocked form of column pivoting:
// the columns are not moved, the panel and trailing kernels address them
// through the map, which ends as the logical -> stored column permutation).
// Early stop of the re-ordered first QR.  Per job: the squared norms (below
// the factored rows) of the columns from logical position j0 on, summed,
// against budget_sq times the squared leading diagonal entry of R (at most
// s_1^2): dropping that rest perturbs M P by at most its Frobenius norm, so
// the singular values move by at most sqrt(budget_sq) s_1.  A job within it
// stops here (stopped[job] = j0: its rows of R from j0 on are dropped and
// its column order is frozen, so that its result does not depend on the
// other jobs, which the batch keeps factoring); *any becomes 1 while some
// job has not stopped.
__global__ __launch_bounds__(256) void trailing_above_kernel(int n_pad, int j0, double budget_sq,
                                                             const double* __restrict__ S,
                                                             const int32_t* __restrict__ colmap,
                                                             const double* __restrict__ colnorm, int* __restrict__ any,
                                                             int* __restrict__ stopped) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (stopped[job] < n_pad) return;   // stopped at an earlier check (uniform)
  const int32_t* cm = colmap + job * n_pad;
  __shared__ double red[4];
  double sum = 0.0;
  for (int p = j0 + tid; p < n_pad; p += 256) sum += colnorm[job * n_pad + cm[p]];
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
  if (lane == 0) red[wave] = sum;
  __syncthreads();
  if (tid == 0) {
    const double tot = (red[0] + red[1]) + (red[2] + red[3]);
    const double r00 = S[(size_t)job * n_pad * n_pad + (size_t)cm[0] * n_pad];
    if (tot <= budget_sq * r00 * r00) stopped[job] = j0;
    else atomicMax(any, 1);   // NaN counts as above
  }
}

__global__ void fill_int_kernel(int64_t n, int* __restrict__ p, int v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Rows of R1 from each job's own rank limit on become zero: rows >= the
// job's rank rows rounded up to 128 (at least 128, at most n_pad), as a
// batch of that job alone would set them.  One workgroup per 8 rows and job.
__global__ void zero_rows_from_kernel(int n_pad, double* __restrict__ W, const int* __restrict__ rows_job) {
  const int64_t job = blockIdx.y;
  const int r0 = 8 * blockIdx.x;
  const int rk = rows_job[job];
  const int from = min(n_pad, max(128, 128 * ((rk + 127) / 128)));
  if (r0 + 7 < from) return;
  double* Wj = W + job * (size_t)n_pad * n_pad;
  for (int e = threadIdx.x; e < 8 * n_pad; e += 256) {
    const int r = r0 + e / n_pad;
    if (r >= from) Wj[(size_t)r * n_pad + e % n_pad] = 0.0;
  }
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

// p[job * stride + e] = 0 for e < n (one job per grid row).
__global__ void zero_tail_kernel(int64_t n, double* __restrict__ p, int64_t stride) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) p[blockIdx.y * stride + e] = 0.0;
}

template <int NT, int MAXQ, int PW>
static hipError_t qr_factor_t(int64_t njobs, int n_pad, double* S, double* Tws, bool keep_T, int32_t* colmap,
                              double* colnorm, double* T64, bool lower, hipStream_t stream, KernelTimer* tq,
                              double* tq_flops, int ncols, QrStop* stop) {
  if (PW == 32 && !colmap && T64) {
    // ncols (a multiple of 128, or n_pad): only the first ncols columns are
    // factored and updated; the others must be zero (then they stay zero,
    // and the kept T of their panels is set to zero: those reflectors are
    // the identity)
    // Steps of 128 columns, each two 64-column blocks A (j .. j + 63) and B
    // (j + 64 .. j + 127) of two 32-column panels: A is factored and
    // applied to B's columns only, B is factored, and both are applied to
    // the rest in one pass (T of the 128 columns from the two 64-column
    // T).  T of every 32-column panel at (c / 32) * 1024 when kept, else two
    // slots per job; T64 holds kQrBlockScratch doubles per job.
    const int64_t ts = keep_T ? (int64_t)n_pad * 32 : 2048;
    auto block64 = [&](int c, double* Tslot) -> bool {   // false: the matrix ends inside the block
      const int64_t o1 = keep_T ? (int64_t)(c / 32) * 1024 : 0, o2 = keep_T ? o1 + 1024 : 1024;
      launch_panel32(dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, c, S, Tws, ts, o1, (const int32_t*)nullptr);
      if (c + 32 >= n_pad) return false;
      hipLaunchKernelGGL(qr_trailing32_kernel, xcd_tile_grid(1, njobs), dim3(256), 0, stream, njobs, n_pad, c, c + 64,
                         S, (const double*)Tws, ts, o1, (const int32_t*)nullptr, (double*)nullptr, 0);
      launch_panel32(dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, c + 32, S, Tws, ts, o2,
                     (const int32_t*)nullptr);
      if (c + 64 >= n_pad) return false;
      hipLaunchKernelGGL(qr_t64_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, c, (const double*)S,
                         (const double*)Tws, ts, o1, o2, Tslot, (const int32_t*)nullptr);
      return true;
    };
    for (int j = 0; j < ncols; j += 128) {
      if (!block64(j, T64)) break;
      hipLaunchKernelGGL(qr_trailing64_kernel, xcd_tile_grid(1, njobs), dim3(256), 0, stream, njobs, n_pad, j,
                         min(j + 128, n_pad), S, (const double*)T64, (const int32_t*)nullptr, (double*)nullptr);
      if (!block64(j + 64, T64 + 4096)) break;
      if (j + 128 >= ncols) break;   // no columns left to update
      hipLaunchKernelGGL(qr_t128_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j, (const double*)S,
                         T64);
      if (tq) {
        const hipError_t e = tq->begin(stream);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(qr_trailing128_kernel, xcd_tile_grid(ceil_div(ncols - j - 128, 64), njobs), dim3(256), 0,
                         stream, njobs, n_pad, j, S, (const double*)T64, (int)(lower && j == 0));
      if (tq) {
        const hipError_t e = tq->end(stream);
        if (e != hipSuccess) return e;
        // dense count of C <- C - V (T^T (V^T C)): m = n_pad - j rows,
        // c = n_pad - j - 128 columns, V m x 128, T triangular
        const double m = n_pad - j, c = ncols - j - 128;
        *tq_flops += (double)njobs * (4.0 * m * 128.0 * c + 128.0 * 128.0 * c);
      }
    }
    if (keep_T && ncols < n_pad) {
      const int64_t nz = (int64_t)(n_pad - ncols) * 32;   // T of the panels from column ncols on
      hipLaunchKernelGGL(zero_tail_kernel, dim3((unsigned)ceil_div(nz, 256), (unsigned)njobs), dim3(256), 0, stream,
                         nz, Tws + (int64_t)ncols * 32, ts);
    }
    return hipGetLastError();
  }
  if (PW == 32 && colmap && colnorm && T64) {
    // Re-ordered columns in 64-column steps: panel A (the 32 columns of
    // largest remaining norm), a read-only pass that gives every remaining
    // column its squared norm below A's rows by downdating, the re-ordering,
    // A applied to the 32 columns chosen for panel B only, panel B, and one
    // pass of both over the rest, which also leaves the exact norms below
    // the step's rows for the next re-ordering: four passes over the
    // trailing columns per 64 columns instead of six.
    hipError_t e = launch_iota(njobs, n_pad, colmap, stream);
    if (e != hipSuccess) return e;
    int* const stopped = stop ? stop->rows_job : nullptr;
    if (stopped)
      hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)ceil_div(njobs, 256)), dim3(256), 0, stream, njobs, stopped,
                         n_pad);
    const int64_t ts = keep_T ? (int64_t)n_pad * 32 : 2048;
    for (int j = 0; j < n_pad; j += 64) {
      const int64_t o1 = keep_T ? (int64_t)(j / 32) * 1024 : 0, o2 = keep_T ? o1 + 1024 : 1024;
      if (j > 0)
        hipLaunchKernelGGL(resort_cols_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j,
                           (const double*)colnorm, colmap, (const int*)stopped);
      launch_panel32(dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j, S, Tws, ts, o1, (const int32_t*)colmap);
      const int rest = n_pad - j - 32;
      if (rest <= 0) break;
      hipLaunchKernelGGL(qr_trailing32_kernel, xcd_tile_grid(ceil_div(rest, 64), njobs), dim3(256), 0, stream, njobs,
                         n_pad, j, n_pad, S, (const double*)Tws, ts, o1, (const int32_t*)colmap, colnorm, 1);
      hipLaunchKernelGGL(resort_cols_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j + 32,
                         (const double*)colnorm, colmap, (const int*)stopped);
      hipLaunchKernelGGL(qr_trailing32_kernel, xcd_tile_grid(1, njobs), dim3(256), 0, stream, njobs, n_pad, j, j + 64,
                         S, (const double*)Tws, ts, o1, (const int32_t*)colmap, (double*)nullptr, 0);
      launch_panel32(dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j + 32, S, Tws, ts, o2,
                     (const int32_t*)colmap);
      if (j + 64 >= n_pad) break;
      hipLaunchKernelGGL(qr_t64_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j, (const double*)S,
                         (const double*)Tws, ts, o1, o2, T64, (const int32_t*)colmap);
      hipLaunchKernelGGL(qr_trailing64_kernel, xcd_tile_grid(ceil_div(n_pad - j - 64, 64), njobs), dim3(256), 0,
                         stream, njobs, n_pad, j, n_pad, S, (const double*)T64, (const int32_t*)colmap, colnorm);
      if (stop) {   // every job within the budget (each stopped at its own check): stop here
        hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, stream, stop->dev, 0);
        hipLaunchKernelGGL(trailing_above_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j + 64,
                           stop->budget * stop->budget, (const double*)S, (const int32_t*)colmap,
                           (const double*)colnorm, stop->dev, stopped);
        hipError_t e = hipMemcpyAsync(stop->host, stop->dev, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (*stop->host == 0) {
          stop->rows = j + 64;
          break;
        }
      }
    }
    return hipGetLastError();
  }
  const int64_t t_stride = keep_T ? (int64_t)n_pad * PW : (int64_t)PW * PW;
  if (colmap) {
    hipError_t e = launch_iota(njobs, n_pad, colmap, stream);
    if (e != hipSuccess) return e;
  }
  for (int j = 0; j < n_pad; j += PW) {
    const int64_t t_off = keep_T ? (int64_t)(j / PW) * PW * PW : 0;
    if (NT == 256 && MAXQ == 4 && PW == 32)
      launch_panel32( dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j, S, Tws, t_stride,
                         t_off, (const int32_t*)colmap);
    else
      hipLaunchKernelGGL((qr_panel_kernel<NT, MAXQ, PW>), dim3((unsigned)njobs), dim3(NT), 0, stream, n_pad, j, S,
                         Tws, t_stride, t_off);
    const int rest = n_pad - j - PW;
    if (rest > 0) {
      if (PW == 32)
        hipLaunchKernelGGL(qr_trailing32_kernel, xcd_tile_grid(ceil_div(rest, 64), njobs), dim3(256), 0, stream,
                           njobs, n_pad, j, n_pad, S, Tws, t_stride, t_off, (const int32_t*)colmap,
                           colmap ? colnorm : nullptr, 0);
      else
        hipLaunchKernelGGL((qr_trailing_kernel<PW>), dim3(ceil_div(rest, 64), (unsigned)njobs), dim3(256), 0, stream,
                           n_pad, j, S, Tws, t_stride, t_off, (const int32_t*)colmap, colmap ? colnorm : nullptr);
      if (colmap)
        hipLaunchKernelGGL(resort_cols_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, j + PW,
                           (const double*)colnorm, colmap, (const int*)nullptr);
    }
  }
  return hipGetLastError();
}

// T64 (kQrBlockScratch doubles per job, or NULL): scratch that enables the
// 64-column blocks when the columns are not re-ordered (n_pad <= 1024).
// lower: S is lower triangular on entry (the transpose of an R factor).
// tq / tq_flops (or NULL): HIP-event timer of the 128-column trailing
// updates and the running sum of their algorithmic flops.
// ncols (0: n_pad): with T64 and no column map, factor the first ncols
// columns only (the rest zero).
static hipError_t qr_factor(int64_t njobs, int n_pad, double* S, double* Tws, bool keep_T, int32_t* colmap,
                            double* colnorm, hipStream_t stream, double* T64 = nullptr, bool lower = false,
                            KernelTimer* tq = nullptr, double* tq_flops = nullptr, int ncols = 0,
                            QrStop* stop = nullptr) {
  if (ncols <= 0 || ncols > n_pad) ncols = n_pad;
  if (stop) stop->rows = n_pad;
  if (n_pad <= 1024)
    return qr_factor_t<256, 4, 32>(njobs, n_pad, S, Tws, keep_T, colmap, colnorm, T64, lower, stream, tq, tq_flops,
                                   ncols, stop);
  return qr_factor_t<512, 8, 8>(njobs, n_pad, S, Tws, keep_T, nullptr, nullptr, nullptr, false, stream, nullptr,
                                nullptr, n_pad, nullptr);
}

static hipError_t order_and_unfold(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src,
                                   const int32_t* split, int32_t* perm, int32_t* iperm, double* S,
                                   hipStream_t stream) {
  int P = 1;
  while (P < n_pad) P <<= 1;
  hipLaunchKernelGGL(colnorm_order_kernel, dim3((unsigned)njobs), dim3(256), (size_t)P * 12, stream, n, D, n_pad, T,
                     src, split, perm, iperm);
  hipLaunchKernelGGL(unfold_cols_kernel, dim3((unsigned)ceil_div(n_pad, 64), (unsigned)ceil_div(n_pad, 32),
                                              (unsigned)njobs),
                     dim3(256), 0, stream, n, D, n_pad, T, src, split, (const int32_t*)iperm, S);
  return hipGetLastError();
}

// Three QRs: M P = Q1 R1, R1^T = Q2 R2, R2^T = Q3 R3 (P: the static norm
// order, refined panel by panel through colmap when n_pad <= 1024).  Each
// factorisation of the transposed triangle is one step of the unshifted QR
// iteration and moves the factor closer to diagonal, so the Jacobi on the
// rows of R3 needs fewer sweeps.  The rows of R_i are the columns of R_i^T,
// so each row copy is directly the column storage of the next QR.
// Since R1 = Q3 R3 Q2^T, M P = (Q1 Q3) R3 Q2^T: the right singular vectors
// y of R3 (the normalised rows of the Jacobi result) give those of M P as
// z = Q2 y, and those of M as v = P z; u = M v / s.  Q2 is kept (V in W1,
// the panel T factors in Tws2); Q1 and Q3 are not needed.  Buffers: S1 (QR1
// in place, then the rows of R3, returned in *rows), W1 (QR2 in place), W2
// (rows of R2, QR3 in place); Tws1 is scratch.
hipError_t run_qr3_precondition(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src,
                                const int32_t* split, int32_t* perm, int32_t* iperm, double* S1, double* Tws1, double* W1,
                                double* Tws2, double* W2, int32_t* colmap, double* colnorm, double** rows,
                                hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  if (n_pad > kQrMaxN) return hipErrorInvalidValue;
  if (n_pad > 1024) colmap = nullptr;   // re-ordering only with 32-column panels
  hipError_t e = order_and_unfold(njobs, n, D, n_pad, T, src, split, perm, iperm, S1, stream);
  if (e != hipSuccess) return e;
  e = qr_factor(njobs, n_pad, S1, Tws1, false, colmap, colnorm, stream);
  if (e != hipSuccess) return e;
  const dim3 rg(n_pad / 32, n_pad / 32, (unsigned)njobs);
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, S1, W1, (const int32_t*)colmap, n_pad, n_pad);
  // (n_pad > 1024: 8-column panels throughout, no block T scratch)
  e = qr_factor(njobs, n_pad, W1, Tws2, true, nullptr, nullptr, stream, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, W1, W2, (const int32_t*)nullptr, n_pad, n_pad);
  e = qr_factor(njobs, n_pad, W2, Tws1, false, nullptr, nullptr, stream, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, W2, S1, (const int32_t*)nullptr, n_pad, n_pad);
  *rows = S1;
  return hipGetLastError();
}

// Five QRs (n_pad <= 1024): M P = Q1 R1 and R_i^T = Q_{i+1} R_{i+1} for i =
// 1..4, so R1 = Q3 R3 Q2^T, R3 = Q5 R5 Q4^T and M P = Q1 Q3 Q5 R5 (Q2 Q4)^T:
// the right singular vectors y of R5 (the normalised Jacobi rows) give v =
// P Q2 Q4 y and u = M v / s; Q1, Q3 and Q5 are not needed.  Every further
// step of this unshifted QR iteration moves R towards diagonal form and
// saves Jacobi work (rotated block pairs in units of a full sweep on steady
// k = 32 unfoldings: about 5.3 after three QRs, 4.5 after four, 3.8 after
// five) at the cost of one more 64-column QR.
// Q2 stays in W1 with its panel T factors in Tws2, Q4 in S1 with its T
// factors in Tws4 (n_pad * 32 doubles per job each); the first, third and
// fifth QR use Tscr (kQrTscr doubles per job) for their T factors.  The rows of
// R5 end in W3; W2 is free afterwards.
hipError_t run_qr1(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src, const int32_t* split,
                   int32_t* perm, int32_t* iperm, double* S1, double* W1, double* Tscr, int32_t* colmap,
                   double* colnorm, hipStream_t stream, QrStop* stop) {
  if (njobs == 0) return hipSuccess;
  if (n_pad > 1024) return hipErrorInvalidValue;
  hipError_t e = order_and_unfold(njobs, n, D, n_pad, T, src, split, perm, iperm, S1, stream);
  if (e != hipSuccess) return e;
  e = qr_factor(njobs, n_pad, S1, Tscr, false, colmap, colnorm, stream, Tscr + (size_t)njobs * 2048, false, nullptr,
                nullptr, 0, stop);
  if (e != hipSuccess) return e;
  const dim3 rg(n_pad / 32, n_pad / 32, (unsigned)njobs);
  // rows from the stop on (the unfactored rest, within the budget) are written as zero
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, S1, W1, (const int32_t*)colmap,
                     stop ? stop->rows : n_pad, n_pad, stop ? (const int*)stop->rows_job : nullptr);
  return hipGetLastError();
}

hipError_t run_qr23(int64_t njobs, int n_pad, int ncols, double* W1, double* Tws2, double* W2, double* W3,
                    double* Tscr, hipStream_t stream, KernelTimer* tq, double* tq_flops, const int* rows_job) {
  if (njobs == 0) return hipSuccess;
  if (n_pad > 1024 || ncols <= 0 || ncols > n_pad || (ncols % 128 && ncols != n_pad)) return hipErrorInvalidValue;
  if (tq && !tq_flops) return hipErrorInvalidValue;
  double* T64 = Tscr + (size_t)njobs * 2048;
  const dim3 rg(n_pad / 32, n_pad / 32, (unsigned)njobs);
  if (rows_job) {
    // every job's rows of R1 from its own limit on (within the budget in
    // total) become zero; the batch factors the leading ncols columns, the
    // largest limit, where the zero columns of a job are exact no-ops
    hipLaunchKernelGGL(zero_rows_from_kernel, dim3((unsigned)(n_pad / 8), (unsigned)njobs), dim3(256), 0, stream,
                       n_pad, W1, rows_job);
  } else if (ncols < n_pad) {   // the rows of R1 from ncols on (within the budget in total) become zero
    const int64_t nz = (int64_t)(n_pad - ncols) * n_pad;
    hipLaunchKernelGGL(zero_tail_kernel, dim3((unsigned)ceil_div(nz, 256), (unsigned)njobs), dim3(256), 0, stream, nz,
                       W1 + (int64_t)ncols * n_pad, (int64_t)n_pad * n_pad);
  }
  hipError_t e = qr_factor(njobs, n_pad, W1, Tws2, true, nullptr, nullptr, stream, Tscr, true, tq, tq_flops, ncols);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, W1, W2, (const int32_t*)nullptr, ncols, ncols);
  e = qr_factor(njobs, n_pad, W2, Tscr, false, nullptr, nullptr, stream, T64, true, tq, tq_flops, ncols);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, W2, W3, (const int32_t*)nullptr, ncols, ncols);
  return hipGetLastError();
}

hipError_t run_qr5_precondition(int64_t njobs, int n, int D, int n_pad, const double* T, const int32_t* src,
                                const int32_t* split, int32_t* perm, int32_t* iperm, double* S1, double* W1, double* Tws2,
                                double* W2, double* Tws4, double* W3, double* Tscr, int32_t* colmap, double* colnorm,
                                hipStream_t stream, KernelTimer* tq, double* tq_flops, int nqr) {
  if (njobs == 0) return hipSuccess;
  if (n_pad > 1024 || (nqr != 3 && nqr != 5)) return hipErrorInvalidValue;
  hipError_t e = run_qr1(njobs, n, D, n_pad, T, src, split, perm, iperm, S1, W1, Tscr, colmap, colnorm, stream,
                         nullptr);
  if (e != hipSuccess) return e;
  e = run_qr23(njobs, n_pad, n_pad, W1, Tws2, W2, W3, Tscr, stream, tq, tq_flops, nullptr);
  if (e != hipSuccess || nqr == 3) return e;
  return run_qr45(njobs, n_pad, n_pad, S1, W2, Tws4, W3, Tscr, stream, tq, tq_flops);
}

hipError_t run_qr45(int64_t njobs, int n_pad, int ncols, double* S1, double* W2, double* Tws4, double* W3,
                    double* Tscr, hipStream_t stream, KernelTimer* tq, double* tq_flops) {
  if (njobs == 0) return hipSuccess;
  if (n_pad > 1024 || ncols <= 0 || ncols > n_pad || (ncols % 128 && ncols != n_pad)) return hipErrorInvalidValue;
  if (tq && !tq_flops) return hipErrorInvalidValue;
  double* T64 = Tscr + (size_t)njobs * 2048;
  const dim3 rg(n_pad / 32, n_pad / 32, (unsigned)njobs);
  hipError_t e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, W2, S1, (const int32_t*)nullptr, ncols, ncols);
  e = qr_factor(njobs, n_pad, S1, Tws4, true, nullptr, nullptr, stream, Tscr, true, tq, tq_flops, ncols);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, S1, W2, (const int32_t*)nullptr, ncols, ncols);
  e = qr_factor(njobs, n_pad, W2, Tscr, false, nullptr, nullptr, stream, T64, true, tq, tq_flops, ncols);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(r_rows_kernel, rg, dim3(256), 0, stream, n_pad, W2, W3, (const int32_t*)nullptr, ncols, ncols);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// X[:, a] = w_a Q x_a for the kept rows x_a = W[order[sel[a]]] / s of the
// Jacobi result, Q = prod_p (I - V_p T_p V_p^T) the orthogonal factor of a
// blocked Householder QR (V below the diagonal of S, stored column c in
// colmap[c]), applied from the last panel to the first.  One workgroup per
// (a, job).
// ---------------------------------------------------------------------------
template <int MAXQ, int PW>
__global__ __launch_bounds__(256) void apply_q1_kernel(int n, int n_pad, int kcap, const double* __restrict__ S1,
                                                       const double* __restrict__ Tws1, const double* __restrict__ W2,
                                                       const double* __restrict__ sigma,
                                                       const int32_t* __restrict__ order,
                                                       const int32_t* __restrict__ kept,
                                                       const int32_t* __restrict__ sel,
                                                       const double* __restrict__ weight, double* __restrict__ F) {
  const int a = blockIdx.x;
  const int64_t job = blockIdx.y;
  const int tid = threadIdx.x;
  double* Fj = F + (size_t)job * n * kcap;
  if (a >= kept[job]) {
    for (int r = tid; r < n; r += 256) Fj[(size_t)r * kcap + a] = 0.0;
    return;
  }
  const int i = sel[job * kcap + a];
  const double s = sigma[(size_t)job * n + i];
  const double* row = W2 + (size_t)job * n_pad * n_pad + (size_t)order[(size_t)job * n + i] * n_pad;
  const double* Sj = S1 + (size_t)job * n_pad * n_pad;
  const double* Tj = Tws1 + (size_t)job * n_pad * PW;
  __shared__ double x[4096];
  __shared__ double red[5][33];
  __shared__ double y2[PW];
  for (int r = tid; r < n_pad; r += 256) x[r] = row[r] / s;
  __syncthreads();
  for (int j = n_pad - PW; j >= 0; j -= PW) {
    double vv[MAXQ][PW];
    double part[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) part[c] = 0.0;
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int r = j + tid + 256 * q;
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        const int d = j + c;
        const double v = (r < n_pad && r > d) ? Sj[(size_t)d * n_pad + r] : (r == d ? 1.0 : 0.0);
        vv[q][c] = v;
        if (r < n_pad) part[c] += v * x[r];
      }
    }
    block_reduce_vec<256>(part, PW, red, tid);
    if (tid < PW) {
      double t = 0.0;
      for (int p = tid; p < PW; ++p) t += Tj[(j / PW) * PW * PW + tid * PW + p] * red[0][p];
      y2[tid] = t;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int r = j + tid + 256 * q;
      if (r < n_pad) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < PW; ++c) acc += vv[q][c] * y2[c];
        x[r] -= acc;
      }
    }
    __syncthreads();
  }
  const double w = weight[job * kcap + a];
  for (int r = tid; r < n; r += 256) Fj[(size_t)r * kcap + a] = w * x[r];
}

// The same product for n_pad <= 1024 with all kept vectors of a job handled
// together: one workgroup per (job, group of 16 vectors), X (n_pad x 16) in
// LDS, and for each panel p (last to first, 32 columns d = j .. j + 31)
//   Y = V_p^T X     (32 x 16, v_mfma_f64_16x16x4, waves split the rows),
//   Z = T_p Y       (T_p upper triangular, 32 x 32),
//   X <- X - V_p Z  (v_mfma_f64_16x16x4 over 16-row tiles).
// V_p (row d of S1, entries r > d; unit diagonal implied) is streamed from
// HBM twice per panel and workgroup instead of once per vector.
__global__ __launch_bounds__(256) void apply_q1_mfma_kernel(int n, int n_pad, int kcap, const double* __restrict__ S1,
                                                            const int32_t* __restrict__ colmap,
                                                            const double* __restrict__ Tws1,
                                                            const double* __restrict__ S1b,
                                                            const double* __restrict__ Tws1b,
                                                            const double* __restrict__ W2,
                                                            const double* __restrict__ sigma,
                                                            const int32_t* __restrict__ order,
                                                            const int32_t* __restrict__ kept,
                                                            const int32_t* __restrict__ sel,
                                                            const double* __restrict__ weight, double* __restrict__ F,
                                                            const int* __restrict__ nob) {
  extern __shared__ unsigned char smem[];
  double* X = reinterpret_cast<double*>(smem);   // [n_pad][16]
  double* Yp = X + (size_t)n_pad * 16;     // [4 waves][2 tiles][256]
  double* Ys = Yp + 4 * 2 * 256;           // [32][16]
  double* Zs = Ys + 32 * 16;               // [32][16], holds -Z
  __shared__ double sv[16], wv[16];
  __shared__ const double* rowp[16];
  const int64_t job = blockIdx.y;
  const int a0 = 16 * blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int nk = kept[job];
  if (tid < 16) {
    const int a = a0 + tid;
    if (a < nk) {
      const int i = sel[job * kcap + a];
      sv[tid] = sigma[(size_t)job * n + i];
      wv[tid] = weight[job * kcap + a];
      rowp[tid] = W2 + (size_t)job * n_pad * n_pad + (size_t)order[(size_t)job * n + i] * n_pad;
    } else {
      sv[tid] = 1.0;
      wv[tid] = 0.0;
      rowp[tid] = nullptr;
    }
  }
  __syncthreads();
  for (int e = tid; e < n_pad * 16; e += 256) {
    const int r = e >> 4, v = e & 15;
    X[e] = rowp[v] ? rowp[v][r] / sv[v] : 0.0;
  }
  __syncthreads();
  // the second factor (if any, and not masked off for this job) first
  for (int set = (S1b && !(nob && nob[job])) ? 0 : 1; set < 2; ++set) {
  const double* Sj = (set == 0 ? S1b : S1) + (size_t)job * n_pad * n_pad;
  const int32_t* cm = (set == 1 && colmap) ? colmap + job * n_pad : nullptr;   // V_d is stored in column cm[d]
  const double* Tj = (set == 0 ? Tws1b : Tws1) + (size_t)job * n_pad * 32;
  for (int j = n_pad - 32; j >= 0; j -= 32) {
    // ---- Y = V_p^T X: rows r = j .. n_pad - 1 in chunks of 16 ------------
    f64x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    for (int r0 = j + 16 * wave; r0 < n_pad; r0 += 64) {
      const int rb = r0 + 4 * lg;
      double av[2][4];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int d = j + 16 * t + lr;
        const double* src = Sj + (size_t)(cm ? cm[d] : d) * n_pad + rb;
        const double2 x01 = *reinterpret_cast<const double2*>(src);
        const double2 x23 = *reinterpret_cast<const double2*>(src + 2);
        av[t][0] = x01.x; av[t][1] = x01.y; av[t][2] = x23.x; av[t][3] = x23.y;
        if (r0 < j + 32) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = rb + q;
            av[t][q] = r > d ? av[t][q] : (r == d ? 1.0 : 0.0);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double b = X[(rb + q) * 16 + lr];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0][q], b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1][q], b, acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = acc_row_f64(lg, i) * 16 + lr;
      Yp[(wave * 2 + 0) * 256 + idx] = acc0[i];
      Yp[(wave * 2 + 1) * 256 + idx] = acc1[i];
    }
    __syncthreads();
    for (int e = tid; e < 512; e += 256) {   // Y[c][v], c = 16 t + row
      const int t = e >> 8, idx = e & 255;
      Ys[e] = ((Yp[(0 * 2 + t) * 256 + idx] + Yp[(1 * 2 + t) * 256 + idx]) + Yp[(2 * 2 + t) * 256 + idx]) +
              Yp[(3 * 2 + t) * 256 + idx];
    }
    __syncthreads();
    for (int e = tid; e < 512; e += 256) {   // -Z[c][v] = -sum_{c' >= c} T[c][c'] Y[c'][v]
      const int c = e >> 4, v = e & 15;
      const double* Trow = Tj + (size_t)(j / 32) * 1024 + c * 32;
      double z = 0.0;
      for (int c2 = c; c2 < 32; ++c2) z += Trow[c2] * Ys[c2 * 16 + v];
      Zs[e] = -z;
    }
    __syncthreads();
    // ---- X <- X - V_p Z over 16-row tiles r0 = j + 16 m -----------------
    double bz[8];
    int vc[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      bz[s] = Zs[(4 * s + lg) * 16 + lr];
      vc[s] = cm ? cm[j + 4 * s + lg] : j + 4 * s + lg;
    }
    for (int r0 = j + 16 * wave; r0 < n_pad; r0 += 64) {
      f64x4 cx;
#pragma unroll
      for (int i = 0; i < 4; ++i) cx[i] = X[(r0 + acc_row_f64(lg, i)) * 16 + lr];
      const int r = r0 + lr;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int d = j + 4 * s + lg;
        double v = Sj[(size_t)vc[s] * n_pad + r];
        if (r0 < j + 32) v = r > d ? v : (r == d ? 1.0 : 0.0);
        cx = __builtin_amdgcn_mfma_f64_16x16x4f64(v, bz[s], cx, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) X[(r0 + acc_row_f64(lg, i)) * 16 + lr] = cx[i];
    }
    __syncthreads();
  }
  }
  double* Fj = F + (size_t)job * n * kcap;
  for (int e = tid; e < n * 16; e += 256) {
    const int r = e >> 4, v = e & 15, a = a0 + v;
    if (a < kcap) Fj[(size_t)r * kcap + a] = (a < nk) ? wv[v] * X[e] : 0.0;
  }
}

// The same for up to 32 kept vectors and n_pad <= 1024, one workgroup of 8
// waves per job with X (n_pad x 32) in registers: wave w owns the 16-row
// tiles g = 8 t + w (t < n_pad / 128), lane (lr, lg) holding X[16 g + 4 i +
// lg][16 vt + lr] in xr[t][vt][i], which is both the B operand layout of Y =
// V^T X (k-step i of tile g) and the accumulator layout of X - V Z.  Each V
// tile is read by the wave that owns its rows only; Y is summed over the
// waves in a fixed order.
constexpr int kApplyTiles = 8;   // row tiles per wave (n_pad <= 1024)
__global__ __launch_bounds__(512) void apply_q_reg_kernel(int n, int n_pad, int kcap, const double* __restrict__ S1,
                                                          const int32_t* __restrict__ colmap,
                                                          const double* __restrict__ Tws1,
                                                          const double* __restrict__ S1b,
                                                          const double* __restrict__ Tws1b,
                                                          const double* __restrict__ W2,
                                                          const double* __restrict__ sigma,
                                                          const int32_t* __restrict__ order,
                                                          const int32_t* __restrict__ kept,
                                                          const int32_t* __restrict__ sel,
                                                          const double* __restrict__ weight, double* __restrict__ F,
                                                            const int* __restrict__ nob) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int nk = kept[job];
  __shared__ double Yp[8][4][256];   // per wave: tiles (ct, vt) of its partial Y
  __shared__ double Ys[32][33];      // Y = V^T X (32 reflectors x 32 vectors)
  __shared__ double Zs[32][33];      // -T Y
  __shared__ double sv[32], wv[32];
  __shared__ const double* rowp[32];
  if (tid < 32) {
    const int a = tid;
    if (a < nk && a < kcap) {
      const int i = sel[job * kcap + a];
      sv[a] = sigma[(size_t)job * n + i];
      wv[a] = weight[job * kcap + a];
      rowp[a] = W2 + (size_t)job * n_pad * n_pad + (size_t)order[(size_t)job * n + i] * n_pad;
    } else {
      sv[a] = 1.0;
      wv[a] = 0.0;
      rowp[a] = nullptr;
    }
  }
  __syncthreads();
  const int ntile = n_pad / 16;   // row tiles of the job
  f64x4 xr[kApplyTiles][2];
#pragma unroll
  for (int t = 0; t < kApplyTiles; ++t)
#pragma unroll
    for (int vt = 0; vt < 2; ++vt) {
      const int g = 8 * t + wave, v = 16 * vt + lr;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * g + 4 * i + lg;
        xr[t][vt][i] = (g < ntile && rowp[v]) ? rowp[v][r] / sv[v] : 0.0;
      }
    }
  // the second factor (if any, and not masked off for this job) first
  for (int set = (S1b && !(nob && nob[job])) ? 0 : 1; set < 2; ++set) {
    const double* Sj = (set == 0 ? S1b : S1) + (size_t)job * n_pad * n_pad;
    const int32_t* cm = (set == 1 && colmap) ? colmap + job * n_pad : nullptr;   // V_d is stored in column cm[d]
    const double* Tj = (set == 0 ? Tws1b : Tws1) + (size_t)job * n_pad * 32;
    for (int j = n_pad - 32; j >= 0; j -= 32) {
      // ---- partial Y over this wave's tiles at or below row j -------------
      f64x4 yp[2][2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int vt = 0; vt < 2; ++vt) yp[ct][vt] = f64x4{0, 0, 0, 0};
      const int d0 = j + lr, d1 = j + 16 + lr;   // V columns of the A fragments (ct = 0, 1)
      const double* c0 = Sj + (size_t)(cm ? cm[d0] : d0) * n_pad;
      const double* c1 = Sj + (size_t)(cm ? cm[d1] : d1) * n_pad;
#pragma unroll
      for (int t = 0; t < kApplyTiles; ++t) {
        const int g = 8 * t + wave;
        if (g >= ntile || 16 * g + 15 < j) continue;   // (uniform per wave)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = 16 * g + 4 * i + lg;
          double a0 = c0[r], a1 = c1[r];
          a0 = r > d0 ? a0 : (r == d0 ? 1.0 : 0.0);
          a1 = r > d1 ? a1 : (r == d1 ? 1.0 : 0.0);
#pragma unroll
          for (int vt = 0; vt < 2; ++vt) {
            yp[0][vt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, xr[t][vt][i], yp[0][vt], 0, 0, 0);
            yp[1][vt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, xr[t][vt][i], yp[1][vt], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int vt = 0; vt < 2; ++vt)
#pragma unroll
          for (int x = 0; x < 4; ++x) Yp[wave][2 * ct + vt][acc_row_f64(lg, x) * 16 + lr] = yp[ct][vt][x];
      __syncthreads();
      for (int e = tid; e < 1024; e += 512) {   // Y[c][v], summed over the waves in order
        const int c = e >> 5, v = e & 31, tile = 2 * (c >> 4) + (v >> 4), idx = (c & 15) * 16 + (v & 15);
        double y = Yp[0][tile][idx];
#pragma unroll
        for (int w = 1; w < 8; ++w) y += Yp[w][tile][idx];
        Ys[c][v] = y;
      }
      __syncthreads();
      for (int e = tid; e < 1024; e += 512) {   // -Z[c][v] = -sum_{c' >= c} T[c][c'] Y[c'][v]
        const int c = e >> 5, v = e & 31;
        const double* Trow = Tj + (size_t)(j / 32) * 1024 + c * 32;
        double z = 0.0;
        for (int c2 = c; c2 < 32; ++c2) z += Trow[c2] * Ys[c2][v];
        Zs[c][v] = -z;
      }
      __syncthreads();
      // ---- X <- X - V Z on this wave's tiles -------------------------------
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const double bz0 = Zs[4 * ks + lg][lr], bz1 = Zs[4 * ks + lg][16 + lr];
        const int d = j + 4 * ks + lg;
        const double* vc = Sj + (size_t)(cm ? cm[d] : d) * n_pad;
#pragma unroll
        for (int t = 0; t < kApplyTiles; ++t) {
          const int g = 8 * t + wave;
          if (g >= ntile || 16 * g + 15 < j) continue;   // (uniform per wave)
          const int r = 16 * g + lr;
          double v = vc[r];
          v = r > d ? v : (r == d ? 1.0 : 0.0);
          xr[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(v, bz0, xr[t][0], 0, 0, 0);
          xr[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(v, bz1, xr[t][1], 0, 0, 0);
        }
      }
    }
  }
  double* Fj = F + (size_t)job * n * kcap;
#pragma unroll
  for (int t = 0; t < kApplyTiles; ++t)
#pragma unroll
    for (int vt = 0; vt < 2; ++vt) {
      const int g = 8 * t + wave, a = 16 * vt + lr;
      if (g >= ntile || a >= kcap) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * g + 4 * i + lg;
        if (r < n) Fj[(size_t)r * kcap + a] = (a < nk) ? wv[a] * xr[t][vt][i] : 0.0;
      }
    }
}

size_t apply_q1_mfma_lds(int n_pad) { return sizeof(double) * ((size_t)n_pad * 16 + 4 * 2 * 256 + 2 * 32 * 16); }

hipError_t launch_apply_q1(int64_t njobs, int n, int n_pad, int kcap, const double* S1, const int32_t* colmap,
                           const double* Tws1, const double* S1b, const double* Tws1b, const double* W2,
                           const double* sigma, const int32_t* order, const int32_t* kept, const int32_t* sel,
                           const double* weight, double* F, hipStream_t stream, const int* nob) {
  if (njobs == 0) return hipSuccess;
  if (S1b && n_pad > 1024) return hipErrorInvalidValue;   // two factors only with 32-column panels
  if (n_pad <= 1024 && kcap > 16 && kcap <= 32) {
    hipLaunchKernelGGL(apply_q_reg_kernel, dim3((unsigned)njobs), dim3(512), 0, stream, n, n_pad, kcap, S1, colmap,
                       Tws1, S1b, Tws1b, W2, sigma, order, kept, sel, weight, F, nob);
  } else if (n_pad <= 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&apply_q1_mfma_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)apply_q1_mfma_lds(n_pad));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(apply_q1_mfma_kernel, dim3((kcap + 15) / 16, (unsigned)njobs), dim3(256),
                       apply_q1_mfma_lds(n_pad), stream, n, n_pad, kcap, S1, colmap, Tws1, S1b, Tws1b, W2, sigma,
                       order, kept, sel, weight, F, nob);
  } else
    hipLaunchKernelGGL((apply_q1_kernel<16, 8>), dim3(kcap, (unsigned)njobs), dim3(256), 0, stream, n, n_pad, kcap, S1,
                       Tws1, W2, sigma, order, kept, sel, weight, F);
  return hipGetLastError();
}

__global__ void iota_kernel(int64_t njobs, int n_pad, int32_t* perm) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < njobs * n_pad) perm[i] = (int32_t)(i % n_pad);
}

hipError_t launch_iota(int64_t njobs, int n_pad, int32_t* perm, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(ceil_div(njobs * n_pad, 256)), dim3(256), 0, stream, njobs, n_pad, perm);
  return hipGetLastError();
}

}  // namespace mctrg
