// Decomposition step: FP64 SVD of a batch of square unfoldings by one-sided
// block Jacobi (Hestenes), the "full singular value decomposition" of each
// tensor that precedes the stochastic truncation (paper Section III, first
// paragraph after Eq. infiniteSum; Section II Eq. exactSVD).
//
// Each job holds W (n_pad x n_pad, row-major).  The rows of W are the
// columns of A = M^T.  Rotating rows so that they become mutually orthogonal
// gives W_final = Q^T W with rows sigma_i * v_i, where v_i are the right
// singular vectors of M and sigma_i its singular values; left vectors follow
// as u_i = M v_i / sigma_i (see the factor kernels).
//
// Rows are grouped into blocks of 16 (32 when n_pad is a multiple of 64, see
// jacobi_round64_kernel); a sweep visits every pair of blocks once, in nb-1
// rounds of nb/2 disjoint pairs (circle ordering).  One workgroup handles one
// (job, pair); for 16-row blocks:
//   1. Gram G = W_pair W_pair^T (32 x 32) with v_mfma_f64_16x16x4, each wave
//      streaming a quarter of the row length from HBM;
//   2. if some |g_ij| > tol * sqrt(g_ii g_jj): two cyclic Jacobi sweeps on G
//      in LDS (two-sided, with the diagonal updated as g_pp - t g_pq for
//      relative accuracy) accumulating Q (32 x 32);
//   3. W_pair <- Q^T W_pair with v_mfma_f64_16x16x4 (Q^T fragments held in
//      registers, W streamed chunk by chunk and written back in place).
// A job has converged when a whole sweep applied no rotation; the host
// checks a device counter once per sweep.
#include "mctrg_internal.h"

namespace mctrg {

// Position -> block index in round r of the circle ordering on nb blocks.
__device__ __forceinline__ int circle_block(int pos, int r, int nb) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (nb - 1);
}

__global__ __launch_bounds__(256) void jacobi_round_kernel(double* __restrict__ W, int n_pad, int nb_all,
                                                           const int* __restrict__ nb_job, int round,
                                                           const int* __restrict__ active,
                                                           int* __restrict__ rotated, int* __restrict__ pairs,
                                                           double tol, double tabs) {
  const int job = blockIdx.y;
  if (!active[job]) return;
  // rows beyond the job's active blocks sit below the noise floor and stay
  // as they are (see deflate_plan_kernel)
  const int nb = nb_job ? nb_job[job] : nb_all;
  const int pair = (int)((blockIdx.x + blockIdx.y) % gridDim.x);   // XCD balance (see jacobi_round64_kernel)
  if (round >= nb - 1 || pair >= nb / 2) return;
  const int I = circle_block(pair, round, nb);
  const int J = circle_block(nb - 1 - pair, round, nb);
  double* Wj = W + (size_t)job * n_pad * n_pad;
  double* rowI = Wj + (size_t)(16 * I) * n_pad;
  double* rowJ = Wj + (size_t)(16 * J) * n_pad;

  // per-wave partial Gram tiles, later reused for Q (32 x 33)
  __shared__ double part_q[4 * 3 * 256];
  __shared__ double G[32][33];
  double(*part)[3][256] = reinterpret_cast<double(*)[3][256]>(part_q);
  double(*Q)[33] = reinterpret_cast<double(*)[33]>(part_q);
  __shared__ double rc[16], rs[16], rdp[16], rdq[16];
  __shared__ int rp[16], rq[16];
  __shared__ int flag_any;
  __shared__ double redbuf[8];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;

  // ---- 1. Gram of the 32 rows -------------------------------------------
  f64x4 aII = {0, 0, 0, 0}, aIJ = {0, 0, 0, 0}, aJJ = {0, 0, 0, 0};
  for (int k0 = 16 * wave; k0 < n_pad; k0 += 64) {
    const double* pa = rowI + (size_t)lr * n_pad + k0 + 4 * lg;
    const double* pb = rowJ + (size_t)lr * n_pad + k0 + 4 * lg;
    double2 a01 = *reinterpret_cast<const double2*>(pa);
    double2 a23 = *reinterpret_cast<const double2*>(pa + 2);
    double2 b01 = *reinterpret_cast<const double2*>(pb);
    double2 b23 = *reinterpret_cast<const double2*>(pb + 2);
    double av[4] = {a01.x, a01.y, a23.x, a23.y};
    double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      aII = __builtin_amdgcn_mfma_f64_16x16x4f64(av[jj], av[jj], aII, 0, 0, 0);
      aIJ = __builtin_amdgcn_mfma_f64_16x16x4f64(av[jj], bv[jj], aIJ, 0, 0, 0);
      aJJ = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[jj], bv[jj], aJJ, 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int idx = acc_row_f64(lg, i) * 16 + lr;
    part[wave][0][idx] = aII[i];
    part[wave][1][idx] = aIJ[i];
    part[wave][2][idx] = aJJ[i];
  }
  __syncthreads();
  for (int e = tid; e < 1024; e += 256) {
    int i = e >> 5, j = e & 31;
    int ti = i >> 4, tj = j >> 4, ii = i & 15, jj = j & 15;
    int t, idx;
    if (ti == 0 && tj == 0) { t = 0; idx = ii * 16 + jj; }
    else if (ti == 0) { t = 1; idx = ii * 16 + jj; }
    else if (tj == 0) { t = 1; idx = jj * 16 + ii; }
    else { t = 2; idx = ii * 16 + jj; }
    G[i][j] = ((part[0][t][idx] + part[1][t][idx]) + part[2][t][idx]) + part[3][t][idx];
  }
  __syncthreads();
  for (int e = tid; e < 1024; e += 256) Q[e >> 5][e & 31] = ((e >> 5) == (e & 31)) ? 1.0 : 0.0;

  // ---- convergence test of this pair ------------------------------------
  double off = 0.0;   // (tabs: as in jacobi_round64_kernel)
  for (int e = tid; e < 1024; e += 256) {
    int i = e >> 5, j = e & 31;
    if (i < j) {
      const double gi = G[i][i], gj = G[j][j], d = gi * gj, g = fabs(G[i][j]);
      if (d > 0.0 && g > tabs * fmax(gi, gj)) off = fmax(off, g / sqrt(d));
    }
  }
  for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
  if (lane == 0) redbuf[wave] = off;
  __syncthreads();
  off = fmax(fmax(redbuf[0], redbuf[1]), fmax(redbuf[2], redbuf[3]));
  if (!(off > tol)) return;            // pair already orthogonal (uniform)
  if (tid == 0) { atomicOr(&rotated[job], 1); atomicAdd(pairs, 1); }

  // ---- 2. cyclic Jacobi on G, accumulating Q ------------------------------
  // Two inner sweeps are enough: the outer iteration recomputes the pair's
  // Gram from W, and capping the latency-bound inner solve does not add
  // outer sweeps (checked on TRG unfoldings).
  const double tol_in = 0x1.0p-53;
  for (int sweep = 0; sweep < 2; ++sweep) {
    if (tid == 0) flag_any = 0;
    __syncthreads();   // also orders the Q initialisation before its first use
    for (int r = 0; r < 31; ++r) {
      if (tid < 16) {
        int p = tid == 0 ? 0 : 1 + (tid - 1 + r) % 31;
        int q = 1 + (31 - tid - 1 + r) % 31;
        if (p > q) { int tmp = p; p = q; q = tmp; }
        double gpp = G[p][p], gqq = G[q][q], gpq = G[p][q];
        double c = 1.0, s = 0.0, dp = gpp, dq = gqq;
        // |.| guards the tiny diagonal entries that rounding can push below 0
        if (gpq != 0.0 && fabs(gpq) > tol_in * sqrt(fabs(gpp * gqq))) {
          double theta = (gqq - gpp) / (2.0 * gpq);
          double t = (fabs(theta) > 1e150) ? 0.5 / theta
                                           : copysign(1.0, theta) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          dp = gpp - t * gpq;
          dq = gqq + t * gpq;
          flag_any = 1;
        }
        rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s; rdp[tid] = dp; rdq[tid] = dq;
      }
      __syncthreads();
      {  // column rotations of G and Q: pair i = tid/16, rows tid%16 and +16
        int i = tid >> 4, row0 = tid & 15;
        int p = rp[i], q = rq[i];
        double c = rc[i], s = rs[i];
        if (s != 0.0) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            int row = row0 + 16 * h;
            double gp = G[row][p], gq = G[row][q];
            G[row][p] = c * gp - s * gq;
            G[row][q] = s * gp + c * gq;
            double qp = Q[row][p], qq = Q[row][q];
            Q[row][p] = c * qp - s * qq;
            Q[row][q] = s * qp + c * qq;
          }
        }
      }
      __syncthreads();
      {  // row rotations of G
        int i = tid >> 4, col0 = tid & 15;
        int p = rp[i], q = rq[i];
        double c = rc[i], s = rs[i];
        if (s != 0.0) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            int col = col0 + 16 * h;
            double gp = G[p][col], gq = G[q][col];
            G[p][col] = c * gp - s * gq;
            G[q][col] = s * gp + c * gq;
          }
        }
      }
      __syncthreads();
      if (tid < 16 && rs[tid] != 0.0) {
        int p = rp[tid], q = rq[tid];
        G[p][p] = rdp[tid];
        G[q][q] = rdq[tid];
        G[p][q] = 0.0;
        G[q][p] = 0.0;
      }
      __syncthreads();
    }
    const int any = flag_any;
    __syncthreads();   // every thread has read the flag before it is reset
    if (!any) break;
  }

  // ---- 3. W_pair <- Q^T W_pair ------------------------------------------
  // A fragment (output rows i = 16t + l%16, K index j = 4s + l/16): Q[j][i].
  double qa[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int s = 0; s < 8; ++s) qa[t][s] = Q[4 * s + lg][16 * t + lr];

  for (int k0 = 16 * wave; k0 < n_pad; k0 += 64) {
    double bvals[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int j = 4 * s + lg;
      const double* src = (j < 16 ? rowI + (size_t)j * n_pad : rowJ + (size_t)(j - 16) * n_pad);
      bvals[s] = src[k0 + lr];
    }
    f64x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[0][s], bvals[s], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[1][s], bvals[s], c1, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = acc_row_f64(lg, i);              // new row within the tile
      rowI[(size_t)r * n_pad + k0 + lr] = c0[i];
      rowJ[(size_t)r * n_pad + k0 + lr] = c1[i];
    }
  }
}

// Circle ordering on 64 indices: slot t of every round pairs the indices at
// positions t and 63 - t; in round r position 0 holds index 0 and position
// k >= 1 holds index 1 + (k - 1 + r) mod 63.  Between two rounds the index
// at position k moves to circle_next64(k).
__device__ __forceinline__ int circle_next64(int k) { return k == 0 ? 0 : (k == 1 ? 63 : k - 1); }

// Packed strictly upper triangle of a 64 x 64 symmetric matrix: entry (i, j),
// i < j, row by row, kGpk entries.
constexpr int kGpk = 64 * 63 / 2;
__device__ __forceinline__ int gpk_index(int i, int j) { return 63 * i - ((i * (i + 1)) >> 1) + j - 1; }

// Position of (Q^T)[row][col] (64 x 64) in A-fragment order for
// v_mfma_f64_16x16x4: fragment (row / 16, col / 4), lane (row % 16) +
// 16 (col % 4).
__device__ __forceinline__ int qt_frag_index(int row, int col) {
  return (((row >> 4) << 4) + (col >> 2)) * 64 + ((col & 3) << 4) + (row & 15);
}

// Tangent of the Jacobi rotation annihilating g_pq of (g_pp, g_pq; g_pq,
// g_qq): t = sign(theta) / (|theta| + sqrt(1 + theta^2)), theta =
// (g_qq - g_pp) / (2 g_pq), the smaller root (|t| <= 1).  Hardware
// reciprocal / reciprocal square root with one Newton step each: t need not
// be exact (the rotation stays orthogonal whatever t is; the cosine below is
// what has to be accurate).
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return r * fma(-x, r, 2.0);
}
__device__ __forceinline__ double jacobi_tangent(double gpp, double gqq, double gpq) {
  const double theta = (gqq - gpp) * rcp_nr(2.0 * gpq);
  if (fabs(theta) > 1e150) return 0.5 / theta;
  const double h = fma(theta, theta, 1.0);
  double y = __builtin_amdgcn_rsq(h);
  y = y * fma(-0.5 * h, y * y, 1.5);
  return copysign(rcp_nr(fabs(theta) + h * y), theta);
}
// c = 1 / sqrt(1 + t^2) to full precision (two Newton steps on the hardware
// reciprocal square root), so that c^2 + s^2 = 1 with s = t c up to rounding.
__device__ __forceinline__ double unit_cosine(double t) {
  const double h = fma(t, t, 1.0);
  double y = __builtin_amdgcn_rsq(h);
  y = y * fma(-0.5 * h, y * y, 1.5);
  y = y * fma(-0.5 * h, y * y, 1.5);
  return y;
}

// ---------------------------------------------------------------------------
// The same rotation step with 32-row blocks (pairs of 64 rows), used when
// n_pad is a multiple of 64.  A sweep then takes nb - 1 = n_pad/32 - 1
// rounds instead of n_pad/16 - 1, which halves the HBM traffic per sweep
// (every round streams each active row through the Gram and update passes).
//   1. Gram G (64 x 64): the ten distinct 16 x 16 tiles of the four 16-row
//      sub-blocks, each wave over a quarter of the row length, partial tiles
//      summed into wave 0's registers through LDS in a fixed order;
//   2. one cyclic Jacobi sweep on G (63 rounds of 32 disjoint rotations, two
//      barriers per round: after the rotations are formed and after the
//      rotated entries are stored, see below);
//   3. W_pair <- Q^T W_pair with v_mfma_f64_16x16x4 (Q^T fragments read
//      from LDS).
// One inner sweep is enough: the outer iteration recomputes the Gram from
// the rows, and a second inner sweep did not reduce the number of outer
// sweeps on TRG unfoldings.  The 64 rotated rows are written in decreasing
// norm order, the larger half to the lower-numbered block (a few percent
// fewer outer sweeps on TRG unfoldings).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 4) void jacobi_round64_kernel(double* __restrict__ W, int n_pad, int ncol, int nb_all,
                                                                const int* __restrict__ nb_job, int round,
                                                                const int* __restrict__ active,
                                                                int* __restrict__ rotated, int* __restrict__ pairs,
                                                                double tol, int* __restrict__ lastmod,
                                                                int* __restrict__ lastchk, int stamp, double tabs) {
  const int job = blockIdx.y;
  if (!active[job]) return;
  const int nb = nb_job ? nb_job[job] : nb_all;   // 32-row blocks
  // Workgroups reach the XCDs round-robin by linear index, so with pair =
  // blockIdx.x each XCD would always get the same pair slots; how often a
  // pair still rotates depends strongly on its slot (rows are kept sorted by
  // norm), which would load some XCDs with most of the rotations.  Rotating
  // the slot by the decomposition index spreads every slot over all XCDs.
  const int pair = (int)((blockIdx.x + blockIdx.y) % gridDim.x);
  if (round >= nb - 1 || pair >= nb / 2) return;
  // the lower-numbered block of the pair takes the larger rotated rows
  const int I0 = circle_block(pair, round, nb), J0 = circle_block(nb - 1 - pair, round, nb);
  const int I = min(I0, J0), J = max(I0, J0);
  // a pair found orthogonal after the last change of both its blocks still
  // is: skip it without reading the rows (uniform)
  int* const chk = lastmod ? lastchk + ((size_t)job * kJacobiMaxBlocks + I) * kJacobiMaxBlocks + J : nullptr;
  if (lastmod) {
    const int tI = lastmod[(size_t)job * kJacobiMaxBlocks + I], tJ = lastmod[(size_t)job * kJacobiMaxBlocks + J];
    if (*chk > max(tI, tJ)) return;
  }
  double* Wj = W + (size_t)job * n_pad * n_pad;
  double* rowI = Wj + (size_t)(32 * I) * n_pad;
  double* rowJ = Wj + (size_t)(32 * J) * n_pad;

  // U: the staged partial Gram tiles, then the two position-space buffers of
  // the strictly upper triangle of G (packed, kGpk entries each), then Q^T in
  // A-fragment order.
  __shared__ double U[4096];
  double* const QTf = U;                                              // qt_frag_index
  double(*stage)[5][256] = reinterpret_cast<double(*)[5][256]>(U);   // [wave-1][tile][16x16]
  __shared__ double2 rcs[32];      // (c, s) of the round's rotations, by slot
  __shared__ double dg[2][64];     // diagonal of G by position, by round parity
  __shared__ int rank_s[64];       // output position of each index (decreasing new row norm)
  __shared__ double xch[4][2][64];      // rows of Q^T handed to the neighbouring wave
  __shared__ double redbuf[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;

  // ---- 1. Gram ------------------------------------------------------------
  // sub-block sb: rows 16 sb .. 16 sb + 15 of the pair
  const double* sub[4] = {rowI, rowI + (size_t)16 * n_pad, rowJ, rowJ + (size_t)16 * n_pad};
  f64x4 acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = f64x4{0, 0, 0, 0};
  // Each wave takes 16-column chunks k0 = 16 wave + 64 i in two halves of 8
  // columns: lane (lr, lg) holds columns k0 + 8 h + 2 lg + {0, 1} of row lr
  // of every sub-block (one 16-byte load each, 64 contiguous bytes per row
  // and half), which are the K indices of two k-steps.  The next half is
  // loaded while the current one is multiplied; 48 VGPRs of operands and
  // the 80 of the ten accumulator tiles keep four waves per SIMD.
  double2 hc[4], hn[4];
  const int go = lr * n_pad + 2 * lg;   // the lane's offset from a sub-block's uniform base
  auto load_half = [&](int c, double2 (&v)[4]) {
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) v[sb] = *reinterpret_cast<const double2*>(sub[sb] + (go + c));
  };
  auto mfma_half = [&](const double2 (&v)[4]) {
    int t = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = x; y < 4; ++y) {
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[x].x, v[y].x, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[x].y, v[y].y, acc[t], 0, 0, 0);
        ++t;
      }
  };
  int k0 = 16 * wave;
  if (k0 < ncol) load_half(k0, hc);
  for (; k0 < ncol; k0 += 64) {
    load_half(k0 + 8, hn);
    mfma_half(hc);
    if (k0 + 64 < ncol) load_half(k0 + 64, hc);
    mfma_half(hn);
  }
  // partial tiles: waves 1..3 stage five tiles at a time, wave 0 adds them
  // to its own (same order for every entry), then stores G by position
  // (= index before the first round): the diagonal in dg, the strictly upper
  // triangle packed
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (wave > 0) {
#pragma unroll
      for (int t = 5 * half; t < 5 * half + 5; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) stage[wave - 1][t - 5 * half][acc_row_f64(lg, i) * 16 + lr] = acc[t][i];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int t = 5 * half; t < 5 * half + 5; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = acc_row_f64(lg, i) * 16 + lr;
          acc[t][i] = ((acc[t][i] + stage[0][t - 5 * half][idx]) + stage[1][t - 5 * half][idx]) +
                      stage[2][t - 5 * half][idx];
        }
    }
    __syncthreads();
  }
  if (wave == 0) {
    int t = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * a + acc_row_f64(lg, i), col = 16 * b + lr;
          if (row < col) U[gpk_index(row, col)] = acc[t][i];
          else if (row == col) dg[0][row] = acc[t][i];
        }
        ++t;
      }
  }
  __syncthreads();

  // ---- convergence test of this pair ------------------------------------
  // An entry needs a rotation when its cosine exceeds tol and (tabs > 0, a
  // job still rotating after many sweeps) the entry itself exceeds tabs
  // times the larger squared row norm: below that, rounding of the larger
  // row keeps the smaller one from becoming more orthogonal, and leaving
  // the entry moves the singular values by less than the approximation
  // budget's share (see run_jacobi).
  double off = 0.0;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    if (i < j) {
      const double gi = dg[0][i], gj = dg[0][j], d = gi * gj, g = fabs(U[gpk_index(i, j)]);
      if (d > 0.0 && g > tabs * fmax(gi, gj)) off = fmax(off, g / sqrt(d));
    }
  }
  for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
  if (lane == 0) redbuf[wave] = off;
  __syncthreads();
  off = fmax(fmax(redbuf[0], redbuf[1]), fmax(redbuf[2], redbuf[3]));
  if (!(off > tol)) {                  // pair already orthogonal (uniform)
    if (chk && tid == 0) *chk = stamp;
    return;
  }
  if (tid == 0) {
    atomicOr(&rotated[job], 1);
    atomicAdd(pairs, 1);
    if (lastmod) {
      lastmod[(size_t)job * kJacobiMaxBlocks + I] = stamp;
      lastmod[(size_t)job * kJacobiMaxBlocks + J] = stamp;
    }
  }

  // ---- 2. one cyclic Jacobi sweep on G, accumulating Q --------------------
  // The sweep works in the positions of the circle ordering: slot t rotates
  // positions t and 63 - t in every round, and between rounds the index at
  // position k + 1 moves to position k (position 1 to 63; position 0 stays),
  // so after 63 rounds every index is back at its own position.  G and its
  // diagonal are kept by position: round r reads the off-diagonal upper
  // triangle from one buffer and writes the rotated entries, already moved
  // to their next positions, into the other, so each thread reads and
  // writes the same LDS addresses in every round (no index tables).
  // Round r: (1) lanes 0..31 form the rotations of the 32 slots from the
  // diagonal and the slot's off-diagonal entry; (2) every 2 x 2 block
  // (positions t_i, 63 - t_i; t_j, 63 - t_j; t_i <= t_j) of G becomes
  // J_i^T A J_j, one owner per block, the off-diagonal entry of a rotated
  // slot set to 0, and the columns of Q are rotated.  A rotation formed with
  // the two positions in either order gives the same two rotated rows.
  //
  // Q lives in registers, by position: wave w holds the Q^T rows at
  // positions 8w .. 8w + 7 (qr[0..7]) and 56 - 8w .. 63 - 8w (qr[8..15]),
  // lane = row of Q, so its slots 8w + a pair qr[a] with qr[15 - a]; each
  // shift moves one row in from each neighbouring wave.  The rows handed
  // over in round r - 1 are read before the first barrier of round r and
  // the new ones written after it, so one exchange buffer serves all rounds
  // (with the G buffers below 40 KB of LDS: four workgroups per CU).
  //
  // The block grid is enumerated as 16 folded rows of 33 (row m and row
  // 31 - m); thread tid owns blocks tid, tid + 256 and (tid < 16) tid + 512.
  // Off-diagonal blocks (t_i < t_j, 496 of them): thread tid owns blocks
  // tid and tid + 256 (tid < 240).  A slot's own block only has its
  // off-diagonal entry to update (0 after a rotation; its diagonal entries
  // are in dg), which the lane that forms the slot's rotation writes.
  int rd[2][4], wr[2][4], bi[2], bj[2];   // per block: read / write offsets, slots
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int rem = min(tid + 256 * u, 495), ti = 0;
    while (rem >= 31 - ti) { rem -= 31 - ti; ++ti; }
    const int tj = ti + 1 + rem;
    bi[u] = ti; bj[u] = tj;
    const int pos[4][2] = {{ti, tj}, {ti, 63 - tj}, {63 - ti, tj}, {63 - ti, 63 - tj}};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = pos[v][0], b = pos[v][1];
      const int na = circle_next64(a), nb2 = circle_next64(b);
      rd[u][v] = gpk_index(min(a, b), max(a, b));
      wr[u][v] = gpk_index(min(na, nb2), max(na, nb2));
    }
  }
  const bool two = tid < 240;
  // lanes 0..31: the slot's own entry (positions tid, 63 - tid), read and
  // written after the move
  const int own_rd = gpk_index(tid & 31, 63 - (tid & 31));
  const int own_nx = circle_next64(tid & 31), own_ny = circle_next64(63 - (tid & 31));
  const int own_wr = gpk_index(min(own_nx, own_ny), max(own_nx, own_ny));
  const int ws = __builtin_amdgcn_readfirstlane(wave);
  double qr[16];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    qr[a] = (8 * ws + a == lane) ? 1.0 : 0.0;
    qr[8 + a] = (56 - 8 * ws + a == lane) ? 1.0 : 0.0;
  }
  for (int r = 0; r < 63; ++r) {
    const double* Gc = U + (r & 1) * kGpk;
    double* Gn = U + ((r + 1) & 1) * kGpk;
    // Q: finish the shift of the previous round (its rows were handed over
    // before that round's second barrier)
    if (r > 0) {
      double nq[16];
#pragma unroll
      for (int a = 0; a < 7; ++a) nq[a] = qr[a + 1];
      nq[7] = ws < 3 ? xch[ws + 1][0][lane] : qr[8];          // position 8w + 8
#pragma unroll
      for (int b = 0; b < 7; ++b) nq[8 + b] = qr[9 + b];
      nq[15] = ws > 0 ? xch[ws - 1][1][lane] : qr[1];         // position 64 - 8w (64 -> 1)
      if (ws == 0) nq[0] = qr[0];                             // position 0 stays
#pragma unroll
      for (int a = 0; a < 16; ++a) qr[a] = nq[a];
    }
    if (tid < 32) {
      const int x = tid, y = 63 - tid;
      const double gxx = dg[r & 1][x], gyy = dg[r & 1][y], gxy = Gc[own_rd];
      double c = 1.0, t = 0.0, dx = gxx, dy = gyy, gn = gxy;
      // |.| guards the tiny diagonal entries that rounding can push below 0
      if (gxy != 0.0 && gxy * gxy > 0x1.0p-106 * fabs(gxx * gyy)) {
        t = jacobi_tangent(gxx, gyy, gxy);
        c = unit_cosine(t);
        dx = fma(-t, gxy, gxx);
        dy = fma(t, gxy, gyy);
        gn = 0.0;
      }
      rcs[tid] = make_double2(c, t);   // cosine and tangent
      dg[(r + 1) & 1][own_nx] = dx;
      dg[(r + 1) & 1][own_ny] = dy;
      Gn[own_wr] = gn;
    }
    __syncthreads();
    // Q: rotate this round's slots (every wave has read the previous
    // round's hand-over before the barrier above, so it may be overwritten)
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double2 ct = rcs[8 * ws + a];
      const double x = qr[a], y = qr[15 - a];
      qr[a] = ct.x * fma(-ct.y, y, x);
      qr[15 - a] = ct.x * fma(ct.y, x, y);
    }
    xch[ws][0][lane] = qr[0];   // position 8w, wanted by wave w - 1
    xch[ws][1][lane] = qr[8];   // position 56 - 8w, wanted by wave w + 1
    // G blocks: read from this round's buffer, store into the other.  With
    // J = c [[1, t], [-t, 1]] acting on the columns (x, y) -> (c (x - t y),
    // c (t x + y)), J_i^T A J_j = c_i c_j (the tangent products below).
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      const double2 ci = rcs[bi[u]], cj = rcs[bj[u]];
      const double ga = Gc[rd[u][0]], gb = Gc[rd[u][1]], gc = Gc[rd[u][2]], gd = Gc[rd[u][3]];
      const double tj = cj.y, ti = ci.y;
      const double u1 = fma(-tj, gb, ga), u2 = fma(tj, ga, gb);   // columns of A J_j / c_j, row x
      const double u3 = fma(-tj, gd, gc), u4 = fma(tj, gc, gd);   // row y
      const double cc = ci.x * cj.x;
      Gn[wr[u][0]] = cc * fma(-ti, u3, u1);
      Gn[wr[u][1]] = cc * fma(-ti, u4, u2);
      Gn[wr[u][2]] = cc * fma(ti, u1, u3);
      Gn[wr[u][3]] = cc * fma(ti, u2, u4);
    }
    __syncthreads();
  }
  // output order: decreasing diagonal of Q^T G Q (the new squared row norms),
  // ties by index, so that the rows drift towards their final order
  if (tid < 64) {   // (a NaN sorts last, so the ranks always form a permutation)
    const double* dgf = dg[63 & 1];
    const double d = dgf[tid] == dgf[tid] ? dgf[tid] : -INFINITY;
    int rk = 0;
    for (int m = 0; m < 64; ++m) {
      const double e = dgf[m] == dgf[m] ? dgf[m] : -INFINITY;
      rk += (e > d || (e == d && m < tid)) ? 1 : 0;
    }
    rank_s[tid] = rk;
  }
  __syncthreads();
  {  // last shift (positions back to indices), then Q^T to LDS for the update
    double nq[16];
#pragma unroll
    for (int a = 0; a < 7; ++a) nq[a] = qr[a + 1];
    nq[7] = ws < 3 ? xch[ws + 1][0][lane] : qr[8];
#pragma unroll
    for (int b = 0; b < 7; ++b) nq[8 + b] = qr[9 + b];
    nq[15] = ws > 0 ? xch[ws - 1][1][lane] : qr[1];
    if (ws == 0) nq[0] = qr[0];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      QTf[qt_frag_index(rank_s[8 * ws + a], lane)] = nq[a];
      QTf[qt_frag_index(rank_s[56 - 8 * ws + a], lane)] = nq[8 + a];
    }
  }
  __syncthreads();

  // ---- 3. W_pair <- Q^T W_pair ------------------------------------------
  // Each wave takes 16-column chunks c0 = 16 wave + 64 i; lane (lr, lg) of
  // the B fragment of k-step s holds W_pair[4 s + lg][c0 + lr].  The A
  // fragments are read from LDS (64 consecutive doubles each, no bank
  // conflicts), which leaves the registers for the next chunk's loads, so
  // every wave keeps one chunk in flight while it multiplies the other.
  // Addresses: a uniform row base (rows 0..31 of the pair in block I, 32..63
  // in J) plus the lane's own offset of lg rows and lr columns, so that no
  // per-lane 64-bit row pointers stay live across the loop.
  auto urow = [&](int r) -> double* {
    return r < 32 ? rowI + (size_t)r * n_pad : rowJ + (size_t)(r - 32) * n_pad;
  };
  const int lo = lg * n_pad + lr;
  double bc[16];
  for (int c0 = 16 * wave; c0 < ncol; c0 += 64) {
#pragma unroll
    for (int s = 0; s < 16; ++s) bc[s] = urow(4 * s)[lo + c0];       // row 4 s + lg
    asm volatile("" ::: "memory");   // keep the fragment reads inside the loop
    f64x4 out[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 16; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        out[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(QTf[(16 * t + s) * 64 + lane], bc[s], out[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) urow(16 * t + 4 * i)[lo + c0] = out[t][i];   // row 16 t + acc_row_f64(lg, i)
  }
}

__global__ void jacobi_init_kernel(int64_t njobs, int* active, int* rotated, int* sweeps) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < njobs) { active[j] = 1; rotated[j] = 0; sweeps[j] = -1; }
}

__global__ void jacobi_sweep_end_kernel(int64_t njobs, int sweep, int* active, int* rotated,
                                        int* sweeps, int* counter) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int still = 0;
  if (j < njobs && active[j]) {
    if (rotated[j]) still = 1;
    else { active[j] = 0; sweeps[j] = sweep + 1; }
    rotated[j] = 0;
  }
  // one atomic per wave
  unsigned long long m = __ballot(still);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(counter, __popcll(m));
}

__global__ void zero_int_kernel(int* p) { p[threadIdx.x] = 0; }

hipError_t KernelTimer::begin(hipStream_t s) {
  if (!enabled) return hipSuccess;
  if (used + 2 > 2 * 256) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    e = collect();
    if (e != hipSuccess) return e;
  }
  if (ev[used] == nullptr) {
    hipError_t e = hipEventCreate(&ev[used]);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(ev[used++], s);
}

hipError_t KernelTimer::end(hipStream_t s) {
  if (!enabled) return hipSuccess;
  if (ev[used] == nullptr) {
    hipError_t e = hipEventCreate(&ev[used]);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(ev[used++], s);
}

hipError_t KernelTimer::collect() {
  for (int i = 0; i + 1 < used; i += 2) {
    float t = 0.0f;
    hipError_t e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
    if (e != hipSuccess) return e;
    ms += t;
    ++launches;
    if (ref) {
      float a = 0.0f, b = 0.0f;
      e = hipEventElapsedTime(&a, ref, ev[i]);
      if (e == hipSuccess) e = hipEventElapsedTime(&b, ref, ev[i + 1]);
      if (e != hipSuccess) return e;
      spans.emplace_back(a, b);
    }
  }
  used = 0;
  return hipSuccess;
}

__global__ void zero_ints_kernel(int n, int* p) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t run_jacobi(int64_t njobs, int n_pad, double* W, const JacobiWork& wk, int max_sweeps,
                      hipStream_t stream, KernelTimer* timer, int* sweeps_done, const int* nb_job, int nb_max,
                      int* history, int ncol, int blind, double tabs, int abs_from) {
  if (ncol <= 0 || ncol > n_pad || ncol % 64) ncol = n_pad;
  if (njobs == 0) return hipSuccess;
  const int brows = jacobi_block_rows(n_pad);
  const int nb = nb_job ? nb_max : n_pad / brows;
  const double tol = fmax(32.0, 8.0 * sqrt((double)n_pad)) * 0x1.0p-53;
  // per-sweep counters (jobs still rotating, block pairs rotated) in their own
  // slots when the work area has room for every sweep: the first `blind`
  // sweeps then run without waiting for the host (a sweep of converged jobs
  // leaves every workgroup idle), and one copy brings all their counters back
  const bool slots = wk.hist_len >= max_sweeps;
  if (!slots) blind = 0;
  blind = blind < 0 ? 0 : (blind > max_sweeps ? max_sweeps : blind);
  int g = ceil_div(njobs, 256);
  hipLaunchKernelGGL(jacobi_init_kernel, dim3(g), dim3(256), 0, stream, njobs, wk.active, wk.rotated,
                     wk.sweeps);
  if (slots) hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(256), 0, stream, 2 * max_sweeps, wk.counter);
  if (wk.lastmod && brows == 32) {
    hipError_t e = hipMemsetAsync(wk.lastmod, 0, sizeof(int) * njobs * kJacobiMaxBlocks, stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(wk.lastchk, 0, sizeof(int) * njobs * kJacobiMaxBlocks * kJacobiMaxBlocks, stream);
    if (e != hipSuccess) return e;
  }
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    int* cnt = slots ? wk.counter + 2 * sweep : wk.counter;
    const double ta = (abs_from > 0 && sweep >= abs_from) ? tabs : 0.0;
    if (!slots) hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(2), 0, stream, wk.counter);
    for (int r = 0; r < nb - 1; ++r) {
      if (timer) { hipError_t e = timer->begin(stream); if (e != hipSuccess) return e; }
      if (brows == 32)
        hipLaunchKernelGGL(jacobi_round64_kernel, dim3(nb / 2, (unsigned)njobs), dim3(256), 0, stream, W,
                           n_pad, ncol, nb, nb_job, r, wk.active, wk.rotated, cnt + 1, tol, wk.lastmod, wk.lastchk,
                           1 + sweep * (nb - 1) + r, ta);
      else
        hipLaunchKernelGGL(jacobi_round_kernel, dim3(nb / 2, (unsigned)njobs), dim3(256), 0, stream, W,
                           n_pad, nb, nb_job, r, wk.active, wk.rotated, cnt + 1, tol, ta);
      if (timer) { hipError_t e = timer->end(stream); if (e != hipSuccess) return e; }
    }
    hipLaunchKernelGGL(jacobi_sweep_end_kernel, dim3(g), dim3(256), 0, stream, njobs, sweep, wk.active,
                       wk.rotated, wk.sweeps, cnt);
    if (sweep + 1 < blind) continue;   // no host round trip yet
    const int nslot = slots ? sweep + 1 : 1;      // counter slots to bring back
    hipError_t e = hipMemcpyAsync(wk.counter_host, wk.counter, 2 * nslot * sizeof(int), hipMemcpyDeviceToHost,
                                  stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    if (timer && timer->enabled) {
      e = timer->collect();
      if (e != hipSuccess) return e;
    }
    // the sweeps covered by this copy, up to the first after which no job rotated
    int last = sweep;
    for (int s = (slots ? 0 : sweep); s <= sweep; ++s) {
      const int* h = wk.counter_host + 2 * (slots ? s : 0);
      if (history) { history[2 * s] = h[1]; history[2 * s + 1] = h[0]; }
      if (h[0] == 0) { last = s; break; }
    }
    if (sweeps_done) *sweeps_done = last + 1;
    if (wk.counter_host[2 * (slots ? last : 0)] == 0) break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Noise-floor deflation.  Rows whose squared norm is at most budget^2 / n_pad
// times the largest squared row norm (budget = approx_budget(tau_null)) are
// moved behind the others (stable partition) and excluded from the
// rotations.  Together they hold at most budget^2 times the largest squared
// row norm (at most s_1^2), so leaving them unrotated perturbs the singular
// values of the rest by at most budget s_1 (Weyl; to second order when, as
// after the QR preconditioning, they are nearly orthogonal to the larger
// rows), and their own values (each below budget s_1, a thirtieth of the
// cut) can never be candidates.  nb_job receives the number of row blocks
// (even, at least 2) that cover the active rows.
// Three kernels: squared row norms and the row copy (one wave per row), and
// the partition between them (one workgroup per job); n_pad <= 4096.
// ---------------------------------------------------------------------------
// Squared row norms, one wave per row (lane-strided sum, then a butterfly).
__global__ __launch_bounds__(256) void deflate_norms_kernel(int n_pad, const double* __restrict__ Win,
                                                            double* __restrict__ nrm) {
  const int64_t job = blockIdx.y;
  const int lane = threadIdx.x & 63, r = 4 * blockIdx.x + (threadIdx.x >> 6);
  if (r >= n_pad) return;
  const double* row = Win + ((size_t)job * n_pad + r) * n_pad;
  double sq = 0.0;
  for (int c = lane; c < n_pad; c += 64) sq += row[c] * row[c];
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
  if (lane == 0) nrm[(size_t)job * n_pad + r] = sq;
}

// Per job: the rows above the floor (squared norm > floor_sq times the
// largest) keep their order at the front, the others follow in order
// (stable partition by a block scan, n_pad <= 4096: m = n_pad / 256 rows per
// thread); nb_job = the number of row blocks to rotate (even, >= 2).
__global__ __launch_bounds__(256) void deflate_plan_kernel(int n_pad, int brows, double floor_sq,
                                                           const double* __restrict__ nrm,
                                                           int32_t* __restrict__ newpos, int* __restrict__ nb_job) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* nj = nrm + (size_t)job * n_pad;
  __shared__ double red[4];
  __shared__ int cnt[256];
  double mx = 0.0;
  for (int r = tid; r < n_pad; r += 256) mx = fmax(mx, nj[r]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  const double thr = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * floor_sq;
  const int m = (n_pad + 255) / 256, r0 = tid * m;
  int own = 0;
  for (int q = 0; q < m; ++q)
    if (r0 + q < n_pad && nj[r0 + q] > thr) ++own;
  cnt[tid] = own;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {   // inclusive scan
    const int v = tid >= o ? cnt[tid - o] : 0;
    __syncthreads();
    cnt[tid] += v;
    __syncthreads();
  }
  const int a = cnt[255];                   // rows above the floor
  int before = cnt[tid] - own;              // active rows before r0
  int32_t* pj = newpos + (size_t)job * n_pad;
  for (int q = 0; q < m; ++q) {
    const int r = r0 + q;
    if (r >= n_pad) break;
    if (nj[r] > thr) pj[r] = before++;
    else pj[r] = a + (r - before);
  }
  if (tid == 0) {
    int nbk = 2 * ((a + 2 * brows - 1) / (2 * brows));
    nb_job[job] = nbk < 2 ? 2 : nbk;
  }
}

// Row r moves to newpos[r], one wave per row with 16-byte accesses.
__global__ __launch_bounds__(256) void deflate_copy_kernel(int n_pad, const double* __restrict__ Win,
                                                           const int32_t* __restrict__ newpos,
                                                           double* __restrict__ Wout) {
  const int64_t job = blockIdx.y;
  const int lane = threadIdx.x & 63, r = 4 * blockIdx.x + (threadIdx.x >> 6);
  if (r >= n_pad) return;
  const int d = newpos[(size_t)job * n_pad + r];
  const double2* src = reinterpret_cast<const double2*>(Win + ((size_t)job * n_pad + r) * n_pad);
  double2* dst = reinterpret_cast<double2*>(Wout + ((size_t)job * n_pad + d) * n_pad);
  for (int c = lane; c < n_pad / 2; c += 64) dst[c] = src[c];
}

// Per job: the smallest L such that the rows from L on hold at most
// budget_sq times the largest squared row norm in total (suffix sums of the
// squared norms, which do not increase with L; n_pad <= 4096: m = n_pad / 256
// consecutive rows per thread, scanned from the end).
__global__ __launch_bounds__(256) void last_row_above_kernel(int n_pad, double budget_sq,
                                                             const double* __restrict__ nrm, int* __restrict__ last) {
  const int64_t job = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* nj = nrm + (size_t)job * n_pad;
  __shared__ double red[4];
  __shared__ double suf[256];
  __shared__ int redi[4];
  double mx = 0.0;
  for (int r = tid; r < n_pad; r += 256) mx = fmax(mx, nj[r]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if (lane == 0) red[wave] = mx;
  const int m = (n_pad + 255) / 256, r0 = tid * m;
  double own = 0.0;
  for (int q = 0; q < m; ++q)
    if (r0 + q < n_pad) own += nj[r0 + q];
  suf[tid] = own;
  __syncthreads();
  const double thr = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * budget_sq;
  for (int o = 1; o < 256; o <<= 1) {   // inclusive suffix scan over the chunks
    const double v = tid + o < 256 ? suf[tid + o] : 0.0;
    __syncthreads();
    suf[tid] += v;
    __syncthreads();
  }
  double acc = suf[tid] - own;   // the rows after this thread's chunk
  int cand = n_pad;
  if (acc <= thr) {
    for (int q = m - 1; q >= 0; --q) {
      const int r = r0 + q;
      if (r >= n_pad) continue;
      acc += nj[r];
      if (!(acc <= thr)) break;   // NaN counts as above
      cand = r;
    }
  }
  for (int o = 32; o > 0; o >>= 1) cand = min(cand, __shfl_xor(cand, o));
  if (lane == 0) redi[wave] = cand;
  __syncthreads();
  if (tid == 0) last[job] = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
}

__global__ void max_int_kernel(int64_t n, const int* __restrict__ v, int* __restrict__ out) {
  int m = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = max(m, v[i]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  __shared__ int red[16];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, red[w]);
    *out = max(m, red[0]);
  }
}

hipError_t run_deflate(int64_t njobs, int n_pad, double tau_null, const double* Win, double* Wout, int* nb_job,
                       double* nrm, int32_t* newpos, int* scratch_dev, int* scratch_host, int* nb_max,
                       hipStream_t stream) {
  if (njobs == 0) { *nb_max = 2; return hipSuccess; }
  if (n_pad > 4096) return hipErrorInvalidValue;
  const double budget = approx_budget(tau_null);
  const dim3 rg((unsigned)ceil_div(n_pad, 4), (unsigned)njobs);
  hipLaunchKernelGGL(deflate_norms_kernel, rg, dim3(256), 0, stream, n_pad, Win, nrm);
  hipLaunchKernelGGL(deflate_plan_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, jacobi_block_rows(n_pad),
                     budget * budget / (double)n_pad, (const double*)nrm, newpos, nb_job);
  hipLaunchKernelGGL(deflate_copy_kernel, rg, dim3(256), 0, stream, n_pad, Win, (const int32_t*)newpos, Wout);
  hipLaunchKernelGGL(max_int_kernel, dim3(1), dim3(1024), 0, stream, njobs, nb_job, scratch_dev);
  hipError_t e = hipMemcpyAsync(scratch_host, scratch_dev, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  *nb_max = *scratch_host;
  return hipGetLastError();
}

// The decomposition of a job stops after three QR steps when its rows left
// to rotate after the deflation are at most half of the matrix (2 nb brows
// <= n_pad), else it takes five; decided per job, so that a job's result
// does not depend on the others in its batch.  three[j] / nb_first[j]: the
// decision and the active blocks after this first deflation; *count: the
// jobs that take five.
__global__ void choose_qr_count_kernel(int64_t njobs, int n_pad, int brows, const int* __restrict__ nb_job,
                                       int* __restrict__ three, int* __restrict__ nb_first, int* __restrict__ count) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int five = 0;
  if (j < njobs) {
    const int nb = nb_job[j];
    const int t = 2 * nb * brows <= n_pad ? 1 : 0;
    three[j] = t;
    nb_first[j] = nb;
    five = 1 - t;
  }
  unsigned long long m = __ballot(five);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, __popcll(m));
}

hipError_t run_choose_qr_count(int64_t njobs, int n_pad, const int* nb_job, int* three, int* nb_first,
                               int* scratch_dev, int* scratch_host, int* n_five, hipStream_t stream) {
  if (njobs == 0) { *n_five = 0; return hipSuccess; }
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, stream, 1, scratch_dev);
  hipLaunchKernelGGL(choose_qr_count_kernel, dim3((unsigned)ceil_div(njobs, 256)), dim3(256), 0, stream, njobs, n_pad,
                     jacobi_block_rows(n_pad), nb_job, three, nb_first, scratch_dev);
  hipError_t e = hipMemcpyAsync(scratch_host, scratch_dev, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  *n_five = *scratch_host;
  return hipGetLastError();
}

// The jobs that stop after three QRs (three[j]) take back their deflated
// rows of R3 (Wsrc) as the Jacobi input (Wdst) and their active block count.
__global__ void keep_three_kernel(int n_pad, const int* __restrict__ three, const double* __restrict__ Wsrc,
                                  double* __restrict__ Wdst, const int* __restrict__ nb_first, int* __restrict__ nb_job) {
  const int64_t job = blockIdx.y;
  if (!three[job]) return;
  const size_t per = (size_t)n_pad * n_pad;
  const double2* src = reinterpret_cast<const double2*>(Wsrc + job * per);
  double2* dst = reinterpret_cast<double2*>(Wdst + job * per);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < per / 2; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) nb_job[job] = nb_first[job];
}

hipError_t launch_keep_three(int64_t njobs, int n_pad, const int* three, const double* Wsrc, double* Wdst,
                             const int* nb_first, int* nb_job, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  const size_t half = (size_t)n_pad * n_pad / 2;
  int gx = (int)((half + 255) / 256);
  if (gx > 512) gx = 512;
  hipLaunchKernelGGL(keep_three_kernel, dim3(gx, (unsigned)njobs), dim3(256), 0, stream, n_pad, three, Wsrc, Wdst,
                     nb_first, nb_job);
  return hipGetLastError();
}

hipError_t run_rank_rows(int64_t njobs, int n_pad, double tau_null, const double* W, double* nrm, int* last,
                         int* scratch_dev, int* scratch_host, int* rows_max, hipStream_t stream) {
  if (njobs == 0) { *rows_max = 0; return hipSuccess; }
  if (n_pad > 4096) return hipErrorInvalidValue;
  const double budget = approx_budget(tau_null);
  const dim3 rg((unsigned)ceil_div(n_pad, 4), (unsigned)njobs);
  hipLaunchKernelGGL(deflate_norms_kernel, rg, dim3(256), 0, stream, n_pad, W, nrm);
  hipLaunchKernelGGL(last_row_above_kernel, dim3((unsigned)njobs), dim3(256), 0, stream, n_pad, budget * budget,
                     (const double*)nrm, last);
  hipLaunchKernelGGL(max_int_kernel, dim3(1), dim3(1024), 0, stream, njobs, (const int*)last, scratch_dev);
  hipError_t e = hipMemcpyAsync(scratch_host, scratch_dev, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  *rows_max = *scratch_host;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finalisation: sigma_i = ||row_i||, sorted descending (ties by row index).
// One workgroup of 256 threads per job; bitonic sort over n_pad <= 4096 keys.
// nrm (or NULL): the squared row norms, already summed by deflate_norms_kernel
// (one wavefront per row over the whole grid, the same summation order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void jacobi_finalize_kernel(int n, int n_pad, const double* __restrict__ W,
                                                              const double* __restrict__ nrm,
                                                              double* __restrict__ sigma,
                                                              int32_t* __restrict__ order) {
  extern __shared__ unsigned char smem[];
  int P = 1;
  while (P < n_pad) P <<= 1;
  double* key = reinterpret_cast<double*>(smem);
  int* idx = reinterpret_cast<int*>(key + P);
  const int job = blockIdx.x;
  const double* Wj = W + (size_t)job * n_pad * n_pad;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (nrm) {
    for (int r = threadIdx.x; r < P; r += 256) {
      key[r] = r < n_pad ? sqrt(nrm[(size_t)job * n_pad + r]) : -1.0;   // padding sorts last
      idx[r] = r;
    }
  }
  for (int r = wave; r < P && !nrm; r += 4) {
    double s = 0.0;
    if (r < n_pad) {
      const double* row = Wj + (size_t)r * n_pad;
      for (int c = lane; c < n_pad; c += 64) s += row[c] * row[c];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    } else {
      s = -1.0;   // padding sorts last
    }
    if (lane == 0) { key[r] = (r < n_pad) ? sqrt(s) : -1.0; idx[r] = r; }
  }
  __syncthreads();
  // bitonic sort: descending key, ascending index on ties
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += 256) {
        int i = 2 * stride * (t / stride) + (t % stride);
        int jx = i + stride;
        bool up = ((i & size) == 0);
        double ki = key[i], kj = key[jx];
        int ii = idx[i], ij = idx[jx];
        bool i_first = (ki > kj) || (ki == kj && ii < ij);   // i should precede j
        bool swap = up ? !i_first : i_first;
        if (swap) { key[i] = kj; key[jx] = ki; idx[i] = ij; idx[jx] = ii; }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += 256) {
    sigma[(size_t)job * n + i] = key[i];
    order[(size_t)job * n + i] = idx[i];
  }
}

// ---------------------------------------------------------------------------
// QR-iteration basis (the decomposition that skips the Jacobi): with M P Q =
// Q' R (Q = Q2 or Q2 Q4, R the last triangular factor, rows stored row-major
// in R), the columns of M P Q have the norms of the columns of R.
// basis_colnorm_kernel: their squares, one thread per column, summed over
// the first nrows rows (the rest are zero).  basis_rows_kernel: W = diag of
// those norms, so that the vector recovery reads the unit vector e_j as the
// j-th "rotated row" over its norm.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void basis_colnorm_kernel(int n_pad, int nrows, const double* __restrict__ R,
                                                            double* __restrict__ nrm) {
  const int64_t job = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n_pad) return;
  const double* Rj = R + (size_t)job * n_pad * n_pad + j;
  double s = 0.0;
  for (int r = 0; r < nrows; ++r) {
    const double x = Rj[(size_t)r * n_pad];
    s += x * x;
  }
  nrm[(size_t)job * n_pad + j] = s;
}

__global__ __launch_bounds__(256) void basis_rows_kernel(int n_pad, const double* __restrict__ nrm,
                                                         double* __restrict__ W) {
  const int64_t job = blockIdx.y;
  const int lane = threadIdx.x & 63, r = 4 * blockIdx.x + (threadIdx.x >> 6);
  if (r >= n_pad) return;
  double2* row = reinterpret_cast<double2*>(W + ((size_t)job * n_pad + r) * n_pad);
  const double d = sqrt(nrm[(size_t)job * n_pad + r]);
  for (int c = lane; c < n_pad / 2; c += 64) {
    double2 v;
    v.x = (2 * c == r) ? d : 0.0;
    v.y = (2 * c + 1 == r) ? d : 0.0;
    row[c] = v;
  }
}

hipError_t launch_qr_basis(int64_t njobs, int n, int n_pad, int nrows, const double* R, double* nrm, double* W,
                           double* sigma, int32_t* order, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  if (n_pad % 32 || nrows < 0 || nrows > n_pad) return hipErrorInvalidValue;
  hipLaunchKernelGGL(basis_colnorm_kernel, dim3((unsigned)ceil_div(n_pad, 256), (unsigned)njobs), dim3(256), 0, stream,
                     n_pad, nrows, R, nrm);
  hipLaunchKernelGGL(basis_rows_kernel, dim3((unsigned)ceil_div(n_pad, 4), (unsigned)njobs), dim3(256), 0, stream,
                     n_pad, (const double*)nrm, W);
  int P = 1;
  while (P < n_pad) P <<= 1;
  const size_t sh = (size_t)P * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(jacobi_finalize_kernel, dim3((unsigned)njobs), dim3(256), sh, stream, n, n_pad,
                     (const double*)W, (const double*)nrm, sigma, order);
  return hipGetLastError();
}

hipError_t launch_jacobi_finalize(int64_t njobs, int n, int n_pad, const double* W, double* sigma,
                                  int32_t* order, hipStream_t stream, double* nrm) {
  if (njobs == 0) return hipSuccess;
  int P = 1;
  while (P < n_pad) P <<= 1;
  size_t sh = (size_t)P * (sizeof(double) + sizeof(int));
  if (nrm)
    hipLaunchKernelGGL(deflate_norms_kernel, dim3((unsigned)ceil_div(n_pad, 4), (unsigned)njobs), dim3(256), 0,
                       stream, n_pad, W, nrm);
  hipLaunchKernelGGL(jacobi_finalize_kernel, dim3((unsigned)njobs), dim3(256), sh, stream, n, n_pad, W,
                     (const double*)nrm, sigma, order);
  return hipGetLastError();
}

}  // namespace mctrg
