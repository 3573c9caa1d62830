// Contraction step: the four factor halves around a plaquette form the
// coarse tensor (Levin-Nave TRG, paper Section III):
//   T'[a,b,c,e] = sum_{p,q,s,t} G_A[a,p,t] G_B[b,q,p] F_A[s,q,c] F_B[t,s,e].
// It is evaluated as
//   X[(a,b)][(t,q)]  = sum_p G_A[a,p,t] G_B[b,q,p]     (2 k^2 D^3 flops, FP64)
//   Yt[(c,e)][(t,q)] = sum_s F_A[s,q,c] F_B[t,s,e]     (2 k^2 D^3 flops, FP64)
//   T'[(a,b)][(c,e)] = sum_{(t,q)} X Yt^T              (2 k^4 D^2 flops, MFMA)
// The last product dominates; it runs in the contraction dtype:
//   F64  v_mfma_f64_16x16x4_f64, FP64 output
//   F32  v_mfma_f32_16x16x4_f32
//   BF16 v_mfma_f32_16x16x32_bf16, FP32 accumulation
//   FP8  v_mfma_f32_16x16x32_fp8_fp8 (OCP e4m3), FP32 accumulation
// Narrow operands are scaled per (tensor, operand) by a power of two so
// that max|x| < 2^target (1 for BF16/F32, 256 for e4m3) before rounding;
// the normalisation step divides the scales back out.
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "mctrg_internal.h"
#include "../../include/mctrg.h"

namespace mctrg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// X and Yt (FP64).  One workgroup per (a or c, output tensor).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void contract_X_kernel(int D, int kk, int kcap, const double* __restrict__ GApool,
                                                         const double* __restrict__ GBpool, int64_t g_stride,
                                                         const int32_t* __restrict__ jobs, double* __restrict__ X) {
  extern __shared__ double sh[];
  const int a = blockIdx.x;
  const int64_t o = blockIdx.y;
  const int DD = D * D, ld = D + 1;
  double* GAa = sh;               // [p][t]
  double* GBb = sh + D * ld;      // [q][p]
  const double* GA = GApool + (size_t)jobs[4 * o + 0] * g_stride + (size_t)a * DD;
  const double* GBbase = GBpool + (size_t)jobs[4 * o + 1] * g_stride;
  for (int e = threadIdx.x; e < DD; e += 256) GAa[(e / D) * ld + e % D] = GA[e];
  double* Xo = X + (size_t)o * kk * kk * DD;
  const bool stage_b = D <= 45;   // both operands fit 32 KB of LDS each
  for (int b = 0; b < kk; ++b) {
    __syncthreads();
    const double* GB = GBbase + (size_t)b * DD;
    if (stage_b)
      for (int e = threadIdx.x; e < DD; e += 256) GBb[(e / D) * ld + e % D] = GB[e];
    __syncthreads();
    for (int e = threadIdx.x; e < DD; e += 256) {
      const int t = e / D, q = e % D;
      double s = 0.0;
      if (stage_b)
        for (int p = 0; p < D; ++p) s += GAa[p * ld + t] * GBb[q * ld + p];
      else
        for (int p = 0; p < D; ++p) s += GAa[p * ld + t] * GB[q * D + p];
      Xo[((size_t)a * kk + b) * DD + e] = s;
    }
  }
  (void)kcap;
}

__global__ __launch_bounds__(256) void contract_Y_kernel(int D, int kk, int kcap, const double* __restrict__ FApool,
                                                         const double* __restrict__ FBpool, int64_t f_stride,
                                                         const int32_t* __restrict__ jobs, double* __restrict__ Yt) {
  extern __shared__ double sh[];
  const int c = blockIdx.x;
  const int64_t o = blockIdx.y;
  const int DD = D * D, ld = D + 1;
  double* FAc = sh;               // [s][q]
  double* FBe = sh + D * ld;      // [t][s]
  // F by kept index: u_c of FA and u_ee of FB are D^2 contiguous doubles each
  const double* FA = FApool + (size_t)jobs[4 * o + 2] * f_stride + (size_t)c * DD;
  const double* FB = FBpool + (size_t)jobs[4 * o + 3] * f_stride;
  for (int e = threadIdx.x; e < DD; e += 256) FAc[(e / D) * ld + e % D] = FA[e];
  double* Yo = Yt + (size_t)o * kk * kk * DD;
  const bool stage_b = D <= 45;
  for (int ee = 0; ee < kk; ++ee) {
    const double* FBee = FB + (size_t)ee * DD;
    __syncthreads();
    if (stage_b)
      for (int e = threadIdx.x; e < DD; e += 256) FBe[(e / D) * ld + e % D] = FBee[e];
    __syncthreads();
    for (int e = threadIdx.x; e < DD; e += 256) {
      const int t = e / D, q = e % D;
      double s = 0.0;
      if (stage_b)
        for (int ss = 0; ss < D; ++ss) s += FBe[t * ld + ss] * FAc[ss * ld + q];
      else
        for (int ss = 0; ss < D; ++ss) s += FBee[t * D + ss] * FAc[ss * ld + q];
      Yo[((size_t)c * kk + ee) * DD + e] = s;
    }
  }
  (void)kcap;
}

// out[j][c][e] = in[j][e][c]: 32 x 32 tiles transposed through LDS.
__global__ __launch_bounds__(256) void f_by_kept_kernel(int DD, int kk, const double* __restrict__ in,
                                                        double* __restrict__ out) {
  __shared__ double tile[32][33];
  const int64_t j = blockIdx.z;
  const int e0 = 32 * blockIdx.x, c0 = 32 * blockIdx.y;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double* ij = in + (size_t)j * DD * kk;
  double* oj = out + (size_t)j * DD * kk;
  for (int yy = ty; yy < 32; yy += 8) {
    const int e = e0 + yy, c = c0 + tx;
    tile[yy][tx] = (e < DD && c < kk) ? ij[(size_t)e * kk + c] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int c = c0 + yy, e = e0 + tx;
    if (c < kk && e < DD) oj[(size_t)c * DD + e] = tile[tx][yy];
  }
}

hipError_t launch_f_by_kept(int64_t njobs, int D, int kk, const double* in, double* out, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  const int DD = D * D;
  hipLaunchKernelGGL(f_by_kept_kernel, dim3((unsigned)ceil_div(DD, 32), (unsigned)ceil_div(kk, 32), (unsigned)njobs),
                     dim3(256), 0, stream, DD, kk, in, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-(tensor, operand) power-of-two scales and narrow casts.
// ---------------------------------------------------------------------------
__global__ void absmax_kernel(int64_t per, const double* __restrict__ A, double* __restrict__ mx) {
  const int64_t o = blockIdx.y;
  const double* Ao = A + o * per;
  double m = 0.0;
  // unrolled so that each thread keeps four loads in flight
#pragma unroll 4
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < per; e += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(Ao[e]));
  for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(&mx[o], m);
}

__global__ void fill_kernel(int64_t n, double* p, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// scale = 2^(target - E) with max = f 2^E, f in [0.5, 1)  (1 if max == 0)
__global__ void make_scale_kernel(int64_t n, double* mx_to_scale, int target) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m = mx_to_scale[i];
  double s = 1.0;
  if (m > 0.0 && isfinite(m)) {
    int E;
    frexp(m, &E);
    s = ldexp(1.0, target - E);
  }
  mx_to_scale[i] = s;
}

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <int DT>
__global__ void cast_kernel(int64_t per, const double* __restrict__ A, const double* __restrict__ scale,
                            void* __restrict__ out) {
  const int64_t o = blockIdx.y;
  const double s = scale[o];
  const double* Ao = A + o * per;
#pragma unroll 4
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < per; e += (int64_t)gridDim.x * blockDim.x) {
    const float v = (float)(Ao[e] * s);
    if (DT == MCTRG_F32) {
      reinterpret_cast<float*>(out)[o * per + e] = v;
    } else if (DT == MCTRG_BF16) {
      reinterpret_cast<unsigned short*>(out)[o * per + e] = f32_to_bf16_rne(v);
    } else {
      int packed = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false);
      reinterpret_cast<unsigned char*>(out)[o * per + e] = (unsigned char)(packed & 0xFF);
    }
  }
}

// ---------------------------------------------------------------------------
// Batched GEMM C[o] = A[o] (M x K, row-major) * B[o]^T (B: N x K, row-major).
// 64 x 64 tile per workgroup, four waves of 32 x 32 (2 x 2 MFMA 16x16 tiles),
// K staged through LDS in chunks of 32.
// ---------------------------------------------------------------------------
template <int DT> struct Mma;
// KSTEP: K per MFMA; BK: K per LDS tile (one barrier pair per tile), 32 for
// the four-element MFMAs and 128 for the narrow types (BF16: 256 bytes of K
// per row; FP8: 128 bytes, which keeps its 128-tile variant within two waves
// per SIMD), so that a wave issues 4 x 4 x 4 MFMAs between barriers.
template <> struct Mma<MCTRG_F64> {
  typedef double elt; typedef double acc_t; typedef f64x4 frag_c;
  static constexpr int KSTEP = 4, PAD = 1, BK = 32;
};
template <> struct Mma<MCTRG_F32> {
  typedef float elt; typedef float acc_t; typedef f32x4 frag_c;
  static constexpr int KSTEP = 4, PAD = 1, BK = 32;
};
template <> struct Mma<MCTRG_BF16> {
  typedef unsigned short elt; typedef float acc_t; typedef f32x4 frag_c;
  static constexpr int KSTEP = 32, PAD = 8, BK = 128;
};
template <> struct Mma<MCTRG_FP8_E4M3> {
  typedef unsigned char elt; typedef float acc_t; typedef f32x4 frag_c;
  static constexpr int KSTEP = 32, PAD = 16, BK = 128;
};

template <int DT>
__device__ __forceinline__ typename Mma<DT>::frag_c mma_step(const typename Mma<DT>::elt* a,
                                                             const typename Mma<DT>::elt* b,
                                                             typename Mma<DT>::frag_c c) {
  if constexpr (DT == MCTRG_F64) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(*a, *b, c, 0, 0, 0);
  } else if constexpr (DT == MCTRG_F32) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
  } else if constexpr (DT == MCTRG_BF16) {
    bf16x8 av = *reinterpret_cast<const bf16x8*>(a);
    bf16x8 bv = *reinterpret_cast<const bf16x8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  } else {
    long av = *reinterpret_cast<const long*>(a);
    long bv = *reinterpret_cast<const long*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, c, 0, 0, 0);
  }
}

// Tile shapes (template parameter BM, picked per dtype and GEMM shape by the
// autotuner in launch_contract): BM x BM workgroup tiles of four waves, each
// wave a (BM/2) x (BM/2) block of WT x WT MFMA 16 x 16 tiles, WT = BM / 32.
// BM = 128 halves the operand loads per flop of BM = 64 at four times the
// accumulator registers (FP64: 128 VGPRs) and twice the LDS (FP64: 67 KB,
// two workgroups per CU).

// The 128-tile variants of the narrow types are held to two workgroups per
// CU (256 registers per lane): left to itself the compiler preloads enough
// LDS operands to drop them to one wave per SIMD.
template <int DT, int BM>
__global__ __launch_bounds__(256, (BM == 128 && (DT == MCTRG_BF16 || DT == MCTRG_FP8_E4M3)) ? 2 : 1) void gemm_tn_kernel(int M, int N, int K, const void* __restrict__ Av,
                                                      const void* __restrict__ Bv, void* __restrict__ Cv) {
  typedef typename Mma<DT>::elt elt;
  typedef typename Mma<DT>::acc_t acc_t;
  typedef typename Mma<DT>::frag_c frag_c;
  constexpr int WT = BM / 32;                              // MFMA tiles per wave side
  constexpr int BK = Mma<DT>::BK, LD = BK + Mma<DT>::PAD, KS = Mma<DT>::KSTEP;
  constexpr int EPL = (KS == 4) ? 1 : 8;                  // elements per lane per MFMA
  __shared__ __attribute__((aligned(16))) elt As[BM * LD];
  __shared__ __attribute__((aligned(16))) elt Bs[BM * LD];
  const int64_t o = blockIdx.z;
  const elt* A = reinterpret_cast<const elt*>(Av) + (size_t)o * M * K;
  const elt* B = reinterpret_cast<const elt*>(Bv) + (size_t)o * N * K;
  acc_t* C = reinterpret_cast<acc_t*>(Cv) + (size_t)o * M * N;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (16 * WT), wn = (wave & 1) * (16 * WT);
  const int lr = lane & 15, lg = lane >> 4;
  frag_c acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = frag_c{0, 0, 0, 0};

  // Tile-aligned shapes (the steady state): 16-byte loads with the lanes along
  // K, so every wave reads whole 64..256-byte row segments.  Other shapes use
  // masked element loads.
  constexpr int VB = 16 / (int)sizeof(elt);   // elements per 16-byte vector
  constexpr int LPR = BK / VB;                // lanes per tile row
  constexpr int RPI = 256 / LPR;              // tile rows per pass
  constexpr int ITERS = (BM + RPI - 1) / RPI;  // (8-bit, BM = 64: one pass over half the threads)
  const bool vec = (M % BM == 0) && (N % BM == 0) && (K % BK == 0);
  const int vrow = tid / LPR, vk = (tid % LPR) * VB;
  uint4 va[ITERS], vb[ITERS];
  auto gload = [&](int k0) {   // the next tile into registers (tile-aligned shapes)
    if (!vec) return;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int row = it * RPI + vrow;
      if (RPI * ITERS > BM && row >= BM) continue;
      va[it] = *reinterpret_cast<const uint4*>(A + (size_t)(m0 + row) * K + k0 + vk);
      vb[it] = *reinterpret_cast<const uint4*>(B + (size_t)(n0 + row) * K + k0 + vk);
    }
  };
  auto lstore = [&](int k0) {
    if (vec) {
#pragma unroll
      for (int it = 0; it < ITERS; ++it) {
        const int row = it * RPI + vrow;
        if (RPI * ITERS > BM && row >= BM) continue;
        const elt* ea = reinterpret_cast<const elt*>(&va[it]);
        const elt* eb = reinterpret_cast<const elt*>(&vb[it]);
#pragma unroll
        for (int v = 0; v < VB; ++v) {
          As[row * LD + vk + v] = ea[v];
          Bs[row * LD + vk + v] = eb[v];
        }
      }
      return;
    }
    // other shapes: element loads straight into LDS, zero outside M x K / N x K
    for (int e = tid; e < BM * BK; e += 256) {
      const int row = e / BK, kk = e % BK, gk = k0 + kk;
      const int gm = m0 + row, gn = n0 + row;
      As[row * LD + kk] = (gm < M && gk < K) ? A[(size_t)gm * K + gk] : elt(0);
      Bs[row * LD + kk] = (gn < N && gk < K) ? B[(size_t)gn * K + gk] : elt(0);
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    lstore(k0);
    __syncthreads();
    if (k0 + BK < K) gload(k0 + BK);    // next K tile in flight during the MFMAs
#pragma unroll
    for (int ks = 0; ks < BK; ks += KS) {
      const int kofs = ks + lg * EPL;
#pragma unroll
      for (int i = 0; i < WT; ++i) {
        const elt* ap = &As[(wm + 16 * i + lr) * LD + kofs];
#pragma unroll
        for (int j = 0; j < WT; ++j) {
          const elt* bp = &Bs[(wn + 16 * j + lr) * LD + kofs];
          acc[i][j] = mma_step<DT>(ap, bp, acc[i][j]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + (DT == MCTRG_F64 ? acc_row_f64(lg, r) : acc_row_f32(lg, r));
        const int gn = n0 + wn + 16 * j + lr;
        if (gm < M && gn < N) C[(size_t)gm * N + gn] = acc[i][j][r];
      }
}

template <typename T>
__global__ void unscale_kernel(int64_t elems, const T* __restrict__ C, const double* __restrict__ scales,
                               int64_t nout, double* __restrict__ out) {
  const int64_t o = blockIdx.y;
  const double inv = 1.0 / (scales[o] * scales[nout + o]);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < elems; e += (int64_t)gridDim.x * blockDim.x)
    out[o * elems + e] = (double)C[o * elems + e] * inv;
}

hipError_t launch_unscale(int64_t nout, int64_t elems, int src_is_f32, const void* C, const double* scales,
                          double* T_out, hipStream_t stream) {
  if (nout == 0) return hipSuccess;
  int gx = (int)((elems + 255) / 256);
  if (gx > 256) gx = 256;
  if (src_is_f32)
    hipLaunchKernelGGL(unscale_kernel<float>, dim3(gx, (unsigned)nout), dim3(256), 0, stream, elems,
                       (const float*)C, scales, nout, T_out);
  else
    hipLaunchKernelGGL(unscale_kernel<double>, dim3(gx, (unsigned)nout), dim3(256), 0, stream, elems,
                       (const double*)C, scales, nout, T_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile autotuner: the first GEMM of a (dtype, M, N, K, batch) shape on a
// device times both tile shapes on the call's own operands (best of three
// launches each, HIP events on the call's stream) and keeps the faster for
// every later call of that shape.  The environment variable MCTRG_GEMM_TILE
// (64 or 128) forces a shape (used by the tests to check both).
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
  int dev, dt, M, N, K;
  int64_t batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, dt, M, N, K, batch) < std::tie(o.dev, o.dt, o.M, o.N, o.K, o.batch);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

template <int DT, int BM>
hipError_t launch_gemm_bm(int M, int N, int K, int64_t nout, const void* A, const void* B, void* C,
                          hipStream_t stream) {
  dim3 grid(ceil_div(N, BM), ceil_div(M, BM), (unsigned)nout);
  hipLaunchKernelGGL((gemm_tn_kernel<DT, BM>), grid, dim3(256), 0, stream, M, N, K, A, B, C);
  return hipGetLastError();
}

template <int DT>
hipError_t launch_gemm_tile(int bm, int M, int N, int K, int64_t nout, const void* A, const void* B, void* C,
                            hipStream_t stream) {
  return bm == 128 ? launch_gemm_bm<DT, 128>(M, N, K, nout, A, B, C, stream)
                   : launch_gemm_bm<DT, 64>(M, N, K, nout, A, B, C, stream);
}

hipError_t launch_gemm_dt(int dt, int bm, int M, int N, int K, int64_t nout, const void* A, const void* B, void* C,
                          hipStream_t stream) {
  switch (dt) {
    case MCTRG_F64: return launch_gemm_tile<MCTRG_F64>(bm, M, N, K, nout, A, B, C, stream);
    case MCTRG_F32: return launch_gemm_tile<MCTRG_F32>(bm, M, N, K, nout, A, B, C, stream);
    case MCTRG_BF16: return launch_gemm_tile<MCTRG_BF16>(bm, M, N, K, nout, A, B, C, stream);
    case MCTRG_FP8_E4M3: return launch_gemm_tile<MCTRG_FP8_E4M3>(bm, M, N, K, nout, A, B, C, stream);
    default: return hipErrorInvalidValue;
  }
}

// The tile shape for this GEMM: forced, cached, or measured now.
hipError_t pick_tile(int dt, int M, int N, int K, int64_t nout, const void* A, const void* B, void* C,
                     hipStream_t stream, int* bm) {
  if (const char* f = std::getenv("MCTRG_GEMM_TILE")) {
    const int v = std::atoi(f);
    if (v == 64 || v == 128) { *bm = v; return hipSuccess; }
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const TuneKey key{dev, dt, M, N, K, nout};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { *bm = it->second; return hipSuccess; }
  }
  // below one tile of 128 in either dimension the small tile always wins
  if (M < 128 || N < 128) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = 64;
    *bm = 64;
    return hipSuccess;
  }
  hipEvent_t ev[2];
  if ((e = hipEventCreate(&ev[0])) != hipSuccess) return e;
  if ((e = hipEventCreate(&ev[1])) != hipSuccess) { (void)hipEventDestroy(ev[0]); return e; }
  float best_ms[2] = {1e30f, 1e30f};
  const int shapes[2] = {64, 128};
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
    for (int t = 0; t < 2 && e == hipSuccess; ++t) {
      e = hipEventRecord(ev[0], stream);
      if (e == hipSuccess) e = launch_gemm_dt(dt, shapes[t], M, N, K, nout, A, B, C, stream);
      if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e == hipSuccess) best_ms[t] = std::min(best_ms[t], ms);
    }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return e;
  *bm = best_ms[1] < best_ms[0] ? 128 : 64;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = *bm;
  return hipSuccess;
}
}  // namespace

int gemm_tile_chosen(int dt, int M, int N, int K, int64_t nout) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(TuneKey{dev, dt, M, N, K, nout});
  return it == g_tune.end() ? 0 : it->second;
}

static hipError_t run_gemm(int dt, int M, int N, int K, int64_t nout, const void* A, const void* B, void* C,
                           hipStream_t stream, KernelTimer* gt) {
  int bm = 64;
  hipError_t e = pick_tile(dt, M, N, K, nout, A, B, C, stream, &bm);
  if (e != hipSuccess) return e;
  if (gt) { e = gt->begin(stream); if (e != hipSuccess) return e; }
  e = launch_gemm_dt(dt, bm, M, N, K, nout, A, B, C, stream);
  if (e != hipSuccess) return e;
  if (gt) { e = gt->end(stream); if (e != hipSuccess) return e; }
  return hipSuccess;
}

hipError_t launch_contract(const ContractArgs& a, hipStream_t stream, KernelTimer* gt) {
  if (a.nout == 0) return hipSuccess;
  const int D = a.D, kk = a.kk, DD = D * D, MM = kk * kk;
  const size_t sh = (size_t)(D <= 45 ? 2 : 1) * D * (D + 1) * sizeof(double);
  const int kcap = kk;
  hipLaunchKernelGGL(contract_X_kernel, dim3(kk, (unsigned)a.nout), dim3(256), sh, stream, D, kk, kcap, a.GA,
                     a.GB, a.g_stride, a.jobs, a.X);
  hipLaunchKernelGGL(contract_Y_kernel, dim3(kk, (unsigned)a.nout), dim3(256), sh, stream, D, kk, kcap, a.FA,
                     a.FB, a.f_stride, a.jobs, a.Y);
  const int64_t per = (int64_t)MM * DD;
  if (a.dtype == MCTRG_F64) {
    hipLaunchKernelGGL(fill_kernel, dim3(ceil_div(2 * a.nout, 256)), dim3(256), 0, stream, 2 * a.nout, a.scales, 1.0);
    hipError_t e = run_gemm(MCTRG_F64, MM, MM, DD, a.nout, a.X, a.Y, a.Tout, stream, gt);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  // scales: the first nout entries for X, the next nout for Yt
  const int target = (a.dtype == MCTRG_FP8_E4M3) ? 8 : 0;
  hipLaunchKernelGGL(fill_kernel, dim3(ceil_div(2 * a.nout, 256)), dim3(256), 0, stream, 2 * a.nout, a.scales, 0.0);
  int gx = (int)((per + 255) / 256);
  if (gx > 256) gx = 256;
  double* mxX = a.scales;
  double* mxY = a.scales + a.nout;
  hipLaunchKernelGGL(absmax_kernel, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.X, mxX);
  hipLaunchKernelGGL(absmax_kernel, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.Y, mxY);
  hipLaunchKernelGGL(make_scale_kernel, dim3(ceil_div(2 * a.nout, 256)), dim3(256), 0, stream, 2 * a.nout,
                     a.scales, target);
  switch (a.dtype) {
    case MCTRG_F32:
      hipLaunchKernelGGL(cast_kernel<MCTRG_F32>, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.X, mxX, a.Xlp);
      hipLaunchKernelGGL(cast_kernel<MCTRG_F32>, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.Y, mxY, a.Ylp);
      break;
    case MCTRG_BF16:
      hipLaunchKernelGGL(cast_kernel<MCTRG_BF16>, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.X, mxX, a.Xlp);
      hipLaunchKernelGGL(cast_kernel<MCTRG_BF16>, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.Y, mxY, a.Ylp);
      break;
    case MCTRG_FP8_E4M3:
      hipLaunchKernelGGL(cast_kernel<MCTRG_FP8_E4M3>, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.X, mxX, a.Xlp);
      hipLaunchKernelGGL(cast_kernel<MCTRG_FP8_E4M3>, dim3(gx, (unsigned)a.nout), dim3(256), 0, stream, per, a.Y, mxY, a.Ylp);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = run_gemm(a.dtype, MM, MM, DD, a.nout, a.Xlp, a.Ylp, a.Tout, stream, gt);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace mctrg
