// Host runtime and C ABI of the MI355X Monte Carlo TRG library.
//
// run_samples buckets samples by kept count k, splits every bucket into
// waves that fit the device memory, and runs each wave as a chain: the
// starting tensors are gathered per sample, n_steps TRG steps are applied
// (unfold -> Jacobi SVD -> sample/reweight -> factors -> contraction ->
// normalisation), and the last tensor is traced (paper Section III).
// In independent mode the batch is (sample x lattice position) and the
// contraction gathers its four halves from the plaquette's four positions.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "../../include/mctrg.h"
#include "mctrg_internal.h"

using namespace mctrg;

struct mctrg_tensor_set {
  int ngroups;
  int d0;
  int device;
  double* T0;   // device, ngroups * d0^4
};

namespace {

constexpr int kMaxSweeps = 120;
// Sweeps after which the Jacobi also accepts pairs at the approximation
// budget's absolute floor (the FP64 forms converge in at most about a dozen)
constexpr int kAbsFromSweep = 30;

// ---------------------------------------------------------------------------
// Independent-mode lattice (TRG geometry on a torus).
// Legs (l,u,r,d) = 0..3; leg r of a site joins leg l of its right neighbour,
// leg d joins leg u of the site below.  One new tensor per A site p0, from
// G_A(p0), G_B(q0 = r of p0), F_A(p1 = d of q0), F_B(q1 = d of p0); its new
// l' leg joins r' of the tensor of (l of (u of p0)) and its u' leg joins d'
// of the tensor of (u of (r of p0)).  New ids are ranks of the A-site ids;
// new sublattices come from a 2-colouring started at position 0.
// ---------------------------------------------------------------------------
struct Level {
  int n = 0;
  std::vector<int> nbr;     // 4 per position
  std::vector<char> is_a;
};

Level square_torus(int L) {
  Level v;
  v.n = L * L;
  v.nbr.resize(4 * v.n);
  v.is_a.resize(v.n);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int i = x + L * y;
      v.nbr[4 * i + 0] = (x + L - 1) % L + L * y;
      v.nbr[4 * i + 1] = x + L * ((y + L - 1) % L);
      v.nbr[4 * i + 2] = (x + 1) % L + L * y;
      v.nbr[4 * i + 3] = x + L * ((y + 1) % L);
      v.is_a[i] = ((x + y) % 2) == 0;
    }
  return v;
}

bool coarsen(const Level& lev, std::vector<int>& plaq, Level& nxt) {
  std::vector<int> newid(lev.n, -1);
  int m = 0;
  for (int p = 0; p < lev.n; ++p)
    if (lev.is_a[p]) newid[p] = m++;
  plaq.assign(4 * m, 0);
  nxt.n = m;
  nxt.nbr.assign(4 * m, -1);
  nxt.is_a.assign(m, 0);
  auto nb = [&](int p, int d) { return lev.nbr[4 * p + d]; };
  for (int p0 = 0; p0 < lev.n; ++p0) {
    if (!lev.is_a[p0]) continue;
    const int P = newid[p0];
    const int q0 = nb(p0, 2), p1 = nb(q0, 3), q1 = nb(p0, 3);
    if (nb(q1, 2) != p1 || lev.is_a[q0] || lev.is_a[q1] || !lev.is_a[p1]) return false;
    plaq[4 * P + 0] = p0; plaq[4 * P + 1] = q0; plaq[4 * P + 2] = p1; plaq[4 * P + 3] = q1;
  }
  for (int p0 = 0; p0 < lev.n; ++p0) {
    if (!lev.is_a[p0]) continue;
    const int P = newid[p0];
    const int Ql = newid[nb(nb(p0, 1), 0)], Qu = newid[nb(nb(p0, 2), 1)];
    if (Ql < 0 || Qu < 0) return false;
    if (nxt.nbr[4 * P + 0] >= 0 || nxt.nbr[4 * Ql + 2] >= 0) return false;
    nxt.nbr[4 * P + 0] = Ql; nxt.nbr[4 * Ql + 2] = P;
    if (nxt.nbr[4 * P + 1] >= 0 || nxt.nbr[4 * Qu + 3] >= 0) return false;
    nxt.nbr[4 * P + 1] = Qu; nxt.nbr[4 * Qu + 3] = P;
  }
  for (int v : nxt.nbr)
    if (v < 0) return false;
  // 2-colouring
  std::vector<int> col(m, -1), queue;
  col[0] = 0;
  queue.push_back(0);
  for (size_t h = 0; h < queue.size(); ++h) {
    const int p = queue[h];
    for (int d = 0; d < 4; ++d) {
      const int q = nxt.nbr[4 * p + d];
      if (col[q] < 0) { col[q] = 1 - col[p]; queue.push_back(q); }
      else if (m > 1 && col[q] == col[p]) return false;
    }
  }
  for (int p = 0; p < m; ++p) {
    if (col[p] < 0) return false;
    nxt.is_a[p] = col[p] == 0;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Device arena: one allocation carved into 256-byte aligned pieces.
// ---------------------------------------------------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool counting = true;
  template <typename T>
  T* take(size_t count) {
    const size_t bytes = ((count * sizeof(T) + 255) / 256) * 256 + 256;
    T* p = counting ? nullptr : reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

struct HostPinned {
  void* p = nullptr;
  ~HostPinned() { if (p) (void)hipHostFree(p); }
};

int32_t capacity_next(int32_t D, int32_t k) {
  const int64_t sq = (int64_t)D * D;
  return (int32_t)std::min<int64_t>(k, sq);
}

struct StepShape {
  int D, kc, n, n_pad, P, jps, ops;
};

struct Chain {
  hipStream_t st = nullptr;
  int mode = 0, dtype = 0, k = 0, n_steps = 0, kmax_rec = 0;
  int n_det = 0;   // leading deterministic (top-k) steps; independent mode: on one shared tensor
  int dec = MCTRG_DEC_SVD;   // decomposition: SVD, or the QR-iteration basis of 3 or 5 QRs
  double tau = 1e-11;
  uint64_t seed = 0;
  int64_t nsamp = 0;
  int step = 0;
  uint32_t flags = 0;
  int32_t* record = nullptr;
  std::vector<int> Dsched;
  std::vector<Level> levels;
  std::vector<std::vector<int>> plaqs;
  std::vector<int64_t> sids;
  // device
  char* mem = nullptr;
  double *Ta = nullptr, *Tb = nullptr, *Tn = nullptr, *W = nullptr, *sigma = nullptr, *logr = nullptr,
         *weight = nullptr, *sscr = nullptr, *G = nullptr, *Gt = nullptr, *F = nullptr, *X = nullptr, *Y = nullptr,
         *scales = nullptr, *cbuf = nullptr, *lnc = nullptr, *lnc_steps = nullptr, *lnabs = nullptr;
  void *Xlp = nullptr, *Ylp = nullptr;
  double *S = nullptr, *Tws = nullptr, *W2 = nullptr, *Tws2 = nullptr, *W3 = nullptr, *Tscr = nullptr;
  double* W4 = nullptr;         // deflated rows of R3 of the jobs that stop after three QRs (n_pad <= 1024)
  int* three_job = nullptr;     // per job: stopped after three QRs
  int* nb_first = nullptr;      // per job: active blocks after the first deflation
  int32_t* perm = nullptr;
  int32_t* colmap = nullptr;   // column re-ordering of the first QR (n_pad <= 1024)
  double* colnorm = nullptr;
  int32_t *order = nullptr, *kept = nullptr, *cand = nullptr, *sel = nullptr, *src = nullptr, *split = nullptr,
          *cjobs = nullptr;
  uint64_t* rng = nullptr;
  int64_t* idx = nullptr;
  int* failed = nullptr;
  int8_t* sign = nullptr;
  JacobiWork jw{};
  int* nb_job = nullptr;
  double* dnrm = nullptr;    // deflation: squared row norms, target rows (n_pad per job)
  int32_t* dpos = nullptr;
  // host staging (pinned)
  HostPinned pin;
  int32_t *h_src = nullptr, *h_split = nullptr, *h_cjobs = nullptr;
  uint64_t* h_rng = nullptr;
  int64_t max_jobs = 0, max_out = 0;
  KernelTimer tj, tg, tq;   // Jacobi rounds, GEMMs, 128-column QR trailing updates
  double tq_flops = 0.0;    // algorithmic flops of the timed QR trailing updates
  int last_sweeps = 0;
  int sweep_hist[2 * kMaxSweeps] = {};   // last decomposition: (pairs rotated, jobs active) per sweep
  int64_t rotated_pairs = 0;              // block pairs rotated, summed over all steps and sweeps
  double jacobi_flops = 0.0;              // their Gram + update flops at the row length used
  int step_sweeps[64] = {};               // Jacobi sweeps of every step
  int64_t fail_sid = -1;                  // test hook: global sample id whose last ln c is made non-finite

  ~Chain() {
    if (mem) (void)hipFree(mem);
  }

  StepShape shape(int s) const {
    StepShape sh;
    sh.D = Dsched[s];
    sh.kc = Dsched[s + 1];
    sh.n = sh.D * sh.D;
    sh.n_pad = std::max(32, round_up32(sh.n));
    if (mode == MCTRG_INDEPENDENT && s >= n_det) {
      sh.P = levels[s].n;
      sh.jps = sh.P;
      sh.ops = sh.P / 2;
    } else {
      sh.P = 1;
      sh.jps = 2;
      sh.ops = 1;
    }
    return sh;
  }

  double* Tcur() { return Ta; }
};

// Lays out (or, when counting, sizes) every device buffer of a chain.
void layout(Chain& c, Arena& ar) {
  size_t tmax = 0, wmax = 0, w4max = 0, nmax = 0, selmax = 0, sscr = 0, gmax = 0, xmax = 0, tnmax = 0, pmax = 0;
  int64_t jmax = 0, omax = 0;
  for (int s = 0; s < c.n_steps; ++s) {
    const StepShape sh = c.shape(s);
    const int64_t nj = c.nsamp * sh.jps, no = c.nsamp * sh.ops;
    const size_t D4 = (size_t)sh.D * sh.D * sh.D * sh.D, K4 = (size_t)sh.kc * sh.kc * sh.kc * sh.kc;
    tmax = std::max(tmax, (size_t)c.nsamp * sh.P * D4);
    tmax = std::max(tmax, (size_t)no * K4);
    wmax = std::max(wmax, (size_t)nj * sh.n_pad * sh.n_pad);
    if (sh.n_pad <= 1024) w4max = std::max(w4max, (size_t)nj * sh.n_pad * sh.n_pad);
    nmax = std::max(nmax, (size_t)nj * sh.n);
    pmax = std::max(pmax, (size_t)nj * sh.n_pad);
    selmax = std::max(selmax, (size_t)nj * sh.kc);
    sscr = std::max(sscr, sample_scratch_doubles(nj, sh.n, sh.kc));
    gmax = std::max(gmax, (size_t)nj * sh.kc * sh.n);
    xmax = std::max(xmax, (size_t)no * sh.kc * sh.kc * sh.n);
    tnmax = std::max(tnmax, (size_t)no * K4);
    jmax = std::max(jmax, nj);
    omax = std::max(omax, no);
  }
  c.max_jobs = jmax;
  c.max_out = omax;
  c.Ta = ar.take<double>(tmax);
  c.Tb = ar.take<double>(tmax);
  c.Tn = ar.take<double>(tnmax);
  c.W = ar.take<double>(wmax);
  c.S = ar.take<double>(wmax);
  c.W2 = ar.take<double>(wmax);
  c.W3 = ar.take<double>(wmax);
  c.W4 = ar.take<double>(w4max);
  c.Tscr = ar.take<double>((size_t)jmax * kQrTscr);
  c.Tws = ar.take<double>((size_t)jmax * 32 * 1024);
  c.Tws2 = ar.take<double>((size_t)jmax * 32 * 1024);
  c.perm = ar.take<int32_t>((size_t)jmax * 4096);
  c.colmap = ar.take<int32_t>((size_t)jmax * 1024);
  c.colnorm = ar.take<double>((size_t)jmax * 1024);
  c.sigma = ar.take<double>(nmax);
  c.order = ar.take<int32_t>(nmax);
  c.kept = ar.take<int32_t>(jmax);
  c.cand = ar.take<int32_t>(jmax);
  c.sel = ar.take<int32_t>(selmax);
  c.logr = ar.take<double>(selmax);
  c.weight = ar.take<double>(selmax);
  c.sscr = ar.take<double>(sscr);
  c.G = ar.take<double>(gmax);
  c.Gt = ar.take<double>(gmax);
  c.F = ar.take<double>(gmax);
  c.X = ar.take<double>(xmax);
  c.Y = ar.take<double>(xmax);
  if (c.dtype != MCTRG_F64) {
    c.Xlp = ar.take<float>(xmax);
    c.Ylp = ar.take<float>(xmax);
  }
  c.scales = ar.take<double>(2 * omax);
  c.cbuf = ar.take<double>(omax);
  c.lnc = ar.take<double>(omax);
  c.src = ar.take<int32_t>(jmax);
  c.split = ar.take<int32_t>(jmax);
  c.rng = ar.take<uint64_t>(3 * jmax);
  c.cjobs = ar.take<int32_t>(4 * omax);
  c.idx = ar.take<int64_t>(c.nsamp);
  c.lnc_steps = ar.take<double>((size_t)c.nsamp * c.n_steps);
  c.failed = ar.take<int>(c.nsamp);
  c.sign = ar.take<int8_t>(c.nsamp);
  c.lnabs = ar.take<double>(c.nsamp);
  c.jw.active = ar.take<int>(jmax);
  c.jw.rotated = ar.take<int>(jmax);
  c.jw.sweeps = ar.take<int>(jmax);
  c.jw.counter = ar.take<int>(2 * kMaxSweeps);
  c.jw.lastmod = ar.take<int>((size_t)jmax * kJacobiMaxBlocks);
  c.jw.lastchk = ar.take<int>((size_t)jmax * kJacobiMaxBlocks * kJacobiMaxBlocks);
  c.nb_job = ar.take<int>(jmax);
  c.three_job = ar.take<int>(jmax);
  c.nb_first = ar.take<int>(jmax);
  c.dnrm = ar.take<double>(pmax);
  c.dpos = ar.take<int32_t>(pmax);
}

std::vector<int> schedule(int d0, int k, int n_steps) {
  std::vector<int> D(n_steps + 1);
  D[0] = d0;
  for (int s = 0; s < n_steps; ++s) D[s + 1] = capacity_next(D[s], k);
  return D;
}

int build_levels(Chain& c) {
  const int L = 1 << (c.n_steps / 2);
  Level lev = square_torus(L);
  for (int s = 0; s < c.n_steps; ++s) {
    std::vector<int> plaq;
    Level nxt;
    if (!coarsen(lev, plaq, nxt)) return MCTRG_EINVAL;
    c.levels.push_back(lev);
    c.plaqs.push_back(plaq);
    lev = nxt;
  }
  if (lev.n != 1) return MCTRG_EINVAL;
  return MCTRG_OK;
}

// int32 entries of the selection record per sample: shared and top-k
// n_steps * (4 + 2 kmax); independent mode (2 + kmax) per position of every
// level.
int64_t record_per_sample(const Chain& c) {
  if (c.mode != MCTRG_INDEPENDENT) return (int64_t)c.n_steps * (4 + 2 * c.kmax_rec);
  int64_t n = 0;
  for (int t = 0; t < c.n_steps; ++t) n += (int64_t)c.levels[t].n * (2 + c.kmax_rec);
  return n;
}

size_t chain_bytes(Chain& c) {
  Arena ar;
  layout(c, ar);
  return ar.off;
}

#define CKH(x)                                  \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return MCTRG_EDEVICE; \
  } while (0)

// ---------------------------------------------------------------------------
// The decomposition of a batch of unfoldings (paper Section II, Eq.
// exactSVD), shared by the chains and the step-level SVD entry point.
// ---------------------------------------------------------------------------
struct DecompBufs {
  double *S, *W, *W2, *W3, *W4, *Tscr, *Tws, *Tws2, *colnorm, *dnrm, *sigma;
  int32_t *perm, *colmap, *dpos, *order;
  int *nb_job, *three_job, *nb_first;
  JacobiWork jw;
};

DecompBufs decomp_bufs(const Chain& c) {
  return DecompBufs{c.S,    c.W,      c.W2,    c.W3,   c.W4,    c.Tscr,   c.Tws,       c.Tws2,     c.colnorm,
                    c.dnrm, c.sigma,  c.perm,  c.colmap, c.dpos, c.order, c.nb_job, c.three_job, c.nb_first,
                    c.jw};
}

struct DecompCtl {
  int dec = MCTRG_DEC_SVD;
  double tau = 0.0;        // candidate cut: sets the approximation budget
  int blind = 0;           // Jacobi sweeps launched before the first host round trip
  KernelTimer* tq = nullptr;
  double* tq_flops = nullptr;
  KernelTimer* tj = nullptr;
  int* sweep_hist = nullptr;   // host, 2 kMaxSweeps ints, or NULL
};

// Where the result is: the rows Wj whose norms are the singular values
// (sigma / order hold them sorted), and which orthogonal factors map the
// normalised rows to the right singular vectors: Q2 (W / Tws2) and Q4 (S /
// Tws) after five QRs (qr5 && !three; nob, if not NULL, marks per job those
// that stopped after three, for which Q4 is not applied), Q2 alone after
// three (three: every job, or qr without qr5), none on the direct route.
struct DecompOut {
  double* Wj = nullptr;
  const int* nob = nullptr;
  bool qr5 = false, qr = false, three = false, qr_basis = false;
  int jcols = 0;    // the Jacobi rows are zero from this column on (0: none)
  int sweeps = 0;   // Jacobi sweeps of the slowest job
};

// Three or five QRs (n_pad <= 1024) or three (n_pad <= 4096), then Jacobi on
// the rows of the last R; larger unfoldings go straight to the Jacobi.  Rows
// at the noise floor or below a tenth of the candidate cut move behind the
// active ones and are not rotated (deflation).  The early stop of the first
// QR, the rank limit of the later ones and the deflation each drop at most
// approx_budget(tau) s_1 in Frobenius norm.
hipError_t decompose(int64_t nj, int n, int D, int n_pad, const double* T, const int32_t* src, const int32_t* split,
                     const DecompBufs& b, const DecompCtl& ctl, DecompOut& out, hipStream_t st) {
#define HKE(x)                           \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) return e_;     \
  } while (0)
  out = DecompOut{};
  const bool qr5 = n_pad <= 1024;
  const bool qr = n_pad <= kQrMaxN;
  out.qr5 = qr5;
  out.qr = qr;
  double* rows = b.W2;   // the rows handed to the Jacobi
  double* Wj = b.W;      // the Jacobi workspace
  int nb_max = 0;
  const bool qr_basis = qr5 && ctl.dec != MCTRG_DEC_SVD;
  out.qr_basis = qr_basis;
  if (qr5) {
    // a job's first QR stops once the columns it has not factored hold at most
    // the approximation budget (its later rows of R1 are set to zero and its
    // column order is frozen); the batch factors on until every job has stopped
    QrStop stop;
    stop.budget = approx_budget(ctl.tau);
    stop.dev = b.jw.counter;
    stop.host = b.jw.counter_host;
    stop.rows_job = b.nb_job;   // free until the rank rows below
    HKE(run_qr1(nj, n, D, n_pad, T, src, split, b.perm, b.dpos, b.S, b.W, b.Tscr, b.colmap, b.colnorm, st, &stop));
    // The first QR re-orders the columns by norm, so the rows of R1 come in
    // roughly decreasing norm: the later QRs run over the leading ncols
    // columns only.  Every job's rows of R1 from its own limit on hold at
    // most the approximation budget in total and are set to zero (which
    // moves the singular values by at most their Frobenius norm); ncols is
    // the largest limit, and a job's zero columns below it are exact no-ops.
    int rows1 = 0;
    HKE(run_rank_rows(nj, n_pad, ctl.tau, b.W, b.dnrm, b.nb_job, b.jw.counter, b.jw.counter_host, &rows1, st));
    const int ncols = std::min(n_pad, std::max(128, 128 * ceil_div(rows1, 128)));
    HKE(run_qr23(nj, n_pad, ncols, b.W, b.Tws2, b.W2, b.W3, b.Tscr, st, ctl.tq, ctl.tq_flops, b.nb_job));
    if (qr_basis) {
      // the cheaper decomposition: the basis V = P Q2 (Q4) of three (five) QR
      // steps, the terms (M v_j) v_j^T weighted by |M v_j| = the column norms
      // of R3 (R5); no Jacobi
      if (ctl.dec == MCTRG_DEC_QR5) HKE(run_qr45(nj, n_pad, ncols, b.S, b.W2, b.Tws, b.W3, b.Tscr, st, ctl.tq, ctl.tq_flops));
      out.three = ctl.dec == MCTRG_DEC_QR3;
      out.Wj = b.W2;
      return launch_qr_basis(nj, n, n_pad, ncols, b.W3, b.dnrm, b.W2, b.sigma, b.order, st);
    }
    out.jcols = ncols;
    // The QR iteration of a job stops after three steps when its rows left to
    // rotate are at most half of the matrix (a cut above the tensor's
    // rounding floor deflates its noise subspace): the Jacobi on them then
    // costs less than the fourth and fifth QR would save.  Otherwise those
    // follow.  Decided per job: in a batch of both kinds the fourth and
    // fifth QR run on all, and the jobs that stop after three take back
    // their deflated rows of R3 (kept in W4) before the Jacobi.
    HKE(run_deflate(nj, n_pad, ctl.tau, b.W3, b.W4, b.nb_job, b.dnrm, b.dpos, b.jw.counter, b.jw.counter_host,
                    &nb_max, st));
    int n_five = 0;
    HKE(run_choose_qr_count(nj, n_pad, b.nb_job, b.three_job, b.nb_first, b.jw.counter, b.jw.counter_host, &n_five,
                            st));
    if (n_five == 0) {
      out.three = true;
      Wj = b.W4;         // W / Tws2 keep Q2
    } else {
      HKE(run_qr45(nj, n_pad, ncols, b.S, b.W2, b.Tws, b.W3, b.Tscr, st, ctl.tq, ctl.tq_flops));
      rows = b.W3;       // W / Tws2 keep Q2, S / Tws keep Q4
      Wj = b.W2;
      if (n_five < nj) out.nob = b.three_job;
    }
  } else if (qr) {
    HKE(run_qr3_precondition(nj, n, D, n_pad, T, src, split, b.perm, b.dpos, b.S, b.Tws, b.W, b.Tws2, b.W2, b.colmap,
                             b.colnorm, &rows, st));
    Wj = b.W2;           // W keeps Q2
  } else {
    HKE(launch_unfold(nj, D, n_pad, T, src, split, b.W2, st));
    HKE(launch_iota(nj, n_pad, b.perm, st));
  }
  if (!out.three) {
    int nb2 = 0;
    HKE(run_deflate(nj, n_pad, ctl.tau, rows, Wj, b.nb_job, b.dnrm, b.dpos, b.jw.counter, b.jw.counter_host, &nb2,
                    st));
    if (out.nob) {   // the jobs that stopped after three QRs
      HKE(launch_keep_three(nj, n_pad, b.three_job, b.W4, Wj, b.nb_first, b.nb_job, st));
      nb_max = std::max(nb_max, nb2);
    } else {
      nb_max = nb2;
    }
  }
  // a job still rotating after kAbsFromSweep sweeps (rows stalled at the
  // rounding of the larger ones) converges at the budget's absolute floor
  HKE(run_jacobi(nj, n_pad, Wj, b.jw, kMaxSweeps, st, ctl.tj, &out.sweeps, b.nb_job, nb_max, ctl.sweep_hist,
                 out.jcols, ctl.blind, approx_budget(ctl.tau) / std::sqrt((double)n_pad), kAbsFromSweep));
  out.Wj = Wj;
  return launch_jacobi_finalize(nj, n, n_pad, Wj, b.sigma, b.order, st, b.dnrm);
#undef HKE
}

// Allocates the chain's memory and gathers its starting tensors.
int chain_start(Chain& c, const mctrg_tensor_set* ts, const std::vector<int32_t>& groups,
                const std::vector<int64_t>& out_index) {
  Arena ar;
  layout(c, ar);
  const size_t bytes = ar.off;
  if (hipMalloc(&c.mem, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c.mem = nullptr;
    return MCTRG_ENOMEM;
  }
  ar.base = c.mem;
  ar.off = 0;
  ar.counting = false;
  layout(c, ar);
  const int64_t J = c.max_jobs, O = c.max_out;
  const size_t hb = sizeof(int32_t) * (2 * J + 4 * O) + sizeof(uint64_t) * 3 * J + 2 * kMaxSweeps * sizeof(int) + 64;
  if (hipHostMalloc(&c.pin.p, hb, hipHostMallocDefault) != hipSuccess) return MCTRG_ENOMEM;
  char* hp = reinterpret_cast<char*>(c.pin.p);
  c.h_rng = reinterpret_cast<uint64_t*>(hp);
  hp += sizeof(uint64_t) * 3 * J;
  c.h_src = reinterpret_cast<int32_t*>(hp);
  hp += sizeof(int32_t) * J;
  c.h_split = reinterpret_cast<int32_t*>(hp);
  hp += sizeof(int32_t) * J;
  c.h_cjobs = reinterpret_cast<int32_t*>(hp);
  hp += sizeof(int32_t) * 4 * O;
  c.jw.counter_host = reinterpret_cast<int*>(hp);
  c.jw.hist_len = kMaxSweeps;

  // groups -> device (staged through the cjobs area, int32 per sample)
  int32_t* dgroups = c.cjobs;  // reused before the first step
  std::vector<int32_t> g = groups;
  if ((int64_t)g.size() > 4 * O) return MCTRG_EINVAL;
  CKH(hipMemcpyAsync(dgroups, g.data(), g.size() * sizeof(int32_t), hipMemcpyHostToDevice, c.st));
  CKH(hipMemcpyAsync(c.idx, out_index.data(), out_index.size() * sizeof(int64_t), hipMemcpyHostToDevice, c.st));
  // every position of a sample starts from the sample's group tensor
  const int P0 = (c.mode == MCTRG_INDEPENDENT && c.n_det == 0) ? c.levels[0].n : 1;
  if (P0 == 1) {
    CKH(launch_gather_tensors(c.nsamp, ts->d0, ts->T0, dgroups, c.Ta, c.st));
  } else {
    // expand groups to (sample, position)
    std::vector<int32_t> gp((size_t)c.nsamp * P0);
    for (int64_t s = 0; s < c.nsamp; ++s)
      for (int p = 0; p < P0; ++p) gp[(size_t)s * P0 + p] = groups[s];
    int32_t* dg2 = c.src;   // J >= nsamp * P0 at step 0
    CKH(hipMemcpyAsync(dg2, gp.data(), gp.size() * sizeof(int32_t), hipMemcpyHostToDevice, c.st));
    CKH(launch_gather_tensors(c.nsamp * P0, ts->d0, ts->T0, dg2, c.Ta, c.st));
  }
  CKH(launch_izero(c.nsamp, c.failed, c.st));
  CKH(hipMemsetAsync(c.lnc_steps, 0, sizeof(double) * c.nsamp * c.n_steps, c.st));
  CKH(hipStreamSynchronize(c.st));
  c.tj.enabled = c.tg.enabled = c.tq.enabled = (c.flags & MCTRG_PROFILE) != 0;
  return MCTRG_OK;
}

int chain_step(Chain& c) {
  const int s = c.step;
  const StepShape sh = c.shape(s);
  const int64_t nj = c.nsamp * sh.jps, no = c.nsamp * sh.ops;
  // job descriptors
  const bool indep = c.mode == MCTRG_INDEPENDENT && s >= c.n_det;
  if (indep) {
    const Level& lev = c.levels[s];
    const std::vector<int>& pl = c.plaqs[s];
    for (int64_t i = 0; i < c.nsamp; ++i) {
      for (int p = 0; p < sh.P; ++p) {
        const int64_t j = i * sh.P + p;
        c.h_src[j] = (int32_t)j;
        c.h_split[j] = lev.is_a[p] ? 0 : 1;
        c.h_rng[3 * j + 0] = (uint64_t)c.sids[i];
        c.h_rng[3 * j + 1] = (uint64_t)p;
        c.h_rng[3 * j + 2] = (uint64_t)s;
      }
      for (int P = 0; P < sh.ops; ++P) {
        const int64_t o = i * sh.ops + P;
        for (int t = 0; t < 4; ++t) c.h_cjobs[4 * o + t] = (int32_t)(i * sh.P + pl[4 * P + t]);
      }
    }
  } else {
    for (int64_t i = 0; i < c.nsamp; ++i) {
      for (int sp = 0; sp < 2; ++sp) {
        const int64_t j = 2 * i + sp;
        c.h_src[j] = (int32_t)i;
        c.h_split[j] = sp;
        c.h_rng[3 * j + 0] = (uint64_t)c.sids[i];
        c.h_rng[3 * j + 1] = 0;
        c.h_rng[3 * j + 2] = (uint64_t)s;
      }
      c.h_cjobs[4 * i + 0] = (int32_t)(2 * i);
      c.h_cjobs[4 * i + 1] = (int32_t)(2 * i + 1);
      c.h_cjobs[4 * i + 2] = (int32_t)(2 * i);
      c.h_cjobs[4 * i + 3] = (int32_t)(2 * i + 1);
    }
  }
  CKH(hipMemcpyAsync(c.src, c.h_src, nj * sizeof(int32_t), hipMemcpyHostToDevice, c.st));
  CKH(hipMemcpyAsync(c.split, c.h_split, nj * sizeof(int32_t), hipMemcpyHostToDevice, c.st));
  CKH(hipMemcpyAsync(c.rng, c.h_rng, 3 * nj * sizeof(uint64_t), hipMemcpyHostToDevice, c.st));
  CKH(hipMemcpyAsync(c.cjobs, c.h_cjobs, 4 * no * sizeof(int32_t), hipMemcpyHostToDevice, c.st));

  DecompOut dout;
  {
    DecompCtl ctl;
    ctl.dec = c.dec;
    ctl.tau = c.tau;
    // the first sweeps run without host round trips: as many as the previous
    // step needed, less two (a sweep after convergence only launches idle
    // workgroups)
    ctl.blind = c.last_sweeps - 2;
    if (c.tq.enabled) {
      ctl.tq = &c.tq;
      ctl.tq_flops = &c.tq_flops;
    }
    if (c.tj.enabled) ctl.tj = &c.tj;
    ctl.sweep_hist = c.sweep_hist;
    CKH(decompose(nj, sh.n, sh.D, sh.n_pad, c.Ta, c.src, c.split, decomp_bufs(c), ctl, dout, c.st));
    c.last_sweeps = dout.sweeps;
  }
  const bool qr5 = dout.qr5, qr = dout.qr, three = dout.three, qr_basis = dout.qr_basis;
  double* const Wj = dout.Wj;
  if (s < 64) c.step_sweeps[s] = c.last_sweeps;
  if (!qr_basis) {
    int64_t rp = 0;
    for (int w = 0; w < c.last_sweeps && w < kMaxSweeps; ++w) rp += c.sweep_hist[2 * w];
    // per rotated pair of two row blocks (2 brows rows): the symmetric Gram
    // (2 brows)^2 len and the update W <- Q^T W, 2 (2 brows)^2 len
    const double rows = 2.0 * jacobi_block_rows(sh.n_pad), len = dout.jcols > 0 ? dout.jcols : sh.n_pad;
    c.rotated_pairs += rp;
    c.jacobi_flops += (double)rp * 3.0 * rows * rows * len;
    CKH(launch_jacobi_fail(nj, sh.jps, c.jw.sweeps, c.failed, c.st));
  }
  SampleArgs sa{};
  sa.njobs = nj; sa.n = sh.n; sa.k = sh.kc; sa.mode = s < c.n_det ? MCTRG_TOPK : c.mode; sa.seed = c.seed;
  sa.tau = c.tau;
  sa.sigma = c.sigma; sa.rng = c.rng; sa.split = c.split; sa.kept = c.kept; sa.cand = c.cand;
  sa.sel = c.sel; sa.log_r = c.logr; sa.weight = c.weight; sa.scratch = c.sscr;
  CKH(launch_sample(sa, c.st));
  if ((c.flags & MCTRG_RECORD) && c.record) {
    if (c.mode == MCTRG_INDEPENDENT) {
      int64_t base = 0;
      for (int t = 0; t < s; ++t) base += (int64_t)c.levels[t].n * (2 + c.kmax_rec);
      // the deterministic prefix decomposes one tensor per sample: its A and
      // B split fill positions 0 and 1 of the level
      CKH(launch_record_positions(c.nsamp, indep ? sh.P : 2, record_per_sample(c), base, c.kmax_rec, sh.kc, c.idx,
                                  c.cand, c.kept, c.sel, c.record, c.st));
    } else {
      CKH(launch_record(c.nsamp, s, c.n_steps, c.kmax_rec, sh.kc, c.idx, c.cand, c.kept, c.sel, c.record, c.st));
    }
  }
  if (qr5 && !three) {
    // z = Q2 Q4 y (in F as scratch), v = P z into G with the gauge, u = M v / s
    CKH(launch_apply_q1(nj, sh.n, sh.n_pad, sh.kc, c.W, nullptr, c.Tws2, c.S, c.Tws, Wj, c.sigma, c.order, c.kept,
                        c.sel, c.weight, c.F, c.st, dout.nob));
    CKH(launch_scatter_G(nj, sh.D, sh.n_pad, sh.kc, c.F, c.perm, c.colmap, c.kept, c.G, c.st));
    CKH(launch_factor_F(nj, sh.D, sh.kc, c.Ta, c.src, c.split, c.sigma, c.kept, c.sel, c.G, c.Gt, c.F, c.st));
  } else if (qr) {
    // z = Q2 y (in F as scratch; three QRs), v = P z into G with the gauge, u = M v / s
    CKH(launch_apply_q1(nj, sh.n, sh.n_pad, sh.kc, c.W, nullptr, c.Tws2, nullptr, nullptr, Wj, c.sigma, c.order,
                        c.kept, c.sel, c.weight, c.F, c.st));
    CKH(launch_scatter_G(nj, sh.D, sh.n_pad, sh.kc, c.F, c.perm, sh.n_pad <= 1024 ? c.colmap : nullptr, c.kept, c.G,
                         c.st));
    CKH(launch_factor_F(nj, sh.D, sh.kc, c.Ta, c.src, c.split, c.sigma, c.kept, c.sel, c.G, c.Gt, c.F, c.st));
  } else {
    CKH(launch_factor_G(nj, sh.D, sh.n_pad, sh.kc, Wj, c.sigma, c.order, c.kept, c.sel, c.weight, c.perm, c.G,
                        c.st));
    CKH(launch_factor_F(nj, sh.D, sh.kc, c.Ta, c.src, c.split, c.sigma, c.kept, c.sel, c.G, c.Gt, c.F, c.st));
  }
  ContractArgs ca{};
  ca.nout = no; ca.D = sh.D; ca.kk = sh.kc; ca.dtype = c.dtype;
  ca.GA = c.G; ca.GB = c.G; ca.FA = c.F; ca.FB = c.F;
  ca.g_stride = (int64_t)sh.kc * sh.n; ca.f_stride = (int64_t)sh.n * sh.kc;
  ca.jobs = c.cjobs; ca.X = c.X; ca.Y = c.Y; ca.Xlp = c.Xlp; ca.Ylp = c.Ylp; ca.scales = c.scales; ca.Tout = c.Tn;
  CKH(launch_contract(ca, c.st, c.tg.enabled ? &c.tg : nullptr));
  const int64_t K4 = (int64_t)sh.kc * sh.kc * sh.kc * sh.kc;
  CKH(launch_normalize(no, K4, c.dtype != MCTRG_F64, c.Tn, c.scales, c.cbuf, c.Tb, c.lnc, c.st));
  if (c.fail_sid >= 0 && s == c.n_steps - 1)
    for (int64_t i = 0; i < c.nsamp; ++i)
      if (c.sids[i] == c.fail_sid) CKH(launch_set_double(c.lnc + i * sh.ops, std::nan(""), c.st));
  // independent mode sums ln c over the level's tensors: a step of the
  // deterministic prefix stands for all 2^(n_steps - s - 1) equal new tensors
  const double mult = (c.mode == MCTRG_INDEPENDENT && s < c.n_det) ? std::ldexp(1.0, c.n_steps - s - 1) : 1.0;
  CKH(launch_lnc_accum(c.nsamp, sh.ops, s, c.n_steps, mult, c.lnc, c.lnc_steps, c.failed, c.st));
  std::swap(c.Ta, c.Tb);
  c.step++;
  if (c.mode == MCTRG_INDEPENDENT && c.step == c.n_det && c.n_det < c.n_steps) {
    // switch to the independent estimator: every position of the coarse
    // lattice starts from the sample's deterministic tensor
    const int P = c.levels[c.n_det].n;
    for (int64_t j = 0; j < c.nsamp * P; ++j) c.h_src[j] = (int32_t)(j / P);
    CKH(hipMemcpyAsync(c.src, c.h_src, c.nsamp * P * sizeof(int32_t), hipMemcpyHostToDevice, c.st));
    CKH(launch_gather_tensors(c.nsamp * P, c.Dsched[c.n_det], c.Ta, c.src, c.Tb, c.st));
    // the next step refills the pinned staging buffer: the copy above must be done first
    CKH(hipStreamSynchronize(c.st));
    std::swap(c.Ta, c.Tb);
  }
  if (c.tg.enabled) {
    CKH(hipStreamSynchronize(c.st));
    CKH(c.tg.collect());
    CKH(c.tq.collect());
  }
  return MCTRG_OK;
}

int chain_finish(Chain& c, int8_t* out_sign, double* out_ln, double* out_lnc, double* out_tensor) {
  const int Df = c.Dsched[c.step];
  if (c.mode == MCTRG_INDEPENDENT && c.step != c.n_steps) return MCTRG_EINVAL;
  CKH(launch_trace(c.nsamp, Df, c.Ta, c.lnc_steps, c.n_steps, c.step, c.mode != MCTRG_INDEPENDENT, c.failed,
                   c.sign, c.lnabs, c.st));
  CKH(launch_scatter(c.nsamp, c.n_steps, c.idx, c.sign, c.lnabs, c.lnc_steps, out_sign, out_ln, out_lnc, c.st));
  if (out_tensor) {
    const size_t per = (size_t)Df * Df * Df * Df;
    std::vector<int64_t> idx(c.nsamp);
    CKH(hipMemcpyAsync(idx.data(), c.idx, c.nsamp * sizeof(int64_t), hipMemcpyDeviceToHost, c.st));
    CKH(hipStreamSynchronize(c.st));
    for (int64_t s = 0; s < c.nsamp; ++s)
      CKH(hipMemcpyAsync(out_tensor + (size_t)idx[s] * per, c.Ta + (size_t)s * per, per * sizeof(double),
                         hipMemcpyDeviceToDevice, c.st));
  }
  return MCTRG_OK;
}

// A wave of samples advanced as up to kParts parts: each part is a Chain with
// its own device memory and stream (part 0 on the caller's stream, the others
// on non-blocking streams of default priority created here), stepped by its
// own host thread.  A part's host thread waits for the convergence count after
// every Jacobi sweep, and its QR panels are latency-bound; meanwhile the
// other parts' kernels fill the GPU.  Per-sample results do not depend on the
// split: every random draw is addressed by the global sample id and every
// decomposition is independent.
constexpr int kParts = 3;

struct ChainParts {
  int device = 0;
  hipStream_t caller = nullptr;
  std::vector<std::unique_ptr<Chain>> parts;
  std::vector<hipStream_t> own;   // streams of parts 1, 2, ...
  hipEvent_t ref = nullptr;    // common origin of the kernel timers
  hipEvent_t done = nullptr;
  ~ChainParts() {
    parts.clear();   // frees the parts' device memory
    for (hipStream_t s : own) (void)hipStreamDestroy(s);
    if (ref) (void)hipEventDestroy(ref);
    if (done) (void)hipEventDestroy(done);
  }
};

// Starts the parts of samples [0, n) (groups, out_index and sids per
// sample); configure sets a fresh Chain's configuration fields.
int parts_start(ChainParts& cp, const std::function<void(Chain&)>& configure, const mctrg_tensor_set* ts,
                const std::vector<int32_t>& groups, const std::vector<int64_t>& out_index,
                const std::vector<int64_t>& sids, hipStream_t caller, bool one_part, bool profile) {
  cp.caller = caller;
  CKH(hipGetDevice(&cp.device));
  const int64_t n = (int64_t)groups.size();
  const int P = one_part ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(kParts, n));
  CKH(hipEventCreateWithFlags(&cp.done, hipEventDisableTiming));
  if (profile) {
    CKH(hipEventCreate(&cp.ref));
    CKH(hipEventRecord(cp.ref, caller));
  }
  if (P > 1) {   // the other parts start after the work already queued on the caller's stream
    CKH(hipEventRecord(cp.done, caller));
    for (int p = 1; p < P; ++p) {
      hipStream_t s = nullptr;
      CKH(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      cp.own.push_back(s);
      CKH(hipStreamWaitEvent(s, cp.done, 0));
    }
  }
  int64_t b = 0;
  for (int p = 0; p < P; ++p) {
    const int64_t e = (n * (p + 1) + P - 1) / P;
    std::unique_ptr<Chain> c(new (std::nothrow) Chain());
    if (!c) return MCTRG_ENOMEM;
    configure(*c);
    c->st = p == 0 ? caller : cp.own[p - 1];
    c->nsamp = e - b;
    c->sids.assign(sids.begin() + b, sids.begin() + e);
    const std::vector<int32_t> g(groups.begin() + b, groups.begin() + e);
    const std::vector<int64_t> oi(out_index.begin() + b, out_index.begin() + e);
    const int rc = chain_start(*c, ts, g, oi);
    if (rc != MCTRG_OK) return rc;
    c->tj.ref = c->tg.ref = c->tq.ref = cp.ref;
    cp.parts.push_back(std::move(c));
    b = e;
  }
  return MCTRG_OK;
}

// The caller's stream waits for the work queued on the other parts' streams.
int parts_join(ChainParts& cp) {
  for (size_t p = 1; p < cp.parts.size(); ++p) {
    CKH(hipEventRecord(cp.done, cp.parts[p]->st));
    CKH(hipStreamWaitEvent(cp.caller, cp.done, 0));
  }
  return MCTRG_OK;
}

// n TRG steps on every part, part 0 on the calling thread and the others on
// threads of their own (one after the other if a thread cannot be started).
int parts_step(ChainParts& cp, int n) {
  const int P = (int)cp.parts.size();
  std::vector<int> rcs(P, MCTRG_OK);
  auto run = [&](int p) {   // no exception leaves a part's thread
    try {
      if (p > 0 && hipSetDevice(cp.device) != hipSuccess) {
        rcs[p] = MCTRG_EDEVICE;
        return;
      }
      for (int i = 0; i < n && rcs[p] == MCTRG_OK; ++i) rcs[p] = chain_step(*cp.parts[p]);
    } catch (...) {
      rcs[p] = MCTRG_ENOMEM;
    }
  };
  std::vector<std::thread> th;
  try {
    th.reserve(P);
  } catch (...) {
  }
  for (int p = 1; p < P; ++p) {
    try {
      th.emplace_back(run, p);
    } catch (...) {   // no thread: step this part here
      run(p);
    }
  }
  run(0);
  for (auto& t : th) t.join();
  for (int p = 0; p < P; ++p)
    if (rcs[p] != MCTRG_OK) return rcs[p];
  return parts_join(cp);
}

int parts_finish(ChainParts& cp, int8_t* out_sign, double* out_ln, double* out_lnc, double* out_tensor) {
  for (auto& c : cp.parts) {
    const int rc = chain_finish(*c, out_sign, out_ln, out_lnc, out_tensor);
    if (rc != MCTRG_OK) return rc;
  }
  return parts_join(cp);
}

// Length of the union of [begin, end) intervals.
double union_ms(std::vector<std::pair<float, float>> v) {
  std::sort(v.begin(), v.end());
  double tot = 0.0;
  bool open = false;
  float lo = 0.0f, hi = 0.0f;
  for (const auto& iv : v) {
    if (open && iv.first <= hi) {
      hi = std::max(hi, iv.second);
    } else {
      if (open) tot += hi - lo;
      lo = iv.first;
      hi = iv.second;
      open = true;
    }
  }
  if (open) tot += hi - lo;
  return tot;
}

bool is_fin(double x) { return std::isfinite(x); }

int validate_config(const mctrg_run_config* cfg) {
  if (!cfg) return MCTRG_EINVAL;
  if (cfg->n_steps < 1 || cfg->n_steps > 40) return MCTRG_EINVAL;
  if (cfg->k < 1 || cfg->k > 64) return MCTRG_EINVAL;
  if (cfg->mode < MCTRG_SHARED || cfg->mode > MCTRG_TOPK) return MCTRG_EINVAL;
  if (cfg->contract_dtype < MCTRG_F64 || cfg->contract_dtype > MCTRG_FP8_E4M3) return MCTRG_EINVAL;
  if (!is_fin(cfg->tau_null) || cfg->tau_null < 0.0 || cfg->tau_null >= 1.0) return MCTRG_EINVAL;
  if (cfg->sample_offset < 0) return MCTRG_EINVAL;
  if (cfg->mode == MCTRG_INDEPENDENT) {
    if ((cfg->n_steps % 2) != 0 || cfg->n_steps > 12) return MCTRG_EINVAL;
  }
  if (cfg->n_det < 0 || cfg->n_det > cfg->n_steps) return MCTRG_EINVAL;
  if (cfg->decomposition < MCTRG_DEC_SVD || cfg->decomposition > MCTRG_DEC_QR5) return MCTRG_EINVAL;
  if (cfg->decomposition != MCTRG_DEC_SVD && cfg->k > 32) return MCTRG_EUNSUPPORTED;
  return MCTRG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* mctrg_status_string(int status) {
  switch (status) {
    case MCTRG_OK: return "ok";
    case MCTRG_EINVAL: return "invalid argument";
    case MCTRG_ENOMEM: return "out of device memory";
    case MCTRG_EDEVICE: return "HIP device error";
    case MCTRG_ENUMERIC: return "numerical failure in some samples";
    case MCTRG_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
  }
}

void mctrg_default_config(mctrg_run_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n_steps = 8;
  cfg->k = 8;
  cfg->mode = MCTRG_SHARED;
  cfg->contract_dtype = MCTRG_F64;
  cfg->tau_null = 1e-11;
}

int32_t mctrg_capacity_dim(int32_t d0, int32_t k, int32_t n_steps) {
  if (d0 < 1 || k < 1 || n_steps < 0) return -1;
  int32_t D = d0;
  for (int s = 0; s < n_steps; ++s) D = capacity_next(D, k);
  return D;
}

int mctrg_init_tensor(int model, int32_t n_groups, const double* beta, const double* h, int32_t d_user,
                      const double* user_T, mctrg_tensor_set** out) {
  if (!out || n_groups < 1 || n_groups > (1 << 20)) return MCTRG_EINVAL;
  if (model != MCTRG_ISING_SITE && model != MCTRG_ISING_PLAQUETTE && model != MCTRG_USER) return MCTRG_EINVAL;
  int d0 = 2;
  if (model == MCTRG_USER) {
    if (!user_T || d_user < 2 || d_user > 4) return MCTRG_EINVAL;
    d0 = d_user;
    const size_t per = (size_t)d0 * d0 * d0 * d0;
    for (size_t i = 0; i < per * n_groups; ++i)
      if (!is_fin(user_T[i])) return MCTRG_EINVAL;
  } else {
    if (!beta || !h) return MCTRG_EINVAL;
    for (int g = 0; g < n_groups; ++g)
      if (!is_fin(beta[g]) || beta[g] < 0.0 || beta[g] > 50.0 || !is_fin(h[g]) || std::fabs(h[g]) > 50.0)
        return MCTRG_EINVAL;
  }
  mctrg_tensor_set* ts = new (std::nothrow) mctrg_tensor_set();
  if (!ts) return MCTRG_ENOMEM;
  ts->ngroups = n_groups;
  ts->d0 = d0;
  if (hipGetDevice(&ts->device) != hipSuccess) { delete ts; return MCTRG_EDEVICE; }
  const size_t per = (size_t)d0 * d0 * d0 * d0;
  if (hipMalloc(&ts->T0, per * n_groups * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    delete ts;
    return MCTRG_ENOMEM;
  }
  int rc = MCTRG_OK;
  if (model == MCTRG_USER) {
    if (hipMemcpy(ts->T0, user_T, per * n_groups * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      rc = MCTRG_EDEVICE;
  } else {
    double* dbh = nullptr;
    if (hipMalloc(&dbh, 2 * n_groups * sizeof(double)) != hipSuccess) {
      rc = MCTRG_ENOMEM;
    } else {
      if (hipMemcpy(dbh, beta, n_groups * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(dbh + n_groups, h, n_groups * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          launch_init_tensors(model, n_groups, dbh, dbh + n_groups, ts->T0, nullptr) != hipSuccess ||
          hipDeviceSynchronize() != hipSuccess)
        rc = MCTRG_EDEVICE;
      (void)hipFree(dbh);
    }
  }
  if (rc != MCTRG_OK) {
    (void)hipFree(ts->T0);
    delete ts;
    return rc;
  }
  *out = ts;
  return MCTRG_OK;
}

int mctrg_tensor_set_info(const mctrg_tensor_set* ts, int32_t* n_groups, int32_t* d0) {
  if (!ts) return MCTRG_EINVAL;
  if (n_groups) *n_groups = ts->ngroups;
  if (d0) *d0 = ts->d0;
  return MCTRG_OK;
}

void mctrg_destroy(mctrg_tensor_set* ts) {
  if (!ts) return;
  (void)hipFree(ts->T0);
  delete ts;
}

int mctrg_run_samples(mctrg_tensor_set* ts, const mctrg_run_config* cfg, int64_t n_samples,
                      const int32_t* group_of_sample, const int32_t* k_of_sample, int8_t* out_sign,
                      double* out_ln_abs_Z, double* out_ln_c, void* hip_stream) {
  if (!ts) return MCTRG_EINVAL;
  int rc = validate_config(cfg);
  if (rc != MCTRG_OK) return rc;
  if (n_samples < 0 || n_samples > (int64_t)1 << 31) return MCTRG_EINVAL;
  if (n_samples == 0) return MCTRG_OK;
  if (!out_sign || !out_ln_abs_Z) return MCTRG_EINVAL;
  if (group_of_sample)
    for (int64_t i = 0; i < n_samples; ++i)
      if (group_of_sample[i] < 0 || group_of_sample[i] >= ts->ngroups) return MCTRG_EINVAL;
  if (k_of_sample)
    for (int64_t i = 0; i < n_samples; ++i) {
      if (k_of_sample[i] < 1 || k_of_sample[i] > 64) return MCTRG_EINVAL;
      if (cfg->decomposition != MCTRG_DEC_SVD && k_of_sample[i] > 32) return MCTRG_EUNSUPPORTED;
    }
  const bool record = (cfg->flags & MCTRG_RECORD) != 0;
  if (record) {
    if (!cfg->record_buf) return MCTRG_EINVAL;
    if (k_of_sample)
      for (int64_t i = 0; i < n_samples; ++i)
        if (k_of_sample[i] > cfg->k) return MCTRG_EINVAL;
  }
  if (cfg->out_tensor) {
    if (cfg->mode == MCTRG_INDEPENDENT) return MCTRG_EUNSUPPORTED;
    if (k_of_sample)
      for (int64_t i = 0; i < n_samples; ++i)
        if (k_of_sample[i] != cfg->k) return MCTRG_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != ts->device) return MCTRG_EINVAL;

  // bucket samples by k
  std::vector<int> ks;
  if (k_of_sample) {
    for (int64_t i = 0; i < n_samples; ++i) ks.push_back(k_of_sample[i]);
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
  } else {
    ks.push_back(cfg->k);
  }
  bool any_fail = false;
  int64_t fail_sid = -1;   // test hook (see mctrg.h): this sample's last normalisation is made non-finite
  if (const char* e = std::getenv("MCTRG_TEST_FAIL_SAMPLE")) fail_sid = std::strtoll(e, nullptr, 10);
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return MCTRG_EDEVICE;
  double budget = 0.70 * (double)freeb;
  if (cfg->max_workspace_bytes > 0) budget = std::min(budget, (double)cfg->max_workspace_bytes);
  // every bucket's chains are sized before anything is enqueued: one sample
  // that does not fit the workspace budget gives ENOMEM with the outputs untouched
  std::vector<Chain> probes(ks.size());
  for (size_t b = 0; b < ks.size(); ++b) {
    Chain& probe = probes[b];
    probe.mode = cfg->mode; probe.dtype = cfg->contract_dtype; probe.k = ks[b]; probe.n_steps = cfg->n_steps;
    probe.Dsched = schedule(ts->d0, ks[b], cfg->n_steps);
    if (cfg->mode == MCTRG_INDEPENDENT && build_levels(probe) != MCTRG_OK) return MCTRG_EINVAL;
    probe.nsamp = 1;
    if ((double)chain_bytes(probe) > budget) return MCTRG_ENOMEM;
  }
  // Buckets of different k run concurrently (each wave of a bucket as its
  // parts on streams and host threads of its own), the workspace budget
  // shared in proportion to what each bucket would need in one wave; when a
  // share cannot hold one sample, the buckets run one after another with the
  // whole budget.
  const int parts = (cfg->flags & MCTRG_ONE_STREAM) ? 1 : kParts;
  struct Bucket {
    std::vector<int64_t> members;
    size_t per1 = 0, per_sample = 0;
    int64_t wave = 1;
  };
  std::vector<Bucket> bk(ks.size());
  double need_tot = 0.0;
  for (size_t b = 0; b < ks.size(); ++b) {
    Chain& probe = probes[b];
    for (int64_t i = 0; i < n_samples; ++i)
      if ((k_of_sample ? k_of_sample[i] : cfg->k) == ks[b]) bk[b].members.push_back(i);
    probe.nsamp = 1;
    bk[b].per1 = chain_bytes(probe);
    probe.nsamp = 2;
    bk[b].per_sample = std::max<size_t>(1, chain_bytes(probe) - bk[b].per1);
    const double fixed = std::max(0.0, (double)bk[b].per1 - (double)bk[b].per_sample);
    need_tot += parts * fixed + (double)bk[b].per_sample * bk[b].members.size();
  }
  bool together = ks.size() > 1;
  for (size_t b = 0; b < ks.size(); ++b) {
    const double fixed = std::max(0.0, (double)bk[b].per1 - (double)bk[b].per_sample);
    const double need = parts * fixed + (double)bk[b].per_sample * bk[b].members.size();
    const double share = need_tot > budget && together ? budget * need / need_tot : budget;
    if (share < (double)bk[b].per1) together = false;
    bk[b].wave = (int64_t)std::max(1.0, std::floor((share - parts * fixed) / (double)bk[b].per_sample));
    bk[b].wave = std::min<int64_t>(bk[b].wave, (int64_t)bk[b].members.size());
  }
  if (!together)   // one after another, each with the whole budget
    for (size_t b = 0; b < ks.size(); ++b) {
      const double fixed = std::max(0.0, (double)bk[b].per1 - (double)bk[b].per_sample);
      bk[b].wave = (int64_t)std::max(1.0, std::floor((budget - parts * fixed) / (double)bk[b].per_sample));
      bk[b].wave = std::min<int64_t>(bk[b].wave, (int64_t)bk[b].members.size());
    }
  // streams of the buckets after the first (which uses the caller's)
  std::vector<hipStream_t> bst(ks.size(), st);
  hipEvent_t ready = nullptr;
  int brc = MCTRG_OK;
  auto cleanup = [&]() {
    for (size_t b = 1; b < bst.size(); ++b)
      if (bst[b] != st) (void)hipStreamDestroy(bst[b]);
    if (ready) (void)hipEventDestroy(ready);
  };
  if (together) {
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return MCTRG_EDEVICE;
    for (size_t b = 1; b < ks.size(); ++b)
      if (hipStreamCreateWithFlags(&bst[b], hipStreamNonBlocking) != hipSuccess) { bst[b] = st; cleanup(); return MCTRG_EDEVICE; }
  }
  // one wave of bucket b: samples members[w0, w1)
  auto run_wave = [&](size_t b, size_t w0, ChainParts& cp) -> int {
    const int kb = ks[b];
    Chain& probe = probes[b];
    const size_t w1 = std::min(bk[b].members.size(), w0 + (size_t)bk[b].wave);
    const int64_t nw = (int64_t)(w1 - w0);
    std::vector<int32_t> groups(nw);
    std::vector<int64_t> out_index(nw), sids(nw);
    for (int64_t s = 0; s < nw; ++s) {
      const int64_t i = bk[b].members[w0 + s];
      groups[s] = group_of_sample ? group_of_sample[i] : 0;
      out_index[s] = i;
      sids[s] = cfg->sample_offset + i;
    }
    auto configure = [&](Chain& c) {
      c.mode = cfg->mode; c.dtype = cfg->contract_dtype; c.k = kb; c.n_steps = cfg->n_steps;
      c.tau = cfg->tau_null; c.seed = cfg->seed; c.flags = cfg->flags; c.record = cfg->record_buf;
      c.kmax_rec = cfg->k;
      c.n_det = cfg->n_det;
      c.dec = cfg->decomposition;
      c.Dsched = probe.Dsched;
      c.levels = probe.levels;
      c.plaqs = probe.plaqs;
      c.fail_sid = fail_sid;
    };
    int r = parts_start(cp, configure, ts, groups, out_index, sids, bst[b], (cfg->flags & MCTRG_ONE_STREAM) != 0,
                        false);
    if (r != MCTRG_OK) return r;
    r = parts_step(cp, cfg->n_steps);
    if (r != MCTRG_OK) return r;
    return parts_finish(cp, out_sign, out_ln_abs_Z, out_ln_c, cfg->out_tensor);
  };
  auto check_signs = [&](ChainParts& cp) -> int {
    for (auto& c : cp.parts) {
      std::vector<int8_t> sg(c->nsamp);
      if (hipMemcpy(sg.data(), c->sign, c->nsamp, hipMemcpyDeviceToHost) != hipSuccess) return MCTRG_EDEVICE;
      for (int8_t v : sg)
        if (v == 0) any_fail = true;
    }
    return MCTRG_OK;
  };
  if (!together) {
    for (size_t b = 0; b < ks.size() && brc == MCTRG_OK; ++b)
      for (size_t w0 = 0; w0 < bk[b].members.size() && brc == MCTRG_OK; w0 += (size_t)bk[b].wave) {
        ChainParts cp;
        brc = run_wave(b, w0, cp);
        if (brc == MCTRG_OK && hipStreamSynchronize(st) != hipSuccess) brc = MCTRG_EDEVICE;
        if (brc == MCTRG_OK) brc = check_signs(cp);
      }
    cleanup();
    if (brc != MCTRG_OK) return brc;
    return any_fail ? MCTRG_ENUMERIC : MCTRG_OK;
  }
  size_t rounds = 0;
  for (const Bucket& x : bk) rounds = std::max(rounds, (x.members.size() + x.wave - 1) / x.wave);
  for (size_t w = 0; w < rounds && brc == MCTRG_OK; ++w) {
    // the buckets' streams start after the work already queued on the caller's
    if (hipEventRecord(ready, st) != hipSuccess) { brc = MCTRG_EDEVICE; break; }
    for (size_t b = 1; b < ks.size(); ++b)
      if (hipStreamWaitEvent(bst[b], ready, 0) != hipSuccess) brc = MCTRG_EDEVICE;
    std::vector<ChainParts> cps(ks.size());
    std::vector<int> rcs(ks.size(), MCTRG_OK);
    std::vector<std::thread> th;
    auto go = [&](size_t b) {
      try {
        if (hipSetDevice(dev) != hipSuccess) { rcs[b] = MCTRG_EDEVICE; return; }
        const size_t w0 = w * (size_t)bk[b].wave;
        if (w0 < bk[b].members.size()) rcs[b] = run_wave(b, w0, cps[b]);
      } catch (...) {
        rcs[b] = MCTRG_ENOMEM;
      }
    };
    for (size_t b = 1; b < ks.size() && brc == MCTRG_OK; ++b) {
      try {
        th.emplace_back(go, b);
      } catch (...) {
        go(b);
      }
    }
    if (brc == MCTRG_OK) go(0);
    for (auto& t : th) t.join();
    for (size_t b = 0; b < ks.size(); ++b)
      if (rcs[b] != MCTRG_OK && brc == MCTRG_OK) brc = rcs[b];
    // the caller's stream waits for every bucket
    for (size_t b = 1; b < ks.size() && brc == MCTRG_OK; ++b) {
      if (hipEventRecord(ready, bst[b]) != hipSuccess || hipStreamWaitEvent(st, ready, 0) != hipSuccess)
        brc = MCTRG_EDEVICE;
    }
    if (brc == MCTRG_OK && hipStreamSynchronize(st) != hipSuccess) brc = MCTRG_EDEVICE;
    for (size_t b = 0; b < ks.size() && brc == MCTRG_OK; ++b)
      if (!cps[b].parts.empty()) brc = check_signs(cps[b]);
  }
  cleanup();
  if (brc != MCTRG_OK) return brc;
  return any_fail ? MCTRG_ENUMERIC : MCTRG_OK;
}

struct mctrg_chain {
  ChainParts cp;
  int n_steps = 0, steps = 0;
};

int mctrg_chain_create(mctrg_tensor_set* ts, const mctrg_run_config* cfg, int64_t n_samples,
                       const int32_t* group_of_sample, void* hip_stream, mctrg_chain** out) {
  if (!ts || !out) return MCTRG_EINVAL;
  int rc = validate_config(cfg);
  if (rc != MCTRG_OK) return rc;
  if (n_samples < 1 || n_samples > (int64_t)1 << 31) return MCTRG_EINVAL;
  if (group_of_sample)
    for (int64_t i = 0; i < n_samples; ++i)
      if (group_of_sample[i] < 0 || group_of_sample[i] >= ts->ngroups) return MCTRG_EINVAL;
  if ((cfg->flags & MCTRG_RECORD) && !cfg->record_buf) return MCTRG_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != ts->device) return MCTRG_EINVAL;
  Chain probe;
  probe.mode = cfg->mode; probe.n_steps = cfg->n_steps;
  probe.Dsched = schedule(ts->d0, cfg->k, cfg->n_steps);
  if (probe.mode == MCTRG_INDEPENDENT && build_levels(probe) != MCTRG_OK) return MCTRG_EINVAL;
  mctrg_chain* ch = new (std::nothrow) mctrg_chain();
  if (!ch) return MCTRG_ENOMEM;
  ch->n_steps = cfg->n_steps;
  std::vector<int32_t> groups(n_samples);
  std::vector<int64_t> out_index(n_samples), sids(n_samples);
  for (int64_t i = 0; i < n_samples; ++i) {
    groups[i] = group_of_sample ? group_of_sample[i] : 0;
    out_index[i] = i;
    sids[i] = cfg->sample_offset + i;
  }
  int64_t fail_sid = -1;   // test hook (see mctrg.h), as in run_samples
  if (const char* e = std::getenv("MCTRG_TEST_FAIL_SAMPLE")) fail_sid = std::strtoll(e, nullptr, 10);
  auto configure = [&](Chain& c) {
    c.mode = cfg->mode; c.dtype = cfg->contract_dtype; c.k = cfg->k; c.n_steps = cfg->n_steps;
    c.tau = cfg->tau_null; c.seed = cfg->seed; c.flags = cfg->flags & (MCTRG_PROFILE | MCTRG_RECORD);
    c.record = (cfg->flags & MCTRG_RECORD) ? cfg->record_buf : nullptr;
    c.kmax_rec = cfg->k;
    c.n_det = cfg->n_det;
    c.dec = cfg->decomposition;
    c.fail_sid = fail_sid;
    c.Dsched = probe.Dsched;
    c.levels = probe.levels;
    c.plaqs = probe.plaqs;
  };
  rc = parts_start(ch->cp, configure, ts, groups, out_index, sids, reinterpret_cast<hipStream_t>(hip_stream),
                   (cfg->flags & MCTRG_ONE_STREAM) != 0, (cfg->flags & MCTRG_PROFILE) != 0);
  if (rc != MCTRG_OK) { delete ch; return rc; }
  *out = ch;
  return MCTRG_OK;
}

int mctrg_chain_step(mctrg_chain* ch, int32_t n) {
  if (!ch || n < 0 || ch->steps + n > ch->n_steps) return MCTRG_EINVAL;
  const int rc = parts_step(ch->cp, n);
  if (rc != MCTRG_OK) return rc;
  ch->steps += n;
  return MCTRG_OK;
}

int mctrg_chain_finish(mctrg_chain* ch, int8_t* out_sign, double* out_ln_abs_Z, double* out_ln_c) {
  if (!ch || !out_sign || !out_ln_abs_Z) return MCTRG_EINVAL;
  const int rc = parts_finish(ch->cp, out_sign, out_ln_abs_Z, out_ln_c, nullptr);
  if (rc != MCTRG_OK) return rc;
  if (hipStreamSynchronize(ch->cp.caller) != hipSuccess) return MCTRG_EDEVICE;
  // a failed sample (sign 0) makes the call return ENUMERIC, as run_samples
  int64_t n = 0;
  for (const auto& c : ch->cp.parts) n += c->nsamp;
  std::vector<int8_t> sg((size_t)n);
  if (n > 0 && hipMemcpy(sg.data(), out_sign, (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) return MCTRG_EDEVICE;
  for (int8_t v : sg)
    if (v == 0) return MCTRG_ENUMERIC;
  return MCTRG_OK;
}

int mctrg_chain_tensor(const mctrg_chain* ch, double* out) {
  if (!ch || !out || ch->cp.parts.empty()) return MCTRG_EINVAL;
  if (ch->cp.parts[0]->mode == MCTRG_INDEPENDENT) return MCTRG_EUNSUPPORTED;
  size_t off = 0;
  for (const auto& c : ch->cp.parts) {
    const size_t D = (size_t)c->Dsched[c->step], per = D * D * D * D;
    CKH(hipMemcpyAsync(out + off, c->Ta, (size_t)c->nsamp * per * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    off += (size_t)c->nsamp * per;
  }
  const int rc = parts_join(const_cast<ChainParts&>(ch->cp));
  if (rc != MCTRG_OK) return rc;
  CKH(hipStreamSynchronize(ch->cp.caller));
  return MCTRG_OK;
}

int mctrg_chain_get_profile(const mctrg_chain* ch, mctrg_chain_profile* out) {
  if (!ch || !out) return MCTRG_EINVAL;
  std::memset(out, 0, sizeof(*out));
  std::vector<std::pair<float, float>> js, gs, qs;
  for (const auto& c : ch->cp.parts) {
    out->jacobi_ms += c->tj.ms;
    out->jacobi_launches += c->tj.launches;
    out->gemm_ms += c->tg.ms;
    out->gemm_launches += c->tg.launches;
    out->qr128_ms += c->tq.ms;
    out->qr128_launches += c->tq.launches;
    out->qr128_flops += c->tq_flops;
    out->jacobi_rotated_pairs += c->rotated_pairs;
    out->jacobi_flops += c->jacobi_flops;
    out->last_sweeps = std::max(out->last_sweeps, c->last_sweeps);
    for (int s = 0; s < 64; ++s) out->step_sweeps[s] = std::max(out->step_sweeps[s], c->step_sweeps[s]);
    for (int s = 0; s < 64; ++s) {
      const bool in = s < c->last_sweeps && s < kMaxSweeps;
      out->last_pairs[s] += in ? c->sweep_hist[2 * s] : 0;
      out->last_active[s] += in ? c->sweep_hist[2 * s + 1] : 0;
    }
    js.insert(js.end(), c->tj.spans.begin(), c->tj.spans.end());
    gs.insert(gs.end(), c->tg.spans.begin(), c->tg.spans.end());
    qs.insert(qs.end(), c->tq.spans.begin(), c->tq.spans.end());
  }
  out->steps_done = ch->steps;
  out->jacobi_busy_ms = union_ms(std::move(js));
  out->gemm_busy_ms = union_ms(std::move(gs));
  out->qr128_busy_ms = union_ms(std::move(qs));
  out->parts = (int32_t)ch->cp.parts.size();
  return MCTRG_OK;
}

void mctrg_chain_destroy(mctrg_chain* ch) { delete ch; }

int mctrg_estimate_lnZ(int64_t n_samples, const int8_t* sign, const double* ln_abs_Z, double n_sites,
                       mctrg_estimate* out, void* hip_stream) {
  if (n_samples < 1 || !sign || !ln_abs_Z || !out || !(n_sites > 0.0) || !is_fin(n_sites)) return MCTRG_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  double* d = nullptr;
  if (hipMalloc(&d, 8 * sizeof(double)) != hipSuccess) return MCTRG_ENOMEM;
  double h[8];
  int rc = MCTRG_OK;
  if (launch_estimate(n_samples, sign, ln_abs_Z, n_sites, d, st) != hipSuccess ||
      hipMemcpyAsync(h, d, 8 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    rc = MCTRG_EDEVICE;
  (void)hipFree(d);
  if (rc != MCTRG_OK) return rc;
  out->ln_meanZ_per_site = h[0];
  out->rel_stderr_Z = h[1];
  out->mean_lnZ_per_site = h[2];
  out->stderr_mean_lnZ = h[3];
  out->n_used = (int64_t)h[4];
  out->n_negative = (int64_t)h[5];
  out->n_failed = (int64_t)h[6];
  return MCTRG_OK;
}

// ---- step-level entry points ----------------------------------------------

int mctrg_svd_batched(int64_t n_mats, int32_t d1, int32_t d2, const double* M, double tau_null, double* sigma_out,
                      double* V_out, int32_t* sweeps_out, void* hip_stream) {
  if (n_mats < 0 || d1 < 1 || d2 < 1 || (int64_t)d1 * d2 > 4096) return MCTRG_EINVAL;
  if (!(tau_null >= 0.0 && tau_null < 1.0)) return MCTRG_EINVAL;
  if (n_mats == 0) return MCTRG_OK;
  if (!M || !sigma_out) return MCTRG_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int n = d1 * d2, n_pad = std::max(32, round_up32(n));
  const size_t per = (size_t)n_pad * n_pad;
  const int64_t nm = n_mats;
  // the chains' buffers at one step's shape, the right vectors' scratch after them
  DecompBufs b{};
  double *X = nullptr, *wgt = nullptr;
  int32_t *ss = nullptr, *kept = nullptr, *sel = nullptr;
  auto lay = [&](Arena& ar) {
    b.S = ar.take<double>(nm * per);
    b.W = ar.take<double>(nm * per);
    b.W2 = ar.take<double>(nm * per);
    b.W3 = ar.take<double>(nm * per);
    b.W4 = ar.take<double>(n_pad <= 1024 ? nm * per : 0);
    b.Tscr = ar.take<double>((size_t)nm * kQrTscr);
    b.Tws = ar.take<double>((size_t)nm * 32 * 1024);
    b.Tws2 = ar.take<double>((size_t)nm * 32 * 1024);
    b.colnorm = ar.take<double>((size_t)nm * n_pad);
    b.dnrm = ar.take<double>((size_t)nm * n_pad);
    b.sigma = sigma_out;
    b.perm = ar.take<int32_t>((size_t)nm * n_pad);
    b.colmap = ar.take<int32_t>((size_t)nm * n_pad);
    b.dpos = ar.take<int32_t>((size_t)nm * n_pad);
    b.order = ar.take<int32_t>((size_t)nm * n);
    b.nb_job = ar.take<int>(nm);
    b.three_job = ar.take<int>(nm);
    b.nb_first = ar.take<int>(nm);
    b.jw.active = ar.take<int>(nm);
    b.jw.rotated = ar.take<int>(nm);
    b.jw.sweeps = ar.take<int>(nm);
    b.jw.counter = ar.take<int>(2 * kMaxSweeps);
    b.jw.lastmod = ar.take<int>((size_t)nm * kJacobiMaxBlocks);
    b.jw.lastchk = ar.take<int>((size_t)nm * kJacobiMaxBlocks * kJacobiMaxBlocks);
    b.jw.hist_len = kMaxSweeps;
    ss = ar.take<int32_t>(2 * nm);
    if (V_out) {
      X = ar.take<double>((size_t)nm * n * n);
      wgt = ar.take<double>((size_t)nm * n);
      kept = ar.take<int32_t>(nm);
      sel = ar.take<int32_t>((size_t)nm * n);
    }
  };
  Arena ar;
  lay(ar);
  char* mem = nullptr;
  if (hipMalloc(&mem, ar.off) != hipSuccess) { (void)hipGetLastError(); return MCTRG_ENOMEM; }
  HostPinned pin;
  if (hipHostMalloc(&pin.p, 2 * kMaxSweeps * sizeof(int) + 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(mem);
    return MCTRG_ENOMEM;
  }
  Arena a2;
  a2.base = mem;
  a2.counting = false;
  lay(a2);
  b.jw.counter_host = reinterpret_cast<int*>(pin.p);
  // every matrix is its own source, read as a plain row-major n x n matrix (split 2)
  std::vector<int32_t> hs(2 * nm);
  for (int64_t i = 0; i < nm; ++i) { hs[i] = (int32_t)i; hs[nm + i] = 2; }
  int rc = MCTRG_OK;
  if (hipMemcpyAsync(ss, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
    rc = MCTRG_EDEVICE;
  DecompOut out;
  if (rc == MCTRG_OK) {
    DecompCtl ctl;
    ctl.tau = tau_null;
    if (decompose(nm, n, 1, n_pad, M, ss, ss + nm, b, ctl, out, st) != hipSuccess) rc = MCTRG_EDEVICE;
  }
  if (rc == MCTRG_OK && V_out) {
    // v = P Q2 (Q4) y for every positive value, the rows of zero values zero
    const bool five = out.qr5 && !out.three;
    hipError_t e = launch_select_all(nm, n, sigma_out, kept, sel, wgt, st);
    if (e == hipSuccess)
      e = launch_apply_q1(nm, n, n_pad, n, b.W, nullptr, b.Tws2, five ? b.S : nullptr, five ? b.Tws : nullptr, out.Wj,
                          sigma_out, b.order, kept, sel, wgt, X, st, out.nob);
    if (e == hipSuccess) e = launch_scatter_V(nm, n, d2, n_pad, X, b.perm, out.qr5 ? b.colmap : nullptr, kept, V_out, st);
    if (e != hipSuccess) rc = MCTRG_EDEVICE;
  }
  if (rc == MCTRG_OK && sweeps_out &&
      hipMemcpyAsync(sweeps_out, b.jw.sweeps, nm * sizeof(int32_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
    rc = MCTRG_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) rc = MCTRG_EDEVICE;
  (void)hipFree(mem);
  return rc;
}

int mctrg_sample_batched(int64_t n_jobs, int32_t n, int32_t k, int32_t mode, uint64_t seed, double tau_null,
                         const double* sigma, const uint64_t* rng, const int32_t* split, int32_t* kept,
                         int32_t* cand, int32_t* sel, double* log_r, double* weight, void* hip_stream) {
  if (n_jobs < 0 || n < 1 || n > 4096 || k < 1 || k > 64 || mode < 0 || mode > MCTRG_TOPK) return MCTRG_EINVAL;
  if (!is_fin(tau_null) || tau_null < 0 || tau_null >= 1) return MCTRG_EINVAL;
  if (n_jobs == 0) return MCTRG_OK;
  if (!sigma || !rng || !split || !kept || !cand || !sel || !log_r || !weight) return MCTRG_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  double* scr = nullptr;
  if (hipMalloc(&scr, sample_scratch_doubles(n_jobs, n, k) * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return MCTRG_ENOMEM;
  }
  SampleArgs sa{};
  sa.njobs = n_jobs; sa.n = n; sa.k = k; sa.mode = mode; sa.seed = seed; sa.tau = tau_null; sa.sigma = sigma;
  sa.rng = rng; sa.split = split; sa.kept = kept; sa.cand = cand; sa.sel = sel; sa.log_r = log_r;
  sa.weight = weight; sa.scratch = scr;
  int rc = MCTRG_OK;
  if (launch_sample(sa, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = MCTRG_EDEVICE;
  (void)hipFree(scr);
  return rc;
}

int mctrg_sample_batched_noalloc(int64_t n_jobs, int32_t n, int32_t k, int32_t mode, uint64_t seed, double tau_null,
                                 const double* sigma, const uint64_t* rng, const int32_t* split, int32_t* kept,
                                 int32_t* cand, int32_t* sel, double* log_r, double* weight, void* hip_stream) {
  if (n_jobs < 0 || n < 1 || n > 4096 || k < 1 || k > 64 || mode < 0 || mode > MCTRG_TOPK) return MCTRG_EINVAL;
  if (!is_fin(tau_null) || tau_null < 0 || tau_null >= 1) return MCTRG_EINVAL;
  if (n_jobs == 0) return MCTRG_OK;
  if (!sigma || !rng || !split || !kept || !cand || !sel || !log_r || !weight) return MCTRG_EINVAL;
  if (sample_scratch_doubles(n_jobs, n, k) > noalloc_scratch_doubles()) return MCTRG_ENOMEM;
  double* scr = nullptr;
  if (noalloc_scratch(&scr) != hipSuccess) return MCTRG_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  SampleArgs sa{};
  sa.njobs = n_jobs; sa.n = n; sa.k = k; sa.mode = mode; sa.seed = seed; sa.tau = tau_null; sa.sigma = sigma;
  sa.rng = rng; sa.split = split; sa.kept = kept; sa.cand = cand; sa.sel = sel; sa.log_r = log_r;
  sa.weight = weight; sa.scratch = scr;
  if (launch_sample(sa, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return MCTRG_EDEVICE;
  return MCTRG_OK;
}

int mctrg_contract_batched(int64_t n_jobs, int32_t D, int32_t kk, int32_t dtype, const double* GA,
                           const double* GB, const double* FA, const double* FB, double* T_out, void* hip_stream) {
  if (n_jobs < 0 || D < 1 || D > 64 || kk < 1 || kk > 64 || dtype < MCTRG_F64 || dtype > MCTRG_FP8_E4M3)
    return MCTRG_EINVAL;
  if (n_jobs == 0) return MCTRG_OK;
  if (!GA || !GB || !FA || !FB || !T_out) return MCTRG_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t xe = (size_t)n_jobs * kk * kk * D * D, te = (size_t)n_jobs * kk * kk * kk * kk;
  const size_t fe = (size_t)n_jobs * D * D * kk;   // each F pool, by kept index
  Arena ar;
  ar.take<double>(xe); ar.take<double>(xe); ar.take<float>(xe); ar.take<float>(xe);
  ar.take<double>(2 * n_jobs); ar.take<double>(te); ar.take<int32_t>(4 * n_jobs);
  ar.take<double>(fe); ar.take<double>(fe);
  char* mem = nullptr;
  if (hipMalloc(&mem, ar.off) != hipSuccess) { (void)hipGetLastError(); return MCTRG_ENOMEM; }
  Arena a2;
  a2.base = mem; a2.counting = false;
  ContractArgs ca{};
  ca.X = a2.take<double>(xe); ca.Y = a2.take<double>(xe); ca.Xlp = a2.take<float>(xe); ca.Ylp = a2.take<float>(xe);
  ca.scales = a2.take<double>(2 * n_jobs);
  double* C = a2.take<double>(te);
  int32_t* jobs = a2.take<int32_t>(4 * n_jobs);
  double* FAk = a2.take<double>(fe);
  double* FBk = a2.take<double>(fe);
  std::vector<int32_t> hj(4 * n_jobs);
  for (int64_t o = 0; o < n_jobs; ++o)
    for (int t = 0; t < 4; ++t) hj[4 * o + t] = (int32_t)o;
  ca.nout = n_jobs; ca.D = D; ca.kk = kk; ca.dtype = dtype;
  ca.GA = GA; ca.GB = GB; ca.FA = FAk; ca.FB = FBk;
  ca.g_stride = (int64_t)kk * D * D; ca.f_stride = (int64_t)D * D * kk;
  ca.jobs = jobs; ca.Tout = C;
  int rc = MCTRG_OK;
  if (hipMemcpyAsync(jobs, hj.data(), hj.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess ||
      launch_f_by_kept(n_jobs, D, kk, FA, FAk, st) != hipSuccess ||
      launch_f_by_kept(n_jobs, D, kk, FB, FBk, st) != hipSuccess || launch_contract(ca, st) != hipSuccess ||
      launch_unscale(n_jobs, (int64_t)kk * kk * kk * kk, dtype != MCTRG_F64, C, ca.scales, T_out, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    rc = MCTRG_EDEVICE;
  (void)hipFree(mem);
  return rc;
}

}  // extern "C"
