// Kernels of the boundary sweep (paper Sec. 4) for a batch of networks.
//
// Gauge and truncation.  Every site tensor T_s is stored with sqrt(lambda_b)
// absorbed on each of its bond legs (both ends of a bond carry one factor),
// so the contraction of all T_s is the represented value and no tensor ever
// holds 1/lambda.  A gate sum_k OA_k (x) OB_k on the bond b between A and B is
// absorbed with the simple-update environment (the lambdas of the other legs):
//   G_A   = sum_o lambda_other(o) T_A[o,:]^T T_A[o,:]      (Gram, (p,b) x (p,b))
//   Z_A   = sum_{p,q} (OA_k^T OA_k')[p,q] G_A[(p,b),(q,b')] (the Gram of the
//           gated A-side block X_A[(o,p'),(k,b)] = (OA_k N_A)[o,p',b])
//   F_A   pivoted Cholesky factor, F_A^T F_A = Z_A; same for B
//   C     = F_A F_B^T, whose singular values are those of the gated two-site
//           block Omega = X_A X_B^T; one-sided Jacobi gives C = U' S V'^T
//   D'    rank rule; lambda' = S[:D'] / S_1; log S_1 to the scale accumulator
//   T_A'  = T_A W_A with W_A[(p,b),(p',m)] = sum_k OA_k[p',p] Phi_A[(k,b),m],
//           Phi_A = F_B^T V'[:, m] sqrt(lambda'_m) / S_m (and Phi_B from F_A,
//           U'), i.e. the left singular vectors of Omega expressed through
//           X_A itself, so no pseudo-inverse and no division by lambda occurs.
// This is the simple-update truncation of the paper (Sec. 4) evaluated through
// Gram matrices; it equals the QR form used by the CPU oracle in exact
// arithmetic.
#include "linalg.h"
#include "sweep.h"

namespace tn3d {
namespace {

constexpr int NT = 256;
constexpr int ET = 64;  // one-site ops, rescaling, final vectors: one wavefront per (site, sweep)
constexpr int SNT = 64;       // one wavefront per bond truncation of order 9 to 16
constexpr int SNT_BIG = 256;  // four wavefronts per bond truncation of order above 16
constexpr int TR = 32;     // rows per tile in the Gram / reabsorption kernels
constexpr int MAXCHI = 64;
constexpr uint32_t WHT_NEG = 1u << 30;  // per-sweep flag: the signed network's value is negative

template <typename T>
__device__ __forceinline__ T* tens(const SweepArgs& A, int par, int sweep, int site) {
  T* b = static_cast<T*>(par ? A.buf1 : A.buf0);
  return b + int64_t(sweep) * A.sweep_stride + A.site_off[site];
}

__device__ __forceinline__ void site_dims(const SweepArgs& A, int sweep, int site, int D[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    int b = A.leg_bond[site * 4 + l];
    D[l] = b >= 0 ? A.bond_dim[int64_t(sweep) * A.n_bonds + b] : 1;
  }
}

__device__ __forceinline__ int synd_bit(const SweepArgs& A, int sweep, int det) {
  int item = A.items[sweep / A.n_cosets];
  return A.synd[A.synd_off[item] + det] & 1;
}

// The op matrices and initial tensors a sweep reads: one pool, or with psel
// one of several copies of equal layout (the same network at other rates).
__device__ __forceinline__ const double* pool_of(const SweepArgs& A, int sweep) {
  return A.psel ? A.pool + int64_t(A.psel[A.items[sweep / A.n_cosets]]) * A.pool_stride : A.pool;
}

// A gate whose terms depend on a per-item bit uses its second term set when
// the bit is set.
__device__ __forceinline__ bool gate_alt(const SweepArgs& A, const DevGate& g, int sweep) {
  return g.det >= 0 && synd_bit(A, sweep, g.det);
}

__device__ double block_max_abs_reduce(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < int(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
    red[0] = m;
  }
  __syncthreads();
  double r = red[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// initial state
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_init_sites(SweepArgs A, const int32_t* init_dims, const int32_t* init_off) {
  const int site = blockIdx.x, sweep = blockIdx.y;
  const int c = sweep % A.n_cosets;
  const int32_t* dm = init_dims + (int64_t(c) * A.n_sites + site) * 5;
  const int n = dm[0] * dm[1] * dm[2] * dm[3] * dm[4];
  const double* src = pool_of(A, sweep) + init_off[c * A.n_sites + site];
  T* dst = tens<T>(A, 0, sweep, site);
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = T(src[i]);
}

__global__ void k_init_bonds(SweepArgs A, const int32_t* bond_dim0) {
  const int sweep = blockIdx.x;
  for (int b = threadIdx.x; b < A.n_bonds; b += blockDim.x) {
    const int64_t bi = int64_t(sweep) * A.n_bonds + b;
    A.bond_dim[bi] = bond_dim0[b];
    A.logb[bi] = 0.0;
    for (int k = 0; k < A.lam_ld; ++k) A.lam[bi * A.lam_ld + k] = 1.0;
  }
  for (int s = threadIdx.x; s < A.n_sites; s += blockDim.x) A.logs[int64_t(sweep) * A.n_sites + s] = 0.0;
  if (threadIdx.x == 0) A.flags[sweep] = 0u;
}

// ---------------------------------------------------------------------------
// one-site ops: T'[r, p'] = sum_p M[p', p] T[r, p]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(ET) void k_onesite(SweepArgs A, const DevOneSite* ops) {
  const DevOneSite op = ops[blockIdx.x];
  const int sweep = blockIdx.y;
  __shared__ double M[256];
  const int bit = op.det >= 0 ? synd_bit(A, sweep, op.det) : 0;
  const double* src = pool_of(A, sweep) + (bit ? op.m1 : op.m0);
  for (int i = threadIdx.x; i < op.din * op.dout; i += blockDim.x) M[i] = src[i];
  __syncthreads();
  int D[4];
  site_dims(A, sweep, op.site, D);
  const int rows = D[0] * D[1] * D[2] * D[3];  // at most legcap^4 * d elements: 32-bit
  const T* in = tens<T>(A, op.src, sweep, op.site);
  T* out = tens<T>(A, op.src ^ 1, sweep, op.site);
  const int din = op.din, dout = op.dout;
  if (din <= 4) {
    // RU rows per lane and step, all their loads issued before any is used
    // (rows past the end read row 0 and are not written); four inputs per row
    // keep the registers, and with them the occupancy, low
    constexpr int RU = 4;
    for (int r0 = threadIdx.x; r0 < rows; r0 += RU * ET) {
      T v[RU][4];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = r0 + u * ET < rows ? r0 + u * ET : 0;
#pragma unroll
        for (int p = 0; p < 4; ++p)
          if (p < din) v[u][p] = in[r * din + p];
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int r = r0 + u * ET;
        if (r < rows)
          for (int q = 0; q < dout; ++q) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 4; ++p)
              if (p < din) s += M[q * din + p] * double(v[u][p]);
            out[r * dout + q] = T(s);
          }
      }
    }
  } else {
    for (int r = threadIdx.x; r < rows; r += ET) {
      double v[16];  // din <= 16 (checked when the network is built)
      for (int p = 0; p < din; ++p) v[p] = double(in[r * din + p]);
      for (int q = 0; q < dout; ++q) {
        double s = 0.0;
        for (int p = 0; p < din; ++p) s += M[q * din + p] * v[p];
        out[r * dout + q] = T(s);
      }
    }
  }
}

// Site tensors are stored [w][e][n][s][p].  For the bond on leg `leg` the
// element (a, x, c, p) sits at ((a * Dx + x) * Cp + c) * d + p, a running over
// the legs before `leg`, c over the legs after it.

// ---------------------------------------------------------------------------
// Gram of one side of each gated bond, FP64 accumulation
// ---------------------------------------------------------------------------
// Element offsets of the (legs before, gated leg, legs after, physical) view of
// a site tensor: row r = (a, c) starts at (a * Dx * Cp + c) * d and column
// col = p * Dx + x sits at x * Cp * d + p from there.  Rows are split once per
// tile and columns once per workgroup, so the element loops use no division.
struct Split {
  int Dx, Cp, d, rows;
};

__device__ __forceinline__ Split make_split(const int D[4], int leg, int d) {
  Split v;
  v.Dx = D[leg];
  v.d = d;
  int apre = 1;
  v.Cp = 1;
  for (int l = 0; l < leg; ++l) apre *= D[l];
  for (int l = leg + 1; l < 4; ++l) v.Cp *= D[l];
  v.rows = apre * v.Cp;
  return v;
}

// A workgroup's start and end in the execution window of its launch (slot by
// workgroup so that few atomics share an address).  The start is read at entry
// and recorded together with the end, so the workgroup never waits for the
// clock read on its way.  win_close must be reached by every thread.
__device__ __forceinline__ int win_slot() { return (blockIdx.x + 7 * blockIdx.y) & 63; }
__device__ __forceinline__ unsigned long long win_open(const unsigned long long* win) {
  return win ? (unsigned long long)wall_clock64() : 0ull;
}
__device__ __forceinline__ void win_close(unsigned long long* win, unsigned long long t0) {
  if (!win) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMin(win + win_slot(), t0);
    atomicMax(win + 64 + win_slot(), (unsigned long long)wall_clock64());
  }
}

// One wavefront per (gate side, sweep): G = X^T X for the row-weighted view X
// (rows x ncols) of the site tensor (each row scaled by the product of
// sqrt(lambda) over the three other legs, the simple-update environment), on
// the FP64 matrix cores for every storage type.  Each chunk of 32 rows is
// fetched in memory order (consecutive lanes read consecutive addresses:
// along the rows when the legs after the gated one hold more than one index,
// Cp > 1, else along the columns), scaled by the rows' weights and stored
// column-major in LDS; the next chunk's values are fetched into registers
// while the current one is multiplied.  Lane (li, lq) = (lane % 16, lane / 16)
// takes X[r][16 b + li] for the four rows r = 4 s + lq of a step and every
// 16-column block b, and one v_mfma_f64_16x16x4f64 per block pair b1 <= b2
// accumulates X_b1^T X_b2 (the A and B operands are the same values).  FP32
// storage is multiplied as FP64: a Gram accumulated in FP32 (as a split-BF16
// product would be) carries FP32 rounding into its small eigenvalues, the
// squares of the small singular values the reduced rank rule keeps.  The
// launch handles the Grams with ncols in (nlo, 16 NB].
constexpr int GR = 32;  // rows per chunk

// Up to 64 columns the kernel is held to two wavefronts per SIMD (at its
// natural 272 registers one would fit); the 96-column variant would spill.
template <typename T, int NB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NB <= 4 ? 2 : 1))) void k_gram2(
    SweepArgs A, const DevGate* gates, int n_g, double* gout, int ncap,
                                              int nlo) {
  constexpr int NC = 16 * NB;
  constexpr int NL = GR * NC / 64;  // elements each lane fetches per chunk
  const int gi = blockIdx.x >> 1, side = blockIdx.x & 1, sweep = blockIdx.y, lane = threadIdx.x;
  const DevGate g = gates[gi];
  const int site = side ? g.sb : g.sa, leg = side ? g.lb : g.la;
  const int d = side ? g.dB : g.dA, par = side ? g.srcB : g.srcA;
  int D[4];
  site_dims(A, sweep, site, D);
  const Split v = make_split(D, leg, d);
  const int ncols = d * v.Dx;
  if (ncols <= nlo || ncols > NC) return;
  const unsigned long long w0 = win_open(A.win);
  __shared__ double slam[4][MAXCHI];
  __shared__ int rowbase[2][GR];
  __shared__ double rowsc[2][GR];
  __shared__ T Xs[NC * (GR + 1)];  // column-major, stride GR + 1
  for (int e = lane; e < 4 * MAXCHI; e += 64) {
    const int lg = e / MAXCHI, k = e % MAXCHI;
    const int b = A.leg_bond[site * 4 + lg];
    double val = 1.0;
    if (lg != leg && b >= 0 && k < D[lg]) val = sqrt(A.lam[(int64_t(sweep) * A.n_bonds + b) * A.lam_ld + k]);
    slam[lg][k] = val;
  }
  // memory-order column mc = x d + p: offset x Cp d + p in a row, Gram column p Dx + x
  __shared__ int coff[NC], ccan[NC];
  for (int mc = lane; mc < NC; mc += 64) {
    const int x = mc / d, p = mc - x * d;
    coff[mc] = mc < ncols ? x * v.Cp * d + p : -1;
    ccan[mc] = p * v.Dx + x;
  }
  for (int e = lane; e < NC * (GR + 1); e += 64) Xs[e] = T(0);
  __syncthreads();
  const bool rowfast = v.Cp > 1;
  const T* t = tens<T>(A, par, sweep, site);
  // row offsets and weights of a chunk, one lane per row, into buffer q
  auto rows_of = [&](int r0, int q) {
    if (lane < GR) {
      const int r = r0 + lane;
      int base = 0;
      double sc = 0.0;
      if (r < v.rows) {
        const int a = r / v.Cp, c = r - a * v.Cp;
        base = (a * v.Dx * v.Cp + c) * d;
        sc = 1.0;
        int cc = c;
        for (int lg = 3; lg > leg; --lg) {
          const int qq = cc / D[lg];
          sc *= slam[lg][cc - qq * D[lg]];
          cc = qq;
        }
        int aa = a;
        for (int lg = leg - 1; lg >= 0; --lg) {
          const int qq = aa / D[lg];
          sc *= slam[lg][aa - qq * D[lg]];
          aa = qq;
        }
      }
      rowbase[q][lane] = base;
      rowsc[q][lane] = sc;
    }
  };
  constexpr int NP = NB * (NB + 1) / 2;
  dbl4 acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  // element j of a lane's fetch: local row and memory-order column; the next
  // chunk's values are fetched into registers while the current one is used
  T reg[NL];
  auto fetch = [&](int r0, int q) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = lane + 64 * j;
      const int rl = rowfast ? e % GR : e / NC, mc = rowfast ? e / GR : e % NC;
      const int co = coff[mc];
      reg[j] = (co >= 0 && r0 + rl < v.rows) ? t[rowbase[q][rl] + co] : T(0);
    }
  };
  auto store = [&](int q) {
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = lane + 64 * j;
      const int rl = rowfast ? e % GR : e / NC, mc = rowfast ? e / GR : e % NC;
      if (coff[mc] >= 0) Xs[ccan[mc] * (GR + 1) + rl] = T(double(reg[j]) * rowsc[q][rl]);
    }
  };
  rows_of(0, 0);
  __syncthreads();
  fetch(0, 0);
  int q = 0;
  for (int r0 = 0; r0 < v.rows; r0 += GR, q ^= 1) {
    store(q);
    if (r0 + GR < v.rows) rows_of(r0 + GR, q ^ 1);
    __syncthreads();
    if (r0 + GR < v.rows) fetch(r0 + GR, q ^ 1);
    const int li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int s4 = 0; s4 < GR / 4; ++s4) {
      double xv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) xv[b] = double(Xs[(16 * b + li) * (GR + 1) + 4 * s4 + lq]);
      int k = 0;
#pragma unroll
      for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
        for (int b2 = b1; b2 < NB; ++b2) {
          acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[b1], xv[b2], acc[k], 0, 0, 0);
          ++k;
        }
    }
    __syncthreads();  // this chunk's tile is read before the next one replaces it
  }
  if (A.bytes_ctr && lane == 0)
    atomicAdd(A.bytes_ctr + ((blockIdx.x + 7 * blockIdx.y) & 63),
              (unsigned long long)(int64_t(v.rows) * ncols * int64_t(sizeof(T))));
  if (side == 0 && lane == 0) A.gate_n[int64_t(sweep) * n_g + gi] = g.K * v.Dx;
  double* out = gout + (int64_t(sweep * n_g + gi) * 2 + side) * ncap * ncap;
  const int li = lane & 15, lq = lane >> 4;
  int k = 0;
#pragma unroll
  for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
    for (int b2 = b1; b2 < NB; ++b2) {
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        // FP64 16x16x4: item r of lane j + 16 q is C[q + 4 r][j]
        const int i = 16 * b1 + lq + 4 * it, j = 16 * b2 + li;
        if (i < ncols && j < ncols) {
          out[i * ncols + j] = acc[k][it];
          if (b1 != b2) out[j * ncols + i] = acc[k][it];
        }
      }
      ++k;
    }
  win_close(A.win, w0);
}

// FP64 route: the triangular factor R (R^T R = X^T X) of the same row-weighted
// view X as k_gram2, by Householder QR streamed over the rows (tsqr_block), so
// no Gram matrix is formed and the small singular values of X keep the
// accuracy of an orthogonal factorisation (a Gram squares their condition).
// One wavefront per (gate side, sweep), split into 64 / TL teams of TL lanes
// (ncols <= TL, lane l of a team owns column l): team t factors rows
// t TL .. t TL + TL - 1 of every chunk of 64 rows into a factor of its own,
// then team 0 absorbs the other teams' factors (a two-level TSQR tree).  R is
// written where k_gram2 writes the Gram (row-major, ncols x ncols).
template <typename T, int TL>
__global__ __launch_bounds__(64) void k_qr(SweepArgs A, const DevGate* gates, int n_g, double* gout, int ncap,
                                           int nlo) {
  constexpr int G = 64 / TL;
  const int gi = blockIdx.x >> 1, side = blockIdx.x & 1, sweep = blockIdx.y, lane = threadIdx.x;
  const int t = lane / TL, l = lane - t * TL;
  const DevGate g = gates[gi];
  const int site = side ? g.sb : g.sa, leg = side ? g.lb : g.la;
  const int d = side ? g.dB : g.dA, par = side ? g.srcB : g.srcA;
  int D[4];
  site_dims(A, sweep, site, D);
  const Split v = make_split(D, leg, d);
  const int ncols = d * v.Dx;
  if (ncols <= nlo || ncols > TL) return;
  const unsigned long long w0 = win_open(A.win);
  __shared__ double slam[4][MAXCHI];
  __shared__ int rowbase[64];
  __shared__ double rowsc[64];
  __shared__ double Fs[G * TL * TL];
  __shared__ double vbs[G][TL + 1];
  for (int e = lane; e < 4 * MAXCHI; e += 64) {
    const int lg = e / MAXCHI, k = e % MAXCHI;
    const int b = A.leg_bond[site * 4 + lg];
    double val = 1.0;
    if (lg != leg && b >= 0 && k < D[lg]) val = sqrt(A.lam[(int64_t(sweep) * A.n_bonds + b) * A.lam_ld + k]);
    slam[lg][k] = val;
  }
  int cofs = -1;
  if (l < ncols) {
    const int p = l / v.Dx, x = l - p * v.Dx;
    cofs = x * v.Cp * d + p;
  }
  double* F = Fs + t * ncols * ncols;
  for (int e = l; e < ncols * ncols; e += TL) F[e] = 0.0;
  const T* tt = tens<T>(A, par, sweep, site);
  __syncthreads();
  for (int r0 = 0; r0 < v.rows; r0 += 64) {
    {
      const int r = r0 + lane;
      int base = 0;
      double sc = 0.0;
      if (r < v.rows) {
        const int a = r / v.Cp, c = r - a * v.Cp;
        base = (a * v.Dx * v.Cp + c) * d;
        sc = 1.0;
        int cc = c;
        for (int lg = 3; lg > leg; --lg) {
          const int q = cc / D[lg];
          sc *= slam[lg][cc - q * D[lg]];
          cc = q;
        }
        int aa = a;
        for (int lg = leg - 1; lg >= 0; --lg) {
          const int q = aa / D[lg];
          sc *= slam[lg][aa - q * D[lg]];
          aa = q;
        }
      }
      rowbase[lane] = base;
      rowsc[lane] = sc;
    }
    __syncthreads();
    double b[TL];
    double sg = 0.0;
#pragma unroll
    for (int i = 0; i < TL; ++i) {
      const int rl = t * TL + i;
      const bool ok = r0 + rl < v.rows && cofs >= 0;
      b[i] = ok ? double(tt[rowbase[rl] + (ok ? cofs : 0)]) * rowsc[rl] : 0.0;
      sg = fma(b[i], b[i], sg);
    }
    tsqr_block<TL, TL>(F, ncols, b, sg, vbs[t], l);
    __syncthreads();  // the next chunk's offsets replace these
  }
  if (G > 1 && t == 0)
    team_tsqr<TL, TL>(
        F, ncols, (G - 1) * ncols,
        [&](int row, int c) { return Fs[(1 + row / ncols) * ncols * ncols + (row % ncols) * ncols + c]; }, vbs[0], l);
  __syncthreads();
  if (A.bytes_ctr && lane == 0)
    atomicAdd(A.bytes_ctr + ((blockIdx.x + 7 * blockIdx.y) & 63),
              (unsigned long long)(int64_t(v.rows) * ncols * int64_t(sizeof(T))));
  if (side == 0 && lane == 0) A.gate_n[int64_t(sweep) * n_g + gi] = g.K * v.Dx;
  double* out = gout + (int64_t(sweep * n_g + gi) * 2 + side) * ncap * ncap;
  for (int e = lane; e < ncols * ncols; e += 64) out[e] = Fs[e];
  win_close(A.win, w0);
}

// Entry (row, col) of the gated block Y of one gate side through its factor R
// (nR x nR, nR = dd D, row-major): Y[(i, r), (k, b)] = sum_p R[i][p D + b] O_k[r][p]
// (O_k at O[(k dd + r) dd + p]), so that Y^T Y is the side's gated Gram Z.
__device__ __forceinline__ double gated_y(const double* R, const double* O, int dd, int D, int row, int col) {
  const int nR = dd * D;
  const int i = row / dd, r = row - i * dd;
  const int k = col / D, b = col - k * D;
  double y = 0.0;
  for (int p = 0; p < dd; ++p) y = fma(R[i * nR + p * D + b], O[(k * dd + r) * dd + p], y);
  return y;
}

// ---------------------------------------------------------------------------
// truncation of each gated bond: FP64, one workgroup per bond
// ---------------------------------------------------------------------------
// Z_A, Z_B (n x n, n = K D) of a gated bond from the Grams of its two sides:
// Z[(k,b),(k',b')] = sum_{p,q} (O_k^T O_k')[p,q] G[(p,b),(q,b')].
__device__ void build_gated_grams(const SweepArgs& A, const DevGate& g, const double* gin, int ncap, int n_g,
                                  int gi, int sweep, int D, double* ZA, double* ZB, int first, int stride) {
  const int K = g.K, dA = g.dA, dB = g.dB, n = K * D;
  const double* GA = gin + (int64_t(sweep * n_g + gi) * 2 + 0) * ncap * ncap;
  const double* GB = gin + (int64_t(sweep * n_g + gi) * 2 + 1) * ncap * ncap;
  const bool alt = gate_alt(A, g, sweep);
  const double* PA = pool_of(A, sweep) + (alt ? g.pA1 : g.pA);
  const double* PB = pool_of(A, sweep) + (alt ? g.pB1 : g.pB);
  const int nA = dA * D, nB = dB * D;
  if (dA <= 4 && dB <= 4) {
    // one bond pair (b, b2) per thread: its dA^2 and dB^2 Gram entries loaded
    // together into registers, then every (k, k2) block entry from them (the
    // gate tables are read at thread-uniform addresses)
    for (int e = first; e < D * D; e += stride) {
      const int b = e / D, b2 = e - b * D;
      double ga[16], gb[16];
#pragma unroll
      for (int pq = 0; pq < 16; ++pq) {
        const int p = pq >> 2, q = pq & 3;
        const int pa = p < dA ? p : 0, qa = q < dA ? q : 0, pb = p < dB ? p : 0, qb = q < dB ? q : 0;
        // multiplied by a 0/1 mask rather than selected, so that every load is
        // issued together (a selected value lets the compiler branch around it)
        ga[pq] = GA[(pa * D + b) * nA + qa * D + b2] * ((p < dA && q < dA) ? 1.0 : 0.0);
        gb[pq] = GB[(pb * D + b) * nB + qb * D + b2] * ((p < dB && q < dB) ? 1.0 : 0.0);
      }
      for (int k = 0; k < K; ++k)
        for (int k2 = 0; k2 < K; ++k2) {
          const double* wa = PA + (k * K + k2) * dA * dA;
          const double* wb = PB + (k * K + k2) * dB * dB;
          double za = 0.0, zb = 0.0;
#pragma unroll
          for (int pq = 0; pq < 16; ++pq) {
            const int p = pq >> 2, q = pq & 3;
            if (p < dA && q < dA) za = fma(wa[p * dA + q], ga[pq], za);
            if (p < dB && q < dB) zb = fma(wb[p * dB + q], gb[pq], zb);
          }
          ZA[(k * D + b) * n + k2 * D + b2] = za;
          ZB[(k * D + b) * n + k2 * D + b2] = zb;
        }
    }
    return;
  }
  for (int e = first; e < n * n; e += stride) {
    const int r = e / n, c = e % n;
    const int k = r / D, b = r % D, k2 = c / D, b2 = c % D;
    double za = 0.0, zb = 0.0;
    for (int p = 0; p < dA; ++p)
      for (int q = 0; q < dA; ++q) za = fma(PA[((k * K + k2) * dA + p) * dA + q], GA[(p * D + b) * nA + q * D + b2], za);
    for (int p = 0; p < dB; ++p)
      for (int q = 0; q < dB; ++q) zb = fma(PB[((k * K + k2) * dB + p) * dB + q], GB[(p * D + b) * nB + q * D + b2], zb);
    ZA[e] = za;
    ZB[e] = zb;
  }
}

// W_A, W_B of a truncation (the kept singular vectors of C mapped back
// through the gate), threads first, first + stride, ... of the caller.
__device__ void write_w(const SweepArgs& A, const DevGate& g, int sweep, int D, int Dn, bool bad, int n, int rA, int rB,
                        const double* CM, const double* VM, const double* ZA, const double* ZB, const int* ord,
                        const double* Ss, double s1, double* WA, double* WB, int first, int stride, int ldc = 0,
                        int ldj = 0) {
  // ZA holds C' (rA x rB, leading dimension ldc), ZB the rotations V'
  // (rB x rB, leading dimension ldj); 0 means rB
  if (ldc == 0) ldc = rB;
  if (ldj == 0) ldj = rB;
  const int K = g.K, dA = g.dA, dB = g.dB, nA = dA * D, nB = dB * D;
  const bool alt = gate_alt(A, g, sweep);
  const double* OA = pool_of(A, sweep) + (alt ? g.oA1 : g.oA);
  const double* OB = pool_of(A, sweep) + (alt ? g.oB1 : g.oB);
  const int ncA = dA * Dn, ncB = dB * Dn;
  if (bad) {
    for (int e = first; e < nA * ncA; e += stride) WA[2 + e] = 0.0;
    for (int e = first; e < nB * ncB; e += stride) WB[2 + e] = 0.0;
  } else if (K <= 4) {
    // one (bond index b, kept vector m) pair per thread: the K projections
    // phi_k(b, m) of side B's factor (for W_A) and of side A's (for W_B) onto
    // the kept singular vector once, then every (p, p2) entry from them
    for (int e = first; e < D * Dn; e += stride) {
      const int b = e / Dn, m = e - b * Dn, om = ord[m];
      double phA[4], phB[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double pa = 0.0, pb = 0.0;
        if (k < K) {
          for (int j = 0; j < rB; ++j) pa = fma(VM[j * n + k * D + b], ZB[j * ldj + om], pa);
          for (int i = 0; i < rA; ++i) pb = fma(CM[i * n + k * D + b], ZA[i * ldc + om], pb);
        }
        phA[k] = pa;
        phB[k] = pb;
      }
      const double sA = sqrt(Ss[m] / s1) / Ss[m], sB = sqrt(Ss[m] / s1) / (Ss[m] * Ss[m]);
      for (int p = 0; p < dA; ++p)
        for (int p2 = 0; p2 < dA; ++p2) {
          double w = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < K) w = fma(OA[(k * dA + p2) * dA + p], phA[k], w);
          WA[2 + (p * D + b) * ncA + p2 * Dn + m] = w * sA;
        }
      for (int p = 0; p < dB; ++p)
        for (int p2 = 0; p2 < dB; ++p2) {
          double w = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < K) w = fma(OB[(k * dB + p2) * dB + p], phB[k], w);
          WB[2 + (p * D + b) * ncB + p2 * Dn + m] = w * sB;
        }
    }
  } else {
    for (int e = first; e < nA * ncA; e += stride) {
      const int row = e / ncA, col = e % ncA;
      const int p = row / D, b = row % D, p2 = col / Dn, m = col % Dn;
      double w = 0.0;
      for (int k = 0; k < K; ++k) {
        double phi = 0.0;
        for (int j = 0; j < rB; ++j) phi = fma(VM[j * n + k * D + b], ZB[j * ldj + ord[m]], phi);
        w = fma(OA[(k * dA + p2) * dA + p], phi, w);
      }
      WA[2 + e] = w * (sqrt(Ss[m] / s1) / Ss[m]);
    }
    for (int e = first; e < nB * ncB; e += stride) {
      const int row = e / ncB, col = e % ncB;
      const int p = row / D, b = row % D, p2 = col / Dn, m = col % Dn;
      double w = 0.0;
      for (int k = 0; k < K; ++k) {
        double phi = 0.0;
        for (int i = 0; i < rA; ++i) phi = fma(CM[i * n + k * D + b], ZA[i * ldc + ord[m]], phi);
        w = fma(OB[(k * dB + p2) * dB + p], phi, w);
      }
      WB[2 + e] = w * (sqrt(Ss[m] / s1) / (Ss[m] * Ss[m]));
    }
  }
}

// Gates with nlo < K D <= nhi only: the launch's LDS holds matrices of order
// nhi, so small gates run in a launch with small LDS and many workgroups per CU.
template <int NT>
__global__ __launch_bounds__(NT) void k_solve(SweepArgs A, const DevGate* gates, int n_g, const double* gin,
                                             double* wout, int ncap, int nlo, int nhi) {
  extern __shared__ double sm[];
  const int gi = blockIdx.x, sweep = blockIdx.y, tid = threadIdx.x;
  const DevGate g = gates[gi];
  const int64_t bidx = int64_t(sweep) * A.n_bonds + g.bond;
  const int D = A.bond_dim[bidx];
  const int K = g.K, dA = g.dA, dB = g.dB, n = K * D;
  // the size class is decided on the order the Gram recorded (the other
  // launch of the pair may already have changed this bond's dimension)
  const int n0 = A.gate_n[int64_t(sweep) * n_g + gi];
  if (n0 <= nlo || n0 > nhi) return;
  const double logb_in = A.logb[bidx];  // loaded early, used at the end
  // four n x n matrices; above order 64 (the Gram route only) the second one
  // lives in the per-gate global scratch, so the rest fits the LDS
  // Up to order 64 each matrix takes n (n + 1) doubles, so that C and the
  // rotations can sit at an odd leading dimension: the Jacobi teams then read
  // a column's consecutive entries from different LDS banks.
  double* ZA = sm;
  const bool zb_global = n > 64;
  const int slot = zb_global ? n * n : n * (n + 1);
  double* ZB = zb_global ? A.solve_big + int64_t(sweep * n_g + gi) * A.sbig_ld : ZA + slot;
  double* CM = zb_global ? ZA + slot : ZB + slot;
  double* VM = CM + slot;
  double* S = VM + slot;
  double* Ss = S + n;
  double* red = Ss + n;
  int* ord = reinterpret_cast<int*>(red + 4);
  int* perm = ord + n;
  int* flag = perm + n;
  const int nA = dA * D, nB = dB * D;
  int rA, rB;
  if (A.qr) {
    // F_A, F_B: triangular factors of the gated blocks Y_A, Y_B from the
    // sides' factors R (k_qr), by Householder QR (no gated Gram is formed);
    // one team per side: of 16 lanes (orders up to 16) or a wavefront
    constexpr int TQ = NT >= 256 ? 64 : 16;
    for (int e = tid; e < n * n; e += NT) CM[e] = VM[e] = 0.0;
    __syncthreads();
    const bool alt = gate_alt(A, g, sweep);
    const int team = tid / TQ, l = tid - team * TQ;
    if (team < 2) {
      const double* R = gin + (int64_t(sweep * n_g + gi) * 2 + team) * ncap * ncap;
      const int dd = team ? dB : dA;
      const double* O = pool_of(A, sweep) + (team ? (alt ? g.oB1 : g.oB) : (alt ? g.oA1 : g.oA));
      team_tsqr<TQ, TQ>(
          team ? VM : CM, n, dd * dd * D, [&](int row, int col) { return gated_y(R, O, dd, D, row, col); },
          team ? ZB : ZA, l);
    }
    __syncthreads();
    rA = rB = n;
  } else {
    build_gated_grams(A, g, gin, ncap, n_g, gi, sweep, D, ZA, ZB, tid, NT);
    __syncthreads();
    rA = block_pchol(ZA, CM, n, A.pchol_tol, perm, red);  // F_A: CM, rA x n
    rB = block_pchol(ZB, VM, n, A.pchol_tol, perm, red);  // F_B: VM, rB x n
  }
  // C = F_A F_B^T (rA x rB) into ZA, leading dimension ldc; the rotations V'
  // (rB x rB) go to ZB at leading dimension ldj
  const int ldc = zb_global ? rB : (rB | 1), ldj = ldc;
  for (int i = tid >> 4; i < rA; i += NT >> 4)
    for (int j = tid & 15; j < rB; j += 16) {
      double s = 0.0;
      for (int c = 0; c < n; ++c) s += CM[i * n + c] * VM[j * n + c];
      ZA[i * ldc + j] = s;
    }
  __syncthreads();
  int Dn = 0, split = 0;
  double s1 = 0.0;
  if (rA > 0 && rB > 0) {
    const int nsw = block_jacobi(ZA, 1, ldc, rB, rA, ZB, A.jtol, A.jfloor, 40, flag, red, ldj);  // columns of C; V' in ZB
    if (tid == 0) {
      atomicMax(&A.sweeps_max[0], nsw);
      if (nsw >= 40) atomicOr(&A.flags[sweep], 8u);
    }
    block_norms_sorted(ZA, 1, ldc, rB, rA, S, ord);
    for (int m = tid; m < rB; m += NT) Ss[m] = S[ord[m]];
    __syncthreads();
    Dn = rank_rule(Ss, rB, A.chi_cut, A.eps, A.tau, &split);
    s1 = Ss[0];
  }
  const bool bad = !(Dn > 0) || !(s1 > 0.0) || !isfinite(s1);
  if (bad) {
    Dn = 1;
    s1 = 1.0;
  }
  double* WA = wout + (int64_t(sweep * n_g + gi) * 2 + 0) * (2 + ncap * ncap);
  double* WB = wout + (int64_t(sweep * n_g + gi) * 2 + 1) * (2 + ncap * ncap);
  __syncthreads();
  if (tid == 0) {
    WA[0] = WB[0] = double(D);
    WA[1] = WB[1] = double(Dn);
    A.bond_dim[bidx] = Dn;
    A.logb[bidx] = logb_in + log(s1);
    uint32_t f = 0;
    if (bad) f |= 1u;
    if (split) f |= 2u;
    if (f) atomicOr(&A.flags[sweep], f);
  }
  for (int m = tid; m < Dn; m += NT) A.lam[bidx * A.lam_ld + m] = bad ? 1.0 : Ss[m] / s1;
  write_w(A, g, sweep, D, Dn, bad, n, rA, rB, CM, VM, ZA, ZB, ord, Ss, s1, WA, WB, tid, NT, ldc, ldj);
}

// ---------------------------------------------------------------------------
// truncations of order K D <= 16: four or eight per wavefront
// ---------------------------------------------------------------------------
// The steps of k_solve (gated Grams, pivoted Cholesky of both, C = F_A F_B^T,
// one-sided Jacobi SVD of C, rank rule, W_A, W_B) for gates of order n with
// nlo < n <= TL (8 or 16), each on a team of TL lanes of one wavefront: team t
// of a workgroup takes sweep blockIdx.y * (64 / TL) + t of gate blockIdx.x.
// Teams share nothing.  Inside a team, values move through the team's LDS,
// ordered by team_sync (one wavefront executes its LDS accesses in order, so a
// wavefront-scope fence that keeps the compiler from moving them suffices), or
// by DPP moves within the team's lanes.  All lanes of a team take the same
// branches.

// Over the TL (8 or 16) lanes of a team: quad butterflies, then the half-row
// mirror (lane i <-> 7 - i) brings in the other quad, and for 16 the row
// mirror the other half-row.
template <int TL>
__device__ __forceinline__ double team_max(double v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x141>(v));
  if (TL == 16) v = fmax(v, dpp_move<0x140>(v));
  return v;
}

template <int TL>
__device__ __forceinline__ void team_argmax(double& v, int& idx) {
  auto step = [&](double w, int j) {
    if (w > v || (w == v && j < idx)) {
      v = w;
      idx = j;
    }
  };
  step(dpp_move<0xB1>(v), __builtin_amdgcn_update_dpp(0, idx, 0xB1, 0xF, 0xF, false));
  step(dpp_move<0x4E>(v), __builtin_amdgcn_update_dpp(0, idx, 0x4E, 0xF, 0xF, false));
  step(dpp_move<0x141>(v), __builtin_amdgcn_update_dpp(0, idx, 0x141, 0xF, 0xF, false));
  if (TL == 16) step(dpp_move<0x140>(v), __builtin_amdgcn_update_dpp(0, idx, 0x140, 0xF, 0xF, false));
}

// Pivoted Cholesky (as block_pchol) of the n x n Z (n <= TL) by one team:
// lane l owns column l.  Returns the rank; F (r x n) as in block_pchol.
template <int TL>
__device__ int team_pchol(double* Z, double* F, int n, double tol, int* perm, int l) {
  if (l < n) perm[l] = l;
  const double thr = tol * fmax(team_max<TL>(l < n ? Z[l * n + l] : 0.0), 0.0);
  team_sync();
  int r = 0;
  for (int k = 0; k < n; ++k) {
    double piv = (l >= k && l < n) ? Z[l * n + l] : -1e300;
    int j = l;
    team_argmax<TL>(piv, j);
    if (!(piv > thr)) break;
    if (j != k) {
      if (l < n) {  // columns k, j
        const double t = Z[l * n + k];
        Z[l * n + k] = Z[l * n + j];
        Z[l * n + j] = t;
      }
      team_sync();
      if (l < n) {  // rows k, j
        const double t = Z[k * n + l];
        Z[k * n + l] = Z[j * n + l];
        Z[j * n + l] = t;
      }
      if (l == 0) {
        const int t = perm[k];
        perm[k] = perm[j];
        perm[j] = t;
      }
      team_sync();
    }
    const double rk = sqrt(piv), rinv = 1.0 / rk;
    if (l == k) Z[k * n + k] = rk;
    if (l > k && l < n) Z[k * n + l] *= rinv;
    team_sync();
    if (l > k && l < n) {
      const double zl = Z[k * n + l];
      for (int a = k + 1; a < n; ++a) Z[a * n + l] -= Z[k * n + a] * zl;
    }
    team_sync();
    r = k + 1;
  }
  if (l < n)
    for (int i = 0; i < r; ++i) F[i * n + perm[l]] = l >= i ? Z[i * n + l] : 0.0;
  team_sync();
  return r;
}

// One-sided Jacobi (as block_jacobi) on the nv <= TL columns of length len of
// A (column v, entry e at A[v + e * nv]) by one team, with J (nv x nv): the
// pairs of a round take two lanes each (each lane half of the entries, the
// sums exchanged within the pair).  t: the team's index in the wavefront.
template <int TL>
__device__ int team_jacobi(double* A, int nv, int len, double* J, double tol, double floor_rel, int max_sweeps,
                           int l, int t) {
  if (l < nv)
    for (int c = 0; c < nv; ++c) J[l * nv + c] = l == c ? 1.0 : 0.0;
  double s = 0.0;
  if (l < nv)
    for (int e = 0; e < len; ++e) s += A[l + e * nv] * A[l + e * nv];
  const double floor2 = floor_rel * floor_rel * team_max<TL>(s);
  const double sqrt_tol = sqrt(tol);
  team_sync();
  const int ne = nv + (nv & 1), npairs = ne / 2;
  const int pp = l >> 1, h = l & 1;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    bool rot = false, big = false;
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      int i = -1, j = -1;
      if (pp < npairs) {
        if (pp == 0) {
          i = ne - 1;
          j = rnd;
        } else {
          i = rnd + pp;
          i = i >= ne - 1 ? i - (ne - 1) : i;
          j = rnd - pp + ne - 1;
          j = j >= ne - 1 ? j - (ne - 1) : j;
        }
        if (i > j) {
          const int q = i;
          i = j;
          j = q;
        }
      }
      const bool live = pp < npairs && j < nv;  // the same in both lanes of a pair
      double a = 0.0, b = 0.0, g = 0.0;
      if (live)
        for (int e = h; e < len; e += 2) {
          const double x = A[i + e * nv], y = A[j + e * nv];
          a += x * x;
          b += y * y;
          g += x * y;
        }
      // the pair's two halves (lanes 2p, 2p + 1), every lane active
      a += dpp_move<0xB1>(a);
      b += dpp_move<0xB1>(b);
      g += dpp_move<0xB1>(g);
      const double sab = sqrt(a) * sqrt(b);
      if (live && a > floor2 && b > floor2 && fabs(g) > tol * sab) {
        const double zeta = (b - a) / (2.0 * g);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int e = h; e < len; e += 2) {
          const double x = A[i + e * nv], y = A[j + e * nv];
          A[i + e * nv] = cs * x - sn * y;
          A[j + e * nv] = sn * x + cs * y;
        }
        for (int e = h; e < nv; e += 2) {
          const double x = J[e * nv + i], y = J[e * nv + j];
          J[e * nv + i] = cs * x - sn * y;
          J[e * nv + j] = sn * x + cs * y;
        }
        rot = true;
        if (fabs(g) > sqrt_tol * sab) big = true;
      }
      team_sync();
    }
    const unsigned long long rb = __ballot(rot), bb = __ballot(big);
    const unsigned long long tm = (1ull << TL) - 1;
    if (!((rb >> (t * TL)) & tm)) break;
    if (!((bb >> (t * TL)) & tm)) break;
  }
  return sweep;
}

template <int TL>
__global__ __launch_bounds__(64) void k_solve_team(SweepArgs A, const DevGate* gates, int n_g, const double* gin,
                                                   double* wout, int ncap, int nlo) {
  constexpr int TSW = 64 / TL;  // problems per workgroup
  __shared__ double tz[TSW][4 * TL * TL + 2 * TL];  // Z_A, Z_B, F_A, F_B, S, Ss
  __shared__ int ti[TSW][2 * TL + 2];                // ord, perm, rank rule result
  const int gi = blockIdx.x, tid = threadIdx.x;
  const int t = tid / TL, l = tid - t * TL;
  const int sweep = blockIdx.y * TSW + t;
  if (sweep >= A.n_sweeps) return;  // the whole team
  const DevGate g = gates[gi];
  const int64_t bidx = int64_t(sweep) * A.n_bonds + g.bond;
  // the class is decided on the order the Gram recorded (see k_solve)
  const int n0 = A.gate_n[int64_t(sweep) * n_g + gi];
  if (n0 <= nlo || n0 > TL) return;
  const int D = A.bond_dim[bidx];
  const int K = g.K, n = K * D;
  const double logb_in = A.logb[bidx];
  double* ZA = tz[t];
  double* ZB = ZA + TL * TL;
  double* CM = ZB + TL * TL;
  double* VM = CM + TL * TL;
  double* S = VM + TL * TL;
  double* Ss = S + TL;
  int* ord = ti[t];
  int* perm = ord + TL;
  int* rr = perm + TL;
  int rA, rB;
  if (A.qr) {
    // F_A, F_B by Householder QR of the gated blocks (see k_solve)
    for (int e = l; e < n * n; e += TL) CM[e] = VM[e] = 0.0;
    team_sync();
    const bool alt = gate_alt(A, g, sweep);
    const double* RA = gin + (int64_t(sweep * n_g + gi) * 2 + 0) * ncap * ncap;
    const double* RB = gin + (int64_t(sweep * n_g + gi) * 2 + 1) * ncap * ncap;
    const double* OA = pool_of(A, sweep) + (alt ? g.oA1 : g.oA);
    const double* OB = pool_of(A, sweep) + (alt ? g.oB1 : g.oB);
    const int dA = g.dA, dB = g.dB;
    team_tsqr<TL, TL>(CM, n, dA * dA * D, [&](int row, int col) { return gated_y(RA, OA, dA, D, row, col); }, ZA, l);
    team_tsqr<TL, TL>(VM, n, dB * dB * D, [&](int row, int col) { return gated_y(RB, OB, dB, D, row, col); }, ZA, l);
    rA = rB = n;
  } else {
    build_gated_grams(A, g, gin, ncap, n_g, gi, sweep, D, ZA, ZB, l, TL);
    team_sync();
    rA = team_pchol<TL>(ZA, CM, n, A.pchol_tol, perm, l);
    rB = team_pchol<TL>(ZB, VM, n, A.pchol_tol, perm, l);
  }
  if (l < rB)  // C = F_A F_B^T (rA x rB) into Z_A, lane j takes column j
    for (int i = 0; i < rA; ++i) {
      double c = 0.0;
      for (int k = 0; k < n; ++k) c += CM[i * n + k] * VM[l * n + k];
      ZA[i * rB + l] = c;
    }
  team_sync();
  int Dn = 0, split = 0;
  double s1 = 0.0;
  if (rA > 0 && rB > 0) {
    const int nsw = team_jacobi<TL>(ZA, rB, rA, ZB, A.jtol, A.jfloor, 40, l, t);  // columns of C; V' in Z_B
    if (l == 0) {
      atomicMax(&A.sweeps_max[0], nsw);
      if (nsw >= 40) atomicOr(&A.flags[sweep], 8u);
    }
    if (l < rB) {
      double q = 0.0;
      for (int e = 0; e < rA; ++e) q += ZA[l + e * rB] * ZA[l + e * rB];
      S[l] = sqrt(q);
    }
    team_sync();
    if (l < rB) {
      int rank = 0;
      for (int u = 0; u < rB; ++u)
        if (sorts_before(S[u], u, S[l], l)) ++rank;
      ord[rank] = l;
    }
    team_sync();
    if (l < rB) Ss[l] = S[ord[l]];
    team_sync();
    if (l == 0) {
      rr[0] = rank_rule(Ss, rB, A.chi_cut, A.eps, A.tau, &rr[1]);
    }
    team_sync();
    Dn = rr[0];
    split = rr[1];
    s1 = Ss[0];
  }
  const bool bad = !(Dn > 0) || !(s1 > 0.0) || !isfinite(s1);
  if (bad) {
    Dn = 1;
    s1 = 1.0;
  }
  double* WA = wout + (int64_t(sweep * n_g + gi) * 2 + 0) * (2 + ncap * ncap);
  double* WB = wout + (int64_t(sweep * n_g + gi) * 2 + 1) * (2 + ncap * ncap);
  if (l == 0) {
    WA[0] = WB[0] = double(D);
    WA[1] = WB[1] = double(Dn);
    A.bond_dim[bidx] = Dn;
    A.logb[bidx] = logb_in + log(s1);
    uint32_t f = 0;
    if (bad) f |= 1u;
    if (split) f |= 2u;
    if (f) atomicOr(&A.flags[sweep], f);
  }
  for (int m = l; m < Dn; m += TL) A.lam[bidx * A.lam_ld + m] = bad ? 1.0 : Ss[m] / s1;
  write_w(A, g, sweep, D, Dn, bad, n, rA, rB, CM, VM, ZA, ZB, ord, Ss, s1, WA, WB, l, TL);
}

// ---------------------------------------------------------------------------
// reabsorption T' = T W on the (p, bond) columns
// ---------------------------------------------------------------------------
// One wavefront per (gate side, sweep), one thread per tensor row: the row's
// nin entries are held in registers in FP64 and multiplied by W (FP64, staged
// in LDS and read by all lanes at the same address), four outputs at a time;
// only the result is rounded to the storage type.  A launch handles the gates
// with nlo < nin <= NMAX, so narrow gates run with fewer registers.
template <typename T, int NMAX>
__global__ __launch_bounds__(64) void k_reabsorb(SweepArgs A, const DevGate* gates, int n_g, const double* win,
                                                 int ncap, int nlo) {
  const int gi = blockIdx.x >> 1, side = blockIdx.x & 1, sweep = blockIdx.y, tid = threadIdx.x;
  const DevGate g = gates[gi];
  const int site = side ? g.sb : g.sa, leg = side ? g.lb : g.la;
  const int d = side ? g.dB : g.dA, par = side ? g.srcB : g.srcA;
  const double* W = win + (int64_t(sweep * n_g + gi) * 2 + side) * (2 + ncap * ncap);
  const int Dold = int(W[0]), Dn = int(W[1]);
  const int nin = d * Dold, nout = d * Dn, nst = (nout + 3) & ~3;
  // classes by row width: nin in (nlo, NMAX] with at most 64 outputs, and
  // the widest (NMAX > 64) every row with more than 64 inputs or outputs
  constexpr int NO = NMAX > 64 ? NMAX : 64;
  if (NMAX > 64 ? (nin <= 64 && nout <= 64) || nin > NMAX || nout > NMAX : nin <= nlo || nin > NMAX || nout > 64)
    return;
  const unsigned long long w0 = win_open(A.win);
  int D[4];
  site_dims(A, sweep, site, D);
  D[leg] = Dold;
  const Split v = make_split(D, leg, d);
  __shared__ double4 Ws4[NMAX * NO / 4];
  __shared__ int colin[NMAX], colout[NO];
  double* Ws = reinterpret_cast<double*>(Ws4);
  for (int e = tid; e < nin * nst; e += 64) {
    const int k = e / nst, q = e - k * nst;
    Ws[e] = q < nout ? W[2 + k * nout + q] : 0.0;
  }
  for (int col = tid; col < nin; col += 64) {
    const int p = col / Dold, x = col - p * Dold;
    colin[col] = x * v.Cp * d + p;
  }
  for (int col = tid; col < nout; col += 64) {
    const int p = col / Dn, m = col - p * Dn;
    colout[col] = m * v.Cp * d + p;
  }
  __syncthreads();
  const T* in = tens<T>(A, par, sweep, site);
  T* out = tens<T>(A, par ^ 1, sweep, site);
  if (A.bytes_ctr && tid == 0)
    atomicAdd(A.bytes_ctr + ((blockIdx.x + 7 * blockIdx.y) & 63),
              (unsigned long long)(int64_t(v.rows) * (nin + nout) * int64_t(sizeof(T))));
  const int n4 = nst / 4;
  for (int r = tid; r < v.rows; r += 64) {
    const int a = r / v.Cp, c = r - a * v.Cp;
    const T* src = in + (a * Dold * v.Cp + c) * d;
    T* dst = out + (a * Dn * v.Cp + c) * d;
    double x[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k)  // every load issued (a valid address, times 0 past nin)
      x[k] = double(src[colin[k < nin ? k : 0]]) * (k < nin ? 1.0 : 0.0);
    for (int q4 = 0; q4 < n4; ++q4) {
      double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k < nin) {
          const double4 w = Ws4[k * n4 + q4];
          s0 += x[k] * w.x;
          s1 += x[k] * w.y;
          s2 += x[k] * w.z;
          s3 += x[k] * w.w;
        }
      const int q = 4 * q4;
      dst[colout[q]] = T(s0);
      if (q + 1 < nout) dst[colout[q + 1]] = T(s1);
      if (q + 2 < nout) dst[colout[q + 2]] = T(s2);
      if (q + 3 < nout) dst[colout[q + 3]] = T(s3);
    }
  }
  win_close(A.win, w0);
}

// A workgroup of one wavefront: this wave's LDS accesses so far complete
// before any that follow, and the compiler moves no memory access across.
// Global stores still in flight are not waited for (__syncthreads would).
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// The reabsorption T' = T W on the matrix cores, for rows of up to NMAX
// (32 or 64) entries: one wavefront per (gate side, sweep), chunks of 32
// rows.  A chunk of T is fetched in memory order (as k_gram2: consecutive
// lanes at consecutive addresses) into LDS, multiplied by W, staged in LDS
// again and written back in memory order.  BF = 0: FP64 matrix cores
// (v_mfma_f64_16x16x4f64: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// item r of lane j + 16 q is C[q + 4 r][j]); W sits in LDS in FP64.  BF = 1
// (float storage): BF16 matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16: lane i + 16 q holds A[i][8 q .. 8 q + 7] and
// B[8 q .. 8 q + 7][i]; item r of lane j + 16 q is C[4 q + r][j]), T and W
// split into three BF16 terms each and the six leading products summed (as
// k_gram2); W's terms stay in registers.
template <typename T, int NMAX, int BF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_reabsorb2(SweepArgs A, const DevGate* gates, int n_g, const double* win,
                                                  int ncap, int nlo) {
  constexpr int NL = GR * NMAX / 64;  // elements a lane moves per chunk
  constexpr int KB = BF ? NMAX / 32 : 1, KS = BF ? 1 : NMAX / 4;
  static_assert(NMAX == 64 && GR == 32, "the chunk's lane assignment assumes 32 rows of 64 columns");
  const int gi = blockIdx.x >> 1, side = blockIdx.x & 1, sweep = blockIdx.y, lane = threadIdx.x;
  const DevGate g = gates[gi];
  const int site = side ? g.sb : g.sa, leg = side ? g.lb : g.la;
  const int d = side ? g.dB : g.dA, par = side ? g.srcB : g.srcA;
  const double* W = win + (int64_t(sweep * n_g + gi) * 2 + side) * (2 + ncap * ncap);
  const int Dold = int(W[0]), Dn = int(W[1]);
  const int nin = d * Dold, nout = d * Dn;
  if (nin <= nlo || nin > NMAX || nout > 64) return;  // wider outputs: k_reabsorb<T, 96>
  const unsigned long long w0 = win_open(A.win);
  int D[4];
  site_dims(A, sweep, site, D);
  D[leg] = Dold;
  const Split v = make_split(D, leg, d);
  // one chunk of T (row-major, canonical input columns), then of T' (canonical
  // output columns) in the same place
  constexpr int TS = NMAX + 1;
  __shared__ T Tb[GR * TS];
  __shared__ int rb_in[GR], rb_out[GR];
  const T* in = tens<T>(A, par, sweep, site);
  T* out = tens<T>(A, par ^ 1, sweep, site);
  const bool rowfast = v.Cp > 1;
  const int li = lane & 15, lq = lane >> 4;
  // W in registers: BF16 terms (BF = 1) or FP64 values (BF = 0), per B operand
  bf16x8 wh[KB][4], wm[KB][4], wl[KB][4];
  double wd[BF ? 1 : 4][KS];
  if (BF) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        float vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = 32 * kb + 8 * lq + u, n = 16 * nb + li;
          vv[u] = (k < nin && n < nout) ? float(W[2 + k * nout + n]) : 0.f;
        }
        split3(vv, wh[kb][nb], wm[kb][nb], wl[kb][nb]);
      }
  } else {
#pragma unroll
    for (int nb = 0; nb < (BF ? 1 : 4); ++nb)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + lq, n = 16 * nb + li;
        wd[nb][ks] = (k < nin && n < nout) ? W[2 + k * nout + n] : 0.0;
      }
  }
  // memory-order columns mc = x d + p: offsets in a row and canonical columns,
  // of the input (bond Dold) and of the output (bond Dn)
  __shared__ int ioff[NMAX], ican[NMAX], ooff[NMAX], ocan[NMAX];
  for (int mc = lane; mc < NMAX; mc += 64) {
    const int x = mc / d, p = mc - x * d;
    ioff[mc] = mc < nin ? x * v.Cp * d + p : -1;
    ican[mc] = p * Dold + x;
    ooff[mc] = mc < nout ? x * v.Cp * d + p : -1;
    ocan[mc] = p * Dn + x;
  }
  for (int e = lane; e < GR * TS; e += 64) Tb[e] = T(0);
  if (A.bytes_ctr && lane == 0)
    atomicAdd(A.bytes_ctr + ((blockIdx.x + 7 * blockIdx.y) & 63),
              (unsigned long long)(int64_t(v.rows) * (nin + nout) * int64_t(sizeof(T))));
  for (int r0 = 0; r0 < v.rows; r0 += GR) {
    if (lane < GR) {
      const int r = r0 + lane;
      int bi = 0, bo = 0;
      if (r < v.rows) {
        const int a = r / v.Cp, c = r - a * v.Cp;
        bi = (a * Dold * v.Cp + c) * d;
        bo = (a * Dn * v.Cp + c) * d;
      }
      rb_in[lane] = bi;
      rb_out[lane] = bo;
    }
    wave_lds_sync();
    // the chunk into registers with every load in flight at once (each from
    // an offset inside the tensor: element 0 stands in for the columns and
    // rows past its end), then into LDS.  Rows run along memory (Cp > 1):
    // lane l takes row l % 32 and columns l / 32 + 2 j; otherwise lane l
    // takes column l of rows j.
    T rv[NL];
    if (rowfast) {
      const int rl = lane & 31, m0 = lane >> 5;
      const bool rok = r0 + rl < v.rows;
      const int rbase = rb_in[rl];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const int io = ioff[m0 + 2 * j];
        rv[j] = in[rok && io >= 0 ? rbase + io : 0];
      }
#pragma unroll
      for (int j = 0; j < NL; ++j)
        if (ioff[m0 + 2 * j] >= 0) Tb[rl * TS + ican[m0 + 2 * j]] = rok ? rv[j] : T(0);
    } else {
      const int io = ioff[lane], ic = ican[lane];
#pragma unroll
      for (int j = 0; j < NL; ++j) rv[j] = in[io >= 0 && r0 + j < v.rows ? rb_in[j] + io : 0];
      if (io >= 0)
#pragma unroll
        for (int j = 0; j < NL; ++j) Tb[j * TS + ic] = r0 + j < v.rows ? rv[j] : T(0);
    }
    wave_lds_sync();
    // A operands of both 16-row blocks into registers, then the products into Tb
    if (BF == 0) {
      double a[2][KS];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) a[mb][ks] = double(Tb[(16 * mb + li) * TS + 4 * ks + lq]);
      wave_lds_sync();
      const int nbn = (nout + 15) >> 4;
      dbl4 c[2][4];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) c[mb][nb] = dbl4{0.0, 0.0, 0.0, 0.0};
      // eight independent accumulators interleaved, so consecutive products
      // never wait for each other
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          if (nb < nbn) {
            c[0][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][ks], wd[nb][ks], c[0][nb], 0, 0, 0);
            c[1][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][ks], wd[nb][ks], c[1][nb], 0, 0, 0);
          }
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          if (nb < nbn)
#pragma unroll
            for (int r = 0; r < 4; ++r) Tb[(16 * mb + lq + 4 * r) * TS + 16 * nb + li] = T(c[mb][nb][r]);
    } else {
      bf16x8 ah[2][KB], am[2][KB], al[2][KB];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          float vv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) vv[u] = float(Tb[(16 * mb + li) * TS + 32 * kb + 8 * lq + u]);
          split3(vv, ah[mb][kb], am[mb][kb], al[mb][kb]);
        }
      wave_lds_sync();
      const int nbn = (nout + 15) >> 4;
      flt4 c[2][4];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) c[mb][nb] = flt4{0.f, 0.f, 0.f, 0.f};
      // the six products of a block pair, smallest first, each step over the
      // eight independent accumulators
      auto step = [&](const bf16x8 (&x)[2][KB], const bf16x8 (&y)[KB][4], int kb) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          if (nb < nbn) {
            c[0][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[0][kb], y[kb][nb], c[0][nb], 0, 0, 0);
            c[1][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[1][kb], y[kb][nb], c[1][nb], 0, 0, 0);
          }
      };
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        step(al, wh, kb);
        step(am, wm, kb);
        step(ah, wl, kb);
        step(am, wh, kb);
        step(ah, wm, kb);
        step(ah, wh, kb);
      }
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          if (nb < nbn)
#pragma unroll
            for (int r = 0; r < 4; ++r) Tb[(16 * mb + 4 * lq + r) * TS + 16 * nb + li] = T(c[mb][nb][r]);
    }
    wave_lds_sync();
    // write back in memory order (output rows of nout entries), the same
    // lane assignment: the LDS reads first, then the stores, which the next
    // chunk does not wait for
    if (rowfast) {
      const int rl = lane & 31, m0 = lane >> 5;
      const bool rok = r0 + rl < v.rows;
      const int rbase = rb_out[rl];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const int oc = ocan[m0 + 2 * j];
        rv[j] = Tb[rl * TS + (ooff[m0 + 2 * j] >= 0 ? oc : 0)];
      }
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const int oo = ooff[m0 + 2 * j];
        if (rok && oo >= 0) out[rbase + oo] = rv[j];
      }
    } else {
      const int oo = ooff[lane], oc = oo >= 0 ? ocan[lane] : 0;
#pragma unroll
      for (int j = 0; j < NL; ++j) rv[j] = Tb[j * TS + oc];
      if (oo >= 0)
#pragma unroll
        for (int j = 0; j < NL; ++j)
          if (r0 + j < v.rows) out[rb_out[j] + oo] = rv[j];
    }
    wave_lds_sync();
  }
  win_close(A.win, w0);
}

// ---------------------------------------------------------------------------
// per-site rescale after each layer
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(ET) void k_rescale(SweepArgs A, const int32_t* d_after, const int32_t* par_after) {
  __shared__ double red[8];
  const int site = blockIdx.x, sweep = blockIdx.y;
  int D[4];
  site_dims(A, sweep, site, D);
  const int64_t n = int64_t(d_after[site]) * D[0] * D[1] * D[2] * D[3];
  T* t = tens<T>(A, par_after[site], sweep, site);
  // EU elements per lane and step, their loads issued together
  constexpr int EU = 8;
  double m = 0.0;
  int64_t e = threadIdx.x;
  for (; e + (EU - 1) * ET < n; e += EU * ET) {
    T v[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) v[u] = t[e + u * ET];
#pragma unroll
    for (int u = 0; u < EU; ++u) m = fmax(m, fabs(double(v[u])));
  }
  for (; e < n; e += ET) m = fmax(m, fabs(double(t[e])));
  m = block_max_abs_reduce(m, red);
  const bool bad = !(m > 0.0) || !isfinite(m);
  const double c = bad ? 1.0 : m;
  const double inv = 1.0 / c;
  e = threadIdx.x;
  for (; e + (EU - 1) * ET < n; e += EU * ET) {
    T v[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) v[u] = t[e + u * ET];
#pragma unroll
    for (int u = 0; u < EU; ++u) t[e + u * ET] = T(double(v[u]) * inv);
  }
  for (; e < n; e += ET) t[e] = T(double(t[e]) * inv);
  if (threadIdx.x == 0) {
    A.logs[int64_t(sweep) * A.n_sites + site] += log(c);
    if (bad) atomicOr(&A.flags[sweep], 1u);
  }
}

// ---------------------------------------------------------------------------
// final stage: contract f_s into the physical leg (FP64 output)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(ET) void k_finalize(SweepArgs A, const int32_t* d_final, const int32_t* f_off,
                                                 const int32_t* par_final, double* fin, int64_t fin_stride,
                                                 const int64_t* fin_off) {
  const int site = blockIdx.x, sweep = blockIdx.y;
  int D[4];
  site_dims(A, sweep, site, D);
  const int64_t rows = int64_t(D[0]) * D[1] * D[2] * D[3];
  const int d = d_final[site];
  const double* f = pool_of(A, sweep) + f_off[site];
  const T* t = tens<T>(A, par_final[site], sweep, site);
  double* o = fin + int64_t(sweep) * fin_stride + fin_off[site];
  if (d <= 4) {
    // RU rows per lane and step, all their loads issued before any is used
    // (rows past the end read row 0 and are not written)
    constexpr int RU = 4;
    for (int64_t r0 = threadIdx.x; r0 < rows; r0 += RU * ET) {
      T v[RU][4];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int64_t r = r0 + u * ET < rows ? r0 + u * ET : 0;
#pragma unroll
        for (int p = 0; p < 4; ++p)
          if (p < d) v[u][p] = t[r * d + p];
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p)
          if (p < d) s += f[p] * double(v[u][p]);
        if (r0 + u * ET < rows) o[r0 + u * ET] = s;
      }
    }
  } else {
    for (int64_t r = threadIdx.x; r < rows; r += ET) {
      double s = 0.0;
      for (int p = 0; p < d; ++p) s += f[p] * double(t[r * d + p]);
      o[r] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// boundary MPS, zip-up, one workgroup per sweep per (row, column) step
// ---------------------------------------------------------------------------
__global__ void k_zip_init(ZipArgs Z) {
  const int s = blockIdx.x;
  for (int x = threadIdx.x; x < Z.Lx; x += blockDim.x) {
    int* md = Z.mdim + ((int64_t(s) * 2 + 0) * Z.Lx + x) * 3;
    md[0] = md[1] = md[2] = 1;
    Z.mps0[(int64_t(s) * Z.Lx + x) * Z.mcap] = 1.0;
  }
  if (threadIdx.x == 0) {
    Z.logm[s] = 0.0;
    Z.flags[s] = 0u;
  }
}

__device__ __forceinline__ int zbd(const ZipArgs& Z, int s, int b) {
  return Z.bond_dim[int64_t(s) * Z.n_bonds + b];
}

constexpr int ZNT = 512;  // threads of the contraction / output kernels of a boundary-MPS step
constexpr int ZBT = 64;   // threads of the decomposition kernel (one wavefront)
constexpr int ZBIG = 64;  // FP32 mode: larger Gram blocks go to the 512-thread kernel

// One zip-up step of the boundary MPS (row y, column x) for one sweep, in
// three kernels:
//   a: L4[nu,w,n,a'] = sum_a K[nu,a,w] M[a,n,a'];
//      Th[(nu,s'),(a',w')] = sum_{w,n} L4[nu,w,n,a'] T[w,w',n,s'];
//      in FP32 mode also the Gram G of the smaller family of Th (its rows if
//      R <= C, else its columns)
//   b: orthonormal singular vectors Fv of that family and singular values S:
//      one-sided Jacobi on the columns of G (FP32 mode; G is PSD, so the
//      rotated column norms are its eigenvalues S^2), or on the family of Th
//      itself (FP64 mode); rank rule with chi_m
//   c: rows family: new MPS site U = Fv, carry K = Fv^T Th;
//      columns family: U = Th Fv / S, carry K = S Fv^T;
//      the last column keeps Th whole; the new site is divided by its max.
// zdim per sweep: R, C, nu, sD, aR, wR, rows, nv, Dn.

__device__ __forceinline__ void zip_dims(const ZipArgs& Z, int s, int x, int y, int& sd, int& aR, int& wL,
                                         int& wR, int& nU, int& sD) {
  const int Lx = Z.Lx, Ly = Z.Ly, nbh = (Lx - 1) * Ly, cur = y & 1;
  const int* mo = Z.mdim + ((int64_t(s) * 2 + cur) * Lx + x) * 3;
  sd = mo[1];
  aR = mo[2];
  wL = x > 0 ? zbd(Z, s, y * (Lx - 1) + x - 1) : 1;
  wR = x + 1 < Lx ? zbd(Z, s, y * (Lx - 1) + x) : 1;
  nU = y > 0 ? zbd(Z, s, nbh + (y - 1) * Lx + x) : 1;
  sD = y + 1 < Ly ? zbd(Z, s, nbh + y * Lx + x) : 1;
}

// inline_dec: the step's decomposition is done here, not by a launch of its
// own: in the last row R = nu sD = 1 (the carry starts at 1 and stays at the
// rank 1 of its family; the bond below is 1), so the family is Th's one row,
// its singular value the row's norm and its vector [1].
__global__ __launch_bounds__(ZNT) void k_zip_a(ZipArgs Z, int x, int y, int inline_dec) {
  __shared__ double gst[GEMM_LDS];
  __shared__ double red[16];
  const int s = blockIdx.x, tid = threadIdx.x;
  const unsigned long long w0 = win_open(Z.win_a);
  const int cur = y & 1;
  const double* Mold = (cur ? Z.mps1 : Z.mps0) + (int64_t(s) * Z.Lx + x) * Z.mcap;
  int sd, aR, wL, wR, nU, sD;
  zip_dims(Z, s, x, y, sd, aR, wL, wR, nU, sD);
  const double* Tt = Z.fin + int64_t(s) * Z.fin_stride + Z.fin_off[y * Z.Lx + x];
  double* Kp = Z.K + int64_t(s) * Z.kcap;
  int* kd = Z.kdim + int64_t(s) * 3;
  if (x == 0) {
    if (tid == 0) {
      kd[0] = kd[1] = kd[2] = 1;
      Kp[0] = 1.0;
    }
    __syncthreads();
  }
  const int nu = kd[0], ka = kd[1];
  double* L4 = Z.L4 + int64_t(s) * Z.bigcap;
  double* Th = Z.Th + int64_t(s) * Z.bigcap;
  const int sa = sd * aR;
  const int R = nu * sD, C = aR * wR;
  // The operand offsets of both contractions separate into a row part and a
  // column part (e.g. L4[nu, w, n, a'] at (m / aR) wL sd aR + m % aR + k aR);
  // the parts are tabulated once in LDS so the fetches do no division.
  constexpr int TAB = 1024;
  __shared__ int tm[TAB], tk[TAB], tn[TAB], tn2[TAB];
  const bool tabs = nu * wL <= TAB && nu * aR <= TAB && wL * sd <= TAB && wR * sD <= TAB;
  if (tabs) {
    for (int m = tid; m < nu * wL; m += ZNT) tm[m] = (m / wL) * ka * wL + m % wL;
    __syncthreads();
    block_gemm512(
        nu * wL, sa, ka, [&](int m, int k) { return Kp[tm[m] + k * wL]; }, [&](int k, int n) { return Mold[k * sa + n]; },
        [&](int m, int n, double v) { L4[m * sa + n] = v; }, gst);
    for (int m = tid; m < nu * aR; m += ZNT) tm[m] = (m / aR) * wL * sd * aR + m % aR;
    for (int k = tid; k < wL * sd; k += ZNT) tk[k] = (k / sd) * wR * nU * sD + (k % sd) * sD;
    for (int n = tid; n < wR * sD; n += ZNT) {
      tn[n] = (n / sD) * nU * sD + n % sD;
      tn2[n] = (n % sD) * C + n / sD;
    }
    __syncthreads();
    auto l4_at = [&](int m, int k) { return L4[tm[m] + k * aR]; };
    auto t_at = [&](int k, int n) { return Tt[tk[k] + tn[n]]; };
    auto th_put = [&](int m, int n, double v) { Th[(m / aR) * sD * C + (m % aR) * wR + tn2[n]] = v; };
    // the reduced precisions form Theta on the BF16 matrix cores (FP32-accurate
    // products of the FP32-accurate tensors); FP64 on the FP64 ones
    if (Z.bf_theta)
      block_gemm512_bf(nu * aR, wR * sD, wL * sd, l4_at, t_at, th_put, gst);
    else
      block_gemm512(nu * aR, wR * sD, wL * sd, l4_at, t_at, th_put, gst);
  } else {
    block_gemm512(
        nu * wL, sa, ka, [&](int m, int k) { return Kp[((m / wL) * ka + k) * wL + m % wL]; },
        [&](int k, int n) { return Mold[k * sa + n]; }, [&](int m, int n, double v) { L4[m * sa + n] = v; }, gst);
    auto l4_at = [&](int m, int k) { return L4[(((m / aR) * wL + k / sd) * sd + k % sd) * aR + m % aR]; };
    auto t_at = [&](int k, int n) { return Tt[(((k / sd) * wR + n / sD) * nU + k % sd) * sD + n % sD]; };
    auto th_put = [&](int m, int n, double v) { Th[((m / aR) * sD + n % sD) * C + (m % aR) * wR + n / sD] = v; };
    if (Z.bf_theta)
      block_gemm512_bf(nu * aR, wR * sD, wL * sd, l4_at, t_at, th_put, gst);
    else
      block_gemm512(nu * aR, wR * sD, wL * sd, l4_at, t_at, th_put, gst);
  }
  const bool rows = R <= C;
  const int nv = rows ? R : C;
  if (inline_dec) {
    double q = 0.0;
    for (int k = tid; k < C; k += ZNT) q = fma(Th[k], Th[k], q);
    const double S0 = sqrt(block_sum(q, red));
    if (tid == 0) {
      Z.zS[int64_t(s) * 1024] = S0;
      Z.L4[int64_t(s) * Z.bigcap] = 1.0;  // Fv: L4 is dead after the second product
      // a zero row is the rank rule's empty case; R != 1 cannot happen
      if (!(S0 > 0.0) || R != 1) atomicOr(&Z.flags[s], 3u);
    }
  } else if (x + 1 < Z.Lx && Z.gram_path) {
    double* G = Z.Gm + int64_t(s) * Z.bigcap;
    if (rows)
      block_gemm512<true, true>(
          R, R, C, [&](int m, int k) { return Th[m * C + k]; }, [&](int k, int n) { return Th[n * C + k]; },
          [&](int m, int n, double v) { G[m * R + n] = v; }, gst);
    else
      block_gemm512(
          C, C, R, [&](int m, int k) { return Th[k * C + m]; }, [&](int k, int n) { return Th[k * C + n]; },
          [&](int m, int n, double v) { G[m * C + n] = v; }, gst);
  }
  if (Z.flop_a && tid == 0) {
    // algorithmic flops: the two contractions and, on the Gram route, the Gram
    double f = 2.0 * (nu * wL) * double(sa) * ka + 2.0 * double(nu * aR) * double(wR * sD) * double(wL * sd);
    if (!inline_dec && x + 1 < Z.Lx && Z.gram_path) f += rows ? 2.0 * R * double(R) * C : 2.0 * C * double(C) * R;
    atomicAdd(Z.flop_a + (s & 63), (unsigned long long)f);
  }
  if (tid == 0) {
    int* zd = Z.zdim + int64_t(s) * 12;
    zd[0] = R;
    zd[1] = C;
    zd[2] = nu;
    zd[3] = sD;
    zd[4] = aR;
    zd[5] = wR;
    zd[6] = rows ? 1 : 0;
    zd[7] = nv;
    zd[8] = 1;
  }
  win_close(Z.win_a, w0);
}

// Rank rule on the sorted singular values Sout of the smaller family, then the
// kept vectors into Fv (nv x Dn, row-major): component r of the vector with
// the c-th largest value is Zv[ord[c] * cs + r * rs].  Records Dn and the flags.
__device__ void zip_keep(const ZipArgs& Z, int s, int* zd, int nv, const double* Sout, const int* ord,
                         const double* Zv, int cs, int rs, int nsw) {
  int split = 0;
  int Dn = rank_rule(Sout, nv, Z.chi_m, Z.eps, Z.tau, &split);
  bool bad = false;
  if (Dn < 1) {
    Dn = 1;
    bad = true;
  }
  double* Fv = Z.L4 + int64_t(s) * Z.bigcap;  // L4 is dead after kernel a
  for (int e = threadIdx.x; e < nv * Dn; e += blockDim.x) Fv[e] = Zv[ord[e % Dn] * cs + (e / Dn) * rs];
  if (threadIdx.x == 0) {
    zd[8] = Dn;
    atomicMax(&Z.sweeps_max[1], nsw);
    uint32_t f = (bad ? 1u : 0u) | (split ? 2u : 0u) | (nsw >= 40 ? 8u : 0u);
    if (f) atomicOr(&Z.flags[s], f);
  }
}

// FP64 mode: one-sided Jacobi SVD of the smaller family of Theta.
__global__ __launch_bounds__(ZBT) void k_zip_b(ZipArgs Z, int x, int y, int lds_doubles) {
  extern __shared__ double zsm[];
  __shared__ double S[1024];
  __shared__ int ord[1024];
  __shared__ int flag[4];
  __shared__ double red[8];
  const int s = blockIdx.x, tid = threadIdx.x;
  int* zd = Z.zdim + int64_t(s) * 12;
  const int R = zd[0], C = zd[1];
  const bool rows = zd[6] != 0;
  const int nv = zd[7], len = rows ? C : R;
  double* Th = Z.Th + int64_t(s) * Z.bigcap;
  double* Jm = Z.Jm + int64_t(s) * Z.jcap;
  double* Sout = Z.zS + int64_t(s) * 1024;
  double* A;
  double* J;
  long vs, es;
  const bool fits = int64_t(nv) * len + int64_t(nv) * nv <= lds_doubles;
  if (fits) {
    A = zsm;
    J = zsm + nv * len;
    for (int e = tid; e < nv * len; e += ZBT) {
      const int v = e / len, k = e % len;
      A[e] = rows ? Th[v * C + k] : Th[k * C + v];
    }
    vs = len;
    es = 1;
  } else {
    // the next kernel reads Theta itself again: rotate a copy, in L4, which
    // is free until the kept vectors are written over it (after the norms)
    A = Z.L4 + int64_t(s) * Z.bigcap;
    J = Jm;
    for (int e = tid; e < nv * len; e += ZBT) {
      const int v = e / len, k = e % len;
      A[e] = rows ? Th[v * C + k] : Th[k * C + v];
    }
    vs = len;
    es = 1;
  }
  __syncthreads();
  const int nsw = block_jacobi(A, vs, es, nv, len, J, Z.jtol, Z.jfloor, 40, flag, red);
  block_norms_sorted(A, vs, es, nv, len, S, ord);
  for (int m = tid; m < nv; m += ZBT) Sout[m] = S[ord[m]];
  __syncthreads();
  zip_keep(Z, s, zd, nv, Sout, ord, J, 1, nv, nsw);
}

// The small-order branch of k_zip_beig (nv <= 16): the scaled Gram into a
// 16 x 17 LDS block, all eigenpairs by wave_jacobi16, the values sorted
// descending into Sout, the rank rule, the kept vectors into Fv.
__device__ __forceinline__ void zip_beig_small(const ZipArgs& Z, int s, int* zd, int nv, const double* G, double gsc,
                                            double* Sout, double* Fv, double* zsm, double* scr, int* cs) {
  const int tid = threadIdx.x;
  double* Aj = zsm;
  double* Vj = zsm + 272;
  int* part = cs;
  int* ord = cs + 16;
  const int c = tid & 15, q = tid >> 4;
  const double gs = 1.0 / gsc;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = q + 4 * t;
    Aj[r * 17 + c] = (r < nv && c < nv) ? G[r * nv + c] * gs : 0.0;
  }
  const int nsw = wave_jacobi16(Aj, Vj, nv, scr, part);
  if (tid < nv) {
    const double li = Aj[tid * 18];
    int rank = 0;
    for (int j = 0; j < nv; ++j) rank += sorts_before(Aj[j * 18], j, li, tid) ? 1 : 0;
    ord[rank] = tid;
    Sout[rank] = sqrt(fmax(li * gsc, 0.0));
  }
  __syncthreads();
  int split = 0;
  int Dn = rank_rule(Sout, nv, Z.chi_m, Z.eps, Z.tau, &split);
  const bool bad = Dn < 1;
  if (bad) Dn = 1;
  for (int e = tid; e < nv * Dn; e += 64) Fv[e] = Vj[(e / Dn) * 17 + ord[e % Dn]];
  if (Z.flop_ctr && tid == 0) {
    const double n = nv, D = Dn;
    const double f = 4.0 / 3.0 * n * n * n + 2.0 * D * n * n + 7.0 * D * n + 12.0 * D * D * n;
    atomicAdd(Z.flop_ctr + (s & 63), (unsigned long long)f);
  }
  if (tid == 0) {
    zd[8] = Dn;
    atomicMax(&Z.sweeps_max[1], nsw);
    const uint32_t f = (bad ? 1u : 0u) | (split ? 2u : 0u) | (nsw >= 40 ? 8u : 0u);
    if (f) atomicOr(&Z.flags[s], f);
  }
}

// Dynamic LDS of k_zip_beig: the eigenvectors and the orthogonalisation's
// triangle at row stride ys, and at least the two 16 x 17 blocks of the
// small-order path.
static inline size_t beig_lds_bytes(int ys) {
  const size_t d = size_t(64 + ys) * ys;
  return (d > 544 ? d : 544) * sizeof(double);
}

// Families of at most ZBIG vectors when the rank rule allows the Gram route:
// leading eigenpairs of the PSD Gram (eigenvalues S^2) in one wavefront.  The
// Gram is scaled by its largest diagonal entry.  Orders up to 16 take every
// eigenpair by Jacobi rotations.  Larger ones compute only the
// min(nv, chi_m + 1) largest eigenvalues (all the rank rule reads) and the
// vectors it keeps; the reflectors of the tridiagonal reduction overwrite the
// Gram and the kept vectors sit in LDS (row stride eig_ys) before they are
// copied to Fv.
// The order-17-and-up branch of k_zip_beig: Householder reduction, the
// leading eigenvalues by multisection, the rank rule, the kept vectors by
// inverse iteration and the back-transformation, copied to Fv.
__device__ __forceinline__ void zip_beig_large(const ZipArgs& Z, int s, int* zd, int nv, double* G, double gsc,
                                            double* Sout, double* Fv, double* zsm, double* scr, double* lam,
                                            int* cs) {
  const int tid = threadIdx.x;
  double* vw = scr;
  double* tri = scr + 128;
  double* xs = scr + 256;  // 64 * SP
  double* de = scr + 256;
  double* rk = scr + 512;
  static_assert(256 + 64 * SP <= 512, "bisection points overlap rk");
  double dr, er, br;
  wave_tridiag(G, 1.0 / gsc, nv, vw, G, dr, er, br);
  const int K = nv < Z.chi_m + 1 ? nv : Z.chi_m + 1;
  const double nrm = wave_tri_topk(dr, er, nv, K, tri, xs, cs, lam);
  if (tid < K) Sout[tid] = sqrt(fmax(lam[tid] * gsc, 0.0));
  __syncthreads();
  int split = 0;
  int Dn = rank_rule(Sout, nv, Z.chi_m, Z.eps, Z.tau, &split);
  const bool bad = Dn < 1;
  if (bad) Dn = 1;
  const int ys = Z.eig_ys;
  wave_tri_vectors(dr, er, nv, Dn, nrm, lam, de, zsm, ys, zsm + 64 * ys, rk, Z.Jm + int64_t(s) * Z.jcap);
  wave_tri_backtransform(G, br, nv, Dn, zsm, ys, scr);
  if (Z.flop_ctr && tid == 0) {
    // algorithmic flops: Householder reduction 4n^3/3, back-transform 2Dn^2,
    // factorisation and two inverse-iteration solves 7Dn, three Cholesky-QR
    // passes 12D^2n
    const double n = nv, D = Dn;
    const double f = 4.0 / 3.0 * n * n * n + 2.0 * D * n * n + 7.0 * D * n + 12.0 * D * D * n;
    atomicAdd(Z.flop_ctr + (s & 63), (unsigned long long)f);
  }
  for (int e = tid; e < nv * Dn; e += 64) Fv[e] = zsm[(e / Dn) * ys + e % Dn];
  if (tid == 0) {
    zd[8] = Dn;
    atomicMax(&Z.sweeps_max[1], 1);
    const uint32_t f = (bad ? 1u : 0u) | (split ? 2u : 0u);
    if (f) atomicOr(&Z.flags[s], f);
  }
}

// (at most 256 registers: two wavefronts per SIMD, the launch's 2048
// problems resident at once)
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_zip_beig(ZipArgs Z, int x, int y) {
  extern __shared__ double zsm[];  // 64 * eig_ys vectors, then eig_ys^2 for the orthogonalisation
  // one 16-byte aligned block for the phases' scratch: the broadcast vectors
  // of the reduction, the tridiagonal and the bisection points, then the
  // factorisation's rows (over the dead points), and (once those are dead)
  // the staged reflectors
  __shared__ __attribute__((aligned(16))) double scr[576];
  __shared__ double lam[64];
  __shared__ int cs[64 * SP];
  const int s = blockIdx.x, tid = threadIdx.x;
  int* zd = Z.zdim + int64_t(s) * 12;
  const int nv = zd[7];
  if (nv > ZBIG) return;  // k_zip_bbig takes it
  const unsigned long long w0 = win_open(Z.win);
  double* G = Z.Gm + int64_t(s) * Z.bigcap;
  double* Sout = Z.zS + int64_t(s) * 1024;
  const double gd = wave_max(tid < nv ? G[tid * nv + tid] : 0.0);
  const double gsc = gd > 0.0 ? gd : 1.0;
  double* Fv = Z.L4 + int64_t(s) * Z.bigcap;  // L4 is dead after kernel a
  if (nv <= 16)
    zip_beig_small(Z, s, zd, nv, G, gsc, Sout, Fv, zsm, scr, cs);
  else
    zip_beig_large(Z, s, zd, nv, G, gsc, Sout, Fv, zsm, scr, lam, cs);
  win_close(Z.win, w0);
}

// Decomposition of the Gram blocks larger than ZBIG (FP32 mode) with the
// whole 512-thread workgroup; matrix and eigenvectors in LDS when they fit.
__global__ __launch_bounds__(ZNT) void k_zip_bbig(ZipArgs Z, int x, int y, int lds_doubles) {
  extern __shared__ double zsm[];
  __shared__ int ord[1024];
  __shared__ double red[16];
  const int s = blockIdx.x, tid = threadIdx.x;
  int* zd = Z.zdim + int64_t(s) * 12;
  const int nv = zd[7];
  if (nv <= ZBIG) return;
  double* G = Z.Gm + int64_t(s) * Z.bigcap;
  double* Jm = Z.Jm + int64_t(s) * Z.jcap;
  double* Sout = Z.zS + int64_t(s) * 1024;
  const int nw = ZNT / 64;
  const int small = 3 * nv + 2 * nw * nv;  // d, e, beta, per-wavefront (d, e)
  const bool fits = 2 * int64_t(nv) * nv + small <= lds_doubles;
  double* dv = zsm;
  double* dw = zsm + 3 * nv;
  double* A = fits ? zsm + small : G;
  double* Zm = fits ? zsm + small + nv * nv : Jm;
  if (fits)
    for (int e = tid; e < nv * nv; e += ZNT) A[e] = G[e];
  __syncthreads();
  const int fail = block_sym_eig(A, nv, Zm, dv, dv + nv, dv + 2 * nv, dw, red);
  for (int v = tid; v < nv; v += ZNT) {
    const double lv = dv[v];
    int rk = 0;
    for (int u = 0; u < nv; ++u)
      if (sorts_before(dv[u], u, lv, v)) ++rk;
    ord[rk] = v;
  }
  __syncthreads();
  for (int m = tid; m < nv; m += ZNT) Sout[m] = sqrt(fmax(dv[ord[m]], 0.0));
  __syncthreads();
  zip_keep(Z, s, zd, nv, Sout, ord, Zm, 1, nv, fail ? 40 : 1);
}

// ---------------------------------------------------------------------------
// Large families on the Gram route: block subspace iteration
// ---------------------------------------------------------------------------
// The K = min(nv, chi_m + 1) largest eigenpairs of the PSD Gram G (order
// nv > ZBIG) by subspace iteration with Rayleigh-Ritz (Saad, "Numerical
// Methods for Large Eigenvalue Problems", Sec. 5.2) on a block of SB vectors,
// every product on the FP64 matrix cores (block_gemm512):
//   Y = G X;  H = X^T Y;  H = V diag(theta) V^T (cyclic Jacobi);
//   U = X V (Ritz vectors), P = Y V (= G U);  stop when every ||P_j -
//   theta_j U_j|| (j < K) is below tol theta_1;  else X <- orth(P
//   diag(1 / theta)) (the columns near U, so Cholesky QR is well conditioned).
// The start is the columns of G at its SB largest diagonal entries.  Block
// vectors (nv x SB, row-major) live in the sweep's Jm scratch.
constexpr int SB = 64;
constexpr int CHEB = 4;  // degree of the subspace iteration's Chebyshev filter
static_assert(CHEB % 3 == 1, "the filter's buffer rotation ends in Y for CHEB = 1 (mod 3)");

// Cyclic Jacobi on the symmetric n x n A (n <= 64, LDS, row stride 65) by a
// 512-thread workgroup: the round-robin order gives 32 disjoint rotations per
// round, applied as A <- J^T A J in one pass over 2 x 2 blocks and V <- V J
// (Golub and Van Loan, Sec. 8.5, the symmetric Schur rotation).  V starts as
// the identity.  Returns the number of sweeps.
__device__ int block_jacobi_sym64(double* A, double* V, int n, double* cs, int* any) {
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += ZNT) {
    const int i = e >> 6, j = e & 63;
    V[i * 65 + j] = i == j ? 1.0 : 0.0;
    if (i >= n || j >= n) A[i * 65 + j] = i == j ? 0.0 : 0.0;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    if (tid == 0) *any = 0;
    __syncthreads();
    for (int rnd = 0; rnd < 63; ++rnd) {
      if (tid < 32) {
        int i, j;
        if (tid == 0) {
          i = 63;
          j = rnd;
        } else {
          i = rnd + tid;
          i = i >= 63 ? i - 63 : i;
          j = rnd - tid + 63;
          j = j >= 63 ? j - 63 : j;
        }
        const int p = i < j ? i : j, q = i < j ? j : i;
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double app = A[p * 65 + p], aqq = A[q * 65 + q], apq = A[p * 65 + q];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq)) && fabs(apq) > 1e-300) {
            const double zeta = (aqq - app) / (2.0 * apq);
            const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = c * t;
            *any = 1;
          }
        }
        cs[4 * tid] = c;
        cs[4 * tid + 1] = sn;
        reinterpret_cast<int*>(cs)[8 * tid + 4] = p;
        reinterpret_cast<int*>(cs)[8 * tid + 5] = q;
      }
      __syncthreads();
      // A <- J^T A J by 2 x 2 blocks: the round's pairs partition the indices,
      // so each element lies in one (row pair, column pair) block; per block
      // the column rotation, then the row rotation.  V <- V J alongside.
      for (int e = tid; e < 32 * 32; e += ZNT) {
        const int k1 = e >> 5, k2 = e & 31;
        const double c1 = cs[4 * k1], s1 = cs[4 * k1 + 1], c2 = cs[4 * k2], s2 = cs[4 * k2 + 1];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = reinterpret_cast<const int*>(cs)[8 * k1 + 4], q1 = reinterpret_cast<const int*>(cs)[8 * k1 + 5];
        const int p2 = reinterpret_cast<const int*>(cs)[8 * k2 + 4], q2 = reinterpret_cast<const int*>(cs)[8 * k2 + 5];
        double xpp = A[p1 * 65 + p2], xpq = A[p1 * 65 + q2], xqp = A[q1 * 65 + p2], xqq = A[q1 * 65 + q2];
        if (s2 != 0.0) {
          const double app = xpp, apq = xpq, aqp = xqp, aqq = xqq;
          xpp = c2 * app - s2 * apq;
          xpq = s2 * app + c2 * apq;
          xqp = c2 * aqp - s2 * aqq;
          xqq = s2 * aqp + c2 * aqq;
        }
        if (s1 != 0.0) {
          A[p1 * 65 + p2] = c1 * xpp - s1 * xqp;
          A[q1 * 65 + p2] = s1 * xpp + c1 * xqp;
          A[p1 * 65 + q2] = c1 * xpq - s1 * xqq;
          A[q1 * 65 + q2] = s1 * xpq + c1 * xqq;
        } else {
          A[p1 * 65 + p2] = xpp;
          A[q1 * 65 + p2] = xqp;
          A[p1 * 65 + q2] = xpq;
          A[q1 * 65 + q2] = xqq;
        }
      }
      for (int e = tid; e < 32 * 64; e += ZNT) {
        const int k = e >> 6, r = e & 63;
        const double c = cs[4 * k], sn = cs[4 * k + 1];
        if (sn == 0.0) continue;
        const int p = reinterpret_cast<const int*>(cs)[8 * k + 4], q = reinterpret_cast<const int*>(cs)[8 * k + 5];
        const double vp = V[r * 65 + p], vq = V[r * 65 + q];
        V[r * 65 + p] = c * vp - sn * vq;
        V[r * 65 + q] = sn * vp + c * vq;
      }
      __syncthreads();
    }
    const int a = *any;
    __syncthreads();
    if (!a) break;
  }
  return sweep;
}

// A deterministic pseudo-random value in [-1, 1) from two indices.
__device__ __forceinline__ double hash_unit(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return double(h) * (2.0 / 4294967296.0) - 1.0;
}

// Elementwise pass over [0, n) by a ZNT-thread workgroup: a thread takes EU
// elements per step and evaluates all of them (ld(e), whose loads read at
// index e; indices past n read element 0) before storing any (st(e, v)), so
// a step's loads are in flight together instead of each waiting behind the
// previous element's store.
template <int EU = 8, class LD, class ST>
__device__ __forceinline__ void block_stream(int n, LD ld, ST st) {
  for (int e0 = threadIdx.x; e0 < n; e0 += EU * ZNT) {
    double v[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) v[u] = ld(e0 + u * ZNT < n ? e0 + u * ZNT : 0);
#pragma unroll
    for (int u = 0; u < EU; ++u)
      if (e0 + u * ZNT < n) st(e0 + u * ZNT, v[u]);
  }
}

// X (nv x SB, row-major) <- an orthonormal basis of the span of Z (same
// shape, destroyed) by Cholesky QR twice with column equilibration; a column
// whose pivot shows it dependent on the previous ones is replaced by a hashed
// vector before the second pass.  R, Ri: SB x 65 LDS, red: 16 doubles.
__device__ void block_cholqr2(double* Z, double* X, int nv, double* R, double* Ri, double* gl, double* red, int* dead,
                              unsigned seed) {
  const int tid = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    // S = Z^T Z into R
    block_gemm512<false, false>(
        SB, SB, nv, [&](int m, int k) { return Z[k * SB + m]; }, [&](int k, int n) { return Z[k * SB + n]; },
        [&](int m, int n, double v) { R[m * 65 + n] = v; }, gl);
    // equilibrate: D^-1/2 S D^-1/2, and the Cholesky factor of that
    __shared__ double dsc[SB];
    if (tid < SB) {
      const double dd = R[tid * 65 + tid];
      dsc[tid] = dd > 0.0 ? 1.0 / sqrt(dd) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < SB * SB; e += ZNT) {
      const int i = e >> 6, j = e & 63;
      R[i * 65 + j] *= dsc[i] * dsc[j];
    }
    if (tid == 0) *dead = 0;
    __syncthreads();
    // right-looking Cholesky, R upper triangular in the upper part
    for (int j = 0; j < SB; ++j) {
      __shared__ double piv;
      if (tid == 0) {
        const double a = R[j * 65 + j];
        if (!(a > 1e-16)) {  // dependent (or zero) column: below the rounding of S
          piv = 0.0;
          *dead = 1;
        } else {
          piv = sqrt(a);
        }
      }
      __syncthreads();
      const double pj = piv;
      if (pj == 0.0) {
        for (int k = tid; k < SB; k += ZNT) R[j * 65 + k] = k == j ? 1.0 : 0.0;
        for (int k = tid; k < SB; k += ZNT) if (k > j) R[k * 65 + j] = 0.0;
        __syncthreads();
        if (tid == 0) dsc[j] = -dsc[j] - 1.0;  // marks the column (dsc >= 0 otherwise)
        __syncthreads();
        continue;
      }
      for (int k = j + tid; k < SB; k += ZNT) R[j * 65 + k] = k == j ? pj : R[j * 65 + k] / pj;
      __syncthreads();
      for (int e = tid; e < (SB - j - 1) * (SB - j - 1); e += ZNT) {
        const int a = j + 1 + e / (SB - j - 1), b = j + 1 + e % (SB - j - 1);
        if (b >= a) R[a * 65 + b] -= R[j * 65 + a] * R[j * 65 + b];
      }
      __syncthreads();
    }
    // R^-1 into Ri (column j by back substitution in thread j), then
    // X = Z D^-1/2 R^-1 on the matrix cores
    if (tid < SB) {
      const int j = tid;
      for (int i = SB - 1; i >= 0; --i) {
        double y = 0.0;
        if (i <= j) {
          y = i == j ? 1.0 : 0.0;
          for (int k = i + 1; k <= j; ++k) y = fma(-R[i * 65 + k], Ri[k * 65 + j], y);
          y /= R[i * 65 + i];
        }
        Ri[i * 65 + j] = y;
      }
    }
    __syncthreads();
    block_gemm512<true, false>(
        nv, SB, SB,
        [&](int m, int k) {
          const double dk = dsc[k];
          return dk >= 0.0 ? Z[m * SB + k] * dk : 0.0;
        },
        [&](int k, int n) { return Ri[k * 65 + n]; }, [&](int m, int n, double v) { X[m * SB + n] = v; }, gl);
    if (pass == 0) {
      // dead columns get a hashed vector; the second pass orthonormalises
      block_stream(
          nv * SB,
          [&](int e) {
            const int j = e % SB;
            return dsc[j] < 0.0 ? hash_unit(seed + unsigned(j), unsigned(e / SB)) : X[e];
          },
          [&](int e, double v) { Z[e] = v; });
      __syncthreads();
    }
    __syncthreads();
  }
  (void)red;
}

__global__ __launch_bounds__(ZNT) void k_zip_bsub(ZipArgs Z, int x, int y) {
  extern __shared__ double zsm[];
  double* gl = zsm;                 // GEMM_LDS
  double* H = zsm + GEMM_LDS;       // SB x 65: H, then the Cholesky factor
  double* Vv = H + SB * 65;         // SB x 65: Jacobi vectors
  __shared__ double cs[4 * 32 + 8];
  __shared__ double th[SB], rn[SB], red[16];
  __shared__ int ord[SB], flag[4];
  __shared__ int jsel[SB];
  const int s = blockIdx.x, tid = threadIdx.x;
  int* zd = Z.zdim + int64_t(s) * 12;
  const int nv = zd[7];
  if (nv <= ZBIG) return;
  const unsigned long long w0 = win_open(Z.win_b);
  const double* G = Z.Gm + int64_t(s) * Z.bigcap;
  double* X = Z.Jm + int64_t(s) * Z.jcap;
  double* Y = X + int64_t(nv) * SB;
  double* U = Y + int64_t(nv) * SB;
  double* P = U + int64_t(nv) * SB;
  double* Sout = Z.zS + int64_t(s) * 1024;
  const int K = nv < Z.chi_m + 1 ? nv : Z.chi_m + 1;
  // start: the columns of G at its SB largest diagonal entries (ties by
  // index); the diagonal is staged in the GEMM area, free until the first
  // product (nv <= 1024 < GEMM_LDS)
  for (int i = tid; i < nv; i += ZNT) gl[i] = G[int64_t(i) * nv + i];
  __syncthreads();
  for (int i = tid; i < nv; i += ZNT) {
    const double gi = gl[i];
    int rank = 0;
    for (int j = 0; j < nv; ++j) rank += sorts_before(gl[j], j, gi, i) ? 1 : 0;
    if (rank < SB) jsel[rank] = i;
  }
  __syncthreads();
  block_stream(
      nv * SB, [&](int e) { return G[int64_t(e / SB) * nv + jsel[e % SB]]; }, [&](int e, double v) { Y[e] = v; });
  __syncthreads();
  block_cholqr2(Y, X, nv, H, Vv, gl, red, &flag[0], 0x1234u);
  const double tol = Z.sub_tol;
  int it = 0, conv = 0, n_gemm = 0;
  const int maxit = 48;
  for (; it < maxit; ++it) {
    ++n_gemm;
    // Y = G X
    block_gemm512<true, false>(
        nv, SB, nv, [&](int m, int k) { return G[int64_t(m) * nv + k]; }, [&](int k, int n) { return X[k * SB + n]; },
        [&](int m, int n, double v) { Y[m * SB + n] = v; }, gl);
    // H = X^T Y, symmetrised
    block_gemm512<false, false>(
        SB, SB, nv, [&](int m, int k) { return X[k * SB + m]; }, [&](int k, int n) { return Y[k * SB + n]; },
        [&](int m, int n, double v) { H[m * 65 + n] = v; }, gl);
    for (int e = tid; e < SB * SB; e += ZNT) {
      const int i = e >> 6, j = e & 63;
      if (i < j) {
        const double a = 0.5 * (H[i * 65 + j] + H[j * 65 + i]);
        H[i * 65 + j] = a;
        H[j * 65 + i] = a;
      }
    }
    __syncthreads();
    block_jacobi_sym64(H, Vv, SB, cs, &flag[1]);
    if (tid < SB) {
      const double li = H[tid * 65 + tid];
      int rank = 0;
      for (int j = 0; j < SB; ++j) rank += sorts_before(H[j * 65 + j], j, li, tid) ? 1 : 0;
      ord[rank] = tid;
      th[rank] = li;
    }
    __syncthreads();
    // U = X V, P = Y V (columns in descending order of theta)
    block_gemm512<true, false>(
        nv, SB, SB, [&](int m, int k) { return X[m * SB + k]; }, [&](int k, int n) { return Vv[k * 65 + ord[n]]; },
        [&](int m, int n, double v) { U[m * SB + n] = v; }, gl);
    block_gemm512<true, false>(
        nv, SB, SB, [&](int m, int k) { return Y[m * SB + k]; }, [&](int k, int n) { return Vv[k * 65 + ord[n]]; },
        [&](int m, int n, double v) { P[m * SB + n] = v; }, gl);
    // residual norms of the K leading Ritz pairs
    if (tid < SB) rn[tid] = 0.0;
    __syncthreads();
    {
      const int j = tid & 63;
      double acc = 0.0;
      if (j < K) {
        // eight rows' loads in flight per step, accumulated in row order
        constexpr int RS = ZNT / 64;
        int r = tid >> 6;
        for (; r + 7 * RS < nv; r += 8 * RS) {
          double dv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) dv[u] = P[(r + u * RS) * SB + j] - th[j] * U[(r + u * RS) * SB + j];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = fma(dv[u], dv[u], acc);
        }
        for (; r < nv; r += RS) {
          const double d = P[r * SB + j] - th[j] * U[r * SB + j];
          acc = fma(d, d, acc);
        }
      }
      atomicAdd(&rn[j], acc);
    }
    __syncthreads();
    double worst = 0.0;
    for (int j = 0; j < K; ++j) worst = fmax(worst, sqrt(rn[j]));
    const double t1 = th[0] > 0.0 ? th[0] : 1.0;
    if (worst <= tol * t1) {
      conv = 1;
      break;
    }
    if (it + 1 == maxit) break;
    const double c_lo = th[SB - 1];
    if (c_lo > 1e-12 * t1 && t1 > 1.05 * c_lo && th[K - 1] >= 1e-2 * t1) {
      // next block: a Chebyshev filter of degree CHEB applied to the Ritz
      // vectors U (G U = P is at hand): T_CHEB((G - cen) / hw) damps the
      // interval [0, c_lo] below the block's smallest Ritz value and grows
      // the wanted end; the three-term recurrence is scaled so that the
      // component at the largest Ritz value t1 stays near one (no overflow).
      // One orthonormalisation and Rayleigh-Ritz step per CHEB products.
      // Only where the wanted Ritz values span at most two decades: the
      // filter grows the largest wanted component over the smallest by up to
      // (t1 / theta_K)^CHEB, and a wider span would leave the smallest ones
      // below the rounding of the block before it is orthonormalised again.
      const double hw = 0.5 * c_lo, cen = 0.5 * c_lo;
      const double sig1 = hw / (t1 - cen);
      double sig = sig1;
      block_stream(
          nv * SB, [&](int e) { return (P[e] - cen * U[e]) * (sig1 / hw); }, [&](int e, double v) { Y[e] = v; });
      __syncthreads();
      double *pa = U, *pb = Y, *pt = X;  // steps j-1, j and the product buffer
      for (int deg = 2; deg <= CHEB; ++deg) {
        const double sn = 1.0 / (2.0 / sig1 - sig);
        block_gemm512<true, false>(
            nv, SB, nv, [&](int m, int k) { return G[int64_t(m) * nv + k]; },
            [&](int k, int n) { return pb[k * SB + n]; }, [&](int m, int n, double v) { pt[m * SB + n] = v; }, gl);
        __syncthreads();
        const double ca = 2.0 * sn / hw, cb = sig * sn;
        block_stream(
            nv * SB, [&](int e) { return ca * (pt[e] - cen * pb[e]) - cb * pa[e]; },
            [&](int e, double v) { pt[e] = v; });
        __syncthreads();
        double* q = pa;
        pa = pb;
        pb = pt;
        pt = q;
        sig = sn;
        ++n_gemm;
      }
      // CHEB = 1 (mod 3): the filtered block is back in Y
      block_cholqr2(Y, X, nv, H, Vv, gl, red, &flag[0], 0x51ED27u + unsigned(it) * 977u);
    } else {
      // no interval to damp (a flat or rank-deficient block): a power step,
      // P diag(1 / theta), orthonormalised
      const double fl = 1e-15 * t1;
      block_stream(
          nv * SB, [&](int e) { return P[e] / fmax(th[e % SB], fl); }, [&](int e, double v) { Y[e] = v; });
      __syncthreads();
      block_cholqr2(Y, X, nv, H, Vv, gl, red, &flag[0], 0x51ED27u + unsigned(it) * 977u);
    }
  }
  // the rank rule on sqrt(theta), the kept Ritz vectors into Fv
  for (int j = tid; j < SB; j += ZNT) Sout[j] = sqrt(fmax(th[j], 0.0));
  __syncthreads();
  int split = 0;
  int Dn = rank_rule(Sout, nv, Z.chi_m, Z.eps, Z.tau, &split);
  const bool bad = Dn < 1;
  if (bad) Dn = 1;
  double* Fv = Z.L4 + int64_t(s) * Z.bigcap;
  block_stream(
      nv * Dn, [&](int e) { return U[(e / Dn) * SB + e % Dn]; }, [&](int e, double v) { Fv[e] = v; });
  if (Z.flop_b && tid == 0) {
    // algorithmic flops: 2 nv^2 SB per block product by G (one per Ritz step
    // and CHEB - 1 more per filter); per Ritz step the projection and
    // rotations 6 nv SB^2 and Cholesky QR twice 8 nv SB^2
    const double n = nv, b = SB;
    const double f = double(n_gemm) * 2.0 * n * n * b + double(it + 1) * 14.0 * n * b * b;
    atomicAdd(Z.flop_b + (s & 63), (unsigned long long)f);
  }
  if (tid == 0) {
    zd[8] = Dn;
    atomicMax(&Z.sweeps_max[1], it + 1);
    const uint32_t f = (bad ? 1u : 0u) | (split ? 2u : 0u) | (conv ? 0u : 8u);
    if (f) atomicOr(&Z.flags[s], f);
  }
  win_close(Z.win_b, w0);
}

// (at most 80 registers: six wavefronts per SIMD)
__global__ __launch_bounds__(ZNT) __attribute__((amdgpu_waves_per_eu(6))) void k_zip_c(ZipArgs Z, int x, int y) {
  __shared__ double gst[GEMM_LDS];
  __shared__ double red[8];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int Lx = Z.Lx, cur = y & 1;
  double* Mnew = (cur ? Z.mps0 : Z.mps1) + (int64_t(s) * Lx + x) * Z.mcap;
  int* mn = Z.mdim + ((int64_t(s) * 2 + (cur ^ 1)) * Lx + x) * 3;
  const int* zd = Z.zdim + int64_t(s) * 12;
  const int R = zd[0], C = zd[1], nu = zd[2], sD = zd[3], aR = zd[4], wR = zd[5];
  const bool rows = zd[6] != 0;
  const int nv = zd[7];
  const double* Th = Z.Th + int64_t(s) * Z.bigcap;
  double* Kp = Z.K + int64_t(s) * Z.kcap;
  int* kd = Z.kdim + int64_t(s) * 3;
  int Dn = 1;
  if (x + 1 < Lx) {
    Dn = zd[8];
    const int D = Dn;
    const double* Fv = Z.L4 + int64_t(s) * Z.bigcap;
    const double* Sv = Z.zS + int64_t(s) * 1024;
    if (rows) {
      for (int e = tid; e < R * D; e += ZNT) Mnew[e] = Fv[e];
      block_gemm512(
          D, C, R, [&](int m, int k) { return Fv[k * D + m]; }, [&](int k, int n) { return Th[k * C + n]; },
          [&](int m, int n, double v) { Kp[m * C + n] = v; }, gst);
    } else {
      block_gemm512(
          R, D, C, [&](int m, int k) { return Th[m * C + k]; }, [&](int k, int n) { return Fv[k * D + n]; },
          [&](int m, int n, double v) {
            const double sv = Sv[n];
            Mnew[m * D + n] = sv > 0.0 ? v / sv : 0.0;
          },
          gst);
      for (int e = tid; e < D * C; e += ZNT) Kp[e] = Sv[e / C] * Fv[(e % C) * D + e / C];
    }
    (void)nv;
    if (tid == 0) {
      kd[0] = Dn;
      kd[1] = aR;
      kd[2] = wR;
    }
  } else {
    for (int e = tid; e < R; e += ZNT) Mnew[e] = Th[e * C];
  }
  if (tid == 0) {
    mn[0] = nu;
    mn[1] = sD;
    mn[2] = Dn;
  }
  __syncthreads();
  const int tot = R * Dn;
  double m = 0.0;
  for (int e = tid; e < tot; e += ZNT) m = fmax(m, fabs(Mnew[e]));
  m = block_max_abs_reduce(m, red);
  const bool zero = !(m > 0.0) || !isfinite(m);
  const double c = zero ? 1.0 : m;
  for (int e = tid; e < tot; e += ZNT) Mnew[e] /= c;
  if (tid == 0) {
    Z.logm[s] += log(c);
    if (zero) atomicOr(&Z.flags[s], 1u);
  }
}

__global__ void k_finish(SweepArgs A, ZipArgs Z, double* logp) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_sweeps) return;
  const int cur = Z.Ly & 1;
  double v[MAXCHI * 2];
  int nv = 1;
  v[0] = 1.0;
  bool ok = true;
  for (int x = 0; x < Z.Lx && ok; ++x) {
    const int* md = Z.mdim + ((int64_t(s) * 2 + cur) * Z.Lx + x) * 3;
    const double* M = (cur ? Z.mps1 : Z.mps0) + (int64_t(s) * Z.Lx + x) * Z.mcap;
    const int aL = md[0], sd = md[1], aR = md[2];
    if (aL != nv || sd != 1 || aR > MAXCHI * 2) {
      ok = false;
      break;
    }
    double w[MAXCHI * 2];
    for (int j = 0; j < aR; ++j) {
      double acc = 0.0;
      for (int i = 0; i < aL; ++i) acc += v[i] * M[i * aR + j];
      w[j] = acc;
    }
    for (int j = 0; j < aR; ++j) v[j] = w[j];
    nv = aR;
  }
  double lsum = Z.logm[s];
  for (int b = 0; b < A.n_bonds; ++b) lsum += A.logb[int64_t(s) * A.n_bonds + b];
  for (int i = 0; i < A.n_sites; ++i) lsum += A.logs[int64_t(s) * A.n_sites + i];
  const double z = (ok && nv == 1) ? v[0] : 0.0;
  const int item = A.items[s / A.n_cosets], c = s % A.n_cosets;
  double out;
  uint32_t f = A.flags[s] | Z.flags[s];
  bool inconsistent = false;
  if (A.n_inc > 0) {
    const uint8_t* bits = A.synd + A.synd_off[item] + A.inc0;
    for (int k = 0; k < A.n_inc; ++k) inconsistent |= (bits[k] & 1) != 0;
  }
  if (inconsistent) {
    out = -INFINITY;
    f = 32u;
  } else if (z > 0.0 && isfinite(z) && isfinite(lsum)) {
    out = lsum + log(z);
  } else if (A.wht && z < 0.0 && isfinite(z) && isfinite(lsum)) {
    // signed network: log |Z| here, the sign for k_wht_combine
    out = lsum + log(-z);
    f |= WHT_NEG;
  } else {
    out = __longlong_as_double(0x7ff8000000000000LL);
    f |= 1u;
  }
  logp[int64_t(item) * 4 + c] = out;
  A.flags[s] = f;
  if (c == 0)
    for (int k = A.n_cosets; k < 4; ++k) logp[int64_t(item) * 4 + k] = -INFINITY;
}

// Walsh-Hadamard form (paper Sec. 3.1): the two sweeps of an item are the
// signed networks Z_0 (the syndrome probability, positive) and Z_1 (the
// difference of the two cosets), k_finish left log |Z_b| in the coset slots
// and the sign of Z_b in WHT_NEG.  log p_{m,L} = log Z_0 + log1p((-1)^L r) -
// log 2 with r = Z_1 / Z_0.  A truncated Z_1 beyond Z_0 in magnitude, or a
// negative Z_0, is NUMERIC (NaN); equality gives -inf.
__global__ void k_wht_combine(int n_items, const int32_t* items, double* logp, uint32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const int item = items[i];
  uint32_t f0 = flags[int64_t(i) * 2], f1 = flags[int64_t(i) * 2 + 1];
  double* lp = logp + int64_t(item) * 4;
  const bool inc = ((f0 | f1) & 32u) != 0;
  if (!inc) {
    const double l0 = lp[0], l1 = lp[1];
    double p0, p1;
    if ((f0 & WHT_NEG) || isnan(l0) || isnan(l1) || !isfinite(l0)) {
      p0 = p1 = __longlong_as_double(0x7ff8000000000000LL);
    } else {
      const double r = ((f1 & WHT_NEG) ? -1.0 : 1.0) * exp(l1 - l0);
      p0 = l0 + log1p(r) - 0.69314718055994530942;
      p1 = l0 + log1p(-r) - 0.69314718055994530942;
    }
    if (isnan(p0) || isnan(p1)) {
      f0 |= 1u;
      f1 |= 1u;
    }
    lp[0] = p0;
    lp[1] = p1;
  }
  flags[int64_t(i) * 2] = f0 & ~WHT_NEG;
  flags[int64_t(i) * 2 + 1] = f1 & ~WHT_NEG;
}

__global__ void k_collect_flags(int n_items, int n_cosets, const int32_t* items, const uint32_t* sweep_flags,
                                uint32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  uint32_t f = 0;
  for (int c = 0; c < n_cosets; ++c) f |= sweep_flags[int64_t(i) * n_cosets + c];
  out[items[i]] = f;
}

__global__ void k_decode(int n_items, int n_cosets, const int32_t* items, const double* logp, double near_tie,
                         int32_t* coset, double* logratio, uint32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const int it = items[i];
  const double* lp = logp + int64_t(it) * 4;
  // a NaN (a value the contraction found non-positive) ranks below every
  // number; with every coset NaN the decision is coset 0 and the log-ratio NaN
  int best = -1;
  for (int c = 0; c < n_cosets; ++c)
    if (!isnan(lp[c]) && (best < 0 || lp[c] > lp[best])) best = c;
  double lr = __longlong_as_double(0x7ff8000000000000LL);
  if (best < 0) {
    best = 0;
  } else {
    double other = -INFINITY;
    for (int c = 0; c < n_cosets; ++c)
      if (c != best && lp[c] > other) other = lp[c];
    lr = lp[best] - other;
  }
  if (coset) coset[it] = best;
  if (logratio) logratio[it] = lr;
  if (flags && !(lr >= near_tie)) flags[it] |= 4u;
}

// Items whose decision is within the near-tie band (or not a number), for the
// FP64 re-sweep; the list order is arbitrary (the host sorts it).
__global__ void k_pick_ties(int n_items, const double* logratio, double near_tie, int32_t* list, int32_t* count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const double lr = logratio[i];
  if (!(lr >= near_tie)) list[atomicAdd(count, 1)] = i;
}

__global__ void k_gather_offsets(int n, const int32_t* items, const int64_t* offs, int64_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = offs[items[i]];
}

__global__ void k_gather_i32(int n, const int32_t* items, const int32_t* src, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = src[items[i]];
}

// Results of the re-sweep (row i of logp_sub, flags_sub) back to items[i].
__global__ void k_scatter_resweep(int n, const int32_t* items, const double* logp_sub, const uint32_t* flags_sub,
                                  double* logp, uint32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int it = items[i];
  for (int c = 0; c < 4; ++c) logp[int64_t(it) * 4 + c] = logp_sub[int64_t(i) * 4 + c];
  if (flags) flags[it] = flags_sub[i] | 16u;
}

// ---------------------------------------------------------------------------
// Gradient of the syndrome log-likelihood with respect to the rates (the
// Sec. 2.4 definition of p_{m,L}).  P(m) = sum_L p_{m,L} is affine in every
// rate p_i, since each mechanism enters every term of the sum once, as p_i
// or as 1 - p_i.  With P_c(m) the value at p_i = c (c = 0 or 1),
//   d log P(m) / d p_i = (P_c(m) / P(m) - 1) / (c - p_i).
// The rows of lp come in blocks of B items: block 0 holds the network at the
// given rates, block i + 1 the network with rate i set to c_i (the end of
// [0, 1] farther from p_i, so |c_i - p_i| >= 1/2).

// log sum_c exp(r[c]) over the coset columns.  A NaN column (a value the
// contraction found non-positive, below its own error) counts as zero; with
// every column NaN the result is NaN, or -inf with all_nan_zero.
__device__ double lse_cosets(const double* r, int nc, bool all_nan_zero = false) {
  double m = -INFINITY;
  int n_nan = 0;
  for (int c = 0; c < nc; ++c) {
    if (isnan(r[c])) ++n_nan;
    if (r[c] > m) m = r[c];
  }
  if (n_nan == nc) return all_nan_zero ? -INFINITY : NAN;
  if (m == -INFINITY) return m;
  double s = 0.0;
  for (int c = 0; c < nc; ++c)
    if (!isnan(r[c])) s += exp(r[c] - m);
  return m + log(s);
}

// term[s][i] = d log P(m_s) / d p_i for every item s < B and mechanism i < n.
// cp[2 i] = c_i, cp[2 i + 1] = p_i.  A changed network whose cosets are all
// found non-positive counts as zero; at the given rates that leaves log P
// NaN and so the item's derivatives.
__global__ void k_grad_terms(int B, int n, int nc, const double* lp, const double* cp, double* term) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(B) * n) return;
  const int s = int(idx / n), i = int(idx % n);
  const double base = lse_cosets(lp + int64_t(s) * 4, nc);
  const double var = lse_cosets(lp + (int64_t(i + 1) * B + s) * 4, nc, true);
  term[idx] = expm1(var - base) / (cp[2 * i] - cp[2 * i + 1]);
}

// loglik[s] = log P(m_s) at the given rates (nullable); flags[s] = the OR of
// the flags of item s's n + 1 contractions (nullable).
__global__ void k_grad_items(int B, int n, int nc, const double* lp, const uint32_t* fl, double* loglik,
                             uint32_t* flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  if (loglik) loglik[s] = lse_cosets(lp + int64_t(s) * 4, nc);
  if (flags) {
    uint32_t f = 0;
    for (int v = 0; v <= n; ++v) f |= fl[int64_t(v) * B + s];
    flags[s] = f;
  }
}

// grad[k] = sum over items s and the mechanisms i of rate k (rm[ptr[k] ..
// ptr[k + 1])) of term[s][i]: one workgroup of 256 per rate, a fixed
// summation order (strided partial sums, then a tree in LDS).
__global__ void __launch_bounds__(256) k_grad_reduce(int B, int n, const double* term, const int32_t* ptr,
                                                     const int32_t* rm, double* grad) {
  __shared__ double part[256];
  const int k = blockIdx.x, t = threadIdx.x;
  const int j0 = ptr[k], cnt = ptr[k + 1] - j0;
  const int64_t tot = int64_t(B) * cnt;
  double acc = 0.0;
  for (int64_t j = t; j < tot; j += 256) acc += term[(j / cnt) * n + rm[j0 + j % cnt]];
  part[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) grad[k] = part[0];
}

// total[0] = sum over items of log P(m_s) at the given rates (one workgroup,
// a fixed summation order).
__global__ void __launch_bounds__(256) k_grad_total(int B, int nc, const double* lp, double* total) {
  __shared__ double part[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int s = t; s < B; s += 256) acc += lse_cosets(lp + int64_t(s) * 4, nc);
  part[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  if (t == 0) total[0] = part[0];
}

// offs_all[v B + s] = offs[s] for the n_blocks blocks of B items.
__global__ void k_tile_offsets(int B, int n_blocks, const int64_t* offs, int64_t* offs_all) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < int64_t(B) * n_blocks) offs_all[idx] = offs[idx % B];
}

// Device wall-clock stamp, for timing that also works inside a captured graph
// (events recorded in a graph cannot be read back as elapsed times).
__global__ void k_stamp(unsigned long long* out) {
  if (threadIdx.x == 0) *out = wall_clock64();
}

__global__ void k_win_init(unsigned long long* win, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * 128) win[e] = (e & 127) < 64 ? ~0ull : 0ull;
}

// One workgroup per window (the last one also takes the stamps and counters):
// the window's span, added to its accumulator.
__global__ void k_timing_reduce(const unsigned long long* stamps, const unsigned long long* win, int n_cls_win,
                                int Lx, int Ly, int eig, const unsigned long long* ctr, double ms_per_tick,
                                double* acc) {
  const int w = blockIdx.x, l = threadIdx.x;
  const int n_win = n_cls_win + 3 * Lx * Ly;
  if (w < n_win) {
    // class windows, then per boundary-MPS step: small decomposition,
    // contraction, large decomposition (subspace iteration)
    const int kind = w < n_cls_win ? 0 : 1 + (w - n_cls_win) / (Lx * Ly);
    const int xy = (w - n_cls_win) % (Lx * Ly);
    if (kind == 1 && (!eig || xy % Lx + 1 >= Lx)) return;
    unsigned long long t0 = win[size_t(w) * 128 + l], t1 = win[size_t(w) * 128 + 64 + l];
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long u0 = __shfl_xor(t0, o, 64), u1 = __shfl_xor(t1, o, 64);
      t0 = u0 < t0 ? u0 : t0;
      t1 = u1 > t1 ? u1 : t1;
    }
    const int slot = kind == 0 ? 2 : (kind == 1 ? 5 : (kind == 2 ? 8 : 10));
    if (l == 0 && t1 > t0) atomicAdd(acc + slot, double(t1 - t0) * ms_per_tick);
    return;
  }
  unsigned long long b = ctr[l], f = ctr[65 + l], fa = ctr[129 + l], fb = ctr[193 + l];
  for (int o = 32; o > 0; o >>= 1) {
    b += __shfl_xor(b, o, 64);
    f += __shfl_xor(f, o, 64);
    fa += __shfl_xor(fa, o, 64);
    fb += __shfl_xor(fb, o, 64);
  }
  if (l == 0) {
    acc[0] += double(stamps[1] - stamps[0]) * ms_per_tick;
    acc[1] += double(stamps[2] - stamps[1]) * ms_per_tick;
    acc[4] += double(b);
    acc[7] += double(f);
    acc[9] += double(fa);
    acc[11] += double(fb);
  }
}

// Graph replay support: the captured sequence reads and writes only
// workspace buffers, filled and drained by these kernels outside it.
__global__ void k_gather_synd(int n, const int32_t* items, const uint8_t* synd, const int64_t* offs, int n_det,
                              int64_t stride, uint8_t* out) {
  const int i = blockIdx.y;
  const int64_t src = offs[items[i]];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_det; k += gridDim.x * blockDim.x)
    out[int64_t(i) * stride + k] = synd[src + k];
}

// Derived per-item bits: bit n_det + e of item i is the parity of
// rows[e] & (syndrome bits [src0, src0 + src_n) packed 64 to a word).  One
// workgroup of 256 per item; the packed syndrome goes through LDS.
__global__ __launch_bounds__(256) void k_ext_bits(int n, uint8_t* bits, int64_t stride, int n_det, int src0,
                                                  int src_n, int words, const uint64_t* rows, int n_ext) {
  __shared__ uint64_t mw[EXT_MAXW];
  const int i = blockIdx.x;
  uint8_t* b = bits + int64_t(i) * stride;
  for (int w = threadIdx.x; w < words; w += blockDim.x) {
    uint64_t v = 0;
    for (int k = 0; k < 64; ++k) {
      const int j = w * 64 + k;
      if (j < src_n) v |= uint64_t(b[src0 + j] & 1) << k;
    }
    mw[w] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n_ext; e += blockDim.x) {
    const uint64_t* r = rows + int64_t(e) * words;
    int par = 0;
    for (int w = 0; w < words; ++w) par ^= __popcll(r[w] & mw[w]) & 1;
    b[n_det + e] = uint8_t(par);
  }
}

__global__ void k_seq(int n, int32_t* items, int64_t* offs, int64_t stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    items[i] = i;
    offs[i] = int64_t(i) * stride;
  }
}

__global__ void k_zero_words(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_scatter_out(int n, const int32_t* items, const double* lp_local, const uint32_t* fl_local,
                              double* logp, uint32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int it = items[i];
  for (int c = 0; c < 4; ++c) logp[int64_t(it) * 4 + c] = lp_local[int64_t(i) * 4 + c];
  if (flags) flags[it] = fl_local[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Dynamic-LDS limits of the kernels that can need more than the default
// 64 KB, set once per device to the most any launch requests (static LDS
// included stays within the 160 KB of a workgroup).  Setting attributes is not
// allowed while a stream is being captured, so no launcher does it.
static inline size_t bsub_lds_bytes() { return size_t(GEMM_LDS + 2 * SB * 65) * sizeof(double); }

hipError_t set_kernel_lds_limits() {
  const int kmax = 64;  // gate rank x chi, checked by the host
  const int solve = 4 * kmax * (kmax + 1) * 8 + 2 * kmax * 8 + 32 + (2 * kmax + 4) * 4;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_solve<SNT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, solve);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_solve<SNT_BIG>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            solve);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_zip_b), hipFuncAttributeMaxDynamicSharedMemorySize,
                            18432 * 8);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_zip_bbig), hipFuncAttributeMaxDynamicSharedMemorySize,
                            19200 * 8);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_zip_bsub), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(bsub_lds_bytes()));
  return e;
}

void launch_init(int prec, const SweepArgs& A, const int32_t* init_dims, const int32_t* init_off,
                 const int32_t* bond_dim0, hipStream_t st) {
  dim3 g(A.n_sites, A.n_sweeps);
  if (prec == 0)
    hipLaunchKernelGGL(k_init_sites<double>, g, dim3(64), 0, st, A, init_dims, init_off);
  else
    hipLaunchKernelGGL(k_init_sites<float>, g, dim3(64), 0, st, A, init_dims, init_off);
  hipLaunchKernelGGL(k_init_bonds, dim3(A.n_sweeps), dim3(64), 0, st, A, bond_dim0);
}

void launch_onesite(int prec, const SweepArgs& A, const DevOneSite* ops, int n_ops, hipStream_t st) {
  if (n_ops <= 0) return;
  dim3 g(n_ops, A.n_sweeps);
  if (prec == 0)
    hipLaunchKernelGGL(k_onesite<double>, g, dim3(ET), 0, st, A, ops);
  else
    hipLaunchKernelGGL(k_onesite<float>, g, dim3(ET), 0, st, A, ops);
}

template <typename T>
static void gram_dispatch(const SweepArgs& A, const DevGate* gates, int n_g, int n_wide, int n_w64, double* gout,
                          int ncap, hipStream_t st) {
  // ncap <= 64 is checked by the host before any launch; Grams of up to 32
  // columns (three block pairs) and of 33 to 64 (ten) in separate launches,
  // the second over the leading n_wide gates (the only ones that can be wide)
  hipLaunchKernelGGL((k_gram2<T, 2>), dim3(2 * n_g, A.n_sweeps), dim3(64), 0, st, A, gates, n_g, gout, ncap, 0);
  if (ncap > 32 && n_wide > 0)
    hipLaunchKernelGGL((k_gram2<T, 4>), dim3(2 * n_wide, A.n_sweeps), dim3(64), 0, st, A, gates, n_g, gout,
                       ncap, 32);
  // 65 to 96 columns (physical dim 4 at chi up to 24): 21 block pairs
  if (ncap > 64 && n_w64 > 0)
    hipLaunchKernelGGL((k_gram2<T, 6>), dim3(2 * n_w64, A.n_sweeps), dim3(64), 0, st, A, gates, n_g, gout,
                       ncap, 64);
}

void launch_gram(int prec, const SweepArgs& A, const DevGate* gates, int n_g, int n_w16, int n_wide, int n_w64,
                 double* gout, int ncap, hipStream_t st) {
  if (n_g <= 0) return;
  if (A.qr) {
    // factors of up to 16 columns (four teams per wavefront), 32 (two) and 64
    // (one), the wider classes over the leading gates that can be that wide
    hipLaunchKernelGGL((k_qr<double, 16>), dim3(2 * n_g, A.n_sweeps), dim3(64), 0, st, A, gates, n_g, gout, ncap, 0);
    if (ncap > 16 && n_w16 > 0)
      hipLaunchKernelGGL((k_qr<double, 32>), dim3(2 * n_w16, A.n_sweeps), dim3(64), 0, st, A, gates, n_g, gout, ncap,
                         16);
    if (ncap > 32 && n_wide > 0)
      hipLaunchKernelGGL((k_qr<double, 64>), dim3(2 * n_wide, A.n_sweeps), dim3(64), 0, st, A, gates, n_g, gout, ncap,
                         32);
    return;
  }
  // the BF16 mode forms its Grams like FP32 (FP64 products of the FP32
  // values): the BF16 split with FP32 accumulation squares the FP32 rounding
  // of the Gram into the small eigenvalues, and the singular values below
  // about 3e-4 of the largest, which the reduced rule keeps, came out wrong
  // (0.5 nats on the loop sector at L = 8, chi = 32)
  if (prec == 0)
    gram_dispatch<double>(A, gates, n_g, n_wide, n_w64, gout, ncap, st);
  else
    gram_dispatch<float>(A, gates, n_g, n_wide, n_w64, gout, ncap, st);
}

// Dynamic LDS of a k_solve launch whose orders reach kd: four n x n matrices
// up to order 64, three above (see k_solve), the most any order <= kd needs.
static size_t solve_lds(int kd) {
  // matrices of n (n + 1) doubles up to order 64 (odd leading dimensions),
  // of n x n above, where the second one lives in global scratch
  auto need = [](int n, int mats, int ld) {
    return size_t(mats) * n * ld * 8 + size_t(2) * n * 8 + 32 + size_t(2 * n + 4) * 4;
  };
  const int k64 = std::min(kd, 64);
  size_t b = need(k64, 4, k64 + 1);
  if (kd > 64) b = std::max(b, need(kd, 3, kd));
  return b;
}

void launch_solve(const LaunchTuning& T, const SweepArgs& A, const DevGate* gates, int n_g, const double* gin,
                  double* wout, int ncap, int kdcap, hipStream_t st) {
  if (n_g <= 0) return;
  // three size classes: order <= 8 (eight problems per wavefront, a team of
  // eight lanes each; most gates), up to T.mid (one wavefront, at most 8 KB of
  // LDS) and the rest up to kdcap (up to 130 KB of LDS, so few workgroups fit
  // a CU: four wavefronts share each problem).  A team of 16 lanes for the
  // middle class measured slower than one wavefront per problem.
  const int lo = T.team ? 8 : 0;
  const int mid = std::max(lo, std::min(kdcap, T.mid));
  if (T.team)
    hipLaunchKernelGGL(k_solve_team<8>, dim3(n_g, (A.n_sweeps + 7) / 8), dim3(64), 0, st, A, gates, n_g, gin, wout,
                       ncap, 0);
  if (mid > lo)
    hipLaunchKernelGGL(k_solve<SNT>, dim3(n_g, A.n_sweeps), dim3(SNT), solve_lds(mid), st, A, gates, n_g, gin, wout,
                       ncap, lo, mid);
  if (kdcap > mid)
    hipLaunchKernelGGL(k_solve<SNT_BIG>, dim3(n_g, A.n_sweeps), dim3(SNT_BIG), solve_lds(kdcap), st, A, gates, n_g,
                       gin, wout, ncap, mid, kdcap);
}

void launch_reabsorb(const LaunchTuning& T, int prec, const SweepArgs& A, const DevGate* gates, int n_g, int n_w16,
                     int n_w32, int n_w64, const double* win, int ncap, hipStream_t st) {
  if (n_g <= 0) return;
  dim3 g(2 * n_g, A.n_sweeps), g16(2 * n_w16, A.n_sweeps), g32(2 * n_w32, A.n_sweeps), g64(2 * n_w64, A.n_sweeps);
  // rows with more than 64 inputs or outputs (physical dim 4 at chi up to 24):
  // W staged in LDS, over the leading gates that can be that wide
  const bool w64 = ncap > 64 && n_w64 > 0;
  // three size classes: rows of at most 16 and 32 entries, then the rest up to
  // 64 (the W staging takes 8, 16 and 32 KB of LDS); the wider classes run
  // over the leading gates that can have such rows.  Without the narrow
  // class (T.narrow = 0) the 32-entry kernel takes every row up to 32.
  const bool merge = !T.narrow && ncap > 16;
  const bool w16 = ncap > 16 && n_w16 > 0, w32 = ncap > 32 && n_w32 > 0;
  // the widest class (rows of 33 to 64 entries) on the matrix cores
  if (prec == 0) {
    if (merge) {
      hipLaunchKernelGGL((k_reabsorb<double, 32>), g, dim3(64), 0, st, A, gates, n_g, win, ncap, 0);
    } else {
      hipLaunchKernelGGL((k_reabsorb<double, 16>), g, dim3(64), 0, st, A, gates, n_g, win, ncap, 0);
      if (w16) hipLaunchKernelGGL((k_reabsorb<double, 32>), g16, dim3(64), 0, st, A, gates, n_g, win, ncap, 16);
    }
    if (w32) hipLaunchKernelGGL((k_reabsorb2<double, 64, 0>), g32, dim3(64), 0, st, A, gates, n_g, win, ncap, 32);
    if (w64) hipLaunchKernelGGL((k_reabsorb<double, 96>), g64, dim3(64), 0, st, A, gates, n_g, win, ncap, 64);
  } else {
    if (merge) {
      hipLaunchKernelGGL((k_reabsorb<float, 32>), g, dim3(64), 0, st, A, gates, n_g, win, ncap, 0);
    } else {
      hipLaunchKernelGGL((k_reabsorb<float, 16>), g, dim3(64), 0, st, A, gates, n_g, win, ncap, 0);
      if (w16) hipLaunchKernelGGL((k_reabsorb<float, 32>), g16, dim3(64), 0, st, A, gates, n_g, win, ncap, 16);
    }
    if (w32) {
      if (prec == 2)
        hipLaunchKernelGGL((k_reabsorb2<float, 64, 1>), g32, dim3(64), 0, st, A, gates, n_g, win, ncap, 32);
      else
        hipLaunchKernelGGL((k_reabsorb2<float, 64, 0>), g32, dim3(64), 0, st, A, gates, n_g, win, ncap, 32);
    }
    if (w64) hipLaunchKernelGGL((k_reabsorb<float, 96>), g64, dim3(64), 0, st, A, gates, n_g, win, ncap, 64);
  }
}

void launch_rescale(int prec, const SweepArgs& A, const int32_t* d_after, const int32_t* par_after,
                    hipStream_t st) {
  dim3 g(A.n_sites, A.n_sweeps);
  if (prec == 0)
    hipLaunchKernelGGL(k_rescale<double>, g, dim3(ET), 0, st, A, d_after, par_after);
  else
    hipLaunchKernelGGL(k_rescale<float>, g, dim3(ET), 0, st, A, d_after, par_after);
}

void launch_finalize(int prec, const SweepArgs& A, const int32_t* d_final, const int32_t* f_off,
                     const int32_t* par_final, double* fin, int64_t fin_stride, const int64_t* fin_off,
                     hipStream_t st) {
  dim3 g(A.n_sites, A.n_sweeps);
  if (prec == 0)
    hipLaunchKernelGGL(k_finalize<double>, g, dim3(ET), 0, st, A, d_final, f_off, par_final, fin, fin_stride,
                       fin_off);
  else
    hipLaunchKernelGGL(k_finalize<float>, g, dim3(ET), 0, st, A, d_final, f_off, par_final, fin, fin_stride,
                       fin_off);
}

void launch_zip_init(const ZipArgs& Z, hipStream_t st) {
  hipLaunchKernelGGL(k_zip_init, dim3(Z.n_sweeps), dim3(64), 0, st, Z);
}

int zip_step_large(const ZipArgs& Z, int x, int y, int legcap) {
  const int inline_dec = (x + 1 < Z.Lx && y + 1 == Z.Ly) ? 1 : 0;
  if (!(x + 1 < Z.Lx && !inline_dec && Z.gram_path)) return 0;
  // the order min(R, C) of the Gram, R = nu sD and C = aR wR, is bounded by
  // the structure: nu = 1 in the first column, aR = 1 in the first row,
  // sD = 1 in the last row
  const int64_t rcap = int64_t(x == 0 ? 1 : Z.chi_m) * (y + 1 == Z.Ly ? 1 : legcap);
  const int64_t ccap = int64_t(y == 0 ? 1 : Z.chi_m) * legcap;
  if ((rcap < ccap ? rcap : ccap) <= ZBIG) return 0;
  return Z.chi_m + 1 <= SB ? 1 : 2;
}

void launch_zip_step(const ZipArgs& Z, int x, int y, int legcap, hipStream_t st) {
  const int inline_dec = (x + 1 < Z.Lx && y + 1 == Z.Ly) ? 1 : 0;
  hipLaunchKernelGGL(k_zip_a, dim3(Z.n_sweeps), dim3(ZNT), 0, st, Z, x, y, inline_dec);
  if (x + 1 < Z.Lx && !inline_dec) {
    if (Z.gram_path) {
      hipLaunchKernelGGL(k_zip_beig, dim3(Z.n_sweeps), dim3(64), beig_lds_bytes(Z.eig_ys), st, Z, x,
                         y);
      // the larger-order kernels run only where the structural bound on the
      // family passes ZBIG
      const int big = zip_step_large(Z, x, y, legcap);
      if (big == 1)
        hipLaunchKernelGGL(k_zip_bsub, dim3(Z.n_sweeps), dim3(ZNT), bsub_lds_bytes(), st, Z, x, y);
      else if (big == 2)
        hipLaunchKernelGGL(k_zip_bbig, dim3(Z.n_sweeps), dim3(ZNT), size_t(19200) * 8, st, Z, x, y, 19200);
    } else {
      hipLaunchKernelGGL(k_zip_b, dim3(Z.n_sweeps), dim3(ZBT), size_t(18432) * 8, st, Z, x, y, 18432);
    }
  }
  hipLaunchKernelGGL(k_zip_c, dim3(Z.n_sweeps), dim3(ZNT), 0, st, Z, x, y);
}

void launch_finish(const SweepArgs& A, const ZipArgs& Z, double* logp, uint32_t* flags_out, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3((A.n_sweeps + 63) / 64), dim3(64), 0, st, A, Z, logp);
  const int n_items = A.n_sweeps / A.n_cosets;
  if (A.wht && A.n_cosets == 2)
    hipLaunchKernelGGL(k_wht_combine, dim3((n_items + 63) / 64), dim3(64), 0, st, n_items, A.items, logp, A.flags);
  if (flags_out)
    hipLaunchKernelGGL(k_collect_flags, dim3((n_items + 63) / 64), dim3(64), 0, st, n_items, A.n_cosets, A.items,
                       A.flags, flags_out);
}

void launch_ext_bits(int n, uint8_t* bits, int64_t stride, int n_det, int src0, int src_n, int words,
                     const uint64_t* rows, int n_ext, hipStream_t st) {
  if (n <= 0 || n_ext <= 0) return;
  hipLaunchKernelGGL(k_ext_bits, dim3(n), dim3(256), 0, st, n, bits, stride, n_det, src0, src_n, words, rows, n_ext);
}

void launch_gather_synd(int n, const int32_t* items, const uint8_t* synd, const int64_t* offs, int n_det,
                        int64_t stride, uint8_t* out, hipStream_t st) {
  if (n <= 0 || n_det <= 0) return;
  hipLaunchKernelGGL(k_gather_synd, dim3((n_det + 255) / 256, n), dim3(256), 0, st, n, items, synd, offs, n_det,
                     stride, out);
}

void launch_stamp(unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, st, out);
}

void launch_seq(int n, int32_t* items, int64_t* offs, int64_t stride, hipStream_t st) {
  hipLaunchKernelGGL(k_seq, dim3((n + 255) / 256), dim3(256), 0, st, n, items, offs, stride);
}

void launch_timing_reduce(const unsigned long long* stamps, const unsigned long long* win, int n_cls_win, int Lx,
                          int Ly, int eig, const unsigned long long* ctr, double ms_per_tick, double* acc,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_timing_reduce, dim3(n_cls_win + 3 * Lx * Ly + 1), dim3(64), 0, st, stamps, win, n_cls_win, Lx,
                     Ly, eig, ctr, ms_per_tick, acc);
}

void launch_win_init(unsigned long long* win, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_win_init, dim3((n * 128 + 255) / 256), dim3(256), 0, st, win, n);
}

void launch_zero_words(uint32_t* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}

void launch_scatter_out(int n, const int32_t* items, const double* lp_local, const uint32_t* fl_local, double* logp,
                        uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_out, dim3((n + 255) / 256), dim3(256), 0, st, n, items, lp_local, fl_local, logp,
                     flags);
}

void launch_pick_ties(int n_items, const double* logratio, double near_tie, int32_t* list, int32_t* count,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_pick_ties, dim3((n_items + 255) / 256), dim3(256), 0, st, n_items, logratio, near_tie, list,
                     count);
}

void launch_gather_offsets(int n, const int32_t* items, const int64_t* offs, int64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_offsets, dim3((n + 255) / 256), dim3(256), 0, st, n, items, offs, out);
}

void launch_gather_i32(int n, const int32_t* items, const int32_t* src, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_i32, dim3((n + 255) / 256), dim3(256), 0, st, n, items, src, out);
}

void launch_scatter_resweep(int n, const int32_t* items, const double* logp_sub, const uint32_t* flags_sub,
                            double* logp, uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_resweep, dim3((n + 255) / 256), dim3(256), 0, st, n, items, logp_sub, flags_sub, logp,
                     flags);
}

void launch_decode(int n_items, int n_cosets, const int32_t* items, const double* logp, double near_tie,
                   int32_t* coset, double* logratio, uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_decode, dim3((n_items + 63) / 64), dim3(64), 0, st, n_items, n_cosets, items, logp,
                     near_tie, coset, logratio, flags);
}

void launch_grad(int B, int n, int nc, int n_rates, const double* lp, const uint32_t* fl, const double* cp,
                 const int32_t* ptr, const int32_t* rm, double* term, double* grad, double* loglik, double* total,
                 uint32_t* flags, hipStream_t st) {
  const int64_t tot = int64_t(B) * n;
  hipLaunchKernelGGL(k_grad_terms, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, B, n, nc, lp, cp, term);
  hipLaunchKernelGGL(k_grad_items, dim3((B + 255) / 256), dim3(256), 0, st, B, n, nc, lp, fl, loglik, flags);
  hipLaunchKernelGGL(k_grad_reduce, dim3(n_rates), dim3(256), 0, st, B, n, term, ptr, rm, grad);
  if (total) hipLaunchKernelGGL(k_grad_total, dim3(1), dim3(256), 0, st, B, nc, lp, total);
}

void launch_tile_offsets(int B, int n_blocks, const int64_t* offs, int64_t* offs_all, hipStream_t st) {
  const int64_t tot = int64_t(B) * n_blocks;
  hipLaunchKernelGGL(k_tile_offsets, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, B, n_blocks, offs,
                     offs_all);
}

}  // namespace tn3d
