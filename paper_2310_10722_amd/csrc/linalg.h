// Workgroup-level dense linear algebra in FP64 for the small truncation
// problems of the sweep.  Every function is called by all threads of the
// workgroup with identical arguments and contains its own barriers.
#pragma once

#include <hip/hip_runtime.h>

namespace tn3d {

// Value of v in lane src (uniform) of the wavefront, in every lane.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Lowest lane whose pred is true (64 if none).
__device__ __forceinline__ int wave_first(bool pred) {
  const unsigned long long m = __ballot(pred);
  return m ? __builtin_ctzll(m) : 64;
}

// v moved across lanes by a DPP pattern (a compile-time dpp_ctrl code).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over aligned teams of `team` (a power of two up to 64) consecutive
// lanes, the same value in every lane of a team: DPP moves within rows of 16
// lanes, lane shuffles across rows.  Every lane of a team must be active.
__device__ __forceinline__ double team_sum(double v, int team) {
  if (team >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  if (team >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  if (team >= 8) v += dpp_move<0x141>(v);  // row_half_mirror: the other quad of the 8
  if (team >= 16) v += dpp_move<0x140>(v); // row_mirror: the other 8 of the row
  if (team >= 32) v += __shfl_xor(v, 16, 64);
  if (team >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// The largest v over the wavefront and the lowest lane holding it, in every
// lane: DPP exchanges within rows of 16 lanes, then the four row winners read
// out in order.  Every lane must be active.
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
  auto step = [&](double w, int j) {
    if (w > v || (w == v && j < idx)) {
      v = w;
      idx = j;
    }
  };
  step(dpp_move<0xB1>(v), __builtin_amdgcn_update_dpp(0, idx, 0xB1, 0xF, 0xF, false));
  step(dpp_move<0x4E>(v), __builtin_amdgcn_update_dpp(0, idx, 0x4E, 0xF, 0xF, false));
  step(dpp_move<0x141>(v), __builtin_amdgcn_update_dpp(0, idx, 0x141, 0xF, 0xF, false));
  step(dpp_move<0x140>(v), __builtin_amdgcn_update_dpp(0, idx, 0x140, 0xF, 0xF, false));
  double bv = wave_bcast(v, 0);
  int bi = __builtin_amdgcn_readlane(idx, 0);
  for (int r = 16; r < 64; r += 16) {
    const double w = wave_bcast(v, r);
    const int j = __builtin_amdgcn_readlane(idx, r);
    if (w > bv || (w == bv && j < bi)) {
      bv = w;
      bi = j;
    }
  }
  v = bv;
  idx = bi;
}

// Pivoted Cholesky of the symmetric positive semidefinite n x n matrix Z
// (row-major, leading dimension n; destroyed).  Writes F (r x n, row-major,
// leading dimension n) with F^T F = Z up to the dropped trailing part, in the
// original column order, and returns the rank r: elimination stops when the
// largest remaining diagonal is <= tol * max(diag Z).  Any n (the diagonal
// is scanned by the first wavefront, lane l taking entries l, l + 64, ...).
// perm is scratch of n ints, red scratch of 2 doubles.
__device__ int block_pchol(double* Z, double* F, int n, double tol, int* perm, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) perm[i] = i;
  if (tid < 64) {
    double m = 0.0;
    for (int i = tid; i < n; i += 64) m = fmax(m, Z[i * n + i]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (tid == 0) red[0] = fmax(m, 0.0);
  }
  __syncthreads();
  const double thr = tol * red[0];
  __syncthreads();
  int r = 0;
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {  // pivot: the largest remaining diagonal, lowest index on ties
      double best = -1e300;
      int j = n + tid;  // no candidate in this lane: loses every tie to a real index
      for (int i = tid; i < n; i += 64)
        if (i >= k) {
          const double v = Z[i * n + i];
          if (v > best) {  // ascending i: the lowest index of a lane's ties stays
            best = v;
            j = i;
          }
        }
      wave_argmax(best, j);
      if (tid == 0) {
        red[1] = double(j);
        red[0] = best;
      }
    }
    __syncthreads();
    const int j = int(red[1]);
    const double piv = red[0];
    if (!(piv > thr)) break;
    if (j != k) {
      for (int i = tid; i < n; i += nt) {  // swap columns k, j
        double t = Z[i * n + k];
        Z[i * n + k] = Z[i * n + j];
        Z[i * n + j] = t;
      }
      __syncthreads();
      for (int i = tid; i < n; i += nt) {  // swap rows k, j
        double t = Z[k * n + i];
        Z[k * n + i] = Z[j * n + i];
        Z[j * n + i] = t;
      }
      if (tid == 0) {
        int t = perm[k];
        perm[k] = perm[j];
        perm[j] = t;
      }
      __syncthreads();
    }
    const double rk = sqrt(piv);
    for (int i = tid; i < n; i += nt) {
      if (i == k) Z[k * n + k] = rk;
      else if (i > k) Z[k * n + i] /= rk;
    }
    __syncthreads();
    // trailing update: 16 columns per pass of a row, nt / 16 rows per pass
    // (no integer division in the loop)
    for (int a = k + 1 + (tid >> 4); a < n; a += nt >> 4) {
      const double za = Z[k * n + a];
      for (int b = k + 1 + (tid & 15); b < n; b += 16) Z[a * n + b] -= za * Z[k * n + b];
    }
    __syncthreads();
    r = k + 1;
  }
  // F[i][perm[c]] = R[i][c] for c >= i, else 0
  for (int e = tid; e < r * n; e += nt) {
    int i = e / n, c = e % n;
    F[i * n + perm[c]] = c >= i ? Z[i * n + c] : 0.0;
  }
  __syncthreads();
  return r;
}

// One-sided Jacobi: orthogonalises the `nv` vectors of length `len` stored at
// A[v * vs + e * es] by plane rotations, applying the same rotations to the
// rows of the nv x nv matrix J (row-major, leading dimension nv, initialised to
// the identity here), so that A_out = A_in J.  A pair is rotated while
// |a_i . a_j| > tol |a_i| |a_j|; pairs in which a vector's norm is below
// floor_rel * (largest initial norm) are left alone: such vectors hold only
// rounding noise of the large ones, cannot be orthogonalised to relative
// precision tol, and lie below the truncation threshold.  Returns the number
// of sweeps before the last; max_sweeps means no convergence.  A sweep whose
// rotations all had |a_i . a_j| <= sqrt(tol) |a_i| |a_j| ends the iteration:
// one-sided Jacobi converges quadratically, so what it leaves is of order
// tol.  red: 2 doubles scratch, flag: 2 ints.  ldj: J's leading dimension
// (0: nv).
__device__ int block_jacobi(double* A, long vs, long es, int nv, int len, double* J, double tol,
                            double floor_rel, int max_sweeps, int* flag, double* red, int ldj = 0) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (ldj == 0) ldj = nv;
  for (int r = tid >> 4; r < nv; r += nt >> 4)
    for (int c = tid & 15; c < nv; c += 16) J[r * ldj + c] = r == c ? 1.0 : 0.0;
  const int ne = nv + (nv & 1);
  const int npairs = ne / 2;
  int team = 64;
  while (team > 1 && team * npairs > nt) team >>= 1;
  const int pair = tid / team, lane = tid % team;
  if (tid == 0) red[0] = 0.0;
  __syncthreads();
  // largest squared norm
  for (int v = tid / 64; v < nv; v += nt / 64) {
    double s = 0.0;
    for (int e = tid % 64; e < len; e += 64) {
      double x = A[v * vs + e * es];
      s += x * x;
    }
    s = team_sum(s, 64);
    if (tid % 64 == 0) atomicMax(reinterpret_cast<unsigned long long*>(red), __double_as_longlong(s));
  }
  __syncthreads();
  const double floor2 = floor_rel * floor_rel * red[0];
  __syncthreads();
  const double sqrt_tol = sqrt(tol);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) {
      flag[0] = 0;  // a rotation was applied
      flag[1] = 0;  // a rotation had cosine of the angle above sqrt(tol)
    }
    __syncthreads();
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      for (int pp = pair; pp < npairs; pp += nt / team) {
        int i, j;
        if (pp == 0) {
          i = ne - 1;
          j = rnd;
        } else {  // (rnd + pp) and (rnd - pp) mod (ne - 1), both in range after one correction
          i = rnd + pp;
          i = i >= ne - 1 ? i - (ne - 1) : i;
          j = rnd - pp + ne - 1;
          j = j >= ne - 1 ? j - (ne - 1) : j;
        }
        if (i >= nv || j >= nv) continue;
        if (i > j) {
          int t = i;
          i = j;
          j = t;
        }
        double a = 0, b = 0, g = 0;
        for (int e = lane; e < len; e += team) {
          double x = A[i * vs + e * es], y = A[j * vs + e * es];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        a = team_sum(a, team);
        b = team_sum(b, team);
        g = team_sum(g, team);
        const double sab = sqrt(a) * sqrt(b);
        if (a > floor2 && b > floor2 && fabs(g) > tol * sab) {
          double zeta = (b - a) / (2.0 * g);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int e = lane; e < len; e += team) {
            double x = A[i * vs + e * es], y = A[j * vs + e * es];
            A[i * vs + e * es] = cs * x - sn * y;
            A[j * vs + e * es] = sn * x + cs * y;
          }
          for (int e = lane; e < nv; e += team) {
            double x = J[e * ldj + i], y = J[e * ldj + j];
            J[e * ldj + i] = cs * x - sn * y;
            J[e * ldj + j] = sn * x + cs * y;
          }
          if (lane == 0) {
            flag[0] = 1;
            if (fabs(g) > sqrt_tol * sab) flag[1] = 1;
          }
        }
      }
      __syncthreads();
    }
    if (flag[0] == 0) break;
    if (flag[1] == 0) break;  // every cosine below sqrt(tol): the next sweep would only square them
    __syncthreads();
  }
  __syncthreads();
  return sweep;
}

// Strict total order for a descending sort with ties broken by index: a NaN
// sorts after every number, so the ranks it gives always form a permutation
// (indices taken from them stay in range whatever the data).
__device__ __forceinline__ bool sorts_before(double a, int ia, double b, int ib) {
  const bool na = a != a, nb = b != b;
  if (na || nb) return !na && nb ? true : (na && nb && ia < ib);
  return a > b || (a == b && ia < ib);
}

// Norms of the nv vectors into S and the permutation `order` that sorts them
// descending (ties by index).
__device__ void block_norms_sorted(const double* A, long vs, long es, int nv, int len, double* S,
                                   int* order) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int v = tid; v < nv; v += nt) {
    double s = 0;
    for (int e = 0; e < len; ++e) {
      double x = A[v * vs + e * es];
      s += x * x;
    }
    S[v] = sqrt(s);
  }
  __syncthreads();
  for (int v = tid; v < nv; v += nt) {
    int rank = 0;
    for (int u = 0; u < nv; ++u)
      if (sorts_before(S[u], u, S[v], v)) ++rank;
    order[rank] = v;
  }
  __syncthreads();
}

// The truncation rank: the largest D <= min(chi, n) with S_D > eps S_1 and
// (D = n or S_{D+1} < (1 - tau) S_D).  Ss sorted descending.  *split is set
// when no such D exists (then D = min(chi, n)).
__device__ __forceinline__ int rank_rule(const double* Ss, int n, int chi, double eps, double tau,
                                         int* split) {
  int top = n < chi ? n : chi;
  *split = 0;
  if (n == 0 || !(Ss[0] > 0.0)) {
    *split = 1;
    return 0;
  }
  for (int D = top; D >= 1; --D) {
    if (Ss[D - 1] <= eps * Ss[0]) continue;
    if (D == n || Ss[D] < (1.0 - tau) * Ss[D - 1]) return D;
  }
  *split = 1;
  return top;
}

// C[m][n] = sum_k A(m, k) B(k, n) for a 512-thread workgroup, FP64 on the
// matrix cores, through 64 x 64 output tiles and 32-deep K slices staged in
// LDS (lds: GEMM_LDS doubles, k-major rows of 64, or of 65 when a fetch runs
// along k so that its stores spread over the banks), each slice's global loads issued into
// registers while the previous slice is multiplied.  a_at / b_at return
// operands (any layout); c_put(m, n, v) stores.  KA (KB): A's (B's) elements
// are contiguous along k, so the lanes of a fetch run along k rather than
// along m (n), and a load instruction touches few cache lines.  v_mfma_f64_16x16x4f64 takes a 16 x 4
// block of A (lane i + 16 k holds A[i][k]) and a 4 x 16 block of B (lane
// j + 16 k holds B[k][j]) and accumulates the 16 x 16 block of C, item r of
// lane j + 16 q holding row q + 4 r of column j.  The 64 x 64 output tile
// is split over the eight wavefronts as four 16-row bands times two 32-column
// halves (two accumulator blocks each); a wavefront whose band or half lies
// outside M x N skips the products, and a K slice runs only as many 4-deep
// steps as it holds.
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int GEMM_LDS = 2 * 32 * 65;  // doubles of LDS block_gemm512 takes
template <bool KA = false, bool KB = false, class FA, class FB, class FC>
__device__ void block_gemm512(int M, int N, int K, FA a_at, FB b_at, FC c_put, double* lds) {
  constexpr int GEMM_LS = (KA || KB) ? 65 : 64;  // LDS row stride of a staged slice
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int rb = (wv & 3) * 16, cb = (wv >> 2) * 32;
  double* As = lds;                 // [32][GEMM_LS]  (k, m)
  double* Bs = lds + 32 * GEMM_LS;  // [32][GEMM_LS]  (k, n)
  // element e of a thread's four: (k, m) = (e / 64, e % 64) along m, or
  // (e % 32, e / 32) along k
  auto kk_of = [](int e, bool alongk) { return alongk ? (e & 31) : (e >> 6); };
  auto mm_of = [](int e, bool alongk) { return alongk ? (e >> 5) : (e & 63); };
  for (int m0 = 0; m0 < M; m0 += 64)
    for (int n0 = 0; n0 < N; n0 += 64) {
      const bool act = m0 + rb < M && n0 + cb < N;  // uniform per wavefront
      const bool act2 = n0 + cb + 16 < N;
      dbl4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
      double ra[4], rb4[4];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = tid + 512 * i;
          const int ka = k0 + kk_of(e, KA), m = m0 + mm_of(e, KA);
          const int kb = k0 + kk_of(e, KB), n = n0 + mm_of(e, KB);
          ra[i] = (m < M && ka < K) ? a_at(m, ka) : 0.0;
          rb4[i] = (n < N && kb < K) ? b_at(kb, n) : 0.0;
        }
      };
      __syncthreads();  // the previous tile's stores land before this tile's loads
      fetch(0);
      for (int k0 = 0; k0 < K; k0 += 32) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = tid + 512 * i;  // with rows of 64 and m-ordered fetches the position is e itself
          As[(KA || GEMM_LS != 64) ? kk_of(e, KA) * GEMM_LS + mm_of(e, KA) : e] = ra[i];
          Bs[(KB || GEMM_LS != 64) ? kk_of(e, KB) * GEMM_LS + mm_of(e, KB) : e] = rb4[i];
        }
        __syncthreads();
        if (k0 + 32 < K) fetch(k0 + 32);
        if (act) {
          const int nks = K - k0 >= 32 ? 8 : (K - k0 + 3) >> 2;
          constexpr int KS = 4 * GEMM_LS;  // LDS distance of one 4-deep step
          const double* ap = As + lq * GEMM_LS + rb + li;
          const double* bp = Bs + lq * GEMM_LS + cb + li;
          if (act2) {
            for (int ks = 0; ks < nks; ++ks) {
              const double a = ap[ks * KS], b0 = bp[ks * KS], b1 = bp[ks * KS + 16];
              c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, c0, 0, 0, 0);
              c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, c1, 0, 0, 0);
            }
          } else {
            for (int ks = 0; ks < nks; ++ks)
              c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[ks * KS], bp[ks * KS], c0, 0, 0, 0);
          }
        }
      }
      if (act) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + rb + lq + 4 * r, n = n0 + cb + li;
          if (m < M) {
            if (n < N) c_put(m, n, c0[r]);
            if (n + 16 < N) c_put(m, n + 16, c1[r]);
          }
        }
      }
    }
  __syncthreads();
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// v = h + m + l exactly (to 24 bits) with three BF16 terms of 8 significant
// bits each (round to nearest at every step; the residuals are exact).
__device__ __forceinline__ void split3(const float (&v)[8], bf16x8& h, bf16x8& m, bf16x8& l) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 a = __bf16(v[t]);
    const float r1 = v[t] - float(a);
    const __bf16 b = __bf16(r1);
    const float r2 = r1 - float(b);
    h[t] = a;
    m[t] = b;
    l[t] = __bf16(r2);
  }
}

// block_gemm512 on the BF16 matrix cores: the operands rounded to FP32, split
// into three BF16 terms each (split3) and the six leading products (h.h, h.m,
// m.h, h.l, m.m, l.h, the dropped ones below 2^-24 relative) accumulated in
// FP32 over each 32-deep K slice, the slices summed in FP64.  Same tiling and
// staging as block_gemm512; v_mfma_f32_16x16x32_bf16 takes A[i][8q .. 8q + 7]
// in lane i + 16 q and B[8q .. 8q + 7][j] in lane j + 16 q, and item r of lane
// j + 16 q is C[4 q + r][j].
template <bool KA = false, bool KB = false, class FA, class FB, class FC>
__device__ void block_gemm512_bf(int M, int N, int K, FA a_at, FB b_at, FC c_put, double* lds) {
  constexpr int GEMM_LS = (KA || KB) ? 65 : 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int rb = (wv & 3) * 16, cb = (wv >> 2) * 32;
  double* As = lds;
  double* Bs = lds + 32 * GEMM_LS;
  auto kk_of = [](int e, bool alongk) { return alongk ? (e & 31) : (e >> 6); };
  auto mm_of = [](int e, bool alongk) { return alongk ? (e >> 5) : (e & 63); };
  for (int m0 = 0; m0 < M; m0 += 64)
    for (int n0 = 0; n0 < N; n0 += 64) {
      const bool act = m0 + rb < M && n0 + cb < N;
      const bool act2 = n0 + cb + 16 < N;
      dbl4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
      double ra[4], rb4[4];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = tid + 512 * i;
          const int ka = k0 + kk_of(e, KA), m = m0 + mm_of(e, KA);
          const int kb = k0 + kk_of(e, KB), n = n0 + mm_of(e, KB);
          ra[i] = (m < M && ka < K) ? a_at(m, ka) : 0.0;
          rb4[i] = (n < N && kb < K) ? b_at(kb, n) : 0.0;
        }
      };
      __syncthreads();
      fetch(0);
      for (int k0 = 0; k0 < K; k0 += 32) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = tid + 512 * i;
          As[(KA || GEMM_LS != 64) ? kk_of(e, KA) * GEMM_LS + mm_of(e, KA) : e] = ra[i];
          Bs[(KB || GEMM_LS != 64) ? kk_of(e, KB) * GEMM_LS + mm_of(e, KB) : e] = rb4[i];
        }
        __syncthreads();
        if (k0 + 32 < K) fetch(k0 + 32);
        if (act) {
          float va[8], vb0[8], vb1[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int kr = (8 * lq + u) * GEMM_LS;
            va[u] = float(As[kr + rb + li]);
            vb0[u] = float(Bs[kr + cb + li]);
            vb1[u] = act2 ? float(Bs[kr + cb + 16 + li]) : 0.f;
          }
          bf16x8 ah, am, al, bh0, bm0, bl0, bh1, bm1, bl1;
          split3(va, ah, am, al);
          split3(vb0, bh0, bm0, bl0);
          split3(vb1, bh1, bm1, bl1);
          flt4 f0 = {0.f, 0.f, 0.f, 0.f}, f1 = {0.f, 0.f, 0.f, 0.f};
          f0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh0, f0, 0, 0, 0);
          f1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh1, f1, 0, 0, 0);
          f0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm0, f0, 0, 0, 0);
          f1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm1, f1, 0, 0, 0);
          f0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl0, f0, 0, 0, 0);
          f1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl1, f1, 0, 0, 0);
          f0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh0, f0, 0, 0, 0);
          f1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh1, f1, 0, 0, 0);
          f0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm0, f0, 0, 0, 0);
          f1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm1, f1, 0, 0, 0);
          f0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh0, f0, 0, 0, 0);
          f1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh1, f1, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            c0[r] += double(f0[r]);
            c1[r] += double(f1[r]);
          }
        }
      }
      if (act) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + rb + 4 * lq + r, n = n0 + cb + li;
          if (m < M) {
            if (n < N) c_put(m, n, c0[r]);
            if (n + 16 < N) c_put(m, n + 16, c1[r]);
          }
        }
      }
    }
  __syncthreads();
}

// Sum over the 64 lanes, the same value in every lane: butterflies within each
// row of 16 lanes (quad permutations, half-row and row mirrors), then the four
// row sums read out in a fixed order.  Every lane must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (wave_bcast(v, 0) + wave_bcast(v, 16)) + (wave_bcast(v, 32) + wave_bcast(v, 48));
}

// 1 / q from the hardware reciprocal and two Newton steps (a few ulps).
__device__ __forceinline__ double approx_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return fma(r, fma(-q, r, 1.0), r);
}

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// Leading eigenpairs of a symmetric matrix of order n <= 64 in one wavefront
// (64 threads): Householder reduction to a tridiagonal T = Q^T A Q, the K
// largest eigenvalues of T by multisection on Sturm sequence counts, their
// eigenvectors by inverse iteration, and the back-transformation by Q.  Only
// the leading pairs are computed, so every lane works on its own eigenvalue or
// vector instead of all lanes repeating one scalar recurrence.
// ---------------------------------------------------------------------------

// Steps k in [kb, ke) of the Householder reduction with the matrix in
// registers: lane i holds column i in a[0..63].  J0 <= kb, so rows below J0
// are finished and every index into a[] is a compile-time constant; row k of
// the current matrix is picked out of the 16 rows [J0, J0 + 16).  v and w of a
// step are broadcast through vw (v in vw[0, 64), w in vw[64, 128), 16-byte
// aligned LDS), read two at a time with the next group's reads issued before
// the current group's FMAs.  Only rows below NR (n rounded up to 16) are
// visited: past n the matrix, v and w are zero.  The Householder vector of step k is kept in row k
// of Hv (stride n); lane i writes only column i, the column it read from the
// input.
template <int J0, int NR>
__device__ __forceinline__ void tri_block(double (&a)[64], int n, int kb, int ke, double* vw, double* Hv,
                                          double& er, double& br) {
  const int i = threadIdx.x;
  const bool own = i < n;
  const double2* v2 = reinterpret_cast<const double2*>(vw);
  const double2* w2 = reinterpret_cast<const double2*>(vw + 64);
  for (int k = kb; k < ke; ++k) {
    double ak = 0.0;
#pragma unroll
    for (int j = J0; j < J0 + 16; ++j)
      if (j == k) ak = a[j];
    const bool act = own && i > k;
    double v = act ? ak : 0.0;
    const double sigma = wave_sum(v * v);
    const double x0 = wave_bcast(v, k + 1);
    if (!(sigma > 0.0) || sigma - x0 * x0 <= 1e-300) {
      if (i == k) {
        er = x0;
        br = 0.0;
      }
      continue;
    }
    const double alpha = x0 >= 0.0 ? -sqrt(sigma) : sqrt(sigma);
    const double bk = 1.0 / (sigma - x0 * alpha);  // 2 / (v.v) with v_{k+1} = x0 - alpha
    if (i == k + 1) v = x0 - alpha;
    if (i == k) {
      er = alpha;
      br = bk;
    }
    if (own) Hv[k * n + i] = v;
    vw[i] = v;
    __syncthreads();
    // p = bk A v in four partial sums, v read 16 rows at a time
    double p4[4] = {0.0, 0.0, 0.0, 0.0};
    double2 c[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) c[t] = v2[J0 / 2 + t];
#pragma unroll
    for (int g = J0; g < NR; g += 16) {
      double2 nx[8];
      if (g + 16 < NR) {
#pragma unroll
        for (int t = 0; t < 8; ++t) nx[t] = v2[(g + 16) / 2 + t];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        p4[(2 * t) & 3] = fma(a[g + 2 * t], c[t].x, p4[(2 * t) & 3]);
        p4[(2 * t + 1) & 3] = fma(a[g + 2 * t + 1], c[t].y, p4[(2 * t + 1) & 3]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (g + 16 < NR) {
#pragma unroll
        for (int t = 0; t < 8; ++t) c[t] = nx[t];
      }
    }
    const double p = ((p4[0] + p4[1]) + (p4[2] + p4[3])) * bk;
    const double K = 0.5 * bk * wave_sum(p * v);
    const double w = act ? p - K * v : 0.0;
    vw[64 + i] = w;
    __syncthreads();
    // A <- A - v w^T - w v^T, v and w read 8 rows at a time
    double2 cv[4], cw[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      cv[t] = v2[J0 / 2 + t];
      cw[t] = w2[J0 / 2 + t];
    }
#pragma unroll
    for (int g = J0; g < NR; g += 8) {
      double2 nv[4], nw[4];
      if (g + 8 < NR) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          nv[t] = v2[(g + 8) / 2 + t];
          nw[t] = w2[(g + 8) / 2 + t];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[g + 2 * t] = fma(-v, cw[t].x, fma(-w, cv[t].x, a[g + 2 * t]));
        a[g + 2 * t + 1] = fma(-v, cw[t].y, fma(-w, cv[t].y, a[g + 2 * t + 1]));
      }
      __builtin_amdgcn_sched_barrier(0);
      if (g + 8 < NR) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          cv[t] = nv[t];
          cw[t] = nw[t];
        }
      }
    }
    __syncthreads();
  }
}

// Householder reduction of the symmetric n x n matrix G (row-major, n >= 1)
// times gs, for n <= NR.  Lane i returns d_i = T[i][i], e_i = T[i][i+1] (0 for
// i >= n - 1) and the scalar beta_i of reflector i (0 when step i needed no
// reflection); Hv receives the reflectors (row k, stride n, components
// k+1 .. n-1, zeros before) and may alias G.  vw: 128 doubles of 16-byte
// aligned LDS.
template <int NR>
__device__ __forceinline__ void tridiag_nr(const double* G, double gs, int n, double* vw, double* Hv, double& dr,
                                           double& er, double& br) {
  const int i = threadIdx.x;
  double a[64];
  // every lane loads the NR entries of its column (clamped into the matrix)
  // and scales them by gs or by 0 outside the n x n block: every loaded value
  // is used, so the loads cannot be moved behind branches and are issued
  // together; entries past NR are zero and never read
  const int ic = i < n ? i : n - 1;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    if (j < NR) {
      const int jc = j < n ? j : n - 1;
      a[j] = G[jc * n + ic] * ((j < n && i < n) ? gs : 0.0);
    } else {
      a[j] = 0.0;
    }
  }
  er = 0.0;
  br = 0.0;
  const int ke = n - 2;
  if (NR > 16) {
    tri_block<0, NR>(a, n, 0, 16, vw, Hv, er, br);
    if (NR > 32) {
      tri_block<16, NR>(a, n, 16, 32, vw, Hv, er, br);
      if (NR > 48) {
        tri_block<32, NR>(a, n, 32, 48, vw, Hv, er, br);
        tri_block<48, NR>(a, n, 48, ke, vw, Hv, er, br);
      } else {
        tri_block<32, NR>(a, n, 32, ke, vw, Hv, er, br);
      }
    } else {
      tri_block<16, NR>(a, n, 16, ke, vw, Hv, er, br);
    }
  } else {
    tri_block<0, NR>(a, n, 0, ke, vw, Hv, er, br);
  }
  double di = 0.0, en = 0.0;
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (j == i) di = a[j];
    if (j == n - 1) en = a[j];
  }
  dr = i < n ? di : 0.0;
  if (i == n - 2) {
    er = en;
    br = 0.0;
  }
  if (i >= n - 1) {
    er = 0.0;
    br = 0.0;
  }
}

// The reduction above with the row bound NR = n rounded up to 16: rows past n
// hold zeros, so the shorter loops give the same result.
__device__ void wave_tridiag(const double* G, double gs, int n, double* vw, double* Hv, double& dr, double& er,
                             double& br) {
  if (n > 48)
    tridiag_nr<64>(G, gs, n, vw, Hv, dr, er, br);
  else if (n > 32)
    tridiag_nr<48>(G, gs, n, vw, Hv, dr, er, br);
  else if (n > 16)
    tridiag_nr<32>(G, gs, n, vw, Hv, dr, er, br);
  else
    tridiag_nr<16>(G, gs, n, vw, Hv, dr, er, br);
}

// Numbers of eigenvalues of T below each of the P points x[q]: sign changes
// along the leading principal minors m_0 = 1, m_1, ..., m_n of T - x I, from
// the three-term recurrence m_{r+1} = (d_r - x) m_r - e_{r-1}^2 m_{r-1} (P
// recurrences interleaved on the same rows, no division; a zero minor counts
// as non-negative).  Every four rows the two carried minors of each point are
// scaled by the same power of two so that they stay in range.  tri[2i] = d_i,
// tri[2i+1] = e_{i-1}^2 raised to at least 2^-700 (so that a zero minor cannot
// zero the rest of the sequence; for T scaled to norm about 1 the change is
// far below rounding), read by all lanes at the same 16-byte aligned LDS
// address.  Rows are taken four at a time: rows n .. 63 must hold d = 4,
// e^2 = 0, which adds no sign change for |x| < 2.
template <int P>
__device__ __forceinline__ void sturm_count(const double* tri, int n, const double (&x)[P], int (&cnt)[P]) {
  const double2* t2 = reinterpret_cast<const double2*>(tri);
  double m1[P], m2[P];
  int nc[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    m1[q] = 1.0;
    m2[q] = 0.0;
    nc[q] = 0;
  }
  double2 de[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) de[t] = t2[t];
  for (int r0 = 0; r0 < n; r0 += 4) {
    double2 dn[4];  // the next four rows, read while these are used
#pragma unroll
    for (int t = 0; t < 4; ++t) dn[t] = t2[(r0 + 4 + t) & 63];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const double pq = fma(de[t].x - x[q], m1[q], -de[t].y * m2[q]);
        nc[q] += (pq < 0.0) != (m1[q] < 0.0) ? 1 : 0;
        m2[q] = m1[q];
        m1[q] = pq;
      }
#pragma unroll
    for (int t = 0; t < 4; ++t) de[t] = dn[t];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int e = -__builtin_amdgcn_frexp_exp(m1[q]);
      m1[q] = __builtin_amdgcn_ldexp(m1[q], e);
      m2[q] = __builtin_amdgcn_ldexp(m2[q], e);
    }
  }
#pragma unroll
  for (int q = 0; q < P; ++q) cnt[q] = nc[q];
}

// The K (<= n) largest eigenvalues of T (lane i holds d_i, e_i) into lam[0..K)
// in decreasing order, by multisection of the Gershgorin interval: g = 64 / K
// lanes (at most 3) share an eigenvalue and each evaluates SP interior points
// per round, until the bracket is within a few ulps of the eigenvalue or of
// the norm of T.  tri: 2 * 64 doubles (16-byte aligned), xs: 64 * SP doubles,
// cs: 64 * SP ints (LDS).
// Returns the norm bound max |Gershgorin end|.
constexpr int SP = 2;
__device__ double wave_tri_topk(double dr, double er, int n, int K, double* tri, double* xs, int* cs, double* lam) {
  const int i = threadIdx.x;
  const bool own = i < n;
  const double eu = __shfl_up(er, 1, 64);
  const double el = (own && i > 0) ? eu : 0.0;
  const double ei = (own && i + 1 < n) ? er : 0.0;
  double lo = wave_min(own ? dr - fabs(el) - fabs(ei) : 1e300);
  double hi = wave_max(own ? dr + fabs(el) + fabs(ei) : -1e300);
  const double nrm = fmax(fabs(lo), fabs(hi));
  const int g = K >= 1 && 64 / K < 3 ? 64 / K : 3;
  const int t = i / g, r = i - t * g;
  const bool act = t < K;
  if (!(nrm > 0.0)) {  // T = 0
    if (act && r == 0) lam[t] = 0.0;
    __syncthreads();
    return nrm;
  }
  // the counts run on T / 2^e with 2^e the power of two at or above ||T||, so
  // the minors stay near 1 whatever the scale of T
  const double sc = __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(nrm));
  tri[2 * i] = own ? dr * sc : 4.0;  // rows past n: no sign change for |x| < 2
  tri[2 * i + 1] = own ? fmax(el * el * (sc * sc), 0x1p-700) : 0.0;
  const double atol = 4.0 * 2.220446049250313e-16 * nrm;
  const double pad = 1e-290 * fmax(1.0, nrm * nrm);
  lo -= atol + pad;
  hi += atol + pad;
  __syncthreads();
  const int sidx = n - 1 - t;  // position of the target in ascending order
  const int npt = SP * g;      // points per eigenvalue and round
  for (int it = 0; it < 128; ++it) {
    const double w = (hi - lo) / double(npt + 1);
    double xq[SP], xsc[SP];
    int cq[SP];
#pragma unroll
    for (int q = 0; q < SP; ++q) {
      xq[q] = lo + w * double(SP * r + q + 1);
      xsc[q] = xq[q] * sc;
    }
    sturm_count<SP>(tri, n, xsc, cq);
#pragma unroll
    for (int q = 0; q < SP; ++q) {
      xs[SP * i + q] = xq[q];
      cs[SP * i + q] = cq[q];
    }
    __syncthreads();
    if (act) {
      double nlo = lo, nhi = hi;
      for (int q = 0; q < npt; ++q) {
        const double xv = xs[SP * t * g + q];
        if (cs[SP * t * g + q] <= sidx)
          nlo = fmax(nlo, xv);
        else
          nhi = fmin(nhi, xv);
      }
      lo = nlo;
      hi = nhi;
    }
    __syncthreads();
    const bool done = !act || hi - lo <= fmax(atol, 4.5e-16 * fmax(fabs(lo), fabs(hi)));
    if (wave_first(!done) == 64) break;
  }
  if (act && r == 0) lam[t] = 0.5 * (lo + hi);
  __syncthreads();
  return nrm;
}

// One inverse-iteration solve (T - lam I) y = y for lane j's vector
// Y[r * ys + j], with the LU factors of lane j at U[(r * ys + j) * 4 + c]
// (c = 0 the reciprocal pivot, 1 and 2 the next two entries of U's row, 3 the
// multiplier) and the row swaps in the bits of swm, then y normalised.  The
// rows are taken in groups of eight held in registers: after a row is used its
// slot is refilled with the row eight further on, so eight rows of loads are
// always in flight.
__device__ __forceinline__ void tri_solve(int n, const double* U, double* Y, int ys, int j,
                                          unsigned long long swm) {
  const double* Uj = U + 4 * j;
  const int rs = 4 * ys;
  double cur = Y[j];
  const int last = n - 2;  // rows 0 .. n-2 carry an elimination step
  if (last >= 0) {
    double mA[8], yA[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = t < last ? t : last;
      mA[t] = Uj[r * rs + 3];
      yA[t] = Y[(r + 1) * ys + j];
    }
    for (int r0 = 0; r0 <= last; r0 += 8) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int r = r0 + t;
        if (r <= last) {
          const bool sw = (swm >> r) & 1ull;
          const double top = sw ? yA[t] : cur, bot = sw ? cur : yA[t];
          Y[r * ys + j] = top;
          cur = fma(-mA[t], top, bot);
        }
        const int rn = r + 8 < last ? r + 8 : last;
        mA[t] = Uj[rn * rs + 3];
        yA[t] = Y[(rn + 1) * ys + j];
      }
    }
  }
  Y[(n - 1) * ys + j] = cur;
  double y1 = 0.0, y2 = 0.0, ss = 0.0;
  double pA[8], uA[8], vA[8], yB[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int r = n - 1 - t >= 0 ? n - 1 - t : 0;
    pA[t] = Uj[r * rs];
    uA[t] = Uj[r * rs + 1];
    vA[t] = Uj[r * rs + 2];
    yB[t] = Y[r * ys + j];
  }
  for (int r0 = n - 1; r0 >= 0; r0 -= 8) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = r0 - t;
      if (r >= 0) {
        double yr = (yB[t] - uA[t] * y1 - vA[t] * y2) * pA[t];
        if (fabs(yr) > 1e150) {  // keep the partial solution representable
          for (int q = r + 1; q < n; ++q) Y[q * ys + j] *= 1e-150;
          y1 *= 1e-150;
          y2 *= 1e-150;
          ss *= 1e-300;
          yr *= 1e-150;
        }
        Y[r * ys + j] = yr;
        ss = fma(yr, yr, ss);
        y2 = y1;
        y1 = yr;
      }
      const int rn = r - 8 >= 0 ? r - 8 : 0;
      pA[t] = Uj[rn * rs];
      uA[t] = Uj[rn * rs + 1];
      vA[t] = Uj[rn * rs + 2];
      yB[t] = Y[rn * ys + j];
    }
  }
  const double sc = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  for (int r = 0; r < n; ++r) Y[r * ys + j] *= sc;
}

// Orthonormalises the D vectors of Y in order, Y <- Y R^-1 with R^T R = Y^T Y
// (Cholesky QR: vector j keeps the part of itself orthogonal to vectors
// 0..j-1, as in Gram-Schmidt).  A vector that is dependent on its
// predecessors (pivot below 1e-28 of its squared norm) is left unnormalised
// and unused by the later ones.  One pass loses about eps * cond(Y)^2 of
// orthogonality; call it twice.  R: ys * ys doubles of LDS (ys odd, so that
// the row and the column accesses of Y avoid bank conflicts), rk: 64 doubles
// of LDS.
//
// D <= 16: lane (i4, j) = (lane / 16, lane % 16) forms the Gram entries
// (i4 + 4u, j), four independent sums over the rows; lane j then factors
// column j of the Gram in registers, row k of R broadcast through rk, and
// every lane solves its row of Y against R.  Larger D: lane j forms column j
// of the Gram and the factorisation runs by rows of R in LDS.
__device__ __forceinline__ void wave_cholqr(int n, int D, double* Y, int ys, double* R, double* rk) {
  const int lane = threadIdx.x;
  if (D <= 16) {
    const int jj = lane & 15, iq = lane >> 4;
    const int jc = jj < D ? jj : D - 1;
    int ic[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) ic[u] = iq + 4 * u < D ? iq + 4 * u : D - 1;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int r = 0; r < n; ++r) {
      const double yj = Y[r * ys + jc];
#pragma unroll
      for (int u = 0; u < 4; ++u) g[u] = fma(Y[r * ys + ic[u]], yj, g[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (iq + 4 * u < D && jj < D) R[(iq + 4 * u) * ys + jj] = g[u];
    __syncthreads();
    const bool col = lane < D;
    const int cl = col ? lane : 0;
    double c[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] = (col && i < D) ? R[(i < D ? i : 0) * ys + cl] : 0.0;
    const double gjj = R[cl * ys + cl];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k < D) {  // uniform; no early exit, so the loops unroll fully
        const double g0 = wave_bcast(c[k], k);
        const bool ok = g0 > 1e-28 * wave_bcast(gjj, k) && g0 > 0.0;
        const double rkk = ok ? sqrt(g0) : 1.0;
        const double rinv = 1.0 / rkk;
        const double rkj = lane == k ? rkk : (lane > k && ok ? c[k] * rinv : 0.0);
        c[k] = rkj;
        rk[lane] = rkj;
        __syncthreads();
        double rr[16];
#pragma unroll
        for (int i = k + 1; i < 16; ++i) rr[i] = rk[i];
#pragma unroll
        for (int i = k + 1; i < 16; ++i) c[i] = lane >= i ? fma(-rr[i], rkj, c[i]) : c[i];
        __syncthreads();
      }
    }
    // column j of R back to LDS, with the reciprocal diagonal in rk
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (col && i <= lane) R[i * ys + cl] = c[i];
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i == lane && col) rk[lane] = 1.0 / c[i];
    __syncthreads();
    if (lane < n) {
      double y[16];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) y[cc] = cc < D ? Y[lane * ys + cc] : 0.0;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) {
        if (cc < D) {
          double v = y[cc];
#pragma unroll
          for (int i = 0; i < cc; ++i) v = fma(-y[i], R[i * ys + cc], v);
          y[cc] = v * rk[cc];
        }
      }
#pragma unroll
      for (int cc = 0; cc < 16; ++cc)
        if (cc < D) Y[lane * ys + cc] = y[cc];
    }
    __syncthreads();
    return;
  }
  const int j = lane;
  double gjj = 0.0;  // squared norm of vector j, for the breakdown test
  if (j < D)
    for (int i = 0; i <= j; ++i) {
      double g = 0.0;
      for (int r = 0; r < n; ++r) g += Y[r * ys + i] * Y[r * ys + j];
      R[i * ys + j] = g;
      gjj = g;
    }
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    const double g0 = R[k * ys + k];
    const bool ok = g0 > 1e-28 * wave_bcast(gjj, k) && g0 > 0.0;
    const double rkk = ok ? sqrt(g0) : 1.0;
    __syncthreads();
    if (j >= k && j < D) R[k * ys + j] = j == k ? rkk : (ok ? R[k * ys + j] / rkk : 0.0);
    __syncthreads();
    if (j > k && j < D) {
      const double rkj = R[k * ys + j];
      for (int i = k + 1; i <= j; ++i) R[i * ys + j] -= R[k * ys + i] * rkj;
    }
    __syncthreads();
  }
  if (j < n)
    for (int c = 0; c < D; ++c) {
      double v = Y[j * ys + c];
      for (int i = 0; i < c; ++i) v -= Y[j * ys + i] * R[i * ys + c];
      Y[j * ys + c] = v / R[c * ys + c];
    }
  __syncthreads();
}

// Eigenvectors of T for lam[0..D) (D <= 64) by inverse iteration: lane j
// factors T - lam_j I by Gaussian elimination with partial pivoting (pivots
// below tiny = 4 ulp * nrm raised to tiny) and solves once from a
// pseudo-random start (the shift is within a few ulps of the norm, so one
// solve already leaves other eigenvectors at about ulp / gap); the D vectors are orthonormalised (Cholesky QR once:
// it only has to separate the members of a cluster), solved once more (which
// removes what the orthogonalisation of a nearly dependent member amplified
// outside the cluster) and orthonormalised again, twice.  Vector j is Y[r * ys + j] (LDS, ys odd); R: ys * ys
// doubles of LDS; de: 2 * 64 doubles of LDS; rk: 64 doubles of LDS; U:
// 4 * n * ys doubles of scratch, four per row and lane.
__device__ void wave_tri_vectors(double dr, double er, int n, int D, double nrm, const double* lam, double* de,
                                 double* Y, int ys, double* R, double* rk, double* U) {
  const int j = threadIdx.x;
  if (j < n) {
    de[2 * j] = dr;
    de[2 * j + 1] = j + 1 < n ? er : 0.0;
  }
  __syncthreads();
  const double tiny = 4.0 * 2.220446049250313e-16 * fmax(nrm, 1e-300);
  unsigned long long swm = 0;
  if (j < D) {
    const double lj = lam[j];
    double cp = de[0] - lj, cq = de[1];
#pragma unroll 4
    for (int r = 0; r + 1 < n; ++r) {
      const double sub = de[2 * r + 1], nd = de[2 * r + 2] - lj, ns = de[2 * r + 3];
      const bool sw = fabs(cp) < fabs(sub);
      const double piv = sw ? sub : (fabs(cp) < tiny ? (cp < 0.0 ? -tiny : tiny) : cp);
      const double rp = approx_rcp(piv);
      const double m = (sw ? cp : sub) * rp;
      double* u = U + (r * ys + j) * 4;
      u[0] = rp;
      u[1] = sw ? nd : cq;
      u[2] = sw ? ns : 0.0;
      u[3] = m;
      if (sw) swm |= 1ull << r;
      const double ncp = sw ? fma(-m, nd, cq) : fma(-m, cq, nd);
      cq = sw ? -m * ns : ns;
      cp = ncp;
    }
    double* u = U + ((n - 1) * ys + j) * 4;
    u[0] = approx_rcp(fabs(cp) < tiny ? (cp < 0.0 ? -tiny : tiny) : cp);
    u[1] = 0.0;
    u[2] = 0.0;
    u[3] = 0.0;
    for (int r = 0; r < n; ++r) {  // start vector: an integer mixing hash of (r, j)
      unsigned h = unsigned(r) * 0x9e3779b1u + unsigned(j) * 0x85ebca77u + 0x165667b1u;
      h ^= h >> 15;
      h *= 0x2c1b3c6du;
      h ^= h >> 12;
      h *= 0x297a2d39u;
      h ^= h >> 15;
      Y[r * ys + j] = double(h >> 8) * (1.0 / 16777216.0) - 0.5;
    }
  }
  // a solve and one orthonormalisation, then a solve and two more (one
  // inlined copy of each step)
  for (int round = 0; round < 2; ++round) {
    if (j < D)
      tri_solve(n, U, Y, ys, j, swm);
    __syncthreads();
    for (int pass = 1 - round; pass < 2; ++pass) wave_cholqr(n, D, Y, ys, R, rk);
  }
}

template <int T>
__device__ __forceinline__ double quad_sum(double v) {
  if (T >= 2) v += dpp_move<0xB1>(v);  // quad_perm [1,0,3,2]
  if (T >= 4) v += dpp_move<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}

// x <- Q x for the D <= 64 / LPV vectors of Y, Q = H_0 ... H_{n-3} with
// H_k = I - beta_k v_k v_k^T, v_k in row k of Hv (stride n, zero at and above
// component k) and beta_k in lane k's br.  LPV consecutive lanes share a
// vector, each holding 64 / LPV consecutive rows of it in registers.  The
// reflectors are staged through hb (8 * 72 doubles of 16-byte aligned LDS, a
// padded row per reflector) eight at a time, the next eight loaded from
// global memory into registers while the current eight are applied.
template <int LPV>
__device__ void tri_backtransform_regs(const double* Hv, double br, int n, int D, double* Y, int ys, double* hb) {
  constexpr int RPL = 64 / LPV;
  const int lane = threadIdx.x;
  const int j = lane / LPV, q = lane - j * LPV;
  const bool act = j < D;
  const int r0 = q * RPL;
  const int off = r0 + 2 * (r0 / 16);  // padded position of row r0 in an hb row
  const int jc = act ? j : 0;
  double y[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = r0 + t;
    y[t] = (act && r < n) ? Y[(r < n ? r : 0) * ys + jc] : 0.0;
  }
  const int nk = n - 2;  // reflectors k = n-3 .. 0
  const int ng = nk > 0 ? (nk + 7) / 8 : 0;
  const int lc = lane < n ? lane : n - 1;
  const int lpos = lane + 2 * (lane / 16);
  double pf[8];
  if (ng > 0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = n - 3 - s;
      pf[s] = Hv[(k >= 0 ? k : 0) * n + lc] * ((k >= 0 && lane < n) ? 1.0 : 0.0);
    }
  }
  for (int g = 0; g < ng; ++g) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) hb[s * 72 + lpos] = pf[s];
    if (g + 1 < ng) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = n - 3 - 8 * (g + 1) - s;
        pf[s] = Hv[(k >= 0 ? k : 0) * n + lc] * ((k >= 0 && lane < n) ? 1.0 : 0.0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = n - 3 - 8 * g - s;
      if (k < 0) break;
      const double bk = wave_bcast(br, k);
      const double2* h2 = reinterpret_cast<const double2*>(hb + s * 72 + off);
      double vv[RPL];
#pragma unroll
      for (int t = 0; t < RPL / 2; ++t) {
        const double2 x = h2[t + t / 8];  // rows r0 + 2t, r0 + 2t + 1 (two pad doubles per 16 rows)
        vv[2 * t] = x.x;
        vv[2 * t + 1] = x.y;
      }
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; t += 2) {
        d0 = fma(vv[t], y[t], d0);
        d1 = fma(vv[t + 1], y[t + 1], d1);
      }
      const double sd = quad_sum<LPV>(d0 + d1) * bk;
#pragma unroll
      for (int t = 0; t < RPL; ++t) y[t] = fma(-sd, vv[t], y[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = r0 + t;
    if (act && r < n) Y[r * ys + j] = y[t];
  }
  __syncthreads();
}

// x <- Q x for the D vectors of Y (see tri_backtransform_regs); one lane per
// vector for D > 32.
__device__ void wave_tri_backtransform(const double* Hv, double br, int n, int D, double* Y, int ys, double* hb) {
  if (D <= 16) {
    tri_backtransform_regs<4>(Hv, br, n, D, Y, ys, hb);
    return;
  }
  if (D <= 32) {
    tri_backtransform_regs<2>(Hv, br, n, D, Y, ys, hb);
    return;
  }
  const int j = threadIdx.x;
  for (int k = n - 3; k >= 0; --k) {
    const double bk = wave_bcast(br, k);
    if (bk == 0.0) continue;
    const double* v = Hv + k * n;
    if (j < D) {
      double sdot = 0.0;
      for (int r = k + 1; r < n; ++r) sdot += v[r] * Y[r * ys + j];
      sdot *= bk;
      for (int r = k + 1; r < n; ++r) Y[r * ys + j] -= sdot * v[r];
    }
  }
  __syncthreads();
}

// 1 / sqrt(x) for x >= 1 from the hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// All eigenpairs of a symmetric n x n matrix (1 <= n <= 16) in one wavefront
// by the cyclic Jacobi method: n rounded up to even, nn, players meet in the
// round-robin order, nn / 2 disjoint plane rotations per step and nn - 1
// steps per sweep, each rotation the one that zeroes its off-diagonal pair
// (the symmetric Schur decomposition of the 2 x 2 block; cos = 1 / sqrt(1 +
// t^2) to working precision, so the rotation is orthogonal whatever the
// rounding of t).  A pair is skipped when its entry is below 2^-53
// sqrt(|a_pp a_qq|) or below 1e-18 (the matrix is expected scaled to a
// largest diagonal entry of about 1); the sweeps stop when a whole sweep is
// skipped, after at most 40.  Lane (q, c) = (lane / 16, lane % 16) updates rows
// q, q + 4, q + 8, q + 12 of column c of A <- J^T A J and of V <- V J in one
// pass from the old entries.  A and V: 16 x 17 doubles of LDS each (row stride
// 17); A holds the matrix, zero outside n x n; on return its diagonal holds
// the eigenvalues and column i of V the eigenvector of A[i][i].  rot: 32
// doubles of LDS, part: 16 ints of LDS.  Returns the number of sweeps.
__device__ int wave_jacobi16(double* A, double* V, int n, double* rot, int* part) {
  const int lane = threadIdx.x, c = lane & 15, q = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) V[(q + 4 * t) * 17 + c] = q + 4 * t == c ? 1.0 : 0.0;
  __syncthreads();
  if (n < 2) return 0;
  const int nn = (n + 1) & ~1, m = nn - 1;
  int sw = 0;
  for (; sw < 40; ++sw) {
    bool turned = false;
    for (int st = 0; st < m; ++st) {
      if (lane < nn) {
        // partner of player i in step st: the last player meets st, the others
        // i and j with i + j = 2 st (mod nn - 1)
        const int i = lane;
        int p;
        if (i == m) {
          p = st;
        } else {
          int j = (2 * st - i) % m;
          if (j < 0) j += m;
          p = j == i ? m : j;
        }
        const int lo = i < p ? i : p, hi = i < p ? p : i;
        const double a = A[lo * 18], b = A[hi * 18], o = A[lo * 17 + hi];
        double cr = 1.0, sr = 0.0;
        if (fabs(o) > 1e-18 && fabs(o) > 0x1p-53 * sqrt(fabs(a * b))) {
          const double tau = (b - a) * approx_rcp(2.0 * o);
          const double at = fabs(tau);
          // t = sign(tau) / (|tau| + sqrt(1 + tau^2)), the smaller root
          double t;
          if (at < 1e100) {
            const double x = fma(tau, tau, 1.0);
            t = approx_rcp(at + x * rsqrt_nr(x));
          } else {
            t = 0.5 / at;
          }
          if (tau < 0.0) t = -t;
          const double cv = rsqrt_nr(fma(t, t, 1.0));
          cr = cv;
          sr = i == lo ? -t * cv : t * cv;  // new column i = cr col_i + sr col_p
          turned = true;
        }
        part[i] = p;
        rot[i] = cr;
        rot[16 + i] = sr;
      }
      __syncthreads();
      // A'[r][c] = sum over r0 in {r, pr}, c0 in {c, pc} of J[r0][r] A[r0][c0] J[c0][c]
      const bool cin = c < nn;
      const int pc = cin ? part[c] : c;
      const double cc = cin ? rot[c] : 1.0, sc = cin ? rot[16 + c] : 0.0;
      double h[4], v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = q + 4 * t;
        const bool rin = r < nn;
        const int pr = rin ? part[r] : r;
        const double cq = rin ? rot[r] : 1.0, sq = rin ? rot[16 + r] : 0.0;
        const double rowr = fma(cc, A[r * 17 + c], sc * A[r * 17 + pc]);
        const double rowp = fma(cc, A[pr * 17 + c], sc * A[pr * 17 + pc]);
        h[t] = (pr == c && r != c && sq != 0.0) ? 0.0 : fma(cq, rowr, sq * rowp);
        v[t] = fma(cc, V[r * 17 + c], sc * V[r * 17 + pc]);
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = q + 4 * t;
        A[r * 17 + c] = h[t];
        V[r * 17 + c] = v[t];
      }
      __syncthreads();
    }
    if (wave_first(turned) == 64) break;
  }
  return sw;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = team_sum(v, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Multi-wavefront version of wave_sym_eig for larger n: the reduction to
// tridiagonal form and the accumulation of Q use the whole workgroup; in the
// QL phase each wavefront repeats the scalar recurrence on its own copy of
// (d, e) (dw: 2 n doubles per wavefront) and rotates only the rows of Z its
// lanes own (row k belongs to thread k mod blockDim, at most 4 rows each),
// carrying the moving column in registers.  red: 16 doubles.
__device__ int block_sym_eig(double* A, int n, double* Z, double* d, double* e, double* beta, double* dw,
                             double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // A stays symmetric (the whole trailing block is updated), so row k stands
  // for column k and thread i updates column i: every access below runs
  // along a row across the threads
  for (int k = 0; k + 2 < n; ++k) {
    double q = 0.0;
    for (int i = k + 1 + tid; i < n; i += nt) q += A[k * n + i] * A[k * n + i];
    const double sigma = block_sum(q, red);
    const double x0 = A[(k + 1) * n + k];
    __syncthreads();
    if (!(sigma > 0.0) || sigma - x0 * x0 <= 1e-300) {
      if (tid == 0) {
        e[k] = x0;
        beta[k] = 0.0;
      }
      __syncthreads();
      continue;
    }
    const double alpha = x0 >= 0.0 ? -sqrt(sigma) : sqrt(sigma);
    const double bk = 1.0 / (sigma - x0 * alpha);
    if (tid == 0) {
      A[(k + 1) * n + k] = x0 - alpha;  // the reflector, in column k (read back below)
      A[k * n + k + 1] = x0 - alpha;    // and in row k (read here)
      e[k] = alpha;
      beta[k] = bk;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = k + 1 + tid; i < n; i += nt) {
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += A[j * n + i] * A[k * n + j];
      acc *= bk;
      Z[k * n + i] = acc;
      pv += acc * A[k * n + i];
    }
    const double K = 0.5 * bk * block_sum(pv, red);
    for (int i = k + 1 + tid; i < n; i += nt) Z[k * n + i] -= K * A[k * n + i];
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += nt) {
      const double vi = A[k * n + i], wi = Z[k * n + i];
      for (int j = k + 1; j < n; ++j) A[j * n + i] -= A[k * n + j] * wi + Z[k * n + j] * vi;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += nt) d[i] = A[i * n + i];
  if (tid == 0) {
    if (n >= 2) e[n - 2] = A[(n - 1) * n + n - 2];
    e[n - 1] = 0.0;
    if (n >= 2) beta[n - 2] = 0.0;
    beta[n - 1] = 0.0;
  }
  __syncthreads();
  for (int x = tid; x < n * n; x += nt) Z[x] = (x / n == x % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double bk = beta[k];
    if (bk == 0.0) continue;
    for (int j = k + 1 + tid; j < n; j += nt) {
      double u = 0.0;
      for (int i = k + 1; i < n; ++i) u += A[i * n + k] * Z[i * n + j];
      u *= bk;
      for (int i = k + 1; i < n; ++i) Z[i * n + j] -= u * A[i * n + k];
    }
    __syncthreads();
  }
  // QL: per-wavefront copies of (d, e)
  const int w = tid >> 6;
  double* dd = dw + size_t(w) * 2 * n;
  double* ee = dd + n;
  const int ws = nt < 64 ? nt : 64;
  for (int i = tid % ws; i < n; i += ws) {
    dd[i] = d[i];
    ee[i] = e[i];
  }
  __syncthreads();
#ifndef TN3D_EIG_RPT
#define TN3D_EIG_RPT 4
#endif
  constexpr int RPT = TN3D_EIG_RPT;
  int fail = 0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double sm = fabs(dd[m]) + fabs(dd[m + 1]);
        if (fabs(ee[m]) <= 1e-16 * sm || ee[m] == 0.0) break;
      }
      if (m == l) break;
      if (iter >= 60) {
        fail = 1;
        break;
      }
      double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
      double r = hypot(g, 1.0);
      g = dd[m] - dd[l] + ee[l] / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, p = 0.0;
      double zc[RPT];
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int kr = tid + j * nt;
        zc[j] = kr < n ? Z[kr * n + m] : 0.0;
      }
      bool early = false;
      int i = m - 1;
      for (; i >= l; --i) {
        double zi[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int kr = tid + j * nt;
          zi[j] = kr < n ? Z[kr * n + i] : 0.0;
        }
        const double f = sn * ee[i], b = cs * ee[i];
        r = hypot(f, g);
        ee[i + 1] = r;
        if (r == 0.0) {
          dd[i + 1] -= p;
          ee[m] = 0.0;
          early = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = dd[i + 1] - p;
        r = (dd[i] - g) * sn + 2.0 * cs * b;
        p = sn * r;
        dd[i + 1] = g + p;
        g = cs * r - b;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const int kr = tid + j * nt;
          if (kr < n) Z[kr * n + i + 1] = sn * zi[j] + cs * zc[j];
          zc[j] = cs * zi[j] - sn * zc[j];
        }
      }
      // write back the carried column (i + 1 after an early exit, l otherwise)
      const int col = early ? i + 1 : l;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int kr = tid + j * nt;
        if (kr < n) Z[kr * n + col] = zc[j];
      }
      if (early) continue;
      dd[l] -= p;
      ee[l] = g;
      ee[m] = 0.0;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) d[i] = dw[i];
  __syncthreads();
  return fail;
}

// Orders the LDS accesses of the lanes of one wavefront (they execute in
// program order; the fence keeps the compiler from moving them).
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Householder QR, one block of rows (Golub and Van Loan, Sec. 5.2, applied to
// a triangular factor stacked on new rows): F (n x n, upper triangular, row
// stride n, in LDS, shared by the TL lanes of a team of one wavefront) is
// replaced by the triangular factor of [F; B] for the RB x n block B, whose
// column l lane l holds in b[] (n <= TL).  sg: the lane's sum of b[i]^2.
// Reflector j acts on row j of F and the rows of B only (F is triangular):
// with alpha = F[j][j], mu = sqrt(alpha^2 + |B_j|^2) and beta = -sign(alpha) mu,
// v = [1; B_j / (alpha - beta)], tau = (beta - alpha) / beta; every column
// l > j is updated by w = F[j][l] + v.B_l, F[j][l] -= tau w, B_l -= tau w v.
// vb: RB + 1 doubles of LDS for the broadcast reflector.  So F^T F gains
// B^T B exactly in exact arithmetic, with the backward stability of an
// orthogonal factorisation (no Gram matrix is formed).
template <int TL, int RB>
__device__ __forceinline__ void tsqr_block(double* F, int n, double (&b)[RB], double sg, double* vb, int l) {
  for (int j = 0; j < n; ++j) {
    if (l == j) {
      const double al = F[j * n + j];
      double be = al, tau = 0.0, sc = 0.0;
      if (sg > 0.0) {
        const double mu = sqrt(fma(al, al, sg));
        be = al > 0.0 ? -mu : mu;
        tau = (be - al) / be;
        sc = 1.0 / (al - be);
      }
      F[j * n + j] = be;
#pragma unroll
      for (int i = 0; i < RB; ++i) vb[i] = b[i] * sc;
      vb[RB] = tau;
    }
    team_sync();
    const double tau = vb[RB];
    if (l > j && l < n && tau != 0.0) {
      double w = F[j * n + l];
#pragma unroll
      for (int i = 0; i < RB; ++i) w = fma(vb[i], b[i], w);
      F[j * n + l] = fma(-tau, w, F[j * n + l]);
      const double tw = tau * w;
      sg = 0.0;
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        b[i] = fma(-tw, vb[i], b[i]);
        sg = fma(b[i], b[i], sg);
      }
    }
    team_sync();
  }
}

// F <- triangular factor of [F; Y] for the nrows x n matrix Y given by
// yv(row, col), streamed RB rows at a time (see tsqr_block).  Every lane of
// the team calls it.
template <int TL, int RB, class YF>
__device__ void team_tsqr(double* F, int n, int nrows, YF yv, double* vb, int l) {
  for (int r0 = 0; r0 < nrows; r0 += RB) {
    double b[RB];
    double sg = 0.0;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      b[i] = (l < n && r0 + i < nrows) ? yv(r0 + i, l) : 0.0;
      sg = fma(b[i], b[i], sg);
    }
    tsqr_block<TL, RB>(F, n, b, sg, vb, l);
  }
}

}  // namespace tn3d
