// Workgroup-level dense linear algebra in FP64 for the small truncation
// problems of the sweep.  Every function is called by all threads of the
// workgroup with identical arguments and contains its own barriers.
#pragma once

#include <hip/hip_runtime.h>

namespace tn3d {

__device__ __forceinline__ double team_sum(double v, int team) {
  for (int o = team >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pivoted Cholesky of the symmetric positive semidefinite n x n matrix Z
// (row-major, leading dimension n; destroyed).  Writes F (r x n, row-major,
// leading dimension n) with F^T F = Z up to the dropped trailing part, in the
// original column order, and returns the rank r: elimination stops when the
// largest remaining diagonal is <= tol * max(diag Z).  perm is scratch of n
// ints, red scratch of 2 doubles.
__device__ int block_pchol(double* Z, double* F, int n, double tol, int* perm, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) perm[i] = i;
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, Z[i * n + i]);
    red[0] = m;
  }
  __syncthreads();
  const double thr = tol * red[0];
  __syncthreads();
  int r = 0;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      int j = k;
      double best = Z[k * n + k];
      for (int i = k + 1; i < n; ++i)
        if (Z[i * n + i] > best) {
          best = Z[i * n + i];
          j = i;
        }
      red[1] = double(j);
      red[0] = best;
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
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += nt) {
      int a = k + 1 + e / m, b = k + 1 + e % m;
      Z[a * n + b] -= Z[k * n + a] * Z[k * n + b];
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
// the identity here), so that A_out = A_in J.  Afterwards the vectors are
// mutually orthogonal to relative precision tol.  Returns the number of sweeps.
__device__ int block_jacobi(double* A, long vs, long es, int nv, int len, double* J, double tol,
                            int max_sweeps, int* flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < nv * nv; e += nt) J[e] = (e / nv == e % nv) ? 1.0 : 0.0;
  const int ne = nv + (nv & 1);
  const int npairs = ne / 2;
  int team = 64;
  while (team > 1 && team * npairs > nt) team >>= 1;
  const int pair = tid / team, lane = tid % team;
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int rnd = 0; rnd < ne - 1; ++rnd) {
      for (int pp = pair; pp < npairs; pp += nt / team) {
        int i, j;
        if (pp == 0) {
          i = ne - 1;
          j = rnd;
        } else {
          i = (rnd + pp) % (ne - 1);
          j = (rnd - pp + ne - 1) % (ne - 1);
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
        if (fabs(g) > tol * sqrt(a * b) && g != 0.0) {
          double zeta = (b - a) / (2.0 * g);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int e = lane; e < len; e += team) {
            double x = A[i * vs + e * es], y = A[j * vs + e * es];
            A[i * vs + e * es] = cs * x - sn * y;
            A[j * vs + e * es] = sn * x + cs * y;
          }
          for (int e = lane; e < nv; e += team) {
            double x = J[e * nv + i], y = J[e * nv + j];
            J[e * nv + i] = cs * x - sn * y;
            J[e * nv + j] = sn * x + cs * y;
          }
          if (lane == 0) *flag = 1;
        }
      }
      __syncthreads();
    }
    if (*flag == 0) break;
    __syncthreads();
  }
  __syncthreads();
  return sweep;
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
      if (S[u] > S[v] || (S[u] == S[v] && u < v)) ++rank;
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

}  // namespace tn3d
