// Device-side state of a batch of sweeps and the host launchers of the
// sweep kernels.  One "sweep" is one (syndrome, coset) network.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "program.h"

namespace tn3d {

struct SweepArgs {
  int32_t n_sweeps, n_sites, n_bonds, n_cosets, chi, Lx, Ly;
  int64_t sweep_stride;     // site-tensor elements per sweep per buffer
  const int64_t* site_off;  // [n_sites] offset of each site within a sweep
  void* buf0;               // site tensors, parity 0
  void* buf1;               // site tensors, parity 1
  int32_t* bond_dim;        // [sweep][n_bonds]
  double* lam;              // [sweep][n_bonds][lam_ld]
  int32_t lam_ld;           // entries per bond in lam: the bond capacity max(chi, 2)
  double* logb;             // [sweep][n_bonds] sum of log S_1 of the gates on the bond
  double* logs;             // [sweep][n_sites] sum of log rescale factors
  uint32_t* flags;          // [sweep]
  const int32_t* leg_bond;  // [site][4]
  const uint8_t* synd;      // syndrome bits
  const int64_t* synd_off;  // [global item] offset into synd
  const int32_t* items;     // [local item] -> global item
  const double* pool;       // op matrices and initial tensors
  const int32_t* psel;      // null, or per item (indexed as synd_off) the copy of the pool it reads
  int64_t pool_stride;      // doubles per pool copy
  double eps, tau, pchol_tol;
  int32_t qr;                     // 1: truncation factors by Householder QR (FP64 route), 0: through Grams
  int32_t inc0, n_inc;            // consistency bits of an item (Program::inc0, n_inc)
  int32_t wht;                    // 1: the two sweeps of an item are the signed networks Z_0, Z_1
  int32_t chi_cut;                // rank-rule cap of the truncations of this layer (<= chi)
  double* solve_big;              // truncations of order above 64: one n x n matrix per (sweep, gate)
  int64_t sbig_ld;                // its doubles per (sweep, gate)
  double jtol, jfloor;            // one-sided Jacobi: orthogonality tolerance, noise floor
  unsigned long long* bytes_ctr;  // 64 counters (indexed by workgroup) or null
  int32_t* sweeps_max;            // [2] most Jacobi sweeps (sweep truncations, boundary MPS)
  int32_t* gate_n;                // [sweep][gate of the class] K D before the gate (set by the Gram)
  unsigned long long* win;        // execution window of this launch (see k_win_init) or null
};

struct ZipArgs {
  int32_t n_sweeps, Lx, Ly, chi_m, n_bonds;
  const double* fin;        // final site tensors [sweep][fin_stride], T[w][e][n][s]
  int64_t fin_stride;
  const int64_t* fin_off;   // [n_sites]
  const int32_t* bond_dim;
  double* mps0;             // boundary MPS, two row buffers [sweep][Lx][mcap]
  double* mps1;
  int64_t mcap;
  int32_t* mdim;            // [sweep][2][Lx][3]
  double* K;                // [sweep][kcap] carry, dims in kdim
  int64_t kcap;
  int32_t* kdim;            // [sweep][3]
  double* L4;               // [sweep][bigcap]
  double* Th;
  double* Jm;               // [sweep][jcap] Jacobi vectors (FP64) / solver scratch (FP32)
  int64_t bigcap;
  int64_t jcap;
  int32_t eig_ys;           // FP32: row stride of the eigenvector block, odd, >= min(chi_m, 64)
  double* logm;             // [sweep]
  uint32_t* flags;
  double eps, tau;
  double jtol, jfloor;
  int32_t gram_path;        // 1: FP32 mode, step SVDs through the Gram of the smaller family
  int32_t* sweeps_max;
  double* Gm;               // [sweep][bigcap] that Gram
  int32_t* zdim;            // [sweep][12] shapes passed between the step kernels
  double* zS;               // [sweep][1024] singular values of the step
  unsigned long long* flop_ctr;  // 64 counters of algorithmic flops of the decomposition, or null
  unsigned long long* win;       // execution window of the decomposition launch, or null
  double sub_tol;                // subspace iteration: residual bound relative to the largest eigenvalue
  int32_t bf_theta;              // 1: Theta on the BF16 matrix cores (reduced precisions)
  unsigned long long* win_a;     // execution window of the contraction launch (k_zip_a), or null
  unsigned long long* flop_a;    // 64 counters of the contraction's algorithmic flops, or null
  unsigned long long* win_b;     // execution window of the subspace-iteration launch (k_zip_bsub), or null
  unsigned long long* flop_b;    // 64 counters of its algorithmic flops, or null
};

// Raises the dynamic-LDS limits of the kernels that need more than 64 KB;
// call once per device before any launch (and outside stream capture).
hipError_t set_kernel_lds_limits();

// Launchers (all enqueue on `st`).  T: 0 = double, 1 = float storage.
void launch_init(int prec, const SweepArgs& A, const int32_t* init_dims, const int32_t* init_off,
                 const int32_t* bond_dim0, hipStream_t st);
void launch_onesite(int prec, const SweepArgs& A, const DevOneSite* ops, int n_ops, hipStream_t st);
// n_wide (and n_w16, n_w32 below): the leading gates of the class whose Grams
// (rows) can be wider than 32 (16, 32) entries; the others are never wider
// (A.qr: the triangular factors of k_qr instead of the Grams)
void launch_gram(int prec, const SweepArgs& A, const DevGate* gates, int n_g, int n_w16, int n_wide, int n_w64,
                 double* gout, int ncap, hipStream_t st);
// Launch-shape choices of the layer absorption (the autotuner's search
// space): team = 1 runs truncations of order <= 8 eight per wavefront;
// truncations of order up to mid (8 or 16) run on one wavefront, larger ones
// on four; narrow = 1 gives rows of at most 16 entries their own
// reabsorption class.
struct LaunchTuning {
  int32_t team = 1, mid = 16, narrow = 1;
};

void launch_solve(const LaunchTuning& T, const SweepArgs& A, const DevGate* gates, int n_g, const double* gin,
                  double* wout,
                  int ncap, int kdcap, hipStream_t st);
void launch_reabsorb(const LaunchTuning& T, int prec, const SweepArgs& A, const DevGate* gates, int n_g, int n_w16,
                     int n_w32, int n_w64,
                     const double* win, int ncap, hipStream_t st);
void launch_rescale(int prec, const SweepArgs& A, const int32_t* d_after, const int32_t* par_after,
                    hipStream_t st);
void launch_finalize(int prec, const SweepArgs& A, const int32_t* d_final, const int32_t* f_off,
                     const int32_t* par_final, double* fin, int64_t fin_stride, const int64_t* fin_off,
                     hipStream_t st);
void launch_zip_init(const ZipArgs& Z, hipStream_t st);
// one zip-up step (x, y) of the boundary MPS: contraction, decomposition (all
// but the last column), new site and carry; legcap bounds the network's bonds
void launch_zip_step(const ZipArgs& Z, int x, int y, int legcap, hipStream_t st);
// Whether step (x, y) decomposes a family above 64 vectors: 1 by subspace
// iteration (k_zip_bsub), 2 by the full eigen-decomposition (k_zip_bbig), 0 not.
int zip_step_large(const ZipArgs& Z, int x, int y, int legcap);
void launch_finish(const SweepArgs& A, const ZipArgs& Z, double* logp, uint32_t* flags_out, hipStream_t st);
// Graph replay helpers: gather each item's syndrome into a dense buffer,
// local item indices with their offsets, zero a counter block (no memset
// node in a captured graph), and scatter the local results to the caller.
void launch_gather_synd(int n, const int32_t* items, const uint8_t* synd, const int64_t* offs, int n_det,
                        int64_t stride, uint8_t* out, hipStream_t st);
// Derived bits n_det + e, e < n_ext, of n items laid out at `stride` bytes
// (Program::ext_rows; words <= EXT_MAXW).
constexpr int EXT_MAXW = 64;
void launch_ext_bits(int n, uint8_t* bits, int64_t stride, int n_det, int src0, int src_n, int words,
                     const uint64_t* rows, int n_ext, hipStream_t st);
void launch_seq(int n, int32_t* items, int64_t* offs, int64_t stride, hipStream_t st);
// Writes the device wall clock (hipDeviceAttributeWallClockRate ticks) to *out.
void launch_stamp(unsigned long long* out, hipStream_t st);
// Execution windows: n windows of 128 words, words 0..63 the earliest start
// and 64..127 the latest end (device wall clock) over the workgroups of the
// launches that record into it, spread over 64 slots by workgroup.
void launch_win_init(unsigned long long* win, int n, hipStream_t st);
// Adds one contraction's times to acc: acc[0] layers (stamps 0..1), acc[1]
// boundary MPS (stamps 1..2), acc[2] the windows [0, n_cls_win) (Gram and
// reabsorption), acc[4] bytes (ctr[0..64)), acc[5] the decomposition windows
// of steps x < Lx - 1 (if eig, windows n_cls_win + step), acc[7] their flops
// (ctr[65..129)), acc[8] the contraction windows (n_cls_win + Lx Ly + step),
// acc[9] their flops (ctr[129..193)), acc[10] the subspace-iteration windows
// (n_cls_win + 2 Lx Ly + step), acc[11] their flops (ctr[193..257));
// milliseconds.
void launch_timing_reduce(const unsigned long long* stamps, const unsigned long long* win, int n_cls_win, int Lx,
                          int Ly, int eig, const unsigned long long* ctr, double ms_per_tick, double* acc,
                          hipStream_t st);
void launch_zero_words(uint32_t* p, int n, hipStream_t st);
void launch_scatter_out(int n, const int32_t* items, const double* lp_local, const uint32_t* fl_local, double* logp,
                        uint32_t* flags, hipStream_t st);
// Near-tie FP64 re-sweep helpers: the items whose log-ratio is below
// near_tie (or NaN), their syndrome offsets, and the write-back of the
// re-swept rows (flags of the FP64 sweep plus the re-swept bit 16).
void launch_pick_ties(int n_items, const double* logratio, double near_tie, int32_t* list, int32_t* count,
                      hipStream_t st);
void launch_gather_offsets(int n, const int32_t* items, const int64_t* offs, int64_t* out, hipStream_t st);
void launch_gather_i32(int n, const int32_t* items, const int32_t* src, int32_t* out, hipStream_t st);
void launch_scatter_resweep(int n, const int32_t* items, const double* logp_sub, const uint32_t* flags_sub,
                            double* logp, uint32_t* flags, hipStream_t st);
void launch_decode(int n_items, int n_cosets, const int32_t* items, const double* logp, double near_tie,
                   int32_t* coset, double* logratio, uint32_t* flags, hipStream_t st);

// Gradient of log P(m) (k_grad_terms, k_grad_items, k_grad_reduce): lp and
// fl hold (n + 1) blocks of B items (block 0 at the given rates, block i + 1
// with rate i at cp[2 i]); cp[2 i + 1] = p_i; rate k sums the mechanisms
// rm[ptr[k] .. ptr[k + 1]).  term: [B][n] per-item derivatives; loglik
// ([B]), total (the sum of loglik) and flags nullable.
void launch_grad(int B, int n, int nc, int n_rates, const double* lp, const uint32_t* fl, const double* cp,
                 const int32_t* ptr, const int32_t* rm, double* term, double* grad, double* loglik, double* total,
                 uint32_t* flags, hipStream_t st);
void launch_tile_offsets(int B, int n_blocks, const int64_t* offs, int64_t* offs_all, hipStream_t st);

}  // namespace tn3d
