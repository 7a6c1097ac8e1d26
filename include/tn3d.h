/*
 * tn3d.h -- coset probabilities of a detector error model by approximate
 * contraction of a layered 3D tensor network, on one AMD Instinct MI355X
 * (gfx950).
 *
 * The problem (Piveteau, Chubb, Renes, "Tensor Network Decoding Beyond 2D",
 * Sec. 2.3-2.4): for a detector error model (H, p, l) and a detector outcome
 * m, the joint probability of m and logical value L is
 *     p_{m,L} = sum_{x : Hx = m, l.x = L} prod_i p_i^{x_i} (1 - p_i)^{1 - x_i}
 * and the optimal decision is argmax_L p_{m,L}.  The library evaluates
 * log p_{m,L} with the paper's method (Sec. 4): the detector-picture network
 * (Sec. 3.1, 3.3, 3.4) is arranged as a stack of layers, a 2D network absorbs
 * one layer at a time as two-site gates, every gated bond is truncated back to
 * at most chi with simple-update environments, and the remaining 2D network is
 * contracted with a boundary MPS of bond chi_m.  The value is exact when chi
 * and chi_m never truncate and approximate otherwise.
 *
 * Conventions for every entry point:
 *   - Every function returns tn3d_status (0 = TN3D_OK); no C++ exception
 *     crosses this boundary.  On failure tn3d_last_error(ctx) describes it.
 *   - Natural logarithms throughout.
 *   - Pointers named *_dev are device pointers (hipMalloc / torch CUDA
 *     tensors) on the context's device; all other pointers are host memory.
 *     Inputs are read-only and owned by the caller; outputs are allocated by
 *     the caller.  Host inputs are copied before the call returns.
 *   - Device work is enqueued on the context's stream (set at creation; NULL
 *     means the default stream).  Functions that take device outputs return
 *     after enqueueing; synchronise the stream before reading the outputs.
 *   - Calls on one context must not overlap in time (the context owns one
 *     workspace); use one context per host thread.
 */
#ifndef TN3D_H
#define TN3D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TN3D_OK = 0,
  TN3D_E_INVALID = -1,      /* bad argument (null pointer, size out of range) */
  TN3D_E_INCONSISTENT = -2, /* inputs contradict each other */
  TN3D_E_UNSUPPORTED = -3,  /* valid but not implemented (e.g. precision) */
  TN3D_E_OOM = -4,          /* device or host allocation failed */
  TN3D_E_DEVICE = -5,       /* a HIP runtime call failed */
  TN3D_E_NUMERIC = -6       /* reserved; per-item numeric trouble is a flag */
} tn3d_status;

/* Per-item result flags (bitwise OR). */
#define TN3D_FLAG_NUMERIC 1u       /* a value was zero, negative or not finite */
#define TN3D_FLAG_TRUNC_CLUSTER 2u /* a truncation cut inside a cluster of equal singular values */
#define TN3D_FLAG_NEAR_TIE 4u      /* |log ratio| of the decision below params.near_tie */
#define TN3D_FLAG_NO_CONVERGE 8u   /* a Jacobi SVD stopped at its sweep limit */
#define TN3D_FLAG_RESWEPT 16u      /* decode: contracted again in FP64 (near tie of a reduced-precision pass) */
#define TN3D_FLAG_INCONSISTENT 32u /* no error pattern has this syndrome: log p = -inf for every coset */

/* Arithmetic of the layer absorption (site tensors and their contractions).
 * The truncation factorisations, singular values and log accumulators are
 * always FP64.
 *   FP64: FP64 site tensors, Grams on FP64 matrix cores, truncations factored
 *         by Householder QR and one-sided Jacobi (see TN3D_OPT_GRAM_FACTOR).
 *   FP32: FP32 site tensors, Grams on FP64 matrix cores.
 *   BF16: FP32 site tensors; the reabsorption products and the boundary-MPS
 *         contraction Theta on BF16 matrix cores with FP32 accumulation (per
 *         chunk of 32 rows; FP64 across chunks), every operand split into
 *         three BF16 terms so the products keep FP32 accuracy; the Grams on
 *         FP64 matrix cores from the FP32 values (a Gram accumulated in FP32
 *         loses the singular values below about 3e-4 of the largest, which
 *         the reduced rank rule keeps); everything else as FP32. */
#define TN3D_PREC_FP64 0
#define TN3D_PREC_FP32 1
#define TN3D_PREC_BF16 2

/* params.flags bits. */
/* FP64 only: factor the truncations through Gram matrices (MFMA Grams,
 * Cholesky, eigenpairs of boundary-MPS family Grams) instead of orthogonal
 * factorisations (Householder QR of the gate sides, one-sided Jacobi SVD of
 * the boundary-MPS families).  Faster at large chi; a Gram squares the
 * condition of the smallest kept singular values, about 1e-8 in log p
 * instead of about 1e-11.  Reduced precisions always use the Gram route. */
#define TN3D_OPT_GRAM_FACTOR 1u

#define TN3D_MAX_CHI_LAYERS 32

typedef struct tn3d_ctx_s* tn3d_ctx;
typedef struct tn3d_net_s* tn3d_net;

typedef struct {
  int32_t chi;       /* max bond dimension of the swept 2D network (>= 1) */
  int32_t chi_mps;   /* max bond dimension of the final boundary MPS (>= 1) */
  int32_t precision; /* TN3D_PREC_* */
  int32_t reserved0;
  double eps_rel;    /* singular values <= eps_rel * S_1 are dropped */
  double tau_gap;    /* never cut where S_{D+1} >= (1 - tau_gap) S_D */
  double near_tie;   /* decode: flag items whose |log ratio| is below this */
  int64_t workspace_bytes; /* cap on the context workspace (0 = no cap) */
  uint32_t flags;    /* TN3D_OPT_* bits (0 = defaults) */
  uint32_t reserved1;
  /* chi-schedule: when n_chi_layers > 0, the truncations of absorbed layer l
   * (0-based) keep at most chi_layers[min(l, n_chi_layers - 1)] <= chi
   * values; chi stays the capacity and the cap of layers past the list.
   * 0 = the constant chi.  The schedule changes the computed value: a
   * reference must run the same schedule. */
  int32_t n_chi_layers;
  int32_t chi_layers[TN3D_MAX_CHI_LAYERS];
} tn3d_params;

/* Fill *p with the defaults for a precision: eps_rel 1e-9 (FP64) / 1e-6
 * (FP32, BF16), tau_gap 1e-6 / 1e-2, near_tie 4e-3, no workspace cap.  The
 * gap threshold stays well above the rounding of the smallest singular value
 * the rule can keep, so two correct implementations take the same cuts; in
 * the reduced precisions the kept subspace at a cut moves with the FP32
 * rounding of the site tensors by about eps_32 / tau_gap, so their cuts sit
 * only at gaps of a percent. */
void tn3d_params_default(tn3d_params* p, int32_t chi, int32_t chi_mps, int32_t precision);

/* Create a context on HIP device `device`, enqueueing on `stream` (a
 * hipStream_t; NULL = default stream).  The context owns a device workspace
 * that grows on demand.  Errors: TN3D_E_INVALID, TN3D_E_DEVICE. */
tn3d_status tn3d_ctx_create(int32_t device, void* stream, tn3d_ctx* out);
/* Frees the context.  Networks built on it should be destroyed first; any
 * still alive lose their device arrays here and are detached: they can then
 * only be passed to tn3d_net_destroy (which frees the handle). */
void tn3d_ctx_destroy(tn3d_ctx ctx);
/* Text of the last error on this context; owned by the context, valid until
 * its next call. */
const char* tn3d_last_error(tn3d_ctx ctx);

/* Point sector of the 3D planar surface code of size L (paper Sec. 5.1):
 * vertex checks at (x, y, z), x, y in [0, L), z in [1, L), detector index
 * ((z-1) L + y) L + x; qubits on lattice edges including the dangling z-edges
 * below level 1 and above level L-1; logical = parity of flips on the bottom
 * dangling edges.  Flip rates p_mech[n] with n = L^3 + 2 L (L-1)^2 in the
 * order: z-edge (x, y) from level z to z+1 -> z L^2 + y L + x; x-edge
 * (x..x+1, y) at level z -> L^3 + ((z-1) L + y)(L-1) + x; y-edge (x, y..y+1)
 * at level z -> L^3 + L (L-1)^2 + ((z-1)(L-1) + y) L + x.  The network is
 * swept along z over an L x L grid.  Errors: TN3D_E_INVALID (L < 2, rate
 * outside [0, 1], null pointer). */
tn3d_status tn3d_net_surface3d_point(tn3d_ctx ctx, int32_t L, const double* p_mech, tn3d_net* out);

/* Rotated distance-d surface code, X flips decoded with Z-checks, T noisy
 * measurement rounds followed by one perfect round (phenomenological noise;
 * the 2D-code-with-noisy-syndromes problem the paper maps to 3D, Sec. 1 and
 * 5.4).  Data qubit (column i, row j) -> j d + i.  Z-checks lie in gap rows g
 * in [0, d-1) between data rows g and g+1: for even g plaquettes on columns
 * (0,1), (2,3), ... and a weight-2 check on column d-1; for odd g a weight-2
 * check on column 0 and plaquettes on (1,2), (3,4), ...; checks are numbered
 * by gap row, then left to right (nZ = (d^2-1)/2).  Detector (c, t), t in
 * [1, T+1] -> (t-1) nZ + c is the change of check c between rounds t-1 and t.
 * Mechanisms: data flip (q, t), t in [1, T] -> (t-1) d^2 + q, flipping the
 * detectors (c, t) of q's checks; measurement flip (c, t) -> T d^2 +
 * (t-1) nZ + c, flipping (c, t) and (c, t+1).  Logical = parity of flips on
 * data row 0.  p_mech has T d^2 + T nZ rates.  The network is swept across
 * data rows over a d x (T+1) grid of (check column, round).
 * Errors: TN3D_E_INVALID (even d, d < 3, T < 1, bad rates). */
tn3d_status tn3d_net_rotated_phenom(tn3d_ctx ctx, int32_t d, int32_t T, const double* p_mech,
                                    tn3d_net* out);

/* The 3D planar surface code of size L (qubit numbering and vertex checks as
 * in tn3d_net_surface3d_point) under depolarizing noise, both error types
 * decoded at once (paper Sec. 2.1-2.3 for the coset probabilities, Sec. 3.3
 * for the generator picture, Sec. 5.1 for the code).  Qubit e suffers X, Y
 * or Z with probability p_qubit[e]/3 each.  Syndrome: the L^2 (L-1) vertex
 * checks (detector ((z-1) L + y) L + x, they see the Z parts), then the
 * face checks (they see the X parts), offset by L^2 (L-1):
 *   xy-face (x..x+1, y..y+1) at level z in [1, L)  -> ((z-1)(L-1) + y)(L-1) + x
 *   xz-face (x..x+1, y, z..z+1), z in [0, L)       -> (L-1)^3 + (z L + y)(L-1) + x
 *   yz-face (x, y..y+1, z..z+1), z in [0, L)       -> (L-1)^3 + L^2 (L-1) + (z (L-1) + y) L + x
 * (faces at the rough top and bottom have three edges).  Four cosets,
 * c = a + 2 b: a is the parity of the X part on the z-edges above (0, 0),
 * b that of the Z part on the bottom dangling z-edges.  The network uses the
 * detector picture for the Z parts and the generator picture over the
 * vertex stabilizers for the X parts (physical dim 4 on every site, gates
 * of operator-Schmidt rank 3 whose terms depend on a representative of the
 * face syndrome, derived on the device per item by a fixed GF(2) map), so
 * contractions need 4 chi <= 64.  A face syndrome that violates a cube
 * relation (no X part has it) gives log p = -inf for every coset and only
 * the flag TN3D_FLAG_INCONSISTENT; the relations are checked on the device
 * per item with the same map.
 * Errors: TN3D_E_INVALID (L < 2, a rate outside [0, 3/4], null pointer),
 * TN3D_E_UNSUPPORTED (more than 4096 faces). */
tn3d_status tn3d_net_surface3d_depolarizing(tn3d_ctx ctx, int32_t L, const double* p_qubit, tn3d_net* out);

/* Loop sector of the 3D planar surface code of size L (the loop-sector
 * experiment of paper Sec. 5, generator picture of Sec. 3.2): independent
 * bit flips with rate p_mech[e] on every edge (qubit numbering of
 * tn3d_net_surface3d_point, n = L^3 + 2 L (L-1)^2 rates), detected by the
 * face checks only (face numbering of tn3d_net_surface3d_depolarizing
 * without its vertex offset: n_det = (L-1)^3 + 2 L^2 (L-1)).  Two cosets: the
 * parity of the flips on the vertical string of z-edges above (0, 0).  The
 * network sums over one generator bit per vertex (physical dim 2 on every
 * site); its gates depend on a representative of the face syndrome derived
 * on the device per item, and a face syndrome that violates a cube relation
 * gives log p = -inf for both cosets and TN3D_FLAG_INCONSISTENT.
 * Errors: TN3D_E_INVALID (L < 2, a rate outside [0, 1], null pointer),
 * TN3D_E_UNSUPPORTED (more than 4096 faces). */
tn3d_status tn3d_net_surface3d_loop(tn3d_ctx ctx, int32_t L, const double* p_mech, tn3d_net* out);

/* The Walsh-Hadamard form of the coset selection (paper Sec. 3.1) for the
 * 3D planar code: instead of one non-negative network per coset, two signed
 * networks per syndrome, Z_0 = P_0 + P_1 and Z_1 = P_0 - P_1 (the logical
 * check node becomes a sign on the legs it joins), contracted with the same
 * sweep, and log p_{m,L} = log((Z_0 + (-1)^L Z_1) / 2).  sector
 * TN3D_SECTOR_POINT: the network of tn3d_net_surface3d_point with the
 * product initial state of the signed bottom-edge weights (1 - q, (-1)^b q);
 * TN3D_SECTOR_LOOP: that of tn3d_net_surface3d_loop with the generator bit
 * below level 1 shared by all sites and signed (-1)^(a b).  Numbering,
 * rates and syndromes as for those builders; results come back per coset
 * like theirs.  The minority coset is a difference of two nearly equal
 * values here: its relative error grows as e^gap times the precision of
 * Z_b, so reduced precisions resolve it poorly.  A truncated |Z_1| above Z_0
 * gives NaN with TN3D_FLAG_NUMERIC.
 * Errors: TN3D_E_INVALID (unknown sector, and as the builders). */
#define TN3D_SECTOR_POINT 0
#define TN3D_SECTOR_LOOP 1
tn3d_status tn3d_net_surface3d_wht(tn3d_ctx ctx, int32_t L, int32_t sector, const double* p_mech, tn3d_net* out);

/* Generic front end (paper Sec. 2.4 problem statement, Sec. 3.1 and 3.4
 * detector picture): a detector error model given as the COO pattern of H
 * (nnz pairs det_idx[k], mech_idx[k]; a pair listed twice cancels), rates
 * p_mech[n_mech], one observable row obs[n_mech] (0/1) and detector
 * coordinates det_coord[n_det][3] = (x, y, t) >= 0, which define the sweep:
 * layers by t, one detector per (x, y, t) on an x-by-y grid.  Supported
 * models are graph-like on that grid: every mechanism flips one detector, or
 * two at grid-adjacent (x, y) of one layer, or two at one (x, y) in layers t
 * and t + 1; parallel mechanisms are merged exactly.  The observable must
 * consist of single-detector mechanisms of the first layer (the coset is
 * chained over their flips).  The syndrome of an item is n_det bytes in
 * detector order; two cosets.  All inputs are host pointers, copied.
 * Errors: TN3D_E_INVALID (null pointers, index or rate out of range,
 * negative coordinates, two detectors at one grid point),
 * TN3D_E_UNSUPPORTED (a model outside that class, more than one
 * observable). */
tn3d_status tn3d_net_from_dem(tn3d_ctx ctx, int32_t n_det, int32_t n_mech, int64_t nnz, const int32_t* det_idx,
                              const int32_t* mech_idx, const double* p_mech, int32_t n_obs, const uint8_t* obs,
                              const int32_t* det_coord, tn3d_net* out);

/* Generic layered network (paper Sec. 4: layers of one topology absorbed
 * into a 2D network; two-site operators split into operator-Schmidt terms by
 * a truncated SVD, the paper's general gate splitting).  An lx-by-ly grid
 * (lx, ly >= 2) of sites; per coset c < n_cosets (1..4) an initial tensor per
 * site s = y lx + x with dims init_dims[c][s][5] = (p, w, e, n, s) (physical,
 * then the bonds to the west, east, north and south neighbours; 1 on the
 * grid boundary; every coset with the same dims; bonds of equal dimension
 * at both ends, at most 64, and at most max(chi, 2) when contracted), its
 * values T[p][w][e][n][s] (row-major) at values[init_off[c][s]].  Then
 * n_layers layers of ops (ops[] in nondecreasing `layer` order; within a
 * layer the one-site ops before the gates act first, in array order, then
 * the gates in four classes, (x, y)-(x+1, y) with x even, then x odd, then
 * (x, y)-(x, y+1) with y even, then y odd (the gates of a class act on
 * disjoint bonds), then the one-site ops after the gates, in array order):
 *   TN3D_OP_PRE / TN3D_OP_POST on site (x, y): a d_out x d_in matrix
 *     (row-major [p'][p], d_in the site's current physical dim, both <= 16);
 *   TN3D_OP_GATE_H / _V on (x, y)-(x+1, y) or (x, y)-(x, y+1): a two-site
 *     operator G[a'][b'][a][b] with d_in = dim at (x, y), d_out = dim at the
 *     other site (unchanged by the gate), split into the terms of singular
 *     value above split_tol times the largest (split_tol in [0, 1)); at
 *     most one gate per bond and layer.
 * det >= 0 makes an op depend on that syndrome bit (values at off1 when it
 * is set, off0 otherwise); n_det bits per item.  Finally the vector of the
 * site's final physical dim at values[final_off[s]] closes every site, and
 * log p_{m,c} is the log of the contracted value of coset c (non-positive
 * values: NaN with NUMERIC).  All inputs are host pointers, copied; the
 * network has no rates (tn3d_grad_loglik refuses it).
 * Errors: TN3D_E_INVALID with the reason (shapes, ranges, dims that do not
 * match, non-finite values). */
typedef struct {
  int32_t layer, kind, x, y, d_in, d_out, det, reserved;
  int64_t off0, off1;
} tn3d_layer_op;
#define TN3D_OP_PRE 0
#define TN3D_OP_GATE_H 1
#define TN3D_OP_GATE_V 2
#define TN3D_OP_POST 3
tn3d_status tn3d_net_from_layers(tn3d_ctx ctx, int32_t lx, int32_t ly, int32_t n_layers, int32_t n_det,
                                 int32_t n_cosets, const int32_t* init_dims, const int64_t* init_off, int32_t n_ops,
                                 const tn3d_layer_op* ops, const int64_t* final_off, const double* values,
                                 int64_t n_values, double split_tol, tn3d_net* out);

/* Gauge rounds (paper Sec. 6: better truncation environments by repeated
 * simple updates with trivial gates, towards the Vidal gauge): a new network
 * equal to `base` (same builder, rates or layers) with `rounds` (0..16)
 * rounds of identity gates on every bond before each layer after the first.
 * A round runs the four bond classes in the layer order, each gate truncated
 * by the rank rule at the chi cap of the layer before it (no bond grows), and
 * rescales like a layer; the contracted value is unchanged where nothing is
 * truncated.  tn3d_net_shape reports the layers of the network, without the
 * rounds; chi-schedules count those layers too.  Errors: TN3D_E_INVALID,
 * TN3D_E_UNSUPPORTED (a network without a recorded builder). */
tn3d_status tn3d_net_with_gauge_rounds(tn3d_ctx ctx, tn3d_net base, int32_t rounds, tn3d_net* out);

int32_t tn3d_net_num_detectors(tn3d_net net);
int32_t tn3d_net_num_mechanisms(tn3d_net net);
int32_t tn3d_net_num_cosets(tn3d_net net);
/* Grid of the swept 2D network and number of absorbed layers. */
void tn3d_net_shape(tn3d_net net, int32_t* lx, int32_t* ly, int32_t* n_layers);
/* Frees the network (its device arrays, and the context's captured launch
 * sequences that use it); valid after its context was destroyed as well. */
void tn3d_net_destroy(tn3d_net net);

/* log p_{m,L} for a batch of syndromes (paper Sec. 2.4 definition; Sec. 4
 * method).  Item i uses nets[i] (host array of `batch` handles) and its
 * syndrome bits syndromes_dev[offsets_dev[i] .. + num_detectors) (one uint8 0/1
 * per detector, device memory; offsets_dev int64 device array).  Outputs:
 * logp_dev[batch * 4] (FP64, row i holds the cosets of item i, unused columns
 * -inf; NaN with TN3D_FLAG_NUMERIC when the approximate value is not
 * positive) and flags_dev[batch] (uint32, may be NULL).  Items sharing a
 * network are contracted together in one batched pass per layer.
 * Errors: TN3D_E_INVALID, TN3D_E_OOM (workspace cap below one item),
 * TN3D_E_DEVICE. */
tn3d_status tn3d_contract_cosets(tn3d_ctx ctx, int32_t batch, const tn3d_net* nets,
                                 const uint8_t* syndromes_dev, const int64_t* offsets_dev,
                                 const tn3d_params* params, double* logp_dev, uint32_t* flags_dev);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): tn3d_contract_cosets
 * with the same arguments, results and errors, except that its workspace is
 * a fixed device array of TN3D_NOALLOC_BYTES that the library holds on every
 * GPU it runs on until the process ends (no hipMalloc, hipFree or graph
 * instantiation: the launches are issued eagerly).  Items are processed in
 * chunks that fit the array; an item that alone needs more returns
 * TN3D_E_OOM with the sizes in tn3d_last_error.  Every call on a GPU shares
 * that GPU's array and leaves its contents behind (the kernels initialise
 * what they read): calls that overlap in time on one GPU, from any context or
 * thread, race and must be serialised by the caller. */
#define TN3D_NOALLOC_BYTES (256ull << 20)
tn3d_status tn3d_contract_cosets_noalloc(tn3d_ctx ctx, int32_t batch, const tn3d_net* nets,
                                         const uint8_t* syndromes_dev, const int64_t* offsets_dev,
                                         const tn3d_params* params, double* logp_dev, uint32_t* flags_dev);

/* Decode (paper Sec. 2.3, eq. optimal_decoder): as tn3d_contract_cosets, then
 * per item coset_dev[i] = argmax_L log p_{m,L} (lowest index on exact ties;
 * a NaN value ranks below every number, and an item with every value NaN
 * decodes to 0 with a NaN log-ratio),
 * logratio_dev[i] = log p of the chosen coset minus the largest other one
 * (>= 0; +inf when every other value is NaN or -inf), TN3D_FLAG_NEAR_TIE
 * when logratio < params->near_tie.  With a reduced precision
 * (TN3D_PREC_FP32, TN3D_PREC_BF16) and near_tie > 0, every item whose log-ratio is
 * below near_tie (or not a number) is contracted again in FP64 at the same chi,
 * chi_mps and rank rule, through the Gram route (TN3D_OPT_GRAM_FACTOR; the
 * decision needs far less than that route's accuracy); its logp row, flags
 * (those of the FP64 pass plus TN3D_FLAG_RESWEPT)
 * and decision are replaced.  This synchronises the context stream once.
 * logp_dev and flags_dev may be NULL. */
tn3d_status tn3d_decode(tn3d_ctx ctx, int32_t batch, const tn3d_net* nets,
                        const uint8_t* syndromes_dev, const int64_t* offsets_dev,
                        const tn3d_params* params, int32_t* coset_dev, double* logratio_dev,
                        double* logp_dev, uint32_t* flags_dev);

/* Gradient of the syndrome log-likelihood with respect to the rates (the
 * Sec. 2.4 definition of p_{m,L}; used to fit a noise model to syndrome
 * data).  P(m) = sum_L p_{m,L} is affine in each mechanism's rate p_i (every
 * term of the sum holds p_i or 1 - p_i once), so for any c != p_i,
 * d log P(m) / d p_i = (P_c(m) / P(m) - 1) / (c - p_i) with P_c(m) the value
 * at p_i = c.  The library takes c_i a quarter of the rate range [0, r_max]
 * away from p_i, towards its middle (r_max = 1, or 3/4 for the depolarizing
 * family), where no term of the network vanishes, and contracts `net` at its
 * rates and, per mechanism i, at p_i = c_i, every contraction at params' chi,
 * chi_mps, precision and rank rule (no near-tie re-sweep): batch *
 * (n_mech + 1) contractions, those of networks with the original's structure
 * (the usual case) in one batched pass.  Each P is the fixed-chi
 * approximation, so the result is the exact gradient where chi truncates
 * nothing and otherwise carries the truncation error of the contractions
 * (it is not the derivative of the truncated contraction itself).
 * Rates: the builder's rate array (p_mech, or p_qubit of the depolarizing
 * family); rate_of_mech (host int32[n_mech], nullable) maps each to one of
 * n_rates parameters, and grad_dev[k] (FP64, device, n_rates entries) is the
 * sum over items s and the mechanisms of parameter k of d log P(m_s) / d p_i
 * (chain rule through p_i = r_k); without a map n_rates = n_mech.
 * Syndromes as in tn3d_contract_cosets (batch items, device offsets).
 * Optional outputs (device, nullable): loglik_sum_dev[1] = sum_s log P(m_s),
 * loglik_dev[batch] = log P(m_s), grad_items_dev[batch][n_mech] the
 * per-item derivatives d log P(m_s) / d p_i, flags_dev[batch] the OR of the
 * flags of an item's contractions.  A coset that a contraction finds
 * non-positive (NaN, NUMERIC in the item's flags) counts as zero (its value
 * is below the contraction's error); an item whose cosets at the given rates
 * are all NaN, or whose syndrome is impossible (log P = -inf), makes the
 * gradient NaN.  The changed networks are built on the first call and kept with `net`
 * (released by tn3d_net_destroy); the pass allocates workspace like
 * tn3d_contract_cosets over batch * (n_mech + 1) items and launches eagerly.
 * Synchronises the context stream.
 * Errors: TN3D_E_INVALID (bad handles, params, map entries out of range),
 * TN3D_E_UNSUPPORTED (as tn3d_contract_cosets), TN3D_E_OOM, TN3D_E_DEVICE. */
tn3d_status tn3d_grad_loglik(tn3d_ctx ctx, tn3d_net net, int32_t batch, const uint8_t* syndromes_dev,
                             const int64_t* offsets_dev, const tn3d_params* params, int32_t n_rates,
                             const int32_t* rate_of_mech, double* grad_dev, double* loglik_sum_dev,
                             double* loglik_dev, double* grad_items_dev, uint32_t* flags_dev);

/* Autotuner (batching): searches the launch shapes of the layer absorption
 * (the size-class split points of the truncation kernels: teams of eight
 * lanes for orders <= 8 on or off, one-wavefront truncations up to order 8
 * or 16; a separate reabsorption class for rows of at most 16 entries on or
 * off) by contracting the given batch under each candidate (twice: capture,
 * then a timed replay), and caches the fastest for each network of the batch
 * under params' precision, chi and chi_mps in the context; later contractions
 * with those parameters use it.  A candidate whose decoded-coset log p leaves
 * the default shape's by more than 1e-9 (FP64) or 1e-4 (reduced precisions),
 * or that changes a decision, is not chosen.  out (nullable, n_out <= 6):
 * chosen candidate index, team, mid, narrow, its time and the default
 * shape's time (ms, one contraction of the batch).  The batch arguments are
 * those of tn3d_contract_cosets; the call synchronises the context stream
 * and allocates two result buffers.  Errors: as tn3d_contract_cosets. */
tn3d_status tn3d_autotune(tn3d_ctx ctx, int32_t batch, const tn3d_net* nets, const uint8_t* syndromes_dev,
                          const int64_t* offsets_dev, const tn3d_params* params, double* out, int32_t n_out);

/* Timing of the contractions on this context: enable = 0 off, 1 kernel times,
 * 2 kernel times and bond statistics (tn3d_last_stats; this level copies the
 * bond dimensions and lambdas of every sweep to the host after each call).
 * Every call of tn3d_ctx_set_timing restarts the sums; tn3d_last_timing and
 * tn3d_last_stats report the sums over the contractions since then.  Level 1
 * keeps its sums on the device (no host synchronisation per contraction);
 * tn3d_last_timing waits for the context stream.
 * Times come from the device wall clock: the phase times from one-thread
 * kernels enqueued at the phase boundaries, the kernel times from execution
 * windows the kernels record themselves (earliest workgroup start to latest
 * workgroup end of the launch), so they hold inside captured graphs as well
 * and add no launches around the kernels.  tn3d_last_timing: out[0] = layer
 * absorption (one-site ops, Grams, truncations, reabsorption, rescaling),
 * out[1] = final boundary MPS, out[2] = Gram + reabsorption kernels only,
 * out[3] = number of Gram + reabsorption launches, out[4] = algorithmic bytes
 * those launches moved (each site tensor read by the Gram, read and written
 * by the reabsorption), out[5] = time of the boundary-MPS eigen-decomposition
 * launches (when the rank rule allows that path), out[6] = their number,
 * out[7] = their algorithmic flops (per problem of order n keeping D vectors:
 * 4n^3/3 + 2Dn^2 + 7Dn + 12D^2n for the one-wavefront solver; per iteration
 * 2n^2 b + 14 n b^2 with b = 64 for the subspace iteration of larger families),
 * out[8] = time of the boundary-MPS contraction launches (the two
 * contractions forming Theta and, on the Gram route, its Gram), out[9] = their
 * algorithmic flops, out[10] = their number, out[11] = time of the
 * subspace-iteration launches (boundary-MPS families above 64 vectors on the
 * Gram route; out[5] then covers only the one-wavefront solver), out[12] =
 * their algorithmic flops, out[13] = their number, out[14] = the sweeps they
 * covered (summed over the launches).  Milliseconds for times; n <= 15
 * values are written.
 * Returns TN3D_E_INVALID if timing is not enabled. */
tn3d_status tn3d_ctx_set_timing(tn3d_ctx ctx, int32_t enable);
tn3d_status tn3d_last_timing(tn3d_ctx ctx, double* out, int32_t n);

/* Launch-sequence replay (on by default).  The first contraction of a chunk
 * shape for a network, parameter set and timing level captures its whole
 * kernel sequence into a HIP graph that reads and writes only the context
 * workspace; later calls of the same shape copy the syndromes in, replay the
 * graph and copy the results out, instead of issuing each launch.  Capture
 * runs on a stream the context owns, so any caller stream (the legacy default
 * one included) can replay.  Graphs are dropped when the workspace is
 * reallocated, the network destroyed or replay switched off; if capture fails
 * the context launches eagerly from then on.  Results are identical either
 * way.  Errors: TN3D_E_INVALID (null ctx). */
tn3d_status tn3d_ctx_set_graphs(tn3d_ctx ctx, int32_t enable);
/* Number of captured launch sequences the context holds (0 when replay is
 * off or capture was refused; setting TN3D_VERBOSE in the environment prints
 * the reason of a refusal to stderr). */
int32_t tn3d_ctx_graphs_cached(tn3d_ctx ctx);

/* Bond statistics of the last contraction with timing level 2, over all its
 * sweeps, taken after the last layer: out[0] = mean bond dimension of the
 * swept 2D network, out[1] = largest, out[2] = number of sweeps, out[3] = mean
 * over sweeps of the smallest kept lambda (relative to its bond's largest),
 * out[4] = most Jacobi sweeps any truncation needed, out[5] = same for the
 * boundary MPS, out[6] = items the last tn3d_decode re-swept in FP64 (n <= 7
 * values are written).
 * Returns TN3D_E_INVALID if the timing level is below 2. */
tn3d_status tn3d_last_stats(tn3d_ctx ctx, double* out, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* TN3D_H */
