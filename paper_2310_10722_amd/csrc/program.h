// Layered op program of a 3D network and the flat structs the kernels read.
//
// A network is a stack of layers over an Lx x Ly grid (paper Sec. 4: layers of
// identical topology, connections between layers only between equal sites).
// The swept 2D network holds one tensor per site with a physical leg and four
// virtual legs (w, e, n, s); a layer is absorbed as
//   pre-ops (one-site linear maps on the physical leg),
//   two-site gates in four classes of disjoint bonds
//     (x,y)-(x+1,y) with x even, x odd, (x,y)-(x,y+1) with y even, y odd,
//   post-ops, then a per-site rescale.
// A one-site op may depend on one syndrome bit (it is then M1 when the bit is
// set, else M0).  A gate is given by its operator-Schmidt terms
// sum_k OA_k (x) OB_k, and may also depend on one per-item bit (a second set
// of terms of the same count).  Per-item bits are the syndrome followed by
// bits derived from it by a fixed GF(2) map (ext_rows).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace tn3d {

enum Leg : int32_t { LEG_W = 0, LEG_E = 1, LEG_N = 2, LEG_S = 3 };

struct DevOneSite {
  int32_t site, din, dout, det;  // det < 0: op independent of the syndrome
  int32_t m0, m1;                // pool offsets of dout x din matrices, row-major [p'][p]
  int32_t src;                   // buffer parity read (the other one is written)
  int32_t pad;
};

struct DevGate {
  int32_t sa, sb;      // sites; sb is east (H) or south (V) of sa
  int32_t la, lb;      // leg of sa / sb carrying the bond
  int32_t dA, dB;      // physical dims during the gate
  int32_t K;           // number of operator-Schmidt terms
  int32_t bond;        // bond id
  int32_t oA, oB;      // pool: K matrices [k][p'][p] of dA x dA / dB x dB
  int32_t pA, pB;      // pool: K*K matrices OA_k^T OA_k' ([k][k'][p][q]) / same for B
  int32_t srcA, srcB;  // buffer parities read
  int32_t det;         // >= 0: the terms depend on this per-item bit (set: oA1 .. pB1)
  int32_t oA1, oB1, pA1, pB1;
  int32_t pad[3];
};

struct LayerRange {
  int32_t pre0, pre1;      // [pre0, pre1) in the one-site op array
  int32_t gate0[4], gate1[4];
  int32_t post0, post1;
  int32_t gauge;           // 1: a gauge round (identity gates on every bond), not a layer of the network
};

struct Program {
  int32_t Lx = 0, Ly = 0;
  int32_t n_det = 0, n_mech = 0, n_cosets = 2;
  std::string name;
  // static geometry
  std::vector<int32_t> leg_bond;  // [site][4] bond id or -1
  int32_t n_bonds_h = 0, n_bonds = 0;
  std::vector<int32_t> dmax;      // per site, max physical dim over the sweep
  // initial state per coset: per site dims (d, Dw, De, Dn, Ds) and values
  std::vector<int32_t> init_dims;  // [coset][site][5]
  std::vector<int32_t> init_off;   // [coset][site] pool offset
  std::vector<int32_t> bond_dim0;  // [bond] initial bond dim (same for all cosets)
  // ops
  std::vector<DevOneSite> ones;
  std::vector<DevGate> gates;
  std::vector<LayerRange> layers;
  std::vector<int32_t> d_after;    // [layer][site] physical dim after the layer
  std::vector<int32_t> par_after;  // [layer][site] buffer parity after the layer
  std::vector<int32_t> d_final;    // per site
  std::vector<int32_t> f_off;      // per site pool offset of the final vector
  std::vector<double> pool;
  int32_t max_K = 0, max_dgate = 0;
  // Derived per-item bits: bit n_det + e of an item is the parity of
  // ext_rows[e] (ext_words 64-bit words) with syndrome bits
  // [ext_src0, ext_src0 + 64 ext_words), for e in [0, n_ext).
  int32_t n_ext = 0, ext_src0 = 0, ext_src_n = 0, ext_words = 0;
  std::vector<uint64_t> ext_rows;
  // Consistency: per-item bits [inc0, inc0 + n_inc) (among the derived bits)
  // are parities that vanish for every syndrome the code can produce; an item
  // with one of them set is inconsistent (log p = -inf for every coset).
  int32_t inc0 = 0, n_inc = 0;
  // Walsh-Hadamard form: the two "cosets" are the signed networks Z_0, Z_1
  // (their values may be negative) and log p_{m,L} = log((Z_0 + (-1)^L Z_1)/2).
  int32_t wht = 0;
  // every rate of the builder lies in [0, rate_max] (3/4 for depolarizing noise)
  double rate_max = 1.0;
};

// Gauge rounds: while a GaugeRounds object lives on this thread, the builders
// put `rounds` rounds of identity gates on every bond before each layer after
// the first (simple update with trivial gates, which moves the bond
// environments towards the Vidal gauge before the layer's truncations).
struct GaugeRounds {
  explicit GaugeRounds(int rounds);
  ~GaugeRounds();
  int saved;
};

// Builders; return an empty string on success, else an error message.
std::string build_surface3d_point(int32_t L, const double* p_mech, Program& out, bool wht = false);
std::string build_rotated_phenom(int32_t d, int32_t T, const double* p_mech, Program& out);
std::string build_surface3d_depol(int32_t L, const double* p_qubit, Program& out);
std::string build_surface3d_loop(int32_t L, const double* p_mech, Program& out, bool wht = false);
std::string build_from_dem(int32_t n_det, int32_t n_mech, int64_t nnz, const int32_t* det_idx,
                           const int32_t* mech_idx, const double* p_mech, int32_t n_obs, const uint8_t* obs,
                           const int32_t* det_coord, Program& out);

// A generic layered network (the flat description of tn3d_net_from_layers).
struct LayerOp {
  int32_t layer, kind, x, y, d_in, d_out, det, pad;
  int64_t off0, off1;
};
enum : int32_t { OP_PRE = 0, OP_GATE_H = 1, OP_GATE_V = 2, OP_POST = 3 };
std::string build_from_layers(int32_t lx, int32_t ly, int32_t n_layers, int32_t n_det, int32_t n_cosets,
                              const int32_t* init_dims, const int64_t* init_off, int32_t n_ops, const LayerOp* ops,
                              const int64_t* final_off, const double* values, int64_t n_values, double split_tol,
                              Program& out);

}  // namespace tn3d
