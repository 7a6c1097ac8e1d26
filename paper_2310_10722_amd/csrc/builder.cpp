// Layered op programs for the detector-picture networks of the paper
// (Sec. 3.1, 3.3, 3.4, 5.1) arranged for a boundary sweep (Sec. 4).
//
// Every physical leg carries flip parities, so a flip mechanism shared by two
// sites is the gate (1-p) I (x) I + p X (x) X (operator-Schmidt rank 2), a
// mechanism inside one site is the one-site op (1-p) I + p X.., and a detector
// outcome is imposed by a one-site op that depends on one syndrome bit.  The
// logical check node is replaced by a parity chain over the first layer's
// legs (one positive network per coset).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "program.h"

namespace tn3d {

static thread_local int g_gauge_rounds = 0;
GaugeRounds::GaugeRounds(int rounds) : saved(g_gauge_rounds) { g_gauge_rounds = rounds; }
GaugeRounds::~GaugeRounds() { g_gauge_rounds = saved; }

namespace {

using Mat = std::vector<double>;  // row-major dout x din

Mat eye(int d) {
  Mat m(size_t(d) * d, 0.0);
  for (int i = 0; i < d; ++i) m[size_t(i) * d + i] = 1.0;
  return m;
}

// X on the bits of `mask` of a physical index of dim d (a permutation).
Mat xmask(int d, int mask) {
  Mat m(size_t(d) * d, 0.0);
  for (int a = 0; a < d; ++a) m[size_t(a ^ mask) * d + a] = 1.0;
  return m;
}

Mat scaled(Mat m, double s) {
  for (auto& v : m) v *= s;
  return m;
}

Mat matmul(const Mat& A, int ar, int ac, const Mat& B, int bc) {
  Mat C(size_t(ar) * bc, 0.0);
  for (int i = 0; i < ar; ++i)
    for (int k = 0; k < ac; ++k) {
      double a = A[size_t(i) * ac + k];
      if (a == 0.0) continue;
      for (int j = 0; j < bc; ++j) C[size_t(i) * bc + j] += a * B[size_t(k) * bc + j];
    }
  return C;
}

struct Term {
  Mat A, B;
};

// (1-p) I (x) I + p XmA (x) XmB as operator-Schmidt terms with sqrt weights on
// both sides (terms with zero weight are dropped).
std::vector<Term> flip_gate(double p, int dA, int maskA, int dB, int maskB) {
  std::vector<Term> t;
  if (1.0 - p > 0.0) t.push_back({scaled(eye(dA), std::sqrt(1.0 - p)), scaled(eye(dB), std::sqrt(1.0 - p))});
  if (p > 0.0) t.push_back({scaled(xmask(dA, maskA), std::sqrt(p)), scaled(xmask(dB, maskB), std::sqrt(p))});
  return t;
}

// (1-p) I + p X_mask
Mat flip_op(double p, int d, int mask) {
  Mat m = scaled(eye(d), 1.0 - p);
  Mat x = xmask(d, mask);
  for (size_t i = 0; i < m.size(); ++i) m[i] += p * x[i];
  return m;
}

class Assembler {
 public:
  Assembler(Program& P, int Lx, int Ly) : P(P), Lx(Lx), Ly(Ly) {
    P.Lx = Lx;
    P.Ly = Ly;
    int ns = Lx * Ly;
    P.n_bonds_h = (Lx - 1) * Ly;
    P.n_bonds = P.n_bonds_h + Lx * (Ly - 1);
    P.leg_bond.assign(size_t(ns) * 4, -1);
    for (int y = 0; y < Ly; ++y)
      for (int x = 0; x < Lx; ++x) {
        int s = y * Lx + x;
        if (x > 0) P.leg_bond[s * 4 + LEG_W] = hbond(x - 1, y);
        if (x + 1 < Lx) P.leg_bond[s * 4 + LEG_E] = hbond(x, y);
        if (y > 0) P.leg_bond[s * 4 + LEG_N] = vbond(x, y - 1);
        if (y + 1 < Ly) P.leg_bond[s * 4 + LEG_S] = vbond(x, y);
      }
    d.assign(ns, 1);
    par.assign(ns, 0);
    P.dmax.assign(ns, 1);
    pre.assign(ns, {});
    post.assign(ns, {});
  }
  int hbond(int x, int y) const { return y * (Lx - 1) + x; }
  int vbond(int x, int y) const { return P.n_bonds_h + y * Lx + x; }

  int put(const Mat& m) {
    int off = int(P.pool.size());
    P.pool.insert(P.pool.end(), m.begin(), m.end());
    return off;
  }

  // Parity chain over the sites in boustrophedon order: value
  // prod_s w_s(b_s) if the parity of all bits is `coset`; w[s] empty for a
  // site without a bit (physical dim 1).
  // With dfull > 0 every site has physical dim dfull and its bit sits at
  // index base + bit.  The state is stored as coset `slot` (default: coset).
  void snake_init(const std::vector<std::vector<double>>& w, int coset, int dfull = 0, int base = 0, int slot = -1) {
    const int sl = slot >= 0 ? slot : coset;
    int ns = Lx * Ly;
    std::vector<std::pair<int, int>> order;
    for (int y = 0; y < Ly; ++y)
      for (int i = 0; i < Lx; ++i) order.push_back({y % 2 == 0 ? i : Lx - 1 - i, y});
    auto leg_to = [](std::pair<int, int> a, std::pair<int, int> b) {
      if (b.first == a.first + 1) return int(LEG_E);
      if (b.first == a.first - 1) return int(LEG_W);
      if (b.second == a.second + 1) return int(LEG_S);
      return int(LEG_N);
    };
    if (int(P.init_dims.size()) < (sl + 1) * ns * 5) {
      P.init_dims.resize(size_t(sl + 1) * ns * 5, 1);
      P.init_off.resize(size_t(sl + 1) * ns, 0);
    }
    P.bond_dim0.assign(P.n_bonds, 1);
    for (int k = 0; k < ns; ++k) {
      auto [x, y] = order[k];
      int s = y * Lx + x;
      int dp = w[s].empty() ? 1 : 2;
      int dphys = dfull > 0 ? dfull : dp;
      int lin = k > 0 ? leg_to(order[k], order[k - 1]) : -1;
      int lout = k + 1 < ns ? leg_to(order[k], order[k + 1]) : -1;
      int dims[5] = {dphys, 1, 1, 1, 1};
      if (lin >= 0) dims[1 + lin] = 2;
      if (lout >= 0) dims[1 + lout] = 2;
      if (lout >= 0) P.bond_dim0[P.leg_bond[s * 4 + lout]] = 2;
      size_t n = size_t(dims[0]) * dims[1] * dims[2] * dims[3] * dims[4];
      Mat t(n, 0.0);
      // storage order [w][e][n][s][p], p fastest
      for (int cin = 0; cin < (lin >= 0 ? 2 : 1); ++cin)
        for (int b = 0; b < dp; ++b) {
          int cout = cin ^ b;
          if (lout < 0 && cout != coset) continue;
          int idx[4] = {0, 0, 0, 0};
          if (lin >= 0) idx[lin] = cin;
          if (lout >= 0) idx[lout] = cout;
          size_t off = ((((size_t(idx[0]) * dims[2] + idx[1]) * dims[3] + idx[2]) * dims[4] + idx[3]) * dphys) +
                       (dfull > 0 ? base : 0) + b;
          t[off] = w[s].empty() ? 1.0 : w[s][b];
        }
      for (int i = 0; i < 5; ++i) P.init_dims[(size_t(sl) * ns + s) * 5 + i] = dims[i];
      P.init_off[size_t(sl) * ns + s] = put(t);
      d[s] = dphys;
      P.dmax[s] = std::max(P.dmax[s], dphys);
    }
  }

  // Product state: site s holds the vector v[s] on its physical leg (dim
  // v[s].size()), every bond of dimension 1; stored as coset `slot`.
  void product_init(const std::vector<std::vector<double>>& v, int slot) {
    int ns = Lx * Ly;
    if (int(P.init_dims.size()) < (slot + 1) * ns * 5) {
      P.init_dims.resize(size_t(slot + 1) * ns * 5, 1);
      P.init_off.resize(size_t(slot + 1) * ns, 0);
    }
    P.bond_dim0.assign(P.n_bonds, 1);
    for (int s = 0; s < ns; ++s) {
      int dp = int(v[s].size());
      for (int i = 0; i < 5; ++i) P.init_dims[(size_t(slot) * ns + s) * 5 + i] = i == 0 ? dp : 1;
      P.init_off[size_t(slot) * ns + s] = put(v[s]);
      d[s] = dp;
      P.dmax[s] = std::max(P.dmax[s], dp);
    }
  }

  // Chain of equal bits in boustrophedon order (bond 2 along the chain,
  // physical dim 2): value (-1)^(a sgn) when every site holds the same bit
  // a, else 0; stored as coset `sgn`.
  void copy_chain_init(int sgn) {
    const int ns = Lx * Ly, slot = sgn;
    std::vector<std::pair<int, int>> order;
    for (int y = 0; y < Ly; ++y)
      for (int i = 0; i < Lx; ++i) order.push_back({y % 2 == 0 ? i : Lx - 1 - i, y});
    auto leg_to = [](std::pair<int, int> a, std::pair<int, int> b) {
      if (b.first == a.first + 1) return int(LEG_E);
      if (b.first == a.first - 1) return int(LEG_W);
      if (b.second == a.second + 1) return int(LEG_S);
      return int(LEG_N);
    };
    if (int(P.init_dims.size()) < (slot + 1) * ns * 5) {
      P.init_dims.resize(size_t(slot + 1) * ns * 5, 1);
      P.init_off.resize(size_t(slot + 1) * ns, 0);
    }
    P.bond_dim0.assign(P.n_bonds, 1);
    for (int k = 0; k < ns; ++k) {
      auto [x, y] = order[k];
      const int s = y * Lx + x;
      const int lin = k > 0 ? leg_to(order[k], order[k - 1]) : -1;
      const int lout = k + 1 < ns ? leg_to(order[k], order[k + 1]) : -1;
      int dims[5] = {2, 1, 1, 1, 1};
      if (lin >= 0) dims[1 + lin] = 2;
      if (lout >= 0) dims[1 + lout] = 2;
      if (lout >= 0) P.bond_dim0[P.leg_bond[s * 4 + lout]] = 2;
      Mat t(size_t(dims[0]) * dims[1] * dims[2] * dims[3] * dims[4], 0.0);
      for (int a = 0; a < 2; ++a) {
        int idx[4] = {0, 0, 0, 0};
        if (lin >= 0) idx[lin] = a;
        if (lout >= 0) idx[lout] = a;
        // storage order [w][e][n][s][p], p fastest
        size_t off = ((((size_t(idx[0]) * dims[2] + idx[1]) * dims[3] + idx[2]) * dims[4] + idx[3]) * 2) + a;
        t[off] = (k == 0 && (a & sgn)) ? -1.0 : 1.0;
      }
      for (int i = 0; i < 5; ++i) P.init_dims[(size_t(slot) * ns + s) * 5 + i] = dims[i];
      P.init_off[size_t(slot) * ns + s] = put(t);
      d[s] = 2;
      P.dmax[s] = std::max(P.dmax[s], 2);
    }
  }

  // ---- layer assembly -------------------------------------------------
  struct Pending {
    bool has = false;
    int din = 0, dout = 0, det = -1;
    Mat M0, M1;
  };
  struct PGate {
    int kind, x, y, dA, dB;
    std::vector<Term> terms;
    int det;
    std::vector<Term> terms1;  // when the per-item bit det is set
  };

  void begin_layer() {
    // gauge rounds before every layer but the first: identity gates on all
    // bonds at the current physical dims (their own layers, marked gauge)
    if (!P.layers.empty())
      for (int r = 0; r < g_gauge_rounds; ++r) {
        reset_layer();
        for (int y = 0; y < Ly; ++y)
          for (int x = 0; x < Lx; ++x) {
            const int s = y * Lx + x;
            if (x + 1 < Lx) add_gate(0, x, y, {Term{eye(d[s]), eye(d[s + 1])}});
            if (y + 1 < Ly) add_gate(1, x, y, {Term{eye(d[s]), eye(d[s + Lx])}});
          }
        end_layer();
        P.layers.back().gauge = 1;
      }
    reset_layer();
  }
  void reset_layer() {
    for (auto& p : pre) p = Pending{};
    for (auto& p : post) p = Pending{};
    gates.clear();
    staged = d;
  }
  int staged_dim(int s) const { return staged[s]; }

  // Compose M (dout x din) after whatever is pending on site s.
  std::string add_pre(int s, const Mat& M0, int dout, int det = -1, const Mat& M1 = {}) {
    return compose(pre[s], s, M0, M1, dout, det, true);
  }
  std::string add_post(int s, const Mat& M0, int dout, int det = -1, const Mat& M1 = {}) {
    return compose(post[s], s, M0, M1, dout, det, false);
  }
  void add_gate(int kind, int x, int y, std::vector<Term> terms, int det = -1, std::vector<Term> terms1 = {}) {
    int sa = y * Lx + x, sb = kind == 0 ? sa + 1 : sa + Lx;
    gates.push_back({kind, x, y, staged_pre(sa), staged_pre(sb), std::move(terms), det, std::move(terms1)});
  }

  std::string end_layer() {
    LayerRange R{};
    int ns = Lx * Ly;
    R.pre0 = int(P.ones.size());
    emit_ones(pre);
    R.pre1 = int(P.ones.size());
    for (int c = 0; c < 4; ++c) {
      R.gate0[c] = int(P.gates.size());
      // the bonds of a class are disjoint, so their order is free: gates with
      // the larger physical dims first, so that the launches for wide Grams
      // and reabsorptions cover a prefix of the class only
      std::vector<const PGate*> cg;
      for (auto& g : gates)
        if ((g.kind == 0 ? (g.x % 2) : 2 + (g.y % 2)) == c) cg.push_back(&g);
      std::stable_sort(cg.begin(), cg.end(), [](const PGate* a, const PGate* b) {
        return std::max(a->dA, a->dB) > std::max(b->dA, b->dB);
      });
      for (const PGate* gpt : cg) {
        const PGate& g = *gpt;
        int sa = g.y * Lx + g.x, sb = g.kind == 0 ? sa + 1 : sa + Lx;
        if (g.dA != d[sa] || g.dB != d[sb]) return "gate dims do not match site dims";
        DevGate G{};
        G.sa = sa;
        G.sb = sb;
        G.la = g.kind == 0 ? LEG_E : LEG_S;
        G.lb = g.kind == 0 ? LEG_W : LEG_N;
        G.dA = g.dA;
        G.dB = g.dB;
        G.K = int(g.terms.size());
        G.bond = g.kind == 0 ? hbond(g.x, g.y) : vbond(g.x, g.y);
        if (g.det >= 0 && g.terms1.size() != g.terms.size()) return "the two term sets of a gate differ in count";
        // P_kk'[p][q] = sum_p' O_k[p'][p] O_k'[p'][q]
        auto gram = [](const std::vector<Term>& ts, bool sideA, int dd) {
          Mat out;
          for (auto& t1 : ts)
            for (auto& t2 : ts) {
              const Mat& a = sideA ? t1.A : t1.B;
              const Mat& b = sideA ? t2.A : t2.B;
              for (int p = 0; p < dd; ++p)
                for (int q = 0; q < dd; ++q) {
                  double s = 0;
                  for (int r = 0; r < dd; ++r) s += a[size_t(r) * dd + p] * b[size_t(r) * dd + q];
                  out.push_back(s);
                }
            }
          return out;
        };
        auto put_terms = [&](const std::vector<Term>& ts, int32_t& oA, int32_t& oB, int32_t& pA, int32_t& pB) {
          Mat oa, ob;
          for (auto& t : ts) {
            oa.insert(oa.end(), t.A.begin(), t.A.end());
            ob.insert(ob.end(), t.B.begin(), t.B.end());
          }
          oA = put(oa);
          oB = put(ob);
          pA = put(gram(ts, true, g.dA));
          pB = put(gram(ts, false, g.dB));
        };
        put_terms(g.terms, G.oA, G.oB, G.pA, G.pB);
        G.det = g.det;
        if (g.det >= 0)
          put_terms(g.terms1, G.oA1, G.oB1, G.pA1, G.pB1);
        else {
          G.oA1 = G.oA;
          G.oB1 = G.oB;
          G.pA1 = G.pA;
          G.pB1 = G.pB;
        }
        G.srcA = par[sa];
        G.srcB = par[sb];
        par[sa] ^= 1;
        par[sb] ^= 1;
        P.max_K = std::max(P.max_K, G.K);
        P.max_dgate = std::max({P.max_dgate, G.dA, G.dB});
        P.gates.push_back(G);
      }
      R.gate1[c] = int(P.gates.size());
    }
    R.post0 = int(P.ones.size());
    emit_ones(post);
    R.post1 = int(P.ones.size());
    P.layers.push_back(R);
    for (int s = 0; s < ns; ++s) {
      P.d_after.push_back(d[s]);
      P.par_after.push_back(par[s]);
    }
    return "";
  }

  void finish(const std::vector<Mat>& f) {
    int ns = Lx * Ly;
    P.d_final.assign(ns, 1);
    P.f_off.assign(ns, 0);
    for (int s = 0; s < ns; ++s) {
      P.d_final[s] = d[s];
      P.f_off[s] = put(f[s]);
    }
  }

  Program& P;
  int Lx, Ly;
  std::vector<int> d, par, staged;

 private:
  int staged_pre(int s) const { return pre[s].has ? pre[s].dout : d[s]; }

  std::string compose(Pending& pd, int s, const Mat& M0, const Mat& M1in, int dout, int det, bool is_pre) {
    int din = pd.has ? pd.dout : (is_pre ? d[s] : staged_pre(s));
    if (int(M0.size()) != dout * din) return "one-site op has the wrong shape";
    Mat M1 = det >= 0 ? M1in : M0;
    if (int(M1.size()) != dout * din) return "one-site op has the wrong shape";
    if (!pd.has) {
      pd.has = true;
      pd.din = din;
      pd.dout = dout;
      pd.det = det;
      pd.M0 = M0;
      pd.M1 = M1;
    } else {
      if (det >= 0 && pd.det >= 0) return "two syndrome-dependent ops on one site";
      pd.M0 = matmul(M0, dout, din, pd.M0, pd.din);
      pd.M1 = matmul(M1, dout, din, pd.M1, pd.din);
      pd.dout = dout;
      if (det >= 0) pd.det = det;
    }
    // the one-site kernel holds the matrix in 256 doubles and a row of the
    // input in 16 registers
    if (pd.din > 16 || pd.dout > 16 || pd.din * pd.dout > 256) return "one-site op larger than 16 x 16";
    if (is_pre) staged[s] = dout;
    return "";
  }

  void emit_ones(std::vector<Pending>& v) {
    for (int s = 0; s < int(v.size()); ++s) {
      auto& pd = v[s];
      if (!pd.has) continue;
      DevOneSite o{};
      o.site = s;
      o.din = pd.din;
      o.dout = pd.dout;
      o.det = pd.det;
      o.m0 = put(pd.M0);
      o.m1 = pd.det >= 0 ? put(pd.M1) : o.m0;
      o.src = par[s];
      par[s] ^= 1;
      d[s] = pd.dout;
      P.dmax[s] = std::max(P.dmax[s], pd.dout);
      P.ones.push_back(o);
    }
  }

  std::vector<Pending> pre, post;
  std::vector<PGate> gates;
};

bool bad_rate(double p) { return !(p >= 0.0 && p <= 1.0); }

}  // namespace

// ---------------------------------------------------------------------------
// 3D planar code, point sector: sweep along z over the L x L vertex grid.
// Physical leg of site (x, y) before layer z = flip of the z-edge entering
// vertex (x, y, z) from below.  Initial state: the L^2 bottom dangling edges
// with their weights, chained to parity = coset (the logical membrane).  Layer
// z: gate (1-p) II + p XX per in-plane edge of level z; post-op at every vertex
// diag(1-q, q) X^{m} with q the rate of the edge leaving it upwards.  After
// the last level the top dangling edges are summed: f = (1, 1).
// ---------------------------------------------------------------------------
std::string build_surface3d_point(int32_t L, const double* p, Program& P, bool wht) {
  if (L < 2) return "L must be >= 2";
  if (!p) return "null rates";
  const int nz = L * L * L, nx = L * (L - 1) * (L - 1);
  const int n = nz + 2 * nx;
  for (int i = 0; i < n; ++i)
    if (bad_rate(p[i])) return "rate outside [0, 1]";
  P = Program{};
  P.name = "surface3d_point_L" + std::to_string(L);
  P.n_det = L * L * (L - 1);
  P.n_mech = n;
  P.n_cosets = 2;
  P.wht = wht ? 1 : 0;
  Assembler A(P, L, L);
  for (int c = 0; c < 2; ++c) {
    std::vector<std::vector<double>> w(L * L);
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        double q = p[y * L + x];
        // Walsh-Hadamard form: the logical check becomes the sign (-1)^(c x_e)
        // on each bottom dangling edge, a product state
        w[y * L + x] = {1.0 - q, (wht && c == 1) ? -q : q};
      }
    A.d.assign(L * L, 1);
    if (wht)
      A.product_init(w, c);
    else
      A.snake_init(w, c);
  }
  for (int z = 1; z < L; ++z) {
    A.begin_layer();
    for (int y = 0; y < L; ++y)
      for (int x = 0; x + 1 < L; ++x)
        A.add_gate(0, x, y, flip_gate(p[nz + ((z - 1) * L + y) * (L - 1) + x], 2, 1, 2, 1));
    for (int y = 0; y + 1 < L; ++y)
      for (int x = 0; x < L; ++x)
        A.add_gate(1, x, y, flip_gate(p[nz + nx + ((z - 1) * (L - 1) + y) * L + x], 2, 1, 2, 1));
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        double q = p[z * L * L + y * L + x];
        Mat w = {1.0 - q, 0.0, 0.0, q};
        Mat wx = matmul(w, 2, 2, xmask(2, 1), 2);
        std::string e = A.add_post(y * L + x, w, 2, ((z - 1) * L + y) * L + x, wx);
        if (!e.empty()) return e;
      }
    std::string e = A.end_layer();
    if (!e.empty()) return e;
  }
  A.finish(std::vector<Mat>(L * L, Mat{1.0, 1.0}));
  return "";
}

// ---------------------------------------------------------------------------
// Rotated code with phenomenological noise: sweep across data rows.
// Grid: site column x in [0, d) (check column), y = t-1 for round t in
// [1, T+1].  The Z-checks of a gap row are open while the data rows on both
// sides are absorbed; the check with centre x2 (twice the x coordinate)
// sits at column (x2-1)/2, the left-edge checks at column 0, so one gap row's
// checks occupy distinct columns and consecutive gap rows share column 0 only.
// A site's physical leg lists the partial parities of the open checks it
// holds (older gap row in the low bit).
//   initial state: flips of data row 0 (they touch gap row 0 only and carry the
//     logical), per site the distribution of the parity feeding its check,
//     chained to total parity = coset.
//   layer j = 1..d-1: pre: open a zero bit for each check of gap row j
//     (j <= d-2) and apply the row-j flips whose two checks share a site;
//     gates: the other row-j flips between the sites of their two checks
//     (neighbours along x) and the measurement flips (c, t) of gap row j-1
//     between rounds t and t+1; post: restrict gap row j-1's bits to the
//     syndrome.
// ---------------------------------------------------------------------------
std::string build_rotated_phenom(int32_t d, int32_t T, const double* p, Program& P) {
  if (d < 3 || d % 2 == 0) return "d must be odd and >= 3";
  if (T < 1) return "T must be >= 1";
  if (!p) return "null rates";
  const int nq = d * d, nZ = (d * d - 1) / 2;
  const int n = T * nq + T * nZ;
  for (int i = 0; i < n; ++i)
    if (bad_rate(p[i])) return "rate outside [0, 1]";
  // checks: per gap row, left to right; column of each check; covering check
  // of (gap row, data column)
  std::vector<int> chk_row, chk_col;
  std::vector<std::vector<int>> chk_cols;
  std::map<std::pair<int, int>, int> cover;
  for (int g = 0; g < d - 1; ++g) {
    std::vector<std::pair<int, std::vector<int>>> row;  // (x2, data columns)
    if (g % 2 == 0) {
      for (int i = 0; i + 1 < d; i += 2) row.push_back({2 * i + 1, {i, i + 1}});
      row.push_back({2 * d - 1, {d - 1}});
    } else {
      row.push_back({-1, {0}});
      for (int i = 1; i + 1 < d; i += 2) row.push_back({2 * i + 1, {i, i + 1}});
    }
    std::sort(row.begin(), row.end(), [](auto& a, auto& b) { return a.first < b.first; });
    for (auto& [x2, cols] : row) {
      int c = int(chk_row.size());
      chk_row.push_back(g);
      chk_col.push_back(x2 < 0 ? 0 : (x2 - 1) / 2);
      chk_cols.push_back(cols);
      for (int i : cols) cover[{g, i}] = c;
    }
  }
  if (int(chk_row.size()) != nZ) return "internal: check count";
  auto pdata = [&](int i, int j, int t) { return p[(t - 1) * nq + j * d + i]; };
  auto pmeas = [&](int c, int t) { return p[T * nq + (t - 1) * nZ + c]; };

  P = Program{};
  P.name = "rotated_phenom_d" + std::to_string(d) + "_T" + std::to_string(T);
  P.n_det = nZ * (T + 1);
  P.n_mech = n;
  P.n_cosets = 2;
  const int Lx = d, Ly = T + 1, ns = Lx * Ly;
  Assembler A(P, Lx, Ly);
  // bits held per site (gap rows, oldest first)
  std::vector<std::vector<int>> held(ns);
  for (int c = 0; c < 2; ++c) {
    std::vector<std::vector<double>> w(ns);
    for (int ch = 0; ch < nZ; ++ch) {
      if (chk_row[ch] != 0) continue;
      for (int t = 1; t <= T + 1; ++t) {
        std::vector<double> v = {1.0, 0.0};
        if (t <= T)
          for (int i : chk_cols[ch]) {
            double q = pdata(i, 0, t);
            v = {v[0] * (1 - q) + v[1] * q, v[0] * q + v[1] * (1 - q)};
          }
        w[(t - 1) * Lx + chk_col[ch]] = v;
      }
    }
    A.d.assign(ns, 1);
    A.snake_init(w, c);
  }
  for (int ch = 0; ch < nZ; ++ch)
    if (chk_row[ch] == 0)
      for (int t = 1; t <= T + 1; ++t) held[(t - 1) * Lx + chk_col[ch]].push_back(0);
  auto bitpos = [&](int s, int g) {
    auto it = std::find(held[s].begin(), held[s].end(), g);
    return int(it - held[s].begin());
  };
  for (int j = 1; j < d; ++j) {
    const int gc = j - 1, go = j <= d - 2 ? j : -1;
    A.begin_layer();
    if (go >= 0)
      for (int ch = 0; ch < nZ; ++ch) {
        if (chk_row[ch] != go) continue;
        for (int t = 1; t <= T + 1; ++t) {
          int s = (t - 1) * Lx + chk_col[ch];
          int dold = 1 << held[s].size();
          Mat E(size_t(2 * dold) * dold, 0.0);
          for (int a = 0; a < dold; ++a) E[size_t(a) * dold + a] = 1.0;
          std::string e = A.add_pre(s, E, 2 * dold);
          if (!e.empty()) return e;
          held[s].push_back(go);
        }
      }
    for (int t = 1; t <= T; ++t) {
      const int y = t - 1;
      for (int i = 0; i < d; ++i) {
        int cc = cover[{gc, i}];
        int sa = y * Lx + chk_col[cc];
        int ba = bitpos(sa, gc);
        double q = pdata(i, j, t);
        if (go < 0) {
          int dd = 1 << held[sa].size();
          std::string e = A.add_pre(sa, flip_op(q, dd, 1 << ba), dd);
          if (!e.empty()) return e;
          continue;
        }
        int co = cover[{go, i}];
        int sb = y * Lx + chk_col[co];
        int bb = bitpos(sb, go);
        if (sa == sb) {
          int dd = 1 << held[sa].size();
          std::string e = A.add_pre(sa, flip_op(q, dd, (1 << ba) | (1 << bb)), dd);
          if (!e.empty()) return e;
          continue;
        }
        int xa = chk_col[cc], xb = chk_col[co];
        if (std::abs(xa - xb) != 1) return "internal: flip between non-neighbour sites";
        if (xa < xb)
          A.add_gate(0, xa, y, flip_gate(q, 1 << held[sa].size(), 1 << ba, 1 << held[sb].size(), 1 << bb));
        else
          A.add_gate(0, xb, y, flip_gate(q, 1 << held[sb].size(), 1 << bb, 1 << held[sa].size(), 1 << ba));
      }
      for (int ch = 0; ch < nZ; ++ch) {
        if (chk_row[ch] != gc) continue;
        int x = chk_col[ch];
        int sa = y * Lx + x, sb = (y + 1) * Lx + x;
        A.add_gate(1, x, y, flip_gate(pmeas(ch, t), 1 << held[sa].size(), 1 << bitpos(sa, gc),
                                      1 << held[sb].size(), 1 << bitpos(sb, gc)));
      }
    }
    for (int ch = 0; ch < nZ; ++ch) {
      if (chk_row[ch] != gc) continue;
      for (int t = 1; t <= T + 1; ++t) {
        int s = (t - 1) * Lx + chk_col[ch];
        int k = bitpos(s, gc);
        int dold = 1 << held[s].size();
        Mat P0(size_t(dold / 2) * dold, 0.0), P1 = P0;
        for (int a = 0; a < dold; ++a) {
          int low = a & ((1 << k) - 1), high = a >> (k + 1);
          int r = low | (high << k);
          if (((a >> k) & 1) == 0)
            P0[size_t(r) * dold + a] = 1.0;
          else
            P1[size_t(r) * dold + a] = 1.0;
        }
        std::string e = A.add_post(s, P0, dold / 2, (t - 1) * nZ + ch, P1);
        if (!e.empty()) return e;
        held[s].erase(held[s].begin() + k);
      }
    }
    std::string e = A.end_layer();
    if (!e.empty()) return e;
  }
  for (auto& h : held)
    if (!h.empty()) return "internal: open checks left after the sweep";
  A.finish(std::vector<Mat>(ns, Mat{1.0}));
  return "";
}

// ---------------------------------------------------------------------------
// 3D planar code under depolarizing noise, both sectors at once (coset
// c = a + 2b: a the class of the X part, read on the vertical string of
// z-edges above (0, 0); b that of the Z part, read on the bottom membrane).
// Sweep along z over the L x L vertex grid; the physical index of a site is
// s + 2 g with
//   s  the Z part of the z-edge entering the next vertex (detector picture,
//      as in the point sector), and
//   g  the generator bit of the vertex last absorbed: the X parts of a coset
//      are u = r + sum_v g_v S_v over the vertex stabilizers S_v, for one
//      representative r of the coset's face syndrome and class.
// An edge e between vertices v, w carries the Pauli with X part
// r_e + g_v + g_w and Z part t, weight W = 1-p_e (I) or p_e/3 (X, Y, Z).
// Its gate, summed over t, is
//   sum_t X_s^t (x) X_s^t [alpha_t + beta_t (-1)^{r_e} Z_g (x) Z_g]
// with alpha_t, beta_t the even and odd parts of W(., t) in the X part:
// operator-Schmidt rank 3 (beta_1 = 0), and r_e flips the sign of the Z_g
// term.  r = B m_Z for a fixed GF(2) map B with zero on the string above
// (0, 0) and on the top dangling edges, so the class a enters only through
// the bottom edges' weights: the initial generator bit below level 1 is a
// (r + a times the bottom membrane).  The r bits are derived per item from
// the face syndrome on the device (Program::ext_rows).
// ---------------------------------------------------------------------------
namespace {

using Bits = std::vector<uint64_t>;

inline void bx(Bits& a, const Bits& b) {
  for (size_t i = 0; i < a.size(); ++i) a[i] ^= b[i];
}
inline int bget(const Bits& a, int i) { return int((a[i >> 6] >> (i & 63)) & 1u); }
inline void bflip(Bits& a, int i) { a[i >> 6] ^= uint64_t(1) << (i & 63); }

// The face checks of the 3D planar code of size L (canonical order) and the
// fixed GF(2) map B from a face syndrome to a representative bit-flip
// pattern r = B m: r has that face syndrome when m is consistent, class 0
// (even parity on the string of z-edges above (0, 0)) and zero on the top
// dangling edges.  cube[i] (i < n_cube) are the rows of the elimination that
// combine the face checks into zero: m is consistent iff every cube[i].m = 0.
struct FaceMap {
  int nf = 0, n = 0, wf = 0;
  std::vector<Bits> B;     // [edge] bits over faces
  std::vector<Bits> cube;  // cube relations, bits over faces
};

FaceMap face_map(int L) {
  const int nz = L * L * L, nx = L * (L - 1) * (L - 1);
  const int n = nz + 2 * nx;
  auto ze = [&](int x, int y, int z) { return z * L * L + y * L + x; };
  auto xe = [&](int x, int y, int z) { return nz + ((z - 1) * L + y) * (L - 1) + x; };
  auto ye = [&](int x, int y, int z) { return nz + nx + ((z - 1) * (L - 1) + y) * L + x; };
  std::vector<std::vector<int>> faces;
  for (int z = 1; z < L; ++z)
    for (int y = 0; y + 1 < L; ++y)
      for (int x = 0; x + 1 < L; ++x) faces.push_back({xe(x, y, z), xe(x, y + 1, z), ye(x, y, z), ye(x + 1, y, z)});
  for (int z = 0; z < L; ++z)
    for (int y = 0; y < L; ++y)
      for (int x = 0; x + 1 < L; ++x) {
        std::vector<int> f = {ze(x, y, z), ze(x + 1, y, z)};
        if (z >= 1) f.push_back(xe(x, y, z));
        if (z + 1 < L) f.push_back(xe(x, y, z + 1));
        faces.push_back(f);
      }
  for (int z = 0; z < L; ++z)
    for (int y = 0; y + 1 < L; ++y)
      for (int x = 0; x < L; ++x) {
        std::vector<int> f = {ze(x, y, z), ze(x, y + 1, z)};
        if (z >= 1) f.push_back(ye(x, y, z));
        if (z + 1 < L) f.push_back(ye(x, y, z + 1));
        faces.push_back(f);
      }
  FaceMap M;
  const int nf = int(faces.size());
  const int wq = (n + 63) / 64, wf = (nf + 63) / 64;
  M.nf = nf;
  M.n = n;
  M.wf = wf;
  // Gauss-Jordan on H_Z (rows = faces, bit columns = qubits), tracking the
  // row operations E, so that E H_Z is reduced: for a consistent m_Z,
  // r[pivot col of row i] = (E m_Z)_i and zero elsewhere.
  std::vector<Bits> H(nf, Bits(wq, 0)), E(nf, Bits(wf, 0));
  for (int f = 0; f < nf; ++f) {
    for (int e : faces[f]) bflip(H[f], e);
    bflip(E[f], f);
  }
  M.B.assign(n, Bits(wf, 0));
  std::vector<int> pcol;
  int rank = 0;
  for (int col = 0; col < n && rank < nf; ++col) {
    int piv = -1;
    for (int r = rank; r < nf; ++r)
      if (bget(H[r], col)) {
        piv = r;
        break;
      }
    if (piv < 0) continue;
    std::swap(H[piv], H[rank]);
    std::swap(E[piv], E[rank]);
    for (int r = 0; r < nf; ++r)
      if (r != rank && bget(H[r], col)) {
        bx(H[r], H[rank]);
        bx(E[r], E[rank]);
      }
    pcol.push_back(col);
    ++rank;
  }
  for (int i = 0; i < rank; ++i) M.B[pcol[i]] = E[i];
  // class of r is its parity on the string above (0, 0); remove it by adding
  // the bottom membrane (which meets the string once)
  Bits zrow(wf, 0);
  for (int z = 0; z < L; ++z) bx(zrow, M.B[ze(0, 0, z)]);
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) bx(M.B[ze(x, y, 0)], zrow);
  // clear the top dangling edges with the stabilizers of the top vertices
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const Bits t = M.B[ze(x, y, L - 1)];
      std::vector<int> st = {ze(x, y, L - 1), ze(x, y, L - 2)};
      if (x > 0) st.push_back(xe(x - 1, y, L - 1));
      if (x + 1 < L) st.push_back(xe(x, y, L - 1));
      if (y > 0) st.push_back(ye(x, y - 1, L - 1));
      if (y + 1 < L) st.push_back(ye(x, y, L - 1));
      for (int e : st) bx(M.B[e], t);
    }
  // rows rank..nf of E combine the face checks into zero (E H_Z = 0 there)
  for (int i = rank; i < nf; ++i) M.cube.push_back(E[i]);
  return M;
}

// Per-item derived bits of a face-syndrome family: bit n_det + e is r_e
// (e < n), then the cube-relation parities (INCONSISTENT when one is set).
void set_face_ext(Program& P, const FaceMap& M, int src0) {
  const int n_chk = int(M.cube.size());
  P.n_ext = M.n + n_chk;
  P.ext_src0 = src0;
  P.ext_src_n = M.nf;
  P.ext_words = M.wf;
  P.ext_rows.resize(size_t(M.n + n_chk) * M.wf);
  for (int e = 0; e < M.n; ++e)
    for (int w = 0; w < M.wf; ++w) P.ext_rows[size_t(e) * M.wf + w] = M.B[e][w];
  for (int i = 0; i < n_chk; ++i)
    for (int w = 0; w < M.wf; ++w) P.ext_rows[size_t(M.n + i) * M.wf + w] = M.cube[i][w];
  P.inc0 = P.n_det + M.n;
  P.n_inc = n_chk;
}

}  // namespace

std::string build_surface3d_depol(int32_t L, const double* p, Program& P) {
  if (L < 2) return "L must be >= 2";
  if (!p) return "null rates";
  const int nz = L * L * L, nx = L * (L - 1) * (L - 1);
  const int n = nz + 2 * nx;
  for (int i = 0; i < n; ++i)
    if (!(p[i] >= 0.0 && p[i] <= 0.75)) return "depolarizing rate outside [0, 3/4]";
  auto ze = [&](int x, int y, int z) { return z * L * L + y * L + x; };
  auto xe = [&](int x, int y, int z) { return nz + ((z - 1) * L + y) * (L - 1) + x; };
  auto ye = [&](int x, int y, int z) { return nz + nx + ((z - 1) * (L - 1) + y) * L + x; };
  const FaceMap FM = face_map(L);
  const int nf = FM.nf, nv = L * L * (L - 1);

  P = Program{};
  P.name = "surface3d_depolarizing_L" + std::to_string(L);
  P.n_det = nv + nf;
  P.n_mech = n;
  P.n_cosets = 4;
  P.rate_max = 0.75;
  set_face_ext(P, FM, nv);

  auto W = [&](int e, int u, int v) { return (u == 0 && v == 0) ? 1.0 - p[e] : p[e] / 3.0; };
  auto I4 = eye(4);
  Mat Zg(16, 0.0), Xs = xmask(4, 1);
  for (int i = 0; i < 4; ++i) Zg[i * 4 + i] = (i >> 1) ? -1.0 : 1.0;
  auto gate_terms = [&](int e, int sgn) {
    const double al = 0.5 * (W(e, 0, 0) + W(e, 1, 0)), be = 0.5 * (W(e, 0, 0) - W(e, 1, 0)), t1 = W(e, 0, 1);
    std::vector<Term> ts;
    ts.push_back({scaled(I4, std::sqrt(al)), scaled(I4, std::sqrt(al))});
    if (be != 0.0)
      ts.push_back({scaled(Zg, be > 0 ? std::sqrt(be) : -std::sqrt(-be)), scaled(Zg, sgn * std::sqrt(std::fabs(be)))});
    if (t1 != 0.0) ts.push_back({scaled(Xs, std::sqrt(t1)), scaled(Xs, std::sqrt(t1))});
    return ts;
  };

  Assembler A(P, L, L);
  for (int c = 0; c < 4; ++c) {
    A.d.assign(L * L, 1);
    A.snake_init(std::vector<std::vector<double>>(L * L, {1.0, 1.0}), c >> 1, 4, 2 * (c & 1), c);
  }
  const int ndet = P.n_det;
  for (int z = 1; z < L; ++z) {
    A.begin_layer();
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int e = ze(x, y, z - 1);
        Mat M0(16, 0.0), M1(16, 0.0);
        for (int g = 0; g < 2; ++g)
          for (int g2 = 0; g2 < 2; ++g2)
            for (int sb = 0; sb < 2; ++sb) {
              M0[(sb + 2 * g2) * 4 + sb + 2 * g] = W(e, g ^ g2, sb);
              M1[(sb + 2 * g2) * 4 + sb + 2 * g] = W(e, 1 ^ g ^ g2, sb);
            }
        std::string er = A.add_pre(y * L + x, M0, 4, ndet + e, M1);
        if (!er.empty()) return er;
      }
    for (int y = 0; y < L; ++y)
      for (int x = 0; x + 1 < L; ++x) {
        const int e = xe(x, y, z);
        A.add_gate(0, x, y, gate_terms(e, 1), ndet + e, gate_terms(e, -1));
      }
    for (int y = 0; y + 1 < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int e = ye(x, y, z);
        A.add_gate(1, x, y, gate_terms(e, 1), ndet + e, gate_terms(e, -1));
      }
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        std::string er = A.add_post(y * L + x, I4, 4, ((z - 1) * L + y) * L + x, Xs);
        if (!er.empty()) return er;
      }
    std::string er = A.end_layer();
    if (!er.empty()) return er;
  }
  std::vector<Mat> f;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int e = ze(x, y, L - 1);
      f.push_back({W(e, 0, 0), W(e, 0, 1), W(e, 1, 0), W(e, 1, 1)});
    }
  A.finish(f);
  return "";
}

// ---------------------------------------------------------------------------
// 3D planar code, loop sector: bit flips on the edges seen by the face checks,
// in the generator picture (paper Sec. 3.2; the loop-sector network of the
// experiments has the cubic shape of the point sector with the roles of the
// parity and copy nodes exchanged).  Every flip pattern u with face syndrome
// m and class a is r + a (bottom membrane) + sum_v g_v s_v for the
// representative r = B m of the face map and one bit g_v per vertex, so the
// physical leg of a site is the generator bit g of the vertex last absorbed,
// dimension 2.  The initial state of coset a is the product state g = a (the
// bit of a virtual vertex below level 1, which adds the bottom membrane).
// Layer z: pre-op per site for the z-edge below (x, y, z), g -> g' with weight
// W(e, r_e + g + g'); a diagonal gate per in-plane edge, W(e, r_e + g_A +
// g_B) = 1/2 + (1/2 - p_e) (-1)^r_e Z (x) Z (operator-Schmidt rank 2, the
// sign of the Z term follows the per-item bit r_e).  Final vectors: the top
// dangling edges, W(e, g) (r is zero there).
// ---------------------------------------------------------------------------
std::string build_surface3d_loop(int32_t L, const double* p, Program& P, bool wht) {
  if (L < 2) return "L must be >= 2";
  if (!p) return "null rates";
  const int nz = L * L * L, nx = L * (L - 1) * (L - 1);
  const int n = nz + 2 * nx;
  for (int i = 0; i < n; ++i)
    if (!(p[i] >= 0.0 && p[i] <= 1.0)) return "flip rate outside [0, 1]";
  auto ze = [&](int x, int y, int z) { return z * L * L + y * L + x; };
  auto xe = [&](int x, int y, int z) { return nz + ((z - 1) * L + y) * (L - 1) + x; };
  auto ye = [&](int x, int y, int z) { return nz + nx + ((z - 1) * (L - 1) + y) * L + x; };
  const FaceMap FM = face_map(L);

  P = Program{};
  P.name = "surface3d_loop_L" + std::to_string(L);
  P.n_det = FM.nf;
  P.n_mech = n;
  P.n_cosets = 2;
  set_face_ext(P, FM, 0);

  auto W = [&](int e, int u) { return u ? p[e] : 1.0 - p[e]; };
  Mat Zg = {1.0, 0.0, 0.0, -1.0};
  auto gate_terms = [&](int e, int sgn) {
    const double al = 0.5, be = 0.5 - p[e];
    std::vector<Term> ts;
    ts.push_back({scaled(eye(2), std::sqrt(al)), scaled(eye(2), std::sqrt(al))});
    if (be != 0.0)
      ts.push_back({scaled(Zg, be > 0 ? std::sqrt(be) : -std::sqrt(-be)), scaled(Zg, sgn * std::sqrt(std::fabs(be)))});
    return ts;
  };

  P.wht = wht ? 1 : 0;
  Assembler A(P, L, L);
  for (int c = 0; c < 2; ++c) {
    if (wht) {
      // Z_c = sum_a (-1)^(a c) P_a: the bit a below level 1 is shared by
      // every site, a chain of equal bits carrying the sign on its first site
      A.copy_chain_init(c);
    } else {
      std::vector<std::vector<double>> v(L * L, {c == 0 ? 1.0 : 0.0, c == 0 ? 0.0 : 1.0});
      A.product_init(v, c);
    }
  }
  const int ndet = P.n_det;
  for (int z = 1; z < L; ++z) {
    A.begin_layer();
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int e = ze(x, y, z - 1);
        Mat M0(4, 0.0), M1(4, 0.0);
        for (int g = 0; g < 2; ++g)
          for (int g2 = 0; g2 < 2; ++g2) {
            M0[g2 * 2 + g] = W(e, g ^ g2);
            M1[g2 * 2 + g] = W(e, 1 ^ g ^ g2);
          }
        std::string er = A.add_pre(y * L + x, M0, 2, ndet + e, M1);
        if (!er.empty()) return er;
      }
    for (int y = 0; y < L; ++y)
      for (int x = 0; x + 1 < L; ++x) {
        const int e = xe(x, y, z);
        A.add_gate(0, x, y, gate_terms(e, 1), ndet + e, gate_terms(e, -1));
      }
    for (int y = 0; y + 1 < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int e = ye(x, y, z);
        A.add_gate(1, x, y, gate_terms(e, 1), ndet + e, gate_terms(e, -1));
      }
    std::string er = A.end_layer();
    if (!er.empty()) return er;
  }
  std::vector<Mat> f;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      const int e = ze(x, y, L - 1);
      f.push_back({W(e, 0), W(e, 1)});
    }
  A.finish(f);
  return "";
}

// ---------------------------------------------------------------------------
// Generic front end: the detector-picture network (paper Sec. 3.1, 3.4) of a
// graph-like DEM whose detectors sit on a grid, swept along the detector
// coordinate t (layers) over the (x, y) grid.  Every mechanism flips one or
// two detectors: two at grid-adjacent sites of one layer (an in-plane gate
// (1-p) I I + p X X), two at one site in consecutive layers (time-like: the
// flip carried on the site's physical leg from the lower detector to the
// upper one), or one (a boundary flip (1-p) I + p X on the detector's
// parity).  Parallel mechanisms are merged exactly (the parity of independent
// flips).  The physical leg of a site holds the parity of its current
// detector; after the layer's gates the detector's check sets it to m_d:
// with a time-like edge upwards the leg then carries that edge's flip
// (weight diag(1-q, q)), otherwise it is projected on parity m_d and the site
// holds no bit until its next detector.  The observable (one row) must
// consist of boundary mechanisms of the first layer: their flips are the
// initial bits, chained to the coset parity (as the bottom dangling edges of
// the 3D planar code).
// ---------------------------------------------------------------------------
std::string build_from_dem(int32_t n_det, int32_t n_mech, int64_t nnz, const int32_t* det_idx,
                           const int32_t* mech_idx, const double* p, int32_t n_obs, const uint8_t* obs,
                           const int32_t* coord, Program& P) {
  if (n_det < 1 || n_mech < 1 || nnz < 0) return "empty DEM";
  if (!det_idx || !mech_idx || !p || !obs || !coord) return "null pointer";
  if (n_obs != 1) return "UNSUPPORTED: exactly one observable row is supported";
  for (int i = 0; i < n_mech; ++i)
    if (!(p[i] >= 0.0 && p[i] <= 1.0)) return "rate outside [0, 1]";
  // detectors of each mechanism (a detector listed twice cancels)
  std::vector<std::vector<int>> md(n_mech);
  for (int64_t k = 0; k < nnz; ++k) {
    const int d = det_idx[k], m = mech_idx[k];
    if (d < 0 || d >= n_det || m < 0 || m >= n_mech) return "COO index out of range";
    auto& v = md[m];
    auto it = std::find(v.begin(), v.end(), d);
    if (it == v.end())
      v.push_back(d);
    else
      v.erase(it);
  }
  int Lx = 0, Ly = 0, t0 = INT32_MAX, t1 = INT32_MIN;
  for (int d = 0; d < n_det; ++d) {
    const int x = coord[3 * d], y = coord[3 * d + 1], t = coord[3 * d + 2];
    if (x < 0 || y < 0) return "negative detector coordinate";
    Lx = std::max(Lx, x + 1);
    Ly = std::max(Ly, y + 1);
    t0 = std::min(t0, t);
    t1 = std::max(t1, t);
  }
  if (int64_t(Lx) * Ly > 4096) return "UNSUPPORTED: grid above 4096 sites";
  const int nl = t1 - t0 + 1, ns = Lx * Ly;
  if (nl > 4096) return "UNSUPPORTED: more than 4096 layers";
  std::vector<int> at(size_t(ns) * nl, -1);  // detector at (site, layer)
  std::vector<int> dsite(n_det), dlay(n_det);
  for (int d = 0; d < n_det; ++d) {
    const int s = coord[3 * d + 1] * Lx + coord[3 * d], l = coord[3 * d + 2] - t0;
    if (at[size_t(s) * nl + l] >= 0) return "two detectors share a grid point";
    at[size_t(s) * nl + l] = d;
    dsite[d] = s;
    dlay[d] = l;
  }
  // merged odd-parity probabilities: q_odd of independent flips q_a, q_b
  auto merge = [](double a, double b) { return a + b - 2.0 * a * b; };
  std::vector<double> bnd(n_det, 0.0), up(n_det, 0.0), obs0(ns, 0.0);
  std::vector<char> has_up(n_det, 0), has_obs(ns, 0);
  std::map<std::pair<int, int>, double> inplane;  // (lower det, higher det) -> q
  for (int m = 0; m < n_mech; ++m) {
    const auto& v = md[m];
    const bool in_obs = obs[m] != 0;
    if (v.empty()) {
      if (in_obs) return "UNSUPPORTED: a mechanism flips the observable but no detector";
      continue;  // sums to one
    }
    if (v.size() > 2) return "UNSUPPORTED: a mechanism flips more than two detectors";
    if (v.size() == 1) {
      const int d = v[0];
      if (in_obs) {
        if (dlay[d] != 0) return "UNSUPPORTED: observable mechanisms must be boundary flips of the first layer";
        obs0[dsite[d]] = merge(obs0[dsite[d]], p[m]);
        has_obs[dsite[d]] = 1;
      } else {
        bnd[d] = merge(bnd[d], p[m]);
      }
      continue;
    }
    if (in_obs) return "UNSUPPORTED: observable mechanisms must be boundary flips of the first layer";
    int a = v[0], b = v[1];
    if (dlay[a] > dlay[b] || (dlay[a] == dlay[b] && dsite[a] > dsite[b])) std::swap(a, b);
    const int xa = dsite[a] % Lx, ya = dsite[a] / Lx, xb = dsite[b] % Lx, yb = dsite[b] / Lx;
    if (dlay[a] == dlay[b] && std::abs(xa - xb) + std::abs(ya - yb) == 1) {
      auto key = std::make_pair(a, b);
      auto it = inplane.find(key);
      inplane[key] = it == inplane.end() ? p[m] : merge(it->second, p[m]);
    } else if (dsite[a] == dsite[b] && dlay[b] == dlay[a] + 1) {
      up[a] = merge(up[a], p[m]);
      has_up[a] = 1;
    } else {
      return "UNSUPPORTED: a mechanism joins detectors that are neither grid neighbours of one layer nor one site "
             "in consecutive layers";
    }
  }

  P = Program{};
  P.name = "dem_" + std::to_string(n_det) + "x" + std::to_string(n_mech);
  P.n_det = n_det;
  P.n_mech = n_mech;
  P.n_cosets = 2;
  Assembler A(P, Lx, Ly);
  for (int c = 0; c < 2; ++c) {
    std::vector<std::vector<double>> w(ns);
    for (int s2 = 0; s2 < ns; ++s2)
      if (has_obs[s2]) w[s2] = {1.0 - obs0[s2], obs0[s2]};
    A.d.assign(ns, 1);
    A.snake_init(w, c);
  }
  const Mat I2 = eye(2);
  for (int l = 0; l < nl; ++l) {
    A.begin_layer();
    for (int s2 = 0; s2 < ns; ++s2) {
      const int d = at[size_t(s2) * nl + l];
      if (d < 0) continue;
      if (A.staged_dim(s2) == 1) {
        // no bit on the site yet: the detector's parity starts at 0
        std::string er = A.add_pre(s2, Mat{1.0, 0.0}, 2);
        if (!er.empty()) return er;
      }
      if (bnd[d] > 0.0) {
        std::string er = A.add_pre(s2, flip_op(bnd[d], 2, 1), 2);
        if (!er.empty()) return er;
      }
    }
    for (const auto& kv : inplane) {
      const int a = kv.first.first, b = kv.first.second;
      if (dlay[a] != l) continue;
      const int sa = dsite[a], sb = dsite[b];
      const int xa = sa % Lx, ya = sa / Lx;
      // the assembler's gate joins (x, y) with its east or south neighbour
      if (sb == sa + 1)
        A.add_gate(0, xa, ya, flip_gate(kv.second, 2, 1, 2, 1));
      else if (sb == sa + Lx)
        A.add_gate(1, xa, ya, flip_gate(kv.second, 2, 1, 2, 1));
      else
        return "internal: in-plane pair not ordered";
    }
    for (int s2 = 0; s2 < ns; ++s2) {
      const int d = at[size_t(s2) * nl + l];
      if (d < 0) continue;
      std::string er;
      if (has_up[d]) {
        // the leg becomes the flip of the edge to the next detector: X^m,
        // then its weight
        const double q = up[d];
        Mat wq = {1.0 - q, 0.0, 0.0, q};
        er = A.add_post(s2, wq, 2, d, matmul(wq, 2, 2, xmask(2, 1), 2));
      } else {
        // parity must equal m_d: keep b = m_d, the site holds no bit after
        er = A.add_post(s2, Mat{1.0, 0.0}, 1, d, Mat{0.0, 1.0});
      }
      if (!er.empty()) return er;
    }
    std::string er = A.end_layer();
    if (!er.empty()) return er;
  }
  std::vector<Mat> f(ns);
  for (int s2 = 0; s2 < ns; ++s2) {
    if (A.d[s2] != 1) return "internal: a bit left after the last layer";
    f[s2] = {1.0};
  }
  A.finish(f);
  return "";
}


namespace {

// Operator-Schmidt terms of a dense two-site operator G[a'][b'][a][b] (dims
// dA, dB) by a singular value decomposition of its matrix
// M[(a', a)][(b', b)]: one-sided Jacobi (Hestenes) on the columns of M, V
// accumulating the rotations, then OA_k = sqrt(s_k) u_k, OB_k = sqrt(s_k) v_k
// for the singular values s_k > tol s_1 (the paper's general gate splitting,
// Sec. 4).  An all-zero operator gives one zero term.
std::vector<Term> svd_split(const double* G, int dA, int dB, double tol) {
  const int m = dA * dA, n = dB * dB;
  std::vector<double> M(size_t(m) * n), V(size_t(n) * n, 0.0);
  for (int a2 = 0; a2 < dA; ++a2)
    for (int b2 = 0; b2 < dB; ++b2)
      for (int a = 0; a < dA; ++a)
        for (int b = 0; b < dB; ++b)
          M[size_t(a2 * dA + a) * n + (b2 * dB + b)] = G[((size_t(a2) * dB + b2) * dA + a) * dB + b];
  for (int j = 0; j < n; ++j) V[size_t(j) * n + j] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int i = 0; i < n - 1; ++i)
      for (int j = i + 1; j < n; ++j) {
        double alpha = 0, beta = 0, gamma = 0;
        for (int r = 0; r < m; ++r) {
          const double x = M[size_t(r) * n + i], y = M[size_t(r) * n + j];
          alpha += x * x;
          beta += y * y;
          gamma += x * y;
        }
        if (gamma == 0.0 || !(std::fabs(gamma) > 1e-15 * std::sqrt(alpha * beta))) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int r = 0; r < m; ++r) {
          const double x = M[size_t(r) * n + i], y = M[size_t(r) * n + j];
          M[size_t(r) * n + i] = c * x - sn * y;
          M[size_t(r) * n + j] = sn * x + c * y;
        }
        for (int r = 0; r < n; ++r) {
          const double x = V[size_t(r) * n + i], y = V[size_t(r) * n + j];
          V[size_t(r) * n + i] = c * x - sn * y;
          V[size_t(r) * n + j] = sn * x + c * y;
        }
      }
    if (!rotated) break;
  }
  std::vector<std::pair<double, int>> sv;
  for (int j = 0; j < n; ++j) {
    double s2 = 0;
    for (int r = 0; r < m; ++r) s2 += M[size_t(r) * n + j] * M[size_t(r) * n + j];
    sv.push_back({std::sqrt(s2), j});
  }
  std::stable_sort(sv.begin(), sv.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first;
  });
  std::vector<Term> terms;
  const double s1 = sv.empty() ? 0.0 : sv[0].first;
  for (const auto& e : sv) {
    const double sk = e.first;
    const int j = e.second;
    if (!terms.empty() && !(sk > tol * s1)) break;
    Term t{Mat(size_t(dA) * dA, 0.0), Mat(size_t(dB) * dB, 0.0)};
    const double r = std::sqrt(sk);
    // column j of M is s_k u_k: u_k sqrt(s_k) = column / sqrt(s_k)
    for (int a2 = 0; a2 < dA; ++a2)
      for (int a = 0; a < dA; ++a) t.A[size_t(a2) * dA + a] = sk > 0.0 ? M[size_t(a2 * dA + a) * n + j] / r : 0.0;
    for (int b2 = 0; b2 < dB; ++b2)
      for (int b = 0; b < dB; ++b) t.B[size_t(b2) * dB + b] = V[size_t(b2 * dB + b) * n + j] * r;
    terms.push_back(std::move(t));
  }
  return terms;
}

}  // namespace

std::string build_from_layers(int32_t lx, int32_t ly, int32_t n_layers, int32_t n_det, int32_t n_cosets,
                              const int32_t* init_dims, const int64_t* init_off, int32_t n_ops, const LayerOp* ops,
                              const int64_t* final_off, const double* values, int64_t n_values, double split_tol,
                              Program& P) {
  if (!init_dims || !init_off || !final_off || !values || (n_ops > 0 && !ops)) return "null pointer";
  if (lx < 2 || ly < 2 || int64_t(lx) * ly > 4096) return "grid must be at least 2 x 2 and at most 4096 sites";
  if (n_layers < 1 || n_layers > 4096 || n_cosets < 1 || n_cosets > 4 || n_det < 0 || n_ops < 0 || n_values < 0)
    return "bad counts (n_layers in 1..4096, n_cosets in 1..4, n_det >= 0)";
  if (!(split_tol >= 0.0 && split_tol < 1.0)) return "split_tol must lie in [0, 1)";
  for (int64_t i = 0; i < n_values; ++i)
    if (!std::isfinite(values[i])) return "values must be finite";
  const int ns = lx * ly;
  auto in_range = [&](int64_t off, int64_t len) { return off >= 0 && len >= 0 && off <= n_values - len; };
  P = Program{};
  P.name = "layers";
  P.n_det = n_det;
  P.n_mech = 0;
  P.n_cosets = n_cosets;
  Assembler A(P, lx, ly);
  // initial states: every coset with the same physical and bond dimensions
  P.init_dims.assign(size_t(n_cosets) * ns * 5, 1);
  P.init_off.assign(size_t(n_cosets) * ns, 0);
  P.bond_dim0.assign(P.n_bonds, 0);
  for (int c = 0; c < n_cosets; ++c)
    for (int s = 0; s < ns; ++s) {
      const int32_t* dm = init_dims + (size_t(c) * ns + s) * 5;
      for (int i = 0; i < 5; ++i)
        if (dm[i] < 1 || dm[i] != init_dims[size_t(s) * 5 + i])
          return "initial dims must be positive and equal across cosets";
      if (dm[0] > 16) return "physical dimension above 16";
      for (int leg = 0; leg < 4; ++leg) {
        const int b = P.leg_bond[s * 4 + leg];
        if (b < 0 && dm[1 + leg] != 1) return "a boundary leg of an initial tensor must have dimension 1";
        if (b >= 0) {
          if (dm[1 + leg] > 64) return "initial bond dimension above 64";
          if (P.bond_dim0[b] == 0) P.bond_dim0[b] = dm[1 + leg];
          if (P.bond_dim0[b] != dm[1 + leg]) return "the two ends of an initial bond differ in dimension";
        }
      }
      const int64_t n = int64_t(dm[0]) * dm[1] * dm[2] * dm[3] * dm[4];
      const int64_t off = init_off[size_t(c) * ns + s];
      if (!in_range(off, n)) return "initial tensor outside values";
      // given as [p][w][e][n][s]; stored as [w][e][n][s][p]
      Mat t(static_cast<size_t>(n));
      const int64_t nv = n / dm[0];
      for (int p = 0; p < dm[0]; ++p)
        for (int64_t v = 0; v < nv; ++v) t[size_t(v * dm[0] + p)] = values[off + p * nv + v];
      for (int i = 0; i < 5; ++i) P.init_dims[(size_t(c) * ns + s) * 5 + i] = dm[i];
      P.init_off[size_t(c) * ns + s] = A.put(t);
    }
  for (int b = 0; b < P.n_bonds; ++b)
    if (P.bond_dim0[b] == 0) P.bond_dim0[b] = 1;
  for (int s = 0; s < ns; ++s) {
    A.d[s] = init_dims[size_t(s) * 5];
    P.dmax[s] = std::max(P.dmax[s], A.d[s]);
  }
  // layers: per layer the one-site ops before the gates, the gates, then the
  // one-site ops after them, each group in array order
  int32_t k0 = 0;
  for (int l = 0; l < n_layers; ++l) {
    int32_t k1 = k0;
    while (k1 < n_ops && ops[k1].layer == l) ++k1;
    A.begin_layer();
    std::vector<char> bond_used(P.n_bonds, 0);
    for (int pass = 0; pass < 3; ++pass)
      for (int32_t k = k0; k < k1; ++k) {
        const LayerOp& o = ops[k];
        if (o.x < 0 || o.x >= lx || o.y < 0 || o.y >= ly) return "op site outside the grid";
        if (o.det < -1 || o.det >= n_det) return "op detector index out of range";
        if (o.kind != OP_PRE && o.kind != OP_POST && o.kind != OP_GATE_H && o.kind != OP_GATE_V)
          return "unknown op kind";
        const int want = o.kind == OP_PRE ? 0 : o.kind == OP_POST ? 2 : 1;
        if (want != pass) continue;
        const int s = o.y * lx + o.x;
        if (pass != 1) {
          if (o.d_out < 1 || o.d_out > 16 || o.d_in < 1 || o.d_in > 16) return "one-site op dims out of range";
          const int64_t n = int64_t(o.d_in) * o.d_out;
          if (!in_range(o.off0, n) || (o.det >= 0 && !in_range(o.off1, n))) return "one-site op outside values";
          Mat M0(values + o.off0, values + o.off0 + n), M1;
          if (o.det >= 0) M1.assign(values + o.off1, values + o.off1 + n);
          // the assembler composes it after the site's pending op and checks
          // its input dimension against the site's
          std::string e =
              pass == 0 ? A.add_pre(s, M0, o.d_out, o.det, M1) : A.add_post(s, M0, o.d_out, o.det, M1);
          if (!e.empty()) return e;
        } else {
          const bool h = o.kind == OP_GATE_H;
          if ((h && o.x + 1 >= lx) || (!h && o.y + 1 >= ly)) return "gate reaches outside the grid";
          const int b = h ? A.hbond(o.x, o.y) : A.vbond(o.x, o.y);
          if (bond_used[b]) return "two gates on one bond in a layer";
          bond_used[b] = 1;
          const int sb = h ? s + 1 : s + lx;
          if (o.d_in != A.staged_dim(s) || o.d_out != A.staged_dim(sb)) return "gate dims differ from the sites'";
          const int64_t n = int64_t(o.d_in) * o.d_in * o.d_out * o.d_out;
          if (!in_range(o.off0, n) || (o.det >= 0 && !in_range(o.off1, n))) return "gate outside values";
          std::vector<Term> t0 = svd_split(values + o.off0, o.d_in, o.d_out, split_tol), t1;
          if (o.det >= 0) {
            t1 = svd_split(values + o.off1, o.d_in, o.d_out, split_tol);
            // equal term counts for both sets: pad with zero terms
            const size_t K = std::max(t0.size(), t1.size());
            for (std::vector<Term>* ts : {&t0, &t1})
              while (ts->size() < K)
                ts->push_back(Term{Mat(size_t(o.d_in) * o.d_in, 0.0), Mat(size_t(o.d_out) * o.d_out, 0.0)});
          }
          A.add_gate(h ? 0 : 1, o.x, o.y, std::move(t0), o.det, std::move(t1));
        }
      }
    std::string e = A.end_layer();
    if (!e.empty()) return e;
    k0 = k1;
  }
  if (k0 != n_ops) return "op layer indices must be nondecreasing and below n_layers";
  std::vector<Mat> f(ns);
  for (int s = 0; s < ns; ++s) {
    const int64_t off = final_off[s];
    if (!in_range(off, A.d[s])) return "final vector outside values";
    f[s].assign(values + off, values + off + A.d[s]);
  }
  A.finish(f);
  return "";
}

}  // namespace tn3d

