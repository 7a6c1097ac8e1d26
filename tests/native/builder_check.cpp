// Host-side check of the network builders under AddressSanitizer and
// UndefinedBehaviorSanitizer: every family at several sizes, the DEM front
// end, and invalid inputs; each returned program's tables are checked for
// consistency (offsets inside the pool, dims of gates matching their sites'
// capacities).  Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2310_10722_amd/csrc/program.h"

using namespace tn3d;

static int fails = 0;

static void expect(bool ok, const std::string& what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what.c_str());
    ++fails;
  }
}

static void check_program(const Program& P, const std::string& name) {
  const size_t pool = P.pool.size();
  const int ns = P.Lx * P.Ly;
  expect(P.Lx > 0 && P.Ly > 0, name + ": grid");
  expect(P.init_off.size() == size_t(P.n_cosets) * ns, name + ": init offsets per coset and site");
  expect(P.init_dims.size() == size_t(P.n_cosets) * ns * 5, name + ": init dims per coset and site");
  for (size_t i = 0; i < P.init_off.size(); ++i) {
    size_t n = 1;
    for (int k = 0; k < 5; ++k) n *= size_t(P.init_dims[i * 5 + k]);
    expect(size_t(P.init_off[i]) + n <= pool, name + ": initial tensor inside the pool");
  }
  for (const DevGate& g : P.gates) {
    expect(g.sa >= 0 && g.sa < ns && g.sb >= 0 && g.sb < ns, name + ": gate sites");
    expect(g.K >= 1 && g.dA >= 1 && g.dB >= 1, name + ": gate shape");
    expect(size_t(g.oA) + size_t(g.K) * g.dA * g.dA <= pool, name + ": gate terms A inside the pool");
    expect(size_t(g.oB) + size_t(g.K) * g.dB * g.dB <= pool, name + ": gate terms B inside the pool");
    expect(size_t(g.pA) + size_t(g.K) * g.K * g.dA * g.dA <= pool, name + ": gate products A inside the pool");
    expect(g.dA <= P.dmax[g.sa] && g.dB <= P.dmax[g.sb], name + ": gate dims within the site capacity");
  }
  for (const DevOneSite& o : P.ones) {
    expect(o.site >= 0 && o.site < ns, name + ": one-site op site");
    expect(size_t(o.m0) + size_t(o.din) * o.dout <= pool && size_t(o.m1) + size_t(o.din) * o.dout <= pool,
           name + ": one-site matrices inside the pool");
    expect(o.det < P.n_det + P.n_ext, name + ": one-site op bit index");
  }
  expect(P.d_after.size() == P.layers.size() * ns, name + ": dims after each layer");
  expect(P.f_off.size() == size_t(ns), name + ": final vectors");
  for (int s = 0; s < ns; ++s) expect(size_t(P.f_off[s]) + P.d_final[s] <= pool, name + ": final vector in pool");
  if (P.n_ext > 0) expect(P.ext_rows.size() == size_t(P.n_ext) * P.ext_words, name + ": derived-bit rows");
}

int main() {
  for (int L = 2; L <= 6; ++L) {
    const int n = L * L * L + 2 * L * (L - 1) * (L - 1);
    std::vector<double> p(n, 0.1), pd(n, 0.15);
    Program P;
    expect(build_surface3d_point(L, p.data(), P).empty(), "point builds");
    check_program(P, "point L" + std::to_string(L));
    expect(build_surface3d_point(L, p.data(), P, true).empty(), "point wht builds");
    check_program(P, "point wht L" + std::to_string(L));
    expect(build_surface3d_loop(L, p.data(), P).empty(), "loop builds");
    check_program(P, "loop L" + std::to_string(L));
    expect(build_surface3d_loop(L, p.data(), P, true).empty(), "loop wht builds");
    check_program(P, "loop wht L" + std::to_string(L));
    expect(build_surface3d_depol(L, pd.data(), P).empty(), "depolarizing builds");
    check_program(P, "depolarizing L" + std::to_string(L));
  }
  for (int d = 3; d <= 7; d += 2)
    for (int T = 1; T <= 4; ++T) {
      const int nZ = (d * d - 1) / 2;
      std::vector<double> p(size_t(T) * d * d + size_t(T) * nZ, 0.02);
      Program P;
      expect(build_rotated_phenom(d, T, p.data(), P).empty(), "rotated builds");
      check_program(P, "rotated d" + std::to_string(d) + " T" + std::to_string(T));
    }
  // invalid inputs are refused with a message, never read out of range
  {
    Program P;
    std::vector<double> bad(51, 0.1);
    bad[7] = 1.5;
    expect(!build_surface3d_point(3, bad.data(), P).empty(), "rate above 1 refused");
    bad[7] = std::nan("");
    expect(!build_surface3d_loop(3, bad.data(), P).empty(), "NaN rate refused");
    expect(!build_surface3d_point(1, bad.data(), P).empty(), "L = 1 refused");
    expect(!build_surface3d_point(3, nullptr, P).empty(), "null rates refused");
    expect(!build_rotated_phenom(4, 2, bad.data(), P).empty(), "even distance refused");
  }
  // the DEM front end: a 2 x 2 x 3 grid, every mechanism class, then errors
  {
    const int Lx = 2, Ly = 2, T = 3, nd = Lx * Ly * T;
    std::vector<int32_t> coord, di, mi;
    for (int t = 0; t < T; ++t)
      for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) coord.insert(coord.end(), {x, y, t});
    auto det = [&](int x, int y, int t) { return (t * Ly + y) * Lx + x; };
    int nm = 0;
    std::vector<uint8_t> obs;
    auto mech = [&](std::vector<int> ds, bool o) {
      for (int d : ds) {
        di.push_back(d);
        mi.push_back(nm);
      }
      obs.push_back(o ? 1 : 0);
      ++nm;
    };
    for (int y = 0; y < Ly; ++y)
      for (int x = 0; x < Lx; ++x) mech({det(x, y, 0)}, true);  // observable: first-layer boundary flips
    for (int t = 0; t < T; ++t) {
      mech({det(0, 0, t), det(1, 0, t)}, false);
      mech({det(0, 0, t), det(1, 0, t)}, false);  // parallel
      mech({det(0, 1, t), det(1, 1, t)}, false);
      mech({det(0, 0, t), det(0, 1, t)}, false);
      mech({det(1, 0, t), det(1, 1, t)}, false);
      mech({det(1, 1, t)}, false);  // boundary
      if (t + 1 < T)
        for (int y = 0; y < Ly; ++y)
          for (int x = 0; x < Lx; ++x) mech({det(x, y, t), det(x, y, t + 1)}, false);
    }
    std::vector<double> p(nm, 0.05);
    Program P;
    std::string e = build_from_dem(nd, nm, int64_t(di.size()), di.data(), mi.data(), p.data(), 1, obs.data(),
                                   coord.data(), P);
    expect(e.empty(), "DEM builds: " + e);
    if (e.empty()) check_program(P, "DEM 2x2x3");
    // a mechanism two layers apart
    di.push_back(det(0, 0, 0));
    mi.push_back(nm);
    di.push_back(det(0, 0, 2));
    mi.push_back(nm);
    std::vector<double> p2(nm + 1, 0.05);
    std::vector<uint8_t> obs2 = obs;
    obs2.push_back(0);
    e = build_from_dem(nd, nm + 1, int64_t(di.size()), di.data(), mi.data(), p2.data(), 1, obs2.data(),
                       coord.data(), P);
    expect(e.rfind("UNSUPPORTED", 0) == 0, "DEM: non-adjacent mechanism refused");
    std::vector<int32_t> bad_idx = {0, nd};
    std::vector<int32_t> bad_m = {0, 0};
    e = build_from_dem(nd, nm, 2, bad_idx.data(), bad_m.data(), p.data(), 1, obs.data(), coord.data(), P);
    expect(!e.empty(), "DEM: detector index out of range refused");
  }
  {
    // generic layered networks: a 3 x 2 grid, product states of two cosets,
    // one layer with a syndrome-dependent op before the gates, dense gates of
    // known operator-Schmidt rank on every bond (rank 1, 2 and 4), an op after
    // them; then invalid descriptions
    const int lx = 3, ly = 2, ns = lx * ly;
    std::vector<double> vals;
    auto put = [&](const std::vector<double>& v) {
      int64_t off = int64_t(vals.size());
      vals.insert(vals.end(), v.begin(), v.end());
      return off;
    };
    std::vector<int32_t> dims(size_t(2) * ns * 5, 1);
    std::vector<int64_t> ioff(size_t(2) * ns);
    for (int c = 0; c < 2; ++c)
      for (int s = 0; s < ns; ++s) {
        dims[(size_t(c) * ns + s) * 5] = 2;
        ioff[size_t(c) * ns + s] = put({0.3 + 0.1 * s, 0.7 - 0.05 * c});
      }
    std::vector<LayerOp> ops;
    ops.push_back({0, OP_PRE, 0, 0, 2, 3, 0, 0, put({1, 0, 0, 1, 1, 1}), put({0, 1, 1, 0, 1, 1})});
    // gates: sums of `rank` products of functions of distinct frequencies
    // (operator-Schmidt rank 1, 2 and 4)
    auto gate = [&](int da, int db, int rank) {
      std::vector<double> g(size_t(da) * db * da * db, 0.0);
      for (int a2 = 0; a2 < da; ++a2)
        for (int b2 = 0; b2 < db; ++b2)
          for (int a = 0; a < da; ++a)
            for (int b = 0; b < db; ++b) {
              double v = 0.0;
              for (int k = 0; k < rank; ++k)
                v += std::cos((k + 1) * (0.7 * (a2 * da + a) + 0.3)) * std::sin((k + 1) * (0.45 * (b2 * db + b) + 0.2) + k);
              g[((size_t(a2) * db + b2) * da + a) * db + b] = v;
            }
      return g;
    };
    ops.push_back({0, OP_GATE_H, 0, 0, 3, 2, -1, 0, put(gate(3, 2, 1)), 0});
    ops.push_back({0, OP_GATE_H, 1, 1, 2, 2, 1, 0, put(gate(2, 2, 2)), put(gate(2, 2, 4))});
    ops.push_back({0, OP_GATE_V, 2, 0, 2, 2, -1, 0, put(gate(2, 2, 4)), 0});
    ops.push_back({0, OP_POST, 0, 0, 3, 2, -1, 0, put({1, 1, 0, 0, 1, 1}), 0});
    std::vector<int64_t> foff(ns);
    for (int s = 0; s < ns; ++s) foff[s] = put({1.0, 0.5});
    Program P;
    std::string e = build_from_layers(lx, ly, 1, 2, 2, dims.data(), ioff.data(), int32_t(ops.size()), ops.data(),
                                      foff.data(), vals.data(), int64_t(vals.size()), 1e-12, P);
    expect(e.empty(), "layers: valid description built (" + e + ")");
    if (e.empty()) {
      check_program(P, "layers");
      int k1 = -1, k2 = -1, k4 = -1;
      for (const auto& g : P.gates) {
        if (g.dA == 3) k1 = g.K;
        else if (g.det >= 0) k2 = g.K;
        else k4 = g.K;
      }
      expect(k1 == 1, "layers: a rank-1 gate splits into one term");
      expect(k2 == 4, "layers: a syndrome-dependent gate takes the larger term count of its two sets");
      expect(k4 == 4, "layers: a rank-4 gate splits into four terms");
    }
    auto bad = [&](std::vector<LayerOp> o, int nl, const char* what) {
      Program Q;
      std::string e2 = build_from_layers(lx, ly, nl, 2, 2, dims.data(), ioff.data(), int32_t(o.size()), o.data(),
                                         foff.data(), vals.data(), int64_t(vals.size()), 1e-12, Q);
      expect(!e2.empty(), std::string("layers: refused ") + what);
    };
    auto o = ops;
    o[1].x = 2;
    bad(o, 1, "a gate reaching outside the grid");
    o = ops;
    o[1].off0 = int64_t(vals.size()) - 2;
    bad(o, 1, "a gate outside values");
    o = ops;
    o[0].det = 7;
    bad(o, 1, "a detector index out of range");
    o = ops;
    o.push_back(ops[3]);
    bad(o, 1, "two gates on one bond");
    o = ops;
    o[1].d_in = 2;
    bad(o, 1, "gate dims that differ from the sites'");
    bad(ops, 0, "zero layers");
    o = ops;
    o[2].layer = 1;
    bad(o, 1, "an op beyond the last layer");
  }
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("builder checks passed\n");
  return 0;
}
