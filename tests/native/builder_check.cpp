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
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("builder checks passed\n");
  return 0;
}
