// C-ABI of the tn3d library: contexts, networks, batched contraction and
// decoding.  See include/tn3d.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tn3d.h"
#include "program.h"
#include "sweep.h"

using namespace tn3d;

// Workspace of tn3d_contract_cosets_noalloc: a fixed device array, one copy
// per GPU the library runs on, held until the process ends.  Host code never
// uses its name as an address: each device's address comes from
// hipGetSymbolAddress, taken once per device when a context is created on it.
constexpr size_t NOALLOC_BYTES = size_t(256) << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;  // device -> address of scratch there

// A captured per-chunk launch sequence is valid for one network, parameter
// set, chunk shape, timing mode and workspace allocation.
struct GraphKey {
  uint64_t net;
  int prec, chi, chi_mps;
  uint32_t flags;  // params.flags: the factorisation route sets the workspace layout
  double eps, tau;
  int ni;
  int64_t chunk;
  int timing;
  char* ws;
  size_t ws_bytes;
  std::vector<int32_t> sched;  // chi-schedule (empty: constant chi)
  int tune;                    // launch-shape choice (LaunchTuning, packed)
  bool operator<(const GraphKey& o) const {
    return std::tie(net, prec, chi, chi_mps, flags, eps, tau, ni, chunk, timing, ws, ws_bytes, sched, tune) <
           std::tie(o.net, o.prec, o.chi, o.chi_mps, o.flags, o.eps, o.tau, o.ni, o.chunk, o.timing, o.ws,
                    o.ws_bytes, o.sched, o.tune);
  }
};

// The autotuner's cache key: a network under one precision, chi and chi_mps.
struct TuneKey {
  uint64_t net;
  int prec, chi, chi_mps;
  bool operator<(const TuneKey& o) const {
    return std::tie(net, prec, chi, chi_mps) < std::tie(o.net, o.prec, o.chi, o.chi_mps);
  }
};

int pack_tuning(const LaunchTuning& T) { return T.team | (T.mid << 1) | (T.narrow << 8); }

// Rank-rule cap of absorbed layer li under the parameters' chi-schedule.
int32_t layer_chi(const tn3d_params& pr, size_t li) {
  if (pr.n_chi_layers <= 0) return pr.chi;
  const int k = int(std::min<size_t>(li, size_t(pr.n_chi_layers - 1)));
  return std::min(pr.chi, pr.chi_layers[k]);
}

struct GraphEntry {
  hipGraphExec_t exec;
  double hot_l;  // Gram + reabsorption launches in it
};

struct tn3d_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int timing = 0;                  // 1: kernel times, 2: also bond statistics
  int wclk_khz = 100000;           // device wall-clock rate
  double timing_out[15] = {};  // launch counts (3, 6, 10, 13) and sweeps (14) kept on the host
  double* tacc = nullptr;          // device sums of the times, bytes and flops since timing was set
  double stats_out[6] = {0, 0, 0, 0, 0, 0};
  int nb_last = 0;
  int last_resweeps = 0;           // items the last decode re-swept in FP64
  char* aux = nullptr;             // decode scratch
  size_t aux_bytes = 0;
  char* gaux = nullptr;            // gradient scratch
  size_t gaux_bytes = 0;
  char* scratch = nullptr;         // this device's copy of the static scratch array
  bool graphs = true;              // replay captured launch sequences
  std::map<TuneKey, LaunchTuning> tune;  // launch shapes chosen by tn3d_autotune
  std::vector<tn3d_net> nets;             // live networks built on this context
  hipStream_t cap_stream = nullptr;  // private stream the sequences are captured on
  uint64_t next_serial = 1;
  std::map<GraphKey, GraphEntry> gcache;
};

struct tn3d_net_s {
  tn3d_ctx ctx = nullptr;
  uint64_t serial = 0;  // identifies the network in the context's graph cache
  Program P;
  char* dev = nullptr;  // one allocation holding every device array below
  DevOneSite* d_ones = nullptr;
  DevGate* d_gates = nullptr;
  double* d_pool = nullptr;
  int32_t *d_leg_bond = nullptr, *d_init_dims = nullptr, *d_init_off = nullptr, *d_bond_dim0 = nullptr;
  int32_t *d_d_after = nullptr, *d_par_after = nullptr, *d_d_final = nullptr, *d_f_off = nullptr;
  uint64_t* d_ext = nullptr;  // derived-bit rows (Program::ext_rows), or null
  int max_gates_class = 0;
  uint64_t tune_serial = 0;  // launch shapes come from the autotuner's entry of this network
  // the builder call that made P (gauge rounds included), for networks at
  // other rates (gradients); build_plain without the gauge rounds
  std::function<std::string(const double*, Program&)> rebuild, build_plain;
  int gauge_rounds = 0;
  std::vector<double> rates;  // the builder's rate array (P.n_mech entries)
  // tn3d_grad_loglik: per mechanism i, this network with rate i at var_c[i],
  // as pool copy var_slot[i] of d_pool_all (copy 0 is this network's pool)
  // when the structure is the same, else as a network of its own variants[i]
  std::vector<double> var_c;
  std::vector<int32_t> var_slot;
  std::vector<tn3d_net> variants;
  double* d_pool_all = nullptr;
};

namespace {

tn3d_status fail(tn3d_ctx c, tn3d_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, TN3D_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Carves aligned sub-buffers out of one allocation.
struct Carver {
  size_t off = 0;
  template <typename T>
  size_t take(size_t n) {
    size_t o = align256(off);
    off = o + n * sizeof(T);
    return o;
  }
};

tn3d_status upload_net(tn3d_net n) {
  tn3d_ctx c = n->ctx;
  Program& P = n->P;
  Carver cv;
  size_t o_ones = cv.take<DevOneSite>(std::max<size_t>(1, P.ones.size()));
  size_t o_gates = cv.take<DevGate>(std::max<size_t>(1, P.gates.size()));
  size_t o_pool = cv.take<double>(P.pool.size());
  size_t o_leg = cv.take<int32_t>(P.leg_bond.size());
  size_t o_idims = cv.take<int32_t>(P.init_dims.size());
  size_t o_ioff = cv.take<int32_t>(P.init_off.size());
  size_t o_bd0 = cv.take<int32_t>(std::max<size_t>(1, P.bond_dim0.size()));
  size_t o_dafter = cv.take<int32_t>(P.d_after.size());
  size_t o_pafter = cv.take<int32_t>(P.par_after.size());
  size_t o_dfin = cv.take<int32_t>(P.d_final.size());
  size_t o_foff = cv.take<int32_t>(P.f_off.size());
  size_t o_ext = cv.take<uint64_t>(std::max<size_t>(1, P.ext_rows.size()));
  if (P.n_ext > 0 && (P.ext_words > EXT_MAXW || P.ext_words * 64 < P.ext_src_n ||
                      P.ext_rows.size() != size_t(P.n_ext) * P.ext_words || P.ext_src0 + P.ext_src_n > P.n_det))
    return fail(c, TN3D_E_UNSUPPORTED, "derived-bit map too large or inconsistent");
  HIPCHK(c, hipSetDevice(c->device));
  if (hipMalloc(&n->dev, cv.off) != hipSuccess) return fail(c, TN3D_E_OOM, "device allocation of the network");
  auto put = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpy(n->dev + off, src, bytes, hipMemcpyHostToDevice);
  };
  HIPCHK(c, put(o_ones, P.ones.data(), P.ones.size() * sizeof(DevOneSite)));
  HIPCHK(c, put(o_gates, P.gates.data(), P.gates.size() * sizeof(DevGate)));
  HIPCHK(c, put(o_pool, P.pool.data(), P.pool.size() * 8));
  HIPCHK(c, put(o_leg, P.leg_bond.data(), P.leg_bond.size() * 4));
  HIPCHK(c, put(o_idims, P.init_dims.data(), P.init_dims.size() * 4));
  HIPCHK(c, put(o_ioff, P.init_off.data(), P.init_off.size() * 4));
  HIPCHK(c, put(o_bd0, P.bond_dim0.data(), P.bond_dim0.size() * 4));
  HIPCHK(c, put(o_dafter, P.d_after.data(), P.d_after.size() * 4));
  HIPCHK(c, put(o_pafter, P.par_after.data(), P.par_after.size() * 4));
  HIPCHK(c, put(o_dfin, P.d_final.data(), P.d_final.size() * 4));
  HIPCHK(c, put(o_foff, P.f_off.data(), P.f_off.size() * 4));
  HIPCHK(c, put(o_ext, P.ext_rows.data(), P.ext_rows.size() * 8));
  n->d_ones = reinterpret_cast<DevOneSite*>(n->dev + o_ones);
  n->d_gates = reinterpret_cast<DevGate*>(n->dev + o_gates);
  n->d_pool = reinterpret_cast<double*>(n->dev + o_pool);
  n->d_leg_bond = reinterpret_cast<int32_t*>(n->dev + o_leg);
  n->d_init_dims = reinterpret_cast<int32_t*>(n->dev + o_idims);
  n->d_init_off = reinterpret_cast<int32_t*>(n->dev + o_ioff);
  n->d_bond_dim0 = reinterpret_cast<int32_t*>(n->dev + o_bd0);
  n->d_d_after = reinterpret_cast<int32_t*>(n->dev + o_dafter);
  n->d_par_after = reinterpret_cast<int32_t*>(n->dev + o_pafter);
  n->d_d_final = reinterpret_cast<int32_t*>(n->dev + o_dfin);
  n->d_f_off = reinterpret_cast<int32_t*>(n->dev + o_foff);
  n->d_ext = P.n_ext > 0 ? reinterpret_cast<uint64_t*>(n->dev + o_ext) : nullptr;
  n->max_gates_class = 0;
  for (auto& L : P.layers)
    for (int k = 0; k < 4; ++k) n->max_gates_class = std::max(n->max_gates_class, L.gate1[k] - L.gate0[k]);
  return TN3D_OK;
}

tn3d_status make_net(tn3d_ctx c, const std::string& err, Program&& P, tn3d_net* out) {
  if (!err.empty()) return fail(c, TN3D_E_INVALID, err);
  tn3d_net n = new (std::nothrow) tn3d_net_s;
  if (!n) return fail(c, TN3D_E_OOM, "host allocation");
  n->ctx = c;
  n->serial = c->next_serial++;
  n->tune_serial = n->serial;
  n->P = std::move(P);
  tn3d_status s = upload_net(n);
  if (s != TN3D_OK) {
    if (n->dev) (void)hipFree(n->dev);
    delete n;
    return s;
  }
  c->nets.push_back(n);
  *out = n;
  return TN3D_OK;
}

// Builds a network with f at rates p and keeps f and the rates, so that the
// gradient can build the same network at other rates.
tn3d_status build_net(tn3d_ctx c, std::function<std::string(const double*, Program&)> f, const double* p,
                      tn3d_net* out) {
  Program P;
  std::string e = f(p, P);
  tn3d_status s = make_net(c, e, std::move(P), out);
  if (s == TN3D_OK) {
    (*out)->rebuild = f;
    (*out)->build_plain = std::move(f);
    (*out)->rates.assign(p, p + (*out)->P.n_mech);
  }
  return s;
}

// Sizes of every per-sweep array for one network at given chi / chi_m.
struct Layout {
  int legcap, ncap, kdcap, mcap_chi;
  int64_t sbig = 0;  // doubles per (sweep, gate) of the order-above-64 truncation scratch
  std::vector<int64_t> site_off, fin_off;
  int64_t sweep_stride = 0, fin_stride = 0;
  // the final tensors (FP64, without the physical leg) fit in the site slots
  // of the parity the last layer left free, and are written there
  bool fin_alias = false;
  int64_t mcap = 0, kcap = 0, bigcap = 0, jcap = 0;
  int eig_ys = 1;
  size_t per_sweep_bytes = 0;
};

Layout make_layout(const Program& P, int chi, int chi_m, int prec, int max_g) {
  Layout L;
  L.legcap = std::max(chi, 2);
  int ns = P.Lx * P.Ly;
  L.site_off.resize(ns);
  L.fin_off.resize(ns);
  int dm = 1;
  for (int s = 0; s < ns; ++s) {
    int64_t cap = P.dmax[s], fcap = 1;
    for (int l = 0; l < 4; ++l)
      if (P.leg_bond[s * 4 + l] >= 0) {
        cap *= L.legcap;
        fcap *= L.legcap;
      }
    L.site_off[s] = L.sweep_stride;
    L.sweep_stride += (cap + 63) & ~int64_t(63);
    L.fin_off[s] = L.fin_stride;
    L.fin_stride += (fcap + 63) & ~int64_t(63);
    dm = std::max(dm, P.dmax[s]);
  }
  L.ncap = std::max(P.max_dgate, 1) * L.legcap;
  L.kdcap = std::max(P.max_K, 1) * L.legcap;
  const int cm = chi_m;
  L.mcap = int64_t(cm) * L.legcap * cm;
  L.kcap = int64_t(cm) * cm * L.legcap;
  L.bigcap = int64_t(cm) * L.legcap * int64_t(cm) * L.legcap;
  // FP32 boundary MPS: eigenvectors of families of up to 64 vectors in LDS
  // with row stride eig_ys, and the inverse-iteration factors per vector
  L.eig_ys = std::min(cm, 64) | 1;  // odd: conflict-free row and column access
  L.jcap = std::max<int64_t>(L.bigcap, int64_t(4) * std::min<int64_t>(64, int64_t(cm) * L.legcap) * L.eig_ys);
  // the subspace iteration of large families: four blocks of 64 vectors
  L.jcap = std::max<int64_t>(L.jcap, int64_t(4) * 64 * cm * L.legcap);
  const size_t esz = prec == TN3D_PREC_FP64 ? 8 : 4;
  L.fin_alias = true;
  for (int s = 0; s < ns; ++s)
    if (size_t(P.dmax[s]) * esz < 8) L.fin_alias = false;
  size_t b = 0;
  b += 2 * L.sweep_stride * esz;
  b += P.n_bonds * (4 + 8 + 8 * size_t(L.legcap)) + P.Lx * P.Ly * 8 + 4;
  b += size_t(max_g) * 2 * (2 * L.ncap * L.ncap + 2) * 8 + size_t(max_g) * 4;
  L.sbig = L.kdcap > 64 ? int64_t(L.kdcap) * L.kdcap : 0;
  b += size_t(max_g) * L.sbig * 8;
  if (!L.fin_alias) b += L.fin_stride * 8;
  b += size_t(2) * P.Lx * L.mcap * 8 + size_t(2) * P.Lx * 3 * 4 + L.kcap * 8 + 3 * 4 + 3 * L.bigcap * 8 + L.jcap * 8 + 8 + 4 + 12 * 4 + 1024 * 8;
  L.per_sweep_bytes = b + 64 * 20;
  return L;
}

__global__ void k_iota(int32_t* out, int n, int base) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = base + i;
}

// Destroys the cached graphs of one network (net != 0) or all of them.
void drop_graphs(tn3d_ctx c, uint64_t net) {
  for (auto it = c->gcache.begin(); it != c->gcache.end();) {
    if (net == 0 || it->first.net == net) {
      (void)hipGraphExecDestroy(it->second.exec);
      it = c->gcache.erase(it);
    } else {
      ++it;
    }
  }
}

tn3d_status ensure_ws(tn3d_ctx c, size_t bytes) {
  if (c->ws_bytes >= bytes) return TN3D_OK;
  if (c->ws) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c, 0);
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (hipMalloc(&c->ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, TN3D_E_OOM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->ws_bytes = bytes;
  return TN3D_OK;
}

// Contracts items[0..n_items) (global item indices, all using net `n`).
// noalloc: the workspace is the device's static scratch array (no device
// allocation, eager launches: graph instantiation allocates).
// pools: null, or copies of the network's pool of equal layout (the same
// network at other rates) with the copy each global item reads; then the
// launches are eager.
struct PoolSel {
  const double* pool;   // device, copies of stride doubles
  int64_t stride;
  const int32_t* psel;  // device, per global item
};

tn3d_status run_group(tn3d_ctx c, tn3d_net n, const std::vector<int32_t>& items, const uint8_t* synd,
                      const int64_t* synd_off, const tn3d_params& pr, double* logp, uint32_t* flags_out,
                      int prec, bool noalloc, const PoolSel* pools = nullptr) {
  if (items.empty()) return TN3D_OK;  // (the chunk arithmetic below divides by the item count)
  const Program& P = n->P;
  const int nc = P.n_cosets;
  const int max_g = std::max(1, n->max_gates_class);
  Layout L = make_layout(P, pr.chi, pr.chi_mps, prec, max_g);
  LaunchTuning TU;
  {
    auto it = c->tune.find(TuneKey{n->tune_serial, prec, pr.chi, pr.chi_mps});
    if (it != c->tune.end()) TU = it->second;
  }
  // the kernels' fixed-size LDS arrays bound these (sweep.hip)
  if (L.ncap > 96) return fail(c, TN3D_E_UNSUPPORTED, "physical dim x chi above 96 on a gated site");
  if (L.kdcap > 72) return fail(c, TN3D_E_UNSUPPORTED, "gate rank x chi above 72");
  for (int32_t b : P.bond_dim0)
    if (b > L.legcap) return fail(c, TN3D_E_UNSUPPORTED, "an initial bond dimension above max(chi, 2)");
  // the one-site and final-vector kernels hold a row of a site tensor in 16 registers
  for (int32_t dm : P.dmax)
    if (dm > 16) return fail(c, TN3D_E_UNSUPPORTED, "a physical dimension above 16");
  if ((L.ncap > 64 || L.kdcap > 64) && prec == TN3D_PREC_FP64 && !(pr.flags & TN3D_OPT_GRAM_FACTOR))
    return fail(c, TN3D_E_UNSUPPORTED,
                "physical dim x chi or gate rank x chi above 64 needs the Gram route in FP64 (TN3D_OPT_GRAM_FACTOR)");
  if (int64_t(pr.chi_mps) * L.legcap > 1024) return fail(c, TN3D_E_UNSUPPORTED, "chi_mps x chi above 1024");
  if (P.Lx * P.Ly > 65535) return fail(c, TN3D_E_UNSUPPORTED, "grid too large");
  size_t budget;
  if (noalloc) {
    budget = NOALLOC_BYTES;
    if (pr.workspace_bytes > 0) budget = std::min(budget, size_t(pr.workspace_bytes));
  } else if (pr.workspace_bytes > 0) {
    budget = size_t(pr.workspace_bytes);
  } else {
    size_t fr = 0, tot = 0;
    HIPCHK(c, hipMemGetInfo(&fr, &tot));
    budget = size_t(0.85 * double(fr + c->ws_bytes));
  }
  const size_t fixed = size_t(items.size()) * 4 + (64 << 10);
  if (budget <= fixed + L.per_sweep_bytes * nc) {
    if (noalloc)
      return fail(c, TN3D_E_OOM, "one item needs " + std::to_string(fixed + L.per_sweep_bytes * nc) +
                                     " bytes of workspace, beyond the " + std::to_string(budget) +
                                     "-byte static scratch of tn3d_contract_cosets_noalloc");
    return fail(c, TN3D_E_OOM, "workspace cap below one item (one item needs " +
                                   std::to_string(fixed + L.per_sweep_bytes * nc) + " bytes)");
  }
  int64_t chunk_items = int64_t((budget - fixed) / (L.per_sweep_bytes * nc));
  chunk_items = std::max<int64_t>(1, std::min<int64_t>(chunk_items, int64_t(items.size())));
  chunk_items = std::min<int64_t>(chunk_items, 65535 / nc);  // grid y dimension
  {
    // as many chunks as the cap needs, of equal size: a ragged last chunk
    // runs the latency-bound kernels at low occupancy, and a chunk a little
    // above a multiple of the CU count puts a second wave of the
    // one-workgroup-per-CU kernels behind the first
    const int64_t n_it = int64_t(items.size());
    const int64_t n_chunks = (n_it + chunk_items - 1) / chunk_items;
    chunk_items = (n_it + n_chunks - 1) / n_chunks;
  }
  const int64_t nsw_max = chunk_items * nc;
  // carve the workspace
  Carver cv;
  const size_t esz = prec == TN3D_PREC_FP64 ? 8 : 4;
  size_t o_items = cv.take<int32_t>(chunk_items);
  size_t o_soff = cv.take<int64_t>(L.site_off.size());
  size_t o_foff = cv.take<int64_t>(L.fin_off.size());
  size_t o_buf0 = cv.take<char>(nsw_max * L.sweep_stride * esz);
  size_t o_buf1 = cv.take<char>(nsw_max * L.sweep_stride * esz);
  size_t o_bd = cv.take<int32_t>(nsw_max * P.n_bonds);
  size_t o_lam = cv.take<double>(nsw_max * P.n_bonds * L.legcap);
  size_t o_logb = cv.take<double>(nsw_max * P.n_bonds);
  size_t o_logs = cv.take<double>(nsw_max * P.Lx * P.Ly);
  size_t o_flags = cv.take<uint32_t>(nsw_max);
  size_t o_gram = cv.take<double>(nsw_max * max_g * 2 * L.ncap * L.ncap);
  size_t o_w = cv.take<double>(nsw_max * max_g * 2 * (2 + L.ncap * L.ncap));
  size_t o_gn = cv.take<int32_t>(nsw_max * max_g);
  size_t o_sbig = cv.take<double>(std::max<int64_t>(1, nsw_max * max_g * L.sbig));
  size_t o_fin = cv.take<double>(L.fin_alias ? 1 : nsw_max * L.fin_stride);
  size_t o_mps0 = cv.take<double>(nsw_max * P.Lx * L.mcap);
  size_t o_mps1 = cv.take<double>(nsw_max * P.Lx * L.mcap);
  size_t o_mdim = cv.take<int32_t>(nsw_max * 2 * P.Lx * 3);
  size_t o_K = cv.take<double>(nsw_max * L.kcap);
  size_t o_kdim = cv.take<int32_t>(nsw_max * 3);
  size_t o_L4 = cv.take<double>(nsw_max * L.bigcap);
  size_t o_Th = cv.take<double>(nsw_max * L.bigcap);
  size_t o_Jm = cv.take<double>(nsw_max * L.jcap);
  // FP64 factors every truncation orthogonally (Householder QR of the gate
  // sides, one-sided Jacobi on the boundary-MPS families) unless the caller
  // asks for the Gram route; the reduced precisions and that option factor
  // through Grams (the boundary MPS only where the rank rule never needs
  // singular values below 1e-8 of the largest)
  const bool f64_orth = prec == TN3D_PREC_FP64 && !(pr.flags & TN3D_OPT_GRAM_FACTOR);
  const bool gram_path = !f64_orth && (prec != TN3D_PREC_FP64 || pr.eps_rel >= 1e-8);
  size_t o_Gm = cv.take<double>(gram_path ? nsw_max * L.bigcap : 1);
  size_t o_zdim = cv.take<int32_t>(nsw_max * 12);
  size_t o_zS = cv.take<double>(nsw_max * 1024);
  size_t o_logm = cv.take<double>(nsw_max);
  size_t o_zfl = cv.take<uint32_t>(nsw_max);
  // 64 byte counters (spread to keep atomics uncontended), then the sweep maxima
  // 64 byte counters, the sweep maxima, 64 flop counters (spread to keep atomics uncontended)
  size_t o_ctr = cv.take<unsigned long long>(257);
  // timing: stamps 0 start, 1 after the layers, 2 end; execution windows of
  // the Gram and reabsorption launches of each gate class (2 per class) and
  // of the decomposition launch of each boundary-MPS step
  const size_t n_stamp = 3;
  size_t o_stamp = cv.take<unsigned long long>(n_stamp);
  const int n_cls_win = int(P.layers.size()) * 4 * 2;
  const int n_win = n_cls_win + 3 * P.Lx * P.Ly;
  size_t o_win = cv.take<unsigned long long>(size_t(n_win) * 128);
  size_t o_gitems = cv.take<int32_t>(chunk_items);
  size_t o_gsoff = cv.take<int64_t>(chunk_items);
  // per-item bits: the syndrome, then the bits derived from it
  const int64_t bstride = std::max(1, P.n_det + P.n_ext);
  size_t o_gsynd = cv.take<uint8_t>(chunk_items * bstride);
  size_t o_glp = cv.take<double>(chunk_items * 4);
  size_t o_gfl = cv.take<uint32_t>(chunk_items);
  size_t o_gpsel = cv.take<int32_t>(pools ? chunk_items : 1);
  char* ws = nullptr;
  if (noalloc) {
    if (!c->scratch || cv.off > NOALLOC_BYTES) return fail(c, TN3D_E_OOM, "static scratch unavailable or too small");
    ws = c->scratch;
  } else {
    tn3d_status st = ensure_ws(c, cv.off);
    if (st != TN3D_OK) return st;
    ws = c->ws;
  }
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(ws + o_soff, L.site_off.data(), L.site_off.size() * 8, hipMemcpyHostToDevice, s));
  if (L.fin_alias) {
    // site s's final tensor goes to its slot of the parity the last layer
    // left free (a slot holds dmax[s] >= 8 / esz times the final tensor's
    // elements): offsets in doubles from buf0, 8-byte aligned since slots
    // and sweeps start at multiples of 64 elements
    const int ns = P.Lx * P.Ly;
    const int32_t* pf = P.par_after.data() + (P.layers.size() - 1) * size_t(ns);
    for (int si = 0; si < ns; ++si)
      L.fin_off[si] = (int64_t(pf[si] ? 0 : o_buf1 - o_buf0) + L.site_off[si] * int64_t(esz)) / 8;
    L.fin_stride = L.sweep_stride * int64_t(esz) / 8;
  }
  HIPCHK(c, hipMemcpyAsync(ws + o_foff, L.fin_off.data(), L.fin_off.size() * 8, hipMemcpyHostToDevice, s));
  bool contiguous = true;
  for (size_t i = 1; i < items.size(); ++i)
    if (items[i] != items[0] + int32_t(i)) contiguous = false;

  const int timing = c->timing;
  double hot_launches = 0, eig_launches = 0, zip_launches = 0, bsub_launches = 0, bsub_sweeps = 0;
  for (int64_t i0 = 0; i0 < int64_t(items.size()); i0 += chunk_items) {
    const int ni = int(std::min<int64_t>(chunk_items, int64_t(items.size()) - i0));
    int32_t* d_items = reinterpret_cast<int32_t*>(ws + o_items);
    if (contiguous) {
      hipLaunchKernelGGL(k_iota, dim3((ni + 255) / 256), dim3(256), 0, s, d_items, ni, items[0] + int32_t(i0));
    } else {
      HIPCHK(c, hipStreamSynchronize(s));
      HIPCHK(c, hipMemcpy(d_items, items.data() + i0, size_t(ni) * 4, hipMemcpyHostToDevice));
    }
    SweepArgs A{};
    ZipArgs Z{};
    double hot_l = 0;
    // workspace-derived arguments (the same for eager launches and replays)
    A.n_sweeps = ni * nc;
    A.n_sites = P.Lx * P.Ly;
    A.n_bonds = P.n_bonds;
    A.n_cosets = nc;
    A.chi = pr.chi;
    A.chi_cut = pr.chi;
    A.lam_ld = L.legcap;
    A.solve_big = reinterpret_cast<double*>(ws + o_sbig);
    A.sbig_ld = L.sbig;
    A.Lx = P.Lx;
    A.Ly = P.Ly;
    A.sweep_stride = L.sweep_stride;
    A.site_off = reinterpret_cast<int64_t*>(ws + o_soff);
    A.buf0 = ws + o_buf0;
    A.buf1 = ws + o_buf1;
    A.bond_dim = reinterpret_cast<int32_t*>(ws + o_bd);
    A.lam = reinterpret_cast<double*>(ws + o_lam);
    A.logb = reinterpret_cast<double*>(ws + o_logb);
    A.logs = reinterpret_cast<double*>(ws + o_logs);
    A.flags = reinterpret_cast<uint32_t*>(ws + o_flags);
    A.leg_bond = n->d_leg_bond;
    A.pool = pools ? pools->pool : n->d_pool;
    A.pool_stride = pools ? pools->stride : 0;
    A.psel = pools ? pools->psel : nullptr;  // indexed by global item (direct launches)
    A.eps = pr.eps_rel;
    A.tau = pr.tau_gap;
    A.pchol_tol = prec == TN3D_PREC_FP64 ? 1e-15 : 1e-14;
    A.qr = f64_orth ? 1 : 0;
    A.inc0 = P.inc0;
    A.n_inc = P.n_inc;
    A.wht = P.wht;
    A.jtol = prec == TN3D_PREC_FP64 ? 1e-14 : 1e-10;
    A.jfloor = prec == TN3D_PREC_FP64 ? std::min(1e-13, 0.1 * pr.eps_rel) : std::min(1e-8, 0.1 * pr.eps_rel);
    A.bytes_ctr = timing ? reinterpret_cast<unsigned long long*>(ws + o_ctr) : nullptr;
    A.sweeps_max = reinterpret_cast<int32_t*>(ws + o_ctr + 64 * 8);
    A.gate_n = reinterpret_cast<int32_t*>(ws + o_gn);
    // The whole per-chunk sequence; in graph mode it is captured once with the
    // workspace copies of the inputs and outputs and replayed afterwards.
    auto enqueue = [&](const int32_t* items_p, const uint8_t* synd_p, const int64_t* soff_p, double* logp_p,
                       uint32_t* flags_p, hipStream_t st) -> tn3d_status {
    const hipStream_t s = st;
    hot_l = 0;
    Z = ZipArgs{};
    A.synd = synd_p;
    A.synd_off = soff_p;
    A.items = items_p;
    launch_zero_words(reinterpret_cast<uint32_t*>(ws + o_ctr), 514, s);
    double* gram = reinterpret_cast<double*>(ws + o_gram);
    double* wbuf = reinterpret_cast<double*>(ws + o_w);
    unsigned long long* stamp = reinterpret_cast<unsigned long long*>(ws + o_stamp);
    unsigned long long* win = reinterpret_cast<unsigned long long*>(ws + o_win);
    if (timing) {
      launch_win_init(win, n_win, s);
      launch_stamp(stamp + 0, s);
    }
    launch_init(prec, A, n->d_init_dims, n->d_init_off, n->d_bond_dim0, s);
    size_t real_layer = 0;  // the chi-schedule counts the network's layers, not gauge rounds
    int32_t cut = pr.chi;
    for (size_t li = 0; li < P.layers.size(); ++li) {
      const LayerRange& R = P.layers[li];
      if (!R.gauge) cut = layer_chi(pr, real_layer++);
      A.chi_cut = cut;  // gauge rounds keep the cap of the layer before them
      launch_onesite(prec, A, n->d_ones + R.pre0, R.pre1 - R.pre0, s);
      for (int k = 0; k < 4; ++k) {
        const int ng = R.gate1[k] - R.gate0[k];
        if (ng <= 0) continue;
        const DevGate* gp = n->d_gates + R.gate0[k];
        const int cls = int(li) * 4 + k;
        // gates come ordered by physical dim, largest first: the ones whose
        // Gram or reabsorbed rows (d times a bond of at most legcap) can pass
        // a width form a prefix
        auto n_wider = [&](int w) {
          int c = 0;
          while (c < ng && std::max(P.gates[R.gate0[k] + c].dA, P.gates[R.gate0[k] + c].dB) * L.legcap > w) ++c;
          return c;
        };
        A.win = timing ? win + size_t(2 * cls) * 128 : nullptr;
        launch_gram(prec, A, gp, ng, n_wider(16), n_wider(32), n_wider(64), gram, L.ncap, s);
        A.win = nullptr;
        launch_solve(TU, A, gp, ng, gram, wbuf, L.ncap, L.kdcap, s);
        A.win = timing ? win + size_t(2 * cls + 1) * 128 : nullptr;
        launch_reabsorb(TU, prec, A, gp, ng, n_wider(16), n_wider(32), n_wider(64), wbuf, L.ncap, s);
        A.win = nullptr;
        hot_l += 2;
      }
      launch_onesite(prec, A, n->d_ones + R.post0, R.post1 - R.post0, s);
      launch_rescale(prec, A, n->d_d_after + li * A.n_sites, n->d_par_after + li * A.n_sites, s);
    }
    HIPCHK(c, hipGetLastError());
    if (timing) launch_stamp(stamp + 1, s);
    const int32_t* par_final = n->d_par_after + (P.layers.size() - 1) * A.n_sites;
    double* fin = reinterpret_cast<double*>(ws + (L.fin_alias ? o_buf0 : o_fin));
    launch_finalize(prec, A, n->d_d_final, n->d_f_off, par_final, fin, L.fin_stride,
                    reinterpret_cast<int64_t*>(ws + o_foff), s);
    Z.n_sweeps = A.n_sweeps;
    Z.Lx = P.Lx;
    Z.Ly = P.Ly;
    Z.chi_m = pr.chi_mps;
    Z.n_bonds = P.n_bonds;
    Z.fin = fin;
    Z.fin_stride = L.fin_stride;
    Z.fin_off = reinterpret_cast<int64_t*>(ws + o_foff);
    Z.bond_dim = A.bond_dim;
    Z.mps0 = reinterpret_cast<double*>(ws + o_mps0);
    Z.mps1 = reinterpret_cast<double*>(ws + o_mps1);
    Z.mcap = L.mcap;
    Z.mdim = reinterpret_cast<int32_t*>(ws + o_mdim);
    Z.K = reinterpret_cast<double*>(ws + o_K);
    Z.kcap = L.kcap;
    Z.kdim = reinterpret_cast<int32_t*>(ws + o_kdim);
    Z.L4 = reinterpret_cast<double*>(ws + o_L4);
    Z.Th = reinterpret_cast<double*>(ws + o_Th);
    Z.Jm = reinterpret_cast<double*>(ws + o_Jm);
    Z.bigcap = L.bigcap;
    Z.jcap = L.jcap;
    Z.eig_ys = L.eig_ys;
    Z.logm = reinterpret_cast<double*>(ws + o_logm);
    Z.flags = reinterpret_cast<uint32_t*>(ws + o_zfl);
    Z.eps = pr.eps_rel;
    Z.tau = pr.tau_gap;
    Z.jtol = A.jtol;
    Z.jfloor = A.jfloor;
    Z.gram_path = gram_path ? 1 : 0;
    // large boundary-MPS families: residuals of the leading Ritz pairs far
    // below what the precision resolves (FP64) or needs (reduced precisions)
    Z.sub_tol = prec == TN3D_PREC_FP64 ? 1e-12 : 1e-9;
    Z.bf_theta = prec == TN3D_PREC_BF16 ? 1 : 0;
    Z.sweeps_max = A.sweeps_max;
    Z.zdim = reinterpret_cast<int32_t*>(ws + o_zdim);
    Z.zS = reinterpret_cast<double*>(ws + o_zS);
    Z.flop_ctr = timing ? reinterpret_cast<unsigned long long*>(ws + o_ctr + 65 * 8) : nullptr;
    Z.flop_a = timing ? reinterpret_cast<unsigned long long*>(ws + o_ctr + 129 * 8) : nullptr;
    Z.flop_b = timing ? reinterpret_cast<unsigned long long*>(ws + o_ctr + 193 * 8) : nullptr;
    Z.Gm = reinterpret_cast<double*>(ws + o_Gm);
    launch_zip_init(Z, s);
    for (int y = 0; y < P.Ly; ++y)
      for (int x = 0; x < P.Lx; ++x)
      {
        Z.win = timing ? win + size_t(n_cls_win + y * P.Lx + x) * 128 : nullptr;
        Z.win_a = timing ? win + size_t(n_cls_win + P.Lx * P.Ly + y * P.Lx + x) * 128 : nullptr;
        Z.win_b = timing ? win + size_t(n_cls_win + 2 * P.Lx * P.Ly + y * P.Lx + x) * 128 : nullptr;
        launch_zip_step(Z, x, y, L.legcap, s);
      }
    Z.win = nullptr;
    Z.win_a = nullptr;
    Z.win_b = nullptr;
    launch_finish(A, Z, logp_p, flags_p, s);
    if (timing) {
      launch_stamp(stamp + 2, s);
      launch_timing_reduce(stamp, win, n_cls_win, P.Lx, P.Ly, gram_path ? 1 : 0,
                           reinterpret_cast<const unsigned long long*>(ws + o_ctr), 1.0 / double(c->wclk_khz),
                           c->tacc, s);
    }
    HIPCHK(c, hipGetLastError());
    return TN3D_OK;
    };
    bool done = false;
    int32_t* g_items = reinterpret_cast<int32_t*>(ws + o_gitems);
    int64_t* g_soff = reinterpret_cast<int64_t*>(ws + o_gsoff);
    uint8_t* g_synd = reinterpret_cast<uint8_t*>(ws + o_gsynd);
    double* g_lp = reinterpret_cast<double*>(ws + o_glp);
    uint32_t* g_fl = reinterpret_cast<uint32_t*>(ws + o_gfl);
    auto gather_inputs = [&]() {
      launch_gather_synd(ni, d_items, synd, synd_off, P.n_det, bstride, g_synd, s);
      launch_ext_bits(ni, g_synd, bstride, P.n_det, P.ext_src0, P.ext_src_n, P.ext_words, n->d_ext, P.n_ext, s);
    };
    if (c->graphs && !noalloc && !pools) {
      // inputs into the workspace, replay (capturing first if needed), results out
      gather_inputs();
      HIPCHK(c, hipGetLastError());
      const GraphKey key{n->serial, prec, pr.chi, pr.chi_mps, pr.flags, pr.eps_rel, pr.tau_gap, ni, chunk_items, timing,
                         c->ws, c->ws_bytes,
                         std::vector<int32_t>(pr.chi_layers, pr.chi_layers + std::max(0, pr.n_chi_layers)),
                         pack_tuning(TU)};
      auto it = c->gcache.find(key);
      if (it == c->gcache.end()) {
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        tn3d_status es = TN3D_OK;
        // captured on a private stream (the caller's may be the legacy default
        // stream, which cannot be captured); replayed on the caller's
        hipError_t ce = hipSuccess;
        if (!c->cap_stream) ce = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (ce == hipSuccess) ce = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (ce == hipSuccess) {
          launch_seq(ni, g_items, g_soff, bstride, c->cap_stream);
          es = enqueue(g_items, g_synd, g_soff, g_lp, g_fl, c->cap_stream);
          ce = hipStreamEndCapture(c->cap_stream, &gr);
        }
        if (ce == hipSuccess && es == TN3D_OK && gr) ce = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (ce != hipSuccess || es != TN3D_OK || !ex) {
          // capture is not available for this sequence: launch eagerly from now on
          if (std::getenv("TN3D_VERBOSE"))
            std::fprintf(stderr, "tn3d: launch capture failed (%s%s%s); launching eagerly\n",
                         hipGetErrorString(ce), es != TN3D_OK ? "; " : "", es != TN3D_OK ? c->err.c_str() : "");
          (void)hipGetLastError();
          if (ex) (void)hipGraphExecDestroy(ex);
          c->graphs = false;
          c->err.clear();
        } else {
          it = c->gcache.emplace(key, GraphEntry{ex, hot_l}).first;
        }
      }
      if (c->graphs) {
        HIPCHK(c, hipGraphLaunch(it->second.exec, s));
        hot_l = it->second.hot_l;
        launch_scatter_out(ni, d_items, g_lp, g_fl, logp, flags_out, s);
        HIPCHK(c, hipGetLastError());
        done = true;
      }
    }
    if (!done && P.n_ext > 0) {
      // the derived bits live in the workspace copy of the inputs
      gather_inputs();
      if (pools) {
        // the kernels index items locally here: the pool choices follow
        int32_t* g_psel = reinterpret_cast<int32_t*>(ws + o_gpsel);
        launch_gather_i32(ni, d_items, pools->psel, g_psel, s);
        A.psel = g_psel;
      }
      launch_seq(ni, g_items, g_soff, bstride, s);
      tn3d_status es = enqueue(g_items, g_synd, g_soff, g_lp, g_fl, s);
      if (es != TN3D_OK) return es;
      launch_scatter_out(ni, d_items, g_lp, g_fl, logp, flags_out, s);
      HIPCHK(c, hipGetLastError());
    } else if (!done) {
      tn3d_status es = enqueue(d_items, synd, synd_off, logp, flags_out, s);
      if (es != TN3D_OK) return es;
    }
    hot_launches += hot_l;
    // the last row's decompositions are done inside the contraction kernel
    if (timing && gram_path) eig_launches += double(P.Ly - 1) * (P.Lx - 1);
    if (timing) {
      // (from the host's own parameters: replays do not fill Z)
      ZipArgs zq{};
      zq.Lx = P.Lx;
      zq.Ly = P.Ly;
      zq.chi_m = pr.chi_mps;
      zq.gram_path = gram_path ? 1 : 0;
      zip_launches += double(P.Ly) * P.Lx;
      for (int y = 0; y < P.Ly; ++y)
        for (int x = 0; x < P.Lx; ++x)
          if (zip_step_large(zq, x, y, L.legcap) == 1) {
            bsub_launches += 1;
            bsub_sweeps += A.n_sweeps;
          }
    }
    if (timing >= 2) {
      std::vector<int32_t> bd(size_t(A.n_sweeps) * P.n_bonds);
      std::vector<double> lm(size_t(A.n_sweeps) * P.n_bonds * L.legcap);
      HIPCHK(c, hipMemcpy(bd.data(), A.bond_dim, bd.size() * 4, hipMemcpyDeviceToHost));
      HIPCHK(c, hipMemcpy(lm.data(), A.lam, lm.size() * 8, hipMemcpyDeviceToHost));
      for (int sw = 0; sw < A.n_sweeps; ++sw) {
        double mn = 1.0;
        for (int b = 0; b < P.n_bonds; ++b) {
          const int D = bd[size_t(sw) * P.n_bonds + b];
          c->stats_out[0] += D;
          c->stats_out[1] = std::max(c->stats_out[1], double(D));
          mn = std::min(mn, lm[(size_t(sw) * P.n_bonds + b) * L.legcap + D - 1]);
        }
        c->stats_out[3] += mn;
      }
      c->stats_out[2] += A.n_sweeps;
      int32_t smax[2] = {0, 0};
      HIPCHK(c, hipMemcpy(smax, A.sweeps_max, 8, hipMemcpyDeviceToHost));
      c->stats_out[4] = std::max(c->stats_out[4], double(smax[0]));
      c->stats_out[5] = std::max(c->stats_out[5], double(smax[1]));
      c->nb_last = P.n_bonds;
    }
  }
  if (timing) {  // times, bytes and flops are summed on the device (tacc)
    c->timing_out[3] += hot_launches;
    c->timing_out[6] += eig_launches;
    c->timing_out[10] += zip_launches;
    c->timing_out[13] += bsub_launches;
    c->timing_out[14] += bsub_sweeps;
  }
  return TN3D_OK;
}

bool params_ok(const tn3d_params* p, std::string& why) {
  if (!p) {
    why = "null params";
    return false;
  }
  if (p->chi < 1 || p->chi > 64) {
    why = "chi must be in [1, 64]";
    return false;
  }
  if (p->chi_mps < 1 || p->chi_mps > 64) {
    why = "chi_mps must be in [1, 64]";
    return false;
  }
  if (p->precision != TN3D_PREC_FP64 && p->precision != TN3D_PREC_FP32 && p->precision != TN3D_PREC_BF16) {
    why = "unknown precision";
    return false;
  }
  if (!(p->eps_rel >= 0.0 && p->eps_rel < 1.0) || !(p->tau_gap >= 0.0 && p->tau_gap < 1.0)) {
    why = "eps_rel and tau_gap must lie in [0, 1)";
    return false;
  }
  if ((p->flags & ~TN3D_OPT_GRAM_FACTOR) != 0) {
    why = "unknown bit in params.flags";
    return false;
  }
  if (p->n_chi_layers < 0 || p->n_chi_layers > TN3D_MAX_CHI_LAYERS) {
    why = "n_chi_layers must lie in [0, TN3D_MAX_CHI_LAYERS]";
    return false;
  }
  for (int i = 0; i < p->n_chi_layers; ++i)
    if (p->chi_layers[i] < 1 || p->chi_layers[i] > p->chi) {
      why = "chi_layers entries must lie in [1, chi]";
      return false;
    }
  return true;
}

tn3d_status contract_impl(tn3d_ctx c, int32_t batch, const tn3d_net* nets, const uint8_t* synd,
                          const int64_t* offs, const tn3d_params* pr, double* logp, uint32_t* flags,
                          bool noalloc = false) {
  if (!c) return TN3D_E_INVALID;
  c->err.clear();
  std::string why;
  if (!params_ok(pr, why)) return fail(c, TN3D_E_INVALID, why);
  if (batch < 0) return fail(c, TN3D_E_INVALID, "negative batch");
  if (batch == 0) return TN3D_OK;
  if (!nets || !synd || !offs || !logp) return fail(c, TN3D_E_INVALID, "null pointer");
  for (int i = 0; i < batch; ++i)
    if (!nets[i] || nets[i]->ctx != c) return fail(c, TN3D_E_INVALID, "network handle null or of another context");
  HIPCHK(c, hipSetDevice(c->device));
  std::map<tn3d_net, std::vector<int32_t>> groups;
  std::vector<tn3d_net> order;
  for (int i = 0; i < batch; ++i) {
    auto it = groups.find(nets[i]);
    if (it == groups.end()) {
      order.push_back(nets[i]);
      groups[nets[i]] = {};
    }
    groups[nets[i]].push_back(i);
  }
  for (tn3d_net n : order) {
    tn3d_status s = run_group(c, n, groups[n], synd, offs, *pr, logp, flags, pr->precision, noalloc);
    if (s != TN3D_OK) return s;
  }
  return TN3D_OK;
}

}  // namespace

extern "C" {

void tn3d_params_default(tn3d_params* p, int32_t chi, int32_t chi_mps, int32_t precision) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->chi = chi;
  p->chi_mps = chi_mps;
  p->precision = precision;
  const bool f64 = precision == TN3D_PREC_FP64;
  // the smallest kept singular value must carry rounding well below the gap
  // that decides a cut: about 1e-7 relative at 1e-9 of the largest in FP64
  p->eps_rel = f64 ? 1e-9 : 1e-6;
  // reduced precisions: a cut only at a gap of a percent, where the kept
  // subspace moves by about eps_32 / 1e-2 with the FP32 rounding of the sites
  p->tau_gap = f64 ? 1e-6 : 1e-2;
  p->near_tie = 4e-3;
  p->workspace_bytes = 0;
}

tn3d_status tn3d_ctx_create(int32_t device, void* stream, tn3d_ctx* out) {
  if (!out) return TN3D_E_INVALID;
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) return TN3D_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return TN3D_E_DEVICE;
  tn3d_ctx c = new (std::nothrow) tn3d_ctx_s;
  if (!c) return TN3D_E_OOM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  bool ok = set_kernel_lds_limits() == hipSuccess;
  int rate = 0;
  ok = ok && hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0;
  if (!ok) {
    (void)hipGetLastError();
    delete c;
    return TN3D_E_DEVICE;
  }
  c->wclk_khz = rate;
  {
    // this device's address of the static scratch array, taken once per device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        delete c;
        return TN3D_E_DEVICE;
      }
      it = g_scratch_ptr.emplace(device, static_cast<char*>(ptr)).first;
    }
    c->scratch = it->second;
  }
  if (hipMalloc(&c->tacc, 12 * sizeof(double)) != hipSuccess || hipMemset(c->tacc, 0, 12 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    if (c->tacc) (void)hipFree(c->tacc);
    delete c;
    return TN3D_E_DEVICE;
  }
  *out = c;
  return TN3D_OK;
}

void tn3d_ctx_destroy(tn3d_ctx c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  // networks the caller did not destroy first: free their device arrays now
  // and detach them, so that a later tn3d_net_destroy only frees the handle
  if (!c->nets.empty()) (void)hipStreamSynchronize(c->stream);
  for (tn3d_net n : c->nets) {
    if (n->dev) (void)hipFree(n->dev);
    if (n->d_pool_all) (void)hipFree(n->d_pool_all);
    n->dev = nullptr;
    n->d_pool_all = nullptr;
    n->ctx = nullptr;
  }
  c->nets.clear();
  if (c->ws) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ws);
  }
  if (c->aux) (void)hipFree(c->aux);
  if (c->gaux) (void)hipFree(c->gaux);
  if (c->tacc) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->tacc);
  }
  drop_graphs(c, 0);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

const char* tn3d_last_error(tn3d_ctx c) { return c ? c->err.c_str() : "null context"; }

tn3d_status tn3d_net_surface3d_point(tn3d_ctx c, int32_t L, const double* p, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  return build_net(c, [L](const double* q, Program& P) { return build_surface3d_point(L, q, P); }, p, out);
}

tn3d_status tn3d_net_rotated_phenom(tn3d_ctx c, int32_t d, int32_t T, const double* p, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  return build_net(c, [d, T](const double* q, Program& P) { return build_rotated_phenom(d, T, q, P); }, p, out);
}

tn3d_status tn3d_net_surface3d_depolarizing(tn3d_ctx c, int32_t L, const double* p, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  return build_net(c, [L](const double* q, Program& P) { return build_surface3d_depol(L, q, P); }, p, out);
}

tn3d_status tn3d_net_surface3d_loop(tn3d_ctx c, int32_t L, const double* p, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  return build_net(c, [L](const double* q, Program& P) { return build_surface3d_loop(L, q, P); }, p, out);
}

tn3d_status tn3d_net_surface3d_wht(tn3d_ctx c, int32_t L, int32_t sector, const double* p, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  if (sector != TN3D_SECTOR_POINT && sector != TN3D_SECTOR_LOOP) return fail(c, TN3D_E_INVALID, "unknown sector");
  return build_net(c,
                   [L, sector](const double* q, Program& P) {
                     return sector == TN3D_SECTOR_POINT ? build_surface3d_point(L, q, P, true)
                                                        : build_surface3d_loop(L, q, P, true);
                   },
                   p, out);
}

tn3d_status tn3d_net_from_dem(tn3d_ctx c, int32_t n_det, int32_t n_mech, int64_t nnz, const int32_t* det_idx,
                              const int32_t* mech_idx, const double* p_mech, int32_t n_obs, const uint8_t* obs,
                              const int32_t* det_coord, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  Program P;
  std::string e = build_from_dem(n_det, n_mech, nnz, det_idx, mech_idx, p_mech, n_obs, obs, det_coord, P);
  if (e.rfind("UNSUPPORTED: ", 0) == 0) return fail(c, TN3D_E_UNSUPPORTED, e.substr(13));
  // the builder has checked the arrays: keep copies for rebuilds at other rates
  std::vector<int32_t> di(det_idx, det_idx + nnz), mi(mech_idx, mech_idx + nnz), dc;
  std::vector<uint8_t> ob(obs, obs + int64_t(n_obs) * n_mech);
  if (det_coord) dc.assign(det_coord, det_coord + int64_t(n_det) * 3);
  auto f = [n_det, n_mech, nnz, n_obs, di, mi, ob, dc](const double* q, Program& Q) {
    return build_from_dem(n_det, n_mech, nnz, di.data(), mi.data(), q, n_obs, ob.data(),
                          dc.empty() ? nullptr : dc.data(), Q);
  };
  tn3d_status s = make_net(c, e, std::move(P), out);
  if (s == TN3D_OK) {
    (*out)->rebuild = f;
    (*out)->build_plain = f;
    (*out)->rates.assign(p_mech, p_mech + n_mech);
  }
  return s;
}

tn3d_status tn3d_net_from_layers(tn3d_ctx c, int32_t lx, int32_t ly, int32_t n_layers, int32_t n_det,
                                 int32_t n_cosets, const int32_t* init_dims, const int64_t* init_off, int32_t n_ops,
                                 const tn3d_layer_op* ops, const int64_t* final_off, const double* values,
                                 int64_t n_values, double split_tol, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  static_assert(sizeof(tn3d_layer_op) == sizeof(LayerOp), "tn3d_layer_op and LayerOp must match");
  Program P;
  std::string e = build_from_layers(lx, ly, n_layers, n_det, n_cosets, init_dims, init_off, n_ops,
                                    reinterpret_cast<const LayerOp*>(ops), final_off, values, n_values, split_tol, P);
  tn3d_status s = make_net(c, e, std::move(P), out);
  if (s == TN3D_OK) {
    // the builder has checked the arrays: copies for rebuilds with gauge rounds
    const int64_t nc = n_cosets, ns = int64_t(lx) * ly;
    std::vector<int32_t> dv(init_dims, init_dims + nc * ns * 5);
    std::vector<int64_t> iv(init_off, init_off + nc * ns), fv(final_off, final_off + ns);
    std::vector<LayerOp> ov(reinterpret_cast<const LayerOp*>(ops), reinterpret_cast<const LayerOp*>(ops) + n_ops);
    std::vector<double> vv(values, values + n_values);
    (*out)->build_plain = [=](const double*, Program& Q) {
      return build_from_layers(lx, ly, n_layers, n_det, n_cosets, dv.data(), iv.data(), n_ops, ov.data(), fv.data(),
                               vv.data(), int64_t(vv.size()), split_tol, Q);
    };
  }
  return s;
}

tn3d_status tn3d_net_with_gauge_rounds(tn3d_ctx c, tn3d_net base, int32_t rounds, tn3d_net* out) {
  if (!c || !out) return TN3D_E_INVALID;
  *out = nullptr;
  if (!base || base->ctx != c) return fail(c, TN3D_E_INVALID, "network handle null or of another context");
  if (rounds < 0 || rounds > 16) return fail(c, TN3D_E_INVALID, "rounds must lie in [0, 16]");
  if (!base->build_plain) return fail(c, TN3D_E_UNSUPPORTED, "network without a recorded builder");
  auto plain = base->build_plain;
  auto f = [plain, rounds](const double* q, Program& Q) {
    GaugeRounds g(rounds);
    return plain(q, Q);
  };
  Program P;
  std::string e = f(base->rates.data(), P);
  tn3d_status s = make_net(c, e, std::move(P), out);
  if (s == TN3D_OK) {
    (*out)->build_plain = plain;
    (*out)->gauge_rounds = rounds;
    (*out)->rates = base->rates;
    if (base->rebuild) (*out)->rebuild = f;
  }
  return s;
}

int32_t tn3d_net_num_detectors(tn3d_net n) { return n ? n->P.n_det : -1; }
int32_t tn3d_net_num_mechanisms(tn3d_net n) { return n ? n->P.n_mech : -1; }
int32_t tn3d_net_num_cosets(tn3d_net n) { return n ? n->P.n_cosets : -1; }

void tn3d_net_shape(tn3d_net n, int32_t* lx, int32_t* ly, int32_t* nl) {
  if (!n) return;
  if (lx) *lx = n->P.Lx;
  if (ly) *ly = n->P.Ly;
  if (nl) *nl = int32_t(std::count_if(n->P.layers.begin(), n->P.layers.end(),
                                      [](const LayerRange& r) { return r.gauge == 0; }));
}

static void drop_variants(tn3d_net net);

void tn3d_net_destroy(tn3d_net n) {
  if (!n) return;
  drop_variants(n);
  if (n->ctx) {
    tn3d_ctx c = n->ctx;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c, n->serial);
    if (n->dev) (void)hipFree(n->dev);
    c->nets.erase(std::remove(c->nets.begin(), c->nets.end(), n), c->nets.end());
  }
  delete n;
}

int32_t tn3d_ctx_graphs_cached(tn3d_ctx c) { return c ? int32_t(c->gcache.size()) : 0; }

tn3d_status tn3d_ctx_set_graphs(tn3d_ctx c, int32_t enable) {
  if (!c) return TN3D_E_INVALID;
  (void)hipSetDevice(c->device);
  if (!enable) {
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c, 0);
  }
  c->graphs = enable != 0;
  return TN3D_OK;
}

tn3d_status tn3d_contract_cosets(tn3d_ctx c, int32_t batch, const tn3d_net* nets, const uint8_t* synd,
                                 const int64_t* offs, const tn3d_params* pr, double* logp, uint32_t* flags) {
  return contract_impl(c, batch, nets, synd, offs, pr, logp, flags);
}

tn3d_status tn3d_contract_cosets_noalloc(tn3d_ctx c, int32_t batch, const tn3d_net* nets, const uint8_t* synd,
                                         const int64_t* offs, const tn3d_params* pr, double* logp,
                                         uint32_t* flags) {
  return contract_impl(c, batch, nets, synd, offs, pr, logp, flags, true);
}

// Autotuner: every candidate launch shape runs the caller's batch twice (the
// first run captures its launch sequence), the second is timed on the host
// around a synchronised stream; candidates whose results leave the default
// shape's decoded coset by more than the precision's rounding (1e-9 in FP64,
// 1e-4 otherwise) or change a decision are rejected.
tn3d_status tn3d_autotune(tn3d_ctx c, int32_t batch, const tn3d_net* nets, const uint8_t* synd,
                          const int64_t* offs, const tn3d_params* pr, double* out, int32_t n_out) {
  if (!c) return TN3D_E_INVALID;
  std::string why;
  if (!params_ok(pr, why)) return fail(c, TN3D_E_INVALID, why);
  if (batch <= 0 || !nets || !synd || !offs) return fail(c, TN3D_E_INVALID, "empty batch or null pointer");
  std::vector<tn3d_net> uniq;
  for (int i = 0; i < batch; ++i) {
    if (!nets[i] || nets[i]->ctx != c) return fail(c, TN3D_E_INVALID, "network handle null or of another context");
    if (std::find(uniq.begin(), uniq.end(), nets[i]) == uniq.end()) uniq.push_back(nets[i]);
  }
  HIPCHK(c, hipSetDevice(c->device));
  const int prec = pr->precision;
  const std::vector<LaunchTuning> cand = {{1, 16, 1}, {0, 16, 1}, {1, 8, 1}, {1, 16, 0}, {0, 16, 0}, {0, 8, 0}};
  double* d_lp = nullptr;
  uint32_t* d_fl = nullptr;
  if (hipMalloc(&d_lp, size_t(batch) * 4 * sizeof(double)) != hipSuccess ||
      hipMalloc(&d_fl, size_t(batch) * sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    if (d_lp) (void)hipFree(d_lp);
    return fail(c, TN3D_E_OOM, "autotune result buffers");
  }
  std::vector<double> ref(size_t(batch) * 4), cur(size_t(batch) * 4);
  const double tol = prec == TN3D_PREC_FP64 ? 1e-9 : 1e-4;
  double best_ms = 0.0, def_ms = 0.0;
  int best = 0;
  tn3d_status st = TN3D_OK;
  for (size_t k = 0; k < cand.size() && st == TN3D_OK; ++k) {
    for (tn3d_net n : uniq) c->tune[TuneKey{n->serial, prec, pr->chi, pr->chi_mps}] = cand[k];
    st = contract_impl(c, batch, nets, synd, offs, pr, d_lp, d_fl);
    if (st != TN3D_OK) break;
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      st = fail(c, TN3D_E_DEVICE, "autotune: stream synchronisation failed");
      break;
    }
    const auto t0 = std::chrono::steady_clock::now();
    st = contract_impl(c, batch, nets, synd, offs, pr, d_lp, d_fl);
    if (st != TN3D_OK) break;
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      st = fail(c, TN3D_E_DEVICE, "autotune: stream synchronisation failed");
      break;
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (hipMemcpy(cur.data(), d_lp, cur.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
      st = fail(c, TN3D_E_DEVICE, "autotune: result copy failed");
      break;
    }
    bool ok = true;
    if (k == 0) {
      ref = cur;
      def_ms = best_ms = ms;
    } else {
      const int nc = 4;
      for (int i = 0; i < batch && ok; ++i) {
        int a = 0, b = 0;
        for (int q = 1; q < nc; ++q) {
          if (ref[size_t(i) * nc + q] > ref[size_t(i) * nc + a]) a = q;
          if (cur[size_t(i) * nc + q] > cur[size_t(i) * nc + b]) b = q;
        }
        const double x = ref[size_t(i) * nc + a], y = cur[size_t(i) * nc + a];
        if (std::isnan(x) != std::isnan(y)) ok = false;
        else if (std::isfinite(x) && !(std::fabs(x - y) <= tol)) ok = false;
        else if (a != b && std::isfinite(x) && std::fabs(x - cur[size_t(i) * nc + b]) > tol) ok = false;
      }
      if (ok && ms < best_ms) {
        best_ms = ms;
        best = int(k);
      }
    }
  }
  (void)hipFree(d_lp);
  (void)hipFree(d_fl);
  for (tn3d_net n : uniq) c->tune[TuneKey{n->serial, prec, pr->chi, pr->chi_mps}] = cand[best];
  // the trial candidates' captured sequences are not needed any more
  (void)hipStreamSynchronize(c->stream);
  const int keep = pack_tuning(cand[best]);
  for (auto it = c->gcache.begin(); it != c->gcache.end();) {
    const bool ours = std::find_if(uniq.begin(), uniq.end(), [&](tn3d_net n) { return n->serial == it->first.net; }) !=
                      uniq.end();
    if (ours && it->first.prec == prec && it->first.chi == pr->chi && it->first.chi_mps == pr->chi_mps &&
        it->first.tune != keep) {
      (void)hipGraphExecDestroy(it->second.exec);
      it = c->gcache.erase(it);
    } else {
      ++it;
    }
  }
  if (st != TN3D_OK) return st;
  const double vals[6] = {double(best), double(cand[best].team), double(cand[best].mid), double(cand[best].narrow),
                          best_ms, def_ms};
  for (int i = 0; out && i < n_out && i < 6; ++i) out[i] = vals[i];
  return TN3D_OK;
}

// Decision for each item of a batch from its coset log-probabilities, grouped
// by coset count when networks differ.  items: device scratch of batch ints.
static tn3d_status decide(tn3d_ctx c, int32_t n, const tn3d_net* nets, const int32_t* host_items, int32_t* d_items,
                          const double* lp, double near_tie, int32_t* coset, double* logratio, uint32_t* flags) {
  // host_items == nullptr: the items are 0 .. n-1 of nets
  int ncs0 = nets[host_items ? host_items[0] : 0]->P.n_cosets;
  bool uniform = true;
  for (int i = 1; i < n; ++i)
    if (nets[host_items ? host_items[i] : i]->P.n_cosets != ncs0) uniform = false;
  if (uniform) {
    if (host_items)
      HIPCHK(c, hipMemcpyAsync(d_items, host_items, size_t(n) * 4, hipMemcpyHostToDevice, c->stream));
    else
      hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, c->stream, d_items, n, 0);
    launch_decode(n, ncs0, d_items, lp, near_tie, coset, logratio, flags, c->stream);
  } else {
    std::vector<int32_t> idx;
    for (int ncs = 2; ncs <= 4; ++ncs) {
      idx.clear();
      for (int i = 0; i < n; ++i) {
        const int it = host_items ? host_items[i] : i;
        if (nets[it]->P.n_cosets == ncs) idx.push_back(it);
      }
      if (idx.empty()) continue;
      HIPCHK(c, hipStreamSynchronize(c->stream));
      HIPCHK(c, hipMemcpy(d_items, idx.data(), idx.size() * 4, hipMemcpyHostToDevice));
      launch_decode(int(idx.size()), ncs, d_items, lp, near_tie, coset, logratio, flags, c->stream);
    }
  }
  HIPCHK(c, hipGetLastError());
  return TN3D_OK;
}

tn3d_status tn3d_decode(tn3d_ctx c, int32_t batch, const tn3d_net* nets, const uint8_t* synd,
                        const int64_t* offs, const tn3d_params* pr, int32_t* coset, double* logratio,
                        double* logp, uint32_t* flags) {
  if (!c) return TN3D_E_INVALID;
  if (batch > 0 && (!coset || !logratio)) return fail(c, TN3D_E_INVALID, "null output");
  if (batch <= 0) return contract_impl(c, batch, nets, synd, offs, pr, logp, flags);
  HIPCHK(c, hipSetDevice(c->device));
  // context-owned scratch: log p (when the caller passes none), item lists,
  // and the near-tie re-sweep's offsets, log p and flags
  const size_t b = size_t(batch);
  const size_t o_lp = 0, o_items = align256(b * 32), o_cnt = o_items + align256(b * 4),
               o_offs = o_cnt + 256, o_lps = o_offs + align256(b * 8), o_fls = o_lps + align256(b * 32),
               need = o_fls + align256(b * 4);
  if (c->aux_bytes < need) {
    if (c->aux) {
      HIPCHK(c, hipStreamSynchronize(c->stream));
      (void)hipFree(c->aux);
      c->aux = nullptr;
      c->aux_bytes = 0;
    }
    if (hipMalloc(&c->aux, need) != hipSuccess) return fail(c, TN3D_E_OOM, "decode scratch");
    c->aux_bytes = need;
  }
  double* lp = logp ? logp : reinterpret_cast<double*>(c->aux + o_lp);
  int32_t* d_items = reinterpret_cast<int32_t*>(c->aux + o_items);
  c->last_resweeps = 0;
  tn3d_status s = contract_impl(c, batch, nets, synd, offs, pr, lp, flags);
  if (s != TN3D_OK) return s;
  s = decide(c, batch, nets, nullptr, d_items, lp, pr->near_tie, coset, logratio, flags);
  if (s != TN3D_OK) return s;
  if (pr->precision == TN3D_PREC_FP64 || !(pr->near_tie > 0.0)) return TN3D_OK;
  // near ties of the reduced-precision pass are contracted again in FP64
  int32_t* d_cnt = reinterpret_cast<int32_t*>(c->aux + o_cnt);
  HIPCHK(c, hipMemsetAsync(d_cnt, 0, 4, c->stream));
  launch_pick_ties(batch, logratio, pr->near_tie, d_items, d_cnt, c->stream);
  int32_t cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, d_cnt, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (cnt <= 0) return TN3D_OK;
  std::vector<int32_t> ties(cnt);
  HIPCHK(c, hipMemcpy(ties.data(), d_items, size_t(cnt) * 4, hipMemcpyDeviceToHost));
  std::sort(ties.begin(), ties.end());
  HIPCHK(c, hipMemcpy(d_items, ties.data(), size_t(cnt) * 4, hipMemcpyHostToDevice));
  std::vector<tn3d_net> sub(cnt);
  for (int i = 0; i < cnt; ++i) sub[i] = nets[ties[i]];
  int64_t* d_offs = reinterpret_cast<int64_t*>(c->aux + o_offs);
  double* lps = reinterpret_cast<double*>(c->aux + o_lps);
  uint32_t* fls = reinterpret_cast<uint32_t*>(c->aux + o_fls);
  launch_gather_offsets(cnt, d_items, offs, d_offs, c->stream);
  HIPCHK(c, hipMemsetAsync(fls, 0, size_t(cnt) * 4, c->stream));
  // the same chi, chi_mps and rank rule in FP64, through Grams (the decision
  // needs far less than that route's accuracy)
  tn3d_params p64 = *pr;
  p64.precision = TN3D_PREC_FP64;
  p64.flags = TN3D_OPT_GRAM_FACTOR;
  p64.workspace_bytes = pr->workspace_bytes;
  // (with timing on, the re-sweep's kernels add to the sums like the main pass's)
  s = contract_impl(c, cnt, sub.data(), synd, d_offs, &p64, lps, fls);
  if (s != TN3D_OK) return s;
  launch_scatter_resweep(cnt, d_items, lps, fls, lp, flags, c->stream);
  c->last_resweeps = cnt;
  return decide(c, cnt, nets, ties.data(), d_items, lp, pr->near_tie, coset, logratio, flags);
}

// True when two programs differ at most in their pool values (then one
// launch sequence serves both, each sweep reading its own pool copy).
static bool same_structure(const Program& a, const Program& b) {
  auto eqb = [](const auto& x, const auto& y) {
    return x.size() == y.size() && (x.empty() || std::memcmp(x.data(), y.data(), x.size() * sizeof(x[0])) == 0);
  };
  return a.Lx == b.Lx && a.Ly == b.Ly && a.n_det == b.n_det && a.n_mech == b.n_mech && a.n_cosets == b.n_cosets &&
         a.n_bonds_h == b.n_bonds_h && a.n_bonds == b.n_bonds && a.max_K == b.max_K && a.max_dgate == b.max_dgate &&
         a.n_ext == b.n_ext && a.ext_src0 == b.ext_src0 && a.ext_src_n == b.ext_src_n && a.ext_words == b.ext_words &&
         a.inc0 == b.inc0 && a.n_inc == b.n_inc && a.wht == b.wht && a.pool.size() == b.pool.size() &&
         eqb(a.leg_bond, b.leg_bond) && eqb(a.dmax, b.dmax) && eqb(a.init_dims, b.init_dims) &&
         eqb(a.init_off, b.init_off) && eqb(a.bond_dim0, b.bond_dim0) && eqb(a.ones, b.ones) && eqb(a.gates, b.gates) &&
         eqb(a.layers, b.layers) && eqb(a.d_after, b.d_after) && eqb(a.par_after, b.par_after) &&
         eqb(a.d_final, b.d_final) && eqb(a.f_off, b.f_off) && eqb(a.ext_rows, b.ext_rows);
}

// Releases the networks at changed rates of a network.
static void drop_variants(tn3d_net net) {
  for (tn3d_net v : net->variants)
    if (v) tn3d_net_destroy(v);
  net->variants.clear();
  net->var_c.clear();
  net->var_slot.clear();
  if (net->d_pool_all && net->ctx) {
    (void)hipSetDevice(net->ctx->device);
    (void)hipStreamSynchronize(net->ctx->stream);
    (void)hipFree(net->d_pool_all);
  }
  net->d_pool_all = nullptr;
}

// Gradient of sum_s log P(m_s) with respect to the rates: the network at the
// given rates and, per mechanism i, the same network with rate i at c_i, all
// contracted at the caller's parameters; k_grad_* combine them.  Changed
// networks of the original's structure (the usual case: c_i lies inside the
// rate range, where no term vanishes) only bring their pool: they run in one
// batched pass with the original, each sweep reading its own pool copy.
tn3d_status tn3d_grad_loglik(tn3d_ctx c, tn3d_net net, int32_t batch, const uint8_t* synd, const int64_t* offs,
                             const tn3d_params* pr, int32_t n_rates, const int32_t* rate_of_mech, double* grad,
                             double* loglik_sum, double* loglik, double* grad_items, uint32_t* flags) {
  if (!c) return TN3D_E_INVALID;
  c->err.clear();
  std::string why;
  if (!params_ok(pr, why)) return fail(c, TN3D_E_INVALID, why);
  if (!net || net->ctx != c) return fail(c, TN3D_E_INVALID, "network handle null or of another context");
  if (!net->rebuild) return fail(c, TN3D_E_UNSUPPORTED, "network without a rate-dependent builder");
  if (batch < 0) return fail(c, TN3D_E_INVALID, "negative batch");
  const int n = net->P.n_mech;
  if (n < 1) return fail(c, TN3D_E_INVALID, "network without mechanisms");
  if (!rate_of_mech) {
    if (n_rates != n) return fail(c, TN3D_E_INVALID, "without rate_of_mech, n_rates must be the mechanism count");
  } else {
    if (n_rates < 1) return fail(c, TN3D_E_INVALID, "n_rates must be positive");
    for (int i = 0; i < n; ++i)
      if (rate_of_mech[i] < 0 || rate_of_mech[i] >= n_rates)
        return fail(c, TN3D_E_INVALID, "rate_of_mech entry out of [0, n_rates)");
  }
  if (!grad) return fail(c, TN3D_E_INVALID, "null gradient output");
  if (batch > 0 && (!synd || !offs)) return fail(c, TN3D_E_INVALID, "null pointer");
  HIPCHK(c, hipSetDevice(c->device));
  if (batch == 0) {
    HIPCHK(c, hipMemsetAsync(grad, 0, size_t(n_rates) * 8, c->stream));
    if (loglik_sum) HIPCHK(c, hipMemsetAsync(loglik_sum, 0, 8, c->stream));
    return TN3D_OK;
  }
  // the networks at p_i = c_i, built once per network: c_i a quarter of the
  // rate range away from p_i, towards the middle of the range
  if (int(net->var_c.size()) != n) {
    drop_variants(net);
    const double h = 0.25 * net->P.rate_max;
    std::vector<double> q = net->rates, pools = net->P.pool;
    net->var_c.assign(n, 0.0);
    net->var_slot.assign(n, -1);
    net->variants.assign(n, nullptr);
    int slots = 1;
    tn3d_status s = TN3D_OK;
    for (int i = 0; i < n && s == TN3D_OK; ++i) {
      const double ci = net->rates[i] <= 0.5 * net->P.rate_max ? net->rates[i] + h : net->rates[i] - h;
      net->var_c[i] = ci;
      q[i] = ci;
      Program P;
      std::string e = net->rebuild(q.data(), P);
      q[i] = net->rates[i];
      if (e.empty() && same_structure(net->P, P)) {
        net->var_slot[i] = slots++;
        pools.insert(pools.end(), P.pool.begin(), P.pool.end());
      } else {
        s = make_net(c, e, std::move(P), &net->variants[i]);
        if (s == TN3D_OK) net->variants[i]->tune_serial = net->serial;
      }
    }
    if (s == TN3D_OK) {
      if (hipMalloc(&net->d_pool_all, pools.size() * 8) != hipSuccess) {
        net->d_pool_all = nullptr;
        s = fail(c, TN3D_E_OOM, "pools of the networks at changed rates");
      } else if (hipMemcpy(net->d_pool_all, pools.data(), pools.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        s = fail(c, TN3D_E_DEVICE, "pool upload");
      }
    }
    if (s != TN3D_OK) {
      drop_variants(net);
      return s;
    }
  }
  // scratch: tiled offsets, log p and flags of the (n + 1) blocks, the pool
  // copy of each item, the rates (c_i, p_i), the rate -> mechanism lists,
  // the per-item derivatives
  const size_t B = size_t(batch), nb = size_t(n) + 1;
  const size_t o_offs = 0, o_lp = align256(nb * B * 8), o_fl = o_lp + align256(nb * B * 32),
               o_psel = o_fl + align256(nb * B * 4), o_cp = o_psel + align256(nb * B * 4),
               o_ptr = o_cp + align256(size_t(n) * 16), o_rm = o_ptr + align256((size_t(n_rates) + 1) * 4),
               o_term = o_rm + align256(size_t(n) * 4), need = o_term + (grad_items ? 0 : align256(B * n * 8));
  if (c->gaux_bytes < need) {
    if (c->gaux) {
      HIPCHK(c, hipStreamSynchronize(c->stream));
      (void)hipFree(c->gaux);
      c->gaux = nullptr;
      c->gaux_bytes = 0;
    }
    if (hipMalloc(&c->gaux, need) != hipSuccess) return fail(c, TN3D_E_OOM, "gradient scratch");
    c->gaux_bytes = need;
  }
  int64_t* offs_all = reinterpret_cast<int64_t*>(c->gaux + o_offs);
  double* lp = reinterpret_cast<double*>(c->gaux + o_lp);
  uint32_t* fl = reinterpret_cast<uint32_t*>(c->gaux + o_fl);
  int32_t* psel = reinterpret_cast<int32_t*>(c->gaux + o_psel);
  double* cp = reinterpret_cast<double*>(c->gaux + o_cp);
  int32_t* ptr = reinterpret_cast<int32_t*>(c->gaux + o_ptr);
  int32_t* rm = reinterpret_cast<int32_t*>(c->gaux + o_rm);
  double* term = grad_items ? grad_items : reinterpret_cast<double*>(c->gaux + o_term);
  std::vector<double> hcp(2 * size_t(n));
  for (int i = 0; i < n; ++i) {
    hcp[2 * i] = net->var_c[i];
    hcp[2 * i + 1] = net->rates[i];
  }
  std::vector<int32_t> hptr(size_t(n_rates) + 1, 0), hrm(n);
  for (int i = 0; i < n; ++i) hptr[(rate_of_mech ? rate_of_mech[i] : i) + 1]++;
  for (int k = 0; k < n_rates; ++k) hptr[k + 1] += hptr[k];
  {
    std::vector<int32_t> fill(hptr.begin(), hptr.end() - 1);
    for (int i = 0; i < n; ++i) hrm[fill[rate_of_mech ? rate_of_mech[i] : i]++] = i;
  }
  // items v B + s: block v = 0 the network at its rates, v = i + 1 rate i changed
  std::vector<int32_t> hsel(nb * B, 0), shared, own;
  for (size_t v = 0; v < nb; ++v) {
    const int slot = v == 0 ? 0 : net->var_slot[v - 1];
    for (size_t j = 0; j < B; ++j) {
      hsel[v * B + j] = slot < 0 ? 0 : slot;
      (slot < 0 ? own : shared).push_back(int32_t(v * B + j));
    }
  }
  HIPCHK(c, hipMemcpyAsync(cp, hcp.data(), hcp.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(ptr, hptr.data(), hptr.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(rm, hrm.data(), hrm.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(psel, hsel.data(), hsel.size() * 4, hipMemcpyHostToDevice, c->stream));
  launch_tile_offsets(batch, int(nb), offs, offs_all, c->stream);
  HIPCHK(c, hipGetLastError());
  // one batched pass over every item of the shared structure, then the
  // changed networks of another structure one by one
  const PoolSel ps{net->d_pool_all, int64_t(net->P.pool.size()), psel};
  tn3d_status s = run_group(c, net, shared, synd, offs_all, *pr, lp, fl, pr->precision, false, &ps);
  const bool graphs = c->graphs;
  c->graphs = false;
  std::vector<int32_t> items(B);
  for (size_t v = 1; v < nb && s == TN3D_OK; ++v) {
    if (net->var_slot[v - 1] >= 0) continue;
    for (size_t j = 0; j < B; ++j) items[j] = int32_t(v * B + j);
    s = run_group(c, net->variants[v - 1], items, synd, offs_all, *pr, lp, fl, pr->precision, false);
  }
  c->graphs = graphs;
  if (s == TN3D_OK) {
    launch_grad(batch, n, net->P.n_cosets, n_rates, lp, fl, cp, ptr, rm, term, grad, loglik, loglik_sum, flags,
                c->stream);
    if (hipGetLastError() != hipSuccess) s = fail(c, TN3D_E_DEVICE, "gradient kernels");
  }
  // the host arrays above were copied asynchronously
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return s;
}

tn3d_status tn3d_ctx_set_timing(tn3d_ctx c, int32_t enable) {
  if (!c) return TN3D_E_INVALID;
  HIPCHK(c, hipSetDevice(c->device));
  c->timing = enable <= 0 ? 0 : (enable >= 2 ? 2 : 1);
  // the sums restart here (ordered after the work already on the stream)
  for (int k = 0; k < 15; ++k) c->timing_out[k] = 0;
  for (int k = 0; k < 6; ++k) c->stats_out[k] = 0;
  HIPCHK(c, hipMemsetAsync(c->tacc, 0, 12 * sizeof(double), c->stream));
  return TN3D_OK;
}

tn3d_status tn3d_last_stats(tn3d_ctx c, double* out, int32_t n) {
  if (!c || !out) return TN3D_E_INVALID;
  if (c->timing < 2) return fail(c, TN3D_E_INVALID, "bond statistics need timing level 2");
  const double ns = c->stats_out[2] > 0 ? c->stats_out[2] : 1.0;
  double v[7] = {0, c->stats_out[1], c->stats_out[2], c->stats_out[3] / ns, c->stats_out[4], c->stats_out[5],
                 double(c->last_resweeps)};
  // mean over all bonds of all sweeps
  v[0] = c->stats_out[0] / (ns * (c->nb_last > 0 ? c->nb_last : 1));
  for (int i = 0; i < n && i < 7; ++i) out[i] = v[i];
  return TN3D_OK;
}

tn3d_status tn3d_last_timing(tn3d_ctx c, double* out, int32_t n) {
  if (!c || !out) return TN3D_E_INVALID;
  if (!c->timing) return fail(c, TN3D_E_INVALID, "timing not enabled");
  HIPCHK(c, hipSetDevice(c->device));
  double acc[12];
  HIPCHK(c, hipMemcpyAsync(acc, c->tacc, sizeof(acc), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double d[15];
  for (int i = 0; i < 10; ++i) d[i] = acc[i];
  d[3] = c->timing_out[3];
  d[6] = c->timing_out[6];
  d[10] = c->timing_out[10];
  d[11] = acc[10];
  d[12] = acc[11];
  d[13] = c->timing_out[13];
  d[14] = c->timing_out[14];
  for (int i = 0; i < n && i < 15; ++i) out[i] = d[i];
  return TN3D_OK;
}

}  // extern "C"
