// Host runtime of libsdc.so: the C ABI declared in include/sdc.h.
//
// sdc_init validates the configuration, generates the network's device code
// (netgen.cpp), compiles it together with the hand-written kernels
// (kernels/sdc_device.hip) for gfx950 through hipRTC, caches the code object
// on disk and loads it.  The entry points then only marshal arguments and
// enqueue kernels: every arithmetic step of the SDC update runs on the GPU.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sdc.h"
#include "kernels/sdc_args.h"
#include "netgen.hpp"

// kSdcArgsSrc, kSdcDeviceSrc: the kernel sources as string literals
#include "_gen/sdc_device_src.inc"

// Scratch memory of sdc_reaction_solve_noalloc: its deferred-zone queue lives
// in this array of the library's own code object, one copy per device, held
// until the process ends.  In host code the name is only a stand-in for the
// device array: host code resolves the address once per device with
// hipGetSymbolAddress (scratch_address below) and uses that pointer only.
static __device__ __align__(256) unsigned char scratch[SDC_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_init_error;

// Device address of `scratch` per device, resolved once with that device
// current (each device holds its own copy of the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_rc[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Resolve the scratch array of the current device `dev`; returns its address
// or nullptr (then *rc holds the HIP error).
void* scratch_address(int dev, hipError_t* rc) {
  if (dev < 0 || dev >= kMaxDevices) {
    *rc = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* p = nullptr;
    g_scratch_rc[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_rc[dev] == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
  }
  *rc = g_scratch_rc[dev];
  return g_scratch_ptr[dev];
}

// Deferred-zone queue of `cap` zones carved from a scratch block of `bytes`
// (256-byte aligned pieces: counter, zone index, iteration, x, b, rho, last
// step size).  Returns the bytes used, or -1 if they exceed `bytes`.
int64_t carve_queue(unsigned char* base, int64_t bytes, int64_t cap, int nx, DeferQueue* q) {
  auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
  const int64_t o_z = 256, o_it = o_z + up(cap * 8), o_x = o_it + up(cap * 4), o_b = o_x + up(cap * 8 * nx),
                o_aux = o_b + up(cap * 8 * nx), o_pe = o_aux + up(cap * 8), end = o_pe + up(cap * 8);
  if (end > bytes) return -1;
  q->count = (unsigned*)base;
  q->z = (sdc_i64*)(base + o_z);
  q->it = (int*)(base + o_it);
  q->x = (double*)(base + o_x);
  q->b = (double*)(base + o_b);
  q->aux = (double*)(base + o_aux);
  q->perr = (double*)(base + o_pe);
  q->capacity = cap;
  return end;
}

constexpr int kBlock = 256;
// Grid of the deferred-zone finish kernels, which stride over the queue: an
// empty queue then costs a few microseconds instead of a launch over all zones.
constexpr int64_t kFinishThreads = 2048 * kBlock;

// ------------------------------------------------------------ quadrature
// Gauss-Lobatto points on [0, 1] for 2..5 nodes (closed forms).
std::vector<double> lobatto_nodes(int n) {
  switch (n) {
    case 2: return {0.0, 1.0};
    case 3: return {0.0, 0.5, 1.0};
    case 4: {
      const double a = 0.5 / std::sqrt(5.0);
      return {0.0, 0.5 - a, 0.5 + a, 1.0};
    }
    case 5: {
      const double a = 0.5 * std::sqrt(3.0 / 7.0);
      return {0.0, 0.5 - a, 0.5, 0.5 + a, 1.0};
    }
  }
  return {};
}

// Right Radau points for 1..4 points on (0, 1], preceded by tau_0 = 0 (the
// start of the step, not a quadrature point): the zeros of
// P_s(x) - P_{s-1}(x) on [-1, 1] mapped to t = (x + 1) / 2, the largest of
// which is x = 1.  The s - 1 interior zeros are bracketed on a fine grid and
// bisected to the last bit.
std::vector<double> radau_nodes(int n) {
  const int s = n - 1;
  auto q = [s](double x) {  // P_s(x) - P_{s-1}(x) by the three-term recurrence
    double p0 = 1.0, p1 = x;
    if (s == 1) return p1 - p0;
    for (int k = 2; k <= s; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    return p1 - p0;
  };
  std::vector<double> tau{0.0};
  const int grid = 4096;
  for (int i = 0; i < grid; ++i) {
    double lo = -1.0 + 1.9 * i / grid, hi = -1.0 + 1.9 * (i + 1) / grid;
    double flo = q(lo);
    if ((flo < 0.0) == (q(hi) < 0.0)) continue;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      const double fm = q(mid);
      if ((fm < 0.0) == (flo < 0.0)) {
        lo = mid;
        flo = fm;
      } else {
        hi = mid;
      }
    }
    tau.push_back(0.5 * (0.5 * (lo + hi) + 1.0));
  }
  tau.push_back(1.0);
  return tau;
}

// S[m][j] = integral over [tau_m, tau_{m+1}] of the Lagrange polynomial l_j
// through the interpolation points tau[first..]: the node-to-node quadrature
// of the integral in Eq. 2 (columns j < first are zero).  Gauss-Lobatto nodes
// interpolate through every node (first = 0), right Radau nodes through the
// Radau points only (first = 1).
std::vector<std::vector<double>> integration_matrix(const std::vector<double>& tau, int first) {
  const int n = (int)tau.size();
  std::vector<std::vector<double>> S(n - 1, std::vector<double>(n, 0.0));
  for (int j = first; j < n; ++j) {
    std::vector<double> c(1, 1.0);  // power-series coefficients of l_j
    for (int i = first; i < n; ++i) {
      if (i == j) continue;
      const double den = tau[j] - tau[i];
      std::vector<double> nc(c.size() + 1, 0.0);
      for (size_t p = 0; p < c.size(); ++p) {
        nc[p + 1] += c[p] / den;
        nc[p] -= c[p] * tau[i] / den;
      }
      c.swap(nc);
    }
    auto anti = [&](double t) {
      double s = 0.0, tp = t;
      for (size_t p = 0; p < c.size(); ++p, tp *= t) s += c[p] * tp / double(p + 1);
      return s;
    };
    for (int m = 0; m < n - 1; ++m) S[m][j] = anti(tau[m + 1]) - anti(tau[m]);
  }
  return S;
}

// ------------------------------------------------------------ kernel cache
uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string library_dir() {
  Dl_info info;
  if (dladdr((void*)&library_dir, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    auto k = p.rfind('/');
    if (k != std::string::npos) return p.substr(0, k);
  }
  return ".";
}

std::string cache_dir() {
  const char* e = std::getenv("SDC_KERNEL_CACHE");
  if (e && *e) return e;
  return library_dir() + "/_kcache";
}

const std::vector<const char*>& compile_options() {
  static const std::vector<const char*> opts = {
      "--offload-arch=gfx950", "-O3", "-std=c++17",
      // no packed FP32 instructions
      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  return opts;
}

std::mutex g_cache_mutex;
std::map<uint64_t, std::vector<char>> g_code_cache;

bool read_file(const std::string& path, std::vector<char>* out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  out->assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
  return !out->empty();
}

void write_file_atomic(const std::string& dir, const std::string& name, const std::vector<char>& data) {
  ::mkdir(dir.c_str(), 0755);
  std::string tmp = dir + "/." + name + ".tmp" + std::to_string(::getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) return;
  }
  std::rename(tmp.c_str(), (dir + "/" + name).c_str());
}

// Name of the ahead-of-time code object of `src` (compiled with hipcc at build
// time): keyed by the source and the options only.
std::string aot_name(const std::string& src) {
  std::string key_text = src;
  for (const char* o : compile_options()) key_text += std::string("\n//opt ") + o;
  char name[64];
  std::snprintf(name, sizeof name, "sdc_%016llx.aot.co", (unsigned long long)fnv1a(key_text));
  return name;
}

// Code object for `src`: in-process cache, then the ahead-of-time object of
// the build step, then the on-disk cache of run-time compilations, then
// hipRTC.  The run-time key includes the hipRTC version, which depends on the
// process (a hipRTC library loaded earlier by another component wins).
int get_code_object(const std::string& src, std::vector<char>* code, std::string* err) {
  std::string key_text = src;
  for (const char* o : compile_options()) key_text += std::string("\n//opt ") + o;
  int ver_major = 0, ver_minor = 0;
  hiprtcVersion(&ver_major, &ver_minor);
  key_text += "\n//hiprtc " + std::to_string(ver_major) + "." + std::to_string(ver_minor);
  const uint64_t key = fnv1a(key_text);
  char name[64];
  std::snprintf(name, sizeof name, "sdc_%016llx.co", (unsigned long long)key);
  {
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    auto it = g_code_cache.find(key);
    if (it != g_code_cache.end()) {
      *code = it->second;
      return SDC_OK;
    }
  }
  const std::string dir = cache_dir();
  if (read_file(dir + "/" + aot_name(src), code) || read_file(dir + "/" + name, code)) {
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    g_code_cache[key] = *code;
    return SDC_OK;
  }
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "sdc_kernels.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    *err = "hiprtcCreateProgram failed";
    return SDC_ERR_COMPILE;
  }
  const auto& opts = compile_options();
  hiprtcResult rc = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  if (rc != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    *err = std::string("kernel compilation failed: ") + hiprtcGetErrorString(rc) + "\n" + log.substr(0, 4000);
    return SDC_ERR_COMPILE;
  }
  size_t sz = 0;
  hiprtcGetCodeSize(prog, &sz);
  code->resize(sz);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  write_file_atomic(dir, name, *code);
  std::lock_guard<std::mutex> lk(g_cache_mutex);
  g_code_cache[key] = *code;
  return SDC_OK;
}

// ------------------------------------------------------------ validation
struct Prepared {
  sdc_config cfg;
  sdcgen::Topology topo;
  sdcgen::Pattern pat;
  std::vector<double> lnA, b, E, Q, q;
  int64_t Z = 0;
  std::vector<int64_t> box_off;  // [nbox + 1] zone offsets (batched boxes)
  std::vector<int32_t> box_ext;  // [nbox][3]
  std::string source;
};

int prepare(const sdc_config* cfg, const sdc_network* net, Prepared* P, std::string* err) {
  if (!cfg || !net) {
    *err = "null configuration or network";
    return SDC_ERR_ARG;
  }
  const sdc_config& c = *cfg;
  if (c.dim < 1 || c.dim > 3) {
    *err = "dim must be 1, 2 or 3";
    return SDC_ERR_ARG;
  }
  int64_t Z = 1;
  const int64_t minn = c.advection ? 2 : 1;
  for (int d = 0; d < c.dim; ++d) {
    if (!(c.dx[d] > 0.0) || !std::isfinite(c.dx[d])) {
      *err = "dx must be positive and finite";
      return SDC_ERR_ARG;
    }
  }
  if (c.nbox < 0) {
    *err = "nbox must be >= 0";
    return SDC_ERR_ARG;
  }
  if (c.nbox > 0) {
    if (!c.box_n) {
      *err = "box_n must not be NULL when nbox > 0";
      return SDC_ERR_ARG;
    }
    P->box_off.assign(1, 0);
    Z = 0;
    for (int bx = 0; bx < c.nbox; ++bx) {
      int64_t zb = 1;
      for (int d = 0; d < 3; ++d) {
        const int64_t e = d < c.dim ? c.box_n[3 * bx + d] : 1;
        if (d < c.dim && (e < minn || e > (int64_t(1) << 20))) {
          *err = "box extents must be in [2, 2^20] per direction (>= 1 without advection)";
          return SDC_ERR_ARG;
        }
        P->box_ext.push_back((int32_t)e);
        zb *= e;
      }
      Z += zb;
      if (Z > (int64_t(1) << 31) - (int64_t)kBlock) break;
      P->box_off.push_back(Z);
    }
  } else {
    for (int d = 0; d < c.dim; ++d) {
      if (c.n[d] < minn || c.n[d] > (int64_t(1) << 30)) {
        *err = "zone counts must be in [2, 2^30] per direction (>= 1 without advection)";
        return SDC_ERR_ARG;
      }
      Z *= c.n[d];
    }
  }
  if (Z > (int64_t(1) << 31) - (int64_t)kBlock) {
    *err = "grid exceeds 2^31 zones";
    return SDC_ERR_UNSUPPORTED;
  }
  if (!(c.gamma > 1.0) || !std::isfinite(c.gamma)) {
    *err = "gamma must exceed 1";
    return SDC_ERR_ARG;
  }
  if (c.n_nodes < 2 || c.n_nodes > SDC_MAX_NODES) {
    *err = "n_nodes must be in 2..5";
    return SDC_ERR_UNSUPPORTED;
  }
  if (c.node_type != SDC_NODES_LOBATTO && c.node_type != SDC_NODES_RADAU) {
    *err = "node_type must be SDC_NODES_LOBATTO or SDC_NODES_RADAU";
    return SDC_ERR_ARG;
  }
  if (c.space_order != 2 && c.space_order != 4) {
    *err = "space_order must be 2 or 4";
    return SDC_ERR_ARG;
  }
  if (c.space_order == 4 && c.nbox > 0) {
    *err = "the fourth-order method supports single grids only";
    return SDC_ERR_UNSUPPORTED;
  }
  if (c.n_iters < 1) {
    *err = "n_iters must be >= 1";
    return SDC_ERR_ARG;
  }
  if (c.precision != SDC_FP64 && c.precision != SDC_MIXED) {
    *err = "precision must be SDC_FP64 or SDC_MIXED";
    return SDC_ERR_ARG;
  }
  if ((c.advection != 0 && c.advection != 1) || (c.slope != 0 && c.slope != 1)) {
    *err = "advection and slope must be 0 or 1";
    return SDC_ERR_ARG;
  }
  if (!(c.newton_tol > 0.0) || c.newton_maxiter < 1 || !(c.pivot_threshold >= 0.0) || !std::isfinite(c.alpha)) {
    *err = "newton_tol > 0, newton_maxiter >= 1, pivot_threshold >= 0 and finite alpha required";
    return SDC_ERR_ARG;
  }
  const sdc_network& n = *net;
  if (n.nspec < 1 || n.nspec > SDC_MAX_SPECIES || n.nreact < 0 || n.nreact > 4096) {
    *err = "nspec must be in 1..31 and nreact in 0..4096";
    return SDC_ERR_UNSUPPORTED;
  }
  if (n.nreact > 0 && (!n.reactants || !n.stoich || !n.lnA || !n.b || !n.E)) {
    *err = "network arrays must not be NULL";
    return SDC_ERR_ARG;
  }
  if (!n.q) {
    *err = "network q must not be NULL";
    return SDC_ERR_ARG;
  }
  P->cfg = c;
  P->Z = Z;
  auto& t = P->topo;
  t.ns = n.nspec;
  t.nr = n.nreact;
  t.reactants.resize(n.nreact);
  t.stoich.assign(n.stoich, n.stoich + (size_t)n.nreact * n.nspec);
  for (int r = 0; r < n.nreact; ++r) {
    const int a = n.reactants[2 * r], cc = n.reactants[2 * r + 1];
    if (a < 0 || a >= n.nspec || cc < -1 || cc >= n.nspec) {
      *err = "reactant index out of range in reaction " + std::to_string(r);
      return SDC_ERR_ARG;
    }
    t.reactants[r] = {a, cc};
    for (int i = 0; i < n.nspec; ++i)
      if (!std::isfinite(t.stoich[(size_t)r * n.nspec + i])) {
        *err = "non-finite stoichiometric coefficient";
        return SDC_ERR_ARG;
      }
  }
  P->q.assign(n.q, n.q + n.nspec);
  P->lnA.assign(n.lnA ? n.lnA : nullptr, n.lnA ? n.lnA + n.nreact : nullptr);
  P->b.assign(n.b ? n.b : nullptr, n.b ? n.b + n.nreact : nullptr);
  P->E.assign(n.E ? n.E : nullptr, n.E ? n.E + n.nreact : nullptr);
  P->Q.assign(n.nreact, 0.0);
  for (int r = 0; r < n.nreact; ++r) {
    double s = 0.0;
    for (int i = 0; i < n.nspec; ++i) s -= t.stoich[(size_t)r * n.nspec + i] * P->q[i];
    P->Q[r] = s;
  }
  P->pat = sdcgen::build_pattern(t);
  std::ostringstream src;
  src << "// SDC kernels: dim " << c.dim << ", " << c.n_nodes << " nodes, "
      << (c.precision == SDC_MIXED ? "mixed" : "fp64") << "\n";
  src << "#define SDC_DIM " << c.dim << "\n#define SDC_NNODES " << c.n_nodes << "\n";
  if (c.precision == SDC_MIXED) src << "#define SDC_MIXED 1\n";
  src << kSdcArgsSrc << "\n" << sdcgen::generate(t, P->pat) << "\n";
  std::string dev = kSdcDeviceSrc;
  const std::string inc = "#include \"sdc_args.h\"";
  auto k = dev.find(inc);
  if (k != std::string::npos) dev.replace(k, inc.size(), "// (argument blocks defined above)");
  src << dev;
  P->source = src.str();
  return SDC_OK;
}

std::vector<double> params_image(const Prepared& P, int nr_alloc) {
  // NetParams layout: lnA[NRA], b[NRA], E[NRA], Q[NRA], q[NS]
  const int nr = P.topo.nr;
  std::vector<double> img((size_t)4 * nr_alloc + P.topo.ns, 0.0);
  for (int r = 0; r < nr; ++r) {
    img[r] = P.lnA[r];
    img[nr_alloc + r] = P.b[r];
    img[2 * nr_alloc + r] = P.E[r];
    img[3 * nr_alloc + r] = P.Q[r];
  }
  for (int i = 0; i < P.topo.ns; ++i) img[4 * nr_alloc + i] = P.q[i];
  return img;
}

}  // namespace

// ------------------------------------------------------------------ handle
struct sdc_handle_s {
  Prepared P;
  int ns = 0, nc = 0, nx = 0, M = 0, nra = 1;
  std::vector<double> tau;
  std::vector<std::vector<double>> S;
  hipModule_t mod = nullptr;
  hipFunction_t f_advect_vjp = nullptr, f_trans_adj_first = nullptr, f_trans_adj = nullptr, f_source_vjp = nullptr,
                f_theta_reduce = nullptr, f_axpy = nullptr;
  // adjoint workspace (allocated on first use): forward replay nodes, stored
  // node states of every iteration, adjoint arrays, parameter partials
  std::vector<double*> adj_buf;
  hipFunction_t f_first_o2 = nullptr, f_node0_o2 = nullptr, f_later_o2 = nullptr, f_trans_finish = nullptr,
                f_solve_o2 = nullptr, f_solve_finish = nullptr, f_reset = nullptr;
  // fourth order in space: kernels and workspace (allocated on first use):
  // face fluxes F [NC][Z], zone-centre density [Z], Newton rhs, iterate and
  // source [NX][Z] each, iteration counts [Z]
  hipFunction_t f_flux4[3] = {nullptr, nullptr, nullptr}, f_div4[3] = {nullptr, nullptr, nullptr},
                f_favg4[3] = {nullptr, nullptr, nullptr},
                f_conv4 = nullptr, f_source4c = nullptr, f_rhs4[3] = {nullptr, nullptr, nullptr},
                f_newin4 = nullptr, f_avgst4 = nullptr;
  double *o4_F = nullptr, *o4_Uf = nullptr, *o4_rho = nullptr, *o4_b = nullptr, *o4_x = nullptr, *o4_R = nullptr;
  int* o4_it = nullptr;
  // deferred-zone queue (capacity Z, allocated on first use) and the tuned
  // kernel choice: occupancy-2 variants and the fast-pass iteration cap
  DeferQueue q{};
  bool q_ready = false;
  int occ2 = 0;
  int cap = 0;  // 0: no cap (newton_maxiter)
  // split schedule: zone batches whose explicit part (on `aux`) runs beside
  // the Newton kernel of the previous batch; 0 = fused transition kernels
  int split = 0;
  bool tuned = false;
  bool capturing = false;
  hipFunction_t f_pre[3] = {nullptr, nullptr, nullptr}, f_newton = nullptr, f_newton_o2 = nullptr;
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> batch_ev;
  double* split_buf = nullptr;  // [NX + 2][Z]
  hipFunction_t f_advect = nullptr, f_advect_rows = nullptr, f_source = nullptr, f_solve = nullptr, f_first = nullptr,
                f_node0 = nullptr, f_later = nullptr, f_fill = nullptr, f_zero_list = nullptr;
  void* d_params = nullptr;
  unsigned long long* d_stats = nullptr;
  int64_t* d_box_off = nullptr;
  int32_t* d_box_ext = nullptr;
  int32_t* d_blk_box = nullptr;
  RowDesc* d_rows = nullptr;  // row advection kernel: one descriptor per block
  int64_t n_rows = 0;
  int row_bw = 256;  // threads per block of the row kernel (512 for rows of 257..512 zones)
  int zchunk = 0;  // row kernel tile: planes per z chunk (0: heuristic)
  hipStream_t last_stream = nullptr;
  // device of the handle's module and its scratch array (noalloc entry point)
  int device = 0;
  void* scratch = nullptr;
  hipError_t scratch_rc = hipSuccess;
  std::string err;
  // per-kernel timing
  bool profile = false;
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  // captured steps: one executable graph per buffer-rotation phase, valid for
  // the (dt, work arrays) they were captured with
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t step_graph[2] = {nullptr, nullptr};
  std::vector<uintptr_t> graph_key;
};

namespace {

int fail(sdc_handle h, int code, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_init_error = msg;
  return code;
}

#define HIP_CHECK(h, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(h, SDC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int kind_of(const sdc_handle h, hipFunction_t f) {
  if (f == h->f_advect || f == h->f_advect_rows) return SDC_K_ADVECT;
  for (int d = 0; d < 3; ++d)
    if (f && (f == h->f_flux4[d] || f == h->f_div4[d] || f == h->f_favg4[d])) return SDC_K_ADVECT;
  if (f && (f == h->f_source4c || f == h->f_conv4)) return SDC_K_SOURCE;
  if (f && f == h->f_rhs4[0]) return SDC_K_TRANSITION_FIRST;
  if (f && f == h->f_rhs4[1]) return SDC_K_TRANSITION_NODE0;
  if (f && f == h->f_rhs4[2]) return SDC_K_TRANSITION_LATER;
  if (f && (f == h->f_newin4 || f == h->f_avgst4)) return SDC_K_ORDER4;
  if (f == h->f_source) return SDC_K_SOURCE;
  if (f == h->f_solve) return SDC_K_SOLVE;
  if (f == h->f_solve_o2) return SDC_K_SOLVE;
  if (f == h->f_solve_finish || f == h->f_trans_finish) return SDC_K_FINISH;
  if (f == h->f_pre[0] || f == h->f_pre[1] || f == h->f_pre[2] || f == h->f_newton || f == h->f_newton_o2)
    return SDC_K_SPLIT;
  if (f == h->f_first || f == h->f_first_o2) return SDC_K_TRANSITION_FIRST;
  if (f == h->f_node0 || f == h->f_node0_o2) return SDC_K_TRANSITION_NODE0;
  if (f == h->f_later || f == h->f_later_o2) return SDC_K_TRANSITION_LATER;
  if (f == h->f_reset) return SDC_K_FILL;
  if (f == h->f_fill || f == h->f_zero_list) return SDC_K_FILL;
  return SDC_K_ADJOINT;
}

hipEvent_t take_event(sdc_handle h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int launch_blocks(sdc_handle h, hipFunction_t f, int64_t nb, void* args, hipStream_t s, int block = kBlock);

int launch(sdc_handle h, hipFunction_t f, int64_t nthreads, void* args, hipStream_t s) {
  if (nthreads <= 0) return SDC_OK;
  return launch_blocks(h, f, (nthreads + kBlock - 1) / kBlock, args, s);
}

int launch_blocks(sdc_handle h, hipFunction_t f, int64_t nb, void* args, hipStream_t s, int block) {
  if (nb <= 0) return SDC_OK;
  void* params[] = {args};
  hipEvent_t ea = nullptr, eb = nullptr;
  if (h->profile) {
    ea = take_event(h);
    eb = take_event(h);
    if (!ea || !eb) return fail(h, SDC_ERR_HIP, "hipEventCreate failed");
    HIP_CHECK(h, hipEventRecord(ea, s));
  }
  HIP_CHECK(h, hipModuleLaunchKernel(f, (unsigned)nb, 1, 1, (unsigned)block, 1, 1, 0, s, params, nullptr));
  if (h->profile) {
    HIP_CHECK(h, hipEventRecord(eb, s));
    h->timed.push_back({kind_of(h, f), ea, eb});
  }
  return SDC_OK;
}

int fill(sdc_handle h, double* p, int64_t n, double v, hipStream_t s) {
  FillArgs a{p, n, v};
  return launch(h, h->f_fill, n, &a, s);
}

NewtonCtl newton_ctl(const sdc_handle h) {
  NewtonCtl c;
  c.tol = h->P.cfg.newton_tol;
  c.tau = h->P.cfg.pivot_threshold;
  c.maxiter = h->P.cfg.newton_maxiter;
  c.cap = h->cap > 0 ? h->cap : h->P.cfg.newton_maxiter;
  return c;
}

// Deferred-zone queue: capacity Z, so every zone can be deferred.
int ensure_queue(sdc_handle h) {
  if (h->q_ready) return SDC_OK;
  const int64_t Z = h->P.Z;
  DeferQueue& q = h->q;
  q.capacity = Z;
  const size_t aux = 2 + h->P.cfg.dim;
  if (hipMalloc((void**)&q.z, Z * sizeof(sdc_i64)) != hipSuccess ||
      hipMalloc((void**)&q.it, Z * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&q.x, (size_t)h->nx * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&q.b, (size_t)h->nx * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&q.aux, aux * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&q.perr, Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&q.count, sizeof(unsigned)) != hipSuccess)
    return fail(h, SDC_ERR_NOMEM, "hipMalloc(deferred-zone queue) failed");
  h->q_ready = true;
  return SDC_OK;
}

// Stream, events and the [NX + 2][Z] array of the split schedule.
int ensure_split(sdc_handle h) {
  if (!h->aux) HIP_CHECK(h, hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
  if (!h->fork_ev) HIP_CHECK(h, hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
  while ((int)h->batch_ev.size() < h->split) {
    hipEvent_t e = nullptr;
    HIP_CHECK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->batch_ev.push_back(e);
  }
  if (!h->split_buf && hipMalloc((void**)&h->split_buf, (size_t)(h->nx + 2) * h->P.Z * sizeof(double)) != hipSuccess)
    return fail(h, SDC_ERR_NOMEM, "hipMalloc(split schedule array) failed");
  return SDC_OK;
}

void free_split(sdc_handle h) {
  if (h->split_buf) (void)hipFree(h->split_buf);
  for (auto e : h->batch_ev) (void)hipEventDestroy(e);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  h->split_buf = nullptr;
  h->batch_ev.clear();
  h->fork_ev = nullptr;
  h->aux = nullptr;
}

void free_queue(sdc_handle h) {
  DeferQueue& q = h->q;
  for (void* p : {(void*)q.z, (void*)q.it, (void*)q.x, (void*)q.b, (void*)q.aux, (void*)q.perr, (void*)q.count})
    if (p) (void)hipFree(p);
  h->q = DeferQueue{};
  h->q_ready = false;
}

int ensure_o4(sdc_handle h) {
  if (h->o4_F) return SDC_OK;
  const size_t Z = (size_t)h->P.Z;
  if (hipMalloc((void**)&h->o4_F, h->nc * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->o4_Uf, h->nc * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->o4_rho, Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->o4_b, h->nx * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->o4_x, h->nx * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->o4_R, h->nx * Z * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&h->o4_it, Z * sizeof(int)) != hipSuccess)
    return fail(h, SDC_ERR_NOMEM, "hipMalloc(fourth-order workspace) failed");
  return SDC_OK;
}

void free_o4(sdc_handle h) {
  for (void* p : {(void*)h->o4_F, (void*)h->o4_Uf, (void*)h->o4_rho, (void*)h->o4_b, (void*)h->o4_x, (void*)h->o4_R, (void*)h->o4_it})
    if (p) (void)hipFree(p);
  h->o4_F = h->o4_Uf = h->o4_rho = h->o4_b = h->o4_x = h->o4_R = nullptr;
  h->o4_it = nullptr;
}

void grid_extents(const sdc_handle h, int* n) {
  for (int d = 0; d < 3; ++d) n[d] = d < h->P.cfg.dim ? (int)h->P.cfg.n[d] : 1;
}

int reset_queue(sdc_handle h, hipStream_t s) {
  void* params[] = {&h->q.count};
  HIP_CHECK(h, hipModuleLaunchKernel(h->f_reset, 1, 1, 1, 64, 1, 1, 0, s, params, nullptr));
  return SDC_OK;
}

// Blocks of the row advection kernel: every periodic grid (the domain, or
// each box) is cut into slots (x-row y, z chunk), R = bw / n0 slots per
// block.  zmax = 0: the chunk starts at 32 planes and is halved until the
// domain gives at least 2048 blocks (down to 4 planes); zmax > 0 (a tuned
// tile): chunks of min(zmax, n2) planes.  A box's chunk is then halved until
// its slots fill a block (down to 2 planes).
std::vector<RowDesc> row_descriptors(const Prepared& P, int zmax, int bw) {
  std::vector<RowDesc> out;
  auto add_grid = [&](int64_t base, int n0, int n1, int n2, bool domain) {
    const int R = bw / n0;
    const int z0 = zmax > 0 ? zmax : 32;
    int zc = n2 < z0 ? n2 : z0;
    auto slots = [&](int z) { return (int64_t)n1 * ((n2 + z - 1) / z); };
    if (domain) {
      if (zmax == 0)
        while (zc > 4 && (slots(zc) + R - 1) / R < 2048) zc = (zc + 1) / 2;
    } else {
      while (zc > 2 && slots(zc) < R) zc = (zc + 1) / 2;
    }
    const int64_t ns = slots(zc);
    for (int64_t s0 = 0; s0 < ns; s0 += R) {
      RowDesc d;
      d.base = base;
      d.n0 = n0;
      d.n1 = n1;
      d.n2 = n2;
      d.zc = zc;
      d.slot0 = (int)s0;
      d.nslot = (int)ns;
      out.push_back(d);
    }
  };
  const sdc_config& c = P.cfg;
  if (c.nbox > 0)
    for (int b = 0; b < c.nbox; ++b)
      add_grid(P.box_off[b], P.box_ext[3 * b], P.box_ext[3 * b + 1], P.box_ext[3 * b + 2], false);
  else
    add_grid(0, (int)c.n[0], (int)c.n[1], (int)c.n[2], true);
  return out;
}

// Longest x-row of the grid or of any box.
int64_t longest_row(const Prepared& P) {
  const sdc_config& c = P.cfg;
  int64_t n0 = 0;
  if (c.nbox > 0) {
    for (int b = 0; b < c.nbox; ++b) n0 = std::max<int64_t>(n0, P.box_ext[3 * b]);
    return n0;
  }
  return c.n[0];
}

// The row kernel takes 3D grids whose x-rows fit one block (256 threads, or
// 512 for longer rows) and whose component arrays stay below 4 GiB (32-bit
// buffer offsets).
constexpr int64_t kRowMax = 512;
bool rows_kernel_fits(const Prepared& P) {
  const sdc_config& c = P.cfg;
  if (c.dim != 3 || 8 * P.Z >= (int64_t(1) << 32)) return false;
  return longest_row(P) <= kRowMax;
}

// (Re)build the row descriptors for the current tile.
int upload_rows(sdc_handle h) {
  if (!h->f_advect_rows) return SDC_OK;
  const std::vector<RowDesc> rows = row_descriptors(h->P, h->zchunk, h->row_bw);
  if (h->d_rows && (int64_t)rows.size() > h->n_rows) {
    (void)hipFree(h->d_rows);
    h->d_rows = nullptr;
  }
  if (!h->d_rows && hipMalloc((void**)&h->d_rows, rows.size() * sizeof(RowDesc)) != hipSuccess)
    return fail(h, SDC_ERR_NOMEM, "hipMalloc(row descriptors) failed");
  HIP_CHECK(h, hipMemcpy(h->d_rows, rows.data(), rows.size() * sizeof(RowDesc), hipMemcpyHostToDevice));
  h->n_rows = (int64_t)rows.size();
  return SDC_OK;
}

// Fourth-order A: per direction the face-averaged fluxes, then their
// difference into A.
int advect4(sdc_handle h, const double* U, double* A, hipStream_t s) {
  if (int rc = ensure_o4(h)) return rc;
  const sdc_config& c = h->P.cfg;
  Flux4Args a;
  std::memset(&a, 0, sizeof a);
  a.U = U;
  a.F = h->o4_F;
  a.Uf = h->o4_Uf;
  a.A = A;
  a.Z = h->P.Z;
  grid_extents(h, a.n);
  a.gamma = c.gamma;
  for (int d = 0; d < c.dim; ++d) {
    a.first = d == 0;
    a.idx = 1.0 / c.dx[d];
    if (int rc = launch(h, h->f_favg4[d], h->P.Z, &a, s)) return rc;
    if (int rc = launch(h, h->f_flux4[d], h->P.Z, &a, s)) return rc;
    if (int rc = launch(h, h->f_div4[d], h->P.Z, &a, s)) return rc;
  }
  return SDC_OK;
}

int advect(sdc_handle h, const double* U, double* A, hipStream_t s) {
  const sdc_config& c = h->P.cfg;
  if (!c.advection) return fill(h, A, (int64_t)h->nc * h->P.Z, 0.0, s);
  if (c.space_order == 4) return advect4(h, U, A, s);
  AdvArgs a;
  std::memset(&a, 0, sizeof a);
  a.U = U;
  a.A = A;
  a.Z = h->P.Z;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = d < c.dim ? (int)c.n[d] : 1;
    a.idx[d] = d < c.dim ? 1.0 / c.dx[d] : 0.0;
  }
  a.gamma = c.gamma;
  a.alpha = c.alpha;
  a.slope = c.slope;
  if (h->f_advect_rows) {
    a.rows = h->d_rows;
    return launch_blocks(h, h->f_advect_rows, h->n_rows, &a, s, h->row_bw);
  }
  if (c.nbox > 0) {
    a.nbox = c.nbox;
    a.box_off = (const sdc_i64*)h->d_box_off;
    a.box_ext = h->d_box_ext;
    a.blk_box = h->d_blk_box;
  }
  return launch(h, h->f_advect, h->P.Z, &a, s);
}

// Fourth-order <R(U)>: R at the zone-centre values, converted to averages.
int source4(sdc_handle h, const double* U, double* R, hipStream_t s) {
  if (int rc = ensure_o4(h)) return rc;
  O4Args o;
  std::memset(&o, 0, sizeof o);
  o.Z = h->P.Z;
  grid_extents(h, o.n);
  o.U = (double*)U;
  o.R = h->o4_R;
  o.P = h->d_params;
  o.gm1 = h->P.cfg.gamma - 1.0;
  if (int rc = launch(h, h->f_source4c, h->P.Z, &o, s)) return rc;
  ConvArgs cv;
  std::memset(&cv, 0, sizeof cv);
  cv.src = h->o4_R;
  cv.dst = R;
  cv.Z = h->P.Z;
  grid_extents(h, cv.n);
  cv.ncomp = h->nx;
  cv.sign = 1.0;
  return launch(h, h->f_conv4, h->P.Z, &cv, s);
}

int source(sdc_handle h, const double* U, double* R, hipStream_t s) {
  if (h->P.cfg.space_order == 4) return source4(h, U, R, s);
  SourceArgs a{h->P.Z, U, R, h->d_params, h->P.cfg.gamma - 1.0};
  return launch(h, h->f_source, h->P.Z, &a, s);
}

bool nodes_ok(const sdc_handle h, const sdc_nodes* n, bool need_c) {
  for (int j = 0; j <= h->M; ++j)
    if (!n->U[j] || !n->A[j] || !n->R[j]) return false;
  if (need_c)
    for (int j = 0; j < h->M - 1; ++j)
      if (!n->C[j]) return false;
  return true;
}

// One node transition in the split schedule: the explicit-part kernels of
// the zone batches run in order on the auxiliary stream, each Newton batch on
// `s` waits for its own explicit part only, so batch i's Newton overlaps batch
// i+1's explicit part; the finish kernel follows the last batch.  With
// profiling on, the whole transition is timed as one span of its kind.
int split_transition(sdc_handle h, int kind, TransArgs a, hipStream_t s) {
  if (int rc = ensure_split(h)) return rc;
  const int64_t Z = h->P.Z, nb = h->split;
  const int64_t B = (Z + nb - 1) / nb;
  a.split = h->split_buf;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool prof = h->profile;
  if (prof) {
    e0 = take_event(h);
    e1 = take_event(h);
    if (!e0 || !e1) return fail(h, SDC_ERR_HIP, "hipEventCreate failed");
    HIP_CHECK(h, hipEventRecord(e0, s));
  }
  HIP_CHECK(h, hipEventRecord(h->fork_ev, s));
  HIP_CHECK(h, hipStreamWaitEvent(h->aux, h->fork_ev, 0));
  int64_t n = 0;
  for (int64_t i = 0; i < nb && i * B < Z; ++i, ++n) {
    a.zbeg = i * B;
    a.zcount = std::min<int64_t>(B, Z - a.zbeg);
    if (int rc = launch(h, h->f_pre[kind], a.zcount, &a, h->aux)) return rc;
    HIP_CHECK(h, hipEventRecord(h->batch_ev[i], h->aux));
  }
  hipFunction_t fn = h->occ2 ? h->f_newton_o2 : h->f_newton;
  for (int64_t i = 0; i < n; ++i) {
    a.zbeg = i * B;
    a.zcount = std::min<int64_t>(B, Z - a.zbeg);
    HIP_CHECK(h, hipStreamWaitEvent(s, h->batch_ev[i], 0));
    if (int rc = launch(h, fn, a.zcount, &a, s)) return rc;
  }
  h->profile = false;  // the finish kernel is part of the span
  int rc = launch(h, h->f_trans_finish, std::min<int64_t>(Z, kFinishThreads), &a, s);
  h->profile = prof;
  if (rc) return rc;
  if (prof) {
    HIP_CHECK(h, hipEventRecord(e1, s));
    h->timed.push_back({SDC_K_TRANSITION_FIRST + kind, e0, e1});
  }
  return SDC_OK;
}

// Fourth-order transition m -> m+1: the rhs of Eq. 2 (zone averages) into
// the node's output array and the Newton guess into the workspace, the
// zone-centre Newton inputs, the per-zone solve (the sdc_reaction_solve
// kernels), then <R> = R_c + lap R_c / 24 and U^{m+1} = rhs + dt_m <R>.
int transition4(sdc_handle h, int kind, TransArgs a, hipStream_t s) {
  if (int rc = ensure_o4(h)) return rc;
  a.x4 = h->o4_x;
  if (int rc = launch(h, h->f_rhs4[kind], h->P.Z, &a, s)) return rc;
  O4Args o;
  std::memset(&o, 0, sizeof o);
  o.Z = h->P.Z;
  grid_extents(h, o.n);
  o.dtm = a.dtm;
  o.U = a.Uout;
  o.R = a.Rout;
  o.rho_c = h->o4_rho;
  o.b_c = h->o4_b;
  o.R_c = h->o4_R;
  if (int rc = launch(h, h->f_newin4, h->P.Z, &o, s)) return rc;
  SolveArgs v;
  std::memset(&v, 0, sizeof v);
  v.Z = h->P.Z;
  v.dtm = a.dtm;
  v.rho = h->o4_rho;
  v.b = h->o4_b;
  v.x = h->o4_x;
  v.R = h->o4_R;
  v.iters = h->o4_it;
  v.P = h->d_params;
  v.gm1 = h->P.cfg.gamma - 1.0;
  v.ctl = newton_ctl(h);
  v.stats = h->d_stats;
  v.q = h->q;
  if (int rc = reset_queue(h, s)) return rc;
  if (int rc = launch(h, h->occ2 ? h->f_solve_o2 : h->f_solve, h->P.Z, &v, s)) return rc;
  if (int rc = launch(h, h->f_solve_finish, std::min<int64_t>(h->P.Z, kFinishThreads), &v, s)) return rc;
  return launch(h, h->f_avgst4, h->P.Z, &o, s);
}

// Work a refined level inserts into a sweep: after each transition
// (node m's new state, before its advective term) and after that term.
struct SweepHooks {
  virtual int after_state(int node, const sdc_nodes& n, hipStream_t s) const = 0;
  virtual int after_advect(int node, const sdc_nodes& n, hipStream_t s) const = 0;
  virtual ~SweepHooks() = default;
};

// One iteration k -> k+1 over the M transitions, then A at node M.
int sweep(sdc_handle h, double dt, int k, const sdc_nodes& n, hipStream_t s, const SweepHooks* hooks = nullptr) {
  const int M = h->M;
  if (int rc = ensure_queue(h)) return rc;
  for (int m = 0; m < M; ++m) {
    TransArgs a;
    std::memset(&a, 0, sizeof a);
    a.Z = h->P.Z;
    a.m = m;
    a.M = M;
    a.first = k == 0;
    a.dt = dt;
    a.dtm = (h->tau[m + 1] - h->tau[m]) * dt;
    for (int i = 0; i < M; ++i) {
      for (int j = 0; j <= M; ++j) a.S[i][j] = h->S[i][j];
      a.dtj[i] = (h->tau[i + 1] - h->tau[i]) * dt;
    }
    a.Um = n.U[m];
    a.Am = n.A[m];
    for (int j = 0; j <= M; ++j) {
      a.Aold[j] = n.A[j];
      a.Rold[j] = n.R[j];
    }
    if (m >= 1 && k >= 1) a.Cin = n.C[m - 1];
    for (int j = 1; j < M; ++j) a.Cout[j - 1] = n.C[j - 1];
    a.guess = k == 0 ? n.U[0] : n.U[m + 1];
    a.Uout = n.U[m + 1];
    a.Rout = n.R[m + 1];
    a.P = h->d_params;
    a.gm1 = h->P.cfg.gamma - 1.0;
    a.ctl = newton_ctl(h);
    a.stats = h->d_stats;
    a.q = h->q;
    const int kind = k == 0 ? 0 : (m == 0 ? 1 : 2);
    int rc;
    if (h->P.cfg.space_order == 4) {
      if ((rc = transition4(h, kind, a, s))) return rc;
    } else if ((rc = reset_queue(h, s))) {
      return rc;
    } else if (h->split > 0 && !h->capturing) {
      if ((rc = split_transition(h, kind, a, s))) return rc;
    } else {
      hipFunction_t f = kind == 0 ? (h->occ2 ? h->f_first_o2 : h->f_first)
                                  : (kind == 1 ? (h->occ2 ? h->f_node0_o2 : h->f_node0)
                                               : (h->occ2 ? h->f_later_o2 : h->f_later));
      if ((rc = launch(h, f, h->P.Z, &a, s))) return rc;
      if ((rc = launch(h, h->f_trans_finish, std::min<int64_t>(h->P.Z, kFinishThreads), &a, s))) return rc;
    }
    if (hooks && (rc = hooks->after_state(m + 1, n, s))) return rc;
    if (h->P.cfg.advection) {
      rc = advect(h, n.U[m + 1], n.A[m + 1], s);
      if (rc) return rc;
      if (hooks && (rc = hooks->after_advect(m + 1, n, s))) return rc;
    }
  }
  return SDC_OK;
}

void drop_graphs(sdc_handle h) {
  for (auto& g : h->step_graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  h->graph_key.clear();
}

// Capture the K sweeps of one step with node 0 in n.U[0] into an executable
// graph.  Capture runs on the handle's own stream: nothing executes.
int capture_step(sdc_handle h, double dt, const sdc_nodes& n, hipGraphExec_t* out) {
  if (int rc = ensure_queue(h)) return rc;  // no allocation while capturing
  if (!h->capture_stream) HIP_CHECK(h, hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
  HIP_CHECK(h, hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
  int rc = SDC_OK;
  h->capturing = true;  // a captured step uses the fused transition kernels
  for (int k = 0; k < h->P.cfg.n_iters && rc == SDC_OK; ++k) rc = sweep(h, dt, k, n, h->capture_stream);
  h->capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->capture_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(h, SDC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, SDC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return SDC_OK;
}

// ---- adjoint
struct AdjWork {
  sdc_nodes F;                      // forward replay nodes
  double* Ust[8][SDC_MAX_NODES];    // node states of iteration k+1 (m = 1..M)
  double *Ub[SDC_MAX_NODES], *Ab[SDC_MAX_NODES], *Rb[SDC_MAX_NODES];  // [0] = node 0 adjoints
  double *Abo[SDC_MAX_NODES], *Rbo[SDC_MAX_NODES];                    // previous iteration
  double* part;                     // [nblocks][2 nreact]
};

int adjoint_workspace(sdc_handle h, AdjWork* W) {
  const int M = h->M, K = h->P.cfg.n_iters;
  const size_t zc = (size_t)h->nc * h->P.Z, zr = (size_t)h->nx * h->P.Z;
  const size_t nblk = (h->P.Z + kBlock - 1) / kBlock;
  std::vector<size_t> sizes;
  // F: U, A (zc) and R (zr) per node, C (zc) per inner node
  for (int j = 0; j <= M; ++j) {
    sizes.push_back(zc);
    sizes.push_back(zc);
    sizes.push_back(zr);
  }
  for (int j = 0; j < M - 1; ++j) sizes.push_back(zc);
  for (int k = 0; k < K; ++k)
    for (int m = 1; m <= M; ++m) sizes.push_back(zc);
  for (int j = 0; j <= M; ++j) {
    sizes.push_back(zc);  // Ub
    sizes.push_back(zc);  // Ab
    sizes.push_back(zr);  // Rb
    sizes.push_back(zc);  // Abo
    sizes.push_back(zr);  // Rbo
  }
  sizes.push_back(nblk * 2 * (size_t)h->nra);
  if (h->adj_buf.empty()) {
    for (size_t n : sizes) {
      double* p = nullptr;
      if (hipMalloc((void**)&p, n * sizeof(double)) != hipSuccess) {
        for (double* q : h->adj_buf) (void)hipFree(q);
        h->adj_buf.clear();
        return fail(h, SDC_ERR_NOMEM, "hipMalloc(adjoint workspace) failed");
      }
      h->adj_buf.push_back(p);
    }
  }
  size_t i = 0;
  std::memset(&W->F, 0, sizeof W->F);
  for (int j = 0; j <= M; ++j) {
    W->F.U[j] = h->adj_buf[i++];
    W->F.A[j] = h->adj_buf[i++];
    W->F.R[j] = h->adj_buf[i++];
  }
  for (int j = 0; j < M - 1; ++j) W->F.C[j] = h->adj_buf[i++];
  for (int k = 0; k < K; ++k)
    for (int m = 1; m <= M; ++m) W->Ust[k][m] = h->adj_buf[i++];
  for (int j = 0; j <= M; ++j) {
    W->Ub[j] = h->adj_buf[i++];
    W->Ab[j] = h->adj_buf[i++];
    W->Rb[j] = h->adj_buf[i++];
    W->Abo[j] = h->adj_buf[i++];
    W->Rbo[j] = h->adj_buf[i++];
  }
  W->part = h->adj_buf[i++];
  return SDC_OK;
}

int advect_vjp(sdc_handle h, const double* U, const double* Abar, double* Ubar, hipStream_t s) {
  const sdc_config& c = h->P.cfg;
  AdvVjpArgs a;
  std::memset(&a, 0, sizeof a);
  a.U = U;
  a.Abar = Abar;
  a.Ubar = Ubar;
  a.Z = h->P.Z;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = d < c.dim ? (int)c.n[d] : 1;
    a.idx[d] = d < c.dim ? 1.0 / c.dx[d] : 0.0;
  }
  a.gamma = c.gamma;
  a.alpha = c.alpha;
  return launch(h, h->f_advect_vjp, h->P.Z, &a, s);
}

// The arrays of one sdc_zero_list launch.  add() refuses entries beyond
// SDC_ZERO_MAX instead of writing past the argument block; zero_arrays()
// then reports the overflow and launches nothing.
struct ZeroList {
  ZeroListArgs a;
  bool overflow = false;
  ZeroList() { std::memset(&a, 0, sizeof a); }
  void add(double* p, int64_t n) {
    if (a.count >= SDC_ZERO_MAX) {
      overflow = true;
      return;
    }
    a.p[a.count] = p;
    a.n[a.count++] = n;
  }
};

int zero_arrays(sdc_handle h, ZeroList& z, int64_t longest, hipStream_t s) {
  if (z.overflow) return fail(h, SDC_ERR_UNSUPPORTED, "more arrays than one zeroing launch takes");
  return launch(h, h->f_zero_list, std::min<int64_t>(longest, int64_t(4096) * kBlock), &z.a, s);
}

int theta_reduce(sdc_handle h, const double* part, double* thetabar, hipStream_t s) {
  if (h->P.topo.nr == 0) return SDC_OK;
  ThetaReduceArgs a{part, (h->P.Z + kBlock - 1) / kBlock, 2 * h->P.topo.nr, thetabar};
  // one block per parameter
  return launch(h, h->f_theta_reduce, (int64_t)a.nparam * kBlock, &a, s);
}

int step_adjoint(sdc_handle h, double dt, const double* Un, const double* Ubar1, double* Ubar0, double* thetabar,
                 hipStream_t s) {
  const int M = h->M, K = h->P.cfg.n_iters;
  const int64_t zc = (int64_t)h->nc * h->P.Z, zr = (int64_t)h->nx * h->P.Z;
  AdjWork W;
  int rc = adjoint_workspace(h, &W);
  if (rc) return rc;
  // forward replay from U^n, keeping every iteration's node states
  HIP_CHECK(h, hipMemcpyAsync(W.F.U[0], Un, zc * sizeof(double), hipMemcpyDeviceToDevice, s));
  if ((rc = advect(h, W.F.U[0], W.F.A[0], s))) return rc;
  if ((rc = source(h, W.F.U[0], W.F.R[0], s))) return rc;
  if (!h->P.cfg.advection)
    for (int j = 1; j <= M; ++j)
      if ((rc = fill(h, W.F.A[j], zc, 0.0, s))) return rc;
  for (int k = 0; k < K; ++k) {
    if ((rc = sweep(h, dt, k, W.F, s))) return rc;
    for (int m = 1; m <= M; ++m)
      HIP_CHECK(h, hipMemcpyAsync(W.Ust[k][m], W.F.U[m], zc * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // reverse: 3 (M + 1) <= SDC_ZERO_MAX arrays in the first zeroing launch
  {
    ZeroList z;
    for (int j = 0; j <= M; ++j) {
      z.add(W.Ub[j], zc);
      z.add(W.Ab[j], zc);
      z.add(W.Rb[j], zr);
    }
    if ((rc = zero_arrays(h, z, zc, s))) return rc;
  }
  HIP_CHECK(h, hipMemcpyAsync(W.Ub[M], Ubar1, zc * sizeof(double), hipMemcpyDeviceToDevice, s));
  const bool adv = h->P.cfg.advection != 0;
  for (int k = K - 1; k >= 0; --k) {
    {
      ZeroList z;
      for (int j = 1; j <= M; ++j) {
        z.add(W.Abo[j], zc);
        z.add(W.Rbo[j], zr);
      }
      if ((rc = zero_arrays(h, z, zc, s))) return rc;
    }
    if (adv && (rc = advect_vjp(h, W.Ust[k][M], W.Ab[M], W.Ub[M], s))) return rc;
    for (int m = M - 1; m >= 0; --m) {
      TransAdjArgs a;
      std::memset(&a, 0, sizeof a);
      a.Z = h->P.Z;
      a.m = m;
      a.M = M;
      a.first = k == 0;
      a.dt = dt;
      a.dtm = (h->tau[m + 1] - h->tau[m]) * dt;
      for (int i = 0; i < M; ++i)
        for (int j = 0; j <= M; ++j) a.S[i][j] = h->S[i][j];
      a.Uout = W.Ust[k][m + 1];
      a.Uoutbar = W.Ub[m + 1];
      a.Routbar = W.Rb[m + 1];
      a.Umbar = W.Ub[m];
      a.Ambar = (k == 0 || m >= 1) ? W.Ab[m] : nullptr;
      for (int j = 0; j <= M; ++j) {
        a.Aoldbar[j] = j == 0 ? W.Ab[0] : W.Abo[j];
        a.Roldbar[j] = j == 0 ? W.Rb[0] : W.Rbo[j];
      }
      a.P = h->d_params;
      a.gm1 = h->P.cfg.gamma - 1.0;
      a.tau = h->P.cfg.pivot_threshold;
      a.theta_part = W.part;
      if ((rc = launch(h, k == 0 ? h->f_trans_adj_first : h->f_trans_adj, h->P.Z, &a, s))) return rc;
      if ((rc = theta_reduce(h, W.part, thetabar, s))) return rc;
      if (m >= 1 && adv && (rc = advect_vjp(h, W.Ust[k][m], W.Ab[m], W.Ub[m], s))) return rc;
    }
    // iteration k's node adjoints: the "old" accumulators; its states feed
    // only Newton guesses, so their adjoints restart from zero
    ZeroList z;
    for (int j = 1; j <= M; ++j) {
      std::swap(W.Ab[j], W.Abo[j]);
      std::swap(W.Rb[j], W.Rbo[j]);
      z.add(W.Ub[j], zc);
    }
    if ((rc = zero_arrays(h, z, zc, s))) return rc;
  }
  // node 0: U^n itself, A^0 = A(U^n), R^0 = R(U^n)
  HIP_CHECK(h, hipMemcpyAsync(Ubar0, W.Ub[0], zc * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (adv && (rc = advect_vjp(h, Un, W.Ab[0], Ubar0, s))) return rc;
  SourceVjpArgs sv{h->P.Z, Un, W.Rb[0], Ubar0, h->d_params, h->P.cfg.gamma - 1.0, W.part};
  if ((rc = launch(h, h->f_source_vjp, h->P.Z, &sv, s))) return rc;
  return theta_reduce(h, W.part, thetabar, s);
}

// ---- autotuning of the Newton schedule
std::string tune_path(const sdc_handle h) {
  const sdc_config& c = h->P.cfg;
  char name[128];
  std::snprintf(name, sizeof name, "tune4_%016llx_z%lld_k%d_a%d_s%d_n%d.txt", (unsigned long long)fnv1a(h->P.source),
                (long long)h->P.Z, (int)c.n_iters, (int)c.advection, (int)c.space_order, (int)c.node_type);
  return cache_dir() + "/" + name;
}

bool load_tuning(sdc_handle h) {
  std::ifstream f(tune_path(h));
  int o = -1, c = -1, sp = -1, zt = -1;
  if (!(f >> o >> c >> sp >> zt) || o < 0 || o > 1 || c < 0 || sp < 0 || sp > 64 || zt < 0 || zt > 1024)
    return false;
  h->occ2 = o;
  h->cap = c;
  h->split = sp;
  if (zt != h->zchunk) {
    h->zchunk = zt;
    if (upload_rows(h) != SDC_OK) return false;
  }
  h->tuned = true;
  return true;
}

int autotune(sdc_handle h, double dt, const double* U, const sdc_nodes& n, hipStream_t s) {
  const int64_t zc = (int64_t)h->nc * h->P.Z;
  int rc = ensure_queue(h);
  if (rc) return rc;
  unsigned long long saved[SDC_NSTATS];
  HIP_CHECK(h, hipStreamSynchronize(s));
  HIP_CHECK(h, hipMemcpy(saved, h->d_stats, sizeof saved, hipMemcpyDeviceToHost));
  HIP_CHECK(h, hipMemcpyAsync(n.U[0], U, zc * sizeof(double), hipMemcpyDeviceToDevice, s));
  if ((rc = advect(h, n.U[0], n.A[0], s)) || (rc = source(h, n.U[0], n.R[0], s))) return rc;
  if (!h->P.cfg.advection)
    for (int j = 1; j <= h->M; ++j)
      if ((rc = fill(h, n.A[j], zc, 0.0, s))) return rc;
  const bool prof = h->profile;
  h->profile = false;
  hipEvent_t e0, e1;
  HIP_CHECK(h, hipEventCreate(&e0));
  HIP_CHECK(h, hipEventCreate(&e1));
  // the split schedule is not searched: it moves more bytes and measured
  // slower than the fused kernels on the 3D workloads
  const int caps[] = {0, 2, 3, 4, 5, 6}, splits[] = {0};
  float best = 1e30f;
  int bo = 0, bc = 0, bs = 0;
  for (int rep = 0; rep < 2 && rc == SDC_OK; ++rep)  // the first pass warms caches and clocks
    for (int sp : splits)
    for (int o = 0; o < 2 && rc == SDC_OK; ++o)
      for (int c : caps) {
        h->occ2 = o;
        h->cap = c;
        h->split = sp;
        if ((rc = (hipEventRecord(e0, s) == hipSuccess ? SDC_OK : SDC_ERR_HIP))) break;
        for (int k = 0; k < h->P.cfg.n_iters && rc == SDC_OK; ++k) rc = sweep(h, dt, k, n, s);
        if (rc) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(h, SDC_ERR_HIP, "autotune event failed");
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        // the default schedule (tried first) is replaced only by one that is
        // faster by more than 1%, so equal variants do not flip between runs
        if (rep == 1 && ms < (o == 0 && c == 0 && sp == 0 ? best : 0.99f * best)) {
          best = ms;
          bo = o;
          bc = c;
          bs = sp;
        }
      }
  // the advection tile: planes per z chunk of the row kernel, timed on A(U^n)
  int bz = h->zchunk;
  if (rc == SDC_OK && h->f_advect_rows) {
    const int tiles[] = {0, 16, 32, 64, 128};
    float bestz = 1e30f;
    for (int rep = 0; rep < 2 && rc == SDC_OK; ++rep)
      for (int zt : tiles) {
        h->zchunk = zt;
        if ((rc = upload_rows(h))) break;
        if (hipEventRecord(e0, s) != hipSuccess) {
          rc = fail(h, SDC_ERR_HIP, "autotune event failed");
          break;
        }
        for (int i = 0; i < 3 && rc == SDC_OK; ++i) rc = advect(h, n.U[0], n.A[0], s);
        if (rc) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(h, SDC_ERR_HIP, "autotune event failed");
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep == 1 && ms < (zt == 0 ? bestz : 0.99f * bestz)) {
          bestz = ms;
          bz = zt;
        }
      }
    if (rc == SDC_OK && bz != h->zchunk) {
      h->zchunk = bz;
      rc = upload_rows(h);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->profile = prof;
  if (rc) return rc;
  h->occ2 = bo;
  h->cap = bc;
  h->split = bs;
  h->tuned = true;
  drop_graphs(h);
  HIP_CHECK(h, hipMemcpy(h->d_stats, saved, sizeof saved, hipMemcpyHostToDevice));
  const std::string path = tune_path(h);
  std::string text = std::to_string(bo) + " " + std::to_string(bc) + " " + std::to_string(bs) + " " +
                     std::to_string(bz) + "\n";
  std::vector<char> data(text.begin(), text.end());
  const auto k = path.rfind('/');
  write_file_atomic(path.substr(0, k), path.substr(k + 1), data);
  return SDC_OK;
}

int check_handle(sdc_handle h) {
  if (!h) return fail(nullptr, SDC_ERR_ARG, "null handle");
  return SDC_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

int sdc_config_default(sdc_config* cfg) {
  if (!cfg) return SDC_ERR_ARG;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->dim = 1;
  cfg->n[0] = cfg->n[1] = cfg->n[2] = 1;
  cfg->dx[0] = cfg->dx[1] = cfg->dx[2] = 1.0;
  cfg->gamma = 1.4;
  cfg->n_nodes = 3;
  cfg->n_iters = 4;
  cfg->precision = SDC_FP64;
  cfg->advection = 1;
  cfg->slope = 1;
  cfg->alpha = -1.0;
  cfg->newton_tol = 1e-13;
  cfg->newton_maxiter = 50;
  cfg->pivot_threshold = 0.1;
  cfg->nbox = 0;
  cfg->box_n = nullptr;
  cfg->graph = 0;
  cfg->autotune = 0;
  cfg->node_type = SDC_NODES_LOBATTO;
  cfg->space_order = 2;
  return SDC_OK;
}

int64_t sdc_generated_source(const sdc_config* cfg, const sdc_network* net, char* buf, int64_t len) {
  Prepared P;
  std::string err;
  int rc = prepare(cfg, net, &P, &err);
  if (rc) {
    g_init_error = err;
    return -rc;
  }
  const int64_t need = (int64_t)P.source.size() + 1;
  if (buf && len > 0) {
    const int64_t n = need < len ? need : len;
    std::memcpy(buf, P.source.c_str(), (size_t)n - 1);
    buf[n - 1] = '\0';
  }
  return need;
}

int64_t sdc_aot_name(const sdc_config* cfg, const sdc_network* net, char* buf, int64_t len) {
  Prepared P;
  std::string err;
  int rc = prepare(cfg, net, &P, &err);
  if (rc) {
    g_init_error = err;
    return -rc;
  }
  const std::string name = cache_dir() + "/" + aot_name(P.source);
  const int64_t need = (int64_t)name.size() + 1;
  if (buf && len > 0) {
    const int64_t n = need < len ? need : len;
    std::memcpy(buf, name.c_str(), (size_t)n - 1);
    buf[n - 1] = '\0';
  }
  return need;
}

int sdc_compile_only(const sdc_config* cfg, const sdc_network* net) {
  Prepared P;
  std::string err;
  int rc = prepare(cfg, net, &P, &err);
  if (rc) return fail(nullptr, rc, err);
  std::vector<char> code;
  rc = get_code_object(P.source, &code, &err);
  if (rc) return fail(nullptr, rc, err);
  return SDC_OK;
}

int sdc_init(const sdc_config* cfg, const sdc_network* net, sdc_handle* out) {
  if (!out) return fail(nullptr, SDC_ERR_ARG, "null output handle");
  *out = nullptr;
  auto* h = new (std::nothrow) sdc_handle_s;
  if (!h) return fail(nullptr, SDC_ERR_NOMEM, "host allocation failed");
  std::string err;
  int rc = prepare(cfg, net, &h->P, &err);
  if (rc) {
    delete h;
    return fail(nullptr, rc, err);
  }
  h->ns = h->P.topo.ns;
  h->nc = 2 + h->P.cfg.dim + h->ns;
  h->nx = h->ns + 1;
  h->M = h->P.cfg.n_nodes - 1;
  h->nra = h->P.topo.nr > 0 ? h->P.topo.nr : 1;
  const bool radau = h->P.cfg.node_type == SDC_NODES_RADAU;
  h->tau = radau ? radau_nodes(h->P.cfg.n_nodes) : lobatto_nodes(h->P.cfg.n_nodes);
  h->S = integration_matrix(h->tau, radau ? 1 : 0);
  std::vector<char> code;
  rc = get_code_object(h->P.source, &code, &err);
  if (rc) {
    delete h;
    return fail(nullptr, rc, err);
  }
  auto bail = [&](int code_, const std::string& msg) {
    sdc_destroy(h);
    return fail(nullptr, code_, msg);
  };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  h->scratch = scratch_address(h->device, &h->scratch_rc);
  e = hipModuleLoadData(&h->mod, code.data());
  if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
  struct {
    hipFunction_t* f;
    const char* name;
  } fns[] = {{&h->f_advect, "sdc_advect"},         {&h->f_source, "sdc_source"},
             {&h->f_solve, "sdc_reaction_solve"},  {&h->f_first, "sdc_transition_first"},
             {&h->f_node0, "sdc_transition_node0"}, {&h->f_later, "sdc_transition_later"},
             {&h->f_fill, "sdc_fill"}, {&h->f_zero_list, "sdc_zero_list"}, {&h->f_advect_vjp, "sdc_advect_vjp"},
             {&h->f_trans_adj_first, "sdc_transition_adjoint_first"}, {&h->f_trans_adj, "sdc_transition_adjoint"},
             {&h->f_source_vjp, "sdc_source_vjp"}, {&h->f_theta_reduce, "sdc_theta_reduce"},
             {&h->f_axpy, "sdc_axpy"}, {&h->f_first_o2, "sdc_transition_first_o2"},
             {&h->f_node0_o2, "sdc_transition_node0_o2"}, {&h->f_later_o2, "sdc_transition_later_o2"},
             {&h->f_trans_finish, "sdc_transition_finish"}, {&h->f_solve_o2, "sdc_reaction_solve_o2"},
             {&h->f_pre[0], "sdc_transition_pre_first"}, {&h->f_pre[1], "sdc_transition_pre_node0"},
             {&h->f_pre[2], "sdc_transition_pre_later"}, {&h->f_newton, "sdc_transition_newton"},
             {&h->f_newton_o2, "sdc_transition_newton_o2"},
             {&h->f_solve_finish, "sdc_reaction_finish"}, {&h->f_reset, "sdc_reset_counter"}};
  for (auto& fn : fns) {
    e = hipModuleGetFunction(fn.f, h->mod, fn.name);
    if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("missing kernel ") + fn.name);
  }
  // 3D grids with rows of at most 512 zones and state arrays below 4 GiB
  // (32-bit buffer offsets) use the row kernel, in 512-thread blocks when a
  // row is longer than 256 zones (SDC_ADVECT_ROWS=0: the zone-per-thread
  // kernel everywhere)
  const char* ev = std::getenv("SDC_ADVECT_ROWS");
  {
    // fourth-order kernels (the flux and divergence kernels exist per direction)
    const char* f4[] = {"sdc_flux4_0", "sdc_flux4_1", "sdc_flux4_2"};
    const char* d4[] = {"sdc_div4_0", "sdc_div4_1", "sdc_div4_2"};
    const char* a4[] = {"sdc_faceavg4_0", "sdc_faceavg4_1", "sdc_faceavg4_2"};
    for (int d = 0; d < h->P.cfg.dim; ++d) {
      if (hipModuleGetFunction(&h->f_flux4[d], h->mod, f4[d]) != hipSuccess ||
          hipModuleGetFunction(&h->f_favg4[d], h->mod, a4[d]) != hipSuccess ||
          hipModuleGetFunction(&h->f_div4[d], h->mod, d4[d]) != hipSuccess)
        return bail(SDC_ERR_HIP, std::string("missing kernel ") + f4[d]);
    }
    struct {
      hipFunction_t* f;
      const char* name;
    } f4s[] = {{&h->f_conv4, "sdc_convert4"},     {&h->f_source4c, "sdc_source4_centre"},
               {&h->f_rhs4[0], "sdc_rhs4_first"}, {&h->f_rhs4[1], "sdc_rhs4_node0"},
               {&h->f_rhs4[2], "sdc_rhs4_later"}, {&h->f_newin4, "sdc_newton_inputs4"},
               {&h->f_avgst4, "sdc_average_store4"}};
    for (auto& fn : f4s)
      if (hipModuleGetFunction(fn.f, h->mod, fn.name) != hipSuccess)
        return bail(SDC_ERR_HIP, std::string("missing kernel ") + fn.name);
  }
  if (h->P.cfg.advection && h->P.cfg.space_order == 2 && rows_kernel_fits(h->P) && !(ev && ev[0] == '0')) {
    h->row_bw = longest_row(h->P) > kBlock ? 512 : kBlock;
    const bool wide = h->row_bw > kBlock;
    const char* name = h->P.cfg.slope == 0 ? (wide ? "sdc_advect_rows_wc" : "sdc_advect_rows_c")
                                           : (wide ? "sdc_advect_rows_w" : "sdc_advect_rows");
    e = hipModuleGetFunction(&h->f_advect_rows, h->mod, name);
    if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("missing kernel ") + name);
    if (upload_rows(h) != SDC_OK) return bail(SDC_ERR_NOMEM, "row descriptors: " + h->err);
  }
  const std::vector<double> img = params_image(h->P, h->nra);
  e = hipMalloc(&h->d_params, img.size() * sizeof(double));
  if (e != hipSuccess) return bail(SDC_ERR_NOMEM, "hipMalloc(params) failed");
  e = hipMemcpy(h->d_params, img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("hipMemcpy(params): ") + hipGetErrorString(e));
  if (h->P.cfg.nbox > 0) {
    const int nbox = h->P.cfg.nbox;
    const int64_t nblk = (h->P.Z + kBlock - 1) / kBlock;
    std::vector<int32_t> blk(nblk);
    int bx = 0;
    for (int64_t q = 0; q < nblk; ++q) {
      while (q * kBlock >= h->P.box_off[bx + 1]) ++bx;
      blk[q] = bx;
    }
    if (hipMalloc((void**)&h->d_box_off, (nbox + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void**)&h->d_box_ext, 3 * nbox * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&h->d_blk_box, nblk * sizeof(int32_t)) != hipSuccess)
      return bail(SDC_ERR_NOMEM, "hipMalloc(box tables) failed");
    if (hipMemcpy(h->d_box_off, h->P.box_off.data(), (nbox + 1) * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_box_ext, h->P.box_ext.data(), 3 * nbox * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_blk_box, blk.data(), nblk * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
      return bail(SDC_ERR_HIP, "hipMemcpy(box tables) failed");
  }
  e = hipMalloc((void**)&h->d_stats, SDC_NSTATS * sizeof(unsigned long long));
  if (e != hipSuccess) return bail(SDC_ERR_NOMEM, "hipMalloc(stats) failed");
  e = hipMemset(h->d_stats, 0, SDC_NSTATS * sizeof(unsigned long long));
  if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("hipMemset(stats): ") + hipGetErrorString(e));
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return bail(SDC_ERR_HIP, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
  *out = h;
  return SDC_OK;
}

int sdc_destroy(sdc_handle h) {
  if (!h) return SDC_OK;
  if (h->last_stream) (void)hipStreamSynchronize(h->last_stream);
  (void)hipDeviceSynchronize();
  for (auto& t : h->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  drop_graphs(h);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  for (double* p : h->adj_buf) (void)hipFree(p);
  free_queue(h);
  free_split(h);
  free_o4(h);
  if (h->d_params) (void)hipFree(h->d_params);
  if (h->d_box_off) (void)hipFree(h->d_box_off);
  if (h->d_box_ext) (void)hipFree(h->d_box_ext);
  if (h->d_blk_box) (void)hipFree(h->d_blk_box);
  if (h->d_rows) (void)hipFree(h->d_rows);
  if (h->d_stats) (void)hipFree(h->d_stats);
  if (h->mod) (void)hipModuleUnload(h->mod);
  delete h;
  return SDC_OK;
}

const char* sdc_last_error(sdc_handle h) { return h ? h->err.c_str() : g_init_error.c_str(); }

int sdc_sizes(sdc_handle h, int64_t* zones, int32_t* ncomp, int32_t* nreact_vars) {
  if (int rc = check_handle(h)) return rc;
  if (zones) *zones = h->P.Z;
  if (ncomp) *ncomp = h->nc;
  if (nreact_vars) *nreact_vars = h->nx;
  return SDC_OK;
}

int sdc_advective_term(sdc_handle h, const double* U, double* A, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!U || !A) return fail(h, SDC_ERR_ARG, "null array");
  if (U == A) return fail(h, SDC_ERR_ARG, "U and A must not alias");
  h->last_stream = (hipStream_t)stream;
  return advect(h, U, A, (hipStream_t)stream);
}

int sdc_source(sdc_handle h, const double* U, double* R, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!U || !R) return fail(h, SDC_ERR_ARG, "null array");
  h->last_stream = (hipStream_t)stream;
  return source(h, U, R, (hipStream_t)stream);
}

int sdc_reaction_solve(sdc_handle h, double dt_m, const double* rho, const double* b, double* x, double* R,
                       int32_t* iters, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!rho || !b || !x || !R || !iters) return fail(h, SDC_ERR_ARG, "null array");
  if (!std::isfinite(dt_m) || dt_m < 0.0) return fail(h, SDC_ERR_ARG, "dt_m must be finite and >= 0");
  if ((const double*)x == b) return fail(h, SDC_ERR_ARG, "x and b must not alias");
  h->last_stream = (hipStream_t)stream;
  SolveArgs a;
  std::memset(&a, 0, sizeof a);
  a.Z = h->P.Z;
  a.dtm = dt_m;
  a.rho = rho;
  a.b = b;
  a.x = x;
  a.R = R;
  a.iters = iters;
  a.P = h->d_params;
  a.gm1 = h->P.cfg.gamma - 1.0;
  a.ctl = newton_ctl(h);
  a.stats = h->d_stats;
  if (int rc = ensure_queue(h)) return rc;
  a.q = h->q;
  hipStream_t s = (hipStream_t)stream;
  if (int rc = reset_queue(h, s)) return rc;
  if (int rc = launch(h, h->occ2 ? h->f_solve_o2 : h->f_solve, h->P.Z, &a, s)) return rc;
  return launch(h, h->f_solve_finish, std::min<int64_t>(h->P.Z, kFinishThreads), &a, s);
}

int sdc_reaction_solve_noalloc(sdc_handle h, double dt_m, int64_t nzones, const double* rho, const double* b,
                               double* x, double* R, int32_t* iters, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (nzones < 0) return fail(h, SDC_ERR_ARG, "nzones must be >= 0");
  if (nzones == 0) return SDC_OK;
  if (!rho || !b || !x || !R || !iters) return fail(h, SDC_ERR_ARG, "null array");
  if (!std::isfinite(dt_m) || dt_m < 0.0) return fail(h, SDC_ERR_ARG, "dt_m must be finite and >= 0");
  if ((const double*)x == b) return fail(h, SDC_ERR_ARG, "x and b must not alias");
  if (!h->scratch)
    return fail(h, SDC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(h->scratch_rc));
  SolveArgs a;
  std::memset(&a, 0, sizeof a);
  if (carve_queue((unsigned char*)h->scratch, SDC_NOALLOC_SCRATCH_BYTES, nzones, h->nx, &a.q) < 0) {
    const int64_t per = 8 + 4 + 16 * (int64_t)h->nx + 8 + 8;
    return fail(h, SDC_ERR_ARG, "nzones = " + std::to_string(nzones) + " exceeds the scratch array of " +
                                    std::to_string((long long)SDC_NOALLOC_SCRATCH_BYTES) + " bytes (about " +
                                    std::to_string((SDC_NOALLOC_SCRATCH_BYTES - 2048) / per) + " zones at " +
                                    std::to_string(h->nx) + " reacting components)");
  }
  h->last_stream = (hipStream_t)stream;
  a.Z = nzones;
  a.dtm = dt_m;
  a.rho = rho;
  a.b = b;
  a.x = x;
  a.R = R;
  a.iters = iters;
  a.P = h->d_params;
  a.gm1 = h->P.cfg.gamma - 1.0;
  a.ctl = newton_ctl(h);
  a.stats = h->d_stats;
  // plain launches: no profiling events, no allocation of any kind
  hipStream_t s = (hipStream_t)stream;
  void* reset_params[] = {&a.q.count};
  HIP_CHECK(h, hipModuleLaunchKernel(h->f_reset, 1, 1, 1, 64, 1, 1, 0, s, reset_params, nullptr));
  void* params[] = {&a};
  const unsigned nb = (unsigned)((nzones + kBlock - 1) / kBlock);
  HIP_CHECK(h, hipModuleLaunchKernel(h->occ2 ? h->f_solve_o2 : h->f_solve, nb, 1, 1, kBlock, 1, 1, 0, s, params,
                                     nullptr));
  const unsigned nf = (unsigned)((std::min<int64_t>(nzones, kFinishThreads) + kBlock - 1) / kBlock);
  HIP_CHECK(h, hipModuleLaunchKernel(h->f_solve_finish, nf, 1, 1, kBlock, 1, 1, 0, s, params, nullptr));
  return SDC_OK;
}

int sdc_sweep(sdc_handle h, double dt, int32_t k, const sdc_nodes* nodes, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!nodes || k < 0) return fail(h, SDC_ERR_ARG, "null nodes or negative k");
  if (!std::isfinite(dt) || dt <= 0.0) return fail(h, SDC_ERR_ARG, "dt must be positive");
  if (!nodes_ok(h, nodes, k >= 1 && h->M >= 2)) return fail(h, SDC_ERR_ARG, "missing node arrays");
  h->last_stream = (hipStream_t)stream;
  return sweep(h, dt, k, *nodes, (hipStream_t)stream);
}

int sdc_step(sdc_handle h, double dt, int32_t nsteps, double* U, const sdc_nodes* work, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!U || !work || nsteps < 0) return fail(h, SDC_ERR_ARG, "null U/work or negative nsteps");
  if (!std::isfinite(dt) || dt <= 0.0) return fail(h, SDC_ERR_ARG, "dt must be positive");
  if (!nodes_ok(h, work, h->P.cfg.n_iters >= 2 && h->M >= 2)) return fail(h, SDC_ERR_ARG, "missing node arrays");
  for (int j = 0; j <= h->M; ++j)
    if (work->U[j] == U) return fail(h, SDC_ERR_ARG, "work arrays must not alias U");
  if (nsteps == 0) return SDC_OK;
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  sdc_nodes n = *work;
  const size_t bytesU = (size_t)h->nc * h->P.Z * sizeof(double);
  if (h->P.cfg.autotune && !h->tuned && !load_tuning(h))
    if (int rc = autotune(h, dt, U, n, s)) return rc;
  HIP_CHECK(h, hipMemcpyAsync(n.U[0], U, bytesU, hipMemcpyDeviceToDevice, s));
  int rc = advect(h, n.U[0], n.A[0], s);
  if (rc) return rc;
  rc = source(h, n.U[0], n.R[0], s);
  if (rc) return rc;
  if (!h->P.cfg.advection)
    for (int j = 1; j <= h->M; ++j)
      if ((rc = fill(h, n.A[j], (int64_t)h->nc * h->P.Z, 0.0, s))) return rc;
  const bool use_graph = h->P.cfg.graph && !h->profile;
  if (use_graph) {
    // key: dt and every work pointer; a change re-captures both phases
    std::vector<uintptr_t> key;
    uint64_t dtbits;
    std::memcpy(&dtbits, &dt, sizeof dt);
    key.push_back((uintptr_t)dtbits);
    for (int j = 0; j < SDC_MAX_NODES; ++j) {
      key.push_back((uintptr_t)n.U[j]);
      key.push_back((uintptr_t)n.A[j]);
      key.push_back((uintptr_t)n.R[j]);
    }
    for (int j = 0; j < SDC_MAX_NODES - 2; ++j) key.push_back((uintptr_t)n.C[j]);
    if (key != h->graph_key) {
      drop_graphs(h);
      sdc_nodes swapped = n;
      std::swap(swapped.U[0], swapped.U[h->M]);
      std::swap(swapped.A[0], swapped.A[h->M]);
      std::swap(swapped.R[0], swapped.R[h->M]);
      if ((rc = capture_step(h, dt, n, &h->step_graph[0]))) return rc;
      if ((rc = capture_step(h, dt, swapped, &h->step_graph[1]))) return rc;
      h->graph_key = key;
    }
  }
  for (int step = 0; step < nsteps; ++step) {
    if (use_graph) {
      HIP_CHECK(h, hipGraphLaunch(h->step_graph[step & 1], s));
    } else {
      for (int k = 0; k < h->P.cfg.n_iters; ++k)
        if ((rc = sweep(h, dt, k, n, s))) return rc;
    }
    // the last node becomes node 0 of the next step
    std::swap(n.U[0], n.U[h->M]);
    std::swap(n.A[0], n.A[h->M]);
    std::swap(n.R[0], n.R[h->M]);
  }
  HIP_CHECK(h, hipMemcpyAsync(U, n.U[0], bytesU, hipMemcpyDeviceToDevice, s));
  return SDC_OK;
}

int sdc_step_adjoint(sdc_handle h, double dt, const double* U_n, const double* Ubar_np1, double* Ubar_n,
                     double* thetabar, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!U_n || !Ubar_np1 || !Ubar_n || (!thetabar && h->P.topo.nr > 0))
    return fail(h, SDC_ERR_ARG, "null array");
  if (!std::isfinite(dt) || dt <= 0.0) return fail(h, SDC_ERR_ARG, "dt must be positive");
  if ((const double*)Ubar_n == Ubar_np1 || (const double*)Ubar_n == U_n)
    return fail(h, SDC_ERR_ARG, "Ubar_n must not alias U_n or Ubar_np1");
  const sdc_config& c = h->P.cfg;
  if (c.nbox > 0) return fail(h, SDC_ERR_UNSUPPORTED, "the adjoint supports single grids only");
  if (c.space_order != 2) return fail(h, SDC_ERR_UNSUPPORTED, "the adjoint supports the second-order method only");
  if (c.advection && !(c.slope == 0 && c.alpha > 0.0))
    return fail(h, SDC_ERR_UNSUPPORTED, "the adjoint needs the smooth mode: slope 0 and a frozen alpha > 0");
  if (c.n_iters > 8) return fail(h, SDC_ERR_UNSUPPORTED, "the adjoint supports up to 8 SDC iterations");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  return step_adjoint(h, dt, U_n, Ubar_np1, Ubar_n, thetabar, s);
}

int sdc_set_schedule(sdc_handle h, int32_t occ2, int32_t cap, int32_t split, int32_t zchunk) {
  if (int rc = check_handle(h)) return rc;
  if (occ2 < 0 || occ2 > 1 || cap < 0 || split < 0 || split > 64 || zchunk < 0 || zchunk > 1024)
    return fail(h, SDC_ERR_ARG, "occ2 must be 0 or 1, cap >= 0, 0 <= split <= 64 and 0 <= zchunk <= 1024");
  if (zchunk != h->zchunk) {
    if (h->last_stream) HIP_CHECK(h, hipStreamSynchronize(h->last_stream));  // descriptors in use
    h->zchunk = zchunk;
    if (int rc = upload_rows(h)) return rc;
  }
  h->occ2 = occ2;
  h->cap = cap;
  h->split = split;
  h->tuned = true;
  drop_graphs(h);
  return SDC_OK;
}

int sdc_get_schedule(sdc_handle h, int32_t* occ2, int32_t* cap, int32_t* split, int32_t* zchunk) {
  if (int rc = check_handle(h)) return rc;
  if (occ2) *occ2 = h->occ2;
  if (cap) *cap = h->cap;
  if (split) *split = h->split;
  if (zchunk) *zchunk = h->zchunk;
  return SDC_OK;
}

int sdc_autotune(sdc_handle h, double dt, const double* U, const sdc_nodes* work, void* stream) {
  if (int rc = check_handle(h)) return rc;
  if (!U || !work) return fail(h, SDC_ERR_ARG, "null U or work");
  if (!std::isfinite(dt) || dt <= 0.0) return fail(h, SDC_ERR_ARG, "dt must be positive");
  if (!nodes_ok(h, work, h->P.cfg.n_iters >= 2 && h->M >= 2)) return fail(h, SDC_ERR_ARG, "missing node arrays");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  return autotune(h, dt, U, *work, s);
}

int sdc_stats(sdc_handle h, int64_t* out) {
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(h, SDC_ERR_ARG, "null output");
  if (h->last_stream) HIP_CHECK(h, hipStreamSynchronize(h->last_stream));
  HIP_CHECK(h, hipDeviceSynchronize());
  unsigned long long tmp[SDC_NSTATS];
  HIP_CHECK(h, hipMemcpy(tmp, h->d_stats, sizeof tmp, hipMemcpyDeviceToHost));
  for (int i = 0; i < SDC_NSTATS; ++i) out[i] = (int64_t)tmp[i];
  return SDC_OK;
}

int sdc_check(sdc_handle h) {
  int64_t st[SDC_NSTATS];
  if (int rc = sdc_stats(h, st)) return rc;
  const std::string counts = std::to_string(st[SDC_STAT_FAILED]) + " of " + std::to_string(st[SDC_STAT_SOLVES]) +
                             " solves unconverged, " + std::to_string(st[SDC_STAT_NONFINITE]) + " non-finite";
  if (st[SDC_STAT_NONFINITE] > 0) return fail(h, SDC_ERR_NONFINITE, counts);
  if (st[SDC_STAT_FAILED] > 0) return fail(h, SDC_ERR_NEWTON, counts);
  return SDC_OK;
}

int sdc_stats_reset(sdc_handle h, void* stream) {
  if (int rc = check_handle(h)) return rc;
  h->last_stream = (hipStream_t)stream;
  HIP_CHECK(h, hipMemsetAsync(h->d_stats, 0, SDC_NSTATS * sizeof(unsigned long long), (hipStream_t)stream));
  return SDC_OK;
}

int sdc_set_params(sdc_handle h, const double* lnA, const double* E) {
  if (int rc = check_handle(h)) return rc;
  const int nr = h->P.topo.nr;
  if (nr > 0 && (!lnA || !E)) return fail(h, SDC_ERR_ARG, "null parameter array");
  for (int r = 0; r < nr; ++r)
    if (!std::isfinite(lnA[r]) || !std::isfinite(E[r])) return fail(h, SDC_ERR_ARG, "non-finite parameter");
  h->P.lnA.assign(lnA, lnA + nr);
  h->P.E.assign(E, E + nr);
  const std::vector<double> img = params_image(h->P, h->nra);
  if (h->last_stream) HIP_CHECK(h, hipStreamSynchronize(h->last_stream));
  HIP_CHECK(h, hipMemcpy(h->d_params, img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice));
  return SDC_OK;
}

int sdc_profile_enable(sdc_handle h, int32_t enable) {
  if (int rc = check_handle(h)) return rc;
  h->profile = enable != 0;
  return SDC_OK;
}

int sdc_profile_read(sdc_handle h, double* ms, int64_t* launches) {
  if (int rc = check_handle(h)) return rc;
  if (!ms || !launches) return fail(h, SDC_ERR_ARG, "null output");
  for (int k = 0; k < SDC_NKINDS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto& t : h->timed) {
    HIP_CHECK(h, hipEventSynchronize(t.b));
    float v = 0.0f;
    HIP_CHECK(h, hipEventElapsedTime(&v, t.a, t.b));
    ms[t.kind] += v;
    launches[t.kind] += 1;
    h->event_pool.push_back(t.a);
    h->event_pool.push_back(t.b);
  }
  h->timed.clear();
  return SDC_OK;
}

int sdc_cost_model(sdc_handle h, int64_t* out) {
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(h, SDC_ERR_ARG, "null output");
  const sdcgen::FlopCount f = sdcgen::count_flops(h->P.topo, h->P.pat);
  out[0] = f.source;
  out[1] = f.residual_matrix;
  out[2] = f.lu;
  out[3] = f.solve;
  out[4] = f.exps;
  out[5] = h->P.pat.nnz_jac;
  out[6] = h->P.pat.nnz;
  return SDC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- refined patches
// Two-level hierarchy around the SDC step: a periodic coarse handle and a
// handle over the padded patches (batched boxes, each box a patch refined by
// 2 with 2 ghost zones per side).  A coarse step: the coarse level steps; each
// patch takes two steps of dt/2 with ghost zones filled from the coarse node
// states before every evaluation of A and A zeroed in the ghost zones; the
// time-integrated fluxes through the coarse-fine faces are accumulated on both
// levels during the last sweep; then refluxing and average-down.

struct sdc_amr_s {
  sdc_handle c = nullptr, f = nullptr;
  int dim = 1, M = 1;
  std::vector<int64_t> lo, ext;        // [np][3]
  std::vector<int64_t> fbase;          // zone offset of each padded patch
  sdc_nodes nc{}, nf{};                // node arrays of both levels (owned)
  std::vector<double*> bufs;
  AmrGhost* d_ghost = nullptr;
  int64_t nghost = 0;
  AmrFace *d_facec = nullptr, *d_facef = nullptr;
  int64_t nfacec = 0, nfacef = 0;
  double *regc = nullptr, *regf = nullptr;
  AmrReflux* d_reflux = nullptr;
  int64_t nreflux = 0;
  AmrCover* d_cover = nullptr;
  int64_t ncover = 0;
  hipFunction_t f_fill = nullptr, f_zero = nullptr, f_flux = nullptr, f_reflux = nullptr, f_average = nullptr;
};

namespace {

constexpr int kRatio = 2, kGhost = 2;

template <class T>
int upload(sdc_handle h, const std::vector<T>& v, T** out) {
  if (v.empty()) return SDC_OK;
  if (hipMalloc((void**)out, v.size() * sizeof(T)) != hipSuccess)
    return fail(h, SDC_ERR_NOMEM, "hipMalloc(hierarchy tables) failed");
  HIP_CHECK(h, hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return SDC_OK;
}

int amr_alloc_nodes(sdc_amr a, sdc_handle h, sdc_nodes* n) {
  std::memset(n, 0, sizeof *n);
  const size_t Z = (size_t)h->P.Z;
  auto get = [&](int comps, double** p) {
    if (hipMalloc((void**)p, comps * Z * sizeof(double)) != hipSuccess) return false;
    a->bufs.push_back(*p);
    return true;
  };
  for (int j = 0; j <= h->M; ++j)
    if (!get(h->nc, &n->U[j]) || !get(h->nc, &n->A[j]) || !get(h->nx, &n->R[j]))
      return fail(h, SDC_ERR_NOMEM, "hipMalloc(hierarchy node arrays) failed");
  for (int j = 0; j + 1 < h->M; ++j)
    if (!get(h->nc, &n->C[j])) return fail(h, SDC_ERR_NOMEM, "hipMalloc(hierarchy node arrays) failed");
  return SDC_OK;
}

// Lagrange weights of the node times tau at theta.
void lagrange(const std::vector<double>& tau, double theta, double* w) {
  for (size_t i = 0; i < tau.size(); ++i) {
    w[i] = 1.0;
    for (size_t j = 0; j < tau.size(); ++j)
      if (j != i) w[i] *= (theta - tau[j]) / (tau[i] - tau[j]);
  }
}

int amr_launch(sdc_handle h, hipFunction_t f, int64_t n, void* args, hipStream_t s) { return launch(h, f, n, args, s); }

// Fill the ghost zones (or, all_zones, every zone) of the fine array U at
// coarse-step fraction theta from the coarse node states.
int amr_fill(sdc_amr a, double* U, double theta, hipStream_t s) {
  AmrFillArgs f;
  std::memset(&f, 0, sizeof f);
  f.Uf = U;
  for (int j = 0; j <= a->M; ++j) f.Uc[j] = a->nc.U[j];
  lagrange(a->c->tau, theta, f.w);
  f.nnodes = a->M + 1;
  f.list = a->d_ghost;
  f.count = a->nghost;
  f.Zc = a->c->P.Z;
  f.Zf = a->f->P.Z;
  for (int d = 0; d < 3; ++d) f.nc[d] = d < a->dim ? (int)a->c->P.cfg.n[d] : 1;
  return amr_launch(a->c, a->f_fill, a->nghost, &f, s);
}

int amr_zero(sdc_amr a, double* A, hipStream_t s) {
  AmrFillArgs f;
  std::memset(&f, 0, sizeof f);
  f.Uf = A;
  f.list = a->d_ghost;
  f.count = a->nghost;
  f.Zf = a->f->P.Z;
  return amr_launch(a->c, a->f_zero, a->nghost, &f, s);
}

int amr_flux(sdc_amr a, sdc_handle h, const double* U, double* reg, const AmrFace* faces, int64_t n, double coef,
             hipStream_t s) {
  if (!h->P.cfg.advection || n == 0 || coef == 0.0) return SDC_OK;
  AmrFluxArgs f;
  std::memset(&f, 0, sizeof f);
  f.U = U;
  f.reg = reg;
  f.faces = faces;
  f.count = n;
  f.Z = h->P.Z;
  f.coef = coef;
  f.gamma = h->P.cfg.gamma;
  f.alpha = h->P.cfg.alpha;
  f.slope = h->P.cfg.slope;
  return amr_launch(a->c, a->f_flux, n, &f, s);
}

// Ghost fills and ghost-zone A of a patch sweep in substep `sub`.
struct PatchHooks : SweepHooks {
  sdc_amr a;
  int sub;
  PatchHooks(sdc_amr a_, int s_) : a(a_), sub(s_) {}
  int after_state(int node, const sdc_nodes& n, hipStream_t s) const override {
    return amr_fill(a, n.U[node], (sub + a->f->tau[node]) / kRatio, s);
  }
  int after_advect(int node, const sdc_nodes& n, hipStream_t s) const override { return amr_zero(a, n.A[node], s); }
};

// One SDC step of a level from U into its node arrays, with the flux
// register accumulated in the last sweep:
//   reg += dt sum_j w_j F(U^{j,(K-1)}) + sum_{m=1}^{M-1} dt_m (F(U^{m,(K)}) - F(U^{m,(K-1)})).
int amr_level_step(sdc_amr a, sdc_handle h, const sdc_nodes& n, const double* U, double dt, const SweepHooks* hooks,
                   double* reg, const AmrFace* faces, int64_t nfaces, hipStream_t s) {
  const size_t bytes = (size_t)h->nc * h->P.Z * sizeof(double);
  HIP_CHECK(h, hipMemcpyAsync(n.U[0], U, bytes, hipMemcpyDeviceToDevice, s));
  int rc;
  if (hooks && (rc = hooks->after_state(0, n, s))) return rc;
  if ((rc = advect(h, n.U[0], n.A[0], s))) return rc;
  if (hooks && h->P.cfg.advection && (rc = hooks->after_advect(0, n, s))) return rc;
  if ((rc = source(h, n.U[0], n.R[0], s))) return rc;
  if (!h->P.cfg.advection)
    for (int j = 1; j <= h->M; ++j)
      if ((rc = fill(h, n.A[j], (int64_t)h->nc * h->P.Z, 0.0, s))) return rc;
  const int K = h->P.cfg.n_iters, M = h->M;
  std::vector<double> w(M + 1, 0.0), dtm(M, 0.0);
  for (int m = 0; m < M; ++m) {
    dtm[m] = (h->tau[m + 1] - h->tau[m]) * dt;
    for (int j = 0; j <= M; ++j) w[j] += h->S[m][j];
  }
  for (int k = 0; k < K; ++k) {
    if (k == K - 1) {
      for (int j = 0; j <= M; ++j) {
        const double coef = dt * w[j] - (j >= 1 && j < M ? dtm[j] : 0.0);
        if ((rc = amr_flux(a, h, k == 0 ? n.U[0] : n.U[j], reg, faces, nfaces, coef, s))) return rc;
      }
    }
    if ((rc = sweep(h, dt, k, n, s, hooks))) return rc;
  }
  for (int m = 1; m < M; ++m)
    if ((rc = amr_flux(a, h, n.U[m], reg, faces, nfaces, dtm[m], s))) return rc;
  return SDC_OK;
}

}  // namespace

extern "C" {

int sdc_amr_create(const sdc_config* coarse, const sdc_network* net, const sdc_patches* patches, sdc_amr* out) {
  if (!out || !coarse || !net || !patches) return fail(nullptr, SDC_ERR_ARG, "null argument");
  *out = nullptr;
  const sdc_config& cc = *coarse;
  if (cc.nbox != 0 || cc.space_order != 2 || cc.dim < 1 || cc.dim > 3)
    return fail(nullptr, SDC_ERR_UNSUPPORTED, "a hierarchy needs a single periodic coarse grid and space_order 2");
  const int np = patches->npatch, dim = cc.dim;
  if (np < 1 || !patches->lo || !patches->ext) return fail(nullptr, SDC_ERR_ARG, "need at least one patch");
  for (int p = 0; p < np; ++p)
    for (int d = 0; d < dim; ++d) {
      const int64_t l = patches->lo[3 * p + d], e = patches->ext[3 * p + d];
      if (e < 1 || l < 0 || l + e > cc.n[d]) return fail(nullptr, SDC_ERR_ARG, "patch must lie inside the coarse grid");
      if (e + 2 > cc.n[d])
        return fail(nullptr, SDC_ERR_ARG, "a patch must leave two coarse zones uncovered along every direction");
    }
  for (int p = 0; p < np; ++p)
    for (int q = p + 1; q < np; ++q) {
      // gaps of two or more coarse zones on both sides of the periodic grid,
      // along some direction, so that every coarse zone next to a patch is
      // uncovered (its reflux target)
      bool apart = false;
      for (int d = 0; d < dim; ++d) {
        const int64_t lp = patches->lo[3 * p + d], ep = patches->ext[3 * p + d];
        const int64_t lq = patches->lo[3 * q + d], eq = patches->ext[3 * q + d], n = cc.n[d];
        apart = apart || (lp + ep + 2 <= lq && lq + eq + 2 <= lp + n) || (lq + eq + 2 <= lp && lp + ep + 2 <= lq + n);
      }
      if (!apart) return fail(nullptr, SDC_ERR_ARG, "patches must be two or more coarse zones apart");
    }
  auto* a = new (std::nothrow) sdc_amr_s;
  if (!a) return fail(nullptr, SDC_ERR_NOMEM, "host allocation failed");
  a->dim = dim;
  a->lo.assign(patches->lo, patches->lo + 3 * np);
  a->ext.assign(patches->ext, patches->ext + 3 * np);
  int rc = sdc_init(coarse, net, &a->c);
  if (rc) {
    delete a;
    return rc;
  }
  // the fine handle: the padded patches as batched boxes, half the zone width
  std::vector<int64_t> box(3 * np, 1);
  for (int p = 0; p < np; ++p)
    for (int d = 0; d < dim; ++d) box[3 * p + d] = kRatio * a->ext[3 * p + d] + 2 * kGhost;
  sdc_config fc = cc;
  for (int d = 0; d < 3; ++d) fc.dx[d] = cc.dx[d] / kRatio;
  fc.nbox = np;
  fc.box_n = box.data();
  fc.graph = 0;
  auto bail = [&](int code) {
    sdc_amr_destroy(a);
    return code;
  };
  if ((rc = sdc_init(&fc, net, &a->f))) {
    const std::string msg = g_init_error;
    sdc_amr_destroy(a);
    return fail(nullptr, rc, "fine level: " + msg);
  }
  sdc_handle c = a->c, f = a->f;
  a->M = c->M;
  a->fbase.assign(f->P.box_off.begin(), f->P.box_off.end() - 1);
  struct {
    hipFunction_t* fn;
    const char* name;
  } fns[] = {{&a->f_fill, "sdc_amr_fill"}, {&a->f_zero, "sdc_amr_zero"}, {&a->f_flux, "sdc_amr_flux"},
             {&a->f_reflux, "sdc_amr_reflux"}, {&a->f_average, "sdc_amr_average"}};
  for (auto& fn : fns)
    if (hipModuleGetFunction(fn.fn, c->mod, fn.name) != hipSuccess) {
      fail(nullptr, SDC_ERR_HIP, std::string("missing kernel ") + fn.name);
      return bail(SDC_ERR_HIP);
    }
  int ncx[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) ncx[d] = (int)cc.n[d];
  // ghost zones, coarse and fine interface faces, reflux and cover tables
  std::vector<AmrGhost> ghost;
  std::vector<AmrFace> facec, facef;
  std::vector<AmrReflux> reflux;
  std::vector<AmrCover> cover;
  for (int p = 0; p < np; ++p) {
    int nb[3] = {1, 1, 1};
    for (int d = 0; d < 3; ++d) nb[d] = (int)box[3 * p + d];
    const int64_t base = a->fbase[p];
    for (int k = 0; k < nb[2]; ++k)
      for (int j = 0; j < nb[1]; ++j)
        for (int i = 0; i < nb[0]; ++i) {
          const int fi[3] = {i, j, k};
          bool inner = true;
          AmrGhost g;
          g.zf = base + i + (int64_t)nb[0] * (j + (int64_t)nb[1] * k);
          g.sig = 0;
          for (int d = 0; d < 3; ++d) {
            g.pc[d] = 0;
            if (d >= dim) continue;
            inner = inner && fi[d] >= kGhost && fi[d] < nb[d] - kGhost;
            const int64_t gl = kRatio * a->lo[3 * p + d] + (fi[d] - kGhost);  // global fine index
            int64_t par = gl >= 0 ? gl / kRatio : -((-gl + kRatio - 1) / kRatio);
            if (gl - kRatio * par != 0) g.sig |= 1 << d;
            par %= ncx[d];
            if (par < 0) par += ncx[d];
            g.pc[d] = (int)par;
          }
          if (!inner) ghost.push_back(g);
        }
    // interface faces: per direction and side, every transverse position
    for (int d = 0; d < dim; ++d) {
      const int64_t l = a->lo[3 * p + d], e = a->ext[3 * p + d];
      const double h = cc.dx[d];
      int t1 = -1, t2 = -1;  // transverse directions, ascending
      for (int t = 0; t < dim; ++t)
        if (t != d) (t1 < 0 ? t1 : t2) = t;
      const int64_t n1 = t1 >= 0 ? a->ext[3 * p + t1] : 1, n2 = t2 >= 0 ? a->ext[3 * p + t2] : 1;
      for (int side = 0; side < 2; ++side)
        for (int64_t b2 = 0; b2 < n2; ++b2)
          for (int64_t b1 = 0; b1 < n1; ++b1) {
            AmrFace cf;
            std::memset(&cf, 0, sizeof cf);
            cf.base = 0;
            for (int t = 0; t < 3; ++t) cf.n[t] = ncx[t];
            cf.d = d;
            int64_t ci = side == 0 ? l - 1 : l + e - 1;  // coarse zone whose i+1/2 face it is
            ci = ((ci % ncx[d]) + ncx[d]) % ncx[d];
            cf.c[d] = (int)ci;
            if (t1 >= 0) cf.c[t1] = (int)(a->lo[3 * p + t1] + b1);
            if (t2 >= 0) cf.c[t2] = (int)(a->lo[3 * p + t2] + b2);
            AmrReflux r;
            std::memset(&r, 0, sizeof r);
            r.fc = (int64_t)facec.size();
            facec.push_back(cf);
            int uz[3] = {cf.c[0], cf.c[1], cf.c[2]};
            uz[d] = (int)(side == 0 ? ((l - 1) % ncx[d] + ncx[d]) % ncx[d] : (l + e) % ncx[d]);
            r.zu = uz[0] + (int64_t)ncx[0] * (uz[1] + (int64_t)ncx[1] * uz[2]);
            r.sign = side == 0 ? -1.0 : 1.0;
            r.h = h;
            // the fine faces over it: pairs along t1 (inner) then t2
            int q = 0;
            for (int s2 = 0; s2 < (t2 >= 0 ? kRatio : 1); ++s2)
              for (int s1 = 0; s1 < (t1 >= 0 ? kRatio : 1); ++s1) {
                AmrFace ff;
                std::memset(&ff, 0, sizeof ff);
                ff.base = base;
                for (int t = 0; t < 3; ++t) ff.n[t] = nb[t];
                ff.d = d;
                ff.c[d] = side == 0 ? kGhost - 1 : kGhost + (int)(kRatio * e) - 1;
                if (t1 >= 0) ff.c[t1] = kGhost + (int)(kRatio * b1) + s1;
                if (t2 >= 0) ff.c[t2] = kGhost + (int)(kRatio * b2) + s2;
                r.ff[q++] = (int64_t)facef.size();
                facef.push_back(ff);
              }
            reflux.push_back(r);
          }
    }
    // covered coarse zones and their first fine zone
    const int64_t e0 = a->ext[3 * p], e1 = dim > 1 ? a->ext[3 * p + 1] : 1, e2 = dim > 2 ? a->ext[3 * p + 2] : 1;
    for (int64_t k = 0; k < e2; ++k)
      for (int64_t j = 0; j < e1; ++j)
        for (int64_t i = 0; i < e0; ++i) {
          AmrCover cv;
          const int64_t ci = a->lo[3 * p] + i, cj = dim > 1 ? a->lo[3 * p + 1] + j : 0,
                        ck = dim > 2 ? a->lo[3 * p + 2] + k : 0;
          cv.zc = ci + (int64_t)ncx[0] * (cj + (int64_t)ncx[1] * ck);
          const int64_t fi = kGhost + kRatio * i, fj = dim > 1 ? kGhost + kRatio * j : 0,
                        fk = dim > 2 ? kGhost + kRatio * k : 0;
          cv.sy = nb[0];
          cv.sz = (int64_t)nb[0] * nb[1];
          cv.f0 = base + fi + cv.sy * fj + cv.sz * fk;
          cover.push_back(cv);
        }
  }
  // every table entry inside its arrays (the kernels index with them unchecked)
  {
    const int64_t Zc = c->P.Z, Zf = f->P.Z, nfc = (int64_t)facec.size(), nff = (int64_t)facef.size();
    bool ok = true;
    for (const AmrGhost& g : ghost) {
      ok = ok && g.zf >= 0 && g.zf < Zf;
      for (int d = 0; d < 3; ++d) ok = ok && g.pc[d] >= 0 && g.pc[d] < ncx[d];
    }
    auto face_ok = [&](const AmrFace& fa, int64_t Z, bool wrap) {
      int64_t vol = 1;
      bool r = fa.base >= 0;
      for (int d = 0; d < 3; ++d) {
        r = r && fa.c[d] >= 0 && fa.c[d] < fa.n[d] && fa.n[d] >= 1;
        vol *= fa.n[d];
      }
      r = r && fa.d >= 0 && fa.d < dim && fa.base + vol <= Z && fa.n[fa.d] >= 2;
      if (!wrap) r = r && fa.c[fa.d] - 1 >= 0 && fa.c[fa.d] + 2 < fa.n[fa.d];
      return r;
    };
    for (const AmrFace& fa : facec) ok = ok && face_ok(fa, Zc, true);
    for (const AmrFace& fa : facef) ok = ok && face_ok(fa, Zf, false);
    for (const AmrReflux& r : reflux) {
      ok = ok && r.zu >= 0 && r.zu < Zc && r.fc >= 0 && r.fc < nfc;
      for (int q = 0; q < (1 << (dim - 1)); ++q) ok = ok && r.ff[q] >= 0 && r.ff[q] < nff;
    }
    for (const AmrCover& cv : cover)
      ok = ok && cv.zc >= 0 && cv.zc < Zc && cv.f0 >= 0 &&
           cv.f0 + (dim > 2 ? cv.sz : 0) + (dim > 1 ? cv.sy : 0) + 1 < Zf;
    if (!ok) {
      fail(nullptr, SDC_ERR_ARG, "hierarchy tables out of range");
      return bail(SDC_ERR_ARG);
    }
  }
  a->nghost = (int64_t)ghost.size();
  a->nfacec = (int64_t)facec.size();
  a->nfacef = (int64_t)facef.size();
  a->nreflux = (int64_t)reflux.size();
  a->ncover = (int64_t)cover.size();
  if ((rc = upload(c, ghost, &a->d_ghost)) || (rc = upload(c, facec, &a->d_facec)) ||
      (rc = upload(c, facef, &a->d_facef)) || (rc = upload(c, reflux, &a->d_reflux)) ||
      (rc = upload(c, cover, &a->d_cover))) {
    g_init_error = c->err;
    return bail(rc);
  }
  if (hipMalloc((void**)&a->regc, std::max<int64_t>(1, a->nfacec) * c->nc * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&a->regf, std::max<int64_t>(1, a->nfacef) * c->nc * sizeof(double)) != hipSuccess) {
    fail(nullptr, SDC_ERR_NOMEM, "hipMalloc(flux registers) failed");
    return bail(SDC_ERR_NOMEM);
  }
  if ((rc = amr_alloc_nodes(a, c, &a->nc)) || (rc = amr_alloc_nodes(a, f, &a->nf))) {
    g_init_error = rc == SDC_ERR_NOMEM ? "hipMalloc(hierarchy node arrays) failed" : c->err;
    return bail(rc);
  }
  *out = a;
  return SDC_OK;
}

int sdc_amr_destroy(sdc_amr a) {
  if (!a) return SDC_OK;
  (void)hipDeviceSynchronize();
  for (double* p : a->bufs) (void)hipFree(p);
  for (void* p : {(void*)a->d_ghost, (void*)a->d_facec, (void*)a->d_facef, (void*)a->regc, (void*)a->regf,
                  (void*)a->d_reflux, (void*)a->d_cover})
    if (p) (void)hipFree(p);
  sdc_destroy(a->f);
  sdc_destroy(a->c);
  delete a;
  return SDC_OK;
}

int sdc_amr_sizes(sdc_amr a, int64_t* zc, int64_t* zf) {
  if (!a) return SDC_ERR_ARG;
  if (zc) *zc = a->c->P.Z;
  if (zf) *zf = a->f->P.Z;
  return SDC_OK;
}

int sdc_amr_handles(sdc_amr a, sdc_handle* coarse, sdc_handle* fine) {
  if (!a) return SDC_ERR_ARG;
  if (coarse) *coarse = a->c;
  if (fine) *fine = a->f;
  return SDC_OK;
}

int sdc_amr_fill_patches(sdc_amr a, const double* Uc, double* Uf, void* stream) {
  if (!a) return SDC_ERR_ARG;
  if (!Uc || !Uf) return fail(a->c, SDC_ERR_ARG, "null array");
  hipStream_t s = (hipStream_t)stream;
  a->c->last_stream = s;
  // every fine zone takes the interpolated coarse state: the ghost list
  // covers ghost zones only, so fill with a list of all zones built here
  std::vector<AmrGhost> all;
  const int np = (int)a->fbase.size();
  int ncx[3] = {1, 1, 1};
  for (int d = 0; d < a->dim; ++d) ncx[d] = (int)a->c->P.cfg.n[d];
  for (int p = 0; p < np; ++p) {
    int nb[3] = {1, 1, 1};
    for (int d = 0; d < a->dim; ++d) nb[d] = (int)(kRatio * a->ext[3 * p + d] + 2 * kGhost);
    for (int k = 0; k < nb[2]; ++k)
      for (int j = 0; j < nb[1]; ++j)
        for (int i = 0; i < nb[0]; ++i) {
          const int fi[3] = {i, j, k};
          AmrGhost g;
          g.zf = a->fbase[p] + i + (int64_t)nb[0] * (j + (int64_t)nb[1] * k);
          g.sig = 0;
          for (int d = 0; d < 3; ++d) {
            g.pc[d] = 0;
            if (d >= a->dim) continue;
            const int64_t gl = kRatio * a->lo[3 * p + d] + (fi[d] - kGhost);
            int64_t par = gl >= 0 ? gl / kRatio : -((-gl + kRatio - 1) / kRatio);
            if (gl - kRatio * par != 0) g.sig |= 1 << d;
            par = ((par % ncx[d]) + ncx[d]) % ncx[d];
            g.pc[d] = (int)par;
          }
          all.push_back(g);
        }
  }
  AmrGhost* d_all = nullptr;
  if (int rc = upload(a->c, all, &d_all)) return rc;
  AmrFillArgs f;
  std::memset(&f, 0, sizeof f);
  f.Uf = Uf;
  f.Uc[0] = Uc;
  f.w[0] = 1.0;
  f.nnodes = 1;
  f.list = d_all;
  f.count = (int64_t)all.size();
  f.Zc = a->c->P.Z;
  f.Zf = a->f->P.Z;
  for (int d = 0; d < 3; ++d) f.nc[d] = ncx[d];
  int rc = amr_launch(a->c, a->f_fill, f.count, &f, s);
  if (hipStreamSynchronize(s) != hipSuccess && rc == SDC_OK) rc = fail(a->c, SDC_ERR_HIP, "fill failed");
  (void)hipFree(d_all);
  return rc;
}

int sdc_amr_step(sdc_amr a, double dt, int32_t nsteps, double* Uc, double* Uf, void* stream) {
  if (!a) return SDC_ERR_ARG;
  sdc_handle c = a->c, f = a->f;
  if (!Uc || !Uf || nsteps < 0) return fail(c, SDC_ERR_ARG, "null state or negative nsteps");
  if (!std::isfinite(dt) || dt <= 0.0) return fail(c, SDC_ERR_ARG, "dt must be positive");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = f->last_stream = s;
  const size_t bc = (size_t)c->nc * c->P.Z * sizeof(double), bf = (size_t)f->nc * f->P.Z * sizeof(double);
  int rc;
  // autotune = 1: the coarse level's Newton schedule (cached on disk or
  // tuned on Uc) serves both levels
  if (nsteps > 0 && c->P.cfg.autotune && !c->tuned && !load_tuning(c)) {
    if ((rc = autotune(c, dt, Uc, a->nc, s))) return rc;
  }
  f->occ2 = c->occ2;
  f->cap = c->cap;
  for (int step = 0; step < nsteps; ++step) {
    if ((rc = fill(c, a->regc, a->nfacec * c->nc, 0.0, s)) || (rc = fill(c, a->regf, a->nfacef * c->nc, 0.0, s)))
      return rc;
    // coarse level: one step, its node states kept for the ghost fills
    if ((rc = amr_level_step(a, c, a->nc, Uc, dt, nullptr, a->regc, a->d_facec, a->nfacec, s))) return rc;
    // patches: two substeps of dt / 2
    for (int sub = 0; sub < kRatio; ++sub) {
      PatchHooks hooks(a, sub);
      if ((rc = amr_level_step(a, f, a->nf, Uf, dt / kRatio, &hooks, a->regf, a->d_facef, a->nfacef, s))) return rc;
      HIP_CHECK(f, hipMemcpyAsync(Uf, a->nf.U[a->M], bf, hipMemcpyDeviceToDevice, s));
    }
    // synchronisation: reflux the uncovered neighbours, average down
    AmrSyncArgs y;
    std::memset(&y, 0, sizeof y);
    y.Uc = a->nc.U[a->M];
    y.Uf = Uf;
    y.regc = a->regc;
    y.regf = a->regf;
    y.Zc = c->P.Z;
    y.Zf = f->P.Z;
    y.nregc = a->nfacec;
    y.nregf = a->nfacef;
    y.reflux = a->d_reflux;
    y.nreflux = c->P.cfg.advection ? a->nreflux : 0;
    y.cover = a->d_cover;
    y.ncover = a->ncover;
    if ((rc = amr_launch(c, a->f_reflux, y.nreflux, &y, s)) || (rc = amr_launch(c, a->f_average, y.ncover, &y, s)))
      return rc;
    HIP_CHECK(c, hipMemcpyAsync(Uc, a->nc.U[a->M], bc, hipMemcpyDeviceToDevice, s));
  }
  return SDC_OK;
}

}  // extern "C"
