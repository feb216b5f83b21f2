// libwcamg: C ABI entry points and the solver orchestration (V-cycle, setup,
// outer FGMRES) on top of the HIP kernels.  All device work is issued on the
// context's stream; host synchronisation happens only where a host decision
// needs device data (Givens rotations of FGMRES, coarse-solve early exit
// outside graph capture) or at the end of synchronous calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <fstream>
#include <sstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/wcamg.h"
#include "wc_kernels.h"

using namespace wc;
using cd = std::complex<double>;

namespace {

struct WcError : std::runtime_error {
  int code;
  WcError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) {                                                                      \
      /* reset the thread's last-error state so that a failed allocation is */                   \
      /* not reported again by the next launch check                         */                  \
      (void)hipGetLastError();                                                                   \
      throw WcError(e_ == hipErrorOutOfMemory ? WCAMG_ENOMEM : WCAMG_EHIP,                       \
                    std::string(#x) + ": " + hipGetErrorString(e_));                              \
    }                                                                                            \
  } while (0)

void require(bool c, const std::string& m, int code = WCAMG_EINVAL) {
  if (!c) throw WcError(code, m);
}

// Incremented whenever any device buffer of the library is allocated,
// reallocated or freed: captured graphs hold raw addresses and are replayed
// only while this count is unchanged since their capture.
static std::atomic<unsigned long long> g_alloc_epoch{0};

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) {
      ++g_alloc_epoch;
      (void)hipFree(p);
    }
  }
  void* ensure(size_t bytes, bool frozen) {
    if (bytes <= n) return p;
    require(!frozen, "internal: workspace growth during graph capture or a no-allocation call", WCAMG_ESTATE);
    ++g_alloc_epoch;
    if (p) HIPCHK(hipFree(p));
    p = nullptr;
    n = 0;
    HIPCHK(hipMalloc(&p, bytes));
    n = bytes;
    return p;
  }
  void release() {
    ++g_alloc_epoch;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

struct Hier {
  int prec = -1;  // WCAMG_PREC_*
  int nv = 0, N = 0;
  CGeo cg{};
  int sap_sweeps = 4, mr_iters = 6, coarse_iters = 50;
  int smoothing = WCAMG_SMOOTH_POST;
  int sap_eo = 0;  // even-odd preconditioned SAP block solve
  double coarse_tol = 0.1;
  DevBuf V;   // stored test vectors [nv][12][V]
  DevBuf Dc;  // [NC][9][N][N]
  // optional level 1 (three-level hierarchy): blocks of the coarse lattice
  bool l1 = false;
  int nw = 0, N2 = 0, b1[4] = {1, 1, 1, 1};
  int mr1_iters = 4;
  CGeo cg2{};
  DevBuf W;    // level-1 test vectors [nw][NC][N]
  DevBuf Dc2;  // [NC2][9][N2][N2]
};

// a coarse operator: lattice, dof per site, stencil blocks
struct COp {
  CGeo cg;
  int N;
  void* Dc;
  size_t n() const { return (size_t)cg.NC * N; }
};

struct KStat {
  double ms = 0, bytes = 0, flops = 0, units = 0;
  int count = 0;
};

// sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] in the chiral basis, as its two
// diagonal 2x2 blocks per plane (mu<nu), [6][2][2][2][re,im].
std::vector<double> sigma_table() {
  cd I(0, 1);
  cd g[4][4][4] = {};
  // gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, -1], [-1, 0]]
  cd s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g[k][a][2 + b] = -I * s[k][a][b];
        g[k][2 + a][b] = I * s[k][a][b];
      }
  for (int a = 0; a < 2; ++a) {
    g[3][a][2 + a] = -1;
    g[3][2 + a][a] = -1;
  }
  std::vector<double> t(6 * 2 * 2 * 2 * 2);
  int pl = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++pl) {
      cd sg[4][4];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          cd c = 0;
          for (int k = 0; k < 4; ++k) c += g[mu][a][k] * g[nu][k][b] - g[nu][a][k] * g[mu][k][b];
          sg[a][b] = 0.5 * I * c;
        }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          if (std::abs(sg[a][2 + b]) > 1e-14 || std::abs(sg[2 + a][b]) > 1e-14)
            throw WcError(WCAMG_EHIP, "internal: sigma not block diagonal");
      for (int ch = 0; ch < 2; ++ch)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            cd v = sg[2 * ch + a][2 * ch + b];
            size_t o = ((((size_t)pl * 2 + ch) * 2 + a) * 2 + b) * 2;
            t[o] = v.real();
            t[o + 1] = v.imag();
          }
    }
  return t;
}

// Launch-variant autotuner.  The first time a key (kernel, shapes,
// precision, architecture) is seen, every candidate variant is timed with HIP
// events on the real operands (all variants compute identical results: they
// change workgroup shapes or staging only, never the order of a sum) and the
// fastest is kept; choices persist in a flat JSON file {"key": variant, ...}.
struct Tuner {
  bool enabled = true;
  std::string path;
  std::map<std::string, int> best;
  double tune_ms = 0;
  int tuned = 0;

  // merge the entries of the cache file p (if any) into the table, then
  // write the merged table back: the file always lists every known key
  void load(const std::string& p) {
    path = p;
    read(p);
    save();
  }
  void read(const std::string& p) {
    std::ifstream f(p);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string txt = ss.str();
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
      size_t j = txt.find('"', i + 1);
      if (j == std::string::npos) break;
      std::string key = txt.substr(i + 1, j - i - 1);
      size_t c = txt.find(':', j);
      if (c == std::string::npos) break;
      best[key] = std::atoi(txt.c_str() + c + 1);
      i = txt.find_first_of(",}", c);
      if (i == std::string::npos) break;
    }
  }
  void save() const {
    if (path.empty()) return;
    std::ofstream f(path);
    if (!f) return;
    f << "{";
    bool first = true;
    for (auto& kv : best) {
      f << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": " << kv.second;
      first = false;
    }
    f << "\n}\n";
  }
};

}  // namespace

struct wcamg_ctx {
  Geo g{};
  double kappa = 0, csw = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  bool have_gauge = false;
  DevBuf U64, U16, Cl64, Cl16;
  // the FP16 hop matrices of the hops that leave each SAP domain, in face
  // order (launch_face_links), for the mixed SAP's crossing-hop correction
  DevBuf FL16;
  // FP32 copies of the links and clover, made on first use by the comparison
  // solver's inner BiCGStab (single-precision fields, as the paper's)
  DevBuf U32, Cl32;
  bool have_f32 = false;
  // FP16 (1 + F)^-1 - 1, made on first use by the even-odd preconditioned
  // SAP block solve
  DevBuf Mi16;
  bool have_minv = false;
  Hier h;
  bool have_hier = false;
  std::map<std::string, std::unique_ptr<DevBuf>> ws;
  std::string err;
  bool capturing = false;
  // inside wcamg_apply_D_noalloc: no tuning runs, no timing events, and any
  // workspace growth is an error
  bool no_alloc = false;
  void* scratch = nullptr;  // this device's no-allocation scratch area (device address)
  // kernel timing
  bool timing = false;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes, flops, units;
  };
  int timing_excl = 0;  // > 0 inside an exclusive scope: inner scopes are not recorded
  std::vector<Pending> pending;
  std::vector<hipEvent_t> evpool;
  std::map<std::string, KStat> kstats;
  // graphs: key (slot, nrhs) -> exec
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  int graph_prec = -1;
  unsigned long long graph_epoch = 0;  // g_alloc_epoch when the graphs were captured
  std::vector<double> graph_sig;        // hierarchy parameters the graphs were captured with
  hipStream_t cap_st = nullptr;  // library-owned stream used for graph capture
  size_t lds_max = 0;            // LDS bytes available to one workgroup
  Tuner tuner;
  std::string arch;
  // equivariant network for initial test vectors
  struct Net {
    int L = 0, C = 0, t = 0;
    DevBuf W, m, v, grad, part;
    std::vector<void*> acts;  // L+1 activation fields [C][12][V] (FP32)
  } net;
  std::vector<std::unique_ptr<DevBuf>> net_act_bufs;
  size_t net_wsize() const { return (size_t)net.L * 9 * net.C * net.C * 16; }

  // forward pass from C input fields (FP32 [C][12][V]); activations kept for backward
  void net_forward(const void* r) {
    size_t fb = (size_t)net.C * 12 * g.V * sizeof(float2);
    while ((int)net_act_bufs.size() < net.L + 1) net_act_bufs.emplace_back(new DevBuf());
    net.acts.resize(net.L + 1);
    for (int l = 0; l <= net.L; ++l) net.acts[l] = net_act_bufs[l]->ensure(fb, capturing);
    HIPCHK(hipMemcpyAsync(net.acts[0], r, fb, hipMemcpyDeviceToDevice, st));
    size_t ws = (size_t)9 * net.C * net.C * 16;
    for (int l = 0; l < net.L; ++l)
      launch_ptc(g, (const float2*)net.W.p + l * ws, (const float2*)net.acts[l], (float2*)net.acts[l + 1],
                 (const double2*)U64.p, 0, st);
  }

  // subspace loss of the last activation against the teacher Q (FP32 [C][12][V])
  // and its gradient into net.grad; returns the loss (synchronises)
  double net_loss_backward(const void* Q) {
    int C = net.C;
    size_t fb = (size_t)C * 12 * g.V * sizeof(float2);
    size_t rs = (size_t)g.nblk * 2 * C;
    double2* G = (double2*)W("nt_G", (size_t)C * rs * sizeof(double2));
    double2* B = (double2*)W("nt_B", (size_t)C * rs * sizeof(double2));
    float2* cq = (float2*)W("nt_cq", (size_t)C * rs * sizeof(float2));
    float2* ca = (float2*)W("nt_ca", (size_t)C * rs * sizeof(float2));
    double* lp = (double*)W("nt_lp", (size_t)2 * g.nblk * sizeof(double));
    float2* ga = (float2*)W("nt_ga", fb);
    float2* gb = (float2*)W("nt_gb", fb);
    const void* A = net.acts[net.L];
    launch_restrict(g, C, C, A, C64, A, C64, frs(), G, C128, rs, 2 * C, 1, st);
    launch_restrict(g, C, C, A, C64, Q, C64, frs(), B, C128, rs, 2 * C, 1, st);
    launch_net_loss_coef(g.nblk, G, B, rs, 1.0 / (C * 2.0 * g.nblk), cq, ca, lp, st);
    launch_prolong(g, C, C, Q, C64, cq, C64, rs, 2 * C, ga, C64, frs(), 0, 1, st);
    launch_prolong(g, C, C, A, C64, ca, C64, rs, 2 * C, ga, C64, frs(), 1, 1, st);
    size_t ws = (size_t)9 * C * C * 16;
    int nwg = ptc_wgrad_nwg(g);
    net.part.ensure((size_t)nwg * ws * sizeof(float2), capturing);
    float2* gcur = ga;
    float2* gnext = gb;
    for (int l = net.L - 1; l >= 0; --l) {
      launch_ptc_wgrad(g, gcur, (const float2*)net.acts[l], (const double2*)U64.p, (float2*)net.part.p,
                       (float2*)net.grad.p + l * ws, st);
      if (l > 0) {
        launch_ptc(g, (const float2*)net.W.p + l * ws, gcur, gnext, (const double2*)U64.p, 1, st);
        std::swap(gcur, gnext);
      }
    }
    std::vector<double> hl(2 * g.nblk);
    HIPCHK(hipMemcpyAsync(hl.data(), lp, hl.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double loss = 0;
    for (double v : hl) loss += v;
    return loss / hl.size();
  }

  // pick the fastest of `cands` for `key` (runs each on the real operands
  // when the key is new and no graph is being captured)
  int tune(const std::string& key0, const std::vector<int>& cands, const std::function<void(int)>& run) {
    if (cands.size() == 1) return cands[0];
    std::string key = arch + "|" + key0;
    auto it = tuner.best.find(key);
    if (it != tuner.best.end()) return it->second;
    if (!tuner.enabled || capturing || no_alloc) return cands[0];
    bool tm = timing;
    timing = false;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto t0 = std::chrono::steady_clock::now();
    int bestv = cands[0];
    float bestt = 1e30f;
    for (int v : cands) {
      run(v);  // warm-up (and allocation of any workspace)
      HIPCHK(hipEventRecord(e0, st));
      for (int k = 0; k < 3; ++k) run(v);
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < bestt) {
        bestt = ms;
        bestv = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    timing = tm;
    tuner.best[key] = bestv;
    tuner.tuned += 1;
    tuner.tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    tuner.save();
    return bestv;
  }

  ~wcamg_ctx() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : evpool) (void)hipEventDestroy(e);
    if (own_stream && st) (void)hipStreamDestroy(st);
    if (cap_st) (void)hipStreamDestroy(cap_st);
  }

  void* W(const std::string& name, size_t bytes) {
    auto& b = ws[name];
    if (!b) b.reset(new DevBuf());
    return b->ensure(bytes, capturing || no_alloc);
  }
  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  // every scalar of the hierarchy that a captured V-cycle depends on
  std::vector<double> hier_sig() const {
    std::vector<double> s = {(double)h.prec, (double)h.nv, (double)h.sap_sweeps, (double)h.mr_iters,
                             (double)h.coarse_iters, h.coarse_tol, (double)h.l1, (double)h.nw,
                             (double)h.mr1_iters, (double)h.smoothing, (double)h.sap_eo};
    for (int m = 0; m < 4; ++m) s.push_back(h.b1[m]);
    return s;
  }
  // drops the graphs when a buffer was (re)allocated or freed since their
  // capture, or when the hierarchy's parameters changed
  void validate_graphs() {
    if (graphs.empty()) return;
    if (graph_epoch != g_alloc_epoch.load() || graph_sig != hier_sig()) drop_graphs();
  }
  // Workspaces are kept between calls.  reserve() is called on entry to a
  // top-level operation (where no workspace pointer other than the host
  // staging buffers "io_*" is live) with the large workspaces the operation
  // will use (name, bytes): when their growth does not fit into the free
  // device memory (with 2 GiB of headroom), first the workspaces outside this
  // list and then all workspaces except the staging buffers are released,
  // together with the graphs that refer to them.
  size_t ws_grow(const std::string& name, size_t bytes) const {
    auto it = ws.find(name);
    size_t have = (it == ws.end() || !it->second) ? 0 : it->second->n;
    return bytes > have ? bytes - have : 0;
  }
  void reserve(const std::vector<std::pair<std::string, size_t>>& plan) {
    auto fits = [&] {
      size_t need = (size_t)2 << 30;
      for (auto& q : plan) need += ws_grow(q.first, q.second);
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      return fr >= need;
    };
    if (fits()) return;
    drop_graphs();
    // host-transfer staging buffers ("io_*") may already be live in this call
    auto release = [&](bool keep_plan) {
      for (auto it = ws.begin(); it != ws.end();) {
        bool keep = it->first.compare(0, 3, "io_") == 0;
        if (keep_plan)
          for (auto& q : plan) keep = keep || q.first == it->first;
        if (keep)
          ++it;
        else
          it = ws.erase(it);
      }
    };
    release(true);
    if (fits()) return;
    release(false);
  }

  // ---- kernel timing
  hipEvent_t ev() {
    if (!evpool.empty()) {
      hipEvent_t e = evpool.back();
      evpool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  // Brackets the launches of one kernel class with events (when timing is
  // on and no graph is being captured), with the algorithmic bytes / flops /
  // right-hand-side units of the work, for roofline accounting.
  struct Timed {
    wcamg_ctx* c;
    const char* name;
    double bytes, flops, units;
    hipEvent_t a = nullptr, b = nullptr;
    bool excl;
    Timed(wcamg_ctx* c_, const char* n, double by = 0, double fl = 0, double un = 0, bool exclusive = false)
        : c(c_), name(n), bytes(by), flops(fl), units(un), excl(exclusive) {
      if (c->timing && !c->capturing && !c->no_alloc && c->timing_excl == 0) {
        a = c->ev();
        b = c->ev();
        HIPCHK(hipEventRecord(a, c->st));
      }
      if (excl) c->timing_excl++;
    }
    ~Timed() {
      if (excl) c->timing_excl--;
      if (a) {
        (void)hipEventRecord(b, c->st);
        c->pending.push_back({name, a, b, bytes, flops, units});
      }
    }
  };
  // ---- solve phases (Table 1's split of the solve time), timed with events
  // on the library stream while phase_on is set (V-cycles then run without
  // graphs)
  enum { PH_PRECOND = 0, PH_COARSE, PH_SMOOTH, PH_RP, PH_N };
  bool phase_on = false;
  struct PhaseEv {
    int ph;
    hipEvent_t a, b;
  };
  std::vector<PhaseEv> phase_pending;
  double phase_ms[PH_N] = {0, 0, 0, 0};
  struct Phase {
    wcamg_ctx* c;
    int ph;
    hipEvent_t a = nullptr, b = nullptr;
    Phase(wcamg_ctx* c_, int p) : c(c_), ph(p) {
      if (c->phase_on && !c->capturing) {
        a = c->ev();
        b = c->ev();
        HIPCHK(hipEventRecord(a, c->st));
      }
    }
    ~Phase() {
      if (a) {
        (void)hipEventRecord(b, c->st);
        c->phase_pending.push_back({ph, a, b});
      }
    }
  };
  void collect_phases() {
    if (phase_pending.empty()) return;
    HIPCHK(hipStreamSynchronize(st));
    for (auto& p : phase_pending) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
      phase_ms[p.ph] += ms;
      evpool.push_back(p.a);
      evpool.push_back(p.b);
    }
    phase_pending.clear();
  }

  void collect_timing() {
    if (pending.empty()) return;
    HIPCHK(hipStreamSynchronize(st));
    for (auto& p : pending) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
      auto& k = kstats[p.name];
      k.ms += ms;
      k.count += 1;
      k.bytes += p.bytes;
      k.flops += p.flops;
      k.units += p.units;
      evpool.push_back(p.a);
      evpool.push_back(p.b);
    }
    pending.clear();
  }

  // ---- precision helpers
  int spin_t(int prec) const { return prec == WCAMG_PREC_MIXED ? C64 : C128; }
  size_t fsz(int nrhs, int prec) const { return (size_t)nrhs * 12 * g.V * ct_size(spin_t(prec)); }
  size_t frs() const { return (size_t)12 * g.V; }
  // the SAP correction workspace: whole corrections (FP64 path, even-odd
  // block solve) or the mixed path's face projections, whichever is larger
  size_t face_rs() const { return (size_t)g.nblk * 6 * sap_face_slots(g); }
  size_t sapd_sz(int nrhs, int prec) const {
    size_t fb = prec == WCAMG_PREC_MIXED ? (size_t)nrhs * face_rs() * sizeof(float2) : 0;
    return std::max(fsz(nrhs, prec), fb);
  }

  // internal precision code of the FP32-field operator (never accepted at the ABI)
  static constexpr int PREC_F32 = 2;
  // The FP16 link field holds the hop matrices -kappa U (rounded once from
  // FP64), so the kernels that apply it take the hop coefficient -kappa = 1,
  // i.e. kappa = -1.
  static constexpr double HOP16_KAPPA = -1.0;
  void ensure_minv() {
    if (have_minv) return;
    Mi16.ensure((size_t)36 * g.V * sizeof(half2_t), capturing);
    launch_clover_inverse(g, (const double2*)Cl64.p, (half2_t*)Mi16.p, st);
    have_minv = true;
  }
  void ensure_f32() {
    if (have_f32) return;
    U32.ensure((size_t)36 * g.V * sizeof(float2), capturing);
    Cl32.ensure((size_t)36 * g.V * sizeof(float2), capturing);
    launch_convert(U64.p, C128, U32.p, C64, (size_t)36 * g.V, st);
    launch_convert(Cl64.p, C128, Cl32.p, C64, (size_t)36 * g.V, st);
    have_f32 = true;
  }

  // ---- D family on internal fields
  void dslash(const void* in, int in_t, void* out, int out_t, int nrhs, int op, int prec, const void* b = nullptr,
              int hopdir = 0, int chir = -1) {
    DslashArgs a;
    a.g = g;
    a.op = op;
    a.hopdir = hopdir;
    a.chir = chir;
    a.nrhs = nrhs;
    a.in = in;
    a.in_t = in_t;
    a.in_rs = frs();
    a.out = out;
    a.out_t = out_t;
    a.out_rs = frs();
    a.b = b;
    a.kappa = kappa;
    if (prec == WCAMG_PREC_MIXED) {
      a.U = U16.p;
      a.C = Cl16.p;
      a.fields16 = 1;
      a.compute32 = 1;
      a.kappa = HOP16_KAPPA;
    } else if (prec == PREC_F32) {
      ensure_f32();
      a.U = U32.p;
      a.C = Cl32.p;
      a.fields32 = 1;
      a.compute32 = 1;
    } else {
      a.U = U64.p;
      a.C = Cl64.p;
    }
    double site = (double)g.V;
    const double fb = a.fields16 ? 4 : a.fields32 ? 8 : 16;
    double fld = 4.0 * 9 * fb + 36.0 * fb;
    double by = site * (fld + nrhs * 12.0 * (ct_size(in_t) + ct_size(out_t) * (b ? 2 : 1)));
    char key[160];
    snprintf(key, sizeof(key), "dslash|op%d|in%d|out%d|f%d|c%d|res%d|V%d|Vb%d|n%d", op, in_t, out_t,
             a.fields16 ? 1 : a.fields32 ? 2 : 0, a.compute32, b ? 1 : 0, g.V, g.Vb, nrhs);
    std::vector<int> dcands = {64, 128, 256, 512};
    if (op == OP_D) dcands.push_back(-1);                                // colour-split variant
    if (op == OP_D && dslash_lds_slices(g) > 0) {
      dcands.push_back(-2);  // LDS-staged tiles
      dcands.push_back(-3);  // LDS-staged tiles, backward hops exchanged as half-spinors
    }
    if (op == OP_D && nrhs >= 2) dcands.push_back(-12);                 // 2 RHS per thread
    if (op == OP_D && nrhs >= 4 && a.compute32) dcands.push_back(-14);  // 4 RHS per thread
    a.block_size = tune(key, dcands, [&](int v) {
      DslashArgs q = a;
      q.block_size = v;
      launch_dslash(q, st);
    });
    Timed t(this, a.compute32 ? "dslash32" : "dslash64", by, 1920.0 * site * nrhs, nrhs);
    launch_dslash(a, st);
  }

  void sap(const void* b, void* x, const void* xinit, int nrhs, int sweeps, int mr, int prec, int eo = 0) {
    SapArgs a;
    a.g = g;
    if (eo) {
      require(prec == WCAMG_PREC_MIXED, "the even-odd block solve runs in mixed precision only");
      require(g.B[0] % 2 == 0 && g.B[1] % 2 == 0 && g.B[2] % 2 == 0 && g.B[3] % 2 == 0,
              "the even-odd block solve needs even block extents");
      ensure_minv();
      a.eo = 1;
      a.M = Mi16.p;
    }
    a.nrhs = nrhs;
    a.sweeps = sweeps;
    a.mr = mr;
    a.mixed = prec == WCAMG_PREC_MIXED;
    a.kappa = kappa;
    a.b = b;
    a.x = x;
    a.xinit = xinit;
    a.r = W("sap_r", fsz(nrhs, prec));
    a.delta = W("sap_d", sapd_sz(nrhs, prec));
    a.rs = frs();
    a.fs = face_rs();
    a.U = a.mixed ? U16.p : U64.p;
    a.C = a.mixed ? Cl16.p : Cl64.p;
    a.FL = FL16.p;
    if (sweeps <= 0) {
      // x = xinit (or 0)
      if (xinit)
        HIPCHK(hipMemcpyAsync(x, xinit, fsz(nrhs, prec), hipMemcpyDeviceToDevice, st));
      else
        launch_zero(x, fsz(nrhs, prec), st);
      return;
    }
    require((size_t)(a.mixed ? sap_dom_lds_bytes(g) : sap_lds_bytes(g, 0)) <= lds_max,
            "block volume too large for the SAP kernel's LDS at this precision");
    // per half-sweep: links+clover of the active half of the sites; per rhs
    // read r (or b), write r, delta and x (plus read x after the first visit)
    double sb = a.mixed ? 8 : 16, fld = a.mixed ? 4 * 9 * 4 + 36 * 4 : 4 * 9 * 16 + 36 * 16;
    for (int sw = 0; sw < sweeps; ++sw)
      for (int col = 0; col < 2; ++col) {
        double xr = (sw > 0 || xinit) ? 1 : 0;
        if (sap_needs_cross(a, sw, col)) {
          // per site of the active colour and RHS: r in and out, and per
          // crossing hop (sum over the directions of 2 / B_mu: 1.75 for
          // 4^3x8 domains) the neighbouring domain's spin-projected
          // correction (6 complex) and the face copy of the FP16 hop matrix,
          // ~170 flop (SU(3) times two colour vectors, reconstruction); the
          // even-odd variant reads whole corrections (12 complex) and the
          // links in site order, ~240 flop per hop
          double nc = 0;
          for (int m = 0; m < 4; ++m) nc += 2.0 / g.B[m];
          double byc = a.eo ? 0.5 * g.V * (nc * 36.0 + nrhs * 12.0 * sb * (2.0 + nc))
                            : 0.5 * g.V * (nc * 36.0 + nrhs * (24.0 * sb + nc * 6.0 * sb));
          double flc = 0.5 * g.V * nrhs * nc * (a.eo ? 240.0 : 170.0);
          Timed t(this, "sap_cross", byc, flc, nrhs);
          launch_sap_cross(a, sw, col, st);
        }
        // per RHS: r in, x in (after the first visit), x and r out, and the
        // correction out (whole, or its face projections on the mixed path:
        // 6 complex per crossing hop)
        double nc = 0;
        for (int m = 0; m < 4; ++m) nc += 2.0 / g.B[m];
        double dout = a.mixed && !a.eo ? nc * 6.0 * sb : 12.0 * sb;
        double by = 0.5 * g.V * (fld + nrhs * (12.0 * sb * (3.0 + xr) + dout));
        // per site of the active colour, RHS and MR iteration: D_SAP with its
        // in-domain hops only (sum over mu of 2 (B_mu - 1) / B_mu hops of 165
        // flop each, plus 552 for the clover and 48 for the identity and the
        // sums) and MR's vector work (<p, r>, <p, p>, x += alpha r,
        // r -= alpha p: 336 flop); the FP64 kernel also applies the
        // crossing-hop correction (~240 flop per crossing hop)
        double hops_in = 0, hops_x = 0;
        for (int m = 0; m < 4; ++m) {
          hops_in += 2.0 * (g.B[m] - 1) / g.B[m];
          hops_x += 2.0 / g.B[m];
        }
        double fl = 0.5 * g.V * nrhs *
                    (mr * (165.0 * hops_in + 600.0 + 336.0) + (a.mixed || (sw == 0 && col == 0) ? 0.0 : 240.0 * hops_x));
        Timed t(this, "sap_half", by, fl, nrhs);
        launch_sap_half(a, sw, col, st);
      }
  }

  // ---- coarse level
  int vec_t() const { return h.prec == WCAMG_PREC_MIXED ? C32H : C128; }
  int crs_t() const { return h.prec == WCAMG_PREC_MIXED ? C64 : C128; }
  size_t crs_n() const { return (size_t)h.cg.NC * h.N; }
  size_t csz(int nrhs) const { return (size_t)nrhs * crs_n() * ct_size(crs_t()); }

  void restrict_(const void* in, void* out, int nrhs) {
    double by = (double)g.V * 12 * (h.nv * ct_size(vec_t()) + nrhs * ct_size(spin_t(h.prec))) +
                (double)nrhs * crs_n() * ct_size(crs_t());
    char key[160];
    snprintf(key, sizeof(key), "restrict|nv%d|n%d|Vb%d|V%d|p%d", h.nv, nrhs, g.Vb, g.V, h.prec);
    std::vector<int> cands;
    for (int v : {32, 16, 8, 4})
      if (g.Vb % v == 0) cands.push_back(v);
    if (cands.empty()) cands.push_back(0);
    if (h.prec == WCAMG_PREC_FP64 && h.nv <= 32 && nrhs <= 32) cands.push_back(RESTRICT_MFMA64);
    if (h.prec == WCAMG_PREC_MIXED && h.nv <= 32 && nrhs <= 32) cands.push_back(RESTRICT_MFMA32);
    if (h.prec == WCAMG_PREC_MIXED && h.nv <= 32 && nrhs <= 32 && g.Vb % 32 == 0) cands.push_back(RESTRICT_MFMA32D);
    int tile = tune(key, cands, [&](int v) {
      launch_restrict(g, h.nv, nrhs, h.V.p, vec_t(), in, spin_t(h.prec), frs(), out, crs_t(), crs_n(), h.N, 0, st,
                      v);
    });
    Timed t(this, "restrict", by, 96.0 * g.V * h.nv * nrhs, nrhs);
    launch_restrict(g, h.nv, nrhs, h.V.p, vec_t(), in, spin_t(h.prec), frs(), out, crs_t(), crs_n(), h.N, 0, st,
                    tile);
  }
  void prolong_(const void* xc, void* out, int nrhs, int accumulate = 0) {
    double by = (double)g.V * 12 * (h.nv * ct_size(vec_t()) + nrhs * ct_size(spin_t(h.prec))) +
                (double)nrhs * crs_n() * ct_size(crs_t());
    std::vector<int> cands = {0};
    if (h.prec == WCAMG_PREC_MIXED && h.nv <= 32 && nrhs <= 32) cands.push_back(PROLONG_MFMA32);
    char key[160];
    snprintf(key, sizeof(key), "prolong|nv%d|n%d|Vb%d|V%d|p%d", h.nv, nrhs, g.Vb, g.V, h.prec);
    // tuning runs the candidates repeatedly: only where the launch overwrites
    // its output (an accumulating launch takes the tuned or the first choice)
    int var = cands[0];
    if (!accumulate) {
      var = tune(key, cands, [&](int v) {
        launch_prolong(g, h.nv, nrhs, h.V.p, vec_t(), xc, crs_t(), crs_n(), h.N, out, spin_t(h.prec), frs(), 0,
                       h.prec == WCAMG_PREC_MIXED, st, v);
      });
    } else {
      auto it = tuner.best.find(arch + "|" + std::string(key));
      if (it != tuner.best.end()) var = it->second;
    }
    Timed t(this, "prolong", by, 96.0 * g.V * h.nv * nrhs, nrhs);
    launch_prolong(g, h.nv, nrhs, h.V.p, vec_t(), xc, crs_t(), crs_n(), h.N, out, spin_t(h.prec), frs(),
                   accumulate, h.prec == WCAMG_PREC_MIXED, st, var);
  }
  COp op1() { return COp{h.cg, h.N, h.Dc.p}; }
  COp op2() { return COp{h.cg2, h.N2, h.Dc2.p}; }
  size_t csz(const COp& o, int nrhs) const { return (size_t)nrhs * o.n() * ct_size(crs_t()); }

  void coarse_mv(const COp& o, const void* x, void* y, const void* b, int nrhs, const BicgScal* live = nullptr) {
    double nc = o.cg.NC, N = o.N, cb = ct_size(crs_t());
    // compulsory operator bytes: the self block and the 4 forward blocks,
    // from which coarse gamma_5-hermiticity gives the backward ones (the
    // library stores and streams all 9)
    double by = nc * 5 * N * N * cb + nrhs * nc * N * cb * (b ? 3 : 2);
    std::vector<int> cands;
    for (int v : {1, 4, 8, 12, 16})
      if (v == 1 || v <= nrhs + 3) cands.push_back(v);
    if (h.prec == WCAMG_PREC_MIXED && o.N <= 64 && nrhs <= 32) cands.push_back(COARSE_MV_MFMA);
    if (h.prec == WCAMG_PREC_MIXED && o.N <= 64 && nrhs <= 16) cands.push_back(COARSE_MV_MFMA16);
    char key[160];
    snprintf(key, sizeof(key), "coarse_mv|N%d|NC%d|n%d|p%d|res%d", o.N, o.cg.NC, nrhs, h.prec, b ? 1 : 0);
    int var = tune(key, cands, [&](int v) {
      launch_coarse_mv(o.cg, o.N, o.Dc, x, y, b, nrhs, o.n(), h.prec == WCAMG_PREC_MIXED, st, v);
    });
    Timed t(this, "coarse_mv", by, 8.0 * 9 * N * N * nc * nrhs, nrhs);
    launch_coarse_mv(o.cg, o.N, o.Dc, x, y, b, nrhs, o.n(), h.prec == WCAMG_PREC_MIXED, st, var,
                     live ? &live->active : nullptr, (int)(sizeof(BicgScal) / sizeof(int)));
  }
  void coarse_mv(const void* x, void* y, const void* b, int nrhs) { coarse_mv(op1(), x, y, b, nrhs); }

  // BiCGStab with the stabilised omega; early exit checks only outside capture
  void coarse_solve(const COp& o, const void* b, void* x, int nrhs, int iters, double tol) {
    int t = crs_t();
    Timed tc(this, "coarse_solve", 0, 0, nrhs);
    size_t n = o.n();
    size_t bytes = csz(o, nrhs);
    void* r = W("cg_r", bytes);
    void* rt = W("cg_rt", bytes);
    void* p = W("cg_p", bytes);
    void* v = W("cg_v", bytes);
    void* s = W("cg_s", bytes);
    void* tt = W("cg_t", bytes);
    double2* part = (double2*)W("cg_part", (size_t)nrhs * reduce_nwg(n) * 3 * sizeof(double2));
    BicgScal* sc = (BicgScal*)W("cg_sc", (size_t)nrhs * sizeof(BicgScal));
    launch_bicg_init(b, x, r, rt, p, v, t, n, n, nrhs, tol, part, sc, st);
    std::vector<BicgScal> hs(nrhs);
    for (int it = 0; it < iters; ++it) {
      launch_bicg_p(p, r, v, t, n, n, nrhs, sc, st);
      coarse_mv(o, p, v, nullptr, nrhs, sc);
      launch_bicg_alpha(rt, v, t, n, n, nrhs, part, sc, st);
      launch_bicg_s(s, r, v, t, n, n, nrhs, sc, st);
      coarse_mv(o, s, tt, nullptr, nrhs, sc);
      launch_bicg_omega(tt, s, t, n, n, nrhs, part, sc, 0.7, st);
      launch_bicg_xr(x, r, p, s, tt, rt, t, n, n, nrhs, part, sc, st);
      if (!capturing && (it % 4 == 3) && it + 1 < iters) {
        HIPCHK(hipMemcpyAsync(hs.data(), sc, nrhs * sizeof(BicgScal), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool any = false;
        for (auto& q : hs) any |= q.active != 0;
        if (!any) break;
      }
    }
  }

  // x = BiCGStab(D, b) on fine fields in FP32 arithmetic (FP32 links,
  // clover and spinors), from 0, with the omega stabilisation of the coarse
  // solve: the preconditioner of the comparison solver (Sec. 5)
  void bicg32(const void* b, void* x, int nrhs, int iters, double tol) {
    const int t = C64;
    const size_t n = frs(), bytes = fsz(nrhs, WCAMG_PREC_MIXED);
    void* r = W("mb_r", bytes);
    void* rt = W("mb_rt", bytes);
    void* p = W("mb_p", bytes);
    void* v = W("mb_v", bytes);
    void* s = W("mb_s", bytes);
    void* tt = W("mb_t", bytes);
    double2* part = (double2*)W("mb_part", (size_t)nrhs * reduce_nwg(n) * 3 * sizeof(double2));
    BicgScal* sc = (BicgScal*)W("mb_sc", (size_t)nrhs * sizeof(BicgScal));
    launch_bicg_init(b, x, r, rt, p, v, t, n, n, nrhs, tol, part, sc, st);
    std::vector<BicgScal> hs(nrhs);
    for (int it = 0; it < iters; ++it) {
      launch_bicg_p(p, r, v, t, n, n, nrhs, sc, st);
      dslash(p, C64, v, C64, nrhs, OP_D, PREC_F32);
      launch_bicg_alpha(rt, v, t, n, n, nrhs, part, sc, st);
      launch_bicg_s(s, r, v, t, n, n, nrhs, sc, st);
      dslash(s, C64, tt, C64, nrhs, OP_D, PREC_F32);
      launch_bicg_omega(tt, s, t, n, n, nrhs, part, sc, 0.7, st);
      launch_bicg_xr(x, r, p, s, tt, rt, t, n, n, nrhs, part, sc, st);
      if ((it % 4 == 3) && it + 1 < iters) {
        HIPCHK(hipMemcpyAsync(hs.data(), sc, nrhs * sizeof(BicgScal), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool any = false;
        for (auto& q : hs) any |= q.active != 0;
        if (!any) break;
      }
    }
  }

  // x += MR(A, r, iters) on coarse vectors (A = the level-1 stencil); r is overwritten
  void mr_smooth(const COp& o, void* x, void* r, int nrhs, int iters) {
    int t = crs_t();
    size_t n = o.n();
    void* p = W("mr_p", csz(o, nrhs));
    double2* part = (double2*)W("mr_part", (size_t)nrhs * reduce_nwg(n) * 2 * sizeof(double2));
    double2* alpha = (double2*)W("mr_alpha", (size_t)nrhs * sizeof(double2));
    for (int it = 0; it < iters; ++it) {
      coarse_mv(o, r, p, nullptr, nrhs);
      launch_mr_alpha(p, r, t, n, n, nrhs, part, alpha, st);
      launch_mr_update(x, r, p, alpha, t, n, n, nrhs, st);
    }
  }

  // level-1 restriction / prolongation
  void l1_restrict(const void* in, void* out, int nrhs) {
    launch_l1_restrict(h.cg, h.b1, h.N, h.nw, nrhs, h.W.p, crs_t(), in, crs_t(), op1().n(), out, crs_t(),
                       op2().n(), h.N2, st);
  }
  void l1_prolong(const void* xc, void* out, int nrhs) {
    launch_l1_prolong(h.cg, h.b1, h.N, h.nw, nrhs, h.W.p, crs_t(), xc, crs_t(), op2().n(), h.N2, out, crs_t(),
                      op1().n(), st);
  }

  // level-1 V-cycle as the coarse solve of level 0: x = P1 BiCGStab(Dc2, R1 b); x += MR(b - Dc x)
  void vcycle1(const void* b, void* x, int nrhs) {
    COp o1 = op1(), o2 = op2();
    void* b2 = W("l1_b2", csz(o2, nrhs));
    void* x2 = W("l1_x2", csz(o2, nrhs));
    void* r1 = W("l1_r", csz(o1, nrhs));
    l1_restrict(b, b2, nrhs);
    coarse_solve(o2, b2, x2, nrhs, h.coarse_iters, h.coarse_tol);
    l1_prolong(x2, x, nrhs);
    coarse_mv(o1, x, r1, b, nrhs);
    mr_smooth(o1, x, r1, nrhs, h.mr1_iters);
  }

  void coarse_solve(const void* b, void* x, int nrhs, int iters, double tol) {
    coarse_solve(op1(), b, x, nrhs, iters, tol);
  }

  // M v: restrict, coarse solve, prolong, residual, SAP started from the prolonged vector
  // M in (Sec. 3): Richardson steps x <- x + M_i (in - D x) from x = 0 with
  // the coarse-grid step M_1 = (1a) restrict, (1b) coarse solve, (1c)
  // prolong, and the SAP smoother M_2, in the order h.smoothing names
  void vcycle(const void* in, void* out, int nrhs) {
    int prec = h.prec, t = spin_t(prec);
    void* vc = W("vc_b", csz(nrhs));
    void* xc = W("vc_x", csz(nrhs));
    void* x1 = W("vc_x1", fsz(nrhs, prec));
    void* r = W("vc_r", fsz(nrhs, prec));
    auto coarse = [&](const void* rhs) {
      {
        Phase ph(this, PH_RP);
        restrict_(rhs, vc, nrhs);
      }
      Phase ph(this, PH_COARSE);
      if (h.l1)
        vcycle1(vc, xc, nrhs);
      else
        coarse_solve(vc, xc, nrhs, h.coarse_iters, h.coarse_tol);
    };
    auto prolong_p = [&](void* x, int acc) {
      Phase ph(this, PH_RP);
      prolong_(xc, x, nrhs, acc);
    };
    auto smooth = [&](const void* rhs, void* x, const void* x0) {
      Phase ph(this, PH_SMOOTH);
      sap(rhs, x, x0, nrhs, h.sap_sweeps, h.mr_iters, prec, h.sap_eo);
    };
    if (h.smoothing == WCAMG_SMOOTH_POST) {
      coarse(in);
      prolong_p(x1, 0);
      dslash(x1, t, r, t, nrhs, OP_D, prec, in);
      smooth(r, out, x1);
      return;
    }
    // smoother first: x = M_2 in, then x += M_1 (in - D x)
    void* x = h.smoothing == WCAMG_SMOOTH_PRE ? out : x1;
    smooth(in, x, nullptr);
    dslash(x, t, r, t, nrhs, OP_D, prec, in);
    coarse(r);
    prolong_p(x, 1);
    if (h.smoothing == WCAMG_SMOOTH_BOTH) {
      // and the smoother again: out = x + M_2 (in - D x)
      dslash(x, t, r, t, nrhs, OP_D, prec, in);
      smooth(r, out, x);
    }
  }

  // block orthonormalisation (CholQR, twice) of nv working fields in place;
  // tmp: nv fields of scratch (the workspace "or_tmp" when null)
  void orthonormalize(void* Vw, int nv, int prec, void* tmp = nullptr) {
    int t = spin_t(prec);
    Timed tb(this, "ortho", 0, 0, 1, true);
    size_t gbytes = (size_t)nv * g.nblk * 2 * nv * sizeof(double2);
    double2* G = (double2*)W("or_G", gbytes);
    void* coef = W("or_c", (size_t)nv * g.nblk * 2 * nv * ct_size(t));
    if (!tmp) tmp = W("or_tmp", fsz(nv, prec));
    int* bad = (int*)W("or_bad", sizeof(int));
    launch_zero(bad, sizeof(int), st);
    size_t grs = (size_t)g.nblk * 2 * nv;
    // pass 0: Vw -> tmp, pass 1: tmp -> Vw (no copies)
    for (int pass = 0; pass < 2; ++pass) {
      void* src = pass == 0 ? Vw : tmp;
      void* dst = pass == 0 ? tmp : Vw;
      launch_restrict(g, nv, nv, src, t, src, t, frs(), G, C128, grs, 2 * nv, 1, st, nv <= 32 ? RESTRICT_MFMA64 : 0);
      launch_cholesky_coef(g.nblk, nv, G, grs, coef, t, grs, bad, st);
      launch_prolong(g, nv, nv, src, t, coef, t, grs, 2 * nv, dst, t, frs(), 0, prec == WCAMG_PREC_MIXED, st);
    }
    int hb = 0;
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    require(hb == 0, "orthonormalisation: test vectors linearly dependent on a block", WCAMG_ENUMERIC);
  }

  // coarse operator eq.(7) from the stored vectors (fused kernel)
  void build_coarse() {
    int nv = h.nv, N = h.N;
    h.Dc.ensure((size_t)h.cg.NC * 9 * N * N * ct_size(crs_t()), capturing);
    bool mixed = h.prec == WCAMG_PREC_MIXED;
    const void* Uf = mixed ? U16.p : U64.p;
    const void* Cf = mixed ? Cl16.p : Cl64.p;
    const double kh = mixed ? HOP16_KAPPA : kappa;
    std::vector<int> cands = {0};
    if (mixed && nv <= 32) cands = {1, 0};  // matrix-core contraction first
    char key[96];
    snprintf(key, sizeof(key), "coarse_build|nv%d|Vb%d|V%d", nv, g.Vb, g.V);
    void* part = nullptr;
    if (mixed && nv <= 32)
      part = W("cb_part", (size_t)coarse_build_chunks(g) * g.nblk * N * N * sizeof(float2));
    int var = tune(key, cands,
                   [&](int v) { launch_coarse_build(g, nv, kh, h.V.p, Uf, Cf, h.Dc.p, mixed, st, v, part); });
    Timed tb(this, "coarse_build", 0, 0, 1, true);
    launch_coarse_build(g, nv, kh, h.V.p, Uf, Cf, h.Dc.p, mixed, st, var, part);
  }

  // level-1 block orthonormalisation of W in place (CholQR twice, FP64 Gram)
  void orthonormalize1() {
    Timed tb(this, "ortho", 0, 0, 1, true);
    int nw = h.nw, t = crs_t();
    COp o1 = op1(), o2 = op2();
    size_t grs = o2.n();  // NC2 * 2 nw
    double2* G = (double2*)W("or1_G", (size_t)nw * grs * sizeof(double2));
    void* coef = W("or1_c", (size_t)nw * grs * ct_size(t));
    void* tmp = W("or1_tmp", csz(o1, nw));
    int* bad = (int*)W("or_bad", sizeof(int));
    launch_zero(bad, sizeof(int), st);
    for (int pass = 0; pass < 2; ++pass) {
      launch_l1_restrict(h.cg, h.b1, h.N, nw, nw, h.W.p, t, h.W.p, t, o1.n(), G, C128, grs, h.N2, st);
      launch_cholesky_coef(h.cg2.NC, nw, G, grs, coef, t, grs, bad, st);
      launch_l1_prolong(h.cg, h.b1, h.N, nw, nw, h.W.p, t, coef, t, grs, h.N2, tmp, t, o1.n(), st);
      HIPCHK(hipMemcpyAsync(h.W.p, tmp, csz(o1, nw), hipMemcpyDeviceToDevice, st));
    }
    int hb = 0;
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    require(hb == 0, "level-1 orthonormalisation: vectors linearly dependent on a block", WCAMG_ENUMERIC);
  }

  void build_coarse2() {
    Timed tb(this, "coarse_build", 0, 0, 1, true);
    h.Dc2.ensure((size_t)h.cg2.NC * 9 * h.N2 * h.N2 * ct_size(crs_t()), capturing);
    launch_l1_build(h.cg, h.b1, h.N, h.nw, h.Dc.p, h.W.p, h.Dc2.p, h.prec == WCAMG_PREC_MIXED, st);
  }

  void set_l1_params(const wcamg_setup_params* p) {
    h.l1 = false;
    if (p->nlevels <= 2) return;
    require(p->nlevels == 3, "nlevels must be 2 or 3");
    require(p->nv1 >= 1 && p->nv1 <= 64 && 2 * p->nv1 * p->nv1 <= 16 * 256, "nv1 must be in [1, 64]");
    require(p->mr1_iters >= 0 && p->init_mr1_iters >= 0, "negative iteration count");
    int n2[4];
    for (int m = 0; m < 4; ++m) {
      require(p->block1[m] >= 1 && h.cg.N[m] % p->block1[m] == 0, "block1 must divide the coarse lattice");
      h.b1[m] = p->block1[m];
      n2[m] = h.cg.N[m] / p->block1[m];
    }
    h.nw = p->nv1;
    h.N2 = 2 * p->nv1;
    h.cg2 = make_cgeo(n2);
    h.mr1_iters = p->mr1_iters;
    h.l1 = true;
  }

  // level-1 setup on the final level-0 hierarchy (same steps one level down)
  void setup_level1(const wcamg_setup_params* p, const void* W0) {
    COp o1 = op1();
    int nw = h.nw, t = crs_t();
    h.W.ensure(csz(o1, nw), capturing);
    if (W0)
      HIPCHK(hipMemcpyAsync(h.W.p, W0, csz(o1, nw), hipMemcpyDeviceToDevice, st));
    else
      launch_gauss(h.W.p, t, (size_t)nw * o1.n(), p->seed1, st);
    void* Wx = W("su1_x", csz(o1, nw));
    void* Wr = W("su1_r", csz(o1, nw));
    for (int k = 0; k < p->n_init; ++k) {
      launch_zero(Wx, csz(o1, nw), st);
      HIPCHK(hipMemcpyAsync(Wr, h.W.p, csz(o1, nw), hipMemcpyDeviceToDevice, st));
      mr_smooth(o1, Wx, Wr, nw, p->init_mr1_iters);
      HIPCHK(hipMemcpyAsync(h.W.p, Wx, csz(o1, nw), hipMemcpyDeviceToDevice, st));
    }
    orthonormalize1();
    build_coarse2();
    for (int k = 0; k < p->n_adapt; ++k) {
      vcycle1(h.W.p, Wx, nw);
      HIPCHK(hipMemcpyAsync(h.W.p, Wx, csz(o1, nw), hipMemcpyDeviceToDevice, st));
      orthonormalize1();
      build_coarse2();
    }
  }

  void store_vectors(const void* Vw, int nv) {
    h.V.ensure((size_t)nv * 12 * g.V * ct_size(vec_t()), capturing);
    launch_convert(Vw, spin_t(h.prec), h.V.p, vec_t(), (size_t)nv * 12 * g.V, st);
  }

  void set_params(const wcamg_setup_params* p) {
    require(p->nv >= 1 && p->nv <= 64, "nv must be in [1, 64]");
    require(p->prec == WCAMG_PREC_FP64 || p->prec == WCAMG_PREC_MIXED, "invalid prec");
    require(p->sap_sweeps >= 0 && p->mr_iters >= 0 && p->coarse_iters >= 0 && p->n_init >= 0 && p->n_adapt >= 0,
            "negative iteration count");
    require(p->sap_sweeps == 0 || (g.NB[0] % 2 == 0 && g.NB[1] % 2 == 0 && g.NB[2] % 2 == 0 && g.NB[3] % 2 == 0),
            "SAP needs an even number of blocks per direction");
    require(std::isfinite(p->coarse_tol) && p->coarse_tol >= 0, "invalid coarse_tol");
    require(p->smoothing == WCAMG_SMOOTH_POST || p->smoothing == WCAMG_SMOOTH_PRE ||
                p->smoothing == WCAMG_SMOOTH_BOTH,
            "invalid smoothing");
    require(p->sap_eo == 0 || p->sap_eo == 1, "sap_eo must be 0 or 1");
    require(!p->sap_eo || p->prec == WCAMG_PREC_MIXED, "the even-odd block solve runs in mixed precision only");
    require(!p->sap_eo || (g.B[0] % 2 == 0 && g.B[1] % 2 == 0 && g.B[2] % 2 == 0 && g.B[3] % 2 == 0),
            "the even-odd block solve needs even block extents");
    h.sap_eo = p->sap_eo;
    h.smoothing = p->smoothing;
    h.prec = p->prec;
    h.nv = p->nv;
    h.N = 2 * p->nv;
    h.cg = make_cgeo(g.NB);
    h.sap_sweeps = p->sap_sweeps;
    h.mr_iters = p->mr_iters;
    h.coarse_iters = p->coarse_iters;
    h.coarse_tol = p->coarse_tol;
  }
};

// ---------------------------------------------------------------------------
// Fixed scratch area of wcamg_apply_D_noalloc: one copy per GPU, held from the
// loading of the library's code object until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory: kernels and copies
// only ever get the device address that hipGetSymbolAddress returns for the
// current device (scratch_address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[WCAMG_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device id -> device address of its scratch array

// Device address of the current device's scratch array, looked up once per
// device (with that device current).
void* scratch_address() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  require(ptr != nullptr, "no device address for the no-allocation scratch area", WCAMG_EHIP);
  g_scratch_addr[dev] = ptr;
  return ptr;
}
}  // namespace

// ---------------------------------------------------------------------------
// helpers for the ABI wrappers
// ---------------------------------------------------------------------------
namespace {

int guard(wcamg_ctx* c, const std::function<void()>& f);

struct HostIO {
  // stage host buffers through device memory
  wcamg_ctx* c;
  HostIO(wcamg_ctx* c_) : c(c_) {}
  const void* in(const void* p, size_t bytes, int where, const char* name) {
    if (where == WCAMG_DEVICE) return p;
    void* d = c->W(name, bytes);
    HIPCHK(hipMemcpyAsync(d, p, bytes, hipMemcpyHostToDevice, c->st));
    return d;
  }
  void* out(void* p, size_t bytes, int where, const char* name) {
    if (where == WCAMG_DEVICE) return p;
    return c->W(name, bytes);
  }
  void finish(void* host, const void* dev, size_t bytes, int where) {
    if (where == WCAMG_DEVICE) return;
    HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  }
};

int guard(wcamg_ctx* c, const std::function<void()>& f) {
  try {
    if (c) c->err.clear();
    f();
    return WCAMG_OK;
  } catch (const WcError& e) {
    if (c) {
      c->err = e.what();
      c->capturing = false;
    }
    return e.code;
  } catch (const std::exception& e) {
    if (c) {
      c->err = e.what();
      c->capturing = false;
    }
    return WCAMG_EHIP;
  } catch (...) {
    if (c) c->err = "unknown error";
    return WCAMG_EHIP;
  }
}

void check_where(int where) { require(where == WCAMG_DEVICE || where == WCAMG_HOST, "invalid 'where'"); }
void check_nrhs(int n) { require(n >= 1 && n <= WCAMG_MAX_RHS, "nrhs must be in [1, 64]"); }
void check_prec(int p) { require(p == WCAMG_PREC_FP64 || p == WCAMG_PREC_MIXED, "invalid prec"); }

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

int wcamg_create(wcamg_ctx** out, const wcamg_lattice* lat, void* hip_stream) {
  if (!out || !lat) return WCAMG_EINVAL;
  *out = nullptr;
  for (int m = 0; m < 4; ++m) {
    if (lat->dims[m] < 2 || lat->dims[m] % 2) return WCAMG_EINVAL;
    if (lat->block[m] < 1 || lat->dims[m] % lat->block[m]) return WCAMG_EINVAL;
    if (lat->bc[m] != 1 && lat->bc[m] != -1) return WCAMG_EINVAL;
  }
  if (!std::isfinite(lat->kappa) || !std::isfinite(lat->csw)) return WCAMG_EINVAL;
  long long V = 1;
  for (int m = 0; m < 4; ++m) V *= lat->dims[m];
  if (V > (1LL << 28)) return WCAMG_EINVAL;
  int vb = lat->block[0] * lat->block[1] * lat->block[2] * lat->block[3];
  if (vb > 512) return WCAMG_EINVAL;  // one SAP workgroup (<= 512 threads) per domain
  wcamg_ctx* c = new (std::nothrow) wcamg_ctx();
  if (!c) return WCAMG_ENOMEM;
  int rc = guard(c, [&] {
    c->g = make_geo(lat->dims, lat->block, lat->bc);
    c->kappa = lat->kappa;
    c->csw = lat->csw;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (hip_stream) {
      c->st = (hipStream_t)hip_stream;
    } else {
      // a blocking stream: ordered with work on the legacy default stream
      HIPCHK(hipStreamCreateWithFlags(&c->st, hipStreamDefault));
      c->own_stream = true;
    }
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    c->lds_max = prop.sharedMemPerBlock;
    c->arch = prop.gcnArchName;
    c->arch = c->arch.substr(0, c->arch.find(':'));
    const char* cache = std::getenv("WCAMG_AUTOTUNE_CACHE");
    if (cache && *cache) c->tuner.load(cache);
    c->scratch = scratch_address();
  });
  if (rc != WCAMG_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return WCAMG_OK;
}

void wcamg_destroy(wcamg_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  delete c;
}

const char* wcamg_last_error(const wcamg_ctx* c) { return c ? c->err.c_str() : "null context"; }

int wcamg_sync(wcamg_ctx* c) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] { HIPCHK(hipStreamSynchronize(c->st)); });
}

int wcamg_load_gauge(wcamg_ctx* c, const void* U, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(U != nullptr, "null gauge pointer");
    const Geo& g = c->g;
    size_t bytes = (size_t)4 * g.V * 9 * sizeof(double2);
    HostIO io(c);
    const double2* Ud = (const double2*)io.in(U, bytes, where, "io_in");
    c->U64.ensure((size_t)4 * 9 * g.V * sizeof(double2), false);
    c->U16.ensure((size_t)4 * 9 * g.V * sizeof(half2_t), false);
    c->Cl64.ensure((size_t)36 * g.V * sizeof(double2), false);
    c->Cl16.ensure((size_t)36 * g.V * sizeof(half2_t), false);
    launch_pack_gauge(g, Ud, (double2*)c->U64.p, (half2_t*)c->U16.p, -c->kappa, c->st);
    c->FL16.ensure((size_t)g.nblk * 9 * sap_face_slots(g) * sizeof(half2_t), false);
    launch_face_links(g, c->U16.p, c->FL16.p, c->st);
    std::vector<double> sig = sigma_table();
    launch_clover_build(g, (const double2*)c->U64.p, c->kappa, c->csw, sig.data(), (double2*)c->Cl64.p,
                        (half2_t*)c->Cl16.p, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    c->have_gauge = true;
    c->have_hier = false;
    c->have_f32 = false;
    c->have_minv = false;
  });
}

int wcamg_load_clover(wcamg_ctx* c, const void* F, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(F != nullptr, "null clover pointer");
    require(c->have_gauge, "load the gauge field first", WCAMG_ESTATE);
    const Geo& g = c->g;
    HostIO io(c);
    const double2* Fd = (const double2*)io.in(F, (size_t)g.V * 72 * sizeof(double2), where, "io_in");
    launch_pack_clover(g, Fd, (double2*)c->Cl64.p, (half2_t*)c->Cl16.p, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    c->have_hier = false;
    c->have_f32 = false;
    c->have_minv = false;
  });
}

int wcamg_get_clover(wcamg_ctx* c, void* F, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(F != nullptr, "null pointer");
    require(c->have_gauge, "no gauge field", WCAMG_ESTATE);
    const Geo& g = c->g;
    size_t bytes = (size_t)g.V * 72 * sizeof(double2);
    HostIO io(c);
    double2* Fd = (double2*)io.out(F, bytes, where, "io_out");
    launch_unpack_clover(g, (const double2*)c->Cl64.p, Fd, c->st);
    HIPCHK(hipGetLastError());
    io.finish(F, Fd, bytes, where);
  });
}

static int apply_op(wcamg_ctx* c, const void* in, void* out, int nrhs, int prec, int where, int op) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    check_prec(prec);
    require(in && out && in != out, "null or aliasing pointers");
    require(c->have_gauge, "no gauge field", WCAMG_ESTATE);
    const Geo& g = c->g;
    size_t cbytes = (size_t)nrhs * g.V * 12 * sizeof(double2);
    HostIO io(c);
    const double2* ind = (const double2*)io.in(in, cbytes, where, "io_in");
    double2* outd = (double2*)io.out(out, cbytes, where, "io_out");
    int t = c->spin_t(prec);
    c->reserve({{"ap_a", c->fsz(nrhs, prec)}, {"ap_b", c->fsz(nrhs, prec)}});
    void* a = c->W("ap_a", c->fsz(nrhs, prec));
    void* b = c->W("ap_b", c->fsz(nrhs, prec));
    launch_pack_spinor(g, ind, a, t, c->frs(), nrhs, c->st);
    c->dslash(a, t, b, t, nrhs, op, prec);
    launch_unpack_spinor(g, b, t, c->frs(), outd, nrhs, c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, outd, cbytes, where);
  });
}

int wcamg_apply_D(wcamg_ctx* c, const void* in, void* out, int nrhs, int prec, int where) {
  return apply_op(c, in, out, nrhs, prec, where, OP_D);
}

int wcamg_apply_D_noalloc(wcamg_ctx* c, const void* in, void* out, int nrhs, int prec) {
  if (!c) return WCAMG_EINVAL;
  struct NoAlloc {  // the flag is cleared on every exit, errors included
    wcamg_ctx* c;
    explicit NoAlloc(wcamg_ctx* c_) : c(c_) { c->no_alloc = true; }
    ~NoAlloc() { c->no_alloc = false; }
  };
  return guard(c, [&] {
    check_nrhs(nrhs);
    check_prec(prec);
    require(in && out && in != out, "null or aliasing pointers");
    require(c->have_gauge, "no gauge field", WCAMG_ESTATE);
    require(c->scratch != nullptr, "no scratch area on this context's device", WCAMG_ESTATE);
    const Geo& g = c->g;
    // two staging fields in the internal layout, each starting on a 256-byte boundary
    const size_t fb = (c->fsz(nrhs, prec) + 255) / 256 * 256;
    require(2 * fb <= (size_t)WCAMG_NOALLOC_SCRATCH_BYTES,
            "nrhs * lattice volume too large for the no-allocation scratch area (" +
                std::to_string(2 * fb) + " > " + std::to_string((size_t)WCAMG_NOALLOC_SCRATCH_BYTES) + " bytes)");
    NoAlloc guard_flag(c);
    char* a = (char*)c->scratch;
    char* b = a + fb;
    int t = c->spin_t(prec);
    launch_pack_spinor(g, (const double2*)in, a, t, c->frs(), nrhs, c->st);
    c->dslash(a, t, b, t, nrhs, OP_D, prec);
    launch_unpack_spinor(g, b, t, c->frs(), (double2*)out, nrhs, c->st);
    HIPCHK(hipGetLastError());
  });
}
int wcamg_apply_Dsap(wcamg_ctx* c, const void* in, void* out, int nrhs, int prec, int where) {
  return apply_op(c, in, out, nrhs, prec, where, OP_DSAP);
}

int wcamg_sap(wcamg_ctx* c, const void* b, void* x, int nrhs, int sweeps, int mr_iters, int block_solve, int prec,
              int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    check_prec(prec);
    require(b && x, "null pointer");
    require(block_solve == WCAMG_BLOCK_MR || block_solve == WCAMG_BLOCK_EO_MR, "invalid block_solve");
    require(sweeps >= 0 && mr_iters >= 0, "negative iteration count");
    require(c->have_gauge, "no gauge field", WCAMG_ESTATE);
    const Geo& g = c->g;
    require(g.NB[0] % 2 == 0 && g.NB[1] % 2 == 0 && g.NB[2] % 2 == 0 && g.NB[3] % 2 == 0,
            "SAP needs an even number of blocks per direction");
    size_t cbytes = (size_t)nrhs * g.V * 12 * sizeof(double2);
    HostIO io(c);
    const double2* bd = (const double2*)io.in(b, cbytes, where, "io_in");
    double2* xd = (double2*)io.out(x, cbytes, where, "io_out");
    int t = c->spin_t(prec);
    c->reserve({{"ap_a", c->fsz(nrhs, prec)}, {"ap_b", c->fsz(nrhs, prec)}, {"sap_r", c->fsz(nrhs, prec)},
                {"sap_d", c->sapd_sz(nrhs, prec)}});
    void* bi = c->W("ap_a", c->fsz(nrhs, prec));
    void* xi = c->W("ap_b", c->fsz(nrhs, prec));
    launch_pack_spinor(g, bd, bi, t, c->frs(), nrhs, c->st);
    c->sap(bi, xi, nullptr, nrhs, sweeps, mr_iters, prec, block_solve == WCAMG_BLOCK_EO_MR);
    launch_unpack_spinor(g, xi, t, c->frs(), xd, nrhs, c->st);
    HIPCHK(hipGetLastError());
    io.finish(x, xd, cbytes, where);
  });
}

static void install_vectors(wcamg_ctx* c, const void* V, int where, const wcamg_setup_params* p) {
  c->set_params(p);
  const Geo& g = c->g;
  size_t cbytes = (size_t)p->nv * g.V * 12 * sizeof(double2);
  HostIO io(c);
  const double2* Vd = (const double2*)io.in(V, cbytes, where, "io_in");
  c->h.V.ensure((size_t)p->nv * 12 * g.V * ct_size(c->vec_t()), false);
  launch_pack_spinor(g, Vd, c->h.V.p, c->vec_t(), c->frs(), p->nv, c->st);
}

int wcamg_set_test_vectors(wcamg_ctx* c, const void* V, const wcamg_setup_params* p, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(V && p, "null pointer");
    require(c->have_gauge, "no gauge field", WCAMG_ESTATE);
    c->have_hier = false;
    install_vectors(c, V, where, p);
    c->set_l1_params(p);
    c->build_coarse();
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    c->have_hier = true;
  });
}

int wcamg_setup(wcamg_ctx* c, const wcamg_setup_params* p) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    require(p != nullptr, "null parameters");
    require(!p->init_net || p->prec == WCAMG_PREC_MIXED || p->prec == WCAMG_PREC_FP64, "invalid prec");
    check_where(p->init_where);
    require(c->have_gauge, "no gauge field", WCAMG_ESTATE);
    c->have_hier = false;
    c->set_params(p);
    c->set_l1_params(p);
    const Geo& g = c->g;
    int nv = p->nv, prec = p->prec, t = c->spin_t(prec);
    require(p->vec_chunk >= 0, "vec_chunk must be >= 0");
    const int ch = p->vec_chunk > 0 ? std::min(p->vec_chunk, nv) : nv;
    size_t cbytes = (size_t)nv * g.V * 12 * sizeof(double2);
    {
      // the iterates and their update (which also serves as the
      // orthonormalisation's scratch), and the SAP and V-cycle fields of one
      // batch of ch vectors
      const size_t f = c->fsz(nv, prec), fc = c->fsz(ch, prec);
      c->reserve({{"su_w", f}, {"su_t", f}, {"sap_r", fc}, {"sap_d", c->sapd_sz(ch, prec)}, {"vc_r", fc},
                  {"vc_x1", fc}});
    }
    const size_t vstride = c->fsz(1, prec);
    auto batched = [&](void* in, void* out, const std::function<void(const void*, void*, int)>& f) {
      for (int v0 = 0; v0 < nv; v0 += ch)
        f((const char*)in + v0 * vstride, (char*)out + v0 * vstride, std::min(ch, nv - v0));
    };
    HostIO io(c);
    const double2* Vd = nullptr;
    if (p->init_vectors) Vd = (const double2*)io.in(p->init_vectors, cbytes, p->init_where, "io_in");
    void* Vw = c->W("su_w", c->fsz(nv, prec));
    void* Vt = c->W("su_t", c->fsz(nv, prec));
    // start vectors: given (canonical layout) or drawn by the counter-based
    // generator (in the internal layout: the generator's element order is the
    // internal one)
    auto start = [&](void* dst, int dt) {
      if (Vd)
        launch_pack_spinor(g, Vd, dst, dt, c->frs(), nv, c->st);
      else
        launch_gauss(dst, dt, (size_t)nv * 12 * g.V, p->seed, c->st);
    };
    if (p->init_net) {
      // (0-a) replaced by the network: its output from the nv start vectors
      require(c->net.L > 0 && c->net.C == nv, "init_net needs a network with nv channels (wcamg_net_init)");
      void* r32 = c->W("su_r32", (size_t)nv * 12 * g.V * sizeof(float2));
      start(r32, C64);
      c->net_forward(r32);
      launch_convert(c->net.acts[c->net.L], C64, Vw, t, (size_t)nv * 12 * g.V, c->st);
    } else {
      start(Vw, t);
      for (int k = 0; k < p->n_init; ++k) {
        batched(Vw, Vt, [&](const void* in, void* out, int n) {
          c->sap(in, out, nullptr, n, p->sap_sweeps, p->mr_iters, prec, p->sap_eo);
        });
        std::swap(Vw, Vt);
      }
    }
    c->orthonormalize(Vw, nv, prec, Vt);
    c->store_vectors(Vw, nv);
    c->build_coarse();
    // level 0 (0-b) runs with the two-level cycle; level 1 is set up on the final level-0 hierarchy
    bool l1 = c->h.l1;
    c->h.l1 = false;
    for (int k = 0; k < p->n_adapt; ++k) {
      batched(Vw, Vt, [&](const void* in, void* out, int n) { c->vcycle(in, out, n); });
      std::swap(Vw, Vt);
      c->orthonormalize(Vw, nv, prec, Vt);
      c->store_vectors(Vw, nv);
      c->build_coarse();
    }
    if (l1) {
      c->h.l1 = true;
      const void* W0 = nullptr;
      if (p->init_vectors1) {
        size_t nel = (size_t)p->nv1 * c->op1().n();
        void* tmp = c->W("su1_w0", nel * ct_size(c->crs_t()));
        launch_convert(p->init_vectors1, C128, tmp, c->crs_t(), nel, c->st);
        W0 = tmp;
      }
      c->setup_level1(p, W0);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    c->have_hier = true;
  });
}

int wcamg_get_test_vectors(wcamg_ctx* c, void* V, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(V, "null pointer");
    require(c->have_hier, "no hierarchy", WCAMG_ESTATE);
    size_t cbytes = (size_t)c->h.nv * c->g.V * 12 * sizeof(double2);
    HostIO io(c);
    double2* Vd = (double2*)io.out(V, cbytes, where, "io_out");
    launch_unpack_spinor(c->g, c->h.V.p, c->vec_t(), c->frs(), Vd, c->h.nv, c->st);
    HIPCHK(hipGetLastError());
    io.finish(V, Vd, cbytes, where);
  });
}

int wcamg_orthonormalize(wcamg_ctx* c, const void* in, void* out, int nv, int prec, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_prec(prec);
    require(in && out, "null pointer");
    require(nv >= 1 && nv <= 64, "nv must be in [1, 64]");
    const Geo& g = c->g;
    size_t cbytes = (size_t)nv * g.V * 12 * sizeof(double2);
    HostIO io(c);
    const double2* ind = (const double2*)io.in(in, cbytes, where, "io_in");
    double2* outd = (double2*)io.out(out, cbytes, where, "io_out");
    int t = c->spin_t(prec);
    c->reserve({{"ap_a", c->fsz(nv, prec)}, {"or_tmp", c->fsz(nv, prec)}});
    void* Vw = c->W("ap_a", c->fsz(nv, prec));
    launch_pack_spinor(g, ind, Vw, t, c->frs(), nv, c->st);
    c->orthonormalize(Vw, nv, prec);
    launch_unpack_spinor(g, Vw, t, c->frs(), outd, nv, c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, outd, cbytes, where);
  });
}

int wcamg_restrict(wcamg_ctx* c, const void* in, void* out, int nrhs, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    require(in && out, "null pointer");
    require(c->have_hier, "no hierarchy", WCAMG_ESTATE);
    const Geo& g = c->g;
    size_t fb = (size_t)nrhs * g.V * 12 * sizeof(double2);
    size_t cb = (size_t)nrhs * c->crs_n() * sizeof(double2);
    HostIO io(c);
    const double2* ind = (const double2*)io.in(in, fb, where, "io_in");
    double2* outd = (double2*)io.out(out, cb, where, "io_out");
    int t = c->spin_t(c->h.prec);
    c->reserve({{"ap_a", c->fsz(nrhs, c->h.prec)}});
    void* a = c->W("ap_a", c->fsz(nrhs, c->h.prec));
    void* xc = c->W("ap_c", c->csz(nrhs));
    launch_pack_spinor(g, ind, a, t, c->frs(), nrhs, c->st);
    c->restrict_(a, xc, nrhs);
    launch_convert(xc, c->crs_t(), outd, C128, (size_t)nrhs * c->crs_n(), c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, outd, cb, where);
  });
}

int wcamg_prolong(wcamg_ctx* c, const void* in, void* out, int nrhs, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    require(in && out, "null pointer");
    require(c->have_hier, "no hierarchy", WCAMG_ESTATE);
    const Geo& g = c->g;
    size_t fb = (size_t)nrhs * g.V * 12 * sizeof(double2);
    size_t cb = (size_t)nrhs * c->crs_n() * sizeof(double2);
    HostIO io(c);
    const double2* ind = (const double2*)io.in(in, cb, where, "io_in");
    double2* outd = (double2*)io.out(out, fb, where, "io_out");
    int t = c->spin_t(c->h.prec);
    c->reserve({{"ap_a", c->fsz(nrhs, c->h.prec)}});
    void* xc = c->W("ap_c", c->csz(nrhs));
    void* a = c->W("ap_a", c->fsz(nrhs, c->h.prec));
    launch_convert(ind, C128, xc, c->crs_t(), (size_t)nrhs * c->crs_n(), c->st);
    c->prolong_(xc, a, nrhs);
    launch_unpack_spinor(g, a, t, c->frs(), outd, nrhs, c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, outd, fb, where);
  });
}

int wcamg_get_coarse_op(wcamg_ctx* c, int level, void* Dc, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(Dc, "null pointer");
    require(level == 1 || level == 2, "level must be 1 or 2");
    require(c->have_hier || (level == 2 && c->h.l1 && c->h.Dc2.p), "no hierarchy", WCAMG_ESTATE);
    require(level == 1 || c->h.l1, "no level-2 operator (nlevels < 3)", WCAMG_ESTATE);
    COp o = level == 1 ? c->op1() : c->op2();
    int N = o.N;
    size_t nel = (size_t)o.cg.NC * 9 * N * N;
    void* tmp = c->W("gc_tmp", nel * sizeof(double2));
    launch_convert(o.Dc, c->crs_t(), tmp, C128, nel, c->st);
    std::vector<double2> hst(nel), tr(nel);
    HIPCHK(hipMemcpyAsync(hst.data(), tmp, nel * sizeof(double2), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    // internal [X][d][m][n] -> [X][d][n][m]
    for (size_t xd = 0; xd < (size_t)o.cg.NC * 9; ++xd)
      for (int m = 0; m < N; ++m)
        for (int n = 0; n < N; ++n) tr[(xd * N + n) * N + m] = hst[(xd * N + m) * N + n];
    HIPCHK(hipMemcpy(Dc, tr.data(), nel * sizeof(double2),
                     where == WCAMG_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
  });
}

int wcamg_set_level1_vectors(wcamg_ctx* c, const void* Wv, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(Wv, "null pointer");
    require(c->have_hier && c->h.l1, "needs a hierarchy set up with nlevels = 3", WCAMG_ESTATE);
    size_t nel = (size_t)c->h.nw * c->op1().n();
    HostIO io(c);
    const void* Wd = io.in(Wv, nel * sizeof(double2), where, "io_in");
    c->h.W.ensure(nel * ct_size(c->crs_t()), false);
    launch_convert(Wd, C128, c->h.W.p, c->crs_t(), nel, c->st);
    c->build_coarse2();
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcamg_get_level1_vectors(wcamg_ctx* c, void* Wv, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(Wv, "null pointer");
    require(c->have_hier && c->h.l1, "no level-1 vectors", WCAMG_ESTATE);
    size_t nel = (size_t)c->h.nw * c->op1().n();
    HostIO io(c);
    void* Wd = io.out(Wv, nel * sizeof(double2), where, "io_out");
    launch_convert(c->h.W.p, c->crs_t(), Wd, C128, nel, c->st);
    HIPCHK(hipGetLastError());
    io.finish(Wv, Wd, nel * sizeof(double2), where);
  });
}

// the coarse operator of a level (1: Dc; 2: the level-2 operator of a
// three-level hierarchy), with the state checks of the coarse-level entry points
static COp level_op(wcamg_ctx* c, int level) {
  require(level == 1 || level == 2, "level must be 1 or 2");
  require(c->have_hier, "no hierarchy", WCAMG_ESTATE);
  require(level == 1 || c->h.l1, "no level-2 operator (nlevels < 3)", WCAMG_ESTATE);
  return level == 1 ? c->op1() : c->op2();
}

int wcamg_set_coarse_op(wcamg_ctx* c, int level, const void* Dc, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(Dc, "null pointer");
    COp o = level_op(c, level);
    int N = o.N;
    size_t nel = (size_t)o.cg.NC * 9 * N * N;
    std::vector<double2> hst(nel), tr(nel);
    HIPCHK(hipMemcpy(hst.data(), Dc, nel * sizeof(double2),
                     where == WCAMG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    // canonical [X][d][n][m] -> internal [X][d][m][n]
    for (size_t xd = 0; xd < (size_t)o.cg.NC * 9; ++xd)
      for (int m = 0; m < N; ++m)
        for (int n = 0; n < N; ++n) tr[(xd * N + m) * N + n] = hst[(xd * N + n) * N + m];
    void* tmp = c->W("gc_tmp", nel * sizeof(double2));
    HIPCHK(hipMemcpyAsync(tmp, tr.data(), nel * sizeof(double2), hipMemcpyHostToDevice, c->st));
    launch_convert(tmp, C128, o.Dc, c->crs_t(), nel, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcamg_apply_coarse(wcamg_ctx* c, int level, const void* in, void* out, int nrhs, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    require(in && out && in != out, "null or aliasing pointers");
    COp o = level_op(c, level);
    size_t n = (size_t)nrhs * o.n();
    size_t cb = n * sizeof(double2);
    HostIO io(c);
    const double2* ind = (const double2*)io.in(in, cb, where, "io_in");
    double2* outd = (double2*)io.out(out, cb, where, "io_out");
    void* a = c->W("ap_c", c->csz(o, nrhs));
    void* b = c->W("ap_c2", c->csz(o, nrhs));
    launch_convert(ind, C128, a, c->crs_t(), n, c->st);
    c->coarse_mv(o, a, b, nullptr, nrhs);
    launch_convert(b, c->crs_t(), outd, C128, n, c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, outd, cb, where);
  });
}

int wcamg_coarse_solve(wcamg_ctx* c, int level, const void* b, void* x, int nrhs, int iters, double tol,
                       int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    require(b && x && b != x, "null or aliasing pointers");
    require(iters >= 0 && std::isfinite(tol) && tol >= 0, "invalid iteration count or tolerance");
    COp o = level_op(c, level);
    size_t n = (size_t)nrhs * o.n();
    size_t cb = n * sizeof(double2);
    HostIO io(c);
    const double2* bd = (const double2*)io.in(b, cb, where, "io_in");
    double2* xd = (double2*)io.out(x, cb, where, "io_out");
    void* a = c->W("ap_c", c->csz(o, nrhs));
    void* y = c->W("ap_c2", c->csz(o, nrhs));
    launch_convert(bd, C128, a, c->crs_t(), n, c->st);
    c->coarse_solve(o, a, y, nrhs, iters, tol);
    launch_convert(y, c->crs_t(), xd, C128, n, c->st);
    HIPCHK(hipGetLastError());
    io.finish(x, xd, cb, where);
  });
}

int wcamg_vcycle(wcamg_ctx* c, const void* in, void* out, int nrhs, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    check_nrhs(nrhs);
    require(in && out, "null pointer");
    require(c->have_hier, "no hierarchy", WCAMG_ESTATE);
    const Geo& g = c->g;
    size_t fb = (size_t)nrhs * g.V * 12 * sizeof(double2);
    HostIO io(c);
    const double2* ind = (const double2*)io.in(in, fb, where, "io_in");
    double2* outd = (double2*)io.out(out, fb, where, "io_out");
    int prec = c->h.prec, t = c->spin_t(prec);
    c->reserve({{"ap_a", c->fsz(nrhs, prec)}, {"ap_b", c->fsz(nrhs, prec)}, {"vc_r", c->fsz(nrhs, prec)},
                {"vc_x1", c->fsz(nrhs, prec)}, {"sap_r", c->fsz(nrhs, prec)}, {"sap_d", c->sapd_sz(nrhs, prec)}});
    void* a = c->W("ap_a", c->fsz(nrhs, prec));
    void* b = c->W("ap_b", c->fsz(nrhs, prec));
    launch_pack_spinor(g, ind, a, t, c->frs(), nrhs, c->st);
    c->vcycle(a, b, nrhs);
    launch_unpack_spinor(g, b, t, c->frs(), outd, nrhs, c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, outd, fb, where);
  });
}

// ---------------------------------------------------------------------------
// Outer solver: FGMRES(m), FP64, right preconditioning with the V-cycle
// ---------------------------------------------------------------------------
static void fgmres_batch(wcamg_ctx* c, const double2* bb, double2* xx, int nrhs, const wcamg_solve_params* p,
                         int* iters, double* relres, int* conv, int* vcycles) {
  const Geo& g = c->g;
  const int m = p->restart;
  const int prec = c->h.prec;
  const size_t n = (size_t)12 * g.V;  // complex numbers per rhs
  const size_t rs = n;
  const size_t vs = (size_t)nrhs * n;  // stride between basis vectors
  int zt = c->spin_t(prec);
  double2* V = (double2*)c->W("fg_V", (size_t)(m + 1) * vs * sizeof(double2));
  void* Z = c->W("fg_Z", (size_t)m * vs * ct_size(zt));
  void* vin = prec == WCAMG_PREC_MIXED ? c->W("fg_vin", vs * sizeof(float2)) : nullptr;
  double2* part = (double2*)c->W("fg_part", (size_t)nrhs * reduce_nwg(n) * (2 * GS_CHUNK + 3) * sizeof(double2));
  double* wwd = (double*)c->W("fg_ww", (size_t)nrhs * sizeof(double));
  const bool delayed = p->ortho == 0;  // CGS2 with the second pass delayed into the next step
  double2* coef = (double2*)c->W("fg_c", (size_t)2 * (m + 2 + m / GS_CHUNK) * nrhs * sizeof(double2));
  double2* h1 = (double2*)c->W("fg_h1", (size_t)(m + 1) * nrhs * sizeof(double2));
  double2* h2 = (double2*)c->W("fg_h2", (size_t)(m + 1) * nrhs * sizeof(double2));
  double* nrm = (double*)c->W("fg_nrm", (size_t)nrhs * sizeof(double));
  double* scl = (double*)c->W("fg_scl", (size_t)nrhs * sizeof(double));
  double2* ycoef = (double2*)c->W("fg_y", (size_t)m * nrhs * sizeof(double2));

  auto sync_get = [&](void* host, const void* dev, size_t bytes) {
    HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  };

  std::vector<double> bn2(nrhs), hn(nrhs), hs(nrhs), wwh(nrhs), vsc(nrhs);
  launch_norm2(bb, C128, n, rs, nrhs, part, nrm, c->st);
  sync_get(bn2.data(), nrm, nrhs * sizeof(double));
  for (int r = 0; r < nrhs; ++r) require(std::isfinite(bn2[r]), "non-finite right-hand side", WCAMG_ENUMERIC);
  launch_zero(xx, vs * sizeof(double2), c->st);
  std::vector<int> its(nrhs, 0), done(nrhs, 0);
  for (int r = 0; r < nrhs; ++r)
    if (bn2[r] == 0.0) done[r] = 1;

  // graph per Z slot (mixed precision only: the V-cycle input is the fixed FP32 buffer)
  auto run_vcycle = [&](int j) {
    void* zj = (char*)Z + (size_t)j * vs * ct_size(zt);
    const void* in = prec == WCAMG_PREC_MIXED ? vin : (const void*)(V + (size_t)j * vs);
    wcamg_ctx::Phase ph(c, wcamg_ctx::PH_PRECOND);
    if (!p->use_graph || c->timing || c->phase_on) {
      c->vcycle(in, zj, nrhs);
      return;
    }
    c->validate_graphs();
    auto key = std::make_pair(j, nrhs);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end() || c->graph_prec != prec) {
      if (c->graph_prec != prec) c->drop_graphs();
      // allocate every workspace first with an uncaptured run
      if (c->graphs.empty()) c->vcycle(in, zj, nrhs);
      // capture on a library-owned stream (the caller's stream may be one
      // that cannot be captured), replay on the caller's stream
      if (!c->cap_st) HIPCHK(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
      HIPCHK(hipStreamSynchronize(c->st));
      hipGraph_t gr;
      hipStream_t user = c->st;
      c->st = c->cap_st;
      c->capturing = true;
      try {
        HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
        c->vcycle(in, zj, nrhs);
        HIPCHK(hipStreamEndCapture(c->st, &gr));
      } catch (...) {
        hipGraph_t junk;
        (void)hipStreamEndCapture(c->st, &junk);
        c->st = user;
        c->capturing = false;
        throw;
      }
      c->st = user;
      c->capturing = false;
      hipGraphExec_t ex;
      HIPCHK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
      HIPCHK(hipGraphDestroy(gr));
      if (c->graphs.empty()) {
        c->graph_epoch = g_alloc_epoch.load();
        c->graph_sig = c->hier_sig();
      } else if (c->graph_epoch != g_alloc_epoch.load()) {
        // a buffer moved while this graph was captured: the others are stale
        c->drop_graphs();
        c->graph_epoch = g_alloc_epoch.load();
        c->graph_sig = c->hier_sig();
      }
      c->graphs[key] = ex;
      c->graph_prec = prec;
      it = c->graphs.find(key);
    }
    HIPCHK(hipGraphLaunch(it->second, c->st));
  };

  // raw Hessenberg matrix H[i][j][r] of the current cycle; the least-squares
  // problem is solved from it by Givens rotations after every step
  std::vector<cd> H((size_t)(m + 1) * m * nrhs);
  std::vector<double> beta(nrhs);
  std::vector<double2> hh1((size_t)(m + 1) * nrhs), hh2((size_t)(m + 1) * nrhs), hc;
  std::vector<int> kcols(nrhs);
  std::vector<double2> yhost((size_t)m * nrhs);
  auto Hc = [&](int i, int j, int r) -> cd& { return H[((size_t)i * m + j) * nrhs + r]; };
  // min_y || beta e_0 - H y || over the first k columns, rotations (c real,
  // s complex) applied to a copy; returns the residual norm, y if asked
  auto lsq = [&](int r, int k, std::vector<cd>* y) -> double {
    std::vector<cd> R((size_t)(k + 1) * std::max(k, 1)), gv(k + 1, cd(0)), cs(k), sn(k);
    auto Rc = [&](int i, int j) -> cd& { return R[(size_t)i * k + j]; };
    gv[0] = beta[r];
    for (int j = 0; j < k; ++j) {
      for (int i = 0; i <= j + 1; ++i) Rc(i, j) = Hc(i, j, r);
      for (int i = 0; i < j; ++i) {
        cd t = cs[i] * Rc(i, j) + sn[i] * Rc(i + 1, j);
        Rc(i + 1, j) = -std::conj(sn[i]) * Rc(i, j) + cs[i] * Rc(i + 1, j);
        Rc(i, j) = t;
      }
      cd a = Rc(j, j), bq = Rc(j + 1, j);
      double den = std::sqrt(std::norm(a) + std::norm(bq));
      if (den == 0) {
        cs[j] = 1;
        sn[j] = 0;
      } else if (std::abs(a) == 0) {
        cs[j] = 0;
        sn[j] = std::conj(bq) / std::abs(bq);
      } else {
        cs[j] = std::abs(a) / den;
        sn[j] = (a / std::abs(a)) * std::conj(bq) / den;
      }
      Rc(j, j) = cs[j] * Rc(j, j) + sn[j] * Rc(j + 1, j);
      Rc(j + 1, j) = 0;
      gv[j + 1] = -std::conj(sn[j]) * gv[j];
      gv[j] = cs[j] * gv[j];
    }
    if (y) {
      y->assign(k, cd(0));
      for (int i = k - 1; i >= 0; --i) {
        cd sum = gv[i];
        for (int l = i + 1; l < k; ++l) sum -= Rc(i, l) * (*y)[l];
        (*y)[i] = Rc(i, i) != cd(0) ? sum / Rc(i, i) : cd(0);
      }
    }
    return std::abs(gv[k]);
  };
  auto gs_args = [&](int k0, int nq, double2* pv, double2* w) {
    GsArgs a;
    a.Q = V + (size_t)k0 * vs;
    a.vs = vs;
    a.nq = nq;
    a.p = pv;
    a.w = w;
    a.n = n;
    a.rs = rs;
    a.nrhs = nrhs;
    a.part = part;
    return a;
  };

  bool x_zero = true;  // x = 0 until the first update: then r = b exactly
  while (true) {
    // r = b - D x (FP64), into V_0
    std::vector<double> rn2(nrhs);
    if (x_zero) {
      rn2 = bn2;
    } else {
      c->dslash(xx, C128, V, C128, nrhs, OP_D, WCAMG_PREC_FP64, bb);
      launch_norm2(V, C128, n, rs, nrhs, part, nrm, c->st);
      sync_get(rn2.data(), nrm, nrhs * sizeof(double));
    }
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      require(std::isfinite(rn2[r]), "non-finite residual", WCAMG_ENUMERIC);
      relres[r] = bn2[r] > 0 ? std::sqrt(rn2[r] / bn2[r]) : 0.0;
      if (!done[r] && (relres[r] <= p->tol || its[r] >= p->max_iters)) done[r] = 1;
      all = all && done[r];
    }
    if (all) break;
    std::vector<double> sc(nrhs);
    std::fill(H.begin(), H.end(), cd(0));
    for (int r = 0; r < nrhs; ++r) {
      bool act = !done[r];
      beta[r] = act ? std::sqrt(rn2[r]) : 0.0;
      sc[r] = act && beta[r] > 0 ? 1.0 / beta[r] : 0.0;
      kcols[r] = 0;
    }
    HIPCHK(hipMemcpyAsync(scl, sc.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
    launch_scale(x_zero ? bb : V, scl, V, (float2*)vin, n, rs, nrhs, c->st);
    bool vin_done = false;       // sweep 2 wrote the next V-cycle input
    std::vector<int> ext(nrhs);  // still extending its Krylov space in this cycle
    for (int r = 0; r < nrhs; ++r) ext[r] = !done[r];
    for (int j = 0; j < m; ++j) {
      run_vcycle(j);
      *vcycles += 1;
      void* zj = (char*)Z + (size_t)j * vs * ct_size(zt);
      double2* pj = V + (size_t)j * vs;
      double2* w = V + (size_t)(j + 1) * vs;
      c->dslash(zj, zt, w, C128, nrhs, OP_D, WCAMG_PREC_FP64);
      const double vb = (double)vs * sizeof(double2);
      std::vector<int> was = ext;
      if (delayed) {
        // Delayed classical Gram-Schmidt twice.  V_0..V_{j-1} are final and
        // V_j = p holds the previous step's vector after one projection.
        // Sweep 1: the projections of w and p on the basis and on p; from
        // them the second projection of p (s, rho), the correction of
        // column j-1 (H[i][j-1] += s_i, H[j][j-1] = rho) and column j.
        // Sweep 2: V_j = (p - sum_i s_i V_i) / rho and the first projection
        // of w on V_0..V_j; w becomes the next p.  In mixed precision sweep 2
        // also writes the next V-cycle's FP32 input, w normalised by the norm
        // that sweep 1 predicts (|w|^2 minus the squared projections), unless
        // that prediction cancels.  Class "gs": the j + 1 basis vectors and w
        // read twice, w and V_j written, and the FP32 input (half a vector).
        wcamg_ctx::Timed tg(c, "gs", vb * (2.0 * (j + 1) + 2.0 + (j > 0 ? 2.0 : 1.0) + (vin ? 0.5 : 0.0)),
                            8.0 * (4.0 * (j + 1) + 1.0) * (double)vs, nrhs);
        for (int k0 = 0; k0 == 0 || k0 < j; k0 += GS_CHUNK) {
          GsArgs a = gs_args(k0, std::min(GS_CHUNK, j - k0), pj, w);
          a.h1 = h1 + (size_t)k0 * nrhs;
          a.h2 = h2 + (size_t)k0 * nrhs;
          a.h1p = h1 + (size_t)j * nrhs;
          a.h2p = h2 + (size_t)j * nrhs;
          a.ww = wwd;
          launch_gs(GS_DOT2, a, c->st);
        }
        HIPCHK(hipMemcpyAsync(hh1.data(), h1, (size_t)(j + 1) * nrhs * sizeof(double2), hipMemcpyDeviceToHost,
                              c->st));
        HIPCHK(hipMemcpyAsync(wwh.data(), wwd, (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost, c->st));
        sync_get(hh2.data(), h2, (size_t)(j + 1) * nrhs * sizeof(double2));
        // coefficients of sweep 2 per chunk: c1 then c2, (nq + 1) x nrhs each
        const int nch = j == 0 ? 1 : (j + GS_CHUNK - 1) / GS_CHUNK;
        std::vector<std::vector<cd>> c1(nrhs), c2(nrhs);
        std::vector<double> rho(nrhs, 1.0);
        bool fused = vin != nullptr;
        for (int r = 0; r < nrhs; ++r) {
          c1[r].assign(j + 1, cd(0));
          c2[r].assign(j + 1, cd(0));
          vsc[r] = 0.0;
          if (!ext[r]) continue;
          auto cx = [](double2 v) { return cd(v.x, v.y); };
          std::vector<cd> s(j);
          double ss = 0;
          for (int i = 0; i < j; ++i) {
            s[i] = cx(hh2[(size_t)i * nrhs + r]);
            ss += std::norm(s[i]);
          }
          if (j > 0) {
            double rho2 = hh2[(size_t)j * nrhs + r].x - ss;
            require(std::isfinite(rho2), "non-finite Arnoldi norm", WCAMG_ENUMERIC);
            for (int i = 0; i < j; ++i) Hc(i, j - 1, r) += s[i];
            if (!(rho2 > 0)) {
              // p lies in the span of V_0..V_{j-1}: the space is invariant
              Hc(j, j - 1, r) = 0;
              ext[r] = 0;
              continue;
            }
            rho[r] = std::sqrt(rho2);
            Hc(j, j - 1, r) = rho[r];
          }
          cd bj = cx(hh1[(size_t)j * nrhs + r]);
          for (int i = 0; i < j; ++i) {
            cd ai = cx(hh1[(size_t)i * nrhs + r]);
            Hc(i, j, r) = ai;
            bj -= std::conj(s[i]) * ai;
          }
          bj /= rho[r];
          Hc(j, j, r) = bj;
          for (int i = 0; i < j; ++i) {
            c1[r][i] = -s[i] / rho[r];
            c2[r][i] = Hc(i, j, r) - bj * s[i] / rho[r];
          }
          c1[r][j] = 1.0 / rho[r];
          c2[r][j] = bj / rho[r];
          // |new w|^2 = |w|^2 - sum_i |H[i][j]|^2 (V_0..V_j orthonormal)
          double est = wwh[r] - std::norm(bj);
          for (int i = 0; i < j; ++i) est -= std::norm(Hc(i, j, r));
          if (std::isfinite(est) && est > 1e-12 * wwh[r])
            vsc[r] = 1.0 / std::sqrt(est);
          else
            fused = false;
        }
        if (fused) HIPCHK(hipMemcpyAsync(scl, vsc.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
        hc.clear();
        std::vector<size_t> co;
        for (int ch = 0; ch < nch; ++ch) {
          const int k0 = ch * GS_CHUNK, nq = std::min(GS_CHUNK, j - k0);
          co.push_back(hc.size());
          for (int half = 0; half < 2; ++half)
            for (int k = 0; k <= nq; ++k)
              for (int r = 0; r < nrhs; ++r) {
                const std::vector<cd>& cc = half ? c2[r] : c1[r];
                cd v = k < nq ? cc[k0 + k] : ch == 0 ? cc[j] : cd(half ? 0.0 : 1.0);
                hc.push_back(make_double2(v.real(), v.imag()));
              }
        }
        HIPCHK(hipMemcpyAsync(coef, hc.data(), hc.size() * sizeof(double2), hipMemcpyHostToDevice, c->st));
        for (int ch = 0; ch < nch; ++ch) {
          const int k0 = ch * GS_CHUNK, nq = std::min(GS_CHUNK, j - k0);
          GsArgs a = gs_args(k0, nq, pj, w);
          a.c1 = coef + co[ch];
          a.c2 = a.c1 + (size_t)(nq + 1) * nrhs;
          a.write_p = j > 0;
          a.norm2 = ch == nch - 1 ? nrm : nullptr;
          if (fused && ch == nch - 1) {
            a.vin = (float2*)vin;
            a.vscale = scl;
          }
          launch_gs(GS_COMB2, a, c->st);
        }
        vin_done = fused;
      } else {
        // Classical Gram-Schmidt twice; the update of the first pass and the
        // projections of the second share one sweep over the basis.  Class
        // "gs": the j + 1 basis vectors read three times, w read three times
        // and written twice
        wcamg_ctx::Timed tg(c, "gs", vb * (3.0 * (j + 1) + 5.0), 8.0 * 3 * (j + 1) * (double)vs, nrhs);
        const int nk = j + 1;
        auto sweep = [&](int mode, const double2* cf, double2* out, double* norm2) {
          for (int k0 = 0; k0 < nk; k0 += GS_CHUNK) {
            GsArgs a = gs_args(k0, std::min(GS_CHUNK, nk - k0), nullptr, w);
            a.c1 = cf ? cf + (size_t)k0 * nrhs : nullptr;
            a.h1 = out ? out + (size_t)k0 * nrhs : nullptr;
            a.norm2 = k0 + GS_CHUNK >= nk ? norm2 : nullptr;
            launch_gs(mode, a, c->st);
          }
        };
        sweep(GS_DOT, nullptr, h1, nullptr);
        if (nk <= GS_CHUNK) {
          sweep(GS_AXPY_DOT, h1, h2, nullptr);
        } else {
          sweep(GS_AXPY_NORM, h1, nullptr, nullptr);
          sweep(GS_DOT, nullptr, h2, nullptr);
        }
        sweep(GS_AXPY_NORM, h2, nullptr, nrm);
        HIPCHK(hipMemcpyAsync(hh1.data(), h1, (size_t)nk * nrhs * sizeof(double2), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(hh2.data(), h2, (size_t)nk * nrhs * sizeof(double2), hipMemcpyDeviceToHost, c->st));
        for (int r = 0; r < nrhs; ++r)
          if (ext[r])
            for (int i = 0; i <= j; ++i) {
              size_t o = (size_t)i * nrhs + r;
              Hc(i, j, r) = cd(hh1[o].x + hh2[o].x, hh1[o].y + hh2[o].y);
            }
      }
      std::fill(hs.begin(), hs.end(), 0.0);
      sync_get(hn.data(), nrm, nrhs * sizeof(double));
      bool any = false, died = false;
      for (int r = 0; r < nrhs; ++r) {
        if (!ext[r]) {
          died = died || was[r];  // an invariant space found by the delayed pass
          continue;
        }
        double hnr = std::sqrt(std::max(hn[r], 0.0));
        require(std::isfinite(hnr), "non-finite Arnoldi norm", WCAMG_ENUMERIC);
        Hc(j + 1, j, r) = hnr;
        hs[r] = hnr > 0 ? 1.0 / hnr : 0.0;
        its[r] += 1;
        kcols[r] = j + 1;
        double est = lsq(r, j + 1, nullptr);
        if (est <= p->tol * std::sqrt(bn2[r]) || hnr == 0 || its[r] >= p->max_iters) {
          ext[r] = 0;
          hs[r] = 0.0;
          died = true;
        }
        any = any || ext[r];
      }
      if (!any || j == m - 1) break;
      // the next V-cycle input: V_{j+1} normalised (CGS2), or w normalised
      // into the FP32 input (delayed, mixed precision; done by sweep 2 unless
      // its norm prediction cancelled); right-hand sides that stopped get a
      // zero input (after a fused write, those that stopped in this step keep
      // theirs: its V-cycle output enters no solution, y being 0 there)
      if (!delayed) {
        HIPCHK(hipMemcpyAsync(scl, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
        launch_scale(w, scl, w, (float2*)vin, n, rs, nrhs, c->st);
      } else if (vin) {
        if (!vin_done) {
          HIPCHK(hipMemcpyAsync(scl, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
          launch_scale(w, scl, nullptr, (float2*)vin, n, rs, nrhs, c->st);
        }
      } else if (died) {
        for (int r = 0; r < nrhs; ++r) hs[r] = ext[r] ? 1.0 : 0.0;
        HIPCHK(hipMemcpyAsync(scl, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
        launch_scale(w, scl, w, nullptr, n, rs, nrhs, c->st);
      }
    }
    // y = argmin || beta e_0 - H y || per rhs, x += Z y
    int kmax = 0;
    for (int r = 0; r < nrhs; ++r) {
      int k = kcols[r];
      kmax = std::max(kmax, k);
      std::vector<cd> y;
      if (k > 0) lsq(r, k, &y);
      for (int i = 0; i < m; ++i) {
        cd v = i < k ? y[i] : cd(0);
        yhost[(size_t)i * nrhs + r] = make_double2(v.real(), v.imag());
      }
    }
    if (kmax > 0) {
      HIPCHK(hipMemcpyAsync(ycoef, yhost.data(), (size_t)m * nrhs * sizeof(double2), hipMemcpyHostToDevice, c->st));
      launch_update_x(xx, Z, zt, vs, kmax, ycoef, n, rs, nrhs, c->st);
      x_zero = false;
    }
  }
  for (int r = 0; r < nrhs; ++r) {
    iters[r] = its[r];
    conv[r] = relres[r] <= p->tol;
  }
}

// Solve-phase timing for one solve call: switched on when the caller asks
// for it, switched off on every exit; fill() writes the split into info.
struct PhaseScope {
  wcamg_ctx* c;
  PhaseScope(wcamg_ctx* c_, bool on) : c(c_) {
    c->phase_on = on;
    for (double& v : c->phase_ms) v = 0;
    c->phase_pending.clear();
  }
  ~PhaseScope() {
    c->phase_on = false;
    for (auto& p : c->phase_pending) {
      c->evpool.push_back(p.a);
      c->evpool.push_back(p.b);
    }
    c->phase_pending.clear();
  }
  void fill(wcamg_solve_info& inf) {
    if (!c->phase_on) return;
    c->collect_phases();
    const double* ms = c->phase_ms;
    inf.t_precond = ms[wcamg_ctx::PH_PRECOND] * 1e-3;
    inf.t_coarse = ms[wcamg_ctx::PH_COARSE] * 1e-3;
    inf.t_smoother = ms[wcamg_ctx::PH_SMOOTH] * 1e-3;
    inf.t_rp = ms[wcamg_ctx::PH_RP] * 1e-3;
    inf.t_prec_other = std::max(0.0, inf.t_precond - inf.t_coarse - inf.t_smoother - inf.t_rp);
    inf.t_outer = std::max(0.0, inf.t_solve - inf.t_precond);
  }
};

int wcamg_solve(wcamg_ctx* c, const void* b, void* x, int nrhs, const wcamg_solve_params* p,
                wcamg_solve_info* info) {
  if (!c) return WCAMG_EINVAL;
  int status = WCAMG_OK;
  int rc = guard(c, [&] {
    require(b && x && p, "null pointer");
    check_nrhs(nrhs);
    require(p->restart >= 1 && p->restart <= 32, "restart must be in [1, 32]");
    require(p->ortho == 0 || p->ortho == 1, "ortho must be 0 (delayed CGS2) or 1 (CGS2)");
    require(std::isfinite(p->tol) && p->tol >= 0, "invalid tol");
    require(p->max_iters >= 0, "invalid max_iters");
    require(c->have_hier, "no hierarchy: call wcamg_setup first", WCAMG_ESTATE);
    PhaseScope phases(c, p->phase_times != 0);
    auto t0 = std::chrono::steady_clock::now();
    const Geo& g = c->g;
    size_t n = (size_t)12 * g.V;
    int chunk = p->rhs_chunk > 0 ? std::min(p->rhs_chunk, nrhs) : nrhs;
    {
      // packed b and x, the FP64 Krylov basis, the preconditioned vectors,
      // the V-cycle's input and the fine fields inside the V-cycle
      const int prec = c->h.prec;
      const size_t cn = (size_t)chunk * n, f = c->fsz(chunk, prec);
      std::vector<std::pair<std::string, size_t>> plan = {
          {"sv_b", cn * sizeof(double2)},
          {"sv_x", cn * sizeof(double2)},
          {"fg_V", (size_t)(p->restart + 1) * cn * sizeof(double2)},
          {"fg_Z", (size_t)p->restart * cn * ct_size(c->spin_t(prec))},
          {"vc_r", f},
          {"vc_x1", f},
          {"sap_r", f},
          {"sap_d", c->sapd_sz(chunk, prec)}};
      if (prec == WCAMG_PREC_MIXED) plan.push_back({"fg_vin", cn * sizeof(float2)});
      c->reserve(plan);
    }
    wcamg_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    for (int r0 = 0; r0 < nrhs; r0 += chunk) {
      int nr = std::min(chunk, nrhs - r0);
      double2* bb = (double2*)c->W("sv_b", (size_t)nr * n * sizeof(double2));
      double2* xx = (double2*)c->W("sv_x", (size_t)nr * n * sizeof(double2));
      launch_pack_spinor(g, (const double2*)b + (size_t)r0 * n, bb, C128, n, nr, c->st);
      fgmres_batch(c, bb, xx, nr, p, inf.iters + r0, inf.relres + r0, inf.converged + r0, &inf.vcycles);
      launch_unpack_spinor(g, xx, C128, n, (double2*)x + (size_t)r0 * n, nr, c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    inf.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    phases.fill(inf);
    for (int r = 0; r < nrhs; ++r)
      if (!inf.converged[r]) status = WCAMG_NOT_CONVERGED;
    if (info) *info = inf;
  });
  return rc != WCAMG_OK ? rc : status;
}

// The paper's flexible BiCGStab (Sec. 3) in FP64 on one batch of right-hand
// sides, from x = 0, with M = the V-cycle or the FP32 BiCGStab.  Scalars per
// right-hand side live on the device (BicgScal); a right-hand side stops
// when its recursive residual reaches tol (relative to b).
static void fbicg_batch(wcamg_ctx* c, const double2* bb, double2* xx, int nrhs, const wcamg_bicg_params* p,
                        int* iters, double* relres, int* conv, int* vcycles) {
  const Geo& g = c->g;
  const size_t n = (size_t)12 * g.V, rs = n, vs = (size_t)nrhs * n;
  const bool amg = p->precond == WCAMG_PC_AMG;
  const int prec = amg ? c->h.prec : WCAMG_PREC_MIXED;
  const int zt = c->spin_t(prec);
  double2* r = (double2*)c->W("fb_r", vs * sizeof(double2));
  double2* rt = (double2*)c->W("fb_rt", vs * sizeof(double2));
  double2* pp = (double2*)c->W("fb_p", vs * sizeof(double2));
  double2* v = (double2*)c->W("fb_v", vs * sizeof(double2));
  double2* s = (double2*)c->W("fb_s", vs * sizeof(double2));
  double2* t = (double2*)c->W("fb_t", vs * sizeof(double2));
  void* Mp = c->W("fb_mp", vs * ct_size(zt));
  void* Ms = c->W("fb_ms", vs * ct_size(zt));
  float2* vin = prec == WCAMG_PREC_MIXED ? (float2*)c->W("fb_vin", vs * sizeof(float2)) : nullptr;
  double2* part = (double2*)c->W("fb_part", (size_t)nrhs * reduce_nwg(n) * 3 * sizeof(double2));
  BicgScal* sc = (BicgScal*)c->W("fb_sc", (size_t)nrhs * sizeof(BicgScal));
  double* ones = (double*)c->W("fb_one", (size_t)nrhs * sizeof(double));
  double* nrm = (double*)c->W("fb_nrm", (size_t)nrhs * sizeof(double));
  {
    std::vector<double> one(nrhs, 1.0);
    HIPCHK(hipMemcpyAsync(ones, one.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
  }
  // out = M in (in: FP64 batch; the mixed preconditioners take an FP32 copy)
  auto precond = [&](double2* in, void* out) {
    const void* src = in;
    if (vin) {
      launch_scale(in, ones, in, vin, n, rs, nrhs, c->st);
      src = vin;
    }
    wcamg_ctx::Phase ph(c, wcamg_ctx::PH_PRECOND);
    if (amg)
      c->vcycle(src, out, nrhs);
    else
      c->bicg32(src, out, nrhs, p->inner_iters, p->inner_tol);
    *vcycles += 1;
  };
  launch_bicg_init(bb, xx, r, rt, pp, v, C128, n, rs, nrhs, p->tol, part, sc, c->st);
  std::vector<BicgScal> hs(nrhs);
  for (int it = 0; it < p->max_iters; ++it) {
    launch_bicg_p(pp, r, v, C128, n, rs, nrhs, sc, c->st);  // p = r + beta (p - omega v)
    precond(pp, Mp);
    c->dslash(Mp, zt, v, C128, nrhs, OP_D, WCAMG_PREC_FP64);  // v = D M p
    launch_bicg_alpha(rt, v, C128, n, rs, nrhs, part, sc, c->st);
    launch_bicg_s(s, r, v, C128, n, rs, nrhs, sc, c->st);  // s = r - alpha v
    precond(s, Ms);
    c->dslash(Ms, zt, t, C128, nrhs, OP_D, WCAMG_PREC_FP64);  // t = D M s
    launch_bicg_omega(t, s, C128, n, rs, nrhs, part, sc, 0.0, c->st);
    launch_fbicg_x(xx, Mp, Ms, zt, n, rs, nrhs, sc, c->st);  // x += alpha M p + omega M s
    launch_bicg_xr(nullptr, r, nullptr, s, t, rt, C128, n, rs, nrhs, part, sc, c->st);  // r = s - omega t
    HIPCHK(hipMemcpyAsync(hs.data(), sc, nrhs * sizeof(BicgScal), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    bool any = false;
    for (auto& q : hs) {
      require(std::isfinite(q.rnorm2), "non-finite residual", WCAMG_ENUMERIC);
      any |= q.active != 0;
    }
    if (!any) break;
  }
  // true residual with the FP64 operator
  std::vector<double> bn2(nrhs), rn2(nrhs);
  launch_norm2(bb, C128, n, rs, nrhs, part, nrm, c->st);
  HIPCHK(hipMemcpyAsync(bn2.data(), nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, c->st));
  c->dslash(xx, C128, r, C128, nrhs, OP_D, WCAMG_PREC_FP64, bb);  // r = b - D x
  launch_norm2(r, C128, n, rs, nrhs, part, nrm, c->st);
  HIPCHK(hipMemcpyAsync(rn2.data(), nrm, nrhs * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  for (int q = 0; q < nrhs; ++q) {
    relres[q] = bn2[q] > 0 ? std::sqrt(rn2[q] / bn2[q]) : 0.0;
    iters[q] = hs[q].iters;
    conv[q] = relres[q] <= p->tol;
  }
}

int wcamg_solve_bicgstab(wcamg_ctx* c, const void* b, void* x, int nrhs, const wcamg_bicg_params* p,
                         wcamg_solve_info* info) {
  if (!c) return WCAMG_EINVAL;
  int status = WCAMG_OK;
  int rc = guard(c, [&] {
    require(b && x && p, "null pointer");
    check_nrhs(nrhs);
    require(std::isfinite(p->tol) && p->tol >= 0, "invalid tol");
    require(p->max_iters >= 0, "invalid max_iters");
    require(p->precond == WCAMG_PC_AMG || p->precond == WCAMG_PC_BICG32, "unknown preconditioner");
    if (p->precond == WCAMG_PC_AMG) require(c->have_hier, "no hierarchy: call wcamg_setup first", WCAMG_ESTATE);
    if (p->precond == WCAMG_PC_BICG32)
      require(p->inner_iters >= 1 && std::isfinite(p->inner_tol) && p->inner_tol >= 0,
              "inner_iters must be >= 1 and inner_tol finite and >= 0");
    PhaseScope phases(c, p->phase_times != 0);
    auto t0 = std::chrono::steady_clock::now();
    const Geo& g = c->g;
    const size_t n = (size_t)12 * g.V;
    const int chunk = p->rhs_chunk > 0 ? std::min(p->rhs_chunk, nrhs) : nrhs;
    {
      // packed b and x, the six FP64 vectors and two preconditioned ones of
      // the iteration, and the fields inside the preconditioner
      const bool amg = p->precond == WCAMG_PC_AMG;
      const int prec = amg ? c->h.prec : WCAMG_PREC_MIXED;
      const size_t cn = (size_t)chunk * n, d = cn * sizeof(double2), z = cn * ct_size(c->spin_t(prec));
      const size_t f = c->fsz(chunk, prec);
      std::vector<std::pair<std::string, size_t>> plan = {
          {"sv_b", d}, {"sv_x", d}, {"fb_r", d}, {"fb_rt", d}, {"fb_p", d}, {"fb_v", d}, {"fb_s", d}, {"fb_t", d},
          {"fb_mp", z}, {"fb_ms", z}};
      if (prec == WCAMG_PREC_MIXED) plan.push_back({"fb_vin", cn * sizeof(float2)});
      if (amg) {
        for (const char* k : {"vc_r", "vc_x1", "sap_r"}) plan.push_back({k, f});
        plan.push_back({"sap_d", c->sapd_sz(chunk, prec)});
      } else {
        for (const char* k : {"mb_r", "mb_rt", "mb_p", "mb_v", "mb_s", "mb_t"}) plan.push_back({k, f});
      }
      c->reserve(plan);
    }
    wcamg_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    for (int r0 = 0; r0 < nrhs; r0 += chunk) {
      const int nr = std::min(chunk, nrhs - r0);
      double2* bb = (double2*)c->W("sv_b", (size_t)nr * n * sizeof(double2));
      double2* xx = (double2*)c->W("sv_x", (size_t)nr * n * sizeof(double2));
      launch_pack_spinor(g, (const double2*)b + (size_t)r0 * n, bb, C128, n, nr, c->st);
      fbicg_batch(c, bb, xx, nr, p, inf.iters + r0, inf.relres + r0, inf.converged + r0, &inf.vcycles);
      launch_unpack_spinor(g, xx, C128, n, (double2*)x + (size_t)r0 * n, nr, c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    inf.t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    phases.fill(inf);
    for (int r = 0; r < nrhs; ++r)
      if (!inf.converged[r]) status = WCAMG_NOT_CONVERGED;
    if (info) *info = inf;
  });
  return rc != WCAMG_OK ? rc : status;
}

int wcamg_autotune(wcamg_ctx* c, int enable, const char* cache_path) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    c->tuner.enabled = enable != 0;
    if (cache_path) c->tuner.load(cache_path);
  });
}

int wcamg_autotune_info(wcamg_ctx* c, double* tune_ms, int* keys_tuned, int* keys_known) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    if (tune_ms) *tune_ms = c->tuner.tune_ms;
    if (keys_tuned) *keys_tuned = c->tuner.tuned;
    if (keys_known) *keys_known = (int)c->tuner.best.size();
  });
}

int wcamg_net_init(wcamg_ctx* c, int layers, int channels, const void* weights, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(weights, "null pointer");
    require(channels == net_channels(), "the network kernels are built for " + std::to_string(net_channels()) +
                                            " channels");
    require(layers >= 1 && layers <= 16, "layers must be in [1, 16]");
    c->net.L = layers;
    c->net.C = channels;
    c->net.t = 0;
    size_t n = c->net_wsize();
    c->net.W.ensure(n * sizeof(float2), false);
    c->net.grad.ensure(n * sizeof(float2), false);
    c->net.m.ensure(n * sizeof(float2), false);
    c->net.v.ensure(n * sizeof(float2), false);
    HostIO io(c);
    const void* wd = io.in(weights, n * sizeof(float2), where, "io_in");
    HIPCHK(hipMemcpyAsync(c->net.W.p, wd, n * sizeof(float2), hipMemcpyDeviceToDevice, c->st));
    launch_zero(c->net.m.p, n * sizeof(float2), c->st);
    launch_zero(c->net.v.p, n * sizeof(float2), c->st);
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcamg_net_get_weights(wcamg_ctx* c, void* weights, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(weights, "null pointer");
    require(c->net.L > 0, "no network", WCAMG_ESTATE);
    size_t n = c->net_wsize() * sizeof(float2);
    HostIO io(c);
    void* wd = io.out(weights, n, where, "io_out");
    HIPCHK(hipMemcpyAsync(wd, c->net.W.p, n, hipMemcpyDeviceToDevice, c->st));
    io.finish(weights, wd, n, where);
  });
}

int wcamg_net_forward(wcamg_ctx* c, const void* r, void* out, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(r && out, "null pointer");
    require(c->have_gauge && c->net.L > 0, "needs a gauge field and a network", WCAMG_ESTATE);
    const Geo& g = c->g;
    int C = c->net.C;
    size_t cb = (size_t)C * g.V * 12 * sizeof(double2);
    HostIO io(c);
    const double2* rd = (const double2*)io.in(r, cb, where, "io_in");
    double2* od = (double2*)io.out(out, cb, where, "io_out");
    c->reserve({{"nt_r", (size_t)C * 12 * g.V * sizeof(float2)}});
    void* r32 = c->W("nt_r", (size_t)C * 12 * g.V * sizeof(float2));
    launch_pack_spinor(g, rd, r32, C64, c->frs(), C, c->st);
    c->net_forward(r32);
    launch_unpack_spinor(g, c->net.acts[c->net.L], C64, c->frs(), od, C, c->st);
    HIPCHK(hipGetLastError());
    io.finish(out, od, cb, where);
  });
}

int wcamg_net_gradient(wcamg_ctx* c, const void* r, const void* teacher, double* loss, void* grad, int where) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    check_where(where);
    require(r && teacher && loss, "null pointer");
    require(c->have_gauge && c->net.L > 0, "needs a gauge field and a network", WCAMG_ESTATE);
    const Geo& g = c->g;
    int C = c->net.C;
    size_t cb = (size_t)C * g.V * 12 * sizeof(double2);
    HostIO io(c);
    const double2* rd = (const double2*)io.in(r, cb, where, "io_in");
    c->reserve({{"nt_r", (size_t)C * 12 * g.V * sizeof(float2)}, {"nt_q", (size_t)C * 12 * g.V * sizeof(float2)}});
    void* r32 = c->W("nt_r", (size_t)C * 12 * g.V * sizeof(float2));
    launch_pack_spinor(g, rd, r32, C64, c->frs(), C, c->st);
    const double2* qd = (const double2*)io.in(teacher, cb, where, "io_in2");
    void* q32 = c->W("nt_q", (size_t)C * 12 * g.V * sizeof(float2));
    launch_pack_spinor(g, qd, q32, C64, c->frs(), C, c->st);
    c->net_forward(r32);
    *loss = c->net_loss_backward(q32);
    if (grad) {
      size_t n = c->net_wsize() * sizeof(float2);
      void* gd = io.out(grad, n, where, "io_out");
      HIPCHK(hipMemcpyAsync(gd, c->net.grad.p, n, hipMemcpyDeviceToDevice, c->st));
      io.finish(grad, gd, n, where);
    }
  });
}

int wcamg_net_train_step(wcamg_ctx* c, const void* r, const void* teacher, double lr, double* loss, int where) {
  if (!c) return WCAMG_EINVAL;
  int rc = wcamg_net_gradient(c, r, teacher, loss, nullptr, where);
  if (rc != WCAMG_OK) return rc;
  return guard(c, [&] {
    require(std::isfinite(*loss), "non-finite network loss", WCAMG_ENUMERIC);
    c->net.t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f - std::pow(b1, (float)c->net.t), c2 = 1.f - std::pow(b2, (float)c->net.t);
    launch_adam((float2*)c->net.W.p, (const float2*)c->net.grad.p, (float2*)c->net.m.p, (float2*)c->net.v.p,
                c->net_wsize(), (float)lr, b1, b2, 1e-8f, c1, c2, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
  });
}

int wcamg_kernel_timing(wcamg_ctx* c, int enable) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    c->collect_timing();
    c->timing = enable != 0;
    if (enable) c->kstats.clear();
  });
}

int wcamg_kernel_stats(wcamg_ctx* c, const char* name, double* total_ms, int* count, double* bytes,
                       double* flops, double* units) {
  if (!c) return WCAMG_EINVAL;
  return guard(c, [&] {
    require(name && total_ms && count, "null pointer");
    c->collect_timing();
    auto it = c->kstats.find(name);
    KStat k = it == c->kstats.end() ? KStat() : it->second;
    *total_ms = k.ms;
    *count = k.count;
    if (bytes) *bytes = k.bytes;
    if (flops) *flops = k.flops;
    if (units) *units = k.units;
  });
}

}  // extern "C"
