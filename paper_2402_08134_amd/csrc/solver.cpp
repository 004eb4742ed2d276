// Host orchestration and C ABI of libsymnmf.
//
// One context = one symmetric X (borrowed), the two factors W and H (owned),
// their FP64 Gram matrices and every workspace the modes need.  All work is
// enqueued on the caller's stream; the stop rule is evaluated on the device
// (DevState) so an iteration never waits for the host.  The host polls the
// stop flag every `check_every` iterations; iterations enqueued after the
// rule fired return at kernel entry.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace {

thread_local std::string g_create_error;

struct Fail {
  int code;
  std::string msg;
};

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) throw Fail{SYMNMF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define LCHK(expr)                                                             \
  do {                                                                         \
    if ((expr) != 0) throw Fail{SYMNMF_E_DEVICE, std::string("launch failed: ") + #expr}; \
  } while (0)

// Device memory cache.  Blocks a context releases are kept, per device and
// size, and handed out again, so contexts of a shape seen before make no
// hipMalloc / hipFree calls (both are slow and hipFree synchronises the
// device).  Contexts release blocks only after synchronising their stream, so
// a reused block has no pending work.  Above kCacheLimit cached bytes a
// released block is freed for real; a failed hipMalloc first empties the
// cache and tries again.  symnmf_trim_cache() frees every cached block.
class DeviceCache {
 public:
  void* get(size_t bytes) {
    bytes = round_up(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = free_.find({dev, bytes});
      if (it != free_.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        cached_ -= bytes;
        live_[p] = {dev, bytes};
        return p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = {dev, bytes};
    return p;
  }

  void put(void* p) {
    if (!p) return;
    std::unique_lock<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) {
      g.unlock();
      (void)hipFree(p);
      return;
    }
    const auto key = it->second;
    live_.erase(it);
    if (cached_ + key.second > kCacheLimit) {
      g.unlock();
      (void)hipFree(p);
      return;
    }
    free_[key].push_back(p);
    cached_ += key.second;
  }

  void trim() {
    std::vector<std::pair<int, void*>> drop;
    {
      std::lock_guard<std::mutex> g(mu_);
      for (auto& kv : free_)
        for (void* p : kv.second) drop.push_back({kv.first.first, p});
      free_.clear();
      cached_ = 0;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& d : drop) {
      (void)hipSetDevice(d.first);
      (void)hipFree(d.second);
    }
    (void)hipSetDevice(cur);
  }

 private:
  static size_t round_up(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }
  static constexpr size_t kCacheLimit = (size_t)16 << 30;
  std::mutex mu_;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_;
  std::unordered_map<void*, std::pair<int, size_t>> live_;
  size_t cached_ = 0;
};

DeviceCache& device_cache() {
  static DeviceCache* c = new DeviceCache();  // never destroyed: blocks live until exit
  return *c;
}

// Pinned host readback buffers of 64 doubles, kept for reuse (hipHostMalloc
// is slow).
class PinnedPool {
 public:
  double* get() {
    {
      std::lock_guard<std::mutex> g(mu_);
      if (!free_.empty()) {
        double* p = free_.back();
        free_.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return (double*)p;
  }
  void put(double* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back(p);
  }

 private:
  std::mutex mu_;
  std::vector<double*> free_;
};

PinnedPool& pinned_pool() {
  static PinnedPool* p = new PinnedPool();
  return *p;
}

template <typename T>
T* dalloc(size_t count) {
  if (count == 0) count = 1;
  void* p = device_cache().get(count * sizeof(T));
  if (!p) throw Fail{SYMNMF_E_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed"};
  return (T*)p;
}
void dfree(void* p) { device_cache().put(p); }

// k rounded up to the 16-column MFMA tile (the padded width of every k-wide
// operand of the update).
int kpad(int k) { return 16 * ((k + 15) / 16); }

constexpr int CMAX = 96;  // widest product operand (LAI basis)

}  // namespace

struct symnmf_ctx {
  // data
  int kind = 0, xdtype = 0, n = 0;
  int64_t ld = 0, nnz = 0;
  const void* Xv = nullptr;
  const int* rp = nullptr;
  const int* ci = nullptr;
  int cdtype = 0;  // product compute dtype
  int fdtype = 0;  // factor / product-output dtype
  const void* Xc = nullptr;
  void* Xb_owned = nullptr;
  // problem
  int k = 0, kp = 16;
  double alpha = 0.0;
  int64_t s = 0;
  double tau = 0.0;
  uint64_t seed = 0;
  symnmf_options opt{};
  hipStream_t st = nullptr;
  int mode = SYMNMF_MODE_PLAIN;
  int64_t iter_host = 0;  // iterations enqueued (drives the LvS sub-streams)
  // Stop-flag gate handed to iteration kernels: the device state while an
  // iteration is being enqueued, nullptr for every other call (those must run
  // even after the stop rule fired).
  const DevState* gate_ = nullptr;
  // scalars
  double normsq = 0, total = 0, maxval = 0, zeta = 0, normsq_lai = 0;
  // device buffers
  void *W = nullptr, *H = nullptr, *Y = nullptr;
  void* Yk = nullptr;  // CSR product in the update's padded layout (n x kp)
  void* P = nullptr;
  void* Bt = nullptr;
  void* BtW = nullptr;  // transposed factor panels for the dense product, or
  void* BtH = nullptr;  // row-major BF16 copies for the BF16-gather CSR product
  bool btW_ok = false, btH_ok = false;
  double* Yhat = nullptr;   // BPP: right-hand sides, then solutions (n x kp FP64)
  double* part = nullptr;   // fused-update block partials (nbu x pcap)
  size_t pcap = 0;          // doubles per partial row
  double* dpart = nullptr;
  int nbu = 1;              // capacity in blocks of the fused update's partials
  int nb_dot = 1;           // blocks of the update that wrote dpart last
  double *M_W = nullptr, *M_H = nullptr;  // LAI: Lambda U^T W, Lambda U^T H
  bool mW_ok = false, mH_ok = false;
  double *G_W = nullptr, *G_H = nullptr, *Gh_W = nullptr, *Gh_H = nullptr, *Gh_S = nullptr;
  double *Gi_W = nullptr, *Gi_H = nullptr, *Gi_S = nullptr;  // 1 / diag of the regularised Grams
  double* d_scal = nullptr;  // [0] ||X||^2 [1] sum [2] max [3..7] scratch [8] ||Lambda||^2 [9] warm beta
  double* rowsum = nullptr;
  DevState* dstate = nullptr;
  double* hist = nullptr;
  int* d_fail = nullptr;
  double* hbuf = nullptr;  // pinned host readback buffer (64 doubles)
  Workspace ws;
  // LAI
  int l = 0;
  double *Q = nullptr, *Q1 = nullptr, *U = nullptr, *YQ = nullptr;
  float* Uf = nullptr;  // U rounded to FP32, read by the update when the factors are FP32
  double *Tm = nullptr, *QT = nullptr, *Vw = nullptr, *lam = nullptr, *Rl = nullptr, *Rlinv = nullptr, *Z = nullptr;
  // LvS / leverage
  SampleBuffers sb;
  int* rows = nullptr;
  double* weights = nullptr;
  int64_t max_sel = 0;
  double* wmask = nullptr;  // LvS: weight of every row in the current sample, 0 off it
  int* seg_cnt = nullptr;
  int* seg_ptr = nullptr;
  int* seg_src = nullptr;
  double* seg_val = nullptr;
  int64_t seg_cap = 0;
  double* lev = nullptr;
  double *R = nullptr, *Rinv = nullptr;
  std::string err;
  // phase timing (options.timing): event pairs recorded on the stream,
  // harvested into phase_ms when the pool fills or the stats are read
  struct TimedPair {
    hipEvent_t a, b;
    int phase;
  };
  std::vector<hipEvent_t> ev_free;
  std::vector<TimedPair> ev_pending;
  double phase_ms[SYMNMF_NUM_PHASES] = {};
  int64_t phase_calls[SYMNMF_NUM_PHASES] = {};
  // HIP graphs of steady-state iterations: [0] one iteration, [1] a block of
  // several; each valid while its generation and iteration count match (the
  // generation is bumped whenever the launch sequence or its arguments change)
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  int64_t graph_gen_of[2] = {-1, -1};
  int graph_count_of[2] = {0, 0};
  int64_t gen = 0;
  bool graphs_broken = false;
  hipStream_t cap_stream = nullptr;  // private stream the graphs are captured on
  int64_t graph_launches = 0;
  // learned-start temporaries (allocated by the first symnmf_warmstart)
  float* warm_F = nullptr;
  float* warm_Htf = nullptr;
  void* warm_Ht = nullptr;
  bool warm_ran = false;  // d_scal[9] holds the scale of the last warm start
  // PGNCG: CG vectors (n x kp FP64), block partials, scalars [e, beta, step,
  // done, 4 spare, M (k x k)]
  double *cgR = nullptr, *cgP = nullptr, *cgZ = nullptr;
  double *cg_part = nullptr, *cg_l1 = nullptr, *cg_sc = nullptr;
  int nbc = 1;

  ~symnmf_ctx() {
    if (st) (void)hipStreamSynchronize(st);
    else (void)hipDeviceSynchronize();
    void* ptrs[] = {Xb_owned, W, H, Y, Yk, Yhat, P, Bt, BtW, BtH, part, dpart, M_W, M_H, Gi_W, Gi_H, Gi_S, G_W, G_H, Gh_W, Gh_H, Gh_S, d_scal, rowsum, dstate, hist, d_fail,
                    ws.base, Q, Q1, U, Uf, YQ, Tm, QT, Vw, lam, Rl, Rlinv, Z, sb.w, sb.prefix, sb.counts, sb.flags,
                    sb.info, sb.theta, rows, weights, wmask, seg_cnt, seg_ptr, seg_src, seg_val, lev, R, Rinv};
    for (void* p : ptrs) dfree(p);
    pinned_pool().put(hbuf);
    for (auto& t : ev_pending) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
    for (hipGraphExec_t& g : graph_exec)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    dfree(warm_F);
    dfree(warm_Htf);
    dfree(warm_Ht);
    for (double* p : {cgR, cgP, cgZ, cg_part, cg_l1, cg_sc}) dfree(p);
  }

  // Any change of mode, options or operand state that alters the kernels of
  // an iteration or their arguments.
  void bump_generation() { ++gen; }

  // Iterations whose launch sequence is fixed: plain (dense or CSR) and LAI
  // with every product operand already up to date.
  bool steady() const {
    if (opt.timing || !opt.graphs || graphs_broken) return false;
    if (opt.rule == SYMNMF_RULE_PGNCG) {
      if (mode == SYMNMF_MODE_LAI) return mH_ok;
      return kind == SYMNMF_CSR || btH_ok;
    }
    if (mode == SYMNMF_MODE_LAI) return mW_ok && mH_ok;
    if (mode == SYMNMF_MODE_PLAIN) return (kind == SYMNMF_CSR && cdtype != SYMNMF_BF16) || (btW_ok && btH_ok);
    return false;
  }

  // Whether graph `which` holds `count` iterations of the current launch
  // sequence.
  bool graph_ready(int which, int count) const {
    return graph_exec[which] && graph_gen_of[which] == gen && graph_count_of[which] == count;
  }

  // Replay `count` iterations from graph `which`, capturing it
  // first if needed.  Returns false (and stops using graphs) if capture or
  // instantiation fails; the iterations are then not done.
  bool graph_iterations(int which, int count) {
    if (!graph_ready(which, count) && !graph_capture(which, count)) return false;
    HIPCHK(hipGraphLaunch(graph_exec[which], st));
    iter_host += count;
    ++graph_launches;
    return true;
  }

  // Capture and instantiate graph `which` for `count` iterations without
  // launching it.  Returns false (and stops using graphs) on failure.
  bool graph_capture(int which, int count) {
    {
      if (graph_exec[which]) {
        HIPCHK(hipGraphExecDestroy(graph_exec[which]));
        graph_exec[which] = nullptr;
      }
      // Capture on a private stream (the caller's may be the null stream,
      // which cannot be captured); the graph is launched on the caller's.
      if (!cap_stream && hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        cap_stream = nullptr;
        graphs_broken = true;
        return false;
      }
      if (hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        graphs_broken = true;
        return false;
      }
      bool ok = true;
      const int64_t saved = iter_host;
      hipStream_t user = st;
      st = cap_stream;
      try {
        for (int t = 0; t < count; ++t) one_iteration();
      } catch (const Fail&) {
        ok = false;
      }
      st = user;
      iter_host = saved;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cap_stream, &g);
      if (!ok || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        graphs_broken = true;
        return false;
      }
      hipGraphExec_t ex = nullptr;
      const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        (void)hipGetLastError();
        graphs_broken = true;
        return false;
      }
      graph_exec[which] = ex;
      graph_gen_of[which] = gen;
      graph_count_of[which] = count;
    }
    return true;
  }

  hipEvent_t take_event() {
    if (!ev_free.empty()) {
      hipEvent_t e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }

  // Wait for every pending pair and add its duration to its phase.
  void harvest_timers() {
    for (auto& t : ev_pending) {
      float ms = 0.f;
      HIPCHK(hipEventSynchronize(t.b));
      HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
      phase_ms[t.phase] += ms;
      phase_calls[t.phase] += 1;
      ev_free.push_back(t.a);
      ev_free.push_back(t.b);
    }
    ev_pending.clear();
  }

  // Brackets the launches of its scope with an event pair when timing is on.
  struct Timed {
    symnmf_ctx* c;
    hipEvent_t a = nullptr;
    int phase;
    Timed(symnmf_ctx* cc, int ph) : c(cc), phase(ph) {
      if (!c->opt.timing) return;
      if (c->ev_pending.size() >= 4096) c->harvest_timers();
      a = c->take_event();
      HIPCHK(hipEventRecord(a, c->st));
    }
    ~Timed() {
      if (!a) return;
      hipEvent_t b = nullptr;
      try {
        b = c->take_event();
      } catch (...) {
        c->ev_free.push_back(a);
        return;
      }
      if (hipEventRecord(b, c->st) != hipSuccess) {
        (void)hipGetLastError();
        c->ev_free.push_back(a);
        c->ev_free.push_back(b);
        return;
      }
      c->ev_pending.push_back({a, b, phase});
    }
  };

  size_t fsize() const { return dtype_size(fdtype); }
  int64_t nk() const { return (int64_t)n * k; }

  void sync() { HIPCHK(hipStreamSynchronize(st)); }

  // Copy `count` doubles from device to the pinned buffer and wait.
  const double* readback(const double* d, int count) {
    HIPCHK(hipMemcpyAsync(hbuf, d, count * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    return hbuf;
  }

  StopRule rule() const {
    StopRule r;
    r.mode = opt.stop_mode;
    r.tol = opt.stop_tol;
    r.patience = opt.stop_patience;
    r.target = opt.target;
    r.max_hist = opt.max_history;
    return r;
  }

  // ---- products -----------------------------------------------------------
  // Y (n x c, fdtype) = X B with B of bdtype (the factor dtype or F64).
  void product(const void* B, int bdtype, int c, void* Yout) {
    if (kind == SYMNMF_DENSE) {
      const GemmPlan p = gemm_plan(n, c, cdtype);
      LCHK(dense_gemm(Xc, opdtype(), ldxc(), B, bdtype, c, n, c, p, Bt, P, Yout, fdtype, c, gate_, st));
    } else {
      LCHK(csr_spmm(rp, ci, Xv, xdtype, n, B, bdtype, c, Yout, fdtype, gate_, st));
    }
  }

  // Y = (LAI operator) Src = U (Lambda (U^T Src)).
  void lai_product(const void* Src, void* Yout) {
    ws.reset();
    LCHK(gram(U, SYMNMF_F64, l, l, Src, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, Z, nullptr, 0, 0.0,
              gate_, st));
    LCHK(rowmat(U, SYMNMF_F64, l, n, l, Z, lam, k, Yout, fdtype, k, gate_, st));
  }

  void refresh_gram(const void* F, double* G, double* Gh, double* Gi) {
    ws.reset();
    LCHK(gram(F, fdtype, k, k, F, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, G, Gh, kp, alpha, gate_, st,
              Gi));
  }

  void invalidate(int which) {
    if (which == SYMNMF_W) btW_ok = mW_ok = false;
    else btH_ok = mH_ok = false;
  }

  // The product-side operand of a factor, brought up to date if needed: its
  // transposed panel (dense plain mode) or M = Lambda U^T F (LAI mode).
  void ensure_operand(int which) {
    void* F = which == SYMNMF_W ? W : H;
    if (mode == SYMNMF_MODE_LAI) {
      bool& ok = which == SYMNMF_W ? mW_ok : mH_ok;
      if (!ok) {
        ws.reset();
        LCHK(gram(U, SYMNMF_F64, l, l, F, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, Z, nullptr, 0, 0.0,
                  nullptr, st));
        LCHK(scale_rows(Z, lam, l, k, kp, which == SYMNMF_W ? M_W : M_H, st));
        ok = true;
      }
    } else if (mode == SYMNMF_MODE_PLAIN && kind == SYMNMF_DENSE) {
      bool& ok = which == SYMNMF_W ? btW_ok : btH_ok;
      if (!ok) {
        const GemmPlan p = gemm_plan(n, k, cdtype);
        LCHK(factor_transpose(F, fdtype, n, k, which == SYMNMF_W ? BtW : BtH, opdtype(), p, nullptr, st));
        ok = true;
      }
    } else if (mode == SYMNMF_MODE_PLAIN && kind == SYMNMF_CSR && cdtype == SYMNMF_BF16) {
      bool& ok = which == SYMNMF_W ? btW_ok : btH_ok;
      if (!ok) {
        LCHK(to_bf16((const float*)F, (int64_t)n * k, which == SYMNMF_W ? BtW : BtH, st));
        ok = true;
      }
    }
  }

  // One half-iteration: Dst from Src (side 0: W from H; side 1: H from W).
  // want_dot: also accumulate <Dst_new, product part> for the residual.
  void half_step(int side, int64_t half_iter, bool want_dot) {
    const int src_id = side == 0 ? SYMNMF_H : SYMNMF_W;
    const int dst_id = side == 0 ? SYMNMF_W : SYMNMF_H;
    void* Src = side == 0 ? H : W;
    void* Dst = side == 0 ? W : H;
    double* Gs = side == 0 ? G_H : G_W;      // Gram of Src (current)
    double* Ghs = side == 0 ? Gh_H : Gh_W;   // regularised Gram of Src
    double* Gis = side == 0 ? Gi_H : Gi_W;
    double* Gid = side == 0 ? Gi_W : Gi_H;
    double* Gd = side == 0 ? G_W : G_H;      // Gram of Dst (refreshed here)
    double* Ghd = side == 0 ? Gh_W : Gh_H;
    ensure_operand(src_id);
    UpdateArgs a;
    a.n = n;
    a.k = k;
    a.Src = Src;
    a.Dst = Dst;
    a.Ghat = Ghs;
    a.alpha = alpha;
    a.part = part;
    a.pstride = k * k;
    a.dpart = want_dot ? dpart : nullptr;
    int ymode = 0, pdt = fdtype, tdt = fdtype;
    if (mode == SYMNMF_MODE_LVS) {
      Timed tm(this, SYMNMF_PHASE_SAMPLE);
      ws.reset();
      LCHK(chol_inverse(Gs, k, R, Rinv, &dstate->flags, SYMNMF_FLAG_LEV_SHIFT, d_fail, st));
      LCHK(leverage_scores(Src, fdtype, n, k, Rinv, lev, gate_, st));
      LCHK(hybrid_sample(lev, n, k, s, tau, seed, (uint32_t)half_iter, sb, rows, weights, max_sel, ws, gate_, st,
                         wmask));
      ws.reset();
      LCHK(gram(Src, fdtype, k, k, Src, fdtype, k, k, n, rows, weights, sb.info + 2, (int)max_sel, ws, nullptr, Gh_S,
                kp, alpha, gate_, st, Gi_S));
      ws.reset();
      LCHK(sampled_slab(rp, ci, Xv, xdtype, n, rows, sb.info + 2, (int)max_sel, wmask, seg_cnt, seg_ptr,
                        seg_src, seg_val, seg_cap, ws, gate_, st));
      a.seg_ptr = seg_ptr;
      a.seg_src = seg_src;
      a.seg_val = seg_val;
      a.Ghat = Gh_S;
      Gis = Gi_S;
      a.dpart = nullptr;
      ymode = 1;
    } else if (mode == SYMNMF_MODE_LAI) {
      // the update rounds U to the factor type as it loads it: FP32 factors
      // read the FP32 copy (half the bytes, the same values)
      a.U = fdtype == SYMNMF_F32 ? (const void*)Uf : (const void*)U;
      a.M = side == 0 ? M_H : M_W;
      a.l = l;
      a.pstride = k * k + l * k;
      ymode = 2;
    } else if (kind == SYMNMF_DENSE) {
      const GemmPlan p = gemm_plan(n, k, cdtype);
      {
        Timed tm(this, SYMNMF_PHASE_PRODUCT);
        LCHK(dense_gemm_bt(Xc, opdtype(), ldxc(), side == 0 ? BtH : BtW, n, k, p, P, gate_, st));
      }
      a.P = P;
      a.splits = p.splits;
      a.cp = p.cp;
      a.Dt = side == 0 ? BtW : BtH;
      a.ldt = p.ldt;
      pdt = cdtype == SYMNMF_F64 ? SYMNMF_F64 : SYMNMF_F32;
      tdt = opdtype();
    } else if (cdtype == SYMNMF_BF16) {
      // gathers of the BF16 copy of Src; the update writes the copy of Dst
      {
        Timed tm(this, SYMNMF_PHASE_PRODUCT);
        LCHK(csr_spmm(rp, ci, Xv, xdtype, n, side == 0 ? BtH : BtW, SYMNMF_BF16, k, Yk, fdtype, gate_, st, kp));
      }
      a.P = Yk;
      a.splits = 1;
      a.cp = kp;
      a.Dt = side == 0 ? BtW : BtH;
      a.dt_rows = 1;
      a.ldt = k;
      tdt = SYMNMF_BF16;
    } else {
      {
        Timed tm(this, SYMNMF_PHASE_PRODUCT);
        LCHK(csr_spmm(rp, ci, Xv, xdtype, n, Src, fdtype, k, Yk, fdtype, gate_, st, kp));
      }
      a.P = Yk;
      a.splits = 1;
      a.cp = kp;
    }
    const int nb = update_blocks(n, kp, ymode == 2 ? 16 * ceil_div(l, 16) : 0, fdtype);
    if (want_dot) nb_dot = nb;
    if (opt.rule == SYMNMF_RULE_HALS) {
      UpdateRO ro;
      ro.Ghat = a.Ghat;
      ro.Ginv = Gis;
      ro.M = a.M;
      if (opt.timing) {
        // the update kernel's own start and end (events taken by its launch)
        if (ev_pending.size() >= 4096) harvest_timers();
        a.ev_start = take_event();
        a.ev_stop = take_event();
        const int rc = fused_update(a, ro, kp, ymode, fdtype, pdt, tdt, nb, gate_, st);
        ev_pending.push_back({a.ev_start, a.ev_stop, SYMNMF_PHASE_UPDATE});
        LCHK(rc);
      } else {
        LCHK(fused_update(a, ro, kp, ymode, fdtype, pdt, tdt, nb, gate_, st));
      }
      Timed tr(this, SYMNMF_PHASE_REDUCE);
      LCHK(update_reduce(part, nb, a.pstride, k, l, kp, alpha, lam, Gd, Ghd, Gid,
                         side == 0 ? M_W : M_H, gate_, st));
    } else {
      // BPP: the update kernel writes the right-hand sides, the pivoting
      // kernel solves every row in place, and the update kernel then takes
      // the solutions through its usual write-back and partials.
      UpdateRO ro;
      ro.Ghat = a.Ghat;
      ro.Ginv = Gis;
      ro.M = a.M;
      a.Yhat = Yhat;
      {
        Timed tm(this, SYMNMF_PHASE_UPDATE);
        a.rule = 1;
        LCHK(fused_update(a, ro, kp, ymode, fdtype, pdt, tdt, nb, gate_, st));
        LCHK(bpp_update(n, k, kp, Yhat, Dst, fdtype, a.Ghat, &dstate->flags, SYMNMF_FLAG_BPP_CAP, gate_, st));
        a.rule = 2;
        LCHK(fused_update(a, ro, kp, ymode, fdtype, pdt, tdt, nb, gate_, st));
      }
      Timed tr(this, SYMNMF_PHASE_REDUCE);
      LCHK(update_reduce(part, nb, a.pstride, k, l, kp, alpha, lam, Gd, Ghd, Gid,
                         side == 0 ? M_W : M_H, gate_, st));
    }
    invalidate(dst_id);
    if (ymode == 0 && a.Dt) {
      if (dst_id == SYMNMF_W) btW_ok = true;
      else btH_ok = true;
    }
    if (ymode == 2) {
      if (dst_id == SYMNMF_W) mW_ok = true;
      else mH_ok = true;
    }
  }

  int64_t ldxc() const { return cdtype == SYMNMF_BF16 && xdtype != SYMNMF_BF16 ? n : ld; }
  // element type of the product operands (X, B panel): the compute dtype,
  // except that the three-piece BF16 products read FP32 operands
  int opdtype() const { return cdtype; }

  struct Gate {
    symnmf_ctx* c;
    explicit Gate(symnmf_ctx* cc) : c(cc) { c->gate_ = c->dstate; }
    ~Gate() { c->gate_ = nullptr; }
  };

  // One PGNCG iteration (Section 2.1.3): Y = X H (or the LAI product), the
  // gradient pass with the residual of H and the stop rule, cg_iters - 1 CG
  // steps and the last step fused with H <- max(H - Z, 0), then the Gram of
  // the new H (and Lambda U^T H in LAI mode) for the next iteration.
  void pgncg_iteration(const double* nrm) {
    ensure_operand(SYMNMF_H);
    CgArgs a;
    a.n = n;
    a.k = k;
    a.H = H;
    a.W = W;
    a.R = cgR;
    a.Pd = cgP;
    a.Z = cgZ;
    a.part = cg_part;
    a.dpart = dpart;
    int ymode = 0, pdt = fdtype, tdt = fdtype;
    if (mode == SYMNMF_MODE_LAI) {
      a.U = U;
      a.Mlai = M_H;
      a.l = l;
      ymode = 2;
    } else if (kind == SYMNMF_DENSE) {
      const GemmPlan p = gemm_plan(n, k, cdtype);
      {
        Timed tm(this, SYMNMF_PHASE_PRODUCT);
        LCHK(dense_gemm_bt(Xc, opdtype(), ldxc(), BtH, n, k, p, P, gate_, st));
      }
      a.P = P;
      a.splits = p.splits;
      a.cp = p.cp;
      a.Dt = BtH;
      a.ldt = p.ldt;
      pdt = cdtype == SYMNMF_F64 ? SYMNMF_F64 : SYMNMF_F32;
      tdt = opdtype();
    } else {
      {
        Timed tm(this, SYMNMF_PHASE_PRODUCT);
        LCHK(csr_spmm(rp, ci, Xv, xdtype, n, H, fdtype, k, Yk, fdtype, gate_, st, kp));
      }
      a.P = Yk;
      a.splits = 1;
      a.cp = kp;
    }
    Timed tm(this, SYMNMF_PHASE_UPDATE);
    LCHK(cg_pass(0, a, kp, ymode, fdtype, pdt, tdt, G_H, cg_sc, nbc, gate_, st));
    finish_iteration(dpart, nbc, G_H, G_H, k, nrm, dstate, hist, rule(), st);
    LCHK(cg_reduce(cg_part, nbc, k, cg_l1, cg_sc, true, gate_, st));
    for (int j = 0; j + 1 < opt.cg_iters; ++j) {
      a.first = j == 0;
      LCHK(cg_pass(1, a, kp, ymode, fdtype, pdt, tdt, G_H, cg_sc, nbc, gate_, st));
      LCHK(cg_reduce(cg_part, nbc, k, cg_l1, cg_sc, false, gate_, st));
    }
    a.first = opt.cg_iters == 1;
    a.part = part;
    a.pstride = k * k + (ymode == 2 ? l * k : 0);
    LCHK(cg_pass(2, a, kp, ymode, fdtype, pdt, tdt, G_H, cg_sc, nbc, gate_, st));
    LCHK(update_reduce(part, nbc, a.pstride, k, l, kp, alpha, lam, G_H, Gh_H, Gi_H,
                       ymode == 2 ? M_H : nullptr, gate_, st));
    invalidate(SYMNMF_W);
    if (ymode == 2) mH_ok = true;
    if (a.Dt) btH_ok = true;
  }

  void one_iteration() {
    Gate g(this);
    const int64_t t = iter_host++;
    const double* nrm = d_scal + (mode == SYMNMF_MODE_LAI ? 8 : 0);
    if (opt.rule == SYMNMF_RULE_PGNCG) {
      pgncg_iteration(nrm);
      return;
    }
    if (mode == SYMNMF_MODE_LVS) {
      half_step(0, 2 * t, false);
      half_step(1, 2 * t + 1, false);
      const int every = opt.resid_every > 0 ? opt.resid_every : 1;
      if (((t + 1) % every) == 0) {
        {
          Timed tm(this, SYMNMF_PHASE_PRODUCT);
          product(W, fdtype, k, Y);
        }
        ws.reset();
        double* part = nullptr;
        const int nb = dot_partials(H, Y, fdtype, nk(), ws, &part, gate_, st);
        if (nb < 0) throw Fail{SYMNMF_E_DEVICE, "dot launch failed"};
        finish_iteration(part, nb, G_W, G_H, k, nrm, dstate, hist, rule(), st);
      } else {
        finish_iteration(nullptr, 0, G_W, G_H, k, nrm, dstate, hist, rule(), st);
      }
      return;
    }
    half_step(0, 2 * t, false);
    half_step(1, 2 * t + 1, true);
    finish_iteration(dpart, nb_dot, G_W, G_H, k, nrm, dstate, hist, rule(), st);
  }

  DevState read_state() {
    static_assert(sizeof(DevState) <= 64 * sizeof(double), "state fits the readback buffer");
    HIPCHK(hipMemcpyAsync(hbuf, dstate, sizeof(DevState), hipMemcpyDeviceToHost, st));
    sync();
    DevState d;
    std::memcpy(&d, hbuf, sizeof(DevState));
    return d;
  }

  // Trace-identity residual ||op - A B^T|| / ||op|| with op = X, or U Lambda U^T
  // when lai is set; uses fresh Grams of A and B.
  double trace_residual(const void* A, const void* B, bool lai) {
    if (lai) lai_product(A, Y);
    else product(A, fdtype, k, Y);
    ws.reset();
    double* part = nullptr;
    const int nb = dot_partials(B, Y, fdtype, nk(), ws, &part, nullptr, st);
    if (nb < 0) throw Fail{SYMNMF_E_DEVICE, "dot launch failed"};
    sum_partials(part, nb, d_scal + 3, st);
    double* ga = ws.dbl((size_t)k * k);
    double* gb = ws.dbl((size_t)k * k);
    if (!ga || !gb) throw Fail{SYMNMF_E_NOMEM, "workspace"};
    LCHK(gram(A, fdtype, k, k, A, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, ga, nullptr, 0, 0.0, nullptr,
              st));
    LCHK(gram(B, fdtype, k, k, B, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, gb, nullptr, 0, 0.0, nullptr,
              st));
    frob_dot(ga, gb, k * k, d_scal + 4, st);
    const double* h = readback(d_scal + 3, 2);
    const double nx = lai ? normsq_lai : normsq;
    return std::sqrt(std::fmax(nx - 2.0 * h[0] + h[1], 0.0) / nx);
  }

  double exact_residual(const void* A, const void* B) {
    ws.reset();
    if (kind == SYMNMF_DENSE) {
      LCHK(dense_resid_exact(Xv, xdtype, ld, n, k, A, B, fdtype, ws, d_scal + 3, st));
      const double* h = readback(d_scal + 3, 1);
      return std::sqrt(h[0] / normsq);
    }
    LCHK(csr_resid_cross(rp, ci, Xv, xdtype, n, k, A, B, fdtype, ws, d_scal + 3, st));
    double* ga = ws.dbl((size_t)k * k);
    double* gb = ws.dbl((size_t)k * k);
    if (!ga || !gb) throw Fail{SYMNMF_E_NOMEM, "workspace"};
    LCHK(gram(A, fdtype, k, k, A, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, ga, nullptr, 0, 0.0, nullptr, st));
    LCHK(gram(B, fdtype, k, k, B, fdtype, k, k, n, nullptr, nullptr, nullptr, 0, ws, gb, nullptr, 0, 0.0, nullptr, st));
    frob_dot(ga, gb, k * k, d_scal + 4, st);
    const double* h = readback(d_scal + 3, 2);
    return std::sqrt(std::fmax(normsq - 2.0 * h[0] + h[1], 0.0) / normsq);
  }

  // CholeskyQR2: Qout (n x l, FP64) = orthonormal factor of Yin (n x l, fdtype).
  // CholeskyQR of Yin into Q; `twice` repeats it on the result (CholeskyQR2,
  // orthonormal to working precision).  One pass suffices between power
  // iterations, where only the span matters: it keeps the basis well
  // conditioned for the next product.
  void cholqr(const void* Yin, bool twice) {
    ws.reset();
    LCHK(gram(Yin, fdtype, l, l, Yin, fdtype, l, l, n, nullptr, nullptr, nullptr, 0, ws, Tm, nullptr, 0, 0.0,
              nullptr, st));
    LCHK(chol_inverse(Tm, l, Rl, Rlinv, &dstate->flags, SYMNMF_FLAG_CHOLQR_SHIFT, d_fail, st));
    if (!twice) {
      LCHK(rowmat(Yin, fdtype, l, n, l, Rlinv, nullptr, l, Q, SYMNMF_F64, l, nullptr, st));
      return;
    }
    LCHK(rowmat(Yin, fdtype, l, n, l, Rlinv, nullptr, l, Q1, SYMNMF_F64, l, nullptr, st));
    ws.reset();
    LCHK(gram(Q1, SYMNMF_F64, l, l, Q1, SYMNMF_F64, l, l, n, nullptr, nullptr, nullptr, 0, ws, Tm, nullptr, 0, 0.0,
              nullptr, st));
    LCHK(chol_inverse(Tm, l, Rl, Rlinv, &dstate->flags, SYMNMF_FLAG_CHOLQR_SHIFT, d_fail, st));
    LCHK(rowmat(Q1, SYMNMF_F64, l, n, l, Rlinv, nullptr, l, Q, SYMNMF_F64, l, nullptr, st));
  }

  void ensure_sampling_buffers() {
    if (sb.w) return;
    sb.w = dalloc<uint64_t>(n);
    sb.prefix = dalloc<uint64_t>(n);
    sb.counts = dalloc<int>(n);
    sb.flags = dalloc<int>((size_t)n + 1);
    sb.info = dalloc<int>(8);
    sb.theta = dalloc<double>(1);
    HIPCHK(hipMemsetAsync(sb.counts, 0, sizeof(int) * n, st));
    HIPCHK(hipMemsetAsync(sb.info, 0, sizeof(int) * 8, st));
    HIPCHK(hipMemsetAsync(sb.theta, 0, sizeof(double), st));
  }
};

// A network of the learned warm start: parameters, Adam state and the
// training buffers (grown to the largest batch seen).
struct symnmf_mlp {
  int hidden = MLP_HIDDEN;
  int np = 0;
  hipStream_t st = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  int64_t cap = 0;
  float *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *dza = nullptr, *dzb = nullptr;
  double* scratch = nullptr;
  double* d_loss = nullptr;
  double* hbuf = nullptr;
  int64_t t = 0;
  std::string err;

  ~symnmf_mlp() {
    if (st) (void)hipStreamSynchronize(st);
    else (void)hipDeviceSynchronize();
    void* ptrs[] = {p, m, v, g, h1, h2, h3, dza, dzb, scratch, d_loss};
    for (void* q : ptrs) dfree(q);
    pinned_pool().put(hbuf);
  }

  void ensure(int64_t rows) {
    if (rows <= cap) return;
    HIPCHK(hipStreamSynchronize(st));
    float** bufs[] = {&h1, &h2, &h3, &dza, &dzb};
    for (float** b : bufs) {
      dfree(*b);
      *b = nullptr;
    }
    dfree(scratch);
    scratch = nullptr;
    cap = 0;
    for (float** b : bufs) *b = dalloc<float>((size_t)rows * hidden);
    scratch = dalloc<double>(mlp_train_scratch_doubles(rows));
    cap = rows;
  }
};

namespace {

int fail(symnmf_ctx* c, const Fail& f) {
  if (c) c->err = f.msg;
  else g_create_error = f.msg;
  return f.code;
}

template <typename Fn>
int guarded(symnmf_ctx* c, Fn&& fn) {
  if (!c) {
    g_create_error = "null context";
    return SYMNMF_E_INVALID;
  }
  try {
    fn();
    return SYMNMF_OK;
  } catch (const Fail& f) {
    return fail(c, f);
  } catch (const std::bad_alloc&) {
    return fail(c, Fail{SYMNMF_E_NOMEM, "host allocation failed"});
  } catch (...) {
    return fail(c, Fail{SYMNMF_E_DEVICE, "unexpected internal error"});
  }
}

template <typename Fn>
int mlp_guarded(symnmf_mlp* net, Fn&& fn) {
  if (!net) return SYMNMF_E_INVALID;
  try {
    fn();
    return SYMNMF_OK;
  } catch (const Fail& f) {
    net->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    net->err = "host allocation failed";
    return SYMNMF_E_NOMEM;
  } catch (...) {
    net->err = "unexpected internal error";
    return SYMNMF_E_DEVICE;
  }
}

// File of a network's parameters (symnmf_mlp_save / symnmf_mlp_load).
constexpr char kMlpMagic[8] = {'S', 'Y', 'M', 'N', 'M', 'L', 'P', '1'};
struct MlpFileHeader {
  char magic[8];
  int32_t hidden;
  int32_t features;
  int64_t count;
};
static_assert(sizeof(MlpFileHeader) == 24, "file header layout");

void mlp_grad(symnmf_mlp* net, const float* F, const float* T, int64_t rows, double* loss) {
  if (rows < 1 || !F || !T) throw Fail{SYMNMF_E_INVALID, "argument"};
  net->ensure(rows);
  LCHK(mlp_gradient(net->p, F, T, rows, net->h1, net->h2, net->h3, net->dza, net->dzb, net->g, net->scratch,
                    net->d_loss, net->st));
  if (loss) {
    HIPCHK(hipMemcpyAsync(net->hbuf, net->d_loss, sizeof(double), hipMemcpyDeviceToHost, net->st));
    HIPCHK(hipStreamSynchronize(net->st));
    *loss = 0.5 * net->hbuf[0] / (double)rows;
  }
}

// Learned start into the caller-chosen temporaries F ((n k) x 6 FP32
// features), Htf (n k FP32 network outputs) and Ht (n k factor elements).
void warmstart_run(symnmf_ctx* c, const symnmf_mlp* net, float* F, float* Htf, void* Ht, double* beta_out) {
  const int n = c->n, k = c->k;
  const int64_t nk = (int64_t)n * k;
  symnmf_ctx::Timed tm(c, SYMNMF_PHASE_WARM);
  c->ws.reset();
  double* info = c->ws.dbl((size_t)2 * k + 2);
  if (!info) throw Fail{SYMNMF_E_NOMEM, "workspace"};
  LCHK(warm_features(c->U, n, c->l, k, c->lam, c->rowsum, c->d_scal + 1, F, info, c->ws, c->st));
  LCHK(mlp_forward(net->p, F, nk, Htf, c->st));
  LCHK(copy_convert(Htf, SYMNMF_F32, Ht, c->fdtype, nk, c->st));
  // least-squares scale: beta^2 = tr(Ht^T X Ht) / ||Ht^T Ht||_F^2
  c->product(Ht, c->fdtype, k, c->Y);
  double* part = nullptr;
  const int nb = dot_partials(Ht, c->Y, c->fdtype, nk, c->ws, &part, nullptr, c->st);
  if (nb < 0) throw Fail{SYMNMF_E_DEVICE, "dot launch failed"};
  sum_partials(part, nb, c->d_scal + 3, c->st);
  double* ga = c->ws.dbl((size_t)k * k);
  if (!ga) throw Fail{SYMNMF_E_NOMEM, "workspace"};
  LCHK(gram(Ht, c->fdtype, k, k, Ht, c->fdtype, k, k, n, nullptr, nullptr, nullptr, 0, c->ws, ga, nullptr, 0, 0.0,
            nullptr, c->st));
  frob_dot(ga, ga, k * k, c->d_scal + 4, c->st);
  LCHK(warm_apply(Htf, nk, c->d_scal + 3, c->d_scal + 4, info + 2 * k + 1, c->H, c->W, c->fdtype, c->d_scal + 9,
                  c->st));
  c->warm_ran = true;
  c->refresh_gram(c->W, c->G_W, c->Gh_W, c->Gi_W);
  c->refresh_gram(c->H, c->G_H, c->Gh_H, c->Gi_H);
  c->invalidate(SYMNMF_W);
  c->invalidate(SYMNMF_H);
  if (beta_out) *beta_out = c->readback(c->d_scal + 9, 1)[0];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Temporaries of one learned start for n k entries with factor elements of
// fsize bytes, each piece 256-byte aligned.
size_t warm_scratch_bytes(int64_t nk, size_t fsize) {
  return align256((size_t)nk * MLP_D_IN * sizeof(float)) + align256((size_t)nk * sizeof(float)) +
         align256((size_t)nk * fsize);
}

// Static device scratch of symnmf_warmstart_noalloc: one copy per GPU, held
// until the process ends, shared by every call on that GPU.  Host code never
// uses the array's name (on the host it is a stand-in, not a device address);
// it uses the address hipGetSymbolAddress returns for the current device.
constexpr size_t kWarmScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kWarmScratchBytes];

char* warm_scratch_device() {
  static std::mutex mu;
  static std::unordered_map<int, char*> addr;  // device ordinal -> address
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Fail{SYMNMF_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array"};
  addr[dev] = (char*)ptr;
  return (char*)ptr;
}
}  // namespace

extern "C" {

int symnmf_default_options(symnmf_options* opt) {
  if (!opt) return SYMNMF_E_INVALID;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = (int32_t)sizeof(symnmf_options);
  opt->rule = SYMNMF_RULE_HALS;
  opt->compute_dtype = -1;
  opt->stop_mode = SYMNMF_STOP_NONE;
  opt->stop_tol = 1e-4;
  opt->stop_patience = 4;
  opt->check_every = 8;
  opt->target = 0.0;
  opt->tau = -1.0;
  opt->resid_every = 1;
  opt->max_history = 4096;
  opt->timing = 0;
  opt->graphs = 1;
  opt->cg_iters = 5;
  return SYMNMF_OK;
}

int symnmf_create(symnmf_ctx** out, const symnmf_matrix* X, int32_t k, double alpha, int64_t s, uint64_t seed,
                  const symnmf_options* opt, void* hip_stream) {
  if (!out || !X) {
    g_create_error = "null argument";
    return SYMNMF_E_INVALID;
  }
  *out = nullptr;
  symnmf_ctx* c = nullptr;
  try {
    c = new symnmf_ctx();
  } catch (...) {
    g_create_error = "host allocation failed";
    return SYMNMF_E_NOMEM;
  }
  try {
    symnmf_default_options(&c->opt);
    if (opt) {
      if (opt->struct_size != (int32_t)sizeof(symnmf_options)) throw Fail{SYMNMF_E_INVALID, "options struct_size"};
      c->opt = *opt;
    }
    if (c->opt.check_every < 1) c->opt.check_every = 1;
    if (c->opt.max_history < 1) c->opt.max_history = 1;
    if (c->opt.rule != SYMNMF_RULE_HALS && c->opt.rule != SYMNMF_RULE_BPP && c->opt.rule != SYMNMF_RULE_PGNCG)
      throw Fail{SYMNMF_E_INVALID, "rule"};
    if (c->opt.rule == SYMNMF_RULE_PGNCG) {
      if (c->opt.cg_iters < 1 || c->opt.cg_iters > 64) throw Fail{SYMNMF_E_INVALID, "cg_iters must be in 1..64"};
      if (s > 0) throw Fail{SYMNMF_E_UNSUPPORTED, "PGNCG with leverage-score sampling"};
    }
    if (c->opt.stop_mode < SYMNMF_STOP_NONE || c->opt.stop_mode > SYMNMF_STOP_STALL_OR_TARGET)
      throw Fail{SYMNMF_E_INVALID, "stop_mode"};
    c->st = (hipStream_t)hip_stream;
    c->kind = X->kind;
    c->xdtype = X->dtype;
    if (X->n < 1 || X->n > 0x7fffffff) throw Fail{SYMNMF_E_INVALID, "n out of range"};
    c->n = (int)X->n;
    if (k < 1 || k > 64) throw Fail{SYMNMF_E_INVALID, "k must be in 1..64"};
    if (k > c->n) throw Fail{SYMNMF_E_INVALID, "k > n"};
    c->k = k;
    c->kp = kpad(k);
    if (s < 0) throw Fail{SYMNMF_E_INVALID, "s < 0"};
    c->s = s;
    c->seed = seed;
    c->Xv = X->values;
    if (c->kind == SYMNMF_DENSE) {
      if (!X->values) throw Fail{SYMNMF_E_INVALID, "null values"};
      if (X->dtype != SYMNMF_F64 && X->dtype != SYMNMF_F32 && X->dtype != SYMNMF_BF16)
        throw Fail{SYMNMF_E_INVALID, "dtype"};
      c->ld = X->ld;
      if (c->ld < c->n) throw Fail{SYMNMF_E_INVALID, "ld < n"};
      if (s > 0) throw Fail{SYMNMF_E_UNSUPPORTED, "leverage-score sampling needs CSR X"};
      int cd = c->opt.compute_dtype < 0 ? X->dtype : c->opt.compute_dtype;
      if (cd == SYMNMF_F64 && X->dtype != SYMNMF_F64) throw Fail{SYMNMF_E_UNSUPPORTED, "F64 compute needs F64 X"};
      if (X->dtype == SYMNMF_F64 && cd != SYMNMF_F64) throw Fail{SYMNMF_E_UNSUPPORTED, "F64 X needs F64 compute"};
      if (X->dtype == SYMNMF_BF16 && cd != SYMNMF_BF16) throw Fail{SYMNMF_E_UNSUPPORTED, "BF16 X needs BF16 compute"};
      if (cd != SYMNMF_F64 && cd != SYMNMF_F32 && cd != SYMNMF_BF16)
        throw Fail{SYMNMF_E_INVALID, "compute dtype"};
      c->cdtype = cd;
      c->fdtype = cd == SYMNMF_F64 ? SYMNMF_F64 : SYMNMF_F32;
    } else if (c->kind == SYMNMF_CSR) {
      if (X->dtype != SYMNMF_F64 && X->dtype != SYMNMF_F32) throw Fail{SYMNMF_E_INVALID, "CSR dtype"};
      if (!X->row_ptr || (X->nnz > 0 && (!X->col_idx || !X->values))) throw Fail{SYMNMF_E_INVALID, "null CSR array"};
      if (X->nnz < 0 || X->nnz > 0x7fffffff) throw Fail{SYMNMF_E_INVALID, "nnz out of range"};
      c->nnz = X->nnz;
      c->rp = X->row_ptr;
      c->ci = X->col_idx;
      c->cdtype = X->dtype;
      c->fdtype = X->dtype;
      const int cd = c->opt.compute_dtype;
      if (cd == SYMNMF_BF16) {
        if (X->dtype != SYMNMF_F32) throw Fail{SYMNMF_E_UNSUPPORTED, "BF16 gathers need FP32 CSR values"};
        if (c->opt.rule == SYMNMF_RULE_PGNCG) throw Fail{SYMNMF_E_UNSUPPORTED, "BF16 gathers with PGNCG"};
        c->cdtype = SYMNMF_BF16;
      } else if (cd >= 0 && cd != X->dtype) {
        throw Fail{SYMNMF_E_UNSUPPORTED, "CSR compute dtype"};
      }
    } else {
      throw Fail{SYMNMF_E_INVALID, "matrix kind"};
    }

    const int n = c->n;
    // workspace: the largest temporaries of any launcher
    size_t wsd = (size_t)256 * CMAX * CMAX + 4096;
    if (c->kind == SYMNMF_DENSE) {
      wsd = std::max(wsd, (size_t)195 * n + 4096);
      const size_t nb = (size_t)ceil_div(n, 64);
      wsd = std::max(wsd, nb * nb + 4096);
    }
    wsd = std::max(wsd, (size_t)3 * n + 65536);
    // Gram partials of 1024 blocks past 2^16 rows, twice over
    if (n > (1 << 16)) wsd = std::max(wsd, (size_t)4 * 1024 * k * k + 65536);
    c->ws.cap = wsd * sizeof(double);
    c->ws.base = dalloc<char>(c->ws.cap);

    const size_t fs = c->fsize();
    c->W = dalloc<char>((size_t)n * k * fs);
    c->H = dalloc<char>((size_t)n * k * fs);
    c->Y = dalloc<char>((size_t)n * CMAX * fs);
    if (c->kind == SYMNMF_CSR) {
      c->Yk = dalloc<char>((size_t)n * c->kp * fs);
      HIPCHK(hipMemsetAsync(c->Yk, 0, (size_t)n * c->kp * fs, c->st));
      if (c->cdtype == SYMNMF_BF16) {
        c->BtW = dalloc<char>((size_t)n * k * 2);
        c->BtH = dalloc<char>((size_t)n * k * 2);
      }
    }
    if (c->kind == SYMNMF_DENSE) {
      // partials buffer: the largest splits * cp over every product width
      size_t pmax = 0;
      for (int cc = 16; cc <= CMAX; cc += 16) {
        const GemmPlan p = gemm_plan(n, cc, c->cdtype);
        pmax = std::max(pmax, (size_t)p.splits * p.cp);
      }
      const size_t acc = c->cdtype == SYMNMF_F64 ? 8 : 4;
      c->P = dalloc<char>(pmax * n * acc);
      c->Bt = dalloc<char>(gemm_bt_bytes(n, CMAX));
      c->BtW = dalloc<char>(gemm_bt_bytes(n, k));
      c->BtH = dalloc<char>(gemm_bt_bytes(n, k));
      HIPCHK(hipMemsetAsync(c->BtW, 0, gemm_bt_bytes(n, k), c->st));
      HIPCHK(hipMemsetAsync(c->BtH, 0, gemm_bt_bytes(n, k), c->st));
    }
    if (c->opt.rule == SYMNMF_RULE_BPP) c->Yhat = dalloc<double>((size_t)n * c->kp);
    if (c->opt.rule == SYMNMF_RULE_PGNCG) {
      c->nbc = cg_blocks(n);
      c->cgR = dalloc<double>((size_t)n * c->kp);
      c->cgP = dalloc<double>((size_t)n * c->kp);
      c->cgZ = dalloc<double>((size_t)n * c->kp);
      c->cg_part = dalloc<double>((size_t)c->nbc * cg_partial_doubles(k));
      c->cg_l1 = dalloc<double>((size_t)ceil_div(c->nbc, 32) * cg_partial_doubles(k));
      c->cg_sc = dalloc<double>(8 + (size_t)k * k);
      HIPCHK(hipMemsetAsync(c->cg_sc, 0, sizeof(double) * (8 + (size_t)k * k), c->st));
    }
    c->G_W = dalloc<double>((size_t)k * k);
    c->G_H = dalloc<double>((size_t)k * k);
    c->Gh_W = dalloc<double>((size_t)c->kp * c->kp);
    c->Gh_H = dalloc<double>((size_t)c->kp * c->kp);
    c->Gh_S = dalloc<double>((size_t)c->kp * c->kp);
    c->d_scal = dalloc<double>(16);
    c->nbu = update_blocks_max(n);
    c->pcap = (size_t)k * k;
    c->part = dalloc<double>((size_t)c->nbu * c->pcap);
    c->dpart = dalloc<double>(c->nbu);
    c->Gi_W = dalloc<double>(c->kp);
    c->Gi_H = dalloc<double>(c->kp);
    c->Gi_S = dalloc<double>(c->kp);
    LCHK(pad_identity(c->Gh_W, c->Gi_W, k, c->kp, c->st));
    LCHK(pad_identity(c->Gh_H, c->Gi_H, k, c->kp, c->st));
    LCHK(pad_identity(c->Gh_S, c->Gi_S, k, c->kp, c->st));
    c->rowsum = dalloc<double>(n);
    c->dstate = dalloc<DevState>(1);
    c->hist = dalloc<double>(c->opt.max_history);
    c->d_fail = dalloc<int>(1);
    c->R = dalloc<double>((size_t)k * k);
    c->Rinv = dalloc<double>((size_t)k * k);
    c->lev = dalloc<double>(n);
    if (!(c->hbuf = pinned_pool().get()))
      throw Fail{SYMNMF_E_NOMEM, "pinned host buffer"};
    HIPCHK(hipMemsetAsync(c->dstate, 0, sizeof(DevState), c->st));
    HIPCHK(hipMemsetAsync(c->d_fail, 0, sizeof(int), c->st));
    HIPCHK(hipMemsetAsync(c->d_scal, 0, 16 * sizeof(double), c->st));

    // compute copy of X
    c->Xc = c->Xv;
    if (c->kind == SYMNMF_DENSE && c->cdtype == SYMNMF_BF16 && c->xdtype == SYMNMF_F32) {
      c->Xb_owned = dalloc<char>((size_t)n * n * 2);
      LCHK(convert_f32_bf16((const float*)c->Xv, c->ld, c->Xb_owned, n, n, c->st));
      c->Xc = c->Xb_owned;
    }

    // one pass over X for the scalars
    c->ws.reset();
    if (c->kind == SYMNMF_DENSE)
      LCHK(dense_scalars(c->Xv, c->xdtype, c->ld, n, c->ws, c->rowsum, c->d_scal, c->st));
    else
      LCHK(csr_scalars(c->rp, c->Xv, c->xdtype, n, c->nnz, c->ws, c->rowsum, c->d_scal, c->st));
    const double* h = c->readback(c->d_scal, 3);
    c->normsq = h[0];
    c->total = h[1];
    c->maxval = h[2];
    if (c->kind == SYMNMF_CSR && (double)c->nnz < (double)n * (double)n) c->maxval = std::fmax(c->maxval, 0.0);
    if (!std::isfinite(c->normsq) || !std::isfinite(c->total)) throw Fail{SYMNMF_E_INVALID, "X has NaN or Inf"};
    if (!(c->normsq > 0.0)) throw Fail{SYMNMF_E_INVALID, "X is zero"};
    c->alpha = alpha > 0.0 ? alpha : c->maxval;
    if (!(c->alpha > 0.0)) throw Fail{SYMNMF_E_INVALID, "alpha = max(X) is not positive"};
    c->zeta = c->total / ((double)n * (double)n);
    if (!(c->zeta > 0.0)) throw Fail{SYMNMF_E_INVALID, "mean of X is not positive"};
    c->tau = c->opt.tau >= 0.0 ? c->opt.tau : (s > 0 ? 1.0 / (double)s : 0.0);

    // H0 = U[0,1) * 2 sqrt(zeta / k), W0 = H0 (Section 5 initialisation)
    LCHK(init_uniform_factor(c->H, c->fdtype, n, k, 2.0 * std::sqrt(c->zeta / k), seed, c->st));
    HIPCHK(hipMemcpyAsync(c->W, c->H, (size_t)n * k * fs, hipMemcpyDeviceToDevice, c->st));
    c->refresh_gram(c->H, c->G_H, c->Gh_H, c->Gi_H);
    // W0 = H0: its Gram matrices are copies
    HIPCHK(hipMemcpyAsync(c->G_W, c->G_H, sizeof(double) * k * k, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->Gh_W, c->Gh_H, sizeof(double) * c->kp * c->kp, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->Gi_W, c->Gi_H, sizeof(double) * c->kp, hipMemcpyDeviceToDevice, c->st));

    if (s > 0) {
      if (c->kind != SYMNMF_CSR) throw Fail{SYMNMF_E_UNSUPPORTED, "sampling needs CSR X"};
      c->mode = SYMNMF_MODE_LVS;
      // bound on selected rows: the s draws plus the rows with p_i >= tau
      // (sum p_i = 1 up to rounding, so at most about 1/tau of them)
      int64_t ms = c->tau > 0.0 ? s + (int64_t)std::ceil(1.01 / c->tau) + 1 : (int64_t)n;
      c->max_sel = std::min<int64_t>(ms, n);
      // slab capacity: the stored entries of the max_sel longest rows
      std::vector<int> hrp((size_t)n + 1);
      HIPCHK(hipMemcpyAsync(hrp.data(), c->rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, c->st));
      c->sync();
      std::vector<int> len(n);
      for (int i = 0; i < n; ++i) len[i] = hrp[i + 1] - hrp[i];
      std::nth_element(len.begin(), len.begin() + (c->max_sel - 1), len.end(), std::greater<int>());
      int64_t cap = 0;
      for (int64_t i = 0; i < c->max_sel; ++i) cap += len[i];
      c->seg_cap = std::max<int64_t>(cap, 1);
      c->ensure_sampling_buffers();
      c->rows = dalloc<int>(c->max_sel);
      c->weights = dalloc<double>(c->max_sel);
      c->wmask = dalloc<double>(n);
      c->seg_cnt = dalloc<int>(n);
      c->seg_ptr = dalloc<int>((size_t)n + 1);
      c->seg_src = dalloc<int>(c->seg_cap);
      c->seg_val = dalloc<double>(c->seg_cap);
      HIPCHK(hipMemsetAsync(c->seg_cnt, 0, sizeof(int) * n, c->st));
    }
    c->sync();
  } catch (const Fail& f) {
    g_create_error = f.msg;
    delete c;
    return f.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    delete c;
    return SYMNMF_E_NOMEM;
  } catch (...) {
    g_create_error = "unexpected internal error";
    delete c;
    return SYMNMF_E_DEVICE;
  }
  *out = c;
  return SYMNMF_OK;
}

namespace {

// Validation and (re)allocation of the LAI buffers for rank l.
void lai_prepare(symnmf_ctx* c, int l) {
  if (c->mode == SYMNMF_MODE_LVS) throw Fail{SYMNMF_E_UNSUPPORTED, "LAI with sampling"};
  if (l < c->k || l > 96 || l > c->n) throw Fail{SYMNMF_E_INVALID, "need k <= l <= min(n, 96)"};
  const int n = c->n;
  if (c->l != l) {
    double** bufs[] = {&c->Q, &c->Q1, &c->U, &c->YQ, &c->Tm, &c->QT, &c->Vw, &c->lam, &c->Rl, &c->Rlinv, &c->Z};
    c->sync();
    for (double** b : bufs) {
      dfree(*b);
      *b = nullptr;
    }
    dfree(c->Uf);
    c->Uf = nullptr;
    c->l = l;
    c->Q = dalloc<double>((size_t)n * l);
    c->Q1 = dalloc<double>((size_t)n * l);
    c->U = dalloc<double>((size_t)n * l);
    if (c->fdtype == SYMNMF_F32) c->Uf = dalloc<float>((size_t)n * l);
    c->YQ = dalloc<double>((size_t)n * l);  // holds fdtype values
    c->Tm = dalloc<double>((size_t)l * l);
    c->QT = dalloc<double>((size_t)l * l);
    c->Vw = dalloc<double>((size_t)l * l);
    c->lam = dalloc<double>(l);
    c->Rl = dalloc<double>((size_t)l * l);
    c->Rlinv = dalloc<double>((size_t)l * l);
    c->Z = dalloc<double>((size_t)l * c->k);
    dfree(c->M_W);
    dfree(c->M_H);
    const size_t need = (size_t)c->k * c->k + (size_t)l * c->k;
    if (need > c->pcap) {
      dfree(c->part);
      c->part = nullptr;
      c->pcap = need;
      c->part = dalloc<double>((size_t)c->nbu * c->pcap);
    }
    c->M_W = dalloc<double>((size_t)l * c->kp);
    c->M_H = dalloc<double>((size_t)l * c->kp);
    HIPCHK(hipMemsetAsync(c->M_W, 0, sizeof(double) * l * c->kp, c->st));
    HIPCHK(hipMemsetAsync(c->M_H, 0, sizeof(double) * l * c->kp, c->st));
  }
  HIPCHK(hipMemsetAsync(c->d_fail, 0, sizeof(int), c->st));
}

// Algorithm Apx-EVD on the basis in c->Q, then the switch to LAI mode.
void lai_finish(symnmf_ctx* c) {
  const int n = c->n, l = c->l;
  {
    symnmf_ctx::Timed tm(c, SYMNMF_PHASE_LAI);
    // Algorithm Apx-EVD: T = Q^T (X Q), T = Q_T Lambda Q_T^T, U = Q Q_T.
    c->product(c->Q, SYMNMF_F64, l, c->YQ);
    c->ws.reset();
    LCHK(gram(c->Q, SYMNMF_F64, l, l, c->YQ, c->fdtype, l, l, n, nullptr, nullptr, nullptr, 0, c->ws, c->Tm,
            nullptr, 0, 0.0, nullptr, c->st));
    LCHK(jacobi_evd(c->Tm, l, c->QT, c->lam, c->st));
    LCHK(rowmat(c->Q, SYMNMF_F64, l, n, l, c->QT, nullptr, l, c->U, SYMNMF_F64, l, nullptr, c->st));
    c->ws.reset();
    LCHK(column_sign_fix(c->U, n, l, c->ws, c->st));
    if (c->Uf) LCHK(copy_convert(c->U, SYMNMF_F64, c->Uf, SYMNMF_F32, (int64_t)n * l, c->st));
    frob_dot(c->lam, c->lam, l, c->d_scal + 8, c->st);
  }
  HIPCHK(hipMemcpyAsync(c->hbuf, c->d_scal + 8, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(c->hbuf + 1, c->d_fail, sizeof(int), hipMemcpyDeviceToHost, c->st));
  c->sync();
  c->normsq_lai = c->hbuf[0];
  int failed = 0;
  std::memcpy(&failed, c->hbuf + 1, sizeof(int));
  if (failed) throw Fail{SYMNMF_E_NUMERIC, "CholeskyQR2 broke down"};
  if (!(c->normsq_lai > 0.0)) throw Fail{SYMNMF_E_NUMERIC, "low-rank approximation is zero"};
  c->mode = SYMNMF_MODE_LAI;
  c->mW_ok = c->mH_ok = false;
  c->bump_generation();
}

}  // namespace

int symnmf_lai(symnmf_ctx* c, int32_t l, int32_t q) {
  return guarded(c, [&] {
    if (q < 0 || q > 64) throw Fail{SYMNMF_E_INVALID, "q out of range"};
    lai_prepare(c, l);
    const int n = c->n;
    // Algorithm RRF: Omega Gaussian (Philox), then 2q+1 products each followed
    // by CholeskyQR (re-orthonormalising after every product; CholeskyQR2
    // after the last one).
    {
      symnmf_ctx::Timed tm(c, SYMNMF_PHASE_LAI);
      LCHK(gen_gaussian(c->Q, (int64_t)n * l, c->seed, 0, TAG_OMEGA, c->st));
      for (int it = 0; it < 2 * q + 1; ++it) {
        c->product(c->Q, SYMNMF_F64, l, c->YQ);
        c->cholqr(c->YQ, it == 2 * q);
      }
    }
    lai_finish(c);
  });
}

int symnmf_lai_adaptive(symnmf_ctx* c, int32_t l, int32_t q_max, double tol, int32_t* rounds_out,
                        double* qb_residual) {
  return guarded(c, [&] {
    if (q_max < 1 || q_max > 64) throw Fail{SYMNMF_E_INVALID, "q_max out of range"};
    if (!(tol >= 0.0)) throw Fail{SYMNMF_E_INVALID, "tol must be >= 0"};
    lai_prepare(c, l);
    const int n = c->n;
    const int64_t nl = (int64_t)n * l;
    // Algorithm Ada-RRF: Q = qr(X Omega); each round B^T = X Q, the
    // normalised QB residual sqrt((||X||^2 - ||B||_F^2) / ||X||^2) (trace
    // identity), Q = qr(B^T); stop when the residual fell by less than tol,
    // else Y = X Q, Q = qr(Y).  A basis that may be returned is made
    // orthonormal to working precision (CholeskyQR2).
    int rounds = 0;
    double prev = INFINITY, r = 0.0;
    {
      symnmf_ctx::Timed tm(c, SYMNMF_PHASE_LAI);
      LCHK(gen_gaussian(c->Q, nl, c->seed, 0, TAG_OMEGA, c->st));
      c->product(c->Q, SYMNMF_F64, l, c->YQ);
      c->cholqr(c->YQ, false);
      for (int j = 0; j < q_max; ++j) {
        c->product(c->Q, SYMNMF_F64, l, c->YQ);
        c->ws.reset();
        double* part = nullptr;
        const int nb = dot_partials(c->YQ, c->YQ, c->fdtype, nl, c->ws, &part, nullptr, c->st);
        if (nb < 0) throw Fail{SYMNMF_E_DEVICE, "dot launch failed"};
        sum_partials(part, nb, c->d_scal + 5, c->st);
        c->cholqr(c->YQ, true);
        const double b2 = c->readback(c->d_scal + 5, 1)[0];
        r = std::sqrt(std::fmax(c->normsq - b2, 0.0) / c->normsq);
        if (prev - r < tol) break;
        prev = r;
        c->product(c->Q, SYMNMF_F64, l, c->YQ);
        c->cholqr(c->YQ, j == q_max - 1);
        ++rounds;
      }
    }
    lai_finish(c);
    if (rounds_out) *rounds_out = rounds;
    if (qb_residual) *qb_residual = r;
  });
}

int symnmf_refine(symnmf_ctx* c, int32_t stop_mode, double target) {
  return guarded(c, [&] {
    if (c->mode != SYMNMF_MODE_LAI) throw Fail{SYMNMF_E_STATE, "refinement needs a context in LAI mode"};
    if (stop_mode < SYMNMF_STOP_NONE || stop_mode > SYMNMF_STOP_STALL_OR_TARGET)
      throw Fail{SYMNMF_E_INVALID, "stop_mode"};
    DevState d = c->read_state();
    d.done = 0;
    d.stall = 0;
    d.prev = INFINITY;
    std::memcpy(c->hbuf, &d, sizeof(DevState));
    HIPCHK(hipMemcpyAsync(c->dstate, c->hbuf, sizeof(DevState), hipMemcpyHostToDevice, c->st));
    c->sync();
    c->opt.stop_mode = stop_mode;
    c->opt.target = target;
    c->mode = SYMNMF_MODE_PLAIN;
    c->btW_ok = c->btH_ok = false;
    c->bump_generation();
  });
}

int symnmf_iterate(symnmf_ctx* c, int32_t iters, int32_t* done) {
  return guarded(c, [&] {
    if (iters < 0) throw Fail{SYMNMF_E_INVALID, "iters < 0"};
    const DevState before = c->read_state();
    if (!before.done) {
      const bool polled = c->opt.stop_mode != SYMNMF_STOP_NONE;
      const int every = polled ? std::max(1, c->opt.check_every) : iters;
      const int block = polled ? std::min(every, 16) : 8;
      int t = 0, since_poll = 0;
      while (t < iters) {
        int step = 0;
        if (c->steady()) {
          const bool whole_block = block > 1 && iters - t >= block && (!polled || every % block == 0);
          if (whole_block) {
            if (c->graph_ready(1, block)) {
              if (c->graph_iterations(1, block)) step = block;
            } else {
              // run this block with direct launches and capture the graph
              // behind it: instantiation then overlaps the block's device work
              for (int b = 0; b < block; ++b) c->one_iteration();
              step = block;
              (void)c->graph_capture(1, block);
            }
          } else if (c->graph_iterations(0, 1)) {
            step = 1;
          }
        }
        if (step == 0) {
          c->one_iteration();
          step = 1;
        }
        t += step;
        since_poll += step;
        if (polled && since_poll >= every && t < iters) {
          since_poll = 0;
          if (c->read_state().done) break;
        }
      }
    }
    const DevState after = c->read_state();
    if (done) *done = after.iter - before.iter;
  });
}

int symnmf_residual(symnmf_ctx* c, int32_t mode, double out[2]) {
  return guarded(c, [&] {
    if (!out) throw Fail{SYMNMF_E_INVALID, "null out"};
    if (mode == SYMNMF_RESID_FAST) {
      const bool lai = c->mode == SYMNMF_MODE_LAI;
      out[0] = c->trace_residual(c->W, c->H, lai);
      out[1] = c->trace_residual(c->H, c->H, lai);
    } else if (mode == SYMNMF_RESID_EXACT) {
      if (c->k > 64) throw Fail{SYMNMF_E_UNSUPPORTED, "k"};
      out[0] = c->exact_residual(c->W, c->H);
      out[1] = c->exact_residual(c->H, c->H);
    } else if (mode == SYMNMF_RESID_LAI) {
      if (c->l == 0 || c->mode != SYMNMF_MODE_LAI) throw Fail{SYMNMF_E_STATE, "no LAI factors"};
      out[0] = c->trace_residual(c->W, c->H, true);
      out[1] = c->trace_residual(c->H, c->H, true);
    } else {
      throw Fail{SYMNMF_E_INVALID, "residual mode"};
    }
  });
}

int symnmf_set_factor(symnmf_ctx* c, int32_t which, const void* src, int32_t dtype) {
  return guarded(c, [&] {
    if (!src || (which != SYMNMF_W && which != SYMNMF_H)) throw Fail{SYMNMF_E_INVALID, "argument"};
    if (dtype != SYMNMF_F64 && dtype != SYMNMF_F32) throw Fail{SYMNMF_E_INVALID, "dtype"};
    void* dst = which == SYMNMF_W ? c->W : c->H;
    LCHK(copy_convert(src, dtype, dst, c->fdtype, c->nk(), c->st));
    if (which == SYMNMF_W) c->refresh_gram(c->W, c->G_W, c->Gh_W, c->Gi_W);
    else c->refresh_gram(c->H, c->G_H, c->Gh_H, c->Gi_H);
    c->invalidate(which);
  });
}

int symnmf_get_factor(symnmf_ctx* c, int32_t which, void* dst, int32_t dtype) {
  return guarded(c, [&] {
    if (!dst || (which != SYMNMF_W && which != SYMNMF_H)) throw Fail{SYMNMF_E_INVALID, "argument"};
    if (dtype != SYMNMF_F64 && dtype != SYMNMF_F32) throw Fail{SYMNMF_E_INVALID, "dtype"};
    LCHK(copy_convert(which == SYMNMF_W ? c->W : c->H, c->fdtype, dst, dtype, c->nk(), c->st));
  });
}

int symnmf_get_lai(symnmf_ctx* c, void* U, void* lambda) {
  return guarded(c, [&] {
    if (c->l == 0) throw Fail{SYMNMF_E_STATE, "symnmf_lai has not run"};
    if (U) HIPCHK(hipMemcpyAsync(U, c->U, sizeof(double) * c->n * c->l, hipMemcpyDeviceToDevice, c->st));
    if (lambda) HIPCHK(hipMemcpyAsync(lambda, c->lam, sizeof(double) * c->l, hipMemcpyDeviceToDevice, c->st));
  });
}

int symnmf_get_sketch(symnmf_ctx* c, int32_t l, void* Omega) {
  return guarded(c, [&] {
    if (!Omega) throw Fail{SYMNMF_E_INVALID, "null output"};
    if (l < 1 || l > c->n) throw Fail{SYMNMF_E_INVALID, "l must be in 1..n"};
    LCHK(gen_gaussian((double*)Omega, (int64_t)c->n * l, c->seed, 0, TAG_OMEGA, c->st));
  });
}

int symnmf_apply_x(symnmf_ctx* c, const void* B, int32_t cols, void* Yout) {
  return guarded(c, [&] {
    if (!B || !Yout || cols < 1 || cols > CMAX) throw Fail{SYMNMF_E_INVALID, "argument"};
    if (c->kind == SYMNMF_CSR && cols > 128) throw Fail{SYMNMF_E_INVALID, "cols"};
    c->product(B, c->fdtype, cols, Yout);
  });
}

int symnmf_half_step(symnmf_ctx* c, int32_t side, int32_t half_iter) {
  return guarded(c, [&] {
    if (side != 0 && side != 1) throw Fail{SYMNMF_E_INVALID, "side"};
    if (half_iter < 0) throw Fail{SYMNMF_E_INVALID, "half_iter"};
    if (c->opt.rule == SYMNMF_RULE_PGNCG) throw Fail{SYMNMF_E_UNSUPPORTED, "PGNCG has no half-steps"};
    c->half_step(side, half_iter, false);
  });
}

int symnmf_leverage(symnmf_ctx* c, int32_t which, void* lev) {
  return guarded(c, [&] {
    if (!lev || (which != SYMNMF_W && which != SYMNMF_H)) throw Fail{SYMNMF_E_INVALID, "argument"};
    const double* G = which == SYMNMF_W ? c->G_W : c->G_H;
    LCHK(chol_inverse(G, c->k, c->R, c->Rinv, &c->dstate->flags, SYMNMF_FLAG_LEV_SHIFT, c->d_fail, c->st));
    LCHK(leverage_scores(which == SYMNMF_W ? c->W : c->H, c->fdtype, c->n, c->k, c->Rinv, (double*)lev, nullptr,
                         c->st));
  });
}

int symnmf_sample(symnmf_ctx* c, const void* lev, int32_t half_iter, void* rows, void* weights, int64_t cap,
                  int64_t* count) {
  return guarded(c, [&] {
    if (!lev || !rows || !weights || !count || cap < 1) throw Fail{SYMNMF_E_INVALID, "argument"};
    if (c->s < 1) throw Fail{SYMNMF_E_STATE, "context has s = 0"};
    c->ensure_sampling_buffers();
    c->ws.reset();
    LCHK(hybrid_sample((const double*)lev, c->n, c->k, c->s, c->tau, c->seed, (uint32_t)half_iter, c->sb,
                       (int*)rows, (double*)weights, cap, c->ws, nullptr, c->st));
    HIPCHK(hipMemcpyAsync(c->hbuf, c->sb.info, 4 * sizeof(int), hipMemcpyDeviceToHost, c->st));
    c->sync();
    int info[4];
    std::memcpy(info, c->hbuf, sizeof(info));
    if ((int64_t)info[3] > cap) throw Fail{SYMNMF_E_INVALID, "capacity smaller than the number of sampled rows"};
    *count = info[3];
  });
}

int symnmf_history(symnmf_ctx* c, double* out, int32_t cap, int32_t* count) {
  return guarded(c, [&] {
    if (!out || !count || cap < 0) throw Fail{SYMNMF_E_INVALID, "argument"};
    const DevState d = c->read_state();
    const int m = std::min(std::min(d.iter, c->opt.max_history), cap);
    if (m > 0) HIPCHK(hipMemcpy(out, c->hist, sizeof(double) * m, hipMemcpyDeviceToHost));
    *count = m;
  });
}

int symnmf_get_stats(symnmf_ctx* c, symnmf_stats* out) {
  return guarded(c, [&] {
    if (!out || out->struct_size != (int32_t)sizeof(symnmf_stats)) throw Fail{SYMNMF_E_INVALID, "stats struct"};
    const DevState d = c->read_state();
    std::memset(out, 0, sizeof(*out));
    out->struct_size = sizeof(symnmf_stats);
    out->mode = c->mode;
    out->iterations = d.iter;
    out->stopped = d.done;
    out->k = c->k;
    out->l = c->l;
    out->n = c->n;
    out->alpha = c->alpha;
    out->zeta = c->zeta;
    out->normsq = c->normsq;
    out->maxval = c->maxval;
    out->last_residual = d.last;
    out->flags = d.flags;
    out->warm_beta = c->warm_ran ? c->readback(c->d_scal + 9, 1)[0] : 0.0;
    out->graph_launches = c->graph_launches;
    c->harvest_timers();
    for (int p = 0; p < SYMNMF_NUM_PHASES; ++p) {
      out->phase_ms[p] = c->phase_ms[p];
      out->phase_calls[p] = c->phase_calls[p];
    }
    if (c->sb.info) {
      HIPCHK(hipMemcpyAsync(c->hbuf, c->sb.info, 4 * sizeof(int), hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipMemcpyAsync(c->hbuf + 2, c->sb.theta, sizeof(double), hipMemcpyDeviceToHost, c->st));
      c->sync();
      int info[4];
      std::memcpy(info, c->hbuf, sizeof(info));
      out->s_D = info[0];
      out->sample_rows = info[3];
      out->theta_over_k = c->hbuf[2] / c->k;
    }
  });
}

// ---- learned warm start ------------------------------------------------------


int symnmf_mlp_create(symnmf_mlp** out, int32_t hidden, uint64_t seed, void* hip_stream) {
  if (!out) return SYMNMF_E_INVALID;
  *out = nullptr;
  if (mlp_param_count(hidden) < 0) {
    g_create_error = "unsupported hidden width";
    return SYMNMF_E_INVALID;
  }
  symnmf_mlp* net = new (std::nothrow) symnmf_mlp();
  if (!net) return SYMNMF_E_NOMEM;
  const int rc = mlp_guarded(net, [&] {
    net->hidden = hidden;
    net->st = (hipStream_t)hip_stream;
    net->np = mlp_param_count(hidden);
    net->p = dalloc<float>(net->np);
    net->m = dalloc<float>(net->np);
    net->v = dalloc<float>(net->np);
    net->g = dalloc<float>(net->np);
    net->d_loss = dalloc<double>(1);
    if (!(net->hbuf = pinned_pool().get()))
      throw Fail{SYMNMF_E_NOMEM, "pinned allocation failed"};
    LCHK(mlp_init(net->p, seed, net->st));
    HIPCHK(hipMemsetAsync(net->m, 0, sizeof(float) * net->np, net->st));
    HIPCHK(hipMemsetAsync(net->v, 0, sizeof(float) * net->np, net->st));
    HIPCHK(hipStreamSynchronize(net->st));
  });
  if (rc != SYMNMF_OK) {
    g_create_error = net->err;
    delete net;
    return rc;
  }
  *out = net;
  return SYMNMF_OK;
}

int symnmf_mlp_num_params(const symnmf_mlp* net, int64_t* count) {
  if (!net || !count) return SYMNMF_E_INVALID;
  *count = net->np;
  return SYMNMF_OK;
}

int symnmf_mlp_set_params(symnmf_mlp* net, const float* src) {
  return mlp_guarded(net, [&] {
    if (!src) throw Fail{SYMNMF_E_INVALID, "null parameters"};
    HIPCHK(hipMemcpyAsync(net->p, src, sizeof(float) * net->np, hipMemcpyDeviceToDevice, net->st));
    HIPCHK(hipMemsetAsync(net->m, 0, sizeof(float) * net->np, net->st));
    HIPCHK(hipMemsetAsync(net->v, 0, sizeof(float) * net->np, net->st));
    net->t = 0;
  });
}

int symnmf_mlp_get_params(symnmf_mlp* net, float* dst) {
  return mlp_guarded(net, [&] {
    if (!dst) throw Fail{SYMNMF_E_INVALID, "null destination"};
    HIPCHK(hipMemcpyAsync(dst, net->p, sizeof(float) * net->np, hipMemcpyDeviceToDevice, net->st));
  });
}

int symnmf_mlp_forward(symnmf_mlp* net, const float* F, int64_t rows, float* Y) {
  return mlp_guarded(net, [&] {
    if (rows < 0 || (rows > 0 && (!F || !Y))) throw Fail{SYMNMF_E_INVALID, "argument"};
    LCHK(mlp_forward(net->p, F, rows, Y, net->st));
  });
}


int symnmf_mlp_gradient(symnmf_mlp* net, const float* F, const float* T, int64_t rows, float* grad, double* loss) {
  return mlp_guarded(net, [&] {
    if (!grad) throw Fail{SYMNMF_E_INVALID, "null gradient"};
    mlp_grad(net, F, T, rows, loss);
    HIPCHK(hipMemcpyAsync(grad, net->g, sizeof(float) * net->np, hipMemcpyDeviceToDevice, net->st));
  });
}

int symnmf_mlp_train_step(symnmf_mlp* net, const float* F, const float* T, int64_t rows, double lr, double* loss) {
  return mlp_guarded(net, [&] {
    if (!(lr > 0.0)) throw Fail{SYMNMF_E_INVALID, "learning rate"};
    mlp_grad(net, F, T, rows, loss);
    net->t += 1;
    LCHK(mlp_adam(net->p, net->g, net->m, net->v, net->np, lr, net->t, net->st));
  });
}

int symnmf_mlp_save(symnmf_mlp* net, const char* path) {
  return mlp_guarded(net, [&] {
    if (!path) throw Fail{SYMNMF_E_INVALID, "null path"};
    std::vector<float> h((size_t)net->np);
    HIPCHK(hipMemcpyAsync(h.data(), net->p, sizeof(float) * net->np, hipMemcpyDeviceToHost, net->st));
    HIPCHK(hipStreamSynchronize(net->st));
    MlpFileHeader hd;
    std::memcpy(hd.magic, kMlpMagic, sizeof(hd.magic));
    hd.hidden = net->hidden;
    hd.features = MLP_D_IN;
    hd.count = net->np;
    FILE* f = std::fopen(path, "wb");
    if (!f) throw Fail{SYMNMF_E_INVALID, std::string("cannot open ") + path + " for writing"};
    const bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 && std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) throw Fail{SYMNMF_E_INVALID, std::string("write to ") + path + " failed"};
  });
}

int symnmf_mlp_load(symnmf_mlp** out, const char* path, void* hip_stream) {
  if (!out || !path) {
    g_create_error = "null argument";
    return SYMNMF_E_INVALID;
  }
  *out = nullptr;
  MlpFileHeader hd;
  std::vector<float> h;
  {
    FILE* f = std::fopen(path, "rb");
    if (!f) {
      g_create_error = std::string("cannot open ") + path;
      return SYMNMF_E_INVALID;
    }
    bool ok = std::fread(&hd, sizeof(hd), 1, f) == 1 && std::memcmp(hd.magic, kMlpMagic, sizeof(hd.magic)) == 0 &&
              hd.features == MLP_D_IN && mlp_param_count(hd.hidden) > 0 && hd.count == mlp_param_count(hd.hidden);
    if (ok) {
      h.resize((size_t)hd.count);
      ok = std::fread(h.data(), sizeof(float), h.size(), f) == h.size() && std::fgetc(f) == EOF;
    }
    std::fclose(f);
    if (!ok) {
      g_create_error = std::string(path) + " is not a network file of this library (magic, sizes or length)";
      return SYMNMF_E_INVALID;
    }
  }
  symnmf_mlp* net = nullptr;
  int rc = symnmf_mlp_create(&net, hd.hidden, 0, hip_stream);
  if (rc != SYMNMF_OK) return rc;
  rc = mlp_guarded(net, [&] {
    HIPCHK(hipMemcpyAsync(net->p, h.data(), sizeof(float) * net->np, hipMemcpyHostToDevice, net->st));
    HIPCHK(hipStreamSynchronize(net->st));
  });
  if (rc != SYMNMF_OK) {
    g_create_error = net->err;
    delete net;
    return rc;
  }
  *out = net;
  return SYMNMF_OK;
}

const char* symnmf_mlp_last_error(const symnmf_mlp* net) { return net ? net->err.c_str() : g_create_error.c_str(); }

void symnmf_mlp_destroy(symnmf_mlp* net) { delete net; }

int symnmf_warm_features(symnmf_ctx* c, float* F) {
  return guarded(c, [&] {
    if (!F) throw Fail{SYMNMF_E_INVALID, "null output"};
    if (c->l == 0 || !c->U) throw Fail{SYMNMF_E_STATE, "symnmf_lai has not run"};
    c->ws.reset();
    double* info = c->ws.dbl((size_t)2 * c->k + 2);
    if (!info) throw Fail{SYMNMF_E_NOMEM, "workspace"};
    LCHK(warm_features(c->U, c->n, c->l, c->k, c->lam, c->rowsum, c->d_scal + 1, F, info, c->ws, c->st));
  });
}

int symnmf_warmstart(symnmf_ctx* c, const symnmf_mlp* net, double* beta_out) {
  return guarded(c, [&] {
    if (!net) throw Fail{SYMNMF_E_INVALID, "null network"};
    if (c->l == 0 || !c->U) throw Fail{SYMNMF_E_STATE, "symnmf_lai has not run"};
    const int64_t nk = (int64_t)c->n * c->k;
    if (!c->warm_F) {
      c->warm_F = dalloc<float>((size_t)nk * MLP_D_IN);
      c->warm_Htf = dalloc<float>(nk);
      c->warm_Ht = dalloc<char>((size_t)nk * c->fsize());
    }
    warmstart_run(c, net, c->warm_F, c->warm_Htf, c->warm_Ht, beta_out);
  });
}

int symnmf_warmstart_noalloc(symnmf_ctx* c, const symnmf_mlp* net, double* beta_out) {
  return guarded(c, [&] {
    if (!net) throw Fail{SYMNMF_E_INVALID, "null network"};
    const size_t need = warm_scratch_bytes((int64_t)c->n * c->k, c->fsize());
    if (need > kWarmScratchBytes)
      throw Fail{SYMNMF_E_INVALID, "n k = " + std::to_string((int64_t)c->n * c->k) + " needs " +
                                       std::to_string(need) + " bytes of temporaries; the static scratch holds " +
                                       std::to_string(kWarmScratchBytes)};
    if (c->l == 0 || !c->U) throw Fail{SYMNMF_E_STATE, "symnmf_lai has not run"};
    char* base = warm_scratch_device();
    const int64_t nk = (int64_t)c->n * c->k;
    float* F = (float*)base;
    float* Htf = (float*)(base + align256((size_t)nk * MLP_D_IN * sizeof(float)));
    void* Ht = base + align256((size_t)nk * MLP_D_IN * sizeof(float)) + align256((size_t)nk * sizeof(float));
    warmstart_run(c, net, F, Htf, Ht, beta_out);
  });
}

int symnmf_trim_cache(void) {
  device_cache().trim();
  return SYMNMF_OK;
}

const char* symnmf_last_error(const symnmf_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void symnmf_destroy(symnmf_ctx* c) { delete c; }

}  // extern "C"
