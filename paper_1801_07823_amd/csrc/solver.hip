// The KD-MG solve (Sec. 4, Table 1): flexible GCR on the KD-block-parity Schur
// operator S = 1 - A_eo A_oe, preconditioned by a K-cycle
//   MR(2, 0.85) -> restrict -> coarse solve -> prolong -> MR(2, 0.85),
// with GCR(8, max 16, tol 0.2) on intermediate levels and CGNE (tol 0.2,
// max 256) on the coarsest.  Precision: KDMG_FP64 runs every level in FP64;
// KDMG_MIXED keeps the outer FGCR, its residuals and all dot products in
// FP64, runs the V-cycle in FP32 with FP16-stored links and prolongators and
// FP32 coarse operators, and the coarsest CGNE in FP64.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>

#include "algos.h"
#include "api_guard.h"

using namespace kdmg;

namespace kdmg {

template <class F>
void with_prec(Prec p, F f) {
  if (p == Prec::F64) f(double{});
  else f(float{});
}

// Two pinned host slots and events for polling device flags without
// draining the stream: the copy of chunk c is checked while chunk c + 1 runs.
struct AsyncPoll {
  int* host = nullptr;  // [2][n]
  hipEvent_t ev[2] = {nullptr, nullptr};
  int n = 0;
  void init(int nflags) {
    n = nflags;
    std::lock_guard<std::mutex> g(hip_mem_mutex());
    KDMG_HIP(hipHostMalloc((void**)&host, sizeof(int) * 2 * n, hipHostMallocDefault));
    for (auto& e : ev) KDMG_HIP(hipEventCreate(&e));
  }
  AsyncPoll() = default;
  AsyncPoll(const AsyncPoll&) = delete;
  AsyncPoll& operator=(const AsyncPoll&) = delete;
  ~AsyncPoll() {
    std::lock_guard<std::mutex> g(hip_mem_mutex());
    if (host) (void)hipHostFree(host);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// A captured chunk of fused CGNE iterations (k = 0 .. n-1, so parities
// match any chunk that starts at an even k) for one workspace and launch
// shape, replayed with hipGraphLaunch.  The kernels read their per-rhs state
// from device memory, so one capture serves every call on the workspace.
struct ChunkGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;  // private stream the chunk is captured on (the solve stream may be the null stream)
  long long replays = 0;
  TileShape sh;
  int n = 0, nrhs = 0;
  bool failed = false;
  bool matches(const TileShape& s, int iters, int nr) const {
    return exec && n == iters && nrhs == nr && sh.core == s.core && sh.RT == s.RT && sh.TI == s.TI &&
           sh.TR == s.TR && sh.KS == s.KS && sh.MT == s.MT && sh.NT == s.NT && sh.ylds == s.ylds &&
           sh.threads == s.threads && sh.smem == s.smem;
  }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
    exec = nullptr;
    g = nullptr;
  }
  ChunkGraph() = default;
  ChunkGraph(const ChunkGraph&) = delete;
  ChunkGraph& operator=(const ChunkGraph&) = delete;
  ~ChunkGraph() {
    reset();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

struct LevelWS {
  Prec prec = Prec::F64;
  long n = 0;                 // complex entries per rhs in this level's solve space
  size_t esz = 16;            // bytes per complex entry
  DevBuf r1, x, r2, q;        // K-cycle work (levels that have a coarser level)
  DevBuf t, w;                // level-0 Schur temporaries (full layout)
  DevBuf b, xs, rs, Z, W, p;  // coarse solve: input, solution, residual, GCR basis / CGNE p
  DevBuf cg_rr, cg_target, cg_act, PA, PB;  // fused CGNE state (coarsest level)
  DevBuf part;                               // exact coarsest solve: partial products
  std::unique_ptr<AsyncPoll> cg_poll;        // its flag copies and events
  std::unique_ptr<ChunkGraph> cg_graph;      // captured CGNE chunk
  // the fused CGNE's tail problem of `tail` rhs (0: none; batches of more
  // rhs than kdmg_mg_params.coarse_tail only)
  int tail = 0;
  DevBuf tx, tr, tp, trr, ttarget, tact, tints, tPA, tPB, tidx;
  // intermediate GCR above the exact coarsest solve: the iteration count of
  // its last call, the first iteration after which the next call polls
  int gcr_last = 0;
  std::unique_ptr<ChunkGraph> cg_graph_t;
  KrylovAlloc ks, kmr;
  template <class T> Cx<T>* v(DevBuf& d) const { return d.as<Cx<T>>(); }
};

// Captured halves of the K-cycle on the level just above an exact coarsest
// solve: everything before the coarsest product (start, pre-smoothing,
// restriction) and everything after it (prolongation, residual,
// post-smoothing) contains no host decision, so each is one hipGraph per
// (level, output column, input vector) of the intermediate GCR.  The
// coarsest product runs between the two replays as plain launches, where the
// live kernel timing can bracket it.  Captured on a private stream, replayed
// on the solve's stream.
struct KCycleGraphs {
  struct Pair {
    hipGraph_t g[2] = {nullptr, nullptr};
    hipGraphExec_t x[2] = {nullptr, nullptr};
  };
  hipStream_t cap = nullptr;
  std::map<std::tuple<int, const void*, const void*, const void*>, Pair> m;
  bool failed = false;
  KCycleGraphs() = default;
  KCycleGraphs(const KCycleGraphs&) = delete;
  KCycleGraphs& operator=(const KCycleGraphs&) = delete;
  ~KCycleGraphs() {
    for (auto& kv : m)
      for (int i = 0; i < 2; ++i) {
        if (kv.second.x[i]) (void)hipGraphExecDestroy(kv.second.x[i]);
        if (kv.second.g[i]) (void)hipGraphDestroy(kv.second.g[i]);
      }
    if (cap) (void)hipStreamDestroy(cap);
  }
};

struct SolveWS {
  int nrhs = 0;
  kdmg_prec prec = KDMG_FP64;
  std::atomic<int> busy{0};
  CtxAlloc ctx;
  std::unique_ptr<KCycleGraphs> kgraphs = std::make_unique<KCycleGraphs>();
  // outer (FP64, even half)
  DevBuf bfull, yfull, xfull, tfull, wfull, bt, ye, re, Zo, Wo, bnorm2, rnorm2, xin32, xout32;
  KrylovAlloc kout;
  std::vector<LevelWS> lv;
  size_t bytes = 0;
};

void destroy_ws(SolveWS* w) { delete w; }

// Captured K-cycle graphs hold the transfer and operator pointers of the
// hierarchy they were captured on; drop them when those change.
void reset_graphs(SolveWS* w) {
  if (w) w->kgraphs = std::make_unique<KCycleGraphs>();
}
bool ws_busy(const SolveWS* w) { return w && w->busy.load() != 0; }

namespace {

struct OpStridedCopy {  // dst[r][i] = src[r][i] for i < n, with separate strides
  c64* dst; long sd; const c64* src; long ss; long n;
  __device__ bool active(int) const { return true; }
  __device__ void elem(int r, long i) const { dst[r * sd + i] = src[r * ss + i]; }
};

struct OpKCInit {  // x = 0 ; r1 = r
  void* x; void* r1; const void* r; long n; const int* act; int f32;
  __device__ bool active(int rr) const { return is_active(act, rr); }
  __device__ void elem(int rr, long i) const {
    const long o = rr * n + i;
    if (f32) {
      ((c32*)x)[o] = c32{0, 0};
      ((c32*)r1)[o] = ((const c32*)r)[o];
    } else {
      ((c64*)x)[o] = c64{0, 0};
      ((c64*)r1)[o] = ((const c64*)r)[o];
    }
  }
};

struct OpResidNorm {  // ||r||^2 -> out[r]
  const c64* r; long n; long stride; double* out;
  __device__ bool active(int) const { return true; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const { a.v[0] += norm2(r[rr * stride + i]); }
  __device__ void finish(int rr, int, const double* s) const { out[rr] = s[0]; }
};

// Fused CGNE on the coarsest level: two kernels per iteration (see
// coarse_fast.h), host reads the active flags every `poll` iterations.
// Capture `n` CGNE iterations on the (idle-by-construction) capture of c.st.
bool capture_chunk(ChunkGraph& G, const TileShape& sh, const CoarseLevel& L, c64* x, c64* r, c64* p,
                   const CgneState& s, int nrhs, int n) {
  std::lock_guard<std::mutex> lock(hip_mem_mutex());
  G.reset();
  if (!G.cap && hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking) != hipSuccess) {
    G.cap = nullptr;
    return false;
  }
  hipStream_t st = G.cap;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  hipGraph_t g = nullptr;
  try {
    for (int k = 0; k < n; ++k) launch_cgne_iter(sh, L, x, r, p, s, nrhs, k, st);
  } catch (const Error&) {
    if (hipStreamEndCapture(st, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    return false;
  }
  if (hipStreamEndCapture(st, &g) != hipSuccess || !g) return false;
  G.g = g;
  if (hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0) != hipSuccess) {
    G.reset();
    return false;
  }
  G.sh = sh;
  G.n = n;
  G.nrhs = nrhs;
  return true;
}

// Tail of the fused CGNE.  A batched call runs until its slowest rhs
// converges; once at most W.tail rhs are still active, their rows (x, r, p,
// the partial sums of ||p||^2 and the per-rhs scalars of both parity slots)
// are gathered into a W.tail-rhs problem that continues with the launch
// shape tuned for that width, and the solution and iteration counts are
// scattered back at the end.  idx[j] < 0 marks an empty, inactive row.
template <class T>
__global__ __launch_bounds__(256) void k_rows_gather(T* dst, const T* src, const int* idx, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, q = idx[j];
  if (i < n) dst[(long)j * n + i] = q >= 0 ? src[(long)q * n + i] : T{};
}

template <class T>
__global__ __launch_bounds__(256) void k_rows_scatter(T* dst, const T* src, const int* idx, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, q = idx[j];
  if (i < n && q >= 0) dst[(long)q * n + i] = src[(long)j * n + i];
}

__global__ __launch_bounds__(64) void k_cgne_state_gather(CgneState t, CgneState s, const int* idx, int nrhs, int nt) {
  const int j = threadIdx.x;
  if (j >= nt) return;
  const int q = idx[j];
  for (int sl = 0; sl < 2; ++sl) {
    t.rr[sl * nt + j] = q >= 0 ? s.rr[sl * nrhs + q] : 0.0;
    t.act[sl * nt + j] = q >= 0 ? s.act[sl * nrhs + q] : 0;
  }
  t.target[j] = q >= 0 ? s.target[q] : 0.0;
  t.its[j] = q >= 0 ? s.its[q] : 0;
  t.tot[j] = q >= 0 ? s.tot[q] : 0;
  t.calls[j] = q >= 0 ? s.calls[q] : 0;
}

__global__ __launch_bounds__(64) void k_cgne_state_scatter(CgneState s, CgneState t, const int* idx, int nt) {
  const int j = threadIdx.x;
  if (j >= nt || idx[j] < 0) return;
  const int q = idx[j];
  s.its[q] = t.its[j];
  s.tot[q] = t.tot[j];
  s.calls[q] = t.calls[j];
}

int cgne_fused(const Ctx& c, const CoarseLevel& L, LevelWS& W, int nrhs, const c64* b, c64* x, c64* r,
               c64* p, double tol, int maxit, const int* parent, int poll, kdmg_hierarchy::KTimer* tm,
               bool graphs) {
  CgneState s;
  s.rr = W.cg_rr.as<double>();
  s.target = W.cg_target.as<double>();
  s.act = W.cg_act.as<int>();
  s.its = W.ks.k.its;
  s.tot = W.ks.k.tot;
  s.calls = W.ks.k.calls;
  s.parent = parent;
  s.PA = W.PA.as<double>();
  s.PB = W.PB.as<double>();
  TileShape sh = cgne_shape(L, nrhs);
  KDMG_CHECK(sh.smem <= LDS_LIMIT, KDMG_EUNSUPPORTED, "coarsest operator too large for the fused CGNE");
  launch_cgne_init(sh, L, x, r, p, b, s, nrhs, tol * tol, c.st);
  // Chunks of `poll` iterations.  After each chunk the active flags are
  // copied to pinned host memory behind an event, and the previous chunk's
  // copy is checked while this chunk runs, so the stream never drains;
  // iterations launched past convergence return at once (all flags off).
  AsyncPoll& ap = *W.cg_poll;
  bool timed = tm && tm->on;  // live timing covers the full-width launches only
  bool pending[2] = {false, false};
  int done_its[2] = {0, 0};
  int cs = 0, k = 0;
  bool stop = false;
  auto account = [&](int slot) {  // kernel time from the first B launch to the end of a chunk
    if (timed && done_its[slot] * 2 - 1 > 0) {
      float ms = 0.f;
      KDMG_HIP(hipEventElapsedTime(&ms, tm->e0, ap.ev[slot]));
      tm->ms += ms;
      tm->launches += done_its[slot] * 2 - 1;
    }
  };
  // the problem the loop advances: the full batch, later possibly the tail
  int nr = nrhs;
  c64 *xc = x, *rc = r, *pc = p;
  CgneState sc = s;
  ChunkGraph* G = W.cg_graph.get();
  const int nt = W.tail;  // <= 64, the state kernels' block
  const bool can_tail = nt > 0 && W.cg_graph_t && nrhs > nt;
  bool tail = false;
  const long nv = (long)L.nsites * L.ndc;
  auto enter_tail = [&](const int* flags) -> bool {
    // flags: the active flags of iteration k (this chunk's copy, synchronised)
    int* idx_h = ap.host;  // both pinned slots are free here
    int na = 0;
    for (int q = 0; q < nrhs; ++q)
      if (flags[q]) idx_h[na++] = q;
    if (na == 0) return false;
    for (int j = na; j < nt; ++j) idx_h[j] = -1;
    int* idx = W.tidx.as<int>();
    KDMG_HIP(hipMemcpyAsync(idx, idx_h, sizeof(int) * nt, hipMemcpyHostToDevice, c.st));
    CgneState t;
    t.rr = W.trr.as<double>();
    t.target = W.ttarget.as<double>();
    t.act = W.tact.as<int>();
    t.its = W.tints.as<int>();
    t.tot = t.its + nt;
    t.calls = t.tot + nt;
    t.parent = nullptr;
    t.PA = W.tPA.as<double>();
    t.PB = W.tPB.as<double>();
    const dim3 gv(cdiv(nv, 256), nt), gs(cdiv(L.nsites, 256), nt);
    hipLaunchKernelGGL(k_rows_gather<c64>, gv, dim3(256), 0, c.st, W.tx.as<c64>(), x, idx, nv);
    hipLaunchKernelGGL(k_rows_gather<c64>, gv, dim3(256), 0, c.st, W.tr.as<c64>(), r, idx, nv);
    hipLaunchKernelGGL(k_rows_gather<c64>, gv, dim3(256), 0, c.st, W.tp.as<c64>(), p, idx, nv);
    hipLaunchKernelGGL(k_rows_gather<double>, gs, dim3(256), 0, c.st, t.PB, s.PB, idx, (long)L.nsites);
    hipLaunchKernelGGL(k_cgne_state_gather, dim3(1), dim3(64), 0, c.st, t, s, idx, nrhs, nt);
    KDMG_LAUNCH_CHECK();
    xc = W.tx.as<c64>();
    rc = W.tr.as<c64>();
    pc = W.tp.as<c64>();
    sc = t;
    nr = nt;
    sh = cgne_shape(L, nt);
    G = W.cg_graph_t.get();
    tail = true;
    if (tm) ++tm->tail_entries;
    return true;
  };
  while (k < maxit && !stop) {
    const int kend = std::min(k + poll, maxit);
    // the first chunk of a call runs eagerly (it also sets the kernels' LDS
    // limits and takes the timing start); later full chunks replay a graph
    bool replayed = false;
    if (graphs && k > 0 && kend - k == poll && k % 2 == 0 && !G->failed) {
      if (!G->matches(sh, poll, nr) && !capture_chunk(*G, sh, L, xc, rc, pc, sc, nr, poll)) {
        (void)hipGetLastError();
        G->failed = true;  // capture unavailable: stay eager on this workspace
      }
      if (!G->failed) {
        KDMG_HIP(hipGraphLaunch(G->exec, c.st));
        ++G->replays;
        if (tm) ++tm->graph_replays;
        k = kend;
        replayed = true;
      }
    }
    if (!replayed)
      for (; k < kend; ++k)
        launch_cgne_iter(sh, L, xc, rc, pc, sc, nr, k, c.st, timed && k == 0 ? tm->e0 : nullptr);
    KDMG_HIP(hipMemcpyAsync(ap.host + cs * nrhs, sc.act + (k & 1) * nr, sizeof(int) * nr,
                            hipMemcpyDeviceToHost, c.st));
    KDMG_HIP(hipEventRecord(ap.ev[cs], c.st));
    pending[cs] = true;
    done_its[cs] = k;
    const int ps = cs ^ 1;
    if (pending[ps]) {
      KDMG_HIP(hipEventSynchronize(ap.ev[ps]));
      pending[ps] = false;
      int active = 0;
      for (int q = 0; q < nr; ++q) active += ap.host[ps * nrhs + q] != 0;
      if (active == 0) {
        account(ps);
        stop = true;
      } else if (can_tail && !tail && active <= nt && k < maxit) {
        // drain to this chunk's end and take its (newer) flags as the set
        KDMG_HIP(hipEventSynchronize(ap.ev[cs]));
        pending[cs] = false;
        account(cs);
        timed = false;
        std::vector<int> flags(ap.host + cs * nrhs, ap.host + cs * nrhs + nrhs);
        if (!enter_tail(flags.data())) {
          stop = true;  // nothing left active
        } else {
          cs = 0;
          continue;
        }
      }
    }
    cs = ps;
  }
  if (!stop && timed) {  // ended at maxit: account the last chunk
    const int last = cs ^ 1;
    KDMG_HIP(hipEventSynchronize(ap.ev[last]));
    account(last);
  }
  if (tail) {
    const int* idx = W.tidx.as<int>();
    const dim3 gv(cdiv(nv, 256), nt);
    hipLaunchKernelGGL(k_rows_scatter<c64>, gv, dim3(256), 0, c.st, x, xc, idx, nv);
    hipLaunchKernelGGL(k_cgne_state_scatter, dim3(1), dim3(64), 0, c.st, s, sc, idx, nt);
    KDMG_LAUNCH_CHECK();
  }
  return k;
}

class Runner {
 public:
  Runner(kdmg_hierarchy& h, SolveWS& ws) : h_(h), ws_(ws), c_(ws.ctx.c), nrhs_(ws.nrhs) {}
  // the same solve state, launching on another stream (graph capture)
  Runner(kdmg_hierarchy& h, SolveWS& ws, const Ctx& c) : h_(h), ws_(ws), c_(c), nrhs_(ws.nrhs) {}

  // level-l operator in the level's precision: out = op(in) or resid - op(in)
  template <class T>
  void op(int l, Cx<T>* out, const Cx<T>* in, const Cx<T>* resid, const int* act, bool dag = false) {
    if (l == 0) {
      LevelWS& L = ws_.lv[0];
      const kdmg_lattice& lat = *h_.lat;
      if (lat.nd == 4) {
        if constexpr (sizeof(T) == 8)
          schur_apply4<T, double, double>(out, in, resid, L.v<T>(L.t), L.v<T>(L.w), fine4_64(), act, nrhs_, c_.st);
        else
          schur_apply4<T, _Float16, float>(out, in, resid, L.v<T>(L.t), L.v<T>(L.w), fine4_mixed(), act, nrhs_,
                                           c_.st);
      } else if (h_.fine_full) {
        using LT = std::conditional_t<sizeof(T) == 8, double, _Float16>;
        const Fine2<LT> F = fine2<LT>(lat, h_.mass);
        if (h_.naive)
          fine2_D<T, LT>(out, in, resid, F, act, nrhs_, c_.st);
        else
          fine2_A<T, LT>(out, in, resid, L.v<T>(L.t), F, act, nrhs_, c_.st);
      } else if constexpr (sizeof(T) == 8) {
        schur_apply<T, double>(out, in, resid, L.v<T>(L.t), L.v<T>(L.w), lat.links64.as<c64>(), lat.g,
                               h_.mass, act, nrhs_, c_.st);
      } else {
        schur_apply<T, _Float16>(out, in, resid, L.v<T>(L.t), L.v<T>(L.w), lat.links16.as<c16>(),
                                 lat.g, h_.mass, act, nrhs_, c_.st);
      }
    } else {
      if constexpr (sizeof(T) == 8)
        coarse_apply<T, double>(h_.L[l], dag, out, in, resid, resid ? -1.0 : 1.0, act, nrhs_, c_.st);
      else
        coarse_apply<T, float>(h_.L[l], dag, out, in, resid, resid ? -1.0 : 1.0, act, nrhs_, c_.st);
    }
  }

  // restrict level l (vector `in`, precision TI) into level l+1's input buffer
  template <class TI>
  void restrict_to(int l, const Cx<TI>* in, const int* act) {
    LevelWS& N = ws_.lv[l + 1];
    const Transfer& T = h_.T[l];
    const bool p16 = ws_.prec == KDMG_MIXED;
    with_prec(N.prec, [&](auto tag) {
      using TO = decltype(tag);
      Cx<TO>* out = N.v<TO>(N.b);
      const long si = ws_.lv[l].n;
      const int even_only = l == 0 && !h_.fine_full;
      if (p16)
        transfer_restrict<TO, _Float16, TI, TO>(T, *h_.lat, &h_.L[l], out, in, si, even_only, act, nrhs_, c_.st);
      else
        transfer_restrict<TO, double, TI, TO>(T, *h_.lat, &h_.L[l], out, in, si, even_only, act, nrhs_, c_.st);
    });
  }

  // x (level l, precision TO) += P (level l+1 solution)
  template <class TO>
  void prolong_add(int l, Cx<TO>* x, const int* act) {
    LevelWS& N = ws_.lv[l + 1];
    const Transfer& T = h_.T[l];
    const bool p16 = ws_.prec == KDMG_MIXED;
    const long so = ws_.lv[l].n;
    const int npar = l == 0 && h_.fine_full ? 2 : 1;
    with_prec(N.prec, [&](auto tag) {
      using TI = decltype(tag);
      const Cx<TI>* in = N.v<TI>(N.xs);
      if (p16)
        transfer_prolong<TO, _Float16, TI, TO>(T, *h_.lat, x, so, x, so, in, npar, act, nrhs_, c_.st);
      else
        transfer_prolong<TO, double, TI, TO>(T, *h_.lat, x, so, x, so, in, npar, act, nrhs_, c_.st);
    });
  }

  // K-cycle on level l: x ~= op_l^-1 r for the rhs in `act`
  template <class T>
  void kcycle(int l, Cx<T>* x, const Cx<T>* r, const int* act) {
    kcycle_pre<T>(l, x, r, act);
    coarse_solve(l + 1, act);
    kcycle_post<T>(l, x, r, act);
  }

  // x = 0, r1 = r ; MR(r1) ; restrict r1
  template <class T>
  void kcycle_pre(int l, Cx<T>* x, const Cx<T>* r, const int* act) {
    LevelWS& L = ws_.lv[l];
    const kdmg_mg_params& P = h_.params;
    const long n = L.n;
    Cx<T>* r1 = L.v<T>(L.r1);
    Cx<T>* q = L.v<T>(L.q);
    launch_map(OpKCInit{x, r1, r, n, act, sizeof(T) == 4}, n, nrhs_, c_.st);
    auto opf = [&](Cx<T>* o, const Cx<T>* i, const Cx<T>* res, const int* a) { op<T>(l, o, i, res, a); };
    const KrylovState kmr = L.kmr.under(act);
    mr_smooth<T>(c_, nrhs_, n, x, r1, q, P.mr_its, P.mr_omega, kmr, opf);
    restrict_to<T>(l, r1, act);
  }

  // x += P e ; r2 = r - op x ; MR(r2)
  template <class T>
  void kcycle_post(int l, Cx<T>* x, const Cx<T>* r, const int* act) {
    LevelWS& L = ws_.lv[l];
    const kdmg_mg_params& P = h_.params;
    const long n = L.n;
    Cx<T>* r2 = L.v<T>(L.r2);
    Cx<T>* q = L.v<T>(L.q);
    auto opf = [&](Cx<T>* o, const Cx<T>* i, const Cx<T>* res, const int* a) { op<T>(l, o, i, res, a); };
    const KrylovState kmr = L.kmr.under(act);
    prolong_add<T>(l, x, act);
    op<T>(l, r2, x, r, act);
    mr_smooth<T>(c_, nrhs_, n, x, r2, q, P.mr_its, P.mr_omega, kmr, opf);
  }

  // The K-cycle with its halves replayed from captured graphs (see
  // KCycleGraphs); falls back to plain launches if capture is unavailable.
  template <class T>
  void kcycle_graphed(int l, Cx<T>* x, const Cx<T>* r, const int* act) {
    KCycleGraphs& G = *ws_.kgraphs;
    if (G.failed) {
      kcycle<T>(l, x, r, act);
      return;
    }
    const auto key = std::make_tuple(l, (const void*)x, (const void*)r, (const void*)act);
    auto it = G.m.find(key);
    if (it == G.m.end()) {
      KCycleGraphs::Pair pr;
      bool ok = true;
      {
        std::lock_guard<std::mutex> lock(hip_mem_mutex());
        if (!G.cap && hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking) != hipSuccess) {
          G.cap = nullptr;
          ok = false;
        }
        Ctx cc = c_;
        cc.st = G.cap;
        Runner rc(h_, ws_, cc);
        for (int part = 0; part < 2 && ok; ++part) {
          if (hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            ok = false;
            break;
          }
          try {
            if (part == 0) rc.kcycle_pre<T>(l, x, r, act);
            else rc.kcycle_post<T>(l, x, r, act);
          } catch (const Error&) {
            ok = false;
          }
          hipGraph_t g = nullptr;
          if (hipStreamEndCapture(G.cap, &g) != hipSuccess || !g) ok = false;
          pr.g[part] = g;
          if (ok && hipGraphInstantiate(&pr.x[part], g, nullptr, nullptr, 0) != hipSuccess) ok = false;
        }
      }
      if (!ok) {
        (void)hipGetLastError();
        for (int i = 0; i < 2; ++i) {
          if (pr.x[i]) (void)hipGraphExecDestroy(pr.x[i]);
          if (pr.g[i]) (void)hipGraphDestroy(pr.g[i]);
        }
        G.failed = true;
        kcycle<T>(l, x, r, act);
        return;
      }
      it = G.m.emplace(key, pr).first;
    }
    KDMG_HIP(hipGraphLaunch(it->second.x[0], c_.st));
    coarse_solve(l + 1, act);
    KDMG_HIP(hipGraphLaunch(it->second.x[1], c_.st));
    h_.timer.graph_replays += 2;
  }

  // approximate solve on level l >= 1 of  op_l xs = b  (buffers of level l)
  void coarse_solve(int l, const int* parent) {
    LevelWS& L = ws_.lv[l];
    const kdmg_mg_params& P = h_.params;
    with_prec(L.prec, [&](auto tag) {
      using T = decltype(tag);
      const long n = L.n;
      Cx<T>* b = L.v<T>(L.b);
      Cx<T>* x = L.v<T>(L.xs);
      Cx<T>* r = L.v<T>(L.rs);
      auto opf = [&](Cx<T>* o, const Cx<T>* i, const Cx<T>* res, const int* a) { op<T>(l, o, i, res, a); };
      if (l == h_.nlevels - 1 && P.coarse_solver == 1) {
        if constexpr (sizeof(T) == 8) {
          auto& tm = h_.timer;
          std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
          int* worked = nullptr;
          if (tm.on && tm.dn_used < tm.DN_CAP) {
            if (!tm.dn_work.p) tm.dn_work.alloc(sizeof(int) * tm.DN_CAP);
            worked = tm.dn_work.as<int>() + tm.dn_used;
            if (tm.dn_used == tm.dn_ev.size()) {
              std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
              KDMG_HIP(hipEventCreate(&e.first));
              KDMG_HIP(hipEventCreate(&e.second));
              tm.dn_ev.push_back(e);
            }
            ev = &tm.dn_ev[tm.dn_used++];
            KDMG_HIP(hipEventRecord(ev->first, c_.st));
          }
          dense_apply(h_.dinv, x, b, L.part.as<c64>(), nrhs_, parent, L.ks.k.its, L.ks.k.calls, L.ks.k.tot, c_.st,
                      worked);
          if (ev) KDMG_HIP(hipEventRecord(ev->second, c_.st));
        } else {
          throw Error(KDMG_EINVAL, "exact coarsest solve: the coarsest level runs in FP64");
        }
      } else if (l == h_.nlevels - 1) {
        if constexpr (sizeof(T) == 8) {
          cgne_fused(c_, h_.L[l], L, nrhs_, b, x, r, L.v<T>(L.p), P.coarse_tol, P.coarse_maxit, parent,
                     poll_, &h_.timer, h_.use_graphs);
        } else {
          auto opd = [&](Cx<T>* o, const Cx<T>* i, const int* a) { op<T>(l, o, i, nullptr, a, true); };
          auto opn = [&](Cx<T>* o, const Cx<T>* i, const int* a) { op<T>(l, o, i, nullptr, a, false); };
          cgne_solve<T>(c_, nrhs_, n, b, x, r, L.v<T>(L.p), L.v<T>(L.q), P.coarse_tol, P.coarse_maxit,
                        L.ks.k, parent, opn, opd, poll_);
        }
      } else {
        const KrylovState& ks = L.ks.k;
        // below this level only the exact coarsest product: no host decision,
        // so the K-cycle's halves replay as captured graphs
        const bool graphed = h_.use_graphs && P.coarse_solver == 1 && l + 1 == h_.nlevels - 1;
        auto prec = [&](Cx<T>* z, const Cx<T>* rr, const int* a) {
          if (graphed) kcycle_graphed<T>(l, z, rr, a);
          else kcycle<T>(l, z, rr, a);
        };
        // graphed: the host first reads the convergence flags after as many
        // iterations as the last call took, so a call that repeats its
        // count runs from start to finish without a host round trip
        int mx = 0;
        gcr_solve<T>(c_, nrhs_, n, b, x, r, L.v<T>(L.Z), L.v<T>(L.W), P.inter_restart, P.inter_maxit,
                     P.inter_tol, nullptr, ks, parent, opf, prec, false, 0,
                     graphed ? std::max(1, L.gcr_last) : 0, graphed ? &mx : nullptr);
        if (graphed) L.gcr_last = mx;
      }
    });
  }

  // outer FGCR on the fine Schur system, FP64
  int outer(double tol) {
    const kdmg_mg_params& P = h_.params;
    const kdmg_lattice& lat = *h_.lat;
    LevelWS& L0 = ws_.lv[0];
    const long n = L0.n;
    auto op64 = [&](c64* o, const c64* i, const c64* res, const int* a) {
      if (h_.fine_full) {
        const Fine2<double> F = fine2<double>(lat, h_.mass);
        if (h_.naive)
          fine2_D<double, double>(o, i, res, F, a, nrhs_, c_.st);
        else
          fine2_A<double, double>(o, i, res, ws_.tfull.as<c64>(), F, a, nrhs_, c_.st);
      } else if (lat.nd == 4)
        schur_apply4<double, double, double>(o, i, res, ws_.tfull.as<c64>(), ws_.wfull.as<c64>(), fine4_64(), a,
                                             nrhs_, c_.st);
      else
        schur_apply<double, double>(o, i, res, ws_.tfull.as<c64>(), ws_.wfull.as<c64>(), lat.links64.as<c64>(),
                                    lat.g, h_.mass, a, nrhs_, c_.st);
    };
    auto prec = [&](c64* z, const c64* r, const int* a) {
      if (L0.prec == Prec::F64) {
        kcycle<double>(0, z, r, a);
      } else {
        c32* r32 = ws_.xin32.as<c32>();
        c32* z32 = ws_.xout32.as<c32>();
        convert<float, double>(r32, r, n, nrhs_, a, c_.st);
        kcycle<float>(0, z32, r32, a);
        convert<double, float>(z, z32, n, nrhs_, a, c_.st);
      }
    };
    return gcr_solve<double>(c_, nrhs_, n, h_.fine_full ? ws_.bfull.as<c64>() : ws_.bt.as<c64>(),
                             ws_.ye.as<c64>(), ws_.re.as<c64>(),
                             ws_.Zo.as<c64>(), ws_.Wo.as<c64>(), P.outer_restart, P.outer_maxit, tol,
                             ws_.bnorm2.as<double>(), ws_.kout.k, nullptr, op64, prec,
                             trace_enabled(), P.outer_stall);
  }

  int poll_ = 8;

  // 4D fine operands at the hierarchy's mass
  Fine4<double, double> fine4_64() const {
    const kdmg_lattice& lat = *h_.lat;
    return Fine4<double, double>{lat.lk64.as<c64>(), lat.nb4.as<int>(), h_.binv64.as<c64>(), lat.g4, h_.mass};
  }
  Fine4<_Float16, float> fine4_mixed() const {
    const kdmg_lattice& lat = *h_.lat;
    return Fine4<_Float16, float>{lat.lk16.as<c16>(), lat.nb4.as<int>(), h_.binv32.as<c32>(), lat.g4, h_.mass};
  }

 private:
  kdmg_hierarchy& h_;
  SolveWS& ws_;
  const Ctx& c_;
  int nrhs_;
};

SolveWS* make_ws(kdmg_hierarchy& h, int nrhs, kdmg_prec prec, hipStream_t st) {
  auto ws = std::make_unique<SolveWS>();
  ws->nrhs = nrhs;
  ws->prec = prec;
  const kdmg_mg_params& P = h.params;
  const kdmg_lattice& lat = *h.lat;
  const long half = lat.half, f = 2 * half;
  const int maxr = std::max(P.outer_restart, P.inter_restart);
  ws->ctx.init(st, maxr * nrhs + nrhs + 8, nrhs);
  size_t tot = 0;
  auto A = [&](DevBuf& d, size_t bytes) { d.alloc(bytes); tot += bytes; };
  const size_t c64s = sizeof(c64) * nrhs;
  A(ws->bfull, c64s * f);
  A(ws->yfull, c64s * f);
  A(ws->xfull, c64s * f);
  A(ws->tfull, c64s * f);
  A(ws->wfull, c64s * f);
  const long n0 = h.fine_full ? f : half;  // the fine solve's space
  A(ws->bt, c64s * half);
  A(ws->ye, c64s * n0);
  A(ws->re, c64s * n0);
  A(ws->Zo, c64s * n0 * P.outer_restart);
  A(ws->Wo, c64s * n0 * P.outer_restart);
  A(ws->bnorm2, sizeof(double) * nrhs);
  A(ws->rnorm2, sizeof(double) * nrhs);
  ws->kout.init(nrhs, P.outer_restart);
  ws->lv.resize(h.nlevels);
  for (int l = 0; l < h.nlevels; ++l) {
    LevelWS& L = ws->lv[l];
    const bool coarsest = l == h.nlevels - 1;
    L.prec = (prec == KDMG_MIXED && !coarsest) ? Prec::F32 : Prec::F64;
    L.esz = L.prec == Prec::F64 ? sizeof(c64) : sizeof(c32);
    L.n = l == 0 ? n0 : h.L[l].n();
    const size_t v = L.esz * nrhs * L.n;
    if (!coarsest) {
      A(L.r1, v);
      A(L.x, v);
      A(L.r2, v);
      A(L.q, v);
      L.kmr.init(nrhs);
    }
    if (l == 0) {
      A(L.t, L.esz * nrhs * f);
      A(L.w, L.esz * nrhs * f);
    } else {
      A(L.b, v);
      A(L.xs, v);
      A(L.rs, v);
      L.ks.init(nrhs, coarsest ? 0 : P.inter_restart);
      if (coarsest && P.coarse_solver == 1) {
        A(L.part, sizeof(c64) * (size_t)dense_apply_splits(L.n, nrhs) * nrhs * L.n);
      } else if (coarsest) {
        A(L.p, v);
        A(L.q, v);
        A(L.cg_rr, sizeof(double) * 2 * nrhs);
        A(L.cg_target, sizeof(double) * nrhs);
        A(L.cg_act, sizeof(int) * 2 * nrhs);
        A(L.PA, sizeof(double) * (size_t)nrhs * h.L[l].nsites);
        A(L.PB, sizeof(double) * (size_t)nrhs * h.L[l].nsites);
        L.cg_graph = std::make_unique<ChunkGraph>();
        L.cg_poll = std::make_unique<AsyncPoll>();
        L.cg_poll->init(nrhs);
        if (P.coarse_tail > 0 && nrhs > P.coarse_tail) {
          const int nt = L.tail = P.coarse_tail;
          const size_t vt = sizeof(c64) * (size_t)nt * h.L[l].nsites * h.L[l].ndc;
          A(L.tx, vt);
          A(L.tr, vt);
          A(L.tp, vt);
          A(L.trr, sizeof(double) * 2 * nt);
          A(L.ttarget, sizeof(double) * nt);
          A(L.tact, sizeof(int) * 2 * nt);
          A(L.tints, sizeof(int) * 3 * nt);
          A(L.tPA, sizeof(double) * (size_t)nt * h.L[l].nsites);
          A(L.tPB, sizeof(double) * (size_t)nt * h.L[l].nsites);
          A(L.tidx, sizeof(int) * nt);
          L.cg_graph_t = std::make_unique<ChunkGraph>();
        }
      } else {
        A(L.Z, v * P.inter_restart);
        A(L.W, v * P.inter_restart);
      }
    }
  }
  if (prec == KDMG_MIXED) {
    A(ws->xin32, sizeof(c32) * nrhs * n0);
    A(ws->xout32, sizeof(c32) * nrhs * n0);
  }
  ws->bytes = tot;
  return ws.release();
}

size_t ws_bytes_estimate(const kdmg_hierarchy& h, int nrhs, kdmg_prec prec) {
  const kdmg_mg_params& P = h.params;
  const long half = h.lat->half, f = 2 * half, n0 = h.fine_full ? f : half;
  size_t b = sizeof(c64) * (size_t)nrhs * (5 * f + half + (2 + 2 * P.outer_restart) * n0);
  for (int l = 0; l < h.nlevels; ++l) {
    const bool coarsest = l == h.nlevels - 1;
    const size_t esz = (prec == KDMG_MIXED && !coarsest) ? 8 : 16;
    const long n = l == 0 ? n0 : h.L[l].n();
    const size_t v = esz * nrhs * n;
    if (!coarsest) b += 4 * v;
    if (l == 0) b += 2 * esz * nrhs * f;
    else if (coarsest && P.coarse_solver == 1) b += 3 * v + (size_t)dense_apply_splits(n, nrhs) * v;
    else b += 3 * v + (coarsest ? 2 * v : 2 * v * P.inter_restart);
  }
  if (prec == KDMG_MIXED) b += 2 * sizeof(c32) * nrhs * n0;
  return b;
}

}  // namespace

// Device bytes a hierarchy derived from `base` (kdmg_hierarchy_at_mass) holds
// once it has solved `nrhs` right-hand sides at `prec`.
size_t derived_footprint(const kdmg_hierarchy& base, int nrhs, kdmg_prec prec) {
  size_t b = base.gal_w.bytes + base.dinv.bytes() + ws_bytes_estimate(base, nrhs, prec);
  for (const auto& l : base.L) b += l.bytes();
  return b;
}

}  // namespace kdmg

extern "C" kdmg_status kdmg_hierarchy_footprint(const kdmg_hierarchy* h, int nrhs, size_t* bytes) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && bytes && nrhs >= 1, KDMG_EINVAL, "bad argument");
  *bytes = h->bytes() + std::max(ws_bytes_estimate(*h, nrhs, KDMG_MIXED), ws_bytes_estimate(*h, nrhs, KDMG_FP64));
  KDMG_API_END
}

extern "C" kdmg_status kdmg_solve(kdmg_hierarchy* h, const void* b, void* x, int nrhs, double tol,
                                  kdmg_prec prec, kdmg_solve_info* info, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && b && x && b != x, KDMG_EINVAL, "kdmg_solve: bad pointers");
  KDMG_CHECK(nrhs >= 1 && nrhs <= 1024, KDMG_EINVAL, "kdmg_solve: nrhs must be 1..1024");
  KDMG_CHECK(tol > 0.0 && tol < 1.0, KDMG_EINVAL, "kdmg_solve: tol must be in (0, 1)");
  KDMG_CHECK(prec == KDMG_FP64 || prec == KDMG_MIXED, KDMG_EINVAL, "kdmg_solve: bad precision");
  hipStream_t st = (hipStream_t)stream;
  if (h->ws && h->ws->nrhs == nrhs && h->ws->prec == prec && h->ws->ctx.c.st != st) {
    // same shape on another stream: keep the buffers, move the work
    // (kdmg_solve synchronises its stream before returning, so nothing of
    // the previous call is still in flight on the old stream)
    KDMG_CHECK(h->ws->busy.load() == 0, KDMG_EBUSY, "hierarchy busy");
    h->ws->ctx.c.st = st;
  }
  if (!h->ws || h->ws->nrhs != nrhs || h->ws->prec != prec) {
    KDMG_CHECK(!h->ws || h->ws->busy.load() == 0, KDMG_EBUSY, "hierarchy busy");
    if (h->ws) destroy_ws(h->ws);
    h->ws = nullptr;
    h->ws = make_ws(*h, nrhs, prec, st);
  }
  if (autotune_enabled()) {
    for (int l = 1; l < h->nlevels; ++l)
      autotune_level(h->L[l], nrhs, prec == KDMG_MIXED && l < h->nlevels - 1, st);
    if (h->params.coarse_solver == 0) {
      autotune_cgne(h->L[h->nlevels - 1], nrhs, st);
      const int tw = h->params.coarse_tail;
      if (tw > 0 && nrhs > tw) autotune_cgne(h->L[h->nlevels - 1], tw, st);
    }
  }
  SolveWS& ws = *h->ws;
  int expect = 0;
  KDMG_CHECK(ws.busy.compare_exchange_strong(expect, 1), KDMG_EBUSY, "hierarchy busy");
  struct Release { std::atomic<int>& b; ~Release() { b.store(0); } } rel{ws.busy};
  const auto t0 = std::chrono::steady_clock::now();
  const kdmg_lattice& lat = *h->lat;
  const Geo2& g = lat.g;
  const long half = lat.half, f = 2 * half, V = lat.ndof;
  const Ctx& c = ws.ctx.c;
  const c64* L64 = lat.links64.as<c64>();
  const bool d4 = lat.nd == 4;
  Runner run(*h, ws);
  h->timer.dn_used = 0;
  // reset statistics
  KDMG_HIP(hipMemsetAsync(ws.kout.ints.p, 0, ws.kout.ints.bytes, st));
  for (auto& L : ws.lv)
    if (L.ks.ints.p) KDMG_HIP(hipMemsetAsync(L.ks.ints.p, 0, L.ks.ints.bytes, st));
  // b -> block layout, ||b||^2
  launch_permute<double, double>(ws.bfull.as<c64>(), f, (const c64*)b, V, lat.perm_full.as<int>(), V, 1,
                                 nrhs, st);
  launch_map_reduce<1>(OpResidNorm{ws.bfull.as<c64>(), f, f, ws.bnorm2.as<double>()}, f, nrhs, 1, c.rs, st);
  // b~_e = b_e - A_eo b_o = b_e - C_eo B_o^-1 b_o  (the full-lattice solve takes b as it is)
  if (h->fine_full) {
  } else if (d4) {
    const Fine4<double, double> F = run.fine4_64();
    launch4_binv<double, double>(ws.tfull.as<c64>(), f, ws.bfull.as<c64>(), f, nullptr, 0, F.Bv, F.g, 1, 1, 0,
                                 nullptr, nrhs, st);
    launch4_hop<double, double>(ws.bt.as<c64>(), half, ws.tfull.as<c64>(), f, ws.bfull.as<c64>(), f, nullptr, 0,
                                0.0, -1.0, F.lk, F.nb4, F.g, 0, 1, F.m, 0, 0, nullptr, nrhs, st);
  } else {
    launch_binv<double, double, double>(ws.tfull.as<c64>(), f, nullptr, 0, ws.bfull.as<c64>(), f, nullptr, 0,
                                        L64, g, 1, 1, h->mass, 0, nullptr, nrhs, st);
    launch_hop<double, double, double>(ws.bt.as<c64>(), half, ws.tfull.as<c64>(), f, ws.bfull.as<c64>(), f,
                                       nullptr, 0, 0.0, -1.0, L64, g, 0, 1, h->mass, 0, 0, nullptr, nrhs, st);
  }
  const int its = run.outer(tol);
  if (h->fine_full) {
    // x = y (D itself) or x = B^-1 y = B~^-1 y / s
    const Fine2<double> F = fine2<double>(lat, h->mass);
    if (h->naive) {
      launch_map(OpStridedCopy{ws.xfull.as<c64>(), f, ws.ye.as<c64>(), f, f}, f, nrhs, st);
    } else {
      launch_binv<double, double, double>(ws.xfull.as<c64>(), f, nullptr, 0, ws.ye.as<c64>(), f, nullptr, 0, L64, g,
                                          0, 2, F.me, 0, nullptr, nrhs, st);
      if (F.s != 1.0)
        launch_map(OpAxpby<double>{ws.xfull.as<c64>(), ws.xfull.as<c64>(), nullptr, f, 1.0 / F.s, 0.0, nullptr}, f,
                   nrhs, st);
    }
  } else {
  // y_o = b_o - C_oe B_e^-1 y_e ; x = B^-1 y
  launch_map(OpStridedCopy{ws.yfull.as<c64>(), f, ws.ye.as<c64>(), half, half}, half, nrhs, st);
  if (d4) {
    const Fine4<double, double> F = run.fine4_64();
    launch4_binv<double, double>(ws.tfull.as<c64>(), f, ws.ye.as<c64>(), half, nullptr, 0, F.Bv, F.g, 0, 1, 0,
                                 nullptr, nrhs, st);
    launch4_hop<double, double>(ws.yfull.as<c64>(), f, ws.tfull.as<c64>(), f, ws.bfull.as<c64>(), f, nullptr, 0,
                                0.0, -1.0, F.lk, F.nb4, F.g, 1, 1, F.m, 0, 0, nullptr, nrhs, st);
    launch4_binv<double, double>(ws.xfull.as<c64>(), f, ws.yfull.as<c64>(), f, nullptr, 0, F.Bv, F.g, 0, 2, 0,
                                 nullptr, nrhs, st);
  } else {
    launch_binv<double, double, double>(ws.tfull.as<c64>(), f, nullptr, 0, ws.ye.as<c64>(), half, nullptr, 0,
                                        L64, g, 0, 1, h->mass, 0, nullptr, nrhs, st);
    launch_hop<double, double, double>(ws.yfull.as<c64>(), f, ws.tfull.as<c64>(), f, ws.bfull.as<c64>(), f,
                                       nullptr, 0, 0.0, -1.0, L64, g, 1, 1, h->mass, 0, 0, nullptr, nrhs, st);
    launch_binv<double, double, double>(ws.xfull.as<c64>(), f, nullptr, 0, ws.yfull.as<c64>(), f, nullptr, 0,
                                        L64, g, 0, 2, h->mass, 0, nullptr, nrhs, st);
  }
  }
  launch_permute<double, double>((c64*)x, V, ws.xfull.as<c64>(), f, lat.perm_full.as<int>(), V, 0, nrhs, st);
  // true residual ||b - D x|| in FP64
  if (h->fine_full) {
    fine2_D<double, double>(ws.tfull.as<c64>(), ws.xfull.as<c64>(), ws.bfull.as<c64>(),
                            fine2<double>(lat, h->mass), nullptr, nrhs, st);
  } else if (d4) {
    const Fine4<double, double> F = run.fine4_64();
    launch4_hop<double, double>(ws.tfull.as<c64>(), f, ws.xfull.as<c64>(), f, ws.bfull.as<c64>(), f, nullptr, 0,
                                0.0, -1.0, F.lk, F.nb4, F.g, 0, 2, F.m, 2, 0, nullptr, nrhs, st);
  } else {
    launch_dslash_blk<double, double, double>(ws.tfull.as<c64>(), f, ws.xfull.as<c64>(), f, ws.bfull.as<c64>(),
                                              f, L64, g, h->mass, nullptr, nrhs, st);
  }
  launch_map_reduce<1>(OpResidNorm{ws.tfull.as<c64>(), f, f, ws.rnorm2.as<double>()}, f, nrhs, 1, c.rs, st);
  std::vector<double> bn(nrhs), rn(nrhs);
  std::vector<int> kints(4 * nrhs);
  KDMG_HIP(hipMemcpyAsync(bn.data(), ws.bnorm2.p, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  KDMG_HIP(hipMemcpyAsync(rn.data(), ws.rnorm2.p, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  KDMG_HIP(hipMemcpyAsync(kints.data(), ws.kout.ints.p, sizeof(int) * 4 * nrhs, hipMemcpyDeviceToHost, st));
  std::vector<std::vector<int>> lints(h->nlevels);
  for (int l = 1; l < h->nlevels; ++l) {
    lints[l].resize(4 * nrhs);
    KDMG_HIP(hipMemcpyAsync(lints[l].data(), ws.lv[l].ks.ints.p, sizeof(int) * 4 * nrhs,
                            hipMemcpyDeviceToHost, st));
  }
  KDMG_HIP(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  {  // exact coarsest solve: kernel time of the products recorded in this solve
    auto& tm = h->timer;
    std::vector<int> worked(tm.dn_used);
    if (tm.dn_used)
      KDMG_HIP(hipMemcpy(worked.data(), tm.dn_work.p, sizeof(int) * tm.dn_used, hipMemcpyDeviceToHost));
    for (size_t e = 0; e < tm.dn_used; ++e) {
      if (!worked[e]) continue;  // every rhs had converged: the launch returned at once
      float ms = 0.f;
      KDMG_HIP(hipEventElapsedTime(&ms, tm.dn_ev[e].first, tm.dn_ev[e].second));
      tm.ms += ms;
      tm.launches += 1;
    }
    tm.dn_used = 0;
  }
  bool all = true;
  const int per_it = 2 * h->params.mr_its + 2;
  for (int r = 0; r < nrhs; ++r) {
    const double rel = bn[r] > 0 ? std::sqrt(rn[r] / bn[r]) : 0.0;
    const bool conv = rel <= tol * (1.0 + 1e-6) || bn[r] == 0.0;
    all = all && conv;
    if (info) {
      kdmg_solve_info& I = info[r];
      std::memset(&I, 0, sizeof(I));
      I.converged = conv ? 1 : 0;
      I.outer_its = kints[nrhs + r];
      I.fine_applies = I.outer_its * per_it + I.outer_its / h->params.outer_restart;
      for (int l = 1; l < h->nlevels && l <= 3; ++l) {
        const int calls = lints[l][2 * nrhs + r], tot = lints[l][3 * nrhs + r];
        I.level_avg_its[l - 1] = calls ? (double)tot / calls : 0.0;
      }
      I.true_rel_resid = rel;
      I.seconds = secs;
    }
  }
  (void)its;
  if (!all) throw Error(KDMG_ENOCONV, "kdmg_solve: some right-hand sides did not converge");
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_kernel_timing(kdmg_hierarchy* h, int enable, double* ms,
                                                    long long* launches) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && enable >= -1 && enable <= 1, KDMG_EINVAL, "kdmg_hierarchy_kernel_timing: bad argument");
  auto& t = h->timer;
  if (enable == 1) {
    if (!t.e0) KDMG_HIP(hipEventCreate(&t.e0));
    if (!t.e1) KDMG_HIP(hipEventCreate(&t.e1));
    t.ms = 0.0;
    t.launches = 0;
    t.on = true;
  } else if (enable == 0) {
    t.on = false;
  }
  if (ms) *ms = t.ms;
  if (launches) *launches = t.launches;
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_graphs(kdmg_hierarchy* h, int enable, long long* replays) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && enable >= -1 && enable <= 1, KDMG_EINVAL, "kdmg_hierarchy_graphs: bad argument");
  if (enable >= 0) h->use_graphs = enable != 0;
  if (replays) *replays = h->timer.graph_replays;
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_counters(kdmg_hierarchy* h, long long* graph_replays,
                                               long long* tail_entries) {
  KDMG_API_BEGIN
  KDMG_CHECK(h, KDMG_EINVAL, "kdmg_hierarchy_counters: null hierarchy");
  if (graph_replays) *graph_replays = h->timer.graph_replays;
  if (tail_entries) *tail_entries = h->timer.tail_entries;
  KDMG_API_END
}
