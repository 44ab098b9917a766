// Host drivers of the batched Krylov methods (Sec. 4, Table 1).  Operators are
// callables  op(out, in, resid, act)  computing out = op(in), or
// out = resid - op(in) when `resid` is non-null, for the rhs whose flag in
// `act` is set.
#pragma once
#include <cstdlib>
#include <vector>

#include "krylov.h"

namespace kdmg {

// KDMG_TRACE=1 prints the outer solver's per-rhs relative residual after every
// iteration (diagnostics; one extra device-to-host copy per iteration).
inline bool trace_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("KDMG_TRACE");
    return e && e[0] == '1';
  }();
  return on;
}

inline void trace_residuals(const Ctx& c, const KrylovState& k, int nrhs, int its, double tol) {
  std::vector<double> sc((size_t)nrhs * S_COUNT);
  KDMG_HIP(hipMemcpyAsync(sc.data(), k.sc, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, c.st));
  KDMG_HIP(hipStreamSynchronize(c.st));
  std::fprintf(stderr, "[kdmg] it %3d rel.res:", its);
  for (int r = 0; r < nrhs; ++r)
    std::fprintf(stderr, " %.2e", tol * std::sqrt(sc[(size_t)r * S_COUNT + S_RR] /
                                                  sc[(size_t)r * S_COUNT + S_TARGET]));
  std::fprintf(stderr, "\n");
}

// Device allocations for one Krylov state of `nrhs` right-hand sides.
struct KrylovAlloc {
  DevBuf sc, ints, rec;
  KrylovState k;
  // gcr_restart > 0: also the GCR cycle records for that restart length
  void init(int nrhs, int gcr_restart = 0) {
    sc.alloc(sizeof(double) * S_COUNT * nrhs);
    ints.alloc(sizeof(int) * 7 * nrhs);
    KDMG_HIP(hipMemset(sc.p, 0, sc.bytes));
    KDMG_HIP(hipMemset(ints.p, 0, ints.bytes));
    k.sc = sc.as<double>();
    k.act = ints.as<int>();
    k.its = k.act + nrhs;
    k.calls = k.its + nrhs;
    k.tot = k.calls + nrhs;
    k.m = k.tot + nrhs;
    k.re = k.m + nrhs;
    k.xu = k.re + nrhs;
    if (gcr_restart > 0) {
      rec.alloc(sizeof(double) * gcr_record_doubles(gcr_restart) * nrhs);
      KDMG_HIP(hipMemset(rec.p, 0, rec.bytes));
      k.R = gcr_restart;
      k.rec = rec.as<double>();
    }
  }
  // a state sharing another's flags (smoothers run under their caller's mask)
  KrylovState under(const int* act) const {
    KrylovState s = k;
    s.act = const_cast<int*>(act);
    return s;
  }
};

struct CtxAlloc {
  DevBuf partials;
  int* h_poll = nullptr;
  Ctx c;
  void init(hipStream_t st, int slots, int nrhs_max) {
    partials.alloc(sizeof(double) * (size_t)slots * 3 * RED_MAX_BLOCKS);
    {
      std::lock_guard<std::mutex> g(hip_mem_mutex());
      KDMG_HIP(hipHostMalloc((void**)&h_poll, sizeof(int) * (2 * nrhs_max + 8), hipHostMallocDefault));
    }
    c.st = st;
    c.rs.partials = partials.as<double>();
    c.rs.slots = slots;
    c.h_poll = h_poll;
  }
  ~CtxAlloc() {
    if (h_poll) {
      std::lock_guard<std::mutex> g(hip_mem_mutex());
      (void)hipHostFree(h_poll);
    }
  }
};

inline void start_solve(const Ctx& c, const KrylovState& k, const int* parent, int nrhs) {
  launch_map(OpStart{k, parent}, 1, nrhs, c.st);
}

// CG on a Hermitian positive operator (null-vector relaxation, the even/odd
// comparison solver).  Stops a rhs when ||r||^2 <= tol^2 (ext ? ext[r] : ||b||^2).
template <class T, class NormalF>
int cg_solve(const Ctx& c, int nrhs, long n, const Cx<T>* b, Cx<T>* x, Cx<T>* r, Cx<T>* p, Cx<T>* q,
             double tol, int maxit, const KrylovState& k, NormalF normal, int poll, const double* ext = nullptr) {
  start_solve(c, k, nullptr, nrhs);
  launch_map_reduce<1>(OpInit<T>{x, r, p, b, n, k, tol * tol, ext}, n, nrhs, 1, c.rs, c.st);
  int it = 0;
  for (; it < maxit; ++it) {
    normal(q, p, k.act);
    launch_map_reduce<1>(OpCGpq<T>{p, q, n, k}, n, nrhs, 1, c.rs, c.st);
    launch_map_reduce<1>(OpCGupd<T>{x, r, p, q, n, k}, n, nrhs, 1, c.rs, c.st);
    launch_map(OpCGp<T>{p, r, n, k}, n, nrhs, c.st);
    if ((it + 1) % poll == 0 && !any_active(c, k.act, nrhs)) { ++it; break; }
  }
  return it;
}

// Global MR with zero start folded into x: x += sum omega a_k r_k (Sec. 4, Table 1).
template <class T, class OpF>
void mr_smooth(const Ctx& c, int nrhs, long n, Cx<T>* x, Cx<T>* r, Cx<T>* q, int its, double omega,
               const KrylovState& k, OpF op) {
  for (int it = 0; it < its; ++it) {
    op(q, r, (const Cx<T>*)nullptr, k.act);
    launch_map_reduce<3>(OpMRred<T>{q, r, n, k, omega}, n, nrhs, 1, c.rs, c.st);
    launch_map(OpMRupd<T>{x, r, q, n, k}, n, nrhs, c.st);
  }
}

// Flexible restarted GCR.  Each new direction w = op(M r) is orthogonalised
// against the cycle's normalised directions by classical Gram-Schmidt, with a
// second pass where the first one lost more than half the norm (OpOrtho).
// Only w is projected: the preconditioned vectors z = M r stay as computed,
// and x receives each cycle's correction at the cycle's end from the
// triangular record of the projections (k_gcr_backsolve, OpXUpdate).  This
// is the same iteration as projecting z alongside w and updating x every
// step, with a third of the vector traffic.
// Stops a rhs when ||r||^2 <= tol^2 * (ext ? ext[r] : ||b||^2), and with
// stall > 0 also when ||r|| has not halved over the last `stall` iterations.
// poll_from > 0: the host reads the active flags only from iteration
// poll_from on (and at restarts), so the first poll_from iterations run
// without a host round trip; iterations after every rhs has converged are
// no-ops on the device (every kernel skips inactive rhs, and the cycle's
// x update uses each rhs' own column count), so the result is the same as
// with a poll after every iteration.  *max_its_out then receives the largest
// per-rhs iteration count of the call (the count a poll after every
// iteration would have stopped at).
template <class T, class OpF, class PrecF>
int gcr_solve(const Ctx& c, int nrhs, long n, const Cx<T>* b, Cx<T>* x, Cx<T>* r, Cx<T>* Zb,
              Cx<T>* Wb, int restart, int maxit, double tol, const double* ext,
              const KrylovState& k, const int* parent, OpF op, PrecF prec, bool trace = false,
              int stall = 0, int poll_from = 0, int* max_its_out = nullptr) {
  start_solve(c, k, parent, nrhs);
  launch_map_reduce<1>(OpInit<T>{x, r, nullptr, b, n, k, tol * tol, ext}, n, nrhs, 1, c.rs, c.st);
  const long vs = (long)nrhs * n;
  KDMG_CHECK(k.R >= restart && k.rec, KDMG_EINVAL, "GCR: cycle record too small");
  int its = 0;
  // polls the active flags (and, in deferred-poll mode, the iteration counts)
  auto poll = [&]() {
    if (poll_from > 0 && max_its_out)
      KDMG_HIP(hipMemcpyAsync(c.h_poll + nrhs, k.its, sizeof(int) * nrhs, hipMemcpyDeviceToHost, c.st));
    const bool any = any_active(c, k.act, nrhs);
    if (poll_from > 0 && max_its_out) {
      int mx = 0;
      for (int i = 0; i < nrhs; ++i) mx = std::max(mx, c.h_poll[nrhs + i]);
      *max_its_out = mx;
    }
    return any;
  };
  if (poll_from == 0 && !poll()) return 0;
  int ncol = 0;  // columns of the current cycle
  auto end_cycle = [&]() {
    if (ncol == 0) return;
    hipLaunchKernelGGL(k_gcr_backsolve<T>, dim3(cdiv(nrhs, 64)), dim3(64), 0, c.st, k, nrhs);
    KDMG_LAUNCH_CHECK();
    launch_map(OpXUpdate<T>{x, Zb, vs, ncol, n, k}, n, nrhs, c.st);
    ncol = 0;
  };
  while (its < maxit) {
    for (int kk = 0; kk < restart && its < maxit; ++kk) {
      Cx<T>* z = Zb + kk * vs;
      Cx<T>* w = Wb + kk * vs;
      prec(z, r, k.act);
      op(w, z, (const Cx<T>*)nullptr, k.act);
      if (kk > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          launch_multidot<T>(Wb, vs, w, n, kk, nrhs, k, pass ? k.re : nullptr, c.rs, c.st);
          launch_map_reduce<3>(OpOrtho<T>{w, Wb, r, vs, kk, n, k, pass}, n, nrhs, 1, c.rs, c.st);
        }
      } else {
        launch_map_reduce<3>(OpGCRred<T>{w, r, n, k}, n, nrhs, 1, c.rs, c.st);
      }
      launch_map_reduce<1>(OpGCRstep<T>{r, w, n, k, stall, kk}, n, nrhs, 1, c.rs, c.st);
      ncol = kk + 1;
      ++its;
      if (trace) trace_residuals(c, k, nrhs, its, tol);
      if (its >= poll_from && !poll()) {
        end_cycle();
        return its;
      }
    }
    end_cycle();
    if (its >= maxit) break;
    op(r, x, b, k.act);  // r = b - op x (true residual at restart)
    launch_map_reduce<1>(OpResNorm<T>{r, n, k}, n, nrhs, 1, c.rs, c.st);
    if (!poll()) break;
  }
  if (poll_from > 0 && max_its_out) (void)poll();
  return its;
}

// CGNE on the coarsest level: CG on op op^dag y = b, x = op^dag y; stops a rhs
// when ||b - op x|| <= tol ||b||.
template <class T, class OpF, class OpDF>
int cgne_solve(const Ctx& c, int nrhs, long n, const Cx<T>* b, Cx<T>* x, Cx<T>* r, Cx<T>* p,
               Cx<T>* q, double tol, int maxit, const KrylovState& k, const int* parent, OpF op,
               OpDF opdag, int poll) {
  start_solve(c, k, parent, nrhs);
  launch_map_reduce<1>(OpInit<T>{x, r, nullptr, b, n, k, tol * tol, nullptr}, n, nrhs, 1, c.rs, c.st);
  opdag(p, r, k.act);
  launch_map_reduce<1>(OpAlphaFromNorm<T>{p, n, k}, n, nrhs, 1, c.rs, c.st);
  int it = 0;
  for (; it < maxit; ++it) {
    op(q, p, k.act);
    launch_map_reduce<1>(OpCGupd<T>{x, r, p, q, n, k}, n, nrhs, 1, c.rs, c.st);
    opdag(q, r, k.act);
    launch_map_reduce<1>(OpCGp<T>{p, q, n, k}, n, nrhs, 1, c.rs, c.st);
    if ((it + 1) % poll == 0 && !any_active(c, k.act, nrhs)) { ++it; break; }
  }
  return it;
}

}  // namespace kdmg
