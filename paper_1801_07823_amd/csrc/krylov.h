// Batched Krylov building blocks with device-resident scalars and per-rhs
// convergence masks: CG (null-vector relaxation), MR (smoother), flexible GCR
// (fine outer and intermediate solvers) and CGNE (coarsest solver), following
// Sec. 4 and Table 1 of the paper.
//
// Each rhs r owns an `active` flag; a rhs that meets its tolerance clears its
// flag inside a reduction epilogue and every later kernel skips it, so a rhs
// follows exactly the iteration it would follow alone.  The host only reads the
// flags (to stop the loop) every `poll` iterations.
#pragma once
#include <functional>

#include "internal.h"

namespace kdmg {

// device scalar slots per rhs (doubles)
enum ScalarSlot {
  S_RR = 0,      // ||r||^2 of the current iterate
  S_TARGET,      // (tol * ||b||)^2
  S_ALPHA,       // 2 slots (complex)
  S_ALPHA_I,
  S_BETA,
  S_INV,         // 1 / ||w||
  S_H,           // GCR projections: 2 * max_restart slots from here
  S_COUNT = S_H + 2 * 64
};

struct KrylovState {
  double* sc = nullptr;   // [nrhs][S_COUNT]
  int* act = nullptr;     // [nrhs] active flags
  int* its = nullptr;     // [nrhs] iteration counters of the current call
  int* calls = nullptr;   // [nrhs] calls made while active (statistics)
  int* tot = nullptr;     // [nrhs] iterations summed over calls (statistics)
};

struct Ctx {
  hipStream_t st = nullptr;
  RedScratch rs;
  int* h_poll = nullptr;  // pinned host buffer (>= max nrhs ints)
};

// Copies the active flags to the host; true if any rhs is still active.
inline bool any_active(const Ctx& c, const int* act, int nrhs) {
  KDMG_HIP(hipMemcpyAsync(c.h_poll, act, sizeof(int) * nrhs, hipMemcpyDeviceToHost, c.st));
  KDMG_HIP(hipStreamSynchronize(c.st));
  for (int r = 0; r < nrhs; ++r)
    if (c.h_poll[r]) return true;
  return false;
}

// ----------------------------------------------------------------- functors

// act[r] = parent[r]; its[r] = 0 ; (used to start a nested solve)
struct OpStart {
  KrylovState k; const int* parent;
  __device__ bool active(int) const { return true; }
  __device__ void elem(int r, long i) const {
    if (i == 0) {
      int a = parent ? parent[r] : 1;
      k.act[r] = a;
      k.its[r] = 0;
      if (a) k.calls[r] += 1;
    }
  }
};

// x = 0, r = b, [p = b]; ||b||^2 -> RR, TARGET = tol2 * (ext ? ext[r] : ||b||^2)
template <class T>
struct OpInit {
  Cx<T>* x; Cx<T>* r; Cx<T>* p; const Cx<T>* b; long n; KrylovState k; double tol2; const double* ext;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const {
    const long o = rr * n + i;
    Cx<T> v = b[o];
    x[o] = Cx<T>{0, 0};
    r[o] = v;
    if (p) p[o] = v;
    a.v[0] += (double)norm2(ld<double>(v));
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_RR] = s[0];
    S[S_TARGET] = tol2 * (ext ? ext[rr] : s[0]);
    if (!(s[0] > S[S_TARGET]) || s[0] == 0.0) k.act[rr] = 0;
  }
};

// ||r||^2 -> RR, convergence test against TARGET (after a restart recompute)
template <class T>
struct OpResNorm {
  const Cx<T>* r; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const { a.v[0] += (double)norm2(ld<double>(r[rr * n + i])); }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_RR] = s[0];
    if (s[0] <= S[S_TARGET]) k.act[rr] = 0;
  }
};

// CG: <p, q> -> ALPHA = RR / <p,q>
template <class T>
struct OpCGpq {
  const Cx<T>* p; const Cx<T>* q; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const {
    Cx<double> u = ld<double>(p[rr * n + i]), v = ld<double>(q[rr * n + i]);
    a.v[0] += u.re * v.re + u.im * v.im;
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_ALPHA] = S[S_RR] / s[0];
  }
};

// x += alpha p ; r -= alpha q ; ||r||^2 -> convergence, BETA = new/old, RR = new
template <class T>
struct OpCGupd {
  Cx<T>* x; Cx<T>* r; const Cx<T>* p; const Cx<T>* q; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const {
    const T al = (T)k.sc[rr * S_COUNT + S_ALPHA];
    const long o = rr * n + i;
    Cx<T> xv = x[o], rv = r[o];
    const Cx<T> pv = p[o], qv = q[o];
    xv = xv + al * pv;
    rv = rv - al * qv;
    x[o] = xv;
    r[o] = rv;
    a.v[0] += (double)norm2(ld<double>(rv));
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    k.its[rr] += 1;
    k.tot[rr] += 1;
    S[S_BETA] = s[0] / S[S_RR];
    S[S_RR] = s[0];
    if (s[0] <= S[S_TARGET]) k.act[rr] = 0;
  }
};

// p = src + beta p  [; ||p||^2 -> ALPHA = RR / ||p||^2 when `red`]
template <class T>
struct OpCGp {
  Cx<T>* p; const Cx<T>* src; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, long i) const {
    const T be = (T)k.sc[rr * S_COUNT + S_BETA];
    const long o = rr * n + i;
    p[o] = src[o] + be * p[o];
  }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const {
    const T be = (T)k.sc[rr * S_COUNT + S_BETA];
    const long o = rr * n + i;
    Cx<T> v = src[o] + be * p[o];
    p[o] = v;
    a.v[0] += (double)norm2(ld<double>(v));
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_ALPHA] = S[S_RR] / s[0];
  }
};

// ||p||^2 -> ALPHA = RR / ||p||^2
template <class T>
struct OpAlphaFromNorm {
  const Cx<T>* p; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const { a.v[0] += (double)norm2(ld<double>(p[rr * n + i])); }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_ALPHA] = S[S_RR] / s[0];
  }
};

// MR: <q, r>, ||q||^2 -> ALPHA = omega <q,r>/||q||^2
template <class T>
struct OpMRred {
  const Cx<T>* q; const Cx<T>* r; long n; KrylovState k; double omega;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<3>& a) const {
    Cx<double> u = ld<double>(q[rr * n + i]), v = ld<double>(r[rr * n + i]);
    a.v[0] += u.re * v.re + u.im * v.im;
    a.v[1] += u.re * v.im - u.im * v.re;
    a.v[2] += u.re * u.re + u.im * u.im;
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    const double d = s[2] > 0.0 ? omega / s[2] : 0.0;
    S[S_ALPHA] = d * s[0];
    S[S_ALPHA_I] = d * s[1];
  }
};

// x += a r ; r -= a q
template <class T>
struct OpMRupd {
  Cx<T>* x; Cx<T>* r; const Cx<T>* q; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, long i) const {
    const double* S = k.sc + rr * S_COUNT;
    const Cx<T> al{(T)S[S_ALPHA], (T)S[S_ALPHA_I]};
    const long o = rr * n + i;
    const Cx<T> rv = r[o];
    x[o] = x[o] + al * rv;
    r[o] = rv - al * q[o];
  }
};

// GCR: h_j = <w_j, w>  (z-batch over j)
template <class T>
struct OpMultiDot {
  const Cx<T>* Wb; long vstride; const Cx<T>* w; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int j, long i, Acc<2>& a) const {
    Cx<double> u = ld<double>(Wb[j * vstride + rr * n + i]), v = ld<double>(w[rr * n + i]);
    a.v[0] += u.re * v.re + u.im * v.im;
    a.v[1] += u.re * v.im - u.im * v.re;
  }
  __device__ void finish(int rr, int j, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_H + 2 * j] = s[0];
    S[S_H + 2 * j + 1] = s[1];
  }
};

// w -= sum_j h_j w_j ; z -= sum_j h_j z_j
template <class T>
struct OpMultiAxpy {
  Cx<T>* w; Cx<T>* z; const Cx<T>* Wb; const Cx<T>* Zb; long vstride; int nj; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, long i) const {
    const double* S = k.sc + rr * S_COUNT;
    const long o = rr * n + i;
    Cx<T> wv = w[o], zv = z[o];
    for (int j = 0; j < nj; ++j) {
      const Cx<T> h{(T)S[S_H + 2 * j], (T)S[S_H + 2 * j + 1]};
      wv = wv - h * Wb[j * vstride + o];
      zv = zv - h * Zb[j * vstride + o];
    }
    w[o] = wv;
    z[o] = zv;
  }
};

// GCR: ||w||^2, <w, r> -> ALPHA = <w,r>/||w||^2, INV = 1/||w||
template <class T>
struct OpGCRred {
  const Cx<T>* w; const Cx<T>* r; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<3>& a) const {
    Cx<double> u = ld<double>(w[rr * n + i]), v = ld<double>(r[rr * n + i]);
    a.v[0] += u.re * u.re + u.im * u.im;
    a.v[1] += u.re * v.re + u.im * v.im;
    a.v[2] += u.re * v.im - u.im * v.re;
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    S[S_ALPHA] = s[1] / s[0];
    S[S_ALPHA_I] = s[2] / s[0];
    S[S_INV] = 1.0 / sqrt(s[0]);
  }
};

// x += alpha z ; r -= alpha w ; w *= inv ; z *= inv ; ||r||^2 -> convergence
template <class T>
struct OpGCRupd {
  Cx<T>* x; Cx<T>* r; Cx<T>* w; Cx<T>* z; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const {
    const double* S = k.sc + rr * S_COUNT;
    const Cx<T> al{(T)S[S_ALPHA], (T)S[S_ALPHA_I]};
    const T inv = (T)S[S_INV];
    const long o = rr * n + i;
    const Cx<T> zv = z[o], wv = w[o];
    x[o] = x[o] + al * zv;
    const Cx<T> rv = r[o] - al * wv;
    r[o] = rv;
    w[o] = inv * wv;
    z[o] = inv * zv;
    a.v[0] += (double)norm2(ld<double>(rv));
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    k.its[rr] += 1;
    k.tot[rr] += 1;
    S[S_RR] = s[0];
    if (s[0] <= S[S_TARGET]) k.act[rr] = 0;
  }
};

}  // namespace kdmg
