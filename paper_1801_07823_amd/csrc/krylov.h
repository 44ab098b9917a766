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
  S_REF,         // ||r||^2 at the last stall checkpoint (GCR with a stall rule)
  S_H,           // GCR projections, then the cycle's solution coefficients:
                 // 2 * max_restart slots from here
  S_COUNT = S_H + 2 * 64
};

// Per-rhs GCR cycle record (restart length R): the upper triangular T with
// T[j][k] = projection of direction k on normalised direction j (j < k, both
// Gram-Schmidt passes summed) and T[k][k] = ||w_k|| after projection, then
// a[k] = alpha_k ||w_k||.  Complex entries, FP64.
__host__ __device__ constexpr long gcr_record_doubles(int R) { return 2L * ((long)R * R + R); }

struct KrylovState {
  double* sc = nullptr;   // [nrhs][S_COUNT]
  int* act = nullptr;     // [nrhs] active flags
  int* its = nullptr;     // [nrhs] iteration counters of the current call
  int* calls = nullptr;   // [nrhs] calls made while active (statistics)
  int* tot = nullptr;     // [nrhs] iterations summed over calls (statistics)
  // GCR only (R > 0): cycle records, columns recorded per rhs this cycle,
  // second-pass flags, and "x has an update pending" flags
  int R = 0;
  double* rec = nullptr;  // [nrhs][gcr_record_doubles(R)]
  int* m = nullptr;       // [nrhs]
  int* re = nullptr;      // [nrhs]
  int* xu = nullptr;      // [nrhs] columns of the pending x update (0: none)
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
      if (k.m) k.m[r] = 0;  // no GCR columns recorded yet
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
    S[S_REF] = s[0];
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

// The classical Gram-Schmidt projections h[r][j] = <W_j[r], w[r]>, j < nz, in
// two kernels.  k_multidot reads w once per batch of MDJ directions (the
// generic map-reduce re-read it for every direction and paid an atomic and a
// device-scope fence per workgroup) and writes per-workgroup partial sums;
// k_multidot_sum adds each (rhs, j)'s partials in workgroup order with a fixed
// tree, so the result is deterministic without atomics.
constexpr int MDJ = 8;

template <class T>
__global__ __launch_bounds__(256) void k_multidot(double* part, const Cx<T>* Wb, long vstride, const Cx<T>* w,
                                                  long n, int nz, int nrhs, const int* act, const int* act2) {
  const int r = blockIdx.y, j0 = blockIdx.z * MDJ;
  if (!act[r] || (act2 && !act2[r])) return;
  double acc[2 * MDJ];
#pragma unroll
  for (int q = 0; q < 2 * MDJ; ++q) acc[q] = 0.0;
  const Cx<T>* wr = w + (long)r * n;
  const Cx<T>* W0 = Wb + (long)j0 * vstride + (long)r * n;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const Cx<double> v = ld<double>(wr[i]);
#pragma unroll
    for (int q = 0; q < MDJ; ++q)
      if (j0 + q < nz) {
        const Cx<double> u = ld<double>(W0[(long)q * vstride + i]);
        acc[2 * q] += u.re * v.re + u.im * v.im;
        acc[2 * q + 1] += u.re * v.im - u.im * v.re;
      }
  }
  __shared__ double sh[2 * MDJ][RED_THREADS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 2 * MDJ; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sh[q][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2 * MDJ && j0 + (int)threadIdx.x / 2 < nz) {
    const int q = threadIdx.x, j = j0 + q / 2;
    double v = 0.0;
    for (int u = 0; u < RED_THREADS / 64; ++u) v += sh[q][u];
    part[(((long)j * nrhs + r) * 2 + (q & 1)) * RED_MAX_BLOCKS + blockIdx.x] = v;
  }
}

template <class T>
__global__ __launch_bounds__(64) void k_multidot_sum(const double* part, int nb, int nrhs, KrylovState k,
                                                     const int* act2) {
  const int j = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  if (!k.act[r] || (act2 && !act2[r])) return;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double* p = part + (((long)j * nrhs + r) * 2 + c) * RED_MAX_BLOCKS;
    double v = 0.0;
    for (int b = lane; b < nb; b += 64) v += p[b];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) k.sc[(long)r * S_COUNT + S_H + 2 * j + c] = v;
  }
}

template <class T>
void launch_multidot(const Cx<T>* Wb, long vstride, const Cx<T>* w, long n, int nz, int nrhs,
                     const KrylovState& k, const int* act2, const RedScratch& rs, hipStream_t st) {
  KDMG_CHECK(nz * nrhs <= rs.slots && 2 * nz <= S_COUNT - S_H, KDMG_EINVAL, "multi-dot: scratch too small");
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_multidot<T>), dim3(nb, nrhs, cdiv(nz, MDJ)), dim3(RED_THREADS), 0, st, rs.partials, Wb,
                     vstride, w, n, nz, nrhs, (const int*)k.act, act2);
  hipLaunchKernelGGL((k_multidot_sum<T>), dim3(nz, nrhs), dim3(64), 0, st, (const double*)rs.partials, nb, nrhs,
                     k, act2);
  KDMG_LAUNCH_CHECK();
}

// One classical Gram-Schmidt pass on w against the normalised directions
// W_0 .. W_{nj-1} with the projections h_j in S_H, fused with the reductions
// the GCR step needs from the result: ||w||^2 and <w, r> give ALPHA and INV
// (as OpGCRred).  The projections go into column nj of the cycle record.
// Pass 0 runs for every active rhs and flags a second pass where the norm
// collapsed: ||w'|| < ||w|| / sqrt(2) (the Daniel-Gragg-Kaufman-Stewart
// criterion), i.e. ||w'||^2 < ||h||^2 since ||w||^2 = ||w'||^2 + ||h||^2.
// Pass 1 runs only for the flagged rhs and adds its projections.
template <class T>
struct OpOrtho {
  Cx<T>* w; const Cx<T>* Wb; const Cx<T>* r; long vstride; int nj; long n; KrylovState k; int pass;
  __device__ bool active(int rr) const { return k.act[rr] != 0 && (pass == 0 || k.re[rr] != 0); }
  __device__ void elem(int rr, int, long i, Acc<3>& a) const {
    const double* S = k.sc + rr * S_COUNT;
    const long o = rr * n + i;
    Cx<T> wv = w[o];
    for (int j = 0; j < nj; ++j) {
      const Cx<T> h{(T)S[S_H + 2 * j], (T)S[S_H + 2 * j + 1]};
      wv = wv - h * Wb[j * vstride + o];
    }
    w[o] = wv;
    const Cx<double> u = ld<double>(wv), v = ld<double>(r[o]);
    a.v[0] += u.re * u.re + u.im * u.im;
    a.v[1] += u.re * v.re + u.im * v.im;
    a.v[2] += u.re * v.im - u.im * v.re;
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    double* T_ = k.rec + rr * gcr_record_doubles(k.R);
    double hh = 0.0;
    for (int j = 0; j < nj; ++j) {
      const double hr = S[S_H + 2 * j], hi = S[S_H + 2 * j + 1];
      double* t = T_ + 2 * ((long)j * k.R + nj);
      t[0] = pass == 0 ? hr : t[0] + hr;
      t[1] = pass == 0 ? hi : t[1] + hi;
      hh += hr * hr + hi * hi;
    }
    if (pass == 0) k.re[rr] = s[0] < hh ? 1 : 0;
    S[S_ALPHA] = s[1] / s[0];
    S[S_ALPHA_I] = s[2] / s[0];
    S[S_INV] = 1.0 / sqrt(s[0]);
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

// GCR step for column `col` of the cycle: r -= alpha w ; w *= inv ;
// ||r||^2 -> convergence.  The solution is not touched here: the step records
// T[col][col] = ||w|| and a[col] = alpha ||w||, and x receives the whole
// cycle's correction at its end (k_gcr_backsolve, OpXUpdate).
template <class T>
struct OpGCRstep {
  Cx<T>* r; Cx<T>* w; long n; KrylovState k; int stall; int col;
  __device__ bool active(int rr) const { return k.act[rr] != 0; }
  __device__ void elem(int rr, int, long i, Acc<1>& a) const {
    const double* S = k.sc + rr * S_COUNT;
    const Cx<T> al{(T)S[S_ALPHA], (T)S[S_ALPHA_I]};
    const T inv = (T)S[S_INV];
    const long o = rr * n + i;
    const Cx<T> wv = w[o];
    const Cx<T> rv = r[o] - al * wv;
    r[o] = rv;
    w[o] = inv * wv;
    a.v[0] += (double)norm2(ld<double>(rv));
  }
  __device__ void finish(int rr, int, const double* s) const {
    double* S = k.sc + rr * S_COUNT;
    double* T_ = k.rec + rr * gcr_record_doubles(k.R);
    const double g = 1.0 / S[S_INV];
    T_[2 * ((long)col * k.R + col)] = g;
    T_[2 * ((long)col * k.R + col) + 1] = 0.0;
    double* a = T_ + 2 * ((long)k.R * k.R + col);
    a[0] = S[S_ALPHA] * g;
    a[1] = S[S_ALPHA_I] * g;
    k.m[rr] = col + 1;
    k.its[rr] += 1;
    k.tot[rr] += 1;
    S[S_RR] = s[0];
    if (s[0] <= S[S_TARGET]) {
      k.act[rr] = 0;
    } else if (stall > 0 && k.its[rr] % stall == 0) {
      // stall rule: the norm must have halved since the last checkpoint
      if (s[0] > 0.25 * S[S_REF]) k.act[rr] = 0;
      else S[S_REF] = s[0];
    }
  }
};

// End of a GCR cycle, one thread per rhs: c = T^-1 a over the rhs' recorded
// columns (back substitution), written to S_H; hands the column count to the
// x update and clears it.  With the raw
// preconditioned vectors Z~ = Z T (Z the orthonormalised-direction images),
// the cycle's correction sum_k alpha_k ||w_k|| Z_k equals Z~ c.
template <class T>
__global__ __launch_bounds__(64) void k_gcr_backsolve(KrylovState k, int nrhs) {
  const int rr = blockIdx.x * 64 + threadIdx.x;
  if (rr >= nrhs) return;
  const int m = k.m[rr], R = k.R;
  const double* T_ = k.rec + rr * gcr_record_doubles(R);
  const double* a = T_ + 2L * R * R;
  double* c = k.sc + (long)rr * S_COUNT + S_H;
  for (int j = m - 1; j >= 0; --j) {
    double sr = a[2 * j], si = a[2 * j + 1];
    for (int l = j + 1; l < m; ++l) {
      const double tr = T_[2 * ((long)j * R + l)], ti = T_[2 * ((long)j * R + l) + 1];
      sr -= tr * c[2 * l] - ti * c[2 * l + 1];
      si -= tr * c[2 * l + 1] + ti * c[2 * l];
    }
    const double d = T_[2 * ((long)j * R + j)];
    c[2 * j] = sr / d;
    c[2 * j + 1] = si / d;
  }
  k.xu[rr] = m;
  k.m[rr] = 0;
}

// x += sum_j c_j Z~_j over the rhs' own columns, for every rhs with a
// pending update (also rhs that converged during the cycle).  Columns past a
// rhs' own count were not written for it in this call and are never read.
template <class T>
struct OpXUpdate {
  Cx<T>* x; const Cx<T>* Zb; long vstride; int nj; long n; KrylovState k;
  __device__ bool active(int rr) const { return k.xu[rr] != 0; }
  __device__ void elem(int rr, long i) const {
    const double* c = k.sc + rr * S_COUNT + S_H;
    const long o = rr * n + i;
    const int mj = min(nj, k.xu[rr]);
    Cx<T> xv = x[o];
    for (int j = 0; j < mj; ++j) xv = xv + Cx<T>{(T)c[2 * j], (T)c[2 * j + 1]} * Zb[j * vstride + o];
    x[o] = xv;
  }
};

}  // namespace kdmg
