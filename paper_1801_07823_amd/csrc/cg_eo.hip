// Conjugate gradient on the site even/odd (red/black) Schur system of the 2D
// staggered operator: the solver the paper compares KD-MG against (Sec. 1 and
// Sec. 2 state the system; Sec. 4, Figs. "resid" and "iterworst", compares
// iteration counts).
//
// With D = m + H (H the hopping term, anti-Hermitian, connecting opposite
// site parities only), D x = b splits into
//   (m^2 - H_eo H_oe) x_e = m b_e - H_eo b_o,   x_o = (b_o - H_oe x_e) / m,
// and m^2 - H_eo H_oe = m^2 + H_oe^dag H_oe is Hermitian positive definite.
// The even residual r_e of that system gives the full residual exactly,
// ||b - D x|| = ||r_e|| / m, so a rhs stops when ||r_e|| <= tol m ||b||.
// Over many iterations the recursively updated CG residual drifts from the
// true one, so after a CG pass converges the true even residual is
// recomputed, and rhs still above the target solve for a correction with a
// further pass (from zero, on the residual system).
//
// Vectors live in a site-parity compact layout: the site of natural index n
// (x0 fastest) and parity q = sum_mu x_mu & 1 has index n >> 1 within its
// parity half (every extent even), its colours contiguous.  Batched over rhs
// with the library's CG (device scalars, per-rhs stopping), FP64
// throughout.  2D U(1) and 4D SU(3).
#include <algorithm>
#include <vector>

#include "internal.h"
#include "algos.h"
#include "api_guard.h"

namespace kdmg {
namespace {

// out[r][i] = c (H in)[r][i] + a add[r][i] on the sites of parity po; `in`
// holds parity 1 - po.  Links in natural order per direction (U_0 then U_1),
// with the staggered phases, the 1/2 and the time boundary sign folded in.
// A tile of RB rhs per thread, loads without branches (rhs outside the tile
// or inactive read row r0 and are not stored).
template <int RB>
__global__ __launch_bounds__(256) void k_hop_eo(c64* out, const c64* in, const c64* add, const c64* __restrict__ Ux,
                                                const c64* __restrict__ Ut, int Lx, int Lt, int po, long half,
                                                double c, double a, const int* act, int nrhs) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * RB;
  if (i >= half) return;
  const int hx = Lx >> 1;
  const int x1 = (int)(i / hx), k = (int)(i - (long)x1 * hx);
  const int x0 = 2 * k + ((po + x1) & 1);
  const int x0p = x0 + 1 == Lx ? 0 : x0 + 1, x0m = x0 == 0 ? Lx - 1 : x0 - 1;
  const int x1p = x1 + 1 == Lt ? 0 : x1 + 1, x1m = x1 == 0 ? Lt - 1 : x1 - 1;
  const long x = (long)x1 * Lx + x0;
  const long jxp = ((long)x1 * Lx + x0p) >> 1, jxm = ((long)x1 * Lx + x0m) >> 1;
  const long jtp = ((long)x1p * Lx + x0) >> 1, jtm = ((long)x1m * Lx + x0) >> 1;
  const c64 ux = Ux[x], uxm = Ux[(long)x1 * Lx + x0m], ut = Ut[x], utm = Ut[(long)x1m * Lx + x0];
  bool on[RB];
  long row[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    on[b] = r0 + b < nrhs && is_active(act, r0 + b);
    row[b] = on[b] ? r0 + b : r0;
  }
  c64 v1[RB], v2[RB], v3[RB], v4[RB], w[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const c64* v = in + row[b] * half;
    v1[b] = v[jxp];
    v2[b] = v[jxm];
    v3[b] = v[jtp];
    v4[b] = v[jtm];
    w[b] = add ? add[row[b] * half + i] : c64{0, 0};
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    c64 h = ux * v1[b];
    h -= cmul_conj(uxm, v2[b]);
    h += ut * v3[b];
    h -= cmul_conj(utm, v4[b]);
    if (on[b]) out[(long)(r0 + b) * half + i] = c * h + a * w[b];
  }
}

// 4D SU(3): out[r][j] = c (H in)[r][j] + a add[r][j] on the sites of parity
// po (j = n >> 1, three colours each); `in` holds parity 1 - po.  nl: the
// folded links (1/2 eta_mu(x) bc U_mu(x)) in natural order [mu][V][3][3].
// One thread per site, a tile of RB rhs sharing the eight link loads.
template <int RB>
__global__ __launch_bounds__(256) void k_hop_eo4(c64* out, const c64* in, const c64* add, const c64* __restrict__ nl,
                                                 int4 L, int po, long Vh, double c, double a, const int* act,
                                                 int nrhs) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * RB;
  if (j >= Vh) return;
  const long V = 2 * Vh, half = 3 * Vh;
  const int hx = L.x >> 1;
  long rest = j / hx;
  const int k = (int)(j - rest * hx);
  const int x1 = (int)(rest % L.y);
  rest /= L.y;
  const int x2 = (int)(rest % L.z), x3 = (int)(rest / L.z);
  const int x0 = 2 * k + ((po + x1 + x2 + x3) & 1);
  const int xs[4] = {x0, x1, x2, x3}, Ls[4] = {L.x, L.y, L.z, L.w};
  const long str[4] = {1, L.x, (long)L.x * L.y, (long)L.x * L.y * L.z};
  const long n = x0 + str[1] * x1 + str[2] * x2 + str[3] * x3;
  bool on[RB];
  long row[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    on[b] = r0 + b < nrhs && is_active(act, r0 + b);
    row[b] = on[b] ? r0 + b : r0;
  }
  c64 h[RB][3];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int e = 0; e < 3; ++e) h[b][e] = c64{0, 0};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const long nf = n + (xs[mu] + 1 == Ls[mu] ? -(long)(Ls[mu] - 1) * str[mu] : str[mu]);
    const long nb = n + (xs[mu] == 0 ? (long)(Ls[mu] - 1) * str[mu] : -str[mu]);
    const c64* Uf = nl + ((long)mu * V + n) * 9;
    const c64* Ub = nl + ((long)mu * V + nb) * 9;
    c64 uf[9], ub[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      uf[e] = Uf[e];
      ub[e] = Ub[e];
    }
    const long jf = (nf >> 1) * 3, jb = (nb >> 1) * 3;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const c64* v = in + row[b] * half;
      const c64 f0 = v[jf], f1 = v[jf + 1], f2 = v[jf + 2];
      const c64 g0 = v[jb], g1 = v[jb + 1], g2 = v[jb + 2];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        // + U(x) psi(x + mu) - U(x - mu)^dag psi(x - mu)
        cfma(h[b][e], uf[3 * e + 0], f0);
        cfma(h[b][e], uf[3 * e + 1], f1);
        cfma(h[b][e], uf[3 * e + 2], f2);
        h[b][e] -= cmul_conj(ub[0 + e], g0);
        h[b][e] -= cmul_conj(ub[3 + e], g1);
        h[b][e] -= cmul_conj(ub[6 + e], g2);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (!on[b]) continue;
    const long o = (long)(r0 + b) * half + 3 * j;
#pragma unroll
    for (int e = 0; e < 3; ++e) out[o + e] = c * h[b][e] + a * (add ? add[o + e] : c64{0, 0});
  }
}

// natural-order folded links of a 4D lattice from its block layout
// ([site][mu][9] at the block-site index of perm_full)
__global__ __launch_bounds__(256) void k_links_nat4(c64* nl, const c64* lk, const int* perm, long V) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  const long ib = perm[3 * n] / 3;
  for (int mu = 0; mu < 4; ++mu)
    for (int e = 0; e < 9; ++e) nl[((long)mu * V + n) * 9 + e] = lk[(ib * 4 + mu) * 9 + e];
}

// 4D natural order <-> parity halves (three colours per site)
__global__ __launch_bounds__(256) void k_eo_split4(c64* e, c64* o, const c64* v, int4 L, long V) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long r = blockIdx.y;
  if (n >= V) return;
  long rest = n;
  int q = 0;
  const int Ls[4] = {L.x, L.y, L.z, L.w};
  for (int mu = 0; mu < 4; ++mu) {
    q += (int)(rest % Ls[mu]);
    rest /= Ls[mu];
  }
  c64* d = (q & 1) ? o : e;
  const long half = 3 * (V / 2);
  for (int c = 0; c < 3; ++c) d[r * half + 3 * (n >> 1) + c] = v[r * 3 * V + 3 * n + c];
}

__global__ __launch_bounds__(256) void k_eo_merge4(c64* v, const c64* e, const c64* o, int4 L, long V) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long r = blockIdx.y;
  if (n >= V) return;
  long rest = n;
  int q = 0;
  const int Ls[4] = {L.x, L.y, L.z, L.w};
  for (int mu = 0; mu < 4; ++mu) {
    q += (int)(rest % Ls[mu]);
    rest /= Ls[mu];
  }
  const c64* s = (q & 1) ? o : e;
  const long half = 3 * (V / 2);
  for (int c = 0; c < 3; ++c) v[r * 3 * V + 3 * n + c] = s[r * half + 3 * (n >> 1) + c];
}

// natural order <-> parity halves: e[r][i] / o[r][i] with i = x >> 1
__global__ __launch_bounds__(256) void k_eo_split(c64* e, c64* o, const c64* v, int Lx, long V, long half) {
  const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long r = blockIdx.y;
  if (x >= V) return;
  const int q = (int)((x / Lx + x % Lx) & 1);
  (q ? o : e)[r * half + (x >> 1)] = v[r * V + x];
}

__global__ __launch_bounds__(256) void k_eo_merge(c64* v, const c64* e, const c64* o, int Lx, long V, long half) {
  const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long r = blockIdx.y;
  if (x >= V) return;
  const int q = (int)((x / Lx + x % Lx) & 1);
  v[r * V + x] = (q ? o : e)[r * half + (x >> 1)];
}

// x += d (add = 1) or x = a - d (add = 0), over nrhs rows of n entries
__global__ __launch_bounds__(256) void k_combine(c64* x, const c64* a, const c64* d, long n, int add) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long o = (long)blockIdx.y * n + i;
  if (i >= n) return;
  x[o] = add ? x[o] + d[o] : a[o] - d[o];
}

// out[r] = s ||v[r]||^2, one workgroup per rhs, a fixed summation order
__global__ __launch_bounds__(256) void k_norm2_scaled(double* out, const c64* v, long n, double s) {
  __shared__ double part[256];
  const long r = blockIdx.x;
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) acc += norm2(v[r * n + i]);
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = s * part[0];
}

// the 4D hop needs the natural-order links (`nl`); the 2D one reads the lattice's
void hop_eo(c64* out, const c64* in, const c64* add, const kdmg_lattice& lat, const c64* nl, int po, double c,
            double a, const int* act, int nrhs, hipStream_t st) {
  if (lat.nd == 4) {
    const long Vh = lat.volume / 2;
    const int4 L{lat.dims[0], lat.dims[1], lat.dims[2], lat.dims[3]};
    const int RB = nrhs >= 4 ? 4 : nrhs >= 2 ? 2 : 1;
    const dim3 grid(cdiv(Vh, 256), cdiv(nrhs, RB));
    if (RB == 4)
      hipLaunchKernelGGL(k_hop_eo4<4>, grid, dim3(256), 0, st, out, in, add, nl, L, po, Vh, c, a, act, nrhs);
    else if (RB == 2)
      hipLaunchKernelGGL(k_hop_eo4<2>, grid, dim3(256), 0, st, out, in, add, nl, L, po, Vh, c, a, act, nrhs);
    else
      hipLaunchKernelGGL(k_hop_eo4<1>, grid, dim3(256), 0, st, out, in, add, nl, L, po, Vh, c, a, act, nrhs);
    KDMG_LAUNCH_CHECK();
    return;
  }
  const int Lx = lat.dims[0], Lt = lat.dims[1];
  const long V = lat.volume, half = V / 2;
  const c64* Ux = lat.nat64.as<c64>();
  const c64* Ut = Ux + V;
  const int RB = nrhs >= 8 ? 8 : nrhs >= 4 ? 4 : 1;
  const dim3 grid(cdiv(half, 256), cdiv(nrhs, RB));
  if (RB == 8)
    hipLaunchKernelGGL(k_hop_eo<8>, grid, dim3(256), 0, st, out, in, add, Ux, Ut, Lx, Lt, po, half, c, a, act, nrhs);
  else if (RB == 4)
    hipLaunchKernelGGL(k_hop_eo<4>, grid, dim3(256), 0, st, out, in, add, Ux, Ut, Lx, Lt, po, half, c, a, act, nrhs);
  else
    hipLaunchKernelGGL(k_hop_eo<1>, grid, dim3(256), 0, st, out, in, add, Ux, Ut, Lx, Lt, po, half, c, a, act, nrhs);
  KDMG_LAUNCH_CHECK();
}

}  // namespace
}  // namespace kdmg

using namespace kdmg;

extern "C" kdmg_status kdmg_solve_cg_eo(const kdmg_lattice* lat, double mass, const void* b, void* x, int nrhs,
                                        double tol, int maxit, int* its_host, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(lat && b && x && b != x, KDMG_EINVAL, "kdmg_solve_cg_eo: bad pointers");
  KDMG_CHECK(lat->nd == 2 || (lat->nd == 4 && lat->nc == 3), KDMG_EUNSUPPORTED,
             "kdmg_solve_cg_eo: 2D U(1) and 4D SU(3) lattices only");
  for (int mu = 0; mu < lat->nd; ++mu)
    KDMG_CHECK(lat->dims[mu] % 2 == 0, KDMG_EINVAL, "kdmg_solve_cg_eo: even extents required");
  KDMG_CHECK(mass > 0.0, KDMG_EINVAL, "kdmg_solve_cg_eo: mass must be positive");
  KDMG_CHECK(tol > 0.0 && tol < 1.0, KDMG_EINVAL, "kdmg_solve_cg_eo: tol must be in (0, 1)");
  KDMG_CHECK(maxit >= 1, KDMG_EINVAL, "kdmg_solve_cg_eo: maxit must be positive");
  KDMG_CHECK(nrhs >= 1 && nrhs <= 1024, KDMG_EINVAL, "kdmg_solve_cg_eo: nrhs must be 1..1024");
  hipStream_t st = (hipStream_t)stream;
  const long V = lat->volume, nd = lat->ndof, half = nd / 2;
  const int Lx = lat->dims[0];
  const int4 L4{lat->dims[0], lat->dims[1], lat->dims[2], lat->dims[3]};
  const double m = mass;
  CtxAlloc ctx;
  ctx.init(st, nrhs, nrhs);
  KrylovAlloc ks;
  ks.init(nrhs);
  const size_t hv = sizeof(c64) * (size_t)nrhs * half;
  DevBuf be(hv), bo(hv), rhs(hv), xe(hv), xo(hv), r(hv), p(hv), q(hv), t(hv), ext(sizeof(double) * nrhs);
  const dim3 gs(cdiv(V, 256), nrhs);
  DevBuf nl;
  if (lat->nd == 4) {
    nl.alloc(sizeof(c64) * 4 * 9 * (size_t)V);
    hipLaunchKernelGGL(k_links_nat4, dim3(cdiv(V, 256)), dim3(256), 0, st, nl.as<c64>(), lat->lk64.as<c64>(),
                       lat->perm_full.as<int>(), V);
    hipLaunchKernelGGL(k_eo_split4, gs, dim3(256), 0, st, be.as<c64>(), bo.as<c64>(), (const c64*)b, L4, V);
  } else {
    hipLaunchKernelGGL(k_eo_split, gs, dim3(256), 0, st, be.as<c64>(), bo.as<c64>(), (const c64*)b, Lx, V, half);
  }
  KDMG_LAUNCH_CHECK();
  const c64* NL = nl.as<c64>();
  // rhs_e = m b_e - H_eo b_o ; stopping target (tol m ||b||)^2
  hop_eo(rhs.as<c64>(), bo.as<c64>(), be.as<c64>(), *lat, NL, 0, -1.0, m, nullptr, nrhs, st);
  hipLaunchKernelGGL(k_norm2_scaled, dim3(nrhs), dim3(256), 0, st, ext.as<double>(), (const c64*)b, nd, m * m);
  KDMG_LAUNCH_CHECK();
  // q = (m^2 - H_eo H_oe) p via t_o = H_oe p
  auto normal = [&](c64* qq, const c64* pp, const int* act) {
    hop_eo(t.as<c64>(), pp, nullptr, *lat, NL, 1, 1.0, 0.0, act, nrhs, st);
    hop_eo(qq, t.as<c64>(), pp, *lat, NL, 0, -1.0, m * m, act, nrhs, st);
  };
  // CG passes on res = rhs - M x_e (x_e = 0, res = rhs at first); each pass
  // solves M d = res from zero to the same absolute target, x_e += d, and the
  // true residual decides whether a rhs needs another pass
  DevBuf d(hv), res(hv), rn(sizeof(double) * nrhs);
  KDMG_HIP(hipMemsetAsync(xe.p, 0, hv, st));
  KDMG_HIP(hipMemcpyAsync(res.p, rhs.p, hv, hipMemcpyDeviceToDevice, st));
  std::vector<double> target(nrhs), resid(nrhs);
  std::vector<int> its(nrhs, 0), pass_its(nrhs);
  KDMG_HIP(hipMemcpyAsync(target.data(), ext.p, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  const dim3 gh(cdiv(half, 256), nrhs);
  bool ok = false;
  for (int pass = 0; pass < 8 && !ok; ++pass) {
    const int used = *std::max_element(its.begin(), its.end());
    if (used >= maxit) break;
    cg_solve<double>(ctx.c, nrhs, half, res.as<c64>(), d.as<c64>(), r.as<c64>(), p.as<c64>(), q.as<c64>(), tol,
                     maxit - used, ks.k, normal, 16, ext.as<double>());
    hipLaunchKernelGGL(k_combine, gh, dim3(256), 0, st, xe.as<c64>(), (const c64*)nullptr, d.as<c64>(), half, 1);
    KDMG_LAUNCH_CHECK();
    normal(q.as<c64>(), xe.as<c64>(), nullptr);
    hipLaunchKernelGGL(k_combine, gh, dim3(256), 0, st, res.as<c64>(), rhs.as<c64>(), q.as<c64>(), half, 0);
    hipLaunchKernelGGL(k_norm2_scaled, dim3(nrhs), dim3(256), 0, st, rn.as<double>(), res.as<c64>(), half, 1.0);
    KDMG_LAUNCH_CHECK();
    KDMG_HIP(hipMemcpyAsync(pass_its.data(), ks.k.its, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
    KDMG_HIP(hipMemcpyAsync(resid.data(), rn.p, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    KDMG_HIP(hipStreamSynchronize(st));
    ok = true;
    for (int i = 0; i < nrhs; ++i) {
      its[i] += pass_its[i];
      ok = ok && resid[i] <= tol * tol * target[i];
    }
  }
  // x_o = (b_o - H_oe x_e) / m
  hop_eo(xo.as<c64>(), xe.as<c64>(), bo.as<c64>(), *lat, NL, 1, -1.0 / m, 1.0 / m, nullptr, nrhs, st);
  if (lat->nd == 4)
    hipLaunchKernelGGL(k_eo_merge4, gs, dim3(256), 0, st, (c64*)x, xe.as<c64>(), xo.as<c64>(), L4, V);
  else
    hipLaunchKernelGGL(k_eo_merge, gs, dim3(256), 0, st, (c64*)x, xe.as<c64>(), xo.as<c64>(), Lx, V, half);
  KDMG_LAUNCH_CHECK();
  KDMG_HIP(hipStreamSynchronize(st));
  if (its_host) std::copy(its.begin(), its.end(), its_host);
  if (!ok) throw Error(KDMG_ENOCONV, "kdmg_solve_cg_eo: some right-hand sides did not converge");
  KDMG_API_END
}
