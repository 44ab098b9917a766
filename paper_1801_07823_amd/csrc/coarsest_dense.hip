// Exact coarsest-level solve through an explicit inverse: the build (normal
// matrix, blocked Gauss-Jordan, X = A^dag N^-1) and the per-call product
// x = X b for a batch of rhs.  See dense.h for the scheme.
#include <algorithm>

#include "api_guard.h"
#include "internal.h"

using namespace kdmg;

namespace kdmg {
namespace {

// N[r][Z ndc + jj] += sum_k Y_d1(X)[i][k] Yd_d2(W)[k][jj] with W = nbr(d1, X),
// Z = nbr(d2, W): the dense A A^dag from the stencil of A (Yt) and of A^dag
// (Yd), both column-major blocks [dir][site][col][row].  Thread (r, jj) owns
// the entries N[r][* ndc + jj], so the accumulation has no races, also where
// two directions reach the same site (extent-2 lattices).
__global__ __launch_bounds__(256) void k_dn_normal(c64* N, const c64* Yt, const c64* Yd, const int* nbr, int nsites,
                                                   int ndc, int ndir) {
  const long n = (long)nsites * ndc;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ndc) return;
  const long r = t / ndc;
  const int jj = (int)(t - r * ndc);
  const int X = (int)(r / ndc), i = (int)(r - (long)X * ndc);
  const long per = (long)ndc * ndc;
  for (int d1 = 0; d1 < ndir; ++d1) {
    const int W = nbr[(long)d1 * nsites + X];
    const c64* y = Yt + ((long)d1 * nsites + X) * per;  // y[k ndc + i] = Y_d1(X)[i][k]
    for (int d2 = 0; d2 < ndir; ++d2) {
      const int Z = nbr[(long)d2 * nsites + W];
      const c64* yd = Yd + ((long)d2 * nsites + W) * per + (long)jj * ndc;  // yd[k] = Yd_d2(W)[k][jj]
      c64 acc{0, 0};
      for (int k = 0; k < ndc; ++k) cfma(acc, y[(long)k * ndc + i], yd[k]);
      N[r * n + (long)Z * ndc + jj] += acc;
    }
  }
}

// G = (pivot block N[kb.., kb..])^-1 by Gauss-Jordan without pivoting, which
// is stable for the positive definite N.  One workgroup, thread (i, j).
__global__ __launch_bounds__(1024) void k_gj_diag(c64* G, const c64* N, long n, long kb, int w) {
  __shared__ c64 S[DN_W][DN_W + 1];
  const int i = threadIdx.x / DN_W, j = threadIdx.x % DN_W;
  const bool in = i < w && j < w;
  if (in) S[i][j] = N[(kb + i) * n + kb + j];
  __syncthreads();
  for (int p = 0; p < w; ++p) {
    c64 v{0, 0};
    if (in) {
      const c64 a = S[p][p];
      const double den = norm2(a);
      const c64 d{a.re / den, -a.im / den};  // 1 / a
      if (i == p && j == p) v = d;
      else if (i == p) v = S[p][j] * d;
      else if (j == p) v = -(S[i][p] * d);
      else v = S[i][j] - (S[i][p] * d) * S[p][j];
    }
    __syncthreads();
    if (in) S[i][j] = v;
    __syncthreads();
  }
  if (in) G[i * w + j] = S[i][j];
}

// Row panel R = G N[kb.., :] (w x n); in the pivot columns R = 1 + G, so that
// one rank-w update N - C R also produces the pivot column -N[:, kb..] G.
__global__ __launch_bounds__(256) void k_gj_rows(c64* R, const c64* G, const c64* N, long n, long kb, int w) {
  __shared__ c64 Gs[DN_W * DN_W];
  for (int e = threadIdx.x; e < w * w; e += blockDim.x) Gs[e] = G[e];
  __syncthreads();
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  if (c >= kb && c < kb + w) {
    const int jc = (int)(c - kb);
    for (int q = 0; q < w; ++q) {
      c64 g = Gs[q * w + jc];
      if (q == jc) g.re += 1.0;
      R[q * n + c] = g;
    }
    return;
  }
  c64 v[DN_W];
#pragma unroll
  for (int p = 0; p < DN_W; ++p) v[p] = N[(kb + min(p, w - 1)) * n + c];
  for (int q = 0; q < w; ++q) {
    c64 acc{0, 0};
#pragma unroll
    for (int p = 0; p < DN_W; ++p)
      if (p < w) cfma(acc, Gs[q * w + p], v[p]);
    R[q * n + c] = acc;
  }
}

// Column panel C = N[:, kb..kb+w) (n x w), copied before the update overwrites it.
__global__ __launch_bounds__(256) void k_gj_cols(c64* C, const c64* N, long n, long kb, int w) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  const long i = t / w;
  const int q = (int)(t - i * w);
  C[t] = N[i * n + kb + q];
}

// One Gauss-Jordan step on a 64 x 64 tile: rows outside the pivot block get
// N - C R; pivot rows get R (with G on the pivot block).
__global__ __launch_bounds__(256) void k_gj_update(c64* N, const c64* C, const c64* R, long n, long kb, int w) {
  __shared__ c64 Cs[64 * DN_W];  // [row][q]
  __shared__ c64 Rs[DN_W * 64];  // [q][col]
  const long r0 = (long)blockIdx.y * 64, c0 = (long)blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int e = threadIdx.x; e < 64 * DN_W; e += 256) {
    const int rr = e / DN_W, q = e - rr * DN_W;
    const long gr = min(r0 + rr, n - 1);
    const c64 v = C[gr * w + min(q, w - 1)];
    Cs[e] = q < w ? v : c64{0, 0};
  }
  for (int e = threadIdx.x; e < DN_W * 64; e += 256) {
    const int q = e >> 6, cc = e & 63;
    const long gc = min(c0 + cc, n - 1);
    const c64 v = R[(long)min(q, w - 1) * n + gc];
    Rs[e] = q < w ? v : c64{0, 0};
  }
  __syncthreads();
  c64 acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = c64{0, 0};
  for (int q = 0; q < w; ++q) {
    c64 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Cs[(ty + 16 * u) * DN_W + q];
      b[u] = Rs[q * 64 + tx + 16 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) cfma(acc[u][v], a[u], b[v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long gr = r0 + ty + 16 * u;
    if (gr >= n) continue;
    const bool piv = gr >= kb && gr < kb + w;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long gc = c0 + tx + 16 * v;
      if (gc >= n) continue;
      if (piv) {
        c64 val = R[(gr - kb) * n + gc];
        if (gc == gr) val.re -= 1.0;
        N[gr * n + gc] = val;
      } else {
        N[gr * n + gc] -= acc[u][v];
      }
    }
  }
}

// X[r][c] = sum_{d,k} Yd_d(Z)[i][k] Ninv[nbr(d, Z) ndc + k][c] for the rows
// r = Z ndc + i, i in [i0, i0 + 16): X = A^dag N^-1.
__global__ __launch_bounds__(256) void k_dn_adj(c64* X, const c64* Ninv, const c64* Yd, const int* nbr, int nsites,
                                                int ndc, int ndir) {
  const long n = (long)nsites * ndc;
  const int nch = (ndc + 15) / 16;
  const int Z = blockIdx.x / nch, i0 = (blockIdx.x - Z * nch) * 16;
  const long c = (long)blockIdx.y * 256 + threadIdx.x;
  const long cc = min(c, n - 1);
  const long per = (long)ndc * ndc;
  c64 acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = c64{0, 0};
  for (int d = 0; d < ndir; ++d) {
    const int W = nbr[(long)d * nsites + Z];
    const c64* yd = Yd + ((long)d * nsites + Z) * per;  // yd[k ndc + i] = Yd_d(Z)[i][k]
    for (int k = 0; k < ndc; ++k) {
      const c64 v = Ninv[((long)W * ndc + k) * n + cc];
#pragma unroll
      for (int u = 0; u < 16; ++u) cfma(acc[u], yd[(long)k * ndc + min(i0 + u, ndc - 1)], v);
    }
  }
  if (c >= n) return;
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (i0 + u < ndc) X[((long)Z * ndc + i0 + u) * n + c] = acc[u];
}

// k-chunk width of the product and its workgroups per CU (the register
// budget is set so that this many fit: 256 threads each)
constexpr int DN_KC = 16, DN_WPC = 4;

// part[s][r][i] = sum_{k in split s} X[i][k] b[r][k] for a 64-row x (16 NT)-rhs
// tile.  Each DN_KC-wide k-chunk of X and b is staged in LDS from coalesced
// loads; the next chunk's loads are issued into registers before the current
// chunk is contracted, so their latency overlaps the MFMAs.  Wave w contracts
// rows 16w..16w+15 against NT 16-rhs tiles with v_mfma_f64_16x16x4 (Gauss:
// three real products per complex one).  Loads past the end of a split read a
// clamped address and are replaced by zero.  With `act`, a workgroup whose
// rhs tile holds no active rhs returns at once (its partial sums are never
// read: k_dn_reduce skips inactive rhs).
template <int NT>
__global__ __launch_bounds__(256, DN_WPC) void k_dn_apply(c64* part, const c64* __restrict__ X, const c64* __restrict__ b,
                                                  long n, int nrhs, long kc, const int* act) {
  constexpr int RW = 16 * NT, KC = DN_KC;
  __shared__ c64 Xs[64][KC + 1];
  __shared__ c64 Bs[RW][KC + 1];
  using M = Mfma<double>;
  typedef M::v4 v4;
  const int rb = blockIdx.z * RW;
  if (act) {
    int mine = 0;
    for (int t = threadIdx.x; t < RW && rb + t < nrhs; t += blockDim.x) mine |= act[rb + t];
    if (!__syncthreads_or(mine)) return;
  }
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), l = threadIdx.x & 63;
  const long row0 = (long)blockIdx.x * 64;
  const long k0 = (long)blockIdx.y * kc, k1 = min(n, k0 + kc);
  v4 p1[NT], p2[NT], p3[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    p1[t] = v4{0, 0, 0, 0};
    p2[t] = v4{0, 0, 0, 0};
    p3[t] = v4{0, 0, 0, 0};
  }
  constexpr int NX = 64 * KC / 256, NB = RW * KC / 256;
  c64 rx[NX], rbv[NB];
  auto fetch = [&](long kb) {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int e = j * 256 + threadIdx.x, r = e / KC, k = e % KC;
      const long gr = min(row0 + r, n - 1), gk = kb + k;
      const c64 v = X[gr * n + min(gk, n - 1)];
      rx[j] = gk < k1 ? v : c64{0, 0};
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = j * 256 + threadIdx.x, c = e / KC, k = e % KC;
      const long gc = min(rb + c, nrhs - 1), gk = kb + k;
      const c64 v = b[gc * n + min(gk, n - 1)];
      rbv[j] = gk < k1 ? v : c64{0, 0};
    }
  };
  fetch(k0);
  for (long kb = k0; kb < k1; kb += KC) {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int e = j * 256 + threadIdx.x;
      Xs[e / KC][e % KC] = rx[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = j * 256 + threadIdx.x;
      Bs[e / KC][e % KC] = rbv[j];
    }
    __syncthreads();
    if (kb + KC < k1) fetch(kb + KC);  // in flight during the contraction below
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const c64 a = Xs[16 * w + (l & 15)][4 * s + (l >> 4)];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const c64 bb = Bs[16 * t + (l & 15)][4 * s + (l >> 4)];
        p1[t] = M::op(a.re, bb.re, p1[t]);
        p2[t] = M::op(a.im, bb.im, p2[t]);
        p3[t] = M::op(a.re + a.im, bb.re + bb.im, p3[t]);
      }
    }
    __syncthreads();
  }
  // fragments -> LDS tile O[rhs][row] (in Xs' storage, one 16-rhs tile at a
  // time) -> coalesced rows
  static_assert(64 * (KC + 1) >= 16 * 64, "the output tile must fit in Xs");
  c64* O = &Xs[0][0];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + M::row(l, v), c = l & 15;
      const double q1 = p1[t][v], q2 = p2[t][v], q3 = p3[t][v];
      O[c * 64 + i] = c64{q1 - q2, q3 - q1 - q2};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int c = e >> 6, i = e & 63;
      const long gr = row0 + i;
      const int gc = rb + 16 * t + c;
      if (gr < n && gc < nrhs) part[((long)blockIdx.y * nrhs + gc) * n + gr] = O[e];
    }
    __syncthreads();
  }
}

// out[r] = sum over splits in order; the coarse-solve statistics of the
// active rhs (one iteration per call).
__global__ __launch_bounds__(256) void k_dn_reduce(c64* out, const c64* part, long n, int nrhs, int S,
                                                   const int* parent, int* its, int* calls, int* tot,
                                                   int* worked) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (worked && i == 0 && r == 0) {
    int any = 0;
    for (int q = 0; q < nrhs && !any; ++q) any = !parent || parent[q];
    *worked = any;
  }
  if (parent && !parent[r]) return;
  if (i < n) {
    c64 s = part[(long)r * n + i];
    for (int q = 1; q < S; ++q) s += part[((long)q * nrhs + r) * n + i];
    out[(long)r * n + i] = s;
  }
  if (i == 0 && (!parent || parent[r])) {
    if (its) its[r] = 1;
    if (calls) calls[r] += 1;
    if (tot) tot[r] += 1;
  }
}

long split_width(long n, int nrhs) {
  const long tiles = (long)cdiv(n, 64) * cdiv(nrhs, nrhs > 16 ? 32 : 16);
  long s = 256L * DN_WPC / tiles;  // as many splits as stay resident at once
  s = std::max(1L, std::min(s, (long)cdiv(n, DN_KC)));
  return (long)cdiv(cdiv(n, s), DN_KC) * DN_KC;
}

}  // namespace

int dense_apply_splits(long n, int nrhs) { return (int)cdiv(n, split_width(n, nrhs)); }

void build_dense_inverse(DenseInverse& D, const CoarseLevel& L, hipStream_t st) {
  const long n = L.n();
  KDMG_CHECK(n >= 1 && n <= 32768, KDMG_EUNSUPPORTED, "exact coarsest solve: more than 32768 coarsest dofs");
  auto need = [](DevBuf& b, size_t bytes) {
    if (b.bytes != bytes) b.alloc(bytes);
  };
  D.built = false;
  D.n = n;
  need(D.X, sizeof(c64) * n * n);
  need(D.N, sizeof(c64) * n * n);
  need(D.G, sizeof(c64) * DN_W * DN_W);
  need(D.R, sizeof(c64) * DN_W * n);
  need(D.C, sizeof(c64) * n * DN_W);
  c64* N = D.N.as<c64>();
  KDMG_HIP(hipMemsetAsync(N, 0, D.N.bytes, st));
  hipLaunchKernelGGL(k_dn_normal, dim3(cdiv(n * L.ndc, 256)), dim3(256), 0, st, N, L.Yt64.as<c64>(),
                     L.Yd64.as<c64>(), L.nbr.as<int>(), L.nsites, L.ndc, L.ndir);
  KDMG_LAUNCH_CHECK();
  const unsigned nt = cdiv(n, 64);
  for (long kb = 0; kb < n; kb += DN_W) {
    const int w = (int)std::min<long>(DN_W, n - kb);
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(1024), 0, st, D.G.as<c64>(), N, n, kb, w);
    hipLaunchKernelGGL(k_gj_rows, dim3(cdiv(n, 256)), dim3(256), 0, st, D.R.as<c64>(), D.G.as<c64>(), N, n, kb, w);
    hipLaunchKernelGGL(k_gj_cols, dim3(cdiv(n * w, 256)), dim3(256), 0, st, D.C.as<c64>(), N, n, kb, w);
    hipLaunchKernelGGL(k_gj_update, dim3(nt, nt), dim3(256), 0, st, N, D.C.as<c64>(), D.R.as<c64>(), n, kb, w);
    KDMG_LAUNCH_CHECK();
  }
  const int nch = (L.ndc + 15) / 16;
  hipLaunchKernelGGL(k_dn_adj, dim3(L.nsites * nch, cdiv(n, 256)), dim3(256), 0, st, D.X.as<c64>(), N,
                     L.Yd64.as<c64>(), L.nbr.as<int>(), L.nsites, L.ndc, L.ndir);
  KDMG_LAUNCH_CHECK();
  D.built = true;
}

void dense_apply(const DenseInverse& D, c64* out, const c64* in, c64* part, int nrhs, const int* parent, int* its,
                 int* calls, int* tot, hipStream_t st, int* worked) {
  KDMG_CHECK(D.built, KDMG_EINVAL, "exact coarsest solve: inverse not built");
  const long n = D.n, kc = split_width(n, nrhs);
  const int S = (int)cdiv(n, kc);
  const unsigned rt = cdiv(n, 64);
  if (nrhs > 16)
    hipLaunchKernelGGL(k_dn_apply<2>, dim3(rt, S, cdiv(nrhs, 32)), dim3(256), 0, st, part, D.X.as<c64>(), in, n,
                       nrhs, kc, parent);
  else
    hipLaunchKernelGGL(k_dn_apply<1>, dim3(rt, S, 1), dim3(256), 0, st, part, D.X.as<c64>(), in, n, nrhs, kc,
                       parent);
  hipLaunchKernelGGL(k_dn_reduce, dim3(cdiv(n, 256), nrhs), dim3(256), 0, st, out, part, n, nrhs, S, parent, its,
                     calls, tot, worked);
  KDMG_LAUNCH_CHECK();
}

}  // namespace kdmg

extern "C" kdmg_status kdmg_coarsest_solve(kdmg_hierarchy* h, const void* in, void* out, int nrhs, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && in && out && in != out, KDMG_EINVAL, "kdmg_coarsest_solve: bad pointers");
  KDMG_CHECK(nrhs >= 1 && nrhs <= 1024, KDMG_EINVAL, "kdmg_coarsest_solve: nrhs must be 1..1024");
  KDMG_CHECK(h->params.coarse_solver == 1 && h->dinv.built, KDMG_EINVAL,
             "kdmg_coarsest_solve: the hierarchy was not built with the exact coarsest solve");
  hipStream_t st = (hipStream_t)stream;
  DevBuf part(sizeof(c64) * (size_t)dense_apply_splits(h->dinv.n, nrhs) * nrhs * h->dinv.n);
  dense_apply(h->dinv, (c64*)out, (const c64*)in, part.as<c64>(), nrhs, nullptr, nullptr, nullptr, nullptr, st);
  KDMG_HIP(hipStreamSynchronize(st));
  KDMG_API_END
}
