// Asymmetric first coarsening of the 2D KD operator (Sec. 5, eqs. "prcplx"
// and "thinlu"; App. A): restriction R != P^dag, built per aggregate by a
// thin LU bi-orthonormalisation.
//
// With the near-null vectors v_i of A (after the global Gram-Schmidt) and the
// two operators gamma5^R = B eps and gamma5^L = eps B^-1 of A (block-local,
// eqs. "gamma5R" and "gamma5L"), every aggregate Z takes
//   P~ = [ v_1 .. v_n | B eps v_1 .. B eps v_n ]            (|Z| x 2n),
//   R~ = [ v_1^dag ; .. ; v_n^dag ; v_1^dag eps B^-1 ; .. ]  (2n x |Z|),
// the left vectors being the right ones.  R~ P~ = L U (no pivoting, L unit
// lower), R = L^-1 R~, P = P~ U^-1, so that R P = 1 on every aggregate and
// the coarse operator is A_hat = R A P = 1 + R C B^-1 P.  The coarse dofs of
// an aggregate are the n columns from v, then the n columns from B eps v;
// the columns are not split by chirality.
//
// Storage: P as [fine dof][2n] and R transposed, R^T as [fine dof][2n]
// (element (x, j) = R[j][x]), both in the block layout of fine2d.h.
#pragma once
#include "common.h"
#include "blas.h"
#include "fine2d.h"

namespace kdmg {

template <class R>
__device__ __forceinline__ Cx<R> cdivide(Cx<R> a, Cx<R> b) {
  const R d = R(1) / norm2(b);
  return Cx<R>{(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}

// LDS bytes of k_asym_build for nd fine dofs and ndc coarse dofs per aggregate.
inline size_t asym_build_lds(int nd, int ndc) {
  return sizeof(c64) * ((size_t)2 * nd * ndc + (size_t)ndc * ndc) + sizeof(int) * nd;
}

// One workgroup per aggregate Z (grid nZ, at least 2 nd threads).  V: the
// orthonormalised vectors, [n][f] in block layout; m: the mass of B.
// *fail is set when a pivot of the LU is exactly zero.
template <class LT>
__global__ __launch_bounds__(1024) void k_asym_build(c64* P, c64* Rt, const c64* V, long f, const Cx<LT>* links,
                                                     Geo2 g, Agg2 a, double m, int* fail) {
  extern __shared__ __align__(16) unsigned char asym_raw[];
  const int Z = blockIdx.x, nv = a.nv, ndc = 2 * nv, nblk = a.a0 * a.a1, nd = 4 * nblk;
  c64* Pt = reinterpret_cast<c64*>(asym_raw);  // [nd][ndc]
  c64* Rs = Pt + (long)nd * ndc;                // [ndc][nd]
  c64* M = Rs + (long)ndc * nd;                 // [ndc][ndc]
  int* qd = reinterpret_cast<int*>(M + (long)ndc * ndc);
  aggregate_dofs(qd, g, a, Z, 2);
  __syncthreads();
  const int Z0 = Z % a.Ncx, Z1 = Z / a.Ncx;
  for (int t = threadIdx.x; t < nblk * nv; t += blockDim.x) {
    const int k = t / nv, i = t - k * nv;
    const int X0 = Z0 * a.a0 + k % a.a0, X1 = Z1 * a.a1 + k / a.a0, p = (X0 + X1) & 1;
    const int b = blk_index(g, X0, X1);
    c64 L[4], v[4], ev[4], w[4], u[4];
    load_intra<double, LT>(links + ((size_t)p * g.Nb2 + b) * 8, L);
    const long base = (long)p * g.half + 4L * b;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      v[s] = V[(long)i * f + base + s];
      ev[s] = (double)eps2(s) * v[s];
    }
    b_block<double>(L, m, ev, w);     // B eps v
    binv_block<double>(L, m, v, u);   // B^-1 v (eps applied below)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = 4 * k + s;
      Pt[q * ndc + i] = v[s];
      Pt[q * ndc + nv + i] = w[s];
      Rs[i * nd + q] = conj(v[s]);
      Rs[(nv + i) * nd + q] = conj((double)eps2(s) * u[s]);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ndc * ndc; e += blockDim.x) {
    const int r = e / ndc, c = e - r * ndc;
    c64 acc{0, 0};
    for (int q = 0; q < nd; ++q) cfma(acc, Rs[r * nd + q], Pt[q * ndc + c]);
    M[e] = acc;
  }
  __syncthreads();
  // LU without pivoting in place: U on and above the diagonal, L's
  // multipliers below it
  for (int k = 0; k < ndc; ++k) {
    const c64 piv = M[k * ndc + k];
    if (piv.re == 0.0 && piv.im == 0.0) {
      if (threadIdx.x == 0) *fail = 1;
      return;  // uniform across the workgroup: every thread read the same pivot
    }
    const int w = ndc - 1 - k;
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      M[i * ndc + j] -= cdivide(M[i * ndc + k], piv) * M[k * ndc + j];
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < ndc; i += blockDim.x) M[i * ndc + k] = cdivide(M[i * ndc + k], piv);
    __syncthreads();
  }
  // R = L^-1 R~ (thread q owns column q), P = P~ U^-1 (thread nd + q owns row q)
  for (int t = threadIdx.x; t < 2 * nd; t += blockDim.x) {
    if (t < nd) {
      const int q = t;
      for (int r = 1; r < ndc; ++r) {
        c64 acc = Rs[r * nd + q];
        for (int k = 0; k < r; ++k) acc -= M[r * ndc + k] * Rs[k * nd + q];
        Rs[r * nd + q] = acc;
      }
    } else {
      const int q = t - nd;
      for (int c = 0; c < ndc; ++c) {
        c64 acc = Pt[q * ndc + c];
        for (int k = 0; k < c; ++k) acc -= Pt[q * ndc + k] * M[k * ndc + c];
        Pt[q * ndc + c] = cdivide(acc, M[c * ndc + c]);
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nd * ndc; e += blockDim.x) {
    const int q = e / ndc, c = e - q * ndc;
    const long x = qd[q];
    P[x * ndc + c] = Pt[e];
    Rt[x * ndc + c] = Rs[c * nd + q];
  }
}

// W[x][c] = (B^-1 P[., c])(x), block by block.  grid (cdiv(Nb2, 256), ndc, 2).
template <class LT>
__global__ __launch_bounds__(256) void k_galerkin_wa(c64* W, const c64* P, const Cx<LT>* links, Geo2 g, int ndc,
                                                     double m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y, p = blockIdx.z;
  if (b >= g.Nb2) return;
  c64 L[4], v[4], w[4];
  load_intra<double, LT>(links + ((size_t)p * g.Nb2 + b) * 8, L);
  const long base = (long)p * g.half + 4L * b;
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = P[(base + s) * ndc + c];
  binv_block<double>(L, m, v, w);
#pragma unroll
  for (int s = 0; s < 4; ++s) W[(base + s) * ndc + c] = w[s];
}

// A_hat = 1 + R C W on the first coarse level, one workgroup per coarse site
// Z; every fine site of the aggregate contributes to every row.  Output as
// k_galerkin1: Yt[dir][Z][col][row], dir 0 self, 1/2 = +-x, 3/4 = +-t.
template <class LT>
__global__ __launch_bounds__(1024) void k_galerkin1a(c64* Yt, const c64* Rt, const c64* W, const Cx<LT>* links,
                                                     Geo2 g, Agg2 a) {
  const int Z = blockIdx.x;
  const int ndc = 2 * a.nv;
  const long nZ = (long)a.Ncx * a.Nct;
  const int Z0 = Z % a.Ncx, Z1 = Z / a.Ncx;
  for (int pair = threadIdx.x; pair < ndc * ndc; pair += blockDim.x) {
    const int row = pair / ndc, col = pair % ndc;
    c64 acc[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) acc[d] = c64{0, 0};
    for (int k = 0; k < a.a0 * a.a1; ++k) {
      const int X0 = Z0 * a.a0 + k % a.a0, X1 = Z1 * a.a1 + k / a.a0;
      const int p = (X0 + X1) & 1, q = 1 - p;
      const int b = blk_index(g, X0, X1);
      const Nbr2 n = nbr2(g, p, b);
      const Cx<LT>* Lb = links + ((size_t)p * g.Nb2 + b) * 8;
      const Cx<LT>* Lxm = links + ((size_t)q * g.Nb2 + n.xm) * 8;
      const Cx<LT>* Ltm = links + ((size_t)q * g.Nb2 + n.tm) * 8;
      const long base = (long)p * g.half + 4L * b;
      const int dxp = ((X0 + 1) % a.a0 == 0) ? 1 : 0, dxm = (X0 % a.a0 == 0) ? 2 : 0;
      const int dtp = ((X1 + 1) % a.a1 == 0) ? 3 : 0, dtm = (X1 % a.a1 == 0) ? 4 : 0;
      auto Wat = [&](int nb, int s) -> c64 { return W[((long)q * g.half + 4L * nb + s) * ndc + col]; };
      auto Rat = [&](int s) -> c64 { return Rt[(base + s) * ndc + row]; };
      // the hops of C from each site of the block (as in hop_block)
      cfma(acc[dxm], Rat(0), -(conj(ld<double>(Lxm[4])) * Wat(n.xm, 1)));
      cfma(acc[dtm], Rat(0), -(conj(ld<double>(Ltm[6])) * Wat(n.tm, 2)));
      cfma(acc[dxp], Rat(1), ld<double>(Lb[4]) * Wat(n.xp, 0));
      cfma(acc[dtm], Rat(1), -(conj(ld<double>(Ltm[7])) * Wat(n.tm, 3)));
      cfma(acc[dtp], Rat(2), ld<double>(Lb[6]) * Wat(n.tp, 0));
      cfma(acc[dxm], Rat(2), -(conj(ld<double>(Lxm[5])) * Wat(n.xm, 3)));
      cfma(acc[dxp], Rat(3), ld<double>(Lb[5]) * Wat(n.xp, 2));
      cfma(acc[dtp], Rat(3), ld<double>(Lb[7]) * Wat(n.tp, 1));
    }
    if (row == col) acc[0].re += 1.0;
#pragma unroll
    for (int d = 0; d < 5; ++d) Yt[(((long)d * nZ + Z) * ndc + col) * ndc + row] = acc[d];
  }
}

// Restriction with R: out[r][Z][j] = sum_{x in Z} R[j][x] in[r][x]
// (even_only: the parity-0 half only contributes).  The workgroup of
// aggregate Z stages R^T's rows of the aggregate and its tile of RB rhs in
// LDS; thread o adds one (rhs, coarse dof).  grid (nZ, cdiv(nrhs, RB));
// LDS (nd ndc + RB nd) Cx<R> + nd int.
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k_restrict1a(Cx<VO>* out, const Cx<VI>* in, long si, const Cx<PT>* Rt,
                                                    Geo2 g, Agg2 a, int even_only, const int* act, int nrhs,
                                                    int RB) {
  extern __shared__ __align__(16) unsigned char xa_raw[];
  const int Z = xcd_block(blockIdx.x, gridDim.x), r0 = blockIdx.y * RB, ndc = 2 * a.nv;
  const int nd = 4 * a.a0 * a.a1;
  Cx<R>* Rs = reinterpret_cast<Cx<R>*>(xa_raw);  // [nd][ndc]
  Cx<R>* Vs = Rs + (long)nd * ndc;               // [RB][nd]
  int* qd = reinterpret_cast<int*>(Vs + (long)RB * nd);
  aggregate_dofs(qd, g, a, Z, even_only ? 1 : 2);
  __syncthreads();
  stage_rows<R, 4>(Rs, ndc, nd, ndc, [&](int q, int j) {
    const int d = qd[q];
    return d >= 0 ? ld<R>(Rt[(long)d * ndc + j]) : Cx<R>{0, 0};
  });
  stage_rows<R, 4>(Vs, nd, RB, nd, [&](int r, int q) {
    const int d = qd[q], rr = r0 + r;
    return d >= 0 && rr < nrhs && is_active(act, rr) ? ld<R>(in[rr * si + d]) : Cx<R>{0, 0};
  });
  __syncthreads();
  const long nc = (long)a.Ncx * a.Nct * ndc;
  for (int o = threadIdx.x; o < RB * ndc; o += blockDim.x) {
    const int r = o / ndc, j = o - r * ndc, rr = r0 + r;
    if (rr >= nrhs || !is_active(act, rr)) continue;
    const Cx<R>* v = Vs + (long)r * nd;
    Cx<R> acc{0, 0};
    for (int q = 0; q < nd; ++q) cfma(acc, Rs[q * ndc + j], v[q]);
    out[rr * nc + (long)Z * ndc + j] = st<VO>(acc);
  }
}

// Prolongation with P: out[r][x] = [add[r][x] +] sum_j P[x][j] in[r][Z(x)][j]
// (npar = 1: only the parity-0 blocks, out/add being Schur-half vectors).
// grid (nZ, cdiv(nrhs, RB)); LDS (nd (ndc + 1) + RB ndc) Cx<R> + nd int.
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k_prolong1a(Cx<VO>* out, long so, const Cx<VO>* add, long sa,
                                                   const Cx<VI>* in, const Cx<PT>* P, Geo2 g, Agg2 a, int npar,
                                                   const int* act, int nrhs, int RB) {
  extern __shared__ __align__(16) unsigned char xa_raw[];
  const int Z = xcd_block(blockIdx.x, gridDim.x), r0 = blockIdx.y * RB, ndc = 2 * a.nv, RP = ndc + 1;
  const int nd = 4 * a.a0 * a.a1;
  Cx<R>* Ps = reinterpret_cast<Cx<R>*>(xa_raw);  // [nd][ndc + 1]
  Cx<R>* Es = Ps + (long)nd * RP;                // [RB][ndc]
  int* qd = reinterpret_cast<int*>(Es + (long)RB * ndc);
  aggregate_dofs(qd, g, a, Z, npar);
  __syncthreads();
  stage_rows<R, 4>(Ps, RP, nd, ndc, [&](int q, int j) {
    const int d = qd[q];
    return d >= 0 ? ld<R>(P[(long)d * ndc + j]) : Cx<R>{0, 0};
  });
  const long nc = (long)a.Ncx * a.Nct * ndc;
  stage_rows<R, 4>(Es, ndc, RB, ndc, [&](int r, int j) {
    const int rr = r0 + r;
    return rr < nrhs ? ld<R>(in[rr * nc + (long)Z * ndc + j]) : Cx<R>{0, 0};
  });
  __syncthreads();
  for (int o = threadIdx.x; o < RB * nd; o += blockDim.x) {
    const int r = o / nd, q = o - r * nd, rr = r0 + r, x = qd[q];
    if (x < 0 || rr >= nrhs || !is_active(act, rr)) continue;
    const Cx<R>* pq = Ps + q * RP;
    const Cx<R>* er = Es + r * ndc;
    Cx<R> acc{0, 0};
    for (int j = 0; j < ndc; ++j) cfma(acc, pq[j], er[j]);
    if (add) acc += ld<R>(add[rr * sa + x]);
    out[rr * so + x] = st<VO>(acc);
  }
}

}  // namespace kdmg
