// Coarse stencil apply and the fused coarsest-level CGNE, LDS-staged, with
// two compute cores:
//   * MFMA core (>= 16 rhs): the per-site product out(X) = sum_dir Y_dir(X)
//     V(nbr(X, dir)) is a complex (ndc x K) . (K x RT) GEMM, K = ndir*ndc.
//     Complex arithmetic takes three real products (Gauss)
//       P1 = Yr Vr, P2 = Yi Vi, P3 = (Yr + Yi)(Vr + Vi),
//       Re C = P1 - P2,  Im C = P3 - P1 - P2,
//     each a v_mfma_{f32,f64}_16x16x4 on 16x16 output tiles; one wavefront
//     owns one (16 dofs x 16 rhs) tile and runs two independent accumulator
//     sets over even/odd k-chunks to keep the matrix pipe busy;
//   * SIMT core (< 16 rhs): each thread accumulates a TI x TR register tile,
//     with the (dir, j) loop split KS ways for few rhs.
// Both read the site's stencil blocks and the neighbour panel from LDS: the
// workgroup first copies Y_dir(X) (column-major, [dir][j][i]) and
// v[r][nbr(X,dir)][j] for its rhs tile with coalesced loads.
//
// Fused CGNE (Sec. 4, Table 1: CG on A A^dag, x = A^dag y, on the coarsest
// level).  One iteration is two kernels:
//   A_k: alpha = rr_k / ||p||^2 ; q = A p ; x += alpha p ; r -= alpha q
//   B_k: beta = ||r||^2 / rr_k (stop the rhs once ||r|| <= tol ||b||) ;
//        p = A^dag r + beta p
// Every workgroup writes one partial sum per (site, rhs); each workgroup of
// the next kernel adds up all partials of its rhs in the same fixed order, so
// all of them obtain bit-identical scalars with no atomics and no device-scope
// fences.  Per-rhs state (rr, active flag) is double-buffered by iteration
// parity because workgroup 0 updates it while other workgroups of the same
// kernel still read the previous values.
#pragma once
#include <algorithm>

#include "common.h"
#include "blas.h"

namespace kdmg {

// ------------------------------------------------------------------ MFMA traits

template <class R>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element v of lane l holds row (l / 16) + 4 v, column l % 16
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element v of lane l holds row 4 (l / 16) + v, column l % 16
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// ------------------------------------------------------------------ launch shape

struct TileShape {
  int core = 0;  // 0 SIMT, 1 MFMA
  int RT = 1;    // rhs per workgroup
  int TI = 1;    // SIMT: dofs per thread
  int TR = 1;    // SIMT: rhs per thread
  int KS = 1;    // SIMT: split of the (dir, j) loop
  int MT = 1;    // MFMA: 16-row tiles
  int NT = 1;    // MFMA: 16-rhs tiles
  int ylds = 1;  // MFMA: stencil blocks staged in LDS (1) or read from global with prefetch (0)
  int threads = 0;
  size_t smem = 0;
  int nslots() const { return core ? MT * 4 : 0; }
};

struct LdsLayout {
  size_t ys, vs, red, S, sc, live, O, total;
};

// Panel row stride (complex entries) and the place of entry (contraction row
// k, tile rhs r).  Tiles of fewer than 32 rhs keep one pad entry per row, so
// the rhs-strided LDS stores of the dof-fastest gather do not hit a single
// bank.  Tiles of 32 rhs (or a multiple) are unpadded and swizzled instead:
// within each aligned group of 32 columns, column r of row k sits at
// r ^ g(k), g(k) = 16 (k & 1) + ((k >> 1) & 15), a permutation of the 32
// columns for every row.  With 64 four-byte banks and 8-byte entries, a row
// of 32 entries covers every bank once, and
//  * the gather's stores (32 consecutive rows of one rhs per half-wavefront)
//    fall in 32 different columns;
//  * the MFMA B-operand reads (16 consecutive columns of rows k and k + 1,
//    k even, per half-wavefront) fall in opposite 16-column halves;
// so neither access has a bank conflict.
__host__ __device__ __forceinline__ int panel_stride(int RT) { return RT % 32 == 0 ? RT : RT + 1; }
__host__ __device__ __forceinline__ int panel_at(int k, int r, int RT) {
  return RT % 32 == 0 ? k * RT + (r ^ (((k & 1) << 4) | ((k >> 1) & 15))) : k * (RT + 1) + r;
}

// panel rows (contraction index k = dir * ndc + j) rounded up to the 8 of an
// MFMA chunk pair; rows [ndir * ndc, kpad8) are zero
__host__ __device__ __forceinline__ int kpad8(int K) { return (K + 7) & ~7; }

// floor(e / n) through the float reciprocal inv = 1.0f / n: exact whenever
// 0 <= e and e + n < 2^22 (the relative error of the product, < 2^-23, stays
// below the distance 0.5 / n of (e + 0.5) / n to the nearest integer).  All
// index arithmetic of these kernels is far inside that range (< 2^17).
__device__ __forceinline__ int fdiv(int e, float inv) { return (int)(((float)e + 0.5f) * inv); }

// Lanes per rhs for the per-rhs reductions: a power of two <= 64 with
// GS * RT <= blockDim, so every group lies inside one wavefront.
__device__ __forceinline__ int group_size(int RT) {
  int g = 64;
  while (g > 1 && g * RT > (int)blockDim.x) g >>= 1;
  return g;
}

// Sum of v over the GS lanes of each aligned lane group, by an xor butterfly:
// a fixed tree, and every lane of the group ends with the same bits.  Called
// by every lane of the wavefront.
__device__ __forceinline__ double group_sum(double v, int GS) {
  for (int o = GS >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// plain = true: the layout of the stencil apply alone (k_capply_fast), which
// needs none of the fused CGNE's per-rhs scalars (S, sc, live) and writes its
// output tile O over the panel once the contraction is done; with the
// stencil blocks streamed from global memory, the MFMA k-split partials
// (written once every wave has left the contraction) go over the panel too.
// At the level-1 shape (32 dofs, 5 directions) a 32-rhs tile then takes the
// 40 KB panel alone (four workgroups per CU), a 16-rhs tile 22 KB (seven).
inline LdsLayout lds_layout(const TileShape& s, int ndc, int ndir, size_t esz, bool plain = false) {
  LdsLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 15) & ~size_t(15);
    return at;
  };
  // stencil blocks (else read from global); also the MFMA k-split partials,
  // written after the contraction
  const size_t ysz = s.core && s.ylds ? (size_t)ndir * ndc * ndc * esz : 0;
  const size_t ksz = s.core && s.KS > 1 ? (size_t)(s.KS - 1) * s.MT * s.NT * 256 * esz : 0;
  const size_t vsz = (size_t)kpad8(ndir * ndc) * panel_stride(s.RT) * esz;
  const bool alias = plain && ysz == 0 && ksz <= vsz;
  L.ys = take(alias ? 0 : std::max(ysz, ksz));
  L.vs = take(vsz);
  if (alias) L.ys = L.vs;
  int nib = s.core ? 0 : ndc / s.TI, nrb = s.core ? 0 : s.RT / s.TR;
  L.red = take(s.core ? 0 : (size_t)(s.KS - 1) * nib * nrb * s.TI * s.TR * esz);
  const int nsl = s.core ? s.MT * 4 : nib;
  L.S = take(plain ? 0 : (size_t)nsl * s.RT * sizeof(double));
  L.sc = take(plain ? 0 : (size_t)(2 * s.RT + 1024) * sizeof(double));
  L.live = take(plain ? 0 : (size_t)s.RT * sizeof(int));
  L.O = plain ? L.vs : take((size_t)s.RT * ndc * esz);
  L.total = o;
  return L;
}

constexpr size_t LDS_LIMIT = 160 * 1024;

inline TileShape choose_tile(int ndc, int nrhs, int ndir, size_t esz) {
  TileShape s;
  if (nrhs >= 16) {
    s.core = 1;
    s.MT = (ndc + 15) / 16;
    s.NT = nrhs >= 32 ? 2 : 1;
    s.RT = 16 * s.NT;
    while (s.NT > 1 && lds_layout(s, ndc, ndir, esz).total > LDS_LIMIT) {
      s.NT /= 2;
      s.RT = 16 * s.NT;
    }
    s.threads = 64 * s.MT * s.NT;
    if (s.threads < 512) s.threads = 512;
    s.smem = lds_layout(s, ndc, ndir, esz).total;
    if (s.smem <= LDS_LIMIT && s.threads <= 1024) return s;
    s = TileShape();
  }
  s.core = 0;
  if (nrhs >= 4) {
    s.TI = (ndc % 2 == 0) ? 2 : 1;
    s.TR = 1;
    s.RT = nrhs >= 16 ? 16 : nrhs;
  } else {
    s.TI = 1;
    s.TR = 1;
    s.RT = nrhs;
  }
  auto tiles = [&] { return (ndc / s.TI) * (s.RT / s.TR); };
  while (s.RT > 1 && (tiles() > 256 || lds_layout(s, ndc, ndir, esz).total > LDS_LIMIT)) s.RT /= 2;
  s.KS = 256 / tiles();
  if (s.KS < 1) s.KS = 1;
  if (s.KS > 16) s.KS = 16;
  while (s.KS > 1 && lds_layout(s, ndc, ndir, esz).total > LDS_LIMIT) --s.KS;
  s.threads = tiles() * s.KS;
  s.threads = ((s.threads + 63) / 64) * 64;
  if (s.threads < 64) s.threads = 64;
  s.smem = lds_layout(s, ndc, ndir, esz).total;
  return s;
}

// ------------------------------------------------------------------ staging

// Neighbour sites of X in every direction; the addresses are uniform across
// the workgroup, so these are scalar loads issued once at kernel entry.
constexpr int MAX_DIR = 9;
struct Nbrs {
  int s[MAX_DIR];
};

__device__ __forceinline__ Nbrs load_nbrs(const int* __restrict__ nbr, int X, int nsites, int ndir) {
  Nbrs n;
#pragma unroll
  for (int d = 0; d < MAX_DIR; ++d) n.s[d] = d < ndir ? nbr[(long)d * nsites + X] : X;
  return n;
}


// Per-thread loads per pass: stencil-block entries and partial sums (the
// panel takes one element in every direction).
constexpr int YU = 4, SU = 8;

// Stages the workgroup's operands into LDS, one pass per batch:
// every load of a pass (stencil blocks, panel, partial sums) is issued before
// any is consumed, so the common shapes pay a single memory round trip.
//   Ys[(d*ndc + j)*ndc + i] = Y_dir(X)[i][j]            (when Ys != null)
//   Vs[panel_at(d*ndc + j, r)] = v[r0 + r][nbr(X, d)][j] (rhs >= nrhs read as 0;
//                                                         rows up to kpad8 zero)
// With P != null ([rhs][site] partial sums of the previous kernel) the lane
// g of rhs group t (t = tid / GS, g = tid % GS, GS = group_size(RT)) sums
// P[r0 + t][g + k GS] over k in increasing order; the group's lanes are then
// added by group_sum() and lane 0 stores the total in tot[t].  The order is
// fixed, so every workgroup obtains bit-identical totals.
template <class R, class OT, class VI>
__device__ __forceinline__ void stage_all(Cx<R>* Ys, Cx<R>* Vs, const Cx<OT>* __restrict__ Yt,
                                          const Cx<VI>* __restrict__ v, const Nbrs& nb, int X, int nsites,
                                          int ndc, int ndir, int r0, int RT, int nrhs,
                                          const double* __restrict__ P, double* tot) {
  const int per = ndc * ndc, totY = Ys ? ndir * per : 0, totE = RT * ndc, RTP = panel_stride(RT);
  const float inv_per = 1.0f / (float)per, inv_ndc = 1.0f / (float)ndc;
  const int nthr = blockDim.x, tid = threadIdx.x;
  const int GS = group_size(RT), t = tid / GS, g = tid - t * GS;
  const bool sum_on = P != nullptr && t < RT && r0 + t < nrhs;
  const double* prow = P ? P + (long)(r0 + (t < RT ? t : 0)) * nsites : nullptr;
  double acc = 0.0;
  for (int b = 0;; ++b) {
    // per pass: one (rhs, dof) panel element in every direction, YU stencil
    // entries and SU partial sums per thread
    const int e = b * nthr + tid, yb = b * YU * nthr, sb = b * SU;
    if (b * nthr >= totE && yb >= totY && (!P || sb * GS >= nsites)) break;
    const bool pe = e < totE;
    const int r = pe ? fdiv(e, inv_ndc) : 0, j = e - r * ndc;
    const bool pl = pe && r0 + r < nrhs;
    const long vrow = (long)(r0 + r) * nsites;
    Cx<R> tv[MAX_DIR], ty[YU];
    double ts[SU];
#pragma unroll
    for (int d = 0; d < MAX_DIR; ++d) {  // the direction index is a constant here: nb.s[d] stays scalar
      tv[d] = Cx<R>{0, 0};
      if (pl && d < ndir) tv[d] = ld<R>(v[(vrow + nb.s[d]) * ndc + j]);
    }
#pragma unroll
    for (int u = 0; u < YU; ++u) {
      const int ey = yb + tid + u * nthr;
      ty[u] = Cx<R>{0, 0};
      if (ey < totY) {
        const int d = fdiv(ey, inv_per), q = ey - d * per;
        ty[u] = ld<R>(Yt[((long)d * nsites + X) * per + q]);
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int Xs = g + (sb + u) * GS;
      ts[u] = (sum_on && Xs < nsites) ? prow[Xs] : 0.0;
    }
#pragma unroll
    for (int d = 0; d < MAX_DIR; ++d)
      if (pe && d < ndir) Vs[panel_at(d * ndc + j, r, RT)] = tv[d];
#pragma unroll
    for (int u = 0; u < YU; ++u) {
      const int ey = yb + tid + u * nthr;
      if (ey < totY) Ys[ey] = ty[u];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) acc += ts[u];
  }
  // zero panel rows [ndir * ndc, kpad8) for the MFMA core's last chunk pair
  const int K = ndir * ndc, kz = (kpad8(K) - K) * RTP;
  for (int e = tid; e < kz; e += nthr) Vs[K * RTP + e] = Cx<R>{0, 0};
  if (P) {
    const double sum = group_sum(acc, GS);
    if (g == 0 && t < RT) tot[t] = sum;
  }
}

// ------------------------------------------------------------------ fragments

// The outputs a thread owns after the compute core: N entries (dof i, tile
// rhs t, value), and the partial-sum slot its entries belong to.
template <class R, int N>
struct Frag {
  Cx<R> val[N];
  int i[N];
  int t[N];
  bool ok[N];  // inside ndc x RT and owned (final) by this thread
  int slot;    // row group for deterministic per-rhs partials (-1: none)
};

template <int CORE, int TI, int TR>
struct FragN {
  static constexpr int value = CORE ? 4 : TI * TR;
};

// SIMT core: acc[a][b] over (dir, j) in steps of KS (stencil blocks read from
// global memory, k-loop unrolled so several loads are in flight), then the
// k-split partial tiles are summed via LDS.
template <class R, class OT, int TI, int TR>
__device__ __forceinline__ void core_simt(Frag<R, TI * TR>& f, const Cx<OT>* __restrict__ Yt, int X, int nsites,
                                          const Cx<R>* Vs, Cx<R>* red, int ndc, int ndir, int RT, int KS) {
  const int nib = ndc / TI, nrb = RT / TR;
  const int tid = threadIdx.x;
  const int ib = tid % nib, rb = (tid / nib) % nrb, ks = tid / (nib * nrb);
  const bool valid = ks < KS;
  Cx<R> acc[TI][TR];
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b) acc[a][b] = Cx<R>{0, 0};
  if (valid) {
    const int nk = ndir * ndc;
    const int i0 = ib * TI, r0l = rb * TR;
    const long per = (long)ndc * ndc;
    const float inv_ndc = 1.0f / (float)ndc;
#pragma unroll 8
    for (int k = ks; k < nk; k += KS) {
      const int d = fdiv(k, inv_ndc), j = k - d * ndc;
      const Cx<OT>* yp = Yt + ((long)d * nsites + X) * per + (long)j * ndc + i0;
      Cx<R> y[TI], v[TR];
#pragma unroll
      for (int a = 0; a < TI; ++a) y[a] = ld<R>(yp[a]);
#pragma unroll
      for (int b = 0; b < TR; ++b) v[b] = Vs[panel_at(k, r0l + b, RT)];
#pragma unroll
      for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TR; ++b) cfma(acc[a][b], y[a], v[b]);
    }
  }
  if (KS > 1) {
    const int nslots = nib * nrb, sb = rb * nib + ib;
    if (valid && ks > 0)
#pragma unroll
      for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TR; ++b) red[((ks - 1) * nslots + sb) * TI * TR + a * TR + b] = acc[a][b];
    __syncthreads();
    if (valid && ks == 0)
      for (int q = 1; q < KS; ++q)
#pragma unroll
        for (int a = 0; a < TI; ++a)
#pragma unroll
          for (int b = 0; b < TR; ++b) acc[a][b] += red[((q - 1) * nslots + sb) * TI * TR + a * TR + b];
  }
  const bool owner = valid && ks == 0;
  f.slot = owner ? ib : -1;
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b) {
      const int e = a * TR + b;
      f.val[e] = acc[a][b];
      f.i[e] = ib * TI + a;
      f.t[e] = rb * TR + b;
      f.ok[e] = owner;
    }
}

// MFMA core: wave w owns the 16x16 tile (mt, nt) = (w % MT, w / MT).  The A
// operand (stencil blocks) comes from LDS (YL = 1) or straight from global
// memory with loads issued one chunk pair ahead (YL = 0).
template <class R, class OT, int YL>
__device__ __forceinline__ void core_mfma(Frag<R, 4>& f, Cx<R>* Ys, const Cx<OT>* __restrict__ Yt, int X,
                                          int nsites, const Cx<R>* Vs, int ndc, int ndir, int RT, int MT, int NT,
                                          int KS) {
  using M = Mfma<R>;
  typedef typename M::v4 v4;
  // the wave index is uniform over the wave: keeping it in a scalar register
  // makes the tile bookkeeping and the k-loop control scalar
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), l = threadIdx.x & 63;
  const int ntile = MT * NT, tile = w % ntile, split = w / ntile;
  // k-split factor, limited to the wave groups the workgroup actually has
  const int KSP = max(1, min(KS, (int)(blockDim.x >> 6) / ntile));
  const bool on = split < KSP;
  const int mt = on ? tile % MT : 0, nt = on ? tile / MT : 0;
  const int K = ndir * ndc, K8 = kpad8(K), nkc = K8 / 4;
  // k-split: wave group `split` takes a contiguous range of chunk pairs
  const int npairs = nkc / 2, share = (npairs + KSP - 1) / KSP;
  const int pb = on ? split * share : 0, pe = on ? min(npairs, (split + 1) * share) : 0;
  const int ia = mt * 16 + (l & 15);      // A-operand row held by this lane
  const int cb = nt * 16 + (l & 15);      // B-operand column held by this lane
  const int kk = l >> 4;
  const long per = (long)ndc * ndc;
  // Operand loads carry no condition, so the compiler can keep the next
  // chunk pair's loads in flight across the current pair's MFMAs:
  //  * rows ia >= ndc of the last 16-row tile read row ndc - 1; their outputs
  //    are dropped;
  //  * k >= K reads stencil column K - 1 against the panel's zero rows
  //    [K, K8); prefetches past the end are clamped and never used.
  const int iac = min(ia, ndc - 1);
  auto loadA = [&](int k) -> Cx<R> {
    const int kc = min(k, K - 1);
    if constexpr (YL == 1) {
      return Ys[kc * ndc + iac];
    } else {
      const int d = fdiv(kc, 1.0f / (float)ndc), j = kc - d * ndc;
      return ld<R>(Yt[((long)d * nsites + X) * per + (long)j * ndc + iac]);
    }
  };
  auto loadB = [&](int k) -> Cx<R> { return Vs[panel_at(min(k, K8 - 1), cb, RT)]; };
  // Three real products per complex one (Gauss): with P1 = Ar Br,
  // P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi):  Re = P1 - P2, Im = P3 - P1 - P2.
  // Two accumulator sets (even / odd k-chunks) keep independent MFMAs in
  // flight.
  v4 p1a = {0, 0, 0, 0}, p2a = {0, 0, 0, 0}, p3a = {0, 0, 0, 0};
  v4 p1b = {0, 0, 0, 0}, p2b = {0, 0, 0, 0}, p3b = {0, 0, 0, 0};
  if (on && pb < pe) {
    const int kb0 = 8 * pb + kk;
    Cx<R> a0 = loadA(kb0), a1 = loadA(kb0 + 4), b0 = loadB(kb0), b1 = loadB(kb0 + 4);
    for (int kc = 2 * pb; kc < 2 * pe; kc += 2) {
      const int k0 = 4 * kc + kk, k1 = k0 + 4;
      // operands of the next chunk pair, fetched before this pair's MFMAs
      const Cx<R> na0 = loadA(k0 + 8), na1 = loadA(k1 + 8);
      const Cx<R> nb0 = loadB(k0 + 8), nb1 = loadB(k1 + 8);
      p1a = M::op(a0.re, b0.re, p1a);
      p1b = M::op(a1.re, b1.re, p1b);
      p2a = M::op(a0.im, b0.im, p2a);
      p2b = M::op(a1.im, b1.im, p2b);
      p3a = M::op(a0.re + a0.im, b0.re + b0.im, p3a);
      p3b = M::op(a1.re + a1.im, b1.re + b1.im, p3b);
      a0 = na0;
      a1 = na1;
      b0 = nb0;
      b1 = nb1;
    }
  }
  f.slot = on && split == 0 ? mt * 4 + (l >> 4) : -1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = mt * 16 + M::row(l, v);
    const R q1 = p1a[v] + p1b[v], q2 = p2a[v] + p2b[v], q3 = p3a[v] + p3b[v];
    f.val[v] = Cx<R>{q1 - q2, q3 - q1 - q2};
    f.i[v] = i;
    f.t[v] = cb;
    f.ok[v] = on && split == 0 && i < ndc && cb < RT;
  }
  if (KSP > 1) {
    // wave groups 1 .. KSP-1 hand their partial tiles to group 0 through the
    // (now unused) stencil-block region; group 0 adds them in split order
    __syncthreads();
    if (on && split > 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ys[((split - 1) * ntile + tile) * 256 + l * 4 + v] = f.val[v];
    __syncthreads();
    if (on && split == 0)
      for (int q = 1; q < KSP; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) f.val[v] += Ys[((q - 1) * ntile + tile) * 256 + l * 4 + v];
  }
}

template <class R, class OT, int CORE, int TI, int TR, int YL>
__device__ __forceinline__ void run_core(Frag<R, FragN<CORE, TI, TR>::value>& f, unsigned char* raw,
                                         const LdsLayout& L, const Cx<OT>* Yt, int X, int nsites, int ndc,
                                         int ndir, int RT, int KS, int MT, int NT) {
  Cx<R>* Ys = reinterpret_cast<Cx<R>*>(raw + L.ys);
  const Cx<R>* Vs = reinterpret_cast<const Cx<R>*>(raw + L.vs);
  if constexpr (CORE == 1)
    core_mfma<R, OT, YL>(f, Ys, Yt, X, nsites, Vs, ndc, ndir, RT, MT, NT, KS);
  else
    core_simt<R, OT, TI, TR>(f, Yt, X, nsites, Vs, reinterpret_cast<Cx<R>*>(raw + L.red), ndc, ndir, RT, KS);
}

// Device-side recomputation of the LDS layout (same arithmetic as the host).
__device__ __forceinline__ LdsLayout lds_layout_dev(int core, int ylds, int RT, int TI, int TR, int KS, int MT,
                                                    int ndc, int ndir, int esz, bool plain = false) {
  LdsLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 15) & ~size_t(15);
    return at;
  };
  const size_t ysz = core && ylds ? (size_t)ndir * ndc * ndc * esz : 0;
  const size_t ksz = core && KS > 1 ? (size_t)(KS - 1) * MT * (RT / 16) * 256 * esz : 0;
  const size_t vsz = (size_t)kpad8(ndir * ndc) * panel_stride(RT) * esz;
  const bool alias = plain && ysz == 0 && ksz <= vsz;
  L.ys = take(alias ? 0 : (ysz > ksz ? ysz : ksz));
  L.vs = take(vsz);
  if (alias) L.ys = L.vs;
  const int nib = core ? 0 : ndc / TI, nrb = core ? 0 : RT / TR;
  L.red = take(core ? 0 : (size_t)(KS - 1) * nib * nrb * TI * TR * esz);
  const int nsl = core ? MT * 4 : nib;
  L.S = take(plain ? 0 : (size_t)nsl * RT * sizeof(double));
  L.sc = take(plain ? 0 : (size_t)(2 * RT + 1024) * sizeof(double));
  L.live = take(plain ? 0 : (size_t)RT * sizeof(int));
  L.O = plain ? L.vs : take((size_t)RT * ndc * esz);
  L.total = o;
  return L;
}

struct TileArgs {
  int RT, TI, TR, KS, MT, NT;
};

// out[r][X][i] = [add +] sgn * (A v)[r][X][i]
template <class R, class OT, class VI, class VO, int CORE, int TI, int TR, int YL>
__global__ __launch_bounds__(1024) void k_capply_fast(Cx<VO>* __restrict__ out, const Cx<VI>* __restrict__ in,
                                                      const Cx<VO>* add, R sgn, const Cx<OT>* __restrict__ Yt,
                                                      const int* __restrict__ nbr, int nsites, int ndc, int ndir,
                                                      TileArgs ta, int nrhs, const int* act) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const LdsLayout L = lds_layout_dev(CORE, YL, ta.RT, TI, TR, ta.KS, ta.MT, ndc, ndir, sizeof(Cx<R>), true);
  const int X = blockIdx.x, r0 = blockIdx.y * ta.RT;
  if (act) {  // a tile of converged rhs has nothing to write
    // every thread reads the same flags (uniform, scalar loads): no barrier
    // and no LDS of the block-wide reduction
    int any = 0;
    for (int t = 0; t < ta.RT && r0 + t < nrhs; ++t) any |= act[r0 + t];
    if (!any) return;
  }
  const Nbrs nb = load_nbrs(nbr, X, nsites, ndir);
  stage_all<R, OT, VI>(CORE == 1 && YL == 1 ? reinterpret_cast<Cx<R>*>(smem_raw + L.ys) : nullptr,
                       reinterpret_cast<Cx<R>*>(smem_raw + L.vs), Yt, in, nb, X, nsites, ndc, ndir, r0, ta.RT,
                       nrhs, nullptr, nullptr);
  __syncthreads();
  Frag<R, FragN<CORE, TI, TR>::value> f;
  run_core<R, OT, CORE, TI, TR, YL>(f, smem_raw, L, Yt, X, nsites, ndc, ndir, ta.RT, ta.KS, ta.MT, ta.NT);
  __syncthreads();  // the output tile O overwrites the panel every wave has read
  Cx<R>* O = reinterpret_cast<Cx<R>*>(smem_raw + L.O);
  frag_to_tile<R, FragN<CORE, TI, TR>::value>(O, f, ndc);
  const float inv_ndc = 1.0f / (float)ndc;
  for (int e = threadIdx.x; e < ta.RT * ndc; e += blockDim.x) {
    const int t = fdiv(e, inv_ndc), i = e - t * ndc, rr = r0 + t;
    if (rr >= nrhs || !is_active(act, rr)) continue;
    const long o = ((long)rr * nsites + X) * ndc + i;
    Cx<R> res = sgn * O[e];
    if (add) res += ld<R>(add[o]);
    out[o] = st<VO>(res);
  }
}


// ------------------------------------------------------------------ fused CGNE

struct CgneState {
  double* rr;         // [2][nrhs]  ||r||^2 at the start of iteration k (slot k & 1)
  double* target;     // [nrhs]     (tol ||b||)^2
  int* act;           // [2][nrhs]  active during iteration k (slot k & 1)
  int* its;           // [nrhs]     iterations of the current call
  int* tot;           // [nrhs]     iterations over all calls
  int* calls;         // [nrhs]     calls while active
  const int* parent;  // rhs the caller wants solved
  double* PA;         // [nrhs][nsites] partial ||r||^2
  double* PB;         // [nrhs][nsites] partial ||p||^2
};

// Scatter a thread's fragment into the workgroup's output tile O[t*ndc + i]
// (every (t < RT, i < ndc) entry is owned by exactly one thread), so the
// epilogue can walk the tile dof-fastest with coalesced global accesses.
template <class R, int N>
__device__ __forceinline__ void frag_to_tile(Cx<R>* O, const Frag<R, N>& f, int ndc) {
#pragma unroll
  for (int e = 0; e < N; ++e)
    if (f.ok[e]) O[f.t[e] * ndc + f.i[e]] = f.val[e];
  __syncthreads();
}

// P[r0 + t][X] = sum_i |O[t*ndc + i]|^2: lane g of rhs group t adds dofs
// g, g + GS, ... in order, then the group's lanes are added by group_sum().
template <class R>
__device__ __forceinline__ void tile_partials(double* P, const Cx<R>* O, int X, int nsites, int nrhs, int r0,
                                              int RT, int ndc) {
  __syncthreads();
  const int GS = group_size(RT), t = threadIdx.x / GS, g = threadIdx.x - t * GS;
  double s = 0.0;
  if (t < RT)
    for (int i = g; i < ndc; i += GS) s += (double)norm2(O[t * ndc + i]);
  s = group_sum(s, GS);
  if (g == 0 && t < RT && r0 + t < nrhs) P[(long)(r0 + t) * nsites + X] = s;
}

// init 1: x = 0, r = b, PA = partial ||b||^2 (one thread per rhs, dofs in order).
template <class R>
__global__ __launch_bounds__(256) void k_cgne_init1(Cx<R>* x, Cx<R>* r, const Cx<R>* b, int nsites, int ndc,
                                                     int nrhs, CgneState s) {
  const int X = blockIdx.x;
  for (int rr = threadIdx.x; rr < nrhs; rr += blockDim.x) {
    const bool on = s.parent == nullptr || s.parent[rr] != 0;
    double acc = 0.0;
    for (int i = 0; i < ndc; ++i) {
      const long o = ((long)rr * nsites + X) * ndc + i;
      const Cx<R> v = b[o];
      if (on) {
        x[o] = Cx<R>{0, 0};
        r[o] = v;
      }
      acc += (double)norm2(v);
    }
    s.PA[(long)rr * nsites + X] = acc;
  }
}

// Common prologue of the CGNE kernels: stages the operands with the previous
// kernel's partial sums, whose per-rhs totals land in tot[0 .. RT).
template <class R, class OT, int CORE, int YL>
__device__ __forceinline__ void cgne_stage(unsigned char* raw, const LdsLayout& L, const Cx<OT>* Y, const Cx<R>* v,
                                           const Nbrs& nb, int X, int nsites, int ndc, int ndir, int r0, int RT,
                                           int nrhs, const double* P, double* tot) {
  stage_all<R, OT, R>(CORE == 1 && YL == 1 ? reinterpret_cast<Cx<R>*>(raw + L.ys) : nullptr,
                      reinterpret_cast<Cx<R>*>(raw + L.vs), Y, v, nb, X, nsites, ndc, ndir, r0, RT, nrhs, P, tot);
}

// Prefetch of the thread's first epilogue element (e = threadIdx.x of the
// RT x ndc output tile).
struct FirstElem {
  bool on;
  long o;
};

__device__ __forceinline__ FirstElem first_elem(int X, int nsites, int ndc, int r0, int RT, int nrhs) {
  const int e = threadIdx.x, t = fdiv(e, 1.0f / (float)ndc), i = e - t * ndc;
  FirstElem f;
  f.on = e < RT * ndc && r0 + t < nrhs;
  f.o = ((long)(r0 + t) * nsites + X) * ndc + i;
  return f;
}

// init 2: rr_0, target, act_0 ; p = A^dag r ; PB = partial ||p||^2
template <class R, class OT, int CORE, int TI, int TR, int YL>
__global__ __launch_bounds__(1024) void k_cgne_init2(Cx<R>* p, const Cx<R>* r, const Cx<OT>* Yd, const int* nbr,
                                                      int nsites, int ndc, int ndir, TileArgs ta, int nrhs,
                                                      CgneState s, double tol2) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const LdsLayout L = lds_layout_dev(CORE, YL, ta.RT, TI, TR, ta.KS, ta.MT, ndc, ndir, sizeof(Cx<R>));
  double* sc = reinterpret_cast<double*>(smem_raw + L.sc);
  int* live = reinterpret_cast<int*>(smem_raw + L.live);
  const int X = blockIdx.x, r0 = blockIdx.y * ta.RT, RT = ta.RT;
  const Nbrs nb = load_nbrs(nbr, X, nsites, ndir);
  cgne_stage<R, OT, CORE, YL>(smem_raw, L, Yd, r, nb, X, nsites, ndc, ndir, r0, RT, nrhs, s.PA, sc + 2 * RT);
  __syncthreads();
  if (threadIdx.x < RT) {
    const int t = threadIdx.x, rr = r0 + t;
    const double b2 = sc[2 * RT + t];
    int lv = 0;
    if (rr < nrhs) {
      const double tg = tol2 * b2;
      const bool on = s.parent == nullptr || s.parent[rr] != 0;
      lv = on && b2 > tg && b2 > 0.0;
      if (X == 0) {
        s.rr[rr] = b2;
        s.target[rr] = tg;
        s.act[rr] = lv;
        s.its[rr] = 0;
        if (on) s.calls[rr] += 1;
      }
    }
    live[t] = lv;
  }
  Frag<R, FragN<CORE, TI, TR>::value> f;
  run_core<R, OT, CORE, TI, TR, YL>(f, smem_raw, L, Yd, X, nsites, ndc, ndir, RT, ta.KS, ta.MT, ta.NT);
  Cx<R>* O = reinterpret_cast<Cx<R>*>(smem_raw + L.O);
  frag_to_tile<R, FragN<CORE, TI, TR>::value>(O, f, ndc);
  const float inv_ndc = 1.0f / (float)ndc;
  for (int e = threadIdx.x; e < RT * ndc; e += blockDim.x) {
    const int t = fdiv(e, inv_ndc), i = e - t * ndc, rr = r0 + t;
    if (rr >= nrhs || !live[t]) {
      O[e] = Cx<R>{0, 0};
      continue;
    }
    p[((long)rr * nsites + X) * ndc + i] = O[e];
  }
  tile_partials<R>(s.PB, O, X, nsites, nrhs, r0, RT, ndc);
}


// A_k: alpha = rr_k/||p||^2 ; q = A p ; x += alpha p ; r -= alpha q ; PA = partial ||r||^2
template <class R, class OT, int CORE, int TI, int TR, int YL>
__global__ __launch_bounds__(1024) void k_cgne_A(Cx<R>* x, Cx<R>* r, const Cx<R>* p, const Cx<OT>* Yt,
                                                  const int* nbr, int nsites, int ndc, int ndir, TileArgs ta,
                                                  int nrhs, CgneState s, int k) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const LdsLayout L = lds_layout_dev(CORE, YL, ta.RT, TI, TR, ta.KS, ta.MT, ndc, ndir, sizeof(Cx<R>));
  double* sc = reinterpret_cast<double*>(smem_raw + L.sc);
  int* live = reinterpret_cast<int*>(smem_raw + L.live);
  const int X = blockIdx.x, r0 = blockIdx.y * ta.RT, RT = ta.RT, sl = (k & 1) * nrhs;
  // Nothing to do once every rhs of the tile has stopped (the host polls the
  // flags asynchronously, so a few iterations past convergence are
  // launched).  The flags are tested at the barrier after the staging, so
  // their load overlaps the staging loads (which only read).
  const int mine = threadIdx.x < RT && r0 + (int)threadIdx.x < nrhs ? s.act[sl + r0 + threadIdx.x] : 0;
  const Nbrs nb = load_nbrs(nbr, X, nsites, ndir);
  const FirstElem fe = first_elem(X, nsites, ndc, r0, RT, nrhs);
  Cx<R> x0{0, 0}, r0v{0, 0};
  if (fe.on) {
    x0 = x[fe.o];
    r0v = r[fe.o];
  }
  cgne_stage<R, OT, CORE, YL>(smem_raw, L, Yt, p, nb, X, nsites, ndc, ndir, r0, RT, nrhs, s.PB, sc + 2 * RT);
  if (!__syncthreads_or(mine)) return;
  if (threadIdx.x < RT) {
    const int t = threadIdx.x, rr = r0 + t;
    const double pp = sc[2 * RT + t];
    const int lv = rr < nrhs ? s.act[sl + rr] : 0;
    live[t] = lv;
    sc[RT + t] = lv ? s.rr[sl + rr] / pp : 0.0;  // alpha
  }
  Frag<R, FragN<CORE, TI, TR>::value> f;
  run_core<R, OT, CORE, TI, TR, YL>(f, smem_raw, L, Yt, X, nsites, ndc, ndir, RT, ta.KS, ta.MT, ta.NT);
  const Cx<R>* Vs = reinterpret_cast<const Cx<R>*>(smem_raw + L.vs);
  Cx<R>* O = reinterpret_cast<Cx<R>*>(smem_raw + L.O);
  frag_to_tile<R, FragN<CORE, TI, TR>::value>(O, f, ndc);
  const float inv_ndc = 1.0f / (float)ndc;
  for (int e = threadIdx.x; e < RT * ndc; e += blockDim.x) {
    const int t = fdiv(e, inv_ndc), i = e - t * ndc, rr = r0 + t;
    if (rr >= nrhs || !live[t]) {
      O[e] = Cx<R>{0, 0};
      continue;
    }
    const R al = (R)sc[RT + t];
    const long o = ((long)rr * nsites + X) * ndc + i;
    const bool first = e == (int)threadIdx.x;
    const Cx<R> xv = first ? x0 : x[o];
    const Cx<R> rv_old = first ? r0v : r[o];
    const Cx<R> pv = Vs[panel_at(i, t, RT)];  // direction 0 is the site itself
    x[o] = xv + al * pv;
    const Cx<R> rv = rv_old - al * O[e];
    r[o] = rv;
    O[e] = rv;
  }
  tile_partials<R>(s.PA, O, X, nsites, nrhs, r0, RT, ndc);
}


// B_k: ||r||^2 -> stop test, beta ; p = A^dag r + beta p ; PB = partial ||p||^2
template <class R, class OT, int CORE, int TI, int TR, int YL>
__global__ __launch_bounds__(1024) void k_cgne_B(Cx<R>* p, const Cx<R>* r, const Cx<OT>* Yd, const int* nbr,
                                                  int nsites, int ndc, int ndir, TileArgs ta, int nrhs,
                                                  CgneState s, int k) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const LdsLayout L = lds_layout_dev(CORE, YL, ta.RT, TI, TR, ta.KS, ta.MT, ndc, ndir, sizeof(Cx<R>));
  double* sc = reinterpret_cast<double*>(smem_raw + L.sc);
  int* live = reinterpret_cast<int*>(smem_raw + L.live);
  const int X = blockIdx.x, r0 = blockIdx.y * ta.RT, RT = ta.RT;
  const int sl = (k & 1) * nrhs, sn = ((k + 1) & 1) * nrhs;
  // flags tested after the staging, as in k_cgne_A
  const int mine = threadIdx.x < RT && r0 + (int)threadIdx.x < nrhs ? s.act[sl + r0 + threadIdx.x] : 0;
  const Nbrs nb = load_nbrs(nbr, X, nsites, ndir);
  const FirstElem fe = first_elem(X, nsites, ndc, r0, RT, nrhs);
  Cx<R> p0{0, 0};
  if (fe.on) p0 = p[fe.o];
  cgne_stage<R, OT, CORE, YL>(smem_raw, L, Yd, r, nb, X, nsites, ndc, ndir, r0, RT, nrhs, s.PA, sc + 2 * RT);
  if (!__syncthreads_or(mine)) {
    // every rhs of the tile has stopped: carry the state into the next slot
    if (X == 0 && threadIdx.x < RT && r0 + (int)threadIdx.x < nrhs) {
      const int rr = r0 + threadIdx.x;
      s.rr[sn + rr] = s.rr[sl + rr];
      s.act[sn + rr] = 0;
    }
    return;
  }
  if (threadIdx.x < RT) {
    const int t = threadIdx.x, rr = r0 + t;
    const double rn = sc[2 * RT + t];
    int lv = 0;
    double beta = 0.0;
    if (rr < nrhs) {
      const int was = s.act[sl + rr];
      const double ro = s.rr[sl + rr];
      lv = was && rn > s.target[rr];
      beta = lv ? rn / ro : 0.0;
      if (X == 0) {
        s.rr[sn + rr] = was ? rn : ro;
        s.act[sn + rr] = lv;
        if (was) {
          s.its[rr] += 1;
          s.tot[rr] += 1;
        }
      }
    }
    live[t] = lv;
    sc[RT + t] = beta;
  }
  Frag<R, FragN<CORE, TI, TR>::value> f;
  run_core<R, OT, CORE, TI, TR, YL>(f, smem_raw, L, Yd, X, nsites, ndc, ndir, RT, ta.KS, ta.MT, ta.NT);
  Cx<R>* O = reinterpret_cast<Cx<R>*>(smem_raw + L.O);
  frag_to_tile<R, FragN<CORE, TI, TR>::value>(O, f, ndc);
  const float inv_ndc = 1.0f / (float)ndc;
  for (int e = threadIdx.x; e < RT * ndc; e += blockDim.x) {
    const int t = fdiv(e, inv_ndc), i = e - t * ndc, rr = r0 + t;
    if (rr >= nrhs || !live[t]) {
      O[e] = Cx<R>{0, 0};
      continue;
    }
    const R be = (R)sc[RT + t];
    const long o = ((long)rr * nsites + X) * ndc + i;
    const Cx<R> pold = e == (int)threadIdx.x ? p0 : p[o];
    const Cx<R> pv = O[e] + be * pold;
    p[o] = pv;
    O[e] = pv;
  }
  tile_partials<R>(s.PB, O, X, nsites, nrhs, r0, RT, ndc);
}


}  // namespace kdmg
