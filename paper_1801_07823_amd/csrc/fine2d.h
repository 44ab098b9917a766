// Fine-level kernels for the 2D U(1) staggered operator in Kahler-Dirac block
// layout.
//
// Layout.  The L_x x L_t lattice is cut into 2x2 Kahler-Dirac blocks anchored
// at even coordinates (Sec. 2.1).  Block X = (X0, X1) has parity
// p = (X0 + X1) & 1 and index b = X1 * (B_x/2) + X0/2 within its parity, so a
// vector is [rhs][p][b][s] with s = (x0 & 1) + 2 (x1 & 1) the site inside the
// block; each block's four complex values are contiguous (64 B in FP64, 32 B
// in FP32) and consecutive threads read consecutive blocks.  The Schur space
// of the solver is the p = 0 half.
//
// Links.  Per block 8 complex values with the staggered phase eta_mu(x), the
// factor 1/2 of eq. "staggeredD" and the antiperiodic sign folded in
// (U~_mu(x) = 1/2 eta_mu(x) bc_mu(x) U_mu(x)); eta_mu(x - mu) = eta_mu(x)
// makes the backward hop -U~_mu(x - mu)^* psi(x - mu).  Entries 0..3 are the
// intra-block links U~_0(s0), U~_1(s0), U~_1(s1), U~_0(s2) (the part of B);
// entries 4..7 the forward inter-block links U~_0(s1), U~_0(s3), U~_1(s2),
// U~_1(s3) (the part of C).
//
// Operators.  D = B + C with B = m + intra-block hops (Sec. 2.1).  In block
// site order the even sites (eps = +1) are s0, s3 and the odd s1, s2, so
// B = [[m, K], [-K^dag, m]] with K = [[a, c], [-d^*, -f^*]] in the links
// (a, c, d, f) = entries 0..3, and
//   B^-1 b = ( S_e^-1 (m b_e - K b_o),  S_o^-1 (m b_o + K^dag b_e) ),
//   S_e = m^2 + K K^dag,  S_o = m^2 + K^dag K  (2x2 Hermitian positive).
// B^-1 is recomputed from the four intra-block links in every kernel that
// needs it instead of being stored.
#pragma once
#include <type_traits>

#include "common.h"
#include "blas.h"

namespace kdmg {

struct Geo2 {
  int Lx, Lt;   // sites
  int Bx, Bt;   // KD blocks
  int hBx;      // Bx / 2
  int Nb2;      // blocks per parity
  long half;    // complex entries in one parity half (= 4 * Nb2)
};

__host__ __device__ __forceinline__ void blk_coords(const Geo2& g, int p, int b, int& X0, int& X1) {
  X1 = b / g.hBx;
  X0 = 2 * (b % g.hBx) + ((p + X1) & 1);
}
__host__ __device__ __forceinline__ int blk_index(const Geo2& g, int X0, int X1) {
  return X1 * g.hBx + (X0 >> 1);
}
// chirality of site s in a block: 0 for eps=+1 (s0, s3), 1 for eps=-1 (s1, s2)
__host__ __device__ __forceinline__ int chir2(int s) { return (s == 1 || s == 2) ? 1 : 0; }

// Workgroup index renumbered so that each of the 8 XCDs (which receive
// workgroups round-robin, XCD = index % 8, each with its own L2) takes one
// contiguous range of the grid: data shared by neighbouring workgroups (the
// rows x1 +- 1 of the Dslash, the 128-byte lines split between neighbouring
// aggregates of the transfers) is then read through the same L2.
__device__ __forceinline__ int xcd_block(unsigned b, unsigned nb) {
  return (int)((nb % 8u == 0) ? (b & 7u) * (nb >> 3) + (b >> 3) : b);
}

// Two adjacent complex values, loaded or stored as one 8-byte (FP16) or
// 16-byte (FP32) access.
struct alignas(8) HPair {
  Cx<_Float16> a, b;
};
struct alignas(16) FPair {
  Cx<float> a, b;
};

// A block's four values (32 B in FP32: two 16-byte accesses; FP64: four).
// p is 4-entry aligned: every block-layout vector here is.
template <class R, class VT>
__device__ __forceinline__ void load4(const Cx<VT>* p, Cx<R> v[4]) {
  if constexpr (std::is_same<VT, float>::value) {
    const FPair a = reinterpret_cast<const FPair*>(p)[0], b = reinterpret_cast<const FPair*>(p)[1];
    v[0] = ld<R>(a.a);
    v[1] = ld<R>(a.b);
    v[2] = ld<R>(b.a);
    v[3] = ld<R>(b.b);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = ld<R>(p[s]);
  }
}
template <class R, class VT>
__device__ __forceinline__ void store4(Cx<VT>* p, const Cx<R> v[4]) {
  if constexpr (std::is_same<VT, float>::value) {
    FPair a, b;
    a.a = st<VT>(v[0]);
    a.b = st<VT>(v[1]);
    b.a = st<VT>(v[2]);
    b.b = st<VT>(v[3]);
    reinterpret_cast<FPair*>(p)[0] = a;
    reinterpret_cast<FPair*>(p)[1] = b;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) p[s] = st<VT>(v[s]);
  }
}

template <class R, class LT>
__device__ __forceinline__ void load_intra(const Cx<LT>* L, Cx<R> k[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) k[i] = ld<R>(L[i]);
}

// out = B^-1 in for one block (links a, c, d, f = L[0..3])
template <class R>
__device__ __forceinline__ void binv_block(const Cx<R> L[4], R m, const Cx<R> in[4], Cx<R> out[4]) {
  const Cx<R> K00 = L[0], K01 = L[1], K10 = -conj(L[2]), K11 = -conj(L[3]);
  const R m2 = m * m;
  const R se00 = m2 + norm2(K00) + norm2(K01);
  const R se11 = m2 + norm2(K10) + norm2(K11);
  const Cx<R> se01 = K00 * conj(K10) + K01 * conj(K11);
  const R so00 = m2 + norm2(K00) + norm2(K10);
  const R so11 = m2 + norm2(K01) + norm2(K11);
  const Cx<R> so01 = conj(K00) * K01 + conj(K10) * K11;
  const Cx<R> ye0 = m * in[0] - (K00 * in[1] + K01 * in[2]);
  const Cx<R> ye1 = m * in[3] - (K10 * in[1] + K11 * in[2]);
  const Cx<R> yo0 = m * in[1] + (conj(K00) * in[0] + conj(K10) * in[3]);
  const Cx<R> yo1 = m * in[2] + (conj(K01) * in[0] + conj(K11) * in[3]);
  const R de = R(1) / (se00 * se11 - norm2(se01));
  const R dd = R(1) / (so00 * so11 - norm2(so01));
  out[0] = de * (se11 * ye0 - se01 * ye1);
  out[3] = de * (se00 * ye1 - conj(se01) * ye0);
  out[1] = dd * (so11 * yo0 - so01 * yo1);
  out[2] = dd * (so00 * yo1 - conj(so01) * yo0);
}

// out = B in for one block
template <class R>
__device__ __forceinline__ void b_block(const Cx<R> L[4], R m, const Cx<R> in[4], Cx<R> out[4]) {
  out[0] = m * in[0] + L[0] * in[1] + L[1] * in[2];
  out[1] = m * in[1] - conj(L[0]) * in[0] + L[2] * in[3];
  out[2] = m * in[2] - conj(L[1]) * in[0] + L[3] * in[3];
  out[3] = m * in[3] - conj(L[2]) * in[1] - conj(L[3]) * in[2];
}

// Neighbour blocks of (p, b): indices within parity 1-p.
struct Nbr2 {
  int xp, xm, tp, tm;  // X+0, X-0, X+1, X-1
  int X0, X1;
};
__device__ __forceinline__ Nbr2 nbr2(const Geo2& g, int p, int b) {
  Nbr2 n;
  blk_coords(g, p, b, n.X0, n.X1);
  const int x0p = n.X0 + 1 == g.Bx ? 0 : n.X0 + 1, x0m = n.X0 == 0 ? g.Bx - 1 : n.X0 - 1;
  const int x1p = n.X1 + 1 == g.Bt ? 0 : n.X1 + 1, x1m = n.X1 == 0 ? g.Bt - 1 : n.X1 - 1;
  n.xp = blk_index(g, x0p, n.X1);
  n.xm = blk_index(g, x0m, n.X1);
  n.tp = blk_index(g, n.X0, x1p);
  n.tm = blk_index(g, n.X0, x1m);
  return n;
}

// out = C in on block (p, b); `in` is the parity-(1-p) half of the source
// (already offset to this rhs).  eps_in multiplies the source by eps(s).
template <class R, class LT, class VT>
__device__ __forceinline__ void hop_block(const Geo2& g, int p, int b, const Nbr2& n,
                                          const Cx<LT>* links, const Cx<VT>* in, bool eps_in,
                                          Cx<R> out[4]) {
  const int q = 1 - p;
  const Cx<LT>* Lo = links + ((size_t)p * g.Nb2 + b) * 8;
  const Cx<LT>* Lxm = links + ((size_t)q * g.Nb2 + n.xm) * 8;
  const Cx<LT>* Ltm = links + ((size_t)q * g.Nb2 + n.tm) * 8;
  Cx<R> xp0, xp2, xm1, xm3, tp0, tp1, tm2, tm3;
  if constexpr (std::is_same<VT, float>::value) {
    // whole neighbour blocks in 16-byte accesses (the unused halves come from
    // the same cache lines)
    Cx<R> a[4], c[4], e[4], f[4];
    load4<R, VT>(in + 4L * n.xp, a);
    load4<R, VT>(in + 4L * n.xm, c);
    load4<R, VT>(in + 4L * n.tp, e);
    load4<R, VT>(in + 4L * n.tm, f);
    xp0 = a[0], xp2 = a[2], xm1 = c[1], xm3 = c[3], tp0 = e[0], tp1 = e[1], tm2 = f[2], tm3 = f[3];
  } else {
    xp0 = ld<R>(in[4 * n.xp + 0]), xp2 = ld<R>(in[4 * n.xp + 2]);
    xm1 = ld<R>(in[4 * n.xm + 1]), xm3 = ld<R>(in[4 * n.xm + 3]);
    tp0 = ld<R>(in[4 * n.tp + 0]), tp1 = ld<R>(in[4 * n.tp + 1]);
    tm2 = ld<R>(in[4 * n.tm + 2]), tm3 = ld<R>(in[4 * n.tm + 3]);
  }
  if (eps_in) { xp2 = -xp2; xm1 = -xm1; tp1 = -tp1; tm2 = -tm2; }
  out[0] = -(cmul_conj(ld<R>(Lxm[4]), xm1) + cmul_conj(ld<R>(Ltm[6]), tm2));
  out[1] = ld<R>(Lo[4]) * xp0 - cmul_conj(ld<R>(Ltm[7]), tm3);
  out[2] = ld<R>(Lo[6]) * tp0 - cmul_conj(ld<R>(Lxm[5]), xm3);
  out[3] = ld<R>(Lo[5]) * xp2 + ld<R>(Lo[7]) * tp1;
}

__device__ __forceinline__ float eps2(int s) { return (s == 1 || s == 2) ? -1.f : 1.f; }

// ------------------------------------------------------------------ kernels
// Grid: x over blocks of one parity, y = rhs, z = parity offset (p = p0 + z).
// Every vector argument is the base of a [p][b][s] layout (parity-0 half
// first); `s*` is its per-rhs stride in complex entries.  A vector that only
// holds the even half (the Schur space) has stride `half` and is only ever
// addressed at p = 0.

// out = [add +] [eps] B^-1 in ; optionally out2 = B^-1 out
template <class R, class LT, class VT>
__global__ __launch_bounds__(256) void k_binv(Cx<VT>* out, long so, Cx<VT>* out2, long so2,
                                               const Cx<VT>* in, long si, const Cx<VT>* add, long sa,
                                               const Cx<LT>* links, Geo2 g, int p0, R m, int eps_out,
                                               const int* act) {
  const int b = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, p = p0 + blockIdx.z;
  if (b >= g.Nb2 || !is_active(act, r)) return;
  Cx<R> L[4], v[4], w[4];
  load_intra<R, LT>(links + ((size_t)p * g.Nb2 + b) * 8, L);
  const long o = (long)p * g.half + 4L * b;
  load4<R, VT>(in + r * si + o, v);
  binv_block<R>(L, m, v, w);
  if (eps_out) {
    w[1] = -w[1];
    w[2] = -w[2];
  }
  if (add) {
    Cx<R> a[4];
    load4<R, VT>(add + r * sa + o, a);
#pragma unroll
    for (int s = 0; s < 4; ++s) w[s] += a[s];
  }
  store4<R, VT>(out + r * so + o, w);
  if (out2) {
    binv_block<R>(L, m, w, v);
    store4<R, VT>(out2 + r * so2 + o, v);
  }
}

// mode 0: out = [add +] [c2 add2 +] sgn C in ;  mode 1: out = B^-1 (C in)
template <class R, class LT, class VT>
__global__ __launch_bounds__(256) void k_hop(Cx<VT>* out, long so, const Cx<VT>* in, long si,
                                              const Cx<VT>* add, long sa, const Cx<VT>* add2,
                                              long sa2, R c2, R sgn, const Cx<LT>* links, Geo2 g,
                                              int p0, R m, int mode, int eps_in, const int* act) {
  const int b = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, p = p0 + blockIdx.z;
  if (b >= g.Nb2 || !is_active(act, r)) return;
  const Nbr2 n = nbr2(g, p, b);
  const Cx<VT>* src = in + r * si + (long)(1 - p) * g.half;
  Cx<R> h[4];
  hop_block<R, LT, VT>(g, p, b, n, links, src, eps_in != 0, h);
  const long o = (long)p * g.half + 4L * b;
  if (mode == 1) {
    Cx<R> L[4], w[4];
    load_intra<R, LT>(links + ((size_t)p * g.Nb2 + b) * 8, L);
    binv_block<R>(L, m, h, w);
    store4<R, VT>(out + r * so + o, w);
    return;
  }
  Cx<R> v[4], a[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = sgn * h[s];
  if (add) {
    load4<R, VT>(add + r * sa + o, a);
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] += a[s];
  }
  if (add2) {
    load4<R, VT>(add2 + r * sa2 + o, a);
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] += c2 * a[s];
  }
  store4<R, VT>(out + r * so + o, v);
}

// out = D in on full block-layout vectors; with `sub`, out = sub - D in.
template <class R, class LT, class VT>
__global__ __launch_bounds__(256) void k_dslash_blk(Cx<VT>* out, long so, const Cx<VT>* in, long si,
                                                    const Cx<VT>* sub, long ss, const Cx<LT>* links,
                                                    Geo2 g, R m, const int* act) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, p = blockIdx.z;
  if (b >= g.Nb2 || !is_active(act, r)) return;
  const Nbr2 n = nbr2(g, p, b);
  const Cx<VT>* src = in + r * si;
  Cx<R> h[4], L[4], v[4], w[4];
  hop_block<R, LT, VT>(g, p, b, n, links, src + (long)(1 - p) * g.half, false, h);
  load_intra<R, LT>(links + ((size_t)p * g.Nb2 + b) * 8, L);
  const long o = (long)p * g.half + 4L * b;
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = ld<R>(src[o + s]);
  b_block<R>(L, m, v, w);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    Cx<R> d = w[s] + h[s];
    if (sub) d = ld<R>(sub[r * ss + o + s]) - d;
    out[r * so + o + s] = st<VT>(d);
  }
}


// D in natural site order: one thread per site and RB right-hand sides (the
// site's four links are loaded once for all of them; every vector load of
// the RB rhs is issued before any is used).  links_nat[mu][site] folded.
template <class R, class LT, class VT, int RB>
__global__ __launch_bounds__(256) void k_dslash_nat(Cx<VT>* __restrict__ out, const Cx<VT>* __restrict__ in,
                                                    const Cx<LT>* __restrict__ Ux,
                                                    const Cx<LT>* __restrict__ Ut, int Lx, int Lt,
                                                    long vol, R m, int nrhs) {
  const long x = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * RB;
  if (x >= vol) return;
  const int x1 = (int)(x / Lx), x0 = (int)(x - (long)x1 * Lx);
  const int x0p = x0 + 1 == Lx ? 0 : x0 + 1, x0m = x0 == 0 ? Lx - 1 : x0 - 1;
  const int x1p = x1 + 1 == Lt ? 0 : x1 + 1, x1m = x1 == 0 ? Lt - 1 : x1 - 1;
  const long ixp = (long)x1 * Lx + x0p, ixm = (long)x1 * Lx + x0m;
  const long itp = (long)x1p * Lx + x0, itm = (long)x1m * Lx + x0;
  const Cx<R> ux = ld<R>(Ux[x]), uxm = ld<R>(Ux[ixm]), ut = ld<R>(Ut[x]), utm = ld<R>(Ut[itm]);
  Cx<R> v0[RB], v1[RB], v2[RB], v3[RB], v4[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const bool on = r0 + b < nrhs;
    const Cx<VT>* v = in + (long)(r0 + b) * vol;
    v0[b] = on ? ld<R>(v[x]) : Cx<R>{0, 0};
    v1[b] = on ? ld<R>(v[ixp]) : Cx<R>{0, 0};
    v2[b] = on ? ld<R>(v[ixm]) : Cx<R>{0, 0};
    v3[b] = on ? ld<R>(v[itp]) : Cx<R>{0, 0};
    v4[b] = on ? ld<R>(v[itm]) : Cx<R>{0, 0};
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (r0 + b >= nrhs) continue;
    Cx<R> acc = m * v0[b];
    acc += ux * v1[b];
    acc -= cmul_conj(uxm, v2[b]);
    acc += ut * v3[b];
    acc -= cmul_conj(utm, v4[b]);
    out[(long)(r0 + b) * vol + x] = st<VT>(acc);
  }
}

// Mixed-precision D in natural site order with two sites per thread: the
// sites x, x + 1 (x even) of a thread and their x-neighbours x - 1, x + 2 lie
// in three aligned pairs, and the t-neighbours in two more, so every rhs
// costs five 16-byte loads and one 16-byte store (FP32 complex), the links
// four 8-byte loads (FP16 complex pairs) per thread.  Same arithmetic per
// site as k_dslash_nat.  Lx even; vectors 16-byte aligned per rhs (vol even).
template <int RB>
__global__ __launch_bounds__(256) void k_dslash_nat2(Cx<float>* __restrict__ out, const Cx<float>* __restrict__ in,
                                                     const Cx<_Float16>* __restrict__ Ux,
                                                     const Cx<_Float16>* __restrict__ Ut, int Lx, int Lt, long vol,
                                                     float m, int nrhs) {
  const long pr = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * RB;
  const long x = 2 * pr;
  if (x >= vol) return;
  const int x1 = (int)(x / Lx), x0 = (int)(x - (long)x1 * Lx);
  const int x0l = x0 == 0 ? Lx - 2 : x0 - 2, x0r = x0 + 2 == Lx ? 0 : x0 + 2;
  const int x1p = x1 + 1 == Lt ? 0 : x1 + 1, x1m = x1 == 0 ? Lt - 1 : x1 - 1;
  // pair indices (a pair holds sites 2k, 2k + 1)
  const long pc = x >> 1, pl = ((long)x1 * Lx + x0l) >> 1, prr = ((long)x1 * Lx + x0r) >> 1;
  const long pu = ((long)x1p * Lx + x0) >> 1, pd = ((long)x1m * Lx + x0) >> 1;
  const HPair* Uxp = reinterpret_cast<const HPair*>(Ux);
  const HPair* Utp = reinterpret_cast<const HPair*>(Ut);
  const HPair uxc = Uxp[pc], uxl = Uxp[pl], utc = Utp[pc], utd = Utp[pd];
  const Cx<float> uxa = ld<float>(uxc.a), uxb = ld<float>(uxc.b), uxm = ld<float>(uxl.b);
  const Cx<float> uta = ld<float>(utc.a), utb = ld<float>(utc.b), utma = ld<float>(utd.a), utmb = ld<float>(utd.b);
  const FPair* vp = reinterpret_cast<const FPair*>(in);
  const long hv = vol >> 1;
  FPair c[RB], l[RB], rr[RB], u[RB], d[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const long row = (long)(r0 + b < nrhs ? r0 + b : r0) * hv;
    c[b] = vp[row + pc];
    l[b] = vp[row + pl];
    rr[b] = vp[row + prr];
    u[b] = vp[row + pu];
    d[b] = vp[row + pd];
  }
  FPair* op = reinterpret_cast<FPair*>(out);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (r0 + b >= nrhs) continue;
    FPair o;
    // site x: +x -> x + 1, -x -> x - 1 (left pair's second), +-t
    Cx<float> acc = m * c[b].a;
    acc += uxa * c[b].b;
    acc -= cmul_conj(uxm, l[b].b);
    acc += uta * u[b].a;
    acc -= cmul_conj(utma, d[b].a);
    o.a = acc;
    // site x + 1: +x -> x + 2 (right pair's first), -x -> x
    acc = m * c[b].b;
    acc += uxb * rr[b].a;
    acc -= cmul_conj(uxa, c[b].a);
    acc += utb * u[b].b;
    acc -= cmul_conj(utmb, d[b].b);
    o.b = acc;
    op[(long)(r0 + b) * hv + pc] = o;
  }
}

// ------------------------------------------------------- Naik three-link hops
// The Naik-improved operator (Sec. 2.1, eq. "freehisq") adds to every site
// the hops x -> x +- 3 mu with the three-link transporter W_mu(x) =
// U_mu(x) U_mu(x+mu) U_mu(x+2mu).  Stored folded like the one-link hops:
// W~_mu(x) = 1/2 eta_mu(x) bc W_mu(x) (bc: the boundary sign when the hop
// crosses the boundary), [mu][site]; the backward hop is -W~_mu(x-3mu)^*,
// since eta_mu(x - 3mu) = eta_mu(x).  A three-link hop always leaves the KD
// block (and joins sites of opposite eps).

// block-layout index of site (x0, x1)
__host__ __device__ __forceinline__ long blk_site_index(const Geo2& g, int x0, int x1) {
  const int X0 = x0 >> 1, X1 = x1 >> 1;
  return (long)((X0 + X1) & 1) * g.half + 4L * blk_index(g, X0, X1) + (x0 & 1) + 2 * (x1 & 1);
}

// Block-layout site e -> its four three-hop neighbours (+x, -x, +t, -t).
struct Hop3 {
  long xp, xm, tp, tm;
  float eps;  // eps(x) of the site itself
};
__device__ __forceinline__ Hop3 hop3_of(const Geo2& g, long e) {
  const int p = e >= g.half ? 1 : 0;
  const long rem = e - (long)p * g.half;
  const int b = (int)(rem >> 2), s = (int)(rem & 3);
  int X0, X1;
  blk_coords(g, p, b, X0, X1);
  const int x0 = 2 * X0 + (s & 1), x1 = 2 * X1 + (s >> 1);
  const int x0p = x0 + 3 >= g.Lx ? x0 + 3 - g.Lx : x0 + 3, x0m = x0 < 3 ? x0 - 3 + g.Lx : x0 - 3;
  const int x1p = x1 + 3 >= g.Lt ? x1 + 3 - g.Lt : x1 + 3, x1m = x1 < 3 ? x1 - 3 + g.Lt : x1 - 3;
  Hop3 h;
  h.xp = blk_site_index(g, x0p, x1);
  h.xm = blk_site_index(g, x0m, x1);
  h.tp = blk_site_index(g, x0, x1p);
  h.tm = blk_site_index(g, x0, x1m);
  h.eps = ((x0 + x1) & 1) ? -1.f : 1.f;
  return h;
}

// out += coef * C3 in on full block-layout vectors (C3: the three-link hops),
// one thread per site; eps_in multiplies the source by eps (the targets all
// have eps = -eps(x)).  Grid (sites / 256, rhs).
template <class R, class LT, class VT>
__global__ __launch_bounds__(256) void k_hop3(Cx<VT>* out, long so, const Cx<VT>* in, long si, R coef,
                                               const Cx<LT>* wl, Geo2 g, int eps_in, const int* act) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const long f = 2 * g.half;
  if (e >= f || !is_active(act, r)) return;
  const Hop3 n = hop3_of(g, e);
  const Cx<VT>* src = in + r * si;
  const Cx<R> vxp = ld<R>(src[n.xp]), vxm = ld<R>(src[n.xm]), vtp = ld<R>(src[n.tp]), vtm = ld<R>(src[n.tm]);
  const Cx<R> wx = ld<R>(wl[e]), wxm = ld<R>(wl[n.xm]), wt = ld<R>(wl[f + e]), wtm = ld<R>(wl[f + n.tm]);
  Cx<R> h = wx * vxp - cmul_conj(wxm, vxm) + wt * vtp - cmul_conj(wtm, vtm);
  const R c = eps_in ? coef * (R)(-n.eps) : coef;
  Cx<VT>& o = out[r * so + e];
  o = st<VT>(ld<R>(o) + c * h);
}

// Naik-improved D in natural site order, one thread per site:
// out = m in + c1 (one-link hops) + c3 (three-link hops), links folded
// ([mu][site]: U~ one-link, W~ three-link).
template <class R, class LT, class VT>
__global__ __launch_bounds__(256) void k_dslash_naik_nat(Cx<VT>* __restrict__ out, const Cx<VT>* __restrict__ in,
                                                         const Cx<LT>* __restrict__ U, const Cx<LT>* __restrict__ W,
                                                         int Lx, int Lt, long vol, R m, R c1, R c3) {
  const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (x >= vol) return;
  const int x1 = (int)(x / Lx), x0 = (int)(x - (long)x1 * Lx);
  auto wrap = [](int a, int L) { return a >= L ? a - L : (a < 0 ? a + L : a); };
  const long i1xp = (long)x1 * Lx + wrap(x0 + 1, Lx), i1xm = (long)x1 * Lx + wrap(x0 - 1, Lx);
  const long i1tp = (long)wrap(x1 + 1, Lt) * Lx + x0, i1tm = (long)wrap(x1 - 1, Lt) * Lx + x0;
  const long i3xp = (long)x1 * Lx + wrap(x0 + 3, Lx), i3xm = (long)x1 * Lx + wrap(x0 - 3, Lx);
  const long i3tp = (long)wrap(x1 + 3, Lt) * Lx + x0, i3tm = (long)wrap(x1 - 3, Lt) * Lx + x0;
  const Cx<VT>* v = in + (long)r * vol;
  Cx<R> h1 = ld<R>(U[x]) * ld<R>(v[i1xp]) - cmul_conj(ld<R>(U[i1xm]), ld<R>(v[i1xm])) +
             ld<R>(U[vol + x]) * ld<R>(v[i1tp]) - cmul_conj(ld<R>(U[vol + i1tm]), ld<R>(v[i1tm]));
  Cx<R> h3 = ld<R>(W[x]) * ld<R>(v[i3xp]) - cmul_conj(ld<R>(W[i3xm]), ld<R>(v[i3xm])) +
             ld<R>(W[vol + x]) * ld<R>(v[i3tp]) - cmul_conj(ld<R>(W[vol + i3tm]), ld<R>(v[i3tm]));
  out[(long)r * vol + x] = st<VT>(m * ld<R>(v[x]) + c1 * h1 + c3 * h3);
}

// gather / scatter between an external ordering and the block layout:
// dst[r][i] = src[r][idx[i]]  (gather)   or  dst[r][idx[i]] = src[r][i]  (scatter)
template <class TO, class TI>
__global__ __launch_bounds__(256) void k_permute(Cx<TO>* dst, long sd, const Cx<TI>* src, long ss,
                                                 const int* idx, long n, int scatter) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  if (scatter) dst[r * sd + idx[i]] = st<TO>(ld<double>(src[r * ss + i]));
  else dst[r * sd + i] = st<TO>(ld<double>(src[r * ss + idx[i]]));
}

// --------------------------------------------------- level-1 transfer (2D)

struct Agg2 {
  int a0, a1;     // aggregate extent in KD blocks
  int Ncx, Nct;   // coarse lattice
  int nv;         // null vectors (coarse dofs = 2 nv)
};

// Shared by the multi-rhs transfers: the fine dof of every aggregate-local
// index q = 4 k + s (block k of the aggregate in row-major order, site s),
// -1 where it does not take part (parity >= npar), written to qd[0 .. nd)
// by the first nd threads.
__device__ __forceinline__ void aggregate_dofs(int* qd, const Geo2& g, const Agg2& a, int Z, int npar) {
  const int nd = 4 * a.a0 * a.a1;
  for (int q = threadIdx.x; q < nd; q += blockDim.x) {
    const int k = q >> 2, Z0 = Z % a.Ncx, Z1 = Z / a.Ncx;
    const int X0 = Z0 * a.a0 + k % a.a0, X1 = Z1 * a.a1 + k / a.a0, p = (X0 + X1) & 1;
    qd[q] = p < npar ? (int)((long)p * g.half + 4L * blk_index(g, X0, X1) + (q & 3)) : -1;
  }
}

// Copies n = rows * cols elements src(row, col) -> dst[row * ds + col] with
// every thread's loads issued before its stores (XU per batch); the row and
// column come from the float-reciprocal division (exact for these sizes).
template <class R, int XU, class F>
__device__ __forceinline__ void stage_rows(Cx<R>* dst, int ds, int rows, int cols, F src) {
  const int n = rows * cols;
  const float inv = 1.0f / (float)cols;
  for (int e0 = threadIdx.x; e0 < n; e0 += XU * blockDim.x) {
    Cx<R> v[XU];
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int e = e0 + u * blockDim.x, row = (int)(((float)e + 0.5f) * inv), col = e - row * cols;
      v[u] = e < n ? src(row, col) : Cx<R>{0, 0};
    }
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int e = e0 + u * blockDim.x, row = (int)(((float)e + 0.5f) * inv), col = e - row * cols;
      if (e < n) dst[row * ds + col] = v[u];
    }
  }
}

// Restriction, several rhs per workgroup:
//   out[r][Z][c*nv+i] = sum_{x in Z, chir(x)=c} conj(P[x][i]) in[r][x]
// in: full block-layout vector (even_only: the parity-0 half only
// contributes).  The workgroup of aggregate Z stages the aggregate's P rows
// (nd = 4 a0 a1 fine dofs, converted to R) and its tile of RB rhs in LDS,
// so P is read once per rhs tile; thread o then adds TI consecutive coarse
// dofs of one (rhs, chirality) over the aggregate's blocks in order.
// grid (nZ, cdiv(nrhs, RB)); LDS (nd nv + RB nd) Cx<R> + nd int.
template <class R, class PT, class VI, class VO, int TI>
__global__ __launch_bounds__(256) void k_restrict1(Cx<VO>* out, const Cx<VI>* in, long si,
                                                   const Cx<PT>* P, Geo2 g, Agg2 a, int even_only,
                                                   const int* act, int nrhs, int RB) {
  extern __shared__ __align__(16) unsigned char xf_raw[];
  const int Z = xcd_block(blockIdx.x, gridDim.x), r0 = blockIdx.y * RB, nv = a.nv, ndc = 2 * nv;
  const int nblk = a.a0 * a.a1, nd = 4 * nblk;
  Cx<R>* Ps = reinterpret_cast<Cx<R>*>(xf_raw);  // [nd][nv]
  Cx<R>* Vs = Ps + (long)nd * nv;                // [RB][nd]
  int* qd = reinterpret_cast<int*>(Vs + (long)RB * nd);
  aggregate_dofs(qd, g, a, Z, even_only ? 1 : 2);
  __syncthreads();
  stage_rows<R, 4>(Ps, nv, nd, nv, [&](int q, int i) {
    const int d = qd[q];
    return d >= 0 ? ld<R>(P[(long)d * nv + i]) : Cx<R>{0, 0};
  });
  stage_rows<R, 4>(Vs, nd, RB, nd, [&](int r, int q) {
    const int d = qd[q], rr = r0 + r;
    return d >= 0 && rr < nrhs && is_active(act, rr) ? ld<R>(in[rr * si + d]) : Cx<R>{0, 0};
  });
  __syncthreads();
  const int ng = nv / TI, nout = RB * 2 * ng;
  const long nc = (long)a.Ncx * a.Nct * ndc;
  for (int o = threadIdx.x; o < nout; o += blockDim.x) {
    const int r = o / (2 * ng), rem = o - r * 2 * ng, c = rem / ng, i0 = (rem - c * ng) * TI, rr = r0 + r;
    if (rr >= nrhs || !is_active(act, rr)) continue;
    Cx<R> acc[TI];
#pragma unroll
    for (int u = 0; u < TI; ++u) acc[u] = Cx<R>{0, 0};
    const int s0 = c ? 1 : 0, s1 = c ? 2 : 3;
    const Cx<R>* v = Vs + (long)r * nd;
    for (int k = 0; k < nblk; ++k) {
      const int q0 = 4 * k + s0, q1 = 4 * k + s1;
      const Cx<R> v0 = v[q0], v1 = v[q1];
#pragma unroll
      for (int u = 0; u < TI; ++u) {
        cfma_conj(acc[u], Ps[q0 * nv + i0 + u], v0);
        cfma_conj(acc[u], Ps[q1 * nv + i0 + u], v1);
      }
    }
#pragma unroll
    for (int u = 0; u < TI; ++u) out[rr * nc + (long)Z * ndc + c * nv + i0 + u] = st<VO>(acc[u]);
  }
}

// Prolongation, several rhs per workgroup:
//   out[r][x] = [add[r][x] +] sum_i P[x][i] in[r][Z(x)][c(x)*nv+i]
// The workgroup of aggregate Z stages the aggregate's P rows (row stride
// nv + 1 against LDS bank conflicts) and the coarse values of its rhs tile in
// LDS, so P is read once per tile; output o is (rhs o / nd, aggregate-local
// dof o % nd).  npar = 1: only the parity-0 blocks (out/add are Schur-half
// vectors), npar = 2: all.  grid (nZ, cdiv(nrhs, RB)); LDS
// (nd (nv + 1) + RB 2 nv) Cx<R> + nd int.
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k_prolong1(Cx<VO>* out, long so, const Cx<VO>* add, long sa,
                                                  const Cx<VI>* in, const Cx<PT>* P, Geo2 g, Agg2 a, int npar,
                                                  const int* act, int nrhs, int RB) {
  extern __shared__ __align__(16) unsigned char xf_raw[];
  const int Z = xcd_block(blockIdx.x, gridDim.x), r0 = blockIdx.y * RB, nv = a.nv, ndc = 2 * nv, RP = nv + 1;
  const int nd = 4 * a.a0 * a.a1;
  Cx<R>* Ps = reinterpret_cast<Cx<R>*>(xf_raw);  // [nd][nv + 1]
  Cx<R>* Es = Ps + (long)nd * RP;                // [RB][2 nv]
  int* qd = reinterpret_cast<int*>(Es + (long)RB * ndc);
  aggregate_dofs(qd, g, a, Z, npar);
  __syncthreads();
  stage_rows<R, 4>(Ps, RP, nd, nv, [&](int q, int i) {
    const int d = qd[q];
    return d >= 0 ? ld<R>(P[(long)d * nv + i]) : Cx<R>{0, 0};
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
    const Cx<R>* er = Es + r * ndc + chir2(q & 3) * nv;
    Cx<R> acc{0, 0};
    for (int i = 0; i < nv; ++i) cfma(acc, pq[i], er[i]);
    if (add) acc += ld<R>(add[rr * sa + x]);
    out[rr * so + x] = st<VO>(acc);
  }
}

// W[x][c'][j] = sum_{s' in block(x), chir(s')=c'} B^-1[x][s'] P[s'][j]   (FP64)
// grid: (blocks, nv, 2 parities)
template <class LT>
// wmode 0: W = B^-1 P (the KD Galerkin product); 1: W = P (Galerkin on D
// itself); 2: W = B P (its block-local part P^dag B P).
__global__ __launch_bounds__(256) void k_galerkin_w1(c64* W, const c64* P, const Cx<LT>* links,
                                                     Geo2 g, int nv, double m, int wmode) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, p = blockIdx.z;
  if (b >= g.Nb2) return;
  c64 L[4], v[4], w[4];
  load_intra<double, LT>(links + ((size_t)p * g.Nb2 + b) * 8, L);
  const long base = (long)p * g.half + 4L * b;
  for (int cp = 0; cp < 2; ++cp) {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = chir2(s) == cp ? P[(base + s) * nv + j] : c64{0, 0};
    if (wmode == 0) {
      binv_block<double>(L, m, v, w);
    } else if (wmode == 2) {
      b_block<double>(L, m, v, w);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) w[s] = v[s];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) W[((base + s) * 2 + cp) * nv + j] = w[s];
  }
}

// A_hat = 1 + P^dag C W, level 1.  One workgroup per coarse site Z.
// Output Yt[dir][Z][col][row] (column-major blocks), dir 0 self, 1/2 = +-x,
// 3/4 = +-t.
template <class LT>
__global__ __launch_bounds__(1024) void k_galerkin1(c64* Yt, const c64* P, const c64* W,
                                                    const Cx<LT>* links, Geo2 g, Agg2 a, int ident) {
  const int Z = blockIdx.x;
  const int nv = a.nv, ndc = 2 * nv;
  const long nZ = (long)a.Ncx * a.Nct;
  const int Z0 = Z % a.Ncx, Z1 = Z / a.Ncx;
  for (int pair = threadIdx.x; pair < ndc * ndc; pair += blockDim.x) {
    const int row = pair / ndc, col = pair % ndc;
    const int c = row / nv, i = row % nv, cp = col / nv, j = col % nv;
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
      auto Wat = [&](int nb, int s) -> c64 {
        return W[(((long)q * g.half + 4L * nb + s) * 2 + cp) * nv + j];
      };
      if (c == 0) {
        // s0: bwd x -> (X-0, s1), bwd t -> (X-1, s2)
        const c64 P0 = P[(base + 0) * nv + i];
        cfma_conj(acc[dxm], P0, -(conj(ld<double>(Lxm[4])) * Wat(n.xm, 1)));
        cfma_conj(acc[dtm], P0, -(conj(ld<double>(Ltm[6])) * Wat(n.tm, 2)));
        // s3: fwd x -> (X+0, s2), fwd t -> (X+1, s1)
        const c64 P3 = P[(base + 3) * nv + i];
        cfma_conj(acc[dxp], P3, ld<double>(Lb[5]) * Wat(n.xp, 2));
        cfma_conj(acc[dtp], P3, ld<double>(Lb[7]) * Wat(n.tp, 1));
      } else {
        // s1: fwd x -> (X+0, s0), bwd t -> (X-1, s3)
        const c64 P1 = P[(base + 1) * nv + i];
        cfma_conj(acc[dxp], P1, ld<double>(Lb[4]) * Wat(n.xp, 0));
        cfma_conj(acc[dtm], P1, -(conj(ld<double>(Ltm[7])) * Wat(n.tm, 3)));
        // s2: fwd t -> (X+1, s0), bwd x -> (X-0, s3)
        const c64 P2 = P[(base + 2) * nv + i];
        cfma_conj(acc[dtp], P2, ld<double>(Lb[6]) * Wat(n.tp, 0));
        cfma_conj(acc[dxm], P2, -(conj(ld<double>(Lxm[5])) * Wat(n.xm, 3)));
      }
    }
    if (ident && row == col) acc[0].re += 1.0;
#pragma unroll
    for (int d = 0; d < 5; ++d) Yt[(((long)d * nZ + Z) * ndc + col) * ndc + row] = acc[d];
  }
}

// Galerkin on D itself: the block-local part, self block += coef P^dag W_B
// with W_B = B P (k_galerkin_w1 mode 2).  One workgroup per coarse site.
template <class LT>
__global__ __launch_bounds__(1024) void k_galerkin1_self(c64* Yt, const c64* P, const c64* WB, Geo2 g, Agg2 a,
                                                          double coef) {
  const int Z = blockIdx.x;
  const int nv = a.nv, ndc = 2 * nv;
  const int Z0 = Z % a.Ncx, Z1 = Z / a.Ncx;
  for (int pair = threadIdx.x; pair < ndc * ndc; pair += blockDim.x) {
    const int row = pair / ndc, col = pair % ndc;
    const int c = row / nv, i = row % nv, cp = col / nv, j = col % nv;
    c64 acc{0, 0};
    for (int k = 0; k < a.a0 * a.a1; ++k) {
      const int X0 = Z0 * a.a0 + k % a.a0, X1 = Z1 * a.a1 + k / a.a0;
      const long base = (long)((X0 + X1) & 1) * g.half + 4L * blk_index(g, X0, X1);
      for (int s = 0; s < 4; ++s)
        if (chir2(s) == c) cfma_conj(acc, P[(base + s) * nv + i], WB[((base + s) * 2 + cp) * nv + j]);
    }
    c64& y = Yt[((long)Z * ndc + col) * ndc + row];
    y.re += coef * acc.re;
    y.im += coef * acc.im;
  }
}

// The Naik term of the level-1 Galerkin product: blocks += coef P^dag C3 W,
// with C3 the three-link hops.  A hop that leaves the aggregate lands in the
// neighbouring one (aggregates at least 2 KD blocks = 4 sites wide) and is
// filed under its direction, as the one-link hops are.
template <class LT>
__global__ __launch_bounds__(1024) void k_galerkin1_hop3(c64* Yt, const c64* P, const c64* W, const Cx<LT>* wl,
                                                          Geo2 g, Agg2 a, double coef) {
  const int Z = blockIdx.x;
  const int nv = a.nv, ndc = 2 * nv;
  const long nZ = (long)a.Ncx * a.Nct, f = 2 * g.half;
  const int Z0 = Z % a.Ncx, Z1 = Z / a.Ncx, e0 = 2 * a.a0, e1 = 2 * a.a1;
  for (int pair = threadIdx.x; pair < ndc * ndc; pair += blockDim.x) {
    const int row = pair / ndc, col = pair % ndc;
    const int c = row / nv, i = row % nv, cp = col / nv, j = col % nv;
    c64 acc[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) acc[d] = c64{0, 0};
    for (int k = 0; k < a.a0 * a.a1; ++k) {
      const int X0 = Z0 * a.a0 + k % a.a0, X1 = Z1 * a.a1 + k / a.a0;
      const long base = (long)((X0 + X1) & 1) * g.half + 4L * blk_index(g, X0, X1);
      for (int s = 0; s < 4; ++s) {
        if (chir2(s) != c) continue;
        const long e = base + s;
        const int lx = (2 * X0 + (s & 1)) % e0, lt = (2 * X1 + (s >> 1)) % e1;  // position in the aggregate
        const Hop3 n = hop3_of(g, e);
        const c64 Pv = P[e * nv + i];
        auto Wat = [&](long y) { return W[(y * 2 + cp) * nv + j]; };
        cfma_conj(acc[lx + 3 >= e0 ? 1 : 0], Pv, ld<double>(wl[e]) * Wat(n.xp));
        cfma_conj(acc[lx < 3 ? 2 : 0], Pv, -(conj(ld<double>(wl[n.xm])) * Wat(n.xm)));
        cfma_conj(acc[lt + 3 >= e1 ? 3 : 0], Pv, ld<double>(wl[f + e]) * Wat(n.tp));
        cfma_conj(acc[lt < 3 ? 4 : 0], Pv, -(conj(ld<double>(wl[f + n.tm])) * Wat(n.tm)));
      }
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      c64& y = Yt[(((long)d * nZ + Z) * ndc + col) * ndc + row];
      y.re += coef * acc[d].re;
      y.im += coef * acc[d].im;
    }
  }
}

}  // namespace kdmg
