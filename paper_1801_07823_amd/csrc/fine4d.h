// Fine-level kernels for the 4D SU(3) staggered operator in Kahler-Dirac
// block layout (eq. "staggeredD" with d = 4, N_c = 3; Sec. 2.1 blocking).
//
// Layout.  The lattice is cut into 2^4 Kahler-Dirac blocks anchored at even
// coordinates.  Block coordinates B (B_mu = x_mu / 2) have linear index
// lin = B0 + NB0 (B1 + NB1 (B2 + NB2 B3)); with NB0 even, lin and lin ^ 1
// have opposite parity p = (sum_mu B_mu) & 1, so b = lin / 2 numbers the
// blocks of one parity.  A site is ib = (p Nb2 + b) 16 + s with
// s = sum_mu (x_mu & 1) 2^mu, and a colour vector entry is ib * 3 + c: the 48
// complex values of a block are contiguous and the Schur space (p = 0) is
// the first half.  The chirality of a site is eps(x) = (-1)^popcount(s).
//
// Links.  lk[ib][mu][a][b] = 1/2 eta_mu(x) bc_mu(x) U_mu(x)_{ab} (forward
// link, staggered phase, factor 1/2 and the antiperiodic sign folded in); the
// backward hop uses the neighbour's forward link: since eta_mu(x - mu) =
// eta_mu(x), D psi(x) = m psi(x) + sum_mu [U~_mu(x) psi(x + mu)
// - U~_mu(x - mu)^dag psi(x - mu)].  nb4[ib][2 mu] = x + mu and
// nb4[ib][2 mu + 1] = x - mu (block-layout site indices).
//
// Blocking.  A forward hop from x stays in the block iff x_mu is even
// (bit mu of s clear), a backward hop iff x_mu is odd.  D = B + C with
// B = m + intra-block hops and C the rest.  B is block diagonal with 48 x 48
// blocks; in (even-site, odd-site) order B = [[m, K], [-K^dag, m]], so with
// S_e = m^2 + K K^dag and S_o = m^2 + K^dag K (Hermitian positive definite)
//   B^-1 = [[m S_e^-1, -K S_o^-1], [K^dag S_e^-1, m S_o^-1]],
// which k4_binv_build evaluates per block (Gauss-Jordan on S_e and S_o,
// stable without pivoting for positive definite matrices) and stores as a
// dense column-major 48 x 48 matrix per block.
#pragma once
#include "common.h"
#include "blas.h"

namespace kdmg {

struct Geo4 {
  int L[4];    // sites per direction
  int NB[4];   // KD blocks per direction
  int Nb2;     // blocks per parity
  long half;   // complex entries per parity half (Nb2 * 48)
};

__host__ __device__ __forceinline__ void blk4_coords(const Geo4& g, int p, int b, int Bc[4]) {
  int r = 2 * b;
  Bc[0] = r % g.NB[0];
  r /= g.NB[0];
  Bc[1] = r % g.NB[1];
  r /= g.NB[1];
  Bc[2] = r % g.NB[2];
  Bc[3] = r / g.NB[2];
  if (((Bc[0] + Bc[1] + Bc[2] + Bc[3]) & 1) != p) Bc[0] += 1;
}

__host__ __device__ __forceinline__ int blk4_index(const Geo4& g, const int Bc[4]) {
  const int lin = Bc[0] + g.NB[0] * (Bc[1] + g.NB[1] * (Bc[2] + g.NB[2] * Bc[3]));
  return lin >> 1;
}

__host__ __device__ __forceinline__ int blk4_parity(const int Bc[4]) { return (Bc[0] + Bc[1] + Bc[2] + Bc[3]) & 1; }

// chirality of a site from its in-block index: 0 for eps = +1, 1 for eps = -1
__host__ __device__ __forceinline__ int chir4(int s) { return __builtin_popcount((unsigned)s) & 1; }

// ------------------------------------------------------------------ hops

// out = [add +] [c2 add2 +] sgn * H in on the sites of parity p = p0 + blockIdx.z, where
//   mode 0: H = C (inter-block hops)
//   mode 2: H = D (all hops + m)
//   mode 3: H = B (intra-block hops + m)
// eps_in multiplies the source by eps.  Vectors are full-layout ([p][b][s][c],
// `s*` = per-rhs stride) except that a vector only addressed at p = 0 may be
// the even half alone.  One thread per site and a tile of RB rhs
// (blockIdx.y): each link and neighbour index is loaded once per tile.
template <class R, class LT, class VT, int RB>
__global__ __launch_bounds__(256) void k4_hop(Cx<VT>* out, long so, const Cx<VT>* in, long si,
                                               const Cx<VT>* add, long sa, const Cx<VT>* add2, long sa2, R c2,
                                               R sgn, const Cx<LT>* __restrict__ lk,
                                               const int* __restrict__ nb4, Geo4 g, int p0, R m, int mode,
                                               int eps_in, const int* act, int nrhs) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * RB, p = p0 + blockIdx.z;
  if (i >= 16L * g.Nb2) return;
  bool on[RB];
  bool any = false;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    on[b] = r0 + b < nrhs && is_active(act, r0 + b);
    any = any || on[b];
  }
  if (!any) return;
  const long ib = (long)p * g.Nb2 * 16 + i;
  const int s = (int)(i & 15);
  // Loads carry no branch (a load under a divergent branch is waited for at
  // the branch's end, which serialises them): inactive rhs of the tile read
  // row r0 and are never stored, and the hop direction a site takes is
  // selected arithmetically.
  long rr[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) rr[b] = on[b] ? r0 + b : r0;
  Cx<R> acc[RB][3];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[b][c] = Cx<R>{0, 0};
  // the mass term reads the site itself; mode is uniform over the launch, and
  // in mode 0 the source may hold only the other parity
  if (mode >= 2)
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[b][c] = m * ld<R>(in[rr[b] * si + ib * 3 + c]);
  // mode 2 takes both directions of every mu; modes 0 and 3 one each:
  // forward (dir 0) is intra-block iff x_mu is even, so C (mode 0) takes
  // dir = 1 - bit and B (mode 3) takes dir = bit
  const int ndir = mode == 2 ? 2 : 1;
  // all neighbour indices first, so their latency is paid once
  int jn[4][2];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int bit = (s >> mu) & 1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int dir = mode == 2 ? t : (mode == 0 ? 1 - bit : bit);
      jn[mu][t] = t < ndir ? nb4[ib * 8 + 2 * mu + dir] : 0;
    }
  }
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int bit = (s >> mu) & 1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t >= ndir) break;
      const int dir = mode == 2 ? t : (mode == 0 ? 1 - bit : bit);
      const long j = jn[mu][t];
      const Cx<LT>* U = lk + ((dir == 0 ? ib : j) * 4 + mu) * 9;
      Cx<R> u[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) u[q] = ld<R>(U[q]);
      Cx<R> v[RB][3];
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[b][c] = ld<R>(in[rr[b] * si + j * 3 + c]);
      // forward: + U v ; backward: - U^dag v (U the link from the neighbour)
      Cx<R> M[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[a * 3 + c] = dir == 0 ? u[a * 3 + c] : -conj(u[c * 3 + a]);
      const R e = (eps_in && chir4((int)(j & 15))) ? R(-1) : R(1);
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[b][a] += M[a * 3 + c] * (e * v[b][c]);
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cx<R> o = sgn * acc[b][c];
      if (add) o += ld<R>(add[rr[b] * sa + ib * 3 + c]);
      if (add2) o += c2 * ld<R>(add2[rr[b] * sa2 + ib * 3 + c]);
      acc[b][c] = o;
    }
#pragma unroll
  for (int b = 0; b < RB; ++b)
    if (on[b])
#pragma unroll
      for (int c = 0; c < 3; ++c) out[(long)(r0 + b) * so + ib * 3 + c] = st<VT>(acc[b][c]);
}

// ------------------------------------------------------------------ block inverse

constexpr int B4_RB = 8;  // rhs per workgroup of the B^-1 apply

// out = [add +] [eps] B^-1 in on the blocks of parity p0 + blockIdx.z; one
// workgroup per block, thread i < 48 owns row i, B4_RB rhs per workgroup.
// Bv[(blk 48 + j) 48 + i] = (B^-1)_{ij} for block blk = p Nb2 + b.
template <class R, class BT, class VT>
__global__ __launch_bounds__(64) void k4_binv(Cx<VT>* out, long so, const Cx<VT>* in, long si, const Cx<VT>* add,
                                              long sa, const Cx<BT>* __restrict__ Bv, Geo4 g, int p0, int eps_out,
                                              const int* act, int nrhs) {
  __shared__ Cx<R> vin[B4_RB][48];
  const int b = blockIdx.x, p = p0 + blockIdx.z, r0 = blockIdx.y * B4_RB;
  const long blk = (long)p * g.Nb2 + b, base = blk * 48;
  // loads carry no branch (inactive rhs read row r0, then count as zero)
  for (int e = threadIdx.x; e < B4_RB * 48; e += blockDim.x) {
    const int rb = e / 48, j = e - rb * 48, rr = r0 + rb;
    const bool use = rr < nrhs && is_active(act, rr);
    const Cx<R> x = ld<R>(in[(long)(use ? rr : r0) * si + base + j]);
    vin[rb][j] = use ? x : Cx<R>{0, 0};
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= 48) return;
  Cx<R> acc[B4_RB];
#pragma unroll
  for (int rb = 0; rb < B4_RB; ++rb) acc[rb] = Cx<R>{0, 0};
  const Cx<BT>* col = Bv + blk * 48 * 48 + i;
  // sixteen entries of the row loaded before any is used, so their loads are
  // in flight together (one at a time, the row costs 48 memory latencies)
  for (int j0 = 0; j0 < 48; j0 += 16) {
    Cx<BT> raw[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) raw[u] = col[(j0 + u) * 48];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const Cx<R> bij = ld<R>(raw[u]);
#pragma unroll
      for (int rb = 0; rb < B4_RB; ++rb) acc[rb] += bij * vin[rb][j0 + u];
    }
  }
  const bool neg = eps_out && chir4(i / 3);
  bool use[B4_RB];
#pragma unroll
  for (int rb = 0; rb < B4_RB; ++rb) {
    use[rb] = r0 + rb < nrhs && is_active(act, r0 + rb);
    if (neg) acc[rb] = -acc[rb];
  }
  if (add)
#pragma unroll
    for (int rb = 0; rb < B4_RB; ++rb) acc[rb] += ld<R>(add[(long)(use[rb] ? r0 + rb : r0) * sa + base + i]);
#pragma unroll
  for (int rb = 0; rb < B4_RB; ++rb)
    if (use[rb]) out[(long)(r0 + rb) * so + base + i] = st<VT>(acc[rb]);
}


// ------------------------------------------------------------------ transfers (level 0 <-> 1)

// Restriction out[r][Z][c nv + i] = sum_{dof in (Z, c)} P[dof][i]^* in[r][dof]
// (rows[(Z 2 + c) nrows + k] lists the group's fine dofs in increasing order;
// with even_only the dofs of odd blocks (dof >= half) count as zero).  Grid (2 nZ, nv / RI,
// nrhs / RR); the workgroup's partial sums are combined in a fixed tree.
constexpr int R4_RI = 4, R4_RR = 4;
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k4_restrict(Cx<VO>* out, const Cx<VI>* in, long si, const Cx<PT>* __restrict__ P,
                                                   const int* __restrict__ rows, const int* __restrict__ neven,
                                                   int nrows, int nv, int even_only, const int* act, int nrhs) {
  __shared__ Cx<R> red[4][R4_RI * R4_RR];
  const int gid = blockIdx.x, i0 = blockIdx.y * R4_RI, r0 = blockIdx.z * R4_RR;
  Cx<R> acc[R4_RR][R4_RI];
#pragma unroll
  for (int a = 0; a < R4_RR; ++a)
#pragma unroll
    for (int q = 0; q < R4_RI; ++q) acc[a][q] = Cx<R>{0, 0};
  bool on[R4_RR];
#pragma unroll
  for (int a = 0; a < R4_RR; ++a) on[a] = r0 + a < nrhs && is_active(act, r0 + a);
  // Loads carry no branch (a load under a divergent branch is waited for at
  // the branch's end, which serialises them): indices are clamped to valid
  // entries and unused values replaced by zero afterwards.
  long ra[R4_RR];
#pragma unroll
  for (int a = 0; a < R4_RR; ++a) ra[a] = on[a] ? r0 + a : r0;
  // The group's dofs are listed in increasing order, so with even_only the
  // rows that count form a prefix, of length neven[gid] (dofs < half).
  const int* grow = rows + (long)gid * nrows;
  const int nuse = even_only ? neven[gid] : nrows;
  for (int k = threadIdx.x; k < nuse; k += blockDim.x) {
    const long dof = grow[k];
    Cx<R> pv[R4_RI], v[R4_RR];
#pragma unroll
    for (int q = 0; q < R4_RI; ++q) {
      const Cx<R> x = conj(ld<R>(P[dof * nv + min(i0 + q, nv - 1)]));
      pv[q] = i0 + q < nv ? x : Cx<R>{0, 0};
    }
#pragma unroll
    for (int a = 0; a < R4_RR; ++a) {
      const Cx<R> x = ld<R>(in[ra[a] * si + dof]);
      v[a] = on[a] ? x : Cx<R>{0, 0};
    }
#pragma unroll
    for (int a = 0; a < R4_RR; ++a)
#pragma unroll
      for (int q = 0; q < R4_RI; ++q) acc[a][q] += pv[q] * v[a];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < R4_RR; ++a)
#pragma unroll
    for (int q = 0; q < R4_RI; ++q) {
      R re = acc[a][q].re, im = acc[a][q].im;
      for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
      }
      if (lane == 0) red[w][a * R4_RI + q] = Cx<R>{re, im};
    }
  __syncthreads();
  const int nw = blockDim.x >> 6;
  for (int e = threadIdx.x; e < R4_RI * R4_RR; e += blockDim.x) {
    const int a = e / R4_RI, q = e - a * R4_RI;
    if (!on[a] || i0 + q >= nv) continue;
    Cx<R> s = red[0][e];
    for (int v = 1; v < nw; ++v) s += red[v][e];
    const int Z = gid >> 1, c = gid & 1;
    out[((long)(r0 + a) * (gridDim.x >> 1) + Z) * 2 * nv + c * nv + i0 + q] = st<VO>(s);
  }
}

// Prolongation out[r][dof] = [add +] sum_i P[dof][i] in[r][Z][c nv + i] for
// dof < n_out, (Z, c) the group of the dof (dgrp[dof] = 2 Z + c).  A
// workgroup of BS threads stages the P rows of its BS consecutive dofs (one
// contiguous range of P) in LDS with coalesced loads, at an odd row stride
// against bank conflicts; each thread then forms its dof for every rhs in
// tiles of RR, so P is read from memory once.  The coarse values are shared
// by the thousands of dofs of a group and come from cache.
template <class R, class PT, class VI, class VO, int BS, int RR>
__global__ __launch_bounds__(BS) void k4_prolong(Cx<VO>* out, long so, const Cx<VO>* add, long sa, const Cx<VI>* in,
                                                 const Cx<PT>* __restrict__ P, const int* __restrict__ dgrp,
                                                 int nv, long n_out, long ncoarse, const int* act, int nrhs) {
  extern __shared__ __align__(16) unsigned char k4p_smem[];
  Cx<R>* Ps = reinterpret_cast<Cx<R>*>(k4p_smem);
  const int ps = nv | 1;
  const long d0 = (long)blockIdx.x * BS;
  const int cnt = (int)(n_out - d0 < BS ? n_out - d0 : BS);
  const Cx<PT>* Pb = P + d0 * nv;
  for (int e = threadIdx.x; e < cnt * nv; e += BS) {
    const int rw = e / nv;
    Ps[rw * ps + (e - rw * nv)] = ld<R>(Pb[e]);
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= cnt) return;
  const long dof = d0 + t;
  const int gidx = dgrp[dof];
  const Cx<VI>* e = in + (long)(gidx >> 1) * 2 * nv + (gidx & 1) * nv;
  const Cx<R>* pr = Ps + t * ps;
  // Loads carry no branch (a load under a divergent branch is waited for at
  // the branch's end, which serialises them): rows of rhs outside the tile or
  // inactive read row r0 instead, and their results are never stored.
  for (int r0 = 0; r0 < nrhs; r0 += RR) {
    bool on[RR];
    long rb[RR];
    Cx<R> acc[RR];
#pragma unroll
    for (int b = 0; b < RR; ++b) {
      on[b] = r0 + b < nrhs && is_active(act, r0 + b);
      rb[b] = on[b] ? r0 + b : r0;
      acc[b] = Cx<R>{0, 0};
    }
    for (int i = 0; i < nv; ++i) {
      const Cx<R> pv = pr[i];
      Cx<R> ev[RR];
#pragma unroll
      for (int b = 0; b < RR; ++b) ev[b] = ld<R>(e[rb[b] * ncoarse + i]);
#pragma unroll
      for (int b = 0; b < RR; ++b) acc[b] += pv * ev[b];
    }
    if (add) {
      Cx<R> av[RR];
#pragma unroll
      for (int b = 0; b < RR; ++b) av[b] = ld<R>(add[rb[b] * sa + dof]);
#pragma unroll
      for (int b = 0; b < RR; ++b) acc[b] += av[b];
    }
#pragma unroll
    for (int b = 0; b < RR; ++b)
      if (on[b]) out[(long)(r0 + b) * so + dof] = st<VO>(acc[b]);
  }
}

// ------------------------------------------------------------------ setup kernels (setup4d.hip)

// B^-1 of every block of parity blockIdx.z at mass m, FP64 (see the header).
__global__ __launch_bounds__(256) void k4_binv_build(c64* Bv, const c64* __restrict__ lk, Geo4 g, double m);

// Gram matrices of the (aggregate, chirality) groups: G[g][i][j] =
// sum_{dof in g} V(dof, i)^* V(dof, j), with V(dof, i) = V[i sv + dof sd].
// One workgroup per group; rows are staged through LDS in chunks of 64.
__global__ __launch_bounds__(256) void k4_gram(c64* G, const c64* __restrict__ V, long sv, long sd,
                                               const int* __restrict__ rows, int nrows, int nv);

// Rinv[g] = R^-1 with G[g] = R^dag R (Cholesky, R upper triangular with a
// positive real diagonal).  One thread per group.
__global__ void k4_chol_inv(c64* Rinv, const c64* G, int ngroups, int nv);

// Q[dof][j] = sum_{i <= j} V(dof, i) Rinv[g][i][j] for the dofs of every group
// (Q in the prolongator layout [dof][nv]).
__global__ __launch_bounds__(256) void k4_qapply(c64* Q, const c64* __restrict__ V, long sv, long sd,
                                                 const c64* __restrict__ Rinv, const int* __restrict__ rows,
                                                 int nrows, int nv);

// W = B^-1 P per block: W[dof][c nv + i] = sum_{j in block, chir(j) = c}
// (B^-1)_{dof, j} P[j][i].  One workgroup per block.
__global__ __launch_bounds__(256) void k4_gal_w(c64* W, const c64* __restrict__ P, const c64* __restrict__ Bv, Geo4 g,
                                                int nv);

// Coarse stencil block of direction `dir` (blockIdx.y) of coarse site Z
// (blockIdx.x):  A_hat(Z, Z') = delta + P^dag C W restricted to the hops from
// sites of aggregate Z that land in Z' = Z (dir 0: hops inside the aggregate)
// or cross its face in direction dir (1 + 2 mu: +mu, 2 + 2 mu: -mu).
// Output Yt[dir][Z] column-major: Yt[((dir nZ + Z) ndc + col) ndc + row].
// Hops are staged through LDS in batches of GB4.
constexpr int GB4 = 8;
__global__ __launch_bounds__(256) void k4_galerkin(c64* Yt, const c64* __restrict__ P, const c64* __restrict__ W,
                                                   const c64* __restrict__ lk, const int* __restrict__ nb4, Geo4 g,
                                                   int agg0, int agg1, int agg2, int agg3, int nZ, int nv);

}  // namespace kdmg
