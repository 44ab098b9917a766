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
#include "blas.cuh"

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
  Cx<R> acc[RB][3];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      acc[b][c] = mode >= 2 && on[b] ? m * ld<R>(in[(r0 + b) * si + ib * 3 + c]) : Cx<R>{0, 0};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int bit = (s >> mu) & 1;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      // forward (dir 0): intra-block iff x_mu even; backward: iff x_mu odd
      if (!(mode == 2 || (mode == 0) == (bit == (dir == 0 ? 1 : 0)))) continue;
      const long j = nb4[ib * 8 + 2 * mu + dir];
      const Cx<LT>* U = lk + ((dir == 0 ? ib : j) * 4 + mu) * 9;
      Cx<R> u[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) u[q] = ld<R>(U[q]);
      const R e = (eps_in && chir4((int)(j & 15))) ? R(-1) : R(1);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (!on[b]) continue;
        const Cx<VT>* src = in + (r0 + b) * si + j * 3;
        Cx<R> v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = e * ld<R>(src[c]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (dir == 0)
              acc[b][a] += u[a * 3 + c] * v[c];
            else
              acc[b][a] -= cmul_conj(u[c * 3 + a], v[c]);
          }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (!on[b]) continue;
    const int r = r0 + b;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cx<R> o = sgn * acc[b][c];
      if (add) o += ld<R>(add[r * sa + ib * 3 + c]);
      if (add2) o += c2 * ld<R>(add2[r * sa2 + ib * 3 + c]);
      out[r * so + ib * 3 + c] = st<VT>(o);
    }
  }
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
  for (int e = threadIdx.x; e < B4_RB * 48; e += blockDim.x) {
    const int rb = e / 48, j = e - rb * 48, rr = r0 + rb;
    vin[rb][j] = (rr < nrhs && is_active(act, rr)) ? ld<R>(in[rr * si + base + j]) : Cx<R>{0, 0};
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= 48) return;
  Cx<R> acc[B4_RB];
#pragma unroll
  for (int rb = 0; rb < B4_RB; ++rb) acc[rb] = Cx<R>{0, 0};
  const Cx<BT>* col = Bv + blk * 48 * 48 + i;
  for (int j = 0; j < 48; ++j) {
    const Cx<R> bij = ld<R>(col[j * 48]);
#pragma unroll
    for (int rb = 0; rb < B4_RB; ++rb) acc[rb] += bij * vin[rb][j];
  }
  const bool neg = eps_out && chir4(i / 3);
#pragma unroll
  for (int rb = 0; rb < B4_RB; ++rb) {
    const int rr = r0 + rb;
    if (rr >= nrhs || !is_active(act, rr)) continue;
    Cx<R> o = neg ? -acc[rb] : acc[rb];
    if (add) o += ld<R>(add[rr * sa + base + i]);
    out[rr * so + base + i] = st<VT>(o);
  }
}


// ------------------------------------------------------------------ transfers (level 0 <-> 1)

// Restriction out[r][Z][c nv + i] = sum_{dof in (Z, c)} P[dof][i]^* in[r][dof]
// (rows[(Z 2 + c) nrows + k] lists the group's fine dofs; with even_only the
// dofs of odd blocks (dof >= half) count as zero).  Grid (2 nZ, nv / RI,
// nrhs / RR); the workgroup's partial sums are combined in a fixed tree.
constexpr int R4_RI = 4, R4_RR = 4;
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k4_restrict(Cx<VO>* out, const Cx<VI>* in, long si, const Cx<PT>* __restrict__ P,
                                                   const int* __restrict__ rows, int nrows, int nv, int even_only,
                                                   long half, const int* act, int nrhs) {
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
  for (int k = threadIdx.x; k < nrows; k += blockDim.x) {
    const long dof = rows[(long)gid * nrows + k];
    if (even_only && dof >= half) continue;
    Cx<R> pv[R4_RI];
#pragma unroll
    for (int q = 0; q < R4_RI; ++q) pv[q] = i0 + q < nv ? conj(ld<R>(P[dof * nv + i0 + q])) : Cx<R>{0, 0};
#pragma unroll
    for (int a = 0; a < R4_RR; ++a) {
      if (!on[a]) continue;
      const Cx<R> v = ld<R>(in[(long)(r0 + a) * si + dof]);
#pragma unroll
      for (int q = 0; q < R4_RI; ++q) acc[a][q] += pv[q] * v;
    }
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
// dof < n_out, (Z, c) = group of the dof (dgrp[dof] = 2 Z + c).  One thread
// per dof and a tile of R4_PB rhs (blockIdx.y): each P[dof][i] is read once
// per tile; the coarse values are shared by the thousands of dofs of a group
// and come from cache.
constexpr int R4_PB = 4;
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k4_prolong(Cx<VO>* out, long so, const Cx<VO>* add, long sa, const Cx<VI>* in,
                                                  const Cx<PT>* __restrict__ P, const int* __restrict__ dgrp,
                                                  int nv, long n_out, long ncoarse, const int* act, int nrhs) {
  const long dof = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * R4_PB;
  if (dof >= n_out) return;
  bool on[R4_PB];
#pragma unroll
  for (int b = 0; b < R4_PB; ++b) on[b] = r0 + b < nrhs && is_active(act, r0 + b);
  const int gidx = dgrp[dof];
  const Cx<VI>* e = in + (long)(gidx >> 1) * 2 * nv + (gidx & 1) * nv;
  Cx<R> acc[R4_PB];
#pragma unroll
  for (int b = 0; b < R4_PB; ++b) acc[b] = Cx<R>{0, 0};
  for (int i = 0; i < nv; ++i) {
    const Cx<R> pv = ld<R>(P[dof * nv + i]);
#pragma unroll
    for (int b = 0; b < R4_PB; ++b)
      if (on[b]) acc[b] += pv * ld<R>(e[(long)(r0 + b) * ncoarse + i]);
  }
#pragma unroll
  for (int b = 0; b < R4_PB; ++b) {
    if (!on[b]) continue;
    const long r = r0 + b;
    Cx<R> o = acc[b];
    if (add) o += ld<R>(add[r * sa + dof]);
    out[r * so + dof] = st<VO>(o);
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
