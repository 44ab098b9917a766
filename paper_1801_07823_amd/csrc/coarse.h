// Coarse-level kernels: block-stencil apply (and its adjoint), restriction and
// prolongation between coarse levels, the Galerkin triple product, and the
// per-aggregate thin QR that builds every prolongator.
//
// A coarse operator on a lattice of `nsites` sites with `ndc` dofs per site is
// a (2 nd + 1)-point block stencil (Sec. 3: the Galerkin projection of a
// nearest-neighbour operator couples nearest-neighbour aggregates only):
//   (A v)(X) = sum_dir Y_dir(X) v(nbr(X, dir)),
// dir 0 = X itself, 1 + 2 mu = X + mu, 2 + 2 mu = X - mu.  Blocks are stored
// column-major, Yt[dir][X][j][i] = Y_dir(X)[i][j], so that the lanes of a
// wavefront (consecutive i) read consecutive addresses.  The adjoint is
// stored as its own stencil, Yd_dir(X) = Y_{-dir}(X + dir)^dag.
// Vectors are [rhs][X][dof].
#pragma once
#include "common.h"
#include "blas.h"
#include "fine2d.h"

namespace kdmg {

// out[r][X][i] = [add[r][X][i] +] sgn * sum_{dir,j} Y_dir(X)[i][j] in[r][nbr][j]
// Block: ndc * js * rpb threads; grid (nsites, ceil(nrhs/rpb)).
template <class R, class OT, class VI, class VO>
__global__ __launch_bounds__(1024) void k_capply(Cx<VO>* out, const Cx<VI>* in, const Cx<VO>* add,
                                                  R sgn, const Cx<OT>* Yt, const int* nbr,
                                                  int nsites, int ndc, int ndir, int js, int rpb,
                                                  int nrhs, const int* act) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* sh = reinterpret_cast<Cx<R>*>(smem_raw);
  const int X = blockIdx.x;
  const int t = threadIdx.x;
  const int i = t % ndc, jp = (t / ndc) % js, rr = t / (ndc * js);
  const int r = blockIdx.y * rpb + rr;
  const bool live = r < nrhs && is_active(act, r);
  Cx<R> acc{0, 0};
  if (live) {
    const long vs = (long)nsites * ndc;
    const Cx<VI>* v = in + r * vs;
    const int nf = ndir * ndc;
    for (int f = jp; f < nf; f += js) {
      const int d = f / ndc, j = f - d * ndc;
      const int Xn = nbr[(long)d * nsites + X];
      cfma(acc, ld<R>(Yt[(((long)d * nsites + X) * ndc + j) * ndc + i]), ld<R>(v[(long)Xn * ndc + j]));
    }
  }
  if (js > 1) {
    sh[t] = acc;
    __syncthreads();
    if (jp != 0) return;
    for (int q = 1; q < js; ++q) acc += sh[(rr * js + q) * ndc + i];
  }
  if (!live) return;
  const long o = ((long)r * nsites + X) * ndc + i;
  Cx<R> res = sgn * acc;
  if (add) res += ld<R>(add[o]);
  out[o] = st<VO>(res);
}

// Yd[dir][X][col][row] = conj(Yt[opp(dir)][nbr(X,dir)][row][col])
template <class T>
__global__ void k_dagger_build(Cx<T>* Yd, const Cx<T>* Yt, const int* nbr, int nsites, int ndc,
                               int ndir) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)ndc * ndc;
  if (e >= (long)ndir * nsites * per) return;
  const int row = (int)(e % ndc);
  const int col = (int)((e / ndc) % ndc);
  const long X = (e / per) % nsites;
  const int d = (int)(e / (per * nsites));
  const int opp = d == 0 ? 0 : (d & 1 ? d + 1 : d - 1);
  const int Xn = nbr[(long)d * nsites + X];
  Yd[e] = conj(Yt[(((long)opp * nsites + Xn) * ndc + row) * ndc + col]);
}

// Restriction between coarse levels:
// out[r][Z][c*nv + j] = sum_{X in Z} sum_{i<nvp} conj(Pst[X][c*nvp+i][j]) in[r][X][c*nvp+i]
// One workgroup per (aggregate Z, tile of RB rhs): the aggregate's P rows
// (nchild * ndf of them) and the tile's input values are staged in LDS, so P
// is read once per tile and the inputs with coalesced loads; thread o then
// forms outputs (rhs o / ndn, coarse dof o % ndn).  grid (nZ, cdiv(nrhs, RB));
// LDS (nchild ndf nv + RB nchild ndf) Cx<R>.  children[Z][nchild].
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k_restrict_c(Cx<VO>* out, const Cx<VI>* in, const Cx<PT>* Pst,
                                                    const int* children, int nchild, int nsf,
                                                    int ndf, int nZ, int nv, const int* act, int nrhs, int RB) {
  extern __shared__ __align__(16) unsigned char xc_raw[];
  const int Z = blockIdx.x, r0 = blockIdx.y * RB;
  const int ndn = 2 * nv, nvp = ndf / 2, nrow = nchild * ndf;
  Cx<R>* Ps = reinterpret_cast<Cx<R>*>(xc_raw);  // [nrow][nv]
  Cx<R>* Vs = Ps + (long)nrow * nv;              // [RB][nrow]
  const int* kids = children + (long)Z * nchild;
  stage_rows<R, 4>(Ps, nv, nrow, nv, [&](int q, int j) {
    const int ch = q / ndf, a = q - ch * ndf;
    return ld<R>(Pst[((long)kids[ch] * ndf + a) * nv + j]);
  });
  stage_rows<R, 4>(Vs, nrow, RB, nrow, [&](int t, int q) {
    const int ch = q / ndf, a = q - ch * ndf, r = r0 + t;
    return r < nrhs && is_active(act, r) ? ld<R>(in[((long)r * nsf + kids[ch]) * ndf + a]) : Cx<R>{0, 0};
  });
  __syncthreads();
  for (int o = threadIdx.x; o < RB * ndn; o += blockDim.x) {
    const int t = o / ndn, col = o - t * ndn, r = r0 + t;
    if (r >= nrhs || !is_active(act, r)) continue;
    const int c = col / nv, j = col - c * nv;
    const Cx<R>* v = Vs + (long)t * nrow;
    Cx<R> acc{0, 0};
    for (int ch = 0; ch < nchild; ++ch)
      for (int i = 0; i < nvp; ++i) {
        const int q = ch * ndf + c * nvp + i;
        cfma_conj(acc, Ps[q * nv + j], v[q]);
      }
    out[((long)r * nZ + Z) * ndn + col] = st<VO>(acc);
  }
}

// Prolongation between coarse levels:
// out[r][X][a] = [add +] sum_j Pst[X][a][j] in[r][parent(X)][c(a)*nv + j]
// One workgroup per (aggregate Z, tile of RB rhs), P rows (padded to nv + 1
// against bank conflicts) and the tile's coarse values staged in LDS; thread
// o forms outputs (rhs o / nrow, row o % nrow of the aggregate).
// grid (nZ, cdiv(nrhs, RB)); LDS (nchild ndf (nv + 1) + RB ndn) Cx<R>.
template <class R, class PT, class VI, class VO>
__global__ __launch_bounds__(256) void k_prolong_c(Cx<VO>* out, const Cx<VO>* add, const Cx<VI>* in,
                                                   const Cx<PT>* Pst, const int* children, int nchild, int nsf,
                                                   int ndf, int nZ, int nv, const int* act, int nrhs, int RB) {
  extern __shared__ __align__(16) unsigned char xc_raw[];
  const int Z = blockIdx.x, r0 = blockIdx.y * RB;
  const int ndn = 2 * nv, nvp = ndf / 2, nrow = nchild * ndf, RP = nv + 1;
  Cx<R>* Ps = reinterpret_cast<Cx<R>*>(xc_raw);  // [nrow][nv + 1]
  Cx<R>* Es = Ps + (long)nrow * RP;              // [RB][ndn]
  const int* kids = children + (long)Z * nchild;
  stage_rows<R, 4>(Ps, RP, nrow, nv, [&](int q, int j) {
    const int ch = q / ndf, a = q - ch * ndf;
    return ld<R>(Pst[((long)kids[ch] * ndf + a) * nv + j]);
  });
  stage_rows<R, 4>(Es, ndn, RB, ndn, [&](int t, int j) {
    const int r = r0 + t;
    return r < nrhs ? ld<R>(in[((long)r * nZ + Z) * ndn + j]) : Cx<R>{0, 0};
  });
  __syncthreads();
  for (int o = threadIdx.x; o < RB * nrow; o += blockDim.x) {
    const int t = o / nrow, q = o - t * nrow, r = r0 + t;
    if (r >= nrhs || !is_active(act, r)) continue;
    const int ch = q / ndf, a = q - ch * ndf, c = a / nvp;
    const long X = children[(long)Z * nchild + ch];
    const Cx<R>* pq = Ps + q * RP;
    const Cx<R>* er = Es + t * ndn + c * nv;
    Cx<R> acc{0, 0};
    for (int j = 0; j < nv; ++j) cfma(acc, pq[j], er[j]);
    const long ob = ((long)r * nsf + X) * ndf + a;
    if (add) acc += ld<R>(add[ob]);
    out[ob] = st<VO>(acc);
  }
}

// Galerkin triple product between coarse levels (FP64):
// Y'_D(Z) += Pfull(X)^dag Y_d(X) Pfull(nbr(X,d)) for every child X of Z and
// direction d, D = gdir[d][X] (the coarse direction the hop maps to).
// One workgroup per Z; ndn*ndn <= blockDim threads each own one output entry.
__global__ __launch_bounds__(1024) void k_galerkin_c(c64* Ytn, const c64* Yt, const c64* Pst,
                                                     const int* nbr, const int* gdir,
                                                     const int* children, int nchild, int nsf,
                                                     int ndf, int nZ, int nv, int ndir);

// Thin QR with positive real diagonal (modified Gram-Schmidt in vector order)
// of nv vectors restricted to the rows of each (aggregate, chirality) group.
// V: [v][n] FP64 vectors; rows[g][nrows] global dof indices; P[dof][i] out.
__global__ __launch_bounds__(256) void k_blockqr(c64* P, const c64* V, long n, const int* rows,
                                                 int nrows, int nv);

}  // namespace kdmg
