// Setup kernels shared by every coarsening: per-aggregate thin QR and the
// coarse-to-coarser Galerkin product.
#include "internal.h"

namespace kdmg {

__device__ __forceinline__ c64 block_sum_c64(c64 v, c64* red) {
  // wave64 shuffles, then one partial per wave through LDS; result broadcast
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_down(v.re, off, 64);
    v.im += __shfl_down(v.im, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  c64 s{0, 0};
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// Thin QR (modified Gram-Schmidt, positive real diagonal) of the nv vectors
// restricted to the rows of group blockIdx.x.  Rows of a group are global dof
// indices rows[g*nrows + k]; the result column i is written to P[dof*nv + i].
__global__ __launch_bounds__(256) void k_blockqr(c64* P, const c64* V, long n, const int* rows,
                                                 int nrows, int nv) {
  extern __shared__ unsigned char smem_raw[];
  c64* M = reinterpret_cast<c64*>(smem_raw);  // [nrows][nv]
  __shared__ c64 red[4];
  const int grp = blockIdx.x;
  const int* rw = rows + (long)grp * nrows;
  for (int e = threadIdx.x; e < nrows * nv; e += blockDim.x) {
    const int k = e / nv, i = e % nv;
    M[e] = V[(long)i * n + rw[k]];
  }
  __syncthreads();
  for (int i = 0; i < nv; ++i) {
    for (int j = 0; j < i; ++j) {
      c64 d{0, 0};
      for (int k = threadIdx.x; k < nrows; k += blockDim.x) cfma_conj(d, M[k * nv + j], M[k * nv + i]);
      d = block_sum_c64(d, red);
      for (int k = threadIdx.x; k < nrows; k += blockDim.x) {
        c64 q = M[k * nv + j];
        M[k * nv + i] -= d * q;
      }
      __syncthreads();
    }
    c64 nn{0, 0};
    for (int k = threadIdx.x; k < nrows; k += blockDim.x) nn.re += norm2(M[k * nv + i]);
    nn = block_sum_c64(nn, red);
    const double inv = 1.0 / sqrt(nn.re);
    for (int k = threadIdx.x; k < nrows; k += blockDim.x) M[k * nv + i] = inv * M[k * nv + i];
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nrows * nv; e += blockDim.x) {
    const int k = e / nv, i = e % nv;
    P[(long)rw[k] * nv + i] = M[e];
  }
}

__global__ __launch_bounds__(1024) void k_galerkin_c(c64* Ytn, const c64* Yt, const c64* Pst,
                                                     const int* nbr, const int* gdir,
                                                     const int* children, int nchild, int nsf,
                                                     int ndf, int nZ, int nv, int ndir) {
  extern __shared__ unsigned char smem_raw[];
  c64* T = reinterpret_cast<c64*>(smem_raw);  // [ndf][ndn]
  const int Z = blockIdx.x, t = threadIdx.x;
  const int ndn = 2 * nv, nvp = ndf / 2;
  const bool owner = t < ndn * ndn;
  const int row = owner ? t / ndn : 0, col = owner ? t % ndn : 0;
  c64 acc[9];
  for (int d = 0; d < 9; ++d) acc[d] = c64{0, 0};
  for (int ch = 0; ch < nchild; ++ch) {
    const int X = children[(long)Z * nchild + ch];
    for (int d = 0; d < ndir; ++d) {
      const int Xn = nbr[(long)d * nsf + X];
      const int D = gdir[(long)d * nsf + X];
      __syncthreads();
      for (int e = t; e < ndf * ndn; e += blockDim.x) {
        const int a = e / ndn, cl = e % ndn;
        const int cc = cl / nv, jj = cl % nv;
        c64 s{0, 0};
        for (int ib = 0; ib < nvp; ++ib) {
          const int bb = cc * nvp + ib;
          cfma(s, Yt[(((long)d * nsf + X) * ndf + bb) * ndf + a], Pst[((long)Xn * ndf + bb) * nv + jj]);
        }
        T[e] = s;
      }
      __syncthreads();
      if (owner) {
        const int c = row / nv, i = row % nv;
        c64 s{0, 0};
        for (int ia = 0; ia < nvp; ++ia) {
          const int aa = c * nvp + ia;
          cfma_conj(s, Pst[((long)X * ndf + aa) * nv + i], T[aa * ndn + col]);
        }
        for (int q = 0; q < 9; ++q)
          if (q == D) acc[q] += s;
      }
    }
  }
  if (owner)
    for (int d = 0; d < ndir; ++d) Ytn[(((long)d * nZ + Z) * ndn + col) * ndn + row] = acc[d];
}

}  // namespace kdmg
