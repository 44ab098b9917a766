// Setup kernels of the 4D SU(3) fine level: dense Kahler-Dirac block
// inverses, block orthonormalisation (Cholesky-QR) and the level-1 Galerkin
// product (layouts and formulas in fine4d.h).
#include "fine4d.h"

namespace kdmg {

// B^-1 of every block of parity blockIdx.z at mass m, FP64 (see the header).
__global__ __launch_bounds__(256) void k4_binv_build(c64* Bv, const c64* __restrict__ lk, Geo4 g, double m) {
  __shared__ c64 K[24][24];       // even-site dofs x odd-site dofs
  __shared__ c64 Ae[24][48];      // [S_e | I] -> [I | S_e^-1]
  __shared__ c64 Ao[24][48];      // [S_o | I] -> [I | S_o^-1]
  __shared__ c64 fe[24], fo[24];
  __shared__ int esite[8], osite[8], epos[16];
  const int b = blockIdx.x, p = blockIdx.z, tid = threadIdx.x, nt = blockDim.x;
  const long blk = (long)p * g.Nb2 + b;
  if (tid == 0) {
    int ne = 0, no = 0;
    for (int s = 0; s < 16; ++s) {
      if (chir4(s) == 0) {
        epos[s] = ne;
        esite[ne++] = s;
      } else {
        epos[s] = no;
        osite[no++] = s;
      }
    }
  }
  __syncthreads();
  // K: B restricted to (even rows, odd columns); intra-block hop partners differ in one bit
  for (int t = tid; t < 576; t += nt) {
    const int row = t / 24, col = t - row * 24;
    const int se = esite[row / 3], so_ = osite[col / 3], a = row % 3, bb = col % 3;
    const int d = se ^ so_;
    c64 v{0, 0};
    if (__builtin_popcount((unsigned)d) == 1) {
      const int mu = __builtin_ctz((unsigned)d);
      if (((se >> mu) & 1) == 0) {  // forward hop se -> so_: +U~_mu(se)
        v = lk[((blk * 16 + se) * 4 + mu) * 9 + a * 3 + bb];
      } else {                      // backward hop se -> so_: -U~_mu(so_)^dag
        const c64 u = lk[((blk * 16 + so_) * 4 + mu) * 9 + bb * 3 + a];
        v = c64{-u.re, u.im};
      }
    }
    K[row][col] = v;
  }
  __syncthreads();
  const double m2 = m * m;
  for (int t = tid; t < 24 * 48; t += nt) {
    const int i = t / 48, j = t - i * 48;
    c64 se{0, 0}, sov{0, 0};
    if (j < 24) {
      for (int k = 0; k < 24; ++k) {
        se += K[i][k] * conj(K[j][k]);   // (K K^dag)_{ij}
        sov += conj(K[k][i]) * K[k][j];  // (K^dag K)_{ij}
      }
      if (i == j) {
        se.re += m2;
        sov.re += m2;
      }
    } else {
      se = sov = c64{j - 24 == i ? 1.0 : 0.0, 0.0};
    }
    Ae[i][j] = se;
    Ao[i][j] = sov;
  }
  for (int k = 0; k < 24; ++k) {
    __syncthreads();
    const double pe = 1.0 / Ae[k][k].re, po = 1.0 / Ao[k][k].re;  // positive real pivots
    __syncthreads();
    for (int j = tid; j < 48; j += nt) {
      Ae[k][j] = pe * Ae[k][j];
      Ao[k][j] = po * Ao[k][j];
    }
    for (int i = tid; i < 24; i += nt) {
      fe[i] = Ae[i][k];
      fo[i] = Ao[i][k];
    }
    __syncthreads();
    for (int t = tid; t < 24 * 48; t += nt) {
      const int i = t / 48, j = t - i * 48;
      if (i == k) continue;
      Ae[i][j] -= fe[i] * Ae[k][j];
      Ao[i][j] -= fo[i] * Ao[k][j];
    }
  }
  __syncthreads();
  // assemble B^-1 in (s, c) order, column-major
  for (int t = tid; t < 48 * 48; t += nt) {
    const int j = t / 48, i = t - j * 48;  // column j, row i
    const int si = i / 3, ci = i % 3, sj = j / 3, cj = j % 3;
    const int ie = epos[si] * 3 + ci, je = epos[sj] * 3 + cj;
    const bool ev_i = chir4(si) == 0, ev_j = chir4(sj) == 0;
    c64 v{0, 0};
    if (ev_i && ev_j) {
      v = m * Ae[ie][24 + je];
    } else if (!ev_i && !ev_j) {
      v = m * Ao[ie][24 + je];
    } else if (ev_i) {  // -(K S_o^-1)_{ie, jo}
      for (int k = 0; k < 24; ++k) v -= K[ie][k] * Ao[k][24 + je];
    } else {            // (K^dag S_e^-1)_{io, je}
      for (int k = 0; k < 24; ++k) v += conj(K[k][ie]) * Ae[k][24 + je];
    }
    Bv[(blk * 48 + j) * 48 + i] = v;
  }
}

// Gram matrices of the (aggregate, chirality) groups: G[g][i][j] =
// sum_{dof in g} V(dof, i)^* V(dof, j), with V(dof, i) = V[i sv + dof sd].
// One workgroup per group; rows are staged through LDS in chunks of 64.
__global__ __launch_bounds__(256) void k4_gram(c64* G, const c64* __restrict__ V, long sv, long sd,
                                               const int* __restrict__ rows, int nrows, int nv) {
  __shared__ c64 tile[64][33];
  const int gid = blockIdx.x, tid = threadIdx.x;
  const int ne = nv * nv;
  c64 acc[4] = {c64{0, 0}, c64{0, 0}, c64{0, 0}, c64{0, 0}};
  for (int k0 = 0; k0 < nrows; k0 += 64) {
    __syncthreads();
    for (int t = tid; t < 64 * nv; t += blockDim.x) {
      const int kr = t / nv, i = t - kr * nv, k = k0 + kr;
      tile[kr][i] = k < nrows ? V[i * sv + (long)rows[(long)gid * nrows + k] * sd] : c64{0, 0};
    }
    __syncthreads();
    const int kmax = nrows - k0 < 64 ? nrows - k0 : 64;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * blockDim.x;
      if (e >= ne) continue;
      const int i = e / nv, j = e - i * nv;
      for (int kr = 0; kr < kmax; ++kr) acc[q] += conj(tile[kr][i]) * tile[kr][j];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * blockDim.x;
    if (e < ne) G[(long)gid * ne + e] = acc[q];
  }
}

// Rinv[g] = R^-1 with G[g] = R^dag R (Cholesky, R upper triangular with a
// positive real diagonal).  One thread per group.
__global__ void k4_chol_inv(c64* Rinv, const c64* G, int ngroups, int nv) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ngroups) return;
  const c64* A = G + (long)gid * nv * nv;
  c64* Ri = Rinv + (long)gid * nv * nv;
  c64 Rm[32][32];
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) Rm[i][j] = c64{0, 0};
  for (int j = 0; j < nv; ++j) {
    double d = A[j * nv + j].re;
    for (int k = 0; k < j; ++k) d -= norm2(Rm[k][j]);
    d = sqrt(d > 0 ? d : 1e-300);
    Rm[j][j] = c64{d, 0};
    for (int i = j + 1; i < nv; ++i) {
      c64 s = A[j * nv + i];  // (R^dag R)_{ji} = sum_k conj(R_kj) R_ki
      for (int k = 0; k < j; ++k) s -= conj(Rm[k][j]) * Rm[k][i];
      Rm[j][i] = (1.0 / d) * s;
    }
  }
  // upper-triangular inverse, column by column
  for (int j = 0; j < nv; ++j)
    for (int i = nv - 1; i >= 0; --i) {
      c64 s = c64{i == j ? 1.0 : 0.0, 0.0};
      for (int k = i + 1; k <= j; ++k) s -= Rm[i][k] * Ri[k * nv + j];
      Ri[i * nv + j] = (i <= j) ? (1.0 / Rm[i][i].re) * s : c64{0, 0};
    }
}

// Q[dof][j] = sum_{i <= j} V(dof, i) Rinv[g][i][j] for the dofs of every group
// (Q in the prolongator layout [dof][nv]).
__global__ __launch_bounds__(256) void k4_qapply(c64* Q, const c64* __restrict__ V, long sv, long sd,
                                                 const c64* __restrict__ Rinv, const int* __restrict__ rows,
                                                 int nrows, int nv) {
  const int gid = blockIdx.x;
  const c64* Ri = Rinv + (long)gid * nv * nv;
  for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < nrows; k += gridDim.y * blockDim.x) {
    const long dof = rows[(long)gid * nrows + k];
    c64 v[32];
    for (int i = 0; i < nv; ++i) v[i] = V[i * sv + dof * sd];
    for (int j = 0; j < nv; ++j) {
      c64 s{0, 0};
      for (int i = 0; i <= j; ++i) s += v[i] * Ri[i * nv + j];
      Q[dof * nv + j] = s;
    }
  }
}

// W = B^-1 P per block: W[dof][c nv + i] = sum_{j in block, chir(j) = c}
// (B^-1)_{dof, j} P[j][i].  One workgroup per block.
__global__ __launch_bounds__(256) void k4_gal_w(c64* W, const c64* __restrict__ P, const c64* __restrict__ Bv, Geo4 g,
                                                int nv) {
  const int b = blockIdx.x, p = blockIdx.z;
  const long blk = (long)p * g.Nb2 + b, base = blk * 48;
  const int ncol = 2 * nv;
  for (int t = threadIdx.x; t < 48 * ncol; t += blockDim.x) {
    const int il = t / ncol, col = t - il * ncol, c = col / nv, i = col - c * nv;
    c64 s{0, 0};
    for (int j = 0; j < 48; ++j) {
      if (chir4(j / 3) != c) continue;
      s += Bv[(blk * 48 + j) * 48 + il] * P[(base + j) * nv + i];
    }
    W[(base + il) * ncol + col] = s;
  }
}

// Coarse stencil block of direction `dir` (blockIdx.y) of coarse site Z
// (blockIdx.x):  A_hat(Z, Z') = delta + P^dag C W restricted to the hops from
// sites of aggregate Z that land in Z' = Z (dir 0: hops inside the aggregate)
// or cross its face in direction dir (1 + 2 mu: +mu, 2 + 2 mu: -mu).
// Output Yt[dir][Z] column-major: Yt[((dir nZ + Z) ndc + col) ndc + row].
// Hops are staged through LDS in batches of GB4.
__global__ __launch_bounds__(256) void k4_galerkin(c64* Yt, const c64* __restrict__ P, const c64* __restrict__ W,
                                                   const c64* __restrict__ lk, const int* __restrict__ nb4, Geo4 g,
                                                   int agg0, int agg1, int agg2, int agg3, int nZ, int nv) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int Z = blockIdx.x, dir = blockIdx.y, tid = threadIdx.x;
  const int ndc = 2 * nv;
  c64* Pc = reinterpret_cast<c64*>(smem_raw);        // [GB4][3][nv]   conj(P) of the hop's source site
  c64* CW = Pc + GB4 * 3 * nv;                        // [GB4][3][ndc]  C W at the source site
  int* hsrc = reinterpret_cast<int*>(CW + GB4 * 3 * ndc);  // [GB4] source site (block layout)
  int* hdst = hsrc + GB4;                                  // [GB4] destination site
  int* hmu = hdst + GB4;                                   // [GB4] 2 mu + (0 forward, 1 backward)
  const int agg[4] = {agg0, agg1, agg2, agg3};
  const int Lc[4] = {g.NB[0] / agg0, g.NB[1] / agg1, g.NB[2] / agg2, g.NB[3] / agg3};
  int Zc[4], rem = Z;
  for (int mu = 0; mu < 4; ++mu) {
    Zc[mu] = rem % Lc[mu];
    rem /= Lc[mu];
  }
  const int nblk = agg0 * agg1 * agg2 * agg3, nsite = nblk * 16;
  // each thread owns output entries e = tid + q * blockDim (row, col) of the ndc x ndc block
  constexpr int MAXQ = 16;
  c64 acc[MAXQ];
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) acc[q] = c64{0, 0};
  // Every thread walks the aggregate's sites and hops in the same order and
  // records the matching ones; batches are processed when full.
  int nh = 0;
  auto flush = [&](int count) {
    __syncthreads();
    // stage conj(P) and C W for the batch
    for (int t = tid; t < count * 3 * nv; t += blockDim.x) {
      const int h = t / (3 * nv), rq = t - h * 3 * nv, a = rq / nv, i = rq - a * nv;
      Pc[(h * 3 + a) * nv + i] = conj(P[((long)hsrc[h] * 3 + a) * nv + i]);
    }
    for (int t = tid; t < count * 3 * ndc; t += blockDim.x) {
      const int h = t / (3 * ndc), rq = t - h * 3 * ndc, a = rq / ndc, col = rq - a * ndc;
      const long x = hsrc[h], y = hdst[h];
      const int mu = hmu[h] >> 1, bwd = hmu[h] & 1;
      c64 s{0, 0};
      for (int bb = 0; bb < 3; ++bb) {
        c64 cab;
        if (!bwd) {
          cab = lk[(x * 4 + mu) * 9 + a * 3 + bb];
        } else {
          const c64 u = lk[(y * 4 + mu) * 9 + bb * 3 + a];
          cab = c64{-u.re, u.im};  // -U~_mu(y)^dag
        }
        s += cab * W[(y * 3 + bb) * ndc + col];
      }
      CW[(h * 3 + a) * ndc + col] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int e = tid + q * blockDim.x;
      if (e >= ndc * ndc) break;
      const int col = e / ndc, row = e - col * ndc, crow = row / nv, i = row - crow * nv;
      for (int h = 0; h < count; ++h) {
        if (chir4(hsrc[h] & 15) != crow) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[q] += Pc[(h * 3 + a) * nv + i] * CW[(h * 3 + a) * ndc + col];
      }
    }
    __syncthreads();  // the batch tables are rewritten next
  };
  for (int k = 0; k < nsite; ++k) {
    const int kb = k >> 4, s = k & 15;
    int lb = kb, Bc[4];
    for (int mu = 0; mu < 4; ++mu) {
      Bc[mu] = Zc[mu] * agg[mu] + lb % agg[mu];
      lb /= agg[mu];
    }
    const long x = ((long)blk4_parity(Bc) * g.Nb2 + blk4_index(g, Bc)) * 16 + s;
    for (int mu = 0; mu < 4; ++mu) {
      const int bit = (s >> mu) & 1;
      for (int bwd = 0; bwd < 2; ++bwd) {
        if (bwd == bit) continue;  // intra-block hop: part of B, not C
        // the hop leaves the KD block; does it leave the aggregate?
        const int local = Bc[mu] - Zc[mu] * agg[mu];
        const bool cross = bwd ? local == 0 : local == agg[mu] - 1;
        const int hd = cross ? 1 + 2 * mu + bwd : 0;
        if (hd != dir) continue;
        if (tid == 0) {
          hsrc[nh] = (int)x;
          hdst[nh] = nb4[x * 8 + 2 * mu + bwd];
          hmu[nh] = 2 * mu + bwd;
        }
        if (++nh == GB4) {
          flush(GB4);
          nh = 0;
        }
      }
    }
  }
  if (nh) flush(nh);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXQ; ++q) {
    const int e = tid + q * blockDim.x;
    if (e >= ndc * ndc) break;
    const int col = e / ndc, row = e - col * ndc;
    c64 v = acc[q];
    if (dir == 0 && row == col) v.re += 1.0;
    Yt[((long)dir * nZ + Z) * ndc * ndc + e] = v;
  }
}

}  // namespace kdmg
