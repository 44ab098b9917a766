// Multigrid setup (Sec. 4 and Table 1, "setup" rows): near-null vectors by CG
// on A A^dag, global modified Gram-Schmidt, chiral doubling with
// block-orthonormalisation into P, Galerkin coarse operators A_hat = P^dag A P.
#include <cstring>

#include "algos.h"
#include "api_guard.h"

using namespace kdmg;

namespace {

struct Scalars1 {  // one device complex scalar for the global Gram-Schmidt
  DevBuf d;
  Scalars1() : d(sizeof(double) * 4) {}
};

// y *= 1/sqrt(s[0])
struct OpScaleInvSqrt {
  c64* y; long n; const double* s;
  __device__ bool active(int) const { return true; }
  __device__ void elem(int, long i) const { y[i] = (1.0 / sqrt(s[0])) * y[i]; }
};

// y = -y
struct OpNeg {
  c64* y; long n;
  __device__ bool active(int) const { return true; }
  __device__ void elem(int r, long i) const { y[r * n + i] = -y[r * n + i]; }
};

// x += e
struct OpAdd {
  c64* x; const c64* e; long n;
  __device__ bool active(int) const { return true; }
  __device__ void elem(int r, long i) const { x[r * n + i] += e[r * n + i]; }
};

// Modified Gram-Schmidt over whole vectors, in vector order (FP64).
void global_mgs(const Ctx& c, c64* V, long n, int nv) {
  Scalars1 s;
  double* d = s.d.as<double>();
  for (int i = 0; i < nv; ++i) {
    c64* vi = V + (long)i * n;
    for (int j = 0; j < i; ++j) {
      const c64* vj = V + (long)j * n;
      launch_map_reduce<2>(OpDot<double>{vj, vi, n, d, nullptr}, n, 1, 1, c.rs, c.st);
      launch_map(OpAxpyDev<double>{vi, vj, n, d, 2, -1.0, nullptr}, n, 1, c.st);
    }
    launch_map_reduce<1>(OpNorm2<double>{vi, n, d + 2, nullptr}, n, 1, 1, c.rs, c.st);
    launch_map(OpScaleInvSqrt{vi, n, d + 2}, n, 1, c.st);
  }
}

void run_blockqr(const Ctx& c, c64* P, const c64* V, long n, const std::vector<int>& rows, int ngroups,
                 int nrows, int nv) {
  DevBuf drows(sizeof(int) * rows.size());
  KDMG_HIP(hipMemcpyAsync(drows.p, rows.data(), drows.bytes, hipMemcpyHostToDevice, c.st));
  const size_t smem = sizeof(c64) * (size_t)nrows * nv;
  KDMG_CHECK(smem <= 65536, KDMG_EUNSUPPORTED, "aggregate too large for the block QR kernel");
  int threads = ((nrows + 63) / 64) * 64;
  if (threads > 256) threads = 256;
  hipLaunchKernelGGL(k_blockqr, dim3(ngroups), dim3(threads), smem, c.st, P, V, n, drows.as<int>(),
                     nrows, nv);
  KDMG_LAUNCH_CHECK();
  KDMG_HIP(hipStreamSynchronize(c.st));
}

void finish_coarse_level(const Ctx& c, CoarseLevel& L) {
  const long nbytes = (long)L.ndir * L.nsites * L.ndc * L.ndc;
  if (!L.Yd64.p) L.Yd64.alloc(sizeof(c64) * nbytes);
  if (!L.Yt32.p) L.Yt32.alloc(sizeof(c32) * nbytes);
  if (!L.Yd32.p) L.Yd32.alloc(sizeof(c32) * nbytes);
  hipLaunchKernelGGL(k_dagger_build<double>, dim3(cdiv(nbytes, 256)), dim3(256), 0, c.st,
                     L.Yd64.as<c64>(), L.Yt64.as<c64>(), L.nbr.as<int>(), L.nsites, L.ndc, L.ndir);
  KDMG_LAUNCH_CHECK();
  convert<float, double>(L.Yt32.as<c32>(), L.Yt64.as<c64>(), nbytes, 1, nullptr, c.st);
  convert<float, double>(L.Yd32.as<c32>(), L.Yd64.as<c64>(), nbytes, 1, nullptr, c.st);
}

void make_nbr(CoarseLevel& L) {
  const int nd = L.nd;
  L.ndir = 2 * nd + 1;
  L.nsites = 1;
  for (int mu = 0; mu < nd; ++mu) L.nsites *= L.dims[mu];
  L.h_nbr.assign((size_t)L.ndir * L.nsites, 0);
  for (int X = 0; X < L.nsites; ++X) {
    int co[4], rem = X;
    for (int mu = 0; mu < nd; ++mu) { co[mu] = rem % L.dims[mu]; rem /= L.dims[mu]; }
    L.h_nbr[X] = X;
    for (int mu = 0; mu < nd; ++mu)
      for (int sgn = 0; sgn < 2; ++sgn) {
        int cc[4];
        std::memcpy(cc, co, sizeof(cc));
        cc[mu] = (co[mu] + (sgn == 0 ? 1 : L.dims[mu] - 1)) % L.dims[mu];
        int idx = 0, str = 1;
        for (int nu = 0; nu < nd; ++nu) { idx += cc[nu] * str; str *= L.dims[nu]; }
        L.h_nbr[(size_t)(1 + 2 * mu + sgn) * L.nsites + X] = idx;
      }
  }
  L.nbr.alloc(sizeof(int) * L.h_nbr.size());
  KDMG_HIP(hipMemcpy(L.nbr.p, L.h_nbr.data(), L.nbr.bytes, hipMemcpyHostToDevice));
}

// Relax the columns of V (nv vectors of length n) with CG on `normal`:
// solve normal e = -normal V to tol (relative) or maxit iterations, V += e.
template <class NormalF>
void relax(const Ctx& c, c64* V, long n, int nv, double tol, int maxit, NormalF normal) {
  DevBuf b(sizeof(c64) * n * nv), x(sizeof(c64) * n * nv), r(sizeof(c64) * n * nv),
      p(sizeof(c64) * n * nv), q(sizeof(c64) * n * nv);
  KrylovAlloc ka;
  ka.init(nv);
  normal(b.as<c64>(), V, (const int*)nullptr);
  launch_map(OpNeg{b.as<c64>(), n}, n, nv, c.st);
  cg_solve<double>(c, nv, n, b.as<c64>(), x.as<c64>(), r.as<c64>(), p.as<c64>(), q.as<c64>(), tol,
                   maxit, ka.k, normal, 10);
  launch_map(OpAdd{V, x.as<c64>(), n}, n, nv, c.st);
  KDMG_HIP(hipStreamSynchronize(c.st));
}

void upload(const Ctx& c, DevBuf& dst, const double* host, size_t bytes) {
  dst.alloc(bytes);
  KDMG_HIP(hipMemcpyAsync(dst.p, host, bytes, hipMemcpyHostToDevice, c.st));
}

// Level-1 Galerkin operator at the hierarchy's mass (Sec. 3, Sec. 4):
// W = B^-1 P block by block, then A_hat = 1 + P^dag C W.  Storage is reused
// when the level already exists (a rebuild at another mass).
void galerkin_level1_4d(kdmg_hierarchy& h, const Ctx& c);

// Asymmetric form (asym2d.h): W = B^-1 P, then A_hat = 1 + R C W.
void galerkin_level1_asym(kdmg_hierarchy& h, const Ctx& c) {
  const kdmg_lattice& lat = *h.lat;
  const Geo2& g = lat.g;
  const Transfer& T = h.T[0];
  const int ndc = 2 * T.nv;
  hipLaunchKernelGGL((k_galerkin_wa<double>), dim3(cdiv(g.Nb2, 256), ndc, 2), dim3(256), 0, c.st,
                     h.gal_w.as<c64>(), T.P64.as<c64>(), lat.links64.as<c64>(), g, ndc, h.mass);
  KDMG_LAUNCH_CHECK();
  CoarseLevel& C1 = h.L[1];
  if (!C1.Yt64.p) {
    C1.nd = 2;
    C1.dims[0] = T.a2.Ncx;
    C1.dims[1] = T.a2.Nct;
    C1.ndc = ndc;
    make_nbr(C1);
    C1.Yt64.alloc(sizeof(c64) * (size_t)C1.ndir * C1.nsites * C1.ndc * C1.ndc);
  }
  const int thr = ndc * ndc > 1024 ? 1024 : ndc * ndc;
  hipLaunchKernelGGL((k_galerkin1a<double>), dim3(T.a2.Ncx * T.a2.Nct), dim3(thr), 0, c.st, C1.Yt64.as<c64>(),
                     T.R64.as<c64>(), h.gal_w.as<c64>(), lat.links64.as<c64>(), g, T.a2);
  KDMG_LAUNCH_CHECK();
  finish_coarse_level(c, C1);
}

void galerkin_level1(kdmg_hierarchy& h, const Ctx& c) {
  if (h.lat->nd == 4) {
    galerkin_level1_4d(h, c);
    return;
  }
  const kdmg_lattice& lat = *h.lat;
  const Geo2& g = lat.g;
  const Transfer& T = h.T[0];
  const int nv = T.nv;
  const long f = 2 * g.half;
  const Fine2<double> F = fine2<double>(lat, h.mass);
  if (!h.gal_w.p) h.gal_w.alloc(sizeof(c64) * f * 2 * nv);
  if (T.asym) {
    galerkin_level1_asym(h, c);
    return;
  }
  // KD: W = B~^-1 P (at the rescaled mass); on D itself: W = P
  hipLaunchKernelGGL((k_galerkin_w1<double>), dim3(cdiv(g.Nb2, 256), nv, 2), dim3(256), 0, c.st,
                     h.gal_w.as<c64>(), T.P64.as<c64>(), lat.links64.as<c64>(), g, nv, F.me, h.naive ? 1 : 0);
  KDMG_LAUNCH_CHECK();
  CoarseLevel& C1 = h.L[1];
  if (!C1.Yt64.p) {
    C1.nd = 2;
    C1.dims[0] = T.a2.Ncx;
    C1.dims[1] = T.a2.Nct;
    C1.ndc = 2 * nv;
    make_nbr(C1);
    C1.Yt64.alloc(sizeof(c64) * (size_t)C1.ndir * C1.nsites * C1.ndc * C1.ndc);
  }
  const int nZ = T.a2.Ncx * T.a2.Nct;
  const int thr = C1.ndc * C1.ndc > 1024 ? 1024 : C1.ndc * C1.ndc;
  hipLaunchKernelGGL((k_galerkin1<double>), dim3(nZ), dim3(thr), 0, c.st, C1.Yt64.as<c64>(),
                     T.P64.as<c64>(), h.gal_w.as<c64>(), lat.links64.as<c64>(), g, T.a2, h.naive ? 0 : 1);
  KDMG_LAUNCH_CHECK();
  if (F.W) {  // Naik: + x P^dag C3 W
    hipLaunchKernelGGL((k_galerkin1_hop3<double>), dim3(nZ), dim3(thr), 0, c.st, C1.Yt64.as<c64>(),
                       T.P64.as<c64>(), h.gal_w.as<c64>(), lat.wl64.as<c64>(), g, T.a2, F.x);
    KDMG_LAUNCH_CHECK();
  }
  if (h.naive) {
    // the block-local part P^dag B~ P, then the overall factor s of D = s (B~ + C~)
    hipLaunchKernelGGL((k_galerkin_w1<double>), dim3(cdiv(g.Nb2, 256), nv, 2), dim3(256), 0, c.st,
                       h.gal_w.as<c64>(), T.P64.as<c64>(), lat.links64.as<c64>(), g, nv, F.me, 2);
    hipLaunchKernelGGL(k_galerkin1_self<double>, dim3(nZ), dim3(thr), 0, c.st, C1.Yt64.as<c64>(), T.P64.as<c64>(),
                       h.gal_w.as<c64>(), g, T.a2, 1.0);
    KDMG_LAUNCH_CHECK();
    if (F.s != 1.0) {
      const long ny = (long)C1.ndir * C1.nsites * C1.ndc * C1.ndc;
      launch_map(OpAxpby<double>{C1.Yt64.as<c64>(), C1.Yt64.as<c64>(), nullptr, ny, F.s, 0.0, nullptr}, ny, 1, c.st);
    }
  }
  finish_coarse_level(c, C1);
}

// Level-(k+1) Galerkin operator P^dag A_hat_k P from level k's operator.
void galerkin_coarse(kdmg_hierarchy& h, int k, const Ctx& c) {
  const CoarseLevel& Lf = h.L[k];
  CoarseLevel& Lc = h.L[k + 1];
  const Transfer& T = h.T[k];
  const kdmg_level_params& lp = h.params.lvl[k];
  if (!Lc.Yt64.p) {
    Lc.nd = Lf.nd;
    for (int mu = 0; mu < Lf.nd; ++mu) Lc.dims[mu] = Lf.dims[mu] / lp.agg[mu];
    Lc.ndc = 2 * T.nv;
    make_nbr(Lc);
    Lc.Yt64.alloc(sizeof(c64) * (size_t)Lc.ndir * Lc.nsites * Lc.ndc * Lc.ndc);
  }
  const size_t smem = sizeof(c64) * (size_t)T.ndf * Lc.ndc;
  KDMG_CHECK(smem <= 65536 && Lc.ndc * Lc.ndc <= 1024 && Lf.ndir <= 9, KDMG_EUNSUPPORTED,
             "coarse Galerkin shape not supported");
  hipLaunchKernelGGL(k_galerkin_c, dim3(T.nZ), dim3(Lc.ndc * Lc.ndc), smem, c.st, Lc.Yt64.as<c64>(),
                     Lf.Yt64.as<c64>(), T.P64.as<c64>(), Lf.nbr.as<int>(), T.gdir.as<int>(),
                     T.children.as<int>(), T.nchild, T.nsf, T.ndf, T.nZ, T.nv, Lf.ndir);
  KDMG_LAUNCH_CHECK();
  finish_coarse_level(c, Lc);
}

// ------------------------------------------------------------------ 4D SU(3), level 1

// Level-1 Galerkin operator on a 4D lattice at h.mass: B^-1 blocks at this
// mass, W = B^-1 P block by block, then A_hat = 1 + P^dag C W per (coarse
// site, direction).
void galerkin_level1_4d(kdmg_hierarchy& h, const Ctx& c) {
  const kdmg_lattice& lat = *h.lat;
  const Geo4& g = lat.g4;
  const Transfer& T = h.T[0];
  const int nv = T.nv, ndc = 2 * nv;
  const long f = 2 * g.half;
  build_binv4(h.binv64, h.binv32, lat, h.mass, c.st);
  if (!h.gal_w.p) h.gal_w.alloc(sizeof(c64) * f * ndc);
  hipLaunchKernelGGL(k4_gal_w, dim3(g.Nb2, 1, 2), dim3(256), 0, c.st, h.gal_w.as<c64>(), T.P64.as<c64>(),
                     h.binv64.as<c64>(), g, nv);
  KDMG_LAUNCH_CHECK();
  CoarseLevel& C1 = h.L[1];
  if (!C1.Yt64.p) {
    C1.nd = 4;
    for (int mu = 0; mu < 4; ++mu) C1.dims[mu] = g.NB[mu] / T.agg4[mu];
    C1.ndc = ndc;
    make_nbr(C1);
    C1.Yt64.alloc(sizeof(c64) * (size_t)C1.ndir * C1.nsites * ndc * ndc);
  }
  KDMG_CHECK(ndc * ndc <= 16 * 256, KDMG_EUNSUPPORTED, "4D Galerkin: 2 n_vec must be <= 64");
  const size_t smem = sizeof(c64) * GB4 * 3 * (nv + ndc) + sizeof(int) * 3 * GB4;
  hipLaunchKernelGGL(k4_galerkin, dim3(C1.nsites, C1.ndir), dim3(256), smem, c.st, C1.Yt64.as<c64>(),
                     T.P64.as<c64>(), h.gal_w.as<c64>(), lat.lk64.as<c64>(), lat.nb4.as<int>(), g, T.agg4[0],
                     T.agg4[1], T.agg4[2], T.agg4[3], C1.nsites, nv);
  KDMG_LAUNCH_CHECK();
  finish_coarse_level(c, C1);
}

// Cholesky-QR applied twice per (aggregate, chirality) group: the thin QR
// with positive real diagonal of the group's rows of V (unique, so equal to
// the oracle's Householder QR up to rounding).  V(dof, i) = V[i sv + dof sd];
// P receives Q in the prolongator layout [dof][nv].
void block_cholqr2(c64* P, const c64* V, long sv, long sd, const Transfer& T, long f, hipStream_t st) {
  const int nv = T.nv, ng = 2 * T.nZ;
  DevBuf G(sizeof(c64) * ng * nv * nv), Ri(sizeof(c64) * ng * nv * nv), Q1(sizeof(c64) * f * nv);
  const int* rows = T.rows4.as<int>();
  const int ychunks = (T.nrows4 + 255) / 256 < 64 ? (T.nrows4 + 255) / 256 : 64;
  // pass 1: V -> Q1
  hipLaunchKernelGGL(k4_gram, dim3(ng), dim3(256), 0, st, G.as<c64>(), V, sv, sd, rows, T.nrows4, nv);
  hipLaunchKernelGGL(k4_chol_inv, dim3(cdiv(ng, 64)), dim3(64), 0, st, Ri.as<c64>(), G.as<c64>(), ng, nv);
  hipLaunchKernelGGL(k4_qapply, dim3(ng, ychunks), dim3(256), 0, st, Q1.as<c64>(), V, sv, sd, Ri.as<c64>(), rows,
                     T.nrows4, nv);
  // pass 2: Q1 -> P
  hipLaunchKernelGGL(k4_gram, dim3(ng), dim3(256), 0, st, G.as<c64>(), Q1.as<c64>(), 1L, (long)nv, rows, T.nrows4, nv);
  hipLaunchKernelGGL(k4_chol_inv, dim3(cdiv(ng, 64)), dim3(64), 0, st, Ri.as<c64>(), G.as<c64>(), ng, nv);
  hipLaunchKernelGGL(k4_qapply, dim3(ng, ychunks), dim3(256), 0, st, P, Q1.as<c64>(), 1L, (long)nv, Ri.as<c64>(),
                     rows, T.nrows4, nv);
  KDMG_LAUNCH_CHECK();
  KDMG_HIP(hipStreamSynchronize(st));
}

// fine 4D lattice -> first coarse lattice
void build_level1_4d(kdmg_hierarchy& h, const Ctx& c, const double* psi0, int relaxed) {
  const kdmg_lattice& lat = *h.lat;
  const Geo4& g = lat.g4;
  const kdmg_level_params& lp = h.params.lvl[0];
  const int nv = lp.nvec;
  Transfer& T = h.T[0];
  T.k = 0;
  T.nv = nv;
  int nblk = 1;
  T.nZ = 1;
  for (int mu = 0; mu < 4; ++mu) {
    T.agg4[mu] = lp.agg[mu];
    KDMG_CHECK(lp.agg[mu] >= 1 && g.NB[mu] % lp.agg[mu] == 0, KDMG_EINVAL,
               "first aggregate must divide the KD-block lattice");
    nblk *= lp.agg[mu];
    T.nZ *= g.NB[mu] / lp.agg[mu];
  }
  T.nrows4 = nblk * 16 * 3 / 2;
  KDMG_CHECK(nv >= 1 && nv <= T.nrows4 && 2 * nv <= 64 && nv <= 32, KDMG_EINVAL,
             "n_vec must not exceed the dofs of one aggregate chirality (and n_vec <= 32)");
  const long f = 2 * g.half, V = lat.volume, nd = lat.ndof;
  T.nfine = f;
  // (aggregate, chirality) groups, dofs in increasing block-layout order
  std::vector<int> rows((size_t)2 * T.nZ * T.nrows4), dgrp(f), fill(2 * T.nZ, 0), neven(2 * T.nZ, 0);
  int Lc[4];
  for (int mu = 0; mu < 4; ++mu) Lc[mu] = g.NB[mu] / T.agg4[mu];
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < g.Nb2; ++b) {
      int Bc[4];
      blk4_coords(g, p, b, Bc);
      int Z = 0, str = 1;
      for (int mu = 0; mu < 4; ++mu) {
        Z += (Bc[mu] / T.agg4[mu]) * str;
        str *= Lc[mu];
      }
      for (int s = 0; s < 16; ++s)
        for (int a = 0; a < 3; ++a) {
          const long dof = (((long)p * g.Nb2 + b) * 16 + s) * 3 + a;
          const int gid = 2 * Z + chir4(s);
          rows[(size_t)gid * T.nrows4 + fill[gid]++] = (int)dof;
          dgrp[dof] = gid;
          if (p == 0) ++neven[gid];  // parity-0 blocks come first: dof < half
        }
    }
  for (int q = 0; q < 2 * T.nZ; ++q) KDMG_CHECK(fill[q] == T.nrows4, KDMG_EINVAL, "aggregate group size mismatch");
  T.rows4.alloc(sizeof(int) * rows.size());
  T.dgrp4.alloc(sizeof(int) * dgrp.size());
  T.neven4.alloc(sizeof(int) * neven.size());
  KDMG_HIP(hipMemcpy(T.neven4.p, neven.data(), T.neven4.bytes, hipMemcpyHostToDevice));
  KDMG_HIP(hipMemcpy(T.rows4.p, rows.data(), T.rows4.bytes, hipMemcpyHostToDevice));
  KDMG_HIP(hipMemcpy(T.dgrp4.p, dgrp.data(), T.dgrp4.bytes, hipMemcpyHostToDevice));
  // starting vectors: natural order -> block layout
  DevBuf nat;
  upload(c, nat, psi0, sizeof(c64) * nd * nv);
  DevBuf Vb(sizeof(c64) * f * nv);
  launch_permute<double, double>(Vb.as<c64>(), f, nat.as<c64>(), nd, lat.perm_full.as<int>(), nd, 1, nv, c.st);
  if (!relaxed) {
    build_binv4(h.binv64, h.binv32, lat, h.mass, c.st);
    const Fine4<double, double> F{lat.lk64.as<c64>(), lat.nb4.as<int>(), h.binv64.as<c64>(), g, h.mass};
    DevBuf u(sizeof(c64) * f * nv), t(sizeof(c64) * f * nv);
    auto normal = [&](c64* out, const c64* in, const int* act) {
      fullAdag_apply4<double, double>(u.as<c64>(), in, t.as<c64>(), F, act, nv, c.st);
      fullA_apply4<double, double>(out, u.as<c64>(), t.as<c64>(), F, act, nv, c.st);
    };
    relax(c, Vb.as<c64>(), f, nv, h.params.setup_tol, h.params.setup_maxit, normal);
  }
  T.relaxed.alloc(Vb.bytes);
  KDMG_HIP(hipMemcpyAsync(T.relaxed.p, Vb.p, Vb.bytes, hipMemcpyDeviceToDevice, c.st));
  global_mgs(c, Vb.as<c64>(), f, nv);
  T.P64.alloc(sizeof(c64) * f * nv);
  block_cholqr2(T.P64.as<c64>(), Vb.as<c64>(), f, 1, T, f, c.st);
  T.P16.alloc(sizeof(c16) * f * nv);
  convert<_Float16, double>(T.P16.as<c16>(), T.P64.as<c64>(), f * nv, 1, nullptr, c.st);
  galerkin_level1_4d(h, c);
  KDMG_HIP(hipStreamSynchronize(c.st));
}

// P and R of the asymmetric first coarsening from the orthonormalised
// vectors V (block layout [nv][f]), at the hierarchy's mass.
void build_asym_transfer(kdmg_hierarchy& h, const Ctx& c, const c64* V) {
  const kdmg_lattice& lat = *h.lat;
  Transfer& T = h.T[0];
  const int ndc = 2 * T.nv, nd = 4 * T.a2.a0 * T.a2.a1, nZ = T.a2.Ncx * T.a2.Nct;
  const long f = T.nfine;
  const size_t smem = asym_build_lds(nd, ndc);
  KDMG_CHECK(smem <= LDS_LIMIT, KDMG_EUNSUPPORTED, "asymmetric coarsening: aggregate too large for LDS");
  T.asym = true;
  T.P64.alloc(sizeof(c64) * f * ndc);
  T.R64.alloc(sizeof(c64) * f * ndc);
  DevBuf fail(sizeof(int));
  KDMG_HIP(hipMemsetAsync(fail.p, 0, sizeof(int), c.st));
  auto fn = k_asym_build<double>;
  ensure_smem((const void*)fn, smem);
  int threads = 2 * nd > 256 ? ((2 * nd + 63) / 64) * 64 : 256;
  if (threads > 1024) threads = 1024;
  hipLaunchKernelGGL(fn, dim3(nZ), dim3(threads), smem, c.st, T.P64.as<c64>(), T.R64.as<c64>(), V, f,
                     lat.links64.as<c64>(), lat.g, T.a2, h.mass, fail.as<int>());
  KDMG_LAUNCH_CHECK();
  int failed = 0;
  KDMG_HIP(hipMemcpyAsync(&failed, fail.p, sizeof(int), hipMemcpyDeviceToHost, c.st));
  KDMG_HIP(hipStreamSynchronize(c.st));
  KDMG_CHECK(!failed, KDMG_EINVAL, "asymmetric coarsening: zero pivot in the thin LU of an aggregate");
  T.P32.alloc(sizeof(c32) * f * ndc);
  T.R32.alloc(sizeof(c32) * f * ndc);
  convert<float, double>(T.P32.as<c32>(), T.P64.as<c64>(), f * ndc, 1, nullptr, c.st);
  convert<float, double>(T.R32.as<c32>(), T.R64.as<c64>(), f * ndc, 1, nullptr, c.st);
}

// fine lattice -> first coarse lattice (2D U(1))
void build_level1(kdmg_hierarchy& h, const Ctx& c, const double* psi0, int relaxed) {
  const kdmg_lattice& lat = *h.lat;
  const Geo2& g = lat.g;
  const kdmg_level_params& lp = h.params.lvl[0];
  const int nv = lp.nvec, a0 = lp.agg[0], a1 = lp.agg[1];
  KDMG_CHECK(a0 >= 1 && a1 >= 1 && g.Bx % a0 == 0 && g.Bt % a1 == 0, KDMG_EINVAL,
             "first aggregate must divide the KD-block lattice");
  KDMG_CHECK(!lat.naik || (a0 >= 2 && a1 >= 2), KDMG_EINVAL,
             "Naik operator: first aggregates must be at least 2 KD blocks wide (three-link hops)");
  KDMG_CHECK(nv >= 1 && nv <= 2 * a0 * a1 && 2 * nv <= 64, KDMG_EINVAL,
             "n_vec must not exceed the sites of one aggregate chirality (and 2 n_vec <= 64)");
  Transfer& T = h.T[0];
  T.k = 0;
  T.nv = nv;
  T.a2 = Agg2{a0, a1, g.Bx / a0, g.Bt / a1, nv};
  const long f = 2 * g.half, V = lat.volume;
  T.nfine = f;
  const double m = h.mass;
  // starting vectors: natural order -> block layout
  DevBuf nat;
  upload(c, nat, psi0, sizeof(c64) * V * nv);
  DevBuf Vb(sizeof(c64) * f * nv);
  launch_permute<double, double>(Vb.as<c64>(), f, nat.as<c64>(), V, lat.perm_full.as<int>(), V, 1, nv,
                                 c.st);
  const c64* L = lat.links64.as<c64>();
  if (!relaxed) {
    DevBuf u(sizeof(c64) * f * nv), t(sizeof(c64) * f * nv), t2(sizeof(c64) * f * nv);
    if (!h.fine_full) {
      auto normal = [&](c64* out, const c64* in, const int* act) {
        fullAdag_apply<double>(u.as<c64>(), t2.as<c64>(), in, t.as<c64>(), L, g, m, act, nv, c.st);
        launch_hop<double, double, double>(out, f, t2.as<c64>(), f, u.as<c64>(), f, nullptr, 0, 0.0, 1.0,
                                           L, g, 0, 2, m, 0, 0, act, nv, c.st);
      };
      relax(c, Vb.as<c64>(), f, nv, h.params.setup_tol, h.params.setup_maxit, normal);
    } else {
      // the operator that is coarsened: A A^dag (Naik KD) or D D^dag (D itself)
      const Fine2<double> F = fine2<double>(lat, m);
      auto normal = [&](c64* out, const c64* in, const int* act) {
        if (h.naive) {
          fine2_Ddag<double, double>(u.as<c64>(), in, F, act, nv, c.st);
          fine2_D<double, double>(out, u.as<c64>(), nullptr, F, act, nv, c.st);
        } else {
          fine2_Adag<double, double>(u.as<c64>(), nullptr, in, t.as<c64>(), F, act, nv, c.st);
          fine2_A<double, double>(out, u.as<c64>(), nullptr, t.as<c64>(), F, act, nv, c.st);
        }
      };
      relax(c, Vb.as<c64>(), f, nv, h.params.setup_tol, h.params.setup_maxit, normal);
    }
  }
  T.relaxed.alloc(Vb.bytes);
  KDMG_HIP(hipMemcpyAsync(T.relaxed.p, Vb.p, Vb.bytes, hipMemcpyDeviceToDevice, c.st));
  global_mgs(c, Vb.as<c64>(), f, nv);
  if (h.params.asymmetric) {
    build_asym_transfer(h, c, Vb.as<c64>());
    galerkin_level1(h, c);
    KDMG_HIP(hipStreamSynchronize(c.st));
    return;
  }
  // block QR per (aggregate, chirality)
  const int nZ = T.a2.Ncx * T.a2.Nct, nrows = 2 * a0 * a1;
  std::vector<int> rows((size_t)nZ * 2 * nrows);
  for (int Z = 0; Z < nZ; ++Z) {
    const int Z0 = Z % T.a2.Ncx, Z1 = Z / T.a2.Ncx;
    for (int cc = 0; cc < 2; ++cc) {
      int k = 0;
      for (int kb = 0; kb < a0 * a1; ++kb) {
        const int X0 = Z0 * a0 + kb % a0, X1 = Z1 * a1 + kb / a0;
        const int p = (X0 + X1) & 1, b = blk_index(g, X0, X1);
        for (int s = 0; s < 4; ++s)
          if (chir2(s) == cc) rows[((size_t)Z * 2 + cc) * nrows + k++] = (int)(((long)p * g.Nb2 + b) * 4 + s);
      }
    }
  }
  T.P64.alloc(sizeof(c64) * f * nv);
  run_blockqr(c, T.P64.as<c64>(), Vb.as<c64>(), f, rows, nZ * 2, nrows, nv);
  T.P16.alloc(sizeof(c16) * f * nv);
  convert<_Float16, double>(T.P16.as<c16>(), T.P64.as<c64>(), f * nv, 1, nullptr, c.st);
  galerkin_level1(h, c);
  KDMG_HIP(hipStreamSynchronize(c.st));
}

// coarse level k -> k+1
void build_coarse(kdmg_hierarchy& h, int k, const Ctx& c, const double* psi0, int relaxed) {
  CoarseLevel& Lf = h.L[k];
  const kdmg_level_params& lp = h.params.lvl[k];
  const int nv = lp.nvec, nd = Lf.nd;
  int nchild = 1;
  CoarseLevel& Lc = h.L[k + 1];
  Lc.nd = nd;
  for (int mu = 0; mu < nd; ++mu) {
    KDMG_CHECK(lp.agg[mu] >= 1 && Lf.dims[mu] % lp.agg[mu] == 0, KDMG_EINVAL,
               "coarse aggregate must divide the coarse lattice");
    Lc.dims[mu] = Lf.dims[mu] / lp.agg[mu];
    nchild *= lp.agg[mu];
  }
  const int ndf = Lf.ndc, nvp = ndf / 2;
  KDMG_CHECK(nv >= 1 && nv <= nchild * nvp && 2 * nv <= 32, KDMG_EINVAL,
             "coarse n_vec must fit the aggregate and 2 n_vec <= 32");
  Transfer& T = h.T[k];
  T.k = k;
  T.nv = nv;
  T.nchild = nchild;
  T.nZ = 1;
  for (int mu = 0; mu < nd; ++mu) T.nZ *= Lc.dims[mu];
  T.nsf = Lf.nsites;
  T.ndf = ndf;
  const long n = Lf.n();
  T.nfine = n;
  // children / parent / coarse direction of each hop
  std::vector<int> children((size_t)T.nZ * nchild), parent(T.nsf), gdir((size_t)Lf.ndir * T.nsf);
  std::vector<int> fill(T.nZ, 0);
  for (int X = 0; X < T.nsf; ++X) {
    int co[4], rem = X;
    for (int mu = 0; mu < nd; ++mu) { co[mu] = rem % Lf.dims[mu]; rem /= Lf.dims[mu]; }
    int Z = 0, str = 1;
    for (int mu = 0; mu < nd; ++mu) { Z += (co[mu] / lp.agg[mu]) * str; str *= Lc.dims[mu]; }
    parent[X] = Z;
    // children in local lexicographic order (x fastest)
    int loc = 0, lstr = 1;
    for (int mu = 0; mu < nd; ++mu) { loc += (co[mu] % lp.agg[mu]) * lstr; lstr *= lp.agg[mu]; }
    children[(size_t)Z * nchild + loc] = X;
    fill[Z]++;
    gdir[X] = 0;
    for (int mu = 0; mu < nd; ++mu) {
      gdir[(size_t)(1 + 2 * mu) * T.nsf + X] = ((co[mu] + 1) % lp.agg[mu] == 0) ? 1 + 2 * mu : 0;
      gdir[(size_t)(2 + 2 * mu) * T.nsf + X] = (co[mu] % lp.agg[mu] == 0) ? 2 + 2 * mu : 0;
    }
  }
  T.children.alloc(sizeof(int) * children.size());
  T.parent.alloc(sizeof(int) * parent.size());
  T.gdir.alloc(sizeof(int) * gdir.size());
  KDMG_HIP(hipMemcpy(T.children.p, children.data(), T.children.bytes, hipMemcpyHostToDevice));
  KDMG_HIP(hipMemcpy(T.parent.p, parent.data(), T.parent.bytes, hipMemcpyHostToDevice));
  KDMG_HIP(hipMemcpy(T.gdir.p, gdir.data(), T.gdir.bytes, hipMemcpyHostToDevice));
  DevBuf Vb;
  upload(c, Vb, psi0, sizeof(c64) * n * nv);
  if (!relaxed) {
    DevBuf u(sizeof(c64) * n * nv);
    auto normal = [&](c64* out, const c64* in, const int* act) {
      coarse_apply<double, double>(Lf, true, u.as<c64>(), in, nullptr, 1.0, act, nv, c.st);
      coarse_apply<double, double>(Lf, false, out, u.as<c64>(), nullptr, 1.0, act, nv, c.st);
    };
    relax(c, Vb.as<c64>(), n, nv, h.params.setup_tol, h.params.setup_maxit, normal);
  }
  T.relaxed.alloc(Vb.bytes);
  KDMG_HIP(hipMemcpyAsync(T.relaxed.p, Vb.p, Vb.bytes, hipMemcpyDeviceToDevice, c.st));
  global_mgs(c, Vb.as<c64>(), n, nv);
  const int nrows = nchild * nvp;
  std::vector<int> rows((size_t)T.nZ * 2 * nrows);
  for (int Z = 0; Z < T.nZ; ++Z)
    for (int cc = 0; cc < 2; ++cc) {
      int kk = 0;
      for (int ch = 0; ch < nchild; ++ch)
        for (int ia = 0; ia < nvp; ++ia)
          rows[((size_t)Z * 2 + cc) * nrows + kk++] = children[(size_t)Z * nchild + ch] * ndf + cc * nvp + ia;
    }
  T.P64.alloc(sizeof(c64) * n * nv);
  run_blockqr(c, T.P64.as<c64>(), Vb.as<c64>(), n, rows, T.nZ * 2, nrows, nv);
  T.P16.alloc(sizeof(c16) * n * nv);
  convert<_Float16, double>(T.P16.as<c16>(), T.P64.as<c64>(), n * nv, 1, nullptr, c.st);
  galerkin_coarse(h, k, c);
  KDMG_HIP(hipStreamSynchronize(c.st));
}

}  // namespace

kdmg_hierarchy::~kdmg_hierarchy() {
  if (ws) kdmg::destroy_ws(ws);
  if (timer.e0) (void)hipEventDestroy(timer.e0);
  if (timer.e1) (void)hipEventDestroy(timer.e1);
  for (auto& e : timer.dn_ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
}

extern "C" kdmg_status kdmg_hierarchy_build(const kdmg_lattice* lat, double mass,
                                            const kdmg_mg_params* params,
                                            const double* const* psi0_host, int relaxed,
                                            void* stream, kdmg_hierarchy** out) {
  KDMG_API_BEGIN
  KDMG_CHECK(lat && params && psi0_host && out, KDMG_EINVAL, "kdmg_hierarchy_build: null argument");
  *out = nullptr;
  KDMG_CHECK(params->nlevels >= 2 && params->nlevels <= 4, KDMG_EINVAL, "nlevels must be 2..4");
  KDMG_CHECK(mass > 0.0, KDMG_EINVAL, "mass must be positive");
  KDMG_CHECK(params->setup_maxit >= 0 && params->outer_restart >= 1 && params->outer_restart <= 64 &&
                 params->inter_restart >= 1 && params->inter_restart <= 64 && params->outer_stall >= 0 &&
                 params->coarse_tail >= 0 && params->coarse_tail <= 64 &&
                 (params->coarse_solver == 0 || params->coarse_solver == 1),
             KDMG_EINVAL, "bad solver parameters");
  for (int k = 0; k < params->nlevels - 1; ++k)
    KDMG_CHECK(psi0_host[k] != nullptr, KDMG_EINVAL, "missing starting vectors");
  KDMG_CHECK(params->fine_op == 0 || params->fine_op == 1, KDMG_EINVAL, "fine_op must be 0 or 1");
  KDMG_CHECK(lat->nd == 2 || (params->fine_op == 0 && !lat->naik), KDMG_EUNSUPPORTED,
             "fine_op = 1 is built for 2D lattices");
  KDMG_CHECK(params->asymmetric == 0 || params->asymmetric == 1, KDMG_EINVAL, "asymmetric must be 0 or 1");
  KDMG_CHECK(!params->asymmetric || (lat->nd == 2 && lat->nc == 1 && !lat->naik && params->fine_op == 0 &&
                                     params->nlevels == 2),
             KDMG_EUNSUPPORTED, "asymmetric coarsening: two levels of the 2D KD operator without Naik terms only");
  auto h = std::make_unique<kdmg_hierarchy>();
  h->lat = lat;
  h->mass = mass;
  h->params = *params;
  h->nlevels = params->nlevels;
  h->naive = params->fine_op == 1;
  h->fine_full = h->naive || lat->naik;
  h->L.resize(h->nlevels);
  h->T.resize(h->nlevels - 1);
  int nvmax = 1;
  for (int k = 0; k < h->nlevels - 1; ++k) nvmax = std::max(nvmax, params->lvl[k].nvec);
  CtxAlloc ca;
  ca.init((hipStream_t)stream, nvmax * 2 + 8, nvmax);
  if (lat->nd == 4)
    build_level1_4d(*h, ca.c, psi0_host[0], relaxed);
  else
    build_level1(*h, ca.c, psi0_host[0], relaxed);
  for (int k = 1; k < h->nlevels - 1; ++k) build_coarse(*h, k, ca.c, psi0_host[k], relaxed);
  if (params->coarse_solver == 1) build_dense_inverse(h->dinv, h->L[h->nlevels - 1], (hipStream_t)stream);
  KDMG_HIP(hipStreamSynchronize((hipStream_t)stream));
  *out = h.release();
  KDMG_API_END
}

namespace {

bool same_shape(const kdmg_hierarchy& a, const kdmg_hierarchy& b) {
  if (a.nlevels != b.nlevels || a.lat->nd != b.lat->nd || a.lat->nc != b.lat->nc) return false;
  if (a.fine_full != b.fine_full || a.naive != b.naive || a.lat->naik != b.lat->naik ||
      a.params.coarse_solver != b.params.coarse_solver)
    return false;
  for (int mu = 0; mu < 4; ++mu)
    if (a.lat->dims[mu] != b.lat->dims[mu]) return false;
  for (int k = 0; k < a.nlevels - 1; ++k) {
    if (a.params.lvl[k].nvec != b.params.lvl[k].nvec) return false;
    for (int mu = 0; mu < 4; ++mu)
      if (a.params.lvl[k].agg[mu] != b.params.lvl[k].agg[mu]) return false;
  }
  return true;
}

// Galerkin-build every coarse operator of h at h.mass from its transfers.
void rebuild_coarse_ops(kdmg_hierarchy& h, hipStream_t st) {
  Ctx c{};
  c.st = st;
  galerkin_level1(h, c);
  for (int k = 1; k < h.nlevels - 1; ++k) galerkin_coarse(h, k, c);
  if (h.params.coarse_solver == 1) build_dense_inverse(h.dinv, h.L[h.nlevels - 1], st);
  KDMG_HIP(hipStreamSynchronize(st));
}

void copy_tuned(const kdmg_hierarchy& from, kdmg_hierarchy& to) {
  for (int l = 1; l < from.nlevels; ++l) {
    std::map<long, TileShape> t;
    {
      std::lock_guard<std::mutex> g(*from.L[l].tune_mu);
      t = from.L[l].tuned;
    }
    std::lock_guard<std::mutex> g(*to.L[l].tune_mu);
    to.L[l].tuned = t;  // the base's launch shapes, so results depend on (base, mass, b) only
  }
}

}  // namespace

extern "C" kdmg_status kdmg_hierarchy_at_mass(const kdmg_hierarchy* base, double mass, void* stream,
                                              kdmg_hierarchy** out) {
  KDMG_API_BEGIN
  KDMG_CHECK(base && out, KDMG_EINVAL, "kdmg_hierarchy_at_mass: null argument");
  *out = nullptr;
  KDMG_CHECK(mass > 0.0, KDMG_EINVAL, "mass must be positive");
  KDMG_CHECK(!base->params.asymmetric, KDMG_EUNSUPPORTED,
             "asymmetric transfers depend on the mass: build a hierarchy at the new mass");
  auto h = std::make_unique<kdmg_hierarchy>();
  h->lat = base->lat;
  h->mass = mass;
  h->params = base->params;
  h->nlevels = base->nlevels;
  h->T = base->T;
  h->derived = true;
  h->naive = base->naive;
  h->fine_full = base->fine_full;
  h->L.resize(h->nlevels);
  rebuild_coarse_ops(*h, (hipStream_t)stream);
  copy_tuned(*base, *h);
  *out = h.release();
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_set_mass(kdmg_hierarchy* h, const kdmg_hierarchy* base, double mass,
                                               void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h, KDMG_EINVAL, "kdmg_hierarchy_set_mass: null hierarchy");
  KDMG_CHECK(mass > 0.0, KDMG_EINVAL, "mass must be positive");
  KDMG_CHECK(!h->params.asymmetric && !(base && base->params.asymmetric), KDMG_EUNSUPPORTED,
             "asymmetric transfers depend on the mass: build a hierarchy at the new mass");
  if (base && base != h) {
    KDMG_CHECK(same_shape(*h, *base), KDMG_EINVAL,
               "kdmg_hierarchy_set_mass: base has a different lattice shape or level structure");
    KDMG_CHECK(!ws_busy(h->ws), KDMG_EBUSY, "hierarchy busy");
    h->lat = base->lat;
    h->T = base->T;
    h->derived = true;
    h->naive = base->naive;
    h->fine_full = base->fine_full;
    copy_tuned(*base, *h);
  }
  KDMG_CHECK(!ws_busy(h->ws), KDMG_EBUSY, "hierarchy busy");
  h->mass = mass;
  reset_graphs(h->ws);
  rebuild_coarse_ops(*h, (hipStream_t)stream);
  KDMG_API_END
}

extern "C" void kdmg_hierarchy_destroy(kdmg_hierarchy* h) { delete h; }

extern "C" kdmg_status kdmg_hierarchy_level_info(const kdmg_hierarchy* h, int level, int* dims_out,
                                                 int* ndof_out) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && level >= 1 && level < h->nlevels, KDMG_EINVAL, "bad level");
  const CoarseLevel& L = h->L[level];
  if (dims_out)
    for (int mu = 0; mu < L.nd; ++mu) dims_out[mu] = L.dims[mu];
  if (ndof_out) *ndof_out = L.ndc;
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_get_nullvecs(const kdmg_hierarchy* h, int k, double* host_out) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && host_out && k >= 0 && k < h->nlevels - 1, KDMG_EINVAL, "bad level");
  const Transfer& T = h->T[k];
  const long n = T.nfine;
  if (k == 0) {
    const kdmg_lattice& lat = *h->lat;
    const long V = lat.ndof;
    DevBuf nat(sizeof(c64) * V * T.nv);
    launch_permute<double, double>(nat.as<c64>(), V, T.relaxed.as<c64>(), n, lat.perm_full.as<int>(), V,
                                   0, T.nv, 0);
    KDMG_HIP(hipMemcpy(host_out, nat.p, nat.bytes, hipMemcpyDeviceToHost));
  } else {
    KDMG_HIP(hipMemcpy(host_out, T.relaxed.p, T.relaxed.bytes, hipMemcpyDeviceToHost));
  }
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_get_prolongator(const kdmg_hierarchy* h, int k, double* host_out) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && host_out && k >= 0 && k < h->nlevels - 1, KDMG_EINVAL, "bad level");
  const Transfer& T = h->T[k];
  KDMG_CHECK(!T.asym, KDMG_EINVAL, "asymmetric hierarchy: use kdmg_hierarchy_get_asym_transfer");
  std::vector<c64> buf(T.P64.bytes / sizeof(c64));
  KDMG_HIP(hipMemcpy(buf.data(), T.P64.p, T.P64.bytes, hipMemcpyDeviceToHost));
  c64* o = reinterpret_cast<c64*>(host_out);
  if (k == 0) {
    const kdmg_lattice& lat = *h->lat;
    for (long x = 0; x < lat.ndof; ++x)
      for (int i = 0; i < T.nv; ++i) o[x * T.nv + i] = buf[(size_t)lat.h_perm_full[x] * T.nv + i];
  } else {
    std::memcpy(o, buf.data(), T.P64.bytes);
  }
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_get_asym_transfer(const kdmg_hierarchy* h, int k, double* p_out,
                                                        double* r_out) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && k == 0 && h->nlevels >= 2 && h->T[0].asym, KDMG_EINVAL,
             "kdmg_hierarchy_get_asym_transfer: not an asymmetric coarsening");
  const Transfer& T = h->T[0];
  const kdmg_lattice& lat = *h->lat;
  const int ndc = 2 * T.nv;
  std::vector<c64> buf(T.P64.bytes / sizeof(c64));
  for (int which = 0; which < 2; ++which) {
    double* out = which == 0 ? p_out : r_out;
    if (!out) continue;
    const DevBuf& src = which == 0 ? T.P64 : T.R64;
    KDMG_HIP(hipMemcpy(buf.data(), src.p, src.bytes, hipMemcpyDeviceToHost));
    c64* o = reinterpret_cast<c64*>(out);
    for (long x = 0; x < lat.ndof; ++x)
      for (int j = 0; j < ndc; ++j) o[x * ndc + j] = buf[(size_t)lat.h_perm_full[x] * ndc + j];
  }
  KDMG_API_END
}

extern "C" kdmg_status kdmg_hierarchy_get_coarse_op(const kdmg_hierarchy* h, int level, double* host_out) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && host_out && level >= 1 && level < h->nlevels, KDMG_EINVAL, "bad level");
  const CoarseLevel& L = h->L[level];
  std::vector<c64> buf(L.Yt64.bytes / sizeof(c64));
  KDMG_HIP(hipMemcpy(buf.data(), L.Yt64.p, L.Yt64.bytes, hipMemcpyDeviceToHost));
  c64* o = reinterpret_cast<c64*>(host_out);
  const long nd2 = (long)L.ndc * L.ndc;
  for (long db = 0; db < (long)L.ndir * L.nsites; ++db)
    for (int i = 0; i < L.ndc; ++i)
      for (int j = 0; j < L.ndc; ++j) o[db * nd2 + (long)i * L.ndc + j] = buf[db * nd2 + (long)j * L.ndc + i];
  KDMG_API_END
}

extern "C" kdmg_status kdmg_coarse_apply(const kdmg_hierarchy* h, int level, int dagger, const void* in,
                                         void* out, int nrhs, kdmg_prec prec, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && in && out && in != out, KDMG_EINVAL, "kdmg_coarse_apply: bad pointers");
  KDMG_CHECK(level >= 1 && level < h->nlevels && nrhs >= 1 && nrhs <= 65535, KDMG_EINVAL,
             "kdmg_coarse_apply: bad level or nrhs");
  const CoarseLevel& L = h->L[level];
  hipStream_t st = (hipStream_t)stream;
  if (prec == KDMG_FP64)
    coarse_apply<double, double>(L, dagger != 0, (c64*)out, (const c64*)in, nullptr, 1.0, nullptr, nrhs, st);
  else
    coarse_apply<float, float>(L, dagger != 0, (c32*)out, (const c32*)in, nullptr, 1.0, nullptr, nrhs, st);
  KDMG_API_END
}

// kdmg_restrict / kdmg_prolong in precision R with prolongator storage PT
// (FP64 / FP64, or FP32 vectors with the FP16-stored P of the mixed V-cycle).
template <class R, class PT>
static void restrict_as(const kdmg_hierarchy* h, int k, const void* in, void* out, int nrhs, hipStream_t st) {
  const Transfer& T = h->T[k];
  if (k == 0) {
    const kdmg_lattice& lat = *h->lat;
    const long f = 2 * lat.half, V = lat.ndof;
    DevBuf a(sizeof(Cx<R>) * f * nrhs);
    launch_permute<R, R>(a.as<Cx<R>>(), f, (const Cx<R>*)in, V, lat.perm_full.as<int>(), V, 1, nrhs, st);
    transfer_restrict<R, PT, R, R>(T, lat, nullptr, (Cx<R>*)out, a.as<Cx<R>>(), f, 0, nullptr, nrhs, st);
    KDMG_HIP(hipStreamSynchronize(st));
  } else {
    transfer_restrict<R, PT, R, R>(T, *h->lat, &h->L[k], (Cx<R>*)out, (const Cx<R>*)in, T.nfine, 0, nullptr,
                                   nrhs, st);
  }
}

template <class R, class PT>
static void prolong_as(const kdmg_hierarchy* h, int k, const void* in, void* out, int nrhs, hipStream_t st) {
  const Transfer& T = h->T[k];
  if (k == 0) {
    const kdmg_lattice& lat = *h->lat;
    const long f = 2 * lat.half, V = lat.ndof;
    DevBuf a(sizeof(Cx<R>) * f * nrhs);
    transfer_prolong<R, PT, R, R>(T, lat, a.as<Cx<R>>(), f, nullptr, 0, (const Cx<R>*)in, 2, nullptr, nrhs, st);
    launch_permute<R, R>((Cx<R>*)out, V, a.as<Cx<R>>(), f, lat.perm_full.as<int>(), V, 0, nrhs, st);
    KDMG_HIP(hipStreamSynchronize(st));
  } else {
    transfer_prolong<R, PT, R, R>(T, *h->lat, (Cx<R>*)out, 0, nullptr, 0, (const Cx<R>*)in, 1, nullptr, nrhs, st);
  }
}

extern "C" kdmg_status kdmg_restrict(const kdmg_hierarchy* h, int k, const void* in, void* out, int nrhs,
                                     kdmg_prec prec, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && in && out && k >= 0 && k < h->nlevels - 1 && nrhs >= 1 &&
                 (prec == KDMG_FP64 || prec == KDMG_MIXED),
             KDMG_EINVAL, "kdmg_restrict: bad argument");
  if (prec == KDMG_FP64)
    restrict_as<double, double>(h, k, in, out, nrhs, (hipStream_t)stream);
  else
    restrict_as<float, _Float16>(h, k, in, out, nrhs, (hipStream_t)stream);
  KDMG_API_END
}

extern "C" kdmg_status kdmg_prolong(const kdmg_hierarchy* h, int k, const void* in, void* out, int nrhs,
                                    kdmg_prec prec, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && in && out && k >= 0 && k < h->nlevels - 1 && nrhs >= 1 &&
                 (prec == KDMG_FP64 || prec == KDMG_MIXED),
             KDMG_EINVAL, "kdmg_prolong: bad argument");
  if (prec == KDMG_FP64)
    prolong_as<double, double>(h, k, in, out, nrhs, (hipStream_t)stream);
  else
    prolong_as<float, _Float16>(h, k, in, out, nrhs, (hipStream_t)stream);
  KDMG_API_END
}
