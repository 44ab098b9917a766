// Internal C++ objects behind the C-ABI handles, and the launchers shared by
// the lattice, setup and solver translation units.
#pragma once
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <type_traits>
#include <vector>

#include "common.h"
#include "blas.h"
#include "fine2d.h"
#include "asym2d.h"
#include "fine4d.h"
#include "coarse.h"
#include "coarse_fast.h"
#include "dense.h"

namespace kdmg {

enum class Prec { F64 = 0, F32 = 1 };

}  // namespace kdmg

// ------------------------------------------------------------------ lattice
struct kdmg_lattice {
  int nd = 0, nc = 0;
  int dims[4] = {1, 1, 1, 1};
  long volume = 0;
  int bc[4] = {1, 1, 1, -1};  // boundary sign per direction (+1 periodic, -1 antiperiodic)
  kdmg::Geo2 g{};
  long ndof = 0;   // complex entries of a fine vector (volume * nc)
  long half = 0;   // complex entries of one KD-block parity half (the Schur space)
  // folded links (1/2 eta bc U), block layout [2][Nb2][8]
  kdmg::DevBuf links64, links16, links32;
  // 4D SU(3): geometry, folded forward links [site][mu][3][3] and neighbour
  // table [site][8] in block layout (see fine4d.h)
  kdmg::Geo4 g4{};
  kdmg::DevBuf lk64, lk32, lk16, nb4;
  // folded links in natural order, per direction [mu][site]
  kdmg::DevBuf nat64, nat16;
  // natural site -> block-layout index; even-block rank -> index in the even half
  kdmg::DevBuf perm_full, perm_even;
  std::vector<int> h_perm_full, h_perm_even;
  // Naik-improved operator (2D U(1), kdmg_lattice_set_naik):
  // D = m + c1 (one-link hops) + c3 (three-link hops)
  int naik = 0;
  double c1 = 1.0, c3 = 0.0;
  kdmg::DevBuf wl64, wl16;          // folded three-link transporters, block layout [mu][2 half]
  kdmg::DevBuf natw64, natw16;      // the same in natural order [mu][volume]
  std::vector<kdmg::c64> h_links;   // 2D: the uploaded links, kept for the transporters
  size_t footprint() const {
    return links64.bytes + links16.bytes + links32.bytes + nat64.bytes + nat16.bytes +
           perm_full.bytes + perm_even.bytes + lk64.bytes + lk32.bytes + lk16.bytes + nb4.bytes +
           wl64.bytes + wl16.bytes + natw64.bytes + natw16.bytes;
  }
};

namespace kdmg {

// ------------------------------------------------------------------ launch helpers

inline dim3 fine_grid(const Geo2& g, int nrhs, int npar) { return dim3(cdiv(g.Nb2, 256), nrhs, npar); }

template <class R, class LT, class VT>
void launch_binv(Cx<VT>* out, long so, Cx<VT>* out2, long so2, const Cx<VT>* in, long si,
                 const Cx<VT>* add, long sa, const Cx<LT>* links, const Geo2& g, int p0, int npar,
                 double m, int eps_out, const int* act, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_binv<R, LT, VT>), fine_grid(g, nrhs, npar), dim3(256), 0, st, out, so, out2,
                     so2, in, si, add, sa, links, g, p0, (R)m, eps_out, act);
  KDMG_LAUNCH_CHECK();
}

template <class R, class LT, class VT>
void launch_hop(Cx<VT>* out, long so, const Cx<VT>* in, long si, const Cx<VT>* add, long sa,
                const Cx<VT>* add2, long sa2, double c2, double sgn, const Cx<LT>* links,
                const Geo2& g, int p0, int npar, double m, int mode, int eps_in, const int* act,
                int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_hop<R, LT, VT>), fine_grid(g, nrhs, npar), dim3(256), 0, st, out, so, in, si,
                     add, sa, add2, sa2, (R)c2, (R)sgn, links, g, p0, (R)m, mode, eps_in, act);
  KDMG_LAUNCH_CHECK();
}

template <class R, class LT, class VT>
void launch_dslash_blk(Cx<VT>* out, long so, const Cx<VT>* in, long si, const Cx<VT>* sub, long ss,
                       const Cx<LT>* links, const Geo2& g, double m, const int* act, int nrhs,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_dslash_blk<R, LT, VT>), fine_grid(g, nrhs, 2), dim3(256), 0, st, out, so, in,
                     si, sub, ss, links, g, (R)m, act);
  KDMG_LAUNCH_CHECK();
}

template <class R, class LT, class VT>
void launch_hop3(Cx<VT>* out, long so, const Cx<VT>* in, long si, double coef, const Cx<LT>* wl, const Geo2& g,
                 int eps_in, const int* act, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_hop3<R, LT, VT>), dim3(cdiv(2 * g.half, 256), nrhs), dim3(256), 0, st, out, so, in, si,
                     (R)coef, wl, g, eps_in, act);
  KDMG_LAUNCH_CHECK();
}

template <class TO, class TI>
void launch_permute(Cx<TO>* dst, long sd, const Cx<TI>* src, long ss, const int* idx, long n,
                    int scatter, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_permute<TO, TI>), dim3(cdiv(n, 256), nrhs), dim3(256), 0, st, dst, sd, src, ss,
                     idx, n, scatter);
  KDMG_LAUNCH_CHECK();
}

// Schur operator S = 1 - A_eo A_oe on even-half vectors:
//   t = B_e^-1 v ; w = B_o^-1 C_oe t ; out = v - C_eo w            (resid == null)
//                                       out = resid - v + C_eo w   (= resid - S v)
// t and w are full-layout temporaries (>= nrhs * 2 * half entries).
template <class R, class LT>
void schur_apply(Cx<R>* out, const Cx<R>* v, const Cx<R>* resid, Cx<R>* t, Cx<R>* w,
                 const Cx<LT>* links, const Geo2& g, double m, const int* act, int nrhs,
                 hipStream_t st) {
  const long h = g.half, f = 2 * g.half;
  launch_binv<R, LT, R>(t, f, nullptr, 0, v, h, nullptr, 0, links, g, 0, 1, m, 0, act, nrhs, st);
  launch_hop<R, LT, R>(w, f, t, f, nullptr, 0, nullptr, 0, 0.0, 1.0, links, g, 1, 1, m, 1, 0, act,
                       nrhs, st);
  if (!resid)
    launch_hop<R, LT, R>(out, h, w, f, v, h, nullptr, 0, 0.0, -1.0, links, g, 0, 1, m, 0, 0, act,
                         nrhs, st);
  else
    launch_hop<R, LT, R>(out, h, w, f, resid, h, v, h, -1.0, 1.0, links, g, 0, 1, m, 0, 0, act,
                         nrhs, st);
}

// Full-lattice A = 1 + C B^-1:  t = B^-1 v ; out = v + C t
template <class LT, class R = double>
void fullA_apply(Cx<R>* out, const Cx<R>* v, Cx<R>* t, const Cx<LT>* links, const Geo2& g, double m,
                 const int* act, int nrhs, hipStream_t st) {
  const long f = 2 * g.half;
  launch_binv<R, LT, R>(t, f, nullptr, 0, v, f, nullptr, 0, links, g, 0, 2, m, 0, act, nrhs, st);
  launch_hop<R, LT, R>(out, f, t, f, v, f, nullptr, 0, 0.0, 1.0, links, g, 0, 2, m, 0, 0, act, nrhs, st);
}

// Full-lattice A^dag = 1 + eps B^-1 C eps:  t = C (eps v) ; out = v + eps B^-1 t
// (optionally out2 = B^-1 out, the first half of the next A apply)
template <class LT, class R = double>
void fullAdag_apply(Cx<R>* out, Cx<R>* out2, const Cx<R>* v, Cx<R>* t, const Cx<LT>* links, const Geo2& g,
                    double m, const int* act, int nrhs, hipStream_t st) {
  const long f = 2 * g.half;
  launch_hop<R, LT, R>(t, f, v, f, nullptr, 0, nullptr, 0, 0.0, 1.0, links, g, 0, 2, m, 0, 1, act, nrhs, st);
  launch_binv<R, LT, R>(out, f, out2, f, t, f, v, f, links, g, 0, 2, m, 1, act, nrhs, st);
}

// ------------------------------------------- 2D fine operators, full lattice
// The fine operator of a 2D lattice in one precision, for the solves that
// iterate on the full lattice (the Naik-improved operator, whose three-link
// hops join KD blocks of the same parity, and multigrid on D itself).  With
// D = m + c1 H1 + c3 H3 (H1, H3 the one- and three-link hops) written as
//   D = s (B~ + C1 + x C3),  s = c1,  x = c3 / c1,  B~ = m / c1 + (intra-block H1),
// A = D B^-1 = 1 + (C1 + x C3) B~^-1 needs only the plain block kernels at the
// rescaled mass (the Naik block is the plain one rescaled, Sec. 2.1).
template <class LT>
struct Fine2 {
  const Cx<LT>* L;  // folded one-link hops, block layout
  const Cx<LT>* W;  // folded three-link hops, block layout (null: none)
  Geo2 g;
  double me;        // m / c1
  double s;         // c1
  double x;         // c3 / c1
  double m;         // the mass of D
};

// The 2D fine operator of `lat` at mass m, FP64 (LT = double) or FP16-stored (LT = _Float16).
template <class LT>
Fine2<LT> fine2(const kdmg_lattice& lat, double m) {
  const bool h = sizeof(LT) == 2;
  const void* L = h ? lat.links16.p : lat.links64.p;
  const void* W = lat.naik ? (h ? lat.wl16.p : lat.wl64.p) : nullptr;
  return Fine2<LT>{(const Cx<LT>*)L, (const Cx<LT>*)W, lat.g, m / lat.c1, lat.c1, lat.c3 / lat.c1, m};
}

// out = a x + b y (in place allowed)
template <class T>
struct OpAxpby {
  Cx<T>* out; const Cx<T>* x; const Cx<T>* y; long n; double a, b; const int* act;
  __device__ bool active(int r) const { return is_active(act, r); }
  __device__ void elem(int r, long i) const {
    const long o = r * n + i;
    Cx<T> v = (T)a * x[o];
    if (y) v += (T)b * y[o];
    out[o] = v;
  }
};

// out = A v, or resid - A v;  t: full-lattice temporary
template <class R, class LT>
void fine2_A(Cx<R>* out, const Cx<R>* v, const Cx<R>* resid, Cx<R>* t, const Fine2<LT>& F, const int* act,
             int nrhs, hipStream_t st) {
  const long f = 2 * F.g.half;
  launch_binv<R, LT, R>(t, f, nullptr, 0, v, f, nullptr, 0, F.L, F.g, 0, 2, F.me, 0, act, nrhs, st);
  if (!resid)
    launch_hop<R, LT, R>(out, f, t, f, v, f, nullptr, 0, 0.0, 1.0, F.L, F.g, 0, 2, F.me, 0, 0, act, nrhs, st);
  else
    launch_hop<R, LT, R>(out, f, t, f, resid, f, v, f, -1.0, -1.0, F.L, F.g, 0, 2, F.me, 0, 0, act, nrhs, st);
  if (F.W) launch_hop3<R, LT, R>(out, f, t, f, resid ? -F.x : F.x, F.W, F.g, 0, act, nrhs, st);
}

// out = A^dag v = v + eps B~^-1 (C1 + x C3) eps v;  optionally out2 = B~^-1 out
template <class R, class LT>
void fine2_Adag(Cx<R>* out, Cx<R>* out2, const Cx<R>* v, Cx<R>* t, const Fine2<LT>& F, const int* act, int nrhs,
                hipStream_t st) {
  const long f = 2 * F.g.half;
  launch_hop<R, LT, R>(t, f, v, f, nullptr, 0, nullptr, 0, 0.0, 1.0, F.L, F.g, 0, 2, F.me, 0, 1, act, nrhs, st);
  if (F.W) launch_hop3<R, LT, R>(t, f, v, f, F.x, F.W, F.g, 1, act, nrhs, st);
  launch_binv<R, LT, R>(out, f, out2, f, t, f, v, f, F.L, F.g, 0, 2, F.me, 1, act, nrhs, st);
}

// out = D v, or resid - D v
template <class R, class LT>
void fine2_D(Cx<R>* out, const Cx<R>* v, const Cx<R>* resid, const Fine2<LT>& F, const int* act, int nrhs,
             hipStream_t st) {
  const long f = 2 * F.g.half;
  launch_dslash_blk<R, LT, R>(out, f, v, f, nullptr, 0, F.L, F.g, F.me, act, nrhs, st);
  if (F.W) launch_hop3<R, LT, R>(out, f, v, f, F.x, F.W, F.g, 0, act, nrhs, st);
  if (resid || F.s != 1.0)
    launch_map(OpAxpby<R>{out, out, resid, f, resid ? -F.s : F.s, 1.0, act}, f, nrhs, st);
}

// out = D^dag v = 2 m v - D v  (D - m is anti-Hermitian)
template <class R, class LT>
void fine2_Ddag(Cx<R>* out, const Cx<R>* v, const Fine2<LT>& F, const int* act, int nrhs, hipStream_t st) {
  const long f = 2 * F.g.half;
  fine2_D<R, LT>(out, v, nullptr, F, act, nrhs, st);
  launch_map(OpAxpby<R>{out, out, v, f, -1.0, 2.0 * F.m, act}, f, nrhs, st);
}

// ------------------------------------------------------------ 4D fine operators

template <class R, class LT>
void launch4_hop(Cx<R>* out, long so, const Cx<R>* in, long si, const Cx<R>* add, long sa, const Cx<R>* add2,
                 long sa2, double c2, double sgn, const Cx<LT>* lk, const int* nb4, const Geo4& g, int p0, int npar,
                 double m, int mode, int eps_in, const int* act, int nrhs, hipStream_t st) {
  // a tile of rhs per thread (links and neighbour indices read once per
  // tile): 8 in FP32 from 8 rhs on, else 4 from 4 rhs on (an FP64 tile of 8
  // exceeds the register budget)
  if constexpr (sizeof(R) == 4) {
    if (nrhs >= 8) {
      hipLaunchKernelGGL((k4_hop<R, LT, R, 8>), dim3(cdiv(16L * g.Nb2, 256), cdiv(nrhs, 8), npar), dim3(256), 0,
                         st, out, so, in, si, add, sa, add2, sa2, (R)c2, (R)sgn, lk, nb4, g, p0, (R)m, mode, eps_in,
                         act, nrhs);
      KDMG_LAUNCH_CHECK();
      return;
    }
  }
  if (nrhs >= 4)
    hipLaunchKernelGGL((k4_hop<R, LT, R, 4>), dim3(cdiv(16L * g.Nb2, 256), cdiv(nrhs, 4), npar), dim3(256), 0, st,
                       out, so, in, si, add, sa, add2, sa2, (R)c2, (R)sgn, lk, nb4, g, p0, (R)m, mode, eps_in, act,
                       nrhs);
  else
    hipLaunchKernelGGL((k4_hop<R, LT, R, 1>), dim3(cdiv(16L * g.Nb2, 256), nrhs, npar), dim3(256), 0, st, out, so,
                       in, si, add, sa, add2, sa2, (R)c2, (R)sgn, lk, nb4, g, p0, (R)m, mode, eps_in, act, nrhs);
  KDMG_LAUNCH_CHECK();
}

template <class R, class BT>
void launch4_binv(Cx<R>* out, long so, const Cx<R>* in, long si, const Cx<R>* add, long sa, const Cx<BT>* Bv,
                  const Geo4& g, int p0, int npar, int eps_out, const int* act, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k4_binv<R, BT, R>), dim3(g.Nb2, cdiv(nrhs, B4_RB), npar), dim3(64), 0, st, out, so, in, si, add,
                     sa, Bv, g, p0, eps_out, act, nrhs);
  KDMG_LAUNCH_CHECK();
}

// Operands of the 4D fine operators in one precision: links, neighbours and
// B^-1 at the operator's mass.
template <class LT, class BT>
struct Fine4 {
  const Cx<LT>* lk;
  const int* nb4;
  const Cx<BT>* Bv;
  Geo4 g;
  double m;
};

// S = 1 - A_eo A_oe on even-half vectors (as schur_apply):
//   t_e = B_e^-1 v ; w_o = C_oe t_e ; t_o = B_o^-1 w_o ;
//   out = v - C_eo t_o   or   out = resid - v + C_eo t_o
template <class R, class LT, class BT>
void schur_apply4(Cx<R>* out, const Cx<R>* v, const Cx<R>* resid, Cx<R>* t, Cx<R>* w, const Fine4<LT, BT>& F,
                  const int* act, int nrhs, hipStream_t st) {
  const long h = F.g.half, f = 2 * h;
  launch4_binv<R, BT>(t, f, v, h, nullptr, 0, F.Bv, F.g, 0, 1, 0, act, nrhs, st);
  launch4_hop<R, LT>(w, f, t, f, nullptr, 0, nullptr, 0, 0.0, 1.0, F.lk, F.nb4, F.g, 1, 1, F.m, 0, 0, act, nrhs, st);
  launch4_binv<R, BT>(t, f, w, f, nullptr, 0, F.Bv, F.g, 1, 1, 0, act, nrhs, st);
  if (!resid)
    launch4_hop<R, LT>(out, h, t, f, v, h, nullptr, 0, 0.0, -1.0, F.lk, F.nb4, F.g, 0, 1, F.m, 0, 0, act, nrhs, st);
  else
    launch4_hop<R, LT>(out, h, t, f, resid, h, v, h, -1.0, 1.0, F.lk, F.nb4, F.g, 0, 1, F.m, 0, 0, act, nrhs, st);
}

// A = 1 + C B^-1 on full vectors:  t = B^-1 v ; out = v + C t
template <class LT, class BT, class R = double>
void fullA_apply4(Cx<R>* out, const Cx<R>* v, Cx<R>* t, const Fine4<LT, BT>& F, const int* act, int nrhs,
                  hipStream_t st) {
  const long f = 2 * F.g.half;
  launch4_binv<R, BT>(t, f, v, f, nullptr, 0, F.Bv, F.g, 0, 2, 0, act, nrhs, st);
  launch4_hop<R, LT>(out, f, t, f, v, f, nullptr, 0, 0.0, 1.0, F.lk, F.nb4, F.g, 0, 2, F.m, 0, 0, act, nrhs, st);
}

// A^dag = 1 + eps B^-1 C eps:  t = C (eps v) ; out = v + eps B^-1 t
template <class LT, class BT, class R = double>
void fullAdag_apply4(Cx<R>* out, const Cx<R>* v, Cx<R>* t, const Fine4<LT, BT>& F, const int* act, int nrhs,
                     hipStream_t st) {
  const long f = 2 * F.g.half;
  launch4_hop<R, LT>(t, f, v, f, nullptr, 0, nullptr, 0, 0.0, 1.0, F.lk, F.nb4, F.g, 0, 2, F.m, 0, 1, act, nrhs, st);
  launch4_binv<R, BT>(out, f, t, f, v, f, F.Bv, F.g, 0, 2, 1, act, nrhs, st);
}

// Dense B^-1 blocks of a 4D lattice at mass m (FP64 and an FP32 copy).
inline void build_binv4(DevBuf& b64, DevBuf& b32, const kdmg_lattice& lat, double m, hipStream_t st) {
  const Geo4& g = lat.g4;
  const long n = 2L * g.Nb2 * 48 * 48;
  if (!b64.p) b64.alloc(sizeof(c64) * n);
  if (!b32.p) b32.alloc(sizeof(c32) * n);
  hipLaunchKernelGGL(k4_binv_build, dim3(g.Nb2, 1, 2), dim3(256), 0, st, b64.as<c64>(), lat.lk64.as<c64>(), g, m);
  KDMG_LAUNCH_CHECK();
  launch_map(OpCopy<float, double>{b32.as<c32>(), b64.as<c64>(), n, nullptr}, n, 1, st);
}

}  // namespace kdmg

namespace kdmg {

// One coarse lattice (level >= 1): geometry and its block-stencil operator.
struct CoarseLevel {
  int nd = 0;
  int dims[4] = {1, 1, 1, 1};
  int nsites = 0, ndc = 0, ndir = 0;
  DevBuf nbr;                    // int [ndir][nsites]
  DevBuf Yt64, Yd64, Yt32, Yd32; // operator and adjoint, FP64 and FP32 copies
  std::vector<int> h_nbr;
  // autotuned launch shapes, keyed by nrhs * 64 + bytes per complex entry
  mutable std::map<long, TileShape> tuned;
  std::unique_ptr<std::mutex> tune_mu = std::make_unique<std::mutex>();
  long n() const { return (long)nsites * ndc; }
  size_t bytes() const { return nbr.bytes + Yt64.bytes + Yd64.bytes + Yt32.bytes + Yd32.bytes; }
};

// Transfer from level k to level k+1.
struct Transfer {
  int k = 0, nv = 0;
  Agg2 a2{};                     // k == 0 (fine -> first coarse)
  int nchild = 0, nZ = 0, nsf = 0, ndf = 0;  // k >= 1
  DevBuf P64, P16;               // prolongator values [ndof_k][nv]
  DevBuf children, parent;       // k >= 1: int [nZ][nchild], int [nsf]
  DevBuf gdir;                   // k >= 1: int [ndir][nsf], coarse direction of each fine hop (0: internal)
  // k == 0 on a 4D lattice: aggregates of agg4 KD blocks; rows4 = fine dofs of
  // each (aggregate, chirality) group [2 nZ][nrows4], dgrp4 = group of each dof
  int agg4[4] = {1, 1, 1, 1};
  int nrows4 = 0;
  DevBuf rows4, dgrp4;
  DevBuf neven4;                 // rows of each group with dof < half (a prefix of rows4)
  DevBuf relaxed;                // relaxed null vectors, FP64, internal layout [nv][n_k]
  long nfine = 0;                // entries per null vector (internal layout)
  // k == 0, 2D, asymmetric coarsening: P64 holds [fine dof][2 nv] and R64
  // the restriction transposed, [fine dof][2 nv] (asym2d.h); the mixed
  // V-cycle reads the FP32 copies P32/R32 (the thin LU can make P's entries
  // exceed the FP16 range when R~ P~ is ill-conditioned)
  bool asym = false;
  DevBuf R64, P32, R32;
  size_t bytes() const {
    return P64.bytes + P16.bytes + children.bytes + parent.bytes + gdir.bytes + relaxed.bytes + rows4.bytes +
           neven4.bytes + dgrp4.bytes + R64.bytes + P32.bytes + R32.bytes;
  }
};

// The transfers of a hierarchy, shared (read-only) between a hierarchy and
// the hierarchies derived from it at other masses.
struct TransferSet {
  std::shared_ptr<std::vector<Transfer>> p = std::make_shared<std::vector<Transfer>>();
  Transfer& operator[](size_t i) const { return (*p)[i]; }
  void resize(size_t n) { p->resize(n); }
  size_t size() const { return p->size(); }
};

void autotune_level(const CoarseLevel& L, int nrhs, bool fp32, hipStream_t st);
bool autotune_enabled();

struct SolveWS;  // solver workspace (solver.hip)
void destroy_ws(SolveWS*);
bool ws_busy(const SolveWS*);
void reset_graphs(SolveWS*);
size_t derived_footprint(const kdmg_hierarchy& base, int nrhs, kdmg_prec prec);

}  // namespace kdmg

struct kdmg_hierarchy {
  const kdmg_lattice* lat = nullptr;
  double mass = 0.0;
  kdmg_mg_params params{};
  int nlevels = 0;
  kdmg::TransferSet T;                // null vectors and prolongators (mass independent)
  bool derived = false;               // T borrowed from another hierarchy (kdmg_hierarchy_at_mass)
  std::vector<kdmg::CoarseLevel> L;   // index by level; L[0] unused
  kdmg::DevBuf gal_w;                 // Galerkin scratch W = B^-1 P (level 1), kept for rebuilds
  kdmg::DevBuf binv64, binv32;        // 4D: dense B^-1 blocks at this mass (FP64, FP32)
  kdmg::DenseInverse dinv;            // coarsest inverse (params.coarse_solver == 1)
  // The fine level: iterate on the KD-block-parity Schur system (false), or on
  // the full lattice (true: the Naik-improved operator, or multigrid on D
  // itself, params.fine_op == 1, which is `naive`).
  bool fine_full = false, naive = false;
  bool use_graphs = true;             // replay captured chunks of the coarsest CGNE
  kdmg::SolveWS* ws = nullptr;
  // event timing of the coarsest CGNE kernels (kdmg_hierarchy_kernel_timing)
  struct KTimer {
    bool on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double ms = 0.0;
    long long launches = 0;
    long long graph_replays = 0;  // captured CGNE chunks replayed (counted whether or not timing is on)
    long long tail_entries = 0;   // coarsest CGNE calls that continued as the narrower tail problem
    // exact coarsest solve: event pairs around each product launch, summed
    // when the solve ends
    std::vector<std::pair<hipEvent_t, hipEvent_t>> dn_ev;
    size_t dn_used = 0;
    // per event pair: whether the product had an active rhs (a product whose
    // rhs had all converged returns at once and is not counted)
    kdmg::DevBuf dn_work;
    static constexpr size_t DN_CAP = 4096;
  } timer;
  ~kdmg_hierarchy();
  // device bytes owned by this hierarchy (borrowed transfers not included)
  size_t bytes() const {
    size_t b = gal_w.bytes + binv64.bytes + binv32.bytes + dinv.bytes();
    if (!derived)
      for (size_t k = 0; k < T.size(); ++k) b += T[k].bytes();
    for (auto& l : L) b += l.bytes();
    return b;
  }
};

namespace kdmg {

// ------------------------------------------------------------ coarse launchers

inline void capply_shape(int ndc, int nrhs, int& js, int& rpb) {
  static const int force = [] {
    const char* e = std::getenv("KDMG_CAPPLY_JS1");
    return e ? std::atoi(e) : 0;
  }();
  if (force) {
    rpb = nrhs >= 8 ? 8 : nrhs;
    if (ndc * rpb > 1024) rpb = 1024 / ndc;
    js = 1;
    return;
  }
  rpb = nrhs >= 8 ? 8 : nrhs;
  if (ndc * rpb > 1024) rpb = 1024 / ndc;
  if (rpb < 1) rpb = 1;
  js = 256 / (ndc * rpb);
  if (js < 1) js = 1;
}

// Dispatch on the compute core of a TileShape: KERNEL(CORE, TI, TR).
#define KDMG_TILE_DISPATCH(S, KERNEL)                      \
  do {                                                     \
    if ((S).core == 1 && (S).ylds) KERNEL(1, 1, 1, 1)      \
    else if ((S).core == 1) KERNEL(1, 1, 1, 0)             \
    else if ((S).TI == 2) KERNEL(0, 2, 1, 0)               \
    else KERNEL(0, 1, 1, 0)                                \
  } while (0)

// Raise a kernel's dynamic-LDS limit above the 64 KB default, once per
// (device, kernel, size); the attribute call is not repeated on every launch.
inline void ensure_smem(const void* fn, size_t bytes) {
  if (bytes <= 65536) return;
  int dev = 0;
  KDMG_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> done;
  std::lock_guard<std::mutex> g(mu);
  size_t& d = done[{dev, fn}];
  if (d >= bytes) return;
  KDMG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  d = bytes;
}

inline TileArgs tile_args(const TileShape& s) { return TileArgs{s.RT, s.TI, s.TR, s.KS, s.MT, s.NT}; }

// ------------------------------------------------------------ fused CGNE launchers

// Key of the CGNE-specific tuned shape in CoarseLevel::tuned.
inline long cgne_key(int nrhs) { return (1L << 40) + (long)nrhs * 64 + (long)sizeof(c64); }

inline void launch_cgne_init(const TileShape& sh, const CoarseLevel& L, c64* x, c64* r, c64* p, const c64* b,
                             const CgneState& s, int nrhs, double tol2, hipStream_t st) {
  const dim3 grid(L.nsites, cdiv(nrhs, sh.RT));
  const TileArgs ta = tile_args(sh);
  hipLaunchKernelGGL(k_cgne_init1<double>, dim3(L.nsites), dim3(64), 0, st, x, r, b, L.nsites, L.ndc, nrhs, s);
#define KDMG_L_INIT2(C_, TI_, TR_, YL_)                                                                   \
  {                                                                                                  \
    auto fn = k_cgne_init2<double, double, C_, TI_, TR_, YL_>;                                         \
    ensure_smem((const void*)fn, sh.smem);                                                           \
    hipLaunchKernelGGL(fn, grid, dim3(sh.threads), sh.smem, st, p, r, L.Yd64.as<c64>(), L.nbr.as<int>(), \
                       L.nsites, L.ndc, L.ndir, ta, nrhs, s, tol2);                                  \
  }
  KDMG_TILE_DISPATCH(sh, KDMG_L_INIT2);
#undef KDMG_L_INIT2
  KDMG_LAUNCH_CHECK();
}

// iteration k: kernel A then kernel B
inline void launch_cgne_iter(const TileShape& sh, const CoarseLevel& L, c64* x, c64* r, c64* p,
                             const CgneState& s, int nrhs, int k, hipStream_t st, hipEvent_t after_A = nullptr) {
  const dim3 grid(L.nsites, cdiv(nrhs, sh.RT));
  const TileArgs ta = tile_args(sh);
  const int* nbr = L.nbr.as<int>();
#define KDMG_L_A(C_, TI_, TR_, YL_)                                                                        \
  {                                                                                                   \
    auto fn = k_cgne_A<double, double, C_, TI_, TR_, YL_>;                                              \
    ensure_smem((const void*)fn, sh.smem);                                                            \
    hipLaunchKernelGGL(fn, grid, dim3(sh.threads), sh.smem, st, x, r, p, L.Yt64.as<c64>(), nbr, L.nsites, \
                       L.ndc, L.ndir, ta, nrhs, s, k);                                                \
  }
#define KDMG_L_B(C_, TI_, TR_, YL_)                                                                        \
  {                                                                                                   \
    auto fn = k_cgne_B<double, double, C_, TI_, TR_, YL_>;                                              \
    ensure_smem((const void*)fn, sh.smem);                                                            \
    hipLaunchKernelGGL(fn, grid, dim3(sh.threads), sh.smem, st, p, r, L.Yd64.as<c64>(), nbr, L.nsites,   \
                       L.ndc, L.ndir, ta, nrhs, s, k);                                                \
  }
  KDMG_TILE_DISPATCH(sh, KDMG_L_A);
  if (after_A) KDMG_HIP(hipEventRecord(after_A, st));
  KDMG_TILE_DISPATCH(sh, KDMG_L_B);
#undef KDMG_L_A
#undef KDMG_L_B
  KDMG_LAUNCH_CHECK();
}



// The launch shape for a coarse level: the autotuned one if present, else the
// default heuristic.
inline TileShape level_shape(const CoarseLevel& L, int nrhs, size_t esz) {
  {
    std::lock_guard<std::mutex> g(*L.tune_mu);
    auto it = L.tuned.find((long)nrhs * 64 + (long)esz);
    if (it != L.tuned.end()) return it->second;
  }
  return choose_tile(L.ndc, nrhs, L.ndir, esz);
}

// launch shape of the fused CGNE: its own tuned shape if present, else the
// level's stencil shape
inline TileShape cgne_shape(const CoarseLevel& L, int nrhs) {
  {
    std::lock_guard<std::mutex> g(*L.tune_mu);
    auto it = L.tuned.find(cgne_key(nrhs));
    if (it != L.tuned.end()) return it->second;
  }
  return level_shape(L, nrhs, sizeof(c64));
}

void autotune_cgne(const CoarseLevel& L, int nrhs, hipStream_t st);

template <class R, class OT>
void coarse_apply_shape(const CoarseLevel& L, bool dag, Cx<R>* out, const Cx<R>* in, const Cx<R>* add,
                        double sgn, const int* act, int nrhs, hipStream_t st, const TileShape& s);

template <class R, class OT>
void coarse_apply(const CoarseLevel& L, bool dag, Cx<R>* out, const Cx<R>* in, const Cx<R>* add,
                  double sgn, const int* act, int nrhs, hipStream_t st) {
  coarse_apply_shape<R, OT>(L, dag, out, in, add, sgn, act, nrhs, st, level_shape(L, nrhs, sizeof(Cx<R>)));
}

template <class R, class OT>
void coarse_apply_shape(const CoarseLevel& L, bool dag, Cx<R>* out, const Cx<R>* in, const Cx<R>* add,
                        double sgn, const int* act, int nrhs, hipStream_t st, const TileShape& s) {
  const Cx<OT>* Y;
  if (sizeof(OT) == 8) Y = (const Cx<OT>*)(dag ? L.Yd64.p : L.Yt64.p);
  else Y = (const Cx<OT>*)(dag ? L.Yd32.p : L.Yt32.p);
  if (s.smem > LDS_LIMIT) {
    // stencil blocks too large for LDS: one thread per output, blocks from global memory
    int js, rpb;
    capply_shape(L.ndc, nrhs, js, rpb);
    const int threads = L.ndc * js * rpb;
    hipLaunchKernelGGL((k_capply<R, OT, R, R>), dim3(L.nsites, cdiv(nrhs, rpb)), dim3(threads),
                       threads * sizeof(Cx<R>), st, out, in, add, (R)sgn, Y, L.nbr.as<int>(), L.nsites, L.ndc,
                       L.ndir, js, rpb, nrhs, act);
    KDMG_LAUNCH_CHECK();
    return;
  }
  const dim3 grid(L.nsites, cdiv(nrhs, s.RT));
  const TileArgs ta = tile_args(s);
  // the stencil apply alone needs less LDS than the fused CGNE sharing the shape
  const size_t smem = lds_layout(s, L.ndc, L.ndir, sizeof(Cx<R>), true).total;
#define KDMG_LAUNCH_CAPPLY(C_, TI_, TR_, YL_)                                                              \
  {                                                                                                        \
    auto fn = k_capply_fast<R, OT, R, R, C_, TI_, TR_, YL_>;                                                    \
    ensure_smem((const void*)fn, smem);                                                                    \
    hipLaunchKernelGGL(fn, grid, dim3(s.threads), smem, st, out, in, add, (R)sgn, Y, L.nbr.as<int>(),      \
                       L.nsites, L.ndc, L.ndir, ta, nrhs, act);                                            \
  }
  KDMG_TILE_DISPATCH(s, KDMG_LAUNCH_CAPPLY);
#undef KDMG_LAUNCH_CAPPLY
  KDMG_LAUNCH_CHECK();
}

// restriction level k -> k+1 ; in: level-k vector (fine: block layout with
// stride `si`, even_only selects the Schur half), out: level-(k+1) vector
template <class R, class PT, class VI, class VO>
void transfer_restrict(const Transfer& T, const kdmg_lattice& lat, const CoarseLevel* Lk,
                       Cx<VO>* out, const Cx<VI>* in, long si, int even_only, const int* act,
                       int nrhs, hipStream_t st) {
  const Cx<PT>* P = (const Cx<PT>*)(sizeof(PT) == 8 ? T.P64.p : T.P16.p);
  if (T.k == 0 && T.asym) {
    // FP64 values, or the FP32 copy where the symmetric form reads FP16
    using PA = std::conditional_t<sizeof(PT) == 8, double, float>;
    const Cx<PA>* Rt = (const Cx<PA>*)(sizeof(PT) == 8 ? T.R64.p : T.R32.p);
    const int nd = 4 * T.a2.a0 * T.a2.a1, ndc = 2 * T.nv;
    int RB = nrhs < 32 ? nrhs : 32;
    auto bytes = [&] { return ((size_t)nd * ndc + (size_t)RB * nd) * sizeof(Cx<R>) + nd * sizeof(int); };
    while (RB > 1 && bytes() > 64 * 1024) RB /= 2;
    KDMG_CHECK(bytes() <= LDS_LIMIT, KDMG_EUNSUPPORTED, "restriction: aggregate too large for LDS staging");
    auto fn = k_restrict1a<R, PA, VI, VO>;
    ensure_smem((const void*)fn, bytes());
    hipLaunchKernelGGL(fn, dim3(T.a2.Ncx * T.a2.Nct, cdiv(nrhs, RB)), dim3(256), bytes(), st, out, in, si, Rt,
                       lat.g, T.a2, even_only, act, nrhs, RB);
  } else if (T.k == 0 && lat.nd == 4) {
    dim3 grid(2 * T.nZ, cdiv(T.nv, R4_RI), cdiv(nrhs, R4_RR));
    hipLaunchKernelGGL((k4_restrict<R, PT, VI, VO>), grid, dim3(256), 0, st, out, in, si, P, T.rows4.as<int>(),
                       T.neven4.as<int>(), T.nrows4, T.nv, even_only, act, nrhs);
  } else if (T.k == 0) {
    // rhs tile: up to 32, with the staged P rows and rhs values within the LDS
    const int nd = 4 * T.a2.a0 * T.a2.a1;
    int RB = nrhs < 32 ? nrhs : 32;
    auto bytes = [&] { return ((size_t)nd * T.nv + (size_t)RB * nd) * sizeof(Cx<R>) + nd * sizeof(int); };
    while (RB > 1 && bytes() > 64 * 1024) RB /= 2;
    KDMG_CHECK(bytes() <= LDS_LIMIT, KDMG_EUNSUPPORTED, "restriction: aggregate too large for LDS staging");
    dim3 grid(T.a2.Ncx * T.a2.Nct, cdiv(nrhs, RB));
    // four coarse dofs per thread only when that still fills the workgroup
    if (T.nv % 4 == 0 && RB * 2 * T.nv >= 4 * 256) {
      auto fn = k_restrict1<R, PT, VI, VO, 4>;
      ensure_smem((const void*)fn, bytes());
      hipLaunchKernelGGL(fn, grid, dim3(256), bytes(), st, out, in, si, P, lat.g, T.a2, even_only, act, nrhs, RB);
    } else {
      auto fn = k_restrict1<R, PT, VI, VO, 1>;
      ensure_smem((const void*)fn, bytes());
      hipLaunchKernelGGL(fn, grid, dim3(256), bytes(), st, out, in, si, P, lat.g, T.a2, even_only, act, nrhs, RB);
    }
  } else {
    // tiles of up to 8 rhs: four or more workgroups per aggregate at 32 rhs
    const int nrow = T.nchild * T.ndf;
    int RB = nrhs < 8 ? nrhs : 8;
    auto bytes = [&] { return ((size_t)nrow * T.nv + (size_t)RB * nrow) * sizeof(Cx<R>); };
    while (RB > 1 && bytes() > 64 * 1024) RB /= 2;
    KDMG_CHECK(bytes() <= LDS_LIMIT, KDMG_EUNSUPPORTED, "restriction: aggregate too large for LDS staging");
    auto fn = k_restrict_c<R, PT, VI, VO>;
    ensure_smem((const void*)fn, bytes());
    hipLaunchKernelGGL(fn, dim3(T.nZ, cdiv(nrhs, RB)), dim3(256), bytes(), st, out, in, P, T.children.as<int>(),
                       T.nchild, T.nsf, T.ndf, T.nZ, T.nv, act, nrhs, RB);
  }
  KDMG_LAUNCH_CHECK();
}

// prolongation level k+1 -> k: out = [add +] P in (fine: npar parities from p=0)
template <class R, class PT, class VI, class VO>
void transfer_prolong(const Transfer& T, const kdmg_lattice& lat, Cx<VO>* out, long so,
                      const Cx<VO>* add, long sa, const Cx<VI>* in, int npar, const int* act,
                      int nrhs, hipStream_t st) {
  const Cx<PT>* P = (const Cx<PT>*)(sizeof(PT) == 8 ? T.P64.p : T.P16.p);
  if (T.k == 0 && T.asym) {
    using PA = std::conditional_t<sizeof(PT) == 8, double, float>;
    const Cx<PA>* Pa = (const Cx<PA>*)(sizeof(PT) == 8 ? T.P64.p : T.P32.p);
    const int nd = 4 * T.a2.a0 * T.a2.a1, ndc = 2 * T.nv;
    int RB = nrhs < 32 ? nrhs : 32;
    auto bytes = [&] { return ((size_t)nd * (ndc + 1) + (size_t)RB * ndc) * sizeof(Cx<R>) + nd * sizeof(int); };
    while (RB > 1 && bytes() > 64 * 1024) RB /= 2;
    KDMG_CHECK(bytes() <= LDS_LIMIT, KDMG_EUNSUPPORTED, "prolongation: aggregate too large for LDS staging");
    auto fn = k_prolong1a<R, PA, VI, VO>;
    ensure_smem((const void*)fn, bytes());
    hipLaunchKernelGGL(fn, dim3(T.a2.Ncx * T.a2.Nct, cdiv(nrhs, RB)), dim3(256), bytes(), st, out, so, add, sa, in,
                       Pa, lat.g, T.a2, npar, act, nrhs, RB);
  } else if (T.k == 0 && lat.nd == 4) {
    const long n_out = npar == 1 ? lat.half : 2 * lat.half;
    constexpr int BS = sizeof(R) == 8 ? 128 : 256;
    const size_t bytes = (size_t)BS * (T.nv | 1) * sizeof(Cx<R>);
    auto fn = k4_prolong<R, PT, VI, VO, BS, 8>;
    ensure_smem((const void*)fn, bytes);
    hipLaunchKernelGGL(fn, dim3(cdiv(n_out, BS)), dim3(BS), bytes, st, out, so, add, sa, in, P, T.dgrp4.as<int>(),
                       T.nv, n_out, (long)T.nZ * 2 * T.nv, act, nrhs);
  } else if (T.k == 0) {
    const int nd = 4 * T.a2.a0 * T.a2.a1;
    int RB = nrhs < 32 ? nrhs : 32;
    auto bytes = [&] { return ((size_t)nd * (T.nv + 1) + (size_t)RB * 2 * T.nv) * sizeof(Cx<R>) + nd * sizeof(int); };
    while (RB > 1 && bytes() > 64 * 1024) RB /= 2;
    KDMG_CHECK(bytes() <= LDS_LIMIT, KDMG_EUNSUPPORTED, "prolongation: aggregate too large for LDS staging");
    auto fn = k_prolong1<R, PT, VI, VO>;
    ensure_smem((const void*)fn, bytes());
    hipLaunchKernelGGL(fn, dim3(T.a2.Ncx * T.a2.Nct, cdiv(nrhs, RB)), dim3(256), bytes(), st, out, so, add, sa, in,
                       P, lat.g, T.a2, npar, act, nrhs, RB);
  } else {
    const int nrow = T.nchild * T.ndf;
    int RB = nrhs < 8 ? nrhs : 8;
    auto bytes = [&] { return ((size_t)nrow * (T.nv + 1) + (size_t)RB * 2 * T.nv) * sizeof(Cx<R>); };
    while (RB > 1 && bytes() > 64 * 1024) RB /= 2;
    KDMG_CHECK(bytes() <= LDS_LIMIT, KDMG_EUNSUPPORTED, "prolongation: aggregate too large for LDS staging");
    auto fn = k_prolong_c<R, PT, VI, VO>;
    ensure_smem((const void*)fn, bytes());
    hipLaunchKernelGGL(fn, dim3(T.nZ, cdiv(nrhs, RB)), dim3(256), bytes(), st, out, add, in, P, T.children.as<int>(),
                       T.nchild, T.nsf, T.ndf, T.nZ, T.nv, act, nrhs, RB);
  }
  KDMG_LAUNCH_CHECK();
}

template <class TO, class TI>
void convert(Cx<TO>* y, const Cx<TI>* x, long n, int nrhs, const int* act, hipStream_t st) {
  launch_map(OpCopy<TO, TI>{y, x, n, act}, n, nrhs, st);
}

}  // namespace kdmg
