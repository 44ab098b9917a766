// Lattice handle (gauge field upload, layouts) and the fine-level operator
// entry points: D, A, A^dag, B^-1 and the Schur operator.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "internal.h"
#include "api_guard.h"

using namespace kdmg;

namespace kdmg {

// Work space of kdmg_apply_schur_noalloc, for callers that cannot allocate:
// a fixed array in device memory, one per GPU, held until the process ends.
// Host code never uses the symbol itself (on the host it is only a stand-in
// for the device address): it uses the address hipGetSymbolAddress returns
// for the current device, looked up once per device (scratch_address).
constexpr size_t SCRATCH_BYTES = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

}  // namespace kdmg

namespace {

// Fold 1/2 eta_mu(x) bc_mu(x) into the links (2D, U(1)): the boundary sign
// of direction mu sits on the links that leave the last slice in mu.
void fold_links_2d(const kdmg_lattice& lat, const double* links, std::vector<c64>& nat) {
  const int Lx = lat.dims[0], Lt = lat.dims[1];
  const long V = lat.volume;
  nat.assign(2 * V, c64{0, 0});
  for (long x = 0; x < V; ++x) {
    const int x0 = (int)(x % Lx), x1 = (int)(x / Lx);
    const double eta1 = (x0 & 1) ? -1.0 : 1.0;
    const double bc0 = x0 == Lx - 1 ? (double)lat.bc[0] : 1.0;
    const double bc1 = x1 == Lt - 1 ? (double)lat.bc[1] : 1.0;
    const double* u0 = links + 2 * (0 * V + x);
    const double* u1 = links + 2 * (1 * V + x);
    nat[x] = c64{0.5 * bc0 * u0[0], 0.5 * bc0 * u0[1]};
    nat[V + x] = c64{0.5 * eta1 * bc1 * u1[0], 0.5 * eta1 * bc1 * u1[1]};
  }
}

// 4D SU(3): geometry, folded links, neighbour table and permutations.
void create_4d(kdmg_lattice& lat, const double* links, hipStream_t st) {
  Geo4& g = lat.g4;
  for (int mu = 0; mu < 4; ++mu) {
    g.L[mu] = lat.dims[mu];
    g.NB[mu] = lat.dims[mu] / 2;
  }
  const long V = lat.volume;
  g.Nb2 = (int)(V / 16 / 2);
  g.half = (long)g.Nb2 * 48;
  lat.ndof = 3 * V;
  lat.half = g.half;
  const int* L = g.L;
  auto nat_index = [&](const int x[4]) { return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3])); };
  auto blk_site = [&](const int x[4]) {
    int Bc[4], s = 0;
    for (int mu = 0; mu < 4; ++mu) {
      Bc[mu] = x[mu] >> 1;
      s |= (x[mu] & 1) << mu;
    }
    return ((long)blk4_parity(Bc) * g.Nb2 + blk4_index(g, Bc)) * 16 + s;
  };
  std::vector<c64> lk((size_t)V * 4 * 9);
  std::vector<int> nb((size_t)V * 8);
  lat.h_perm_full.assign(3 * V, 0);
  int x[4];
  for (long n = 0; n < V; ++n) {
    long r = n;
    for (int mu = 0; mu < 4; ++mu) {
      x[mu] = (int)(r % L[mu]);
      r /= L[mu];
    }
    const long ib = blk_site(x);
    for (int c = 0; c < 3; ++c) lat.h_perm_full[3 * n + c] = (int)(3 * ib + c);
    int parity = 0;  // sum_{nu < mu} x_nu
    for (int mu = 0; mu < 4; ++mu) {
      const double eta = (parity & 1) ? -1.0 : 1.0;
      parity += x[mu];
      const double bc = x[mu] == L[mu] - 1 ? (double)lat.bc[mu] : 1.0;
      const double* u = links + 2 * (((long)mu * V + n) * 9);
      for (int e = 0; e < 9; ++e)
        lk[((size_t)ib * 4 + mu) * 9 + e] = c64{0.5 * eta * bc * u[2 * e], 0.5 * eta * bc * u[2 * e + 1]};
      int y[4] = {x[0], x[1], x[2], x[3]};
      y[mu] = (x[mu] + 1) % L[mu];
      nb[ib * 8 + 2 * mu] = (int)blk_site(y);
      y[mu] = (x[mu] + L[mu] - 1) % L[mu];
      nb[ib * 8 + 2 * mu + 1] = (int)blk_site(y);
    }
  }
  lat.h_perm_even.assign(3 * V / 2, 0);
  long rank = 0;
  for (long n = 0; n < V; ++n) {
    const long bd = lat.h_perm_full[3 * n];
    if (bd < 3 * (V / 2))
      for (int c = 0; c < 3; ++c) lat.h_perm_even[rank++] = (int)(bd + c);
  }
  KDMG_CHECK(rank == 3 * V / 2, KDMG_EINVAL, "even-block count mismatch");
  lat.lk64.alloc(lk.size() * sizeof(c64));
  lat.lk32.alloc(lk.size() * sizeof(c32));
  lat.lk16.alloc(lk.size() * sizeof(c16));
  lat.nb4.alloc(nb.size() * sizeof(int));
  lat.perm_full.alloc(lat.h_perm_full.size() * sizeof(int));
  lat.perm_even.alloc(lat.h_perm_even.size() * sizeof(int));
  KDMG_HIP(hipMemcpyAsync(lat.lk64.p, lk.data(), lat.lk64.bytes, hipMemcpyHostToDevice, st));
  KDMG_HIP(hipMemcpyAsync(lat.nb4.p, nb.data(), lat.nb4.bytes, hipMemcpyHostToDevice, st));
  KDMG_HIP(hipMemcpyAsync(lat.perm_full.p, lat.h_perm_full.data(), lat.perm_full.bytes, hipMemcpyHostToDevice, st));
  KDMG_HIP(hipMemcpyAsync(lat.perm_even.p, lat.h_perm_even.data(), lat.perm_even.bytes, hipMemcpyHostToDevice, st));
  convert<_Float16, double>(lat.lk16.as<c16>(), lat.lk64.as<c64>(), (long)lk.size(), 1, nullptr, st);
  convert<float, double>(lat.lk32.as<c32>(), lat.lk64.as<c64>(), (long)lk.size(), 1, nullptr, st);
  KDMG_HIP(hipStreamSynchronize(st));
}

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of its `scratch`

// Resolves (once per device, with that device current) and returns the
// current device's scratch address.
void* scratch_address() {
  int dev = 0;
  KDMG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw Error(KDMG_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

}  // namespace

extern "C" kdmg_status kdmg_init(int device) {
  KDMG_API_BEGIN
  int n = 0;
  KDMG_HIP(hipGetDeviceCount(&n));
  KDMG_CHECK(device >= 0 && device < n, KDMG_EINVAL, "kdmg_init: no such device");
  KDMG_HIP(hipSetDevice(device));
  (void)scratch_address();
  KDMG_API_END
}

extern "C" kdmg_status kdmg_lattice_create(int nd, const int* dims, int ncolor, const int* bc_sign,
                                           const double* links_host, void* stream, kdmg_lattice** out) {
  KDMG_API_BEGIN
  KDMG_CHECK(out && dims && links_host, KDMG_EINVAL, "kdmg_lattice_create: null argument");
  *out = nullptr;
  if (bc_sign)
    for (int mu = 0; mu < nd && mu < 4; ++mu)
      KDMG_CHECK(bc_sign[mu] == 1 || bc_sign[mu] == -1, KDMG_EINVAL,
                 "kdmg_lattice_create: boundary signs must be +1 or -1");
  if (!((nd == 2 && ncolor == 1) || (nd == 4 && ncolor == 3)))
    throw Error(KDMG_EUNSUPPORTED, "kdmg_lattice_create: built for nd=2 with ncolor=1 and nd=4 with ncolor=3");
  for (int mu = 0; mu < nd; ++mu)
    KDMG_CHECK(dims[mu] >= 4 && dims[mu] % 4 == 0, KDMG_EINVAL,
               "kdmg_lattice_create: extents must be positive multiples of 4");
  auto lat = std::make_unique<kdmg_lattice>();
  lat->nd = nd;
  lat->nc = ncolor;
  lat->volume = 1;
  for (int mu = 0; mu < nd; ++mu) {
    lat->dims[mu] = dims[mu];
    lat->volume *= dims[mu];
  }
  for (int mu = 0; mu < nd; ++mu) lat->bc[mu] = bc_sign ? bc_sign[mu] : (mu == nd - 1 ? -1 : 1);
  hipStream_t st = (hipStream_t)stream;
  if (nd == 4) {
    KDMG_CHECK(lat->volume <= (1L << 26), KDMG_EINVAL, "kdmg_lattice_create: 4D volume too large");
    create_4d(*lat, links_host, st);
    *out = lat.release();
    return KDMG_OK;
  }
  Geo2& g = lat->g;
  g.Lx = dims[0];
  g.Lt = dims[1];
  g.Bx = g.Lx / 2;
  g.Bt = g.Lt / 2;
  g.hBx = g.Bx / 2;
  g.Nb2 = g.Bx * g.Bt / 2;
  g.half = 4L * g.Nb2;
  lat->ndof = lat->volume;
  lat->half = g.half;
  const long V = lat->volume;

  std::vector<c64> nat;
  fold_links_2d(*lat, links_host, nat);
  lat->h_links.assign(reinterpret_cast<const c64*>(links_host), reinterpret_cast<const c64*>(links_host) + 2 * V);
  std::vector<c64> blk(2L * g.Nb2 * 8);
  lat->h_perm_full.assign(V, 0);
  lat->h_perm_even.assign(V / 2, 0);
  auto site = [&](int x0, int x1) { return (long)x1 * g.Lx + x0; };
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < g.Nb2; ++b) {
      int X0, X1;
      blk_coords(g, p, b, X0, X1);
      const long s0 = site(2 * X0, 2 * X1), s1 = site(2 * X0 + 1, 2 * X1);
      const long s2 = site(2 * X0, 2 * X1 + 1), s3 = site(2 * X0 + 1, 2 * X1 + 1);
      c64* L = &blk[((long)p * g.Nb2 + b) * 8];
      L[0] = nat[s0];          // U~_0(s0)
      L[1] = nat[V + s0];      // U~_1(s0)
      L[2] = nat[V + s1];      // U~_1(s1)
      L[3] = nat[s2];          // U~_0(s2)
      L[4] = nat[s1];          // U~_0(s1)  -> X+0
      L[5] = nat[s3];          // U~_0(s3)  -> X+0
      L[6] = nat[V + s2];      // U~_1(s2)  -> X+1
      L[7] = nat[V + s3];      // U~_1(s3)  -> X+1
      const long sites[4] = {s0, s1, s2, s3};
      for (int s = 0; s < 4; ++s) lat->h_perm_full[sites[s]] = (int)(((long)p * g.Nb2 + b) * 4 + s);
    }
  long rank = 0;
  for (long x = 0; x < V; ++x) {
    const int x0 = (int)(x % g.Lx), x1 = (int)(x / g.Lx);
    if ((((x0 >> 1) + (x1 >> 1)) & 1) == 0) lat->h_perm_even[rank++] = lat->h_perm_full[x];
  }
  KDMG_CHECK(rank == V / 2, KDMG_EINVAL, "even-block count mismatch");

  lat->links64.alloc(blk.size() * sizeof(c64));
  lat->links32.alloc(blk.size() * sizeof(c32));
  lat->links16.alloc(blk.size() * sizeof(c16));
  lat->nat64.alloc(nat.size() * sizeof(c64));
  lat->nat16.alloc(nat.size() * sizeof(c16));
  lat->perm_full.alloc(V * sizeof(int));
  lat->perm_even.alloc(V / 2 * sizeof(int));
  KDMG_HIP(hipMemcpyAsync(lat->links64.p, blk.data(), lat->links64.bytes, hipMemcpyHostToDevice, st));
  KDMG_HIP(hipMemcpyAsync(lat->nat64.p, nat.data(), lat->nat64.bytes, hipMemcpyHostToDevice, st));
  KDMG_HIP(hipMemcpyAsync(lat->perm_full.p, lat->h_perm_full.data(), lat->perm_full.bytes, hipMemcpyHostToDevice,
                          st));
  KDMG_HIP(hipMemcpyAsync(lat->perm_even.p, lat->h_perm_even.data(), lat->perm_even.bytes, hipMemcpyHostToDevice,
                          st));
  convert<_Float16, double>(lat->links16.as<c16>(), lat->links64.as<c64>(), (long)blk.size(), 1, nullptr, st);
  convert<float, double>(lat->links32.as<c32>(), lat->links64.as<c64>(), (long)blk.size(), 1, nullptr, st);
  convert<_Float16, double>(lat->nat16.as<c16>(), lat->nat64.as<c64>(), (long)nat.size(), 1, nullptr, st);
  KDMG_HIP(hipStreamSynchronize(st));
  *out = lat.release();
  KDMG_API_END
}

extern "C" kdmg_status kdmg_lattice_set_naik(kdmg_lattice* lat, int enable, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(lat, KDMG_EINVAL, "kdmg_lattice_set_naik: null lattice");
  KDMG_CHECK(lat->nd == 2 && lat->nc == 1, KDMG_EUNSUPPORTED, "kdmg_lattice_set_naik: 2D U(1) lattices only");
  if (!enable) {
    lat->naik = 0;
    lat->c1 = 1.0;
    lat->c3 = 0.0;
    return KDMG_OK;
  }
  KDMG_CHECK(lat->dims[0] >= 8 && lat->dims[1] >= 8, KDMG_EINVAL,
             "kdmg_lattice_set_naik: extents must be at least 8 (three-link hops)");
  hipStream_t st = (hipStream_t)stream;
  const int Lx = lat->dims[0], Lt = lat->dims[1];
  const long V = lat->volume, f = 2 * lat->half;
  const c64* U = lat->h_links.data();
  std::vector<c64> natw(2 * V), blkw(2 * V);
  for (long x = 0; x < V; ++x) {
    const int x0 = (int)(x % Lx), x1 = (int)(x / Lx);
    for (int mu = 0; mu < 2; ++mu) {
      const int L = mu == 0 ? Lx : Lt, xm = mu == 0 ? x0 : x1;
      c64 w{1.0, 0.0};
      for (int k = 0; k < 3; ++k) {
        const int y0 = mu == 0 ? (x0 + k) % Lx : x0, y1 = mu == 1 ? (x1 + k) % Lt : x1;
        w = w * U[(long)mu * V + (long)y1 * Lx + y0];
      }
      const double eta = mu == 1 && (x0 & 1) ? -1.0 : 1.0;
      const double bc = xm + 3 >= L ? (double)lat->bc[mu] : 1.0;
      const c64 wf{0.5 * eta * bc * w.re, 0.5 * eta * bc * w.im};
      natw[(long)mu * V + x] = wf;
      blkw[(long)mu * f + blk_site_index(lat->g, x0, x1)] = wf;
    }
  }
  lat->natw64.alloc(sizeof(c64) * 2 * V);
  lat->natw16.alloc(sizeof(c16) * 2 * V);
  lat->wl64.alloc(sizeof(c64) * 2 * f);
  lat->wl16.alloc(sizeof(c16) * 2 * f);
  KDMG_HIP(hipMemcpyAsync(lat->natw64.p, natw.data(), lat->natw64.bytes, hipMemcpyHostToDevice, st));
  KDMG_HIP(hipMemcpyAsync(lat->wl64.p, blkw.data(), lat->wl64.bytes, hipMemcpyHostToDevice, st));
  convert<_Float16, double>(lat->natw16.as<c16>(), lat->natw64.as<c64>(), 2 * V, 1, nullptr, st);
  convert<_Float16, double>(lat->wl16.as<c16>(), lat->wl64.as<c64>(), 2 * f, 1, nullptr, st);
  KDMG_HIP(hipStreamSynchronize(st));
  lat->naik = 1;
  lat->c1 = 9.0 / 8.0;
  lat->c3 = -1.0 / 24.0;
  KDMG_API_END
}

extern "C" void kdmg_lattice_destroy(kdmg_lattice* lat) { delete lat; }

extern "C" kdmg_status kdmg_lattice_footprint(const kdmg_lattice* lat, size_t* bytes) {
  KDMG_API_BEGIN
  KDMG_CHECK(lat && bytes, KDMG_EINVAL, "null argument");
  *bytes = lat->footprint();
  KDMG_API_END
}

extern "C" kdmg_status kdmg_apply_D(const kdmg_lattice* lat, double mass, const void* in, void* out,
                                    int nrhs, kdmg_prec prec, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(lat && in && out, KDMG_EINVAL, "kdmg_apply_D: null argument");
  KDMG_CHECK(nrhs >= 1 && nrhs <= 65535, KDMG_EINVAL, "kdmg_apply_D: bad nrhs");
  KDMG_CHECK(in != out, KDMG_EINVAL, "kdmg_apply_D: in and out must not alias");
  hipStream_t st = (hipStream_t)stream;
  const long V = lat->volume;
  if (lat->nd == 4) {
    // block layout: gather, D, scatter
    const long f = 2 * lat->half, n = lat->ndof;
    const int* perm = lat->perm_full.as<int>();
    if (prec == KDMG_FP64) {
      DevBuf a(sizeof(c64) * f * nrhs), b(sizeof(c64) * f * nrhs);
      launch_permute<double, double>(a.as<c64>(), f, (const c64*)in, n, perm, n, 1, nrhs, st);
      launch4_hop<double, double>(b.as<c64>(), f, a.as<c64>(), f, nullptr, 0, nullptr, 0, 0.0, 1.0,
                                  lat->lk64.as<c64>(), lat->nb4.as<int>(), lat->g4, 0, 2, mass, 2, 0, nullptr, nrhs,
                                  st);
      launch_permute<double, double>((c64*)out, n, b.as<c64>(), f, perm, n, 0, nrhs, st);
      KDMG_HIP(hipStreamSynchronize(st));
    } else if (prec == KDMG_MIXED) {
      DevBuf a(sizeof(c32) * f * nrhs), b(sizeof(c32) * f * nrhs);
      launch_permute<float, float>(a.as<c32>(), f, (const c32*)in, n, perm, n, 1, nrhs, st);
      launch4_hop<float, _Float16>(b.as<c32>(), f, a.as<c32>(), f, nullptr, 0, nullptr, 0, 0.0, 1.0,
                                   lat->lk16.as<c16>(), lat->nb4.as<int>(), lat->g4, 0, 2, mass, 2, 0, nullptr,
                                   nrhs, st);
      launch_permute<float, float>((c32*)out, n, b.as<c32>(), f, perm, n, 0, nrhs, st);
      KDMG_HIP(hipStreamSynchronize(st));
    } else {
      throw Error(KDMG_EINVAL, "kdmg_apply_D: bad precision");
    }
    return KDMG_OK;
  }
  if (lat->naik) {
    const dim3 gn(cdiv(V, 256), nrhs);
    if (prec == KDMG_FP64)
      hipLaunchKernelGGL((k_dslash_naik_nat<double, double, double>), gn, dim3(256), 0, st, (c64*)out,
                         (const c64*)in, lat->nat64.as<c64>(), lat->natw64.as<c64>(), lat->dims[0], lat->dims[1], V,
                         mass, lat->c1, lat->c3);
    else if (prec == KDMG_MIXED)
      hipLaunchKernelGGL((k_dslash_naik_nat<float, _Float16, float>), gn, dim3(256), 0, st, (c32*)out,
                         (const c32*)in, lat->nat16.as<c16>(), lat->natw16.as<c16>(), lat->dims[0], lat->dims[1], V,
                         (float)mass, (float)lat->c1, (float)lat->c3);
    else
      throw Error(KDMG_EINVAL, "kdmg_apply_D: bad precision");
    KDMG_LAUNCH_CHECK();
    return KDMG_OK;
  }
  // several rhs per thread (links read once per site, more loads in flight)
  // when there are enough sites to fill the device
  const int RB = V < 16384 ? 1 : nrhs >= 8 ? 8 : nrhs >= 4 ? 4 : 1;
  dim3 grid(cdiv(V, 256), cdiv(nrhs, RB));
  auto launch = [&](auto r_tag, auto l_tag, const auto* U) {
    using R = decltype(r_tag);
    using LT = decltype(l_tag);
    const Cx<LT>* Ul = (const Cx<LT>*)U;
    if (RB == 8)
      hipLaunchKernelGGL((k_dslash_nat<R, LT, R, 8>), grid, dim3(256), 0, st, (Cx<R>*)out, (const Cx<R>*)in, Ul,
                         Ul + V, lat->dims[0], lat->dims[1], V, (R)mass, nrhs);
    else if (RB == 4)
      hipLaunchKernelGGL((k_dslash_nat<R, LT, R, 4>), grid, dim3(256), 0, st, (Cx<R>*)out, (const Cx<R>*)in, Ul,
                         Ul + V, lat->dims[0], lat->dims[1], V, (R)mass, nrhs);
    else
      hipLaunchKernelGGL((k_dslash_nat<R, LT, R, 1>), grid, dim3(256), 0, st, (Cx<R>*)out, (const Cx<R>*)in, Ul,
                         Ul + V, lat->dims[0], lat->dims[1], V, (R)mass, nrhs);
  };
  if (prec == KDMG_FP64) {
    launch(double{}, double{}, lat->nat64.as<c64>());
  } else if (prec == KDMG_MIXED && (((uintptr_t)in | (uintptr_t)out) & 15) != 0) {
    launch(float{}, _Float16{}, lat->nat16.as<c16>());  // vectors not 16-byte aligned: one site per thread
  } else if (prec == KDMG_MIXED) {
    // two sites per thread with 16-byte vector accesses (k_dslash_nat2)
    const Cx<_Float16>* Ul = lat->nat16.as<c16>();
    const dim3 g2(cdiv(V / 2, 256), cdiv(nrhs, RB));
    if (RB == 8)
      hipLaunchKernelGGL(k_dslash_nat2<8>, g2, dim3(256), 0, st, (c32*)out, (const c32*)in, Ul, Ul + V, lat->dims[0],
                         lat->dims[1], V, (float)mass, nrhs);
    else if (RB == 4)
      hipLaunchKernelGGL(k_dslash_nat2<4>, g2, dim3(256), 0, st, (c32*)out, (const c32*)in, Ul, Ul + V, lat->dims[0],
                         lat->dims[1], V, (float)mass, nrhs);
    else
      hipLaunchKernelGGL(k_dslash_nat2<1>, g2, dim3(256), 0, st, (c32*)out, (const c32*)in, Ul, Ul + V, lat->dims[0],
                         lat->dims[1], V, (float)mass, nrhs);
  } else {
    throw Error(KDMG_EINVAL, "kdmg_apply_D: bad precision");
  }
  KDMG_LAUNCH_CHECK();
  KDMG_API_END
}

namespace {

enum FineOp { OP_A, OP_ADAG, OP_BINV, OP_SCHUR };

// Complex entries of work space a fine-operator call needs per rhs: gathered
// input a, output b, and the temporaries t and w (the Schur operator's input
// and output are even-block halves).
long fine_op_scratch_entries(const kdmg_lattice& lat, FineOp op) {
  const long h = lat.half, f = 2 * h;
  return op == OP_SCHUR ? 2 * h + 2 * f : 4 * f;
}

// One fine operator on natural-order vectors: gather into the block layout,
// apply, scatter back.  R = double: complex128 vectors and FP64 links;
// R = float: complex64 vectors, FP16-stored links (FP32 B^-1 blocks in 4D).
// `work`: caller-provided space of fine_op_scratch_entries * nrhs entries, or
// null to allocate it for the call.
template <class R>
void fine_op_natural(const kdmg_lattice* lat, double mass, const void* in, void* out, int nrhs, FineOp op,
                     hipStream_t st, Cx<R>* work) {
  KDMG_CHECK(lat && in && out, KDMG_EINVAL, "null argument");
  KDMG_CHECK(nrhs >= 1 && nrhs <= 65535, KDMG_EINVAL, "bad nrhs");
  KDMG_CHECK(in != out, KDMG_EINVAL, "in and out must not alias");
  using LT = std::conditional_t<sizeof(R) == 8, double, _Float16>;
  const Geo2& g = lat->g;
  const long h = lat->half, f = 2 * h, V = lat->ndof;
  const long na = op == OP_SCHUR ? h : f;
  DevBuf own;
  if (!work) {
    own.alloc(sizeof(Cx<R>) * fine_op_scratch_entries(*lat, op) * nrhs);
    work = own.as<Cx<R>>();
  }
  Cx<R>* a = work;
  Cx<R>* b = a + na * nrhs;
  Cx<R>* t = b + na * nrhs;
  Cx<R>* w = t + f * nrhs;
  const Cx<R>* vin = (const Cx<R>*)in;
  Cx<R>* vout = (Cx<R>*)out;
  if (lat->nd == 4) {
    DevBuf b64, b32;
    build_binv4(b64, b32, *lat, mass, st);
    const Cx<LT>* lk = (const Cx<LT>*)(sizeof(R) == 8 ? lat->lk64.p : lat->lk16.p);
    const Cx<R>* Bv = (const Cx<R>*)(sizeof(R) == 8 ? b64.p : b32.p);
    const Fine4<LT, R> F{lk, lat->nb4.as<int>(), Bv, lat->g4, mass};
    if (op == OP_SCHUR) {
      launch_permute<R, R>(a, h, vin, V / 2, lat->perm_even.as<int>(), V / 2, 1, nrhs, st);
      schur_apply4<R, LT, R>(b, a, nullptr, t, w, F, nullptr, nrhs, st);
      launch_permute<R, R>(vout, V / 2, b, h, lat->perm_even.as<int>(), V / 2, 0, nrhs, st);
    } else {
      launch_permute<R, R>(a, f, vin, V, lat->perm_full.as<int>(), V, 1, nrhs, st);
      if (op == OP_A)
        fullA_apply4<LT, R, R>(b, a, t, F, nullptr, nrhs, st);
      else if (op == OP_ADAG)
        fullAdag_apply4<LT, R, R>(b, a, t, F, nullptr, nrhs, st);
      else
        launch4_binv<R, R>(b, f, a, f, nullptr, 0, F.Bv, F.g, 0, 2, 0, nullptr, nrhs, st);
      launch_permute<R, R>(vout, V, b, f, lat->perm_full.as<int>(), V, 0, nrhs, st);
    }
    KDMG_HIP(hipStreamSynchronize(st));  // the B^-1 blocks are freed on return
    return;
  }
  const Cx<LT>* L = (const Cx<LT>*)(sizeof(R) == 8 ? lat->links64.p : lat->links16.p);
  if (op == OP_SCHUR) {
    KDMG_CHECK(!lat->naik, KDMG_EUNSUPPORTED,
               "the Naik-improved operator has no KD-block-parity Schur form (its three-link hops join "
               "blocks of the same parity)");
    launch_permute<R, R>(a, h, vin, V / 2, lat->perm_even.as<int>(), V / 2, 1, nrhs, st);
    schur_apply<R, LT>(b, a, nullptr, t, w, L, g, mass, nullptr, nrhs, st);
    launch_permute<R, R>(vout, V / 2, b, h, lat->perm_even.as<int>(), V / 2, 0, nrhs, st);
  } else {
    const Fine2<LT> F = fine2<LT>(*lat, mass);
    launch_permute<R, R>(a, f, vin, V, lat->perm_full.as<int>(), V, 1, nrhs, st);
    if (op == OP_A) {
      fine2_A<R, LT>(b, a, nullptr, t, F, nullptr, nrhs, st);
    } else if (op == OP_ADAG) {
      fine2_Adag<R, LT>(b, nullptr, a, t, F, nullptr, nrhs, st);
    } else {
      // B^-1 = B~^-1 / s for the rescaled block
      launch_binv<R, LT, R>(b, f, nullptr, 0, a, f, nullptr, 0, L, g, 0, 2, F.me, 0, nullptr, nrhs, st);
      if (F.s != 1.0) launch_map(OpAxpby<R>{b, b, nullptr, f, 1.0 / F.s, 0.0, nullptr}, f, nrhs, st);
    }
    launch_permute<R, R>(vout, V, b, f, lat->perm_full.as<int>(), V, 0, nrhs, st);
  }
  if (own.p) KDMG_HIP(hipStreamSynchronize(st));  // the work space is freed on return
}

void fine_op_prec(const kdmg_lattice* lat, double mass, const void* in, void* out, int nrhs, FineOp op,
                  kdmg_prec prec, hipStream_t st) {
  if (prec == KDMG_FP64)
    fine_op_natural<double>(lat, mass, in, out, nrhs, op, st, nullptr);
  else if (prec == KDMG_MIXED)
    fine_op_natural<float>(lat, mass, in, out, nrhs, op, st, nullptr);
  else
    throw Error(KDMG_EINVAL, "bad precision");
}

}  // namespace

extern "C" kdmg_status kdmg_apply_A(const kdmg_lattice* lat, double mass, const void* in, void* out,
                                    int nrhs, int dagger, kdmg_prec prec, void* stream) {
  KDMG_API_BEGIN
  fine_op_prec(lat, mass, in, out, nrhs, dagger ? OP_ADAG : OP_A, prec, (hipStream_t)stream);
  KDMG_API_END
}

extern "C" kdmg_status kdmg_apply_Binv(const kdmg_lattice* lat, double mass, const void* in,
                                       void* out, int nrhs, void* stream) {
  KDMG_API_BEGIN
  fine_op_prec(lat, mass, in, out, nrhs, OP_BINV, KDMG_FP64, (hipStream_t)stream);
  KDMG_API_END
}

extern "C" kdmg_status kdmg_apply_schur(const kdmg_lattice* lat, double mass, const void* in_even,
                                        void* out_even, int nrhs, void* stream) {
  KDMG_API_BEGIN
  fine_op_prec(lat, mass, in_even, out_even, nrhs, OP_SCHUR, KDMG_FP64, (hipStream_t)stream);
  KDMG_API_END
}

extern "C" kdmg_status kdmg_apply_schur_noalloc(const kdmg_lattice* lat, double mass, const void* in_even,
                                                void* out_even, int nrhs, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(lat, KDMG_EINVAL, "kdmg_apply_schur_noalloc: null lattice");
  KDMG_CHECK(lat->nd == 2, KDMG_EUNSUPPORTED,
             "kdmg_apply_schur_noalloc: 2D lattices only (the 4D B^-1 blocks are built per call)");
  KDMG_CHECK(nrhs >= 1 && nrhs <= 65535, KDMG_EINVAL, "kdmg_apply_schur_noalloc: bad nrhs");
  const size_t need = sizeof(c64) * (size_t)fine_op_scratch_entries(*lat, OP_SCHUR) * (size_t)nrhs;
  if (need > SCRATCH_BYTES)
    throw Error(KDMG_EINVAL, "kdmg_apply_schur_noalloc: " + std::to_string(nrhs) + " rhs need " +
                                 std::to_string(need) + " bytes of work space, above the fixed " +
                                 std::to_string(SCRATCH_BYTES) + " (at most " +
                                 std::to_string(SCRATCH_BYTES / (sizeof(c64) * fine_op_scratch_entries(*lat, OP_SCHUR))) +
                                 " rhs on this lattice)");
  c64* work = static_cast<c64*>(scratch_address());
  fine_op_natural<double>(lat, mass, in_even, out_even, nrhs, OP_SCHUR, (hipStream_t)stream, work);
  KDMG_API_END
}

extern "C" const char* kdmg_status_string(kdmg_status s) {
  switch (s) {
    case KDMG_OK: return "ok";
    case KDMG_EINVAL: return "invalid argument";
    case KDMG_ENOMEM: return "out of device memory";
    case KDMG_EHIP: return "HIP runtime error";
    case KDMG_ENOCONV: return "solver did not converge";
    case KDMG_EBUSY: return "busy";
    case KDMG_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" const char* kdmg_last_error(void) { return kdmg::last_error(); }

extern "C" void kdmg_default_params(kdmg_mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nlevels = 3;
  p->lvl[0].agg[0] = p->lvl[0].agg[1] = p->lvl[0].agg[2] = p->lvl[0].agg[3] = 4;
  p->lvl[0].nvec = 8;
  p->lvl[1].agg[0] = p->lvl[1].agg[1] = p->lvl[1].agg[2] = p->lvl[1].agg[3] = 2;
  p->lvl[1].nvec = 12;
  p->lvl[2] = p->lvl[1];
  p->setup_tol = 1e-4;
  p->setup_maxit = 250;
  p->outer_restart = 32;
  p->outer_maxit = 2000;
  p->mr_its = 2;
  p->mr_omega = 0.85;
  p->inter_restart = 8;
  p->inter_maxit = 16;
  p->inter_tol = 0.2;
  p->coarse_tol = 0.2;
  p->coarse_maxit = 256;
  p->outer_stall = 0;
  p->coarse_tail = 16;
  p->coarse_solver = 0;
  p->fine_op = 0;
  p->asymmetric = 0;
}
