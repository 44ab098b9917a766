// Autotuner for the coarse stencil kernels: for one coarse level, rhs count
// and precision it times every candidate launch shape (MFMA tiles with the
// stencil blocks in LDS or streamed from global memory, 16 or 32 rhs per
// workgroup; SIMT register tiles with different rhs tiles and k-splits) on
// the level's real operator and keeps the fastest.  The fused coarsest-level
// CGNE kernels share the choice, since they run the same stencil core.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "internal.h"
#include "api_guard.h"

using namespace kdmg;

namespace kdmg {

std::vector<TileShape> tile_candidates(int ndc, int nrhs, int ndir, size_t esz) {
  std::vector<TileShape> out;
  if (nrhs >= 16) {
    for (int NT : {1, 2}) {
      if (NT == 2 && nrhs < 32) continue;
      for (int ylds : {1, 0}) {
        for (int minthr : {256, 512, 1024}) {
          TileShape s;
          s.core = 1;
          s.MT = (ndc + 15) / 16;
          s.NT = NT;
          s.RT = 16 * NT;
          s.ylds = ylds;
          s.threads = std::max(64 * s.MT * s.NT, minthr);
          s.smem = lds_layout(s, ndc, ndir, esz).total;
          if (s.smem <= LDS_LIMIT && s.threads <= 1024) out.push_back(s);
        }
      }
    }
  }
  for (int TI : {1, 2}) {
    if (TI == 2 && ndc % 2) continue;
    for (int RT : {16, 8, 4, 2, 1}) {
      if (RT > nrhs) continue;
      for (int KS : {1, 2, 4, 8, 16}) {
        TileShape s;
        s.core = 0;
        s.TI = TI;
        s.TR = 1;
        s.RT = RT;
        s.KS = KS;
        const int tiles = (ndc / TI) * RT;
        int thr = tiles * KS;
        if (thr > 256 || thr < 32) continue;
        s.threads = std::max(64, ((thr + 63) / 64) * 64);
        s.smem = lds_layout(s, ndc, ndir, esz).total;
        if (s.smem <= LDS_LIMIT) out.push_back(s);
      }
    }
  }
  return out;
}

template <class R, class OT>
TileShape tune_one(const CoarseLevel& L, int nrhs, hipStream_t st, bool verbose) {
  const size_t n = (size_t)nrhs * L.nsites * L.ndc;
  DevBuf a(sizeof(Cx<R>) * n), b(sizeof(Cx<R>) * n);
  KDMG_HIP(hipMemsetAsync(a.p, 0, a.bytes, st));
  const auto cands = tile_candidates(L.ndc, nrhs, L.ndir, sizeof(Cx<R>));
  hipEvent_t e0, e1;
  KDMG_HIP(hipEventCreate(&e0));
  KDMG_HIP(hipEventCreate(&e1));
  TileShape best = choose_tile(L.ndc, nrhs, L.ndir, sizeof(Cx<R>));
  float best_ms = 1e30f;
  for (const TileShape& s : cands) {
    for (int w = 0; w < 2; ++w)
      coarse_apply_shape<R, OT>(L, false, b.as<Cx<R>>(), a.as<Cx<R>>(), nullptr, 1.0, nullptr, nrhs, st, s);
    KDMG_HIP(hipEventRecord(e0, st));
    const int reps = 10;
    for (int w = 0; w < reps; ++w)
      coarse_apply_shape<R, OT>(L, false, b.as<Cx<R>>(), a.as<Cx<R>>(), nullptr, 1.0, nullptr, nrhs, st, s);
    KDMG_HIP(hipEventRecord(e1, st));
    KDMG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    KDMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    if (verbose)
      std::fprintf(stderr, "[kdmg-tune] nsites %d ndc %d nrhs %d esz %zu core %d RT %d TI %d KS %d ylds %d thr %d: %.2f us\n",
                   L.nsites, L.ndc, nrhs, sizeof(Cx<R>), s.core, s.RT, s.TI, s.KS, s.ylds, s.threads, ms * 1e3);
    if (ms < best_ms) {
      best_ms = ms;
      best = s;
    }
  }
  KDMG_HIP(hipEventDestroy(e0));
  KDMG_HIP(hipEventDestroy(e1));
  return best;
}

void autotune_level(const CoarseLevel& L, int nrhs, bool fp32, hipStream_t st) {
  const size_t esz = fp32 ? sizeof(c32) : sizeof(c64);
  const long key = (long)nrhs * 64 + (long)esz;
  {
    std::lock_guard<std::mutex> g(*L.tune_mu);
    if (L.tuned.count(key)) return;
  }
  const char* e = std::getenv("KDMG_TUNE_VERBOSE");
  const bool verbose = e && e[0] == '1';
  TileShape best = fp32 ? tune_one<float, float>(L, nrhs, st, verbose) : tune_one<double, double>(L, nrhs, st, verbose);
  std::lock_guard<std::mutex> g(*L.tune_mu);
  L.tuned.emplace(key, best);  // a concurrent tuner that finished first wins
}

bool autotune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("KDMG_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

}  // namespace kdmg

extern "C" kdmg_status kdmg_hierarchy_autotune(kdmg_hierarchy* h, int nrhs, kdmg_prec prec, void* stream) {
  KDMG_API_BEGIN
  KDMG_CHECK(h && nrhs >= 1 && nrhs <= 1024, KDMG_EINVAL, "kdmg_hierarchy_autotune: bad argument");
  hipStream_t st = (hipStream_t)stream;
  for (int l = 1; l < h->nlevels; ++l) {
    const bool coarsest = l == h->nlevels - 1;
    const bool fp32 = prec == KDMG_MIXED && !coarsest;
    autotune_level(h->L[l], nrhs, fp32, st);
  }
  KDMG_HIP(hipStreamSynchronize(st));
  KDMG_API_END
}
