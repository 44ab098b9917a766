// Exact coarsest-level solve through an explicit inverse (an option beside
// the CGNE(0.2) of Table 1).
//
// Build, once per hierarchy and mass, in FP64:
//   N = A A^dag                 (Hermitian positive definite; dense, formed
//                                from the nearest-neighbour stencil blocks),
//   N^-1                        (blocked Gauss-Jordan in place: positive
//                                definite, so no pivoting is needed),
//   X = A^dag N^-1 = A^-1.
// Each coarsest call is then one dense product x = X b for all rhs of the
// batch: X is streamed once per call and every element serves the whole rhs
// tile (FP64 MFMA, three real products per complex one).  Going through the
// normal matrix costs its squared condition number in rounding (kappa(A)^2
// times 1e-16; kappa(A) is about 10^3 at the masses used here), far inside
// what a preconditioner needs.
#pragma once
#include "common.h"

namespace kdmg {

struct CoarseLevel;
struct KrylovState;

struct DenseInverse {
  long n = 0;           // coarsest dofs
  DevBuf X;             // A^-1, row-major [n][n] complex FP64
  DevBuf N;             // build work: A A^dag, inverted in place
  DevBuf G, R, C;       // Gauss-Jordan panels: pivot-block inverse [w][w], row panel [w][n], column panel [n][w]
  bool built = false;
  size_t bytes() const { return X.bytes + N.bytes + G.bytes + R.bytes + C.bytes; }
};

// Gauss-Jordan block width.
constexpr int DN_W = 32;

// Builds (or rebuilds, reusing the buffers) the inverse of level L's operator.
void build_dense_inverse(DenseInverse& D, const CoarseLevel& L, hipStream_t st);

// K-split of the product for nrhs rhs: number of partial products.
int dense_apply_splits(long n, int nrhs);

// out[r] = X in[r] for the rhs r < nrhs that `parent` marks active (all when
// null; the others' outputs are left as they were); `part` holds
// dense_apply_splits(n, nrhs) * nrhs * n complex entries.  The statistics of
// a coarse solve (one iteration per call) are recorded in `its`, `calls`,
// `tot` for the active rhs; *worked receives whether any rhs was active.  Any
// of these may be null.
void dense_apply(const DenseInverse& D, c64* out, const c64* in, c64* part, int nrhs, const int* parent, int* its,
                 int* calls, int* tot, hipStream_t st, int* worked = nullptr);

}  // namespace kdmg
