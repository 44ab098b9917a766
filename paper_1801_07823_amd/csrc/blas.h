// Level-1 vector kernels with device-resident scalars.
//
// Every vector holds `nrhs` right-hand sides back to back ([rhs][n] complex).
// Scalars (dot products, Krylov coefficients, convergence flags) live in device
// memory, one slot per rhs, so a Krylov iteration never waits for the host.
// Reductions are deterministic: fixed grid, fixed tree order, and a second
// kernel adds the per-block partials in block order (no atomics).
#pragma once
#include "common.h"

namespace kdmg {

constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 240;

// Per-stream scratch for reductions.
struct RedScratch {
  double* partials = nullptr;  // [slots][K][RED_MAX_BLOCKS]
  int slots = 0;
};

inline int red_blocks(long n) {
  long b = (n + RED_THREADS * 4 - 1) / (RED_THREADS * 4);
  if (b < 1) b = 1;
  if (b > RED_MAX_BLOCKS) b = RED_MAX_BLOCKS;
  return (int)b;
}

template <int K>
struct Acc {
  double v[K];
};

// Wave64 + LDS tree reduction of K doubles; result valid in thread 0.
template <int K>
__device__ __forceinline__ void block_reduce(Acc<K>& a) {
  __shared__ double sh[K][RED_THREADS / 64];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = a.v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    a.v[k] = v;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][wid] = a.v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < RED_THREADS / 64; ++w) s += sh[k][w];
      a.v[k] = s;
    }
  }
}

// Generic map + reduce.  Op provides
//   __device__ bool active(int r) const;
//   __device__ void elem(int r, int z, long i, Acc<K>& a) const;   (may also write)
//   __device__ void finish(int r, int z, const double* sums) const; (one thread)
// Two kernels: k_map_reduce (grid x = blocks over i, y = rhs, z = batch index,
// e.g. which basis vector) writes one partial sum per workgroup;
// k_reduce_finish adds each (rhs, z) slot's partials in workgroup order with a
// fixed lane tree and calls finish.  No atomics and no device-scope fences
// (on this part a fence writes back L2, and one per workgroup made the
// reductions several times slower than their memory traffic).
template <int K, class Op>
__global__ __launch_bounds__(RED_THREADS) void k_map_reduce(Op op, long n, int nrhs, double* partials) {
  const int r = blockIdx.y, z = blockIdx.z;
  if (!op.active(r)) return;
  Acc<K> a;
#pragma unroll
  for (int k = 0; k < K; ++k) a.v[k] = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    op.elem(r, z, i, a);
  block_reduce<K>(a);
  if (threadIdx.x == 0) {
    double* pp = partials + (size_t)(z * nrhs + r) * K * RED_MAX_BLOCKS;
#pragma unroll
    for (int k = 0; k < K; ++k) pp[k * RED_MAX_BLOCKS + blockIdx.x] = a.v[k];
  }
}

template <int K, class Op>
__global__ __launch_bounds__(64) void k_reduce_finish(Op op, int nb, int nrhs, const double* partials) {
  const int r = blockIdx.x, z = blockIdx.y, lane = threadIdx.x;
  if (!op.active(r)) return;
  const double* pp = partials + (size_t)(z * nrhs + r) * K * RED_MAX_BLOCKS;
  double s[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = 0.0;
    for (int b = lane; b < nb; b += 64) v += pp[k * RED_MAX_BLOCKS + b];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    s[k] = v;
  }
  if (lane == 0) op.finish(r, z, s);
}

template <int K, class Op>
void launch_map_reduce(const Op& op, long n, int nrhs, int nz, const RedScratch& rs,
                       hipStream_t st) {
  KDMG_CHECK(nz * nrhs <= rs.slots, KDMG_EINVAL, "reduction scratch too small");
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_map_reduce<K, Op>), dim3(nb, nrhs, nz), dim3(RED_THREADS), 0, st, op, n, nrhs,
                     rs.partials);
  hipLaunchKernelGGL((k_reduce_finish<K, Op>), dim3(nrhs, nz), dim3(64), 0, st, op, nb, nrhs,
                     (const double*)rs.partials);
  KDMG_LAUNCH_CHECK();
}

// Generic elementwise map: Op provides active(r) and elem(r, i).
template <class Op>
__global__ __launch_bounds__(256) void k_map(Op op, long n) {
  const int r = blockIdx.y;
  if (!op.active(r)) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    op.elem(r, i);
}

template <class Op>
void launch_map(const Op& op, long n, int nrhs, hipStream_t st) {
  long b = (n + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  hipLaunchKernelGGL((k_map<Op>), dim3((unsigned)b, nrhs), dim3(256), 0, st, op, n);
  KDMG_LAUNCH_CHECK();
}

__device__ __forceinline__ bool is_active(const int* act, int r) { return !act || act[r] != 0; }

// ------------------------------------------------------------- elementwise ops

// y = x (with precision conversion)
template <class TO, class TI>
struct OpCopy {
  Cx<TO>* y; const Cx<TI>* x; long n; const int* act;
  __device__ bool active(int r) const { return is_active(act, r); }
  __device__ void elem(int r, long i) const { y[r * n + i] = st<TO>(ld<double>(x[r * n + i])); }
};

template <class T>
struct OpZero {
  Cx<T>* y; long n; const int* act;
  __device__ bool active(int r) const { return is_active(act, r); }
  __device__ void elem(int r, long i) const { y[r * n + i] = Cx<T>{0, 0}; }
};

// y += s[r] * x   (s complex, from device, optionally negated)
template <class T>
struct OpAxpyDev {
  Cx<T>* y; const Cx<T>* x; long n; const double* s; int sstride; double sign; const int* act;
  __device__ bool active(int r) const { return is_active(act, r); }
  __device__ void elem(int r, long i) const {
    Cx<T> a{(T)(sign * s[r * sstride]), (T)(sign * s[r * sstride + 1])};
    cfma(y[r * n + i], a, x[r * n + i]);
  }
};

// ------------------------------------------------------------- reductions

// sums = (Re, Im) of <x, y> = sum conj(x) y ; stores to out[r*2 + 0/1]
template <class T>
struct OpDot {
  const Cx<T>* x; const Cx<T>* y; long n; double* out; const int* act;
  __device__ bool active(int r) const { return is_active(act, r); }
  __device__ void elem(int r, int, long i, Acc<2>& a) const {
    Cx<double> u = ld<double>(x[r * n + i]), v = ld<double>(y[r * n + i]);
    a.v[0] += u.re * v.re + u.im * v.im;
    a.v[1] += u.re * v.im - u.im * v.re;
  }
  __device__ void finish(int r, int, const double* s) const { out[2 * r] = s[0]; out[2 * r + 1] = s[1]; }
};

template <class T>
struct OpNorm2 {
  const Cx<T>* x; long n; double* out; const int* act;
  __device__ bool active(int r) const { return is_active(act, r); }
  __device__ void elem(int r, int, long i, Acc<1>& a) const { a.v[0] += (double)norm2(ld<double>(x[r * n + i])); }
  __device__ void finish(int r, int, const double* s) const { out[r] = s[0]; }
};

}  // namespace kdmg
