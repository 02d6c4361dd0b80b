// Per-slice building blocks shared by the slice-operator kernels: a real
// Nx x Nx matrix applied along each axis of a slice (z in registers, y and x
// through LDS with rows padded to Nx+1 complex).
#pragma once

#include "ufg_internal.h"

namespace ufg {
namespace hopc {

template <typename R>
__device__ __forceinline__ C2<R> mk(R a, R b) {
  C2<R> c;
  c.x = a;
  c.y = b;
  return c;
}

// out_i = sum_j mat[i][j] * in_j for one line of NX complex values.
template <typename R, int NX>
__device__ __forceinline__ void line_transform(const R* __restrict__ mat, const C2<R> (&in)[NX],
                                               C2<R> (&out)[NX]) {
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    R re = R(0), im = R(0);
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const R m = mat[i * NX + j];
      re = fma(m, in[j].x, re);
      im = fma(m, in[j].y, im);
    }
    out[i] = mk<R>(re, im);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum 4 per-thread doubles over the workgroup; thread 0 writes them to out.
__device__ void block_sum4(double a0, double a1, double a2, double a3, double* out, double* scratch) {
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  a3 = wave_sum(a3);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();  // scratch may alias LDS used before
  if (lane == 0) {
    scratch[wid * 4 + 0] = a0;
    scratch[wid * 4 + 1] = a1;
    scratch[wid * 4 + 2] = a2;
    scratch[wid * 4 + 3] = a3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int w = 0; w < nw; ++w) {
      s0 += scratch[w * 4 + 0];
      s1 += scratch[w * 4 + 1];
      s2 += scratch[w * 4 + 2];
      s3 += scratch[w * 4 + 3];
    }
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
    out[3] = s3;
  }
}

template <int NX>
struct HopShape {
  static constexpr int P = NX * NX;                 // threads per slice
  static constexpr int V = NX * NX * NX;            // sites per slice
  static constexpr int LD = NX + 1;                 // padded LDS row
  static constexpr int SL = NX * NX * (NX + 1);     // LDS complex per slice
  static constexpr int SPW = (256 / P) > 0 ? 256 / P : 1;
  static constexpr int THREADS = P * SPW;
};

// Apply mat^{(x)3} to the slice held as z-lines in v (thread (y,x) of its slice),
// leaving the result as z-lines in w. `my` is this slice's LDS region.
template <typename R, int NX>
__device__ __forceinline__ void slice_transform(const R* __restrict__ mat, C2<R>* my, int l,
                                                C2<R> (&v)[NX], C2<R> (&w)[NX]) {
  using S = HopShape<NX>;
  constexpr int LD = S::LD;
  const int y = l / NX, x = l - (l / NX) * NX;
  line_transform<R, NX>(mat, v, w);  // along z
#pragma unroll
  for (int z = 0; z < NX; ++z) my[(z * NX + y) * LD + x] = w[z];
  __syncthreads();
  {  // along y: thread (z, x)
    const int z = l / NX, xx = l - (l / NX) * NX;
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) v[yy] = my[(z * NX + yy) * LD + xx];
    line_transform<R, NX>(mat, v, w);
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) my[(z * NX + yy) * LD + xx] = w[yy];
  }
  __syncthreads();
  {  // along x: thread (z, y)
    const int z = l / NX, yy = l - (l / NX) * NX;
    C2<R>* row = my + (z * NX + yy) * LD;
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) v[xx] = row[xx];
    line_transform<R, NX>(mat, v, w);
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) row[xx] = w[xx];
  }
  __syncthreads();
#pragma unroll
  for (int z = 0; z < NX; ++z) w[z] = my[(z * NX + y) * LD + x];
}


}  // namespace hopc
}  // namespace ufg
