// Slice operator kernels for gfx950.
//
// Every application of M, M^T, M1, M1^T (paper, Sec. 1 Eq. MatrixM and Sec. 3
// Eq. MatrixM_1) and every change of spatial basis used by M0^{-1} is the same
// shape of work: for each right-hand side and output time slice t, take one
// source slice (t-1, t+1 or t), optionally scale it by a real field, apply a
// real Nx x Nx matrix along each of the three spatial axes (exp(-tau K) is
// separable: T (x) T (x) T), and combine the result with other slices of other
// vectors in an epilogue.
//
// One workgroup handles SPW slices of one right-hand side; each slice is
// Nx^2 threads. Data path per slice:
//   global -> registers : thread (y, x) loads its z-line (coalesced over x)
//   registers           : transform along z
//   LDS (rows padded to Nx+1 complex to spread banks)
//   LDS                 : threads (z, x) transform y-columns in place
//   LDS                 : threads (z, y) transform x-rows in place
//   LDS -> registers    : thread (y, x) reads its z-line back
//   epilogue            : coalesced loads of the identity / auxiliary terms,
//                         one coalesced store, optional fused dot products.
#include "ufg_internal.h"
#include "hop_stream.h"

namespace ufg {
namespace {

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

template <typename R, int NX, bool GENERAL>
__global__ void __launch_bounds__(HopShape<NX>::THREADS)
    hop_kernel(HopArgs<R> a, int ntau) {
  using S = HopShape<NX>;
  constexpr int P = S::P, V = S::V, SPW = S::SPW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* lds = reinterpret_cast<C2<R>*>(smem_raw);

  const int tgroups = (ntau + SPW - 1) / SPW;
  const int r = blockIdx.x / tgroups;
  const int tg = blockIdx.x - r * tgroups;
  if (a.gate && a.gate[r] == 0) return;  // uniform over the block

  const int sub = threadIdx.x / P;
  const int l = threadIdx.x - sub * P;
  const int t = tg * SPW + sub;
  const bool valid = t < ntau;
  int ts = t + a.shift;
  if (ts < 0) ts += ntau;
  if (ts >= ntau) ts -= ntau;
  const long long rbase = (long long)r * ntau * V;

  C2<R> v[NX], w[NX];
  if (valid) {
    const C2<R>* s = a.src + rbase + (long long)ts * V + l;
#pragma unroll
    for (int z = 0; z < NX; ++z) v[z] = s[z * P];
    if (a.pre) {
      const R* f = a.pre + (long long)ts * V + l;
#pragma unroll
      for (int z = 0; z < NX; ++z) {
        const R fz = f[z * P];
        v[z].x *= fz;
        v[z].y *= fz;
      }
    }
  } else {
#pragma unroll
    for (int z = 0; z < NX; ++z) v[z] = mk<R>(R(0), R(0));
  }

  slice_transform<R, NX>(a.mat, lds + sub * S::SL, l, v, w);

  R sgn = R(1);
  if (a.shift < 0) sgn = (ts == ntau - 1) ? R(1) : R(-1);
  if (a.shift > 0) sgn = (t == ntau - 1) ? R(1) : R(-1);

  double acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  if (valid) {
    const long long o = rbase + (long long)t * V + l;
    const R* post = a.post ? a.post + (long long)t * V + l : nullptr;
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      const long long idx = o + z * P;
      R f = sgn;
      if (post) f *= post[z * P];
      C2<R> base = mk<R>(f * w[z].x, f * w[z].y);
      if (a.id) {
        const C2<R> i0 = a.id[idx];
        base.x += i0.x;
        base.y += i0.y;
      }
      C2<R> out = base;
      if (GENERAL) {
        const R ar = R(a.alpha.x), ai = R(a.alpha.y);
        out = mk<R>(ar * base.x - ai * base.y, ar * base.y + ai * base.x);
        if (a.aux) {
          const C2<R> q = a.aux[idx];
          const R br = R(a.beta.x), bi = R(a.beta.y);
          out.x += br * q.x - bi * q.y;
          out.y += br * q.y + bi * q.x;
        }
      }
      a.dst[idx] = out;
      if (a.red_mode == 1) {  // <w, out> = sum conj(w) out
        const C2<R> q = a.red_w[idx];
        acc0 += double(q.x) * out.x + double(q.y) * out.y;
        acc1 += double(q.x) * out.y - double(q.y) * out.x;
      } else if (a.red_mode == 2) {  // <out, w> and <out, out>
        const C2<R> q = a.red_w[idx];
        acc0 += double(out.x) * q.x + double(out.y) * q.y;
        acc1 += double(out.x) * q.y - double(out.y) * q.x;
        acc2 += double(out.x) * out.x + double(out.y) * out.y;
      }
    }
  }
  if (a.red_mode) {
    double* scratch = reinterpret_cast<double*>(smem_raw);
    block_sum4(acc0, acc1, acc2, acc3, a.red_out + ((long long)r * tgroups + tg) * 4, scratch);
  }
}

// Force contraction (paper, Sec. 1): per site of slice t,
//   grad = -2 A cos sigma * s_t * sum_r Re[X_t conj((T^3 y_{t+1}))].
template <typename R, int NX>
__global__ void __launch_bounds__(HopShape<NX>::THREADS)
    force_kernel(const C2<R>* __restrict__ X, const C2<R>* __restrict__ y, const R* __restrict__ mat,
                 const double* __restrict__ sigma, double A, int ntau, int nrhs, double* grad) {
  using S = HopShape<NX>;
  constexpr int P = S::P, V = S::V, SPW = S::SPW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* lds = reinterpret_cast<C2<R>*>(smem_raw);
  const int sub = threadIdx.x / P;
  const int l = threadIdx.x - sub * P;
  const int t = blockIdx.x * SPW + sub;
  const bool valid = t < ntau;
  const int tp = (t + 1 >= ntau) ? t + 1 - ntau : t + 1;
  double acc[NX];
#pragma unroll
  for (int z = 0; z < NX; ++z) acc[z] = 0.0;
  C2<R> v[NX], w[NX];
  for (int r = 0; r < nrhs; ++r) {
    const long long rbase = (long long)r * ntau * V;
    if (valid) {
      const C2<R>* s = y + rbase + (long long)tp * V + l;
#pragma unroll
      for (int z = 0; z < NX; ++z) v[z] = s[z * P];
    } else {
#pragma unroll
      for (int z = 0; z < NX; ++z) v[z] = mk<R>(R(0), R(0));
    }
    slice_transform<R, NX>(mat, lds + sub * S::SL, l, v, w);
    if (valid) {
      const C2<R>* xs = X + rbase + (long long)t * V + l;
#pragma unroll
      for (int z = 0; z < NX; ++z) {
        const C2<R> q = xs[z * P];
        acc[z] += double(q.x) * w[z].x + double(q.y) * w[z].y;
      }
    }
    __syncthreads();  // LDS is reused by the next right-hand side
  }
  if (valid) {
    const double sgn = (t == ntau - 1) ? 1.0 : -1.0;
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      const long long i = (long long)t * V + z * P + l;
      grad[i] = -2.0 * A * cos(sigma[i]) * sgn * acc[z];
    }
  }
}

template <typename R, int NX>
int launch_hop_nx(const Lattice& L, const HopArgs<R>& args) {
  using S = HopShape<NX>;
  HopArgs<R> a = args;
  if (a.beta.x == 0.0 && a.beta.y == 0.0) a.aux = nullptr;  // never read an unused operand
  const int tgroups = (L.ntau + S::SPW - 1) / S::SPW;
  const size_t lds = size_t(S::SPW) * S::SL * sizeof(C2<R>);
  const bool general = (a.alpha.x != 1.0 || a.alpha.y != 0.0 || a.aux != nullptr);
  dim3 grid(tgroups * a.nrhs), block(S::THREADS);
  if (general) {
    static bool attr = false;
    if (!attr) {
      UFG_HIP(hipFuncSetAttribute((const void*)hop_kernel<R, NX, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      attr = true;
    }
    hipLaunchKernelGGL((hop_kernel<R, NX, true>), grid, block, lds, L.stream, a, L.ntau);
  } else {
    static bool attr = false;
    if (!attr) {
      UFG_HIP(hipFuncSetAttribute((const void*)hop_kernel<R, NX, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      attr = true;
    }
    hipLaunchKernelGGL((hop_kernel<R, NX, false>), grid, block, lds, L.stream, a, L.ntau);
  }
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R, int NX>
int launch_force_nx(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs, double* grad) {
  using S = HopShape<NX>;
  const int tgroups = (L.ntau + S::SPW - 1) / S::SPW;
  const size_t lds = size_t(S::SPW) * S::SL * sizeof(C2<R>);
  static bool attr = false;
  if (!attr) {
    UFG_HIP(hipFuncSetAttribute((const void*)force_kernel<R, NX>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  const Fields<R>& F = fields<R>(L);
  hipLaunchKernelGGL((force_kernel<R, NX>), dim3(tgroups), dim3(S::THREADS), lds, L.stream, X, y,
                     F.T, L.sigma, L.A, L.ntau, nrhs, grad);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

}  // namespace

#define UFG_NX_SWITCH(nx, CALL)          \
  switch (nx) {                          \
    case 2: return CALL(2);              \
    case 4: return CALL(4);              \
    case 6: return CALL(6);              \
    case 8: return CALL(8);              \
    case 10: return CALL(10);            \
    case 12: return CALL(12);            \
    case 14: return CALL(14);            \
    case 16: return CALL(16);            \
    default: set_error("unsupported nx"); return UFG_EINVAL; \
  }

template <typename R>
int launch_hop(const Lattice& L, const HopArgs<R>& a) {
  // M and M^T with the kinetic factor T go through the streaming kernel
  if (a.shift != 0 && a.mat == fields<R>(L).T && (a.id == nullptr || a.id == a.src) &&
      stream_supported(L))
    return launch_hop_stream<R>(L, a);
#define CALL_HOP(NX) launch_hop_nx<R, NX>(L, a)
  UFG_NX_SWITCH(L.nx, CALL_HOP)
#undef CALL_HOP
}

int hop_blocks_per_rhs(const Lattice& L) {
  if (stream_supported(L)) {
    const int slab = stream_slab(L);
    return (L.ntau + slab - 1) / slab;
  }
  int spw = 256 / (L.nx * L.nx);
  if (spw < 1) spw = 1;
  return (L.ntau + spw - 1) / spw;
}

template <typename R>
int launch_force(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs, double* grad) {
#define CALL_F(NX) launch_force_nx<R, NX>(L, X, y, nrhs, grad)
  UFG_NX_SWITCH(L.nx, CALL_F)
#undef CALL_F
}

template int launch_hop<float>(const Lattice&, const HopArgs<float>&);
template int launch_hop<double>(const Lattice&, const HopArgs<double>&);
template int launch_force<float>(const Lattice&, const float2*, const float2*, int, double*);
template int launch_force<double>(const Lattice&, const double2*, const double2*, int, double*);

}  // namespace ufg
