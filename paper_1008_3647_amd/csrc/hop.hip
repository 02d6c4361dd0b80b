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
#include "hop_common.h"
#include "hop_stream.h"

namespace ufg {
namespace {
using namespace hopc;

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
      } else if (a.red_mode == 2) {  // <out, w>, <out, out>, <w, w>
        const C2<R> q = a.red_w[idx];
        acc0 += double(out.x) * q.x + double(out.y) * q.y;
        acc1 += double(out.x) * q.y - double(out.y) * q.x;
        acc2 += double(out.x) * out.x + double(out.y) * out.y;
        acc3 += double(q.x) * q.x + double(q.y) * q.y;
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
  if (L.dim < 3) return launch_hop_lowd<R>(L, a);
  // M and M^T with the kinetic factor T go through the streaming kernel
  if (a.shift != 0 && a.mat == fields<R>(L).T && (a.id == nullptr || a.id == a.src) &&
      stream_supported(L))
    return launch_hop_stream<R>(L, a);
  // basis changes of the eigenbasis: the mode-space vectors are in the block
  // order of the streaming basis kernel whenever it exists for this nx
  if (a.shift == 0 && !L.mode_perm.empty() &&
      (a.mat == fields<R>(L).U || a.mat == fields<R>(L).Ut))
    return launch_basis_stream<R>(L, a, a.mat == fields<R>(L).Ut);
#define CALL_HOP(NX) launch_hop_nx<R, NX>(L, a)
  UFG_NX_SWITCH(L.nx, CALL_HOP)
#undef CALL_HOP
}

int hop_blocks_per_rhs(const Lattice& L) {
  if (L.dim < 3) return lowd_blocks_per_rhs(L);
  if (stream_supported(L)) return stream_nslab(L);
  int spw = 256 / (L.nx * L.nx);
  if (spw < 1) spw = 1;
  return (L.ntau + spw - 1) / spw;
}

template <typename R>
int launch_force(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs, double* grad) {
  if (L.dim < 3) return launch_force_lowd<R>(L, X, y, nrhs, grad);
#define CALL_F(NX) launch_force_nx<R, NX>(L, X, y, nrhs, grad)
  UFG_NX_SWITCH(L.nx, CALL_F)
#undef CALL_F
}

template int launch_hop<float>(const Lattice&, const HopArgs<float>&);
template int launch_hop<double>(const Lattice&, const HopArgs<double>&);
template int launch_force<float>(const Lattice&, const float2*, const float2*, int, double*);
template int launch_force<double>(const Lattice&, const double2*, const double2*, int, double*);

}  // namespace ufg
