// Slice operator and force for lattices of spatial dimension 1 and 2 (the
// lower dimensions the paper's concluding section names as an extension).
//
// A slice has Nx (dimension 1) or Nx^2 (dimension 2) sites and exp(-tau K)
// is T or T (x) T with the same symmetric circulant T as in three dimensions.
// One thread per site of SPW = 256 / Nx^d slices of one right-hand side, and
// four such groups of slices per workgroup, whose loads each thread issues
// together. The scaled source slices and the matrix go to LDS, each thread
// forms its output along x as a row of T (read into registers once) times the
// slice row, and in dimension 2 the result goes through LDS once more for the
// y axis. The epilogue (identity, auxiliary term, complex scaling, fused dot
// products) is that of the general three-dimensional slice kernel, with the
// same operand conventions (HopArgs): shift -1 / +1 / 0 for M-type /
// M^T-type / basis changes, mat the Nx x Nx matrix applied along every axis.
#include "hop_common.h"

namespace ufg {
namespace {
using namespace hopc;

constexpr int kLowdThreads = 256;
// slices per thread of the operator kernel (its loads are issued together):
// four, two on 2D lattices of Nx <= 8, where a workgroup then still covers 8
// or more slices (measured on 8^2 x 8000, 16 rhs: complex128 apply_M 72.6 ->
// 59.8 us, apply_Mdag 54.6 -> 49.8 us, complex64 within 4 %; two on 2D
// Nx = 16 was 6-14 % slower). A function of the shape alone, so that the
// reduction's partial-sum count (lowd_blocks_per_rhs) follows it.
constexpr int lowd_slices(int nx, int d) { return (d == 2 && nx <= 8) ? 2 : 4; }

template <int NX, int D>
struct LowdShape {
  static constexpr int V = D == 1 ? NX : NX * NX;  // sites per slice
  static constexpr int SPW = kLowdThreads / V;     // slices per workgroup
};

// (T^d s)(l) for the slice s held in LDS (row-major [y][x]); tmp: a second
// LDS slice for the y stage. Every thread of the block calls it (barriers);
// `active` threads own a site.
template <typename R, int NX, int D>
__device__ __forceinline__ C2<R> lowd_transform(const R* __restrict__ mat, C2<R>* s, C2<R>* tmp,
                                                int l, bool active) {
  const int x = l % NX, row = l - x;
  C2<R> w = mk<R>(R(0), R(0));
  if (active) {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const R m = mat[x * NX + j];
      const C2<R> v = s[row + j];
      w.x = fma(m, v.x, w.x);
      w.y = fma(m, v.y, w.y);
    }
  }
  if constexpr (D == 2) {
    if (active) tmp[l] = w;
    __syncthreads();
    const int y = l / NX;
    w = mk<R>(R(0), R(0));
    if (active) {
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        const R m = mat[y * NX + j];
        const C2<R> v = tmp[j * NX + x];
        w.x = fma(m, v.x, w.x);
        w.y = fma(m, v.y, w.y);
      }
    }
  }
  return w;
}

template <typename R, int NX, int D, bool GENERAL>
__global__ void __launch_bounds__(kLowdThreads) hop_lowd_kernel(HopArgs<R> a, int ntau) {
  using S = LowdShape<NX, D>;
  constexpr int V = S::V, SPW = S::SPW, KS = lowd_slices(NX, D), W = SPW * V;
  __shared__ C2<R> src_lds[KS][W];
  __shared__ C2<R> tmp_lds[D == 2 ? KS : 1][D == 2 ? W : 1];
  __shared__ double red_lds[4 * (kLowdThreads / 64)];
  __shared__ R mat_lds[NX * NX];
  const int tgroups = (ntau + SPW * KS - 1) / (SPW * KS);
  const int r = blockIdx.x / tgroups;
  const int tg = blockIdx.x - r * tgroups;
  if (a.gate && a.gate[r] == 0) return;  // uniform over the block

  const int sub = threadIdx.x / V;
  const int l = threadIdx.x - sub * V;
  const bool active = sub < SPW;
  const int x = l % NX, y = l / NX, row = l - x;
  const long long rbase = (long long)r * ntau * V;
  // slice k of this workgroup: t = (tg KS + k) SPW + sub, so that for every k
  // the workgroup reads SPW consecutive slices (one contiguous block)
  C2<R> v[KS];
  int ts[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int t = (tg * KS + k) * SPW + sub;
    int q = t + a.shift;
    if (q < 0) q += ntau;
    if (q >= ntau) q -= ntau;
    ts[k] = q;
    v[k] = mk<R>(R(0), R(0));
    if (active && t < ntau) v[k] = a.src[rbase + (long long)q * V + l];
  }
  // the output field (M^T-type) is loaded with the sources (measured:
  // apply_Mdag 5-9 % faster than loading it in the epilogue)
  R postv[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int t = (tg * KS + k) * SPW + sub;
    postv[k] = (active && t < ntau && a.post) ? a.post[(long long)t * V + l] : R(1);
  }
  // so is the identity term, except for complex64 in dimension 1 (measured:
  // 4-13 % faster elsewhere, apply_Mdag complex128 1D 123 -> 107 us; 1D
  // complex64 apply_M 68 -> 72 us)
  constexpr bool kEarlyId = !(D == 1 && sizeof(R) == 4);
  C2<R> idv[kEarlyId ? KS : 1];
  if constexpr (kEarlyId) {
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int t = (tg * KS + k) * SPW + sub;
      idv[k] = (active && t < ntau && a.id) ? a.id[rbase + (long long)t * V + l]
                                            : mk<R>(R(0), R(0));
    }
  }
  if (a.pre) {
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int t = (tg * KS + k) * SPW + sub;
      if (active && t < ntau) {
        const R f = a.pre[(long long)ts[k] * V + l];
        v[k].x *= f;
        v[k].y *= f;
      }
    }
  }
  // the matrix goes through LDS, one coalesced load per thread (measured: the
  // operator 5-11 % faster than with each thread loading its rows itself)
  if (threadIdx.x < NX * NX) mat_lds[threadIdx.x] = a.mat[threadIdx.x];
  if (active) {
#pragma unroll
    for (int k = 0; k < KS; ++k) src_lds[k][sub * V + l] = v[k];
  }
  __syncthreads();
  R mrow[NX], mcol[D == 2 ? NX : 1];
#pragma unroll
  for (int j = 0; j < NX; ++j) mrow[j] = mat_lds[x * NX + j];
  if constexpr (D == 2) {
#pragma unroll
    for (int j = 0; j < NX; ++j) mcol[j] = mat_lds[y * NX + j];
  }
  // along x: a row of T times the slice row
  C2<R> w[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    w[k] = mk<R>(R(0), R(0));
    if (active) {
      const C2<R>* sl = &src_lds[k][sub * V + row];
#pragma unroll
      for (int j = 0; j < NX; ++j) {
        w[k].x = fma(mrow[j], sl[j].x, w[k].x);
        w[k].y = fma(mrow[j], sl[j].y, w[k].y);
      }
    }
  }
  if constexpr (D == 2) {  // along y
    if (active) {
#pragma unroll
      for (int k = 0; k < KS; ++k) tmp_lds[k][sub * V + l] = w[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      w[k] = mk<R>(R(0), R(0));
      if (active) {
        const C2<R>* sl = &tmp_lds[k][sub * V + x];
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          w[k].x = fma(mcol[j], sl[j * NX].x, w[k].x);
          w[k].y = fma(mcol[j], sl[j * NX].y, w[k].y);
        }
      }
    }
  }

  double acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int t = (tg * KS + k) * SPW + sub;
    if (!(active && t < ntau)) continue;
    R sgn = R(1);
    if (a.shift < 0) sgn = (ts[k] == ntau - 1) ? R(1) : R(-1);
    if (a.shift > 0) sgn = (t == ntau - 1) ? R(1) : R(-1);
    const long long idx = rbase + (long long)t * V + l;
    R f = sgn;
    if (a.post) f *= postv[k];
    C2<R> base = mk<R>(f * w[k].x, f * w[k].y);
    if (a.id) {
      C2<R> i0;
      if constexpr (kEarlyId)
        i0 = idv[k];
      else
        i0 = a.id[idx];
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
  if (a.red_mode)
    block_sum4(acc0, acc1, acc2, acc3, a.red_out + ((long long)r * tgroups + tg) * 4, red_lds);
}

// grad(n, t) = -2 A cos sigma(n, t) s_t sum_r Re[X_t(n) conj((T^d y_{t+1})(n))]
// (paper, Sec. 1), as the three-dimensional force kernel.
template <typename R, int NX, int D>
__global__ void __launch_bounds__(kLowdThreads)
    force_lowd_kernel(const C2<R>* __restrict__ X, const C2<R>* __restrict__ y,
                      const R* __restrict__ mat, const double* __restrict__ sigma, double A,
                      int ntau, int nrhs, double* grad) {
  using S = LowdShape<NX, D>;
  constexpr int V = S::V, SPW = S::SPW;
  __shared__ C2<R> src_lds[SPW * V];
  __shared__ C2<R> tmp_lds[D == 2 ? SPW * V : 1];
  const int sub = threadIdx.x / V;
  const int l = threadIdx.x - sub * V;
  const int t = blockIdx.x * SPW + sub;
  const bool active = sub < SPW;
  const bool valid = active && t < ntau;
  const int tp = (t + 1 >= ntau) ? t + 1 - ntau : t + 1;
  C2<R>* s = src_lds + (active ? sub : 0) * V;
  C2<R>* tmp = tmp_lds + (D == 2 && active ? sub * V : 0);
  double acc = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    const long long rbase = (long long)r * ntau * V;
    if (active) s[l] = valid ? y[rbase + (long long)tp * V + l] : mk<R>(R(0), R(0));
    __syncthreads();
    const C2<R> w = lowd_transform<R, NX, D>(mat, s, tmp, l, active);
    if (valid) {
      const C2<R> q = X[rbase + (long long)t * V + l];
      acc += double(q.x) * w.x + double(q.y) * w.y;
    }
    __syncthreads();  // LDS is reused by the next right-hand side
  }
  if (valid) {
    const double sgn = (t == ntau - 1) ? 1.0 : -1.0;
    const long long i = (long long)t * V + l;
    grad[i] = -2.0 * A * cos(sigma[i]) * sgn * acc;
  }
}

template <typename R, int NX, int D>
int launch_lowd(const Lattice& L, const HopArgs<R>& args) {
  using S = LowdShape<NX, D>;
  HopArgs<R> a = args;
  if (a.beta.x == 0.0 && a.beta.y == 0.0) a.aux = nullptr;  // never read an unused operand
  constexpr int per = S::SPW * lowd_slices(NX, D);  // slices per workgroup
  const int tgroups = (L.ntau + per - 1) / per;
  const bool general = (a.alpha.x != 1.0 || a.alpha.y != 0.0 || a.aux != nullptr);
  const dim3 grid(tgroups * a.nrhs), block(kLowdThreads);
  if (general)
    hipLaunchKernelGGL((hop_lowd_kernel<R, NX, D, true>), grid, block, 0, L.stream, a, L.ntau);
  else
    hipLaunchKernelGGL((hop_lowd_kernel<R, NX, D, false>), grid, block, 0, L.stream, a, L.ntau);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R, int NX, int D>
int launch_force_lowd_nx(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs,
                         double* grad) {
  using S = LowdShape<NX, D>;
  const int tgroups = (L.ntau + S::SPW - 1) / S::SPW;
  const Fields<R>& F = fields<R>(L);
  hipLaunchKernelGGL((force_lowd_kernel<R, NX, D>), dim3(tgroups), dim3(kLowdThreads), 0,
                     L.stream, X, y, F.T, L.sigma, L.A, L.ntau, nrhs, grad);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

}  // namespace

#define UFG_LOWD_SWITCH(CALL)                                        \
  switch (L.nx) {                                                    \
    case 2: return L.dim == 1 ? CALL(2, 1) : CALL(2, 2);             \
    case 4: return L.dim == 1 ? CALL(4, 1) : CALL(4, 2);             \
    case 6: return L.dim == 1 ? CALL(6, 1) : CALL(6, 2);             \
    case 8: return L.dim == 1 ? CALL(8, 1) : CALL(8, 2);             \
    case 10: return L.dim == 1 ? CALL(10, 1) : CALL(10, 2);          \
    case 12: return L.dim == 1 ? CALL(12, 1) : CALL(12, 2);          \
    case 14: return L.dim == 1 ? CALL(14, 1) : CALL(14, 2);          \
    case 16: return L.dim == 1 ? CALL(16, 1) : CALL(16, 2);          \
    default: set_error("unsupported nx"); return UFG_EINVAL;         \
  }

template <typename R>
int launch_hop_lowd(const Lattice& L, const HopArgs<R>& a) {
  if (L.dim != 1 && L.dim != 2) {
    set_error("slice kernel: lattice dimension must be 1 or 2 here");
    return UFG_EINVAL;
  }
#define CALL_LOWD(NX, D) launch_lowd<R, NX, D>(L, a)
  UFG_LOWD_SWITCH(CALL_LOWD)
#undef CALL_LOWD
}

int lowd_blocks_per_rhs(const Lattice& L) {
  const int v = L.dim == 1 ? L.nx : L.nx * L.nx;
  const int per = (kLowdThreads / v) * lowd_slices(L.nx, L.dim);  // slices per workgroup
  return (L.ntau + per - 1) / per;
}

template <typename R>
int launch_force_lowd(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs, double* grad) {
  if (L.dim != 1 && L.dim != 2) {
    set_error("force kernel: lattice dimension must be 1 or 2 here");
    return UFG_EINVAL;
  }
#define CALL_FL(NX, D) launch_force_lowd_nx<R, NX, D>(L, X, y, nrhs, grad)
  UFG_LOWD_SWITCH(CALL_FL)
#undef CALL_FL
}

template int launch_hop_lowd<float>(const Lattice&, const HopArgs<float>&);
template int launch_hop_lowd<double>(const Lattice&, const HopArgs<double>&);
template int launch_force_lowd<float>(const Lattice&, const float2*, const float2*, int, double*);
template int launch_force_lowd<double>(const Lattice&, const double2*, const double2*, int,
                                       double*);

}  // namespace ufg
