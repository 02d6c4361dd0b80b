// Streaming slice operator for M and M^T (paper, Sec. 1, Eq. MatrixM) on gfx950.
//
// One workgroup owns a slab of S consecutive time slices of one right-hand
// side and walks it in the direction of the time shift, so every input slice
// is loaded from HBM once: the slice x_t loaded for the identity term of y_t
// is the slice whose transform feeds y_{t+1} (M) or y_{t-1} (M^T); only one
// halo slice per slab is loaded twice, and it is usually an L2 hit.
//
// Workgroups are numbered so that each XCD receives a contiguous run of
// (slab, rhs) pairs with the rhs index fastest: the eight right-hand sides of
// a slab run together on one XCD and share the field slab and the halo slices
// through that XCD's L2.
//
// exp(-tau K) along one axis is the symmetric circulant T. T commutes with the
// reflections i -> -i and i -> Nx/2 - i (mod Nx), so in the basis of their
// joint eigenvectors (built by two levels of add/subtract butterflies) T is
// block diagonal with blocks of sizes Nx/4+1, Nx/4, Nx/4, Nx/4-1. A line of Nx
// values then costs 4 (Nx-2) additions for the butterflies and sum(block^2)
// multiply-adds (56 + 66 for Nx = 16) instead of Nx^2 = 256 multiply-adds.
//
// Fused BiCGStab sources: the kernel can build its source on the fly from the
// Krylov vectors (p = r + beta (p_old - omega v_old), or s = r - alpha v) so
// that BiCGStab's vector updates ride on the operator's memory stream.
#include "hop_stream.h"
#include "krylov.h"

namespace ufg {
namespace {

template <typename R>
__device__ __forceinline__ C2<R> add(C2<R> a, C2<R> b) {
  C2<R> c;
  c.x = a.x + b.x;
  c.y = a.y + b.y;
  return c;
}
template <typename R>
__device__ __forceinline__ C2<R> sub(C2<R> a, C2<R> b) {
  C2<R> c;
  c.x = a.x - b.x;
  c.y = a.y - b.y;
  return c;
}
template <typename R>
__device__ __forceinline__ C2<R> zero2() {
  C2<R> c;
  c.x = R(0);
  c.y = R(0);
  return c;
}

// y = T a for one line held in registers (in place), through the butterflies.
template <typename R, int NX>
__device__ __forceinline__ void split_line(const SplitCoef<R, NX>& c, C2<R> (&a)[NX]) {
  constexpr int H = NX / 2, Q = NX / 4;
  C2<R> E[H + 1], O[H + 1];
  E[0] = a[0];
  E[H] = a[H];
#pragma unroll
  for (int j = 1; j < H; ++j) {
    E[j] = add<R>(a[j], a[NX - j]);
    O[j] = sub<R>(a[j], a[NX - j]);
  }
  C2<R> es[Q + 1], ea[Q + 1], os[Q + 1], oa[Q + 1];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    es[j] = add<R>(E[j], E[H - j]);
    ea[j] = sub<R>(E[j], E[H - j]);
  }
  es[Q] = E[Q];
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    os[j] = add<R>(O[j], O[H - j]);
    oa[j] = sub<R>(O[j], O[H - j]);
  }
  os[Q] = O[Q];
  C2<R> es2[Q + 1], ea2[Q + 1], os2[Q + 1], oa2[Q + 1];
#pragma unroll
  for (int i = 0; i <= Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 0; k <= Q; ++k) {
      const R m = c.es[i * (Q + 1) + k];
      s.x = fma(m, es[k].x, s.x);
      s.y = fma(m, es[k].y, s.y);
    }
    es2[i] = s;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const R m = c.ea[i * Q + k];
      s.x = fma(m, ea[k].x, s.x);
      s.y = fma(m, ea[k].y, s.y);
    }
    ea2[i] = s;
  }
#pragma unroll
  for (int i = 1; i <= Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 1; k <= Q; ++k) {
      const R m = c.os[(i - 1) * Q + (k - 1)];
      s.x = fma(m, os[k].x, s.x);
      s.y = fma(m, os[k].y, s.y);
    }
    os2[i] = s;
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const R m = c.oa[(i - 1) * (Q - 1) + (k - 1)];
      s.x = fma(m, oa[k].x, s.x);
      s.y = fma(m, oa[k].y, s.y);
    }
    oa2[i] = s;
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    E[j] = add<R>(es2[j], ea2[j]);
    E[H - j] = sub<R>(es2[j], ea2[j]);
  }
  E[Q] = es2[Q];
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    O[j] = add<R>(os2[j], oa2[j]);
    O[H - j] = sub<R>(os2[j], oa2[j]);
  }
  O[Q] = os2[Q];
  a[0] = E[0];
  a[H] = E[H];
#pragma unroll
  for (int j = 1; j < H; ++j) {
    a[j] = add<R>(E[j], O[j]);
    a[NX - j] = sub<R>(E[j], O[j]);
  }
}

// T^3 of the slice held as z-lines in v (thread (y, x)); result left in v.
template <typename R, int NX>
__device__ __forceinline__ void slice_T3(const SplitCoef<R, NX>& c, C2<R>* lds, int l,
                                         C2<R> (&v)[NX]) {
  constexpr int LD = NX + 1;
  const int y = l / NX, x = l - (l / NX) * NX;
  split_line<R, NX>(c, v);  // along z
  __syncthreads();          // the previous slice's readers are done with lds
#pragma unroll
  for (int z = 0; z < NX; ++z) lds[(z * NX + y) * LD + x] = v[z];
  __syncthreads();
  C2<R> w[NX];
  {
    const int z = l / NX, xx = l - (l / NX) * NX;
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) w[yy] = lds[(z * NX + yy) * LD + xx];
    split_line<R, NX>(c, w);  // along y
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) lds[(z * NX + yy) * LD + xx] = w[yy];
  }
  __syncthreads();
  {
    const int z = l / NX, yy = l - (l / NX) * NX;
    C2<R>* row = lds + (z * NX + yy) * LD;
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) w[xx] = row[xx];
    split_line<R, NX>(c, w);  // along x
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) row[xx] = w[xx];
  }
  __syncthreads();
#pragma unroll
  for (int z = 0; z < NX; ++z) v[z] = lds[(z * NX + y) * LD + x];
}

// Per-rhs scalars of the fused BiCGStab sources.
template <typename R>
struct SrcScal {
  R br, bi, wr, wi, ar, ai;
};

template <typename R, int SRC>
__device__ __forceinline__ SrcScal<R> src_scalars(const HopArgs<R>& a, int r) {
  SrcScal<R> q{};
  if (SRC == 0) return q;
  const RhsState s = reinterpret_cast<const RhsState*>(a.st)[r];
  if (SRC == 1) {
    // beta = (rho / rho_old)(alpha / omega)
    const double d1 = s.rho_old.x * s.rho_old.x + s.rho_old.y * s.rho_old.y;
    const double q1x = (s.rho.x * s.rho_old.x + s.rho.y * s.rho_old.y) / d1;
    const double q1y = (s.rho.y * s.rho_old.x - s.rho.x * s.rho_old.y) / d1;
    const double d2 = s.omega.x * s.omega.x + s.omega.y * s.omega.y;
    const double q2x = (s.alpha.x * s.omega.x + s.alpha.y * s.omega.y) / d2;
    const double q2y = (s.alpha.y * s.omega.x - s.alpha.x * s.omega.y) / d2;
    q.br = R(q1x * q2x - q1y * q2y);
    q.bi = R(q1x * q2y + q1y * q2x);
    q.wr = R(s.omega.x);
    q.wi = R(s.omega.y);
  } else {
    q.ar = R(s.alpha.x);
    q.ai = R(s.alpha.y);
  }
  return q;
}

// z-line of the source vector at element offset o (already includes rhs, slice, lane).
template <typename R, int NX, int SRC>
__device__ __forceinline__ void load_source(const HopArgs<R>& a, const SrcScal<R>& q, long long o,
                                            C2<R> (&X)[NX]) {
  constexpr int P = NX * NX;
#pragma unroll
  for (int z = 0; z < NX; ++z) {
    const long long i = o + z * P;
    if (SRC == 0) {
      X[z] = a.src[i];
    } else if (SRC == 1) {
      const C2<R> rv = a.fr[i], pv = a.fp[i], vv = a.fv[i];
      const R dx = pv.x - (q.wr * vv.x - q.wi * vv.y);
      const R dy = pv.y - (q.wr * vv.y + q.wi * vv.x);
      X[z].x = rv.x + q.br * dx - q.bi * dy;
      X[z].y = rv.y + q.br * dy + q.bi * dx;
    } else {
      const C2<R> rv = a.fr[i], vv = a.fv[i];
      X[z].x = rv.x - (q.ar * vv.x - q.ai * vv.y);
      X[z].y = rv.y - (q.ar * vv.y + q.ai * vv.x);
    }
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// DIR = -1: M-type (output t reads source t-1, walk t upwards)
// DIR = +1: M^T-type (output t reads source t+1, walk t upwards with lookahead)
template <typename R, int NX, int DIR, bool GENERAL, int SRC>
__global__ void __launch_bounds__(NX * NX)
    hop_stream_kernel(HopArgs<R> a, SplitCoef<R, NX> c, int ntau, int slab, int nslab) {
  constexpr int P = NX * NX, V = NX * NX * NX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* lds = reinterpret_cast<C2<R>*>(smem_raw);

  // XCD-aware numbering: contiguous logical ids per XCD, rhs fastest
  const int nb = gridDim.x;
  const int full = nb & ~7;
  int lid = blockIdx.x;
  if (lid < full) lid = (lid & 7) * (full >> 3) + (lid >> 3);
  const int r = lid % a.nrhs;
  const int sb = lid / a.nrhs;
  if (a.gate && a.gate[r] == 0) return;

  const int l = threadIdx.x;
  const int t0 = sb * slab;
  const int t1 = min(t0 + slab, ntau);  // exclusive
  const long long rbase = (long long)r * ntau * V;
  const SrcScal<R> q = src_scalars<R, SRC>(a, r);

  double acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  const int count = t1 - t0;
  // Both directions walk t upwards (ascending addresses stream best).
  //   M  : W holds T^3(b_{t-1} x_{t-1}); X = x_t is loaded, used as the
  //        identity term, then becomes the next W.
  //   M^T: X = x_t was loaded one step earlier; Xn = x_{t+1} is loaded and its
  //        transform W = T^3 x_{t+1} combines with X into y_t; Xn becomes X.
  C2<R> W[NX], X[NX];
  if (DIR < 0) {
    const int th = (t0 == 0) ? ntau - 1 : t0 - 1;
    load_source<R, NX, SRC>(a, q, rbase + (long long)th * V + l, W);
    if (a.pre) {
      const R* f = a.pre + (long long)th * V + l;
#pragma unroll
      for (int z = 0; z < NX; ++z) {
        const R fz = f[z * P];
        W[z].x *= fz;
        W[z].y *= fz;
      }
    }
    slice_T3<R, NX>(c, lds, l, W);
  } else {
    const long long o = rbase + (long long)t0 * V + l;
    load_source<R, NX, SRC>(a, q, o, X);
    if (SRC == 1) {
#pragma unroll
      for (int z = 0; z < NX; ++z) a.fpnew[o + z * P] = X[z];
    }
  }
  for (int k = 0; k < count; ++k) {
    const int t = t0 + k;
    const long long o = rbase + (long long)t * V + l;
    C2<R> Xn[NX];
    if (DIR < 0) {
      load_source<R, NX, SRC>(a, q, o, X);
      if (SRC == 1) {
#pragma unroll
        for (int z = 0; z < NX; ++z) a.fpnew[o + z * P] = X[z];
      }
    } else {
      const int tn = (t + 1 == ntau) ? 0 : t + 1;
      const long long on = rbase + (long long)tn * V + l;
      load_source<R, NX, SRC>(a, q, on, Xn);
      if (SRC == 1 && k + 1 < count) {  // x_{t+1} belongs to this slab
#pragma unroll
        for (int z = 0; z < NX; ++z) a.fpnew[on + z * P] = Xn[z];
      }
#pragma unroll
      for (int z = 0; z < NX; ++z) W[z] = Xn[z];
      slice_T3<R, NX>(c, lds, l, W);
    }
    // sign of the block that connects the source slice to slice t
    R sgn;
    if (DIR < 0)
      sgn = (t == 0) ? R(1) : R(-1);
    else
      sgn = (t == ntau - 1) ? R(1) : R(-1);
    const R* post = a.post ? a.post + (long long)t * V + l : nullptr;
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      const long long idx = o + z * P;
      const C2<R> id = X[z];
      R f = sgn;
      if (post) f *= post[z * P];
      C2<R> base;
      base.x = f * W[z].x;
      base.y = f * W[z].y;
      if (a.id) {
        base.x += id.x;
        base.y += id.y;
      }
      C2<R> out = base;
      if (GENERAL) {
        const R ar = R(a.alpha.x), ai = R(a.alpha.y);
        out.x = ar * base.x - ai * base.y;
        out.y = ar * base.y + ai * base.x;
        if (a.aux) {
          const C2<R> u = a.aux[idx];
          const R br = R(a.beta.x), bi = R(a.beta.y);
          out.x += br * u.x - bi * u.y;
          out.y += br * u.y + bi * u.x;
        }
      }
      // streaming store: y is not re-read by this launch, keep L2 for the
      // halo slices and the field
      __builtin_nontemporal_store(out.x, &a.dst[idx].x);
      __builtin_nontemporal_store(out.y, &a.dst[idx].y);
      if (a.red_mode == 1) {
        const C2<R> u = a.red_w[idx];
        acc0 += double(u.x) * out.x + double(u.y) * out.y;
        acc1 += double(u.x) * out.y - double(u.y) * out.x;
      } else if (a.red_mode == 2) {
        const C2<R> u = a.red_w[idx];
        acc0 += double(out.x) * u.x + double(out.y) * u.y;
        acc1 += double(out.x) * u.y - double(out.y) * u.x;
        acc2 += double(out.x) * out.x + double(out.y) * out.y;
        acc3 += double(u.x) * u.x + double(u.y) * u.y;
      } else if (a.red_mode == 3) {  // <out, source>, |out|^2, |source|^2
        acc0 += double(out.x) * id.x + double(out.y) * id.y;
        acc1 += double(out.x) * id.y - double(out.y) * id.x;
        acc2 += double(out.x) * out.x + double(out.y) * out.y;
        acc3 += double(id.x) * id.x + double(id.y) * id.y;
      }
    }
    if (DIR > 0) {
#pragma unroll
      for (int z = 0; z < NX; ++z) X[z] = Xn[z];
    }
    if (DIR < 0 && k + 1 < count) {
      // transform slice t for the next output slice
      if (a.pre) {
        const R* f = a.pre + (long long)t * V + l;
#pragma unroll
        for (int z = 0; z < NX; ++z) {
          const R fz = f[z * P];
          X[z].x *= fz;
          X[z].y *= fz;
        }
      }
#pragma unroll
      for (int z = 0; z < NX; ++z) W[z] = X[z];
      slice_T3<R, NX>(c, lds, l, W);
    }
  }
  if (a.red_mode) {
    acc0 = wsum(acc0);
    acc1 = wsum(acc1);
    acc2 = wsum(acc2);
    acc3 = wsum(acc3);
    __syncthreads();
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      sm[wid * 4 + 0] = acc0;
      sm[wid * 4 + 1] = acc1;
      sm[wid * 4 + 2] = acc2;
      sm[wid * 4 + 3] = acc3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
      for (int w = 0; w < (P + 63) / 64; ++w) {
        s0 += sm[w * 4 + 0];
        s1 += sm[w * 4 + 1];
        s2 += sm[w * 4 + 2];
        s3 += sm[w * 4 + 3];
      }
      double* out = a.red_out + ((long long)r * nslab + sb) * 4;
      out[0] = s0;
      out[1] = s1;
      out[2] = s2;
      out[3] = s3;
    }
  }
}

template <typename R, int NX, int DIR, bool GENERAL, int SRC>
int launch_one(const Lattice& L, const HopArgs<R>& a, const SplitCoef<R, NX>& c, dim3 grid,
               size_t lds, int slab, int nslab) {
  static bool attr = false;
  if (!attr) {
    UFG_HIP(hipFuncSetAttribute((const void*)hop_stream_kernel<R, NX, DIR, GENERAL, SRC>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((hop_stream_kernel<R, NX, DIR, GENERAL, SRC>), grid, dim3(NX * NX), lds,
                     L.stream, a, c, L.ntau, slab, nslab);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R, int NX, int DIR>
int launch_dir(const Lattice& L, const HopArgs<R>& a, const SplitCoef<R, NX>& c) {
  const int slab = stream_slab(L);
  const int nslab = (L.ntau + slab - 1) / slab;
  const size_t lds = size_t(NX) * NX * (NX + 1) * sizeof(C2<R>);
  const bool general = (a.alpha.x != 1.0 || a.alpha.y != 0.0 || a.aux != nullptr);
  const dim3 grid(nslab * a.nrhs);
  if (a.src_mode == 1) return launch_one<R, NX, DIR, false, 1>(L, a, c, grid, lds, slab, nslab);
  if (a.src_mode == 2) return launch_one<R, NX, DIR, false, 2>(L, a, c, grid, lds, slab, nslab);
  if (general) return launch_one<R, NX, DIR, true, 0>(L, a, c, grid, lds, slab, nslab);
  return launch_one<R, NX, DIR, false, 0>(L, a, c, grid, lds, slab, nslab);
}

template <typename R, int NX>
int launch_nx(const Lattice& L, const HopArgs<R>& a) {
  SplitCoef<R, NX> c;
  const std::vector<double>& h = L.split_host;
  int k = 0;
  for (auto& v : c.es) v = R(h[k++]);
  for (auto& v : c.ea) v = R(h[k++]);
  for (auto& v : c.os) v = R(h[k++]);
  for (auto& v : c.oa) v = R(h[k++]);
  if (a.shift < 0) return launch_dir<R, NX, -1>(L, a, c);
  return launch_dir<R, NX, +1>(L, a, c);
}

}  // namespace

int stream_slab(const Lattice& L) {
  if (L.slab > 0) return std::min(L.slab, L.ntau);
  return std::min(2, L.ntau);  // best measured for 16^3 slices with HBM-resident data
}

bool stream_supported(const Lattice& L) {
  return (L.nx == 8 || L.nx == 12 || L.nx == 16) && !L.split_host.empty();
}

template <typename R>
int launch_hop_stream(const Lattice& L, const HopArgs<R>& args) {
  HopArgs<R> a = args;
  if (a.beta.x == 0.0 && a.beta.y == 0.0) a.aux = nullptr;
  switch (L.nx) {
    case 8: return launch_nx<R, 8>(L, a);
    case 12: return launch_nx<R, 12>(L, a);
    case 16: return launch_nx<R, 16>(L, a);
    default: set_error("streaming kernel: unsupported nx"); return UFG_EINVAL;
  }
}

template int launch_hop_stream<float>(const Lattice&, const HopArgs<float>&);
template int launch_hop_stream<double>(const Lattice&, const HopArgs<double>&);

}  // namespace ufg
