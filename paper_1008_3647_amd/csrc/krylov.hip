// Krylov vector kernels for CG and BiCGStab on [nrhs][N] complex vectors.
//
// Every right-hand side runs its own iteration: its scalars (rho, alpha,
// omega, ...) live on the device in RhsState and are updated by one-block
// "finalize" kernels that sum per-block partials in a fixed order (FP64, so
// results are reproducible run to run). Flags gate whole right-hand sides:
// a kernel block whose rhs is not active returns at once, which lets the
// host enqueue the same sequence every iteration without reading anything
// back. Reductions always accumulate in FP64, whatever the vector type.
#include <algorithm>

#include "krylov.h"
#include "krylov_fin.h"

namespace ufg {
namespace {

template <typename R>
__device__ __forceinline__ C2<R> c2(R a, R b) {
  C2<R> c;
  c.x = a;
  c.y = b;
  return c;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-reduce 4 doubles (blockDim.x == 256) into out[0..3] (thread 0).
__device__ void bsum4(double a0, double a1, double a2, double a3, double* out) {
  __shared__ double sm[4][4];
  a0 = wsum(a0);
  a1 = wsum(a1);
  a2 = wsum(a2);
  a3 = wsum(a3);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sm[wid][0] = a0;
    sm[wid][1] = a1;
    sm[wid][2] = a2;
    sm[wid][3] = a3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[4] = {0, 0, 0, 0};
    for (int w = 0; w < 4; ++w)
      for (int j = 0; j < 4; ++j) s[j] += sm[w][j];
    for (int j = 0; j < 4; ++j) out[j] = s[j];
  }
}

// Non-temporal access of one element (operands a kernel touches for the last
// time, or x, which only the update kernels touch): keeps the cache for the
// vectors the next launches read.
template <typename R>
__device__ __forceinline__ C2<R> ldnt(const C2<R>* p) {
  return c2<R>(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
template <typename R>
__device__ __forceinline__ void stnt(C2<R> v, C2<R>* p) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

#define KR_LOOP(n) \
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < (n); i += (long long)gridDim.x * 256)

// p = r + beta (p - omega v), beta = (rho / rho_old)(alpha / omega) from the state
template <typename R>
__global__ void __launch_bounds__(256) bicg_p_kernel(const C2<R>* r, C2<R>* p, const C2<R>* v,
                                                     const RhsState* st, const int* active,
                                                     long long n) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const RhsState s = st[k];
  const R br = R(s.beta.x), bi = R(s.beta.y), wr = R(s.omega.x), wi = R(s.omega.y);
  const long long off = (long long)k * n;
  KR_LOOP(n) {
    const C2<R> rv = r[off + i], pv = p[off + i], vv = v[off + i];
    const R dx = pv.x - (wr * vv.x - wi * vv.y);
    const R dy = pv.y - (wr * vv.y + wi * vv.x);
    p[off + i] = c2<R>(rv.x + br * dx - bi * dy, rv.y + br * dy + bi * dx);
  }
}

// s = r - alpha v
template <typename R>
__global__ void __launch_bounds__(256) bicg_s_kernel(const C2<R>* r, const C2<R>* v, C2<R>* s,
                                                     const RhsState* st, const int* active,
                                                     long long n) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const double2 al = st[k].alpha;
  const R ar = R(al.x), ai = R(al.y);
  const long long off = (long long)k * n;
  KR_LOOP(n) {
    const C2<R> rv = r[off + i], vv = v[off + i];
    s[off + i] = c2<R>(rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
  }
}

// x += alpha phat + omega shat; r = s - omega t; partials <rhat, r>, |r|^2
template <typename R>
__global__ void __launch_bounds__(256) bicg_xr_kernel(C2<R>* x, const C2<R>* phat,
                                                      const C2<R>* shat, const C2<R>* s,
                                                      const C2<R>* t, C2<R>* r, const C2<R>* rhat,
                                                      const RhsState* st, const int* active,
                                                      long long n, double* part) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const RhsState q = st[k];
  const R ar = R(q.alpha.x), ai = R(q.alpha.y), wr = R(q.omega.x), wi = R(q.omega.y);
  const long long off = (long long)k * n;
  double d0 = 0, d1 = 0, d2 = 0;
  KR_LOOP(n) {
    const long long j = off + i;
    // phat, shat, s and t are used for the last time in this iteration
    const C2<R> pv = ldnt<R>(phat + j), sv = ldnt<R>(shat + j), ss = ldnt<R>(s + j);
    const C2<R> tv = ldnt<R>(t + j), h = rhat[j];
    C2<R> xv = ldnt<R>(x + j);
    xv.x += (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y);
    xv.y += (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x);
    stnt<R>(xv, x + j);
    const C2<R> rv = c2<R>(ss.x - (wr * tv.x - wi * tv.y), ss.y - (wr * tv.y + wi * tv.x));
    r[j] = rv;
    d0 += double(h.x) * rv.x + double(h.y) * rv.y;
    d1 += double(h.x) * rv.y - double(h.y) * rv.x;
    d2 += double(rv.x) * rv.x + double(rv.y) * rv.y;
  }
  bsum4(d0, d1, d2, 0.0, part + ((long long)k * gridDim.x + blockIdx.x) * 4);
}

// Fused BiCGStab update with s = r - alpha v recomputed instead of stored:
// x += alpha p + omega s; r = s - omega t; partials <rhat, r>, |r|^2.
template <typename R>
__global__ void __launch_bounds__(256) bicg_xr_fused_kernel(C2<R>* x, const C2<R>* p, C2<R>* r,
                                                            const C2<R>* v, const C2<R>* t,
                                                            const C2<R>* rhat, const RhsState* st,
                                                            const int* active, long long n,
                                                            double* part) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const RhsState q = st[k];
  const R ar = R(q.alpha.x), ai = R(q.alpha.y), wr = R(q.omega.x), wi = R(q.omega.y);
  const long long off = (long long)k * n;
  double d0 = 0, d1 = 0, d2 = 0;
  KR_LOOP(n) {
    const long long j = off + i;
    // p and v are read again by the p update after the check point, t is not
    const C2<R> pv = p[j], vv = v[j], tv = ldnt<R>(t + j), h = rhat[j], rv = r[j];
    const C2<R> sv = c2<R>(rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
    C2<R> xv = ldnt<R>(x + j);
    xv.x += (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y);
    xv.y += (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x);
    stnt<R>(xv, x + j);
    const C2<R> rn = c2<R>(sv.x - (wr * tv.x - wi * tv.y), sv.y - (wr * tv.y + wi * tv.x));
    r[j] = rn;
    d0 += double(h.x) * rn.x + double(h.y) * rn.y;
    d1 += double(h.x) * rn.y - double(h.y) * rn.x;
    d2 += double(rn.x) * rn.x + double(rn.y) * rn.y;
  }
  bsum4(d0, d1, d2, 0.0, part + ((long long)k * gridDim.x + blockIdx.x) * 4);
}

// The x, r update of one iteration merged with the p update of the next
// (beta from the rho that FIN_OMEGA_RHO derived): s = r - alpha v,
// x += alpha p + omega s, r = s - omega t, p = r + beta (p - omega v);
// partial |r|^2 in slot 2.
template <typename R>
__global__ void __launch_bounds__(256) bicg_xrp_kernel(C2<R>* x, C2<R>* p, C2<R>* r,
                                                       const C2<R>* v, const C2<R>* t,
                                                       const RhsState* st, const int* active,
                                                       long long n, double* part) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const RhsState q = st[k];
  const R ar = R(q.alpha.x), ai = R(q.alpha.y), wr = R(q.omega.x), wi = R(q.omega.y);
  const R br = R(q.beta.x), bi = R(q.beta.y);
  const long long off = (long long)k * n;
  double d2 = 0;
  KR_LOOP(n) {
    const long long j = off + i;
    // x is touched only here, v and t for the last time in this iteration:
    // non-temporal, so that r and p stay cached for the next launches
    const C2<R> pv = p[j], rv = r[j];
    const C2<R> vv = ldnt<R>(v + j), tv = ldnt<R>(t + j);
    C2<R> xv = ldnt<R>(x + j);
    const C2<R> sv = c2<R>(rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
    xv.x += (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y);
    xv.y += (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x);
    stnt<R>(xv, x + j);
    const C2<R> rn = c2<R>(sv.x - (wr * tv.x - wi * tv.y), sv.y - (wr * tv.y + wi * tv.x));
    r[j] = rn;
    const R dx = pv.x - (wr * vv.x - wi * vv.y);
    const R dy = pv.y - (wr * vv.y + wi * vv.x);
    p[j] = c2<R>(rn.x + br * dx - bi * dy, rn.y + br * dy + bi * dx);
    d2 += double(rn.x) * rn.x + double(rn.y) * rn.y;
  }
  bsum4(0.0, 0.0, d2, 0.0, part + ((long long)k * gridDim.x + blockIdx.x) * 4);
}

// Generic reductions: mode 0 |a|^2 -> [2]; mode 1 <a, b> -> [0,1];
// mode 2 <a, b> -> [0,1] and |a|^2 -> [2]; mode 3 <b, a> -> [0,1] and |a|^2 -> [2].
template <typename R>
__global__ void __launch_bounds__(256) reduce_kernel(const C2<R>* a, const C2<R>* b, int mode,
                                                     const int* gate, long long n, double* part) {
  const int k = blockIdx.y;
  if (gate && !gate[k]) return;
  const long long off = (long long)k * n;
  double d0 = 0, d1 = 0, d2 = 0;
  KR_LOOP(n) {
    const C2<R> av = a[off + i];
    if (mode != 0) {
      const C2<R> bv = b[off + i];
      d0 += double(av.x) * bv.x + double(av.y) * bv.y;
      d1 += (mode == 3) ? double(bv.x) * av.y - double(bv.y) * av.x
                        : double(av.x) * bv.y - double(av.y) * bv.x;
    }
    if (mode != 1) d2 += double(av.x) * av.x + double(av.y) * av.y;
  }
  bsum4(d0, d1, d2, 0.0, part + ((long long)k * gridDim.x + blockIdx.x) * 4);
}

// y = a * x + b * y (complex scalars, same for every rhs); gate may be null.
template <typename R>
__global__ void __launch_bounds__(256) axpby_kernel(double2 a, const C2<R>* x, double2 b, C2<R>* y,
                                                    const int* gate, long long n) {
  const int k = blockIdx.y;
  if (gate && !gate[k]) return;
  const long long off = (long long)k * n;
  const R ar = R(a.x), ai = R(a.y), br = R(b.x), bi = R(b.y);
  const bool read_y = (b.x != 0.0 || b.y != 0.0);  // y may be uninitialised when b = 0
  KR_LOOP(n) {
    const C2<R> xv = x[off + i];
    C2<R> out = c2<R>(ar * xv.x - ai * xv.y, ar * xv.y + ai * xv.x);
    if (read_y) {
      const C2<R> yv = y[off + i];
      out.x += br * yv.x - bi * yv.y;
      out.y += br * yv.y + bi * yv.x;
    }
    y[off + i] = out;
  }
}

template <typename RI, typename RO>
__global__ void __launch_bounds__(256) convert_kernel(const C2<RI>* in, C2<RO>* out,
                                                      const int* gate, long long n) {
  const int k = blockIdx.y;
  if (gate && !gate[k]) return;
  const long long off = (long long)k * n;
  KR_LOOP(n) {
    const C2<RI> v = in[off + i];
    out[off + i] = c2<RO>(RO(v.x), RO(v.y));
  }
}

// Mixed precision: x64 += x32, x32 = 0 (gated by the update flag).
__global__ void __launch_bounds__(256) promote_kernel(double2* x64, float2* x32, const int* gate,
                                                      long long n) {
  const int k = blockIdx.y;
  if (gate && !gate[k]) return;
  const long long off = (long long)k * n;
  KR_LOOP(n) {
    const float2 v = x32[off + i];
    double2 w = x64[off + i];
    w.x += v.x;
    w.y += v.y;
    x64[off + i] = w;
    x32[off + i] = float2{0.f, 0.f};
  }
}

// r32 = r64 and partials <rhat, r>, |r64|^2 (gated).
__global__ void __launch_bounds__(256) demote_kernel(const double2* r64, float2* r32,
                                                     const float2* rhat, const int* gate,
                                                     long long n, double* part) {
  const int k = blockIdx.y;
  if (gate && !gate[k]) return;
  const long long off = (long long)k * n;
  double d0 = 0, d1 = 0, d2 = 0;
  KR_LOOP(n) {
    const double2 v = r64[off + i];
    r32[off + i] = float2{float(v.x), float(v.y)};
    if (rhat) {
      const float2 h = rhat[off + i];
      d0 += double(h.x) * v.x + double(h.y) * v.y;
      d1 += double(h.x) * v.y - double(h.y) * v.x;
    }
    d2 += v.x * v.x + v.y * v.y;
  }
  bsum4(d0, d1, d2, 0.0, part + ((long long)k * gridDim.x + blockIdx.x) * 4);
}

// CG: x += alpha p; r -= alpha w; partial |r|^2.
template <typename R>
__global__ void __launch_bounds__(256) cg_xr_kernel(C2<R>* x, const C2<R>* p, C2<R>* r,
                                                    const C2<R>* w, const RhsState* st,
                                                    const int* active, long long n, double* part) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const double2 al = st[k].alpha;
  const R ar = R(al.x), ai = R(al.y);
  const long long off = (long long)k * n;
  double d2 = 0;
  KR_LOOP(n) {
    const long long j = off + i;
    // w is used for the last time, x only here
    const C2<R> pv = p[j], wv = ldnt<R>(w + j);
    C2<R> xv = ldnt<R>(x + j), rv = r[j];
    xv.x += ar * pv.x - ai * pv.y;
    xv.y += ar * pv.y + ai * pv.x;
    rv.x -= ar * wv.x - ai * wv.y;
    rv.y -= ar * wv.y + ai * wv.x;
    stnt<R>(xv, x + j);
    r[j] = rv;
    d2 += double(rv.x) * rv.x + double(rv.y) * rv.y;
  }
  bsum4(0.0, 0.0, d2, 0.0, part + ((long long)k * gridDim.x + blockIdx.x) * 4);
}

// CG: p = z + beta p (beta = st.omega slot).
template <typename R>
__global__ void __launch_bounds__(256) cg_p_kernel(const C2<R>* z, C2<R>* p, const RhsState* st,
                                                   const int* active, long long n) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const double2 be = st[k].omega;
  const R br = R(be.x), bi = R(be.y);
  const long long off = (long long)k * n;
  KR_LOOP(n) {
    const C2<R> zv = z[off + i], pv = p[off + i];
    p[off + i] = c2<R>(zv.x + br * pv.x - bi * pv.y, zv.y + br * pv.y + bi * pv.x);
  }
}

// BiCGStab restart after a breakdown (rho = 0): rhat = r, p = v = 0.
template <typename R>
__global__ void __launch_bounds__(256) restart_kernel(const C2<R>* r, C2<R>* rhat, C2<R>* p,
                                                      C2<R>* v, const int* gate, long long n) {
  const int k = blockIdx.y;
  if (!gate[k]) return;
  const long long off = (long long)k * n;
  KR_LOOP(n) {
    rhat[off + i] = r[off + i];
    p[off + i] = c2<R>(R(0), R(0));
    v[off + i] = c2<R>(R(0), R(0));
  }
}

// One block per rhs: sum `nblk` partials of `stride` doubles (fixed order)
// into s[0..stride), and nblk2 partials of 4 from part2 into s[4..8), then
// apply `op`. NV: number of sums (4, or 8 with stride 8 or part2).
template <int NV>
__global__ void __launch_bounds__(256) finalize_kernel(int op, const double* part, int nblk,
                                                       int stride, const double* part2,
                                                       int nblk2, RhsState* st, int* active,
                                                       int* update, int* restart,
                                                       const int* gate, KrylovParams prm) {
  const int k = blockIdx.x;
  if (gate && !gate[k]) return;
  // the state is fetched while the partials are summed
  RhsState q;
  int act = 0, upd = 0, rst = 0;
  if (threadIdx.x == 0) {
    q = st[k];
    act = active[k];
    upd = update[k];
    rst = restart[k];
  }
  double a[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) a[j] = 0.0;
  if (NV == 8 && stride == 8) {
    for (int b = threadIdx.x; b < nblk; b += 256) {
      const double* q = part + ((long long)k * nblk + b) * 8;
#pragma unroll
      for (int j = 0; j < NV; ++j) a[j] += q[j];
    }
  } else {
    for (int b = threadIdx.x; b < nblk; b += 256) {
      const double* q = part + ((long long)k * nblk + b) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] += q[j];
    }
    if (NV == 8) {
      for (int b = threadIdx.x; b < nblk2; b += 256) {
        const double* q = part2 + ((long long)k * nblk2 + b) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[NV - 4 + j] += q[j];
      }
    }
  }
  __shared__ double sm[4][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    a[j] = wsum(a[j]);
    if (lane == 0) sm[wid][j] = a[j];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int w = 0; w < 4; ++w)
#pragma unroll
    for (int j = 0; j < NV; ++j) s[j] += sm[w][j];
  apply_fin(op, s, q, act, upd, rst, prm);
  st[k] = q;
  active[k] = act;
  update[k] = upd;
  restart[k] = rst;
}

// Segmented variant: rhs (segment) k owns partials [first[k], first[k] + count[k])
// of `stride` doubles (into s[0..stride)), and, with part2, partials
// [first2[k], first2[k] + count2[k]) of 4 doubles (into s[4..8)).
template <int NV>
__global__ void __launch_bounds__(256) finalize_seg_kernel(int op, const double* part,
                                                           const int* first, const int* count,
                                                           int stride, const double* part2,
                                                           const int* first2, const int* count2,
                                                           RhsState* st, int* active,
                                                           int* update, int* restart,
                                                           const int* gate, KrylovParams prm) {
  const int k = blockIdx.x;
  if (gate && !gate[k]) return;
  RhsState q;
  int act = 0, upd = 0, rst = 0;
  if (threadIdx.x == 0) {
    q = st[k];
    act = active[k];
    upd = update[k];
    rst = restart[k];
  }
  double a[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) a[j] = 0.0;
  const int f = first[k], c = count[k];
  if (NV == 8 && stride == 8) {
    for (int b = threadIdx.x; b < c; b += 256) {
      const double* qq = part + ((long long)f + b) * 8;
#pragma unroll
      for (int j = 0; j < NV; ++j) a[j] += qq[j];
    }
  } else {
    for (int b = threadIdx.x; b < c; b += 256) {
      const double* qq = part + ((long long)f + b) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] += qq[j];
    }
    if (NV == 8) {
      const int f2 = first2[k], c2 = count2[k];
      for (int b = threadIdx.x; b < c2; b += 256) {
        const double* qq = part2 + ((long long)f2 + b) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[NV - 4 + j] += qq[j];
      }
    }
  }
  __shared__ double sm[4][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    a[j] = wsum(a[j]);
    if (lane == 0) sm[wid][j] = a[j];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int w = 0; w < 4; ++w)
#pragma unroll
    for (int j = 0; j < NV; ++j) s[j] += sm[w][j];
  apply_fin(op, s, q, act, upd, rst, prm);
  st[k] = q;
  active[k] = act;
  update[k] = upd;
  restart[k] = rst;
}

}  // namespace

// Workgroups per rhs of the vector kernels: enough 256-thread groups for
// about four elements per thread, capped so that all right-hand sides
// together launch about 2048 groups (grid-stride loops keep them busy).
int vec_blocks(const Lattice& L, int nrhs) {
  if (L.vec_blocks > 0) return L.vec_blocks;
  long long nb = (L.N + 1023) / 1024;
  const long long cap = std::max(16, 2048 / std::max(1, nrhs));
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  return (int)nb;
}

namespace {
inline dim3 vgrid_for(const Lattice& L, int nrhs) {
  return dim3((unsigned)vec_blocks(L, nrhs), (unsigned)nrhs);
}
}  // namespace
#define vgrid(n, nrhs) vgrid_for(L, nrhs)

template <typename R>
int k_bicg_p(const Lattice& L, const C2<R>* r, C2<R>* p, const C2<R>* v, const KrylovState& K) {
  hipLaunchKernelGGL((bicg_p_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, r, p, v, K.st,
                     K.active, L.N);
  return UFG_OK;
}
template <typename R>
int k_bicg_s(const Lattice& L, const C2<R>* r, const C2<R>* v, C2<R>* s, const KrylovState& K) {
  hipLaunchKernelGGL((bicg_s_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, r, v, s, K.st,
                     K.active, L.N);
  return UFG_OK;
}
template <typename R>
int k_bicg_xr(const Lattice& L, C2<R>* x, const C2<R>* phat, const C2<R>* shat, const C2<R>* s,
              const C2<R>* t, C2<R>* r, const C2<R>* rhat, const KrylovState& K) {
  hipLaunchKernelGGL((bicg_xr_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, x, phat, shat,
                     s, t, r, rhat, K.st, K.active, L.N, K.part);
  return UFG_OK;
}
template <typename R>
int k_bicg_xr_fused(const Lattice& L, C2<R>* x, const C2<R>* p, C2<R>* r, const C2<R>* v,
                    const C2<R>* t, const C2<R>* rhat, const KrylovState& K) {
  hipLaunchKernelGGL((bicg_xr_fused_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, x, p,
                     r, v, t, rhat, K.st, K.active, L.N, K.part);
  return UFG_OK;
}
template <typename R>
int k_bicg_xrp(const Lattice& L, C2<R>* x, C2<R>* p, C2<R>* r, const C2<R>* v, const C2<R>* t,
               const KrylovState& K) {
  if (K.part2 == nullptr) {
    set_error("k_bicg_xrp: no second partials buffer");
    return UFG_EINVAL;
  }
  hipLaunchKernelGGL((bicg_xrp_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, x, p, r,
                     v, t, K.st, K.active, L.N, K.part2);
  return UFG_OK;
}
template <typename R>
int k_reduce(const Lattice& L, const C2<R>* a, const C2<R>* b, int mode, const int* gate,
             const KrylovState& K) {
  hipLaunchKernelGGL((reduce_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, a, b, mode,
                     gate, L.N, K.part);
  return UFG_OK;
}
template <typename R>
int k_axpby(const Lattice& L, double2 a, const C2<R>* x, double2 b, C2<R>* y, int nrhs,
            const int* gate) {
  hipLaunchKernelGGL((axpby_kernel<R>), vgrid(L.N, nrhs), dim3(256), 0, L.stream, a, x, b, y, gate,
                     L.N);
  return UFG_OK;
}
template <typename RI, typename RO>
int k_convert(const Lattice& L, const C2<RI>* in, C2<RO>* out, int nrhs, const int* gate) {
  hipLaunchKernelGGL((convert_kernel<RI, RO>), vgrid(L.N, nrhs), dim3(256), 0, L.stream, in, out,
                     gate, L.N);
  return UFG_OK;
}
int k_promote(const Lattice& L, double2* x64, float2* x32, int nrhs, const int* gate) {
  hipLaunchKernelGGL(promote_kernel, vgrid(L.N, nrhs), dim3(256), 0, L.stream, x64, x32, gate, L.N);
  return UFG_OK;
}
int k_demote(const Lattice& L, const double2* r64, float2* r32, const float2* rhat,
             const KrylovState& K, const int* gate) {
  hipLaunchKernelGGL(demote_kernel, vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, r64, r32, rhat,
                     gate, L.N, K.part);
  return UFG_OK;
}
template <typename R>
int k_cg_xr(const Lattice& L, C2<R>* x, const C2<R>* p, C2<R>* r, const C2<R>* w,
            const KrylovState& K) {
  hipLaunchKernelGGL((cg_xr_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, x, p, r, w,
                     K.st, K.active, L.N, K.part);
  return UFG_OK;
}
template <typename R>
int k_cg_p(const Lattice& L, const C2<R>* z, C2<R>* p, const KrylovState& K) {
  hipLaunchKernelGGL((cg_p_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, z, p, K.st,
                     K.active, L.N);
  return UFG_OK;
}
template <typename R>
int k_restart(const Lattice& L, const C2<R>* r, C2<R>* rhat, C2<R>* p, C2<R>* v,
              const KrylovState& K) {
  hipLaunchKernelGGL((restart_kernel<R>), vgrid(L.N, K.nrhs), dim3(256), 0, L.stream, r, rhat, p, v,
                     K.restart, L.N);
  return UFG_OK;
}
int k_finalize_seg(hipStream_t stream, int op, const double* part, const int* first,
                   const int* count, const int* gate, const KrylovState& K, int stride,
                   const double* part2, const int* first2, const int* count2) {
  if ((stride != 4 && stride != 8) || (part2 && (stride != 4 || !first2 || !count2))) {
    set_error("k_finalize_seg: bad partials layout");
    return UFG_EINVAL;
  }
  if (stride == 8 || part2)
    hipLaunchKernelGGL(finalize_seg_kernel<8>, dim3(K.nrhs), dim3(256), 0, stream, op, part,
                       first, count, stride, part2, first2, count2, K.st, K.active, K.update,
                       K.restart, gate, K.prm);
  else
    hipLaunchKernelGGL(finalize_seg_kernel<4>, dim3(K.nrhs), dim3(256), 0, stream, op, part,
                       first, count, stride, part2, first2, count2, K.st, K.active, K.update,
                       K.restart, gate, K.prm);
  return UFG_OK;
}
int k_finalize(const Lattice& L, int op, int nblk, const int* gate, const KrylovState& K,
               int stride, int nblk2) {
  if ((stride != 4 && stride != 8) || (nblk2 > 0 && (stride != 4 || K.part2 == nullptr))) {
    set_error("k_finalize: bad partials layout");
    return UFG_EINVAL;
  }
  if (stride == 8 || nblk2 > 0)
    hipLaunchKernelGGL(finalize_kernel<8>, dim3(K.nrhs), dim3(256), 0, L.stream, op, K.part, nblk,
                       stride, K.part2, nblk2, K.st, K.active, K.update, K.restart, gate, K.prm);
  else
    hipLaunchKernelGGL(finalize_kernel<4>, dim3(K.nrhs), dim3(256), 0, L.stream, op, K.part, nblk,
                       stride, K.part2, nblk2, K.st, K.active, K.update, K.restart, gate, K.prm);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

#define INST(R)                                                                                  \
  template int k_bicg_p<R>(const Lattice&, const C2<R>*, C2<R>*, const C2<R>*,                   \
                           const KrylovState&);                                                  \
  template int k_bicg_s<R>(const Lattice&, const C2<R>*, const C2<R>*, C2<R>*,                   \
                           const KrylovState&);                                                  \
  template int k_bicg_xr<R>(const Lattice&, C2<R>*, const C2<R>*, const C2<R>*, const C2<R>*,    \
                            const C2<R>*, C2<R>*, const C2<R>*, const KrylovState&);             \
  template int k_bicg_xr_fused<R>(const Lattice&, C2<R>*, const C2<R>*, C2<R>*, const C2<R>*,   \
                                  const C2<R>*, const C2<R>*, const KrylovState&);               \
  template int k_bicg_xrp<R>(const Lattice&, C2<R>*, C2<R>*, C2<R>*, const C2<R>*, const C2<R>*, \
                             const KrylovState&);                                                \
  template int k_reduce<R>(const Lattice&, const C2<R>*, const C2<R>*, int, const int*,          \
                           const KrylovState&);                                                  \
  template int k_axpby<R>(const Lattice&, double2, const C2<R>*, double2, C2<R>*, int,           \
                          const int*);                                                           \
  template int k_cg_xr<R>(const Lattice&, C2<R>*, const C2<R>*, C2<R>*, const C2<R>*,            \
                          const KrylovState&);                                                   \
  template int k_cg_p<R>(const Lattice&, const C2<R>*, C2<R>*, const KrylovState&);              \
  template int k_restart<R>(const Lattice&, const C2<R>*, C2<R>*, C2<R>*, C2<R>*,                \
                            const KrylovState&);
INST(float)
INST(double)
template int k_convert<float, double>(const Lattice&, const float2*, double2*, int, const int*);
template int k_convert<double, float>(const Lattice&, const double2*, float2*, int, const int*);
template int k_convert<double, double>(const Lattice&, const double2*, double2*, int, const int*);
template int k_convert<float, float>(const Lattice&, const float2*, float2*, int, const int*);

namespace {
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Plain streaming copy (16-byte loads, non-temporal 16-byte stores), the
// reference for the achievable HBM rate of the streaming kernels.
__global__ void __launch_bounds__(256) copy_kernel(const f32x4* __restrict__ src,
                                                   f32x4* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    __builtin_nontemporal_store(src[i], &dst[i]);
}
}  // namespace

int k_device_copy(const void* src, void* dst, long long bytes, hipStream_t stream) {
  const long long n = bytes / 16;
  const long long want = (n + 255) / 256;
  const int grid = (int)std::min<long long>(std::max<long long>(want, 1), 8192);
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, (const f32x4*)src,
                     (f32x4*)dst, n);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

}  // namespace ufg
