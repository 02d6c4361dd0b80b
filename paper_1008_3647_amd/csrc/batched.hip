// Batched two-step BiCGStab over many independent lattices (uneven Nx, Ntau).
//
// All systems (problem, right-hand side) of the batch are "segments" of one
// set of concatenated Krylov vectors, each with its own device-resident
// scalars and flags. Every phase of an iteration covers the whole batch with
// persistent grids (compute units x occupancy) that walk work tables: one
// operator launch per class of segments sharing Nx and T, over (segment, slab
// group) items, with BiCGStab's p- and s-updates fused into it, and one vector
// launch over (segment, chunk) items, so small lattices share the GPU instead
// of each paying its own launches. Whole check intervals, each closed by the
// check point's reliable updates (FP64 residual of the outer complex128
// vectors) and restarts as launches gated per segment by its device flags, are
// captured once in hipGraphs of one and of about 100 iterations' worth of
// intervals and replayed; the host reads the flags once per replay of the
// larger graph, and the work tables (with their sizes in device memory) are
// compacted without a new capture.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "hop_common.h"
#include "hop_stream.h"
#include "ops.h"
#include "split_line.h"

namespace ufg {
namespace {
using namespace hopc;

struct BSeg {
  int nx, ntau, V;
  long long n;    // elements of one vector of this system
  long long off;  // offset of the segment in the concatenated inner vectors
  const double2* b64;
  double2* x64;
  double2* r64;
  const float* f32;  // 1 + A sin sigma of the problem
  const double* f64;
  const float* T32;  // Nx x Nx transfer factor
  const double* T64;
};
struct BHop {
  int seg, t0;
};
struct BVec {
  int seg;
  long long lo, hi;
};

int g_hop_blocks_per_cu = 4;
int g_vec_blocks_per_cu = 8;
long long g_chunk = 4096;
int g_bop_slab = 2;
// iterations between host reads of the flags (measured on the 64-lattice
// batch: 200 gives 36 host waits instead of 56 at 100 in the same wall time;
// 400 was 1 % slower)
int g_sync_iters = 200;

template <typename R>
__device__ __forceinline__ const R* fld(const BSeg& g);
template <>
__device__ __forceinline__ const float* fld<float>(const BSeg& g) { return g.f32; }
template <>
__device__ __forceinline__ const double* fld<double>(const BSeg& g) { return g.f64; }
template <typename R>
__device__ __forceinline__ const R* tmat(const BSeg& g);
template <>
__device__ __forceinline__ const float* tmat<float>(const BSeg& g) { return g.T32; }
template <>
__device__ __forceinline__ const double* tmat<double>(const BSeg& g) { return g.T64; }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of 4 doubles into out[0..3] (thread 0 writes). `scratch` >= 4 doubles x 4 waves.
__device__ void bsum4b(double a0, double a1, double a2, double a3, double* out, double* scratch) {
  a0 = wsum(a0);
  a1 = wsum(a1);
  a2 = wsum(a2);
  a3 = wsum(a3);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    scratch[wid * 4 + 0] = a0;
    scratch[wid * 4 + 1] = a1;
    scratch[wid * 4 + 2] = a2;
    scratch[wid * 4 + 3] = a3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) {
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
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Batched operator. One launch per class of segments that share Nx and T (the
// same Nx and tau): the class's transform coefficients travel as kernel
// arguments. A workgroup holds SG sub-groups of Nx^2 threads (one z-line per
// thread); a work item is SG consecutive slabs of `slab` time slices of one
// segment, and each sub-group walks its slab like the single-lattice streaming
// kernel (M upwards, M^T downwards): the slice loaded for the identity term of
// one output is the source of the next, so only one halo slice per slab is
// loaded twice. Nx in {8, 12, 16} use the reflection-symmetry block form of T;
// the other Nx apply T as a dense Nx x Nx matrix.

__host__ __device__ constexpr int bop_groups(int nx) {
  return (nx * nx >= 576) ? 1 : 576 / (nx * nx);
}
__host__ __device__ constexpr int bop_threads(int nx) {
  return ((bop_groups(nx) * nx * nx + 63) / 64) * 64;
}
__host__ __device__ constexpr bool bop_split(int nx) { return nx == 8 || nx == 12 || nx == 16; }

template <typename R, int NX, bool SPLIT>
struct BCoef;
template <typename R, int NX>
struct BCoef<R, NX, true> {
  SplitCoef<R, NX> s;
};
template <typename R, int NX>
struct BCoef<R, NX, false> {
  R t[NX * NX];
};

template <typename R, int NX, bool SPLIT>
__device__ __forceinline__ void bline(const BCoef<R, NX, SPLIT>& c, C2<R> (&v)[NX]) {
  if constexpr (SPLIT) {
    splitk::split_line<R, NX>(c.s, v);
  } else {
    C2<R> w[NX];
    line_transform<R, NX>(c.t, v, w);
#pragma unroll
    for (int i = 0; i < NX; ++i) v[i] = w[i];
  }
}

// T^3 of one slice per sub-group (z-lines in v, thread l of the sub-group);
// sub-groups with act == false take part in the barriers only. A thread's
// last read and next first write touch only its own z-line, so the buffer
// needs no barrier before its reuse by the next slice.
template <typename R, int NX, bool SPLIT>
__device__ __forceinline__ void bslice_T3(const BCoef<R, NX, SPLIT>& c, C2<R>* my, int l,
                                          bool act, C2<R> (&v)[NX]) {
  constexpr int LD = NX + 1;
  const int y = l / NX, x = l - (l / NX) * NX;
  if (act) {
    bline<R, NX, SPLIT>(c, v);  // along z
#pragma unroll
    for (int z = 0; z < NX; ++z) my[(z * NX + y) * LD + x] = v[z];
  }
  __syncthreads();
  C2<R> w[NX];
  if (act) {  // along y: thread (z, x)
    const int z = l / NX, xx = l - (l / NX) * NX;
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) w[yy] = my[(z * NX + yy) * LD + xx];
    bline<R, NX, SPLIT>(c, w);
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) my[(z * NX + yy) * LD + xx] = w[yy];
  }
  __syncthreads();
  if (act) {  // along x: thread (z, y)
    const int z = l / NX, yy = l - (l / NX) * NX;
    C2<R>* row = my + (z * NX + yy) * LD;
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) w[xx] = row[xx];
    bline<R, NX, SPLIT>(c, w);
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) row[xx] = w[xx];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int z = 0; z < NX; ++z) v[z] = my[(z * NX + y) * LD + x];
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return double2{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// Fused BiCGStab sources of the batched operator (per segment, like the
// single-lattice streaming kernel): SRC 1 builds p = r + beta (p - omega v)
// while loading and stores it to pout for the sub-group's own slices; SRC 2
// builds s = r - alpha v (not stored). The scalars come from the segment's
// device state. The vectors are the concatenated inner vectors.
template <typename R>
struct BSrc {
  const C2<R>* r;
  const C2<R>* p;
  const C2<R>* v;
  C2<R>* pout;
  const RhsState* st;
};

template <typename R>
struct BScal {
  R br, bi, wr, wi, ar, ai;
};

template <typename R, int SRC>
__device__ __forceinline__ BScal<R> bsrc_scalars(const BSrc<R>& b, int seg) {
  BScal<R> q{};
  if (SRC == 0) return q;
  const RhsState s = b.st[seg];
  if (SRC == 1) {  // beta = (rho / rho_old)(alpha / omega), set by the finalize
    q.br = R(s.beta.x);
    q.bi = R(s.beta.y);
    q.wr = R(s.omega.x);
    q.wi = R(s.omega.y);
  } else {
    q.ar = R(s.alpha.x);
    q.ai = R(s.alpha.y);
  }
  return q;
}

// Non-temporal load of one element (operands the launch reads once).
template <typename R>
__device__ __forceinline__ C2<R> ldnt(const C2<R>* p) {
  C2<R> v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}

// z-line of the source at element offset o (segment offset included)
template <typename R, int NX, int SRC>
__device__ __forceinline__ void bsource(const C2<R>* src, const BSrc<R>& b, const BScal<R>& q,
                                        long long o, C2<R> (&X)[NX]) {
  constexpr int P = NX * NX;
#pragma unroll
  for (int z = 0; z < NX; ++z) {
    const long long i = o + z * P;
    if (SRC == 0) {
      X[z] = src[i];
    } else if (SRC == 1) {
      const C2<R> rv = b.r[i], pv = b.p[i], vv = b.v[i];
      const R dx = pv.x - (q.wr * vv.x - q.wi * vv.y);
      const R dy = pv.y - (q.wr * vv.y + q.wi * vv.x);
      X[z] = mk<R>(rv.x + q.br * dx - q.bi * dy, rv.y + q.br * dy + q.bi * dx);
    } else {
      const C2<R> rv = b.r[i], vv = b.v[i];
      X[z] = mk<R>(rv.x - (q.ar * vv.x - q.ai * vv.y), rv.y - (q.ar * vv.y + q.ai * vv.x));
    }
  }
}

// y_t = x_t + s T^3(...) over the items [range[0], range[1]) of one class (the
// range lives in device memory, so a captured launch follows the work tables
// when they are compacted).
// RES (SRC 0, R = double): y = b - M x on the outer FP64 vectors of the segment;
// else SRC 0 applies the operator to bs.p. SRC 3 is the source of SRC 2 with
// red_mode 4.
// red_mode 1: <w, y>; 3: <y, source>, |y|^2, |source|^2; 4: those of 3, then
// <w, y>, <w, source> (per item partials: 4 doubles, 8 for mode 4).
template <typename R, int NX, int DIR, bool RES, bool SPLIT, int SRC>
__global__ void __launch_bounds__(bop_threads(NX))
    bop_kernel(BCoef<R, NX, SPLIT> c, const BSeg* __restrict__ segs,
               const BHop* __restrict__ items, const int* range, BSrc<R> bs, C2<R>* dst_cat,
               int red_mode, const C2<R>* redw_cat, double* part, const int* gate, int slab) {
  const int i0 = range[0], i1 = range[1];
  constexpr int P = NX * NX, V = NX * NX * NX, SL = NX * NX * (NX + 1), SG = bop_groups(NX);
  constexpr int SM = (SRC == 3) ? 2 : SRC;  // source mode
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double scratch[4 * (bop_threads(NX) / 64)];
  const int tid = threadIdx.x;
  const int sub = tid / P, l = tid - (tid / P) * P;
  const bool member = sub < SG;
  C2<R>* my = reinterpret_cast<C2<R>*>(smem_raw) + (member ? sub : 0) * SL;
  for (int it = i0 + blockIdx.x; it < i1; it += gridDim.x) {
    const BHop h = items[it];
    if (gate && gate[h.seg] == 0) continue;
    const BSeg g = segs[h.seg];
    const C2<R>* src = nullptr;  // SRC 0
    C2<R>* dst;
    const C2<R>* aux = nullptr;
    long long so = 0;  // offset of the segment in the inner vectors
    if (RES) {
      src = reinterpret_cast<const C2<R>*>(g.x64);
      dst = reinterpret_cast<C2<R>*>(g.r64);
      aux = reinterpret_cast<const C2<R>*>(g.b64);
    } else {
      so = g.off;
      dst = dst_cat + so;
      if (SRC == 0) src = bs.p;
    }
    const BScal<R> q = bsrc_scalars<R, SM>(bs, h.seg);
    const C2<R>* redw = redw_cat ? redw_cat + so : nullptr;
    const R* f = fld<R>(g);
    const int ntau = g.ntau;
    const int ts0 = h.t0 + (member ? sub : SG) * slab;
    const int ts1 = min(ts0 + slab, ntau);
    const int count = (member && ts1 > ts0) ? ts1 - ts0 : 0;
    const bool live = count > 0;
    const int tfirst = (DIR < 0) ? ts0 : ts1 - 1;
    const int step = (DIR < 0) ? 1 : -1;
    // halo slice feeding the first output
    const int th = (DIR < 0) ? ((ts0 == 0) ? ntau - 1 : ts0 - 1) : ((ts1 == ntau) ? 0 : ts1);
    C2<R> W[NX], X[NX];
    if (live) {
      bsource<R, NX, SM>(src, bs, q, so + (long long)th * V + l, W);
      if (DIR < 0) {
#pragma unroll
        for (int z = 0; z < NX; ++z) {
          const R fz = f[(long long)th * V + z * P + l];
          W[z].x *= fz;
          W[z].y *= fz;
        }
      }
    }
    bslice_T3<R, NX, SPLIT>(c, my, l, live, W);
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, a7 = 0;
    for (int k = 0; k < slab; ++k) {
      const bool act = k < count;
      const int t = tfirst + k * step;
      if (act) {
        R sgn;
        if (DIR < 0)
          sgn = (t == 0) ? R(1) : R(-1);
        else
          sgn = (t == ntau - 1) ? R(1) : R(-1);
        const long long o = (long long)t * V + l;
        bsource<R, NX, SM>(src, bs, q, so + o, X);
        if (SRC == 1) {
#pragma unroll
          for (int z = 0; z < NX; ++z) bs.pout[so + o + z * P] = X[z];
        }
        R F[NX];
#pragma unroll
        for (int z = 0; z < NX; ++z) F[z] = (DIR > 0) ? sgn * f[o + z * P] : sgn;
        C2<R> B[RES ? NX : 1], Q[NX];
        if (RES) {
#pragma unroll
          for (int z = 0; z < NX; ++z) B[RES ? z : 0] = ldnt<R>(aux + o + z * P);
        }
        if (red_mode == 1 || SRC == 3) {
#pragma unroll
          for (int z = 0; z < NX; ++z) Q[z] = ldnt<R>(redw + o + z * P);
        }
#pragma unroll
        for (int z = 0; z < NX; ++z) {
          C2<R> out = mk<R>(X[z].x + F[z] * W[z].x, X[z].y + F[z] * W[z].y);
          if (RES) {
            const C2<R> bb = B[RES ? z : 0];
            out = mk<R>(bb.x - out.x, bb.y - out.y);
          }
          // y is not re-read by this launch
          __builtin_nontemporal_store(out.x, &dst[o + z * P].x);
          __builtin_nontemporal_store(out.y, &dst[o + z * P].y);
          if (red_mode == 1) {  // <w, y>
            a0 += double(Q[z].x) * out.x + double(Q[z].y) * out.y;
            a1 += double(Q[z].x) * out.y - double(Q[z].y) * out.x;
          } else if (red_mode == 3 || red_mode == 4) {  // <y, source>, |y|^2, |source|^2
            a0 += double(out.x) * X[z].x + double(out.y) * X[z].y;
            a1 += double(out.x) * X[z].y - double(out.y) * X[z].x;
            a2 += double(out.x) * out.x + double(out.y) * out.y;
            a3 += double(X[z].x) * X[z].x + double(X[z].y) * X[z].y;
            if (SRC == 3) {  // <w, y>, <w, source>
              a4 += double(Q[z].x) * out.x + double(Q[z].y) * out.y;
              a5 += double(Q[z].x) * out.y - double(Q[z].y) * out.x;
              a6 += double(Q[z].x) * X[z].x + double(Q[z].y) * X[z].y;
              a7 += double(Q[z].x) * X[z].y - double(Q[z].y) * X[z].x;
            }
          }
        }
      }
      if (k + 1 < slab) {  // transform source slice t for the next output
        const bool tr = act && k + 1 < count;
        if (tr) {
#pragma unroll
          for (int z = 0; z < NX; ++z) {
            W[z] = X[z];
            if (DIR < 0) {
              const R fz = f[(long long)t * V + z * P + l];
              W[z].x *= fz;
              W[z].y *= fz;
            }
          }
        }
        bslice_T3<R, NX, SPLIT>(c, my, l, tr, W);
      }
    }
    if (SRC == 3) {
      bsum4b(a0, a1, a2, a3, part + (long long)it * 8, scratch);
      bsum4b(a4, a5, a6, a7, part + (long long)it * 8 + 4, scratch);
    } else if (red_mode) {
      bsum4b(a0, a1, a2, a3, part + (long long)it * 4, scratch);
    }
  }
}

#define BV_LOOP(v) for (long long i = v.lo + threadIdx.x; i < v.hi; i += blockDim.x)


// Vector phases (the p and s updates ride on the operator launches). op:
// 9 x/r update with s = r - alpha v recomputed (+partials),
// 3 init (x_in = 0, r = b, rhat = r, p = v = 0; |b|^2 partials, x64 = 0),
// 4 promote (x64 += x_in, x_in = 0), 5 demote (r = r64; <rhat, r>, |r64|^2),
// 6 restart (rhat = r, p = v = 0), 7 |b64|^2 partials, 8 |r64|^2 partials,
// 10 the x/r update of op 9 merged with the next p update, pn = r + beta (p -
// omega v) (beta from the rho that FIN_OMEGA_RHO derived; |r|^2 partials).
struct BVecArgs {
  void* x;
  void* r;
  void* rhat;
  void* p;
  void* v;
  void* t;
  void* pn;  // op 10: the new p
};

template <typename R>
__global__ void __launch_bounds__(256)
    bvec_kernel(int op, const BSeg* __restrict__ segs, const BVec* __restrict__ items,
                const int* nitems_dev, BVecArgs A, const RhsState* st, const int* gate,
                double* part) {
  const int nitems = *nitems_dev;
  __shared__ double scratch[16];
  C2<R>* X = reinterpret_cast<C2<R>*>(A.x);
  C2<R>* Rr = reinterpret_cast<C2<R>*>(A.r);
  C2<R>* Rh = reinterpret_cast<C2<R>*>(A.rhat);
  C2<R>* Pp = reinterpret_cast<C2<R>*>(A.p);
  C2<R>* Vv = reinterpret_cast<C2<R>*>(A.v);
  C2<R>* Tt = reinterpret_cast<C2<R>*>(A.t);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BVec item = items[it];
    if (gate && gate[item.seg] == 0) continue;
    const BSeg g = segs[item.seg];
    const long long o = g.off;
    const RhsState q = st[item.seg];
    double a0 = 0, a1 = 0, a2 = 0;
    if (op == 9) {  // x += alpha p + omega s, r = s - omega t, s = r - alpha v
      const R ar = R(q.alpha.x), ai = R(q.alpha.y), wr = R(q.omega.x), wi = R(q.omega.y);
      BV_LOOP(item) {
        // t is used for the last time and x only here: non-temporal (p and v
        // are read again by the p update after the check point)
        const C2<R> pv = Pp[o + i], rv = Rr[o + i], vv = Vv[o + i], tv = ldnt<R>(Tt + o + i),
                    h = Rh[o + i];
        const C2<R> sv = mk<R>(rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
        C2<R> xv = ldnt<R>(X + o + i);
        xv.x += (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y);
        xv.y += (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x);
        __builtin_nontemporal_store(xv.x, &X[o + i].x);
        __builtin_nontemporal_store(xv.y, &X[o + i].y);
        const C2<R> rn = mk<R>(sv.x - (wr * tv.x - wi * tv.y), sv.y - (wr * tv.y + wi * tv.x));
        Rr[o + i] = rn;
        a0 += double(h.x) * rn.x + double(h.y) * rn.y;
        a1 += double(h.x) * rn.y - double(h.y) * rn.x;
        a2 += double(rn.x) * rn.x + double(rn.y) * rn.y;
      }
    } else if (op == 10) {
      const R ar = R(q.alpha.x), ai = R(q.alpha.y), wr = R(q.omega.x), wi = R(q.omega.y);
      const R br = R(q.beta.x), bi = R(q.beta.y);
      C2<R>* Pn = reinterpret_cast<C2<R>*>(A.pn);
      BV_LOOP(item) {
        // the old p, v and t are used for the last time and x only here:
        // non-temporal, so that the cache keeps r and the new p
        const C2<R> pv = ldnt<R>(Pp + o + i), rv = Rr[o + i], vv = ldnt<R>(Vv + o + i),
                    tv = ldnt<R>(Tt + o + i);
        const C2<R> sv = mk<R>(rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
        C2<R> xv = ldnt<R>(X + o + i);
        xv.x += (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y);
        xv.y += (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x);
        __builtin_nontemporal_store(xv.x, &X[o + i].x);
        __builtin_nontemporal_store(xv.y, &X[o + i].y);
        const C2<R> rn = mk<R>(sv.x - (wr * tv.x - wi * tv.y), sv.y - (wr * tv.y + wi * tv.x));
        Rr[o + i] = rn;
        const R dx = pv.x - (wr * vv.x - wi * vv.y);
        const R dy = pv.y - (wr * vv.y + wi * vv.x);
        Pn[o + i] = mk<R>(rn.x + br * dx - bi * dy, rn.y + br * dy + bi * dx);
        a2 += double(rn.x) * rn.x + double(rn.y) * rn.y;
      }
    } else if (op == 3) {
      BV_LOOP(item) {
        const double2 bb = g.b64[i];
        const C2<R> rv = mk<R>(R(bb.x), R(bb.y));
        X[o + i] = mk<R>(R(0), R(0));
        Rr[o + i] = rv;
        Rh[o + i] = rv;
        Pp[o + i] = mk<R>(R(0), R(0));
        Vv[o + i] = mk<R>(R(0), R(0));
        g.x64[i] = double2{0.0, 0.0};
        a2 += bb.x * bb.x + bb.y * bb.y;
      }
    } else if (op == 4) {
      BV_LOOP(item) {
        const C2<R> v = X[o + i];
        double2 w = g.x64[i];
        w.x += double(v.x);
        w.y += double(v.y);
        g.x64[i] = w;
        X[o + i] = mk<R>(R(0), R(0));
      }
    } else if (op == 5) {
      BV_LOOP(item) {
        const double2 v = g.r64[i];
        Rr[o + i] = mk<R>(R(v.x), R(v.y));
        const C2<R> h = Rh[o + i];
        a0 += double(h.x) * v.x + double(h.y) * v.y;
        a1 += double(h.x) * v.y - double(h.y) * v.x;
        a2 += v.x * v.x + v.y * v.y;
      }
    } else if (op == 6) {
      BV_LOOP(item) {
        Rh[o + i] = Rr[o + i];
        Pp[o + i] = mk<R>(R(0), R(0));
        Vv[o + i] = mk<R>(R(0), R(0));
      }
    } else if (op == 7) {
      BV_LOOP(item) {
        const double2 bb = g.b64[i];
        a2 += bb.x * bb.x + bb.y * bb.y;
      }
    } else if (op == 8) {
      BV_LOOP(item) {
        const double2 v = g.r64[i];
        a2 += v.x * v.x + v.y * v.y;
      }
    }
    if (op == 3 || op == 5 || op >= 7)
      bsum4b(a0, a1, a2, 0.0, part + (long long)it * 4, scratch);
  }
}

// --------------------------------------------------------------------------

struct Dev {
  void* p = nullptr;
  ~Dev() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      set_error("solve_batched: device allocation failed");
      return UFG_ENOMEM;
    }
    return UFG_OK;
  }
};

// Operator class: segments with the same Nx and T share one launch.
struct BClass {
  int nx = 0;
  std::vector<double> T, coef;  // coef: block form (Nx in {8, 12, 16}) or T
  int i0 = 0, i1 = 0;           // item range in the operator table (host copy)
  int nmax = 0;                 // items of the class with every segment live
  const int* range = nullptr;   // device copy of {i0, i1}
};

template <typename R, int NX, int DIR, bool RES, int SRC>
int launch_bop_nx(const BClass& k, int ncu, hipStream_t cs, bool prepare, const BSeg* dseg,
                  const BHop* dhop, const BSrc<R>& bsrc, C2<R>* dst, int red_mode,
                  const C2<R>* redw, double* part, const int* gate, int slab) {
  constexpr bool SPLIT = bop_split(NX);
  constexpr int SG = bop_groups(NX);
  const size_t lds = size_t(SG) * NX * NX * (NX + 1) * sizeof(C2<R>);
  const void* fn = (const void*)bop_kernel<R, NX, DIR, RES, SPLIT, SRC>;
  if (prepare) {  // before any capture
    UFG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return UFG_OK;
  }
  // persistent grid sized for the full table; the live range is read on the device
  const int n = k.nmax;
  if (n <= 0) return UFG_OK;
  BCoef<R, NX, SPLIT> c;
  if constexpr (SPLIT) {
    int j = 0;
    for (auto& v : c.s.es) v = R(k.coef[j++]);
    for (auto& v : c.s.ea) v = R(k.coef[j++]);
    for (auto& v : c.s.os) v = R(k.coef[j++]);
    for (auto& v : c.s.oa) v = R(k.coef[j++]);
  } else {
    for (int j = 0; j < NX * NX; ++j) c.t[j] = R(k.coef[j]);
  }
  const dim3 grid(std::max(1, std::min(n, ncu * g_hop_blocks_per_cu)));
  hipLaunchKernelGGL((bop_kernel<R, NX, DIR, RES, SPLIT, SRC>), grid, dim3(bop_threads(NX)), lds,
                     cs, c, dseg, dhop, k.range, bsrc, dst, red_mode, redw, part, gate, slab);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

// One class, one phase: DIR -1 (M) / +1 (M^T); RES: FP64 residual b - A x;
// else SRC 1 (p-update fused, red 1) or 2 (s on the fly, red 3).
template <typename R, int DIR, bool RES, int SRC>
int launch_bop(const BClass& k, int ncu, hipStream_t cs, bool prepare, const BSeg* dseg,
               const BHop* dhop, const BSrc<R>& bsrc, C2<R>* dst, int red_mode,
               const C2<R>* redw, double* part, const int* gate, int slab) {
  switch (k.nx) {
#define BOP(NXV)                                                                           \
  case NXV:                                                                                \
    return launch_bop_nx<R, NXV, DIR, RES, SRC>(k, ncu, cs, prepare, dseg, dhop, bsrc, dst, \
                                                red_mode, redw, part, gate, slab);
    BOP(2) BOP(4) BOP(6) BOP(8) BOP(10) BOP(12) BOP(14) BOP(16)
#undef BOP
    default:
      set_error("solve_batched: unsupported nx");
      return UFG_EINVAL;
  }
}

struct Graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  ~Graph() {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
  }
};

template <typename RI>
int run_batched(std::vector<Lattice*>& Ls, const void* const* bu, void* const* xu,
                const int* nrhs, const ufg_solve_opts& o, ufg_solve_stats* stats) {
  const int nprob = (int)Ls.size();
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, Ls[0]->device);
  // segments, their operator classes (same Nx and T) and the work tables
  std::vector<BSeg> segs;
  std::vector<int> seg_prob, seg_cls;
  std::vector<BClass> cls;
  long long total = 0;
  for (int i = 0; i < nprob; ++i) {
    Lattice& L = *Ls[i];
    int c = 0;
    while (c < (int)cls.size() && !(cls[c].nx == L.nx && cls[c].T == L.T_host)) ++c;
    if (c == (int)cls.size()) {
      BClass k;
      k.nx = L.nx;
      k.T = L.T_host;
      k.coef = bop_split(L.nx) ? L.split_host : L.T_host;
      cls.push_back(k);
    }
    for (int r = 0; r < nrhs[i]; ++r) {
      BSeg g{};
      g.nx = L.nx;
      g.ntau = L.ntau;
      g.V = L.V;
      g.n = L.N;
      g.off = total;
      g.f32 = L.f32.b;
      g.f64 = L.f64.b;
      g.T32 = L.f32.T;
      g.T64 = L.f64.T;
      total += L.N;
      segs.push_back(g);
      seg_prob.push_back(i);
      seg_cls.push_back(c);
    }
  }
  const int S = (int)segs.size();
  const int C = (int)cls.size();
  const int slab = g_bop_slab;
  // Work tables over the segments marked in `use` (the others get no items):
  // operator items (segment, first slice of SG slabs), grouped by class, and
  // vector items (segment, chunk), with each segment's first item and item
  // count (its partial sums).
  std::vector<BHop> hops;
  std::vector<BVec> vecs;
  std::vector<int> htab(4 * S);
  auto make_tables = [&](const std::vector<char>& use) {
    hops.clear();
    vecs.clear();
    for (int c = 0; c < C; ++c) {
      cls[c].i0 = (int)hops.size();
      const int span = bop_groups(cls[c].nx) * slab;
      for (int s = 0; s < S; ++s) {
        if (seg_cls[s] != c) continue;
        htab[s] = (int)hops.size();
        if (use[s])
          for (int t0 = 0; t0 < segs[s].ntau; t0 += span) hops.push_back(BHop{s, t0});
        htab[S + s] = (int)hops.size() - htab[s];
      }
      cls[c].i1 = (int)hops.size();
    }
    for (int s = 0; s < S; ++s) {
      htab[2 * S + s] = (int)vecs.size();
      if (use[s])
        for (long long lo = 0; lo < segs[s].n; lo += g_chunk)
          vecs.push_back(BVec{s, lo, std::min(segs[s].n, lo + g_chunk)});
      htab[3 * S + s] = (int)vecs.size() - htab[2 * S + s];
    }
  };
  const std::vector<char> all_segs(S, 1);
  make_tables(all_segs);
  for (int c = 0; c < C; ++c) cls[c].nmax = cls[c].i1 - cls[c].i0;
  const int nv_max = (int)vecs.size();
  // device memory
  const size_t vbytes = sizeof(C2<RI>) * (size_t)total;
  Dev dvec[8], dr64, dy, dsegs, dhops, dvecs, dtab, dhpart, dvpart, dstate, dcnt;
  for (auto& d : dvec) UFG_TRY(d.alloc(vbytes));
  UFG_TRY(dr64.alloc(sizeof(double2) * (size_t)total));
  UFG_TRY(dy.alloc(sizeof(double2) * (size_t)total));
  UFG_TRY(dsegs.alloc(sizeof(BSeg) * S));
  UFG_TRY(dhops.alloc(sizeof(BHop) * hops.size()));
  UFG_TRY(dvecs.alloc(sizeof(BVec) * vecs.size()));
  UFG_TRY(dtab.alloc(sizeof(int) * 4 * S));
  UFG_TRY(dhpart.alloc(sizeof(double) * 8 * hops.size()));
  UFG_TRY(dvpart.alloc(sizeof(double) * 4 * vecs.size()));
  UFG_TRY(dstate.alloc(sizeof(RhsState) * S + sizeof(int) * 3 * S));
  UFG_TRY(dcnt.alloc(sizeof(int) * (2 * C + 1)));  // class item ranges, vector item count
  int* cnt_dev = reinterpret_cast<int*>(dcnt.p);
  for (int c = 0; c < C; ++c) cls[c].range = cnt_dev + 2 * c;
  const int* nv_dev = cnt_dev + 2 * C;
  std::vector<int> hcnt(2 * C + 1);
  long long n_sync = 0, n_submit = 0;  // host synchronisations and submissions
  hipStream_t cs = nullptr;
  UFG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      if (s) (void)hipStreamDestroy(s);
    }
  } guard{cs};
  int* tab = reinterpret_cast<int*>(dtab.p);
  // persistent vector grid sized for the full table
  const dim3 vgrid(std::max(1, std::min(nv_max, ncu * g_vec_blocks_per_cu)));
  // upload the tables and their sizes (the device buffers were sized for all
  // segments); captured launches read them from there. Synchronous: the host
  // copies must stay alive until the transfer is done.
  auto upload_tables = [&]() -> int {
    UFG_HIP(hipMemcpyAsync(tab, htab.data(), sizeof(int) * 4 * S, hipMemcpyHostToDevice, cs));
    if (!hops.empty())
      UFG_HIP(hipMemcpyAsync(dhops.p, hops.data(), sizeof(BHop) * hops.size(),
                             hipMemcpyHostToDevice, cs));
    if (!vecs.empty())
      UFG_HIP(hipMemcpyAsync(dvecs.p, vecs.data(), sizeof(BVec) * vecs.size(),
                             hipMemcpyHostToDevice, cs));
    for (int c = 0; c < C; ++c) {
      hcnt[2 * c] = cls[c].i0;
      hcnt[2 * c + 1] = cls[c].i1;
    }
    hcnt[2 * C] = (int)vecs.size();
    UFG_HIP(hipMemcpyAsync(cnt_dev, hcnt.data(), sizeof(int) * (2 * C + 1),
                           hipMemcpyHostToDevice, cs));
    UFG_HIP(hipStreamSynchronize(cs));
    n_submit += 4;
    ++n_sync;
    return UFG_OK;
  };
  UFG_TRY(upload_tables());
  KrylovState K;
  K.nrhs = S;
  K.st = reinterpret_cast<RhsState*>(dstate.p);
  K.active = reinterpret_cast<int*>(K.st + S);
  K.update = K.active + S;
  K.restart = K.update + S;
  K.part = reinterpret_cast<double*>(dvpart.p);
  K.prm.tol = o.tol;
  K.prm.delta2 = o.delta * o.delta;
  K.prm.mixed = 1;  // inner vectors are corrections to the FP64 x (reliable updates)
  K.prm.bicg = 1;
  K.prm.unprec = 1;
  K.prm.limit_omega = 1;
  const int* hf = tab;
  const int* hc = tab + S;
  const int* vf = tab + 2 * S;
  const int* vc = tab + 3 * S;
  double* hpart = reinterpret_cast<double*>(dhpart.p);
  double* vpart = reinterpret_cast<double*>(dvpart.p);
  // inner vectors: x, r, rhat, p (two, alternating), v (two, alternating), t
  BVecArgs VA{dvec[0].p, dvec[1].p, dvec[2].p, dvec[3].p, dvec[4].p, dvec[6].p, nullptr};
  C2<RI>* vr = reinterpret_cast<C2<RI>*>(dvec[1].p);
  C2<RI>* vrh = reinterpret_cast<C2<RI>*>(dvec[2].p);
  C2<RI>* vt = reinterpret_cast<C2<RI>*>(dvec[6].p);
  C2<RI>* pbuf[2] = {reinterpret_cast<C2<RI>*>(dvec[3].p), reinterpret_cast<C2<RI>*>(dvec[5].p)};
  C2<RI>* vbuf[2] = {reinterpret_cast<C2<RI>*>(dvec[4].p), reinterpret_cast<C2<RI>*>(dvec[7].p)};
  const BSeg* dseg = reinterpret_cast<const BSeg*>(dsegs.p);
  const BHop* dhop = reinterpret_cast<const BHop*>(dhops.p);
  const BVec* dvv = reinterpret_cast<const BVec*>(dvecs.p);
  // dynamic LDS limits of every operator instance, set before any capture
  const BSrc<RI> nosrc{};
  const BSrc<double> nosrc64{};
  for (const BClass& k : cls) {
    UFG_TRY((launch_bop<RI, -1, false, 1>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                          nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, 1, false, 1>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                         nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, -1, false, 2>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                          nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, 1, false, 2>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                         nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, -1, false, 0>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                          nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, -1, false, 3>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                          nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, 1, false, 3>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                         nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<RI, 1, false, 0>(k, ncu, cs, true, nullptr, nullptr, nosrc, nullptr, 0,
                                         nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<double, -1, true, 0>(k, ncu, cs, true, nullptr, nullptr, nosrc64, nullptr,
                                             0, nullptr, nullptr, nullptr, slab)));
    UFG_TRY((launch_bop<double, 1, true, 0>(k, ncu, cs, true, nullptr, nullptr, nosrc64, nullptr,
                                            0, nullptr, nullptr, nullptr, slab)));
  }
  int check = o.check_every > 0 ? o.check_every : 10;
  check += check & 1;
  std::vector<RhsState> hst(S);
  std::vector<int> hflags(3 * S);
  FlagMirror mirror;
  std::vector<int> iters_step[2];
  std::vector<double> relres_step[2];
  std::vector<int> status(nprob, 0);

  for (int step = 0; step < 2; ++step) {
    const int dir = (step == 0) ? +1 : -1;  // M^T first, then M
    for (int s = 0; s < S; ++s) {
      const int i = seg_prob[s];
      const int r = s - (int)(std::lower_bound(seg_prob.begin(), seg_prob.end(), i) -
                              seg_prob.begin());
      const long long N = Ls[i]->N;
      double2* ycat = reinterpret_cast<double2*>(dy.p) + segs[s].off;
      if (step == 0) {
        segs[s].b64 = reinterpret_cast<const double2*>(bu[i]) + r * N;
        segs[s].x64 = ycat;
      } else {
        segs[s].b64 = ycat;
        segs[s].x64 = reinterpret_cast<double2*>(xu[i]) + r * N;
      }
      segs[s].r64 = reinterpret_cast<double2*>(dr64.p) + segs[s].off;
    }
    UFG_HIP(hipMemcpyAsync(dsegs.p, segs.data(), sizeof(BSeg) * S, hipMemcpyHostToDevice, cs));
    // src_mode 1: p_new = r + beta (p - omega v) fused into v_new = A p_new
    // (+ <rhat, v_new>); 0: v = A p (+ <rhat, v>); 2: s = r - alpha v fused into
    // t = A s (+ <t, s>, |t|^2, |s|^2, and with red 4 <rhat, t>, <rhat, s>).
    // p and v alternate between two buffers so that halo reads never see this
    // launch's writes.
    auto hop = [&](int src_mode, int red, const C2<RI>* pin, C2<RI>* pout, const C2<RI>* vin,
                   C2<RI>* dst) -> int {
      const BSrc<RI> b{vr, pin, vin, pout, K.st};
      const C2<RI>* w = (red == 1 || red == 4) ? vrh : nullptr;
      for (const BClass& k : cls) {
        if (src_mode == 1 && dir < 0)
          UFG_TRY((launch_bop<RI, -1, false, 1>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                                hpart, K.active, slab)));
        else if (src_mode == 1)
          UFG_TRY((launch_bop<RI, 1, false, 1>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                               hpart, K.active, slab)));
        else if (src_mode == 0 && dir < 0)
          UFG_TRY((launch_bop<RI, -1, false, 0>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                                hpart, K.active, slab)));
        else if (src_mode == 0)
          UFG_TRY((launch_bop<RI, 1, false, 0>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                               hpart, K.active, slab)));
        else if (red == 4 && dir < 0)
          UFG_TRY((launch_bop<RI, -1, false, 3>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                                hpart, K.active, slab)));
        else if (red == 4)
          UFG_TRY((launch_bop<RI, 1, false, 3>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                               hpart, K.active, slab)));
        else if (dir < 0)
          UFG_TRY((launch_bop<RI, -1, false, 2>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                                hpart, K.active, slab)));
        else
          UFG_TRY((launch_bop<RI, 1, false, 2>(k, ncu, cs, false, dseg, dhop, b, dst, red, w,
                                               hpart, K.active, slab)));
      }
      return UFG_OK;
    };
    auto residual = [&](const int* gate) -> int {
      for (const BClass& k : cls) {
        if (dir < 0)
          UFG_TRY((launch_bop<double, -1, true, 0>(k, ncu, cs, false, dseg, dhop, nosrc64,
                                                   nullptr, 0, nullptr, hpart, gate, slab)));
        else
          UFG_TRY((launch_bop<double, 1, true, 0>(k, ncu, cs, false, dseg, dhop, nosrc64,
                                                  nullptr, 0, nullptr, hpart, gate, slab)));
      }
      return UFG_OK;
    };
    auto vop = [&](int op, const int* gate, const BVecArgs& args) {
      hipLaunchKernelGGL((bvec_kernel<RI>), vgrid, dim3(256), 0, cs, op, dseg, dvv, nv_dev, args,
                         K.st, gate, vpart);
    };
    // initial state: x = 0, r = b, rhat = r
    vop(3, nullptr, VA);
    UFG_TRY(k_finalize_seg(cs, FIN_INIT_B, vpart, vf, vc, nullptr, K));
    UFG_TRY(k_finalize_seg(cs, FIN_INIT_R, vpart, vf, vc, nullptr, K));
    UFG_HIP(hipGetLastError());
    // One check interval of iterations (an even count; every iteration moves p
    // and v to the other buffer, so they are back in their first buffers at
    // every check point), captured once. As in the single-lattice solver, the
    // x, r update of an iteration is merged with the p update of the next one
    // (rho of the next iteration from <rhat, s> - omega <rhat, t>, reduced by
    // the second operator launch), except in the last iteration of the
    // interval, which runs the separate update so that x and r are current at
    // the check point; the first iteration forms p in its operator launch.
    auto body = [&]() -> int {
      for (int k = 0; k < check; ++k) {
        const bool last = (k + 1 == check);
        C2<RI>* pin = pbuf[k & 1];
        C2<RI>* pout = pbuf[(k + 1) & 1];
        C2<RI>* vin = vbuf[k & 1];
        C2<RI>* vout = vbuf[(k + 1) & 1];
        if (k == 0) {
          UFG_TRY(hop(1, 1, pin, pout, vin, vout));
          UFG_TRY(k_finalize_seg(cs, FIN_ALPHA, hpart, hf, hc, K.active, K));
        } else {  // pout was formed by the merged update of the previous iteration
          UFG_TRY(hop(0, 1, pout, nullptr, nullptr, vout));
          UFG_TRY(k_finalize_seg(cs, FIN_ALPHA_XR, hpart, hf, hc, K.active, K, 4, vpart, vf,
                                 vc));
        }
        UFG_TRY(hop(2, last ? 3 : 4, nullptr, nullptr, vout, vt));
        BVecArgs A = VA;
        A.p = pout;
        A.v = vout;
        if (last) {
          UFG_TRY(k_finalize_seg(cs, FIN_OMEGA, hpart, hf, hc, K.active, K));
          vop(9, K.active, A);
          UFG_TRY(k_finalize_seg(cs, FIN_RHO, vpart, vf, vc, K.active, K));
        } else {
          UFG_TRY(k_finalize_seg(cs, FIN_OMEGA_RHO, hpart, hf, hc, K.active, K, 8));
          A.pn = pin;  // the p of the next iteration
          vop(10, K.active, A);
        }
      }
      return UFG_OK;
    };
    // the check point that closes an interval: reliable update (x64 += x_in,
    // r64 = b - A x64, r = r64) and restart, gated per system by its flags
    auto check_point = [&]() -> int {
      vop(4, K.update, VA);
      UFG_TRY(residual(K.update));
      vop(5, K.update, VA);
      UFG_TRY(k_finalize_seg(cs, FIN_UPDATE, vpart, vf, vc, K.update, K));
      vop(6, K.restart, VA);
      UFG_TRY(k_finalize_seg(cs, FIN_RESTART, vpart, vf, vc, K.restart, K));
      return UFG_OK;
    };
    // Whole check intervals, check points included, are captured once: G1
    // holds one interval, GU holds U of them (about g_sync_iters iterations).
    // The work tables and their sizes live in device memory, so compacting
    // them needs no new capture.
    const int U = std::max(1, g_sync_iters / check);
    Graph G1, GU;
    auto capture = [&](Graph& G, int nint) -> int {
      UFG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      int brc = UFG_OK;
      for (int j = 0; j < nint && brc >= 0; ++j) {
        brc = body();
        if (brc >= 0) brc = check_point();
      }
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(cs, &graph);
      G.g = graph;
      UFG_TRY(brc);
      UFG_HIP(ec);
      UFG_HIP(hipGraphInstantiate(&G.e, G.g, nullptr, nullptr, 0));
      return UFG_OK;
    };
    UFG_TRY(capture(G1, 1));
    if (U > 1) UFG_TRY(capture(GU, U));
    int in_tables = S;  // segments the current tables cover
    const int launches = (o.maxit + check - 1) / check;
    bool done = false;
    UFG_HIP(hipMemcpyAsync(hflags.data(), K.active, sizeof(int) * 3 * S, hipMemcpyDeviceToHost, cs));
    UFG_HIP(hipStreamSynchronize(cs));
    n_submit += 4;  // initial vector pass, two finalizes, flag copy
    ++n_sync;
    done = std::all_of(hflags.begin(), hflags.begin() + S, [](int v) { return v == 0; });
    // The host replays U intervals (or single ones for the last, partial
    // stretch before maxit), then reads the flags once. A system stops on the
    // device at its own check point; the host only ends the loop and, once
    // half of the covered systems have stopped, drops them from the work
    // tables so that the tail of the batch launches only the live work.
    UFG_TRY(mirror.ensure(3 * S));
    int n = 0;
    while (n < launches && !done) {
      if (U > 1 && launches - n >= U) {
        UFG_HIP(hipGraphLaunch(GU.e, cs));
        n += U;
        ++n_submit;
      } else {
        const int k = std::min(U, launches - n);
        for (int j = 0; j < k; ++j) UFG_HIP(hipGraphLaunch(G1.e, cs));
        n += k;
        n_submit += k;
      }
      UFG_HIP(hipMemcpyAsync(mirror.host, K.active, sizeof(int) * 3 * S, hipMemcpyDeviceToHost,
                             cs));
      UFG_HIP(hipStreamSynchronize(cs));
      ++n_submit;
      ++n_sync;
      const int* f = mirror.host;
      const int nactive = (int)std::count_if(f, f + S, [](int v) { return v != 0; });
      done = nactive == 0;
      if (!done && 2 * nactive <= in_tables) {
        std::vector<char> live(S);
        for (int s = 0; s < S; ++s) live[s] = f[s] != 0;
        make_tables(live);
        UFG_TRY(upload_tables());
        in_tables = nactive;
      }
    }
    if (in_tables != S) {  // the epilogue runs over every segment
      make_tables(all_segs);
      UFG_TRY(upload_tables());
    }
    vop(4, nullptr, VA);  // final x64 += x_in
    UFG_HIP(hipMemcpyAsync(hst.data(), K.st, sizeof(RhsState) * S, hipMemcpyDeviceToHost, cs));
    UFG_HIP(hipStreamSynchronize(cs));
    n_submit += 2;
    ++n_sync;
    iters_step[step].assign(nprob, 0);
    for (int s = 0; s < S; ++s) {
      const int i = seg_prob[s];
      iters_step[step][i] = std::max(iters_step[step][i], hst[s].iters);
      if (hst[s].status) status[i] = std::max(status[i], hst[s].status);
      else if (!hst[s].conv) status[i] = std::max(status[i], (int)UFG_NOT_CONVERGED);
    }
    // true residuals of this step, FP64
    UFG_TRY(residual(nullptr));
    vop(7, nullptr, VA);
    UFG_TRY(k_finalize_seg(cs, FIN_INIT_B, vpart, vf, vc, nullptr, K));
    vop(8, nullptr, VA);
    UFG_TRY(k_finalize_seg(cs, FIN_NORM, vpart, vf, vc, nullptr, K));
    UFG_HIP(hipMemcpyAsync(hst.data(), K.st, sizeof(RhsState) * S, hipMemcpyDeviceToHost, cs));
    UFG_HIP(hipStreamSynchronize(cs));
    n_submit += (long long)C + 6;
    ++n_sync;
    relres_step[step].assign(nprob, 0.0);
    for (int s = 0; s < S; ++s) {
      const int i = seg_prob[s];
      const double rr = hst[s].b2 > 0 ? std::sqrt(hst[s].r2 / hst[s].b2) : std::sqrt(hst[s].r2);
      if (!(rr <= relres_step[step][i])) relres_step[step][i] = rr;
    }
  }
  int worst = 0;
  for (int i = 0; i < nprob; ++i) {
    worst = std::max(worst, status[i]);
    if (stats) {
      ufg_solve_stats& q = stats[i];
      std::memset(&q, 0, sizeof(q));
      q.iters[0] = iters_step[0][i];
      q.iters[1] = iters_step[1][i];
      q.mv = 2LL * (q.iters[0] + q.iters[1]);
      q.relres[0] = relres_step[0][i];
      q.relres[1] = relres_step[1][i];
      q.relres_normal = -1.0;
      q.paper_mv = 2.0 * (q.iters[0] + q.iters[1]);
      q.status = status[i];
      q.host_syncs = n_sync;
      q.host_submits = n_submit;
    }
  }
  return worst;
}

}  // namespace

int solve_batched_impl(const ufg_lattice* Ls, int nprob, const void* const* b, void* const* x,
                       const int* nrhs, const ufg_precond* p, const ufg_solve_opts* o,
                       ufg_solve_stats* st) {
  UFG_CHECK(Ls && b && x && nrhs && nprob >= 1, "solve_batched: bad arguments");
  UFG_CHECK(o != nullptr, "solve_batched: options are required");
  UFG_CHECK(o->tol > 0 && o->tol < 1 && o->maxit >= 1, "solve_batched: bad tol or maxit");
  UFG_CHECK(o->delta > 0 && o->delta < 1, "solve_batched: delta must be in (0, 1)");
  UFG_CHECK(!o->use_x0, "solve_batched: starts from x = 0");
  UFG_CHECK(!p || p->kind == UFG_PC_NONE, "solve_batched: no preconditioner in batched solves");
  std::vector<Lattice*> L(nprob);
  for (int i = 0; i < nprob; ++i) {
    L[i] = reinterpret_cast<Lattice*>(Ls[i]);
    UFG_CHECK(L[i] != nullptr, "solve_batched: NULL lattice");
    UFG_CHECK(L[i]->dtype == UFG_C128, "solve_batched: lattices must be complex128");
    UFG_CHECK(L[i]->dim == 3, "solve_batched: lattices must be three-dimensional");
    UFG_CHECK(nrhs[i] >= 1, "solve_batched: nrhs must be >= 1");
    UFG_CHECK(b[i] && x[i] && b[i] != x[i], "solve_batched: bad vectors");
    UFG_CHECK(L[i]->device == L[0]->device, "solve_batched: lattices on different devices");
    UFG_HIP(hipStreamSynchronize(L[i]->stream));
  }
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = o->mixed ? run_batched<float>(L, b, x, nrhs, *o, st)
                          : run_batched<double>(L, b, x, nrhs, *o, st);
  if (rc >= 0 && st) {
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < nprob; ++i) st[i].seconds = sec;
  }
  return rc;
}

int batched_tune(int hop_blocks_per_cu, int vec_blocks_per_cu, long long chunk, int slab,
                 int sync_iters) {
  UFG_CHECK(hop_blocks_per_cu >= 0 && hop_blocks_per_cu <= 64, "bad hop blocks per CU");
  UFG_CHECK(vec_blocks_per_cu >= 0 && vec_blocks_per_cu <= 64, "bad vector blocks per CU");
  UFG_CHECK(chunk == 0 || (chunk >= 256 && chunk <= (1 << 22)), "bad chunk");
  UFG_CHECK(slab >= 0 && slab <= 64, "bad slab");
  UFG_CHECK(sync_iters >= 0 && sync_iters <= 100000, "bad iterations per host check");
  g_hop_blocks_per_cu = hop_blocks_per_cu ? hop_blocks_per_cu : 4;
  g_vec_blocks_per_cu = vec_blocks_per_cu ? vec_blocks_per_cu : 8;
  g_chunk = chunk ? chunk : 4096;
  g_bop_slab = slab ? slab : 2;
  g_sync_iters = sync_iters ? sync_iters : 200;
  return UFG_OK;
}

}  // namespace ufg
