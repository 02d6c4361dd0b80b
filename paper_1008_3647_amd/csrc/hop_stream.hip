// Streaming slice operator for M and M^T (paper, Sec. 1, Eq. MatrixM) on gfx950.
//
// One workgroup owns a slab of S consecutive time slices of one right-hand
// side and walks it in the direction that reuses loads: upwards for M (output
// t reads source t-1), downwards for M^T (output t reads source t+1). The
// slice loaded for the identity term of output t is the source of the next
// output, so every input slice of the slab is loaded once; only one halo
// slice per slab is loaded twice (at two slices per slab the L2 misses come to
// about 1.2 times the algorithmic bytes).
//
// Workgroup numbering (see stream_item): by default consecutive slabs are
// gathered into groups of G that go round-robin to the eight XCDs, and each
// XCD walks its groups right-hand side by right-hand side. Every rhs of a slab
// then runs on the same XCD (the field slab is read from HBM once), the halo
// slice of a slab is the last slice of the previous slab on the same XCD
// (except at group edges), and the workgroups resident at any moment cover one
// contiguous address window of each vector. The earlier numbering, contiguous
// runs of (slab, rhs) pairs per XCD with the rhs fastest (G = 0), spreads the
// resident workgroups over the eight rhs blocks of every vector.
//
// exp(-tau K) along one axis is the symmetric circulant T. T commutes with the
// reflections i -> -i and i -> Nx/2 - i (mod Nx), so in the basis of their
// joint eigenvectors (built by two levels of add/subtract butterflies) T is
// block diagonal with blocks of sizes Nx/4+1, Nx/4, Nx/4, Nx/4-1. A line of Nx
// values then costs 4 (Nx-2) additions for the butterflies and sum(block^2)
// multiply-adds (56 + 66 for Nx = 16) instead of Nx^2 = 256 multiply-adds.
//
// Memory access: raw buffer instructions with one resource per array (base =
// the rhs block), the lane offset in a VGPR and the slice / z offset in an
// SGPR, so a z-line costs no 64-bit address arithmetic. The operands of an
// output slice (field, aux, reduction weights) are loaded before its stores
// start, because loads cannot be moved across buffer stores.
//
// Fused BiCGStab sources: the kernel can build its source on the fly from the
// Krylov vectors (p = r + beta (p_old - omega v_old), or s = r - alpha v) so
// that BiCGStab's vector updates ride on the operator's memory stream, and
// reduce FP64 dot products of its output, its source and a weight vector into
// one partial per workgroup.
#include "hop_stream.h"
#include "krylov.h"
#include "krylov_fin.h"
#include "split_line.h"

namespace ufg {
namespace {
using namespace splitk;

// LDS slot of element (row, col) of a slice stored as NX*NX rows of NX:
// power-of-two NX uses an XOR swizzle (no padding), else one pad column.
template <int NX>
__device__ __forceinline__ int lds_at(int row, int col) {
  if constexpr ((NX & (NX - 1)) == 0)
    return row * NX + (col ^ (row & (NX - 1)));
  else
    return row * (NX + 1) + col;
}
template <int NX>
constexpr int lds_slice_elems() {
  return ((NX & (NX - 1)) == 0) ? NX * NX * NX : NX * NX * (NX + 1);
}

// T^3 of the slice held as z-lines in v (thread (y, x)); result left in v.
// Barriers: stage 1 (thread (y, x) writes its z-line) feeds the y-lines of
// other waves, and the x-lines feed the z-lines of other waves. The y-lines
// (z, x) and x-lines (z, y) of one z-plane belong to the same NX consecutive
// threads, which sit in one wave when NX divides 64: there a wave-level
// ordering point replaces the block barrier. Each thread's last read and its
// next first write touch only its own z-line, so no barrier guards the reuse
// of the buffer by the next slice.
// MODE 0: T (positions -> positions); 1: U^T (positions -> block-ordered
// modes); 2: U (modes -> positions). The same three passes serve all three.
template <int MODE, typename R, int NX>
__device__ __forceinline__ void line_op(const SplitCoef<R, NX>& c, C2<R> (&v)[NX]) {
  if constexpr (MODE == 0)
    split_line<R, NX>(c, v);
  else if constexpr (MODE == 1)
    modes_fwd<R, NX>(c, v);
  else
    modes_bwd<R, NX>(c, v);
}

template <typename R, int NX, int MODE = 0, bool KEEP = false>
__device__ __forceinline__ void slice_T3(const SplitCoef<R, NX>& c, C2<R>* lds, int l,
                                         C2<R> (&v)[NX]) {
  const int y = l / NX, x = l - (l / NX) * NX;
  line_op<MODE, R, NX>(c, v);  // along z
#pragma unroll
  for (int z = 0; z < NX; ++z) lds[lds_at<NX>(z * NX + y, x)] = v[z];
  __syncthreads();
  C2<R> w[NX];
  {
    const int z = l / NX, xx = l - (l / NX) * NX;
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) w[yy] = lds[lds_at<NX>(z * NX + yy, xx)];
    line_op<MODE, R, NX>(c, w);  // along y
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) lds[lds_at<NX>(z * NX + yy, xx)] = w[yy];
  }
  if constexpr (64 % NX == 0) {
    // LDS operations of one wave are performed in order; the fences keep the
    // compiler from moving the reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
  {
    const int z = l / NX, yy = l - (l / NX) * NX;
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) w[xx] = lds[lds_at<NX>(z * NX + yy, xx)];
    line_op<MODE, R, NX>(c, w);  // along x
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) lds[lds_at<NX>(z * NX + yy, xx)] = w[xx];
  }
  __syncthreads();
  if (KEEP) return;  // the result stays in LDS: z-line of thread (y, x) at lds_at(z NX + y, x)
#pragma unroll
  for (int z = 0; z < NX; ++z) v[z] = lds[lds_at<NX>(z * NX + y, x)];
}

// The y and x stages of T^3 as 16x16x4 FP32 MFMA contractions (Nx = 16,
// complex64; lattice_tune_transform route 1). A wave owns z-planes 4w..4w+3,
// as in the VALU stages. For one plane and axis, the lines of the plane form
// the 16 columns of B and T the 16x16 A operand: lane holds
// ta[s] = T[lane % 16][4 s + lane / 16] for k-block s, and B[k][c] = the
// plane's element k of line c (real and imaginary parts separately); the
// product lands as D[4 (lane / 16) + j][lane % 16], element 4 (lane / 16) + j
// of line lane % 16. AX = 1: lines along y (c = x); AX = 0: along x (c = y).
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int AX>
__device__ __forceinline__ void stage_mfma16(const float (&ta)[4], float2* lds, int l) {
  constexpr int NX = 16;
  const int w = l >> 6, lane = l & 63, g = lane >> 4, cc = lane & 15;
#pragma unroll
  for (int zz = 0; zz < 4; ++zz) {
    const int z = 4 * w + zz;
    f32x4 dre = {0.f, 0.f, 0.f, 0.f}, dim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + g;
      const float2 v = AX == 0 ? lds[lds_at<NX>(z * NX + cc, k)] : lds[lds_at<NX>(z * NX + k, cc)];
      dre = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[s], v.x, dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[s], v.y, dim, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = 4 * g + j;
      const float2 r = make_float2(dre[j], dim[j]);
      if (AX == 0)
        lds[lds_at<NX>(z * NX + cc, o)] = r;
      else
        lds[lds_at<NX>(z * NX + o, cc)] = r;
    }
  }
}

// slice_T3 with the y and x stages on MFMA (z stays on the VALU, in registers);
// the result stays in LDS as for slice_T3<..., KEEP = true>.
__device__ __forceinline__ void slice_T3_mfma16(const SplitCoef<float, 16>& c,
                                                const float (&ta)[4], float2* lds, int l,
                                                float2 (&v)[16]) {
  constexpr int NX = 16;
  const int y = l / NX, x = l - (l / NX) * NX;
  split_line<float, NX>(c, v);  // along z
#pragma unroll
  for (int z = 0; z < NX; ++z) lds[lds_at<NX>(z * NX + y, x)] = v[z];
  __syncthreads();
  stage_mfma16<1>(ta, lds, l);  // along y: planes of this wave only
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  stage_mfma16<0>(ta, lds, l);  // along x
  __syncthreads();
}

// T^3 through Fourier transforms (complex64, Nx = 16; lattice_tune_transform
// route 2): T is a symmetric circulant, so along each axis T = F^-1 diag(lam) F
// with F the 16-point DFT and lam_k = sum_j T_0j cos(2 pi j k / 16). Each
// stage is a forward DFT of the line, the scaling by lam_k / 16 and an
// inverse DFT, the DFT in radix 4 x 4 (index n = 4 n1 + n2, k = k1 + 4 k2:
// 4-point DFTs over n1, twiddles W^(n2 k1), 4-point DFTs over n2).
template <int M, bool INV>
__device__ __forceinline__ float2 twiddle16(float2 a) {
  // a * exp(-+2 pi i M / 16) (INV: +)
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f,
                  r2 = 0.70710678118654752f;
  constexpr float cs[10] = {1.f, c1, r2, s1, 0.f, -s1, -r2, -c1, -1.f, -c1};
  constexpr float sn[10] = {0.f, s1, r2, c1, 1.f, c1, r2, s1, 0.f, -s1};
  if constexpr (M == 0) {
    return a;
  } else if constexpr (M == 4) {  // -i (forward) or +i (inverse)
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else if constexpr (M == 8) {
    return make_float2(-a.x, -a.y);
  } else {
    const float c = cs[M], sg = INV ? sn[M] : -sn[M];
    return make_float2(a.x * c - a.y * sg, a.x * sg + a.y * c);
  }
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = make_float2(a0.x + a2.x, a0.y + a2.y);
  const float2 t1 = make_float2(a0.x - a2.x, a0.y - a2.y);
  const float2 t2 = make_float2(a1.x + a3.x, a1.y + a3.y);
  const float2 t3 = make_float2(a1.x - a3.x, a1.y - a3.y);
  a0 = make_float2(t0.x + t2.x, t0.y + t2.y);
  a2 = make_float2(t0.x - t2.x, t0.y - t2.y);
  // forward: A1 = t1 - i t3, A3 = t1 + i t3 (inverse: the other way round)
  const float2 m = make_float2(t1.x + t3.y, t1.y - t3.x);
  const float2 p = make_float2(t1.x - t3.y, t1.y + t3.x);
  a1 = INV ? p : m;
  a3 = INV ? m : p;
}

template <bool INV>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
  float2 y[16];  // y[4 n2 + k1]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
    dft4<INV>(a0, a1, a2, a3);
    y[4 * n2 + 0] = a0;
    y[4 * n2 + 1] = a1;
    y[4 * n2 + 2] = a2;
    y[4 * n2 + 3] = a3;
  }
  y[5] = twiddle16<1, INV>(y[5]);
  y[6] = twiddle16<2, INV>(y[6]);
  y[7] = twiddle16<3, INV>(y[7]);
  y[9] = twiddle16<2, INV>(y[9]);
  y[10] = twiddle16<4, INV>(y[10]);
  y[11] = twiddle16<6, INV>(y[11]);
  y[13] = twiddle16<3, INV>(y[13]);
  y[14] = twiddle16<6, INV>(y[14]);
  y[15] = twiddle16<9, INV>(y[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = y[k1], a1 = y[4 + k1], a2 = y[8 + k1], a3 = y[12 + k1];
    dft4<INV>(a0, a1, a2, a3);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

__device__ __forceinline__ void fft_line16(const float (&lam)[16], float2 (&v)[16]) {
  dft16<false>(v);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k].x *= lam[k];
    v[k].y *= lam[k];
  }
  dft16<true>(v);
}

// lam_k / 16 from the first row of T (row-major Nx x Nx on the device).
__device__ __forceinline__ void fft_lambda16(const float* __restrict__ T, float (&lam)[16]) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f,
                  r2 = 0.70710678118654752f;
  constexpr float cs[16] = {1.f, c1, r2, s1, 0.f, -s1, -r2, -c1,
                            -1.f, -c1, -r2, -s1, 0.f, s1, r2, c1};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc = fmaf(T[j], cs[(j * k) & 15], acc);
    lam[k] = acc * (1.f / 16.f);
  }
}

// slice_T3<float, 16, 0, true> with each line through fft_line16.
__device__ __forceinline__ void slice_T3_fft16(const float (&lam)[16], float2* lds, int l,
                                               float2 (&v)[16]) {
  constexpr int NX = 16;
  const int y = l / NX, x = l - (l / NX) * NX;
  fft_line16(lam, v);  // along z
#pragma unroll
  for (int z = 0; z < NX; ++z) lds[lds_at<NX>(z * NX + y, x)] = v[z];
  __syncthreads();
  float2 w[NX];
  {
    const int z = l / NX, xx = l - (l / NX) * NX;
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) w[yy] = lds[lds_at<NX>(z * NX + yy, xx)];
    fft_line16(lam, w);  // along y
#pragma unroll
    for (int yy = 0; yy < NX; ++yy) lds[lds_at<NX>(z * NX + yy, xx)] = w[yy];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  {
    const int z = l / NX, yy = l - (l / NX) * NX;
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) w[xx] = lds[lds_at<NX>(z * NX + yy, xx)];
    fft_line16(lam, w);  // along x
#pragma unroll
    for (int xx = 0; xx < NX; ++xx) lds[lds_at<NX>(z * NX + yy, xx)] = w[xx];
  }
  __syncthreads();
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
    q.br = R(s.beta.x);  // beta = (rho / rho_old)(alpha / omega), set by the finalize
    q.bi = R(s.beta.y);
    q.wr = R(s.omega.x);
    q.wi = R(s.omega.y);
  } else {
    q.ar = R(s.alpha.x);
    q.ai = R(s.alpha.y);
  }
  return q;
}

// Raw buffer access: one 128-bit resource per array (base = the rhs block),
// a 32-bit lane offset in a VGPR and the slice / z offset in an SGPR.
// Out-of-range accesses are dropped by the hardware (loads return 0).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer, 32-bit data format
constexpr int kAuxNT = 2;               // non-temporal

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kRsrcWord3);
}

template <typename R, int AUX = 0>
__device__ __forceinline__ C2<R> bload(__amdgpu_buffer_rsrc_t rs, int vo, int so) {
  if constexpr (sizeof(R) == 4) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, AUX);
    return __builtin_bit_cast(C2<R>, v);
  } else {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, AUX);
    return __builtin_bit_cast(C2<R>, v);
  }
}

// Store of one element at byte offset so + vo from base (rsrc describes the
// same block). 16-byte elements go through a FLAT store: the compiler's
// wait-state handling for a VALU overwrite of store-data registers does not
// cover buffer stores with an SGPR offset, and 128-bit buffer stores were
// seen to write registers already overwritten by the next instruction.
template <typename R, bool NT>
__device__ __forceinline__ void bstore(C2<R> v, C2<R>* base, __amdgpu_buffer_rsrc_t rs, int vo,
                                       int so) {
  if constexpr (sizeof(R) == 4) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, vo, so,
                                          NT ? kAuxNT : 0);
  } else {
    C2<R>* p = reinterpret_cast<C2<R>*>(reinterpret_cast<char*>(base) + so + vo);
    if (NT) {
      __builtin_nontemporal_store(v.x, &p->x);
      __builtin_nontemporal_store(v.y, &p->y);
    } else {
      *p = v;
    }
  }
}

template <typename R>
__device__ __forceinline__ R bload_real(__amdgpu_buffer_rsrc_t rs, int vo, int so) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
  } else {
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
  }
}

struct Rsrc {
  __amdgpu_buffer_rsrc_t src, fr, fp, fv, fpnew, dst, aux, rw, pre, post;
};

// z-line of the source slice at byte offset so (uniform); vo = lane byte offset.
// AUX: cache policy of the loads (kAuxNT for slices that no other workgroup reads).
template <typename R, int NX, int SRC, int AUX>
__device__ __forceinline__ void load_source(const Rsrc& b, const SrcScal<R>& q, int so, int vo,
                                            C2<R> (&X)[NX]) {
  constexpr int ZB = NX * NX * (int)sizeof(C2<R>);
#pragma unroll
  for (int z = 0; z < NX; ++z) {
    const int s = so + z * ZB;
    if (SRC == 0) {
      X[z] = bload<R, AUX>(b.src, vo, s);
    } else if (SRC == 1) {
      const C2<R> rv = bload<R, AUX>(b.fr, vo, s), pv = bload<R, AUX>(b.fp, vo, s),
                  vv = bload<R, AUX>(b.fv, vo, s);
      const R dx = pv.x - (q.wr * vv.x - q.wi * vv.y);
      const R dy = pv.y - (q.wr * vv.y + q.wi * vv.x);
      X[z].x = rv.x + q.br * dx - q.bi * dy;
      X[z].y = rv.y + q.br * dy + q.bi * dx;
    } else {
      const C2<R> rv = bload<R, AUX>(b.fr, vo, s), vv = bload<R, AUX>(b.fv, vo, s);
      X[z].x = rv.x - (q.ar * vv.x - q.ai * vv.y);
      X[z].y = rv.y - (q.ar * vv.y + q.ai * vv.x);
    }
  }
}

// z-line of a real field slice times X (in place).
template <typename R, int NX>
__device__ __forceinline__ void scale_field(__amdgpu_buffer_rsrc_t f, int so, int vo,
                                            C2<R> (&X)[NX]) {
  constexpr int ZB = NX * NX * (int)sizeof(R);
#pragma unroll
  for (int z = 0; z < NX; ++z) {
    const R fz = bload_real<R>(f, vo, so + z * ZB);
    X[z].x *= fz;
    X[z].y *= fz;
  }
}

// Block -> (rhs r, slab sb); false if the block has no item (it exits).
// xg = 0: contiguous runs of (slab, rhs) per XCD, rhs fastest (grid nslab*nrhs).
// xg > 0: slab groups of xg go round-robin to the XCDs (blocks are dispatched
// to XCD blockIdx % 8); the q-th block of XCD j takes item q of the list
// "for r: for the slabs of XCD j's groups" (ri = 0) or "for XCD j's groups:
// for r: for the group's slabs" (ri = 1); grid stream_grid().
__device__ __forceinline__ bool stream_item(int nslab, int nrhs, int xg, int ri, int& r,
                                            int& sb) {
  const int b = blockIdx.x;
  if (xg <= 0) {
    const int full = (int)gridDim.x & ~7;
    int lid = b;
    if (lid < full) lid = (lid & 7) * (full >> 3) + (lid >> 3);
    r = lid % nrhs;
    sb = lid / nrhs;
    return true;
  }
  const int j = b & 7, q = b >> 3;
  if (ri) {
    const int per = nrhs * xg;  // blocks per group
    const int m = q / per, k = q - m * per;
    r = k / xg;
    sb = (8 * m + j) * xg + (k - r * xg);
    return sb < nslab;
  }
  const int F = nslab / xg, rem = nslab - F * xg;  // full groups, slabs of the partial one
  int nj = xg * (F / 8 + ((j < (F & 7)) ? 1 : 0));
  if (rem > 0 && (F & 7) == j) nj += rem;
  if (q >= nrhs * nj) return false;
  r = q / nj;
  const int k = q - r * nj;
  sb = (k / xg) * 8 * xg + j * xg + (k % xg);
  return true;
}

// Where the transform reads the blocks of T (or U) from. The Nx = 16 blocks
// are 66 numbers. In FP64 (132 SGPRs) they exceed the scalar register file and
// the compiler spills them to VGPR lanes (a v_readlane before each use); with
// IN_LDS the workgroup copies them into LDS once and the transform reads them
// from there (broadcast reads). Measured per kernel: the fused FP64 M-type
// operator (t = A s: 227 -> 206 us), the FP64 basis changes and both
// precisions of basis_pair_kernel (two sets) gain; the plain FP64 operator (103
// -> 122 us), the M^T-type fused ones and every complex64 operator keep the
// kernel-argument copy.
template <bool IN_LDS, typename R, int NX>
using CoefSlot = typename std::conditional<IN_LDS, SplitCoef<R, NX>, char>::type;

template <bool IN_LDS, typename R, int NX>
__device__ __forceinline__ const SplitCoef<R, NX>* coef_copy(const SplitCoef<R, NX>& c,
                                                            CoefSlot<IN_LDS, R, NX>* lds_slot) {
  if constexpr (IN_LDS) {
    constexpr int NC = sizeof(SplitCoef<R, NX>) / sizeof(R);
    for (int i = threadIdx.x; i < NC; i += blockDim.x)
      reinterpret_cast<R*>(lds_slot)[i] = reinterpret_cast<const R*>(&c)[i];
    __syncthreads();
    return lds_slot;
  } else {
    return &c;
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// DIR = -1: M-type, output t reads source t-1; the slab is walked upwards.
// DIR = +1: M^T-type, output t reads source t+1; the slab is walked downwards.
// Either way the slice loaded for the identity term of output t is the source
// of the next output: each thread holds one z-line X (current source) in
// registers, and the transform of the previous source stays in the LDS slice,
// from which the output phase reads the thread's own z-line.
// TR = 1: the transform's y and x stages on MFMA (complex64, Nx = 16, plain
// operator only; see slice_T3_mfma16); TR = 2: every stage through 16-point
// DFTs (same restriction; see slice_T3_fft16).
template <typename R, int NX, int DIR, bool GENERAL, int SRC, int RED, int TR = 0>
__global__ void __launch_bounds__(NX * NX)
    hop_stream_kernel(HopArgs<R> a, SplitCoef<R, NX> c, int ntau, int nslab, int xg, int ri) {
  static_assert(TR == 0 || (sizeof(R) == 4 && NX == 16 && SRC == 0 && RED == 0 && !GENERAL),
                "the MFMA and DFT transform routes exist for the plain complex64 Nx = 16 "
                "operator");
  constexpr int P = NX * NX, V = NX * NX * NX;
  constexpr int ES = sizeof(C2<R>), FS = sizeof(R);
  // Single-use operand slices are loaded non-temporal (measured: faster for
  // every complex64 variant and the fused complex128 ones, slower for the
  // plain complex128 operator, which keeps the default policy).
  constexpr int kNTA = (sizeof(R) == 4 || SRC != 0 || RED != 0) ? kAuxNT : 0;
  // plain complex64 operator: the first output slice's source (and, for M^T,
  // its field) is loaded together with the halo, before the halo's transform
  // (one more z-line of registers; the fused variants would lose a wave per
  // SIMD to it)
  constexpr bool EARLY = sizeof(R) == 4 && SRC == 0 && RED == 0 && !GENERAL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* lds = reinterpret_cast<C2<R>*>(smem_raw);

  int r, sb;
  if (!stream_item(nslab, a.nrhs, xg, ri, r, sb)) return;
  // M^T walks time downwards: with slab groups the XCD takes its slabs in
  // decreasing order, so a slab's halo (the next slab) was loaded first
  if (DIR > 0 && xg > 0) sb = nslab - 1 - sb;
  if (a.gate && a.gate[r] == 0) return;
  constexpr bool kCoefLds = sizeof(R) == 8 && DIR < 0 && (SRC != 0 || RED != 0);
  __shared__ CoefSlot<kCoefLds, R, NX> coef_lds[1];
  const SplitCoef<R, NX>& cc = *coef_copy<kCoefLds, R, NX>(c, coef_lds);

  const int l = threadIdx.x;
  float ta[TR == 1 ? 4 : 1];
  if constexpr (TR == 1) {
    const int lane = l & 63;
#pragma unroll
    for (int j = 0; j < 4; ++j) ta[j] = float(a.mat[(lane & 15) * NX + 4 * j + (lane >> 4)]);
  }
  float lam[TR == 2 ? 16 : 1];
  if constexpr (TR == 2) fft_lambda16(a.mat, lam);
  const int t0 = (int)((long long)sb * ntau / nslab);
  const int t1 = (int)((long long)(sb + 1) * ntau / nslab);  // exclusive
  const long long rbase = (long long)r * ntau * V;
  const unsigned vbytes = (unsigned)ntau * V * ES;
  const unsigned fbytes = (unsigned)ntau * V * FS;
  Rsrc b;
  b.src = make_rsrc(a.src + rbase, vbytes);
  b.fr = make_rsrc(a.fr + rbase, vbytes);
  b.fp = make_rsrc(a.fp + rbase, vbytes);
  b.fv = make_rsrc(a.fv + rbase, vbytes);
  b.fpnew = make_rsrc(a.fpnew + rbase, vbytes);
  b.dst = make_rsrc(a.dst + rbase, vbytes);
  b.aux = make_rsrc(a.aux + rbase, vbytes);
  b.rw = make_rsrc(a.red_w + rbase, vbytes);
  b.pre = make_rsrc(a.pre, fbytes);
  b.post = make_rsrc(a.post, fbytes);
  const int vo = l * ES, fo = l * FS;
  SrcScal<R> q = src_scalars<R, SRC>(a, r);
  if constexpr (SRC == 2 && RED == 4) {
    if (a.fin_part) {  // the alpha step of the rhs state, see HopArgs
      // thread 0 fetches the state and flags while every thread sums partials
      RhsState* st = reinterpret_cast<RhsState*>(const_cast<void*>(a.st));
      int* fl = a.fin_flags;
      RhsState qs{};
      int act = 0, upd = 0, rst = 0;
      if (l == 0) {
        qs = st[r];
        act = fl[r];
        upd = fl[a.nrhs + r];
        rst = fl[2 * a.nrhs + r];
      }
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = 0.0;
      for (int bi = l; bi < a.fin_nblk; bi += P) {
        const double* pp = a.fin_part + ((long long)r * a.fin_nblk + bi) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] += pp[j];
      }
      for (int bi = l; bi < a.fin_nblk2; bi += P) {
        const double* pp = a.fin_part2 + ((long long)r * a.fin_nblk2 + bi) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 + j] += pp[j];
      }
      constexpr int NW = (P + 63) / 64;
      double* sm = reinterpret_cast<double*>(smem_raw);
      const int lane = l & 63, wid = l >> 6;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double w = wsum(v[j]);
        if (lane == 0) sm[wid * 8 + j] = w;
      }
      __syncthreads();
      if (l == 0) {
        double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < NW; ++w)
#pragma unroll
          for (int j = 0; j < 8; ++j) s8[j] += sm[w * 8 + j];
        apply_fin(FIN_ALPHA_XR, s8, qs, act, upd, rst, a.fin_prm);
        if (sb == 0) {
          st[r] = qs;
          fl[r] = act;
          fl[a.nrhs + r] = upd;
          fl[2 * a.nrhs + r] = rst;
        }
        sm[NW * 8] = qs.alpha.x;
        sm[NW * 8 + 1] = qs.alpha.y;
        sm[NW * 8 + 2] = act ? 1.0 : 0.0;
      }
      __syncthreads();
      const double alx = sm[NW * 8], aly = sm[NW * 8 + 1];
      const bool live = sm[NW * 8 + 2] != 0.0;
      __syncthreads();  // the LDS slice is written next
      if (!live) return;
      q.ar = R(alx);
      q.ai = R(aly);
    }
  }
  const int count = t1 - t0;
  // first output slice, step, and the halo slice that feeds it
  const int tfirst = (DIR < 0) ? t0 : t1 - 1;
  const int step = (DIR < 0) ? 1 : -1;
  const int th = (DIR < 0) ? ((t0 == 0) ? ntau - 1 : t0 - 1) : ((t1 == ntau) ? 0 : t1);

  double acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0, acc4 = 0, acc5 = 0, acc6 = 0, acc7 = 0;
  // X: the z-line of the current source slice. The T^3 of the previous one
  // stays in the LDS slice (each thread reads back only its own z-line, which
  // is also the first thing it writes in the next transform).
  C2<R> X[NX];
  C2<R> Y[EARLY ? NX : 1];
  const int ly = l / NX, lx = l - (l / NX) * NX;
  load_source<R, NX, SRC, 0>(b, q, th * V * ES, vo, X);
  R F0[EARLY && DIR > 0 ? NX : 1];
  if constexpr (EARLY) {
    if (count > 1)
      load_source<R, NX, SRC, kNTA>(b, q, tfirst * V * ES, vo, Y);
    else
      load_source<R, NX, SRC, 0>(b, q, tfirst * V * ES, vo, Y);
    if constexpr (DIR > 0) {  // and its output field
#pragma unroll
      for (int z = 0; z < NX; ++z)
        F0[z] = bload_real<R>(b.post, fo, tfirst * V * FS + z * P * FS);
    }
  }
  // plain complex64 operator: once its loads are issued, the workgroup runs
  // the transform and the output at raised wave priority, so that the
  // workgroups started earlier finish (and free their slots) first (measured:
  // apply_Mdag 45.9 -> 43.6 us, apply_M unchanged; the fused and complex128
  // variants ran slower that way)
  if constexpr (EARLY) __builtin_amdgcn_s_setprio(2);
  if (DIR < 0) scale_field<R, NX>(b.pre, th * V * FS, fo, X);
  if constexpr (TR == 1)
    slice_T3_mfma16(cc, ta, lds, l, X);
  else if constexpr (TR == 2)
    slice_T3_fft16(lam, lds, l, X);
  else
    slice_T3<R, NX, 0, true>(cc, lds, l, X);
  for (int k = 0; k < count; ++k) {
    const int t = tfirst + k * step;
    const int so = t * V * ES;  // slice byte offset (uniform)
    // the last slice of the slab is the halo of the neighbouring slab: it
    // stays cacheable, the others are streamed
    bool have = false;
    if constexpr (EARLY) {
      if (k == 0) {
#pragma unroll
        for (int z = 0; z < NX; ++z) X[z] = Y[z];
        have = true;
      }
    }
    if (!have) {
      if (k + 1 < count)
        load_source<R, NX, SRC, kNTA>(b, q, so, vo, X);
      else
        load_source<R, NX, SRC, 0>(b, q, so, vo, X);
    }
    if (SRC == 1) {
#pragma unroll
      for (int z = 0; z < NX; ++z) bstore<R, false>(X[z], a.fpnew + rbase, b.fpnew, vo, so + z * P * ES);
    }
    // sign of the block that connects the source slice to slice t
    R sgn;
    if (DIR < 0)
      sgn = (t == 0) ? R(1) : R(-1);
    else
      sgn = (t == ntau - 1) ? R(1) : R(-1);
    // The output slice is written in chunks of ZC z-planes; the operands of a
    // chunk (field, aux, reduction weights) are loaded ahead of its stores
    // (loads cannot be moved across buffer stores). complex128 with a
    // reduction uses half-slice chunks to stay within the register file.
    constexpr int ZC = (sizeof(R) == 8 && (GENERAL || RED != 0)) ? NX / 2 : NX;
#pragma unroll
    for (int z0 = 0; z0 < NX; z0 += ZC) {
      R F[DIR > 0 ? ZC : 1];
      if (DIR > 0) {  // M^T-type: the field multiplies the output slice
        if (EARLY && k == 0) {
#pragma unroll
          for (int j = 0; j < ZC; ++j) F[j] = sgn * F0[EARLY && DIR > 0 ? z0 + j : 0];
        } else {
#pragma unroll
          for (int j = 0; j < ZC; ++j)
            F[j] = sgn * bload_real<R>(b.post, fo, t * V * FS + (z0 + j) * P * FS);
        }
      }
      C2<R> U[GENERAL ? ZC : 1];
      if (GENERAL && a.aux) {
#pragma unroll
        for (int j = 0; j < ZC; ++j) U[j] = bload<R, kNTA>(b.aux, vo, so + (z0 + j) * P * ES);
      }
      C2<R> Wr[(RED == 1 || RED == 2 || RED == 4) ? ZC : 1];
      if (RED == 1 || RED == 2 || RED == 4) {
#pragma unroll
        for (int j = 0; j < ZC; ++j) Wr[j] = bload<R, kNTA>(b.rw, vo, so + (z0 + j) * P * ES);
      }
#pragma unroll
      for (int j = 0; j < ZC; ++j) {
        const int z = z0 + j;
        const int s = so + z * P * ES;
        const C2<R> id = X[z];
        const C2<R> wz = lds[lds_at<NX>(z * NX + ly, lx)];
        C2<R> base;
        const R f = (DIR > 0) ? F[DIR > 0 ? j : 0] : sgn;
        base.x = f * wz.x;
        base.y = f * wz.y;
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
            const C2<R> u = U[GENERAL ? j : 0];
            const R br = R(a.beta.x), bi = R(a.beta.y);
            out.x += br * u.x - bi * u.y;
            out.y += br * u.y + bi * u.x;
          }
        }
        // streaming store: y is not re-read by this launch, keep L2 for the
        // halo slices and the field
        bstore<R, true>(out, a.dst + rbase, b.dst, vo, s);
        if (RED == 1) {  // <w, out>
          const C2<R> u = Wr[RED == 1 ? j : 0];
          acc0 += double(u.x) * out.x + double(u.y) * out.y;
          acc1 += double(u.x) * out.y - double(u.y) * out.x;
        } else if (RED == 2) {  // <out, w>, |out|^2, |w|^2
          const C2<R> u = Wr[RED == 2 ? j : 0];
          acc0 += double(out.x) * u.x + double(out.y) * u.y;
          acc1 += double(out.x) * u.y - double(out.y) * u.x;
          acc2 += double(out.x) * out.x + double(out.y) * out.y;
          acc3 += double(u.x) * u.x + double(u.y) * u.y;
        } else if (RED == 3 || RED == 4) {  // <out, source>, |out|^2, |source|^2
          acc0 += double(out.x) * id.x + double(out.y) * id.y;
          acc1 += double(out.x) * id.y - double(out.y) * id.x;
          acc2 += double(out.x) * out.x + double(out.y) * out.y;
          acc3 += double(id.x) * id.x + double(id.y) * id.y;
          if (RED == 4) {  // <w, out>, <w, source>
            const C2<R> u = Wr[RED == 4 ? j : 0];
            acc4 += double(u.x) * out.x + double(u.y) * out.y;
            acc5 += double(u.x) * out.y - double(u.y) * out.x;
            acc6 += double(u.x) * id.x + double(u.y) * id.y;
            acc7 += double(u.x) * id.y - double(u.y) * id.x;
          }
        }
      }
    }
    if (RED != 0) {
      // the reductions of this slice are complete here: without this point the
      // compiler sinks them below the next transform and keeps the slice's
      // operands live across it
      asm volatile("" ::"v"(acc0), "v"(acc1), "v"(acc2), "v"(acc3));
      if (RED == 4) asm volatile("" ::"v"(acc4), "v"(acc5), "v"(acc6), "v"(acc7));
    }
    if (k + 1 < count) {
      // transform source slice t for the next output slice
      if (DIR < 0) scale_field<R, NX>(b.pre, t * V * FS, fo, X);
      if constexpr (TR == 1)
        slice_T3_mfma16(cc, ta, lds, l, X);
      else if constexpr (TR == 2)
        slice_T3_fft16(lam, lds, l, X);
      else
        slice_T3<R, NX, 0, true>(cc, lds, l, X);
    }
  }
  if (RED != 0) {
    constexpr int NR = (RED == 4) ? 8 : 4;
    double acc[NR];
    acc[0] = wsum(acc0);
    acc[1] = wsum(acc1);
    acc[2] = wsum(acc2);
    acc[3] = wsum(acc3);
    if (RED == 4) {
      acc[NR - 4] = wsum(acc4);
      acc[NR - 3] = wsum(acc5);
      acc[NR - 2] = wsum(acc6);
      acc[NR - 1] = wsum(acc7);
    }
    __syncthreads();
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < NR; ++j) sm[wid * NR + j] = acc[j];
    }
    __syncthreads();
    if (threadIdx.x < NR) {
      const int j = threadIdx.x;
      double v = 0;
      for (int w = 0; w < (P + 63) / 64; ++w) v += sm[w * NR + j];
      a.red_out[((long long)r * nslab + sb) * NR + j] = v;
    }
  }
}

template <typename R, int NX, int DIR, bool GENERAL, int SRC, int RED, int TR = 0>
int launch_one(const Lattice& L, const HopArgs<R>& a, const SplitCoef<R, NX>& c, dim3 grid,
               size_t lds, int nslab) {
  static bool attr = false;
  if (!attr) {
    UFG_HIP(hipFuncSetAttribute((const void*)hop_stream_kernel<R, NX, DIR, GENERAL, SRC, RED, TR>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((hop_stream_kernel<R, NX, DIR, GENERAL, SRC, RED, TR>), grid, dim3(NX * NX),
                     lds, L.stream, a, c, L.ntau, nslab, stream_group(L), stream_inner(L));
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R, int NX, int DIR>
int launch_dir(const Lattice& L, const HopArgs<R>& a, const SplitCoef<R, NX>& c) {
  const int nslab = stream_nslab(L);
  const size_t lds = size_t(lds_slice_elems<NX>()) * sizeof(C2<R>);
  const bool general = (a.alpha.x != 1.0 || a.alpha.y != 0.0 || a.aux != nullptr);
  const dim3 grid(stream_grid(L, a.nrhs));
  // instantiated combinations: plain apply (any reduction), the residual form
  // b - A x, and the two fused BiCGStab sources with their reductions
  if (a.src_mode == 1 && a.red_mode == 1 && !general)
    return launch_one<R, NX, DIR, false, 1, 1>(L, a, c, grid, lds, nslab);
  if (a.src_mode == 2 && a.red_mode == 3 && !general)
    return launch_one<R, NX, DIR, false, 2, 3>(L, a, c, grid, lds, nslab);
  if (a.src_mode == 2 && a.red_mode == 4 && !general && a.red_w != nullptr)
    return launch_one<R, NX, DIR, false, 2, 4>(L, a, c, grid, lds, nslab);
  if (a.src_mode == 0 && general && a.red_mode == 0)
    return launch_one<R, NX, DIR, true, 0, 0>(L, a, c, grid, lds, nslab);
  if (a.src_mode == 0 && !general) {
    switch (a.red_mode) {
      case 0:
        if constexpr (sizeof(R) == 4 && NX == 16) {
          if (L.t3_route == 1)
            return launch_one<R, NX, DIR, false, 0, 0, 1>(L, a, c, grid, lds, nslab);
          if (L.t3_route == 2)
            return launch_one<R, NX, DIR, false, 0, 0, 2>(L, a, c, grid, lds, nslab);
        }
        return launch_one<R, NX, DIR, false, 0, 0>(L, a, c, grid, lds, nslab);
      case 1: return launch_one<R, NX, DIR, false, 0, 1>(L, a, c, grid, lds, nslab);
      case 2: return launch_one<R, NX, DIR, false, 0, 2>(L, a, c, grid, lds, nslab);
      case 3: return launch_one<R, NX, DIR, false, 0, 3>(L, a, c, grid, lds, nslab);
      default: break;
    }
  }
  set_error("streaming kernel: unsupported combination of source, reduction and scaling");
  return UFG_EINVAL;
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

// Basis change of whole slices (no time shift): y = post . M^3 (pre . x),
// M = U^T (forward: positions -> block-ordered modes) or U (backward), then
// GENERAL: y = alpha y + beta aux. A workgroup walks a slab of slices of one
// right-hand side (XCD-aware numbering as above); the slices are independent.
// SRC 1 / 2: x is built while loading as the BiCGStab p = r + beta (p - omega v)
// or s = r - alpha v of the rhs state and stored to fpnew (the first basis
// change of a weak-coupling application takes over the vector update).
template <typename R, int NX, bool FWD, bool GENERAL, int SRC>
__global__ void __launch_bounds__(NX * NX)
    basis_kernel(HopArgs<R> a, SplitCoef<R, NX> c, int ntau, int nslab, int xg, int ri) {
  constexpr int P = NX * NX, V = NX * NX * NX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* lds = reinterpret_cast<C2<R>*>(smem_raw);
  int r, sb;
  if (!stream_item(nslab, a.nrhs, xg, ri, r, sb)) return;
  if (a.gate && a.gate[r] == 0) return;
  constexpr bool kCoefLds = sizeof(R) == 8;
  __shared__ CoefSlot<kCoefLds, R, NX> coef_lds[1];
  const SplitCoef<R, NX>& cc = *coef_copy<kCoefLds, R, NX>(c, coef_lds);
  const int l = threadIdx.x;
  const int t0 = (int)((long long)sb * ntau / nslab);
  const int t1 = (int)((long long)(sb + 1) * ntau / nslab);
  const long long rbase = (long long)r * ntau * V;
  const SrcScal<R> q = src_scalars<R, SRC>(a, r);
  for (int t = t0; t < t1; ++t) {
    const long long o = rbase + (long long)t * V + l;
    const long long fo = (long long)t * V + l;
    C2<R> X[NX];
    if constexpr (SRC == 0) {
#pragma unroll
      for (int z = 0; z < NX; ++z) X[z] = a.src[o + z * P];
    } else {
#pragma unroll
      for (int z = 0; z < NX; ++z) {
        const long long i = o + z * P;
        const C2<R> rv = a.fr[i], vv = a.fv[i];
        if constexpr (SRC == 1) {
          const C2<R> pv = a.fp[i];
          const R dx = pv.x - (q.wr * vv.x - q.wi * vv.y);
          const R dy = pv.y - (q.wr * vv.y + q.wi * vv.x);
          X[z] = C2<R>{rv.x + q.br * dx - q.bi * dy, rv.y + q.br * dy + q.bi * dx};
        } else {
          X[z] = C2<R>{rv.x - (q.ar * vv.x - q.ai * vv.y), rv.y - (q.ar * vv.y + q.ai * vv.x)};
        }
        a.fpnew[i] = X[z];
      }
    }
    if (a.pre) {
#pragma unroll
      for (int z = 0; z < NX; ++z) {
        const R fz = a.pre[fo + z * P];
        X[z].x *= fz;
        X[z].y *= fz;
      }
    }
    R F[NX];
    C2<R> U[GENERAL ? NX : 1];
#pragma unroll
    for (int z = 0; z < NX; ++z) F[z] = a.post ? a.post[fo + z * P] : R(1);
    if (GENERAL && a.aux) {
#pragma unroll
      for (int z = 0; z < NX; ++z) U[GENERAL ? z : 0] = a.aux[o + z * P];
    }
    slice_T3<R, NX, FWD ? 1 : 2>(cc, lds, l, X);
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      C2<R> out;
      out.x = F[z] * X[z].x;
      out.y = F[z] * X[z].y;
      if (GENERAL) {
        const R ar = R(a.alpha.x), ai = R(a.alpha.y);
        const C2<R> b = out;
        out.x = ar * b.x - ai * b.y;
        out.y = ar * b.y + ai * b.x;
        if (a.aux) {
          const C2<R> u = U[GENERAL ? z : 0];
          const R br = R(a.beta.x), bi = R(a.beta.y);
          out.x += br * u.x - bi * u.y;
          out.y += br * u.y + bi * u.x;
        }
      }
      a.dst[o + z * P] = out;
    }
  }
}

// Two basis changes of each slice in one pass (the weak-coupling series, whose
// consecutive orders meet as U^3 then U^3T with only per-site factors between):
//   z = alpha post . U^3 x + beta aux  (stored to zout when given),
//   y = U^3T (mid . z).
// The second transform's first LDS write touches only the thread's own z-line,
// which the first transform's last read has already consumed.
template <typename R>
struct PairArgs {
  const C2<R>* src = nullptr;
  C2<R>* dst = nullptr;
  C2<R>* zout = nullptr;
  const R* post = nullptr;
  const R* mid = nullptr;
  const C2<R>* aux = nullptr;
  double2 alpha = {1.0, 0.0};
  double2 beta = {0.0, 0.0};
  const int* gate = nullptr;
  int nrhs = 1;
};

template <typename R, int NX>
__global__ void __launch_bounds__(NX * NX)
    basis_pair_kernel(PairArgs<R> a, SplitCoef<R, NX> cb, SplitCoef<R, NX> cf, int ntau,
                      int nslab, int xg, int ri) {
  constexpr int P = NX * NX, V = NX * NX * NX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C2<R>* lds = reinterpret_cast<C2<R>*>(smem_raw);
  int r, sb;
  if (!stream_item(nslab, a.nrhs, xg, ri, r, sb)) return;
  if (a.gate && a.gate[r] == 0) return;
  __shared__ SplitCoef<R, NX> coef_lds[2];
  const SplitCoef<R, NX>& ccb = *coef_copy<true, R, NX>(cb, coef_lds);
  const SplitCoef<R, NX>& ccf = *coef_copy<true, R, NX>(cf, coef_lds + 1);
  const int l = threadIdx.x;
  const int t0 = (int)((long long)sb * ntau / nslab);
  const int t1 = (int)((long long)(sb + 1) * ntau / nslab);
  const long long rbase = (long long)r * ntau * V;
  const R ar = R(a.alpha.x), ai = R(a.alpha.y), br = R(a.beta.x), bi = R(a.beta.y);
  for (int t = t0; t < t1; ++t) {
    const long long o = rbase + (long long)t * V + l;
    const long long fo = (long long)t * V + l;
    C2<R> X[NX];
#pragma unroll
    for (int z = 0; z < NX; ++z) X[z] = a.src[o + z * P];
    R F[NX], G[NX];
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      F[z] = a.post ? a.post[fo + z * P] : R(1);
      G[z] = a.mid ? a.mid[fo + z * P] : R(1);
    }
    C2<R> Au[NX];
    if (a.aux) {
#pragma unroll
      for (int z = 0; z < NX; ++z) Au[z] = a.aux[o + z * P];
    }
    slice_T3<R, NX, 2>(ccb, lds, l, X);  // U^3
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      const C2<R> b = C2<R>{F[z] * X[z].x, F[z] * X[z].y};
      C2<R> w = C2<R>{ar * b.x - ai * b.y, ar * b.y + ai * b.x};
      if (a.aux) {
        w.x += br * Au[z].x - bi * Au[z].y;
        w.y += br * Au[z].y + bi * Au[z].x;
      }
      if (a.zout) {
        __builtin_nontemporal_store(w.x, &a.zout[o + z * P].x);
        __builtin_nontemporal_store(w.y, &a.zout[o + z * P].y);
      }
      X[z] = C2<R>{G[z] * w.x, G[z] * w.y};
    }
    slice_T3<R, NX, 1>(ccf, lds, l, X);  // U^3T
#pragma unroll
    for (int z = 0; z < NX; ++z) {
      a.dst[o + z * P] = X[z];
    }
  }
}

template <typename R, int NX>
int launch_basis_pair_nx(const Lattice& L, const PairArgs<R>& a) {
  SplitCoef<R, NX> cb, cf;
  int k = 0;
  for (auto& v : cb.es) v = R(L.mode_bwd_host[k++]);
  for (auto& v : cb.ea) v = R(L.mode_bwd_host[k++]);
  for (auto& v : cb.os) v = R(L.mode_bwd_host[k++]);
  for (auto& v : cb.oa) v = R(L.mode_bwd_host[k++]);
  k = 0;
  for (auto& v : cf.es) v = R(L.mode_fwd_host[k++]);
  for (auto& v : cf.ea) v = R(L.mode_fwd_host[k++]);
  for (auto& v : cf.os) v = R(L.mode_fwd_host[k++]);
  for (auto& v : cf.oa) v = R(L.mode_fwd_host[k++]);
  const int nslab = stream_nslab(L);
  const size_t lds = size_t(lds_slice_elems<NX>()) * sizeof(C2<R>);
  static bool attr = false;
  if (!attr) {
    UFG_HIP(hipFuncSetAttribute((const void*)basis_pair_kernel<R, NX>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((basis_pair_kernel<R, NX>), dim3(stream_grid(L, a.nrhs)), dim3(NX * NX),
                     lds, L.stream, a, cb, cf, L.ntau, nslab, stream_group(L),
                     stream_inner(L));
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R, int NX, bool FWD, bool GENERAL, int SRC = 0>
int launch_basis_one(const Lattice& L, const HopArgs<R>& a, const SplitCoef<R, NX>& c,
                     dim3 grid, size_t lds, int nslab) {
  static bool attr = false;
  if (!attr) {
    UFG_HIP(hipFuncSetAttribute((const void*)basis_kernel<R, NX, FWD, GENERAL, SRC>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((basis_kernel<R, NX, FWD, GENERAL, SRC>), grid, dim3(NX * NX), lds,
                     L.stream, a, c, L.ntau, nslab, stream_group(L), stream_inner(L));
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R, int NX>
int launch_basis_nx(const Lattice& L, const HopArgs<R>& a, bool forward) {
  SplitCoef<R, NX> c;
  const std::vector<double>& h = forward ? L.mode_fwd_host : L.mode_bwd_host;
  int k = 0;
  for (auto& v : c.es) v = R(h[k++]);
  for (auto& v : c.ea) v = R(h[k++]);
  for (auto& v : c.os) v = R(h[k++]);
  for (auto& v : c.oa) v = R(h[k++]);
  const int nslab = stream_nslab(L);
  const size_t lds = size_t(lds_slice_elems<NX>()) * sizeof(C2<R>);
  const dim3 grid(stream_grid(L, a.nrhs));
  const bool general = (a.alpha.x != 1.0 || a.alpha.y != 0.0 || a.aux != nullptr);
  if (forward && a.src_mode == 1 && !general)
    return launch_basis_one<R, NX, true, false, 1>(L, a, c, grid, lds, nslab);
  if (forward && a.src_mode == 2 && !general)
    return launch_basis_one<R, NX, true, false, 2>(L, a, c, grid, lds, nslab);
  if (a.src_mode != 0) {
    set_error("basis change: a fused source needs the plain forward change");
    return UFG_EINVAL;
  }
  if (forward)
    return general ? launch_basis_one<R, NX, true, true>(L, a, c, grid, lds, nslab)
                   : launch_basis_one<R, NX, true, false>(L, a, c, grid, lds, nslab);
  return general ? launch_basis_one<R, NX, false, true>(L, a, c, grid, lds, nslab)
                 : launch_basis_one<R, NX, false, false>(L, a, c, grid, lds, nslab);
}

}  // namespace

int stream_slab(const Lattice& L) {
  if (L.slab > 0) return std::min(L.slab, L.ntau);
  // One slice per workgroup throughout (with the slab groups of stream_group):
  // complex64 apply_M at 16^3 x 400, 8 rhs: 48.8 us at two slices per
  // workgroup in the contiguous numbering, 43.1 us at one in groups of 10;
  // complex128: 102.9 / 95.3 us (M / M^T) at two slices, 95.4 / 95.8 us at
  // one in groups of 10 taken rhs-inner (16^3 x 800: 200.1 / 177.9 against
  // 178.7 / 178.9 us), the FP64 solve within 0.5 %.
  return 1;
}

int stream_nslab(const Lattice& L) {
  if (L.nslab > 0) return std::min(L.nslab, L.ntau);
  const int slab = stream_slab(L);
  return (L.ntau + slab - 1) / slab;
}

int stream_group(const Lattice& L) {
  if (L.xcd_group >= 0) return std::min(L.xcd_group, stream_nslab(L));
  // Groups of ten slabs per XCD. complex64 walks a group's slabs for one rhs
  // after the other; complex128 lattices of 2^20 sites and more take every rhs
  // of a group in turn (stream_inner), so a field slice is read while the same
  // XCD still holds it. Smaller complex128 lattices (short launches,
  // few slabs) keep the contiguous numbering.
  if (L.dtype == UFG_C64) return std::min(10, stream_nslab(L));
  if ((long long)L.V * L.ntau >= (1ll << 20)) return std::min(10, stream_nslab(L));
  return 0;
}

int stream_inner(const Lattice& L) {
  if (L.xcd_group >= 0) return L.xcd_rhs_inner;
  return (L.dtype == UFG_C128 && (long long)L.V * L.ntau >= (1ll << 20)) ? 1 : 0;
}

int stream_grid(const Lattice& L, int nrhs) {
  const int nslab = stream_nslab(L), xg = stream_group(L);
  if (xg <= 0) return nslab * nrhs;
  if (stream_inner(L)) {
    const int groups = (nslab + xg - 1) / xg;
    return 8 * ((groups + 7) / 8) * nrhs * xg;
  }
  const int F = nslab / xg, rem = nslab - F * xg;
  int most = 0;
  for (int j = 0; j < 8; ++j) {
    int nj = xg * (F / 8 + ((j < (F & 7)) ? 1 : 0));
    if (rem > 0 && (F & 7) == j) nj += rem;
    most = std::max(most, nj);
  }
  return 8 * nrhs * most;
}

bool stream_supported(const Lattice& L) {
  // buffer offsets are 32-bit: one rhs block of complex128 must stay below 2 GiB
  const long long block = (long long)L.ntau * L.nx * L.nx * L.nx * (long long)sizeof(double2);
  return (L.nx == 8 || L.nx == 12 || L.nx == 16) && !L.split_host.empty() &&
         block < (1ll << 31);
}

template <typename R>
int launch_hop_stream(const Lattice& L, const HopArgs<R>& args) {
  HopArgs<R> a = args;
  if (a.beta.x == 0.0 && a.beta.y == 0.0) a.aux = nullptr;
  if (a.fin_part && !(a.src_mode == 2 && a.red_mode == 4 && a.fin_part2 && a.fin_flags &&
                      a.st && a.fin_nblk > 0 && a.fin_nblk2 > 0)) {
    set_error("streaming kernel: the fused alpha step needs source 2, reduction 4 and its "
              "partials, state and flags");
    return UFG_EINVAL;
  }
  // M-type applies the field to the source slice, M^T-type to the output slice
  const bool fields_ok = (a.shift < 0) ? (a.pre != nullptr && a.post == nullptr)
                                       : (a.post != nullptr && a.pre == nullptr);
  if (!fields_ok) {
    set_error("streaming kernel: field must multiply the source (M) or the output (M^T)");
    return UFG_EINVAL;
  }
  switch (L.nx) {
    case 8: return launch_nx<R, 8>(L, a);
    case 12: return launch_nx<R, 12>(L, a);
    case 16: return launch_nx<R, 16>(L, a);
    default: set_error("streaming kernel: unsupported nx"); return UFG_EINVAL;
  }
}

template <typename R>
int launch_basis_stream(const Lattice& L, const HopArgs<R>& args, bool forward) {
  HopArgs<R> a = args;
  if (a.beta.x == 0.0 && a.beta.y == 0.0) a.aux = nullptr;
  if (a.shift != 0 || a.red_mode != 0 || a.id != nullptr) {
    set_error("basis change: no shift, identity term or reduction");
    return UFG_EINVAL;
  }
  if (a.src_mode != 0 && (a.src_mode > 2 || !a.fr || !a.fv || !a.fpnew || !a.st ||
                          (a.src_mode == 1 && !a.fp))) {
    set_error("basis change: incomplete fused source");
    return UFG_EINVAL;
  }
  switch (L.nx) {
    case 8: return launch_basis_nx<R, 8>(L, a, forward);
    case 12: return launch_basis_nx<R, 12>(L, a, forward);
    case 16: return launch_basis_nx<R, 16>(L, a, forward);
    default: set_error("basis change: unsupported nx"); return UFG_EINVAL;
  }
}

template <typename R>
int launch_basis_pair(const Lattice& L, const C2<R>* x, C2<R>* y, C2<R>* zout, const R* post,
                      double2 alpha, const C2<R>* aux, double2 beta, const R* mid, int nrhs,
                      const int* gate) {
  if (L.mode_perm.empty() || !stream_supported(L)) {
    set_error("basis pair: needs the block form of U (nx in {8, 12, 16})");
    return UFG_EINVAL;
  }
  if (x == nullptr || y == nullptr || (zout != nullptr && (zout == x || zout == y))) {
    set_error("basis pair: bad vectors");
    return UFG_EINVAL;
  }
  PairArgs<R> a;
  a.src = x;
  a.dst = y;
  a.zout = zout;
  a.post = post;
  a.mid = mid;
  a.alpha = alpha;
  a.beta = beta;
  a.aux = (beta.x == 0.0 && beta.y == 0.0) ? nullptr : aux;
  a.gate = gate;
  a.nrhs = nrhs;
  switch (L.nx) {
    case 8: return launch_basis_pair_nx<R, 8>(L, a);
    case 12: return launch_basis_pair_nx<R, 12>(L, a);
    case 16: return launch_basis_pair_nx<R, 16>(L, a);
    default: set_error("basis pair: unsupported nx"); return UFG_EINVAL;
  }
}

template int launch_basis_pair<float>(const Lattice&, const float2*, float2*, float2*,
                                      const float*, double2, const float2*, double2,
                                      const float*, int, const int*);
template int launch_basis_pair<double>(const Lattice&, const double2*, double2*, double2*,
                                       const double*, double2, const double2*, double2,
                                       const double*, int, const int*);
template int launch_basis_stream<float>(const Lattice&, const HopArgs<float>&, bool);
template int launch_basis_stream<double>(const Lattice&, const HopArgs<double>&, bool);
template int launch_hop_stream<float>(const Lattice&, const HopArgs<float>&);
template int launch_hop_stream<double>(const Lattice&, const HopArgs<double>&);

}  // namespace ufg
