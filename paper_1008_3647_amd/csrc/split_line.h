// One line of the symmetric-circulant factor T applied in registers through
// its reflection-symmetry block form (the blocks are SplitCoef, built on the
// host by split_coefficients). Shared by the streaming operator and the
// batched operator.
#pragma once

#include "hop_stream.h"

namespace ufg {
namespace splitk {

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
// The four blocks of a line in the reflection-symmetry basis (Q = NX/4):
// es[0..Q], ea[0..Q-1], os[1..Q], oa[1..Q-1].
template <typename R, int NX>
struct Parts {
  static constexpr int Q = NX / 4;
  C2<R> es[Q + 1], ea[Q + 1], os[Q + 1], oa[Q + 1];
};

// positions -> reflection-symmetry components (two butterfly levels)
template <typename R, int NX>
__device__ __forceinline__ void butterflies(const C2<R> (&a)[NX], Parts<R, NX>& p) {
  constexpr int H = NX / 2, Q = NX / 4;
  C2<R> E[H + 1], O[H + 1];
  E[0] = a[0];
  E[H] = a[H];
#pragma unroll
  for (int j = 1; j < H; ++j) {
    E[j] = add<R>(a[j], a[NX - j]);
    O[j] = sub<R>(a[j], a[NX - j]);
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    p.es[j] = add<R>(E[j], E[H - j]);
    p.ea[j] = sub<R>(E[j], E[H - j]);
  }
  p.es[Q] = E[Q];
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    p.os[j] = add<R>(O[j], O[H - j]);
    p.oa[j] = sub<R>(O[j], O[H - j]);
  }
  p.os[Q] = O[Q];
}

// out = blockdiag(c) in, block by block
template <typename R, int NX>
__device__ __forceinline__ void blockmul(const SplitCoef<R, NX>& c, const Parts<R, NX>& in,
                                         Parts<R, NX>& out) {
  constexpr int Q = NX / 4;
#pragma unroll
  for (int i = 0; i <= Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 0; k <= Q; ++k) {
      const R m = c.es[i * (Q + 1) + k];
      s.x = fma(m, in.es[k].x, s.x);
      s.y = fma(m, in.es[k].y, s.y);
    }
    out.es[i] = s;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const R m = c.ea[i * Q + k];
      s.x = fma(m, in.ea[k].x, s.x);
      s.y = fma(m, in.ea[k].y, s.y);
    }
    out.ea[i] = s;
  }
#pragma unroll
  for (int i = 1; i <= Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 1; k <= Q; ++k) {
      const R m = c.os[(i - 1) * Q + (k - 1)];
      s.x = fma(m, in.os[k].x, s.x);
      s.y = fma(m, in.os[k].y, s.y);
    }
    out.os[i] = s;
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    C2<R> s = zero2<R>();
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const R m = c.oa[(i - 1) * (Q - 1) + (k - 1)];
      s.x = fma(m, in.oa[k].x, s.x);
      s.y = fma(m, in.oa[k].y, s.y);
    }
    out.oa[i] = s;
  }
}

// reflection-symmetry components -> positions (additions only)
template <typename R, int NX>
__device__ __forceinline__ void unbutterflies(const Parts<R, NX>& p, C2<R> (&a)[NX]) {
  constexpr int H = NX / 2, Q = NX / 4;
  C2<R> E[H + 1], O[H + 1];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    E[j] = add<R>(p.es[j], p.ea[j]);
    E[H - j] = sub<R>(p.es[j], p.ea[j]);
  }
  E[Q] = p.es[Q];
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    O[j] = add<R>(p.os[j], p.oa[j]);
    O[H - j] = sub<R>(p.os[j], p.oa[j]);
  }
  O[Q] = p.os[Q];
  a[0] = E[0];
  a[H] = E[H];
#pragma unroll
  for (int j = 1; j < H; ++j) {
    a[j] = add<R>(E[j], O[j]);
    a[NX - j] = sub<R>(E[j], O[j]);
  }
}

// y = T a for one line held in registers (in place)
template <typename R, int NX>
__device__ __forceinline__ void split_line(const SplitCoef<R, NX>& c, C2<R> (&a)[NX]) {
  Parts<R, NX> u, w;
  butterflies<R, NX>(a, u);
  blockmul<R, NX>(c, u, w);
  unbutterflies<R, NX>(w, a);
}

// Mode-space packing of a line: the blocks in the order es, ea, os, oa.
template <typename R, int NX>
__device__ __forceinline__ void pack_modes(const Parts<R, NX>& p, C2<R> (&a)[NX]) {
  constexpr int Q = NX / 4;
#pragma unroll
  for (int j = 0; j <= Q; ++j) a[j] = p.es[j];
#pragma unroll
  for (int j = 0; j < Q; ++j) a[Q + 1 + j] = p.ea[j];
#pragma unroll
  for (int j = 1; j <= Q; ++j) a[2 * Q + j] = p.os[j];
#pragma unroll
  for (int j = 1; j < Q; ++j) a[3 * Q + j] = p.oa[j];
}
template <typename R, int NX>
__device__ __forceinline__ void unpack_modes(const C2<R> (&a)[NX], Parts<R, NX>& p) {
  constexpr int Q = NX / 4;
#pragma unroll
  for (int j = 0; j <= Q; ++j) p.es[j] = a[j];
#pragma unroll
  for (int j = 0; j < Q; ++j) p.ea[j] = a[Q + 1 + j];
#pragma unroll
  for (int j = 1; j <= Q; ++j) p.os[j] = a[2 * Q + j];
#pragma unroll
  for (int j = 1; j < Q; ++j) p.oa[j] = a[3 * Q + j];
}

// c = U^T a in the block-ordered eigenbasis of T (positions -> modes)
template <typename R, int NX>
__device__ __forceinline__ void modes_fwd(const SplitCoef<R, NX>& c, C2<R> (&a)[NX]) {
  Parts<R, NX> u, w;
  butterflies<R, NX>(a, u);
  blockmul<R, NX>(c, u, w);
  pack_modes<R, NX>(w, a);
}

// a = U c from block-ordered modes (modes -> positions)
template <typename R, int NX>
__device__ __forceinline__ void modes_bwd(const SplitCoef<R, NX>& c, C2<R> (&a)[NX]) {
  Parts<R, NX> u, w;
  unpack_modes<R, NX>(a, u);
  blockmul<R, NX>(c, u, w);
  unbutterflies<R, NX>(w, a);
}

}  // namespace splitk
}  // namespace ufg
