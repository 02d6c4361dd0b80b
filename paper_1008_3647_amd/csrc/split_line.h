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

}  // namespace splitk
}  // namespace ufg
