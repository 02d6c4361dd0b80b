// Block coefficients of the symmetric-circulant T in the basis of its two
// reflection symmetries, and the streaming M / M^T launcher.
#pragma once

#include "ufg_internal.h"

namespace ufg {

template <typename R, int NX>
struct SplitCoef {
  static constexpr int Q = NX / 4;
  R es[(Q + 1) * (Q + 1)];
  R ea[Q * Q];
  R os[Q * Q];
  R oa[(Q - 1) * (Q - 1) > 0 ? (Q - 1) * (Q - 1) : 1];
};

// Host: the blocks for nx in {8, 12, 16} in the order es, ea, os, oa
// (row-major each); empty for other nx. Returns the largest off-block entry
// of the transformed matrix (a self-check).
double split_coefficients(int nx, const std::vector<double>& T, std::vector<double>* out);

// Host: the block-diagonal forward (U^T) and backward (U) maps of the
// eigenbasis of T, with the block ordering of the modes (perm); empty for nx
// not in {8, 12, 16}. Returns the largest off-block entry (a self-check).
double mode_split_coefficients(int nx, const std::vector<double>& U, std::vector<double>* fwd,
                               std::vector<double>* bwd, std::vector<int>* perm);

// Basis change y = (U or U^T)^{x3} (pre . x) scaled by post, alpha, plus beta aux,
// in the block-ordered mode basis (streaming-supported nx only).
template <typename R>
int launch_basis_stream(const Lattice& L, const HopArgs<R>& a, bool forward);

// Two basis changes per slice in one pass (streaming-supported nx):
// z = alpha post . U^3 x + beta aux (stored to zout unless null), y = U^3T (mid . z).
// post, mid: real fields or null (1); y may alias x; zout must alias neither.
template <typename R>
int launch_basis_pair(const Lattice& L, const C2<R>* x, C2<R>* y, C2<R>* zout, const R* post,
                      double2 alpha, const C2<R>* aux, double2 beta, const R* mid, int nrhs,
                      const int* gate);

int stream_slab(const Lattice& L);
// Slabs per right-hand side: slab s of nslab covers slices [s ntau / nslab,
// (s + 1) ntau / nslab), so every slab holds floor or ceil of ntau / nslab.
int stream_nslab(const Lattice& L);
// Slab groups per XCD of the workgroup numbering (0: contiguous (slab, rhs)
// runs per XCD with the rhs fastest), and the grid of a launch over nrhs.
int stream_group(const Lattice& L);
int stream_grid(const Lattice& L, int nrhs);
// 1: an XCD takes every rhs of a slab group in turn (default or lattice_tune_order)
int stream_inner(const Lattice& L);
bool stream_supported(const Lattice& L);
template <typename R>
int launch_hop_stream(const Lattice& L, const HopArgs<R>& a);

}  // namespace ufg
