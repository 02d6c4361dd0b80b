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

int stream_slab(const Lattice& L);
bool stream_supported(const Lattice& L);
template <typename R>
int launch_hop_stream(const Lattice& L, const HopArgs<R>& a);

}  // namespace ufg
