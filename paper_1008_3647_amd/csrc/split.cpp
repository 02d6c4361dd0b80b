// Host construction of the block-diagonal form of the circulant factor T used
// by the streaming kernel (see hop_stream.hip). With u = P x the two-level
// add/subtract butterfly and y = P' v its inverse written with additions only,
// B = P'^{-1} T P^{-1} is block diagonal (reflection symmetries of T); the
// blocks are returned in the order the kernel consumes them.
#include <cmath>

#include "hop_stream.h"

namespace ufg {

static bool invert(int n, std::vector<double> a, std::vector<double>* inv) {
  inv->assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) (*inv)[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[p * n + c])) p = r;
    if (std::fabs(a[p * n + c]) < 1e-12) return false;
    for (int k = 0; k < n; ++k) {
      std::swap(a[c * n + k], a[p * n + k]);
      std::swap((*inv)[c * n + k], (*inv)[p * n + k]);
    }
    const double d = a[c * n + c];
    for (int k = 0; k < n; ++k) {
      a[c * n + k] /= d;
      (*inv)[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[c * n + k];
        (*inv)[r * n + k] -= f * (*inv)[c * n + k];
      }
    }
  }
  return true;
}

// P: positions -> reflection-symmetry components (block order es, ea, os,
// oa); Pp: the inverse written with additions only (as the kernels do).
static void butterfly_matrices(int nx, std::vector<double>* Pout, std::vector<double>* Ppout) {
  const int n = nx, H = nx / 2, Q = nx / 4;
  // rows of P: E_j = x_j + x_{-j} (x_0, x_H alone), O_j = x_j - x_{-j}
  auto Erow = [&](int j) {
    std::vector<double> v(n, 0.0);
    v[j] += 1.0;
    if (j != 0 && j != H) v[n - j] += 1.0;
    return v;
  };
  auto Orow = [&](int j) {
    std::vector<double> v(n, 0.0);
    v[j] += 1.0;
    v[n - j] -= 1.0;
    return v;
  };
  std::vector<std::vector<double>> rows;
  for (int j = 0; j < Q; ++j) {  // ES_j = E_j + E_{H-j}
    auto a = Erow(j), b = Erow(H - j);
    for (int k = 0; k < n; ++k) a[k] += b[k];
    rows.push_back(a);
  }
  rows.push_back(Erow(Q));
  for (int j = 0; j < Q; ++j) {  // EA_j = E_j - E_{H-j}
    auto a = Erow(j), b = Erow(H - j);
    for (int k = 0; k < n; ++k) a[k] -= b[k];
    rows.push_back(a);
  }
  for (int j = 1; j < Q; ++j) {  // OS_j = O_j + O_{H-j}
    auto a = Orow(j), b = Orow(H - j);
    for (int k = 0; k < n; ++k) a[k] += b[k];
    rows.push_back(a);
  }
  rows.push_back(Orow(Q));
  for (int j = 1; j < Q; ++j) {  // OA_j = O_j - O_{H-j}
    auto a = Orow(j), b = Orow(H - j);
    for (int k = 0; k < n; ++k) a[k] -= b[k];
    rows.push_back(a);
  }
  std::vector<double> P(n * n), Pp(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) P[i * n + k] = rows[i][k];
  // P': v = (ES', EA', OS', OA') -> y with additions only
  const int nES = Q + 1, nEA = Q, nOS = Q;
  auto iES = [&](int j) { return j; };
  auto iEA = [&](int j) { return nES + j; };
  auto iOS = [&](int j) { return nES + nEA + (j - 1); };
  auto iOA = [&](int j) { return nES + nEA + nOS + (j - 1); };
  auto Ep = [&](int j) {
    std::vector<double> v(n, 0.0);
    if (j < Q) {
      v[iES(j)] += 1;
      v[iEA(j)] += 1;
    } else if (j == Q) {
      v[iES(Q)] += 1;
    } else {
      v[iES(H - j)] += 1;
      v[iEA(H - j)] -= 1;
    }
    return v;
  };
  auto Op = [&](int j) {
    std::vector<double> v(n, 0.0);
    if (j < Q) {
      v[iOS(j)] += 1;
      v[iOA(j)] += 1;
    } else if (j == Q) {
      v[iOS(Q)] += 1;
    } else {
      v[iOS(H - j)] += 1;
      v[iOA(H - j)] -= 1;
    }
    return v;
  };
  auto setrow = [&](int r, const std::vector<double>& v) {
    for (int k = 0; k < n; ++k) Pp[r * n + k] = v[k];
  };
  setrow(0, Ep(0));
  setrow(H, Ep(H));
  for (int j = 1; j < H; ++j) {
    auto e = Ep(j), o = Op(j);
    std::vector<double> s(n), d(n);
    for (int k = 0; k < n; ++k) {
      s[k] = e[k] + o[k];
      d[k] = e[k] - o[k];
    }
    setrow(j, s);
    setrow(n - j, d);
  }
  *Pout = P;
  *Ppout = Pp;
}

double split_coefficients(int nx, const std::vector<double>& T, std::vector<double>* out) {
  out->clear();
  if (nx % 4 != 0 || nx < 8) return 0.0;
  const int n = nx, Q = nx / 4;
  std::vector<double> P, Pp;
  butterfly_matrices(nx, &P, &Pp);
  std::vector<double> Pi, Ppi;
  if (!invert(n, P, &Pi) || !invert(n, Pp, &Ppi)) return 1.0;
  std::vector<double> tmp(n * n, 0.0), B(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += T[i * n + k] * Pi[k * n + j];
      tmp[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += Ppi[i * n + k] * tmp[k * n + j];
      B[i * n + j] = s;
    }
  const int sizes[4] = {Q + 1, Q, Q, Q - 1};
  int starts[4];
  starts[0] = 0;
  for (int b = 1; b < 4; ++b) starts[b] = starts[b - 1] + sizes[b - 1];
  double off = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      int bi = 0, bj = 0;
      for (int b = 0; b < 4; ++b) {
        if (i >= starts[b] && i < starts[b] + sizes[b]) bi = b;
        if (j >= starts[b] && j < starts[b] + sizes[b]) bj = b;
      }
      if (bi != bj) off = std::max(off, std::fabs(B[i * n + j]));
    }
  for (int b = 0; b < 4; ++b)
    for (int i = 0; i < sizes[b]; ++i)
      for (int j = 0; j < sizes[b]; ++j) out->push_back(B[(starts[b] + i) * n + starts[b] + j]);
  return off;
}

// The eigenbasis U of T (columns = modes: cosines and sines) in the same
// reflection-symmetry basis. Every mode is even or odd under both reflections,
// so with the modes ordered block by block (perm[i] = the column of U that is
// block-ordered mode i) the forward map c = U^T a = (U^T P^{-1}) (P a) and the
// backward map a = U c = Pp (Pp^{-1} U) c are block diagonal: fwd and bwd hold
// their blocks in the order es, ea, os, oa. Returns the largest off-block
// entry of either map (a self-check), 1 when the parities do not sort.
double mode_split_coefficients(int nx, const std::vector<double>& U, std::vector<double>* fwd,
                               std::vector<double>* bwd, std::vector<int>* perm) {
  fwd->clear();
  bwd->clear();
  perm->clear();
  if (nx % 4 != 0 || nx < 8) return 0.0;
  const int n = nx, Q = nx / 4;
  std::vector<double> P, Pp, Pi, Ppi;
  butterfly_matrices(nx, &P, &Pp);
  if (!invert(n, P, &Pi) || !invert(n, Pp, &Ppi)) return 1.0;
  const int sizes[4] = {Q + 1, Q, Q, Q - 1};
  const int starts[4] = {0, Q + 1, 2 * Q + 1, 3 * Q + 1};
  auto block_of = [&](int j) {
    int b = 0;
    while (b < 3 && j >= starts[b + 1]) ++b;
    return b;
  };
  // C = U^T P^{-1}: row m = mode m in component coordinates
  std::vector<double> C(n * n, 0.0);
  for (int m = 0; m < n; ++m)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += U[k * n + m] * Pi[k * n + j];
      C[m * n + j] = s;
    }
  std::vector<int> blk(n);
  for (int m = 0; m < n; ++m) {
    int arg = 0;
    for (int j = 1; j < n; ++j)
      if (std::fabs(C[m * n + j]) > std::fabs(C[m * n + arg])) arg = j;
    blk[m] = block_of(arg);
  }
  for (int b = 0; b < 4; ++b)
    for (int m = 0; m < n; ++m)
      if (blk[m] == b) perm->push_back(m);
  for (int b = 0; b < 4; ++b) {
    int cnt = 0;
    for (int m = 0; m < n; ++m) cnt += blk[m] == b;
    if (cnt != sizes[b]) return 1.0;
  }
  // D = Pp^{-1} U Pi^T: column i = block-ordered mode i in component coordinates
  std::vector<double> D(n * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += Ppi[r * n + k] * U[k * n + (*perm)[i]];
      D[r * n + i] = s;
    }
  double off = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (block_of(i) == block_of(j)) continue;
      off = std::max(off, std::fabs(C[(*perm)[i] * n + j]));
      off = std::max(off, std::fabs(D[i * n + j]));
    }
  for (int b = 0; b < 4; ++b)
    for (int i = 0; i < sizes[b]; ++i)
      for (int k = 0; k < sizes[b]; ++k) {
        fwd->push_back(C[(*perm)[starts[b] + i] * n + starts[b] + k]);
        bwd->push_back(D[(starts[b] + i) * n + starts[b] + k]);
      }
  return off;
}

}  // namespace ufg
