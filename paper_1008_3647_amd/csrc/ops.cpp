// Operator and preconditioner compositions (host-side launch sequences).
//
// Preconditioners (paper):
//   Chebyshev (Sec. 2): P(Q^) v = prod_k c^{1/2n} (Q/lam_max - z_k) v, roots in
//     bit-reversal order; each factor is an M then an M^T launch whose epilogue
//     does the complex axpby.
//   Strong coupling (Sec. 4): (L^dagger D L)^{-1} by one per-site kernel.
//   Weak coupling (Sec. 3): with T^3 = U^3 diag(lam) U^3T and M0 = 1 - Z T^3,
//     M1 = -Z T^3 S (S = diag sin sigma, Z the antiperiodic one-slice shift):
//       M0^{-1}          = U^3 (1 - lam Z)^{-1} U^3T
//       -A M0^{-1} M1 u  = A U^3 [(1 - lam Z)^{-1} - 1] U^3T S u
//       -A M1^T M0^{-T}v = A S U^3 [(1 - lam Z^T)^{-1} - 1] U^3T v
//     so every order of the expansion costs two spatial basis changes and one
//     temporal sweep, with the M1 factor folded into them.
#include "ops.h"
#include "hop_stream.h"

#include <cmath>
#include <complex>

namespace ufg {

double PcPlan::paper_cost() const {
  switch (kind) {
    case UFG_PC_CHEB: return 2.0 * degree;
    case UFG_PC_SCA: return 1.0;
    case UFG_PC_WCE: return 2.0 * (order + 1) + order;  // (d+1) 2 beta + d, beta = 1
    case UFG_PC_SCA_CHEB: return 2.0 * degree + (degree + 1);  // 2d MV and d + 1 SCA (1 each)
    default: return 0.0;
  }
}

template <typename R>
C2<R>* slot_vec(Lattice& L, int slot, int nrhs, int* rc) {
  const size_t bytes = sizeof(C2<R>) * (size_t)L.N * (size_t)nrhs;
  *rc = L.work[slot].ensure(bytes);
  return reinterpret_cast<C2<R>*>(L.work[slot].p);
}
template float2* slot_vec<float>(Lattice&, int, int, int*);
template double2* slot_vec<double>(Lattice&, int, int, int*);

int krylov_state(Lattice& L, int nrhs, KrylovState* K, int slot_red) {
  const int nblk = std::max(vec_blocks(L, nrhs), hop_blocks_per_rhs(L));
  const size_t st_bytes = sizeof(RhsState) * nrhs;
  const size_t flag_bytes = sizeof(int) * nrhs;
  const size_t red_bytes = sizeof(double) * 8 * (size_t)nblk * nrhs;
  const size_t red2_bytes = sizeof(double) * 4 * (size_t)vec_blocks(L, nrhs) * nrhs;
  const size_t red3_bytes = sizeof(double) * 4 * (size_t)hop_blocks_per_rhs(L) * nrhs;
  DevBuf& b = L.work[slot_red];
  UFG_TRY(b.ensure(st_bytes + 3 * flag_bytes + red_bytes + red2_bytes + red3_bytes + 256));
  char* p = reinterpret_cast<char*>(b.p);
  K->nrhs = nrhs;
  K->part = reinterpret_cast<double*>(p);
  p += red_bytes;
  K->part2 = reinterpret_cast<double*>(p);
  p += red2_bytes;
  K->part3 = reinterpret_cast<double*>(p);
  p += red3_bytes;
  K->st = reinterpret_cast<RhsState*>(p);
  p += st_bytes;
  K->active = reinterpret_cast<int*>(p);
  K->update = K->active + nrhs;
  K->restart = K->update + nrhs;
  return UFG_OK;
}

// ---------------------------------------------------------------------------

template <typename R>
int op_apply(const Lattice& L, int op, const C2<R>* x, C2<R>* y, int nrhs, const int* gate,
             int red_mode, const C2<R>* red_w, double* red_out) {
  const Fields<R>& F = fields<R>(L);
  HopArgs<R> a;
  a.src = x;
  a.id = x;
  a.dst = y;
  a.mat = F.T;
  a.nrhs = nrhs;
  a.gate = gate;
  a.red_mode = red_mode;
  a.red_w = red_w;
  a.red_out = red_out;
  if (op == UFG_OP_M) {
    a.shift = kShiftM;
    a.pre = F.b;
  } else {
    a.shift = kShiftMdag;
    a.post = F.b;
  }
  return launch_hop<R>(L, a);
}

template <typename R>
int op_residual(const Lattice& L, int op, const C2<R>* x, const C2<R>* b, C2<R>* y, int nrhs,
                const int* gate) {
  const Fields<R>& F = fields<R>(L);
  HopArgs<R> a;
  a.src = x;
  a.id = x;
  a.dst = y;
  a.aux = b;
  a.alpha = double2{-1.0, 0.0};
  a.beta = double2{1.0, 0.0};
  a.mat = F.T;
  a.nrhs = nrhs;
  a.gate = gate;
  if (op == UFG_OP_M) {
    a.shift = kShiftM;
    a.pre = F.b;
  } else {
    a.shift = kShiftMdag;
    a.post = F.b;
  }
  return launch_hop<R>(L, a);
}

template <typename R>
int q_apply(const Lattice& L, const C2<R>* x, C2<R>* tmp, C2<R>* y, int nrhs, const int* gate,
            int red_mode, const C2<R>* red_w, double* red_out) {
  UFG_TRY(op_apply<R>(L, UFG_OP_M, x, tmp, nrhs, gate));
  return op_apply<R>(L, UFG_OP_MDAG, tmp, y, nrhs, gate, red_mode, red_w, red_out);
}

template <typename R>
int q_residual(const Lattice& L, const C2<R>* x, const C2<R>* b, C2<R>* tmp, C2<R>* y, int nrhs,
               const int* gate) {
  UFG_TRY(op_apply<R>(L, UFG_OP_M, x, tmp, nrhs, gate));
  return op_residual<R>(L, UFG_OP_MDAG, tmp, b, y, nrhs, gate);
}

// ---------------------------------------------------------------------------
// Chebyshev helpers (host arithmetic, complex128)

static std::vector<std::complex<double>> cheb_roots_paper(int degree, double eps) {
  std::vector<std::complex<double>> z(degree);
  for (int k = 1; k <= degree; ++k) {
    const double th = 2.0 * M_PI * k / (degree + 1);
    z[k - 1] = std::complex<double>(0.5 * (1.0 + eps) * (1.0 - std::cos(th)),
                                    -std::sqrt(eps) * std::sin(th));
  }
  return z;
}

static int bitrev(int i, int m) {
  int r = 0;
  for (int b = 0; b < m; ++b)
    if (i >> b & 1) r |= 1 << (m - 1 - b);
  return r;
}

int cheb_plan(int degree, double eps, std::vector<double2>* roots, double2* cf) {
  if (degree < 1 || (degree & (degree - 1)) != 0) return UFG_EINVAL;
  if (!(eps > 0.0 && eps < 1.0)) return UFG_EINVAL;
  int m = 0;
  while ((1 << m) < degree) ++m;
  auto z = cheb_roots_paper(degree, eps);
  const double h = 0.5 * (1.0 + eps);
  std::complex<double> cinv = h;
  for (auto& zk : z) cinv *= (h - zk);
  const std::complex<double> c = 1.0 / cinv;
  const std::complex<double> cfac = std::pow(c, 1.0 / degree);
  roots->resize(degree);
  for (int i = 0; i < degree; ++i) {
    const auto zk = z[bitrev(i, m)];
    (*roots)[i] = double2{zk.real(), zk.imag()};
  }
  *cf = double2{cfac.real(), cfac.imag()};
  return UFG_OK;
}

int euler_weights(int order, double p, double* w) {
  if (order < 0 || order > kMaxWceOrder) return UFG_EINVAL;
  // S_{d,0} = sum_k C(d,k) p^{d-k} (1-p)^k S_{0,k}; S_{0,k} = sum_{m<=k} u_m
  double binom[kMaxWceOrder + 1];
  binom[0] = 1.0;
  for (int k = 1; k <= order; ++k) binom[k] = binom[k - 1] * (order - k + 1) / k;
  for (int m = 0; m <= order; ++m) {
    double s = 0.0;
    for (int k = m; k <= order; ++k) s += binom[k] * std::pow(p, order - k) * std::pow(1 - p, k);
    w[m] = s;
  }
  return UFG_OK;
}

int resolve_precond(Lattice& L, const ufg_precond* p, PcPlan* out) {
  PcPlan pc;
  if (!p || p->kind == UFG_PC_NONE) {
    *out = pc;
    return UFG_OK;
  }
  pc.kind = p->kind;
  switch (p->kind) {
    case UFG_PC_CHEB: {
      pc.degree = p->degree;
      pc.eps = p->eps;
      if (cheb_plan(p->degree, p->eps, &pc.roots, &pc.cf) != UFG_OK) {
        set_error("Chebyshev preconditioner needs a power-of-two degree and 0 < eps < 1");
        return UFG_EINVAL;
      }
      if (p->lam_max > 0) {
        pc.lam_max = p->lam_max;
      } else if (p->lam_max == 0) {
        pc.lam_max = (1.0 + L.bmax) * (1.0 + L.bmax);
      } else {
        UFG_TRY(estimate_lam_max(L, &pc.lam_max));
      }
      break;
    }
    case UFG_PC_SCA:
      UFG_CHECK(p->alpha > 0, "SCA needs alpha > 0");
      pc.alpha = p->alpha;
      if (L.sca_alpha != p->alpha) UFG_TRY(launch_sca_setup(L, p->alpha));
      break;
    case UFG_PC_SCA_CHEB:
      UFG_CHECK(p->alpha > 0, "SCA needs alpha > 0");
      pc.alpha = p->alpha;
      pc.degree = p->degree;
      pc.eps = p->eps;
      if (cheb_plan(p->degree, p->eps, &pc.roots, &pc.cf) != UFG_OK) {
        set_error("Chebyshev filter needs a power-of-two degree and 0 < eps < 1");
        return UFG_EINVAL;
      }
      if (L.sca_alpha != p->alpha) UFG_TRY(launch_sca_setup(L, p->alpha));
      if (p->lam_max > 0)
        pc.lam_max = p->lam_max;
      else
        UFG_TRY(estimate_lam_max_sq(L, p->alpha, &pc.lam_max));
      break;
    case UFG_PC_WCE:
      UFG_CHECK(p->wce_order >= 0 && p->wce_order <= kMaxWceOrder, "WCE order must be 0..8");
      pc.order = p->wce_order;
      if (p->euler) {
        UFG_CHECK(p->euler_p > 0 && p->euler_p < 1, "Euler p must be in (0, 1)");
        euler_weights(p->wce_order, p->euler_p, pc.w);
      } else {
        for (int m = 0; m <= pc.order; ++m) pc.w[m] = 1.0;
      }
      break;
    default:
      set_error("unknown preconditioner kind");
      return UFG_EINVAL;
  }
  *out = pc;
  return UFG_OK;
}

// ---------------------------------------------------------------------------

template <typename R>
static int basis_change(const Lattice& L, const R* mat, const C2<R>* x, C2<R>* y, int nrhs,
                        const int* gate, const R* pre, const R* post, double2 alpha,
                        const C2<R>* aux, double2 beta) {
  HopArgs<R> a;
  a.src = x;
  a.dst = y;
  a.mat = mat;
  a.shift = kShiftNone;
  a.nrhs = nrhs;
  a.gate = gate;
  a.pre = pre;
  a.post = post;
  a.alpha = alpha;
  a.aux = aux;
  a.beta = beta;
  return launch_hop<R>(L, a);
}

// y = W_d x (adjoint: W_d^T x). Uses three temporaries.
// The truncated series sum_m w_m K^m M0^{-1} x (K = -A M0^{-1} M1) is evaluated
// in Horner form, z_d = w_d u_0, z_m = w_m u_0 + K z_{m+1}: the last basis
// change of each K application adds w_m u_0 itself (alpha / beta form), so no
// separate accumulation pass runs. The adjoint is the transpose of the same
// polynomial: M0^{-T} (sum_m w_m K'^m x), K' = A S U^3 [(1 - lam Z^T)^{-1} - 1] U^3T.
template <typename R>
static int wce_apply(Lattice& L, const PcPlan& pc, bool adjoint, const C2<R>* x, C2<R>* y,
                     int nrhs, const int* gate, Counters* cnt,
                     const PcSource<R>* src = nullptr) {
  const Fields<R>& F = fields<R>(L);
  int rc = 0;
  C2<R>* tmp = slot_vec<R>(L, SLOT_PC0 + 0, nrhs, &rc);
  UFG_TRY(rc);
  C2<R>* cur = slot_vec<R>(L, SLOT_PC0 + 1, nrhs, &rc);
  UFG_TRY(rc);
  const double2 one{1.0, 0.0}, zero{0.0, 0.0};
  const double A = L.A;
  const int d = pc.order;
  // With the block form of U (streaming-supported nx), consecutive orders meet
  // as U^3 then U^3T with only per-site factors between them: one launch does
  // both (launch_basis_pair), and z_m is stored only where it is needed again.
  const bool pair = d > 0 && stream_supported(L) && !L.mode_perm.empty();
  if (src && (!pair || src->out != x)) {
    set_error("weak-coupling apply: fused source without the paired basis changes");
    return UFG_EINVAL;
  }
  // the first change U^3T x; with a fused source x is formed (and stored) here
  auto first_change = [&]() -> int {
    HopArgs<R> a;
    a.src = x;
    a.dst = tmp;
    a.mat = F.Ut;
    a.shift = kShiftNone;
    a.nrhs = nrhs;
    a.gate = gate;
    if (src) {
      a.src_mode = src->mode;
      a.fr = src->r;
      a.fp = src->p;
      a.fv = src->v;
      a.fpnew = src->out;
      a.st = src->st;
    }
    return launch_hop<R>(L, a);
  };
  if (pair && !adjoint) {
    C2<R>* u0 = slot_vec<R>(L, SLOT_PC0 + 2, nrhs, &rc);
    UFG_TRY(rc);
    // mode space of u_0 = M0^{-1} x; then u_0 itself and U^3T (sin sigma u_0)
    UFG_TRY(first_change());
    UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, false, false, gate));
    cnt->m0inv += 1;
    UFG_TRY(launch_basis_pair<R>(L, tmp, tmp, u0, nullptr, one, nullptr, zero, F.sn, nrhs, gate));
    double scale = pc.w[d];
    for (int m = d - 1; m >= 0; --m) {
      // tmp holds U^3T (sin sigma z_{m+1}) up to `scale`; z_m = w_m u_0 + K z_{m+1}
      UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, false, true, gate));
      const double2 al{A * scale, 0.0}, be{pc.w[m], 0.0};
      if (m > 0) {
        UFG_TRY(launch_basis_pair<R>(L, tmp, tmp, nullptr, nullptr, al, u0, be, F.sn, nrhs,
                                     gate));
      } else {
        UFG_TRY(basis_change<R>(L, F.U, tmp, y, nrhs, gate, nullptr, nullptr, al, u0, be));
      }
      scale = 1.0;
      cnt->m0inv += 1;
      cnt->mv += 1;
    }
    return UFG_OK;
  }
  if (pair && adjoint) {
    // z_m = w_m x + K' z_{m+1}, K' v = A S U^3 [(1 - lam Z^T)^{-1} - 1] U^3T v, acc = z_0;
    // y = U^3 (1 - lam Z^T)^{-1} U^3T acc
    UFG_TRY(first_change());
    double scale = pc.w[d];
    for (int m = d - 1; m >= 0; --m) {
      UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, true, true, gate));
      UFG_TRY(launch_basis_pair<R>(L, tmp, tmp, nullptr, F.sn, double2{A * scale, 0.0}, x,
                                   double2{pc.w[m], 0.0}, nullptr, nrhs, gate));
      scale = 1.0;
      cnt->m0inv += 1;
      cnt->mv += 1;
    }
    UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, true, false, gate));
    UFG_TRY(basis_change<R>(L, F.U, tmp, y, nrhs, gate, nullptr, nullptr, one, nullptr, zero));
    cnt->m0inv += 1;
    return UFG_OK;
  }
  if (!adjoint) {
    // u_0 = M0^{-1} x
    UFG_TRY(basis_change<R>(L, F.Ut, x, tmp, nrhs, gate, nullptr, nullptr, one, nullptr, zero));
    UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, false, false, gate));
    cnt->m0inv += 1;
    if (d == 0) {
      return basis_change<R>(L, F.U, tmp, y, nrhs, gate, nullptr, nullptr,
                             double2{pc.w[0], 0.0}, nullptr, zero);
    }
    C2<R>* u0 = slot_vec<R>(L, SLOT_PC0 + 2, nrhs, &rc);
    UFG_TRY(rc);
    UFG_TRY(basis_change<R>(L, F.U, tmp, u0, nrhs, gate, nullptr, nullptr, one, nullptr, zero));
    // K v = A U^3 [(1 - lam Z)^{-1} - 1] U^3T (sin sigma v); z_m = w_m u_0 + K z_{m+1}
    const C2<R>* src = u0;
    double scale = pc.w[d];
    for (int m = d - 1; m >= 0; --m) {
      C2<R>* dst = (m == 0) ? y : cur;
      UFG_TRY(basis_change<R>(L, F.Ut, src, tmp, nrhs, gate, F.sn, nullptr, one, nullptr, zero));
      UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, false, true, gate));
      UFG_TRY(basis_change<R>(L, F.U, tmp, dst, nrhs, gate, nullptr, nullptr,
                              double2{A * scale, 0.0}, u0, double2{pc.w[m], 0.0}));
      src = dst;
      scale = 1.0;
      cnt->m0inv += 1;
      cnt->mv += 1;
    }
  } else {
    // acc = sum_m w_m K'^m x in Horner form (z_m = w_m x + K' z_{m+1}), then
    // y = M0^{-T} acc
    const C2<R>* acc = x;
    double scale = pc.w[0];
    if (d > 0) {
      const C2<R>* src = x;
      double s = pc.w[d];
      for (int m = d - 1; m >= 0; --m) {
        UFG_TRY(basis_change<R>(L, F.Ut, src, tmp, nrhs, gate, nullptr, nullptr, one, nullptr,
                                zero));
        UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, true, true, gate));
        UFG_TRY(basis_change<R>(L, F.U, tmp, cur, nrhs, gate, nullptr, F.sn, double2{A * s, 0.0},
                                x, double2{pc.w[m], 0.0}));
        src = cur;
        s = 1.0;
        cnt->m0inv += 1;
        cnt->mv += 1;
      }
      acc = cur;
      scale = 1.0;
    }
    UFG_TRY(basis_change<R>(L, F.Ut, acc, tmp, nrhs, gate, nullptr, nullptr,
                            double2{scale, 0.0}, nullptr, zero));
    UFG_TRY(launch_m0_temporal<R>(L, tmp, tmp, nrhs, true, false, gate));
    UFG_TRY(basis_change<R>(L, F.U, tmp, y, nrhs, gate, nullptr, nullptr, one, nullptr, zero));
    cnt->m0inv += 1;
  }
  return UFG_OK;
}

// y = P(Q^) x, bit-reversal order. y must not alias x.
template <typename R>
static int cheb_apply(Lattice& L, const PcPlan& pc, const C2<R>* x, C2<R>* y, int nrhs,
                      const int* gate, Counters* cnt) {
  const Fields<R>& F = fields<R>(L);
  int rc = 0;
  C2<R>* tmp = slot_vec<R>(L, SLOT_PC0 + 3, nrhs, &rc);
  UFG_TRY(rc);
  const std::complex<double> cf(pc.cf.x, pc.cf.y);
  const C2<R>* cur = x;
  for (size_t i = 0; i < pc.roots.size(); ++i) {
    const std::complex<double> z(pc.roots[i].x, pc.roots[i].y);
    const std::complex<double> al = cf / pc.lam_max, be = -cf * z;
    UFG_TRY(op_apply<R>(L, UFG_OP_M, cur, tmp, nrhs, gate));
    HopArgs<R> a;
    a.src = tmp;
    a.id = tmp;
    a.dst = y;
    a.aux = cur;
    a.alpha = double2{al.real(), al.imag()};
    a.beta = double2{be.real(), be.imag()};
    a.mat = F.T;
    a.shift = kShiftMdag;
    a.post = F.b;
    a.nrhs = nrhs;
    a.gate = gate;
    UFG_TRY(launch_hop<R>(L, a));
    cur = y;
    cnt->mv += 2;
  }
  return UFG_OK;
}

// y = P(S Q / lam_max) S x: the strong-coupling inverse S first, then the
// Chebyshev factors of the S-preconditioned operator (bit-reversal order,
// c^{1/2n} each). A factor is M, M^T, the SCA sweep and an axpby.
template <typename R>
static int sca_cheb_apply(Lattice& L, const PcPlan& pc, const C2<R>* x, C2<R>* y, int nrhs,
                          const int* gate, Counters* cnt) {
  int rc = 0;
  C2<R>* t1 = slot_vec<R>(L, SLOT_PC0 + 3, nrhs, &rc);
  UFG_TRY(rc);
  C2<R>* t2 = slot_vec<R>(L, SLOT_PC0 + 5, nrhs, &rc);
  UFG_TRY(rc);
  UFG_TRY(launch_sca_apply<R>(L, x, y, nrhs, gate));
  cnt->sca += 1;
  const std::complex<double> cf(pc.cf.x, pc.cf.y);
  for (size_t i = 0; i < pc.roots.size(); ++i) {
    const std::complex<double> z(pc.roots[i].x, pc.roots[i].y);
    const std::complex<double> al = cf / pc.lam_max, be = -cf * z;
    UFG_TRY(op_apply<R>(L, UFG_OP_M, y, t1, nrhs, gate));
    UFG_TRY(op_apply<R>(L, UFG_OP_MDAG, t1, t2, nrhs, gate));
    UFG_TRY(launch_sca_apply<R>(L, t2, t1, nrhs, gate));
    UFG_TRY(k_axpby<R>(L, double2{al.real(), al.imag()}, t1, double2{be.real(), be.imag()}, y,
                       nrhs, gate));
    cnt->mv += 2;
    cnt->sca += 1;
  }
  return UFG_OK;
}

template <typename R>
static int q_pc_apply(Lattice& L, const PcPlan& pc, const C2<R>* x, C2<R>* y, int nrhs,
                      const int* gate, Counters* cnt) {
  switch (pc.kind) {
    case UFG_PC_CHEB:
      return cheb_apply<R>(L, pc, x, y, nrhs, gate, cnt);
    case UFG_PC_SCA_CHEB:
      return sca_cheb_apply<R>(L, pc, x, y, nrhs, gate, cnt);
    case UFG_PC_SCA:
      cnt->sca += 1;
      return launch_sca_apply<R>(L, x, y, nrhs, gate);
    case UFG_PC_WCE: {
      int rc = 0;
      C2<R>* mid = slot_vec<R>(L, SLOT_PC0 + 3, nrhs, &rc);
      UFG_TRY(rc);
      UFG_TRY(wce_apply<R>(L, pc, true, x, mid, nrhs, gate, cnt));
      return wce_apply<R>(L, pc, false, mid, y, nrhs, gate, cnt);
    }
    default:
      set_error("bad preconditioner");
      return UFG_EINVAL;
  }
}

bool pc_fuses_source(const Lattice& L, const PcPlan& pc, int op) {
  return pc.kind == UFG_PC_WCE && op != UFG_OP_Q && pc.order > 0 && stream_supported(L) &&
         !L.mode_perm.empty();
}

template <typename R>
int pc_apply(Lattice& L, const PcPlan& pc, int op, const C2<R>* x, C2<R>* y, int nrhs,
             const int* gate, Counters* cnt, const PcSource<R>* src) {
  if (src && !pc_fuses_source(L, pc, op)) {
    set_error("preconditioner: no fused source for this plan");
    return UFG_EINVAL;
  }
  if (src)
    return wce_apply<R>(L, pc, op == UFG_OP_MDAG, x, y, nrhs, gate, cnt, src);
  if (pc.kind == UFG_PC_NONE) return k_axpby<R>(L, double2{1.0, 0.0}, x, double2{0.0, 0.0}, y,
                                                 nrhs, gate);
  if (op == UFG_OP_Q) return q_pc_apply<R>(L, pc, x, y, nrhs, gate, cnt);
  if (pc.kind == UFG_PC_WCE) return wce_apply<R>(L, pc, op == UFG_OP_MDAG, x, y, nrhs, gate, cnt);
  // Chebyshev / SCA for M or M^T: K^{-1} = P M^T (for M), M P (for M^T)
  int rc = 0;
  C2<R>* mid = slot_vec<R>(L, SLOT_PC0 + 4, nrhs, &rc);
  UFG_TRY(rc);
  if (op == UFG_OP_M) {
    UFG_TRY(op_apply<R>(L, UFG_OP_MDAG, x, mid, nrhs, gate));
    cnt->mv += 1;
    return q_pc_apply<R>(L, pc, mid, y, nrhs, gate, cnt);
  }
  UFG_TRY(q_pc_apply<R>(L, pc, x, mid, nrhs, gate, cnt));
  cnt->mv += 1;
  return op_apply<R>(L, UFG_OP_M, mid, y, nrhs, gate);
}

// Largest eigenvalue of Q (sq = false) or of S Q (sq = true) by 30 power
// iterations in FP64 from a deterministic start, times 1.05. S Q is similar to
// the Hermitian S^{1/2} Q S^{1/2}, so its dominant eigenvalue is real and
// positive and |A v| / |v| converges to it.
static int power_lam_max(Lattice& L, bool sq, double* out) {
  int rc = 0;
  double2* v = slot_vec<double>(L, SLOT_POWER, 1, &rc);
  UFG_TRY(rc);
  double2* w = slot_vec<double>(L, SLOT_POWER2, 1, &rc);
  UFG_TRY(rc);
  double2* tmp = slot_vec<double>(L, SLOT_PC0 + 5, 1, &rc);
  UFG_TRY(rc);
  std::vector<double2> h(L.N);
  for (long long i = 0; i < L.N; ++i) h[i] = double2{1.0 + 0.5 * std::sin(0.7 * i), 0.0};
  UFG_HIP(hipMemcpyAsync(v, h.data(), sizeof(double2) * L.N, hipMemcpyHostToDevice, L.stream));
  KrylovState K;
  UFG_TRY(krylov_state(L, 1, &K, SLOT_PSTATE));
  const int nvb = vec_blocks(L, 1);
  double lam = 0.0;
  RhsState hs;
  for (int it = 0; it < 30; ++it) {
    if (sq) {
      UFG_TRY(q_apply<double>(L, v, w, tmp, 1, nullptr));
      UFG_TRY(launch_sca_apply<double>(L, tmp, w, 1, nullptr));
    } else {
      UFG_TRY(q_apply<double>(L, v, tmp, w, 1, nullptr));
    }
    UFG_TRY(k_reduce<double>(L, w, nullptr, 0, nullptr, K));
    UFG_TRY(k_finalize(L, FIN_NORM, nvb, nullptr, K));
    UFG_HIP(hipMemcpyAsync(&hs, K.st, sizeof(RhsState), hipMemcpyDeviceToHost, L.stream));
    UFG_HIP(hipStreamSynchronize(L.stream));
    const double nw = std::sqrt(hs.r2);
    if (!(nw > 0)) {
      set_error("power iteration failed");
      return UFG_EHIP;
    }
    // |A v| / |v| with |v| = 1 after the first step
    if (it > 0) lam = nw;
    UFG_TRY(k_axpby<double>(L, double2{1.0 / nw, 0.0}, w, double2{0.0, 0.0}, v, 1, nullptr));
  }
  *out = 1.05 * lam;
  return UFG_OK;
}

int estimate_lam_max(Lattice& L, double* out) {
  if (!L.lam_max_valid) {
    UFG_TRY(power_lam_max(L, false, &L.lam_max_cache));
    L.lam_max_valid = 1;
  }
  *out = L.lam_max_cache;
  return UFG_OK;
}

int estimate_lam_max_sq(Lattice& L, double alpha, double* out) {
  if (!L.lam_max_sq_valid || L.lam_max_sq_alpha != alpha) {
    if (L.sca_alpha != alpha) UFG_TRY(launch_sca_setup(L, alpha));
    UFG_TRY(power_lam_max(L, true, &L.lam_max_sq_cache));
    L.lam_max_sq_alpha = alpha;
    L.lam_max_sq_valid = 1;
  }
  *out = L.lam_max_sq_cache;
  return UFG_OK;
}

#define INST_OPS(R)                                                                              \
  template int op_apply<R>(const Lattice&, int, const C2<R>*, C2<R>*, int, const int*, int,      \
                           const C2<R>*, double*);                                               \
  template int op_residual<R>(const Lattice&, int, const C2<R>*, const C2<R>*, C2<R>*, int,      \
                              const int*);                                                       \
  template int q_apply<R>(const Lattice&, const C2<R>*, C2<R>*, C2<R>*, int, const int*, int,    \
                          const C2<R>*, double*);                                                \
  template int q_residual<R>(const Lattice&, const C2<R>*, const C2<R>*, C2<R>*, C2<R>*, int,    \
                             const int*);                                                        \
  template int pc_apply<R>(Lattice&, const PcPlan&, int, const C2<R>*, C2<R>*, int, const int*, \
                           Counters*, const PcSource<R>*);
INST_OPS(float)
INST_OPS(double)

}  // namespace ufg
