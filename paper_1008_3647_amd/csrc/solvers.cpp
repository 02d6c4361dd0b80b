// Krylov solvers of the paper (Sec. 1): CG on the normal equations (Eq. 1,
// left/"PCG" preconditioning, Eq. 3) and BiCGStab (van der Vorst) for M and
// M^T, alone or as the two-step solve M^T y = b, M x = y (Eq. 2), right
// preconditioned so that the iterated residual is that of the original system.
//
// Precision modes
//   plain : every vector in the lattice dtype; the final residual is
//           recomputed from scratch before a right-hand side is declared
//           converged ("reliable update" in the working precision).
//   mixed : complex64 inner iteration; x, b and the true residual stay in
//           complex128. Whenever the inner residual falls below delta times
//           its maximum since the last update (Sleijpen & van der Vorst's
//           reliable updates), x64 += x32, r64 = b - A x64 in FP64, the inner
//           residual restarts from r64 and the search direction is kept.
// All scalar arithmetic is FP64 on the device; the host only enqueues kernels
// and reads the per-rhs "active" flags every check_every iterations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "hop_stream.h"
#include "ops.h"

namespace ufg {

namespace {

// One check interval of a solver's iterations, captured once on a private
// stream and replayed on the lattice's stream. Small lattices run hundreds of
// short launches per interval; a replay submits them at once. The body must
// hold kernel launches only (no allocation, memset or copy): it runs after the
// first interval has been launched eagerly, so every workspace and function
// attribute exists already. Counters advanced by the host code of the body are
// counted per replay.
struct IntervalGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  hipStream_t cs = nullptr;
  Counters delta;
  ~IntervalGraph() {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
  template <typename F>
  int capture(Lattice& L, Counters* cnt, F&& body) {
    if (!cs) UFG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const Counters before = *cnt;
    hipStream_t saved = L.stream;
    L.stream = cs;
    const hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int brc = (eb == hipSuccess) ? body() : UFG_EHIP;
    hipGraph_t graph = nullptr;
    const hipError_t ee = (eb == hipSuccess) ? hipStreamEndCapture(cs, &graph) : eb;
    L.stream = saved;
    g = graph;
    if (eb != hipSuccess || ee != hipSuccess) {
      (void)hipGetLastError();
      set_error("solver: graph capture failed");
      return UFG_EHIP;
    }
    UFG_TRY(brc);
    UFG_HIP(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    delta.mv = cnt->mv - before.mv;
    delta.m0inv = cnt->m0inv - before.m0inv;
    delta.sca = cnt->sca - before.sca;
    *cnt = before;
    return UFG_OK;
  }
  int replay(const Lattice& L, Counters* cnt) {
    UFG_HIP(hipGraphLaunch(e, L.stream));
    cnt->mv += delta.mv;
    cnt->m0inv += delta.m0inv;
    cnt->sca += delta.sca;
    return UFG_OK;
  }
};

struct StepResult {
  int iters = 0;
  int status = 0;
  long long updates = 0;
};

template <typename R>
struct Inner {
  C2<R> *x, *r, *rhat, *p, *v, *s, *t, *phat, *shat, *z, *w, *tmp;
};

template <typename R>
int inner_vectors(Lattice& L, int nrhs, bool need_pc, bool mixed, C2<R>* x_user, Inner<R>* V) {
  int rc = 0;
  C2<R>* slots[12];
  for (int i = 0; i < 12; ++i) {
    slots[i] = slot_vec<R>(L, SLOT_SOLVER0 + i, nrhs, &rc);
    UFG_TRY(rc);
  }
  V->x = mixed ? slots[0] : x_user;
  V->r = slots[1];
  V->rhat = slots[2];
  V->p = slots[3];
  V->v = slots[4];
  V->s = slots[5];
  V->t = slots[6];
  V->phat = need_pc ? slots[7] : V->p;
  V->shat = need_pc ? slots[8] : V->s;
  V->z = need_pc ? slots[9] : V->r;
  V->w = slots[10];
  V->tmp = slots[11];
  return UFG_OK;
}

// Copies active, update and restart flags (3 nrhs ints) to the host.
int read_flags(Lattice& L, const KrylovState& K, int* host_flags, bool* done) {
  UFG_HIP(hipMemcpyAsync(host_flags, K.active, 3 * sizeof(int) * K.nrhs, hipMemcpyDeviceToHost,
                         L.stream));
  UFG_HIP(hipStreamSynchronize(L.stream));
  *done = true;
  for (int i = 0; i < K.nrhs; ++i)
    if (host_flags[i]) *done = false;
  return UFG_OK;
}

int read_states(Lattice& L, const KrylovState& K, std::vector<RhsState>* out) {
  out->resize(K.nrhs);
  UFG_HIP(hipMemcpyAsync(out->data(), K.st, sizeof(RhsState) * K.nrhs, hipMemcpyDeviceToHost,
                         L.stream));
  UFG_HIP(hipStreamSynchronize(L.stream));
  return UFG_OK;
}

// Worst relative true residual ||b - A x|| / ||b|| over the rhs, FP64 when RO = double.
template <typename RO>
int true_relres(Lattice& L, int op, const C2<RO>* x, const C2<RO>* b, int nrhs, double* worst) {
  int rc = 0;
  C2<RO>* res = slot_vec<RO>(L, SLOT_OUTER_T, nrhs, &rc);
  UFG_TRY(rc);
  KrylovState K;
  UFG_TRY(krylov_state(L, nrhs, &K, SLOT_PSTATE));
  const int nvb = vec_blocks(L, nrhs);
  if (op == UFG_OP_Q) {
    C2<RO>* tmp = slot_vec<RO>(L, SLOT_OUTER_R + 3, nrhs, &rc);  // slot 15
    UFG_TRY(rc);
    UFG_TRY(q_residual<RO>(L, x, b, tmp, res, nrhs, nullptr));
  } else {
    UFG_TRY(op_residual<RO>(L, op, x, b, res, nrhs, nullptr));
  }
  UFG_TRY(k_reduce<RO>(L, b, nullptr, 0, nullptr, K));
  UFG_TRY(k_finalize(L, FIN_INIT_B, nvb, nullptr, K));
  UFG_TRY(k_reduce<RO>(L, res, nullptr, 0, nullptr, K));
  UFG_TRY(k_finalize(L, FIN_NORM, nvb, nullptr, K));
  std::vector<RhsState> st;
  UFG_TRY(read_states(L, K, &st));
  double w = 0.0;
  for (auto& q : st) {
    const double rr = q.b2 > 0 ? std::sqrt(q.r2 / q.b2) : std::sqrt(q.r2);
    if (!(rr <= w)) w = rr;  // NaN propagates as worst
  }
  *worst = w;
  return UFG_OK;
}

// ---------------------------------------------------------------------------
// BiCGStab for A = op (M or M^T) on nrhs systems.
//   RI: inner precision; RO: precision of b and x (RO == RI unless mixed).
template <typename RI, typename RO>
int bicgstab_step(Lattice& L, const PcPlan& pc, int op, const C2<RO>* b, C2<RO>* x, int nrhs,
                  const ufg_solve_opts& o, Counters* cnt, StepResult* res) {
  constexpr bool kMixed = !std::is_same<RI, RO>::value;
  const bool need_pc = pc.kind != UFG_PC_NONE;
  Inner<RI> V;
  UFG_TRY(inner_vectors<RI>(L, nrhs, need_pc, kMixed, reinterpret_cast<C2<RI>*>(x), &V));
  KrylovState K;
  UFG_TRY(krylov_state(L, nrhs, &K, SLOT_STATE));
  K.prm.tol = o.tol;
  K.prm.delta2 = o.delta * o.delta;
  K.prm.mixed = kMixed ? 1 : 0;
  K.prm.bicg = 1;
  K.prm.unprec = need_pc ? 0 : 1;
  // The operator itself, and M with the weak-coupling series, have complex
  // spectra; the Q-type preconditioners composed with M^T or M make the
  // preconditioned operator Hermitian-like, where the limit only slows it.
  K.prm.limit_omega = (pc.kind == UFG_PC_NONE || pc.kind == UFG_PC_WCE) ? 1 : 0;
  const int nvb = vec_blocks(L, nrhs);
  const int nhb = hop_blocks_per_rhs(L);
  const double2 one{1.0, 0.0}, zero{0.0, 0.0};
  int rc = 0;
  C2<RO>* r64 = kMixed ? slot_vec<RO>(L, SLOT_OUTER_R, nrhs, &rc) : nullptr;
  UFG_TRY(rc);

  // ||b||^2
  UFG_TRY(k_reduce<RO>(L, b, nullptr, 0, nullptr, K));
  UFG_TRY(k_finalize(L, FIN_INIT_B, nvb, nullptr, K));
  // r_0 = b - A x_0 (x_0 = 0 unless use_x0)
  if (kMixed) {
    if (o.use_x0) {
      UFG_TRY(op_residual<RO>(L, op, x, b, r64, nrhs, nullptr));
    } else {
      UFG_HIP(hipMemsetAsync(x, 0, sizeof(C2<RO>) * L.N * nrhs, L.stream));
      UFG_TRY(k_convert<RO, RO>(L, b, r64, nrhs, nullptr));
    }
    UFG_HIP(hipMemsetAsync(V.x, 0, sizeof(C2<RI>) * L.N * nrhs, L.stream));
    UFG_TRY(k_convert<RO, RI>(L, r64, V.r, nrhs, nullptr));
  } else {
    if (o.use_x0) {
      UFG_TRY(op_residual<RI>(L, op, V.x, reinterpret_cast<const C2<RI>*>(b), V.r, nrhs, nullptr));
    } else {
      UFG_HIP(hipMemsetAsync(V.x, 0, sizeof(C2<RI>) * L.N * nrhs, L.stream));
      UFG_TRY(k_convert<RI, RI>(L, reinterpret_cast<const C2<RI>*>(b), V.r, nrhs, nullptr));
    }
  }
  UFG_TRY(k_convert<RI, RI>(L, V.r, V.rhat, nrhs, nullptr));
  UFG_HIP(hipMemsetAsync(V.p, 0, sizeof(C2<RI>) * L.N * nrhs, L.stream));
  UFG_HIP(hipMemsetAsync(V.v, 0, sizeof(C2<RI>) * L.N * nrhs, L.stream));
  if (kMixed) {
    UFG_TRY(k_reduce<RO>(L, r64, nullptr, 0, nullptr, K));
  } else {
    UFG_TRY(k_reduce<RI>(L, V.r, nullptr, 0, nullptr, K));
  }
  UFG_TRY(k_finalize(L, FIN_INIT_R, nvb, nullptr, K));

  // Unpreconditioned BiCGStab with the streaming operator runs fused. s = r -
  // alpha v is formed on the fly by the second operator launch (t = A s) and
  // again by the x, r update, so s is never stored. Between check points the
  // x, r update of an iteration is merged with the p update of the next one
  // (one vector pass instead of two): the second operator launch also reduces
  // <rhat, s> and <rhat, t>, which give rho of the next iteration as
  // <rhat, r - alpha v - omega t> before r is formed, hence beta; the first
  // launch of the next iteration is then a plain v = A p. Iterations that end
  // at a check point run the separate x, r update (rho from r itself) so that
  // x and r are current there, and the iteration after a check point forms p
  // inside the first operator launch; p and v then alternate between two
  // buffers (a workgroup reads the halo slice of the previous iterate while
  // its neighbour writes the new one).
  const bool fused = !need_pc && stream_supported(L);
  C2<RI>* P2[2] = {V.p, nullptr};
  C2<RI>* V2[2] = {V.v, nullptr};
  if (fused) {
    P2[1] = slot_vec<RI>(L, SLOT_SOLVER0 + 7, nrhs, &rc);
    UFG_TRY(rc);
    V2[1] = slot_vec<RI>(L, SLOT_SOLVER0 + 8, nrhs, &rc);
    UFG_TRY(rc);
  }
  const Fields<RI>& F = fields<RI>(L);

  // reliable update / convergence check for the rhs whose update flag is set
  auto reliable_update = [&]() -> int {
    if (kMixed) {
      UFG_TRY(k_promote(L, reinterpret_cast<double2*>(x), reinterpret_cast<float2*>(V.x), nrhs,
                        K.update));
      UFG_TRY(op_residual<RO>(L, op, x, b, r64, nrhs, K.update));
      UFG_TRY(k_demote(L, reinterpret_cast<const double2*>(r64), reinterpret_cast<float2*>(V.r),
                       reinterpret_cast<const float2*>(V.rhat), K, K.update));
    } else {
      UFG_TRY(op_residual<RI>(L, op, V.x, reinterpret_cast<const C2<RI>*>(b), V.r, nrhs,
                              K.update));
      UFG_TRY(k_reduce<RI>(L, V.r, V.rhat, 3, K.update, K));
    }
    return k_finalize(L, FIN_UPDATE, nvb, K.update, K);
  };
  auto restart = [&]() -> int {
    UFG_TRY(k_restart<RI>(L, V.r, V.rhat, P2[0], V2[0], K));
    if (fused) UFG_TRY(k_restart<RI>(L, V.r, V.rhat, P2[1], V2[1], K));
    return k_finalize(L, FIN_RESTART, 1, K.restart, K);
  };

  std::vector<int> hflags(3 * nrhs);
  const int check = o.check_every > 0 ? o.check_every : 10;
  int it = 0;
  bool done = false;
  UFG_TRY(read_flags(L, K, hflags.data(), &done));
  int cur = 0;          // P2[cur], V2[cur] hold the current p and v
  bool merged = false;  // p was formed by the merged x, r, p update
  // one iteration of the unfused form (preconditioned, or a lattice without
  // the streaming kernel); whole check intervals of it replay from a graph
  // a weak-coupling preconditioner forms p and s in its first basis change
  const bool fuse_src = need_pc && pc_fuses_source(L, pc, op);
  auto classic_iteration = [&]() -> int {
    if (fuse_src) {
      PcSource<RI> ps;
      ps.mode = 1;
      ps.r = V.r;
      ps.p = V.p;
      ps.v = V.v;
      ps.out = V.p;
      ps.st = K.st;
      UFG_TRY(pc_apply<RI>(L, pc, op, V.p, V.phat, nrhs, K.active, cnt, &ps));
    } else {
      UFG_TRY(k_bicg_p<RI>(L, V.r, V.p, V.v, K));
      if (need_pc) UFG_TRY(pc_apply<RI>(L, pc, op, V.p, V.phat, nrhs, K.active, cnt));
    }
    UFG_TRY(op_apply<RI>(L, op, V.phat, V.v, nrhs, K.active, 1, V.rhat, K.part));
    UFG_TRY(k_finalize(L, FIN_ALPHA, nhb, K.active, K));
    if (fuse_src) {
      PcSource<RI> ps;
      ps.mode = 2;
      ps.r = V.r;
      ps.v = V.v;
      ps.out = V.s;
      ps.st = K.st;
      UFG_TRY(pc_apply<RI>(L, pc, op, V.s, V.shat, nrhs, K.active, cnt, &ps));
    } else {
      UFG_TRY(k_bicg_s<RI>(L, V.r, V.v, V.s, K));
      if (need_pc) UFG_TRY(pc_apply<RI>(L, pc, op, V.s, V.shat, nrhs, K.active, cnt));
    }
    UFG_TRY(op_apply<RI>(L, op, V.shat, V.t, nrhs, K.active, 2, V.s, K.part));
    UFG_TRY(k_finalize(L, FIN_OMEGA, nhb, K.active, K));
    UFG_TRY(k_bicg_xr<RI>(L, V.x, V.phat, V.shat, V.s, V.t, V.r, V.rhat, K));
    UFG_TRY(k_finalize(L, FIN_RHO, nvb, K.active, K));
    cnt->mv += 2;
    return UFG_OK;
  };
  // Check points do not wait for the device. The reliable update and the
  // restart are issued at every check point as launches gated per rhs by
  // their device flags; the flags are then copied behind them to pinned host
  // memory, which the host reads at the next check point, when that copy has
  // long completed. The loop so ends one check interval late, on launches that
  // do nothing (every rhs is inactive by then).
  UFG_TRY(L.flags.ensure(3 * nrhs));
  int posted = 0;
  Counters at_prev_post;  // the counters when the previous flags were posted
  IntervalGraph G;
  for (it = 0; it < o.maxit && !done; ++it) {
    const bool check_it = (it + 1) % check == 0 || it + 1 == o.maxit;
    // a whole check interval after the first one: replay the captured interval
    const bool replay = !fused && !o.eager && it >= check && it % check == 0 &&
                        it + check <= o.maxit;
    if (replay && !G.e) {
      UFG_TRY(G.capture(L, cnt, [&]() -> int {
        for (int k = 0; k < check; ++k) UFG_TRY(classic_iteration());
        return UFG_OK;
      }));
    }
    if (fused) {
      HopArgs<RI> a1;  // v = A p; <rhat, v>
      a1.mat = F.T;
      a1.nrhs = nrhs;
      a1.gate = K.active;
      a1.st = K.st;
      a1.red_mode = 1;
      a1.red_w = V.rhat;
      a1.red_out = K.part;
      if (op == UFG_OP_M) {
        a1.shift = kShiftM;
        a1.pre = F.b;
      } else {
        a1.shift = kShiftMdag;
        a1.post = F.b;
      }
      // a merged FP64 iteration that does not end at a check point leaves its
      // alpha step (FIN_ALPHA_XR) to the prologue of the t = A s launch, which
      // reads the partials of v = A p from part3 (measured at 16^3 x 400: the
      // FP64 solve 1.5 % faster; in FP32 the prologue costs more than the
      // finalize launch it replaces, so FP32 keeps the launch)
      const bool fin_in_hop = merged && !check_it && sizeof(RI) == 8;
      if (merged) {
        a1.src = a1.id = P2[cur];
        a1.dst = V2[cur];
        a1.red_out = K.part3;
        UFG_TRY(launch_hop<RI>(L, a1));
        if (!fin_in_hop) {
          KrylovState K3 = K;
          K3.part = K.part3;
          UFG_TRY(k_finalize(L, FIN_ALPHA_XR, nhb, K.active, K3, 4, nvb));
        }
      } else {  // p_new = r + beta (p - omega v) formed by the launch
        a1.src = a1.id = P2[cur ^ 1];
        a1.dst = V2[cur ^ 1];
        a1.src_mode = 1;
        a1.fr = V.r;
        a1.fp = P2[cur];
        a1.fv = V2[cur];
        a1.fpnew = P2[cur ^ 1];
        UFG_TRY(launch_hop<RI>(L, a1));
        UFG_TRY(k_finalize(L, FIN_ALPHA, nhb, K.active, K));
        cur ^= 1;
      }
      HopArgs<RI> a2 = a1;  // t = A s, s = r - alpha v; <t, s>, |t|^2, |s|^2, <rhat, t>, <rhat, s>
      a2.src = a2.id = V2[cur];
      a2.dst = V.t;
      a2.src_mode = 2;
      a2.fr = V.r;
      a2.fv = V2[cur];
      a2.fp = nullptr;
      a2.fpnew = nullptr;
      a2.red_mode = check_it ? 3 : 4;
      a2.red_w = check_it ? nullptr : V.rhat;
      a2.red_out = K.part;
      if (fin_in_hop) {
        a2.fin_part = K.part3;
        a2.fin_nblk = nhb;
        a2.fin_part2 = K.part2;
        a2.fin_nblk2 = nvb;
        a2.fin_flags = K.active;
        a2.fin_prm = K.prm;
      }
      UFG_TRY(launch_hop<RI>(L, a2));
      if (check_it) {
        UFG_TRY(k_finalize(L, FIN_OMEGA, nhb, K.active, K));
        UFG_TRY(k_bicg_xr_fused<RI>(L, V.x, P2[cur], V.r, V2[cur], V.t, V.rhat, K));
        UFG_TRY(k_finalize(L, FIN_RHO, nvb, K.active, K));
        merged = false;
      } else {
        UFG_TRY(k_finalize(L, FIN_OMEGA_RHO, nhb, K.active, K, 8));
        UFG_TRY(k_bicg_xrp<RI>(L, V.x, P2[cur], V.r, V2[cur], V.t, K));
        merged = true;
      }
      cnt->mv += 2;
    } else if (replay) {
      UFG_TRY(G.replay(L, cnt));
      it += check - 1;  // the interval ends at the check point below
    } else {
      UFG_TRY(classic_iteration());
    }
    if ((it + 1) % check == 0 || it + 1 == o.maxit) {
      UFG_TRY(reliable_update());
      UFG_TRY(restart());
      const int slot = posted & 1;
      int* mirror = L.flags.host + slot * L.flags.cap;
      UFG_HIP(hipMemcpyAsync(mirror, K.active, 3 * sizeof(int) * nrhs, hipMemcpyDeviceToHost,
                             L.stream));
      UFG_HIP(hipEventRecord(L.flags.ev[slot], L.stream));
      ++posted;
      const Counters at_post = *cnt;
      if (posted >= 2) {  // the previous check point's flags
        const int prev = slot ^ 1;
        UFG_HIP(hipEventSynchronize(L.flags.ev[prev]));
        const int* f = L.flags.host + prev * L.flags.cap;
        done = true;
        for (int i = 0; i < nrhs; ++i)
          if (f[i]) done = false;
        // every rhs was inactive when those flags were taken: what was issued
        // since then did no work and is not counted
        if (done) *cnt = at_prev_post;
      }
      at_prev_post = at_post;
    }
  }
  if (kMixed) {
    UFG_TRY(k_promote(L, reinterpret_cast<double2*>(x), reinterpret_cast<float2*>(V.x), nrhs,
                      nullptr));
  }
  std::vector<RhsState> st;
  UFG_TRY(read_states(L, K, &st));
  res->iters = 0;
  res->status = 0;
  for (auto& q : st) {
    res->iters = std::max(res->iters, q.iters);
    res->updates = std::max<long long>(res->updates, q.updates);
    if (q.status) res->status = std::max(res->status, q.status);
    else if (!q.conv) res->status = std::max(res->status, (int)UFG_NOT_CONVERGED);
  }
  (void)one;
  (void)zero;
  return UFG_OK;
}

// ---------------------------------------------------------------------------
// CG on Q = M^T M with an HPD preconditioner; or, with `split` (a weak-coupling
// plan E = W_d), CG with split preconditioning (paper, Sec. 5, the remark
// after Table 2): CG on A' = E^T Q E with right-hand side b' = E^T b, whose
// residual the stop rule measures, and x = E z at the end (no preconditioner,
// no mixed precision, x_0 = 0).
template <typename RI, typename RO>
int cg_solve(Lattice& L, const PcPlan& pc, const C2<RO>* b, C2<RO>* x, int nrhs,
             const ufg_solve_opts& o, Counters* cnt, StepResult* res,
             const PcPlan* split = nullptr) {
  constexpr bool kMixed = !std::is_same<RI, RO>::value;
  const bool need_pc = pc.kind != UFG_PC_NONE;
  if (split && (kMixed || need_pc || o.use_x0)) {
    set_error("split-preconditioned CG: no second preconditioner, no mixed precision, x_0 = 0");
    return UFG_EINVAL;
  }
  Inner<RI> V;
  UFG_TRY(inner_vectors<RI>(L, nrhs, need_pc, kMixed, reinterpret_cast<C2<RI>*>(x), &V));
  // split form: b' and two temporaries in solver slots the unpreconditioned
  // iteration leaves free
  C2<RI>* bsp = nullptr;
  C2<RI>* ep = nullptr;
  C2<RI>* qy = nullptr;
  if (split) {
    int src = 0;
    bsp = slot_vec<RI>(L, SLOT_SOLVER0 + 7, nrhs, &src);
    UFG_TRY(src);
    ep = slot_vec<RI>(L, SLOT_SOLVER0 + 8, nrhs, &src);
    UFG_TRY(src);
    qy = slot_vec<RI>(L, SLOT_SOLVER0 + 9, nrhs, &src);
    UFG_TRY(src);
    UFG_TRY(pc_apply<RI>(L, *split, UFG_OP_MDAG, reinterpret_cast<const C2<RI>*>(b), bsp, nrhs,
                         nullptr, cnt));
    b = reinterpret_cast<const C2<RO>*>(bsp);
  }
  // w = A' v (split form) on the rhs of `gate`
  auto split_apply = [&](const C2<RI>* v, C2<RI>* w, const int* gate) -> int {
    UFG_TRY(pc_apply<RI>(L, *split, UFG_OP_M, v, ep, nrhs, gate, cnt));
    UFG_TRY(q_apply<RI>(L, ep, V.tmp, qy, nrhs, gate));
    return pc_apply<RI>(L, *split, UFG_OP_MDAG, qy, w, nrhs, gate, cnt);
  };
  KrylovState K;
  UFG_TRY(krylov_state(L, nrhs, &K, SLOT_STATE));
  K.prm.tol = o.tol;
  K.prm.delta2 = o.delta * o.delta;
  K.prm.mixed = kMixed ? 1 : 0;
  K.prm.bicg = 0;
  K.prm.unprec = need_pc ? 0 : 1;
  const int nvb = vec_blocks(L, nrhs);
  const int nhb = hop_blocks_per_rhs(L);
  int rc = 0;
  C2<RO>* r64 = kMixed ? slot_vec<RO>(L, SLOT_OUTER_R, nrhs, &rc) : nullptr;
  UFG_TRY(rc);
  C2<RO>* t64 = kMixed ? slot_vec<RO>(L, SLOT_OUTER_Y + 2, nrhs, &rc) : nullptr;  // slot 15
  UFG_TRY(rc);

  UFG_TRY(k_reduce<RO>(L, b, nullptr, 0, nullptr, K));
  UFG_TRY(k_finalize(L, FIN_INIT_B, nvb, nullptr, K));
  if (kMixed) {
    if (o.use_x0) {
      UFG_TRY(q_residual<RO>(L, x, b, t64, r64, nrhs, nullptr));
    } else {
      UFG_HIP(hipMemsetAsync(x, 0, sizeof(C2<RO>) * L.N * nrhs, L.stream));
      UFG_TRY(k_convert<RO, RO>(L, b, r64, nrhs, nullptr));
    }
    UFG_HIP(hipMemsetAsync(V.x, 0, sizeof(C2<RI>) * L.N * nrhs, L.stream));
    UFG_TRY(k_convert<RO, RI>(L, r64, V.r, nrhs, nullptr));
    UFG_TRY(k_reduce<RO>(L, r64, nullptr, 0, nullptr, K));
  } else {
    const C2<RI>* bi = reinterpret_cast<const C2<RI>*>(b);
    if (o.use_x0) {
      UFG_TRY(q_residual<RI>(L, V.x, bi, V.tmp, V.r, nrhs, nullptr));
    } else {
      UFG_HIP(hipMemsetAsync(V.x, 0, sizeof(C2<RI>) * L.N * nrhs, L.stream));
      UFG_TRY(k_convert<RI, RI>(L, bi, V.r, nrhs, nullptr));
    }
    UFG_TRY(k_reduce<RI>(L, V.r, nullptr, 0, nullptr, K));
  }
  UFG_TRY(k_finalize(L, FIN_INIT_R, nvb, nullptr, K));
  if (need_pc) {
    UFG_TRY(pc_apply<RI>(L, pc, UFG_OP_Q, V.r, V.z, nrhs, nullptr, cnt));
    UFG_TRY(k_reduce<RI>(L, V.r, V.z, 1, nullptr, K));
  }
  UFG_TRY(k_finalize(L, FIN_CG_INIT_RZ, nvb, nullptr, K));
  UFG_TRY(k_convert<RI, RI>(L, V.z, V.p, nrhs, nullptr));

  Counters pc_cost;  // what one refresh of z adds to the counters
  auto reliable_update = [&]() -> int {
    UFG_HIP(hipMemcpyAsync(K.restart, K.update, sizeof(int) * nrhs, hipMemcpyDeviceToDevice,
                           L.stream));
    if (kMixed) {
      UFG_TRY(k_promote(L, reinterpret_cast<double2*>(x), reinterpret_cast<float2*>(V.x), nrhs,
                        K.update));
      UFG_TRY(q_residual<RO>(L, x, b, t64, r64, nrhs, K.update));
      UFG_TRY(k_demote(L, reinterpret_cast<const double2*>(r64), reinterpret_cast<float2*>(V.r),
                       nullptr, K, K.update));
    } else if (split) {  // r' = b' - A' z
      UFG_TRY(split_apply(V.x, V.w, K.update));
      UFG_TRY(k_convert<RI, RI>(L, reinterpret_cast<const C2<RI>*>(b), V.r, nrhs, K.update));
      UFG_TRY(k_axpby<RI>(L, double2{-1.0, 0.0}, V.w, double2{1.0, 0.0}, V.r, nrhs, K.update));
      UFG_TRY(k_reduce<RI>(L, V.r, nullptr, 0, K.update, K));
    } else {
      UFG_TRY(q_residual<RI>(L, V.x, reinterpret_cast<const C2<RI>*>(b), V.tmp, V.r, nrhs,
                             K.update));
      UFG_TRY(k_reduce<RI>(L, V.r, nullptr, 0, K.update, K));
    }
    UFG_TRY(k_finalize(L, FIN_UPDATE, nvb, K.update, K));
    // the search direction is kept; z and rz are refreshed from the new
    // residual of the updated systems (their set travels in the restart
    // flags, which CG does not use otherwise)
    if (need_pc) {
      pc_cost = Counters{};
      UFG_TRY(pc_apply<RI>(L, pc, UFG_OP_Q, V.r, V.z, nrhs, K.restart, &pc_cost));
      UFG_TRY(k_reduce<RI>(L, V.r, V.z, 1, K.restart, K));
    }
    return k_finalize(L, FIN_CG_INIT_RZ, nvb, K.restart, K);
  };

  std::vector<int> hflags(3 * nrhs);
  const int check = o.check_every > 0 ? o.check_every : 10;
  bool done = false;
  UFG_TRY(read_flags(L, K, hflags.data(), &done));
  auto iteration = [&]() -> int {
    if (split) {  // w = A' p and <p, w> over the vector blocks
      UFG_TRY(split_apply(V.p, V.w, K.active));
      UFG_TRY(k_reduce<RI>(L, V.p, V.w, 1, K.active, K));
      UFG_TRY(k_finalize(L, FIN_CG_ALPHA, nvb, K.active, K));
    } else {
      UFG_TRY(q_apply<RI>(L, V.p, V.tmp, V.w, nrhs, K.active, 1, V.p, K.part));
      UFG_TRY(k_finalize(L, FIN_CG_ALPHA, nhb, K.active, K));
    }
    UFG_TRY(k_cg_xr<RI>(L, V.x, V.p, V.r, V.w, K));
    UFG_TRY(k_finalize(L, FIN_CG_R, nvb, K.active, K));
    cnt->mv += 2;
    if (need_pc) {
      UFG_TRY(pc_apply<RI>(L, pc, UFG_OP_Q, V.r, V.z, nrhs, K.active, cnt));
      UFG_TRY(k_reduce<RI>(L, V.r, V.z, 1, K.active, K));
    }
    UFG_TRY(k_finalize(L, FIN_CG_BETA, nvb, K.active, K));
    return k_cg_p<RI>(L, V.z, V.p, K);
  };
  // Check points do not wait for the device (as in BiCGStab): the reliable
  // update runs as launches gated per rhs by the device flags, and the flags
  // are read from pinned memory at the next check point. A refresh of z is
  // counted when the flags show that it had work.
  UFG_TRY(L.flags.ensure(3 * nrhs));
  int posted = 0, last_read = 0;
  long long refreshes = 0;
  Counters at_prev_post;
  auto read_posted = [&](int k) -> int {  // flags of the k-th check point (1-based)
    const int slot = (k - 1) & 1;
    UFG_HIP(hipEventSynchronize(L.flags.ev[slot]));
    const int* f = L.flags.host + slot * L.flags.cap;
    done = true;
    bool refreshed = false;
    for (int i = 0; i < nrhs; ++i) {
      if (f[i]) done = false;
      if (f[2 * nrhs + i]) refreshed = true;
    }
    if (refreshed) ++refreshes;
    last_read = k;
    return UFG_OK;
  };
  IntervalGraph G;
  for (int it = 0; it < o.maxit && !done; ++it) {
    // whole check intervals after the first one replay a captured interval
    if (!o.eager && it >= check && it % check == 0 && it + check <= o.maxit) {
      if (!G.e) {
        UFG_TRY(G.capture(L, cnt, [&]() -> int {
          for (int k = 0; k < check; ++k) UFG_TRY(iteration());
          return UFG_OK;
        }));
      }
      UFG_TRY(G.replay(L, cnt));
      it += check - 1;
    } else {
      UFG_TRY(iteration());
    }
    if ((it + 1) % check == 0 || it + 1 == o.maxit) {
      UFG_TRY(reliable_update());
      const int slot = posted & 1;
      UFG_HIP(hipMemcpyAsync(L.flags.host + slot * L.flags.cap, K.active, 3 * sizeof(int) * nrhs,
                             hipMemcpyDeviceToHost, L.stream));
      UFG_HIP(hipEventRecord(L.flags.ev[slot], L.stream));
      ++posted;
      const Counters at_post = *cnt;
      if (posted >= 2) {
        UFG_TRY(read_posted(posted - 1));
        // every rhs had stopped there: the interval issued since did no work
        if (done) *cnt = at_prev_post;
      }
      at_prev_post = at_post;
    }
  }
  if (posted > last_read) UFG_TRY(read_posted(posted));
  cnt->mv += refreshes * pc_cost.mv;
  cnt->m0inv += refreshes * pc_cost.m0inv;
  cnt->sca += refreshes * pc_cost.sca;
  if (kMixed) {
    UFG_TRY(k_promote(L, reinterpret_cast<double2*>(x), reinterpret_cast<float2*>(V.x), nrhs,
                      nullptr));
  }
  if (split) {  // x = E z (z was iterated in x's buffer)
    UFG_TRY(pc_apply<RI>(L, *split, UFG_OP_M, V.x, ep, nrhs, nullptr, cnt));
    UFG_TRY(k_convert<RI, RI>(L, ep, V.x, nrhs, nullptr));
  }
  std::vector<RhsState> st;
  UFG_TRY(read_states(L, K, &st));
  res->iters = 0;
  res->status = 0;
  for (auto& q : st) {
    res->iters = std::max(res->iters, q.iters);
    res->updates = std::max<long long>(res->updates, q.updates);
    if (q.status) res->status = std::max(res->status, q.status);
    else if (!q.conv) res->status = std::max(res->status, (int)UFG_NOT_CONVERGED);
  }
  return UFG_OK;
}

int validate_opts(const Lattice& L, const ufg_solve_opts* o, int nrhs) {
  UFG_CHECK(o != nullptr, "solve options are required");
  UFG_CHECK(nrhs >= 1, "nrhs must be >= 1");
  UFG_CHECK(o->tol > 0 && o->tol < 1, "tol must be in (0, 1)");
  UFG_CHECK(o->maxit >= 1, "maxit must be >= 1");
  UFG_CHECK(!o->mixed || L.dtype == UFG_C128, "mixed solves need a complex128 lattice");
  UFG_CHECK(!o->mixed || (o->delta > 0 && o->delta < 1), "delta must be in (0, 1)");
  return UFG_OK;
}

template <typename RI, typename RO>
int bicgstab_dispatch(Lattice& L, const PcPlan& pc, int op, const void* bv, void* xv, int nrhs,
                      const ufg_solve_opts& o, ufg_solve_stats* st) {
  Counters cnt;
  const C2<RO>* b = reinterpret_cast<const C2<RO>*>(bv);
  C2<RO>* x = reinterpret_cast<C2<RO>*>(xv);
  StepResult r1, r2;
  int rc = 0;
  double rel1 = 0, rel2 = 0, relq = -1;
  if (op == UFG_OP_TWO_STEP) {
    C2<RO>* y = slot_vec<RO>(L, SLOT_OUTER_Y, nrhs, &rc);
    UFG_TRY(rc);
    UFG_TRY((bicgstab_step<RI, RO>(L, pc, UFG_OP_MDAG, b, y, nrhs, o, &cnt, &r1)));
    UFG_TRY(true_relres<RO>(L, UFG_OP_MDAG, y, b, nrhs, &rel1));
    UFG_TRY((bicgstab_step<RI, RO>(L, pc, UFG_OP_M, y, x, nrhs, o, &cnt, &r2)));
    UFG_TRY(true_relres<RO>(L, UFG_OP_M, x, y, nrhs, &rel2));
    UFG_TRY(true_relres<RO>(L, UFG_OP_Q, x, b, nrhs, &relq));
  } else {
    UFG_TRY((bicgstab_step<RI, RO>(L, pc, op, b, x, nrhs, o, &cnt, &r1)));
    UFG_TRY(true_relres<RO>(L, op, x, b, nrhs, &rel1));
  }
  if (st) {
    st->iters[0] = r1.iters;
    st->iters[1] = r2.iters;
    st->mv = cnt.mv;
    st->m0inv = cnt.m0inv;
    st->sca_sweeps = cnt.sca;
    st->reliable_updates = r1.updates + r2.updates;
    st->relres[0] = rel1;
    st->relres[1] = rel2;
    st->relres_normal = relq;
    st->paper_mv = (double)(r1.iters + r2.iters) * (2.0 + 2.0 * pc.paper_cost());
    st->status = std::max(r1.status, r2.status);
    st->host_syncs = 0;
    st->host_submits = 0;
  }
  return std::max(r1.status, r2.status);
}

template <typename RI, typename RO>
int cg_dispatch(Lattice& L, const PcPlan& pc, const void* bv, void* xv, int nrhs,
                const ufg_solve_opts& o, ufg_solve_stats* st) {
  Counters cnt;
  StepResult r1;
  const C2<RO>* b = reinterpret_cast<const C2<RO>*>(bv);
  C2<RO>* x = reinterpret_cast<C2<RO>*>(xv);
  UFG_TRY((cg_solve<RI, RO>(L, pc, b, x, nrhs, o, &cnt, &r1)));
  double relq = 0;
  UFG_TRY(true_relres<RO>(L, UFG_OP_Q, x, b, nrhs, &relq));
  if (st) {
    st->iters[0] = r1.iters;
    st->iters[1] = 0;
    st->mv = cnt.mv;
    st->m0inv = cnt.m0inv;
    st->sca_sweeps = cnt.sca;
    st->reliable_updates = r1.updates;
    st->relres[0] = relq;
    st->relres[1] = 0;
    st->relres_normal = relq;
    st->paper_mv = (double)r1.iters * (2.0 + pc.paper_cost());
    st->status = r1.status;
    st->host_syncs = 0;
    st->host_submits = 0;
  }
  return r1.status;
}

template <typename R>
int cg_split_dispatch(Lattice& L, const PcPlan& E, const void* bv, void* xv, int nrhs,
                      const ufg_solve_opts& o, ufg_solve_stats* st) {
  Counters cnt;
  StepResult r1;
  PcPlan none;
  const C2<R>* b = reinterpret_cast<const C2<R>*>(bv);
  C2<R>* x = reinterpret_cast<C2<R>*>(xv);
  UFG_TRY((cg_solve<R, R>(L, none, b, x, nrhs, o, &cnt, &r1, &E)));
  double relq = 0;
  UFG_TRY(true_relres<R>(L, UFG_OP_Q, x, b, nrhs, &relq));
  if (st) {
    st->iters[0] = r1.iters;
    st->iters[1] = 0;
    st->mv = cnt.mv;
    st->m0inv = cnt.m0inv;
    st->sca_sweeps = cnt.sca;
    st->reliable_updates = r1.updates;
    st->relres[0] = relq;
    st->relres[1] = 0;
    st->relres_normal = relq;
    st->paper_mv = (double)r1.iters * (2.0 + 2.0 * E.paper_cost());
    st->status = r1.status;
    st->host_syncs = 0;
    st->host_submits = 0;
  }
  return r1.status;
}

}  // namespace

int solve_cg_split_impl(Lattice& L, const ufg_precond* p, const void* b, void* x, int nrhs,
                        const ufg_solve_opts* o, ufg_solve_stats* st) {
  UFG_TRY(validate_opts(L, o, nrhs));
  UFG_CHECK(b && x && b != x, "solve_cg_split: b and x must be distinct device pointers");
  UFG_CHECK(p && p->kind == UFG_PC_WCE, "solve_cg_split: the split factor is a weak-coupling W_d");
  UFG_CHECK(!o->mixed && !o->use_x0, "solve_cg_split: no mixed precision, x_0 = 0");
  PcPlan E;
  UFG_TRY(resolve_precond(L, p, &E));
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = (L.dtype == UFG_C128) ? cg_split_dispatch<double>(L, E, b, x, nrhs, *o, st)
                                       : cg_split_dispatch<float>(L, E, b, x, nrhs, *o, st);
  if (rc < 0) return rc;
  UFG_HIP(hipStreamSynchronize(L.stream));
  if (st) st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int solve_bicgstab_impl(Lattice& L, const ufg_precond* p, int op, const void* b, void* x,
                        int nrhs, const ufg_solve_opts* o, ufg_solve_stats* st) {
  UFG_TRY(validate_opts(L, o, nrhs));
  UFG_CHECK(op == UFG_OP_M || op == UFG_OP_MDAG || op == UFG_OP_TWO_STEP,
            "solve_bicgstab: op must be M, MDAG or TWO_STEP");
  UFG_CHECK(b && x && b != x, "solve_bicgstab: b and x must be distinct device pointers");
  PcPlan pc;
  UFG_TRY(resolve_precond(L, p, &pc));
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (o->mixed)
    rc = bicgstab_dispatch<float, double>(L, pc, op, b, x, nrhs, *o, st);
  else if (L.dtype == UFG_C128)
    rc = bicgstab_dispatch<double, double>(L, pc, op, b, x, nrhs, *o, st);
  else
    rc = bicgstab_dispatch<float, float>(L, pc, op, b, x, nrhs, *o, st);
  if (rc < 0) return rc;
  UFG_HIP(hipStreamSynchronize(L.stream));
  if (st) st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int solve_cg_impl(Lattice& L, const ufg_precond* p, const void* b, void* x, int nrhs,
                  const ufg_solve_opts* o, ufg_solve_stats* st) {
  UFG_TRY(validate_opts(L, o, nrhs));
  UFG_CHECK(b && x && b != x, "solve_cg_normal: b and x must be distinct device pointers");
  PcPlan pc;
  UFG_TRY(resolve_precond(L, p, &pc));
  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (o->mixed)
    rc = cg_dispatch<float, double>(L, pc, b, x, nrhs, *o, st);
  else if (L.dtype == UFG_C128)
    rc = cg_dispatch<double, double>(L, pc, b, x, nrhs, *o, st);
  else
    rc = cg_dispatch<float, float>(L, pc, b, x, nrhs, *o, st);
  if (rc < 0) return rc;
  UFG_HIP(hipStreamSynchronize(L.stream));
  if (st) st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

}  // namespace ufg
