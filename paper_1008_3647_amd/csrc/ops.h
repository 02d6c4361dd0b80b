// Operators and preconditioners assembled from the kernels.
#pragma once

#include "krylov.h"

namespace ufg {

struct Counters {
  long long mv = 0, m0inv = 0, sca = 0;
};

// A preconditioner with everything resolved (roots, weights, lam_max).
struct PcPlan {
  int kind = UFG_PC_NONE;
  int degree = 0;
  double eps = 0, lam_max = 0, alpha = 1.0;
  int order = 0;
  double w[kMaxWceOrder + 1] = {1.0};
  std::vector<double2> roots;  // application order
  double2 cf = {1.0, 0.0};     // c^{1/(2n)}
  // paper cost model: MV per preconditioner application
  double paper_cost() const;
};

// y = op x (op = UFG_OP_M or UFG_OP_MDAG); optional fused reduction.
template <typename R>
int op_apply(const Lattice& L, int op, const C2<R>* x, C2<R>* y, int nrhs, const int* gate,
             int red_mode = 0, const C2<R>* red_w = nullptr, double* red_out = nullptr);

// y = b - op x.
template <typename R>
int op_residual(const Lattice& L, int op, const C2<R>* x, const C2<R>* b, C2<R>* y, int nrhs,
                const int* gate);

// y = Q x = M^T M x using tmp; optional fused reduction on the M^T step.
template <typename R>
int q_apply(const Lattice& L, const C2<R>* x, C2<R>* tmp, C2<R>* y, int nrhs, const int* gate,
            int red_mode = 0, const C2<R>* red_w = nullptr, double* red_out = nullptr);

// y = b - Q x.
template <typename R>
int q_residual(const Lattice& L, const C2<R>* x, const C2<R>* b, C2<R>* tmp, C2<R>* y, int nrhs,
               const int* gate);

int resolve_precond(Lattice& L, const ufg_precond* p, PcPlan* out);

// BiCGStab source formed inside a weak-coupling application: its first basis
// change builds x from the rhs state while loading (mode 1: p = r + beta (p -
// omega v), mode 2: s = r - alpha v), stores it to `out` (== the x passed to
// pc_apply) and goes on from there. Only where pc_fuses_source holds.
template <typename R>
struct PcSource {
  int mode = 0;
  const C2<R>* r = nullptr;
  const C2<R>* p = nullptr;
  const C2<R>* v = nullptr;
  C2<R>* out = nullptr;
  const void* st = nullptr;  // RhsState array
};

bool pc_fuses_source(const Lattice& L, const PcPlan& pc, int op);

// y = K^{-1} x for the plan and operator (table in ufg.h). y must not alias x.
// With `src`, x is first formed as described for PcSource.
template <typename R>
int pc_apply(Lattice& L, const PcPlan& pc, int op, const C2<R>* x, C2<R>* y, int nrhs,
             const int* gate, Counters* cnt, const PcSource<R>* src = nullptr);

// Workspace slots (each holds nrhs vectors of the requested type).
enum Slot {
  SLOT_SOLVER0 = 0,  // 0..11 solver vectors
  SLOT_OUTER_R = 12,
  SLOT_OUTER_Y = 13,
  SLOT_OUTER_T = 14,
  SLOT_PC0 = 16,     // 16..21 preconditioner temporaries
  SLOT_PSTATE = 22,
  SLOT_POWER = 23,
  SLOT_POWER2 = 24,
  SLOT_STATE = 25
};

template <typename R>
C2<R>* slot_vec(Lattice& L, int slot, int nrhs, int* rc);

int krylov_state(Lattice& L, int nrhs, KrylovState* K, int slot_red);

// lam_max of Q (Chebyshev) or of S Q (strong coupling with the Chebyshev
// filter, S for the SCA shift alpha): 30 power iterations, times 1.05, cached
// per field.
int estimate_lam_max(Lattice& L, double* out);
int estimate_lam_max_sq(Lattice& L, double alpha, double* out);

}  // namespace ufg
