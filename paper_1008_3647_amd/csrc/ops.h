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

// y = K^{-1} x for the plan and operator (table in ufg.h). y must not alias x.
template <typename R>
int pc_apply(Lattice& L, const PcPlan& pc, int op, const C2<R>* x, C2<R>* y, int nrhs,
             const int* gate, Counters* cnt);

// Workspace slots (each holds nrhs vectors of the requested type).
enum Slot {
  SLOT_SOLVER0 = 0,  // 0..11 solver vectors
  SLOT_OUTER_R = 12,
  SLOT_OUTER_Y = 13,
  SLOT_OUTER_T = 14,
  SLOT_PC0 = 16,     // 16..19 preconditioner temporaries
  SLOT_PSTATE = 20,
  SLOT_POWER = 21,
  SLOT_POWER2 = 22,
  SLOT_STATE = 23
};

template <typename R>
C2<R>* slot_vec(Lattice& L, int slot, int nrhs, int* rc);

int krylov_state(Lattice& L, int nrhs, KrylovState* K, int slot_red);

}  // namespace ufg
