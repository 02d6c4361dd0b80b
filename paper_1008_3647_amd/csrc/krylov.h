// Device state and kernel launchers of the Krylov solvers.
#pragma once

#include "ufg_internal.h"

namespace ufg {


// Scalars of one right-hand side, resident on the device.
struct RhsState {
  double2 rho, rho_old, alpha, omega;  // BiCGStab; CG uses rho = <r,z>, alpha, omega = beta
  double2 beta;  // BiCGStab: (rho / rho_old)(alpha / omega), 0 when undefined
  double r2;     // |r|^2 of the iterated residual
  double b2;     // |b|^2
  double maxr2;  // largest |r|^2 since the last reliable update
  double tol2;   // tol^2 |b|^2
  double rhat2;  // |rhat|^2 (shadow residual, fixed between restarts)
  int iters, updates, conv, status;
};

struct KrylovState {
  int nrhs = 0;
  RhsState* st = nullptr;
  int* active = nullptr;
  int* update = nullptr;
  int* restart = nullptr;
  double* part = nullptr;   // [nrhs][nblk][4] (8 per block for the streaming reduction mode 4)
  double* part2 = nullptr;  // [nrhs][vector blocks][4]: partials kept across one operator launch
  double* part3 = nullptr;  // [nrhs][operator blocks][4]: partials read by the next operator launch
  KrylovParams prm{};
};

enum FinOp {
  FIN_INIT_B = 0,
  FIN_INIT_R,
  FIN_ALPHA,
  FIN_OMEGA,
  FIN_RHO,
  FIN_UPDATE,
  FIN_RESTART,
  FIN_CG_ALPHA,
  FIN_CG_R,
  FIN_CG_BETA,
  FIN_CG_INIT_RZ,
  FIN_NORM,
  FIN_ALPHA_XR,   // |r|^2 of the deferred x, r update (part2), then alpha (part)
  FIN_OMEGA_RHO   // omega, then rho of the next iteration from <rhat, s>, <rhat, t>
};

int vec_blocks(const Lattice& L, int nrhs);

template <typename R>
int k_bicg_p(const Lattice& L, const C2<R>* r, C2<R>* p, const C2<R>* v, const KrylovState& K);
template <typename R>
int k_bicg_s(const Lattice& L, const C2<R>* r, const C2<R>* v, C2<R>* s, const KrylovState& K);
template <typename R>
int k_bicg_xr(const Lattice& L, C2<R>* x, const C2<R>* phat, const C2<R>* shat, const C2<R>* s,
              const C2<R>* t, C2<R>* r, const C2<R>* rhat, const KrylovState& K);
template <typename R>
int k_bicg_xr_fused(const Lattice& L, C2<R>* x, const C2<R>* p, C2<R>* r, const C2<R>* v,
                    const C2<R>* t, const C2<R>* rhat, const KrylovState& K);
// x, r update of one iteration merged with the p update of the next:
// s = r - alpha v, x += alpha p + omega s, r = s - omega t,
// p = r + beta (p - omega v); |r|^2 partials into K.part2.
template <typename R>
int k_bicg_xrp(const Lattice& L, C2<R>* x, C2<R>* p, C2<R>* r, const C2<R>* v, const C2<R>* t,
               const KrylovState& K);
template <typename R>
int k_reduce(const Lattice& L, const C2<R>* a, const C2<R>* b, int mode, const int* gate,
             const KrylovState& K);
template <typename R>
int k_axpby(const Lattice& L, double2 a, const C2<R>* x, double2 b, C2<R>* y, int nrhs,
            const int* gate);
template <typename RI, typename RO>
int k_convert(const Lattice& L, const C2<RI>* in, C2<RO>* out, int nrhs, const int* gate);
int k_promote(const Lattice& L, double2* x64, float2* x32, int nrhs, const int* gate);
// Streaming device copy of `bytes` (multiple of 16, 16-byte aligned pointers).
int k_device_copy(const void* src, void* dst, long long bytes, hipStream_t stream);
int k_demote(const Lattice& L, const double2* r64, float2* r32, const float2* rhat,
             const KrylovState& K, const int* gate);
template <typename R>
int k_cg_xr(const Lattice& L, C2<R>* x, const C2<R>* p, C2<R>* r, const C2<R>* w,
            const KrylovState& K);
template <typename R>
int k_cg_p(const Lattice& L, const C2<R>* z, C2<R>* p, const KrylovState& K);
template <typename R>
int k_restart(const Lattice& L, const C2<R>* r, C2<R>* rhat, C2<R>* p, C2<R>* v,
              const KrylovState& K);
// Sums `nblk` partials of `stride` (4 or 8) doubles per rhs from K.part into
// s[0 .. stride), and, with nblk2 > 0, nblk2 partials of 4 from K.part2 into
// s[4 .. 8); then applies `op` to the state.
int k_finalize(const Lattice& L, int op, int nblk, const int* gate, const KrylovState& K,
               int stride = 4, int nblk2 = 0);
// Partials of rhs (segment) k are part[first[k] .. first[k] + count[k]) (`stride`
// doubles each, into s[0 .. stride)); with part2, also part2[first2[k] ..
// first2[k] + count2[k]) (4 doubles each, into s[4 .. 8)).
int k_finalize_seg(hipStream_t stream, int op, const double* part, const int* first,
                   const int* count, const int* gate, const KrylovState& K, int stride = 4,
                   const double* part2 = nullptr, const int* first2 = nullptr,
                   const int* count2 = nullptr);

}  // namespace ufg
