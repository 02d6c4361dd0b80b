// Device-side scalar updates of the Krylov solvers (the "finalize" step):
// shared by the finalize kernels and by operator launches that perform the
// step themselves in their prologue.
#pragma once

#include "krylov.h"

namespace ufg {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return double2{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// Scalar update of one rhs from its summed partials s[0..8).
// The state and the flags of the rhs are held in registers by the caller.
__device__ inline void apply_fin(int op, const double* s, RhsState& q, int& act, int& upd,
                                 int& rst, const KrylovParams& prm) {
  const double s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3];
  const double2 d01 = double2{s0, s1};
  switch (op) {
    case FIN_INIT_B:  // |b|^2
      q.b2 = s2;
      q.tol2 = prm.tol * prm.tol * s2;
      break;
    case FIN_INIT_R:  // rhat = r: rho = <r, r>, r2
      q.rho = double2{s2, 0.0};
      q.rhat2 = s2;
      q.rho_old = q.alpha = q.omega = double2{1.0, 0.0};
      q.beta = double2{0.0, 0.0};
      q.r2 = q.maxr2 = s2;
      q.iters = 0;
      q.updates = 0;
      q.conv = (s2 <= q.tol2) ? 1 : 0;
      act = q.conv ? 0 : 1;
      upd = 0;
      rst = 0;
      q.status = 0;
      break;
    case FIN_ALPHA:  // alpha = rho / <rhat, v>
      if (d01.x == 0.0 && d01.y == 0.0) {
        rst = 1;
        q.alpha = double2{0.0, 0.0};
      } else {
        q.alpha = cdiv(q.rho, d01);
      }
      break;
    case FIN_OMEGA: {  // omega = <t, s> / <t, t>, s3 = |s|^2
      // Sleijpen and van der Vorst's limited omega: when t and s are nearly
      // orthogonal the minimal-residual omega stalls the bi-orthogonal part;
      // enlarge it so that |cos(t, s)| counts as at least 0.7.
      if (s2 > 0.0) {
        double2 w = double2{s0 / s2, s1 / s2};
        const double c = std::sqrt((s0 * s0 + s1 * s1) / (s2 * s3));
        if (prm.limit_omega && s3 > 0.0 && c < 0.7 && c > 0.0) {
          w.x *= 0.7 / c;
          w.y *= 0.7 / c;
        }
        q.omega = w;
      } else {
        q.omega = double2{0.0, 0.0};
      }
      break;
    }
    case FIN_RHO: {  // after x, r update: rho_old = rho; rho = <rhat, r>
      q.rho_old = q.rho;
      q.rho = d01;
      q.r2 = s2;
      q.iters += 1;
      if (!(s2 == s2) || s2 > 1e300) {  // NaN / overflow: stop this rhs
        act = 0;
        q.status = UFG_BREAKDOWN;
        break;
      }
      if (q.omega.x == 0.0 && q.omega.y == 0.0 && s2 > q.tol2) rst = 1;
      // beta of the next p-update; undefined after omega = 0 or rho_old = 0
      // (then p restarts from r, and the restart flag renews rhat)
      if ((q.rho_old.x != 0.0 || q.rho_old.y != 0.0) && (q.omega.x != 0.0 || q.omega.y != 0.0))
        q.beta = cmul(cdiv(q.rho, q.rho_old), cdiv(q.alpha, q.omega));
      else
        q.beta = double2{0.0, 0.0};
      if (s2 <= q.tol2) {
        // verify with a recomputed residual; no further iterations until then
        // (this is the end of an iteration, so the state stays consistent)
        upd = 1;
        act = 0;
      } else if (prm.mixed && s2 < prm.delta2 * q.maxr2) {
        upd = 1;
      }
      if (s2 > q.maxr2) q.maxr2 = s2;
      // near breakdown of the bi-orthogonality: restart with rhat = r
      if (!upd && (d01.x * d01.x + d01.y * d01.y) < 1e-28 * q.rhat2 * s2) rst = 1;
      break;
    }
    case FIN_UPDATE:  // reliable update done: r is b - A x
      q.r2 = s2;
      q.maxr2 = s2;
      q.updates += 1;
      if (prm.bicg) {  // rho = <rhat, r> of the recomputed residual, and its beta
        q.rho = d01;
        if ((q.rho_old.x != 0.0 || q.rho_old.y != 0.0) && (q.omega.x != 0.0 || q.omega.y != 0.0))
          q.beta = cmul(cdiv(q.rho, q.rho_old), cdiv(q.alpha, q.omega));
        else
          q.beta = double2{0.0, 0.0};
      }
      upd = 0;
      if (s2 <= q.tol2) {
        q.conv = 1;
        act = 0;
      } else if (q.status == 0) {
        act = 1;  // the iterated residual met tol, the true one did not
      }
      break;
    case FIN_RESTART:  // rhat = r: rho = |r|^2, scalars reset
      q.rho = double2{q.r2, 0.0};
      q.rhat2 = q.r2;
      q.rho_old = q.alpha = q.omega = double2{1.0, 0.0};
      q.beta = double2{0.0, 0.0};
      rst = 0;
      break;
    case FIN_CG_ALPHA:  // alpha = rz / <p, w>
      if (d01.x == 0.0 && d01.y == 0.0) {
        act = 0;
        q.status = UFG_BREAKDOWN;
        q.alpha = double2{0.0, 0.0};
      } else {
        q.alpha = cdiv(q.rho, d01);
      }
      break;
    case FIN_CG_R:  // |r|^2 after x, r update
      q.r2 = s2;
      q.iters += 1;
      if (!(s2 == s2) || s2 > 1e300) {
        act = 0;
        q.status = UFG_BREAKDOWN;
        break;
      }
      // CG keeps iterating until the check point verifies (the rest of this
      // iteration, beta and p, still has to run for a consistent state)
      if (s2 <= q.tol2) {
        upd = 1;
      } else if (prm.mixed && s2 < prm.delta2 * q.maxr2) {
        upd = 1;
      }
      if (s2 > q.maxr2) q.maxr2 = s2;
      break;
    case FIN_CG_BETA: {  // rz_new = <r, z>: beta = rz_new / rz (stored in omega)
      const double2 rz = prm.unprec ? double2{q.r2, 0.0} : d01;
      q.omega = (q.rho.x == 0.0 && q.rho.y == 0.0) ? double2{0.0, 0.0} : cdiv(rz, q.rho);
      q.rho = rz;
      break;
    }
    case FIN_CG_INIT_RZ:  // rz = <r, z>
      q.rho = prm.unprec ? double2{q.r2, 0.0} : d01;
      break;
    case FIN_NORM:  // true residual norm into r2 (no flags)
      q.r2 = s2;
      break;
    case FIN_ALPHA_XR: {
      // s[6] = |r|^2 after the deferred x, r update (the checks of FIN_RHO,
      // with rho from FIN_OMEGA_RHO), then alpha = rho / <rhat, v> from s0, s1
      const double r2 = s[6];
      q.r2 = r2;
      q.iters += 1;
      if (!(r2 == r2) || r2 > 1e300) {
        act = 0;
        q.status = UFG_BREAKDOWN;
        break;
      }
      if (q.omega.x == 0.0 && q.omega.y == 0.0 && r2 > q.tol2) rst = 1;
      if (r2 <= q.tol2) {
        // stop and verify; p already holds the next direction, so a rhs the
        // check sends back to work restarts from its recomputed residual
        upd = 1;
        rst = 1;
        act = 0;
      } else if (prm.mixed && r2 < prm.delta2 * q.maxr2) {
        upd = 1;
      }
      if (r2 > q.maxr2) q.maxr2 = r2;
      if (!upd && (q.rho.x * q.rho.x + q.rho.y * q.rho.y) < 1e-28 * q.rhat2 * r2)
        rst = 1;
      if (!act) break;
      if (d01.x == 0.0 && d01.y == 0.0) {
        rst = 1;
        q.alpha = double2{0.0, 0.0};
      } else {
        q.alpha = cdiv(q.rho, d01);
      }
      break;
    }
    case FIN_OMEGA_RHO: {
      // omega as FIN_OMEGA; r_new = s - omega t gives
      // rho_new = <rhat, r_new> = <rhat, s> - omega <rhat, t> (s[6,7], s[4,5])
      if (s2 > 0.0) {
        double2 w = double2{s0 / s2, s1 / s2};
        const double c = std::sqrt((s0 * s0 + s1 * s1) / (s2 * s3));
        if (prm.limit_omega && s3 > 0.0 && c < 0.7 && c > 0.0) {
          w.x *= 0.7 / c;
          w.y *= 0.7 / c;
        }
        q.omega = w;
      } else {
        q.omega = double2{0.0, 0.0};
      }
      const double2 wt = cmul(q.omega, double2{s[4], s[5]});
      q.rho_old = q.rho;
      q.rho = double2{s[6] - wt.x, s[7] - wt.y};
      if ((q.rho_old.x != 0.0 || q.rho_old.y != 0.0) && (q.omega.x != 0.0 || q.omega.y != 0.0))
        q.beta = cmul(cdiv(q.rho, q.rho_old), cdiv(q.alpha, q.omega));
      else
        q.beta = double2{0.0, 0.0};
      break;
    }
  }
}

}  // namespace
}  // namespace ufg
