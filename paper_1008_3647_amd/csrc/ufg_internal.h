// Internal declarations shared by the library's translation units.
// Device layout of every vector: complex interleaved, [rhs][t][z][y][x].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ufg.h"

namespace ufg {

template <typename R>
using C2 = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;

constexpr int kMaxNx = 16;
constexpr int kMaxWceOrder = 8;

// ---------------------------------------------------------------------------
// error reporting

void set_error(const std::string& msg);

#define UFG_HIP(...)                                                               \
  do {                                                                             \
    hipError_t e_ = (__VA_ARGS__);                                                 \
    if (e_ != hipSuccess) {                                                        \
      ::ufg::set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));  \
      return UFG_EHIP;                                                             \
    }                                                                              \
  } while (0)

#define UFG_CHECK(cond, msg)                                                       \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      ::ufg::set_error(msg);                                                       \
      return UFG_EINVAL;                                                           \
    }                                                                              \
  } while (0)

#define UFG_TRY(...)                                                               \
  do {                                                                             \
    int rc_ = (__VA_ARGS__);                                                       \
    if (rc_ < 0) return rc_;                                                       \
  } while (0)

// ---------------------------------------------------------------------------
// Per-precision copy of everything derived from sigma and the lattice.
template <typename R>
struct Fields {
  R* b = nullptr;       // 1 + A sin sigma                 [N]
  R* sn = nullptr;      // sin sigma                       [N]
  R* cs = nullptr;      // cos sigma                       [N]
  R* scaD = nullptr;    // strong coupling D_t             [N]
  R* scaL = nullptr;    // strong coupling L_t             [N]
  R* T = nullptr;       // 1D factor of exp(-tau K)        [nx*nx]
  R* U = nullptr;       // eigenvectors of T (columns)     [nx*nx]
  R* Ut = nullptr;      // U^T                             [nx*nx]
  R* lam = nullptr;     // eigenvalue of U^3 mode n        [V]
};

// Device-resident work buffer that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t want);
  void release();
  ~DevBuf() { release(); }
};

// Pinned host mirror of solver flags: two slots of `cap` ints, each with an
// event recorded behind the copy into it.
struct FlagMirror {
  int* host = nullptr;
  int cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int ensure(int n);
  void release();
  ~FlagMirror() { release(); }
};

struct Lattice {
  int nx = 0, ntau = 0, dtype = UFG_C128;
  int dispersion = UFG_DISP_FREE;
  int dim = 3;      // spatial dimension (1, 2 or 3)
  int V = 0;        // nx^dim
  long long N = 0;  // V * ntau
  double tau = 0, g = 0, A = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  double* sigma = nullptr;  // FP64 copy of the field
  double bmax = 1.0;        // max |1 + A sin sigma|
  double sca_alpha = 1.0;   // alpha the SCA blocks were built with
  Fields<double> f64;
  Fields<float> f32;
  std::vector<double> T_host, U_host, lam1_host;  // 1D factors (host)
  std::vector<double> split_host;  // block-diagonal form of T (streaming kernel)
  std::vector<double> mode_fwd_host, mode_bwd_host;  // block form of U^T and U
  std::vector<int> mode_perm;       // block-ordered mode -> column of U
  int slab = 0;                    // time slices per workgroup of the streaming kernel (0: default)
  int nslab = 0;                   // slabs per rhs of the streaming kernel (0: from slab)
  int vec_blocks = 0;              // workgroups per rhs of the vector kernels (0: default)
  int xcd_group = -1;              // slab groups per XCD of the streaming kernels (-1: default)
  int xcd_rhs_inner = 0;           // 1: an XCD takes every rhs of a slab group in turn
  int t3_route = 0;                // 1: y and x stages of T^3 on MFMA, 2: DFTs (complex64, Nx = 16)
  DevBuf work[26];          // vector workspaces (solver / preconditioner)
  DevBuf hmc[7];            // HMC trajectory: sigma0, pi0, grad, phi, y, X, partials
  DevBuf red;               // reduction partials
  DevBuf state;             // solver state
  DevBuf cheb;              // Chebyshev roots on device
  FlagMirror flags;         // check-point flags read one interval late
  double lam_max_cache = -1.0;
  int lam_max_valid = 0;
  double lam_max_sq_cache = -1.0;  // lam_max of S Q, for the SCA shift below
  double lam_max_sq_alpha = 0.0;
  int lam_max_sq_valid = 0;
};

template <typename R>
inline const Fields<R>& fields(const Lattice& L);
template <>
inline const Fields<float>& fields<float>(const Lattice& L) { return L.f32; }
template <>
inline const Fields<double>& fields<double>(const Lattice& L) { return L.f64; }

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files). All are asynchronous on the
// lattice stream and assume sizes were validated by the caller.

enum HopShift { kShiftM = -1, kShiftNone = 0, kShiftMdag = +1 };

// General slice operator: for each rhs and output slice t (ts = t + shift):
//   r_t   = Mat^{(x)3} (pre_ts * src_ts)            (pre may be null)
//   base  = id_t + sgn_t * post_t * r_t               (id, post may be null)
//   dst_t = alpha * base + beta * aux_t               (aux may be null)
// sgn_t = s_{ts} for shift -1, s_t for shift +1, +1 for shift 0.
// `gate` (may be null): rhs r is skipped unless gate[r] != 0.
// Parameters of the Krylov scalar updates (shared by every rhs of a solve).
struct KrylovParams {
  double tol;
  double delta2;  // reliable-update threshold squared
  int mixed;
  int bicg;       // 1: BiCGStab (rho = <rhat, r> refreshed at updates)
  int unprec;     // CG without preconditioner: <r, z> = |r|^2
  int limit_omega;  // BiCGStab: keep |cos(t, s)| >= 0.7 (complex spectra)
};

template <typename R>
struct HopArgs {
  const C2<R>* src = nullptr;
  const C2<R>* id = nullptr;
  const C2<R>* aux = nullptr;
  C2<R>* dst = nullptr;
  const R* pre = nullptr;
  const R* post = nullptr;
  const R* mat = nullptr;
  int shift = 0;
  int nrhs = 1;
  double2 alpha = {1.0, 0.0};
  double2 beta = {0.0, 0.0};
  const int* gate = nullptr;
  // optional fused reduction over the output (per rhs, per block partials):
  //   red_mode 1: <w, dst>  (complex)        red_mode 2: <dst, id>, <dst, dst>
  //   red_mode 4 (streaming kernel, src_mode 2): those of mode 3, then <w, dst>
  //   and <w, source> (8 doubles per partial)
  int red_mode = 0;
  const C2<R>* red_w = nullptr;
  double* red_out = nullptr;  // [nrhs][nblk_per_rhs][4, or 8 for red_mode 4]
  // Fused BiCGStab source (streaming kernel only). src_mode 0: the source is
  // `src`. 1: p = r + beta (p_old - omega v_old) with beta, omega of the rhs
  // state, stored to fpnew for the workgroup's own slices. 2: s = r - alpha v.
  // red_mode 3 then gives <out, source> and |out|^2.
  int src_mode = 0;
  const C2<R>* fr = nullptr;
  const C2<R>* fp = nullptr;
  const C2<R>* fv = nullptr;
  C2<R>* fpnew = nullptr;
  const void* st = nullptr;  // RhsState array
  // Finalize performed by the launch (streaming kernel, src_mode 2 with
  // red_mode 4): before forming s, every workgroup sums the partials of its
  // rhs (fin_part [nrhs][fin_nblk][4] from the previous operator launch,
  // fin_part2 [nrhs][fin_nblk2][4] from the vector update before it) in a
  // fixed order and applies the BiCGStab alpha step (FIN_ALPHA_XR) to the rhs
  // state `st`; the workgroup of slab 0 stores the new state and the flags
  // fin_flags = active, update, restart ([3][nrhs]). That step changes none
  // of the state fields that alpha and the active flag derive from, so a
  // workgroup that reads the state after slab 0 stored it derives the same.
  const double* fin_part = nullptr;
  const double* fin_part2 = nullptr;
  int fin_nblk = 0;
  int fin_nblk2 = 0;
  int* fin_flags = nullptr;
  KrylovParams fin_prm{};
};

template <typename R>
int launch_hop(const Lattice& L, const HopArgs<R>& a);
int hop_blocks_per_rhs(const Lattice& L);

// Slice operator and force of lattices of spatial dimension 1 and 2
// (lowd.hip); launch_hop, hop_blocks_per_rhs and launch_force route there.
template <typename R>
int launch_hop_lowd(const Lattice& L, const HopArgs<R>& a);
int lowd_blocks_per_rhs(const Lattice& L);
template <typename R>
int launch_force_lowd(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs, double* grad);

// Force contraction: grad(n,t) = c(n,t) s_t sum_r Re[X_t conj((T^3 y_{t+1}))],
// c = -2 A cos sigma.
template <typename R>
int launch_force(const Lattice& L, const C2<R>* X, const C2<R>* y, int nrhs, double* grad);

// Temporal kernels.
template <typename R>
int launch_sca_apply(const Lattice& L, const C2<R>* v, C2<R>* x, int nrhs, const int* gate);
int launch_sca_setup(Lattice& L, double alpha);
// (1 - lam Z)^{-1} v per spatial mode (adjoint: Z^T); subtract_input: result - v.
// scale_field (may be null, indexed by t, n) multiplies the result.
template <typename R>
int launch_m0_temporal(const Lattice& L, const C2<R>* v, C2<R>* u, int nrhs, bool adjoint,
                       bool subtract_input, const int* gate);

// Field setup: b, sin, cos from sigma in both precisions; per-block max |b| into bmax_part.
int launch_field_setup(Lattice& L, double* bmax_part, int nblk);

// Everything derived from L.sigma (both precisions, max |b|, SCA blocks);
// synchronizes the lattice stream.
int install_field(Lattice& L);
// out_host[r] = ||x_r||^2 (FP64, fixed order) for nrhs vectors of the lattice
// dtype; synchronous.
int norm2_host(Lattice& L, const void* x, int nrhs, double* out_host);
int solve_bicgstab_impl(Lattice& L, const ufg_precond* p, int op, const void* b, void* x,
                        int nrhs, const ufg_solve_opts* o, ufg_solve_stats* st);


}  // namespace ufg
