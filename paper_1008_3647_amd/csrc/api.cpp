// C ABI entry points (declared in include/ufg.h).
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>

#include "ops.h"
#include "hop_stream.h"

namespace ufg {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int DevBuf::ensure(size_t want) {
  if (want <= bytes && p) return UFG_OK;
  release();
  if (hipMalloc(&p, want) != hipSuccess) {
    p = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    set_error("hipMalloc failed (" + std::to_string(want) + " bytes)");
    return UFG_ENOMEM;
  }
  bytes = want;
  return UFG_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

int FlagMirror::ensure(int n) {
  if (host && n <= cap) return UFG_OK;
  release();
  if (hipHostMalloc(reinterpret_cast<void**>(&host), 2 * sizeof(int) * n,
                    hipHostMallocDefault) != hipSuccess) {
    host = nullptr;
    (void)hipGetLastError();
    set_error("hipHostMalloc failed for the solver flags");
    return UFG_ENOMEM;
  }
  cap = n;
  for (hipEvent_t& e : ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      (void)hipGetLastError();
      release();
      set_error("hipEventCreate failed");
      return UFG_EHIP;
    }
  }
  return UFG_OK;
}

void FlagMirror::release() {
  for (hipEvent_t& e : ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (host) (void)hipHostFree(host);
  host = nullptr;
  cap = 0;
}

int solve_bicgstab_impl(Lattice& L, const ufg_precond* p, int op, const void* b, void* x,
                        int nrhs, const ufg_solve_opts* o, ufg_solve_stats* st);
int solve_cg_impl(Lattice& L, const ufg_precond* p, const void* b, void* x, int nrhs,
                  const ufg_solve_opts* o, ufg_solve_stats* st);
int solve_cg_split_impl(Lattice& L, const ufg_precond* p, const void* b, void* x, int nrhs,
                        const ufg_solve_opts* o, ufg_solve_stats* st);
int cheb_plan(int degree, double eps, std::vector<double2>* roots, double2* cf);
int solve_batched_impl(const ufg_lattice* Ls, int nprob, const void* const* b, void* const* x,
                       const int* nrhs, const ufg_precond* p, const ufg_solve_opts* o,
                       ufg_solve_stats* st);
int batched_tune(int hop_blocks_per_cu, int vec_blocks_per_cu, long long chunk, int slab,
                 int sync_iters);
int euler_weights(int order, double p, double* w);

// Kinetic energy of one axis at momentum k: k^2 / 2 (Sec. 1) or, for the
// Hubbard-model dispersion, 1 - cos k (nearest-neighbour hopping of amplitude
// 1/2, equal to k^2 / 2 up to O(k^4)).
static double axis_energy(int dispersion, double k) {
  return dispersion == UFG_DISP_HUBBARD ? 1.0 - std::cos(k) : 0.5 * k * k;
}

// T_{xy} = (1/Nx) sum_m exp(-tau E(k_m)) cos(k_m (x - y)), k_m = 2 pi m / Nx,
// m = -Nx/2 .. Nx/2-1: the one-axis factor of exp(-tau K) in position space.
static void transfer_matrix(int nx, double tau, int dispersion, double* T) {
  for (int x = 0; x < nx; ++x)
    for (int y = 0; y < nx; ++y) {
      double s = 0.0;
      for (int m = -nx / 2; m < nx / 2; ++m) {
        const double k = 2.0 * M_PI * m / nx;
        s += std::exp(-tau * axis_energy(dispersion, k)) * std::cos(k * (x - y));
      }
      T[x * nx + y] = s / nx;
    }
}

// Real orthonormal eigenvectors of the circulant T (columns of U) and their
// eigenvalues exp(-tau E(k)): constant mode, cos/sin pairs, alternating mode.
static void transfer_eigenbasis(int nx, double tau, int dispersion, double* U, double* lam) {
  auto e = [&](int m) {
    const double k = 2.0 * M_PI * m / nx;
    return std::exp(-tau * axis_energy(dispersion, k));
  };
  int col = 0;
  for (int x = 0; x < nx; ++x) U[x * nx + col] = 1.0 / std::sqrt((double)nx);
  lam[col++] = e(0);
  for (int m = 1; m < nx / 2; ++m) {
    for (int x = 0; x < nx; ++x) U[x * nx + col] = std::sqrt(2.0 / nx) * std::cos(2 * M_PI * m * x / nx);
    lam[col++] = e(m);
    for (int x = 0; x < nx; ++x) U[x * nx + col] = std::sqrt(2.0 / nx) * std::sin(2 * M_PI * m * x / nx);
    lam[col++] = e(m);
  }
  for (int x = 0; x < nx; ++x) U[x * nx + col] = ((x & 1) ? -1.0 : 1.0) / std::sqrt((double)nx);
  lam[col++] = e(nx / 2);
}

static int alloc_fields(Lattice& L) {
  const size_t N = (size_t)L.N, V = (size_t)L.V, m = (size_t)L.nx * L.nx;
  double** d[] = {&L.f64.b, &L.f64.sn, &L.f64.cs, &L.f64.scaD, &L.f64.scaL};
  float** f[] = {&L.f32.b, &L.f32.sn, &L.f32.cs, &L.f32.scaD, &L.f32.scaL};
  for (auto pp : d)
    if (hipMalloc(pp, N * sizeof(double)) != hipSuccess) return UFG_ENOMEM;
  for (auto pp : f)
    if (hipMalloc(pp, N * sizeof(float)) != hipSuccess) return UFG_ENOMEM;
  if (hipMalloc(&L.sigma, N * sizeof(double)) != hipSuccess) return UFG_ENOMEM;
  double** dm[] = {&L.f64.T, &L.f64.U, &L.f64.Ut};
  float** fm[] = {&L.f32.T, &L.f32.U, &L.f32.Ut};
  for (auto pp : dm)
    if (hipMalloc(pp, m * sizeof(double)) != hipSuccess) return UFG_ENOMEM;
  for (auto pp : fm)
    if (hipMalloc(pp, m * sizeof(float)) != hipSuccess) return UFG_ENOMEM;
  if (hipMalloc(&L.f64.lam, V * sizeof(double)) != hipSuccess) return UFG_ENOMEM;
  if (hipMalloc(&L.f32.lam, V * sizeof(float)) != hipSuccess) return UFG_ENOMEM;
  return UFG_OK;
}

static void free_fields(Lattice& L) {
  void* ptrs[] = {L.f64.b, L.f64.sn, L.f64.cs, L.f64.scaD, L.f64.scaL, L.f32.b, L.f32.sn,
                  L.f32.cs, L.f32.scaD, L.f32.scaL, L.sigma, L.f64.T, L.f64.U, L.f64.Ut,
                  L.f32.T, L.f32.U, L.f32.Ut, L.f64.lam, L.f32.lam};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

template <typename T>
static int upload(hipStream_t s, T* dst, const std::vector<double>& src) {
  std::vector<T> h(src.begin(), src.end());
  UFG_HIP(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  UFG_HIP(hipStreamSynchronize(s));
  return UFG_OK;
}

int install_field(Lattice& L) {
  const int nblk = 512;
  int rc = L.red.ensure(nblk * sizeof(double));
  if (rc) return rc;
  double* part = reinterpret_cast<double*>(L.red.p);
  UFG_TRY(launch_field_setup(L, part, nblk));
  std::vector<double> h(nblk);
  UFG_HIP(hipMemcpyAsync(h.data(), part, nblk * sizeof(double), hipMemcpyDeviceToHost, L.stream));
  UFG_HIP(hipStreamSynchronize(L.stream));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  L.bmax = m;
  UFG_TRY(launch_sca_setup(L, 1.0));
  UFG_HIP(hipStreamSynchronize(L.stream));
  L.lam_max_valid = 0;
  L.lam_max_sq_valid = 0;
  return UFG_OK;
}

int norm2_host(Lattice& L, const void* x, int nrhs, double* out_host) {
  KrylovState K;
  UFG_TRY(krylov_state(L, nrhs, &K, SLOT_PSTATE));
  if (L.dtype == UFG_C128)
    UFG_TRY(k_reduce<double>(L, (const double2*)x, nullptr, 0, nullptr, K));
  else
    UFG_TRY(k_reduce<float>(L, (const float2*)x, nullptr, 0, nullptr, K));
  UFG_TRY(k_finalize(L, FIN_NORM, vec_blocks(L, nrhs), nullptr, K));
  std::vector<RhsState> st(nrhs);
  UFG_HIP(hipMemcpyAsync(st.data(), K.st, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost,
                         L.stream));
  UFG_HIP(hipStreamSynchronize(L.stream));
  for (int i = 0; i < nrhs; ++i) out_host[i] = st[i].r2;
  return UFG_OK;
}

static Lattice* check_handle(ufg_lattice h) { return reinterpret_cast<Lattice*>(h); }

}  // namespace ufg

using namespace ufg;

extern "C" {

const char* ufg_last_error(void) { return g_err.c_str(); }
const char* last_error(void) { return g_err.c_str(); }

int create_lattice(int nx, int ntau, double tau, double g, int dtype, void* hip_stream,
                   ufg_lattice* out) {
  return create_lattice_ex(nx, ntau, tau, g, dtype, UFG_DISP_FREE, hip_stream, out);
}

int create_lattice_ex(int nx, int ntau, double tau, double g, int dtype, int dispersion,
                      void* hip_stream, ufg_lattice* out) {
  return create_lattice_dim(nx, ntau, 3, tau, g, dtype, dispersion, hip_stream, out);
}

int create_lattice_dim(int nx, int ntau, int dim, double tau, double g, int dtype,
                       int dispersion, void* hip_stream, ufg_lattice* out) {
  UFG_CHECK(out != nullptr, "create_lattice: out is NULL");
  UFG_CHECK(dim >= 1 && dim <= 3, "create_lattice: dim must be 1, 2 or 3");
  UFG_CHECK(dispersion == UFG_DISP_FREE || dispersion == UFG_DISP_HUBBARD,
            "create_lattice: dispersion must be UFG_DISP_FREE or UFG_DISP_HUBBARD");
  *out = nullptr;
  UFG_CHECK(nx >= 2 && nx <= kMaxNx && nx % 2 == 0, "create_lattice: nx must be even, 2..16");
  UFG_CHECK(ntau >= 2, "create_lattice: ntau must be >= 2");
  UFG_CHECK(tau > 0 && std::isfinite(tau), "create_lattice: tau must be > 0");
  UFG_CHECK(g >= 0 && std::isfinite(g), "create_lattice: g must be >= 0");
  UFG_CHECK(dtype == UFG_C64 || dtype == UFG_C128, "create_lattice: dtype must be C64 or C128");
  Lattice* L = new (std::nothrow) Lattice();
  if (!L) return UFG_ENOMEM;
  L->nx = nx;
  L->ntau = ntau;
  L->dim = dim;
  L->V = dim == 1 ? nx : dim == 2 ? nx * nx : nx * nx * nx;
  L->N = (long long)L->V * ntau;
  L->tau = tau;
  L->g = g;
  L->A = std::sqrt(2.0) * std::sqrt(std::exp(tau * g) - 1.0);
  L->dtype = dtype;
  L->dispersion = dispersion;
  L->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&L->device) != hipSuccess) {
    delete L;
    set_error("create_lattice: no HIP device");
    return UFG_EHIP;
  }
  if (alloc_fields(*L) != UFG_OK) {
    free_fields(*L);
    delete L;
    set_error("create_lattice: device allocation failed");
    return UFG_ENOMEM;
  }
  L->T_host.assign(nx * nx, 0.0);
  L->U_host.assign(nx * nx, 0.0);
  L->lam1_host.assign(nx, 0.0);
  transfer_matrix(nx, tau, dispersion, L->T_host.data());
  transfer_eigenbasis(nx, tau, dispersion, L->U_host.data(), L->lam1_host.data());
  // check T = U diag(lam) U^T before trusting the eigenbasis
  double err = 0.0;
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < nx; ++j) {
      double s = 0.0;
      for (int k = 0; k < nx; ++k) s += L->U_host[i * nx + k] * L->lam1_host[k] * L->U_host[j * nx + k];
      err = std::max(err, std::fabs(s - L->T_host[i * nx + j]));
    }
  if (err > 1e-12) {
    free_fields(*L);
    delete L;
    set_error("create_lattice: eigenbasis check failed");
    return UFG_EHIP;
  }
  // block forms of T and U serve the streaming kernels (three-dimensional
  // slices); lower dimensions use the general slice kernels with T and U
  if (dim == 3 && split_coefficients(nx, L->T_host, &L->split_host) > 1e-13) {
    free_fields(*L);
    delete L;
    set_error("create_lattice: block form of T failed its check");
    return UFG_EHIP;
  }
  if (dim == 3 && mode_split_coefficients(nx, L->U_host, &L->mode_fwd_host,
                                          &L->mode_bwd_host, &L->mode_perm) > 1e-12) {
    free_fields(*L);
    delete L;
    set_error("create_lattice: block form of the eigenbasis failed its check");
    return UFG_EHIP;
  }
  // mode-space vectors of the streaming basis change use the block order of
  // the modes; the mode eigenvalues follow it
  std::vector<double> lam1m = L->lam1_host;
  if (!L->mode_perm.empty())
    for (int i = 0; i < nx; ++i) lam1m[i] = L->lam1_host[L->mode_perm[i]];
  std::vector<double> Ut(nx * nx), lam3(L->V);
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < nx; ++j) Ut[i * nx + j] = L->U_host[j * nx + i];
  // eigenvalue of the mode product: one factor per axis (site index
  // (z nx + y) nx + x; the leading axes are absent in lower dimensions)
  for (int i = 0; i < L->V; ++i) {
    double v = 1.0;
    for (int k = 0, rest = i; k < dim; ++k, rest /= nx) v *= lam1m[rest % nx];
    lam3[i] = v;
  }
  int rc = UFG_OK;
  if (!rc) rc = upload<double>(L->stream, L->f64.T, L->T_host);
  if (!rc) rc = upload<float>(L->stream, L->f32.T, L->T_host);
  if (!rc) rc = upload<double>(L->stream, L->f64.U, L->U_host);
  if (!rc) rc = upload<float>(L->stream, L->f32.U, L->U_host);
  if (!rc) rc = upload<double>(L->stream, L->f64.Ut, Ut);
  if (!rc) rc = upload<float>(L->stream, L->f32.Ut, Ut);
  if (!rc) rc = upload<double>(L->stream, L->f64.lam, lam3);
  if (!rc) rc = upload<float>(L->stream, L->f32.lam, lam3);
  if (!rc && hipMemsetAsync(L->sigma, 0, sizeof(double) * L->N, L->stream) != hipSuccess)
    rc = UFG_EHIP;
  if (!rc) rc = install_field(*L);
  if (rc) {
    free_fields(*L);
    delete L;
    return rc;
  }
  *out = reinterpret_cast<ufg_lattice>(L);
  return UFG_OK;
}

int destroy_lattice(ufg_lattice h) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "destroy_lattice: NULL handle");
  (void)hipStreamSynchronize(L->stream);
  free_fields(*L);
  delete L;
  return UFG_OK;
}

int set_lattice_stream(ufg_lattice h, void* s) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "set_lattice_stream: NULL handle");
  L->stream = reinterpret_cast<hipStream_t>(s);
  return UFG_OK;
}

int set_aux_field(ufg_lattice h, const double* sigma_dev) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "set_aux_field: NULL handle");
  UFG_CHECK(sigma_dev != nullptr, "set_aux_field: sigma is NULL");
  UFG_HIP(hipMemcpyAsync(L->sigma, sigma_dev, sizeof(double) * L->N, hipMemcpyDeviceToDevice,
                         L->stream));
  return install_field(*L);
}

int apply_M(ufg_lattice h, const void* x, void* y, int nrhs) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "apply_M: NULL handle");
  UFG_CHECK(x && y && x != y && nrhs >= 1, "apply_M: bad vectors or nrhs");
  if (L->dtype == UFG_C128)
    return op_apply<double>(*L, UFG_OP_M, (const double2*)x, (double2*)y, nrhs, nullptr);
  return op_apply<float>(*L, UFG_OP_M, (const float2*)x, (float2*)y, nrhs, nullptr);
}

int apply_Mdag(ufg_lattice h, const void* x, void* y, int nrhs) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "apply_Mdag: NULL handle");
  UFG_CHECK(x && y && x != y && nrhs >= 1, "apply_Mdag: bad vectors or nrhs");
  if (L->dtype == UFG_C128)
    return op_apply<double>(*L, UFG_OP_MDAG, (const double2*)x, (double2*)y, nrhs, nullptr);
  return op_apply<float>(*L, UFG_OP_MDAG, (const float2*)x, (float2*)y, nrhs, nullptr);
}

int apply_precond(ufg_lattice h, const ufg_precond* p, int op, const void* x, void* y, int nrhs) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "apply_precond: NULL handle");
  UFG_CHECK(x && y && x != y && nrhs >= 1, "apply_precond: bad vectors or nrhs");
  UFG_CHECK(op == UFG_OP_M || op == UFG_OP_MDAG || op == UFG_OP_Q,
            "apply_precond: op must be M, MDAG or Q");
  PcPlan pc;
  UFG_TRY(resolve_precond(*L, p, &pc));
  Counters cnt;
  if (L->dtype == UFG_C128)
    return pc_apply<double>(*L, pc, op, (const double2*)x, (double2*)y, nrhs, nullptr, &cnt);
  return pc_apply<float>(*L, pc, op, (const float2*)x, (float2*)y, nrhs, nullptr, &cnt);
}

int solve_cg_normal(ufg_lattice h, const ufg_precond* p, const void* b, void* x, int nrhs,
                    const ufg_solve_opts* o, ufg_solve_stats* st) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "solve_cg_normal: NULL handle");
  return solve_cg_impl(*L, p, b, x, nrhs, o, st);
}

int solve_cg_split(ufg_lattice h, const ufg_precond* p, const void* b, void* x, int nrhs,
                   const ufg_solve_opts* o, ufg_solve_stats* st) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "solve_cg_split: NULL handle");
  return solve_cg_split_impl(*L, p, b, x, nrhs, o, st);
}

int solve_bicgstab(ufg_lattice h, const ufg_precond* p, int op, const void* b, void* x, int nrhs,
                   const ufg_solve_opts* o, ufg_solve_stats* st) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "solve_bicgstab: NULL handle");
  return solve_bicgstab_impl(*L, p, op, b, x, nrhs, o, st);
}

int force_dS_dsigma(ufg_lattice h, const void* X, const void* y, int nrhs, double* grad_dev) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "force_dS_dsigma: NULL handle");
  UFG_CHECK(X && y && grad_dev && nrhs >= 1, "force_dS_dsigma: bad pointers or nrhs");
  if (L->dtype == UFG_C128)
    return launch_force<double>(*L, (const double2*)X, (const double2*)y, nrhs, grad_dev);
  return launch_force<float>(*L, (const float2*)X, (const float2*)y, nrhs, grad_dev);
}

int lattice_norm2(ufg_lattice h, const void* x, int nrhs, double* out_host) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "lattice_norm2: NULL handle");
  UFG_CHECK(x && out_host && nrhs >= 1, "lattice_norm2: bad pointers or nrhs");
  return norm2_host(*L, x, nrhs, out_host);
}

int lattice_tune(ufg_lattice h, int slab, int vec_blocks) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "lattice_tune: NULL handle");
  UFG_CHECK(slab >= 0 && slab <= L->ntau, "lattice_tune: slab must be 0..ntau");
  UFG_CHECK(vec_blocks >= 0 && vec_blocks <= 4096, "lattice_tune: vec_blocks must be 0..4096");
  UFG_HIP(hipStreamSynchronize(L->stream));  // launches in flight used the old shapes
  L->slab = slab;
  L->vec_blocks = vec_blocks;
  return UFG_OK;
}

int lattice_tune_slabs(ufg_lattice h, int nslab) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "lattice_tune_slabs: NULL handle");
  UFG_CHECK(nslab >= 0 && nslab <= L->ntau, "lattice_tune_slabs: nslab must be 0..ntau");
  UFG_HIP(hipStreamSynchronize(L->stream));
  L->nslab = nslab;
  return UFG_OK;
}

int precond_lam_max(ufg_lattice h, const ufg_precond* p, double* out_host) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "precond_lam_max: NULL handle");
  UFG_CHECK(p && out_host, "precond_lam_max: NULL preconditioner or output");
  UFG_CHECK(p->kind == UFG_PC_CHEB || p->kind == UFG_PC_SCA_CHEB,
            "precond_lam_max: needs a Chebyshev preconditioner (plain or with SCA)");
  PcPlan pc;
  UFG_TRY(resolve_precond(*L, p, &pc));
  *out_host = pc.lam_max;
  return UFG_OK;
}

int lattice_tune_order(ufg_lattice h, int group, int rhs_inner) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "lattice_tune_order: NULL handle");
  UFG_CHECK(group >= -1 && group <= L->ntau, "lattice_tune_order: group must be -1..ntau");
  UFG_CHECK(rhs_inner == 0 || rhs_inner == 1, "lattice_tune_order: rhs_inner must be 0 or 1");
  UFG_HIP(hipStreamSynchronize(L->stream));
  L->xcd_group = group;
  L->xcd_rhs_inner = rhs_inner;
  return UFG_OK;
}

int lattice_tune_transform(ufg_lattice h, int route) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "lattice_tune_transform: NULL handle");
  UFG_CHECK(route >= 0 && route <= 2, "lattice_tune_transform: route must be 0, 1 or 2");
  UFG_HIP(hipStreamSynchronize(L->stream));
  L->t3_route = route;
  return UFG_OK;
}

int lattice_info(ufg_lattice h, int* nx, int* ntau, int* dtype, double* A) {
  Lattice* L = check_handle(h);
  UFG_CHECK(L != nullptr, "lattice_info: NULL handle");
  if (nx) *nx = L->nx;
  if (ntau) *ntau = L->ntau;
  if (dtype) *dtype = L->dtype;
  if (A) *A = L->A;
  return UFG_OK;
}

int ufg_cheb_roots(int degree, double eps, double* out, double* out_c) {
  UFG_CHECK(out && out_c, "ufg_cheb_roots: NULL output");
  std::vector<double2> roots;
  double2 cf;
  if (cheb_plan(degree, eps, &roots, &cf) != UFG_OK) {
    set_error("ufg_cheb_roots: degree must be a power of two and 0 < eps < 1");
    return UFG_EINVAL;
  }
  for (int i = 0; i < degree; ++i) {
    out[2 * i] = roots[i].x;
    out[2 * i + 1] = roots[i].y;
  }
  out_c[0] = cf.x;
  out_c[1] = cf.y;
  return UFG_OK;
}

int ufg_euler_weights(int order, double p, double* out) {
  UFG_CHECK(out != nullptr, "ufg_euler_weights: NULL output");
  UFG_CHECK(p > 0 && p < 1, "ufg_euler_weights: p must be in (0, 1)");
  if (euler_weights(order, p, out) != UFG_OK) {
    set_error("ufg_euler_weights: order must be 0..8");
    return UFG_EINVAL;
  }
  return UFG_OK;
}

int ufg_transfer_matrix(int nx, double tau, double* out) {
  UFG_CHECK(out != nullptr, "ufg_transfer_matrix: NULL output");
  UFG_CHECK(nx >= 2 && nx <= kMaxNx && nx % 2 == 0, "ufg_transfer_matrix: nx must be even, 2..16");
  UFG_CHECK(tau > 0, "ufg_transfer_matrix: tau must be > 0");
  transfer_matrix(nx, tau, UFG_DISP_FREE, out);
  return UFG_OK;
}

int solve_batched(const ufg_lattice* Ls, int nprob, const void* const* b, void* const* x,
                  const int* nrhs, const ufg_precond* p, const ufg_solve_opts* o,
                  ufg_solve_stats* st) {
  return solve_batched_impl(Ls, nprob, b, x, nrhs, p, o, st);
}

int solve_batched_tune(int hop_blocks_per_cu, int vec_blocks_per_cu, long long chunk,
                       int slab, int sync_iters) {
  return batched_tune(hop_blocks_per_cu, vec_blocks_per_cu, chunk, slab, sync_iters);
}

int ufg_device_copy(const void* src, void* dst, long long bytes, void* hip_stream) {
  UFG_CHECK(src && dst && bytes > 0 && bytes % 16 == 0, "ufg_device_copy: bad pointers or size");
  UFG_CHECK(((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0,
            "ufg_device_copy: pointers must be 16-byte aligned");
  return k_device_copy(src, dst, bytes, (hipStream_t)hip_stream);
}

}  // extern "C"
