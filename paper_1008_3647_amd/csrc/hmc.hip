// HMC of the phi-algorithm (paper, Sec. 1): heat bath, leapfrog molecular
// dynamics on H = sum pi^2 / 2 + S_p[sigma], Metropolis step.
//
// The solves and the force contraction are the library's; this file adds the
// O(N) field updates (one fused kick-drift kernel per force) and the FP64 sum
// of pi^2 (fixed grid, fixed tree order, so the same input always gives the
// same bits). sigma, pi and the gradient are float64 [Ntau][Nx]^3.
#include <chrono>
#include <cmath>

#include "ops.h"

namespace ufg {

namespace {

constexpr int kMdThreads = 256;
constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 256;

// pi -= c grad, then (d != 0) sigma += d pi: the kick after a force and the
// drift before the next one.
__global__ void __launch_bounds__(kMdThreads)
    md_kick_drift_kernel(double* __restrict__ sigma, double* __restrict__ pi,
                         const double* __restrict__ grad, double c, double d, long long n) {
  const long long stride = (long long)gridDim.x * kMdThreads;
  for (long long i = (long long)blockIdx.x * kMdThreads + threadIdx.x; i < n; i += stride) {
    const double p = pi[i] - c * grad[i];
    pi[i] = p;
    if (d != 0.0) sigma[i] += d * p;
  }
}

// Block partial sums of v^2 over a grid-stride walk (kRedBlocks blocks).
__global__ void __launch_bounds__(kRedThreads)
    sq_partial_kernel(const double* __restrict__ v, long long n, double* __restrict__ part) {
  __shared__ double s[kRedThreads];
  double acc = 0.0;
  const long long stride = (long long)kRedBlocks * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride)
    acc += v[i] * v[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// out = scale * sum of the kRedBlocks partials (one block).
__global__ void __launch_bounds__(kRedThreads)
    sum_partials_kernel(const double* __restrict__ part, double scale, double* __restrict__ out) {
  __shared__ double s[kRedThreads];
  double a = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scale * s[0];
}

enum { HB_SIGMA0, HB_PI0, HB_GRAD, HB_PHI, HB_Y, HB_X, HB_RED };

struct Md {
  Lattice& L;
  const ufg_precond* pc;
  ufg_solve_opts so;
  int nphi;
  int chrono;
  const void* phi;
  void* y;
  void* X;
  double* grad;
  double* red;
  ufg_hmc_result* res;
  bool y_guess = false;  // y holds a starting vector for the next M^dagger solve
  bool X_guess = false;
};

int md_kick_drift(const Lattice& L, double* sigma, double* pi, const double* grad, double c,
                  double d) {
  const long long n = L.N;
  long long blocks = (n + kMdThreads - 1) / kMdThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(md_kick_drift_kernel, dim3((unsigned)blocks), dim3(kMdThreads), 0, L.stream,
                     sigma, pi, grad, c, d, n);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

// sum pi^2 / 2 (host value; synchronizes the stream)
int kinetic(const Lattice& L, const double* pi, double* red, double* out) {
  hipLaunchKernelGGL(sq_partial_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, L.stream, pi,
                     L.N, red);
  UFG_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kRedThreads), 0, L.stream, red, 0.5,
                     red + kRedBlocks);
  UFG_HIP(hipGetLastError());
  UFG_HIP(hipMemcpyAsync(out, red + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, L.stream));
  UFG_HIP(hipStreamSynchronize(L.stream));
  return UFG_OK;
}

int solve_step(Md& m, int op, const void* b, void* x, bool guess) {
  ufg_solve_opts o = m.so;
  o.use_x0 = guess ? 1 : 0;
  ufg_solve_stats st{};
  const int rc = solve_bicgstab_impl(m.L, m.pc, op, b, x, m.nphi, &o, &st);
  if (rc < 0) return rc;
  m.res->solves += 1;
  m.res->iters += st.iters[0];
  m.res->mv += st.mv;
  if (st.relres[0] > m.res->worst_relres) m.res->worst_relres = st.relres[0];
  if (st.status != 0) {
    m.res->status = st.status;
    return 1;
  }
  return UFG_OK;
}

// S_p and its gradient (into m.grad) at sigma; 1 when a solve failed.
int force_at(Md& m, const double* sigma, double* S) {
  Lattice& L = m.L;
  UFG_HIP(hipMemcpyAsync(L.sigma, sigma, sizeof(double) * L.N, hipMemcpyDeviceToDevice, L.stream));
  UFG_TRY(install_field(L));
  int rc = solve_step(m, UFG_OP_MDAG, m.phi, m.y, m.y_guess);
  if (rc) return rc;
  std::vector<double> nrm(m.nphi);
  UFG_TRY(norm2_host(L, m.y, m.nphi, nrm.data()));
  double s = 0.0;
  for (double v : nrm) s += v;
  *S = s;
  rc = solve_step(m, UFG_OP_M, m.y, m.X, m.X_guess);
  if (rc) return rc;
  m.y_guess = m.X_guess = (m.chrono != 0);
  if (L.dtype == UFG_C128)
    UFG_TRY(launch_force<double>(L, (const double2*)m.X, (const double2*)m.y, m.nphi, m.grad));
  else
    UFG_TRY(launch_force<float>(L, (const float2*)m.X, (const float2*)m.y, m.nphi, m.grad));
  m.res->forces += 1;
  return UFG_OK;
}

// Leapfrog from (sigma, pi); 1 when a solve failed (state then partial).
int leapfrog(Md& m, double* sigma, double* pi, double dt, int nsteps, double* actions) {
  double S = 0.0;
  int rc = force_at(m, sigma, &S);
  if (rc) return rc;
  m.res->S0 = S;
  if (actions) actions[0] = S;
  UFG_TRY(md_kick_drift(m.L, sigma, pi, m.grad, 0.5 * dt, dt));
  for (int step = 0; step < nsteps; ++step) {
    rc = force_at(m, sigma, &S);
    if (rc) return rc;
    if (actions) actions[step + 1] = S;
    const bool last = step == nsteps - 1;
    UFG_TRY(md_kick_drift(m.L, sigma, pi, m.grad, last ? 0.5 * dt : dt, last ? 0.0 : dt));
  }
  m.res->S1 = S;
  return UFG_OK;
}

int validate(const Lattice* L, double* sigma, double* pi, const void* vec, int nphi,
             const ufg_hmc_opts* o, ufg_hmc_result* res, const char* who) {
  const std::string w(who);
  UFG_CHECK(L != nullptr, w + ": NULL handle");
  UFG_CHECK(o != nullptr && res != nullptr, w + ": options and result are required");
  UFG_CHECK(sigma && pi && vec && sigma != pi, w + ": bad device pointers");
  UFG_CHECK(nphi >= 1, w + ": nphi must be >= 1");
  UFG_CHECK(std::isfinite(o->dt) && o->dt > 0.0, w + ": dt must be finite and > 0");
  UFG_CHECK(o->nsteps >= 1 && o->nsteps <= 1000000, w + ": nsteps must be 1..1e6");
  UFG_CHECK(o->check_every >= 1, w + ": check_every must be >= 1");
  return UFG_OK;
}

int prepare(Lattice& L, int nphi, const ufg_hmc_opts* o, const ufg_precond* pc,
            ufg_hmc_result* res, Md& m) {
  const size_t fbytes = sizeof(double) * L.N;
  const size_t vbytes = size_t(nphi) * L.N * (L.dtype == UFG_C128 ? 16 : 8);
  UFG_TRY(L.hmc[HB_SIGMA0].ensure(fbytes));
  UFG_TRY(L.hmc[HB_PI0].ensure(fbytes));
  UFG_TRY(L.hmc[HB_GRAD].ensure(fbytes));
  UFG_TRY(L.hmc[HB_PHI].ensure(vbytes));
  UFG_TRY(L.hmc[HB_Y].ensure(vbytes));
  UFG_TRY(L.hmc[HB_X].ensure(vbytes));
  UFG_TRY(L.hmc[HB_RED].ensure(sizeof(double) * (kRedBlocks + 1)));
  *res = ufg_hmc_result{};
  res->accept = -1;
  m.so = ufg_solve_opts{o->tol, o->maxit, o->mixed, 0.1, o->check_every, 0, 0};
  m.nphi = nphi;
  m.chrono = o->chrono;
  m.pc = pc;
  m.y = L.hmc[HB_Y].p;
  m.X = L.hmc[HB_X].p;
  m.grad = reinterpret_cast<double*>(L.hmc[HB_GRAD].p);
  m.red = reinterpret_cast<double*>(L.hmc[HB_RED].p);
  m.res = res;
  return UFG_OK;
}

// Back to the saved start; reinstalls its field.
int restore(Lattice& L, double* sigma, double* pi) {
  const size_t fbytes = sizeof(double) * L.N;
  UFG_HIP(hipMemcpyAsync(sigma, L.hmc[HB_SIGMA0].p, fbytes, hipMemcpyDeviceToDevice, L.stream));
  UFG_HIP(hipMemcpyAsync(pi, L.hmc[HB_PI0].p, fbytes, hipMemcpyDeviceToDevice, L.stream));
  UFG_HIP(hipMemcpyAsync(L.sigma, sigma, fbytes, hipMemcpyDeviceToDevice, L.stream));
  return install_field(L);
}

int save_start(Lattice& L, const double* sigma, const double* pi) {
  const size_t fbytes = sizeof(double) * L.N;
  UFG_HIP(hipMemcpyAsync(L.hmc[HB_SIGMA0].p, sigma, fbytes, hipMemcpyDeviceToDevice, L.stream));
  UFG_HIP(hipMemcpyAsync(L.hmc[HB_PI0].p, pi, fbytes, hipMemcpyDeviceToDevice, L.stream));
  return UFG_OK;
}

// MD shared by both entry points, after phi is in place; fills K, dH.
int run_md(Md& m, double* sigma, double* pi, const ufg_hmc_opts* o, double* actions) {
  Lattice& L = m.L;
  double K0 = 0.0, K1 = 0.0;
  UFG_TRY(kinetic(L, pi, m.red, &K0));
  const int rc = leapfrog(m, sigma, pi, o->dt, o->nsteps, actions);
  if (rc < 0) return rc;
  if (rc > 0) return restore(L, sigma, pi);
  UFG_TRY(kinetic(L, pi, m.red, &K1));
  m.res->K0 = K0;
  m.res->K1 = K1;
  m.res->dH = (K1 - K0) + (m.res->S1 - m.res->S0);
  return UFG_OK;
}

}  // namespace

}  // namespace ufg

using namespace ufg;

extern "C" {

int hmc_leapfrog(ufg_lattice h, const ufg_precond* precond, double* sigma_dev, double* pi_dev,
                 const void* phi_dev, int nphi, const ufg_hmc_opts* o, double* actions_host,
                 ufg_hmc_result* res) {
  Lattice* Lp = reinterpret_cast<Lattice*>(h);
  UFG_TRY(validate(Lp, sigma_dev, pi_dev, phi_dev, nphi, o, res, "hmc_leapfrog"));
  Lattice& L = *Lp;
  const auto t0 = std::chrono::steady_clock::now();
  Md m{L};
  UFG_TRY(prepare(L, nphi, o, precond, res, m));
  m.phi = phi_dev;
  UFG_TRY(save_start(L, sigma_dev, pi_dev));
  UFG_TRY(run_md(m, sigma_dev, pi_dev, o, actions_host));
  UFG_HIP(hipStreamSynchronize(L.stream));
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return UFG_OK;
}

int hmc_trajectory(ufg_lattice h, const ufg_precond* precond, double* sigma_dev, double* pi_dev,
                   const void* eta_dev, int nphi, double u, const ufg_hmc_opts* o,
                   void* phi_out, double* actions_host, ufg_hmc_result* res) {
  Lattice* Lp = reinterpret_cast<Lattice*>(h);
  UFG_TRY(validate(Lp, sigma_dev, pi_dev, eta_dev, nphi, o, res, "hmc_trajectory"));
  UFG_CHECK(std::isfinite(u) && u >= 0.0 && u < 1.0, "hmc_trajectory: u must be in [0, 1)");
  Lattice& L = *Lp;
  const auto t0 = std::chrono::steady_clock::now();
  Md m{L};
  UFG_TRY(prepare(L, nphi, o, precond, res, m));
  const size_t vbytes = size_t(nphi) * L.N * (L.dtype == UFG_C128 ? 16 : 8);
  UFG_CHECK(phi_out != eta_dev, "hmc_trajectory: phi_out must not alias eta");
  UFG_TRY(save_start(L, sigma_dev, pi_dev));
  // heat bath at the starting field
  UFG_HIP(hipMemcpyAsync(L.sigma, sigma_dev, sizeof(double) * L.N, hipMemcpyDeviceToDevice,
                         L.stream));
  UFG_TRY(install_field(L));
  void* phi = L.hmc[HB_PHI].p;
  if (L.dtype == UFG_C128)
    UFG_TRY(op_apply<double>(L, UFG_OP_MDAG, (const double2*)eta_dev, (double2*)phi, nphi, nullptr));
  else
    UFG_TRY(op_apply<float>(L, UFG_OP_MDAG, (const float2*)eta_dev, (float2*)phi, nphi, nullptr));
  if (phi_out)
    UFG_HIP(hipMemcpyAsync(phi_out, phi, vbytes, hipMemcpyDeviceToDevice, L.stream));
  m.phi = phi;
  if (o->chrono) {  // M^dagger eta = phi: eta is the first y
    UFG_HIP(hipMemcpyAsync(m.y, eta_dev, vbytes, hipMemcpyDeviceToDevice, L.stream));
    m.y_guess = true;
  }
  UFG_TRY(run_md(m, sigma_dev, pi_dev, o, actions_host));
  if (res->status == 0) {
    res->accept = (u < std::exp(-res->dH)) ? 1 : 0;
    if (!res->accept) UFG_TRY(restore(L, sigma_dev, pi_dev));
  } else {
    res->accept = 0;
  }
  UFG_HIP(hipStreamSynchronize(L.stream));
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return UFG_OK;
}

}  // extern "C"
