// Kernels that run along Euclidean time at fixed spatial site or mode:
//   * field setup: 1 + A sin sigma, sin sigma, cos sigma (paper, Sec. 1)
//   * strong-coupling factorisation and its two sweeps (paper, Sec. 4)
//   * the temporal part of M0^{-1} in the eigenbasis of exp(-tau K)
//     (paper, Sec. 3: M0 is diagonal in frequency-momentum space; per spatial
//     mode the antiperiodic time problem (1 - lam Z) u = v has the closed form
//     u = (1 + lam^Ntau)^{-1} sum_m lam^m Z^m v, evaluated by two sweeps).
// One thread owns one (rhs, site) column; consecutive threads take consecutive
// sites so every access along t is a coalesced row.
#include "ufg_internal.h"

namespace ufg {
namespace {

__global__ void field_setup_kernel(const double* __restrict__ sigma, double A, long long n,
                                   double* b64, double* s64, double* c64, float* b32, float* s32,
                                   float* c32, double* bmax_part) {
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double s = sin(sigma[i]), c = cos(sigma[i]);
    const double b = 1.0 + A * s;
    b64[i] = b;
    s64[i] = s;
    c64[i] = c;
    b32[i] = float(b);
    s32[i] = float(s);
    c32[i] = float(c);
    m = fmax(m, fabs(b));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  __shared__ double sm[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sm[w]);
    bmax_part[blockIdx.x] = r;
  }
}

// D_0 = alpha + b_0^2; D_t = alpha + b_t^2 - b_{t-1}^2 / D_{t-1};
// D_{Ntau-1} additionally loses b_{Ntau-1}^2 / D_0 (the antiperiodic corner);
// L_t = b_t / D_t for t < Ntau-1 and L_{Ntau-1} = b_{Ntau-1} / D_0.
__global__ void sca_setup_kernel(const double* __restrict__ b, int V, int ntau, double alpha,
                                 double* D64, double* L64, float* D32, float* L32) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  const double b0 = b[n];
  const double D0 = alpha + b0 * b0;
  double Dprev = D0, bprev = b0;
  D64[n] = D0;
  for (int t = 1; t < ntau; ++t) {
    const long long i = (long long)t * V + n;
    const double bt = b[i];
    double D = alpha + bt * bt - bprev * bprev / Dprev;
    if (t == ntau - 1) D -= bt * bt / D0;
    D64[i] = D;
    L64[i - V] = bprev / Dprev;
    Dprev = D;
    bprev = bt;
  }
  L64[(long long)(ntau - 1) * V + n] = bprev / D0;
  for (int t = 0; t < ntau; ++t) {
    const long long i = (long long)t * V + n;
    D32[i] = float(D64[i]);
    L32[i] = float(L64[i]);
  }
}

// x = L^{-1} D^{-1} L^{dagger -1} v per site. x may alias v.
template <typename R>
__global__ void sca_apply_kernel(const C2<R>* v, C2<R>* x, const R* __restrict__ D,
                                 const R* __restrict__ Lb, int V, int ntau, int nrhs,
                                 const int* gate) {
  const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (gid >= (long long)V * nrhs) return;
  const int r = int(gid / V);
  const int n = int(gid - (long long)r * V);
  if (gate && gate[r] == 0) return;
  const long long base = (long long)r * ntau * V + n;
  // forward sweep: w_0 = v_0, w_t = v_t + L_{t-1} w_{t-1}, corner on the last slice
  C2<R> w0 = v[base];
  C2<R> w = w0;
  x[base] = C2<R>{w0.x / D[n], w0.y / D[n]};
  for (int t = 1; t < ntau; ++t) {
    const long long i = base + (long long)t * V;
    const long long f = (long long)t * V + n;
    const R l = Lb[f - V];
    const C2<R> vt = v[i];
    C2<R> wt = C2<R>{vt.x + l * w.x, vt.y + l * w.y};
    if (t == ntau - 1) {
      const R lc = Lb[(long long)(ntau - 1) * V + n];
      wt.x -= lc * w0.x;
      wt.y -= lc * w0.y;
    }
    w = wt;
    const R d = D[f];
    x[i] = C2<R>{wt.x / d, wt.y / d};
  }
  // backward sweep: x_{Ntau-1} = w'_{Ntau-1}; x_t = w'_t + L_t x_{t+1};
  // x_0 additionally loses L_{Ntau-1} x_{Ntau-1}
  const long long last = base + (long long)(ntau - 1) * V;
  const C2<R> xl = x[last];
  C2<R> xn = xl;
  for (int t = ntau - 2; t >= 0; --t) {
    const long long i = base + (long long)t * V;
    const R l = Lb[(long long)t * V + n];
    const C2<R> wt = x[i];
    C2<R> xt = C2<R>{wt.x + l * xn.x, wt.y + l * xn.y};
    if (t == 0) {
      const R lc = Lb[(long long)(ntau - 1) * V + n];
      xt.x -= lc * xl.x;
      xt.y -= lc * xl.y;
    }
    x[i] = xt;
    xn = xt;
  }
}

// Per spatial mode n with eigenvalue lam of exp(-tau K):
//   forward : (1 - lam Z) u = v,   (Z w)_t = w_{t-1}, (Z w)_0 = -w_{Ntau-1}
//   adjoint : (1 - lam Z^T) u = v
// Temporal part of M0^{-1} per (rhs, spatial mode): the cyclic first-order
// recurrence u_t = v_t + lam u_{t-1} with the antiperiodic closure
// u_{-1} = -u_{Ntau-1}, split into kChunks time chunks so that 8x more threads
// share the sweep (a thread's chain is Ntau/8 long instead of Ntau):
// workgroup = 64 modes x kChunks chunks (one chunk per wave, modes along the
// lanes). Pass 1: every chunk sweeps its slices from a zero carry (g = last
// value). Then per mode: the chunk carries U_c = g_c + lam^{L_c} U_{c-1} with
// the antiperiodic closure U_{-1} = -U_{last}, i.e. U_last = G / (1 + lam^N)
// where G is the scan from a zero start. Pass 2: every chunk sweeps again from
// its carry. The adjoint runs the same recurrence on reversed time. u may
// alias v (each thread reads and writes only its own chunk).
constexpr int kChunks = 8;
constexpr int kModes = 64;

template <typename R>
__global__ void __launch_bounds__(kModes* kChunks)
    m0_chunked_kernel(const C2<R>* v, C2<R>* u, const R* __restrict__ lam_mode, int V, int ntau,
                      int nrhs, int adjoint, int subtract, const int* gate) {
  __shared__ C2<R> carry[kChunks][kModes];
  const int ml = threadIdx.x % kModes, c = threadIdx.x / kModes;
  const long long gid = (long long)blockIdx.x * kModes + ml;
  const bool inb = gid < (long long)V * nrhs;
  const int r = inb ? int(gid / V) : 0;
  const int n = inb ? int(gid - (long long)r * V) : 0;
  const bool act = inb && !(gate && gate[r] == 0);
  const int Lc = (ntau + kChunks - 1) / kChunks;
  const int s0 = min(c * Lc, ntau), s1 = min(s0 + Lc, ntau);  // chunk [s0, s1) in sweep order
  const long long base = (long long)r * ntau * V + n;
  const R lam = act ? lam_mode[n] : R(0);
  auto at = [&](int k) -> long long {  // sweep position -> element index
    const int t = adjoint ? ntau - 1 - k : k;
    return base + (long long)t * V;
  };
  // pass 1: zero-carry sweep of the chunk
  C2<R> w = C2<R>{R(0), R(0)};
  if (act) {
#pragma unroll 8
    for (int k = s0; k < s1; ++k) {
      const C2<R> q = v[at(k)];
      w = C2<R>{q.x + lam * w.x, q.y + lam * w.y};
    }
  }
  carry[c][ml] = w;
  __syncthreads();
  if (c == 0 && act) {
    R lamL[kChunks];
    R lamN = R(1);
    for (int j = 0; j < kChunks; ++j) {
      const int L = min((j + 1) * Lc, ntau) - min(j * Lc, ntau);
      R p = R(1);
      for (int i = 0; i < L; ++i) p *= lam;
      lamL[j] = p;
      lamN *= p;
    }
    // scan from a zero start: G = carry out of the last chunk
    C2<R> U = C2<R>{R(0), R(0)};
    for (int j = 0; j < kChunks; ++j) {
      const C2<R> g = carry[j][ml];
      U = C2<R>{g.x + lamL[j] * U.x, g.y + lamL[j] * U.y};
    }
    const R inv = R(1) / (R(1) + lamN);
    // carry into chunk 0 is U_{-1} = -U_last
    C2<R> cin = C2<R>{-U.x * inv, -U.y * inv};
    for (int j = 0; j < kChunks; ++j) {
      const C2<R> g = carry[j][ml];
      carry[j][ml] = cin;  // carry into chunk j
      cin = C2<R>{g.x + lamL[j] * cin.x, g.y + lamL[j] * cin.y};
    }
  }
  __syncthreads();
  if (act) {
    C2<R> prev = carry[c][ml];
#pragma unroll 8
    for (int k = s0; k < s1; ++k) {
      // last use of v here, and u is not re-read by this launch
      const long long i = at(k);
      const C2<R> q =
          C2<R>{__builtin_nontemporal_load(&v[i].x), __builtin_nontemporal_load(&v[i].y)};
      prev = C2<R>{q.x + lam * prev.x, q.y + lam * prev.y};
      const C2<R> o = subtract ? C2<R>{prev.x - q.x, prev.y - q.y} : prev;
      __builtin_nontemporal_store(o.x, &u[i].x);
      __builtin_nontemporal_store(o.y, &u[i].y);
    }
  }
}

}  // namespace

int launch_field_setup(Lattice& L, double* bmax_part, int nblk) {
  hipLaunchKernelGGL(field_setup_kernel, dim3(nblk), dim3(256), 0, L.stream, L.sigma, L.A, L.N,
                     L.f64.b, L.f64.sn, L.f64.cs, L.f32.b, L.f32.sn, L.f32.cs, bmax_part);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

int launch_sca_setup(Lattice& L, double alpha) {
  const int threads = 256;
  hipLaunchKernelGGL(sca_setup_kernel, dim3((L.V + threads - 1) / threads), dim3(threads), 0,
                     L.stream, L.f64.b, L.V, L.ntau, alpha, L.f64.scaD, L.f64.scaL, L.f32.scaD,
                     L.f32.scaL);
  UFG_HIP(hipGetLastError());
  L.sca_alpha = alpha;
  return UFG_OK;
}

template <typename R>
int launch_sca_apply(const Lattice& L, const C2<R>* v, C2<R>* x, int nrhs, const int* gate) {
  const Fields<R>& F = fields<R>(L);
  const long long n = (long long)L.V * nrhs;
  const int threads = 128;
  hipLaunchKernelGGL((sca_apply_kernel<R>), dim3((unsigned)((n + threads - 1) / threads)),
                     dim3(threads), 0, L.stream, v, x, F.scaD, F.scaL, L.V, L.ntau, nrhs, gate);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template <typename R>
int launch_m0_temporal(const Lattice& L, const C2<R>* v, C2<R>* u, int nrhs, bool adjoint,
                       bool subtract_input, const int* gate) {
  const Fields<R>& F = fields<R>(L);
  const long long n = (long long)L.V * nrhs;
  hipLaunchKernelGGL((m0_chunked_kernel<R>), dim3((unsigned)((n + kModes - 1) / kModes)),
                     dim3(kModes * kChunks), 0, L.stream, v, u, F.lam, L.V, L.ntau, nrhs,
                     adjoint ? 1 : 0, subtract_input ? 1 : 0, gate);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}

template int launch_sca_apply<float>(const Lattice&, const float2*, float2*, int, const int*);
template int launch_sca_apply<double>(const Lattice&, const double2*, double2*, int, const int*);
template int launch_m0_temporal<float>(const Lattice&, const float2*, float2*, int, bool, bool,
                                       const int*);
template int launch_m0_temporal<double>(const Lattice&, const double2*, double2*, int, bool, bool,
                                        const int*);

}  // namespace ufg
