// lattice_norm2_noalloc: the per-rhs squared norms of lattice_norm2 for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops). Same kernels as lattice_norm2 (block partial sums in
// FP64, fixed-order finalize); their partials, the per-rhs state and flags live
// in a file-scope device array instead of library-allocated buffers, and the
// result goes to a caller-owned device array, so the call is asynchronous and
// makes no host round trip.
#include <mutex>

#include "krylov.h"

namespace ufg {
namespace {

constexpr size_t kScratchBytes = size_t(2) << 20;  // 2 MiB per device
constexpr int kMaxDevices = 64;

// Each GPU the library runs on holds its own copy until the process ends. In
// host code the name is only a stand-in: kernels get the address from
// hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of device `dev`'s copy of `scratch`, looked up once per
// device with that device current.
int scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("lattice_norm2_noalloc: device index out of range");
    return UFG_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    int cur = 0;
    UFG_HIP(hipGetDevice(&cur));
    if (cur != dev) UFG_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) UFG_HIP(hipSetDevice(cur));
    UFG_HIP(e);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return UFG_OK;
}

__global__ void __launch_bounds__(64) norm2_out_kernel(const RhsState* st, double* out, int nrhs) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k < nrhs) out[k] = st[k].r2;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

// Scratch bytes lattice_norm2_noalloc needs for nrhs vectors of lattice L.
size_t norm2_noalloc_bytes(const Lattice& L, int nrhs) {
  const size_t part = sizeof(double) * 4 * (size_t)vec_blocks(L, nrhs) * (size_t)nrhs;
  return align256(part) + align256(sizeof(RhsState) * (size_t)nrhs) +
         align256(sizeof(int) * 3 * (size_t)nrhs);
}

}  // namespace ufg

using namespace ufg;

extern "C" int lattice_norm2_noalloc(ufg_lattice h, const void* x, int nrhs, double* out_dev) {
  Lattice* L = reinterpret_cast<Lattice*>(h);  // a handle from create_lattice
  UFG_CHECK(L != nullptr, "lattice_norm2_noalloc: NULL handle");
  UFG_CHECK(x && out_dev && nrhs >= 1, "lattice_norm2_noalloc: bad pointers or nrhs");
  const size_t need = norm2_noalloc_bytes(*L, nrhs);
  if (need > kScratchBytes) {
    set_error("lattice_norm2_noalloc: " + std::to_string(need) +
              " bytes of scratch needed, more than the static " +
              std::to_string(kScratchBytes) +
              " (lower nrhs or the lattice's vector workgroups, lattice_tune)");
    return UFG_EINVAL;
  }
  void* base = nullptr;
  UFG_TRY(scratch_ptr(L->device, &base));
  char* p = static_cast<char*>(base);
  KrylovState K;
  K.nrhs = nrhs;
  K.part = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * 4 * (size_t)vec_blocks(*L, nrhs) * (size_t)nrhs);
  K.st = reinterpret_cast<RhsState*>(p);
  p += align256(sizeof(RhsState) * (size_t)nrhs);
  K.active = reinterpret_cast<int*>(p);
  K.update = K.active + nrhs;
  K.restart = K.update + nrhs;
  // every partial the finalize reads is written by the reduction, and the
  // finalize's FIN_NORM step writes r2 from them alone: nothing in the scratch
  // has to start at zero
  if (L->dtype == UFG_C128)
    UFG_TRY(k_reduce<double>(*L, (const double2*)x, nullptr, 0, nullptr, K));
  else
    UFG_TRY(k_reduce<float>(*L, (const float2*)x, nullptr, 0, nullptr, K));
  UFG_TRY(k_finalize(*L, FIN_NORM, vec_blocks(*L, nrhs), nullptr, K));
  hipLaunchKernelGGL(norm2_out_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, L->stream, K.st,
                     out_dev, nrhs);
  UFG_HIP(hipGetLastError());
  return UFG_OK;
}
