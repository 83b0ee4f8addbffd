// The over-integrated free-surface right-hand side for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid allocation).
//
// sem_free_surface_rhs keeps its scratch (the per-element right-hand sides
// and their node sums) in the mesh workspace.  This variant keeps it in a
// file-scope device array instead, so the call touches neither the workspace
// scratch nor any allocator: no hipMalloc, hipFree or allocating library
// routine, no host synchronisation.  The array's device address is taken
// once per device with hipGetSymbolAddress (in host code the array's name is
// only a host-side stand-in) and kept; kernels receive that address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "launch.hpp"
#include "mesh.hpp"

using sem::fail;
using sem::TankDev;

namespace {

// 4 MiB per device, held until the process ends
constexpr size_t kScratchDoubles = SEM_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// The array's address on the current device (taken on first use there).
sem_status scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SEM_E_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(SEM_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SEM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return SEM_OK;
}

}  // namespace

extern "C" sem_status sem_free_surface_rhs_noalloc(sem_mesh* M, const double* eta, const double* eta_x,
                                                   const double* phi_x, const double* w_s, double* deta,
                                                   double* dphi, void* stream) {
  sem_status s = sem::check_bound(M);
  if (s) return s;
  if (!eta || !eta_x || !phi_x || !w_s || !deta || !dphi) return fail(SEM_E_INVAL, "null argument");
  const TankDev& h = M->hd;
  const size_t need = 2 * (size_t)h.nx * (h.P + 1) + 2 * (size_t)h.ns;
  if (need > kScratchDoubles)
    return fail(SEM_E_INVAL, "tank too large for the static scratch (" + std::to_string(need * sizeof(double)) +
                                 " bytes needed, " + std::to_string(SEM_NOALLOC_SCRATCH_BYTES) + " available)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != M->device)
    return fail(SEM_E_INVAL, "the current device is not the one the mesh was bound on");
  double* base = nullptr;
  if ((s = scratch_on_current_device(&base))) return s;
  double* loc = base;
  double* re = loc + 2 * (size_t)h.nx * (h.P + 1);
  double* rp = re + h.ns;
  // every scratch value is written before it is read: nothing to clear
  sem::launch_fs_rhs_into(h, M->dtank, eta, eta_x, phi_x, w_s, deta, dphi, loc, re, rp, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return fail(SEM_E_DEVICE, "launch failed");
  return SEM_OK;
}
