// afm_energy_forces_noalloc: afm_energy_forces for callers that cannot
// allocate device memory.  Its workspace is a fixed array in the library's
// own device memory instead of a caller allocation; the kernels are those of
// afm_energy_forces, given this array's device address where they would get
// the caller's workspace.
//
// The array is a file-scope device symbol.  Its name, used in host code, is
// a host-side stand-in and not a device address, so host code never passes
// it anywhere: the device address comes from hipGetSymbolAddress, resolved
// once per device with that device current (at model creation, else at the
// first call on the device) and kept in g_scratch_ptr.  Every call on one
// GPU uses that GPU's single copy: calls that overlap on one GPU race, and
// the array keeps whatever the last call left in it (the energy/force path
// initialises everything it reads).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace afm {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[AFM_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of this device's scratch array (resolved on first use, with
// `device` current).  Returns AFM_OK and sets *out, or an error code.
int static_scratch_resolve(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index out of range for the static scratch table");
    return AFM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    if (e != hipSuccess) {
      set_error(std::string("static scratch: ") + hipGetErrorString(e));
      return AFM_E_HIP;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return AFM_E_HIP;
    }
    g_scratch_ptr[device] = p;
  }
  if (out) *out = g_scratch_ptr[device];
  return AFM_OK;
}

}  // namespace afm

using namespace afm;

extern "C" int afm_energy_forces_noalloc(const afm_model* m, const afm_system* sys, const afm_nlist* nl,
                                         double* e_atom, double* e_struct, double* forces, double* virial,
                                         void* stream) {
  if (!m || !sys || !nl) {
    set_error("null model, system or neighbour list");
    return AFM_E_INVALID;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error(hipGetErrorString(e));
    return AFM_E_HIP;
  }
  if (dev != m->device) {
    set_error("the current device is not the model's device");
    return AFM_E_INVALID;
  }
  void* base = nullptr;
  int rc = static_scratch_resolve(dev, &base);
  if (rc) return rc;
  // the same plan as a caller workspace capped at the array's size; the
  // planner's chunk size comes from a linear fit of the layout, so shrink the
  // cap by any overshoot and plan again
  afm_workspace ws{};
  int64_t cap = AFM_STATIC_SCRATCH_BYTES;
  for (int attempt = 0; attempt < 4; ++attempt) {
    rc = afm_workspace_plan(m, sys->n_atoms, sys->n_struct, nl->capacity, cap, 0, &ws);
    if (rc) {
      set_error("system of " + std::to_string(sys->n_atoms) + " atoms and edge capacity " +
                std::to_string(nl->capacity) + " needs more than the " +
                std::to_string((long long)AFM_STATIC_SCRATCH_BYTES) +
                "-byte static scratch (use afm_energy_forces with a caller workspace)");
      return AFM_E_CAPACITY;
    }
    if (ws.bytes <= AFM_STATIC_SCRATCH_BYTES) break;
    cap -= (ws.bytes - AFM_STATIC_SCRATCH_BYTES) + (int64_t(1) << 20);
  }
  if (ws.bytes > AFM_STATIC_SCRATCH_BYTES) {
    set_error("system of " + std::to_string(sys->n_atoms) + " atoms and edge capacity " +
              std::to_string(nl->capacity) + " does not fit the " +
              std::to_string((long long)AFM_STATIC_SCRATCH_BYTES) + "-byte static scratch");
    return AFM_E_CAPACITY;
  }
  ws.ptr = base;
  return afm_energy_forces(m, sys, nl, e_atom, e_struct, forces, virial, &ws, stream);
}
