// hip_stub.cpp -- a host-memory stand-in for the HIP runtime, so that the
// library's host code (validation, float64 tables, workspace layout, plan
// bookkeeping, launch configuration) runs on a machine without a GPU under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
// "Device" memory is host memory: copies and fills are memcpy / memset on
// the given addresses, so a table written past the end of a workspace sized
// by pwfs_workspace_size is an out-of-bounds host write that ASan reports.
// Kernels are not run; every launch configuration is checked against the
// gfx950 limits (grid, 1..1024 threads, 160 KiB of LDS) and counted.
// Test infrastructure only: linked into tests/host_abi/abi_driver.cpp.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include <hip/hip_runtime_api.h>

namespace {
struct Config {
  dim3 grid, block;
  size_t shared;
  hipStream_t stream;
};
Config g_cfg[16];
int g_depth = 0;
// kernels register from module constructors, which may run before this
// file's own static objects are built: the name table is made on first use
std::map<const void*, std::string>& names() {
  static auto* m = new std::map<const void*, std::string>;
  return *m;
}
long g_launches = 0, g_bad_launches = 0;
hipError_t g_last = hipSuccess;
}  // namespace

extern "C" {

long stub_launches() { return g_launches; }
long stub_bad_launches() { return g_bad_launches; }

void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* host_fn, char*, const char* name, unsigned int, void*, void*, dim3*,
                           dim3*, int*) {
  names()[host_fn] = name;
}
void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shared, hipStream_t stream) {
  if (g_depth >= 16) abort();
  g_cfg[g_depth++] = {grid, block, shared, stream};
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shared, hipStream_t* stream) {
  if (g_depth <= 0) abort();
  const Config& c = g_cfg[--g_depth];
  *grid = c.grid;
  *block = c.block;
  *shared = c.shared;
  *stream = c.stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void* fn, dim3 grid, dim3 block, void** args, size_t shared, hipStream_t) {
  ++g_launches;
  const unsigned long long threads = (unsigned long long)block.x * block.y * block.z;
  const bool ok = args && grid.x >= 1 && grid.y >= 1 && grid.z >= 1 && grid.x <= 0x7fffffffu && grid.y <= 65535 &&
                  grid.z <= 65535 && threads >= 1 && threads <= 1024 && shared <= 160 * 1024;
  if (!ok) {
    ++g_bad_launches;
    auto it = names().find(fn);
    fprintf(stderr, "bad launch of %s: grid (%u, %u, %u) block (%u, %u, %u) lds %zu\n",
            it == names().end() ? "?" : it->second.c_str(), grid.x, grid.y, grid.z, block.x, block.y, block.z,
            shared);
    g_last = hipErrorInvalidConfiguration;
    return g_last;
  }
  return hipSuccess;
}

hipError_t hipGetLastError(void) {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "stub error"; }

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  if (n) memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
// a __device__ variable's host shadow has its size: it serves as the "device" copy
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}

// events: one heap object each, so create/destroy pairing is leak-checked
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t)malloc(16);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  free((void*)e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}

}  // extern "C"
