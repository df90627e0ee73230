// pwfs_mfma.hip -- split-precision DFT-as-GEMM form of the forward model.
#include <hip/hip_runtime.h>

#include "pwfs_internal.hpp"

namespace pwfs {

bool mfma_supported(const pwfs_sensor_desc&) { return false; }
size_t mfma_table_bytes(const pwfs_sensor_desc&) { return 0; }
size_t mfma_scratch_frame_bytes(const pwfs_sensor_desc&) { return 0; }
int upload_mfma_tables(const pwfs_sensor_desc&, char*, hipStream_t, std::vector<std::vector<char>>&, double) {
  return PWFS_EUNSUPPORTED;
}
int forward_mfma(const SensorPlan&, const float*, long long, float*, long long, int, void*, hipStream_t, Prof*) {
  return PWFS_EUNSUPPORTED;
}

}  // namespace pwfs
