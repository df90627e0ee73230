// pwfs_internal.hpp -- host-side plan structures shared by the library's
// translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pwfs.h"

namespace pwfs {

// per-sensor workspace regions, in order
enum Region {
  R_AMP = 0, R_RX, R_RY, R_AK, R_MROW, R_MCOL, R_TW, R_VALID, R_REF, R_REFINT, R_ZERO, R_MFMA,
  kRegions
};

struct Geometry {
  int D, N, n, b, S, o;   // pupil, transform, subapertures, block, separation, pad offset
  int Sx, Sy;             // image separation along x and y (S and S; a roof arm has 0 on one axis)
  int win_lo, win_hi;     // first column of the two image windows (one window when Sx = 0)
  int wy_lo, wy_hi;       // first row of the two image windows (one window when Sy = 0)
  int full, Nc, Dp;       // full-plane mode, columns kept by the row pass, padded D
  int n_mod, n_lam, n_a;  // modulation points, wavelengths, distinct cosines
  int qmax;               // non-zero first-stage inputs per butterfly
};

struct SensorPlan {
  pwfs_sensor_desc desc;
  Geometry g;
  int arms = 1;           // 2 for a double roof: arm x, then arm y, one plane each
  Geometry arm_g[2];
  int ident = 0;          // an arm's flat axis as the identity: 1 = columns (arm x), 2 = rows (arm y)
  void* dev[kRegions];
  int n_valid;
  double sumA2;
  std::vector<uint8_t> valid_host;
  size_t opd_offset, int_offset, slope_offset;
  float2* rbuf = nullptr;   // this sensor's pass scratch
  int row_tile = 0;         // row-pass tile rows (0: the default of its N)
};

struct Layout {
  std::vector<size_t> offsets;  // [sensor][region]
  std::vector<size_t> sensor_rbuf;
  size_t rbuf_offset = 0, rbuf_bytes = 0, counters_offset = 0, total = 0;
  int chunk = 1;
};

struct TiltPoint {
  double tx, ty;   // lambda/D at lambda_ref
  int key;         // index of the distinct x-tilt (row-pass result) it uses
};
void tilt_points(const pwfs_sensor_desc& d, std::vector<TiltPoint>& pts, std::vector<double>& key_tx);
Geometry geometry(const pwfs_sensor_desc& d);
Geometry arm_geometry(const pwfs_sensor_desc& d, int arm);
inline int sensor_arms(const pwfs_sensor_desc& d) { return (d.flags & PWFS_F_DOUBLE_ROOF) ? 2 : 1; }
void set_last_error(const char* msg);   // message returned by pwfs_last_error
void pupil_and_valid(const pwfs_sensor_desc& d, std::vector<float>& A, std::vector<uint8_t>& V);
int fft_lanes(int N);
int fft_r0(int N);
size_t rbuf_field_offset(const pwfs_sensor_desc& d, int nf);

// MFMA (split-precision DFT-as-GEMM) form
bool mfma_supported(const pwfs_sensor_desc& d);
size_t mfma_table_bytes(const pwfs_sensor_desc& d);
size_t mfma_scratch_frame_bytes(const pwfs_sensor_desc& d);
int upload_mfma_tables(const pwfs_sensor_desc& d, char* dst, hipStream_t st, std::vector<std::vector<char>>& keep,
                       double sumA2);
struct Prof;
int forward_mfma(const SensorPlan& sp, const float* opd, long long opd_stride, float* out, long long out_stride,
                 int nf, void* scratch, hipStream_t st, Prof* prof);

// Optional per-kernel timing: HIP events recorded on the launch stream
// around each kernel (pool created when profiling is switched on).
enum KernelId {
  K_ROWS = 0, K_COLS = 1, K_SLOPES = 2, K_MFMA = 3, K_FIELD = 4, K_HETERO = 5, K_CCD = 6, K_FUSED = 7, kKernelIds = 8
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;  // start, stop per slot
  std::vector<int> kid;
  int used = 0;
  int begin(hipStream_t st) {
    if (!on || used >= (int)kid.size()) return -1;
    if (hipEventRecord(ev[2 * used], st) != hipSuccess) return -1;
    return used++;
  }
  void end(int slot, hipStream_t st, int kernel) {
    if (slot < 0) return;
    kid[slot] = kernel;
    (void)hipEventRecord(ev[2 * slot + 1], st);
  }
};

}  // namespace pwfs

struct pwfs_plan_s {
  std::vector<pwfs::SensorPlan> s;
  int max_frames = 0, chunk = 1, max_chunk = 1, n_cu = 256;
  pwfs_tuning tune{};
  int* counters = nullptr;      // persistent-pass claim and dependency counters
  size_t opd_stride = 0, int_stride = 0, slope_stride = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  float2* rbuf = nullptr;
  pwfs::Prof prof;
};

namespace pwfs {
// slope stage on an n_in x n_in input whose four img x img pupil images start
// at (org_r[q], org_c[q]) and are cut into the sensor's n x n subapertures
// (the intensity plane, or the detector pixels of the detector stage); when
// img is not a multiple of n, pixels cut by subaperture edges count with
// their area fraction
int slopes_launch_at(const SensorPlan& sp, const float* in, long long in_stride, float* slopes,
                     long long slope_stride, float* flux, long long flux_stride, const float* ref, int nf, int n_in,
                     int img, const int* org_r, const int* org_c, hipStream_t st, Prof* prof);
int forward_sensor(pwfs_plan_s* p, int i, const float* opd, long long opd_stride, float* out, long long out_stride,
                   int nf, hipStream_t st);
}
