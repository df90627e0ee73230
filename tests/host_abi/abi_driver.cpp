// abi_driver.cpp -- drives every entry point of include/pwfs.h through its
// host code, linked against the HIP stand-in of hip_stub.cpp and built with
// AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).
//
// Sensor descriptions come from a file written by the Python test (the
// workloads and edge sensors the GPU tests use).  For each: validate, size
// the workspace, plan into a host buffer of exactly that size (the float64
// tables are written into it), run forward and slopes on host buffers (the
// launch configurations are checked by the stand-in), switch tunings, query,
// profile, destroy.  Then the detector, the Shack-Hartmann sensor, the dense
// products, the network, the loop kernels and the error paths.  Any
// sanitizer report, bad launch or unexpected status ends the run non-zero.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pwfs.h"

extern "C" long stub_launches();
extern "C" long stub_bad_launches();

namespace {

int g_fail = 0;

void expect(bool ok, const char* what, int line) {
  if (!ok) {
    fprintf(stderr, "FAIL line %d: %s (last error: %s)\n", line, what, pwfs_last_error());
    ++g_fail;
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

// host "device" buffer of exactly n bytes, 256-byte aligned start
struct Buf {
  void* raw = nullptr;
  void* p = nullptr;
  explicit Buf(size_t n) {
    // the request is rounded to 256 (aligned_alloc needs a multiple); every
    // size the library asks for is a multiple of 256 already
    const size_t m = (n + 255) & ~size_t(255);
    raw = aligned_alloc(256, m ? m : 256);
    memset(raw, 0, m ? m : 256);
    p = raw;
  }
  ~Buf() { free(raw); }
  float* f() { return (float*)p; }
};

void run_plan(const pwfs_sensor_desc* d, int n, int frames, const char* label) {
  EXPECT(pwfs_validate(d, n) == PWFS_OK);
  size_t bytes = 0;
  EXPECT(pwfs_workspace_size(d, n, frames, &bytes) == PWFS_OK);
  EXPECT(bytes % 256 == 0);
  Buf ws(bytes);
  pwfs_plan_t plan = nullptr;
  // one byte short is refused before anything is written
  EXPECT(pwfs_plan(d, n, frames, ws.p, bytes - 1, nullptr, &plan) == PWFS_EWORKSPACE && plan == nullptr);
  const int rc = pwfs_plan(d, n, frames, ws.p, bytes, nullptr, &plan);
  EXPECT(rc == PWFS_OK);
  if (rc != PWFS_OK) return;
  pwfs_sensor_info info{};
  EXPECT(pwfs_query(plan, 0, &info) == PWFS_OK);
  EXPECT(pwfs_query(plan, n, &info) == PWFS_EINVAL);
  Buf opd(sizeof(float) * frames * info.opd_stride), inten(sizeof(float) * frames * info.intensity_stride),
      slopes(sizeof(float) * frames * info.slope_stride), flux(sizeof(float) * frames * n);
  EXPECT(pwfs_forward(plan, opd.f(), frames, inten.f(), nullptr) == PWFS_OK);
  EXPECT(pwfs_slopes(plan, inten.f(), frames, slopes.f(), flux.f(), nullptr) == PWFS_OK);
  EXPECT(pwfs_forward(plan, opd.f(), frames + 1, inten.f(), nullptr) == PWFS_ESTATE);
  EXPECT(pwfs_forward(plan, nullptr, frames, inten.f(), nullptr) == PWFS_EINVAL);
  // every tuning the autotuner may set
  pwfs_tuning t{};
  EXPECT(pwfs_get_tuning(plan, &t) == PWFS_OK);
  for (int chunk = 1; chunk <= t.max_chunk; chunk = chunk * 2 + 1) {
    pwfs_tuning u = t;
    u.chunk = chunk;
    u.row_groups = chunk * 97;
    EXPECT(pwfs_set_tuning(plan, &u) == PWFS_OK);
    EXPECT(pwfs_forward(plan, opd.f(), frames, inten.f(), nullptr) == PWFS_OK);
    u.mode = PWFS_MODE_PERSISTENT;
    u.wg_per_cu = 1 + chunk % 8;
    if (pwfs_set_tuning(plan, &u) == PWFS_OK) EXPECT(pwfs_forward(plan, opd.f(), frames, inten.f(), nullptr) == 0);
    u.mode = PWFS_MODE_FUSED;
    if (pwfs_set_tuning(plan, &u) == PWFS_OK) EXPECT(pwfs_forward(plan, opd.f(), frames, inten.f(), nullptr) == 0);
  }
  pwfs_tuning bad = t;
  bad.chunk = t.max_chunk + 1;
  EXPECT(pwfs_set_tuning(plan, &bad) == PWFS_EINVAL);
  bad = t;
  bad.reserved[0] = 1;
  EXPECT(pwfs_set_tuning(plan, &bad) == PWFS_EINVAL);
  EXPECT(pwfs_set_tuning(plan, &t) == PWFS_OK);
  // row tiles: every value the autotuner tries, per sensor; forward with each accepted one
  for (int i = 0; i < n; ++i) {
    int rows = -1;
    EXPECT(pwfs_get_row_tile(plan, i, &rows) == PWFS_OK);
    EXPECT(rows == 8 || rows == 16 || rows == 32);
    for (int r : {4, 8, 16, 32}) {
      const int rc2 = pwfs_set_row_tile(plan, i, r);
      EXPECT(rc2 == PWFS_OK || rc2 == PWFS_EINVAL || rc2 == PWFS_EUNSUPPORTED);
      if (rc2 == PWFS_OK) EXPECT(pwfs_forward(plan, opd.f(), frames, inten.f(), nullptr) == PWFS_OK);
    }
    EXPECT(pwfs_set_row_tile(plan, i, 0) == PWFS_OK);
  }
  EXPECT(pwfs_set_row_tile(plan, n, 8) == PWFS_EINVAL);
  EXPECT(pwfs_get_row_tile(plan, 0, nullptr) == PWFS_EINVAL);
  EXPECT(pwfs_set_row_tile(nullptr, 0, 8) == PWFS_EINVAL);
  EXPECT(pwfs_profile(plan, 7) == PWFS_OK);
  EXPECT(pwfs_forward(plan, opd.f(), frames, inten.f(), nullptr) == PWFS_OK);
  EXPECT(pwfs_slopes(plan, inten.f(), frames, slopes.f(), nullptr, nullptr) == PWFS_OK);
  for (int k = 0; k < 8; ++k) {
    double ms = -1;
    int cnt = -1;
    EXPECT(pwfs_profile_read(plan, k, &ms, &cnt) == PWFS_OK);
  }
  EXPECT(pwfs_profile(plan, 0) == PWFS_OK);
  EXPECT(pwfs_device_status(plan, nullptr) == PWFS_OK);
  std::vector<uint8_t> vm((size_t)d[0].n_subap * d[0].n_subap);
  EXPECT(pwfs_valid_map(plan, 0, vm.data()) == PWFS_OK);
  // the detector stage, where the geometry allows it (integer and 11/2 pitch)
  if (n == 1 && !(d[0].flags & PWFS_F_DOUBLE_ROOF)) {
    for (int rb = 1; rb <= 2; ++rb) {
      pwfs_ccd_desc c{};
      c.rebin = rb == 1 ? 4 : 11;
      c.rebin_den = rb == 1 ? 0 : 2;
      const double r = rb == 1 ? 4.0 : 5.5;
      c.n_det = (int)(d[0].n_fft / r) & ~1;
      c.flags = PWFS_CCD_PHOTON | PWFS_CCD_READOUT | PWFS_CCD_EXCESS;
      c.electrons = 1e5;
      c.readout_e = 0.4;
      c.seed = 7;
      Buf pix(sizeof(float) * frames * c.n_det * c.n_det);
      Buf s2(sizeof(float) * frames * 2 * d[0].n_subap * d[0].n_subap), f2(sizeof(float) * frames);
      const int cc = pwfs_ccd(plan, 0, &c, inten.f(), frames, 1000, pix.f(), nullptr);
      EXPECT(cc == PWFS_OK || cc == PWFS_EINVAL);
      if (cc == PWFS_OK) {
        const int cs = pwfs_ccd_slopes(plan, 0, &c, pix.f(), frames, s2.f(), f2.f(), nullptr);
        EXPECT(cs == PWFS_OK || cs == PWFS_EINVAL);
      }
    }
  }
  pwfs_destroy(plan);
  printf("  %-34s n=%d frames=%d workspace %zu bytes: ok\n", label, n, frames, bytes);
}

void run_sh() {
  pwfs_sh_desc poly = {64, 8, 16, 2, 3, 0, 0.1, 600.0, {}, {}};
  const double lams[3] = {600.0, 750.0, 900.0}, ws3[3] = {0.25, 0.25, 0.5};
  for (int l = 0; l < 3; ++l) {
    poly.lambdas_nm[l] = lams[l];
    poly.lambda_weights[l] = ws3[l];
  }
  const pwfs_sh_desc cases[] = {{160, 20, 56, 7, 0, 0, 0.0, 750.0, {}, {}},
                                {476, 68, 240, 15, 0, 0, 0.28, 750.0, {}, {}},
                                {64, 8, 16, 2, 0, 0, 0.1, 600.0, {}, {}}, poly};
  for (const auto& sh : cases) {
    EXPECT(pwfs_sh_validate(&sh) == PWFS_OK);
    size_t bytes = 0;
    EXPECT(pwfs_sh_workspace_size(&sh, 3, &bytes) == PWFS_OK);
    Buf ws(bytes);
    pwfs_sh_t p = nullptr;
    EXPECT(pwfs_sh_plan(&sh, 3, ws.p, bytes, nullptr, &p) == PWFS_OK);
    int32_t nv = 0, npx = 0;
    EXPECT(pwfs_sh_query(p, &nv, &npx) == PWFS_OK && nv > 0 && npx == sh.n_fft / sh.rebin);
    const size_t n = sh.n_subap;
    Buf opd(sizeof(float) * 3 * sh.n_pupil * sh.n_pupil), sl(sizeof(float) * 3 * 2 * n * n),
        px(sizeof(float) * 3 * n * n * npx * npx);
    EXPECT(pwfs_sh_forward(p, opd.f(), 3, px.f(), sl.f(), nullptr) == PWFS_OK);
    EXPECT(pwfs_sh_forward(p, opd.f(), 4, nullptr, sl.f(), nullptr) == PWFS_ESTATE);
    pwfs_sh_destroy(p);
  }
  pwfs_sh_desc bad = cases[0];
  bad.rebin = 5;  // does not divide 56
  EXPECT(pwfs_sh_validate(&bad) == PWFS_EINVAL);
  bad = cases[0];
  bad.pad_ = 1;
  EXPECT(pwfs_sh_validate(&bad) == PWFS_EINVAL);
  bad = poly;
  bad.n_lambda = PWFS_MAX_LAMBDA + 1;
  EXPECT(pwfs_sh_validate(&bad) == PWFS_EINVAL);
  bad = poly;
  bad.lambdas_nm[0] = 500.0;   // below the reference
  EXPECT(pwfs_sh_validate(&bad) == PWFS_EINVAL);
  bad = poly;
  bad.lambda_weights[2] = 0.4;   // weights sum to 0.9
  EXPECT(pwfs_sh_validate(&bad) == PWFS_EINVAL);
  printf("  shack-hartmann: ok\n");
}

void run_dense() {
  const int M = 300, N = 200, K = 150;
  for (int prec : {PWFS_BF16, PWFS_BF16X3}) {
    size_t bytes = 0;
    EXPECT(pwfs_gemm_workspace_size(M, N, K, prec, &bytes) == PWFS_OK);
    Buf ws(bytes), A(sizeof(float) * M * K), B(sizeof(float) * N * K), C(sizeof(float) * M * N);
    EXPECT(pwfs_gemm(A.f(), K, B.f(), K, C.f(), N, M, N, K, 1.f, 0.f, prec, ws.p, bytes, nullptr) == PWFS_OK);
    EXPECT(pwfs_gemm(A.f(), K, B.f(), K, C.f(), N, M, N, K, 1.f, 0.f, prec, ws.p, bytes - 256, nullptr) ==
           PWFS_EWORKSPACE);
    EXPECT(pwfs_gemm_noalloc(A.f(), K, B.f(), K, C.f(), N, M, N, K, 1.f, 1.f, prec, nullptr) == PWFS_OK);
    EXPECT(pwfs_gemm_noalloc(A.f(), K, B.f(), K, C.f(), N - 1, M, N, K, 1.f, 1.f, prec, nullptr) == PWFS_EINVAL);
    // planes of 65536 x 1024 operands exceed the static scratch (pointers not touched)
    EXPECT(pwfs_gemm_noalloc(A.f(), 1024, B.f(), 1024, C.f(), 1 << 16, 1 << 16, 1 << 16, 1024, 1.f, 0.f, prec,
                             nullptr) == PWFS_EWORKSPACE);
  }
  Buf x(sizeof(float) * 64 * 33), r(sizeof(float) * 64);
  EXPECT(pwfs_row_rms(x.f(), 33, 64, 33, r.f(), nullptr) == PWFS_OK);
  EXPECT(pwfs_row_rms(x.f(), 32, 64, 33, r.f(), nullptr) == PWFS_EINVAL);
  // the network: sizes of the surrogate's shape, scaled down
  const int32_t sizes[] = {50, 96, 96, 130};
  for (int prec : {PWFS_BF16, PWFS_BF16X3}) {
    size_t bytes = 0;
    EXPECT(pwfs_mlp_workspace_size(3, sizes, 64, prec, &bytes) == PWFS_OK);
    Buf ws(bytes);
    pwfs_mlp_t m = nullptr;
    EXPECT(pwfs_mlp_create(3, sizes, 64, prec, ws.p, bytes, nullptr, &m) == PWFS_OK);
    size_t np = 0;
    EXPECT(pwfs_mlp_param_count(m, &np) == PWFS_OK && np == 50 * 96 + 96 + 96 * 96 + 96 + 96 * 130 + 130);
    Buf prm(sizeof(float) * np), g(sizeof(float) * np), in(sizeof(float) * 64 * 50), t(sizeof(float) * 64 * 130),
        y(sizeof(float) * 64 * 130), loss(sizeof(float));
    EXPECT(pwfs_mlp_set_params(m, prm.f(), nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_get_params(m, g.f(), nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_forward(m, in.f(), 37, y.f(), 1.f, nullptr) == PWFS_OK);
    Buf lin(sizeof(float) * 130 * 50);
    EXPECT(pwfs_mlp_set_linear(m, lin.f(), nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_forward(m, in.f(), 64, y.f(), 0.5f, nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_forward(m, in.f(), 64, y.f(), 2.0f, nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_forward(m, in.f(), 64, y.f(), 0.f, nullptr) == PWFS_EINVAL);
    EXPECT(pwfs_mlp_set_linear(m, nullptr, nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_grad(m, in.f(), t.f(), 64, 1.f, loss.f(), g.f(), nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_grad(m, in.f(), t.f(), 33, 1.f, loss.f(), g.f(), nullptr) == PWFS_ESTATE);
    EXPECT(pwfs_mlp_adam(m, 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr) == PWFS_OK);
    Buf mom(sizeof(float) * 2 * np);
    long long step = -1;
    EXPECT(pwfs_mlp_get_state(m, mom.f(), &step, nullptr) == PWFS_OK && step == 1);
    EXPECT(pwfs_mlp_set_state(m, mom.f(), step, nullptr) == PWFS_OK);
    EXPECT(pwfs_mlp_set_state(m, mom.f(), -1, nullptr) == PWFS_EINVAL);
    EXPECT(pwfs_mlp_forward(m, in.f(), 65, y.f(), 1.f, nullptr) == PWFS_ESTATE);
    pwfs_mlp_destroy(m);
  }
  // the loop's kernels
  pwfs_layer layers[2] = {{0.7, 1.5, 2.5, 0.3, -0.2}, {0.3, 0.0, 10.0, -1.0, 0.5}};
  Buf scr(sizeof(float) * 2 * 96 * 128), o(sizeof(float) * 40 * 40), step(sizeof(long long));
  EXPECT(pwfs_layers(scr.f(), 2, 96, 128, layers, 40, (const long long*)step.p, o.f(), nullptr) == PWFS_OK);
  EXPECT(pwfs_layers(scr.f(), 17, 96, 128, layers, 40, (const long long*)step.p, o.f(), nullptr) == PWFS_EINVAL);
  Buf modes(sizeof(float) * 500), gain(sizeof(float) * 500), ff(sizeof(float) * 500), hist(sizeof(float) * 3 * 500),
      applied(sizeof(float) * 500);
  EXPECT(pwfs_integrator(modes.f(), gain.f(), ff.f(), 500, 2, hist.f(), applied.f(), (long long*)step.p, nullptr) ==
         PWFS_OK);
  EXPECT(pwfs_integrator(modes.f(), gain.f(), ff.f(), 500, 65, hist.f(), applied.f(), (long long*)step.p, nullptr) ==
         PWFS_EINVAL);
  Buf Am(sizeof(float) * 100 * 70), xv(sizeof(float) * 70), yv(sizeof(float) * 100);
  EXPECT(pwfs_gemv(Am.f(), 70, xv.f(), yv.f(), 100, 70, 1.f, 0.f, nullptr) == PWFS_OK);
  EXPECT(pwfs_gemv(Am.f(), 69, xv.f(), yv.f(), 100, 70, 1.f, 0.f, nullptr) == PWFS_EINVAL);
  printf("  dense products, network, loop kernels: ok\n");
}

void run_invalid(const pwfs_sensor_desc& good) {
  struct Mut {
    const char* what;
    void (*f)(pwfs_sensor_desc&);
    int want;
  };
  const Mut muts[] = {
      {"odd pupil", [](pwfs_sensor_desc& d) { d.n_pupil += 1; }, PWFS_EINVAL},
      {"N < D", [](pwfs_sensor_desc& d) { d.n_fft = d.n_pupil - 2; }, PWFS_EINVAL},
      {"no radix plan", [](pwfs_sensor_desc& d) { d.n_fft = 200; d.pupil_sep_px = 100; d.n_pupil = 64; },
       PWFS_EUNSUPPORTED},
      {"subap > D", [](pwfs_sensor_desc& d) { d.n_subap = d.n_pupil + 1; }, PWFS_EINVAL},
      {"n_mod 0", [](pwfs_sensor_desc& d) { d.n_mod = 0; }, PWFS_EINVAL},
      {"17 wavelengths", [](pwfs_sensor_desc& d) { d.n_lambda = 17; }, PWFS_EINVAL},
      {"weights", [](pwfs_sensor_desc& d) { d.lambda_weight[0] = 0.5; }, PWFS_EINVAL},
      {"negative wavelength", [](pwfs_sensor_desc& d) { d.lambda_nm[0] = -1; }, PWFS_EINVAL},
      {"odd separation", [](pwfs_sensor_desc& d) { d.pupil_sep_px += 1; }, PWFS_EINVAL},
      {"images overlap", [](pwfs_sensor_desc& d) { d.pupil_sep_px = d.n_pupil - 2; }, PWFS_EINVAL},
      {"images outside", [](pwfs_sensor_desc& d) { d.pupil_sep_px = d.n_fft; }, PWFS_EINVAL},
      {"obstruction 1", [](pwfs_sensor_desc& d) { d.obstruction = 1.0; }, PWFS_EINVAL},
      {"NaN radius", [](pwfs_sensor_desc& d) { d.mod_radius_lod = 0.0 / 0.0; }, PWFS_EINVAL},
      {"flags", [](pwfs_sensor_desc& d) { d.flags |= 64; }, PWFS_EINVAL},
      {"precision", [](pwfs_sensor_desc& d) { d.precision = 9; }, PWFS_EINVAL},
      {"rings", [](pwfs_sensor_desc& d) { d.src_rings = 9; }, PWFS_EINVAL},
      {"fov", [](pwfs_sensor_desc& d) { d.fov_lod = -1; }, PWFS_EINVAL},
      {"stop in bf16", [](pwfs_sensor_desc& d) { d.fov_lod = 5; d.precision = PWFS_BF16X3; }, PWFS_EUNSUPPORTED},
      {"roof in bf16", [](pwfs_sensor_desc& d) { d.flags |= PWFS_F_DOUBLE_ROOF; d.precision = PWFS_BF16; },
       PWFS_EUNSUPPORTED},
  };
  for (const Mut& m : muts) {
    pwfs_sensor_desc d = good;
    m.f(d);
    const int rc = pwfs_validate(&d, 1);
    if (rc != m.want) fprintf(stderr, "mutation '%s': status %d, wanted %d\n", m.what, rc, m.want);
    EXPECT(rc == m.want);
    EXPECT(strlen(pwfs_last_error()) > 0);
    size_t b = 0;
    EXPECT(pwfs_workspace_size(&d, 1, 4, &b) == m.want);
  }
  EXPECT(pwfs_validate(nullptr, 1) == PWFS_EINVAL);
  EXPECT(pwfs_validate(&good, 0) == PWFS_EINVAL);
  pwfs_plan_t p = nullptr;
  EXPECT(pwfs_plan(&good, 1, 4, nullptr, 0, nullptr, &p) == PWFS_EWORKSPACE);
  EXPECT(pwfs_forward(nullptr, nullptr, 1, nullptr, nullptr) == PWFS_EINVAL);
  EXPECT(pwfs_device_status(nullptr, nullptr) == PWFS_EINVAL);
  pwfs_destroy(nullptr);
  printf("  invalid descriptions and arguments: ok\n");
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s descriptions.bin\n", argv[0]);
    return 2;
  }
  // file: int32 count, then per entry int32 group size g, int32 frames,
  // g pwfs_sensor_desc records
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t count = 0;
  if (fread(&count, 4, 1, f) != 1) return 2;
  pwfs_sensor_desc first{};
  for (int i = 0; i < count; ++i) {
    int32_t g = 0, frames = 0;
    if (fread(&g, 4, 1, f) != 1 || fread(&frames, 4, 1, f) != 1 || g < 1 || g > 64) return 2;
    std::vector<pwfs_sensor_desc> d(g);
    if (fread(d.data(), sizeof(pwfs_sensor_desc), g, f) != (size_t)g) return 2;
    if (i == 0) first = d[0];
    char label[64];
    snprintf(label, sizeof label, "entry %d (D=%d N=%d prec=%d flags=%u)", i, d[0].n_pupil, d[0].n_fft,
             d[0].precision, d[0].flags);
    run_plan(d.data(), g, frames, label);
  }
  fclose(f);
  run_sh();
  run_dense();
  run_invalid(first);
  printf("launches %ld, bad %ld, failures %d\n", stub_launches(), stub_bad_launches(), g_fail);
  if (g_fail || stub_bad_launches()) return 1;
  printf("ALL OK\n");
  return 0;
}
