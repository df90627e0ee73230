/*
 * pwfs.h -- C ABI of the MI355X (gfx950) pyramid wavefront sensor library.
 *
 * The library computes the forward model of a tip-tilt-modulated four-face
 * pyramid wavefront sensor and its slope stage: the ``ModulatedPyramid`` and
 * ``PyrSlopec`` processing objects of the paper (Section 2.3 and Table 4; the
 * pyramid block of the SOUL listing in Appendix B gives the parameters).  For
 * every frame, wavelength and modulation point k:
 *
 *   E_k = A exp(i 2 pi OPD / lambda) exp(i 2 pi r (x cos t_k + y sin t_k) / D),
 *   zero-padded to N x N and tilted by half a focal pixel;
 *   e_k = IDFT2( DFT2(E_k) . m(x)m ),  m[u] = exp(i pi S |u + 1/2| / N);
 *   I   = sum_lambda w_lambda (1/n_mod) sum_k |e_k|^2 / sum(A^2);
 *
 * then the four pupil images of I are binned into subapertures and turned
 * into normalised slopes minus the flat-wavefront reference.
 *
 * Conventions shared by every entry point:
 *  - Every call returns a pwfs_status (0 = success); pwfs_last_error() gives
 *    a thread-local message for the last failure.  No C++ exception crosses
 *    this boundary.
 *  - Device pointers are HIP device addresses owned by the caller; the
 *    library never allocates or frees device memory (the one device array it
 *    holds, the static scratch of pwfs_gemm_noalloc, is part of its code
 *    object).  Streams are hipStream_t passed as void* (NULL = the null
 *    stream).
 *  - pwfs_forward / pwfs_slopes only enqueue kernels on the given stream:
 *    they neither allocate nor synchronise, so they may be captured into a
 *    HIP graph.  Argument checks are synchronous; launch errors are read with
 *    hipGetLastError after each launch; asynchronous device faults surface at
 *    the caller's next synchronisation.
 *  - One plan is used by one stream at a time.
 *  - Arrays are row-major float32.  For a plan over several sensors the
 *    per-sensor blocks of one frame are packed one after another, at the
 *    offsets pwfs_query reports.
 */
#ifndef PWFS_H
#define PWFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwfs_plan_s* pwfs_plan_t;

typedef enum {
  PWFS_OK = 0,
  PWFS_EINVAL = -1,        /* bad argument or sensor description        */
  PWFS_EUNSUPPORTED = -2,  /* valid, but a size this library does not run */
  PWFS_EWORKSPACE = -3,    /* workspace missing, too small or misaligned */
  PWFS_EHIP = -4,          /* a HIP runtime call or launch failed       */
  PWFS_ESTATE = -5         /* call out of order (e.g. frames > max)     */
} pwfs_status;

/* Arithmetic of the two transforms of the forward model. */
typedef enum {
  PWFS_FP32 = 0,    /* radix FFTs in float32 on the vector ALUs            */
  PWFS_BF16 = 1,    /* dense DFT operator as bf16 MFMA products, 1 term     */
  PWFS_BF16X3 = 2,  /* bf16 MFMA with hi/lo split, 3 products, fp32 accum   */
  PWFS_FP16X3 = 3,  /* fp16 MFMA with scaled hi/lo split, 3 products        */
  PWFS_FP16 = 4     /* dense DFT operator as fp16 MFMA products, 1 term:
                       the bf16 form's speed with 3 more mantissa bits      */
} pwfs_precision;

enum {
  PWFS_F_REF_SLOPES = 1,  /* subtract flat-wavefront reference slopes        */
  PWFS_F_FULL_PLANE = 2,  /* compute every pixel of the N x N plane; without
                             it only the four D x D pupil images are written
                             and the other pixels are left untouched        */
  PWFS_F_LOCAL_NORM = 4,  /* normalise by per-subaperture flux, not mean    */
  PWFS_F_DOUBLE_ROOF = 8  /* double-roof sensor (Table 4: ModulatedDoubleRoof)
                             instead of the four-face pyramid: a 50/50 splitter
                             feeds two roof prisms, the first with its edge
                             along x (two images S apart in x, centred in y),
                             the second along y; each arm has half the light
                             and a plane of its own, so the sensor's intensity
                             block is two N x N planes (arm x, then arm y).
                             Slopes: s_x from arm x's images, s_y from arm y's,
                             each over its own arm's mean flux (or the
                             subaperture's, with PWFS_F_LOCAL_NORM).  FP32
                             precision, per-sensor launches only; not with the
                             detector stage                                  */
};

/* Wavelengths per sensor.  A polychromatic sensor (Table 4: PolyCromPyramid)
 * is a weighted sum of monochromatic ones; 16 samples cover a broad sensing
 * band (e.g. the 300 nm bandwidth of the SOUL detector) finely.  Cost grows
 * linearly with the count. */
#define PWFS_MAX_LAMBDA 16

/*
 * One sensor.  Pixel conventions: pupil pixel centres at i - (D-1)/2; the
 * pupil sits at offset (N-D)/2 of the N x N grid; focal bins at half-integer
 * coordinates; image q = 2*iy + ix of the four pupil images starts at
 * (N/2 + sy S/2 - D/2, N/2 + sx S/2 - D/2) with s = -1 for i = 0, +1 for i = 1.
 */
typedef struct {
  int32_t n_pupil;        /* D, even, >= 4                                     */
  int32_t n_fft;          /* N: 128, 256, 384, 512 or 768                      */
  int32_t n_subap;        /* subapertures across, 1 .. min(D, 64); D / n_subap
                             need not be whole (SOUL: 220 / 40 = 5.5): pixels
                             cut by subaperture edges then count with their
                             area fraction, in binning and in the valid map
                             (valid: at least half the subaperture's area on
                             lit pupil pixels)                                 */
  int32_t n_mod;          /* modulation points, >= 1                           */
  int32_t n_lambda;       /* 1 .. PWFS_MAX_LAMBDA                              */
  int32_t precision;      /* pwfs_precision                                    */
  uint32_t flags;         /* PWFS_F_*                                          */
  int32_t src_rings;      /* extended source: rings sampling a uniform disk of
                             radius src_radius_lod (centre + 6q points on ring
                             q), 0 = point source; 0..8, FP32 path only        */
  double diameter_m;      /* telescope diameter (> 0; informational)           */
  double obstruction;     /* linear central obstruction ratio, [0, 1)          */
  double pupil_sep_px;    /* S: even integer, D <= S, S + D <= N                */
  double mod_radius_lod;  /* modulation radius in lambda/D at lambda_ref, >= 0  */
  double lambda_ref_nm;   /* wavelength at which the radius is given, > 0       */
  double lambda_nm[PWFS_MAX_LAMBDA];      /* sensing wavelengths, > 0          */
  double lambda_weight[PWFS_MAX_LAMBDA];  /* >= 0, summing to 1 (to 1e-9)      */
  double src_radius_lod;  /* extended-source radius in lambda/D at lambda_ref  */
  double fov_lod;         /* field stop: a square of side fov_lod lambda/D at
                             lambda_ref (a fixed sky angle) centred on the apex,
                             0 = none.  At wavelength l its side in focal samples
                             is side = ((fov_lod * (lambda_ref / l)) * N) / D
                             (float64, in that order); sample u passes when
                             2 |u_bar| <= side, on both axes.  FP32 only       */
} pwfs_sensor_desc;

/* What a plan reports about one of its sensors. */
typedef struct {
  int32_t n_pupil, n_fft, n_subap, n_valid;
  size_t opd_offset;        /* floats into one frame of the packed OPD input   */
  size_t intensity_offset;  /* floats into one frame of the packed intensity   */
  size_t slope_offset;      /* floats into one frame of the packed slopes      */
  size_t opd_stride, intensity_stride, slope_stride;  /* floats per frame, all sensors */
} pwfs_sensor_info;

/*
 * Checks sensor descriptions on the host; touches no device.  Returns
 * PWFS_EINVAL for a malformed description (N < D, odd N - D, n_subap > D,
 * pupil images outside the grid, n_mod <= 0, wavelength <= 0, weights not
 * summing to 1, ...) and PWFS_EUNSUPPORTED for a valid one whose FFT size
 * has no radix plan here.
 */
int pwfs_validate(const pwfs_sensor_desc* sensors, int n_sensors);

/*
 * Device workspace, in bytes, that pwfs_plan needs for these sensors and up
 * to max_frames frames per pwfs_forward call.  Host only.
 */
int pwfs_workspace_size(const pwfs_sensor_desc* sensors, int n_sensors, int max_frames,
                        size_t* bytes);

/*
 * Builds a plan: validates, builds the float64 tables (pupil, ramps, mask,
 * twiddles, valid map) on the host and copies them into d_workspace (caller
 * owned, >= pwfs_workspace_size bytes, 256-byte aligned, alive until
 * pwfs_destroy), then, if PWFS_F_REF_SLOPES is set, computes the reference
 * slopes of a flat wavefront on the device.  Synchronises hip_stream before
 * returning.  The plan handle holds host metadata only.
 */
int pwfs_plan(const pwfs_sensor_desc* sensors, int n_sensors, int max_frames,
              void* d_workspace, size_t ws_bytes, void* hip_stream, pwfs_plan_t* out);

/*
 * Forward model: d_opd_nm [n_frames][opd_stride] optical path difference in
 * nm (float32) -> d_intensity [n_frames][intensity_stride], each sensor's
 * block an N x N plane normalised so that a full plane sums to 1.  Without
 * PWFS_F_FULL_PLANE only the four pupil-image windows are written.
 * 1 <= n_frames <= max_frames.  Asynchronous on hip_stream.
 */
int pwfs_forward(pwfs_plan_t plan, const float* d_opd_nm, int n_frames, float* d_intensity,
                 void* hip_stream);

/*
 * Slope stage: d_intensity as written by pwfs_forward -> d_slopes
 * [n_frames][slope_stride] (per sensor [2][n_subap][n_subap], x then y,
 * zero outside the valid map) and, if d_flux is not NULL, d_flux
 * [n_frames][n_sensors] = total flux of the valid subapertures (summed in
 * float64).  Asynchronous on hip_stream.
 */
int pwfs_slopes(pwfs_plan_t plan, const float* d_intensity, int n_frames, float* d_slopes,
                float* d_flux, void* hip_stream);

/*
 * Execution tuning of a plan (chosen by the autotuner, see autotune.py).
 *  mode       PWFS_MODE_LAUNCHES: per sensor, a field, a row and a column
 *             launch per pass; PWFS_MODE_PERSISTENT: one persistent launch per
 *             pass for all sensors, whose workgroups claim field, row and
 *             column work items from a device counter (a sensor's row items
 *             wait for its field items, its column items for its row items).
 *             Both modes give bit-identical results.  PWFS_MODE_FUSED (FP32
 *             pyramid sensors with N = 64 or 128): one launch for all frames,
 *             one workgroup per frame holding the field, the row-pass output
 *             and the intensity on chip, so a frame reads only its OPD from
 *             HBM and writes only its intensity; the |e|^2 sum runs in point
 *             order, so results match the other modes to rounding, not bits.
 *  chunk      frames per pass, 1 .. max_chunk (set by the workspace size)
 *  wg_per_cu  persistent workgroups per compute unit, 1 .. 8
 *  row_groups minimum number of row-pass work items per pass
 *  spin_limit polls of a persistent pass's dependency wait before it gives
 *             up (0 = the default, 2^24); a wait that gives up skips its
 *             work item and sets the plan's sticky error flag (pwfs_device_status).
 *             A negative value makes every wait give up at once: a failure
 *             forced from the host, for testing that path
 */
enum { PWFS_MODE_LAUNCHES = 0, PWFS_MODE_PERSISTENT = 1, PWFS_MODE_FUSED = 2 };
typedef struct {
  int32_t mode, chunk, wg_per_cu, row_groups, max_chunk, spin_limit, reserved[2];
} pwfs_tuning;
int pwfs_get_tuning(pwfs_plan_t plan, pwfs_tuning* out);
/* PWFS_EUNSUPPORTED for the persistent mode unless every sensor is FP32 with
 * N >= 256 and at most 3 non-zero inputs per first-stage butterfly. */
int pwfs_set_tuning(pwfs_plan_t plan, const pwfs_tuning* tuning);

/*
 * Row-pass tile of one FP32 sensor: rows of the field per row-pass
 * workgroup.  Each N has a default and one alternative (N = 256, 512, 768:
 * 8 and 16; N = 384: 16 and 8; N = 64 and 128 have one tile, 32 and 16).  A
 * taller tile writes longer contiguous segments of the row-pass output (rows
 * x 8 bytes per column) but holds more LDS, so fewer workgroups share a
 * compute unit; the autotuner measures both.  Every tile gives bit-identical
 * results, in both launch modes.  rows = 0 restores the default.
 * PWFS_EINVAL for a sensor out of range, a tile not compiled for the
 * sensor's N or one whose LDS would exceed 160 KiB; PWFS_EUNSUPPORTED for a
 * sensor that is not on the FP32 path.  Takes effect at the next forward
 * call; not to be called while a call on the plan is being enqueued.
 */
int pwfs_set_row_tile(pwfs_plan_t plan, int sensor, int rows);
/* The tile sensor `sensor` runs with (its selection or the default). */
int pwfs_get_row_tile(pwfs_plan_t plan, int sensor, int* rows);

/*
 * Device-side status of the plan's work enqueued on hip_stream so far:
 * synchronises hip_stream, then returns PWFS_EHIP (message in
 * pwfs_last_error) if a persistent pass's dependency wait gave up since the
 * last call (those calls' intensities may be incomplete), and clears the
 * flag; PWFS_OK otherwise.  Not for use under graph capture.
 */
int pwfs_device_status(pwfs_plan_t plan, void* hip_stream);

/* Geometry and packing of sensor `sensor` of the plan. */
int pwfs_query(pwfs_plan_t plan, int sensor, pwfs_sensor_info* info);

/* Copies the valid-subaperture map of `sensor` (n_subap^2 bytes, 0/1) to host. */
int pwfs_valid_map(pwfs_plan_t plan, int sensor, uint8_t* host_out);

/*
 * Kernel timing for benchmarks.  pwfs_profile(plan, n) creates a pool of
 * 2n HIP events and, until called again with n = 0, records a start and a
 * stop event on the launch stream around each of the next n kernel launches
 * of this plan (launches beyond n are not timed).  Calling it again resets
 * the pool.  Not for use under graph capture.
 * pwfs_profile_read waits for the recorded events of one kernel kind
 * (0 = row pass, 1 = column pass, 2 = slope stage, 3 = matrix-core forward,
 * 4 = pupil-field pass, 5 = persistent heterogeneous pass, 6 = detector,
 * 7 = fused pass)
 * and returns their summed duration in ms and their number.
 */
int pwfs_profile(pwfs_plan_t plan, int max_launches);
int pwfs_profile_read(pwfs_plan_t plan, int kernel, double* total_ms, int* launches);

/* ------------------------------------------------------------------------
 * Detector stage: the paper's CCD processing object between the sensor and
 * the slope computer (Table 4), with the parameters of its SOUL
 * configuration (Appendix B): detector size, photon / readout / excess
 * noise switches, readout level; the source flux, integration time,
 * bandwidth and quantum efficiency enter through `electrons`.
 *
 * Detector pixels are r = rebin / rebin_den transform pixels wide (SOUL
 * reads 660 transform pixels onto a 120 px detector: r = 11/2); the
 * detector covers the central (n_det r) square of the plane, which must be
 * whole transform pixels.
 *
 * Per detector pixel p and frame f (global frame index frame0 + f):
 *   lam = electrons * sum over the transform pixels the detector pixel
 *         overlaps, in row-major order and float64, of w * I with
 *         w = (overlap_y * overlap_x) / rebin_den^2, overlaps in units of
 *         1/rebin_den pixel (an integer rebin gives w = 1: block sums);
 *         without PWFS_F_FULL_PLANE only pixels inside the four pupil images
 *         count (the rest of the plane is not written by pwfs_forward);
 *   photon noise: n ~ Poisson(lam) (else the value is lam);
 *   excess noise: n -> Gamma(n, 1) (electron multiplication at high gain);
 *   readout noise: + N(0, readout_e^2).
 * Random numbers: Philox4x64-10 keyed by (seed, 0), counter (p, frame,
 * purpose, block), so results depend only on (seed, frame index, pixel),
 * not on how frames are batched.
 * ------------------------------------------------------------------------ */

enum { PWFS_CCD_PHOTON = 1, PWFS_CCD_READOUT = 2, PWFS_CCD_EXCESS = 4 };

typedef struct {
  int32_t n_det;      /* detector pixels per side */
  int32_t rebin;      /* transform pixels per detector pixel, per side: rebin / rebin_den */
  uint32_t flags;     /* PWFS_CCD_* (excess noise needs photon noise) */
  int32_t rebin_den;  /* 0 or 1: whole transform pixels; else 2 .. 64, rebin >= rebin_den */
  double electrons;   /* expected photo-electrons per frame over the whole normalised plane, >= 0 */
  double readout_e;   /* readout noise RMS [electrons / pixel / frame], >= 0 */
  uint64_t seed;      /* key of the random draws */
} pwfs_ccd_desc;

/*
 * Detector frames of one sensor: d_intensity as written by pwfs_forward
 * ([n_frames][intensity_stride], the sensor's plane at its intensity
 * offset) -> d_pixels [n_frames][n_det][n_det] float32 electrons.
 * Requires n_det r whole and <= N with N - n_det r even; without
 * PWFS_F_FULL_PLANE also that the pupil images fall on whole detector
 * pixels.  PWFS_EINVAL for a bad description, PWFS_ESTATE for n_frames
 * outside [1, max_frames].  Asynchronous on hip_stream.
 */
int pwfs_ccd(pwfs_plan_t plan, int sensor, const pwfs_ccd_desc* ccd, const float* d_intensity, int n_frames,
             long long frame0, float* d_pixels, void* hip_stream);

/*
 * Slope stage on detector frames: the sensor's slope definition applied to
 * the four pupil images on the detector (D / r pixels each, binned
 * D / (r n_subap) per subaperture), minus the sensor's reference slopes when
 * PWFS_F_REF_SLOPES is set (the subapertures then cover the same areas of
 * the plane as the sensor's own, so the reference carries over).  d_slopes [n_frames][2][n][n],
 * d_flux [n_frames] or NULL.  Requires the pupil images to fall on whole
 * detector pixels tiled by the subapertures (PWFS_EINVAL otherwise).
 * Asynchronous on hip_stream.
 */
int pwfs_ccd_slopes(pwfs_plan_t plan, int sensor, const pwfs_ccd_desc* ccd, const float* d_pixels, int n_frames,
                    float* d_slopes, float* d_flux, void* hip_stream);

/* ------------------------------------------------------------------------
 * Closed loop (the SOUL chain of Appendix B: atmosphere -> mirror -> pyramid
 * -> Modalrec -> Integrator, closed through the delayed connection of
 * Section 2.1).  The mirror (OPD -= B c) and the reconstructor (m = R s) are
 * pwfs_gemm products; these two calls are the rest.  The time index t is an
 * int64 in device memory, read by pwfs_layers and advanced by
 * pwfs_integrator, so one captured timestep replays unchanged.
 * ------------------------------------------------------------------------ */

typedef struct {
  double weight;               /* multiplies the layer's screen */
  double origin_x, origin_y;   /* screen coordinates (pixels) of pupil pixel (0, 0) at t = 0 */
  double vel_x, vel_y;         /* pixels per time step */
} pwfs_layer;

/*
 * d_opd [D][D] float32 = sum_l weight_l * S_l(x + origin_x_l + vel_x_l t,
 * y + origin_y_l + vel_y_l t) with t = *d_step: frozen-flow layers, each
 * screen S_l periodic ([n_layers][rows][cols] float32 on the device),
 * sampled bilinearly in float64 (pupil pixel (x, y) = column x, row y).
 * layers is a host array of n_layers (1..16) entries.  Asynchronous.
 */
int pwfs_layers(const float* d_screens, int n_layers, int rows, int cols, const pwfs_layer* layers, int D,
                const long long* d_step, float* d_opd, void* hip_stream);

/*
 * Integrator step at t = *d_step: c(t) = ff * c(t-1) + gain * m(t) per mode
 * (c(-1) = 0), stored in d_hist [delay + 1][n_modes] at slot t mod
 * (delay + 1); d_applied <- c(t + 1 - delay) (zero before it exists), the
 * command the mirror applies at the next step; then *d_step = t + 1.
 * d_hist must be zeroed with *d_step = 0 to start a loop.  delay in [1, 64].
 * Asynchronous (one workgroup).
 */
int pwfs_integrator(const float* d_modes, const float* d_gain, const float* d_ff, int n_modes, int delay,
                    float* d_hist, float* d_applied, long long* d_step, void* hip_stream);

/*
 * y[M] = alpha * A[M][K] x[K] + beta * y in float32 (fma accumulation per
 * row, fixed-order sum): the loop's mirror (OPD -= B c) and reconstructor
 * (m = R s), matrix-vector products bound by reading A once.  Row-major A
 * with lda >= K; with beta == 0 the old y is not read.  Asynchronous.
 */
int pwfs_gemv(const float* d_A, long long lda, const float* d_x, float* d_y, int M, int K, float alpha, float beta,
              void* hip_stream);

/* ------------------------------------------------------------------------
 * Shack-Hartmann sensor (the paper's SH processing object, Table 4; FFT
 * workload shapes in Table 2, e.g. the SCAO SH: 160 px pupil, 20 x 20
 * subapertures, 56 x 56 focal samples each).  Per frame and subaperture:
 * the b x b block (b = n_pupil / n_subap) of A exp(i 2 pi OPD / lambda) is
 * transformed onto n_fft x n_fft focal samples at the half-integer
 * frequencies (u - n_fft/2 + 1/2) / n_fft, |F|^2 / (n_fft^2 sum A^2) is
 * summed over rebin x rebin samples into n_pix x n_pix detector pixels
 * (n_pix = n_fft / rebin), and the slopes are the pixels' centre of gravity
 * in pixels from the subaperture centre (x along columns, then y).  A
 * subaperture is valid when at least half of its pupil pixels are lit
 * (pupil pixel centres at i - (D-1)/2, lit for eps R <= r <= R); invalid
 * ones get zero slopes and pixels.
 *
 * Polychromatic sensor (Table 4: PolyChromSH), n_lambda >= 2: the spot image
 * is sum_l w_l spot_l over the sampled wavelengths.  The focal samples are
 * fixed in angle: the n_fft samples span the pixel-limited field at the
 * reference wavelength lambda_nm, so at lambda_l the block is transformed at
 * the frequencies (u - n_fft/2 + 1/2) s / n_fft with s = lambda_nm / lambda_l
 * (<= 1: lambda_nm may not exceed any lambda_l), and spot_l carries s^2 for
 * the fixed solid angle of a sample.
 * ------------------------------------------------------------------------ */

typedef struct pwfs_sh_s* pwfs_sh_t;

typedef struct {
  int32_t n_pupil;        /* D, a multiple of n_subap                          */
  int32_t n_subap;        /* subapertures across; b = D / n_subap <= 32         */
  int32_t n_fft;          /* focal samples per subaperture and axis, 2..512     */
  int32_t rebin;          /* focal samples per detector pixel; divides n_fft    */
  int32_t n_lambda;       /* 0 or 1: monochromatic at lambda_nm; 2 ..
                             PWFS_MAX_LAMBDA: polychromatic over lambdas_nm   */
  int32_t pad_;           /* must be 0                                         */
  double obstruction;     /* linear central obstruction ratio, [0, 1)          */
  double lambda_nm;       /* wavelength (monochromatic), or the reference that
                             fixes the angular sampling (polychromatic), > 0  */
  double lambdas_nm[PWFS_MAX_LAMBDA];      /* polychromatic: >= lambda_nm      */
  double lambda_weights[PWFS_MAX_LAMBDA];  /* polychromatic: >= 0, summing to 1
                                              (to 1e-9)                        */
} pwfs_sh_desc;

/* Host-only check: PWFS_EINVAL for a malformed description,
 * PWFS_EUNSUPPORTED when b > 32 or the tables do not fit the LDS. */
int pwfs_sh_validate(const pwfs_sh_desc* sh);
int pwfs_sh_workspace_size(const pwfs_sh_desc* sh, int max_frames, size_t* bytes);

/* Builds the tables (pupil, valid map, focal DFT matrix, float64 on the
 * host) into d_workspace (caller owned, 256-byte aligned); synchronises
 * hip_stream.  The handle holds host metadata only. */
int pwfs_sh_plan(const pwfs_sh_desc* sh, int max_frames, void* d_workspace, size_t ws_bytes, void* hip_stream,
                 pwfs_sh_t* out);

/* d_opd_nm [n_frames][D][D] -> d_slopes [n_frames][2][n_subap][n_subap] and,
 * if d_pixels is not NULL, the detector pixels [n_frames][n_subap][n_subap]
 * [n_pix][n_pix].  1 <= n_frames <= max_frames.  Asynchronous. */
int pwfs_sh_forward(pwfs_sh_t plan, const float* d_opd_nm, int n_frames, float* d_pixels, float* d_slopes,
                    void* hip_stream);
int pwfs_sh_query(pwfs_sh_t plan, int32_t* n_valid, int32_t* n_pix);
void pwfs_sh_destroy(pwfs_sh_t plan);

/* ------------------------------------------------------------------------
 * Matrix-core products.  The learned-surrogate form and its data pipeline
 * (modal coefficients -> OPD, the linear interaction-matrix baseline) need
 * dense products; they run on the same split-precision MFMA tiles as the
 * matrix-core forward model.  precision: PWFS_BF16 (bf16 operands, fp32
 * accumulation) or PWFS_BF16X3 (bf16 hi/lo split, three products, ~fp32).
 * ------------------------------------------------------------------------ */

/* Workspace bytes of pwfs_gemm for these sizes. */
int pwfs_gemm_workspace_size(int M, int N, int K, int precision, size_t* bytes);

/*
 * C[M][N] = alpha * sum_k A[M][k] B[N][k] + beta * C[M][N]: all float32
 * device arrays, row-major with leading dimensions lda >= K, ldb >= K,
 * ldc >= N; with beta == 0 the old C is not read (it may hold anything).
 * The operands are converted into 16-bit planes in d_workspace (256-byte
 * aligned, >= pwfs_gemm_workspace_size bytes).  Asynchronous on hip_stream.
 */
int pwfs_gemm(const float* A, long long lda, const float* B, long long ldb, float* C, long long ldc, int M, int N,
              int K, float alpha, float beta, int precision, void* d_workspace, size_t ws_bytes, void* hip_stream);

/*
 * pwfs_gemm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product, kernels and bits as pwfs_gemm, with the 16-bit operand
 * planes in a static device array of PWFS_GEMM_NOALLOC_MAX_BYTES that the
 * library holds on every GPU it runs on until the process ends, instead of
 * a caller workspace.  Sizes whose pwfs_gemm_workspace_size exceeds that
 * return PWFS_EWORKSPACE.  The array of the GPU current at the call is used
 * (hip_stream must belong to it); its address is looked up on the first
 * call on each device.  The call allocates and frees nothing.  Every call on
 * one GPU shares that GPU's array (each call writes all the plane bytes it
 * reads, so nothing needs clearing): calls that can overlap on one GPU
 * (different streams, or host threads enqueueing concurrently) race and must
 * be serialised by the caller.  Asynchronous on hip_stream.
 */
#define PWFS_GEMM_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int pwfs_gemm_noalloc(const float* A, long long lda, const float* B, long long ldb, float* C, long long ldc, int M,
                      int N, int K, float alpha, float beta, int precision, void* hip_stream);

/* out[r] = sqrt(mean_c x[r][c]^2) for r < rows (float32 device arrays). */
int pwfs_row_rms(const float* x, long long ld, int rows, int cols, float* out, void* hip_stream);

/*
 * Surrogate network: n_layers fully connected layers sizes[0] -> ... ->
 * sizes[n_layers], exact-erf GELU after every layer but the last, mean
 * squared error loss, Adam.  Weights are kept as float32 masters plus
 * 16-bit copies used by the products.  All device memory is the caller's
 * workspace (>= pwfs_mlp_workspace_size bytes, 256-byte aligned), cleared
 * by pwfs_mlp_create on hip_stream.  Parameters are exchanged packed and
 * unpadded: for each layer W [out][in] row-major, then b [out].
 */
typedef struct pwfs_mlp_s* pwfs_mlp_t;
int pwfs_mlp_workspace_size(int n_layers, const int32_t* sizes, int max_batch, int precision, size_t* bytes);
int pwfs_mlp_create(int n_layers, const int32_t* sizes, int max_batch, int precision, void* d_workspace,
                    size_t ws_bytes, void* hip_stream, pwfs_mlp_t* out);
int pwfs_mlp_param_count(pwfs_mlp_t mlp, size_t* count);
/* Loads parameters (device, packed) and clears the Adam state and step. */
int pwfs_mlp_set_params(pwfs_mlp_t mlp, const float* d_params, void* hip_stream);
int pwfs_mlp_get_params(pwfs_mlp_t mlp, float* d_params, void* hip_stream);
/*
 * Optimiser state, for checkpoint and resume: d_moments [2 * param_count]
 * holds Adam's first moments then its second moments, each packed like the
 * parameters, and *step the number of Adam steps taken.  Restoring a
 * checkpoint is pwfs_mlp_set_params then pwfs_mlp_set_state (in that order:
 * set_params clears the state); training then continues exactly as it would
 * have without the interruption (same bits, given the same batches).
 */
int pwfs_mlp_get_state(pwfs_mlp_t mlp, float* d_moments, long long* step, void* hip_stream);
int pwfs_mlp_set_state(pwfs_mlp_t mlp, const float* d_moments, long long step, void* hip_stream);
/*
 * Fixed linear term of inference: d_C [sizes[n]][sizes[0]] (device, row-major;
 * NULL removes it).  With it, pwfs_mlp_forward returns
 * out_scale * network(x) + C x, the linear part folded into the output
 * layer's product as a second run of its K loop (the input's 16-bit planes
 * against those of C / out_scale), so no separate product re-reads the
 * output.  Training (pwfs_mlp_grad) is unaffected: it fits the network part.
 * The learned surrogate uses it for its interaction-matrix term.
 */
int pwfs_mlp_set_linear(pwfs_mlp_t mlp, const float* d_C, void* hip_stream);
/* d_y [batch][sizes[n]] = out_scale * network(d_x [batch][sizes[0]]) (+ C x
 * with a linear term), 1 <= batch <= max_batch. */
int pwfs_mlp_forward(pwfs_mlp_t mlp, const float* d_x, int batch, float* d_y, float out_scale, void* hip_stream);
/*
 * Loss and gradients of mean((y - target_scale * t)^2) over the batch
 * (batch a multiple of 32, <= max_batch): d_loss (1 float, nullable),
 * d_grads (packed like the parameters, nullable; the gradients are also
 * kept for pwfs_mlp_adam).
 */
int pwfs_mlp_grad(pwfs_mlp_t mlp, const float* d_x, const float* d_t, int batch, float target_scale, float* d_loss,
                  float* d_grads, void* hip_stream);
/* One Adam step (bias-corrected) with the last gradients. */
int pwfs_mlp_adam(pwfs_mlp_t mlp, float lr, float beta1, float beta2, float eps, void* hip_stream);
void pwfs_mlp_destroy(pwfs_mlp_t mlp);

/* Thread-local message of the last failing call ("" if none). */
const char* pwfs_last_error(void);

/* Frees the host-side plan (the workspace stays the caller's). NULL is a no-op. */
void pwfs_destroy(pwfs_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* PWFS_H */
