"""FP64 CPU oracle of the modulated pyramid wavefront sensor and its slope stage.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call
this module: only the tests, the smoke check of the entry file and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library;
its only common dependency is the ``workloads`` package of seeded inputs.

What it computes is the plain Fourier-optics result of the sensor named by
the paper's ``ModulatedPyramid`` -> ``PyrSlopec`` chain (Section 2.3, Table 4;
parameters of the pyramid block in the SOUL listing of Appendix B).  The
paper never writes the sensor's equations down, so the forward model is the
textbook one, evaluated in complex128 with numpy's FFT as a library step:

  1. pupil amplitude A on a D x D grid, pixel centres at i - (D-1)/2;
  2. field A exp(i 2 pi OPD / lambda) times the modulation tilt of point k,
     zero-padded to N x N at offset (N-D)/2, times the half-pixel tilt h;
  3. unnormalised 2-D DFT, times the separable pyramid mask m (x) m;
  4. inverse 2-D DFT (1/N^2), |e|^2, averaged over k, weighted over lambda,
     divided by sum(A^2);
  5. the four pupil images are binned into b x b subapertures, slopes are
     the normalised face differences minus the flat-wavefront reference.

The readings taken where the paper is silent (apex on the corner of the four
central pixels, separable faces, centre-to-centre separation, geometric valid
map, global normaliser, reference-slope subtraction, sign) are the ones listed
in the design doc; each is stated again at the function that uses it.
"""

from __future__ import annotations

import numpy as np

FLAG_REF_SLOPES = 1
FLAG_FULL_PLANE = 2
FLAG_LOCAL_NORM = 4
FLAG_DOUBLE_ROOF = 8


def is_double_roof(s) -> bool:
    return bool(int(getattr(s, "flags", 0)) & FLAG_DOUBLE_ROOF)


# ---------------------------------------------------------------- geometry --

def centred(n: int) -> np.ndarray:
    """Pixel-centre coordinates of an n-pixel pupil axis, zero at its middle."""
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def pupil_amplitude(n_pupil: int, obstruction: float) -> np.ndarray:
    """Circular pupil stop (Table 3, ``PupilStop``): 1 where the pixel centre
    lies in the annulus obstruction*D/2 <= r <= D/2, else 0 (linear ratio)."""
    c = centred(n_pupil)
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    R = n_pupil / 2.0
    Ro = obstruction * R
    return ((r2 <= R * R) & (r2 >= Ro * Ro)).astype(np.float64)


def focal_coords(n_fft: int) -> np.ndarray:
    """Focal-plane coordinate of DFT bin u in pixels.  With the half-pixel
    input tilt the bins sit at half integers, so the pyramid apex falls on
    the corner between the four central pixels: u + 1/2 below N/2, u - N + 1/2
    from N/2 on."""
    u = np.arange(n_fft, dtype=np.float64)
    return np.where(u < n_fft // 2, u + 0.5, u - n_fft + 0.5)


def mask_vector(n_fft: int, pupil_sep: float) -> np.ndarray:
    """One axis of the four-face pyramid phase mask, exp(i pi S |u_bar| / N).

    The faces split along both axes, so the 2-D mask is m[v] m[u]; a face
    of slope pi S / N shifts its pupil image by S/2 pixels, which puts the
    four image centres S apart (the SOUL block's 'separation between pupil
    centers')."""
    ub = focal_coords(n_fft)
    return np.exp(1j * np.pi * pupil_sep * np.abs(ub) / n_fft)


def half_pixel_tilt(n_fft: int) -> np.ndarray:
    """h[X] = exp(-i pi X / N), X the array index: moves the DFT samples to
    half-integer focal coordinates."""
    return np.exp(-1j * np.pi * np.arange(n_fft, dtype=np.float64) / n_fft)


def modulation_angles(n_mod: int) -> np.ndarray:
    """Equispaced points on the modulation circle, counter-clockwise from +x."""
    return 2.0 * np.pi * np.arange(n_mod, dtype=np.float64) / n_mod


def modulation_ramp(n_pupil: int, radius_lod: float, theta: float) -> np.ndarray:
    """Pupil-plane tilt exp(i 2 pi r (x cos t + y sin t) / D) that moves the
    focal spot to r lambda/D along angle t (x = column, y = row)."""
    c = centred(n_pupil)
    arg = 2.0 * np.pi * radius_lod * (c[None, :] * np.cos(theta) + c[:, None] * np.sin(theta)) / n_pupil
    return np.exp(1j * arg)


def source_points(s) -> np.ndarray:
    """Points of the source in lambda/D at lambda_ref, [P][2] (x, y): the
    centre, plus, for an extended source of radius rho sampled with R rings,
    ring q = 1..R at radius rho q / R with 6 q points at angles 2 pi j / (6 q).
    Equal weights: with 6 q points on ring q the points are uniformly dense
    over the disk.  A point source is the centre alone."""
    R = int(getattr(s, "src_rings", 0))
    rho = float(getattr(s, "src_radius_lod", 0.0))
    pts = [(0.0, 0.0)]
    for q in range(1, R + 1):
        for j in range(6 * q):
            a = 2.0 * np.pi * j / (6 * q)
            pts.append((rho * q / R * np.cos(a), rho * q / R * np.sin(a)))
    return np.array(pts)


def tilt_ramp(n_pupil: int, tx_lod: float, ty_lod: float) -> np.ndarray:
    """Pupil-plane tilt exp(i 2 pi (tx x + ty y) / D): the focal spot moves by
    (tx, ty) lambda/D."""
    c = centred(n_pupil)
    return np.exp(1j * 2.0 * np.pi * (tx_lod * c[None, :] + ty_lod * c[:, None]) / n_pupil)


def image_origins(s) -> list:
    """Top-left corner (row, col) of the four pupil images, quadrant order
    q = 2*iy + ix with iy, ix = 0 for the image at N/2 - S/2 and 1 for N/2 + S/2.
    For a double roof: (plane, row, col) of arm x's images at x = N/2 -/+ S/2
    (q = 0, 1; plane 0, centred in y) and arm y's at y = N/2 -/+ S/2 (q = 2, 3;
    plane 1, centred in x)."""
    N, D, S = s.n_fft, s.n_pupil, int(round(s.pupil_sep_px))
    if is_double_roof(s):
        c = N // 2 - D // 2
        return [(0, c, N // 2 - S // 2 - D // 2), (0, c, N // 2 + S // 2 - D // 2),
                (1, N // 2 - S // 2 - D // 2, c), (1, N // 2 + S // 2 - D // 2, c)]
    out = []
    for sy in (-1, 1):
        for sx in (-1, 1):
            out.append((N // 2 + sy * S // 2 - D // 2, N // 2 + sx * S // 2 - D // 2))
    return out


# ----------------------------------------------------------------- forward --

def focal_field(E_pupil: np.ndarray, n_fft: int) -> np.ndarray:
    """Zero-pad a D x D pupil field to N x N at offset (N-D)/2, apply the
    half-pixel tilt and take the unnormalised 2-D DFT (exp(-2 pi i u x / N))."""
    D = E_pupil.shape[-1]
    o = (n_fft - D) // 2
    E = np.zeros((n_fft, n_fft), np.complex128)
    E[o:o + D, o:o + D] = E_pupil
    h = half_pixel_tilt(n_fft)
    E *= h[:, None] * h[None, :]
    return np.fft.fft2(E)


def pyramid_image(E_pupil: np.ndarray, n_fft: int, m: np.ndarray, m_y: np.ndarray | None = None) -> np.ndarray:
    """Complex field after the pyramid: IDFT2(DFT2(pad(E) h h) (m_y m)), with
    the inverse carrying 1/N^2 (m_y = m: the four faces)."""
    F = focal_field(E_pupil, n_fft)
    my = m if m_y is None else m_y
    return np.fft.ifft2(F * (my[:, None] * m[None, :]))


def forward_frame(opd_nm: np.ndarray, s, mask: np.ndarray | None = None) -> np.ndarray:
    """Normalised modulated intensity of one frame, float64 [N][N] ([2][N][N]
    for a double roof).

    I = sum_l w_l (1/(n_mod P)) sum_k sum_p |e_{l,k,p}|^2 / sum(A^2) over the
    modulation points k and the P source points p; phase 2 pi OPD / lambda,
    modulation radius and source offsets scaled by lambda_ref / lambda (fixed
    angles on the sky), mask in pixel units independent of lambda.

    Double roof (Table 4: ModulatedDoubleRoof; the geometry is a reading): a
    50/50 beam splitter feeds two roof prisms, one with the pyramid's edge
    along x only (mask m(u), 1 along v), one along y only; each arm gets half
    the light and forms two pupil images S apart along its own axis, on a
    plane of its own."""
    N = s.n_fft
    m = mask_vector(N, s.pupil_sep_px) if mask is None else mask
    if is_double_roof(s):
        one = np.ones(N, np.complex128)
        return np.stack([0.5 * _modulated(opd_nm, s, m, one), 0.5 * _modulated(opd_nm, s, one, m)])
    return _modulated(opd_nm, s, m, m)


def field_stop(s, lam: float) -> np.ndarray:
    """Transmission of the square field stop along one focal axis at
    wavelength lam (1 everywhere without one).  The stop is a fixed sky
    angle, fov_lod lambda/D at lambda_ref; at lam its side in samples is
    side = ((fov_lod * (lambda_ref / lam)) * N) / D, and sample u passes when
    2 |u_bar| <= side (the square is centred on the apex, at the corner of the
    four central samples).  The paper names a field of view (Appendix B,
    'fov') but not the stop's shape; square is the reading, which keeps the
    mask separable."""
    N, D = s.n_fft, s.n_pupil
    fov = float(getattr(s, "fov_lod", 0.0))
    if fov <= 0.0:
        return np.ones(N)
    side = ((fov * (s.lambda_ref_nm / lam)) * N) / D
    return (2.0 * np.abs(focal_coords(N)) <= side).astype(np.float64)


def _modulated(opd_nm: np.ndarray, s, m_x: np.ndarray, m_y: np.ndarray) -> np.ndarray:
    D, N = s.n_pupil, s.n_fft
    A = pupil_amplitude(D, s.obstruction)
    sA2 = float((A * A).sum())
    th = modulation_angles(s.n_mod)
    src = source_points(s)
    opd = np.asarray(opd_nm, dtype=np.float64)
    I = np.zeros((N, N), np.float64)
    for lam, w in zip(s.lambdas_nm, s.lambda_weights):
        E0 = A * np.exp(1j * 2.0 * np.pi * opd / lam)
        sc = s.lambda_ref_nm / lam
        r = s.mod_radius_lod * sc
        stop = field_stop(s, lam)
        mx, my = m_x * stop, m_y * stop
        acc = np.zeros((N, N), np.float64)
        for t in th:
            Em = E0 * modulation_ramp(D, r, t)
            for dx, dy in src:
                Ep = Em if (dx == 0.0 and dy == 0.0) else Em * tilt_ramp(D, sc * dx, sc * dy)
                e = pyramid_image(Ep, N, mx, my)
                acc += e.real ** 2 + e.imag ** 2
        I += w * acc / (s.n_mod * len(src) * sA2)
    return I


def forward(opd_nm: np.ndarray, s, mask: np.ndarray | None = None) -> np.ndarray:
    """Intensity for a batch of frames, float64 [F][N][N]."""
    opd_nm = np.asarray(opd_nm)
    if opd_nm.ndim == 2:
        opd_nm = opd_nm[None]
    return np.stack([forward_frame(o, s, mask) for o in opd_nm])


# ------------------------------------------ separable (matrix) form of 3-4 --

def separable_operator(n_fft: int, n_pupil: int, pupil_sep: float) -> np.ndarray:
    """P = IDFT diag(m) DFT diag(h) restricted to the D pupil columns, N x D.

    Because the mask and the tilt are separable, the padded 2-D chain of
    steps 3-4 equals e = P E P^T for a D x D pupil field E."""
    N, D = n_fft, n_pupil
    x = np.arange(N, dtype=np.float64)
    W = np.exp(-2j * np.pi * np.outer(x, x) / N)          # DFT matrix
    Winv = np.conj(W) / N
    m = mask_vector(N, pupil_sep)
    h = half_pixel_tilt(N)
    P = Winv @ (m[:, None] * W) * h[None, :]
    o = (N - D) // 2
    return P[:, o:o + D]


def forward_frame_separable(opd_nm: np.ndarray, s) -> np.ndarray:
    """The same intensity as ``forward_frame`` through e_k = P (E o R_k) P^T
    (point sources only)."""
    if int(getattr(s, "src_rings", 0)) > 0 or is_double_roof(s) or float(getattr(s, "fov_lod", 0.0)) > 0.0:
        raise ValueError("the separable form is written for a four-face pyramid and a point source")
    D, N = s.n_pupil, s.n_fft
    A = pupil_amplitude(D, s.obstruction)
    sA2 = float((A * A).sum())
    P = separable_operator(N, D, s.pupil_sep_px)
    opd = np.asarray(opd_nm, dtype=np.float64)
    I = np.zeros((N, N), np.float64)
    for lam, w in zip(s.lambdas_nm, s.lambda_weights):
        E0 = A * np.exp(1j * 2.0 * np.pi * opd / lam)
        r = s.mod_radius_lod * s.lambda_ref_nm / lam
        acc = np.zeros((N, N), np.float64)
        for t in modulation_angles(s.n_mod):
            e = P @ (E0 * modulation_ramp(D, r, t)) @ P.T
            acc += np.abs(e) ** 2
        I += w * acc / (s.n_mod * sA2)
    return I


# ------------------------------------------------------ binning and slopes --

def subaperture_overlaps(D: int, n: int) -> np.ndarray:
    """W [n][D]: the length of pixel y's overlap with subaperture i along one
    axis, in units of 1/n pixel (integers).  Subaperture i spans pixels
    [i D / n, (i + 1) D / n), which need not be whole pixels: a pixel cut by a
    subaperture edge is shared in proportion to area."""
    W = np.zeros((n, D))
    for i in range(n):
        for y in range(D):
            W[i, y] = max(0, min((y + 1) * n, (i + 1) * D) - max(y * n, i * D))
    return W


def bin_images(I: np.ndarray, s) -> np.ndarray:
    """Sum each of the four D x D pupil images over the subapertures:
    Q[f][q][i][j].  With b = D / n_subap whole, plain b x b block sums;
    otherwise pixels cut by subaperture edges count with their area
    fraction (Q = W I W^T, W the overlaps / n)."""
    I = np.asarray(I, dtype=np.float64)
    if I.ndim == (3 if is_double_roof(s) else 2):
        I = I[None]
    D, n = s.n_pupil, s.n_subap
    Q = np.zeros((I.shape[0], 4, n, n), np.float64)
    W = subaperture_overlaps(D, n) / n
    for q, org in enumerate(image_origins(s)):
        if is_double_roof(s):
            pl, r0, c0 = org
            win = I[:, pl, r0:r0 + D, c0:c0 + D]
        else:
            r0, c0 = org
            win = I[:, r0:r0 + D, c0:c0 + D]
        if D % n == 0:
            b = D // n
            Q[:, q] = win.reshape(I.shape[0], n, b, n, b).sum(axis=(2, 4))
        else:
            Q[:, q] = W @ win @ W.T
    return Q


def valid_subapertures(s) -> np.ndarray:
    """Geometric valid map: a subaperture is valid when at least half of its
    area lies on pixels inside the pupil stop (decided exactly: areas in
    units of 1/n_subap^2 pixel are integers, the subaperture's is D^2)."""
    A = pupil_amplitude(s.n_pupil, s.obstruction)
    W = subaperture_overlaps(s.n_pupil, s.n_subap)
    lit = W @ A @ W.T
    return 2.0 * lit >= float(s.n_pupil) ** 2


def raw_slopes_roof(Q: np.ndarray, valid: np.ndarray, local_norm: bool = False):
    """Double-roof slope computer (Table 4: DoubleRoofSlopec; the form is a
    reading): each axis from its own arm, s_x = (Q0 - Q1) / T_x with T_x the
    mean over valid subapertures of Q0 + Q1 (arm x), s_y = (Q2 - Q3) / T_y
    likewise (arm y); with ``local_norm`` each subaperture's own arm flux.
    Signs as for the pyramid (the image at N/2 - S/2 minus the one at
    N/2 + S/2).  flux = sum over valid subapertures of all four images."""
    Q = np.asarray(Q, dtype=np.float64)
    Tx = Q[:, 0] + Q[:, 1]
    Ty = Q[:, 2] + Q[:, 3]
    nv = valid.sum()
    if local_norm:
        nx = np.where(valid[None], Tx, 1.0)
        ny = np.where(valid[None], Ty, 1.0)
    else:
        nx = (Tx[:, valid].sum(axis=1) / nv)[:, None, None]
        ny = (Ty[:, valid].sum(axis=1) / nv)[:, None, None]
    s = np.stack([(Q[:, 0] - Q[:, 1]) / nx, (Q[:, 2] - Q[:, 3]) / ny], axis=1)
    s[:, :, ~valid] = 0.0
    return s, (Tx + Ty)[:, valid].sum(axis=1)


def raw_slopes(Q: np.ndarray, valid: np.ndarray, local_norm: bool = False):
    """Normalised face differences before reference subtraction.

    The image from the faces covering positive focal x sits at N/2 - S/2
    (quadrants with ix = 0); a positive x tilt moves light onto those faces,
    so s_x = (Q[ix=0] - Q[ix=1]) / T_bar is positive for it (likewise in y).
    T_bar is the mean total flux over valid subapertures (summed in float64);
    with ``local_norm`` each subaperture uses its own total flux instead.
    Returns (slopes [F][2][n][n], flux [F]) with flux = sum over valid T."""
    Q = np.asarray(Q, dtype=np.float64)
    T = Q.sum(axis=1)                                     # [F][n][n]
    sx = (Q[:, 0] + Q[:, 2]) - (Q[:, 1] + Q[:, 3])
    sy = (Q[:, 0] + Q[:, 1]) - (Q[:, 2] + Q[:, 3])
    flux = T[:, valid].sum(axis=1)
    if local_norm:
        norm = np.where(valid[None], T, 1.0)
    else:
        norm = (flux / valid.sum())[:, None, None]
    s = np.stack([sx / norm, sy / norm], axis=1)
    s[:, :, ~valid] = 0.0
    return s, flux


def sensor_raw_slopes(Q: np.ndarray, s, valid: np.ndarray):
    """The slope computer of sensor s: the pyramid's or the double roof's."""
    rs = raw_slopes_roof if is_double_roof(s) else raw_slopes
    return rs(Q, valid, bool(s.flags & FLAG_LOCAL_NORM))


def reference_slopes(s) -> np.ndarray:
    """Raw slopes of a flat wavefront, [2][n][n]."""
    D = s.n_pupil
    I = forward(np.zeros((1, D, D)), s)
    return sensor_raw_slopes(bin_images(I, s), s, valid_subapertures(s))[0][0]


def slopes(I: np.ndarray, s, ref: np.ndarray | None = None):
    """Slopes of intensities I [F][N][N] (``PyrSlopec``): raw slopes minus the
    flat-wavefront reference when the sensor asks for it, zero outside the
    valid map.  Returns (slopes [F][2][n][n], flux [F])."""
    valid = valid_subapertures(s)
    sl, flux = sensor_raw_slopes(bin_images(I, s), s, valid)
    if s.flags & FLAG_REF_SLOPES:
        if ref is None:
            ref = reference_slopes(s)
        sl = sl - ref[None]
        sl[:, :, ~valid] = 0.0
    return sl, flux


# --------------------------------------------------------- error metrics --

def intensity_rel_error(I: np.ndarray, I_ref: np.ndarray) -> np.ndarray:
    """Per-frame normwise relative error ||I - I_ref||_2 / ||I_ref||_2."""
    I = np.asarray(I, np.float64).reshape(len(I_ref), -1)
    R = np.asarray(I_ref, np.float64).reshape(len(I_ref), -1)
    return np.linalg.norm(I - R, axis=1) / np.linalg.norm(R, axis=1)


def slope_rel_rms(s: np.ndarray, s_ref: np.ndarray, valid: np.ndarray) -> float:
    """Pooled relative RMS error over valid subapertures and frames."""
    a = np.asarray(s, np.float64)[:, :, valid]
    b = np.asarray(s_ref, np.float64)[:, :, valid]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
