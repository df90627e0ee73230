"""FP64 CPU oracle of the detector stage that follows the pyramid sensor.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call
this module: only the tests, the smoke check of the entry file and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

The paper lists a ``CCD`` processing object between the sensor and the slope
computer (Table 4) and gives its parameters in the SOUL listing of
Appendix B: detector size, integration time, bandwidth, switches for photon,
readout and excess noise, the readout level and the quantum efficiency.  It
does not write the model down, so the readings here are the textbook ones:

  1. expected photo-electrons per detector pixel: lam = n_e * (sum of the
     rebin x rebin block of the normalised intensity), the block sum taken
     in float64 in row-major order over the central rebin * n_det square of
     the N x N plane.  The detector pitch need not be a whole number of
     transform pixels (the SOUL sensor reads 660 transform pixels onto 120
     detector pixels, Appendix B: 5.5 each): a transform pixel cut by a
     detector pixel edge then counts with its area fraction;
  2. photon noise: a Poisson draw of mean lam;
  3. excess noise (electron-multiplying register at high gain): the output
     of n electrons is Gamma(n, 1) distributed (mean n, variance n);
  4. readout noise: plus a zero-mean Gaussian of RMS sigma_e.

Random numbers come from the counter-based generator Philox4x64-10
(Salmon, Moraes, Dror and Shaw, SC'11), keyed by (seed, 0); each draw has
its own counter (pixel, frame, purpose, block), so any frame of any chunk
gives the same numbers.  From a 64-bit word w, a uniform in [0, 1) is
(w >> 11) * 2^-53; a normal is Box-Muller on two uniforms.  Poisson draws
invert the CDF; the integer they return is decided in float64 with basic
operations only (exp(-mu) is formed by a fixed Taylor series and repeated
squaring), so an implementation that performs the same operations in the
same order returns the same integers.  Gamma draws use Marsaglia and Tsang's
method (ACM TOMS 2000).
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

PHOTON = 1
READOUT = 2
EXCESS = 4

# purposes (third counter word)
P_PHOTON, P_EXCESS, P_READOUT = 0, 1, 2

POISSON_CHUNK = 256.0      # largest mean drawn by one inversion
MAX_LAM = 2.0 ** 24        # larger or non-finite expected counts give NaN (bounds the O(lam) draw)
POISSON_KCAP = 1024        # inversion stops here (unreachable at mean <= 256 in practice)
GAMMA_TRIES = 64           # Marsaglia-Tsang attempts before giving up (returns d)

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


# --------------------------------------------------------------- Philox ---

def _mulhilo(a: np.uint64, b: np.ndarray):
    """(high, low) 64-bit halves of the 128-bit products a * b."""
    b = np.asarray(b, np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    cross = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (cross >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Philox4x64-10 of counters (c0, c1, c2, c3) (uint64 arrays, broadcast)
    under key (k0, k1); returns the four output words."""
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) for x in np.broadcast_arrays(c0, c1, c2, c3))
    k0 = np.uint64(k0)
    k1 = np.uint64(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = np.uint64(k0 + _W0)
                k1 = np.uint64(k1 + _W1)
            h0, l0 = _mulhilo(_M0, c0)
            h1, l1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = h1 ^ c1 ^ k0, l1, h0 ^ c3 ^ k1, l0
    return c0, c1, c2, c3


def uniform(w) -> np.ndarray:
    """[0, 1) float64 from 64-bit words."""
    return (np.asarray(w, np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


# ----------------------------------------------- elementary functions ---
# log, sqrt and cos(2 pi u) of the samplers, evaluated with + - * / and
# exact scalings by powers of two only, each operation rounded on its own,
# so that an implementation doing the same operations in the same order
# gets the same bits.  An accept/reject decision (the Gamma sampler's) then
# no longer depends on which math library evaluates it.

LN2 = 0.6931471805599453              # the float64 nearest ln 2
TWO_PI = 6.283185307179586            # the float64 nearest 2 pi
SQRT_HALF = 0.7071067811865476        # the float64 nearest sqrt(1/2)
LOG_TERMS = 12                        # atanh series terms: |s| <= 0.1716, s^26 / 27 < 1e-21
SQRT_NEWTON = 5                       # Newton steps after a linear first guess


def log_basic(x: np.ndarray) -> np.ndarray:
    """ln x for finite x > 0: x = m 2^e with m in [sqrt(1/2), sqrt 2), then
    ln m = 2 atanh(s), s = (m - 1) / (m + 1), as s times a Horner polynomial
    in s^2 of the series coefficients 1 / (2j + 1); ln x = e ln 2 + ln m."""
    m, e = np.frexp(np.asarray(x, np.float64))      # m in [0.5, 1)
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    p = np.full(s.shape, 1.0 / (2.0 * LOG_TERMS + 1.0))
    for j in range(LOG_TERMS - 1, -1, -1):
        t = p * s2
        p = t + 1.0 / (2.0 * j + 1.0)
    t = s * p
    t = t * 2.0
    return e * LN2 + t


def sqrt_basic(y: np.ndarray) -> np.ndarray:
    """sqrt y for finite y >= 0: y = m 2^e with e even and m in [0.5, 2),
    first guess 0.41731 + 0.59016 m, SQRT_NEWTON Newton steps
    g <- (g + m / g) / 2, then scaled by 2^(e/2)."""
    y = np.asarray(y, np.float64)
    m, e = np.frexp(y)                              # m in [0.5, 1)
    odd = (e % 2) != 0
    m = np.where(odd, m * 2.0, m)
    e = np.where(odd, e - 1, e)
    g = 0.41731 + 0.59016 * m
    for _ in range(SQRT_NEWTON):
        q = m / g
        g = (g + q) * 0.5
    r = np.ldexp(g, e // 2)
    return np.where(y == 0.0, 0.0, r)


def _fact(n: int) -> float:
    """n! as a float64 product formed left to right (exact for n <= 18)."""
    f = 1.0
    for i in range(2, n + 1):
        f = f * float(i)
    return f


def _cos_poly(x: np.ndarray) -> np.ndarray:
    """cos x for |x| <= pi/4: sum over k <= 8 of (-1)^k x^(2k) / (2k)!,
    Horner in x^2 from the highest term."""
    x2 = x * x
    c = np.full(x.shape, 1.0 / _fact(16))
    for k in range(7, -1, -1):
        t = c * x2
        c = (1.0 if k % 2 == 0 else -1.0) / _fact(2 * k) + t
    return c


def _sin_poly(x: np.ndarray) -> np.ndarray:
    """sin x for |x| <= pi/4: x times the sum over k <= 8 of
    (-1)^k x^(2k) / (2k + 1)!, Horner in x^2 from the highest term."""
    x2 = x * x
    c = np.full(x.shape, 1.0 / _fact(17))
    for k in range(7, -1, -1):
        t = c * x2
        c = (1.0 if k % 2 == 0 else -1.0) / _fact(2 * k + 1) + t
    return c * x


def cos_2pi_basic(u: np.ndarray) -> np.ndarray:
    """cos(2 pi u) for u in [0, 1): w = |u - round(u)| in [0, 1/2] (exact),
    then cos(2 pi w) on [0, 1/8], sin(2 pi (1/4 - w)) on (1/8, 3/8] and
    -cos(2 pi (1/2 - w)) above (each reduced argument exact, at most 1/8)."""
    u = np.asarray(u, np.float64)
    w = np.where(u >= 0.5, 1.0 - u, u)
    a = np.where(w <= 0.125, w, np.where(w <= 0.375, 0.25 - w, 0.5 - w))
    x = a * TWO_PI
    return np.where(w <= 0.125, _cos_poly(x), np.where(w <= 0.375, _sin_poly(x), -_cos_poly(x)))


def box_muller(w0, w1) -> np.ndarray:
    """Standard normal from two 64-bit words: sqrt(-2 ln u1) cos(2 pi u2)
    with the basic-operation functions above."""
    u1 = 1.0 - uniform(w0)              # (0, 1]
    u2 = uniform(w1)
    return sqrt_basic(-2.0 * log_basic(u1)) * cos_2pi_basic(u2)


# -------------------------------------------------------------- samplers ---

def exp_neg(mu: np.ndarray) -> np.ndarray:
    """exp(-mu) for 0 <= mu <= 256 with + - * / only: a 24-term Taylor
    series at mu / 256 (Horner), then eight squarings."""
    x = np.asarray(mu, np.float64) / 256.0
    e = np.ones_like(x)
    for i in range(24, 0, -1):
        t = e * x
        t = t / float(i)
        e = 1.0 - t
    for _ in range(8):
        e = e * e
    return e


def poisson_inversion(mu: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Smallest k with u <= F(k) for Poisson(mu), F built by p_k = p_{k-1} mu / k
    in float64; stops at POISSON_KCAP."""
    mu = np.asarray(mu, np.float64)
    u = np.asarray(u, np.float64)
    p = exp_neg(mu)
    F = p.copy()
    k = np.zeros(mu.shape, np.int64)
    live = u > F
    while live.any():
        kk = k[live] + 1
        pp = p[live] * mu[live]
        pp = pp / kk.astype(np.float64)
        FF = F[live] + pp
        k[live] = kk
        p[live] = pp
        F[live] = FF
        idx = np.flatnonzero(live)
        live[idx] = (u[idx] > FF) & (kk < POISSON_KCAP)
    return k


def poisson(lam: np.ndarray, pix: np.ndarray, frame: int, key) -> np.ndarray:
    """Poisson(lam) per pixel (float64): lam split into m = ceil(lam / 256)
    equal parts, one inversion each (part j uses counter block j), summed;
    lam <= 0 gives 0, lam > 2^24 or non-finite gives NaN."""
    lam = np.asarray(lam, np.float64)
    bad = ~(lam <= MAX_LAM)
    ok = np.where(bad, 0.0, lam)
    out = np.zeros(lam.shape, np.int64)
    m = np.where(ok > 0, np.ceil(ok / POISSON_CHUNK), 0).astype(np.int64)
    mu = np.where(m > 0, ok / np.maximum(m, 1), 0.0)
    for j in range(int(m.max()) if m.size else 0):
        sel = m > j
        w = philox4x64(pix[sel], frame, P_PHOTON, j, key[0], key[1])[0]
        out[sel] += poisson_inversion(mu[sel], uniform(w))
    res = out.astype(np.float64)
    res[bad] = np.nan
    return res


def gamma_mt(n: np.ndarray, pix: np.ndarray, frame: int, key) -> np.ndarray:
    """Gamma(n, 1) for shapes n >= 1 (Marsaglia-Tsang); attempt i uses
    counter block i: words 0, 1 -> normal x, word 2 -> uniform u."""
    n = np.asarray(n, np.float64)
    d = n - 1.0 / 3.0
    c = 1.0 / sqrt_basic(9.0 * d)
    out = d.copy()
    live = np.ones(n.shape, bool)
    for i in range(GAMMA_TRIES):
        if not live.any():
            break
        idx = np.flatnonzero(live)
        w = philox4x64(pix[idx], frame, P_EXCESS, i, key[0], key[1])
        x = box_muller(w[0], w[1])
        u = uniform(w[2])
        v = 1.0 + c[idx] * x
        ok = v > 0.0
        v3 = np.where(ok, v * v * v, 1.0)
        with np.errstate(divide="ignore"):
            lhs = np.where(u > 0.0, log_basic(np.where(u > 0.0, u, 1.0)), -np.inf)
            acc = ok & (lhs < 0.5 * x * x + d[idx] - d[idx] * v3 + d[idx] * log_basic(v3))
        out[idx[acc]] = d[idx[acc]] * v3[acc]
        live[idx[acc]] = False
    return out


# ------------------------------------------------------------- detector ---

def _ratio(rebin) -> tuple:
    r = Fraction(rebin)
    return r.numerator, r.denominator


def pixel_spans(n_det: int, num: int, den: int):
    """Per detector pixel p along one axis: the transform pixels y it covers
    (relative to the detector square) and their overlap lengths in units of
    1/den pixel.  Pixel p spans [p num / den, (p + 1) num / den)."""
    out = []
    for p in range(n_det):
        lo, hi = p * num, (p + 1) * num                 # in 1/den pixel
        ys = list(range(lo // den, -(-hi // den)))
        ov = [min((y + 1) * den, hi) - max(y * den, lo) for y in ys]
        out.append((ys, ov))
    return out


def expected_electrons(I: np.ndarray, n_det: int, rebin, electrons: float) -> np.ndarray:
    """lam [n_det][n_det] over the central (n_det rebin) square of the float32
    intensity I [N][N], rebin = transform pixels per detector pixel (an
    integer or a fraction num/den; the square must be whole pixels).  Each
    detector pixel sums, in float64 and row-major order over the transform
    pixels it overlaps, w * I with w = (overlap_y overlap_x) / den^2 (one
    division of integers: the area fraction), then multiplies by electrons.
    For an integer rebin every w is 1 and this is the plain block sum."""
    num, den = _ratio(rebin)
    N = I.shape[-1]
    if (n_det * num) % den:
        raise ValueError("the detector square must be whole transform pixels")
    w = n_det * num // den
    off = (N - w) // 2
    win = np.asarray(I[off:off + w, off:off + w], np.float32).astype(np.float64)
    spans = pixel_spans(n_det, num, den)
    K = max(len(ys) for ys, _ in spans)
    # per axis: index, overlap and presence of the k-th covered pixel of each detector pixel
    idx = np.zeros((n_det, K), np.int64)
    ovl = np.zeros((n_det, K), np.int64)
    has = np.zeros((n_det, K), bool)
    for p, (ys, ov) in enumerate(spans):
        idx[p, :len(ys)] = ys
        ovl[p, :len(ys)] = ov
        has[p, :len(ys)] = True
    s = np.zeros((n_det, n_det), np.float64)
    dd = float(den * den)
    for a in range(K):                       # row-major over the covered pixels
        for b in range(K):
            wgt = (ovl[:, a, None] * ovl[None, :, b]).astype(np.float64) / dd
            val = wgt * win[idx[:, a, None], idx[None, :, b]]
            s = np.where(has[:, a, None] & has[None, :, b], s + val, s)
    return s * float(electrons)


def detector_frame(I: np.ndarray, n_det: int, rebin, electrons: float, flags: int, readout_e: float,
                   seed: int, frame: int) -> np.ndarray:
    """Detector pixels [n_det][n_det] (electrons, float64) of one frame of
    normalised intensity I [N][N] (float32); `frame` is the global frame
    index that keys the random numbers."""
    if (flags & EXCESS) and not (flags & PHOTON):
        raise ValueError("excess noise needs photon noise")
    key = (int(seed) & ((1 << 64) - 1), 0)
    lam = expected_electrons(I, n_det, rebin, electrons).ravel()
    pix = np.arange(n_det * n_det, dtype=np.uint64)
    if flags & PHOTON:
        val = poisson(lam, pix, frame, key)
        if flags & EXCESS:
            pos = val > 0
            val[pos] = gamma_mt(val[pos], pix[pos], frame, key)
    else:
        val = lam.copy()
    if flags & READOUT:
        w = philox4x64(pix, frame, P_READOUT, 0, key[0], key[1])
        val = val + float(readout_e) * box_muller(w[0], w[1])
    return val.reshape(n_det, n_det)


def detector(I: np.ndarray, n_det: int, rebin, electrons: float, flags: int, readout_e: float, seed: int,
             frame0: int = 0) -> np.ndarray:
    """detector_frame over frames I [F][N][N]; frame f uses index frame0 + f."""
    return np.stack([detector_frame(I[f], n_det, rebin, electrons, flags, readout_e, seed, frame0 + f)
                     for f in range(I.shape[0])])


# ---------------------------------------------------------- detector slopes --

def detector_geometry(s, n_det: int, rebin):
    """(image origins in detector pixels, image size, detector pixels per
    subaperture) for sensor s read out on an n_det detector whose pixels are
    rebin (integer or fraction) transform pixels wide; raises if the pupil
    images do not fall on whole detector pixels tiled by the subapertures."""
    from . import pwfs as O
    num, den = _ratio(rebin)
    N, D = s.n_fft, s.n_pupil
    if (n_det * num) % den or (D * den) % num:
        raise ValueError("detector does not tile the pupil images")
    off2 = N - n_det * num // den
    img = D * den // num
    if off2 < 0 or off2 % 2 or img % s.n_subap:
        raise ValueError("detector does not tile the pupil images")
    off = off2 // 2
    org = []
    for r0, c0 in O.image_origins(s):
        if ((r0 - off) * den) % num or ((c0 - off) * den) % num or r0 < off or c0 < off:
            raise ValueError("pupil image not aligned with detector pixels")
        org.append(((r0 - off) * den // num, (c0 - off) * den // num))
    return org, img, img // s.n_subap


def detector_quadrants(P: np.ndarray, s, n_det: int, rebin) -> np.ndarray:
    """Q [F][4][n][n]: the four pupil images of detector frames P [F][n_det][n_det]
    summed over b_det x b_det blocks."""
    org, Dd, b = detector_geometry(s, n_det, rebin)
    P = np.asarray(P, np.float64)
    n = s.n_subap
    Q = np.zeros((P.shape[0], 4, n, n))
    for q, (r0, c0) in enumerate(org):
        Q[:, q] = P[:, r0:r0 + Dd, c0:c0 + Dd].reshape(P.shape[0], n, b, n, b).sum(axis=(2, 4))
    return Q


def detector_slopes(P: np.ndarray, s, n_det: int, rebin):
    """(slopes [F][2][n][n], flux [F]) of detector frames: the sensor's slope
    definition on detector pixels, minus the raw slopes of the noise-free
    detector frame of a flat wavefront (when reference subtraction is on)."""
    from . import pwfs as O
    valid = O.valid_subapertures(s)
    local = bool(s.flags & O.FLAG_LOCAL_NORM)
    sl, flux = O.raw_slopes(detector_quadrants(P, s, n_det, rebin), valid, local)
    if s.flags & O.FLAG_REF_SLOPES:
        I0 = O.forward(np.zeros((1, s.n_pupil, s.n_pupil)), s).astype(np.float32)
        P0 = detector(I0, n_det, rebin, 1.0, 0, 0.0, 0)
        ref = O.raw_slopes(detector_quadrants(P0, s, n_det, rebin), valid, local)[0][0]
        sl = sl - ref[None]
        sl[:, :, ~valid] = 0.0
    return sl, flux
