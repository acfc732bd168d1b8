"""Seeded synthetic inputs shaped like the paper's ground-based and satellite-like workloads.

Every random stream is ``PCG64(SeedSequence([MASTER_SEED, cfg_id, stream, *keys]))`` so any array
can be regenerated independently of the others.  Streams:

    1 detector pixel offsets      2 per-sample / per-detector polarisation angles
    3 knee frequencies            4 noise, keyed by (detector, interval, rhs)
    5 sky maps, keyed by rhs      6 per-sweep boresight rotation
    7 flagged samples             8 random block layouts (small random problems)
    9 serving workload: geometry sizes and the request trace

Data model (Eq. dataModelSingleSlot / Eq. dataModelHwp): d_t = I_p + cos(2psi_t) Q_p +
sin(2psi_t) U_p + n_t, with p = p(t).  The per-sample weights are stored as FP32 and *define* the
problem: the sky signal is formed from the stored FP32 weights promoted to FP64.

Noise (Eq. noisepowermodel with f0 = 0): P(f) = sigma^2 (1 + (f / f_knee)^alpha), alpha = -1.
Each (detector, interval) gets an independent Gaussian realisation drawn in the frequency domain
on twice the interval length and cropped; the DC amplitude is zero.

Inverse-noise band (Eq. MADCAP and the weight recipe of the ML method section): 1/P sampled on a
grid of ``max(2^20, 16 lambda)`` frequencies (1/P(0) := 0), inverse FFT, Gaussian window of
standard deviation lambda/2, cut at |lag| <= lambda, stored as FP32 coefficients c_0..c_lambda.
The band is an input of the solver, like the scan.
"""

from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np
import scipy.fft as sfft

MASTER_SEED = 211203370

_S_OFFSETS, _S_PSI, _S_FKNEE, _S_NOISE, _S_SKY, _S_RHO, _S_FLAGS, _S_LAYOUT, _S_TRACE = range(1, 10)


def _rng(cfg_id: int, stream: int, *keys: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([MASTER_SEED, int(cfg_id), int(stream), *map(int, keys)]))
    )


def _workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


@dataclasses.dataclass
class Problem:
    """A map-making problem: pointing, block-Toeplitz inverse-noise weights and data.

    Arrays (time-ordered arrays have ``n_samples`` entries, detector-major):
      pix        int32   global pixel id per sample, -1 = flagged (no sky response)
      wq, wu     float32 polarisation weights cos(2psi), sin(2psi) (the I weight is 1)
      d          float32 [n_rhs, n_samples] time-ordered data
      blk_start, blk_len  int64 [n_blocks]  stationary intervals (never cross detectors)
      blk_band   int32 [n_blocks]           index into ``bands``
      bands      list of float32 arrays, band b holds c_0..c_lambda_b
      det_offset int64 [n_dets + 1]         first sample of each detector
      m_true     float64 [n_rhs, n_pix_global, 3] or None
    """

    name: str
    pix: np.ndarray
    wq: np.ndarray
    wu: np.ndarray
    d: np.ndarray
    n_pix_global: int
    blk_start: np.ndarray
    blk_len: np.ndarray
    blk_band: np.ndarray
    bands: list
    det_offset: np.ndarray
    m_true: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_rhs(self) -> int:
        return int(self.d.shape[0])

    @property
    def lam_max(self) -> int:
        return max((len(b) - 1 for b in self.bands), default=0)

    def band_table(self):
        """Concatenated band coefficients: (ncoef int32, offset int64, coef float32)."""
        ncoef = np.array([len(b) for b in self.bands], dtype=np.int32)
        offset = np.zeros(len(self.bands), dtype=np.int64)
        if len(self.bands) > 1:
            offset[1:] = np.cumsum(ncoef[:-1])
        coef = (np.concatenate(self.bands).astype(np.float32) if self.bands
                else np.zeros(0, np.float32))
        return ncoef, offset, coef


# --------------------------------------------------------------------------------------------
# Noise model and inverse-noise band
# --------------------------------------------------------------------------------------------

def noise_psd(f, sigma=1.0, fknee=1.0, alpha=-1.0):
    """P(f) = sigma^2 (1 + (f/f_knee)^alpha); f_knee = 0 means white noise."""
    f = np.asarray(f, dtype=np.float64)
    if fknee <= 0.0:
        return np.full_like(f, sigma * sigma)
    with np.errstate(divide="ignore"):
        return sigma * sigma * (1.0 + np.power(f / fknee, alpha))


def inverse_noise_band(lam, fsample, sigma=1.0, fknee=1.0, alpha=-1.0, n_grid=None):
    """First row c_0..c_lam of the banded inverse-noise Toeplitz block, as float32."""
    lam = int(lam)
    if n_grid is None:
        n_grid = max(1 << 20, 1 << int(math.ceil(math.log2(max(16 * lam, 2)))))
    f = np.fft.rfftfreq(n_grid, d=1.0 / fsample)
    inv = np.zeros_like(f)
    p = noise_psd(f[1:], sigma, fknee, alpha)
    inv[1:] = 1.0 / p
    if fknee <= 0.0:
        inv[0] = 1.0 / (sigma * sigma)
    c = sfft.irfft(inv, n_grid)[: lam + 1]
    if lam > 0:
        k = np.arange(lam + 1, dtype=np.float64)
        c = c * np.exp(-2.0 * k * k / float(lam * lam))
    return c.astype(np.float32)


def _noise_batch(rng, n_int, length, fsample, sigma, fknee, alpha, workers=None):
    """``n_int`` independent realisations of ``length`` samples (drawn on 2*length, cropped)."""
    m = 2 * length
    f = np.fft.rfftfreq(m, d=1.0 / fsample)
    p = noise_psd(f, sigma, fknee, alpha)
    p[0] = 0.0
    amp = np.sqrt(m * p / 2.0)
    amp[-1] = np.sqrt(m * p[-1])  # Nyquist bin is real
    g = rng.standard_normal((n_int, f.size)) + 1j * rng.standard_normal((n_int, f.size))
    g[:, -1] = g[:, -1].real
    spec = g * amp
    return sfft.irfft(spec, m, axis=1, workers=workers or _workers())[:, :length]


# --------------------------------------------------------------------------------------------
# Assembly helpers
# --------------------------------------------------------------------------------------------

def _blocks_for(det_offset, interval, band_of_det):
    starts, lens, bands = [], [], []
    for det in range(len(det_offset) - 1):
        s0, s1 = int(det_offset[det]), int(det_offset[det + 1])
        if interval <= 0:
            continue
        for s in range(s0, s1, interval):
            starts.append(s)
            lens.append(min(interval, s1 - s))
            bands.append(band_of_det[det])
    return (np.asarray(starts, np.int64), np.asarray(lens, np.int64), np.asarray(bands, np.int32))


def _sky(cfg_id, n_rhs, n_pix):
    return np.stack([_rng(cfg_id, _S_SKY, j).standard_normal((n_pix, 3)) for j in range(n_rhs)])


def _fill_data(d, pix, wq, wu, m_true, cfg_id, det_offset, interval, fsample, sigma, fknees,
               alpha, noise):
    """d[j] = P m_j + n_j per detector, in FP64, stored FP32 (detectors in parallel threads;
    every detector draws from its own streams, so the bytes do not depend on the threading)."""
    n_rhs = d.shape[0]

    def one(det):
        s0, s1 = int(det_offset[det]), int(det_offset[det + 1])
        p = pix[s0:s1]
        ok = p >= 0
        pp = np.where(ok, p, 0)
        q = wq[s0:s1].astype(np.float64)
        u = wu[s0:s1].astype(np.float64)
        for j in range(n_rhs):
            m = m_true[j]
            sig = m[pp, 0] + q * m[pp, 1] + u * m[pp, 2]
            sig[~ok] = 0.0
            if noise != "none":
                L = interval if interval > 0 else (s1 - s0)
                n_int = (s1 - s0 + L - 1) // L
                fk = 0.0 if noise == "white" else float(fknees[det])
                for i in range(n_int):
                    a, b = i * L, min((i + 1) * L, s1 - s0)
                    g = _rng(cfg_id, _S_NOISE, det, i, j)
                    sig[a:b] += _noise_batch(g, 1, b - a, fsample, sigma, fk, alpha, workers=1)[0]
            d[j, s0:s1] = sig.astype(np.float32)

    n_dets = len(det_offset) - 1
    if n_dets <= 1 or det_offset[-1] < (1 << 16):
        for det in range(n_dets):
            one(det)
        return
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(one, range(n_dets)))


def _bands_for(lam, fsample, sigma, fknees, alpha, noise):
    return [inverse_noise_band(lam, fsample, sigma, 0.0 if noise == "white" else float(f), alpha)
            for f in fknees]


# --------------------------------------------------------------------------------------------
# Scans
# --------------------------------------------------------------------------------------------

def make_raster(cfg_id=0, n_dets=4, side=64, dwell=16, lam=1024, fknee=1.0, fsample=100.0,
                sigma=1.0, alpha=-1.0, n_rhs=1, noise="1/f", repeats=1, name="raster"):
    """Boustrophedon raster over a side x side patch, one full raster per repeat per detector.

    Each detector gets a toroidal pixel offset (dx, dy) ~ U{0..side-1}^2; psi ~ U[0, pi) i.i.d.
    per sample; one stationary interval per detector.  With ``repeats = 1`` every pixel is hit
    exactly ``n_dets * dwell`` times.
    """
    per_det = side * side * dwell * repeats
    n_s = n_dets * per_det
    det_offset = np.arange(n_dets + 1, dtype=np.int64) * per_det
    rows = np.repeat(np.arange(side), side * dwell)
    cols = np.tile(np.repeat(np.arange(side), dwell), side)
    odd = (rows % 2) == 1
    cols = np.where(odd, side - 1 - cols, cols)
    rows = np.tile(rows, repeats)
    cols = np.tile(cols, repeats)
    off = _rng(cfg_id, _S_OFFSETS).integers(0, side, size=(n_dets, 2))
    pix = np.empty(n_s, np.int32)
    for det in range(n_dets):
        r = (rows + off[det, 1]) % side
        c = (cols + off[det, 0]) % side
        pix[det * per_det:(det + 1) * per_det] = (r * side + c).astype(np.int32)
    psi = _rng(cfg_id, _S_PSI).uniform(0.0, np.pi, size=n_s)
    wq = np.cos(2.0 * psi).astype(np.float32)
    wu = np.sin(2.0 * psi).astype(np.float32)
    fknees = np.full(n_dets, fknee if noise == "1/f" else 0.0)
    bands = _bands_for(lam, fsample, sigma, fknees, alpha, noise)
    blk = _blocks_for(det_offset, per_det, list(range(n_dets)))
    n_pix = side * side
    m_true = _sky(cfg_id, n_rhs, n_pix)
    d = np.empty((n_rhs, n_s), np.float32)
    _fill_data(d, pix, wq, wu, m_true, cfg_id, det_offset, per_det, fsample, sigma, fknees,
               alpha, noise)
    return Problem(name, pix, wq, wu, d, n_pix, *blk, bands, det_offset, m_true,
                   dict(cfg_id=cfg_id, kind="raster", side=side, dwell=dwell, lam=lam,
                        fknee=fknee, fsample=fsample, noise=noise))


def make_ground(cfg_id=1, n_dets=256, samples_per_det=1 << 20, interval=1 << 16, side=512,
                dwell=16, lam=8192, fknee_range=(0.1, 2.0), fsample=100.0, sigma=1.0, alpha=-1.0,
                n_rhs=1, noise="1/f", row_step=None, flag_frac=0.0, name="ground"):
    """Constant-elevation azimuth sweeps over a side x side patch.

    A sweep is a triangle-wave pass across the patch columns with ``dwell`` samples per pixel
    (side*dwell samples); the row advances ``row_step`` per sweep (sky drift).  Detector focal
    plane offsets (dx, dy) ~ U{0..side-1}^2 with wrap.  psi = psi_det + rho_sweep, with psi_det
    ~ U[0, pi) per detector and rho_sweep ~ U[0, pi) common to all detectors of a sweep.  f_knee
    ~ U[fknee_range] per detector; one band per detector shared by its intervals.
    """
    sweep = side * dwell
    if row_step is None:
        row_step = max(1, (side * side * dwell) // samples_per_det)
    n_s = n_dets * samples_per_det
    det_offset = np.arange(n_dets + 1, dtype=np.int64) * samples_per_det
    t = np.arange(samples_per_det)
    j = t // sweep
    within = (t % sweep) // dwell
    col0 = np.where(j % 2 == 0, within, side - 1 - within)
    n_sweeps = int(j[-1]) + 1
    rho = _rng(cfg_id, _S_RHO).uniform(0.0, np.pi, size=n_sweeps)
    off = _rng(cfg_id, _S_OFFSETS).integers(0, side, size=(n_dets, 2))
    psi_det = _rng(cfg_id, _S_PSI).uniform(0.0, np.pi, size=n_dets)
    pix = np.empty(n_s, np.int32)
    wq = np.empty(n_s, np.float32)
    wu = np.empty(n_s, np.float32)
    rho_t = rho[j]
    for det in range(n_dets):
        sl = slice(det * samples_per_det, (det + 1) * samples_per_det)
        r = (row_step * j + off[det, 1]) % side
        c = (col0 + off[det, 0]) % side
        pix[sl] = (r * side + c).astype(np.int32)
        psi = psi_det[det] + rho_t
        wq[sl] = np.cos(2.0 * psi)
        wu[sl] = np.sin(2.0 * psi)
    if flag_frac > 0.0:
        fl = _rng(cfg_id, _S_FLAGS).random(n_s) < flag_frac
        pix[fl] = -1
    if noise == "1/f":
        fknees = _rng(cfg_id, _S_FKNEE).uniform(*fknee_range, size=n_dets)
    else:
        fknees = np.zeros(n_dets)
    bands = _bands_for(lam, fsample, sigma, fknees, alpha, noise)
    blk = _blocks_for(det_offset, interval, list(range(n_dets)))
    n_pix = side * side
    m_true = _sky(cfg_id, n_rhs, n_pix)
    d = np.empty((n_rhs, n_s), np.float32)
    _fill_data(d, pix, wq, wu, m_true, cfg_id, det_offset, interval, fsample, sigma, fknees,
               alpha, noise)
    return Problem(name, pix, wq, wu, d, n_pix, *blk, bands, det_offset, m_true,
                   dict(cfg_id=cfg_id, kind="ground", side=side, dwell=dwell, lam=lam,
                        fsample=fsample, noise=noise, row_step=row_step, interval=interval,
                        fknees=fknees.tolist()))


def _pixel_of(vec, n_rings, n_phi):
    """Equal-area pixel: n_rings rings uniform in z = cos(theta), n_phi pixels in phi."""
    z = np.clip(vec[..., 2], -1.0, 1.0)
    ring = np.minimum(((1.0 - z) * 0.5 * n_rings).astype(np.int64), n_rings - 1)
    phi = np.arctan2(vec[..., 1], vec[..., 0])
    iphi = ((phi / (2.0 * np.pi)) * n_phi).astype(np.int64) % n_phi
    return ring * n_phi + iphi


def make_satellite(cfg_id=2, n_dets=32, samples_per_det=1 << 23, interval=1 << 20, n_rings=768,
                   n_phi=1024, lam=1 << 15, fknee=0.05, fsample=20.0, sigma=1.0, alpha=-1.0,
                   spin_period_s=1200.0, prec_period_s=12000.0, spin_angle_deg=50.0,
                   prec_angle_deg=45.0, hwp_hz=0.75, n_rhs=1, noise="1/f", chunk=1 << 22,
                   name="satellite"):
    """Spinning, precessing satellite with an ideal HWP (Eq. dataModelHwp).

    The anti-sun axis makes one full turn over ``samples_per_det`` samples, so one detector's
    stream covers the sky.  Detector offsets: spin angle +/- 2 deg and a spin phase in [0, 2pi).
    Weights cos(2 psi_det + 4 omega t), sin(...), psi_det ~ U[0, pi).
    """
    n_s = n_dets * samples_per_det
    det_offset = np.arange(n_dets + 1, dtype=np.int64) * samples_per_det
    g = _rng(cfg_id, _S_OFFSETS)
    dbeta = np.deg2rad(g.uniform(-2.0, 2.0, size=n_dets))
    dphase = g.uniform(0.0, 2.0 * np.pi, size=n_dets)
    psi_det = _rng(cfg_id, _S_PSI).uniform(0.0, np.pi, size=n_dets)
    pix = np.empty(n_s, np.int32)
    wq = np.empty(n_s, np.float32)
    wu = np.empty(n_s, np.float32)
    a = np.deg2rad(prec_angle_deg)
    year = samples_per_det / fsample

    def one(det):
        b = np.deg2rad(spin_angle_deg) + dbeta[det]
        for s0 in range(0, samples_per_det, chunk):
            s1 = min(samples_per_det, s0 + chunk)
            t = np.arange(s0, s1, dtype=np.float64) / fsample
            th_sun = 2.0 * np.pi * t / year
            th_prec = 2.0 * np.pi * t / prec_period_s
            th_spin = 2.0 * np.pi * t / spin_period_s + dphase[det]
            # boresight in the spin frame, then tilt by the precession angle, then rotate with
            # the precession phase about the anti-sun axis (x), then the anti-sun axis about z
            v0 = np.cos(b)
            v1 = np.sin(b) * np.cos(th_spin)
            v2 = np.sin(b) * np.sin(th_spin)
            x1 = np.cos(a) * v0 - np.sin(a) * v1
            y1 = np.sin(a) * v0 + np.cos(a) * v1
            z1 = v2
            cp, sp = np.cos(th_prec), np.sin(th_prec)
            y2 = cp * y1 - sp * z1
            z2 = sp * y1 + cp * z1
            cs, ss = np.cos(th_sun), np.sin(th_sun)
            vec = np.stack([cs * x1 - ss * y2, ss * x1 + cs * y2, z2], axis=-1)
            sl = slice(det * samples_per_det + s0, det * samples_per_det + s1)
            pix[sl] = _pixel_of(vec, n_rings, n_phi).astype(np.int32)
            ang = 2.0 * psi_det[det] + 4.0 * (2.0 * np.pi * hwp_hz) * t
            wq[sl] = np.cos(ang)
            wu[sl] = np.sin(ang)

    if n_dets == 1:
        one(0)
    else:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=_workers()) as ex:
            list(ex.map(one, range(n_dets)))
    fknees = np.full(n_dets, fknee if noise == "1/f" else 0.0)
    bands = _bands_for(lam, fsample, sigma, fknees, alpha, noise)
    blk = _blocks_for(det_offset, interval, list(range(n_dets)))
    n_pix = n_rings * n_phi
    m_true = _sky(cfg_id, n_rhs, n_pix)
    d = np.empty((n_rhs, n_s), np.float32)
    _fill_data(d, pix, wq, wu, m_true, cfg_id, det_offset, interval, fsample, sigma, fknees,
               alpha, noise)
    return Problem(name, pix, wq, wu, d, n_pix, *blk, bands, det_offset, m_true,
                   dict(cfg_id=cfg_id, kind="satellite", lam=lam, fsample=fsample,
                        noise=noise, interval=interval, n_rings=n_rings, n_phi=n_phi))


def make_random_small(seed=0, n_samples=3000, n_pix=40, n_dets=3, lam_max=16, flag_frac=0.05,
                      gap_frac=0.1, n_rhs=1, noise_sigma=1.0, dwell=4, name="random"):
    """Small random geometry for property tests: runs of equal pixels of random length, random
    psi, random block layout that leaves some samples uncovered, random bands (positive symbol
    by construction: a Gaussian-windowed Lorentzian-like decay plus a dominant diagonal)."""
    cfg = 1000 + int(seed)
    g = _rng(cfg, _S_LAYOUT)
    bounds = np.sort(g.choice(np.arange(1, n_samples), size=n_dets - 1, replace=False))
    det_offset = np.concatenate([[0], bounds, [n_samples]]).astype(np.int64)
    runs = []
    total = 0
    while total < n_samples:
        L = int(g.integers(1, 2 * dwell + 1))
        runs.append((int(g.integers(0, n_pix)), L))
        total += L
    pix = np.concatenate([np.full(L, p, np.int32) for p, L in runs])[:n_samples]
    psi = _rng(cfg, _S_PSI).uniform(0.0, np.pi, size=n_samples)
    wq = np.cos(2.0 * psi).astype(np.float32)
    wu = np.sin(2.0 * psi).astype(np.float32)
    if flag_frac > 0:
        pix[_rng(cfg, _S_FLAGS).random(n_samples) < flag_frac] = -1
    starts, lens, bands_idx = [], [], []
    n_bands = max(1, n_dets)
    for det in range(n_dets):
        s0, s1 = int(det_offset[det]), int(det_offset[det + 1])
        s = s0
        while s < s1:
            L = int(g.integers(1, max(2, (s1 - s0) // 2) + 1))
            L = min(L, s1 - s)
            if g.random() >= gap_frac:
                starts.append(s)
                lens.append(L)
                bands_idx.append(det % n_bands)
            s += L
    bands = []
    for b in range(n_bands):
        lam = int(g.integers(0, lam_max + 1))
        k = np.arange(lam + 1, dtype=np.float64)
        tail = -0.4 * np.exp(-k / max(1.0, lam / 3.0)) * np.exp(-2.0 * k * k / max(1, lam) ** 2)
        c = tail.copy()
        c[0] = 1.0 + 2.0 * np.sum(np.abs(tail[1:])) + g.uniform(0.1, 0.5)
        bands.append(c.astype(np.float32))
    m_true = _sky(cfg, n_rhs, n_pix)
    d = np.empty((n_rhs, n_samples), np.float32)
    ok = pix >= 0
    pp = np.where(ok, pix, 0)
    for j in range(n_rhs):
        m = m_true[j]
        sig = m[pp, 0] + wq.astype(np.float64) * m[pp, 1] + wu.astype(np.float64) * m[pp, 2]
        sig[~ok] = 0.0
        sig += noise_sigma * _rng(cfg, _S_NOISE, 0, 0, j).standard_normal(n_samples)
        d[j] = sig.astype(np.float32)
    return Problem(name, pix, wq, wu, d, n_pix, np.asarray(starts, np.int64),
                   np.asarray(lens, np.int64), np.asarray(bands_idx, np.int32), bands,
                   det_offset, m_true, dict(cfg_id=cfg, kind="random", seed=seed))


def make_templates(cfg_id=5, n_dets=4, samples_per_det=1 << 16, interval=1 << 14, side=32,
                   dwell=8, baseline=1000, n_poly=3, drift_sigma=5.0, sigma_range=(0.5, 2.0),
                   cover=1.0, flag_frac=0.0, n_rhs=1, name="templates"):
    """Ground-like sweeps for template map-making (Eq. dataModel with T = polynomial baselines).

    Geometry of ``make_ground``.  White noise with a detector-dependent sigma ~ U[sigma_range],
    hence diagonal weights: one band per detector with lambda = 0 and c_0 = 1 / sigma^2.
    Baselines of ``baseline`` samples tile every stationary interval (the last one of an
    interval is shorter); with ``cover < 1`` each baseline is kept with that probability and the
    others stay uncovered.  Every kept baseline carries a drift: a polynomial of degree
    < n_poly in the sample index with Gaussian coefficients of scale drift_sigma (the
    low-frequency contribution that the templates describe).  Returns the Problem with
    ``meta["base_start"]``, ``meta["base_len"]`` (int64) and ``meta["n_poly"]``.
    """
    geo = make_ground(cfg_id=cfg_id, n_dets=n_dets, samples_per_det=samples_per_det,
                      interval=interval, side=side, dwell=dwell, lam=0, noise="white",
                      flag_frac=flag_frac, n_rhs=n_rhs, name=name)
    g = _rng(cfg_id, _S_LAYOUT)
    sig = g.uniform(*sigma_range, size=n_dets)
    bands = [np.array([1.0 / (s * s)], np.float32) for s in sig]
    starts, lens = [], []
    for s0, L in zip(geo.blk_start, geo.blk_len):
        for o in range(0, int(L), baseline):
            if cover >= 1.0 or g.random() < cover:
                starts.append(int(s0) + o)
                lens.append(min(baseline, int(L) - o))
    base_start = np.asarray(starts, np.int64)
    base_len = np.asarray(lens, np.int64)
    ok = geo.pix >= 0
    pp = np.where(ok, geo.pix, 0)
    d = np.empty((n_rhs, geo.n_samples), np.float32)
    wq = geo.wq.astype(np.float64)
    wu = geo.wu.astype(np.float64)
    for j in range(n_rhs):
        m = geo.m_true[j]
        sky = np.where(ok, m[pp, 0] + wq * m[pp, 1] + wu * m[pp, 2], 0.0)
        noise = _rng(cfg_id, _S_NOISE, 0, 0, j).standard_normal(geo.n_samples)
        det = np.searchsorted(geo.det_offset, np.arange(geo.n_samples), side="right") - 1
        drift = np.zeros(geo.n_samples)
        coef = _rng(cfg_id, _S_NOISE, 1, 0, j).standard_normal((len(starts), max(1, n_poly)))
        for i, (s0, L) in enumerate(zip(starts, lens)):
            u = np.arange(L) / max(1, L) - 0.5
            drift[s0:s0 + L] = np.polynomial.polynomial.polyval(u, drift_sigma * coef[i, :n_poly])
        d[j] = (sky + sig[det] * noise + drift).astype(np.float32)
    meta = dict(geo.meta, kind="templates", base_start=base_start, base_len=base_len,
                n_poly=n_poly, sigmas=sig.tolist())
    return Problem(name, geo.pix, geo.wq, geo.wu, d, geo.n_pix_global, geo.blk_start,
                   geo.blk_len, geo.blk_band, bands, geo.det_offset, geo.m_true, meta)


# --------------------------------------------------------------------------------------------
# Named workloads (shapes of the benchmark configurations)
# --------------------------------------------------------------------------------------------

CONFIGS = {
    # 4 detectors x 65,536 samples, 64x64 raster, lambda = 1,024, f_knee = 1 Hz, f_s = 100 Hz
    "tiny": dict(kind="raster", cfg_id=0, n_dets=4, side=64, dwell=16, lam=1024, fknee=1.0,
                 fsample=100.0),
    # 256 detectors x 2^20 samples, intervals of 2^16, 512x512 patch, lambda = 8,192
    "ground": dict(kind="ground", cfg_id=1, n_dets=256, samples_per_det=1 << 20,
                   interval=1 << 16, side=512, dwell=16, lam=8192, fknee_range=(0.1, 2.0),
                   fsample=100.0),
    # 32 detectors x 2^23 samples, intervals of 2^20, 786,432 pixels, lambda = 2^15, HWP
    "satellite": dict(kind="satellite", cfg_id=2, n_dets=32, samples_per_det=1 << 23,
                      interval=1 << 20, lam=1 << 15, fknee=0.05, fsample=20.0),
    # ground geometry at 64 detectors with 64 Monte Carlo right-hand sides
    "batched": dict(kind="ground", cfg_id=3, n_dets=64, samples_per_det=1 << 20,
                    interval=1 << 16, side=512, dwell=16, lam=8192, fknee_range=(0.1, 2.0),
                    fsample=100.0, n_rhs=64),
}


def serving_pool(cfg_id=4, n_geoms=24, dets=(4, 32), log2_samples=(16, 18), sides=(32, 128),
                 log2_lam=(8, 13), n_rhs=4, interval=1 << 16):
    """Geometries of the serving workload: ground-like sweeps of uneven size, one draw per
    geometry of detectors ~ U{dets}, samples per detector 2^e with e ~ U{log2_samples}, patch
    side ~ U{sides}, half-bandwidth 2^g with g ~ U{log2_lam}; n_rhs data realizations each.
    Geometry i uses the streams of configuration 100 cfg_id + i."""
    g = _rng(cfg_id, _S_TRACE, 0)
    pool = []
    for i in range(n_geoms):
        nd = int(g.integers(dets[0], dets[1] + 1))
        e = int(g.integers(log2_samples[0], log2_samples[1] + 1))
        side = int(g.integers(sides[0], sides[1] + 1))
        lam = 1 << int(g.integers(log2_lam[0], log2_lam[1] + 1))
        pool.append(make_ground(cfg_id=100 * cfg_id + i, n_dets=nd, samples_per_det=1 << e,
                                interval=interval, side=side, dwell=16, lam=lam, n_rhs=n_rhs,
                                name=f"serving-{i}"))
    return pool


@dataclasses.dataclass
class GeometryView:
    """A serving geometry as a contiguous sample range [s0, s0 + n_samples) of a base stream:
    n_dets virtual detectors of samples_per_det samples each (pieces of the base detectors),
    stationary intervals of ``interval`` samples, its own inverse-noise bands (half-bandwidth
    lam, the knee of the base detector each piece comes from)."""

    s0: int
    n_samples: int
    n_dets: int
    samples_per_det: int
    lam: int
    n_pix_global: int
    blk_start: np.ndarray
    blk_len: np.ndarray
    blk_band: np.ndarray
    bands: list
    det_offset: np.ndarray


def serving_views(cfg_id=6, n_geoms=100, dets=(4, 128), log2_samples=(16, 21),
                  log2_lam=(8, 13), base_dets=128, base_log2=21, side=512, interval=1 << 16):
    """Geometries of the full-range serving workload (4..128 detectors x 2^16..2^21 samples,
    half-bandwidths 2^8..2^13) as views of one ground-like base stream of base_dets x
    2^base_log2 samples, so that the pointing of every geometry is a slice of one device
    buffer.  Geometry i draws detectors ~ U{dets}, samples per detector 2^e with
    e ~ U{log2_samples}, lam = 2^g with g ~ U{log2_lam}, and a start s0 (a multiple of 2^e)
    uniformly among those that fit.  Returns (base Problem with one data realisation, views)."""
    base = make_ground(cfg_id=cfg_id, n_dets=base_dets, samples_per_det=1 << base_log2,
                       interval=interval, side=side, dwell=16, lam=1 << log2_lam[1], n_rhs=1,
                       name="serving-base")
    fknees = np.asarray(base.meta["fknees"])
    g = _rng(cfg_id, _S_TRACE, 2)
    n_base = base.n_samples
    cache = {}
    views = []
    for _ in range(n_geoms):
        nd = int(g.integers(dets[0], dets[1] + 1))
        e = int(g.integers(log2_samples[0], log2_samples[1] + 1))
        lam = 1 << int(g.integers(log2_lam[0], log2_lam[1] + 1))
        per = 1 << e
        n = nd * per
        s0 = per * int(g.integers(0, (n_base - n) // per + 1))
        bands = []
        for i in range(nd):
            fk = round(float(fknees[(s0 + i * per) >> base_log2]), 1)
            key = (fk, lam)
            if key not in cache:
                cache[key] = inverse_noise_band(lam, base.meta["fsample"], 1.0, fk, -1.0)
            bands.append(cache[key])
        det_offset = np.arange(nd + 1, dtype=np.int64) * per
        bs, bl, bb = _blocks_for(det_offset, interval, list(range(nd)))
        views.append(GeometryView(s0, n, nd, per, lam, base.n_pix_global, bs, bl, bb, bands,
                                  det_offset))
    return base, views


def serving_trace(cfg_id=4, n_requests=400, n_geoms=24, zipf_s=1.1, k_range=(1, 4)):
    """Request trace: geometry index by Zipf(zipf_s) popularity over the pool, right-hand sides
    per request ~ U{k_range}, and unit-rate exponential inter-arrival gaps (Poisson arrivals;
    divide by the rate)."""
    g = _rng(cfg_id, _S_TRACE, 1)
    p = 1.0 / np.arange(1, n_geoms + 1) ** zipf_s
    p /= p.sum()
    geom = g.choice(n_geoms, size=n_requests, p=p)
    k = g.integers(k_range[0], k_range[1] + 1, size=n_requests)
    gaps = g.exponential(1.0, size=n_requests)
    return geom.astype(np.int64), k.astype(np.int64), gaps


def make_config(name, **overrides):
    spec = dict(CONFIGS[name])
    spec.update(overrides)
    kind = spec.pop("kind")
    spec.setdefault("name", name)
    if kind == "raster":
        return make_raster(**spec)
    if kind == "ground":
        return make_ground(**spec)
    if kind == "satellite":
        return make_satellite(**spec)
    raise ValueError(kind)
