"""Checks of the seeded input generator (CPU only)."""

import numpy as np

import synth


def test_tiny_raster_hits_exactly_64_per_pixel():
    p = synth.make_config("tiny", n_rhs=1)
    assert p.n_samples == 4 * 65536
    h = np.bincount(p.pix, minlength=p.n_pix_global)
    assert h.min() == 64 and h.max() == 64
    assert p.lam_max == 1024 and len(p.blk_start) == 4


def test_reproducible_bytes():
    a = synth.make_ground(n_dets=3, samples_per_det=4096, interval=1024, side=16, lam=64)
    b = synth.make_ground(n_dets=3, samples_per_det=4096, interval=1024, side=16, lam=64)
    for k in ("pix", "wq", "wu", "d"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert all(np.array_equal(x, y) for x, y in zip(a.bands, b.bands))


def test_ground_blocks_tile_each_detector():
    p = synth.make_ground(n_dets=4, samples_per_det=10000, interval=3000, side=16, lam=32)
    assert np.all(p.blk_len > 0)
    cov = np.zeros(p.n_samples, int)
    for s, L in zip(p.blk_start, p.blk_len):
        cov[s:s + L] += 1
    assert np.all(cov == 1)
    for s, L in zip(p.blk_start, p.blk_len):  # never across a detector boundary
        det = np.searchsorted(p.det_offset, s, side="right") - 1
        assert s + L <= p.det_offset[det + 1]


def test_noise_psd_matches_model():
    # averaged periodogram of the drawn noise against P(f) = sigma^2 (1 + f_knee / f)
    n, m, fs, fk = 4096, 64, 100.0, 1.0
    g = np.random.Generator(np.random.PCG64(5))
    x = synth.problems._noise_batch(g, m, n, fs, 1.0, fk, -1.0)
    f = np.fft.rfftfreq(n, 1 / fs)
    per = np.mean(np.abs(np.fft.rfft(x, axis=1)) ** 2, axis=0) / n
    sel = (f > 5.0) & (f < 45.0)
    ratio = per[sel] / synth.noise_psd(f[sel], 1.0, fk)
    assert abs(ratio.mean() - 1.0) < 0.03


def test_white_band_is_delta_and_bands_have_positive_symbol():
    w = synth.inverse_noise_band(16, 100.0, sigma=2.0, fknee=0.0)
    assert abs(w[0] - 0.25) < 1e-7 and np.abs(w[1:]).max() < 1e-7
    for fk in (0.1, 1.0, 2.0):
        c = synth.inverse_noise_band(1024, 100.0, fknee=fk).astype(np.float64)
        n = 1 << 15
        h = np.zeros(n)
        h[0] = c[0]
        h[1:c.size] = c[1:]
        h[n - c.size + 1:] = c[1:][::-1]
        assert np.fft.rfft(h).real.min() > 0


def test_serving_views_are_slices_of_the_base_stream():
    base, views = synth.serving_views(cfg_id=7, n_geoms=12, dets=(2, 8), log2_samples=(12, 14),
                                      log2_lam=(4, 6), base_dets=8, base_log2=14, side=32,
                                      interval=1 << 12)
    assert base.n_samples == 8 << 14
    for v in views:
        per = v.samples_per_det
        assert 2 <= v.n_dets <= 8 and per in (1 << 12, 1 << 13, 1 << 14)
        assert v.s0 % per == 0 and v.s0 + v.n_samples <= base.n_samples
        assert v.n_samples == v.n_dets * per and v.det_offset[-1] == v.n_samples
        # every piece lies inside one base detector, so its intervals are base intervals
        assert all(((v.s0 + i * per) >> 14) == ((v.s0 + (i + 1) * per - 1) >> 14)
                   for i in range(v.n_dets))
        assert np.array_equal(np.diff(v.det_offset), np.full(v.n_dets, per))
        assert v.blk_len.sum() == v.n_samples and np.all(v.blk_start % (1 << 12) == 0)
        assert len(v.bands) == v.n_dets and v.blk_band.max() == v.n_dets - 1
        assert all(len(b) == v.lam + 1 for b in v.bands) and v.lam in (16, 32, 64)
