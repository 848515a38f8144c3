"""Checks of the synthetic inputs: the impulse-response band holds the
derivative-of-Gaussian pulse at the signed semicircle delay, the phantom is
nonnegative and seeded, and the configurations have the stated sizes."""
import math

import numpy as np
import pytest

import synth


def test_pulse_unit_peak_and_band_truncation():
    s = synth.pulse_sigma_s()
    u = np.linspace(-10 * s, 10 * s, 200001)
    g = synth.pulse(u)
    assert abs(np.abs(g).max() - 1.0) < 1e-6
    tail = np.abs(g[np.abs(u) > synth.BAND_HALF_SIGMAS * s]).max()
    assert tail < 2e-7
    # spectrum of the pulse peaks at the centre frequency
    n = 1 << 16
    dt = s / 50
    tt = (np.arange(n) - n // 2) * dt
    spec = np.abs(np.fft.rfft(synth.pulse(tt)))
    freq = np.fft.rfftfreq(n, dt)
    assert abs(freq[np.argmax(spec)] - synth.F_CENTER_HZ) < 0.02 * synth.F_CENTER_HZ


def test_sir_band_is_pulse_at_signed_delay():
    nz, f, nt = 16, 7, 64
    t0, taps = synth.sir_table(nz, f, nt)
    R = (f - 1) // 2
    assert t0.shape == (nz, f, f) and taps.shape == (nz, f, f, synth.SIR_WIDTH)
    for (iz, jdy, jdx) in [(0, 3, 3), (7, 0, 6), (8, 1, 2), (15, 6, 6)]:
        dy, dx = jdy - R, jdx - R
        tau = synth.delay_s(np.float64(dx), np.float64(dy), np.float64(iz), nz, nt)
        zf = (nz - 1) / 2
        # above the focal plane the delay is earlier than the focal time, below it later
        assert (tau < (nt // 2) * synth.DT_S) == (iz < zf)
        sig = synth.beam_sigma_vox(np.float64(iz), nz, f)
        w = math.exp(-(dx * dx + dy * dy) / (2 * sig * sig))
        for j in range(synth.SIR_WIDTH):
            u = (t0[iz, jdy, jdx] + j) * synth.DT_S - tau
            ref = w * synth.pulse(u) if abs(u) <= 6 * synth.pulse_sigma_s() else 0.0
            assert abs(taps[iz, jdy, jdx, j] - ref) <= 1e-6 * max(1e-30, abs(ref)) + 1e-30
    # number of nonzero taps per column: 9 or 10 (6 s = 4.77 samples each side)
    nnz = (taps != 0).sum(axis=-1)
    assert nnz.min() >= 9 and nnz.max() <= 10
    # beam symmetric in dx, dy: dx -> -dx gives the same column
    np.testing.assert_array_equal(taps, taps[:, :, ::-1, :])
    np.testing.assert_array_equal(t0, t0[:, ::-1, :])


def test_beam_width_grows_linearly_from_focus():
    nz, f = 64, 31
    s = synth.beam_sigma_vox(np.arange(nz, dtype=np.float64), nz, f)
    assert abs(s.min() - (1.0 + 6.5 * 0.5 / 31.5)) < 1e-12
    assert abs(s[0] - 7.5) < 1e-12 and abs(s[-1] - 7.5) < 1e-12


def test_phantom_nonnegative_and_seeded():
    c1 = synth.phantom(synth.C1)
    c2 = synth.phantom(synth.C1)
    assert c1.shape == synth.C1.c_shape and c1.dtype == np.float32
    assert c1.min() >= 0 and c1.max() > 0.4
    np.testing.assert_array_equal(c1, c2)


def test_config_sizes():
    assert synth.C2.c_shape == (3, 128, 128, 64) and synth.C2.y_shape == (32, 128, 128, 256)
    assert synth.C5.r == 25 and synth.C3.r == 20
    for i in range(16):
        c = synth.c4_instance(i)
        assert 64 <= c.nx <= 192 and 48 <= c.nz <= 96 and 16 <= c.n_pulses <= 48
        assert c.n_species in (2, 3) and c.nt % 32 == 0 and 256 <= c.nt <= 384


def test_factorised_inputs():
    """Inputs of the factorised operator: the spatial response image is the
    banded table's beam weight (1 on the axis, symmetric in dx and dy), the
    impulse response is the pulse sampled at dt with its zero lag at the
    origin (odd, zero at lag 0, within its 6 s support), and the radius step
    is c0 dt / pitch."""
    nz, f = 16, 7
    spr = synth.spr_table(nz, f)
    R = (f - 1) // 2
    assert spr.shape == (nz, f, f) and spr.dtype == np.float32
    np.testing.assert_array_equal(spr[:, R, R], np.ones(nz, np.float32))
    np.testing.assert_array_equal(spr, spr[:, ::-1, :])
    np.testing.assert_array_equal(spr, spr[:, :, ::-1])
    np.testing.assert_array_equal(spr, np.transpose(spr, (0, 2, 1)))
    s = synth.beam_sigma_vox(np.arange(nz, dtype=np.float64), nz, f)
    np.testing.assert_allclose(spr[:, R, R + 2], np.exp(-4.0 / (2 * s * s)), rtol=1e-6)
    v, o = synth.eir_taps()
    assert v.dtype == np.float32 and len(v) == 2 * o + 1
    assert v[o] == 0.0
    np.testing.assert_array_equal(v[o + 1:], -v[o - 1::-1])
    lags = (np.arange(len(v)) - o) * synth.DT_S
    assert np.abs(lags).max() <= synth.BAND_HALF_SIGMAS * synth.pulse_sigma_s()
    np.testing.assert_allclose(v, synth.pulse(lags).astype(np.float32))
    dr, zf, tf = synth.shell_geometry(64, 256)
    assert dr == pytest.approx(synth.C0_M_S * synth.DT_S / synth.PITCH_M) and zf == 31.5 and tf == 128
