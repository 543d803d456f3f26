"""Pins of the oracle's frequency-domain front ends, the paper's own forms
(Sec. 2): 1024-point blocks advancing by 512 samples; for KK (second
paragraph) the Hilbert transform as -j sgn(k) on each block's spectrum and
the 203-tap static equaliser on the 1024-point spectrum with a 512-point
inverse transform to 2 samples per symbol; for PAM (first paragraph) the
503-tap static equaliser on the blocks and the clock recovery as a delay
applied to each block's spectrum.  Each pin is fixed by the mathematics,
not by retyping the oracle: exact transforms of tones that are periodic in
a block, equality with the (separately pinned) time-domain FIR, and which
input samples an output may depend on."""
import numpy as np
import pytest

import oracle
import synth

N = 1 << 14
t = np.arange(N)
INNER = slice(512, N - 512)


def _rrc(k):
    h = np.zeros(k)
    oracle.lib().rxo_rrc_taps(k, 4.0, 0.1, h.ctypes.data_as(oracle._dp))
    return h


@pytest.mark.parametrize("k0", [1, 37, 255, 300, 511])
def test_block_hilbert_turns_a_bin_cosine_into_its_sine(k0):
    """A tone on a bin of the 1024-point grid is periodic in every block, so
    -j sgn(k) maps cos to sin exactly, whatever the block framing."""
    phi = oracle.hilbert_fd(np.cos(2 * np.pi * k0 * t / 1024 + 0.3))
    assert np.abs(phi[INNER] - np.sin(2 * np.pi * k0 * t / 1024 + 0.3)[INNER]).max() < 1e-10


@pytest.mark.parametrize("k0", [0, 512])
def test_block_hilbert_zeroes_dc_and_nyquist(k0):
    phi = oracle.hilbert_fd(3.0 + np.cos(np.pi * k0 * t / 512))
    assert np.abs(phi[INNER]).max() < 1e-10


def test_block_hilbert_is_odd_and_linear():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=N), rng.normal(size=N)
    pa, pb = oracle.hilbert_fd(a), oracle.hilbert_fd(b)
    assert np.allclose(oracle.hilbert_fd(2 * a - b), 2 * pa - pb, atol=1e-10)
    # applied twice, -j sgn(k) squared is -1 on every bin but DC and N/2
    ac = a - a.mean()
    twice = oracle.hilbert_fd(oracle.hilbert_fd(ac))
    # block-local: compare on blocks whose outputs come from interior samples only
    assert np.corrcoef(twice[INNER], -ac[INNER])[0, 1] > 0.9


def test_block_hilbert_output_depends_on_its_own_block_only():
    """Outputs 512 b .. 512 b + 511 come from samples 512 b - 256 .. 512 b + 767:
    changing any other sample leaves them unchanged (framing, guard, hop)."""
    rng = np.random.default_rng(4)
    l = rng.normal(size=N)
    b = 7
    base = oracle.hilbert_fd(l)
    for j in (512 * b - 257, 512 * b + 768, 100, N - 3):
        l2 = l.copy()
        l2[j] += 5.0
        assert np.array_equal(oracle.hilbert_fd(l2)[512 * b:512 * b + 512], base[512 * b:512 * b + 512])
    for j in (512 * b - 256, 512 * b + 767):
        l2 = l.copy()
        l2[j] += 5.0
        assert not np.array_equal(oracle.hilbert_fd(l2)[512 * b:512 * b + 512], base[512 * b:512 * b + 512])


def _fir_dec2(y, h):
    x = np.zeros(y.size // 2, dtype=np.complex128)
    oracle.lib().rxo_fir_same_dec2_cplx(y.view(np.float64).ctypes.data_as(oracle._dp), y.size,
                                         h.ctypes.data_as(oracle._dp), h.size,
                                         x.view(np.float64).ctypes.data_as(oracle._dp))
    return x


def test_fd_equaliser_equals_the_decimating_fir_on_kept_bins():
    """Block-periodic input inside |f| < fs/4: the circular convolution, the
    bin selection and the 512-point inverse change nothing, so the result is
    the time-domain FIR's every second output (centring, scale, offset)."""
    rng = np.random.default_rng(1)
    y = np.zeros(N, complex)
    for k in rng.integers(-255, 256, 12):
        y += rng.normal() * np.exp(2j * np.pi * k * t / 1024 + 1j * rng.uniform(0, 2 * np.pi))
    h = _rrc(oracle.FD_EQ_TAPS)
    x = oracle.fd_eq_dec2(y, h)
    xt = _fir_dec2(y, h)
    inner = slice(256, N // 2 - 256)
    assert np.abs(x[inner] - xt[inner]).max() < 1e-10 * np.abs(xt).max()
    # an asymmetric filter pins the direction of the centring
    ha = np.zeros(oracle.FD_EQ_TAPS)
    ha[101 + 5] = 1.0
    assert np.abs(oracle.fd_eq_dec2(y, ha)[inner] - y[2 * np.arange(N // 2) - 5][inner]).max() < 1e-10 * np.abs(y).max()


def test_fd_equaliser_drops_bins_beyond_a_quarter_of_the_rate():
    y = np.exp(2j * np.pi * 300 * t / 1024) + np.exp(-2j * np.pi * 400 * t / 1024)
    x = oracle.fd_eq_dec2(y, _rrc(oracle.FD_EQ_TAPS))
    assert np.abs(x[256:N // 2 - 256]).max() < 1e-10


def test_fd_equaliser_output_depends_on_its_own_block_only():
    rng = np.random.default_rng(5)
    y = rng.normal(size=N) + 1j * rng.normal(size=N)
    h = _rrc(oracle.FD_EQ_TAPS)
    b = 9
    base = oracle.fd_eq_dec2(y, h)[256 * b:256 * b + 256]
    for j in (512 * b - 257, 512 * b + 768):
        y2 = y.copy()
        y2[j] += 5.0
        assert np.array_equal(oracle.fd_eq_dec2(y2, h)[256 * b:256 * b + 256], base)
    y2 = y.copy()
    y2[512 * b - 256] += 5.0
    assert not np.array_equal(oracle.fd_eq_dec2(y2, h)[256 * b:256 * b + 256], base)


@pytest.mark.parametrize("fmt", [4, 5])
def test_fd_chain_noiseless_is_error_free(fmt):
    g = synth.generate(fmt, 1 << 18, seed=40 + fmt, snr_db=None)
    r = oracle.process(fmt, g["packed"], 1 << 18, g["seed"], want=("bits",), front=1)
    assert r["counted_bits"] > 100000 and r["bit_errors"] == 0


def test_fd_chain_agrees_with_the_time_domain_chain():
    """Both front ends are a Hilbert transform, the field, the downshift and a
    matched RRC with decimation; at 16 dB their decisions agree almost
    everywhere and their error counts are alike."""
    g = synth.generate(5, 1 << 18, seed=45, snr_db=16.0)
    fd = oracle.process(5, g["packed"], 1 << 18, g["seed"], want=("bits",), front=1)
    td = oracle.process(5, g["packed"], 1 << 18, g["seed"], want=("bits",))
    diff = np.unpackbits(fd["bits"] ^ td["bits"]).sum()
    assert diff < 2e-3 * fd["counted_bits"]
    assert abs(fd["bit_errors"] - td["bit_errors"]) < 4 * np.sqrt(td["bit_errors"] + 1)


def test_fd_front_rejects_what_it_does_not_cover():
    g = synth.generate(5, 1 << 16, seed=46, snr_db=20.0)
    for kw in ({"rounding": 1}, ):
        with pytest.raises(ValueError):
            oracle.process(5, g["packed"], 1 << 16, g["seed"], front=1, **kw)
    g2 = synth.generate(3, 1 << 16, seed=47, snr_db=20.0)
    with pytest.raises(ValueError):
        oracle.process(3, g2["packed"], 1 << 16, g2["seed"], front=1, equalizer=1,
                       mlp=np.zeros(oracle.MLP_PARAMS))


# ---- the PAM frequency-domain forms (Sec. 2, first paragraph: 503-tap static
# equaliser on the 1024-point blocks, frequency-domain clock recovery) ----
def _rrc2(k):
    h = np.zeros(k)
    oracle.lib().rxo_rrc_taps(k, 2.0, 0.1, h.ctypes.data_as(oracle._dp))
    return h


def _fir_same(x, h):
    y = np.zeros_like(x)
    oracle.lib().rxo_fir_same(x.ctypes.data_as(oracle._dp), x.size, h.ctypes.data_as(oracle._dp), h.size,
                              y.ctypes.data_as(oracle._dp))
    return y


def test_fd_fir_is_the_same_convolution():
    """503 taps fit inside the 256-sample guards, so no central output wraps
    around its block: the block filter equals the time-domain convolution
    with zeros outside the buffer everywhere, edges included."""
    rng = np.random.default_rng(6)
    x = rng.normal(size=N + 1024)
    for h in (_rrc2(oracle.FD_PAM_EQ_TAPS), rng.normal(size=oracle.FD_PAM_EQ_TAPS), rng.normal(size=33)):
        assert np.abs(oracle.fd_fir(x, h) - _fir_same(x, h)).max() < 1e-12 * np.abs(x).max() * np.abs(h).sum()


@pytest.mark.parametrize("k0", [3, 100, 511])
def test_fd_delay_shifts_a_bin_tone_by_each_blocks_delay(k0):
    rng = np.random.default_rng(k0)
    d = rng.uniform(-1.5, 1.5, N // 512)
    xr = oracle.fd_delay(np.cos(2 * np.pi * k0 * t / 1024 + 0.4), d)
    ref = np.cos(2 * np.pi * k0 * (t + np.repeat(d, 512)) / 1024 + 0.4)
    assert np.abs(xr - ref)[INNER].max() < 1e-10


def test_fd_delay_at_half_the_rate_keeps_the_signal_real():
    """The bin at N/2 takes cos(pi d): (-1)^t resampled at t + d is
    (-1)^t cos(pi d), with no imaginary part to discard."""
    d = np.linspace(-1.0, 1.0, N // 512)
    xr = oracle.fd_delay((-1.0) ** t, d)
    assert np.abs(xr - (-1.0) ** t * np.cos(np.pi * np.repeat(d, 512)))[INNER].max() < 1e-10


def test_fd_delay_zero_and_integer_delays():
    rng = np.random.default_rng(7)
    x = rng.normal(size=N)
    assert np.abs(oracle.fd_delay(x, np.zeros(N // 512)) - x).max() < 1e-12
    # an integer delay of a block-periodic signal is an exact shift
    per = rng.normal(size=1024)
    xp = np.tile(per, N // 1024)
    assert np.abs(oracle.fd_delay(xp, np.full(N // 512, 3.0)) - np.roll(xp, -3))[INNER].max() < 1e-10


def test_fd_delay_approaches_band_limited_interpolation():
    """On a band-limited signal (not periodic in the blocks) the block-circular
    delay differs from the exact shift only by the wrap-around of the block
    edges, attenuated across the 256-sample guards."""
    rng = np.random.default_rng(8)
    f = np.fft.rfftfreq(4 * N)
    spec = (rng.normal(size=f.size) + 1j * rng.normal(size=f.size)) * (f < 0.3)
    d = 0.37

    def sig(shift):
        return np.fft.irfft(spec * np.exp(2j * np.pi * f * shift), 4 * N)[:N]
    xr = oracle.fd_delay(sig(0.0), np.full(N // 512, d))
    err = np.abs(xr - sig(d))[INNER]
    assert err.max() < 2e-2 * np.abs(sig(0.0)).max() and np.sqrt(np.mean(err ** 2)) < 2e-3 * np.std(sig(0.0))


@pytest.mark.parametrize("fmt", [1, 2, 3])
def test_pam_fd_chain_noiseless_is_error_free(fmt):
    g = synth.generate(fmt, 1 << 18, seed=60 + fmt, snr_db=None, drive=0.1)
    r = oracle.process(fmt, g["packed"], 1 << 18, g["seed"], want=("bits",), front=1)
    assert r["counted_bits"] > 100000 and r["bit_errors"] == 0


def test_pam_fd_chain_agrees_with_the_time_domain_chain():
    g = synth.generate(3, 1 << 18, seed=63, snr_db=20.0)
    fd = oracle.process(3, g["packed"], 1 << 18, g["seed"], want=("bits",), front=1)
    td = oracle.process(3, g["packed"], 1 << 18, g["seed"], want=("bits",))
    assert abs(fd["bit_errors"] - td["bit_errors"]) < 0.1 * td["bit_errors"]


# ---- the paper's short KK DD-LMS (Sec. 2, second paragraph: a 4-tap
# decision-directed LMS equaliser doing clock- and symbol-phase recovery):
# 4 T/2-spaced taps, the carrier phase carried by the taps (no
# Viterbi-Viterbi stage) ----
def test_four_tap_ffe_alignment():
    """An even tap count keeps the centring c = (K - 1) / 2 = 1: tap i
    multiplies x[2k + 1 - i], so a unit tap 1 passes the symbol sample and a
    unit tap 0 the sample after it."""
    rng = np.random.default_rng(9)
    x = rng.normal(size=400) + 1j * rng.normal(size=400)
    for tap, off in ((1, 0), (0, 1), (2, -1), (3, -2)):
        w = np.zeros(4, complex)
        w[tap] = 1.0
        _, z = oracle.lms(x, w, 10, 100, mu=0.0)
        assert np.allclose(z, x[10 + 2 * np.arange(100) + off])


@pytest.mark.parametrize("theta", [0.0, 1.0, 2.2, -2.0])
def test_four_tap_dd_phase_chain_is_error_free_for_every_quadrant(theta):
    """Noiseless KK-16QAM through the paper's front end and its 4-tap
    DD-LMS without a separate phase stage: the prefix acquisition (CMA,
    static phase, quadrant) and the taps carry any carrier phase."""
    g = synth.generate(5, 1 << 18, seed=90, snr_db=None, theta_c=theta)
    r = oracle.process(5, g["packed"], 1 << 18, g["seed"], want=("bits",), front=1, ffe_taps=4, dd_phase=1)
    assert r["counted_bits"] > 200000 and r["bit_errors"] == 0


def test_four_tap_dd_phase_chain_at_22_db():
    for fmt in (4, 5):
        g = synth.generate(fmt, 1 << 18, seed=91 + fmt, snr_db=22.0)
        r = oracle.process(fmt, g["packed"], 1 << 18, g["seed"], want=("bits",), front=1, ffe_taps=4, dd_phase=1)
        assert r["bit_errors"] <= 2, r["bit_errors"]


def test_dd_phase_and_even_taps_are_limited_to_what_is_defined():
    g = synth.generate(2, 1 << 16, seed=95, snr_db=20.0)
    with pytest.raises(ValueError):
        oracle.process(2, g["packed"], 1 << 16, g["seed"], dd_phase=1)
    g = synth.generate(5, 1 << 16, seed=96, snr_db=20.0)
    with pytest.raises(ValueError):
        oracle.process(5, g["packed"], 1 << 16, g["seed"], ffe_taps=6)
