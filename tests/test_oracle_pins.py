"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: published known-answer values, closed forms, brute force, library
routines used as independent references, and whole-chain invariants."""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- reference sequence ------------------------------------------------------
def test_splitmix64_known_answers(oracle_lib):
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = [oracle_lib.splitmix64(0, k) for k in range(4)]
    assert got == vals
    # the generator's own implementation agrees (it feeds the reference bits)
    assert [int(v) for v in synth.splitmix64(0, np.arange(4))] == vals


# --- 12-bit unpack ------------------------------------------------------------
def test_unpack_explicit_bytes(oracle_lib):
    # codes 0xABC, 0x123 -> b0 = 0xBC, b1 = 0xA | (0x3 << 4), b2 = 0x12
    packed = np.array([0xBC, 0x3A, 0x12], dtype=np.uint8)
    assert list(oracle_lib.unpack12(packed, 2)) == [0xABC, 0x123]


def test_unpack_exhaustive_pairs(oracle_lib):
    a, b = np.meshgrid(np.arange(4096), np.arange(4096), indexing="ij")
    codes = np.stack([a.ravel(), b.ravel()], axis=1).ravel().astype(np.uint16)
    got = oracle_lib.unpack12(synth.pack12(codes), codes.size)
    assert np.array_equal(got, codes)


# --- FFT ------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
def test_fft_vs_bruteforce_dft(oracle_lib, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    k = np.arange(n)
    dft = np.exp(-2j * np.pi * np.outer(k, k) / n) @ x
    got = oracle_lib.fft(x)
    assert np.max(np.abs(got - dft)) <= 1e-13 * max(1.0, np.max(np.abs(dft)))
    inv = np.exp(2j * np.pi * np.outer(k, k) / n) @ x
    assert np.max(np.abs(oracle_lib.fft(x, inverse=True) - inv)) <= 1e-13 * max(1.0, np.max(np.abs(inv)))


def test_fft_parseval_impulse_roundtrip(oracle_lib):
    n = 4096
    rng = np.random.default_rng(1)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = oracle_lib.fft(x)
    assert abs(np.sum(np.abs(X) ** 2) / n - np.sum(np.abs(x) ** 2)) < 1e-9 * np.sum(np.abs(x) ** 2)
    assert np.max(np.abs(oracle_lib.fft(X, inverse=True) / n - x)) < 1e-12
    imp = np.zeros(n, complex)
    imp[0] = 1.0
    assert np.max(np.abs(oracle_lib.fft(imp) - 1.0)) < 1e-15
    assert np.max(np.abs(oracle_lib.fft(np.ones(n, complex)) - n * imp)) < 1e-9


# --- matched filter taps -------------------------------------------------------
@pytest.mark.parametrize("k,sps", [(33, 2), (65, 4)])
def test_rrc_taps(oracle_lib, k, sps):
    beta = 0.1
    h = oracle_lib.rrc_taps(k, sps, beta)
    assert abs(np.sum(h ** 2) - 1.0) < 1e-14
    assert np.max(np.abs(h - h[::-1])) < 1e-15
    # the |t| = 1/(4 beta) tap (exactly on the grid here) equals the limit of
    # the generic expression
    t = 1.0 / (4 * beta)
    i = int(round((k - 1) / 2 + t * sps))

    def generic(tt):
        return (np.sin(np.pi * tt * (1 - beta)) + 4 * beta * tt * np.cos(np.pi * tt * (1 + beta))) / (
            np.pi * tt * (1 - (4 * beta * tt) ** 2))
    scale = h[(k - 1) // 2] / (1 - beta + 4 * beta / np.pi)
    lim = 0.5 * (generic(t + 1e-6) + generic(t - 1e-6)) * scale
    assert abs(h[i] - lim) < 1e-8
    # RRC * RRC sampled at the symbol period is a Nyquist (zero-ISI) pulse,
    # up to truncation of the 16-symbol span
    rc = np.convolve(h, h)
    c = k - 1
    isi = rc[c + sps::sps]
    assert abs(rc[c] - 1.0) < 2e-2 and np.max(np.abs(isi)) < 3e-2


# --- Hilbert transformer ------------------------------------------------------
def test_hilbert_taps_structure(oracle_lib):
    h = oracle_lib.hilbert_taps(4097)
    m = np.arange(4097) - 2048
    assert np.all(h[m % 2 == 0] == 0.0)
    assert np.max(np.abs(h + h[::-1])) < 1e-18
    w = np.linspace(0.02, 0.98, 200) * np.pi
    resp = np.array([np.sum(h * np.sin(wi * m)) for wi in w])   # H(w) = -j*resp
    # an ideal Hilbert transformer has -j sgn(w): |resp| = 1 in band
    assert np.max(np.abs(resp - 1.0)) < 1e-4


def test_hilbert_cos_to_sin(oracle_lib):
    """H{cos(w n)} = sin(w n) away from the buffer edges."""
    h = oracle_lib.hilbert_taps(4097)
    n = np.arange(16384)
    for w in (0.05 * np.pi, 0.3 * np.pi, 0.77 * np.pi):
        phi = oracle_lib.hilbert_direct(np.cos(w * n), h)
        core = slice(2048, 16384 - 2048)
        assert np.max(np.abs(phi[core] - np.sin(w * n)[core])) < 1e-4


def test_hilbert_minimum_phase_closed_form(oracle_lib):
    """E = A exp(g) with g one-sided (positive frequencies only): ln|E| =
    ln A + Re g and its Hilbert transform is Im g = arg E - arg A."""
    n = np.arange(1 << 15)
    rng = np.random.default_rng(3)
    g = np.zeros(n.size, complex)
    for _ in range(12):
        w = rng.uniform(0.03, 0.9) * np.pi
        g += 0.05 * rng.standard_normal() * np.exp(1j * (w * n + rng.uniform(0, 2 * np.pi)))
    ell = np.log(3.0) + g.real
    phi = oracle_lib.hilbert_direct(ell, oracle_lib.hilbert_taps(4097))
    core = slice(4096, n.size - 4096)
    assert np.max(np.abs(phi[core] - g.imag[core])) < 2e-4


@pytest.mark.parametrize("log2n", [13, 14, 16])
def test_hilbert_overlap_save_equals_direct(oracle_lib, log2n):
    rng = np.random.default_rng(log2n)
    ell = np.cumsum(rng.standard_normal(40000)) * 0.01 + 3.0
    h = oracle_lib.hilbert_taps(4097)
    d = oracle_lib.hilbert_direct(ell, h)
    o = oracle_lib.hilbert_os(ell, h, log2n)
    assert np.max(np.abs(o - d)) < 1e-11 * np.max(np.abs(ell))


# --- plain FIRs against numpy's convolution ------------------------------------
def test_fir_same_matches_numpy(oracle_lib):
    rng = np.random.default_rng(5)
    for k in (1, 15, 33, 65):
        x = rng.standard_normal(1000)
        h = rng.standard_normal(k)
        assert np.max(np.abs(oracle_lib.fir_same(x, h) - np.convolve(x, h, "same"))) < 1e-12
        xc = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
        full = np.convolve(xc, h, "same")
        assert np.max(np.abs(oracle_lib.fir_same_dec2_cplx(xc, h) - full[0::2])) < 1e-12


# --- timing interpolation and estimation ---------------------------------------
def test_farrow_exact_on_cubics(oracle_lib):
    """Cubic Lagrange interpolation reproduces any cubic polynomial."""
    n = 4096
    t = np.arange(n, dtype=float)
    poly = lambda u: 1e-9 * u ** 3 - 2e-6 * u ** 2 + 0.01 * u - 3.0
    delta = np.array([0.0, 0.25, -0.6, 1.7, 0.5, -1.25, 2.0, 0.999])
    xr = oracle_lib.farrow(poly(t), delta)
    for b in range(8):
        s = np.arange(b * 512, (b + 1) * 512)
        s = s[(s > 4) & (s < n - 5)]
        assert np.max(np.abs(xr[s] - poly(s + delta[b]))) < 1e-9


@pytest.mark.parametrize("tau0", [0.0, 0.1, 0.35, 0.5, 0.8, 0.95])
def test_gardner_recovers_known_timing(oracle_lib, tau0):
    """Noiseless PAM-2 with a known symbol-timing offset tau0 (in symbol
    periods): the estimated shift is 2*tau0 samples (mod one symbol)."""
    g = synth.generate(synth.PAM2, 1 << 17, 42, None, tau0=tau0, drive=0.1)
    r = oracle_lib.process(1, g["packed"], 1 << 17, g["seed"], want=("timing",))
    d = r["timing"]
    err = (d - 2 * tau0 + 1.0) % 2.0 - 1.0
    assert np.max(np.abs(err)) < 0.06
    assert np.max(np.abs(np.diff(d))) < 0.05      # unwrapped: no 2-sample jumps


# --- decisions / Gray ------------------------------------------------------------
@pytest.mark.parametrize("m", [2, 4, 8])
def test_decisions_exhaustive(oracle_lib, m):
    for i in range(m):
        lvl = 2 * i - (m - 1)
        assert oracle_lib.decide(lvl, m) == i
        assert oracle_lib.decide(lvl + 0.999, m) == i
        assert oracle_lib.decide(lvl - 0.999, m) == i
        if i < m - 1:
            assert oracle_lib.decide(lvl + 1.0, m) == i + 1     # tie -> higher level
    assert oracle_lib.decide(-1e9, m) == 0 and oracle_lib.decide(1e9, m) == m - 1


# --- narrow-format rounding ------------------------------------------------------
def test_rounding_matches_library_conversions(oracle_lib):
    import torch
    rng = np.random.default_rng(9)
    vals = np.concatenate([rng.standard_normal(2000) * 30, [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8)]])
    vals32 = vals.astype(np.float32).astype(np.float64)
    bf = torch.tensor(vals32, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle_lib.round_bf16(v) for v in vals32])
    assert np.array_equal(got, bf)
    fp = vals32.astype(np.float16).astype(np.float64)
    got = np.array([oracle_lib.round_fp16(v) for v in vals32])
    assert np.array_equal(got, fp)
    assert oracle_lib.round_bf16(1 + 2 ** -8) == 1.0
    assert oracle_lib.round_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


# --- MLP and Adam -----------------------------------------------------------------
def _unit_mlp(sel=15):
    p = np.zeros(oracle_lib_params())
    w1 = p[:64 * 31].reshape(64, 31)
    w1[0, sel] = 1.0
    off = 64 * 31 + 64
    w2 = p[off:off + 4096].reshape(64, 64)
    w2[0, 0] = 1.0
    off += 4096 + 64
    p[off] = 1.0          # W3[0]
    return p


def oracle_lib_params():
    return 64 * 31 + 64 + 64 * 64 + 64 + 64 + 1


def test_mlp_forward_hand_network(oracle_lib):
    p = _unit_mlp(15)
    x = np.zeros((3, 31))
    x[0, 15] = 2.5
    x[1, 15] = -1.0
    x[2, 14] = 7.0
    assert np.allclose(oracle_lib.mlp_forward(p, x), [2.5, 0.0, 0.0], atol=0, rtol=0)
    p[-1] = 0.25          # b3
    assert np.allclose(oracle_lib.mlp_forward(p, x), [2.75, 0.25, 0.25])


def test_mlp_gradient_finite_differences(oracle_lib):
    rng = np.random.default_rng(11)
    p = rng.uniform(-0.3, 0.3, oracle_lib_params())
    x = rng.standard_normal((16, 31))
    t = rng.standard_normal(16)
    loss, g = oracle_lib.mlp_grad(p, x, t)
    idx = rng.choice(p.size, 60, replace=False)
    idx = np.concatenate([idx, [p.size - 1, 64 * 31, 64 * 31 + 64 + 4096 + 3]])
    for i in idx:
        e = 1e-6
        pp = p.copy(); pp[i] += e
        pm = p.copy(); pm[i] -= e
        num = (oracle_lib.mlp_grad(pp, x, t)[0] - oracle_lib.mlp_grad(pm, x, t)[0]) / (2 * e)
        assert abs(num - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-8
    y = oracle_lib.mlp_forward(p, x)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-12


def test_adam_constant_gradient_closed_form(oracle_lib):
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves each parameter by lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    p = np.zeros(3); m = np.zeros(3); v = np.zeros(3)
    for step in range(1, 6):
        oracle_lib.adam(p, m, v, g, step, lr=1e-3)
        assert np.allclose(p, -step * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)


# --- whole chains --------------------------------------------------------------
@pytest.mark.parametrize("fmt", [1, 2, 3])
def test_noiseless_pam_is_error_free(oracle_lib, fmt):
    """Near-linear modulator (drive 0.1), no noise: only 12-bit quantisation."""
    n = 1 << 18
    g = synth.generate(fmt, n, 1000 + fmt, None, drive=0.1)
    r = oracle_lib.process(fmt, g["packed"], n, g["seed"])
    assert r["counted_syms"] > 0 and r["bit_errors"] == 0


@pytest.mark.parametrize("fmt", [4, 5])
@pytest.mark.parametrize("quarter", [0, 1, 2, 3])
def test_noiseless_kk_error_free_every_rotation(oracle_lib, fmt, quarter):
    """CSPR 10 dB, no noise: zero errors whatever the carrier phase quadrant
    (the four-fold ambiguity is resolved on the known prefix)."""
    n = 1 << 18
    g = synth.generate(fmt, n, 2000 + fmt, None, theta_c=0.4 + quarter * np.pi / 2)
    r = oracle_lib.process(fmt, g["packed"], n, g["seed"], want=("taps",))
    assert r["bit_errors"] == 0
    # the FFE undoes the carrier rotation: arg of the centre tap = theta_c
    c = r["taps"][10]
    assert abs(np.angle(c * np.exp(-1j * g["theta_c"]))) < 0.05


@pytest.mark.parametrize("fmt,tau0,lag", [(5, 3.25, 3), (5, -2.4, -2), (4, 1.6, 2), (2, 4.3, 4), (2, -1.2, -1)])
def test_integer_delay_found_by_sync(oracle_lib, fmt, tau0, lag):
    n = 1 << 18
    g = synth.generate(fmt, n, 3000 + fmt, None, tau0=tau0, drive=0.1)
    r = oracle_lib.process(fmt, g["packed"], n, g["seed"])
    assert r["lag"] == lag and r["bit_errors"] == 0


def test_kk_reconstruction_converges_with_cspr(oracle_lib):
    """The KK field approaches the true optical field (up to a constant phase
    and scale) as the carrier-to-signal ratio grows; a wrong Hilbert sign or
    a missing sqrt would leave an O(1) error."""
    n = 1 << 17
    errs = []
    for cspr in (10.0, 16.0, 22.0):
        g = synth.generate(5, n, 77, None, cspr_db=cspr)
        r = oracle_lib.process(5, g["packed"], n, g["seed"], want=("field",))
        e, f = r["field"], g["field"]
        core = slice(8192, n - 8192)
        a = np.vdot(e[core], f[core]) / np.vdot(e[core], e[core])   # best complex scale
        res = f[core] - a * e[core]
        sig = f[core] - np.mean(f[core])
        errs.append(np.linalg.norm(res) / np.linalg.norm(sig))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


def test_reference_bits_match_generator(oracle_lib):
    """Error counting regenerates the transmitted bits: a noiseless buffer
    decoded by the oracle reproduces the generator's bits exactly."""
    n = 1 << 18
    g = synth.generate(2, n, 55, None, drive=0.1)
    r = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits",))
    ref = synth.reference_bits(2, g["seed"], n // 2)
    bits = np.unpackbits(r["bits"], bitorder="little")[: ref.size * 2].reshape(-1, 2)
    dec = bits[:, 0] * 2 + bits[:, 1]
    core = slice(4096 + 64, ref.size - 64)
    assert np.array_equal(dec[core], ref[core])


def test_precision_form_error_bound(oracle_lib):
    """BF16/FP16 operands with exact accumulation stay within
    (2u) * sum|h||x| of the unrounded matched filter, elementwise."""
    n = 1 << 17
    g = synth.generate(5, n, 88, 22.0)
    ref = oracle_lib.process(5, g["packed"], n, g["seed"], want=("mf", "shifted", "field"))
    h = oracle_lib.rrc_taps(65, 4, 0.1)
    for rounding, u in ((1, 2.0 ** -8), (2, 2.0 ** -11)):
        r = oracle_lib.process(5, g["packed"], n, g["seed"], want=("mf",), rounding=rounding)
        # both outputs carry the AGC scale of their own run
        y_pre = ref["field"] * np.exp(-2j * np.pi * ((0.1375 * np.arange(n)) % 1.0))
        bound = 2 * u * np.convolve(np.abs(y_pre), np.abs(h), "same")[0::2] * ref["agc"]
        diff = np.abs(r["mf"] - ref["mf"])
        assert np.all(diff <= bound * 1.05 + 1e-12)


@pytest.mark.parametrize("fmt,fs_sim", [(5, 4.0e9), (2, 8.0e9)])
def test_synth_osnr_measured_from_detected_noise(fmt, fs_sim):
    """The optical-noise option of the input generator (the OSNR sweeps'
    noise model): with the same seed, noisy minus noiseless intensity is the
    signal-ASE beat (zero mean) plus |n_co|^2 + |n_or|^2, whose mean is twice
    the per-polarisation variance (the PAM path's 2 GHz low-pass keeps the
    mean).  The OSNR recovered from that mean, P_sig / (ASE of both
    polarisations in 12.5 GHz), is the one asked for."""
    n = 1 << 20
    for osnr in (18.0, 26.0):
        a = synth.generate(fmt, n, 5, None, osnr_db=osnr)
        b = synth.generate(fmt, n, 5, None)
        var = float(np.mean(a["intensity"] - b["intensity"])) / 2.0
        p_sig = float(np.mean(b["intensity"]))
        ase_in_band = 2.0 * var / fs_sim * 12.5e9
        assert 10.0 * np.log10(p_sig / ase_in_band) == pytest.approx(osnr, abs=0.25)


@pytest.mark.parametrize("beta", [0.01, 0.1, 0.5])
@pytest.mark.parametrize("k,sps", [(33, 2), (65, 4)])
def test_rrc_taps_against_the_spectrum(oracle_lib, k, sps, beta):
    """The oracle's matched-filter taps (closed-form impulse response) have
    the shape of the impulse response obtained numerically from the
    root-raised-cosine spectrum (a fine inverse FFT of the input generator's
    closed-form spectrum), for the default roll-off and the trial's 0.01
    (KK) and 0.5 (PAM)."""
    h = oracle_lib.rrc_taps(k, sps, beta)
    m, size = 16, 1 << 20
    dt = 1.0 / (sps * m)
    ref = np.fft.ifft(synth.rrc_spectrum(np.fft.fftfreq(size, d=dt), 1.0, beta)).real / dt
    ref = ref[(np.arange(k) - (k - 1) // 2) * m % size]
    assert np.max(np.abs(h / np.linalg.norm(h) - ref / np.linalg.norm(ref))) < 1e-6
