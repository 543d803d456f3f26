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


@pytest.mark.parametrize("fmt", [1, 2])
def test_gardner_recovers_known_timing(oracle_lib, fmt):
    """Noiseless PAM with a known symbol-timing offset tau0 (in symbol
    periods): the estimated shift is 2*tau0 samples (mod one symbol) within
    1e-2 T = 0.02 samples, at every tau0 of a grid over one symbol, and the
    estimate is unwrapped (no 2-sample jumps)."""
    for tau0 in np.arange(10) / 10 + 0.05:
        g = synth.generate(fmt, 1 << 17, 42, None, tau0=tau0, drive=0.1)
        r = oracle_lib.process(fmt, g["packed"], 1 << 17, g["seed"], want=("timing",))
        d = r["timing"]
        err = (d - 2 * tau0 + 1.0) % 2.0 - 1.0
        assert np.max(np.abs(err)) < 0.02, (tau0, np.max(np.abs(err)))
        assert np.max(np.abs(np.diff(d))) < 0.05


@pytest.mark.parametrize("phi", [0.0, 0.3, -1.1, 2.5])
def test_gardner_tone_closed_form(oracle_lib, phi):
    """A tone at half the symbol rate, x[s] = cos(pi s / 2 + phi): per symbol
    the detector gives G0 = -sin(2 phi) and, through the half-sample cubic
    Lagrange interpolator of gain a = 5 / (4 sqrt 2) at that frequency,
    G1 = -a^2 cos(2 phi) (a^2 = 25/32).  So every interior block sums to
    256 (-sin 2phi - j (25/32) cos 2phi), and the estimated shift is the
    tone's peak position -2 phi / pi samples (mod one symbol)."""
    n = 1 << 16
    s = np.arange(n)
    x = np.cos(np.pi * (s % 4) / 2 + phi)   # the phase reduced exactly (period 4)
    c = oracle_lib.gardner_sums(x)
    want = 256 * (-np.sin(2 * phi) - 1j * (25 / 32) * np.cos(2 * phi))
    assert np.max(np.abs(c[1:-1] - want)) < 1e-11
    d = oracle_lib.gardner(x)
    interior = d[17:-17]
    err = (interior + 2 * phi / np.pi + 1.0) % 2.0 - 1.0
    assert np.max(np.abs(err)) < 1e-12


def test_gardner_s_curve_sinusoidal(oracle_lib):
    """Noiseless PAM-2 (roll-off 0.1): the mean detector outputs over a
    symbol of timing offsets are sinusoids in tau0 (the S-curve of a
    quadratic detector at under 100 % excess bandwidth), G0 and the scaled
    G1 of equal amplitude a quarter period apart, so their angle advances
    by 2 pi per symbol."""
    taus = np.arange(16) / 16
    cs = []
    for tau0 in taus:
        g = synth.generate(1, 1 << 17, 42, None, tau0=tau0, drive=0.1)
        r = oracle_lib.process(1, g["packed"], 1 << 17, g["seed"], want=("mf",))
        cs.append(oracle_lib.gardner_sums(r["mf"])[1:-1].mean())
    cs = np.array(cs)
    g0, g1 = cs.real, cs.imag * 32 / 25
    basis = np.stack([np.sin(2 * np.pi * taus), np.cos(2 * np.pi * taus), np.ones_like(taus)], 1)
    amps = []
    for v in (g0, g1):
        coef = np.linalg.lstsq(basis, v, rcond=None)[0]
        amp = np.hypot(coef[0], coef[1])
        amps.append(amp)
        assert np.max(np.abs(v - basis @ coef)) < 2e-3 * amp
        assert abs(coef[2]) < 2e-3 * amp
    assert abs(amps[0] / amps[1] - 1) < 1e-2
    ang = np.unwrap(np.angle(g0 + 1j * g1))
    slope = np.polyfit(taus, ang, 1)[0]
    assert abs(slope - 2 * np.pi) < 1e-2


# --- adaptive filters -------------------------------------------------------------
@pytest.mark.parametrize("mu", [1e-3, 1e-2])
def test_lms_single_tap_closed_form(oracle_lib, mu):
    """One tap, input +-1, desired d_k = w* x_k, no noise: the error
    recursion is w_k - w* = (1 - mu)^k (w_0 - w*) exactly, which fixes the
    step size's scale, the sign of the update and the conjugate."""
    rng = np.random.default_rng(17)
    nsym = 3000
    x = np.zeros(2 * nsym, complex)
    x[0::2] = rng.choice([-1.0, 1.0], nsym)
    wstar = 0.7 - 0.2j
    d = wstar * x[0::2]
    for k in (1, 10, 700, 3000):
        w, z = oracle_lib.lms(x, [0.3 + 0.1j], 0, k, ref=d, mu=mu)
        want = wstar + (1 - mu) ** k * (0.3 + 0.1j - wstar)
        assert abs(w[0] - want) < 1e-12
    # outputs are formed before each update
    assert abs(z[0] - (0.3 + 0.1j) * x[0]) < 1e-15


def test_lms_converges_to_wiener_solution(oracle_lib):
    """QPSK through a short T/2-spaced channel with noise: data-aided LMS
    settles at the least-squares (Wiener) taps from the normal equations,
    within the steady-state misadjustment of about mu J_min tr(R) / 2."""
    rng = np.random.default_rng(23)
    nsym, K, mu = 200000, 7, 2e-3
    a = rng.choice([-1.0, 1.0], nsym) + 1j * rng.choice([-1.0, 1.0], nsym)
    up = np.zeros(2 * nsym, complex)
    up[0::2] = a
    ch = np.array([0.1, 0.3, 1.0, 0.25 + 0.1j, -0.1])
    x = np.convolve(up, ch)[: 2 * nsym] + 0.05 * (rng.standard_normal(2 * nsym) + 1j * rng.standard_normal(2 * nsym))
    c = (K - 1) // 2
    # regressors u_k[i] = x[2k + c - i]; z_k = sum_i w_i u_k[i]
    idx = 2 * np.arange(nsym)[:, None] + c - np.arange(K)[None, :]
    U = np.where((idx >= 0) & (idx < x.size), x[np.clip(idx, 0, x.size - 1)], 0)
    wopt = np.linalg.lstsq(U, a, rcond=None)[0]
    jmin = np.mean(np.abs(a - U @ wopt) ** 2)
    trR = K * np.mean(np.abs(x) ** 2)
    w, z = oracle_lib.lms(x, np.zeros(K), 0, nsym, ref=a, mu=mu)
    err2 = np.sum(np.abs(w - wopt) ** 2)
    assert err2 < 3.0 * mu * jmin * trR / 2
    # the tail's output error is the Wiener MSE plus the excess mu J_min tr(R)/2
    mse = np.mean(np.abs(a[-20000:] - z[-20000:]) ** 2)
    assert jmin < mse < jmin * (1 + 3 * mu * trR / 2)


@pytest.mark.parametrize("theta", [0.3, -0.6])
def test_cma_radius_and_static_phase(oracle_lib, theta):
    """Noiseless QPSK (unit power, radius R2 = 1) rotated by theta through a
    mild ISI channel: CMA from the centre tap drives |z|^2 to R2, and the
    Viterbi-Viterbi sum of z^4 over its last outputs recovers theta modulo
    pi/2 within 1e-3 rad (CMA is blind to the phase, so the channel's own
    phase is the only other rotation: the channel here is real)."""
    rng = np.random.default_rng(29)
    nsym, K = 30000, 21
    a = (rng.choice([-1.0, 1.0], nsym) + 1j * rng.choice([-1.0, 1.0], nsym)) / np.sqrt(2)
    up = np.zeros(2 * nsym, complex)
    up[0::2] = a * np.exp(1j * theta)
    ch = np.array([0.05, 0.15, 1.0, 0.15, 0.05])
    x = np.convolve(up, ch)[2: 2 * nsym + 2]   # centre of the channel on the symbol sample
    x /= np.sqrt(np.mean(np.abs(x[0::2]) ** 2) + np.mean(np.abs(x[1::2]) ** 2)) / np.sqrt(2) * np.sqrt(1.0)
    w0 = np.zeros(K, complex)
    w0[(K - 1) // 2] = 1.0
    w, s4, z = oracle_lib.cma(x, w0, nsym, mu=1e-3, r2=1.0, nvv=2048)
    tail = z[-2048:]
    assert np.mean((np.abs(tail) ** 2 - 1.0) ** 2) < 1e-4
    est = 0.25 * np.angle(-s4)
    d = (est - theta + np.pi / 4) % (np.pi / 2) - np.pi / 4
    assert abs(d) < 1e-3


def test_downshift_phase_exact(oracle_lib):
    """f_c / f_s = 0.55 / 4 = 11/80 exactly, so the phase of sample n is
    (11 n mod 80) / 80 revolutions; the FP64 value frac(r n) agrees to
    1e-15 n over the largest buffer (2^26 samples)."""
    rng = np.random.default_rng(31)
    ns = np.concatenate([np.arange(200), rng.integers(0, 1 << 26, 2000), [(1 << 26) - 1]])
    r = 0.55e9 / 4e9
    for n in ns:
        n = int(n)
        exact = (11 * n % 80) / 80.0
        got = oracle_lib.downshift_rev(r, n)
        diff = abs(got - exact)
        diff = min(diff, 1.0 - diff)   # 0 and 1 are the same phase
        assert diff <= 1e-15 * max(n, 1), (n, got, exact)


def _qpsk_block_sums(theta, blk=128, seed=37):
    """Sums of z^4 per block for QPSK symbols (odd-integer units) rotated by
    the block phases theta_b: each is E-sum of a^4 e^{4 j theta_b} = -4 blk
    e^{4 j theta_b}."""
    rng = np.random.default_rng(seed)
    s4 = []
    for th in theta:
        a = rng.choice([-1.0, 1.0], blk) + 1j * rng.choice([-1.0, 1.0], blk)
        z = a * np.exp(1j * th)
        s4.append(np.sum(z ** 4))
    return np.array(s4)


def test_vv_unwrap_follows_a_ramp_across_pi_over_4(oracle_lib):
    """A carrier phase ramp of 0.05 rad per block over 400 blocks (crossing
    +-pi/4 many times): the symmetric three-block window of a linear ramp
    has exactly the middle block's angle, so the unwrapped estimate equals
    the ramp up to one constant multiple of pi/2, and the first block (two
    blocks in its window) is off by half a step."""
    nb, step = 400, 0.05
    theta = 0.7 + step * np.arange(nb)
    ph = oracle_lib.vv_phase(_qpsk_block_sums(theta))
    off = ph[1:-1] - theta[1:-1]
    k = np.round(off[0] / (np.pi / 2))
    assert np.max(np.abs(off - k * np.pi / 2)) < 1e-12
    assert abs(ph[0] - theta[0] - k * np.pi / 2 - step / 2) < 1e-12
    # a decreasing ramp, and a slow sinusoidal wander of 3 rad amplitude
    theta2 = -0.2 - 0.07 * np.arange(nb)
    off2 = oracle_lib.vv_phase(_qpsk_block_sums(theta2))[1:-1] - theta2[1:-1]
    k2 = np.round(off2[0] / (np.pi / 2))
    assert np.max(np.abs(off2 - k2 * np.pi / 2)) < 1e-12
    theta3 = 3.0 * np.sin(2 * np.pi * np.arange(nb) / 200)
    off3 = oracle_lib.vv_phase(_qpsk_block_sums(theta3))[1:-1] - theta3[1:-1]
    k3 = np.round(off3[0] / (np.pi / 2))
    assert np.max(np.abs(off3 - k3 * np.pi / 2)) < 2e-3


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


def test_mlp_forward_bf16_hand_network(oracle_lib):
    """rounding=1 rounds every layer's operands to BF16 (inputs, weights,
    hidden activations) and keeps the biases exact.  With x = 1 + 2^-8 (a
    tie: rounds to 1), W1 = 1 + 3 2^-8 (a tie: rounds up to 1 + 2^-6) and
    b1 = 2^-9: h1 = 1 + 2^-6 + 2^-9, which rounds to 1 + 2^-6; W2 = 1 + 2^-9
    rounds to 1, b2 = 2^-12 exact: h2 = 1 + 2^-6 + 2^-12, which rounds to
    1 + 2^-6 (2^-12 is below half an ulp, 2^-8); W3 = 1 + 2^-20 rounds to 1;
    b3 = 2^-30 is added exactly."""
    p = np.zeros(oracle_lib_params())
    p[15] = 1 + 3 * 2.0 ** -8                    # W1[0][15]
    p[64 * 31] = 2.0 ** -9                       # b1[0]
    off = 64 * 31 + 64
    p[off] = 1 + 2.0 ** -9                       # W2[0][0]
    p[off + 4096] = 2.0 ** -12                   # b2[0]
    p[off + 4096 + 64] = 1 + 2.0 ** -20          # W3[0]
    p[-1] = 2.0 ** -30                           # b3
    x = np.zeros((1, 31))
    x[0, 15] = 1 + 2.0 ** -8
    want = (1 + 2.0 ** -6) * 1.0 + 2.0 ** -30
    assert oracle_lib.mlp_forward(p, x, rounding=1)[0] == want
    # unrounded: every term exact in FP64
    h1 = (1 + 3 * 2.0 ** -8) * (1 + 2.0 ** -8) + 2.0 ** -9
    exact = (h1 * (1 + 2.0 ** -9) + 2.0 ** -12) * (1 + 2.0 ** -20) + 2.0 ** -30
    assert oracle_lib.mlp_forward(p, x, rounding=0)[0] == exact
    # FP16 (11 significant bits) holds x, W1 and W2 exactly; h1 = 1 + 2^-6 + 2^-9 + 3 2^-16
    # rounds to 1 + 2^-6 + 2^-9 (3 2^-16 is below half an ulp, 2^-11); then
    # h2 = (1 + 2^-6 + 2^-9)(1 + 2^-9) + 2^-12 = 1 + 2^-6 + 2^-8 + 2^-12 + 2^-15 + 2^-18
    # rounds to 1 + 2^-6 + 2^-8 (the rest is below 2^-11), and W3 rounds to 1
    want16 = (1 + 2.0 ** -6 + 2.0 ** -8) * 1.0 + 2.0 ** -30
    assert oracle_lib.mlp_forward(p, x, rounding=2)[0] == want16


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
    """The precision form's matched filter takes the carrier-free downshifted
    field (E - m) exp(-j 2 pi frac(r n)) and the taps rounded to BF16/FP16
    (unit roundoff u = 2^-8 / 2^-11) with exact accumulation: each output is
    within 2u sum|h||y| of the unrounded filter (each product carries at most
    two roundings), elementwise; both runs apply their own AGC gain."""
    n = 1 << 17
    g = synth.generate(5, n, 88, 22.0)
    ref = oracle_lib.process(5, g["packed"], n, g["seed"], want=("mf", "shifted", "field"))
    h = oracle_lib.rrc_taps(65, 4, 0.1)
    y = ref["shifted"]
    # the carrier-free input is far smaller than the field (CSPR 10 dB)
    assert np.linalg.norm(y) < 0.5 * np.linalg.norm(ref["field"])
    for rounding, u in ((1, 2.0 ** -8), (2, 2.0 ** -11)):
        r = oracle_lib.process(5, g["packed"], n, g["seed"], want=("mf",), rounding=rounding)
        bound = 2 * u * np.convolve(np.abs(y), np.abs(h), "same")[0::2] * ref["agc"]
        diff = np.abs(r["mf"] - ref["mf"])
        assert np.all(diff <= bound * 1.05 + 1e-12)
        # and the error is of the rounding's size, not far below it (the operands are rounded)
        assert np.sqrt(np.mean(diff ** 2)) > 0.02 * np.sqrt(np.mean(bound ** 2))


def _linear_net_from_taps(w, K):
    """A 31-64-64-1 ReLU network computing the real FIR sum_i w_i x[c - i]
    on its centred window: y = relu(relu(z)) - relu(relu(-z))."""
    p = np.zeros(oracle_lib_params())
    c = (K - 1) // 2
    w1 = p[:64 * 31].reshape(64, 31)
    for i in range(K):
        w1[0, 15 + c - i] = w[i]
        w1[1, 15 + c - i] = -w[i]
    off = 64 * 31 + 64
    w2 = p[off:off + 4096].reshape(64, 64)
    w2[0, 0] = 1.0
    w2[1, 1] = 1.0
    off += 4096 + 64
    p[off] = 1.0
    p[off + 1] = -1.0
    return p


def test_mlp_judge_and_fallback(oracle_lib):
    """The learned equaliser replaces the DD-LMS blocks only if it makes no
    more decision errors than the trained LMS taps on the known prefix.  A
    network equal to the frozen prefix FIR ties with LMS and runs (its soft
    values are that FIR's outputs, i.e. the frozen-tap form); an all-zero
    network loses and the block DD-LMS runs instead (the LMS chain's
    decisions, fallback flagged)."""
    n = 1 << 18
    g = synth.generate(2, n, 61, 16.0)
    lms = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits", "soft", "taps"))
    frozen = oracle_lib.process(2, g["packed"], n, g["seed"], want=("soft",), form=1)
    w = lms["taps"].real
    assert np.max(np.abs(lms["taps"].imag)) == 0.0
    net = _linear_net_from_taps(w, 15)
    r = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits", "soft"), equalizer=1, mlp=net)
    assert r["fallback"] == 0
    assert np.max(np.abs(r["soft"] - frozen["soft"])) < 1e-12
    zero = np.zeros(oracle_lib_params())
    r0 = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits", "soft"), equalizer=1, mlp=zero)
    assert r0["fallback"] == 1
    assert np.array_equal(r0["bits"], lms["bits"]) and np.array_equal(r0["soft"], lms["soft"])


def test_forced_decision_stays_in_its_block(oracle_lib):
    """Forcing the block DD-LMS to its own decision changes nothing; forcing
    another level at symbol k leaves every output before and at k (formed
    before its update) and every other block unchanged, and moves the later
    outputs of k's block only."""
    n = 1 << 18
    g = synth.generate(2, n, 62, 14.0)
    base = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits", "soft"))
    nsym = n // 2
    k = 3 * 256 + 40 + 2 * 4096          # a symbol inside DD-LMS block 35
    f = np.full(nsym, -1, dtype=np.int32)
    own = oracle_lib.decide(base["soft"][k], 4)
    f[k] = own
    same = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits", "soft"), force=f)
    assert np.array_equal(same["soft"], base["soft"])
    f[k] = own + 1 if own < 3 else own - 1
    moved = oracle_lib.process(2, g["packed"], n, g["seed"], want=("bits", "soft"), force=f)
    b0, b1 = (k // 256) * 256, (k // 256 + 1) * 256
    d = moved["soft"] - base["soft"]
    assert np.all(d[:k + 1] == 0.0) and np.all(d[b1:] == 0.0)
    assert np.max(np.abs(d[k + 1:b1])) > 1e-6 and b0 < k


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
