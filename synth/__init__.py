"""Seeded synthetic ADC buffers for the receiver tests and benchmark.

This module is test infrastructure: it stands in for the transmitter, the
link and the 12-bit ADC of the field trial (Sec. 3, first paragraph, and
Fig. 2), which cannot be reproduced without the optical hardware.  It holds
none of the receiver's arithmetic: pulse shaping is done in the frequency
domain from the closed-form root-raised-cosine spectrum, and the only thing it
shares with the receiver is the published definition of the counter-based
SplitMix64 generator that fixes the transmitted bits (each side implements it
on its own).

Waveforms (all synthesised circularly over exactly one buffer):

* PAM-M at 2 GBaud (2 samples/symbol at 4 Gs/s): root-raised-cosine pulses
  (roll-off 0.1) with the outer symbol at +-1, optional tanh driver
  compression, a Mach-Zehnder arm biased at quadrature with 0.3 drive
  (field = cos(pi/4 - (pi/2) * drive * v)), optional chromatic dispersion on
  the optical field, square-law detection.  Simulated at 8 Gs/s and reduced to
  4 Gs/s by an ideal 2 GHz low-pass.
* KK-QAM at 1 GBaud (4 samples/symbol): s(t) RRC-shaped QPSK/16QAM placed at
  +f_c above a carrier tone of power CSPR * E|s|^2, square-law detection.
  Its spectrum stays below 1.1 GHz, so it is synthesised at 4 Gs/s directly.

Optionally, before detection, amplified spontaneous emission at a given
OSNR (signal power over the ASE power of both polarisations in a 12.5 GHz,
0.1 nm, reference band): complex white Gaussian noise on the optical field,
half of it co-polarised with the signal (signal-ASE and ASE-ASE beating) and
half orthogonal (ASE-ASE only), white over the simulation bandwidth.

Then electrical AWGN (variance = var(I)/SNR at 4 Gs/s) and the 12-bit
quantiser c = clamp(floor(I / D), 0, 4095) with D = (mean(I) + 6 std(I))/4096,
packed two samples per three bytes, little-endian.
"""
from __future__ import annotations

import numpy as np

PAM2, PAM4, PAM8, KK_QPSK, KK_16QAM = 1, 2, 3, 4, 5
FORMAT_NAMES = {PAM2: "PAM-2", PAM4: "PAM-4", PAM8: "PAM-8",
                KK_QPSK: "KK-QPSK", KK_16QAM: "KK-16QAM"}
FS = 4.0e9

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def is_kk(fmt: int) -> bool:
    return fmt in (KK_QPSK, KK_16QAM)


def bits_per_symbol(fmt: int) -> int:
    return {PAM2: 1, PAM4: 2, PAM8: 3, KK_QPSK: 2, KK_16QAM: 4}[fmt]


def sps_of(fmt: int) -> int:
    return 4 if is_kk(fmt) else 2


def splitmix64(seed: int, k) -> np.ndarray:
    """k-th output (k = 0, 1, ...) of SplitMix64 seeded with `seed`
    (Steele, Lea & Flood, OOPSLA 2014): state_k = seed + (k+1)*gamma, mixed."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def derive_seed(base: int, index: int) -> int:
    """Per-buffer seed from a configuration's base seed."""
    return int(splitmix64(base, index))


def _gray_inverse(g: np.ndarray) -> np.ndarray:
    i = g.copy()
    s = g >> 1
    while np.any(s):
        i ^= s
        s >>= 1
    return i


def reference_bits(fmt: int, seed: int, nsym: int) -> np.ndarray:
    """Top log2(M) bits of SplitMix64(seed, k) for symbols k = 0..nsym-1."""
    bps = bits_per_symbol(fmt)
    r = splitmix64(seed, np.arange(nsym, dtype=np.uint64))
    return (r >> np.uint64(64 - bps)).astype(np.int64)


def reference_levels(fmt: int, seed: int, nsym: int) -> np.ndarray:
    """Transmitted odd-integer levels (real for PAM, complex for QAM)."""
    b = reference_bits(fmt, seed, nsym)
    if is_kk(fmt):
        half = bits_per_symbol(fmt) // 2
        m_axis = 1 << half
        bi = b >> half
        bq = b & (m_axis - 1)
        ii = _gray_inverse(bi)
        iq = _gray_inverse(bq)
        return (2 * ii - (m_axis - 1)) + 1j * (2 * iq - (m_axis - 1))
    m = 1 << bits_per_symbol(fmt)
    return (2 * _gray_inverse(b) - (m - 1)).astype(np.float64)


def rrc_spectrum(f: np.ndarray, rs: float, beta: float) -> np.ndarray:
    """Closed-form root-raised-cosine amplitude spectrum, H(0) = 1."""
    af = np.abs(f) / rs
    lo, hi = (1 - beta) / 2, (1 + beta) / 2
    h = np.zeros_like(af)
    h[af <= lo] = 1.0
    mid = (af > lo) & (af <= hi)
    h[mid] = np.sqrt(0.5 * (1 + np.cos(np.pi / beta * (af[mid] - lo))))
    return h


def _shaped(levels: np.ndarray, sps_sim: int, rs: float, fs_sim: float,
            beta: float, tau0: float) -> np.ndarray:
    """Circular RRC waveform sum_k a_k p(t - kT - tau0), p(0) = 1."""
    nsim = levels.size * sps_sim
    up = np.zeros(nsim, dtype=np.complex128)
    up[::sps_sim] = levels
    f = np.fft.fftfreq(nsim, d=1.0 / fs_sim)
    h = rrc_spectrum(f, rs, beta)
    h = h / (h.sum() / nsim)             # impulse response peak = 1
    spec = np.fft.fft(up) * h * np.exp(-2j * np.pi * f * tau0)
    return np.fft.ifft(spec)


def quantize12(intensity: np.ndarray) -> np.ndarray:
    d = (intensity.mean() + 6.0 * intensity.std()) / 4096.0
    c = np.floor(intensity / d)
    return np.clip(c, 0, 4095).astype(np.uint16)


def pack12(codes: np.ndarray) -> np.ndarray:
    """Two 12-bit codes per three bytes, little-endian (s0 low first)."""
    c = np.asarray(codes, dtype=np.uint16)
    assert c.size % 2 == 0
    s0 = c[0::2].astype(np.uint32)
    s1 = c[1::2].astype(np.uint32)
    out = np.empty((c.size // 2, 3), dtype=np.uint8)
    out[:, 0] = s0 & 0xFF
    out[:, 1] = ((s0 >> 8) & 0xF) | ((s1 & 0xF) << 4)
    out[:, 2] = (s1 >> 4) & 0xFF
    return out.reshape(-1)


def unpack12(packed: np.ndarray) -> np.ndarray:
    p = np.asarray(packed, dtype=np.uint8).reshape(-1, 3).astype(np.uint16)
    out = np.empty(p.shape[0] * 2, dtype=np.uint16)
    out[0::2] = p[:, 0] | ((p[:, 1] & 0xF) << 8)
    out[1::2] = (p[:, 1] >> 4) | (p[:, 2] << 4)
    return out


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed & 0xFFFFFFFFFFFFFFFF, stream]))


def generate(fmt: int, n_samples: int, seed: int, snr_db: float | None = 20.0, *,
             rolloff: float = 0.1, cspr_db: float = 10.0, fc_hz: float = 0.55e9,
             drive: float = 0.3, tanh_driver: bool = False,
             beta2_l_s2: float | None = None, tau0: float | None = None,
             theta_c: float | None = None, osnr_db: float | None = None) -> dict:
    """One synthetic 12-bit ADC buffer.  `snr_db=None` means no electrical
    noise; `osnr_db` adds optical noise before detection (None: none).

    Returns a dict with 'packed' (uint8, 1.5 * n_samples), 'codes',
    'intensity', the drawn impairments ('tau0' in symbol periods,
    'theta_c') and, with optical noise, 'ase_var' (the per-polarisation
    complex noise variance per simulation sample) and 'p_sig'."""
    if n_samples % 2:
        raise ValueError("n_samples must be even")
    sps = sps_of(fmt)
    rs = FS / sps
    nsym = n_samples // sps
    r = _rng(seed, 7)
    if tau0 is None:
        tau0 = float(r.uniform(0.0, 1.0))
    if theta_c is None:
        theta_c = float(r.uniform(0.0, 2 * np.pi))
    a = reference_levels(fmt, seed, nsym)
    if is_kk(fmt):
        s = _shaped(a.astype(np.complex128), sps, rs, FS, rolloff, tau0 / rs)
        ps = np.mean(np.abs(s) ** 2)
        amp = np.sqrt(10.0 ** (cspr_db / 10.0) * ps)
        n = np.arange(n_samples)
        field = amp * np.exp(1j * theta_c) + s * np.exp(2j * np.pi * fc_hz / FS * n)
        true_field = field
        inten, ase = _detect(field, FS, osnr_db, seed)
    else:
        m = 1 << bits_per_symbol(fmt)
        os_ = 2
        v = _shaped(a / (m - 1), sps * os_, rs, FS * os_, rolloff, tau0 / rs).real
        if tanh_driver:
            v = np.tanh(v) / np.tanh(1.0)
        field = np.cos(np.pi / 4 - (np.pi / 2) * drive * v).astype(np.complex128)
        f = np.fft.fftfreq(field.size, d=1.0 / (FS * os_))
        if beta2_l_s2 is not None:
            field = np.fft.ifft(np.fft.fft(field) *
                                np.exp(0.5j * beta2_l_s2 * (2 * np.pi * f) ** 2))
        i_sim, ase = _detect(field, FS * os_, osnr_db, seed)
        spec = np.fft.fft(i_sim)
        spec[np.abs(f) >= FS / 2] = 0.0          # ideal 2 GHz anti-alias filter
        inten = np.fft.ifft(spec).real[::os_]
        true_field = field[::os_]
    if snr_db is not None:
        sigma = np.sqrt(inten.var() / 10.0 ** (snr_db / 10.0))
        inten = inten + sigma * _rng(seed, 11).standard_normal(n_samples)
    codes = quantize12(inten)
    out = {"fmt": fmt, "seed": seed, "n_samples": n_samples, "codes": codes,
           "packed": pack12(codes), "intensity": inten, "field": true_field, "tau0": tau0,
           "theta_c": theta_c}
    out.update(ase)
    return out


B_REF = 12.5e9   # OSNR reference bandwidth (0.1 nm at 1550 nm)


def _detect(field: np.ndarray, fs_sim: float, osnr_db: float | None, seed: int):
    """Square-law detection, with ASE at `osnr_db` added to the field first.

    ASE power in B_REF (both polarisations) = P_sig / OSNR, white, so each
    polarisation carries complex noise of variance P_sig fs_sim / (2 B_REF
    OSNR) per sample at the simulation rate fs_sim."""
    if osnr_db is None:
        return np.abs(field) ** 2, {}
    p_sig = float(np.mean(np.abs(field) ** 2))
    var = p_sig * fs_sim / (2.0 * B_REF * 10.0 ** (osnr_db / 10.0))
    r = _rng(seed, 13)
    sd = np.sqrt(var / 2.0)   # per real component
    n_co = sd * (r.standard_normal(field.size) + 1j * r.standard_normal(field.size))
    n_or = sd * (r.standard_normal(field.size) + 1j * r.standard_normal(field.size))
    return np.abs(field + n_co) ** 2 + np.abs(n_or) ** 2, {"ase_var": var, "p_sig": p_sig}


# Named workloads (sizes and link parameters of the measured configurations).
def pam4_2e20(seed: int = 101, **kw):
    return generate(PAM4, 1 << 20, derive_seed(seed, 0), kw.pop("snr_db", 20.0), **kw)


def kk_2e22(fmt: int = KK_16QAM, seed: int | None = None, index: int = 0, **kw):
    base = seed if seed is not None else (201 if fmt == KK_16QAM else 202)
    return generate(fmt, 1 << 22, derive_seed(base, index), kw.pop("snr_db", 22.0), **kw)


def pam8_91km(index: int, seed: int = 501, n_samples: int = 1 << 22, **kw):
    """PAM-8 over 91 km of SSMF (beta2 = -21.68 ps^2/km), tanh driver, 24 dB."""
    return generate(PAM8, n_samples, derive_seed(seed, index), kw.pop("snr_db", 24.0),
                    tanh_driver=True, beta2_l_s2=-21.68e-27 * 91.0, **kw)


def mixed_batch_formats(count: int, seed: int = 301):
    """Format and SNR of each buffer of a mixed batch: format = SplitMix64 % 5,
    SNR ~ U[14, 26] dB."""
    r = splitmix64(seed, np.arange(count, dtype=np.uint64))
    fmts = (r % np.uint64(5)).astype(int) + 1
    snrs = 14.0 + 12.0 * ((r >> np.uint64(11)).astype(np.float64) / float(1 << 53))
    return list(zip(fmts.tolist(), snrs.tolist()))
