"""ctypes binding of the FP64 receiver oracle (oracle/rxo.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path (paper_2010_14333_amd) never
imports it.  Build with `make -C oracle`.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

PAM2, PAM4, PAM8, KK_QPSK, KK_16QAM = 1, 2, 3, 4, 5
MLP_PARAMS = 64 * 31 + 64 + 64 * 64 + 64 + 64 + 1

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class Out(ctypes.Structure):
    pass


class Cfg(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("mf_taps", ctypes.c_int32), ("ffe_taps", ctypes.c_int32),
                ("prefix", ctypes.c_int32), ("hilbert_taps", ctypes.c_int32),
                ("os_log2", ctypes.c_int32), ("form", ctypes.c_int32),
                ("rounding", ctypes.c_int32), ("equalizer", ctypes.c_int32),
                ("front", ctypes.c_int32), ("rolloff", ctypes.c_double), ("mu", ctypes.c_double),
                ("mu_cma", ctypes.c_double), ("fc_over_fs", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("mlp", _dp), ("force", ctypes.POINTER(ctypes.c_int32)),
                ("frozen", ctypes.POINTER(Out)), ("count_end", ctypes.c_int64),
                ("dd_phase", ctypes.c_int32), ("pad2", ctypes.c_int32)]


Out._fields_ = [("field", _dp), ("shifted", _dp), ("mf", _dp), ("timing", _dp), ("xr", _dp),
                ("soft", _dp), ("taps", _dp), ("phase", _dp), ("ddz", _dp), ("bits", _u8p),
                ("mean_re", ctypes.c_double), ("mean_im", ctypes.c_double),
                ("agc", ctypes.c_double), ("theta0", ctypes.c_double),
                ("lag", ctypes.c_int32), ("rot", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("pad1", ctypes.c_int32), ("nsym", ctypes.c_int64), ("nbits", ctypes.c_int64),
                ("counted_syms", ctypes.c_int64), ("sym_errors", ctypes.c_int64),
                ("counted_bits", ctypes.c_int64), ("bit_errors", ctypes.c_int64)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "librxo.so")
        if not os.path.exists(path):
            raise RuntimeError("oracle/librxo.so is not built (run `make -C oracle`)")
        L = ctypes.CDLL(path)
        L.rxo_process.argtypes = [ctypes.POINTER(Cfg), _u8p, ctypes.c_int64, ctypes.POINTER(Out)]
        L.rxo_process.restype = ctypes.c_int
        L.rxo_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.rxo_splitmix64.restype = ctypes.c_uint64
        L.rxo_unpack12.argtypes = [_u8p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
        L.rxo_fft.argtypes = [_dp, ctypes.c_int64, ctypes.c_int]
        L.rxo_rrc_taps.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, _dp]
        L.rxo_hilbert_taps.argtypes = [ctypes.c_int32, _dp]
        L.rxo_fir_same.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp]
        L.rxo_fir_same_dec2_cplx.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp]
        L.rxo_hilbert_direct.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp]
        L.rxo_hilbert_os.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, ctypes.c_int32, _dp]
        L.rxo_hilbert_fd.argtypes = [_dp, ctypes.c_int64, _dp]
        L.rxo_fd_eq_dec2.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp]
        L.rxo_fd_fir.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, _dp]
        L.rxo_fd_delay.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
        L.rxo_gardner.argtypes = [_dp, ctypes.c_int64, _dp]
        L.rxo_farrow.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
        L.rxo_gardner_sums.argtypes = [_dp, ctypes.c_int64, _dp]
        L.rxo_downshift_rev.argtypes = [ctypes.c_double, ctypes.c_int64]
        L.rxo_downshift_rev.restype = ctypes.c_double
        L.rxo_lms.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _dp,
                              ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32), _dp]
        L.rxo_cma.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int64, _dp, _dp]
        L.rxo_vv_phase.argtypes = [_dp, ctypes.c_int64, _dp]
        L.rxo_decide.argtypes = [ctypes.c_double, ctypes.c_int32]
        L.rxo_decide.restype = ctypes.c_int32
        L.rxo_round_bf16.argtypes = [ctypes.c_double]
        L.rxo_round_bf16.restype = ctypes.c_double
        L.rxo_round_fp16.argtypes = [ctypes.c_double]
        L.rxo_round_fp16.restype = ctypes.c_double
        L.rxo_mlp_forward.argtypes = [_dp, _dp, ctypes.c_int64, ctypes.c_int32, _dp]
        L.rxo_mlp_grad.argtypes = [_dp, _dp, _dp, ctypes.c_int64, _dp]
        L.rxo_mlp_grad.restype = ctypes.c_double
        L.rxo_adam.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def is_kk(fmt):
    return fmt in (KK_QPSK, KK_16QAM)


def bits_per_symbol(fmt):
    return {1: 1, 2: 2, 3: 3, 4: 2, 5: 4}[fmt]


def default_cfg(fmt, seed, **kw) -> dict:
    kk = is_kk(fmt)
    d = dict(fmt=fmt, mf_taps=65 if kk else 33, ffe_taps=21 if kk else 15, prefix=4096,
             hilbert_taps=4097, os_log2=16, form=0, rounding=0, equalizer=0,
             front=0, rolloff=0.1, mu=1e-3, mu_cma=1e-3, fc_over_fs=0.55e9 / 4e9 if kk else 0.0,
             seed=seed, mlp=None, force=None, frozen=None, count_end=0, dd_phase=0, pad2=0)
    d.update(kw)
    return d


def process(fmt, packed, n_samples, seed, want=("bits", "soft"), **kw) -> dict:
    """Run one buffer through the oracle chain.  `want` names the optional
    intermediate arrays to return (field, shifted, mf, timing, xr, soft,
    ddz, taps, phase, bits).  force: optional int32[nsym] decision indices
    the block DD-LMS takes instead of its own (-1: its own)."""
    d = default_cfg(fmt, seed, **kw)
    mlp = d.pop("mlp")
    force = d.pop("force")
    frozen = d.pop("frozen")
    cfg = Cfg(**d)
    keep = []
    n = int(n_samples)
    kk = is_kk(fmt)
    nsym = n // (4 if kk else 2)
    if force is not None:
        force = np.ascontiguousarray(force, dtype=np.int32)
        assert force.size == nsym
        cfg.force = force.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        keep.append(force)
    if mlp is not None:
        mlp = _f64(mlp)
        assert mlp.size == MLP_PARAMS
        cfg.mlp = _p(mlp)
        keep.append(mlp)
    if frozen is not None:
        fz = Out()
        taps = np.ascontiguousarray(np.asarray(frozen["taps"], dtype=np.complex128))
        keep.append(taps)
        fz.taps = taps.view(np.float64).ctypes.data_as(_dp)
        for k in ("mean_re", "mean_im", "agc", "theta0", "lag", "rot", "fallback"):
            setattr(fz, k, frozen[k])
        keep.append(fz)
        cfg.frozen = ctypes.pointer(fz)
    sizes = {"field": 2 * n, "shifted": 2 * n, "mf": n, "timing": n // 512, "xr": n,
             "soft": 2 * nsym if kk else nsym, "ddz": 2 * nsym if kk else nsym, "taps": 2 * d["ffe_taps"],
             "phase": nsym // 128}
    out = Out()
    arrays = {}
    for name in want:
        if name == "bits":
            a = np.zeros((nsym * bits_per_symbol(fmt) + 7) // 8, dtype=np.uint8)
            out.bits = a.ctypes.data_as(_u8p)
        else:
            a = np.zeros(sizes[name], dtype=np.float64)
            setattr(out, name, _p(a))
        arrays[name] = a
    buf = np.ascontiguousarray(packed, dtype=np.uint8)
    assert buf.size == n * 3 // 2
    rc = lib().rxo_process(ctypes.byref(cfg), buf.ctypes.data_as(_u8p), n, ctypes.byref(out))
    if rc != 0:
        raise ValueError(f"oracle rejected the configuration (rc={rc})")
    res = {k: v for k, v in arrays.items()}
    for k in ("field", "shifted", "soft", "ddz", "taps") if kk else ("taps",):
        if k in res:
            res[k] = res[k].view(np.complex128)
    if kk and "mf" in res:
        res["mf"] = res["mf"].view(np.complex128)
    for k in ("mean_re", "mean_im", "agc", "theta0", "lag", "rot", "fallback", "nsym", "nbits",
              "counted_syms", "sym_errors", "counted_bits", "bit_errors"):
        res[k] = getattr(out, k)
    return res


def process_stream(fmt, buffers, seed, hold_back, want=("bits", "soft"), force=None, **kw) -> dict:
    """A contiguous stream cut into buffers (the paper's continuous ADC
    stream with its overlap events): the first buffer is acquired on its own
    (carrier or DC mean, AGC gain, static phase, delay, rotation, prefix
    taps, MLP fallback), then the whole concatenated stream is processed as
    one signal with that acquisition frozen.  A receiver that holds back the
    last `hold_back` samples of every buffer emits the decisions of samples
    [0, total - hold_back): bits and soft values are cut to those symbols and
    errors counted up to them.  force (optional): forced DD-LMS decisions of
    the stream pass (see process)."""
    bufs = [np.ascontiguousarray(b, dtype=np.uint8) for b in buffers]
    ns = [b.size * 2 // 3 for b in bufs]
    sps = 4 if is_kk(fmt) else 2
    acq = process(fmt, bufs[0], ns[0], seed, want=("taps",), **kw)
    total = sum(ns)
    nsym_emit = (total - hold_back) // sps
    if force is not None and len(force) < total // sps:   # forced decisions given for the emitted symbols
        force = np.concatenate([force, np.full(total // sps - len(force), -1, dtype=np.int32)])
    res = process(fmt, np.concatenate(bufs), total, seed, want=tuple(want), frozen=acq, count_end=nsym_emit,
                  force=force, **kw)
    nb = bits_per_symbol(fmt)
    if "bits" in res:
        bits = np.unpackbits(res["bits"], bitorder="little")[: nsym_emit * nb]
        res["bits"] = np.packbits(bits, bitorder="little")
    for k in ("soft", "ddz"):
        if k in res:
            res[k] = res[k][:nsym_emit]
    res["nsym_emitted"] = nsym_emit
    res["acquisition"] = acq
    return res


# --- building blocks -------------------------------------------------------
def splitmix64(seed, k):
    return int(lib().rxo_splitmix64(seed, k))


def unpack12(packed, n):
    out = np.zeros(n, dtype=np.int32)
    buf = np.ascontiguousarray(packed, dtype=np.uint8)
    lib().rxo_unpack12(buf.ctypes.data_as(_u8p), n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out


def fft(x, inverse=False):
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().rxo_fft(a.view(np.float64).ctypes.data_as(_dp), a.size, int(inverse))
    return a


def rrc_taps(k, sps, beta):
    h = np.zeros(k)
    lib().rxo_rrc_taps(k, sps, beta, _p(h))
    return h


def hilbert_taps(ntaps):
    h = np.zeros(ntaps)
    lib().rxo_hilbert_taps(ntaps, _p(h))
    return h


def fir_same(x, h):
    x, h = _f64(x), _f64(h)
    y = np.zeros_like(x)
    lib().rxo_fir_same(_p(x), x.size, _p(h), h.size, _p(y))
    return y


def fir_same_dec2_cplx(x, h):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    h = _f64(h)
    y = np.zeros(x.size // 2, dtype=np.complex128)
    lib().rxo_fir_same_dec2_cplx(x.view(np.float64).ctypes.data_as(_dp), x.size, _p(h), h.size,
                                 y.view(np.float64).ctypes.data_as(_dp))
    return y


def hilbert_direct(l, h):
    l, h = _f64(l), _f64(h)
    y = np.zeros_like(l)
    lib().rxo_hilbert_direct(_p(l), l.size, _p(h), h.size, _p(y))
    return y


def hilbert_os(l, h, log2n):
    l, h = _f64(l), _f64(h)
    y = np.zeros_like(l)
    lib().rxo_hilbert_os(_p(l), l.size, _p(h), h.size, log2n, _p(y))
    return y


def hilbert_fd(l):
    """The paper's block-circular Hilbert transform (1024-point blocks at hop 512)."""
    l = _f64(l)
    y = np.zeros_like(l)
    lib().rxo_hilbert_fd(_p(l), l.size, _p(y))
    return y


def fd_eq_dec2(y, h):
    """Frequency-domain static equaliser h and 512-point IFFT decimation to
    half rate over 1024-point blocks at hop 512 (complex y -> complex y.size / 2)."""
    y = np.ascontiguousarray(y, dtype=np.complex128)
    h = _f64(h)
    x = np.zeros(y.size // 2, dtype=np.complex128)
    lib().rxo_fd_eq_dec2(y.view(np.float64).ctypes.data_as(_dp), y.size, _p(h), h.size,
                         x.view(np.float64).ctypes.data_as(_dp))
    return x


FD_EQ_TAPS = 203
FD_PAM_EQ_TAPS = 503


def fd_fir(x, h):
    """Real FIR h on the frequency-domain blocks (central outputs kept)."""
    x, h = _f64(x), _f64(h)
    y = np.zeros_like(x)
    lib().rxo_fd_fir(_p(x), x.size, _p(h), h.size, _p(y))
    return y


def fd_delay(x, delta):
    """Block b's central samples resampled at t + delta[b] in the frequency domain."""
    x, d = _f64(x), _f64(delta)
    assert d.size >= (x.size + 511) // 512
    y = np.zeros_like(x)
    lib().rxo_fd_delay(_p(x), x.size, _p(d), _p(y))
    return y


def gardner(x):
    x = _f64(x)
    d = np.zeros(x.size // 512)
    lib().rxo_gardner(_p(x), x.size, _p(d))
    return d


def farrow(x, delta):
    x, delta = _f64(x), _f64(delta)
    y = np.zeros_like(x)
    lib().rxo_farrow(_p(x), x.size, _p(delta), _p(y))
    return y


def gardner_sums(x):
    x = _f64(x)
    c = np.zeros(x.size // 512, dtype=np.complex128)
    lib().rxo_gardner_sums(_p(x), x.size, c.view(np.float64).ctypes.data_as(_dp))
    return c


def downshift_rev(r, n):
    return float(lib().rxo_downshift_rev(float(r), int(n)))


def lms(x, w, pos0, count, ref=None, m_axis=2, cplx_axis=True, mu=1e-3, force=None):
    """LMS adaptation of the FFE (rxo_lms): returns (final taps, outputs)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.complex128).copy()
    z = np.zeros(count, dtype=np.complex128)
    rp = None
    if ref is not None:
        ref = np.ascontiguousarray(ref, dtype=np.complex128)
        assert ref.size >= count
        rp = ref.view(np.float64).ctypes.data_as(_dp)
    fp = None
    if force is not None:
        force = np.ascontiguousarray(force, dtype=np.int32)
        assert force.size >= count
        fp = force.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    lib().rxo_lms(x.view(np.float64).ctypes.data_as(_dp), x.size, w.view(np.float64).ctypes.data_as(_dp),
                  w.size, pos0, count, rp, m_axis, int(cplx_axis), mu, fp, z.view(np.float64).ctypes.data_as(_dp))
    return w, z


def cma(x, w, count, mu=1e-3, r2=1.0, nvv=2048):
    """Constant-modulus adaptation (rxo_cma): returns (taps, sum z^4, outputs)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.complex128).copy()
    z = np.zeros(count, dtype=np.complex128)
    s4 = np.zeros(2)
    lib().rxo_cma(x.view(np.float64).ctypes.data_as(_dp), x.size, w.view(np.float64).ctypes.data_as(_dp),
                  w.size, count, mu, r2, nvv, _p(s4), z.view(np.float64).ctypes.data_as(_dp))
    return w, complex(s4[0], s4[1]), z


def vv_phase(s4):
    s4 = np.ascontiguousarray(s4, dtype=np.complex128)
    ph = np.zeros(s4.size)
    lib().rxo_vv_phase(s4.view(np.float64).ctypes.data_as(_dp), s4.size, _p(ph))
    return ph


def decide(v, m):
    return int(lib().rxo_decide(float(v), m))


def round_bf16(v):
    return float(lib().rxo_round_bf16(float(v)))


def round_fp16(v):
    return float(lib().rxo_round_fp16(float(v)))


def mlp_forward(params, x, rounding=0):
    p, x = _f64(params), _f64(x).reshape(-1, 31)
    y = np.zeros(x.shape[0])
    lib().rxo_mlp_forward(_p(p), _p(x), x.shape[0], rounding, _p(y))
    return y


def mlp_grad(params, x, t):
    p, x, t = _f64(params), _f64(x).reshape(-1, 31), _f64(t)
    g = np.zeros(MLP_PARAMS)
    loss = lib().rxo_mlp_grad(_p(p), _p(x), _p(t), x.shape[0], _p(g))
    return loss, g


def adam(p, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays p, m, v."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().rxo_adam(_p(p), _p(m), _p(v), _p(g), p.size, step, lr, b1, b2, eps)
