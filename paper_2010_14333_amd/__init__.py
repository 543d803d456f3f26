"""Python binding of librx.so, the MI355X receiver hot path (include/rx.h).

Argument marshalling only: every step of the chain runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  There is no CPU
fallback: importing the binding without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librx.so")

RX_PAM2, RX_PAM4, RX_PAM8, RX_KK_QPSK, RX_KK_16QAM = 1, 2, 3, 4, 5
RX_FP32, RX_BF16, RX_FP16 = 0, 1, 2
RX_EQ_LMS, RX_EQ_MLP = 0, 1
RX_FRONT_OS, RX_FRONT_FD = 0, 1
RX_OK, RX_E_INVALID, RX_E_UNSUPPORTED, RX_E_NOMEM, RX_E_HIP, RX_E_STATE = 0, -1, -2, -3, -4, -5
RX_W_FALLBACK = 1
RX_DEBUG_KEEP = 0x1
(RX_STAGE_FIELD, RX_STAGE_MF, RX_STAGE_XR, RX_STAGE_TIMING, RX_STAGE_SOFT, RX_STAGE_TAPS,
 RX_STAGE_PHASE, RX_STAGE_SCALARS) = range(1, 9)

RX_PROFILE = 0x2
RX_STREAM = 0x4
RX_DD_PHASE = 0x8
HOLD = {RX_PAM2: 12288, RX_PAM4: 12288, RX_PAM8: 12288, RX_KK_QPSK: 4096, RX_KK_16QAM: 4096}
STAGES = ("kk_front", "kk_debug", "pam_sum", "pam_mf", "pam_gavg", "pam_unwrap", "pam_farrow",
          "prefix", "blocks", "kk_vv", "decide", "mlp_infer", "mlp_judge")
RX_MLP_PARAMS = 6273
EXPORTS = ("rx_params_default", "rx_create", "rx_process", "rx_process_batch", "rx_process_batch_host",
           "rx_sync", "rx_stream_reset", "rx_tuning", "rx_errors",
           "rx_errors_reset", "rx_latencies", "rx_debug_fetch", "rx_train_cfg_default", "rx_mlp_param_count",
           "rx_mlp_order_multiplier", "rx_train_mlp", "rx_train_mlp_data", "rx_mlp_grad", "rx_mlp_grad_static",
           "rx_mlp_infer",
           "rx_set_mlp", "rx_get_mlp", "rx_save_weights", "rx_load_weights", "rx_stage_times",
           "rx_destroy", "rx_strerror")


class rx_params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("mf_taps", ctypes.c_int32),
                ("ffe_taps", ctypes.c_int32), ("prefix_symbols", ctypes.c_int32),
                ("hilbert_taps", ctypes.c_int32), ("fft_log2", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("equalizer", ctypes.c_int32),
                ("rolloff", ctypes.c_double), ("mu", ctypes.c_double), ("mu_cma", ctypes.c_double),
                ("carrier_hz", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("max_samples", ctypes.c_uint64), ("stream", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("deadline_s", ctypes.c_double), ("ref_bits", ctypes.c_void_p),
                ("ref_period", ctypes.c_uint64), ("blocks_bc", ctypes.c_int32), ("ffe_gpw", ctypes.c_int32),
                ("dec_syms", ctypes.c_int32), ("front", ctypes.c_int32)]


class rx_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("buffers", "symbols", "bits", "bit_errors", "symbol_errors", "fallbacks", "late_buffers")]


class rx_train_cfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("init_seed", ctypes.c_uint64),
                ("init", ctypes.POINTER(ctypes.c_float))]


class RxError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {rx_strerror(code)} ({code})")
        self.code = code


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2010_14333_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        L.rx_params_default.argtypes = [i32, ctypes.POINTER(rx_params)]
        L.rx_create.argtypes = [i32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(rx_params),
                                ctypes.POINTER(vp)]
        L.rx_process.argtypes = [vp, vp, sz, vp, ctypes.POINTER(sz)]
        L.rx_process_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(sz),
                                       ctypes.POINTER(vp), i32, i32]
        L.rx_process_batch_host.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(sz),
                                            ctypes.POINTER(vp), i32, i32]
        L.rx_sync.argtypes = [vp]
        L.rx_stream_reset.argtypes = [vp]
        L.rx_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.rx_errors.argtypes = [vp, ctypes.POINTER(rx_stats)]
        L.rx_errors_reset.argtypes = [vp]
        L.rx_latencies.argtypes = [vp, ctypes.POINTER(ctypes.c_double), sz, ctypes.POINTER(sz)]
        L.rx_debug_fetch.argtypes = [vp, i32, vp, sz]
        L.rx_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_uint64), i32]
        fp = ctypes.POINTER(ctypes.c_float)
        dp = ctypes.POINTER(ctypes.c_double)
        L.rx_train_cfg_default.argtypes = [ctypes.POINTER(rx_train_cfg)]
        L.rx_mlp_param_count.argtypes = []
        L.rx_mlp_order_multiplier.argtypes = [ctypes.c_int64]
        L.rx_train_mlp.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_uint64),
                                   i32, ctypes.POINTER(rx_train_cfg), dp]
        L.rx_train_mlp_data.argtypes = [vp, vp, vp, sz, ctypes.POINTER(rx_train_cfg), dp]
        L.rx_mlp_grad.argtypes = [vp, vp, vp, sz, vp, dp]
        L.rx_mlp_grad_static.argtypes = [vp, vp, vp, sz, vp, dp]
        L.rx_mlp_infer.argtypes = [vp, vp, sz, vp]
        L.rx_set_mlp.argtypes = [vp, fp]
        L.rx_get_mlp.argtypes = [vp, fp]
        L.rx_save_weights.argtypes = [vp, ctypes.c_char_p]
        L.rx_load_weights.argtypes = [vp, ctypes.c_char_p]
        L.rx_destroy.argtypes = [vp]
        L.rx_destroy.restype = None
        L.rx_strerror.argtypes = [i32]
        L.rx_strerror.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("rx_destroy", "rx_strerror"):
                getattr(L, name).restype = i32
        _LIB = L
    return _LIB


def _check(code: int, where: str) -> int:
    if code < 0:
        raise RxError(code, where)
    return code


def rx_strerror(code: int) -> str:
    return lib().rx_strerror(code).decode()


def rx_params_default(fmt: int) -> rx_params:
    p = rx_params()
    _check(lib().rx_params_default(fmt, ctypes.byref(p)), "rx_params_default")
    return p


def rx_create(fmt: int, baud: float, fs: float, params: rx_params | None = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().rx_create(fmt, baud, fs, ctypes.byref(params) if params is not None else None,
                           ctypes.byref(h)), "rx_create")
    return h.value


def rx_process(h: int, dev_buffer: int, n_samples: int, dev_bits: int) -> int:
    nb = ctypes.c_size_t()
    _check(lib().rx_process(h, dev_buffer, n_samples, dev_bits, ctypes.byref(nb)), "rx_process")
    return nb.value


def rx_process_batch(handles, dev_buffers, n_samples, dev_bits, graph: bool = False) -> int:
    c = len(handles)
    H = (ctypes.c_void_p * c)(*handles)
    B = (ctypes.c_void_p * c)(*dev_buffers)
    N = (ctypes.c_size_t * c)(*n_samples)
    O = (ctypes.c_void_p * c)(*dev_bits)
    return _check(lib().rx_process_batch(H, B, N, O, c, int(graph)), "rx_process_batch")


def rx_process_batch_host(handles, host_buffers, n_samples, host_bits, graph: bool = False) -> int:
    """Host-resident inputs and outputs (addresses of host memory, pinned for
    asynchronous copies); returns without waiting: call rx_sync first."""
    c = len(handles)
    H = (ctypes.c_void_p * c)(*handles)
    B = (ctypes.c_void_p * c)(*host_buffers)
    N = (ctypes.c_size_t * c)(*n_samples)
    O = (ctypes.c_void_p * c)(*host_bits)
    return _check(lib().rx_process_batch_host(H, B, N, O, c, int(graph)), "rx_process_batch_host")


def rx_sync(h: int) -> None:
    _check(lib().rx_sync(h), "rx_sync")


def rx_tuning(h: int) -> dict:
    """The handle's launch shapes (tuned or given)."""
    a = (ctypes.c_int32 * 4)()
    _check(lib().rx_tuning(h, a), "rx_tuning")
    return {"fft_log2": a[0], "blocks_bc": a[1], "ffe_gpw": a[2], "dec_syms": a[3]}


def rx_stream_reset(h: int) -> None:
    _check(lib().rx_stream_reset(h), "rx_stream_reset")


def rx_errors(h: int) -> dict:
    s = rx_stats()
    _check(lib().rx_errors(h, ctypes.byref(s)), "rx_errors")
    return {k: getattr(s, k) for k, _ in rx_stats._fields_}


def rx_errors_reset(h: int) -> None:
    _check(lib().rx_errors_reset(h), "rx_errors_reset")


def rx_latencies(h: int, max_count: int = 1024) -> np.ndarray:
    """Device-measured latencies (microseconds) of the handle's most recent
    buffers, oldest first."""
    us = (ctypes.c_double * max_count)()
    cnt = ctypes.c_size_t()
    _check(lib().rx_latencies(h, us, max_count, ctypes.byref(cnt)), "rx_latencies")
    return np.array(us[: cnt.value])


def rx_debug_fetch(h: int, stage: int, nbytes: int) -> bytes:
    buf = ctypes.create_string_buffer(nbytes)
    _check(lib().rx_debug_fetch(h, stage, buf, nbytes), "rx_debug_fetch")
    return buf.raw


def rx_train_cfg_default() -> rx_train_cfg:
    c = rx_train_cfg()
    _check(lib().rx_train_cfg_default(ctypes.byref(c)), "rx_train_cfg_default")
    return c


def rx_mlp_order_multiplier(n: int) -> int:
    return int(lib().rx_mlp_order_multiplier(n))


def _cfg(cfg, init):
    c = cfg if cfg is not None else rx_train_cfg_default()
    keep = None
    if init is not None:
        keep = np.ascontiguousarray(init, dtype=np.float32)
        assert keep.size == RX_MLP_PARAMS
        c.init = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    return c, keep


def rx_train_mlp(h: int, dev_buffers, n_samples, seeds, cfg=None, init=None) -> float:
    c, keep = _cfg(cfg, init)
    k = len(dev_buffers)
    B = (ctypes.c_void_p * k)(*dev_buffers)
    N = (ctypes.c_size_t * k)(*n_samples)
    S = (ctypes.c_uint64 * k)(*seeds)
    loss = ctypes.c_double()
    _check(lib().rx_train_mlp(h, B, N, S, k, ctypes.byref(c), ctypes.byref(loss)), "rx_train_mlp")
    del keep
    return loss.value


def rx_train_mlp_data(h: int, dev_x: int, dev_t: int, n: int, cfg=None, init=None) -> float:
    c, keep = _cfg(cfg, init)
    loss = ctypes.c_double()
    _check(lib().rx_train_mlp_data(h, dev_x, dev_t, n, ctypes.byref(c), ctypes.byref(loss)), "rx_train_mlp_data")
    del keep
    return loss.value


def rx_mlp_grad(h: int, dev_x: int, dev_t: int, n: int, dev_grad: int) -> float:
    loss = ctypes.c_double()
    _check(lib().rx_mlp_grad(h, dev_x, dev_t, n, dev_grad, ctypes.byref(loss)), "rx_mlp_grad")
    return loss.value


def rx_mlp_grad_static(h: int, dev_x: int, dev_t: int, n: int, dev_grad: int) -> float:
    """rx_mlp_grad with its partials in the library's static device array
    (no allocation; n <= 8192)."""
    loss = ctypes.c_double()
    _check(lib().rx_mlp_grad_static(h, dev_x, dev_t, n, dev_grad, ctypes.byref(loss)), "rx_mlp_grad_static")
    return loss.value


def rx_mlp_infer(h: int, dev_x: int, n: int, dev_y: int) -> None:
    _check(lib().rx_mlp_infer(h, dev_x, n, dev_y), "rx_mlp_infer")


def rx_set_mlp(h: int, params) -> None:
    a = np.ascontiguousarray(params, dtype=np.float32)
    assert a.size == RX_MLP_PARAMS
    _check(lib().rx_set_mlp(h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "rx_set_mlp")


def rx_get_mlp(h: int) -> np.ndarray:
    a = np.zeros(RX_MLP_PARAMS, dtype=np.float32)
    _check(lib().rx_get_mlp(h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "rx_get_mlp")
    return a


def rx_save_weights(h: int, path: str) -> None:
    _check(lib().rx_save_weights(h, path.encode()), "rx_save_weights")


def rx_load_weights(h: int, path: str) -> None:
    _check(lib().rx_load_weights(h, path.encode()), "rx_load_weights")


def rx_stage_times(h: int, reset: bool = False) -> dict:
    """{stage name: (total ms, launches)} since the last reset."""
    n = len(STAGES)
    if reset:
        _check(lib().rx_stage_times(h, None, None, n), "rx_stage_times")
        return {}
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_uint64 * n)()
    _check(lib().rx_stage_times(h, ms, cnt, n), "rx_stage_times")
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}


def rx_destroy(h: int) -> None:
    lib().rx_destroy(h)


# ---- convenience wrapper on torch tensors (marshalling only) -------------
FMT_RATE = {RX_PAM2: (2e9, 2), RX_PAM4: (2e9, 2), RX_PAM8: (2e9, 2), RX_KK_QPSK: (1e9, 4),
            RX_KK_16QAM: (1e9, 4)}
BPS = {RX_PAM2: 1, RX_PAM4: 2, RX_PAM8: 3, RX_KK_QPSK: 2, RX_KK_16QAM: 4}


class Receiver:
    """One rx handle; buffers and bit outputs are torch uint8 device tensors."""

    def __init__(self, fmt: int, seed: int, max_samples: int = 1 << 22, debug: bool = False,
                 stream=None, dd_phase: bool = False, **overrides):
        self.fmt = fmt
        self.baud, self.sps = FMT_RATE[fmt]
        p = rx_params_default(fmt)
        p.seed = seed
        p.max_samples = max_samples
        p.flags = (RX_DEBUG_KEEP if debug else 0) | (RX_DD_PHASE if dd_phase else 0)
        p.stream = stream.cuda_stream if stream is not None else None
        for k, v in overrides.items():
            if not any(k == f[0] for f in rx_params._fields_):
                raise TypeError(f"rx_params has no field {k!r}")
            setattr(p, k, v)
        self.params = p
        self.h = rx_create(fmt, self.baud, 4e9, p)

    def bits_bytes(self, n_samples: int) -> int:
        return (n_samples // self.sps * BPS[self.fmt] + 7) // 8

    def process(self, buf, n_samples: int, out=None):
        """Bits of the buffer (a stream handle: of the symbols this call
        emits, as many bytes as they fill)."""
        import torch
        if out is None:
            out = torch.empty(self.bits_bytes(n_samples), dtype=torch.uint8, device=buf.device)
        nb = ctypes.c_size_t()
        self.last_status = _check(lib().rx_process(self.h, buf.data_ptr(), n_samples, out.data_ptr(),
                                                   ctypes.byref(nb)), "rx_process")
        self.last_bits = nb.value
        return out[: (nb.value + 7) // 8]

    def errors(self) -> dict:
        return rx_errors(self.h)

    def reset(self) -> None:
        rx_errors_reset(self.h)

    def latencies(self) -> np.ndarray:
        return rx_latencies(self.h)

    def fetch(self, stage: int, n_samples: int) -> np.ndarray:
        nsym = n_samples // self.sps
        kk = self.fmt in (RX_KK_QPSK, RX_KK_16QAM)
        spec = {RX_STAGE_FIELD: (np.complex64, n_samples),
                RX_STAGE_MF: (np.complex64, n_samples // 2) if kk else (np.float32, n_samples),
                RX_STAGE_XR: (np.float32, n_samples), RX_STAGE_TIMING: (np.float32, n_samples // 512),
                RX_STAGE_SOFT: (np.complex64, nsym) if kk else (np.float32, nsym),
                RX_STAGE_TAPS: (np.complex64, self.params.ffe_taps),
                RX_STAGE_PHASE: (np.float32, nsym // 128), RX_STAGE_SCALARS: (np.float64, 8)}[stage]
        dt, cnt = spec
        raw = rx_debug_fetch(self.h, stage, np.dtype(dt).itemsize * cnt)
        return np.frombuffer(raw, dtype=dt).copy()

    def close(self) -> None:
        if self.h:
            rx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
