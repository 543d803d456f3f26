"""Contiguous streams (RX_STREAM) through the C ABI: a continuous signal cut
into buffers of several lengths and processed buffer by buffer on one
handle emits the decisions of the whole signal processed at once with the
stream's acquisition (the oracle's stream mode), symbol by symbol; the cut
does not matter; streams batch with other handles; a repeated pattern
streamed many times keeps giving the same decisions."""
import numpy as np
import pytest

import oracle
import parity
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2010_14333_amd as rx
    rx.lib()
    return rx


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _cut(packed, ns):
    out, o = [], 0
    for n in ns:
        out.append(packed[o * 3 // 2:(o + n) * 3 // 2])
        o += n
    return out


def _stream_gpu(rx, fmt, seed, bufs, ns, **opts):
    r = rx.Receiver(fmt, seed, max_samples=max(ns), flags=rx.RX_STREAM, **opts)
    bits = []
    for b, n in zip(bufs, ns):
        out = r.process(_dev(b), n)
        bits.append(np.unpackbits(out.cpu().numpy(), bitorder="little")[: r.last_bits])
    e = r.errors()
    r.close()
    return np.packbits(np.concatenate(bits), bitorder="little"), sum(len(b) for b in bits), e


STREAMS = [
    (5, 22.0, {}),
    (4, 14.0, {}),
    (2, 16.0, {}),
    (3, 22.0, {}),
    (1, 12.0, {}),
]


@pytest.mark.parametrize("fmt,snr,opts", STREAMS)
def test_stream_equals_the_signal_processed_at_once(rx, fmt, snr, opts):
    n = 1 << 20
    print(f"[stream] fmt={fmt} snr={snr}", flush=True)
    g = synth.generate(fmt, n, 6000 + fmt, snr)
    ns = [1 << 18, 3 << 16, 5 << 16, n - (1 << 18) - (3 << 16) - (5 << 16)]
    bufs = _cut(g["packed"], ns)
    hold = rx.HOLD[fmt]
    bits, nbits, e = _stream_gpu(rx, fmt, g["seed"], bufs, ns, **opts)
    kk = fmt >= 4
    sps = 4 if kk else 2
    nsym = (n - hold) // sps
    assert nbits == nsym * parity.bps(fmt)
    want = ("bits", "soft", "ddz")
    o = oracle.process_stream(fmt, bufs, g["seed"], hold, want=want)
    dec = parity.compare_decisions(
        fmt, bits, o, nsym, 128 if kk else 256,
        rerun=lambda f: oracle.process_stream(fmt, bufs, g["seed"], hold, want=want, force=f))
    print(f"[stream]   mismatches {dec.mismatch}, forced {dec.forced}, bit errors {e['bit_errors']} / "
          f"{dec.oracle['bit_errors']} of {e['bits']}", flush=True)
    assert not dec.untolerated, dec.untolerated[:10]
    assert e["buffers"] == len(ns) and e["bits"] == dec.oracle["counted_bits"]
    assert abs(e["bit_errors"] - dec.oracle["bit_errors"]) <= dec.tolerated_bits


@pytest.mark.parametrize("fmt", [5, 2])
def test_the_cut_does_not_matter(rx, fmt):
    """The same stream cut two ways after the same first buffer: the emitted
    bits agree except where a decision lies on a threshold (the front end's
    overlap-save frames fall elsewhere, so its rounding differs)."""
    n = 3 << 18
    g = synth.generate(fmt, n, 6100 + fmt, 20.0)
    a = [1 << 18, 1 << 18, 1 << 18]
    b = [1 << 18, 5 << 16, 3 << 16]
    ba, nba, ea = _stream_gpu(rx, fmt, g["seed"], _cut(g["packed"], a), a)
    bb, nbb, eb = _stream_gpu(rx, fmt, g["seed"], _cut(g["packed"], b), b)
    assert nba == nbb
    sps = 4 if fmt >= 4 else 2
    nsym = nba // parity.bps(fmt)
    ga = parity.symbols_from_bits(ba, fmt, nsym)
    gb = parity.symbols_from_bits(bb, fmt, nsym)
    diff = np.nonzero(ga != gb)[0]
    print(f"[stream] cut invariance fmt={fmt}: {diff.size} differing symbols of {nsym}", flush=True)
    assert diff.size <= 2
    assert abs(ea["bit_errors"] - eb["bit_errors"]) <= 2 * parity.bps(fmt) and ea["bits"] == eb["bits"]


def test_streams_batch_with_other_handles(rx):
    """Two streams (KK and PAM) and an independent buffer in one batched
    launch sequence per step give the bits of the streams processed alone."""
    import torch
    n = 1 << 19
    gk = synth.generate(5, n, 6201, 20.0)
    gp = synth.generate(2, n, 6202, 18.0)
    gi = synth.generate(4, 1 << 18, 6203, 16.0)
    ns = [1 << 18, 1 << 18]
    ref_k = _stream_gpu(rx, 5, gk["seed"], _cut(gk["packed"], ns), ns)
    ref_p = _stream_gpu(rx, 2, gp["seed"], _cut(gp["packed"], ns), ns)
    rk = rx.Receiver(5, gk["seed"], max_samples=1 << 18, flags=rx.RX_STREAM)
    rp = rx.Receiver(2, gp["seed"], max_samples=1 << 18, flags=rx.RX_STREAM)
    ri = rx.Receiver(4, gi["seed"], max_samples=1 << 18)
    outs = [torch.zeros(r.bits_bytes(1 << 18), dtype=torch.uint8, device="cuda:0") for r in (rk, rp, ri)]
    got_k, got_p = [], []
    bi = _dev(gi["packed"])
    for step, (bk, bp) in enumerate(zip(_cut(gk["packed"], ns), _cut(gp["packed"], ns))):
        dk, dp = _dev(bk), _dev(bp)
        rx.rx_process_batch([rk.h, rp.h, ri.h], [dk.data_ptr(), dp.data_ptr(), bi.data_ptr()], [1 << 18] * 3,
                            [o.data_ptr() for o in outs])
        torch.cuda.synchronize()
        hk = (1 << 18) - (4096 if step == 0 else 0)
        hp = (1 << 18) - (12288 if step == 0 else 0)
        got_k.append(np.unpackbits(outs[0].cpu().numpy(), bitorder="little")[: hk // 4 * 4])
        got_p.append(np.unpackbits(outs[1].cpu().numpy(), bitorder="little")[: hp // 2 * 2])
    with pytest.raises(rx.RxError):   # no graph replay for streams
        rx.rx_process_batch([rk.h, ri.h], [dk.data_ptr(), bi.data_ptr()], [1 << 18] * 2,
                            [outs[0].data_ptr(), outs[2].data_ptr()], graph=True)
    assert np.array_equal(np.packbits(np.concatenate(got_k), bitorder="little"), ref_k[0])
    assert np.array_equal(np.packbits(np.concatenate(got_p), bitorder="little"), ref_p[0])
    ek, ep = rk.errors(), rp.errors()
    assert ek["bit_errors"] == ref_k[2]["bit_errors"] and ep["bit_errors"] == ref_p[2]["bit_errors"]
    for r in (rk, rp, ri):
        r.close()


def test_repeated_pattern_soak_is_stable(rx):
    """A transmitter repeating one pattern (reference period = the pattern's
    symbols) streamed 48 times: after the first buffer every buffer's input
    (tail + pattern) is the same signal, so every later call emits the same
    bits and the same error count; the stream's first three buffers against
    the oracle's stream mode.  The pattern is 1,024,000 samples: a multiple
    of 1024 and of 80, so the tone offset (11/80 of the sample rate) also
    completes whole cycles and the repeated signal stays continuous."""
    import torch
    n = 1024000
    g = synth.generate(5, n, 6301, 20.0)
    r = rx.Receiver(5, g["seed"], max_samples=n, flags=rx.RX_STREAM, ref_period=n // 4)
    d = _dev(g["packed"])
    out = torch.zeros(r.bits_bytes(n), dtype=torch.uint8, device="cuda:0")
    bits, errs = [], []
    for i in range(48):
        r.process(d, n, out=out)
        bits.append(np.unpackbits(out.cpu().numpy(), bitorder="little")[: r.last_bits].copy())
        e = r.errors()
        errs.append(e["bit_errors"])
        r.reset()
    r.close()
    for i in range(2, 48):
        assert np.array_equal(bits[i], bits[1]), i
        assert errs[i] == errs[1], i
    # the first three buffers against the oracle (the pattern repeated three times)
    want = ("bits", "soft", "ddz")
    bufs = [g["packed"]] * 3
    hold = rx.HOLD[5]
    nsym = (3 * n - hold) // 4
    o = oracle.process_stream(5, bufs, g["seed"], hold, want=want)
    # the oracle's reference does not repeat: compare decisions, not counts
    got = np.packbits(np.concatenate(bits[:3]), bitorder="little")
    dec = parity.compare_decisions(5, got, o, nsym, 128,
                                   rerun=lambda f: oracle.process_stream(5, bufs, g["seed"], hold, want=want, force=f))
    assert not dec.untolerated, dec.untolerated[:10]
    print(f"[stream] soak: {errs[1]} bit errors per buffer after the first ({errs[0]} in it)", flush=True)
