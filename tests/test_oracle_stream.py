"""Pins of the oracle's contiguous-stream mode (the paper's continuous ADC
stream, buffers joined by overlap events and a clock-phase unwrap that
continues from the previous buffer): a stream is acquired on its first
buffer and then processed as one signal, and a receiver that holds back the
last D samples of each buffer emits only decisions no later sample can
change."""
import numpy as np
import pytest

import synth

HOLD = {2: 12288, 5: 4096}   # hold-back in samples (PAM, KK), as the library uses


def _cut(packed, ns):
    out, o = [], 0
    for n in ns:
        out.append(packed[o * 3 // 2:(o + n) * 3 // 2])
        o += n
    return out


@pytest.mark.parametrize("fmt", [2, 5])
def test_stream_of_one_buffer_is_the_buffer(oracle_lib, fmt):
    """A stream of one buffer, acquired on itself, is that buffer processed
    on its own (the frozen values are the ones it would compute)."""
    n = 1 << 18
    g = synth.generate(fmt, n, 5100 + fmt, 18.0)
    ind = oracle_lib.process(fmt, g["packed"], n, g["seed"], want=("bits", "soft"))
    st = oracle_lib.process_stream(fmt, [g["packed"]], g["seed"], HOLD[fmt])
    k = st["nsym_emitted"]
    assert np.array_equal(st["soft"], ind["soft"][:k])


@pytest.mark.parametrize("fmt", [2, 5])
def test_emitted_decisions_do_not_depend_on_later_samples(oracle_lib, fmt):
    """What a receiver emits after holding back D samples is final: the
    stream's first buffer's emitted soft values equal that buffer processed
    on its own, and a stream of two buffers gives the same soft values on
    all it emitted as the same stream with a third buffer appended (the
    hold-back covers the Hilbert and matched-filter reach, the timing
    detector's averaging window, the FFE span and delay, the DD-LMS block
    and the carrier-phase window)."""
    n = 3 << 18
    g = synth.generate(fmt, n, 5200 + fmt, 18.0)
    ns = [1 << 18] * 3
    bufs = _cut(g["packed"], ns)
    ind = oracle_lib.process(fmt, bufs[0], ns[0], g["seed"], want=("bits", "soft"))
    s2 = oracle_lib.process_stream(fmt, bufs[:2], g["seed"], HOLD[fmt])
    s3 = oracle_lib.process_stream(fmt, bufs, g["seed"], HOLD[fmt])
    sps = 4 if fmt >= 4 else 2
    k1 = (ns[0] - HOLD[fmt]) // sps
    assert np.max(np.abs(s2["soft"][:k1] - ind["soft"][:k1])) < 1e-9
    k2 = s2["nsym_emitted"]
    assert np.max(np.abs(s3["soft"][:k2] - s2["soft"])) < 1e-9
    # and the last emitted symbols do change if the hold-back is cut short
    short = (ns[0] + ns[1] - 1024) // sps
    s2b = oracle_lib.process_stream(fmt, bufs[:2], g["seed"], 1024)
    assert np.max(np.abs(s3["soft"][k2:short] - s2b["soft"][k2:short])) > 1e-6


@pytest.mark.parametrize("fmt", [2, 5])
def test_noiseless_stream_error_free_across_buffers(oracle_lib, fmt):
    """A continuous noiseless signal cut into four buffers of different
    lengths: no errors on any emitted symbol, across every boundary."""
    n = 1 << 20
    kw = {"drive": 0.1} if fmt < 4 else {}
    g = synth.generate(fmt, n, 5300 + fmt, None, **kw)
    ns = [1 << 18, 3 << 17, 5 << 16, n - (1 << 18) - (3 << 17) - (5 << 16)]
    st = oracle_lib.process_stream(fmt, _cut(g["packed"], ns), g["seed"], HOLD[fmt])
    sps = 4 if fmt >= 4 else 2
    assert st["counted_syms"] == st["nsym_emitted"] - 4096 - 64
    assert st["bit_errors"] == 0
    assert st["nsym_emitted"] == (n - HOLD[fmt]) // sps
