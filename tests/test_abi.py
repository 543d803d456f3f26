"""The C-ABI library loads and exports every entry point include/rx.h
declares, and the Python mirror of its structs has the C layout (checked
against gcc's view of the header).  No compute calls: no GPU needed."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rx_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def rxlib():
    import paper_2010_14333_amd as rx
    if not os.path.exists(rx.LIB_PATH):
        from paper_2010_14333_amd import build
        build.build()
    return rx


def test_every_declared_symbol_is_exported(rxlib):
    lib = rxlib.lib()
    names = _declared()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(rxlib.EXPORTS)


def test_struct_layout_matches_c(rxlib, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rx.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(rx_params),'
                    ' offsetof(rx_params, rolloff), offsetof(rx_params, seed),'
                    ' offsetof(rx_params, stream), offsetof(rx_params, flags), sizeof(rx_stats));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    P = rxlib.rx_params
    want = [ctypes.sizeof(P), P.rolloff.offset, P.seed.offset, P.stream.offset, P.flags.offset,
            ctypes.sizeof(rxlib.rx_stats)]
    assert got == want


def test_defaults_and_strerror_without_gpu(rxlib):
    p = rxlib.rx_params_default(rxlib.RX_KK_16QAM)
    assert (p.mf_taps, p.ffe_taps, p.prefix_symbols, p.hilbert_taps) == (65, 21, 4096, 4097)
    assert abs(p.carrier_hz - 0.55e9) < 1 and p.struct_size == ctypes.sizeof(rxlib.rx_params)
    q = rxlib.rx_params_default(rxlib.RX_PAM4)
    assert (q.mf_taps, q.ffe_taps) == (33, 15)
    with pytest.raises(rxlib.RxError):
        rxlib.rx_params_default(9)
    assert "invalid" in rxlib.rx_strerror(rxlib.RX_E_INVALID)
    # argument checks run before any device call
    assert rxlib.lib().rx_create(rxlib.RX_PAM4, 2e9, 4e9, None, None) == rxlib.RX_E_INVALID
    h = ctypes.c_void_p()
    assert rxlib.lib().rx_create(rxlib.RX_PAM4, 1e9, 4e9, None, ctypes.byref(h)) == rxlib.RX_E_UNSUPPORTED
    bad = rxlib.rx_params_default(rxlib.RX_KK_16QAM)
    bad.max_samples = 1000
    assert rxlib.lib().rx_create(rxlib.RX_KK_16QAM, 1e9, 4e9, ctypes.byref(bad), ctypes.byref(h)) == rxlib.RX_E_INVALID
