"""Launch shapes (the tuner's choices) change the layout of the work, never
the result: every DD-LMS chunk length, FFE grouping and decision workgroup
size gives bit-identical bits and counts, and both overlap-save FFT sizes
match the oracle; the tuner's choices come from its JSON cache file when it
holds them."""
import ast
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import parity
import synth

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2010_14333_amd as rx
    rx.lib()
    return rx


def _run(rx, fmt, g, n, **shapes):
    import torch
    r = rx.Receiver(fmt, g["seed"], max_samples=n, **shapes)
    got = rx.rx_tuning(r.h)
    for k, v in shapes.items():
        if k in got:
            assert got[k] == v, (k, got)
    bits = r.process(torch.from_numpy(g["packed"]).to("cuda:0"), n).cpu().numpy()
    e = r.errors()
    r.close()
    return bits, {k: v for k, v in e.items() if k != "late_buffers"}


@pytest.mark.parametrize("fmt,prec", [(5, 0), (2, 0), (5, 1)])
def test_every_shape_gives_the_same_bits(rx, fmt, prec):
    n = 1 << 18
    g = synth.generate(fmt, n, 7000 + fmt + 10 * prec, 16.0)
    kk = fmt >= 4
    base = dict(fft_log2=14, blocks_bc=8, ffe_gpw=8, dec_syms=2048, precision=prec)
    ref = _run(rx, fmt, g, n, **base)
    knob = "ffe_gpw" if prec else "blocks_bc"
    for k, vals in ((knob, (4, 16)), ("dec_syms", (1024, 4096))):
        for v in vals:
            got = _run(rx, fmt, g, n, **{**base, k: v})
            assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (k, v)
    if kk and not prec:
        # the other FFT size: the same chain up to rounding, against the oracle
        want = ("bits", "soft", "ddz")
        o = oracle.process(fmt, g["packed"], n, g["seed"], want=want)
        for lg in (13, 14):
            bits, e = _run(rx, fmt, g, n, **{**base, "fft_log2": lg})
            dec = parity.compare_decisions(fmt, bits, o, n // 4, 128,
                                           rerun=lambda f: oracle.process(fmt, g["packed"], n, g["seed"], want=want,
                                                                          force=f))
            assert not dec.untolerated
            assert abs(e["bit_errors"] - dec.oracle["bit_errors"]) <= dec.tolerated_bits


def test_tuned_shapes_come_from_the_cache_file(rx, tmp_path):
    """A cache file holding a choice for this GPU's KK/FP32/21-tap chain is
    used as it is (no timing), in a fresh process."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    path = tmp_path / "tune.json"
    choice = {"fft_log2": 13, "blocks_bc": 16, "ffe_gpw": 4, "dec_syms": 1024}
    path.write_text(json.dumps({f"{arch}|kk|0|21": choice}))
    prog = ("import sys; sys.path.insert(0, %r); import paper_2010_14333_amd as rx; "
            "r = rx.Receiver(rx.RX_KK_16QAM, 1, max_samples=1 << 16); print(rx.rx_tuning(r.h)); r.close()" % ROOT)
    env = dict(os.environ, RX_TUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    got = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    # an FP32 KK handle has no precision-form FFE: its ffe_gpw is not used (reported as the default)
    assert {k: got[k] for k in ("fft_log2", "blocks_bc", "dec_syms")} == \
        {k: choice[k] for k in ("fft_log2", "blocks_bc", "dec_syms")}, got
    # a key it lacks is tuned and added to the file
    prog2 = ("import sys; sys.path.insert(0, %r); import paper_2010_14333_amd as rx; "
             "r = rx.Receiver(rx.RX_PAM4, 1, max_samples=1 << 16); print(rx.rx_tuning(r.h)); r.close()" % ROOT)
    out = subprocess.run([sys.executable, "-c", prog2], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    saved = json.loads(path.read_text())
    assert saved[f"{arch}|kk|0|21"] == choice and f"{arch}|pam|0|15" in saved
    print(f"[tuning] PAM-4 tuned: {saved[f'{arch}|pam|0|15']}", flush=True)
