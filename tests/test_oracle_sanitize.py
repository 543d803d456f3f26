"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is the judge of every parity test, so an out-of-bounds read in it
(an edge case of the overlap-save framing, the timing interpolator's
neighbours, the block windows) would hand the tests a wrong expected value
silently.  tests/sanitize/rxo_san_main.c runs each chain, the stream form
and the building blocks with every output at its documented size; the
sanitized build must report nothing and give the bits of the normal build.
Host code only, built with gcc."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N = 1 << 16


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path_factory.mktemp("san") / "rxo_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "rxo.c"),
                    os.path.join(ROOT, "tests", "sanitize", "rxo_san_main.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, text=True)
    return exe


def _run(exe, tmp_path, fmt, packed, seed, rounding=0, form=0, mlp=None):
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    hdr = np.array([fmt, rounding, form, 1 if mlp is not None else 0], dtype=np.int32).tobytes()
    hdr += np.array([N], dtype=np.int64).tobytes() + np.array([seed], dtype=np.uint64).tobytes()
    body = (np.asarray(mlp, dtype=np.float64).tobytes() if mlp is not None else b"") + \
        np.ascontiguousarray(packed, dtype=np.uint8).tobytes()
    inp.write_bytes(hdr + body)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([exe, str(inp), str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-3000:]
    raw = out.read_bytes()
    nbytes = (N // synth.sps_of(fmt) * oracle.bits_per_symbol(fmt) + 7) // 8
    passes = []
    for p in range(2):
        o = p * (24 + nbytes)
        head = np.frombuffer(raw[o:o + 24], dtype=np.int64)
        passes.append((head, np.frombuffer(raw[o + 24:o + 24 + nbytes], dtype=np.uint8)))
    return passes


@pytest.mark.parametrize("fmt,rounding,form", [(1, 0, 0), (2, 0, 0), (3, 0, 0), (4, 0, 0), (5, 0, 0),
                                               (5, 1, 1), (2, 2, 1)])
def test_oracle_clean_under_sanitizers(sanitized, tmp_path, fmt, rounding, form):
    g = synth.generate(fmt, N, seed=900 + fmt, snr_db=18.0)
    (h1, b1), (h2, _) = _run(sanitized, tmp_path, fmt, g["packed"], g["seed"], rounding, form)
    ref = oracle.process(fmt, g["packed"], N, g["seed"], want=("bits",), os_log2=14,
                         rounding=rounding, form=form)
    assert np.array_equal(b1, ref["bits"])
    assert (h1[1], h1[2]) == (ref["sym_errors"], ref["bit_errors"])
    assert h2[0] == h1[0]


def test_oracle_mlp_form_clean_under_sanitizers(sanitized, tmp_path):
    g = synth.generate(3, N, seed=931, snr_db=20.0)
    rng = np.random.default_rng(5)
    p = rng.normal(0.0, 0.1, oracle.MLP_PARAMS)
    (h1, b1), _ = _run(sanitized, tmp_path, 3, g["packed"], g["seed"], 1, 0, mlp=p)
    ref = oracle.process(3, g["packed"], N, g["seed"], want=("bits",), os_log2=14, rounding=1,
                         equalizer=1, mlp=p)
    assert np.array_equal(b1, ref["bits"])
    assert (h1[1], h1[2]) == (ref["sym_errors"], ref["bit_errors"])
