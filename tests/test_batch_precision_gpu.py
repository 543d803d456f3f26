"""Batched mixed-format processing, hipGraph replay, FFT-size invariance and
the BF16/FP16 precision form, through the C ABI."""
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
    return torch.from_numpy(a).to("cuda:0")


def test_mixed_batch_equals_single_buffers_and_graph_replays(rx):
    import torch
    n = 1 << 18
    fmts = [5, 1, 4, 3, 2, 5]
    gens = [synth.generate(f, n, 700 + i, 18.0 + i) for i, f in enumerate(fmts)]
    recs = [rx.Receiver(f, g["seed"], max_samples=n) for f, g in zip(fmts, gens)]
    bufs = [_dev(g["packed"]) for g in gens]
    single = [r.process(b, n).cpu().numpy() for r, b in zip(recs, bufs)]
    torch.cuda.synchronize()
    e_single = [r.errors() for r in recs]
    outs = [torch.zeros(r.bits_bytes(n), dtype=torch.uint8, device="cuda:0") for r in recs]
    args = ([r.h for r in recs], [b.data_ptr() for b in bufs], [n] * len(recs), [o.data_ptr() for o in outs])
    rx.rx_process_batch(*args, graph=False)
    torch.cuda.synchronize()
    for o, s in zip(outs, single):
        assert np.array_equal(o.cpu().numpy(), s)
    for rep in range(3):
        for o in outs:
            o.zero_()
        junk = torch.randn(1 << 20, device="cuda:0").sum()   # eager work between replays
        rx.rx_process_batch(*args, graph=True)
        torch.cuda.synchronize()
        for o, s in zip(outs, single):
            assert np.array_equal(o.cpu().numpy(), s), f"replay {rep}"
        del junk
    for r, e in zip(recs, e_single):
        e5 = r.errors()
        assert e5["buffers"] == 5 * e["buffers"] and e5["bit_errors"] == 5 * e["bit_errors"]
    # one buffer of the batch against the oracle
    o = oracle.process(fmts[0], gens[0]["packed"], n, gens[0]["seed"], want=("bits", "soft"))
    _, _, untol = parity.compare_decisions(fmts[0], single[0], o["bits"], o["soft"], n // 4, 128)
    assert not untol
    for r in recs:
        r.close()


def test_batch_rejects_repeated_handle_and_bad_count(rx):
    import torch
    n = 1 << 16
    r = rx.Receiver(5, 1, max_samples=n)
    b = torch.zeros(n * 3 // 2, dtype=torch.uint8, device="cuda:0")
    o = torch.zeros(r.bits_bytes(n), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(rx.RxError):
        rx.rx_process_batch([r.h, r.h], [b.data_ptr()] * 2, [n] * 2, [o.data_ptr()] * 2)
    with pytest.raises(rx.RxError):
        rx.rx_process_batch([], [], [], [])
    r.close()


def test_fft_size_invariance(rx):
    """The Hilbert transform is a fixed finite kernel, so both overlap-save
    FFT sizes give the same field up to rounding and the same decisions."""
    n = 1 << 19
    g = synth.generate(5, n, 4321, 22.0)
    res = {}
    for lg in (13, 14):
        r = rx.Receiver(5, g["seed"], max_samples=n, debug=True, fft_log2=lg)
        bits = r.process(_dev(g["packed"]), n).cpu().numpy()
        res[lg] = (bits, r.fetch(rx.RX_STAGE_FIELD, n), r.errors())
        r.close()
    assert parity.rel_rms(res[13][1], res[14][1]) < 1e-6
    o = oracle.process(5, g["packed"], n, g["seed"], want=("bits", "soft"))
    for lg in (13, 14):
        _, tol, untol = parity.compare_decisions(5, res[lg][0], o["bits"], o["soft"], n // 4, 128)
        assert not untol and abs(res[lg][2]["bit_errors"] - o["bit_errors"]) <= tol


PREC_NEAR = 2e-2   # one-ulp narrow-operand disagreements can move an output this far


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("n,seed", [(1 << 18, 51), (1 << 24, 401)])
def test_precision_form(rx, prec, n, seed):
    """BF16 (1) / FP16 (2) Toeplitz-GEMM matched filter and frozen-tap FFE on
    MFMA vs the oracle run with the same operand rounding (FP64 accumulate);
    the error against the unrounded FP64 chain is reported."""
    print(f"[precision] prec={prec} n={n} seed={seed}", flush=True)
    g = synth.generate(5, n, synth.derive_seed(seed, 0), 22.0)
    s = g["seed"]
    o_r = oracle.process(5, g["packed"], n, s, want=("bits", "soft", "mf", "taps"), form=1, rounding=prec)
    r = rx.Receiver(5, s, max_samples=n, debug=True, precision=prec)
    bits = r.process(_dev(g["packed"]), n).cpu().numpy()
    sc = r.fetch(rx.RX_STAGE_SCALARS, n)
    mf = r.fetch(rx.RX_STAGE_MF, n)   # already AGC'd
    soft = r.fetch(rx.RX_STAGE_SOFT, n)
    err = r.errors()
    r.close()
    assert int(sc[4]) == o_r["lag"] and int(sc[5]) == o_r["rot"]
    rep = {"mf": parity.rel_rms(mf, o_r["mf"]), "soft": parity.rel_rms(soft, o_r["soft"])}
    assert rep["mf"] < 1e-4 and rep["soft"] < 1e-3, rep
    nsym = n // 4
    g_sym = parity.symbols_from_bits(bits, 5, nsym)
    o_sym = parity.symbols_from_bits(o_r["bits"], 5, nsym)
    dist = parity.threshold_distance(o_r["soft"], 5)
    bad = np.nonzero(g_sym != o_sym)[0]
    assert np.all(dist[bad] <= PREC_NEAR), dist[bad][:10]
    tol_bits = int(sum(bin(int(a ^ b)).count("1") for a, b in zip(g_sym[bad], o_sym[bad])))
    assert abs(err["bit_errors"] - o_r["bit_errors"]) <= tol_bits
    # stated error against the unrounded FP64 chain (same frozen-tap definition)
    o_f = oracle.process(5, g["packed"], n, s, want=("soft",), form=1, rounding=0)
    rep["soft_vs_fp64_frozen"] = parity.rel_rms(soft, o_f["soft"])
    rep["ber_gpu"] = err["bit_errors"] / err["bits"]
    rep["ber_fp64_frozen"] = o_f["bit_errors"] / o_f["counted_bits"]
    rep["mismatch"] = int(bad.size)
    print(f"[precision]   {rep}", flush=True)
    assert rep["soft_vs_fp64_frozen"] < 2e-2
