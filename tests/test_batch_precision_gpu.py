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


@pytest.mark.parametrize("fronts", [(0, 0, 0, 0, 0, 0), (1, 1, 0, 0, 1, 0)], ids=["os", "fd_and_os"])
def test_mixed_batch_equals_single_buffers_and_graph_replays(rx, fronts):
    """fronts: per buffer, the time-domain front end (0) or the paper's
    frequency-domain one (1); a batch mixing them launches each group's
    kernels separately and must equal the buffers processed alone."""
    import torch
    n = 1 << 18
    fmts = [5, 1, 4, 3, 2, 5]
    gens = [synth.generate(f, n, 700 + i, 18.0 + i) for i, f in enumerate(fmts)]
    recs = [rx.Receiver(f, g["seed"], max_samples=n, front=fr) for f, g, fr in zip(fmts, gens, fronts)]
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
    want = ("bits", "soft", "ddz")
    o = oracle.process(fmts[0], gens[0]["packed"], n, gens[0]["seed"], want=want, front=fronts[0])
    dec = parity.compare_decisions(
        fmts[0], single[0], o, n // 4, 128,
        rerun=lambda f: oracle.process(fmts[0], gens[0]["packed"], n, gens[0]["seed"], want=want, force=f,
                                       front=fronts[0]))
    assert not dec.untolerated
    for r in recs:
        r.close()


def test_kk_batch_of_unequal_buffers_through_the_work_queue(rx):
    """Eight KK buffers of unequal lengths in one launch group (both formats,
    lengths multiples of 1024 but not of the front end's block pair): 344
    work items (eight buffers of the longest one's 43 block pairs), more than
    the persistent front end's grid holds at once, so workgroups take items
    from its queue; the 85 items past a shorter buffer's end are skipped.  Each buffer's bits must equal the buffer
    processed alone, on two eager batches in a row (the queue resets itself
    between launches) and on graph replays."""
    import torch
    lens = [1 << 20, (1 << 20) - 25 * 1024, 600 * 1024, (1 << 19) + 7 * 1024, 1 << 20, 24 * 1024,
            900 * 1024, (1 << 20) - 1024]
    fmts = [5, 4, 5, 4, 4, 5, 5, 4]
    gens = [synth.generate(f, n, 1400 + i, 20.0) for i, (f, n) in enumerate(zip(fmts, lens))]
    recs = [rx.Receiver(f, g["seed"], max_samples=1 << 20) for f, g in zip(fmts, gens)]
    bufs = [_dev(g["packed"]) for g in gens]
    single = [r.process(b, n).cpu().numpy() for r, b, n in zip(recs, bufs, lens)]
    torch.cuda.synchronize()
    outs = [torch.zeros(r.bits_bytes(n), dtype=torch.uint8, device="cuda:0") for r, n in zip(recs, lens)]
    args = ([r.h for r in recs], [b.data_ptr() for b in bufs], lens, [o.data_ptr() for o in outs])
    for rep in range(2):
        for o in outs:
            o.zero_()
        rx.rx_process_batch(*args, graph=False)
        torch.cuda.synchronize()
        for i, (o, s) in enumerate(zip(outs, single)):
            assert np.array_equal(o.cpu().numpy(), s), f"eager batch {rep}, buffer {i} (n = {lens[i]})"
    for rep in range(2):
        for o in outs:
            o.zero_()
        rx.rx_process_batch(*args, graph=True)
        torch.cuda.synchronize()
        for i, (o, s) in enumerate(zip(outs, single)):
            assert np.array_equal(o.cpu().numpy(), s), f"graph replay {rep}, buffer {i} (n = {lens[i]})"
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
    want = ("bits", "soft", "ddz")
    o = oracle.process(5, g["packed"], n, g["seed"], want=want)
    for lg in (13, 14):
        dec = parity.compare_decisions(
            5, res[lg][0], o, n // 4, 128,
            rerun=lambda f: oracle.process(5, g["packed"], n, g["seed"], want=want, force=f))
        assert not dec.untolerated
        assert abs(res[lg][2]["bit_errors"] - dec.oracle["bit_errors"]) <= dec.tolerated_bits


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("n,seed", [(1 << 18, 51), (1 << 24, 401)])
def test_precision_form(rx, prec, n, seed):
    """BF16 (1) / FP16 (2) Toeplitz-GEMM matched filter and frozen-tap FFE on
    MFMA with FP32 accumulation, against the oracle's precision form (the
    carrier-free downshifted field, the taps and the FFE operands rounded to
    the narrow type, FP64 accumulation) and against the unrounded FP64 chain
    of the same frozen-tap definition.  The kernel rounds its own operands
    (not the oracle's), so the soft values differ by rounding noise: their
    error against the unrounded chain must be of the same size as the
    oracle's own (at most RATIO times it), decisions may differ only where
    the oracle's soft value lies within DIST_SIGMAS times that noise of a
    threshold, and error counts by at most those symbols' bits."""
    print(f"[precision] prec={prec} n={n} seed={seed}", flush=True)
    g = synth.generate(5, n, synth.derive_seed(seed, 0), 22.0)
    s = g["seed"]
    o_r = oracle.process(5, g["packed"], n, s, want=("bits", "soft", "mf", "taps"), form=1, rounding=prec)
    o_f = oracle.process(5, g["packed"], n, s, want=("bits", "soft", "mf"), form=1, rounding=0)
    r = rx.Receiver(5, s, max_samples=n, debug=True, precision=prec)
    bits = r.process(_dev(g["packed"]), n).cpu().numpy()
    sc = r.fetch(rx.RX_STAGE_SCALARS, n)
    mf = r.fetch(rx.RX_STAGE_MF, n)   # already AGC'd
    soft = r.fetch(rx.RX_STAGE_SOFT, n)
    err = r.errors()
    r.close()
    assert int(sc[4]) == o_r["lag"] and int(sc[5]) == o_r["rot"]
    rep = {"mf_vs_fp64": parity.rel_rms(mf, o_f["mf"]), "mf_oracle_rounded_vs_fp64": parity.rel_rms(o_r["mf"], o_f["mf"]),
           "soft_vs_fp64": parity.rel_rms(soft, o_f["soft"]),
           "soft_oracle_rounded_vs_fp64": parity.rel_rms(o_r["soft"], o_f["soft"]),
           "soft_vs_oracle_rounded": parity.rel_rms(soft, o_r["soft"])}
    nsym = n // 4
    sigma = np.sqrt(np.mean(np.abs(soft - o_r["soft"]) ** 2) / 2)   # per real axis
    g_sym = parity.symbols_from_bits(bits, 5, nsym)
    o_sym = parity.symbols_from_bits(o_r["bits"], 5, nsym)
    dist = parity.threshold_distance(o_r["soft"], 5)
    bad = np.nonzero(g_sym != o_sym)[0]
    tol_bits = int(sum(bin(int(a ^ b)).count("1") for a, b in zip(g_sym[bad], o_sym[bad])))
    rep.update(sigma=float(sigma), mismatch=int(bad.size), max_mismatch_dist=float(dist[bad].max()) if bad.size else 0.0,
               ber_gpu=err["bit_errors"] / err["bits"], ber_oracle_rounded=o_r["bit_errors"] / o_r["counted_bits"],
               ber_fp64=o_f["bit_errors"] / o_f["counted_bits"])
    print(f"[precision]   {rep}", flush=True)
    assert rep["mf_vs_fp64"] <= RATIO * rep["mf_oracle_rounded_vs_fp64"], rep
    assert rep["soft_vs_fp64"] <= RATIO * rep["soft_oracle_rounded_vs_fp64"], rep
    assert np.all(dist[bad] <= max(DIST_SIGMAS * sigma, parity.NEAR)), dist[bad][:10]
    assert abs(err["bit_errors"] - o_r["bit_errors"]) <= tol_bits


RATIO = 4.0          # the kernel's rounding error against the oracle's, both against FP64
DIST_SIGMAS = 8.0    # rounding-noise standard deviations (per axis) around a threshold
