"""Full-scale cases through the C ABI: the largest buffer a handle accepts
(2^26 samples) against the FP64 oracle decision by decision, and a
64 x 2^22-sample batch in the launch configuration the benchmark times
(distinct handles, eight distinct buffers round-robin): sampled buffers of the
batch bit-exact against the same buffers processed alone, one of them against
the oracle."""
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


def _counts(e):
    """The error counters; late_buffers depends on where a buffer sat in its launch."""
    return {k: v for k, v in e.items() if k != "late_buffers"}


def _against_oracle(fmt, g, n, bits, err):
    want = ("bits", "soft", "ddz")
    o = oracle.process(fmt, g["packed"], n, g["seed"], want=want)
    kk = fmt >= 4
    nsym = n // (4 if kk else 2)
    dec = parity.compare_decisions(fmt, bits, o, nsym, 128 if kk else 256,
                                   rerun=lambda f: oracle.process(fmt, g["packed"], n, g["seed"], want=want, force=f))
    of = dec.oracle
    print(f"[scale]   mismatches {dec.mismatch}, tolerated bits {dec.tolerated_bits}, forced {dec.forced}, "
          f"bit errors {err['bit_errors']} / {of['bit_errors']}", flush=True)
    assert not dec.untolerated, dec.untolerated[:10]
    assert err["bits"] == of["counted_bits"]
    assert abs(err["bit_errors"] - of["bit_errors"]) <= dec.tolerated_bits


def test_maximum_buffer_kk16qam(rx):
    import torch
    n = 1 << 26
    print(f"[scale] KK-16QAM n={n}", flush=True)
    g = synth.generate(5, n, 81, 22.0)
    r = rx.Receiver(5, g["seed"], max_samples=n)
    bits = r.process(torch.from_numpy(g["packed"]).to("cuda:0"), n).cpu().numpy()
    err = r.errors()
    r.close()
    assert err["buffers"] == 1 and err["bit_errors"] <= 1e-4 * err["bits"]
    _against_oracle(5, g, n, bits, err)


def test_bench_launch_configuration(rx):
    import torch
    n, batch, distinct = 1 << 22, 64, 8
    print(f"[scale] KK-16QAM batch {batch} x {n}", flush=True)
    gens = [synth.kk_2e22(synth.KK_16QAM, index=i) for i in range(distinct)]
    bufs = [torch.from_numpy(g["packed"]).to("cuda:0") for g in gens]
    recs = [rx.Receiver(5, gens[i % distinct]["seed"], max_samples=n) for i in range(batch)]
    outs = [torch.zeros(r.bits_bytes(n), dtype=torch.uint8, device="cuda:0") for r in recs]
    rx.rx_process_batch([r.h for r in recs], [bufs[i % distinct].data_ptr() for i in range(batch)], [n] * batch,
                        [o.data_ptr() for o in outs])
    torch.cuda.synchronize()
    errs = [r.errors() for r in recs]
    for i in (0, 13, 38, 63):
        alone = rx.Receiver(5, gens[i % distinct]["seed"], max_samples=n)
        single = alone.process(bufs[i % distinct], n).cpu().numpy()
        assert np.array_equal(outs[i].cpu().numpy(), single), f"buffer {i}"
        assert _counts(alone.errors()) == _counts(errs[i])
        alone.close()
    # the same buffer through distinct handles of the batch: identical bits
    assert np.array_equal(outs[5].cpu().numpy(), outs[5 + distinct].cpu().numpy())
    _against_oracle(5, gens[0], n, outs[0].cpu().numpy(), errs[0])
    for r in recs:
        r.close()


def test_every_format_full_size_in_one_batch(rx):
    """One 2^22-sample buffer of each format, each twice, in one batched
    launch: every buffer against the oracle, the two copies bit-exact."""
    import torch
    n = 1 << 22
    fmts = [1, 2, 3, 4, 5]
    print(f"[scale] mixed formats {fmts}, n={n}", flush=True)
    gens = [synth.generate(f, n, 950 + f, 18.0 + f) for f in fmts]
    bufs = [torch.from_numpy(g["packed"]).to("cuda:0") for g in gens]
    order = list(range(len(fmts))) * 2
    recs = [rx.Receiver(fmts[i], gens[i]["seed"], max_samples=n) for i in order]
    outs = [torch.zeros(r.bits_bytes(n), dtype=torch.uint8, device="cuda:0") for r in recs]
    rx.rx_process_batch([r.h for r in recs], [bufs[i].data_ptr() for i in order], [n] * len(order),
                        [o.data_ptr() for o in outs])
    torch.cuda.synchronize()
    errs = [r.errors() for r in recs]
    for j, i in enumerate(order[:len(fmts)]):
        k = j + len(fmts)
        assert np.array_equal(outs[j].cpu().numpy(), outs[k].cpu().numpy()) and _counts(errs[j]) == _counts(errs[k])
        print(f"[scale] format {fmts[i]}", flush=True)
        _against_oracle(fmts[i], gens[i], n, outs[j].cpu().numpy(), errs[j])
    for r in recs:
        r.close()
