"""Host-resident buffers through rx_process_batch_host: bits and error counts
equal those of the device path, for pinned and pageable host memory and for
two calls in a row (the second on smaller buffers, reusing the staging), and
every buffer's decisions against the FP64 oracle."""
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


def _device_reference(rx, recs, gens, n):
    import torch
    bits = [r.process(torch.from_numpy(g["packed"]).to("cuda:0"), n).cpu().numpy() for r, g in zip(recs, gens)]
    errs = [r.errors() for r in recs]
    for r in recs:
        r.reset()
    return bits, errs


@pytest.mark.parametrize("pinned", [True, False])
def test_host_ingest_equals_device_path(rx, pinned):
    import torch
    fmts = [5, 1, 4, 3]
    recs = [rx.Receiver(f, 900 + i, max_samples=1 << 18) for i, f in enumerate(fmts)]
    for call, n in enumerate((1 << 18, 1 << 17)):   # the same handles and staging, then shorter buffers
        print(f"[host-ingest] pinned={pinned} call={call} n={n}", flush=True)
        gens = [synth.generate(f, n, 900 + i, 20.0 - 2 * call) for i, f in enumerate(fmts)]
        ref_bits, ref_errs = _device_reference(rx, recs, gens, n)
        if pinned:
            hin = [torch.from_numpy(g["packed"]).pin_memory() for g in gens]
            hout = [torch.full((r.bits_bytes(n),), 0xA5, dtype=torch.uint8).pin_memory() for r in recs]
            pin_ptrs = [t.data_ptr() for t in hin]
            out_ptrs = [t.data_ptr() for t in hout]
        else:
            hin = [np.ascontiguousarray(g["packed"]) for g in gens]
            hout = [np.full(r.bits_bytes(n), 0xA5, dtype=np.uint8) for r in recs]
            pin_ptrs = [a.ctypes.data for a in hin]
            out_ptrs = [a.ctypes.data for a in hout]
        rx.rx_process_batch_host([r.h for r in recs], pin_ptrs, [n] * len(recs), out_ptrs)
        rx.rx_sync(recs[0].h)
        for i, (o, b) in enumerate(zip(hout, ref_bits)):
            got = o.numpy() if pinned else o
            assert np.array_equal(got, b), f"buffer {i}"
            if pinned:   # the host-ingested decisions against the oracle
                f, g = fmts[i], gens[i]
                want = ("bits", "soft", "ddz")
                kk = f >= 4
                orun = oracle.process(f, g["packed"], n, g["seed"], want=want)
                dec = parity.compare_decisions(
                    f, got, orun, n // (4 if kk else 2), 128 if kk else 256,
                    rerun=lambda fo, f=f, g=g: oracle.process(f, g["packed"], n, g["seed"], want=want, force=fo))
                assert not dec.untolerated, (i, dec.untolerated[:5])
                assert abs(ref_errs[i]["bit_errors"] - dec.oracle["bit_errors"]) <= dec.tolerated_bits
        for r, e in zip(recs, ref_errs):
            got_e = r.errors()
            # latencies differ between the batch and the lone reference runs
            assert {k: v for k, v in got_e.items() if k != "late_buffers"} == \
                {k: v for k, v in e.items() if k != "late_buffers"}
            r.reset()
    for r in recs:
        r.close()


def test_host_ingest_rejects_bad_arguments(rx):
    r = rx.Receiver(1, 1, max_samples=1 << 18)
    buf = np.zeros((1 << 18) // 2 * 3, dtype=np.uint8)
    out = np.zeros(r.bits_bytes(1 << 18), dtype=np.uint8)
    with pytest.raises(RuntimeError):
        rx.rx_process_batch_host([r.h], [buf.ctypes.data], [1000], [out.ctypes.data])   # not a multiple of 1024
    with pytest.raises(RuntimeError):
        rx.rx_process_batch_host([r.h, r.h], [buf.ctypes.data] * 2, [1 << 18] * 2, [out.ctypes.data] * 2)
    r.close()
