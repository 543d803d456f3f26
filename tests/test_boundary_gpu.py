"""Boundary behaviour through the C ABI: cached hipGraphs follow the
handles' state, per-buffer latency and deadline accounting, a caller-owned
reference bit stream, and pointer alignment checks."""
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


def _linear_net(taps):
    """A ReLU network equal to the real FIR with the given 15 taps."""
    p = np.zeros(oracle.MLP_PARAMS)
    w1 = p[:64 * 31].reshape(64, 31)
    for i, w in enumerate(taps):
        w1[0, 15 + 7 - i] = w
        w1[1, 15 + 7 - i] = -w
    off = 64 * 31 + 64
    w2 = p[off:off + 4096].reshape(64, 64)
    w2[0, 0] = w2[1, 1] = 1.0
    off += 4096 + 64
    p[off], p[off + 1] = 1.0, -1.0
    return p.astype(np.float32)


def test_graph_replay_follows_network_and_new_handles(rx):
    """A graph captured while an MLP handle had no network replays the LMS
    stage list; after the network is set the next graph call must run the
    network (a new capture), like an eager call.  The network here is the
    frozen prefix FIR, which ties with LMS on a noiseless prefix and so runs:
    its outputs are not the block DD-LMS's.  A handle destroyed and another
    created (possibly at the same address) must not replay the old capture
    either."""
    import torch
    n = 1 << 18
    gp = synth.generate(synth.PAM4, n, 1201, None, drive=0.1)
    gk = synth.generate(synth.KK_QPSK, n, 1202, 20.0)
    bp, bk = _dev(gp["packed"]), _dev(gk["packed"])
    m = rx.Receiver(rx.RX_PAM4, gp["seed"], max_samples=n, equalizer=rx.RX_EQ_MLP, debug=True)
    k = rx.Receiver(rx.RX_KK_QPSK, gk["seed"], max_samples=n)
    om = torch.zeros(m.bits_bytes(n), dtype=torch.uint8, device="cuda:0")
    ok = torch.zeros(k.bits_bytes(n), dtype=torch.uint8, device="cuda:0")

    def run(hs, graph):
        rx.rx_process_batch(hs, [bp.data_ptr(), bk.data_ptr()], [n, n], [om.data_ptr(), ok.data_ptr()],
                            graph=graph)
        torch.cuda.synchronize()

    run([m.h, k.h], True)                      # captured with the LMS stage list (no network yet)
    lms_soft = m.fetch(rx.RX_STAGE_SOFT, n)
    rx.rx_set_mlp(m.h, _linear_net(m.fetch(rx.RX_STAGE_TAPS, n).real))
    run([m.h, k.h], True)
    graph_soft = m.fetch(rx.RX_STAGE_SOFT, n)
    assert int(m.fetch(rx.RX_STAGE_SCALARS, n)[6]) == 0, "the network ties on the prefix and runs"
    run([m.h, k.h], False)
    eager_soft = m.fetch(rx.RX_STAGE_SOFT, n)
    assert np.array_equal(graph_soft, eager_soft)
    assert not np.array_equal(graph_soft, lms_soft)
    # destroy the KK handle, create another in its place (another reference
    # sequence: other training symbols, so other decisions), replay with graph
    k.close()
    k2 = rx.Receiver(rx.RX_KK_QPSK, gk["seed"] + 1, max_samples=n)
    ok.zero_()
    run([m.h, k2.h], True)
    graph_bits = ok.cpu().numpy().copy()
    e_graph = k2.errors()
    k2.reset()
    ok.zero_()
    run([m.h, k2.h], False)
    assert e_graph["buffers"] == 1
    assert np.array_equal(graph_bits, ok.cpu().numpy())
    e_eager = k2.errors()
    assert e_graph["bit_errors"] == e_eager["bit_errors"] and e_graph["bits"] == e_eager["bits"]
    m.close()
    k2.close()


def test_latency_and_late_buffers(rx):
    """Device timestamps give each buffer's latency; a deadline of 1 ns makes
    every buffer late, one of 100 s none, and the default (the buffer's own
    real-time span, 65.5 us for 2^18 samples at 4 Gs/s) is compared too."""
    n = 1 << 18
    g = synth.generate(synth.KK_16QAM, n, 1301, 22.0)
    buf = _dev(g["packed"])
    res = {}
    for name, dl in (("tight", 1e-9), ("loose", 100.0), ("default", 0.0)):
        r = rx.Receiver(rx.RX_KK_16QAM, g["seed"], max_samples=n, deadline_s=dl)
        for _ in range(3):
            r.process(buf, n)
        e = r.errors()
        lat = r.latencies()
        res[name] = (e, lat)
        assert e["buffers"] == 3 and lat.size == 3 and np.all(lat > 0) and np.all(lat < 1e6)
        r.reset()
        assert r.errors()["late_buffers"] == 0 and r.latencies().size == 0
        r.close()
    assert res["tight"][0]["late_buffers"] == 3
    assert res["loose"][0]["late_buffers"] == 0
    lat_d = res["default"][1]
    assert res["default"][0]["late_buffers"] == int(np.sum(lat_d > n / 4e9 * 1e6))
    print(f"[boundary] latencies (us) of a lone 2^18 KK buffer: {np.round(lat_d, 1)}", flush=True)
    # the ring keeps the most recent 1024
    r = rx.Receiver(rx.RX_PAM2, g["seed"], max_samples=1 << 16)
    gp = synth.generate(synth.PAM2, 1 << 16, 1302, 20.0)
    bp = _dev(gp["packed"])
    for _ in range(1030):
        r.process(bp, 1 << 16)
    assert r.latencies().size == 1024 and r.errors()["buffers"] == 1030
    r.close()


def _packed_reference(fmt, seed, nsym):
    """Reference bits of symbols 0..nsym-1 packed like the output (symbol k
    at stream bits [bps k, bps (k+1)), MSB first; LSB-first bytes), padded
    to whole 32-bit words."""
    b = parity.bps(fmt)
    sym = synth.reference_bits(fmt, seed, nsym)
    bits = ((sym[:, None] >> np.arange(b - 1, -1, -1)[None, :]) & 1).astype(np.uint8).ravel()
    packed = np.packbits(bits, bitorder="little")
    words = -(-packed.size // 4)
    out = np.zeros(4 * words, dtype=np.uint8)
    out[:packed.size] = packed
    return out


@pytest.mark.parametrize("fmt", [3, 5])
def test_caller_reference_stream(rx, fmt):
    """One handle with a caller-owned reference stream counts two buffers of
    different sequences (the stream rewritten on the handle's stream between
    them) exactly as two seed-based handles do.  The stream is sized to the
    exact word count (no slack) for every symbol count check."""
    import torch
    n = 1 << 18
    sps = 4 if fmt >= 4 else 2
    gens = [synth.generate(fmt, n, 1400 + i, 16.0) for i in range(2)]
    refs = [_packed_reference(fmt, g["seed"], n // sps) for g in gens]
    dref = torch.zeros(refs[0].size, dtype=torch.uint8, device="cuda:0")
    r = rx.Receiver(fmt, 0, max_samples=n, ref_bits=dref.data_ptr())
    got = []
    for g, ref in zip(gens, refs):
        dref.copy_(torch.from_numpy(ref))
        torch.cuda.synchronize()
        bits = r.process(_dev(g["packed"]), n).cpu().numpy()
        e = r.errors()
        r.reset()
        got.append((bits, e))
    r.close()
    for (bits, e), g in zip(got, gens):
        s = rx.Receiver(fmt, g["seed"], max_samples=n)
        b2 = s.process(_dev(g["packed"]), n).cpu().numpy()
        e2 = s.errors()
        s.close()
        assert np.array_equal(bits, b2)
        assert {k: v for k, v in e.items() if k != "late_buffers"} == \
            {k: v for k, v in e2.items() if k != "late_buffers"}


def test_misaligned_pointers_rejected(rx):
    import torch
    n = 1 << 16
    r = rx.Receiver(rx.RX_PAM4, 1, max_samples=n)
    buf = torch.zeros(n * 3 // 2 + 8, dtype=torch.uint8, device="cuda:0")
    out = torch.zeros(r.bits_bytes(n) + 8, dtype=torch.uint8, device="cuda:0")
    for db, do in ((1, 0), (0, 2), (3, 1)):
        with pytest.raises(rx.RxError):
            rx.rx_process(r.h, buf.data_ptr() + db, n, out.data_ptr() + do)
        with pytest.raises(rx.RxError):
            rx.rx_process_batch([r.h], [buf.data_ptr() + db], [n], [out.data_ptr() + do])
    with pytest.raises(rx.RxError):
        rx.Receiver(rx.RX_PAM4, 1, max_samples=n, ref_bits=out.data_ptr() + 2)
    rx.rx_process(r.h, buf.data_ptr() + 4, n, out.data_ptr() + 4)   # 4-byte aligned: accepted
    torch.cuda.synchronize()
    r.close()
