#!/usr/bin/env python3
"""Sustained throughput of the KK-16QAM receiver chain on one MI355X.

One step = one batched pass of the whole KK chain (unpack .. error count)
over `--batch` buffers of 2^22 packed 12-bit samples (KK-16QAM, 1 GBaud,
CSPR 10 dB, 22 dB SNR), each buffer in its own device allocation (the
`--distinct` seeded buffers are copied into `--batch` distinct device
buffers, 384 MiB for 64: more than the chip's caches hold), inputs resident
in HBM.  Prints one JSON line.

Beside the headline: each stage timed alone on the chip (one stream, HIP
events on that stream) for the roofline of the dominant kernel, per-kernel
HBM traffic from committed counter records, the BF16/FP16 precision forms,
their error and BER against the FP64 oracle on a 2^24-sample buffer, the
PAM-8 learned-equaliser form, a mixed-format batch with per-buffer device
latencies, the chain fed from host memory, and the FP64 oracle timed on the
host's cores (all of them, and one).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 1 << 22
FS = 4e9
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3          # published MI355X FP32 vector peak (counts packed FP32 FMA)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 FLOP x 2.4 GHz: the kernels issue no packed FP32
METRIC = "sustained Gsamples/s for KK-16QAM chain, plain vs BF16/MLP at matched BER"


def front_flop_per_sample(log2n):
    """Algorithmic FLOP per input sample of the fused KK front end: two
    complex N-point FFTs per 2 hop samples at 5 N log2 N, the Hilbert product
    (2 N per pair), and the 65-tap decimating matched filter on complex
    samples (65 complex-by-real MACs per output, one output per two
    samples: 130)."""
    n = 1 << log2n
    hop = (n - 2048 - 2080 - 32) & ~15
    return (5.0 * n * log2n + 2.0 * n) / hop + 130.0


# Counter records (two rocprofv3 --pmc passes each, FETCH_SIZE and WRITE_SIZE)
# and the sources whose code they were taken on.
KERNEL_SOURCES = ["kk.hip", "fft_lds.hpp", "rx_dev.hpp", "rx_shared.h"]
EQ_SOURCES = ["eq.hip", "rx_dev.hpp", "rx_shared.h"]
TRAFFIC = {
    "kk_front": ("kk_front_kk16qam_2e22_b64_traffic.json", KERNEL_SOURCES),
    "blocks": ("rx_blocks_kk16qam_2e22_b64_traffic.json", EQ_SOURCES),
    "decide": ("rx_decide_kk16qam_2e22_b64_traffic.json", EQ_SOURCES),
}


def kernel_source_hash(root=None, sources=None):
    """SHA-256 of the named kernel sources with comments and blank lines
    removed: the counters were taken on the code, so a change to a comment
    leaves a figure valid and any change to the code does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in sources or KERNEL_SOURCES:
        with open(os.path.join(root or ROOT, "paper_2010_14333_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.split("\n") if line.strip())
        h.update(code.encode())
    return h.hexdigest()


def traffic_record(stage, batch):
    """HBM bytes per launch of a stage from its committed counter record, if
    it was taken at this launch size on the kernel code as it is now (else
    None)."""
    if stage not in TRAFFIC:
        return None
    fname, sources = TRAFFIC[stage]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != kernel_source_hash(sources=sources) or t.get("buffers_per_launch") != batch:
        return None
    return {"bytes_per_launch": t["bytes_per_launch"], "source": os.path.relpath(path, ROOT)}


def front_traffic(batch):
    return traffic_record("kk_front", batch)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---- input generation in worker processes (before the GPU is touched) -------
def _gen(job):
    import synth
    kind, a = job
    if kind == "kk":
        g = synth.kk_2e22(synth.KK_16QAM, index=a)
    elif kind == "kk24":   # the precision workload at its SNR (22 dB) and at 16 dB (BER near 1e-3)
        g = synth.generate(synth.KK_16QAM, 1 << 24, synth.derive_seed(401, 0 if a == 22.0 else 1), a)
        g["snr_db"] = a
    elif kind == "mixed":
        i, fmt, snr = a
        g = synth.generate(fmt, N, synth.derive_seed(301, i), snr)
    elif kind == "pam8":
        seed, i = a
        g = synth.pam8_91km(i, seed=seed)
    elif kind == "soak":
        # a whole number of tone cycles (11/80 of the sample rate) and of 1024 samples,
        # so the repeated pattern is a continuous signal
        g = synth.generate(synth.KK_16QAM, 4096000, synth.derive_seed(801, 0), 22.0)
    else:
        raise ValueError(kind)
    return {"fmt": g["fmt"], "seed": g["seed"], "n": g["n_samples"], "packed": g["packed"],
            "snr_db": g.get("snr_db")}


def _oracle_kk(item):
    import oracle
    import synth
    oracle.process(synth.KK_16QAM, item["packed"], item["n"], item["seed"], want=("bits",))
    return item["n"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))   # the host share of one GPU


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--distinct", type=int, default=8, help="distinct seeded buffers (copied into --batch allocations)")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--streams", type=int, default=3,
                    help="consecutive batches alternate over this many HIP streams (batch pipelining)")
    ap.add_argument("--roofline", type=int, default=1,
                    help="time every stage alone on the chip (one stream, HIP events) for the roofline")
    ap.add_argument("--roof-steps", type=int, default=5)
    ap.add_argument("--cpu-buffers", type=int, default=4, help="oracle buffers per host core (0: no CPU baseline)")
    ap.add_argument("--copy-probe", type=int, default=1, help="run a 256 MiB device copy (counter scale)")
    ap.add_argument("--forms", default="bf16,fp16,fd,paper",
                    help="forms timed beside the plain chain: bf16, fp16 (precision forms), fd (the paper's "
                         "frequency-domain front end), paper (that front end with the paper's 4-tap DD-LMS "
                         "carrying the carrier phase)")
    ap.add_argument("--precision-check", type=int, default=1,
                    help="2^24-sample KK-16QAM buffers (22 and 16 dB) through FP32/BF16/FP16 against the FP64 oracle")
    ap.add_argument("--mlp", type=int, default=1, help="train and time the PAM-8 learned-equaliser form")
    ap.add_argument("--mixed", type=int, default=1, help="time a 64-buffer mixed-format batch (graph replay)")
    ap.add_argument("--latency", type=int, default=1, help="per-buffer latency of small batches on one stream")
    ap.add_argument("--host", type=int, default=1, help="time the plain chain fed from pinned host memory")
    ap.add_argument("--soak", type=int, default=5859,
                    help="buffers of the contiguous-stream soak (KK-16QAM, 4,096,000-sample buffers fed from pinned "
                         "host memory, a repeated transmitter pattern, Q every 20 buffers; 5859 = 6 s of signal)")
    ap.add_argument("--fft-log2", type=int, default=0, choices=(0, 13, 14),
                    help="KK overlap-save FFT size of the timed KK handles: 0 = the library's autotuner, "
                         "13 or 14 to pin it (profiler runs pin 14)")
    ap.add_argument("--sweep", type=int, default=0,
                    help="Q-factor sweeps through the GPU chain, one 2^22 buffer per point: 1 = vs electrical "
                         "SNR for every format, 2 = vs OSNR for the paper's link variants, 3 = both")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}): buffers are independent units, "
              "so N GPUs would each run this single-GPU path on their share", file=sys.stderr)
        sys.exit(2)

    import multiprocessing as mp

    import numpy as np
    import synth

    # every input generated first, in worker processes, before any GPU call
    jobs = [("kk", i) for i in range(a.distinct)]
    plan = synth.mixed_batch_formats(a.batch, seed=301) if a.mixed else []
    jobs += [("mixed", (i, f, snr)) for i, (f, snr) in enumerate(plan)]
    if a.mlp:
        jobs += [("pam8", (501, i)) for i in range(4)] + [("pam8", (502, i)) for i in range(8)]
    if a.precision_check:
        jobs += [("kk24", 22.0), ("kk24", 16.0)]
    if a.soak:
        jobs += [("soak", 0)]
    cores = usable_cores()
    t0 = time.time()
    with mp.get_context("fork").Pool(min(cores, len(jobs))) as pool:
        made = pool.map(_gen, jobs, chunksize=1)
    gens = [m for j, m in zip(jobs, made) if j[0] == "kk"]
    mixed_gens = [m for j, m in zip(jobs, made) if j[0] == "mixed"]
    train = [m for j, m in zip(jobs, made) if j[0] == "pam8" and j[1][0] == 501]
    testg = [m for j, m in zip(jobs, made) if j[0] == "pam8" and j[1][0] == 502]
    big = [m for j, m in zip(jobs, made) if j[0] == "kk24"]
    soak_g = [m for j, m in zip(jobs, made) if j[0] == "soak"]
    log(f"[bench] generated {len(jobs)} input buffers in {time.time() - t0:.1f}s on {cores} processes")

    # the FP64 oracle on the host's cores: all of them, then one (before the
    # GPU is touched, so the worker processes fork from a plain process)
    cpu = None
    if a.cpu_buffers > 0:
        items = [gens[i % len(gens)] for i in range(a.cpu_buffers * cores)]
        t2 = time.perf_counter()
        with mp.get_context("fork").Pool(cores) as pool:
            done = sum(pool.map(_oracle_kk, items, chunksize=1))
        t_all = time.perf_counter() - t2
        one = items[: max(2, a.cpu_buffers)]
        t3 = time.perf_counter()
        done1 = sum(_oracle_kk(it) for it in one)
        t_one = time.perf_counter() - t3
        cpu = {"value": round(done / t_all / 1e9, 5), "unit": "Gsamples/s", "cores": cores, "kind": "oracle",
               "sample": f"{len(items)} x 2^22-sample KK-16QAM buffers (22 dB) through the FP64 oracle, one buffer "
                         f"per process, {cores} processes, {t_all:.1f} s wall",
               "one_core": {"value": round(done1 / t_one / 1e9, 5), "unit": "Gsamples/s", "cores": 1,
                            "sample": f"{len(one)} buffers, one process, {t_one:.1f} s"},
               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        log(f"[bench] cpu baseline {cpu['value']} Gs/s on {cores} cores, {cpu['one_core']['value']} on one")

    import torch

    import paper_2010_14333_amd as rx

    dev = torch.device("cuda:0")
    src = [torch.from_numpy(g["packed"]).to(dev) for g in gens]
    bufs = [src[i % a.distinct].clone() for i in range(a.batch)]   # one allocation per buffer of the batch
    del src
    bp = [b.data_ptr() for b in bufs]
    streams = [torch.cuda.Stream(device=dev) for _ in range(max(1, a.streams))]   # default priority
    torch.cuda.synchronize()

    def seed_of(i):
        return gens[i % a.distinct]["seed"]

    def run_kk(precision, nstreams, steps, profile=False, front=0, taps=21, dd_phase=False):
        """`steps` batches of the KK-16QAM chain, consecutive batches
        alternating over `nstreams` streams (one set of handles each);
        with `profile`, HIP events on the first handle of each set time
        every stage launch on that stream."""
        sets = []
        for st in streams[:nstreams]:
            recs = [rx.Receiver(rx.RX_KK_16QAM, seed_of(i), max_samples=N, stream=st,
                                flags=rx.RX_PROFILE if (i == 0 and profile) else 0,
                                precision=precision, fft_log2=0 if front else a.fft_log2, front=front,
                                ffe_taps=taps, dd_phase=dd_phase)
                    for i in range(a.batch)]
            outs = [torch.empty(r.bits_bytes(N), dtype=torch.uint8, device=dev) for r in recs]
            sets.append((recs, outs, [r.h for r in recs], [o.data_ptr() for o in outs]))
        ns = [N] * a.batch

        def step(i):
            _, _, hs, op = sets[i % len(sets)]
            rx.rx_process_batch(hs, bp, ns, op, graph=bool(a.graph))

        for i in range(a.warmup * len(sets)):
            step(i)
        torch.cuda.synchronize()
        if profile:
            for _, _, hs, _ in sets:
                rx.rx_stage_times(hs[0], reset=True)
        for recs, _, _, _ in sets:
            for r in recs:
                r.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(steps):
            step(i)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        stages = {}
        if profile:
            for _, _, hs, _ in sets:
                for k, (ms, cnt) in rx.rx_stage_times(hs[0]).items():
                    a0, c0 = stages.get(k, (0.0, 0))
                    stages[k] = (a0 + ms, c0 + cnt)
        errs = [r.errors() for recs, _, _, _ in sets for r in recs]
        for recs, _, _, _ in sets:
            for r in recs:
                r.close()
        bits = sum(e["bits"] for e in errs)
        berr = sum(e["bit_errors"] for e in errs)
        return wall, stages, (berr / bits if bits else None)

    def per_buffer(st):
        return {k: round(v[0] / v[1] * 1e3 / a.batch, 3) for k, v in st.items()}

    # headline: no profiling events on the timed launches
    wall, _, ber = run_kk(rx.RX_FP32, a.streams, a.steps)
    ms_step = wall * 1e3 / a.steps
    samples = a.batch * N
    gsps = samples / (ms_step * 1e-3) / 1e9
    log(f"[bench] plain chain: {a.steps} steps x {a.batch} buffers in {wall:.3f}s: {gsps:.2f} Gs/s")

    stages1 = {}
    if a.roofline:
        wall1, stages1, _ = run_kk(rx.RX_FP32, 1, a.roof_steps, profile=True)
        log(f"[bench] plain chain, one stream, stage events: {per_buffer(stages1)}")

    forms = {}
    for name in [f for f in a.forms.split(",") if f]:
        prec, front, taps, ddp = {"bf16": (rx.RX_BF16, 0, 21, False), "fp16": (rx.RX_FP16, 0, 21, False),
                                  "fd": (rx.RX_FP32, rx.RX_FRONT_FD, 21, False),
                                  "paper": (rx.RX_FP32, rx.RX_FRONT_FD, 4, True)}[name]
        w2, _, b2 = run_kk(prec, a.streams, a.steps, front=front, taps=taps, dd_phase=ddp)
        forms[name] = {"value": round(samples / (w2 / a.steps) / 1e9, 3), "unit": "Gsamples/s",
                       "ms_per_step": round(w2 * 1e3 / a.steps, 4), "ber": b2}
        if a.roofline:
            _, st1, _ = run_kk(prec, 1, a.roof_steps, profile=True, front=front, taps=taps, dd_phase=ddp)
            forms[name]["one_stream_stage_us_per_buffer"] = per_buffer(st1)
        log(f"[bench] {name} form: {forms[name]['value']} Gs/s, BER {b2}")

    def time_handles(make_recs, bptrs, steps, graph, host=False):
        """Time `steps` batches, consecutive batches alternating over the
        streams (one set of handles per stream, made by make_recs(stream));
        with host, bptrs are pinned host buffers and the bits come back to
        pinned host memory (rx_process_batch_host).  Returns the wall time,
        BER, per-handle counters and every buffer's device latency (us)."""
        sets = []
        for st in streams:
            recs = make_recs(st)
            if host:
                outs = [torch.empty(r.bits_bytes(N), dtype=torch.uint8, pin_memory=True) for r in recs]
            else:
                outs = [torch.empty(r.bits_bytes(N), dtype=torch.uint8, device=dev) for r in recs]
            sets.append((st, recs, outs, [r.h for r in recs], [o.data_ptr() for o in outs]))
        ns = [N] * len(bptrs)

        def step(i):
            _, _, _, hs, op = sets[i % len(sets)]
            if host:
                rx.rx_process_batch_host(hs, bptrs, ns, op, graph=graph)
            else:
                rx.rx_process_batch(hs, bptrs, ns, op, graph=graph)

        for i in range(a.warmup * len(sets)):
            step(i)
        torch.cuda.synchronize()
        for _, recs, _, _, _ in sets:
            for r in recs:
                r.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(steps):
            step(i)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        errs = [r.errors() for _, recs, _, _, _ in sets for r in recs]
        lat = np.concatenate([r.latencies() for _, recs, _, _, _ in sets for r in recs])
        for _, recs, _, _, _ in sets:
            for r in recs:
                r.close()
        bits = sum(e["bits"] for e in errs)
        ber = sum(e["bit_errors"] for e in errs) / bits if bits else None
        return wall, ber, errs, lat

    def pct(v, q):
        return round(float(np.percentile(v, q)), 1) if len(v) else None

    host_ingest = None
    if a.host:
        # the plain chain fed from pinned host memory: each buffer crosses PCIe
        # in, its bits come back, on the same streams as the kernels
        hb = [torch.from_numpy(g["packed"]).pin_memory() for g in gens]
        hbp = [hb[i % a.distinct].data_ptr() for i in range(a.batch)]
        wall_h, ber_h, _, _ = time_handles(
            lambda st: [rx.Receiver(rx.RX_KK_16QAM, seed_of(i), max_samples=N, stream=st, fft_log2=a.fft_log2)
                        for i in range(a.batch)], hbp, a.steps, False, host=True)
        host_ingest = {"workload": f"KK-16QAM plain chain, {a.batch} x 2^22 buffers per batch from pinned host "
                                   f"memory, bits back to pinned host memory, {len(streams)} streams",
                       "value": round(a.steps * a.batch * N / wall_h / 1e9, 3), "unit": "Gsamples/s",
                       "h2d_gb_per_s": round(a.steps * a.batch * N * 1.5 / wall_h / 1e9, 2), "ber": ber_h}
        log(f"[bench] host ingest {host_ingest}")
        del hb

    precision = None
    if a.precision_check and big:
        # 2^24-sample KK-16QAM buffers at 22 dB (the workload) and 16 dB (a
        # BER near 1e-3, so the BERs are paired over thousands of errors):
        # each dtype's soft values and BER against the FP64 oracle (the same
        # frozen-tap definition, unrounded and with the precision form's
        # rounding), the FP32 field against FP64
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import parity

        def check(gb):
            nb = gb["n"]
            d = torch.from_numpy(gb["packed"]).to(dev)
            o_plain = oracle.process(5, gb["packed"], nb, gb["seed"], want=("field",))
            o_frozen = oracle.process(5, gb["packed"], nb, gb["seed"], want=("soft",), form=1, rounding=0)
            res = {"workload": f"KK-16QAM, one 2^24-sample buffer (1 GBaud, CSPR 10 dB, {gb['snr_db']:g} dB SNR)"}
            r = rx.Receiver(5, gb["seed"], max_samples=nb, debug=True)
            r.process(d, nb)
            field = r.fetch(rx.RX_STAGE_FIELD, nb)
            e = r.errors()
            r.close()
            res["fp32"] = {"field_rel_rms_vs_fp64": parity.rel_rms(field, o_plain["field"]),
                           "ber": e["bit_errors"] / e["bits"], "bit_errors": e["bit_errors"],
                           "ber_fp64": o_plain["bit_errors"] / o_plain["counted_bits"],
                           "bit_errors_fp64": o_plain["bit_errors"]}
            for name, prec in (("bf16", rx.RX_BF16), ("fp16", rx.RX_FP16)):
                o_r = oracle.process(5, gb["packed"], nb, gb["seed"], want=("soft",), form=1, rounding=prec)
                r = rx.Receiver(5, gb["seed"], max_samples=nb, debug=True, precision=prec)
                r.process(d, nb)
                soft = r.fetch(rx.RX_STAGE_SOFT, nb)
                e = r.errors()
                r.close()
                res[name] = {
                    "soft_rel_rms_vs_fp64": parity.rel_rms(soft, o_frozen["soft"]),
                    "oracle_rounded_soft_rel_rms_vs_fp64": parity.rel_rms(o_r["soft"], o_frozen["soft"]),
                    "soft_rel_rms_vs_oracle_rounded": parity.rel_rms(soft, o_r["soft"]),
                    "ber": e["bit_errors"] / e["bits"], "bit_errors": e["bit_errors"],
                    "ber_fp64_frozen": o_frozen["bit_errors"] / o_frozen["counted_bits"],
                    "bit_errors_fp64_frozen": o_frozen["bit_errors"],
                    "ber_oracle_rounded": o_r["bit_errors"] / o_r["counted_bits"],
                    "delta_ber_vs_fp64_frozen": e["bit_errors"] / e["bits"] - o_frozen["bit_errors"] / o_frozen["counted_bits"]}
            del d
            return res

        precision = check(big[0])
        if len(big) > 1:
            precision["at_16db"] = check(big[1])
        log(f"[bench] precision check {precision}")

    q_sweep = q_osnr = None
    if a.sweep:
        q_sweep, q_osnr = sweeps(a, rx, torch, dev, np, synth)

    mlp_form = None
    if a.mlp:
        trainer = rx.Receiver(rx.RX_PAM8, 0, max_samples=N, equalizer=rx.RX_EQ_MLP)
        tb = [torch.from_numpy(g["packed"]).to(dev) for g in train]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        loss = rx.rx_train_mlp(trainer.h, [b.data_ptr() for b in tb], [N] * len(tb), [g["seed"] for g in train])
        train_s = time.perf_counter() - t2
        w = rx.rx_get_mlp(trainer.h)
        trainer.close()
        del tb
        tsrc = [torch.from_numpy(g["packed"]).to(dev) for g in testg]
        pb = [tsrc[i % len(testg)].clone() for i in range(a.batch)]
        del tsrc
        pbp = [b.data_ptr() for b in pb]
        res = {}
        # the learned equaliser, LMS, and LMS behind the paper's frequency-domain
        # front end (503-tap static equaliser, clock recovery on the spectra)
        for eq in ("mlp", "lms", "lms_fd"):
            def make(st, eq=eq):
                recs = [rx.Receiver(rx.RX_PAM8, testg[i % len(testg)]["seed"], max_samples=N, stream=st,
                                    equalizer=rx.RX_EQ_MLP if eq == "mlp" else rx.RX_EQ_LMS,
                                    front=rx.RX_FRONT_FD if eq == "lms_fd" else rx.RX_FRONT_OS)
                        for i in range(a.batch)]
                if eq == "mlp":
                    for r in recs:
                        rx.rx_set_mlp(r.h, w)
                return recs
            wl, ber_f, errs, _ = time_handles(make, pbp, a.steps, bool(a.graph))
            res[eq] = (a.batch * N / (wl / a.steps) / 1e9, ber_f, sum(e["fallbacks"] for e in errs))
        mlp_form = {"workload": f"PAM-8, 2 GBaud, 91 km SSMF, tanh driver, 24 dB; {len(testg)} distinct 2^22-sample "
                                f"test buffers in {a.batch} allocations per batch",
                    "value": round(res["mlp"][0], 3), "unit": "Gsamples/s", "ber": res["mlp"][1],
                    "fallbacks": res["mlp"][2], "lms_value": round(res["lms"][0], 3), "lms_ber": res["lms"][1],
                    "lms_fd_value": round(res["lms_fd"][0], 3), "lms_fd_ber": res["lms_fd"][1],
                    "train_samples": len(train) * N, "train_s": round(train_s, 3), "final_loss": round(loss, 5)}
        if a.roofline:
            # each PAM stage alone on the chip: one stream, stage events on one handle
            for eq in ("mlp", "lms", "lms_fd"):
                recs = [rx.Receiver(rx.RX_PAM8, testg[i % len(testg)]["seed"], max_samples=N, stream=streams[0],
                                    flags=rx.RX_PROFILE if i == 0 else 0,
                                    equalizer=rx.RX_EQ_MLP if eq == "mlp" else rx.RX_EQ_LMS,
                                    front=rx.RX_FRONT_FD if eq == "lms_fd" else rx.RX_FRONT_OS)
                        for i in range(a.batch)]
                if eq == "mlp":
                    for r in recs:
                        rx.rx_set_mlp(r.h, w)
                outs = [torch.empty(r.bits_bytes(N), dtype=torch.uint8, device=dev) for r in recs]
                args = ([r.h for r in recs], pbp, [N] * a.batch, [o.data_ptr() for o in outs])
                for _ in range(2):
                    rx.rx_process_batch(*args)
                torch.cuda.synchronize()
                rx.rx_stage_times(recs[0].h, reset=True)
                for _ in range(a.roof_steps):
                    rx.rx_process_batch(*args)
                stt = rx.rx_stage_times(recs[0].h)
                mlp_form[f"{eq}_one_stream_stage_us_per_buffer"] = {
                    k: round(v[0] / v[1] * 1e3 / a.batch, 3) for k, v in stt.items()}
                for r in recs:
                    r.close()
                del outs
        del pb
        log(f"[bench] MLP form {mlp_form}")

    mixed = None
    if a.mixed:
        msrc = [torch.from_numpy(g["packed"]).to(dev) for g in mixed_gens]
        mbp = [b.data_ptr() for b in msrc]

        def make_mixed(st):
            return [rx.Receiver(g["fmt"], g["seed"], max_samples=N, stream=st) for g in mixed_gens]
        wl, ber_m, errs, lat = time_handles(make_mixed, mbp, a.steps, True)
        cnt = {}
        for g in mixed_gens:
            cnt[synth.FORMAT_NAMES[g["fmt"]]] = cnt.get(synth.FORMAT_NAMES[g["fmt"]], 0) + 1
        mixed = {"workload": f"{a.batch} distinct 2^22-sample buffers, format per buffer SplitMix64 % 5, SNR per "
                             f"buffer U[14, 26] dB, one hipGraph replay per batch, consecutive batches over "
                             f"{len(streams)} streams",
                 "value": round(a.batch * N / (wl / a.steps) / 1e9, 3), "unit": "Gsamples/s", "formats": cnt,
                 "buffer_latency_us_p50": pct(lat, 50), "buffer_latency_us_p99": pct(lat, 99),
                 "buffers_timed": int(lat.size), "late_buffers": int(sum(e["late_buffers"] for e in errs)),
                 "realtime_budget_us_per_buffer": round(N / FS * 1e6, 1), "ber": ber_m}
        del msrc
        log(f"[bench] mixed batch {mixed}")

    latency = None
    if a.latency:
        # small batches on one stream: the latency a buffer sees when the
        # receiver keeps up with the ADC batch by batch
        latency = {}
        for lb in (1, 4, 16):
            recs = [rx.Receiver(rx.RX_KK_16QAM, seed_of(i), max_samples=N, stream=streams[0], fft_log2=a.fft_log2)
                    for i in range(lb)]
            outs = [torch.empty(r.bits_bytes(N), dtype=torch.uint8, device=dev) for r in recs]
            args = ([r.h for r in recs], bp[:lb], [N] * lb, [o.data_ptr() for o in outs])
            for _ in range(3):
                rx.rx_process_batch(*args)
            torch.cuda.synchronize()
            for r in recs:
                r.reset()
            reps = max(8, 256 // lb)
            t1 = time.perf_counter()
            for _ in range(reps):
                rx.rx_process_batch(*args)
            torch.cuda.synchronize()
            wl = time.perf_counter() - t1
            lat = np.concatenate([r.latencies() for r in recs])
            late = sum(r.errors()["late_buffers"] for r in recs)
            latency[f"batch_{lb}"] = {"buffer_latency_us_p50": pct(lat, 50), "buffer_latency_us_p99": pct(lat, 99),
                                      "late_buffers": int(late), "buffers": int(lat.size),
                                      "value": round(reps * lb * N / wl / 1e9, 3), "unit": "Gsamples/s"}
            for r in recs:
                r.close()
        latency["realtime_budget_us_per_buffer"] = round(N / FS * 1e6, 1)
        latency["workload"] = "KK-16QAM plain chain, batches of 1, 4 and 16 2^22-sample buffers on one stream"
        log(f"[bench] latency {latency}")

    soak = None
    if a.soak and soak_g:
        # the paper's 6-second continuity run with its data flow (Fig. 1a: ADC
        # buffers in host RAM, to the GPU, bits back to RAM): one contiguous
        # stream through a ring of 4 pinned host buffers and 4 device buffers;
        # each buffer's host-to-device copy runs on a copy stream while the
        # previous buffer is processed, its bits go back on the copy stream;
        # Q per 20 buffers (about 21 ms of signal) against the real-time rate
        g = soak_g[0]
        ns_ = g["n"]
        R = 4
        nbytes_bits = (ns_ // 4 * 4 + 7) // 8
        host_in = [torch.from_numpy(g["packed"]).pin_memory() for _ in range(R)]   # the ADC's ring in RAM
        dev_in = [torch.empty(g["packed"].size, dtype=torch.uint8, device=dev) for _ in range(R)]
        dev_bits = [torch.empty(nbytes_bits, dtype=torch.uint8, device=dev) for _ in range(R)]
        host_bits = [torch.empty(nbytes_bits, dtype=torch.uint8).pin_memory() for _ in range(R)]
        comp, copy = streams[0], torch.cuda.Stream(device=dev)
        r = rx.Receiver(rx.RX_KK_16QAM, g["seed"], max_samples=ns_, stream=comp, flags=rx.RX_STREAM,
                        ref_period=ns_ // 4, fft_log2=a.fft_log2)
        copied = [torch.cuda.Event() for _ in range(R)]
        done = [torch.cuda.Event() for _ in range(R)]
        from scipy.special import erfcinv
        qs, bers, lat = [], [], []
        late = 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        i = 0
        while i < a.soak:
            for _ in range(min(20, a.soak - i)):
                sl = i % R
                with torch.cuda.stream(copy):
                    if i >= R:
                        copy.wait_event(done[sl])      # the slot's previous buffer is processed
                    dev_in[sl].copy_(host_in[sl], non_blocking=True)
                    copied[sl].record(copy)
                comp.wait_event(copied[sl])
                r.process(dev_in[sl], ns_, out=dev_bits[sl])
                done[sl].record(comp)
                with torch.cuda.stream(copy):
                    copy.wait_event(done[sl])
                    host_bits[sl].copy_(dev_bits[sl], non_blocking=True)
                i += 1
            e = r.errors()          # synchronises the compute stream
            late += e["late_buffers"]
            lat.append(rx.rx_latencies(r.h, 20))
            r.reset()
            ber_p = e["bit_errors"] / e["bits"] if e["bits"] else 0.0
            bers.append(ber_p)
            qs.append(20.0 * np.log10(np.sqrt(2.0) * erfcinv(2.0 * ber_p)) if 0 < ber_p < 0.5 else None)
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t1
        lat = np.concatenate(lat)
        qv = [q for q in qs if q is not None]
        signal_s = a.soak * ns_ / FS
        soak = {"workload": f"KK-16QAM contiguous stream of {a.soak} buffers of {ns_} samples ({signal_s:.2f} s of "
                            f"signal at 4 Gs/s, 22 dB SNR, a repeated transmitter pattern) through a ring of {R} "
                            f"pinned host buffers: host-to-device copies on a copy stream overlapping the previous "
                            f"buffer's processing, bits back to pinned host memory",
                "buffers": a.soak, "wall_s": round(wall_s, 3), "realtime_factor": round(signal_s / wall_s, 2),
                "h2d_gb_per_s": round(a.soak * ns_ * 1.5 / wall_s / 1e9, 2),
                "periods": len(bers), "q_db_min": round(min(qv), 2) if qv else None,
                "q_db_max": round(max(qv), 2) if qv else None, "error_free_periods": sum(q is None for q in qs),
                "ber_mean": float(np.mean(bers)), "buffer_latency_us_p50": pct(lat, 50),
                "buffer_latency_us_p99": pct(lat, 99), "late_buffers": int(late),
                "realtime_budget_us_per_buffer": round(ns_ / FS * 1e6, 1)}
        r.close()
        del host_in, dev_in, dev_bits, host_bits
        log(f"[bench] soak {soak}")

    def roofline(st):
        if not st or "kk_front" not in st:
            return {"bound": "alu", "achieved": None, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": None,
                    "traffic": None, "kernel": "kk_front<14,0>"}
        lg = a.fft_log2 or 14   # the autotuner's choice on MI355X when not pinned
        dom_ms = st["kk_front"][0] / st["kk_front"][1]
        flop = front_flop_per_sample(lg) * samples
        achieved = flop / (dom_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": f"kk_front<{lg},0>", "achieved": round(achieved, 2),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                "frac_nonpacked": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "flop_per_sample": round(front_flop_per_sample(lg), 2), "samples_per_launch": samples,
                "launch_us": round(dom_ms * 1e3, 2), "timing": "HIP events around each launch on its stream, "
                                                              "one stream (the kernel alone on the chip)",
                "traffic": None}
        hbm = {}
        for stage in ("kk_front", "blocks", "decide"):
            t = traffic_record(stage, a.batch)
            if stage in st and t is not None:
                us = st[stage][0] / st[stage][1] * 1e3
                gbs = t["bytes_per_launch"] / (us * 1e-6) / 1e9
                hbm[stage] = {"bytes_per_launch": t["bytes_per_launch"], "launch_us": round(us, 2),
                              "gb_per_s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4), "source": t["source"]}
        if "kk_front" in hbm:
            roof["traffic"] = hbm["kk_front"]["bytes_per_launch"]
            roof["traffic_source"] = hbm["kk_front"]["source"]
        roof["hbm_per_kernel"] = hbm
        return roof

    roof = roofline(stages1)
    if a.copy_probe:
        probe_src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        probe_dst = torch.empty_like(probe_src)
        probe_dst.copy_(probe_src)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": round(gsps, 3), "unit": "Gsamples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "KK-16QAM receiver chain, plain FP32, 2^22-sample 12-bit buffers "
                               "at 4 Gs/s (1 GBaud, CSPR 10 dB, 22 dB SNR)",
                   "buffers_per_step": a.batch, "samples_per_buffer": N, "distinct_inputs": a.distinct,
                   "input_allocations": a.batch, "graph": bool(a.graph), "streams": a.streams},
        "realtime_factor": round(gsps / 4.0, 2),
        "ber": ber,
        "forms": forms,
        "precision_check": precision,
        "mlp_form": mlp_form,
        "mixed_batch": mixed,
        "latency": latency,
        "host_ingest": host_ingest,
        "stream_soak": soak,
        "q_vs_snr": q_sweep,
        "q_vs_osnr": q_osnr,
        "one_stream_stage_us_per_buffer": per_buffer(stages1) if stages1 else None,
        "roofline": roof,
        # algorithmic HBM fraction of the whole chain: 1.5 B in + 0.125 B of bits out per
        # sample (KK-16QAM: 4 bits per 4 samples) at the sustained rate, over 8 TB/s
        "algorithmic_hbm_frac": round(1.625 * gsps / PEAK_HBM_GBS, 5),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def sweeps(a, rx, torch, dev, np, synth):
    """Q against electrical SNR (every format, bit 1 of --sweep) and against
    OSNR with the paper's link parameters (bit 2), one 2^22-sample buffer per
    point through the GPU chain, the oracle's BER at one point per curve."""
    from scipy.special import erfcinv

    import oracle

    def q_db(ber):
        return round(20.0 * np.log10(np.sqrt(2.0) * erfcinv(2.0 * ber)), 2) if ber and ber < 0.5 else None

    def point(fmt, g, **rxo):
        r = rx.Receiver(fmt, g["seed"], max_samples=N, **rxo)
        r.process(torch.from_numpy(g["packed"]).to(dev), N)
        e = r.errors()
        r.close()
        return e["bit_errors"] / e["bits"] if e["bits"] else None

    q_sweep = q_osnr = None
    if a.sweep & 1:
        names = {1: "PAM-2", 2: "PAM-4", 3: "PAM-8", 4: "KK-QPSK", 5: "KK-16QAM"}
        q_sweep = {}
        for fmt in range(1, 6):
            pts = []
            for si, snr in enumerate([10, 12, 14, 16, 18, 20, 22, 24]):
                g = synth.generate(fmt, N, synth.derive_seed(601, 16 * fmt + si), float(snr))
                ber = point(fmt, g)
                pt = {"snr_db": snr, "ber": ber, "q_db": q_db(ber)}
                if snr == 16:
                    o = oracle.process(fmt, g["packed"], N, g["seed"], want=("bits",))
                    pt["oracle_ber"] = o["bit_errors"] / o["counted_bits"] if o["counted_bits"] else None
                pts.append(pt)
            q_sweep[names[fmt]] = pts
            log(f"[bench] sweep {names[fmt]}: " + ", ".join(f"{p['snr_db']} dB {p['ber']:.2e}" for p in pts))
    if a.sweep & 2:
        curves = [("KK-16QAM, CSPR 11 dB, RRC 0.01", 5, {"rolloff": 0.01, "cspr_db": 11.0}, range(14, 27, 2)),
                  ("KK-16QAM, CSPR 6 dB, RRC 0.01", 5, {"rolloff": 0.01, "cspr_db": 6.0}, range(14, 27, 2)),
                  ("KK-QPSK, CSPR 11 dB, RRC 0.01", 4, {"rolloff": 0.01, "cspr_db": 11.0}, range(4, 15, 2)),
                  ("KK-QPSK, CSPR 6 dB, RRC 0.01", 4, {"rolloff": 0.01, "cspr_db": 6.0}, range(4, 15, 2)),
                  ("PAM-4, RRC 0.5", 2, {"rolloff": 0.5}, range(10, 21, 2)),
                  ("PAM-8, RRC 0.5", 3, {"rolloff": 0.5}, range(16, 29, 2))]
        q_osnr = {}
        for ci, (name, fmt, gen, osnrs) in enumerate(curves):
            osnrs = list(osnrs)
            pts = []
            for si, osnr in enumerate(osnrs):
                g = synth.generate(fmt, N, synth.derive_seed(701, 16 * ci + si), None, osnr_db=float(osnr), **gen)
                ber = point(fmt, g, rolloff=gen["rolloff"])
                pt = {"osnr_db": osnr, "ber": ber, "q_db": q_db(ber)}
                if si == len(osnrs) // 2:
                    o = oracle.process(fmt, g["packed"], N, g["seed"], want=("bits",), rolloff=gen["rolloff"])
                    pt["oracle_ber"] = o["bit_errors"] / o["counted_bits"] if o["counted_bits"] else None
                pts.append(pt)
            q_osnr[name] = pts
            log(f"[bench] osnr sweep {name}: " + ", ".join(f"{p['osnr_db']} dB {p['ber']:.2e}" for p in pts))
    return q_sweep, q_osnr


if __name__ == "__main__":
    main()
