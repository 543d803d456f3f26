"""The decision-comparison rule of the parity tests, exercised on the CPU
with the oracle standing in for a second implementation: a run whose block
DD-LMS took one threshold decision the other way (forced in the oracle, with
a larger LMS step so that the flip moves later decisions of its block) is
explained by the re-run search, and nothing else is forgiven."""
import numpy as np
import pytest

import parity
import synth


def _flip_cases(oracle_lib, fmt, seeds, limit):
    """(generator dict, oracle run, rerun, symbol, level index, other run) for
    threshold decisions whose flip moves a later decision beyond NEAR."""
    n = 1 << 18
    kk = fmt >= 4
    nsym, blk = n // (4 if kk else 2), (128 if kk else 256)
    want = ("bits", "soft", "ddz")
    out = []
    for seed in seeds:
        g = synth.generate(fmt, n, seed, 14.0)
        o = oracle_lib.process(fmt, g["packed"], n, g["seed"], want=want, mu=1e-2)

        def rerun(f, g=g):
            return oracle_lib.process(fmt, g["packed"], n, g["seed"], want=want, force=f, mu=1e-2)

        m = parity.axis_levels(fmt)
        dd = parity.threshold_distance(o["ddz"], fmt)
        for k in np.nonzero(dd <= parity.NEAR)[0]:
            if not 4096 + 64 <= k < nsym - 64:
                continue
            v = o["ddz"][k]
            idx = []
            for x in ([v.real, v.imag] if kk else [float(v)]):
                i = int(min(max(np.floor((x + m) / 2.0), 0), m - 1))
                j = int(np.clip(np.round((x + m - 2) / 2.0), 0, m - 2))
                if abs(x - (2.0 * j - (m - 2))) <= parity.NEAR:
                    i = j if x >= 2.0 * j - (m - 2) else j + 1
                idx.append(i)
            alt = idx[0] * m + idx[1] if kk else idx[0]
            f = np.full(nsym, -1, dtype=np.int32)
            f[k] = alt
            other = rerun(f)
            bits = other["bits"].copy()
            if not kk:
                # the second implementation's own output at k decided the other way too
                nb = parity.bps(fmt)
                gray = alt ^ (alt >> 1)
                for t in range(nb):
                    pos = k * nb + t
                    bit = (gray >> (nb - 1 - t)) & 1
                    bits[pos >> 3] = (bits[pos >> 3] & ~np.uint8(1 << (pos & 7))) | np.uint8(bit << (pos & 7))
            if parity.compare_decisions(fmt, bits, o, nsym, blk).untolerated:
                out.append((g, o, rerun, int(k), alt, bits, other))
                if len(out) >= limit:
                    return out, nsym, blk
    return out, nsym, blk


@pytest.mark.parametrize("fmt", [2, 5])
def test_flip_on_a_threshold_is_explained_and_nothing_else(oracle_lib, fmt):
    cases, nsym, blk = _flip_cases(oracle_lib, fmt, (62, 63, 64), 2)
    assert cases, "no cascading threshold flip found"
    for g, o, rerun, k, alt, bits, other in cases:
        dec = parity.compare_decisions(fmt, bits, o, nsym, blk, rerun=rerun)
        assert not dec.untolerated, (k, dec)
        assert (k, alt) in dec.forced and dec.reruns >= 1
        # a decision flipped far from any threshold is never forgiven
        dist = parity.threshold_distance(dec.oracle["soft"], fmt)
        far = int(np.nonzero(dist > 0.5)[0][5000])
        bad = bits.copy()
        nb = parity.bps(fmt)
        bad[(far * nb) >> 3] ^= np.uint8(1 << ((far * nb) & 7))
        dec2 = parity.compare_decisions(fmt, bad, o, nsym, blk, rerun=rerun)
        assert any(u[0] == far for u in dec2.untolerated)
