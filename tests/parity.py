"""Helpers for comparing the HIP path with the oracle (tests only)."""
from typing import NamedTuple

import numpy as np

NEAR = 1e-3      # decisions may differ only this close to a threshold (level units)


def axis_levels(fmt):
    return {1: 2, 2: 4, 3: 8, 4: 2, 5: 4}[fmt]


def bps(fmt):
    return {1: 1, 2: 2, 3: 3, 4: 2, 5: 4}[fmt]


def symbols_from_bits(packed, fmt, nsym):
    b = bps(fmt)
    bits = np.unpackbits(np.asarray(packed, dtype=np.uint8), bitorder="little")[: nsym * b]
    bits = bits.reshape(nsym, b).astype(np.int64)
    w = 1 << np.arange(b - 1, -1, -1)
    return bits @ w


def _gray_inverse(g):
    i = g.copy()
    s = g >> 1
    while np.any(s):
        i ^= s
        s >>= 1
    return i


def decision_index(sym, fmt):
    """Level index of each decided symbol (QAM: i * m + q, the oracle's
    forced-decision encoding) from its Gray-coded bits."""
    if fmt >= 4:
        half = bps(fmt) // 2
        m = axis_levels(fmt)
        return _gray_inverse(sym >> half) * m + _gray_inverse(sym & (m - 1))
    return _gray_inverse(sym)


def threshold_distance(soft, fmt):
    """Per symbol: smallest distance of any real axis to a decision threshold."""
    m = axis_levels(fmt)
    thr = np.arange(m - 1) * 2.0 - (m - 2)
    def d(x):
        return np.min(np.abs(x[:, None] - thr[None, :]), axis=1)
    s = np.asarray(soft)
    if np.iscomplexobj(s):
        return np.minimum(d(s.real), d(s.imag))
    return d(s)


class Decisions(NamedTuple):
    mismatch: int          # symbols decided differently from the (final) oracle run
    tolerated_bits: int    # bits of those symbols (all within NEAR of a threshold)
    untolerated: list      # (symbol, distance) of mismatches farther than NEAR
    reruns: int            # oracle re-runs with DD-LMS decisions forced
    forced: list           # (symbol, forced level index) of the accepted re-run
    oracle: dict           # the oracle run the decisions were finally judged against


def _alternatives(fmt, o, g_sym, lo, hi):
    """DD-LMS decisions in symbols [lo, hi) that another implementation may
    have taken the other way: the oracle's pre-derotation output lies within
    NEAR of a threshold there.  Returns (symbol, level index of the other
    side).  For PAM the output decided on is the soft value itself, so where
    the final decisions agree no flip happened and the GPU's own decision is
    the alternative where they differ."""
    m = axis_levels(fmt)
    ddz = np.asarray(o["ddz"])
    out = []
    for k in range(lo, hi):
        v = ddz[k]
        axes = [v.real, v.imag] if fmt >= 4 else [float(v)]
        idx, near = [], False
        for x in axes:
            i = int(min(max(np.floor((x + m) / 2.0), 0), m - 1))
            j = int(np.clip(np.round((x + m - 2) / 2.0), 0, m - 2))   # nearest threshold 2j - (m - 2)
            t = 2.0 * j - (m - 2)
            if abs(x - t) <= NEAR:
                near = True
                i = j if x >= t else j + 1
            idx.append(i)
        if not near:
            continue
        alt = idx[0] * m + idx[1] if fmt >= 4 else idx[0]
        if fmt < 4 and alt != decision_index(np.array([g_sym[k]]), fmt)[0]:
            continue
        out.append((k, alt))
    return out


def compare_decisions(fmt, gpu_bits, oracle_run, nsym, blk, rerun=None, max_cands=4):
    """Symbols whose decisions differ must lie within NEAR of a threshold in
    the oracle's soft value; no other mismatch is forgiven as such.  The one
    mechanism that can move a symbol farther is explained, not tolerated: in
    the block DD-LMS a decision taken the other way at a symbol whose output
    lies on a threshold changes the block's later taps.  For a block with a
    mismatch beyond NEAR, the oracle is run again (rerun(force), force =
    int32[nsym] level indices, -1 = its own) with the other decision forced
    at such symbols before it (subsets of the first max_cands, smallest
    first); the block counts as explained when a re-run leaves it no
    mismatch beyond NEAR, and the GPU is then judged against that run.
    oracle_run: the oracle's result (bits, soft, and ddz when rerun is
    given)."""
    import itertools
    g = symbols_from_bits(gpu_bits, fmt, nsym)

    def classify(o):
        os_ = symbols_from_bits(o["bits"], fmt, nsym)
        dist = threshold_distance(o["soft"], fmt)
        bad = np.nonzero(g != os_)[0]
        return os_, dist, bad, bad[dist[bad] > NEAR]

    o = oracle_run
    force = np.full(nsym, -1, dtype=np.int32)
    reruns = 0
    os_, dist, bad, far = classify(o)
    done_blocks = set()
    nblk = nsym // blk
    while rerun is not None and far.size:
        k0 = int(far[0])
        b = k0 // blk
        if b in done_blocks:
            break
        done_blocks.add(b)
        # PAM: a flip moves only the later symbols of its own block.  KK: it
        # also changes the block's z^4 sum, so the carrier phase of the
        # blocks either side (the three-block window) and their decisions.
        if fmt >= 4:
            lo, hi = max(b - 1, 0) * blk, min(b + 2, nblk) * blk
            blocks = {b - 1, b, b + 1}
        else:
            lo, hi = b * blk, k0 + 1
            blocks = {b}
        cands = [c for c in _alternatives(fmt, o, g, lo, hi) if force[c[0]] < 0][:max_cands]
        accepted = None
        for r in range(1, len(cands) + 1):
            for sub in itertools.combinations(cands, r):
                f = force.copy()
                for k, a in sub:
                    f[k] = a
                o2 = rerun(f)
                reruns += 1
                c2 = classify(o2)
                if not any(int(k) // blk in blocks for k in c2[3]):
                    accepted = (f, o2, c2)
                    break
            if accepted:
                break
        if accepted is None:
            break
        force, o = accepted[0], accepted[1]
        os_, dist, bad, far = accepted[2]
    near = bad[dist[bad] <= NEAR]
    tol_bits = int(sum(bin(int(a ^ b)).count("1") for a, b in zip(g[near], os_[near])))
    untol = [(int(k), float(dist[k])) for k in far]
    forced = [(int(k), int(force[k])) for k in np.nonzero(force >= 0)[0]]
    return Decisions(int(bad.size), tol_bits, untol, reruns, forced, o)


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
