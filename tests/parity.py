"""Helpers for comparing the HIP path with the oracle (tests only)."""
import numpy as np

NEAR = 1e-3      # decisions may differ only this close to a threshold (level units)
CASCADE = 5e-2   # after a tolerated flip, the same DD-LMS block may flip this close


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


def compare_decisions(fmt, gpu_bits, oracle_bits, oracle_soft, nsym, blk):
    """Symbols whose decisions differ must lie within NEAR of a threshold in
    the oracle, or within CASCADE after an earlier tolerated flip in the same
    DD-LMS block.  Returns (mismatches, tolerated_bits, untolerated list)."""
    g = symbols_from_bits(gpu_bits, fmt, nsym)
    o = symbols_from_bits(oracle_bits, fmt, nsym)
    dist = threshold_distance(oracle_soft, fmt)
    bad = np.nonzero(g != o)[0]
    flipped_blocks = set()
    untol = []
    tol_bits = 0
    for k in bad:
        b = k // blk
        if dist[k] <= NEAR or (b in flipped_blocks and dist[k] <= CASCADE):
            flipped_blocks.add(b)
            tol_bits += bin(int(g[k] ^ o[k])).count("1")
        else:
            untol.append((int(k), float(dist[k])))
    return len(bad), tol_bits, untol


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
