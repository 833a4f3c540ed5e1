"""Plain CPU oracle of the compressed stream's bit-level features (Sec. IV of
Arvanitis, Lalos, Moustakas, arXiv 2111.10105: Eq. 13's bit accounting,
Fig. 5's bits per row of the projected delta coordinates, Fig. 6's coding of
the dictionary as differences of consecutive blocks).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or runs this
file; only the tests, the package's smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library.

Readings (the paper gives the ideas, not the formats):
  * Codes are packed at their bit width with no spare bits: code j of a
    segment occupies bits [j b, (j + 1) b) of the segment's bit string, bit i
    of the string being bit (i mod 32) of 32-bit word floor(i / 32) (least
    significant bit first).  Every segment starts on an 8-byte boundary.
  * Bits per row (Fig. 5): besides Eq. (10)'s b bits for every kept row, a
    caller-given quantisation step s can be asked for; row r then takes the
    fewest bits b_r <= 16 with (hi_r - lo_r) <= s (2^b_r - 1) and is coded by
    Eq. (10) with b_r bits over its own [lo_r, hi_r].  Its step is at most s,
    so every row's error is within s / 2 ("the same reconstruction error"
    whatever the row or block); equal steps are also the allocation that
    minimises the bits for a given total squared error at high rate.
  * Dictionary differences (Fig. 6 and the text before Table II): each column
    of a window's dictionary is sent either as its values or as its
    difference from the same column of the previous window's dequantised
    dictionary, whichever needs fewer bits, over the values' own range
    [lo, hi] (float32, rounded outwards) with the fewest bits whose step is at
    most that of the plain dict_bits code over [-1, 1], so the dictionary is
    never less precise than the plain code.  A window's first window, and any
    window whose predecessor has another length, uses values only.
"""
from __future__ import annotations

import numpy as np

from .dmc_oracle import dequantise_uniform, f32_down, f32_up, quantise_uniform, stored_range


# ---------------------------------------------------------------------------
# packing
# ---------------------------------------------------------------------------

def words_for(count: int, bits: int) -> int:
    """32-bit words of a segment of `count` codes of `bits` bits, rounded up
    to an even number (8-byte boundary)."""
    w = (count * bits + 31) // 32
    return w + (w & 1)


def pack_bits(codes, bits: int) -> np.ndarray:
    """Codes (each < 2^bits) into the segment's words, LSB first."""
    codes = np.asarray(codes, dtype=np.uint64).ravel()
    out = np.zeros(words_for(codes.size, bits), dtype=np.uint64)
    if bits == 0 or codes.size == 0:
        return out.astype(np.uint32)
    if np.any(codes >> np.uint64(bits)):
        raise ValueError("a code does not fit its bit width")
    pos = np.arange(codes.size, dtype=np.uint64) * np.uint64(bits)
    word = pos // np.uint64(32)
    shift = pos % np.uint64(32)
    lo = (codes << shift) & np.uint64(0xFFFFFFFF)
    np.add.at(out, word.astype(np.int64), lo)  # disjoint bit fields: add = or
    spill = shift + np.uint64(bits) > np.uint64(32)
    if np.any(spill):
        hi = codes[spill] >> (np.uint64(32) - shift[spill])
        np.add.at(out, (word[spill] + np.uint64(1)).astype(np.int64), hi)
    return out.astype(np.uint32)


def unpack_bits(words, count: int, bits: int) -> np.ndarray:
    """Inverse of pack_bits: `count` codes of `bits` bits."""
    if bits == 0:
        return np.zeros(count, dtype=np.uint32)
    w = np.asarray(words, dtype=np.uint64)
    pos = np.arange(count, dtype=np.uint64) * np.uint64(bits)
    word = (pos // np.uint64(32)).astype(np.int64)
    shift = pos % np.uint64(32)
    nxt = np.where(word + 1 < w.size, word + 1, word)
    both = w[word] | (np.where(word + 1 < w.size, w[nxt], 0) << np.uint64(32))
    return ((both >> shift) & np.uint64((1 << bits) - 1)).astype(np.uint32)


# ---------------------------------------------------------------------------
# bits per row (Fig. 5)
# ---------------------------------------------------------------------------

def bits_for_step(lo, hi, step: float, max_bits: int = 16) -> int:
    """Fewest bits b (0 <= b <= max_bits) with hi - lo <= step (2^b - 1), or
    max_bits when none is enough; in float64: ratio = (hi - lo) / step, then
    the first b with 2^b - 1 >= ratio."""
    width = np.float64(hi) - np.float64(lo)
    if width == 0.0:
        return 0
    ratio = width / np.float64(step)
    for b in range(1, max_bits + 1):
        if np.float64((1 << b) - 1) >= ratio:
            return b
    return max_bits


def quantise_row(y, lo, hi, bits: int):
    """Eq. (10) on one row with `bits` bits over [lo, hi]; 0 bits means every
    value is sent as lo (the range is a single value).  Returns (codes,
    dequantised)."""
    y = np.asarray(y, dtype=np.float64)
    if bits == 0:
        return np.zeros(y.shape, dtype=np.uint16), np.full(y.shape, np.float64(lo))
    codes = quantise_uniform(y, lo, hi, bits)
    return codes, dequantise_uniform(codes, lo, hi, bits)


def quantise_rows_step(Y, step: float, fp32_data: bool, max_bits: int = 16):
    """Rows of Y (k x n) with the bits per row of a common step: per row the
    stored range (as Eq. 10's), then bits_for_step (at most max_bits), then
    quantise_row.  Returns (codes [k][n] uint16, ranges [k][2] float32,
    bits [k], deq)."""
    k = Y.shape[0]
    codes = np.empty(Y.shape, dtype=np.uint16)
    ranges = np.empty((k, 2), dtype=np.float32)
    bits = np.empty(k, dtype=np.int64)
    deq = np.empty(Y.shape, dtype=np.float64)
    for r in range(k):
        row = Y[r].astype(np.float32) if fp32_data else Y[r]
        lo, hi = stored_range(row)
        ranges[r] = (lo, hi)
        bits[r] = bits_for_step(lo, hi, step, max_bits)
        codes[r], deq[r] = quantise_row(row, lo, hi, int(bits[r]))
    return codes, ranges, bits, deq


# ---------------------------------------------------------------------------
# dictionary as differences of consecutive blocks (Fig. 6)
# ---------------------------------------------------------------------------

DICT_VALUES, DICT_DIFFERENCE = 0, 1


def code_dictionary_column(u, prev, dict_bits: int):
    """One dictionary column u (T values) of a window, given the previous
    window's dequantised column `prev` (or None).  Returns (mode, bits, lo,
    hi, codes, dequantised column)."""
    step = 2.0 / np.float64((1 << dict_bits) - 1)
    u = np.asarray(u, dtype=np.float64)
    cands = [(DICT_VALUES, u)]
    if prev is not None:
        cands.append((DICT_DIFFERENCE, u - np.asarray(prev, dtype=np.float64)))
    best = None
    for mode, vals in cands:
        lo, hi = f32_down(float(vals.min())), f32_up(float(vals.max()))
        b = bits_for_step(lo, hi, step, max_bits=32)
        if best is None or b < best[1]:
            best = (mode, b, lo, hi, vals)
    mode, b, lo, hi, vals = best
    if b > dict_bits:  # only a difference wider than [-1, 1] can need more
        raise AssertionError("values within [-1, 1] never need more than dict_bits")
    codes, deq = quantise_row(vals, lo, hi, b)
    if mode == DICT_DIFFERENCE:
        deq = np.asarray(prev, dtype=np.float64) + deq
    return mode, b, np.float32(lo), np.float32(hi), codes, deq


def code_dictionary(U, prev_tilde, dict_bits: int):
    """A window's dictionary U (T x k) column by column; prev_tilde is the
    previous window's dequantised dictionary (T x k_prev) or None.  Returns
    (list of per-column tuples, dequantised dictionary T x k)."""
    T, k = U.shape
    cols, Ut = [], np.empty((T, k))
    for j in range(k):
        prev = None
        if prev_tilde is not None and prev_tilde.shape[0] == T and j < prev_tilde.shape[1]:
            prev = prev_tilde[:, j]
        c = code_dictionary_column(U[:, j], prev, dict_bits)
        cols.append(c)
        Ut[:, j] = c[5]
    return cols, Ut


def decode_dictionary(cols, prev_tilde, T: int, dict_bits: int):
    """Rebuild a window's dequantised dictionary from its per-column (mode,
    bits, lo, hi, codes) and the previous window's, as a decoder does."""
    k = len(cols)
    Ut = np.empty((T, k))
    for j, (mode, b, lo, hi, codes, _deq) in enumerate(cols):
        vals = np.full(T, np.float64(lo)) if b == 0 else dequantise_uniform(codes, lo, hi, b)
        Ut[:, j] = prev_tilde[:, j] + vals if mode == DICT_DIFFERENCE else vals
    return Ut


# ---------------------------------------------------------------------------
# the record's bits (Eq. 13 per coordinate, for the stream as laid out)
# ---------------------------------------------------------------------------

def _align256(x: int) -> int:
    return (x + 255) // 256 * 256


def _seg_words(count: int, bits: int, raw_bytes: int) -> int:
    """Words of a segment of packed codes, or of raw values when bits is 0."""
    if bits:
        return words_for(count, bits)
    w = (count * raw_bytes + 3) // 4
    return w + (w & 1)


def record_bits(n: int, T: int, k: int, n_anchors: int, coef_bits: int, anchor_bits: int,
                dict_bits: int, raw_bytes: int, row_bits=None, dict_col_bits=None) -> dict:
    """Bits of one window's record by part, per vertex, frame and coordinate
    (divided by 3 n T), for the record layout: a 128-byte header; 16-byte
    table entries for the 3 k dictionary columns and the 3 k coefficient rows;
    three anchor ranges (8 bytes each); then, on 256-byte boundaries, the three
    anchor segments and the variable part (dictionary columns, then rows).
    Parts: q = row segments + row table, q_d = column segments + column
    table, q_a = anchor segments + ranges, q_s = all used bytes (header and
    alignment included).  row_bits / dict_col_bits: [3 k] bit widths (default:
    coef_bits / dict_bits for all)."""
    nq = 3 * k
    rb = [coef_bits] * nq if row_bits is None else [int(b) for b in row_bits]
    db = [dict_bits] * nq if dict_col_bits is None else [int(b) for b in dict_col_bits]
    rows = sum(32 * _seg_words(n, b if coef_bits else 0, raw_bytes) for b in rb)
    cols = sum(32 * _seg_words(T, b if dict_bits else 0, raw_bytes) for b in db)
    aseg = 4 * _seg_words(T * n_anchors, anchor_bits, raw_bytes)
    off_var = _align256(_align256(128 + 2 * nq * 16 + 24) + 3 * aseg)
    used = off_var + (rows + cols) // 8
    vf = 3.0 * n * T
    return {"q": (rows + nq * 128) / vf, "q_d": (cols + nq * 128) / vf,
            "q_a": 3 * (8 * aseg + 64) / vf, "q_s": 8.0 * used / vf}
