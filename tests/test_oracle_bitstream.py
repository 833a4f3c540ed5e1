"""Pins of the stream oracle (oracle/bitstream.py) against brute force and the
bounds its readings promise: packing bit for bit, the fewest bits of a row
for a step, the error bound of the bits per row (Fig. 5), and the dictionary
coded as differences of consecutive blocks (Fig. 6)."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import bitstream as B


@pytest.mark.parametrize("bits", list(range(1, 17)))
def test_pack_unpack_round_trip(bits):
    rng = np.random.default_rng(bits)
    for count in (0, 1, 31, 32, 33, 1000):
        codes = rng.integers(0, 1 << bits, size=count, dtype=np.uint64)
        words = B.pack_bits(codes, bits)
        assert words.dtype == np.uint32
        assert words.size == B.words_for(count, bits)
        assert np.array_equal(B.unpack_bits(words, count, bits), codes.astype(np.uint32))


@pytest.mark.parametrize("bits", [1, 3, 7, 10, 12, 13, 16])
def test_pack_bit_order_brute_force(bits):
    """Bit i of the segment (bit i mod 32 of word i // 32) is bit i mod b of
    code i // b: checked bit by bit in plain Python."""
    rng = np.random.default_rng(100 + bits)
    codes = [int(c) for c in rng.integers(0, 1 << bits, size=77)]
    words = [int(w) for w in B.pack_bits(np.array(codes, dtype=np.uint64), bits)]
    nbits = 77 * bits
    for i in range(32 * len(words)):
        got = (words[i // 32] >> (i % 32)) & 1
        want = (codes[i // bits] >> (i % bits)) & 1 if i < nbits else 0
        assert got == want, (i, got, want)


def test_words_for_rounds_to_eight_bytes():
    for count, bits in itertools.product((0, 1, 5, 64, 65, 1000), (1, 5, 12, 16)):
        w = B.words_for(count, bits)
        assert w % 2 == 0 and 32 * w >= count * bits and 32 * (w - 2) < count * bits or \
            (count * bits == 0 and w == 0)


def test_bits_for_step_is_the_fewest():
    rng = np.random.default_rng(5)
    for _ in range(500):
        lo = float(np.float32(rng.uniform(-3, 1)))
        hi = float(np.float32(lo + rng.uniform(0, 4) * rng.choice([1e-6, 1e-3, 1.0])))
        step = float(rng.uniform(1e-5, 1e-1))
        b = B.bits_for_step(lo, hi, step)
        width = hi - lo
        if width == 0.0:
            assert b == 0
            continue
        assert 1 <= b <= 16
        if b < 16:
            assert width / step <= (1 << b) - 1
        if b > 1:
            assert width / step > (1 << (b - 1)) - 1


def test_rows_with_a_common_step_keep_the_error_bound():
    """Each row's error is within half the common step, the widest row takes
    the bits the step was derived from and codes as Eq. (10) does, and rows
    of smaller range take fewer bits."""
    rng = np.random.default_rng(9)
    k, n = 8, 500
    scales = 2.0 ** -np.arange(k)
    Y = (rng.standard_normal((k, n)) * scales[:, None]).astype(np.float32).astype(np.float64)
    wmax = max(float(O.stored_range(Y[r])[1]) - float(O.stored_range(Y[r])[0]) for r in range(k))
    step = wmax / ((1 << 12) - 1)
    codes, ranges, bits, deq = B.quantise_rows_step(Y, step, fp32_data=True)
    assert bits[0] == 12 and np.all(np.diff(bits) <= 0) and bits[-1] < 12
    for r in range(k):
        assert np.max(np.abs(deq[r] - Y[r])) <= step / 2 * (1 + 1e-12)
    c12, r12, d12 = O.quantise_rows(Y[:1], 12, fp32_data=True)
    assert np.array_equal(codes[0], c12[0]) and np.array_equal(deq[0], d12[0])


def test_dictionary_columns_as_differences():
    """Window 0 is sent as values; later windows take differences where they
    need fewer bits; every entry is within half the plain 16-bit step of U;
    a decoder rebuilds the dequantised dictionaries bit for bit; identical
    consecutive windows cost at most one bit per entry."""
    rng = np.random.default_rng(3)
    T, k, nw = 16, 5, 4
    Us = []
    base = O.orthonormalise(rng.standard_normal((T, k)))
    for w in range(nw):
        drift = 0.02 * rng.standard_normal((T, k)) if w else 0.0
        U = O.sign_fix(O.orthonormalise(base + drift))
        U[:, 0] = O.sign_fix(np.full((T, 1), 1.0 / np.sqrt(T)))[:, 0]  # a constant column
        Us.append(U)
    Us.append(Us[-1].copy())  # a repeated window
    step = 2.0 / 65535
    prev, prev_dec = None, None
    for w, U in enumerate(Us):
        cols, Ut = B.code_dictionary(U, prev, 16)
        if w == 0:
            assert all(c[0] == B.DICT_VALUES for c in cols)
        assert np.max(np.abs(Ut - U)) <= step / 2 * (1 + 1e-9)
        dec = B.decode_dictionary(cols, prev_dec, T, 16)
        assert np.array_equal(dec, Ut)
        assert cols[0][1] == 0  # the constant column: one value, no bits
        if w == len(Us) - 1:
            assert all(c[0] == B.DICT_DIFFERENCE and c[1] <= 1 for c in cols[1:])
        if 0 < w < len(Us) - 1:
            # small drifts: the differences need fewer bits than the values,
            # except where the sign rule flipped a column between windows
            diff = [c for c in cols[1:] if c[0] == B.DICT_DIFFERENCE]
            assert len(diff) >= k - 2 and all(c[1] <= 13 for c in diff)
        prev, prev_dec = Ut, dec
