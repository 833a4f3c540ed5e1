"""The packed stream (Sec. IV: Eq. 13's bits, Fig. 5's bits per row, Fig. 6's
dictionary as differences of consecutive blocks) on the GPU, against the
stream oracle (oracle/bitstream.py): every segment's words equal the oracle's
packing of the oracle's codes of the GPU's own coefficients and dictionary,
the bits per row follow the oracle's rule on the stored ranges, the
adaptive dictionary decodes (on the host, with the oracle's dequantiser) to
within half the plain code's step of the exact eigenvectors, and the GPU's
decode of such streams matches the oracle's decode of the same records.
Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from oracle import bitstream as B
from paper_2111_10105_amd import dmc
from synth import animate, configs, meshes

from gpu_helpers import record_to_oracle, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = dmc.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def _words(count, bits, real):
    w = (count * bits + 31) // 32 if bits else (count * real + 3) // 4
    return w + w % 2


def _check_packing(view, n, T, k, p, fr, anchors, U, Y):
    """Segments of one record against the oracle: dictionary (plain), rows
    (Eq. 10 at coef_bits, or the bits of coef_step), anchors; offsets and
    used bytes as the format lays them out."""
    fp32 = p.precision != dmc.FP64
    real = 4 if fp32 else 8
    off = 0
    # dictionary columns: plain code over [-1, 1] of the GPU's U
    for c in range(3):
        for j in range(k):
            e = view.dict_table[c, j]
            assert int(e["word_off"]) == off
            b = int(e["bits_mode"]) & 0xFF
            seg = view.var_words[off:off + _words(T, b if p.dict_bits else 0, real)]
            if p.dict_bits:
                assert b == p.dict_bits and e["lo"] == -1.0 and e["hi"] == 1.0
                codes = O.quantise_uniform(U[c][:, j], -1.0, 1.0, p.dict_bits)
                assert np.array_equal(seg, B.pack_bits(codes, b))
            off += _words(T, b if p.dict_bits else 0, real)
    # coefficient rows
    for c in range(3):
        yc = Y[c].astype(np.float64)
        if p.coef_bits and p.coef_step > 0:
            codes, ranges, bits, _ = B.quantise_rows_step(Y[c], p.coef_step, fp32,
                                                          max_bits=p.coef_bits)
        elif p.coef_bits:
            codes, ranges, _ = O.quantise_rows(yc if not fp32 else Y[c], p.coef_bits, fp32)
            bits = np.full(k, p.coef_bits)
        for r in range(k):
            assert int(view.row_bits[c, r]) == (int(bits[r]) if p.coef_bits else 0)
            nwd = _words(n, int(bits[r]) if p.coef_bits else 0, real)
            seg = view.var_words[off:off + nwd]
            if p.coef_bits:
                assert np.array_equal(view.ranges[c, r], ranges[r])
                assert np.array_equal(seg, B.pack_bits(codes[r], int(bits[r])))
            else:
                assert np.array_equal(seg.view(Y.dtype)[:n], Y[c, r])
            off += nwd
    assert view.used_bytes == len(view.var_words) * 4 + (view.used_bytes - 4 * off)
    assert len(view.var_words) == off
    # anchors
    for c in range(3):
        a = O.anchor_values(fr, anchors, c)
        if p.anchor_bits:
            lo, hi = O.stored_range(a.astype(np.float32) if fp32 else a)
            assert np.array_equal(view.anchor_range[c], np.array([lo, hi], dtype=np.float32))
            codes = O.quantise_uniform(a, lo, hi, p.anchor_bits).T.ravel()
            assert np.array_equal(view.anchor_words[c], B.pack_bits(codes, p.anchor_bits))


@pytest.mark.parametrize("prec", [dmc.FP32, dmc.FP64])
@pytest.mark.parametrize("bits", [(12, 16, 16, 0.0), (7, 11, 13, 0.0), (16, 16, 16, 1e-4),
                                  (12, 16, 16, 3e-3), (0, 0, 0, 0.0), (5, 3, 1, 0.0)])
def test_window_record_packing(ctx, prec, bits):
    cb, ab, db, step = bits
    T, k = 16, 6
    v, t = meshes.torus(24, 20)
    n = v.shape[0]
    dt = np.float64 if prec == dmc.FP64 else np.float32
    fr = animate.rbf_skinning(v, T, 4, seed=21, dtype=dt)
    anchors = animate.choose_anchors(n, 7, seed=4)
    m = dmc.Mesh(ctx, n, t, anchors)
    p = dmc.make_params(k, coef_bits=cb, anchor_bits=ab, dict_bits=db, precision=prec,
                        coef_step=step, cg_tol=1e-13)
    r = dmc.encode_window(ctx, m, to_dev(fr), p, want_coef=True)
    assert r["status"] == 0
    view = dmc.parse_record(_np(r["code"]), n, T, anchors.size, p)
    assert list(view.header[:10]) == [0x32434D44, T, k, n, anchors.size, cb, ab, db, prec, 0]
    _check_packing(view, n, T, k, p, fr, anchors, _np(r["u"]).astype(np.float64), _np(r["coef"]))
    # the record's bytes beyond its stream are zero; the stats count its parts
    buf = _np(r["code"])
    assert not buf[view.used_bytes:].any()
    st = r["stats"]
    real = 4 if prec == dmc.FP32 else 8
    vf = 3 * n * T
    q = sum(32 * _words(n, int(b) if cb else 0, real) + 128 for b in view.row_bits.ravel()) / vf
    assert st["q"] == pytest.approx(q, rel=1e-12)
    assert st["q_s"] == pytest.approx(8 * view.used_bytes / vf, rel=1e-12)
    # decode: the GPU against the oracle's decode of this record
    out, _, status = dmc.decode_window(ctx, m, r["code"], T, p)
    assert status == 0
    ref = O.decode_window(O.AnchoredSolver(O.laplacian(n, t), anchors), record_to_oracle(view, p, T))
    tol = 1e-20 if prec == dmc.FP64 else 1e-11
    assert O.nmse(_np(out), ref) <= tol


def test_row_step_saves_bits_at_equal_distortion(ctx):
    """Bits per row for a common step (Fig. 5 reading): starting from the
    step whose squared error over all coefficients equals the plain
    quantiser's and halving it until the reconstruction error against the
    input is no larger than the plain one's, the rows still take far fewer
    bits in all."""
    w = configs.torus_fp32(frames=64)
    m = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    fr = to_dev(w.frames)
    p = dmc.make_params(w.k, coef_bits=12, precision=dmc.FP32, init=dmc.INIT_EXACT)
    codes, out, st, status = dmc.compress_sequence(ctx, m, fr, w.T, p)
    assert status == 0
    views = []
    nb = dmc.window_code_bytes(w.n, w.T, m.nc, p)
    buf = _np(codes)
    for wi in range(w.F // w.T):
        views.append(dmc.parse_record(buf[wi * nb:(wi + 1) * nb], w.n, w.T, m.nc, p))
    # the plain steps (hi - lo) / 4095 of all rows; the common step with the same sum of squares
    steps = np.concatenate([(v.ranges[..., 1] - v.ranges[..., 0]).ravel() / 4095.0 for v in views])
    step = float(np.sqrt(np.mean(steps.astype(np.float64) ** 2)))
    q_plain = sum(s["q"] for s in st)
    e_plain = O.nmse(_np(out), w.frames)
    for _ in range(6):
        ps = dmc.make_params(w.k, coef_bits=16, precision=dmc.FP32, init=dmc.INIT_EXACT,
                             coef_step=step)
        codes_s, out_s, st_s, status = dmc.compress_sequence(ctx, m, fr, w.T, ps)
        assert status == 0
        q_step = sum(s["q"] for s in st_s)
        e_step = O.nmse(_np(out_s), w.frames)
        print(f"q plain {q_plain / len(st):.4f} step {q_step / len(st):.4f}  "
              f"NMSE plain {e_plain:.4e} step {e_step:.4e}  step {step:.3e}")
        if e_step <= e_plain:
            break
        step /= 2
    assert e_step <= e_plain
    assert q_step < 0.75 * q_plain
    # every row within the bound its bits promise
    for wi in range(w.F // w.T):
        v = dmc.parse_record(_np(codes_s)[wi * nb:(wi + 1) * nb], w.n, w.T, m.nc, ps)
        for c in range(3):
            for r in range(w.k):
                lo, hi = v.ranges[c, r]
                assert int(v.row_bits[c, r]) == B.bits_for_step(lo, hi, step, 16)


@pytest.mark.parametrize("prec", [dmc.FP64, dmc.FP32])
def test_adaptive_dictionary_sequence(ctx, prec):
    """Dictionaries coded per column as values or as differences from the
    previous window's (gapped windows, so the exact eigenvectors are fixed by
    the data): the first window uses values only; the decoded dictionaries,
    rebuilt on the host with the oracle's dequantiser and the tables, are
    within half the plain 16-bit step of the oracle's eigenvectors; the bits
    of every column follow the oracle's rule on its stored range; decoding
    a single record that refers to its predecessor is refused; and the GPU's
    decode of the sequence matches the oracle's decode of the same records."""
    T, k, F = 16, 6, 56
    v, t = meshes.torus(30, 26)
    n = v.shape[0]
    dt = np.float64 if prec == dmc.FP64 else np.float32
    # nearby eigenvectors from window to window (a small drift of one basis)
    fr = animate.gapped_windows(v, F, T, k, seed=77, drift=0.01, dtype=dt)
    anchors = animate.choose_anchors(n, 9, seed=78)
    m = dmc.Mesh(ctx, n, t, anchors)
    p = dmc.make_params(k, coef_bits=12, precision=prec, init=dmc.INIT_EXACT,
                        dict_mode=dmc.DICT_ADAPTIVE, cg_tol=1e-13)
    codes, out, stats, status = dmc.compress_sequence(ctx, m, to_dev(fr), T, p)
    assert status == 0
    buf = _np(codes)
    L = O.laplacian(n, t)
    solver = O.AnchoredSolver(L, anchors)
    step = 2.0 / 65535
    off, prev, refs = 0, None, []
    views = []
    for wi, (s0, s1) in enumerate(O.windows(F, T)):
        Tw = s1 - s0
        nb = dmc.window_code_bytes(n, Tw, m.nc, p)
        view = dmc.parse_record(buf[off:off + nb], n, Tw, m.nc, p)
        views.append(view)
        modes = view.dict_modes
        if wi == 0 or Tw != T:
            assert not modes.any() and view.header[10] == 0
        rec = record_to_oracle(view, p, Tw, prev_tilde=prev if Tw == T else None)
        for c in range(3):
            _, V = O.exact_subspace(O.autocorrelation(O.coordinate_matrix(fr[s0:s1], c)), min(k, Tw))
            assert np.max(np.abs(rec["U_tilde"][c] - V)) <= step / 2 + 1e-9
            for j in range(min(k, Tw)):
                e = view.dict_table[c, j]
                assert (int(e["bits_mode"]) & 0xFF) == B.bits_for_step(e["lo"], e["hi"], step, 16)
        refs.append(O.decode_window(solver, rec))
        prev = rec["U_tilde"]
        off += nb
    n_diff = sum(int(v.dict_modes.sum()) for v in views)
    print(f"difference-coded columns: {n_diff} of {sum(v.dict_modes.size for v in views)}; "
          f"q_d per window {[round(s['q_d'], 5) for s in stats]}")
    ref = np.concatenate(refs)
    tol = 1e-20 if prec == dmc.FP64 else 1e-11
    assert O.nmse(_np(out), ref) <= tol
    # a record whose dictionary refers to its predecessor cannot be decoded alone
    if any(v.header[10] for v in views):
        wi = next(i for i, v in enumerate(views) if v.header[10])
        nb = dmc.window_code_bytes(n, T, m.nc, p)
        with pytest.raises(dmc.DmcError) as e:
            dmc.decode_window(ctx, m, codes[wi * nb:(wi + 1) * nb], T, p)
        assert e.value.status == 1
