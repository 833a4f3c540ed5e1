"""Shared helpers of the GPU parity tests (not collected by pytest)."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2111_10105_amd import dmc


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def record_to_oracle(view: dmc.RecordView, p: dmc.Params, T: int, prev_tilde=None) -> dict:
    """The oracle's view of one GPU record: dequantised dictionary (per
    column, values or differences from prev_tilde, the previous window's
    [3][T][k] dequantised dictionary), coefficients and anchors, computed by
    the oracle's own dequantiser from the record's codes and tables."""
    k = min(p.k, T)
    rec = {"T": T, "k": k, "U_tilde": [], "Y_hat": [], "A_hat": []}
    for c in range(3):
        if p.dict_bits == 0:
            ut = view.dict_codes[c].astype(np.float64)
        else:
            ut = np.empty((T, k))
            for j in range(k):
                e = view.dict_table[c, j]
                b, mode = int(e["bits_mode"]) & 0xFF, (int(e["bits_mode"]) >> 8) & 0xFF
                vals = (np.full(T, np.float64(e["lo"])) if b == 0 else
                        O.dequantise_uniform(view.dict_codes[c, :, j], e["lo"], e["hi"], b))
                ut[:, j] = prev_tilde[c][:, j] + vals if mode else vals
        rec["U_tilde"].append(ut)
        if p.coef_bits:
            rows = []
            for r in range(k):
                b = int(view.row_bits[c, r])
                lo, hi = view.ranges[c, r, 0], view.ranges[c, r, 1]
                rows.append(np.full(view.codes.shape[2], np.float64(lo)) if b == 0 else
                            O.dequantise_uniform(view.codes[c, r], lo, hi, b))
            rec["Y_hat"].append(np.stack(rows))
        else:
            rec["Y_hat"].append(view.codes[c].astype(np.float64))
        if p.anchor_bits:
            a = O.dequantise_uniform(view.anchor_codes[c], view.anchor_range[c, 0],
                                     view.anchor_range[c, 1], p.anchor_bits)
        else:
            a = view.anchor_codes[c].astype(np.float64)
        rec["A_hat"].append(a.T)  # n_c x T
    return rec


def sin_angle(U, Q):
    """Largest principal angle (sine) between the column spans of U and Q."""
    Uo = O.orthonormalise(U)
    Qo = O.orthonormalise(Q)
    return float(np.linalg.norm(Qo - Uo @ (Uo.T @ Qo), 2))
