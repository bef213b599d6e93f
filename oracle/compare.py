"""Parity rule between a tested result and the oracle.

logL cannot cancel (a weighted sum of negative site terms), so its plain
relative error is used.  A branch gradient g_b can be ~0 through
cancellation between sites; it passes when |g - g*| <= tol * A_b with
A_b = sum_s w_s |term_{b,s}| >= |g*_b| (equality when the sites do not
cancel).  This is plain relative error wherever relative error is defined.
"""
from __future__ import annotations

import numpy as np


def parity_report(logL, grad, ref_logL, ref_grad, ref_abs, tol, branches=None):
    grad = np.asarray(grad, dtype=np.float64)
    ref_grad = np.asarray(ref_grad, dtype=np.float64)
    ref_abs = np.asarray(ref_abs, dtype=np.float64)
    if branches is None:
        branches = np.nonzero(np.isfinite(ref_grad))[0]
    branches = np.asarray(branches)
    err_logL = abs(logL - ref_logL) / abs(ref_logL) if ref_logL != 0 else abs(logL)
    diff = np.abs(grad[branches] - ref_grad[branches])
    scale = np.maximum(ref_abs[branches], np.finfo(np.float64).tiny)
    rel_a = diff / scale
    rel_plain = diff / np.maximum(np.abs(ref_grad[branches]), np.finfo(np.float64).tiny)
    inf_norm = diff.max() / max(np.abs(ref_grad[branches]).max(), np.finfo(np.float64).tiny) \
        if len(branches) else 0.0
    ok = bool(err_logL <= tol and (rel_a <= tol).all())
    return dict(ok=ok, logL_rel=float(err_logL),
                grad_rel_A_max=float(rel_a.max()) if len(branches) else 0.0,
                grad_rel_plain_max=float(rel_plain.max()) if len(branches) else 0.0,
                grad_inf_rel=float(inf_norm),
                n_cancelling=int((ref_abs[branches] > 10 * np.abs(ref_grad[branches])).sum()),
                n_checked=int(len(branches)))
