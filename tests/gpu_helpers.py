"""Shared pieces of the GPU parity tests: tolerances and oracle runs."""
from __future__ import annotations

import sys

import numpy as np

import oracle

# Tolerances of the FP32 GPU path against the FP64 oracle.
SP_ABS = 1e-5        # per-net SP, TR_model, SP_acc, TR_acc, TR_hyb
POWER_REL = 1e-5     # total power
GRAD_REL = 1e-4      # gradients, with a floor of GRAD_FLOOR * max |g_ref|
GRAD_FLOOR = 1e-6


def say(*a):
    """Flushed progress line naming the case before a GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


def assert_grad_close(g, ref, what=""):
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    tol = GRAD_REL * np.abs(ref) + GRAD_FLOOR * (np.abs(ref).max() if ref.size else 0.0)
    err = np.abs(g - ref)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{what}: {bad.size} of {ref.size} gradient entries off; worst "
                           f"{err[bad].max():.3g} at {bad[np.argmax(err[bad])]} (ref "
                           f"{ref[bad[np.argmax(err[bad])]]:.6g})")


# A net's TR_model relative to the oracle's: every cell rule is a sum of
# products of p's and q's (no cancellation), so FP32 keeps relative accuracy
# even where TR_model is tiny; the bar is loose next to the rounding the
# test designs show (about 1e-6).
TR_REL = 1e-4


def assert_beta_close(beta, tr, f, what=""):
    """beta = clip(TR_acc / TR_model) on every net: TR_acc comes from exact
    counts (one float rounding), the quotient adds one more, and the clip
    cannot widen a difference, so |beta - beta_ref| <= beta_ref (r / (1 - r)
    + 2^-21) with r the net's relative TR_model error, itself within TR_REL.
    Where TR_model is 0 in the oracle (P is 0 or 1), beta follows the
    zero-denominator rule exactly."""
    beta = np.asarray(beta, np.float64)
    tr = np.asarray(tr, np.float64)
    ref_tr, ref_beta = f["tr_model"], f["beta"]
    zero = ref_tr == 0
    np.testing.assert_array_equal(beta[zero], ref_beta[zero], err_msg=what)
    r = np.abs(tr[~zero] - ref_tr[~zero]) / ref_tr[~zero]
    assert r.size == 0 or r.max() <= TR_REL, f"{what}: TR_model relative error {r.max():.3g}"
    bound = ref_beta[~zero] * (r / (1 - r) + 2.0 ** -21)
    err = np.abs(beta[~zero] - ref_beta[~zero])
    assert (err <= bound).all(), (f"{what}: beta off by {(err / bound).max():.3g} x its bound")


def assert_power_close(p, ref, what=""):
    p = np.asarray(p, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    np.testing.assert_allclose(p, ref, rtol=POWER_REL, atol=0, err_msg=what)


def oracle_column(o, p, cap, size=None, *, mode="modeled", n_words=0, seed=1, pi_words=None,
                  beta=None, ste=False, kappa=0.5):
    """Oracle forward + adjoint of one query column."""
    hybrid = mode == "hybrid"
    f = o.forward(p, cap, size, hybrid=hybrid, n_words=n_words, seed=seed, pi_words=pi_words,
                  kappa=kappa)
    if mode == "frozen":
        f = {**f, **o.power(f["sp"], cap, size, kappa=kappa, beta=beta)}
    adj = o.adjoint(f["sp"], f["beta"], cap, size, kappa=kappa, beta_ste=ste)
    return f, adj
