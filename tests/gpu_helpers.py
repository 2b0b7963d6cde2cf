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
# test designs show (about 1e-6).  The oracle computes P alone in FP64, so
# its 1 - P cancels near P = 1: its P carries an absolute rounding error of
# a few thousand eps64 at most (about 1e-13 along the deepest paths), and
# its TR_model a relative error of that over min(P, 1 - P), which the bar
# adds (ORACLE_P_ABS).
TR_REL = 1e-4
ORACLE_P_ABS = 2.0 ** -40


def assert_beta_close(beta, tr, f, what="", beta_min=0.1, beta_max=10.0):
    """beta = clip(TR_acc / TR_model) on every net: TR_acc comes from exact
    counts (one float rounding), the quotient adds one more, and the clip
    cannot widen a difference, so |beta - beta_ref| <= beta_ref (r / (1 - r)
    + 2^-21) with r the net's relative TR_model difference, itself within
    TR_REL plus the oracle's own rounding.
    Where the oracle's TR_model is 0 its P is 0 or 1 only to within its
    own rounding (its 1 - P cancels), while the kernels keep the smaller of
    P and 1 - P exactly: there the GPU's TR_model must lie below the
    oracle's resolution, and beta must follow the rule (0/0 -> 1, x/0 ->
    beta_max, else the clipped ratio) on the GPU's own TR_model and the
    exact TR_acc."""
    beta = np.asarray(beta, np.float64)
    tr = np.asarray(tr, np.float64)
    ref_tr, ref_beta = f["tr_model"], f["beta"]
    zero = ref_tr == 0
    assert (tr[zero] <= 4 * ORACLE_P_ABS).all(), f"{what}: TR_model where the oracle's is 0"
    ta = f["tr_acc"][zero]
    with np.errstate(divide="ignore", invalid="ignore"):
        rule = np.where(tr[zero] == 0, np.where(ta == 0, 1.0, beta_max),
                        np.clip(ta / tr[zero], beta_min, beta_max))
    np.testing.assert_allclose(beta[zero], rule, rtol=2.0 ** -20, atol=0, err_msg=what)
    r = np.abs(tr[~zero] - ref_tr[~zero]) / ref_tr[~zero]
    P = f["sp"][~zero]
    allowed = TR_REL + ORACLE_P_ABS / np.minimum(P, 1 - P)
    worst = np.argmax(r / allowed) if r.size else 0
    assert r.size == 0 or (r <= allowed).all(), (
        f"{what}: TR_model relative error {r[worst]:.3g} at P = {P[worst]:.17g}")
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
