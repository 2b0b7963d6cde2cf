"""Rank agreement of two gradient vectors (Sec. V-C): Pearson correlation,
overlap of the top-k sets by magnitude, and their Jaccard index.  Host-side
analysis of results; nothing here is on the device path."""
from __future__ import annotations

import numpy as np


def top_k(v, k: int) -> np.ndarray:
    """Indices of the k largest |v| (ties broken by index)."""
    v = np.abs(np.asarray(v, dtype=np.float64))
    order = np.lexsort((np.arange(v.size), -v))
    return order[:k]


def top_k_overlap(a, b, k: int) -> float:
    """|top_k(a) & top_k(b)| / k."""
    return len(set(top_k(a, k)) & set(top_k(b, k))) / float(k)


def jaccard_top_k(a, b, k: int) -> float:
    """|top_k(a) & top_k(b)| / |top_k(a) | top_k(b)|."""
    sa, sb = set(top_k(a, k)), set(top_k(b, k))
    return len(sa & sb) / float(len(sa | sb))


def pearson(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a = a - a.mean()
    b = b - b.mean()
    den = np.sqrt((a * a).sum() * (b * b).sum())
    return float((a * b).sum() / den) if den > 0 else float("nan")


def agreement(analytic, reference, k: int) -> dict:
    return dict(pearson=pearson(analytic, reference),
                top_k_overlap=top_k_overlap(analytic, reference, k),
                jaccard_top_k=jaccard_top_k(analytic, reference, k), k=k)
