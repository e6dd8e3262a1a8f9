"""Decision statistics of the attribution protocol (Sec. IV): a pair is
declared "same camera" when its PCE exceeds a threshold (60).  Host-side
summaries of PCE values the library computed; no method arithmetic.

* tpr(matched, thr): fraction of same-camera PCEs above thr;
* fpr(unmatched, thr): fraction of different-camera PCEs above thr;
* roc(matched, unmatched): (FPR, TPR) at every distinct threshold, from
  (0, 0) to (1, 1);
* auc(matched, unmatched): area under that curve, equal to the probability
  that a same-camera PCE exceeds a different-camera one (ties count 1/2).
"""
from __future__ import annotations

import numpy as np

THRESHOLD = 60.0


def tpr(matched, thr: float = THRESHOLD) -> float:
    m = np.asarray(matched, dtype=np.float64).ravel()
    return float(np.mean(m > thr)) if m.size else float("nan")


def fpr(unmatched, thr: float = THRESHOLD) -> float:
    u = np.asarray(unmatched, dtype=np.float64).ravel()
    return float(np.mean(u > thr)) if u.size else float("nan")


def roc(matched, unmatched):
    """(fpr, tpr) arrays at thresholds just below every distinct value, in
    increasing FPR; the first point is (0, 0) and the last (1, 1)."""
    m = np.asarray(matched, dtype=np.float64).ravel()
    u = np.asarray(unmatched, dtype=np.float64).ravel()
    thr = np.unique(np.concatenate([m, u]))[::-1]  # descending
    ms, us = np.sort(m), np.sort(u)
    # counts of values >= t for each threshold t
    tp = m.size - np.searchsorted(ms, thr, side="left")
    fp = u.size - np.searchsorted(us, thr, side="left")
    f = np.concatenate([[0.0], fp / max(u.size, 1)])
    t = np.concatenate([[0.0], tp / max(m.size, 1)])
    return f, t


def auc(matched, unmatched) -> float:
    """P(matched > unmatched) + P(equal) / 2 over all pairs (rank statistic)."""
    m = np.asarray(matched, dtype=np.float64).ravel()
    u = np.asarray(unmatched, dtype=np.float64).ravel()
    if not m.size or not u.size:
        return float("nan")
    us = np.sort(u)
    below = np.searchsorted(us, m, side="left")
    equal = np.searchsorted(us, m, side="right") - below
    return float((below.sum() + 0.5 * equal.sum()) / (m.size * u.size))
