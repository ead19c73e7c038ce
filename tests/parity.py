"""Comparison of a GPU result with the oracle under the near-tie rule.

With a shared uniform stream the masks must be identical, except on runs where
the first differing index k has |u_k - d_k| below a threshold (d_k the
oracle's pre-decision probability): such runs are counted as near ties (a
rounding-level difference in d_k decided a comparison that was within rounding
of a tie). Later differences follow from the diverged histories and are not
compared. Pre-decision probabilities are compared up to and including k.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class ParityResult:
    ok: bool
    near_tie: bool
    first_diff: int       # -1 if masks are identical
    max_dd: float         # max |d_gpu - d_oracle| over the compared prefix
    ll_rel: float         # |ll_gpu - ll_oracle| / |ll_oracle| (masks identical), else nan
    min_gap: float        # min_j |u_j - d_j| over the oracle run
    why: str = ""


def compare(gpu_mask, gpu_piv, gpu_ll, ora, u, tol, thr) -> ParityResult:
    gm = np.asarray(gpu_mask).astype(np.uint8)
    om = np.asarray(ora["mask"]).astype(np.uint8)
    n = om.shape[0]
    d_o = np.asarray(ora["predec"])[:n]
    d_g = np.asarray(gpu_piv)[:n] + 1.0 - gm
    u = np.asarray(u)[:n]
    gap = float(np.min(np.abs(u - d_o))) if n else np.inf
    diff = np.nonzero(gm != om)[0]
    if diff.size == 0:
        dd = float(np.max(np.abs(d_g - d_o))) if n else 0.0
        ll_o = ora["loglik"]
        ll_rel = abs(gpu_ll - ll_o) / max(abs(ll_o), 1e-300)
        ok = dd <= tol and ll_rel <= tol
        return ParityResult(ok, False, -1, dd, ll_rel, gap,
                       "" if ok else f"max|dd|={dd:.3g} ll_rel={ll_rel:.3g} > tol={tol:g}")
    k = int(diff[0])
    dd = float(np.max(np.abs(d_g[:k + 1] - d_o[:k + 1])))
    tie = abs(u[k] - d_o[k]) < thr
    ok = tie and dd <= tol
    why = "" if ok else (f"mask differs at {k}: |u-d|={abs(u[k] - d_o[k]):.3g} >= thr={thr:g}"
                         if not tie else f"max|dd|={dd:.3g} > tol={tol:g}")
    return ParityResult(ok, tie, k, dd, float("nan"), gap, why)
