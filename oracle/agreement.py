"""Prop. 1 agreement, measured on the oracle (test infrastructure).

Prop. 1 (Sec. 5.3.1) replaces the exact test of the colour term, H(s) >=
H(s_t), by a comparison of two histogram intersections; the paper reports
that the two agree on 97% of the pixel-level and 89% of the block-level
updates it evaluated (Sec. 6.2). This module repeats that measurement on
synthetic images: before every phase of the oracle's schedule it takes each
proposed move (a boundary unit whose superpixel stays connected, and its best
neighbour n) and compares

  * Prop. 1: int(c_n, c_l) > int(c_{k\\l}, c_l), with normalised histograms,
    compared exactly by cross-multiplication; for one pixel of bin j this is
    h_n(j) (|A_k| - 1) > (h_k(j) - 1) |A_n|;
  * the exact change of H, in two forms: (a) H as defined by eqs. eqColorSum,
    eqColorMain and eqColorHistogram with each histogram normalised by its
    superpixel's size, in exact rational arithmetic; (b) the count form the
    proof of Prop. 1 (appendix) works with once the normalisation is dropped,
    sum_k sum_j h_k(j)^2, whose change is 2 sum_j h_l(j) (h_n(j) - h_k(j) +
    h_l(j)).

Reported over all proposals (agreement of the two tests) and over the moves
Prop. 1 accepts (the share that increase H). Both sides use strict
inequalities (acceptance needs an increase). Only the
colour term enters: Prop. 1 is a statement about H alone. The paper does not
say which of (a) and (b) its figures use; both are reported.

Run ``python -m oracle.agreement`` for the 481x321 workload figures.
"""
from __future__ import annotations

import json
import sys
from fractions import Fraction

import numpy as np

from . import Oracle


def _s2(v) -> int:
    return int(np.dot(v, v))


def _exact_gain_positive(hk, hn, hl, ak, an, m) -> bool:
    """Exact change of H (normalised histograms) when block l (m pixels,
    histogram hl) moves from k to n is > 0."""
    after = Fraction(_s2(hk - hl), (ak - m) ** 2) + Fraction(_s2(hn + hl), (an + m) ** 2)
    before = Fraction(_s2(hk), ak * ak) + Fraction(_s2(hn), an * an)
    return after > before


def _count_gain_positive(hk, hn, hl) -> bool:
    """Change of sum_k sum_j h_k(j)^2 (count form) is > 0."""
    return int(np.dot(hl, hn - hk + hl)) > 0


def _prop1_accepts(hk, hn, hl, ak, an, m) -> bool:
    hkl, akl = hk - hl, ak - m
    sn = int(np.minimum(hn * m, hl * an).sum())        # int(c_n, c_l) * an * m
    skl = int(np.minimum(hkl * m, hl * akl).sum())     # int(c_{k\\l}, c_l) * akl * m
    return sn * akl > skl * an


def agreement(rgb, K: int, levels: int, bins: int = 5, iters: int = 4, gamma: int = 1,
              rule: int = 0) -> dict:
    """Agreement counts over one cold-start refinement of rgb."""
    o = Oracle(rgb, K, levels, bins, iters, gamma, rule)
    B3 = bins ** 3
    px = {"agree": 0, "agree_count": 0, "total": 0, "prop1": 0, "exact": 0, "exact_count": 0,
          "prop1_and_exact": 0, "prop1_and_exact_count": 0}
    bl = dict(px)
    checked = 0
    while True:
        cls = o.next_phase()
        if cls < 0:
            break
        level = o.level
        side = 1 << level
        hist, size = o.histograms()
        b = o.bins()
        for d in o.decide(cls):
            if not d.boundary or not d.connect_ok or d.n < 0:
                continue
            k, n = d.k, d.n
            blk = b[d.uy * side:(d.uy + 1) * side, d.ux * side:(d.ux + 1) * side]
            hl = np.bincount(blk.ravel(), minlength=B3).astype(np.int64)
            m = int(blk.size)
            hk, hn = hist[k], hist[n]
            ak, an = int(size[k]), int(size[n])
            p1 = _prop1_accepts(hk, hn, hl, ak, an, m)
            ex = _exact_gain_positive(hk, hn, hl, ak, an, m)
            exc = _count_gain_positive(hk, hn, hl)
            if level > 0 and rule == 0:
                assert p1 == bool(d.accepted), "Prop. 1 test differs from the oracle's decision"
                checked += 1
            c = px if level == 0 else bl
            c["total"] += 1
            c["agree"] += p1 == ex
            c["agree_count"] += p1 == exc
            c["prop1"] += p1
            c["exact"] += ex
            c["exact_count"] += exc
            c["prop1_and_exact"] += p1 and ex
            c["prop1_and_exact_count"] += p1 and exc
        o.run(1)
    def rates(c):
        t = c["total"]
        p = c["prop1"]
        return dict(c, rate=c["agree"] / t if t else None,
                    rate_count=c["agree_count"] / t if t else None,
                    accepted_increase=c["prop1_and_exact"] / p if p else None,
                    accepted_increase_count=c["prop1_and_exact_count"] / p if p else None)
    return {"pixel": rates(px), "block": rates(bl),
            "block_decisions_checked_against_oracle": checked}


def main() -> int:
    from paper_1309_3848_amd import synth
    seeds = [int(a) for a in sys.argv[1:]] or [1]
    tot = {"pixel": [0, 0, 0, 0, 0, 0], "block": [0, 0, 0, 0, 0, 0]}
    for sd in seeds:
        img = synth.voronoi_image(321, 481, 30, 8.0, sd)
        r = agreement(img, 200, 3, 5, 4, 1, 0)
        for key in tot:
            tot[key][0] += r[key]["agree"]
            tot[key][1] += r[key]["agree_count"]
            tot[key][2] += r[key]["total"]
            tot[key][3] += r[key]["prop1"]
            tot[key][4] += r[key]["prop1_and_exact"]
            tot[key][5] += r[key]["prop1_and_exact_count"]
        print(json.dumps({"seed": sd, **r}), flush=True)
    print(json.dumps({k: {"proposals": t, "agree_normalised": a / t if t else None,
                          "agree_count_form": c / t if t else None, "prop1_accepted": p,
                          "accepted_increase_normalised": pe / p if p else None,
                          "accepted_increase_count_form": pc / p if p else None}
                      for k, (a, c, t, p, pe, pc) in tot.items()}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
