"""Comparison of a GPU output with the oracle's, counted on the signal.

An entry is close when |gpu - oracle| <= rel * max(|oracle|, 1e-3 * max|oracle|).
Time-of-flight images and histograms are mostly zero (a narrow gate lights a
few percent of the pixels, a transient histogram a fraction of a percent of
its bins), so the fraction of close entries is taken over the support: the
entries where either side is non-zero.  The fraction over all entries is
reported beside it, with the support's size and the largest discrepancies.
"""
import math

import numpy as np

REL = 1e-4


def compare(g, o, rel=REL, topk=5):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    scale = max(float(np.abs(o).max()) if o.size else 0.0, 1e-30)
    floor = np.maximum(np.abs(o), 1e-3 * scale)
    err = np.abs(g - o)
    close = err <= rel * floor
    support = (g != 0) | (o != 0)
    n_sup = int(support.sum())
    frac_sup = float(close[support].mean()) if n_sup else 1.0
    d = (g - o)[~close]
    z = float(d.sum() / math.sqrt(float((d * d).sum()))) if d.size else 0.0
    relerr = np.where(support, err / floor, 0.0)
    order = np.argsort(relerr, axis=None)[::-1][:topk]
    top = []
    for flat in order:
        if relerr.flat[flat] <= rel:
            break
        top.append((np.unravel_index(flat, g.shape), float(g.flat[flat]), float(o.flat[flat])))
    return dict(frac_support=frac_sup, frac_all=float(close.mean()) if close.size else 1.0, support=n_sup,
                outside=int((~close).sum()), z=z, top=top, sum_gpu=float(g.sum()), sum_oracle=float(o.sum()),
                close=close)


def describe(what, r):
    s = (f"{what}: {r['frac_support'] * 100:.4f}% of {r['support']} support entries within {REL} "
         f"({r['frac_all'] * 100:.4f}% of all; {r['outside']} outside, sign z {r['z']:+.2f}), "
         f"sums gpu {r['sum_gpu']:.7g} oracle {r['sum_oracle']:.7g}")
    for idx, gv, ov in r["top"]:
        s += f"\n    at {tuple(int(i) for i in idx)}: gpu {gv:.7g} oracle {ov:.7g}"
    return s
