"""Relative force error statistics (test infrastructure, float64 numpy).

e_i = |a_i - a_ref,i|_2 / |a_ref,i|_2; percentiles with
numpy.quantile(method="higher"), so a reported percentile is always one of
the observed errors.  Particles whose reference force is below 1e-6 times
the median reference magnitude are counted apart (``tiny``), since a
relative error is not meaningful there.

Test infrastructure only (see the package docstring).  Parity: pinned by
tests/test_oracle_metrics.py on hand-built errors whose norms, quantiles
and tiny counts are worked out by hand.
"""

from __future__ import annotations

import numpy as np


def relative_errors(acc, ref):
    acc = np.asarray(acc, np.float64)
    ref = np.asarray(ref, np.float64)
    num = np.linalg.norm(acc - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    med = float(np.median(den)) if len(den) else 0.0
    tiny = den <= 1e-6 * med
    e = np.where(tiny, 0.0, num / np.where(tiny, 1.0, den))
    return e, tiny


def error_summary(acc, ref):
    e, tiny = relative_errors(acc, ref)
    ok = e[~tiny]
    if ok.size == 0:
        return dict(n=0, tiny=int(tiny.sum()), median=0.0, p999=0.0, max=0.0)
    return dict(
        n=int(ok.size),
        tiny=int(tiny.sum()),
        median=float(np.quantile(ok, 0.5, method="higher")),
        p99=float(np.quantile(ok, 0.99, method="higher")),
        p999=float(np.quantile(ok, 0.999, method="higher")),
        max=float(ok.max()),
    )
