"""Richardson extrapolation and observed order (sec. 2.4; test only).

Eq. rich_extr:       f_exact ~ f1 + (f1 - f2) / (r^p - 1)
Eq. observed_order:  p = log((f3 - f2) / (f2 - f1)) / log(r)
with f1 the finest and f3 the coarsest of three results refined at a
constant ratio r = h2/h1 = h3/h2.  Here h is the mean panel area, so r is
the ratio of panel counts.
"""

from __future__ import annotations

import math


def observed_order(f1, f2, f3, r):
    return math.log((f3 - f2) / (f2 - f1)) / math.log(r)


def richardson(f1, f2, r, p):
    return f1 + (f1 - f2) / (r ** p - 1.0)
