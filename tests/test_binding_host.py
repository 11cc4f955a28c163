"""Host-side checks of the refinement helpers of the binding module (CPU).

The helpers are Eqs. rich_extr and observed_order applied to three numbers;
on a sequence f(h) = f* + C h^p with h the inverse panel count they must
return p and f* exactly (up to rounding), whatever f*, C and p are.
"""

import pytest

from paper_1309_4018_amd.binding import observed_order, richardson


@pytest.mark.parametrize("p,ratio", [(1.0, 4.0), (2.0, 4.0), (1.5, 2.0)])
def test_exact_power_law(p, ratio):
    fstar, c = -41.2465, 7.5
    f = [fstar + c * (1.0 / n) ** p for n in (512.0, 512.0 * ratio, 512.0 * ratio ** 2)]
    got = observed_order(f[2], f[1], f[0], ratio)
    assert abs(got - p) < 1e-9
    assert abs(richardson(f[2], f[1], ratio, got) - fstar) < 1e-10
