"""Host-side checks of constants the HIP kernels carry (no GPU)."""
import importlib.util
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2606_29794_amd", "csrc")


def _atan_coefficients():
    src = open(os.path.join(CSRC, "hp_offset.h")).read()
    body = src[src.index("hp_atan2_pos(float s, float c)"):]
    body = body[:body.index("return")]
    first = float(re.search(r"float r = ([-0-9.e]+)f;", body).group(1))
    rest = [float(sgn + x) for sgn, x in re.findall(r"r = r \* t2 ([+-]) ([0-9.e]+)f;", body)]
    return [first] + rest + [1.0]


def test_atan_polynomial_error_bound():
    """hp_atan2_pos evaluates atan t = t P(t^2) on [0, 1] with a degree-8 P
    from a minimax fit in relative error: with the float coefficients as
    stored, the polynomial is within 6e-8 relative of atan everywhere on
    [0, 1] (under one float ulp at 1), and a Lawson fit (fit_atan.py)
    reproduces the coefficients."""
    c = _atan_coefficients()
    assert len(c) == 9
    spec = importlib.util.spec_from_file_location("fit_atan", os.path.join(CSRC, "fit_atan.py"))
    fa = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fa)
    assert fa.rel_error(c) < 6e-8
    fit, err = fa.lawson_fit(passes=200)
    assert err < 2e-8
    np.testing.assert_allclose(fit, c, rtol=1e-4, atol=2e-6)
