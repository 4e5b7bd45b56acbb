"""Element-wise and norm-wise comparison of a GPU result with the oracle's.

Both measures are asserted: the relative 2-norm error over the whole array, and the largest
point-wise error relative to the largest oracle value.  The second catches an error confined to
a few tile edges or one boundary row, which the 2-norm dilutes by about the square root of the
number of elements."""
import numpy as np


def errors(got, exp):
    """(relative 2-norm error, max |got - exp| / max |exp|) in float64."""
    g = np.asarray(got, np.float64)
    e = np.asarray(exp, np.float64)
    d = g - e
    rel2 = float(np.linalg.norm(d) / max(float(np.linalg.norm(e)), 1e-300))
    relmax = float(np.max(np.abs(d)) / max(float(np.max(np.abs(e))), 1e-300)) if e.size else 0.0
    return rel2, relmax


def assert_close(got, exp, tol, what="", say=None):
    """Both the norm-wise and the element-wise error of `got` against `exp` are <= tol."""
    rel2, relmax = errors(got, exp)
    if say is not None:
        say(f"  {what} rel2 {rel2:.3e} max {relmax:.3e}")
    assert rel2 <= tol and relmax <= tol, (what, rel2, relmax, tol)
    return rel2, relmax
