"""Error measures of the parity tests: relative L2 error over all outputs of
a field, ||got - ref||_2 / ||ref||_2, and the maximum absolute error over the
largest reference magnitude, max|got - ref| / max|ref| (a local error
confined to a few modes or points shows in the second).  Arrays are compared
as flat vectors; complex spectra by their moduli of differences."""
import numpy as np


def rel_l2(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def max_ratio(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def both(got, ref):
    """The larger of the two measures: a bound on this holds for both."""
    return max(rel_l2(got, ref), max_ratio(got, ref))
