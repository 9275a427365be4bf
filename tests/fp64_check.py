"""Per-event FP64 parity rule shared by the GPU tests.

An event's FP64 |M|^2 must lie within 1e-12 (relative) of the oracle's
double-precision value.  An event outside it is judged against the oracle's
long-double value with a bound scaled by the event's condition number kappa
(oracle.Process.condition: the helicity- and colour-summed square with every
diagram amplitude, colour coefficient and colour-matrix entry replaced by its
absolute value, over |M|^2).  Relative errors of at most eps in every diagram
amplitude move |M|^2 by at most 2 eps kappa; an FP64 amplitude of these tree
diagrams passes through fewer than 256 roundings (external states,
propagators, vertex contractions along the longest chain), so any correct
FP64 evaluation lies within 512 u kappa of the exact value, u = 2^-53.  Where
diagrams cancel (soft and collinear gluons, gauge cancellations) kappa reaches
1e5 and no FP64 evaluation, the oracle's included, meets 1e-12."""
import numpy as np

TOL = 1e-12
U = 2.0 ** -53
K_FP64 = 512.0


def check(got, d, ld, kappa, tol=TOL):
    """got: GPU values; d: the oracle's double values; ld, kappa: the
    oracle's long-double values and condition numbers, as arrays or as
    callables of an index array (so that only the outliers are evaluated).
    Returns (relative error against d, number of outliers, largest outlier
    error against ld in units of u kappa)."""
    rel = np.abs(got / d - 1.0)
    bad = np.nonzero(rel > tol)[0]
    worst = 0.0
    if len(bad):
        ldb = ld(bad) if callable(ld) else ld[bad]
        kb = kappa(bad) if callable(kappa) else kappa[bad]
        rel_ld = np.abs(got[bad] / ldb - 1.0)
        ok = rel_ld <= np.maximum(tol, K_FP64 * U * kb)
        assert np.all(ok), (bad[~ok][:10], rel[bad][~ok][:10], rel_ld[~ok][:10], kb[~ok][:10])
        worst = float(np.max(rel_ld / (U * kb)))
    return rel, len(bad), worst
