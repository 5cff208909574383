"""The decision rule of the parity tests (a helper module, not collected).

Decisions (rank, pivot columns) must match the oracle exactly, with one
admissible exception: a column whose updated pivot lies within the rounding
band of tol (oracle.ambiguity_band) may be decided either way by two correct
float64 evaluations.  Then the first differing decision must lie inside the
band, the oracle is re-run with the GPU's decisions (replay), every GPU
decision must agree with the replayed pivot values outside the band, and
the floating-point results are compared with that replay.
"""
import numpy as np

from oracle import geninv_ref as o


def _mask(piv, n):
    a = np.zeros(n, bool)
    a[np.asarray(piv, dtype=np.int64)] = True
    return a


def decisions_or_replay(G, ref, piv_gpu, tol=None):
    """Oracle result to compare with: ref itself when the GPU took the same
    decisions, else the oracle replayed with the GPU's decisions after
    checking that every difference is a legitimate rounding-band case.
    Returns (result, number of ambiguous decisions)."""
    n = ref.A.shape[0]
    acc_o = _mask(ref.piv, n)
    acc_g = _mask(piv_gpu, n)
    if np.array_equal(acc_o, acc_g):
        return ref, 0
    band = o.ambiguity_band(ref.A, ref.tol, acc_o)
    k = int(np.nonzero(acc_o != acc_g)[0][0])
    print(f"  ambiguous decision at column {k}: oracle d/tol={ref.d[k] / ref.tol:.6f}, band={band[k]:.3e}",
          flush=True)
    assert abs(ref.d[k] / ref.tol - 1.0) <= band[k]
    rep = o.geninv(G, tol, forced=acc_g)
    band = np.maximum(band, o.ambiguity_band(rep.A, rep.tol, acc_g))
    consistent = ((rep.d > rep.tol) == acc_g) | (np.abs(rep.d / rep.tol - 1.0) <= band)
    assert consistent.all(), np.nonzero(~consistent)[0][:10]
    return rep, int((acc_o != acc_g).sum())
