"""Comparison helpers shared by the GPU parity tests."""
import numpy as np

# (+,x) tolerances per entry, relative to the oracle's value
RTOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def assert_same_csc(got, ref, exact_values=False, what=""):
    """got / ref: objects with cp (int64 [n+1]), ir, num.  Patterns must be
    identical; values identical (exact) or within the dtype's tolerance."""
    assert np.array_equal(np.asarray(got.cp, dtype=np.int64), np.asarray(ref.cp, dtype=np.int64)), f"{what}: cp differs"
    assert np.array_equal(got.ir, ref.ir), f"{what}: row indices differ"
    assert_values(got.num, ref.num, exact_values, what)


def assert_values(got, ref, exact, what=""):
    if ref is None:
        assert got is None, f"{what}: expected a pattern result"
        return
    assert got.dtype == ref.dtype, f"{what}: dtype {got.dtype} vs {ref.dtype}"
    if exact or ref.dtype == np.int64:
        u = {8: np.uint64, 4: np.uint32}[ref.itemsize]
        bad = np.nonzero(got.view(u) != ref.view(u))[0]
        assert bad.size == 0, f"{what}: {bad.size} values differ, first at {bad[:5]}: {got[bad[:5]]} vs {ref[bad[:5]]}"
        return
    rtol = RTOL[ref.dtype]
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    lim = rtol * np.abs(ref.astype(np.float64))
    bad = np.nonzero(~(err <= lim))[0]  # NaN fails
    assert bad.size == 0, (f"{what}: {bad.size} values outside rtol {rtol}; first {bad[:5]}: "
                           f"{got[bad[:5]]} vs {ref[bad[:5]]}")
    # a zero must be the oracle's zero, sign included (Algorithm 1 starts each
    # sum from its first product, so products of -0.0 alone sum to -0.0)
    zs = np.nonzero(ref == 0)[0]
    badz = zs[np.signbit(got[zs]) != np.signbit(ref[zs])]
    assert badz.size == 0, f"{what}: {badz.size} zeros with the wrong sign, first at {badz[:5]}"


def columns_of(cp, ir, num, cols):
    """(cp, ir, num) of the listed columns of a CSC."""
    cp = np.asarray(cp, dtype=np.int64)
    lens = cp[np.asarray(cols) + 1] - cp[np.asarray(cols)]
    out_cp = np.zeros(len(cols) + 1, dtype=np.int64)
    np.cumsum(lens, out=out_cp[1:])
    idx = np.concatenate([np.arange(cp[j], cp[j + 1]) for j in cols]) if len(cols) else np.zeros(0, np.int64)
    return out_cp, ir[idx], (None if num is None else num[idx])
