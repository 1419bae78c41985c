"""Order-independent fingerprints of a set of groups (histories + amplitudes).

Test infrastructure: used by the script that writes the stored oracle runs and
by the tests that compare the library's groups with them.  It holds none of
the method's arithmetic -- only a hash of the integer histories and two
weighted sums of the amplitudes, so that two group sets can be compared step
by step without storing them.

For a set {(h_i, w_i)} with h_i the pair index at lags 0..K-1 (uint8) and w_i
complex:

* ``n``     -- the number of groups;
* ``hsum``  -- sum over i of mix64(poly(h_i)) mod 2^64, where
               poly(h) = sum_j (h_j + 1) * B^j mod 2^64 (B = 0x100000001B3) and
               mix64 is the SplitMix64 finaliser (Steele, Lea, Flood 2014);
* ``wsum``  -- sum over i of w_i * u_i with u_i = (mix64(poly(h_i) ^ S) >> 11) * 2^-53,
               a pseudo-random weight in [0, 1) attached to the history;
* ``wabs``  -- sum over i of |w_i|.

Equal sets give equal (n, hsum) exactly and equal (wsum, wabs) up to the
rounding of the amplitudes and of the summation order.
"""
from __future__ import annotations

import numpy as np

_B = np.uint64(0x100000001B3)
_S = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def _poly(hist: np.ndarray) -> np.ndarray:
    n, K = hist.shape
    x = np.zeros(n, dtype=np.uint64)
    b = np.uint64(1)
    for j in range(K):
        x = x + (hist[:, j].astype(np.uint64) + np.uint64(1)) * b
        b = b * _B
    return x


def fingerprint(hist, w) -> dict:
    hist = np.asarray(hist, dtype=np.uint8)
    w = np.asarray(w, dtype=np.complex128)
    with np.errstate(over="ignore"):
        if hist.ndim != 2 or len(hist) == 0:
            return {"n": 0, "hsum": "0", "wsum": [0.0, 0.0], "wabs": 0.0}
        x = _poly(hist)
        h = _mix64(x)
        hs = int(np.sum(h, dtype=np.uint64))
        u = (_mix64(x ^ _S) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    # fixed summation order: sort by the hash so that both sides add in the same order
    order = np.lexsort((u, h))
    ws = np.sum(w[order] * u[order])
    wa = float(np.sum(np.abs(w[order])))
    return {"n": int(len(hist)), "hsum": format(hs, "x"), "wsum": [float(ws.real), float(ws.imag)],
            "wabs": wa}


def compare(got: dict, want: dict, wtol: float) -> str:
    """'' when the fingerprints agree, else a reason.  The amplitude sums must
    agree within wtol * max(1, sum |w|): wtol bounds each amplitude's error
    relative to the largest, so the sums' error is bounded by wtol times the
    sum of the moduli."""
    if got["n"] != want["n"]:
        return f"group count {got['n']} != {want['n']}"
    if got["hsum"] != want["hsum"]:
        return "history sets differ"
    tol = wtol * max(1.0, want["wabs"])
    dw = abs(complex(*got["wsum"]) - complex(*want["wsum"]))
    if dw > tol:
        return f"amplitude sums differ by {dw:.3e} (bound {tol:.1e})"
    da = abs(got["wabs"] - want["wabs"])
    if da > tol:
        return f"|w| sums differ by {da:.3e} (bound {tol:.1e})"
    return ""
