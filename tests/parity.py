"""Error metric of the parity tests: per element and output, ||x - y||_inf / ||y||_inf with y the oracle's
value; when ||y||_inf = 0 the denominator is ||Q||_inf (times 1/h for favg). Reported as the maximum over
elements."""
import numpy as np

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-4}  # FP64, FP32, split-BF16x3


def max_rel_err(got: dict, ref: dict, Q: np.ndarray, h: np.ndarray) -> dict:
    E = Q.shape[0]
    qn = np.abs(Q.reshape(E, -1)).max(axis=1) if E else np.zeros(0)
    out = {}
    for k, y in ref.items():
        if k == "favg_fig5":
            continue
        x = got[k]
        yE = y.reshape(E, -1)
        d = np.abs(x.reshape(E, -1) - yE).max(axis=1)
        den = np.abs(yE).max(axis=1)
        fallback = qn / (h if k == "favg" else 1.0)
        den = np.where(den > 0, den, np.where(fallback > 0, fallback, 1.0))
        out[k] = float((d / den).max()) if E else 0.0
    return out
