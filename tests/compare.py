"""Comparison helpers between the HIP library's outputs and the oracle."""

import numpy as np

import oracle

PAD = 0xFFFFFFFF
# per-parameter floors of the relative fit tolerance: phi0 [rad], d0 [cm],
# q/pT [1/GeV], cot(theta), z0 [cm]
FLOORS = np.array([1.0, 0.01, 0.001, 0.1, 1.0])
FIT_RTOL = 1e-4


def canon_rows(a):
    a = np.asarray(a, dtype=np.uint32)
    if a.ndim != 2 or a.shape[0] == 0:
        return a.reshape(-1, a.shape[-1] if a.ndim == 2 else 1)
    return a[np.lexsort(a.T[::-1])]


def per_event_rows(dump, n_events):
    """Split dump rows (event, ...) by event."""
    out = []
    for e in range(n_events):
        out.append(canon_rows(dump[dump[:, 0] == e][:, 1:]))
    return out


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def fit_errors(p_gpu, p_ref):
    """Per-parameter relative error with floors (phi0 compared modulo 2 pi)."""
    d = np.abs(p_gpu.astype(np.float64) - p_ref)
    d[:, 0] = np.abs(wrap(p_gpu[:, 0].astype(np.float64) - p_ref[:, 0]))
    return d / np.maximum(np.abs(p_ref), FLOORS)


def match_tracks(res, oref, event):
    """GPU tracks of `event` and the oracle's, both in canonical hit order.

    Returns (gpu_hits, gpu_params, gpu_cov, gpu_chi2, gpu_flags, ora_hits,
    ora_params, ora_cov, ora_chi2)."""
    m = res["event_id"] == event
    gh = res["hit_idx"][m].view(np.uint32)
    go = np.lexsort(gh.T[::-1]) if gh.shape[0] else np.zeros(0, int)
    oh = oref["tracks"]
    oo = np.lexsort(oh.T[::-1]) if oh.shape[0] else np.zeros(0, int)
    return (gh[go], res["params"][m][go], res["cov"][m][go], res["chi2"][m][go],
            res["flags"][m][go], oh[oo], oref["params"][oo], oref["cov"][oo], oref["chi2"][oo])


def oracle_events(events, det, workers=None):
    """The oracle on every event, one event per host thread (the C oracle
    releases the interpreter while it runs)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    oracle.lib()
    if workers is None:
        try:
            workers = len(os.sched_getaffinity(0))
        except AttributeError:
            workers = os.cpu_count() or 1
        workers = max(1, min(16, workers))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda e: oracle.reconstruct(e.x, e.y, e.z, e.layer, det), events))


def correlations(c15):
    """Correlation coefficients of packed 5x5 covariances [n, 15] -> [n, 10]
    (the off-diagonal entries of the lower triangle over sqrt of their
    diagonals)."""
    c = np.asarray(c15, np.float64)
    diag = [0, 2, 5, 9, 14]
    out = []
    k = 0
    for a in range(5):
        for b in range(a + 1):
            if a != b:
                out.append(c[:, k] / np.sqrt(c[:, diag[a]] * c[:, diag[b]]))
            k += 1
    return np.stack(out, axis=1) if out else np.zeros((c.shape[0], 0))
