"""Test helpers: convert oracle localization regions to the C-ABI layout and
back, and compare library results with the oracle.  Tests only."""
import numpy as np

import paper_1401_7441_amd as W
from oracle.locreg import Locreg, seg_count


def _with_offsets(seg):
    seg = np.asarray(seg, np.int64).reshape(-1, 4)
    out = np.zeros(len(seg), W.SEG_DTYPE)
    if len(seg):
        out["i1s"], out["i1e"], out["i2"], out["i3"] = seg[:, 0], seg[:, 1], seg[:, 2], seg[:, 3]
        lens = seg[:, 1] - seg[:, 0] + 1
        out["off"] = np.concatenate([[0], np.cumsum(lens)[:-1]])
    return out


def to_abi(lrs):
    """oracle Locreg list -> (locregs, segs) structured arrays with
    coefficients laid out back to back in function order."""
    recs = np.zeros(len(lrs), W.LOCREG_DTYPE)
    chunks = []
    nseg = 0
    coef = 0
    ocoef = 0
    for k, l in enumerate(lrs):
        r = recs[k]
        r["center"] = l.center
        r["radius"] = l.radius
        r["ext"] = l.ext
        r["lo"] = l.lo
        r["dims"] = l.dims
        for name, seg in (("seg_c", l.cseg), ("seg_f", l.fseg), ("oseg_c", l.ocseg),
                          ("oseg_f", l.ofseg)):
            s = _with_offsets(seg)
            r[name] = nseg
            r["n" + name] = len(s)
            nseg += len(s)
            chunks.append(s)
        r["n_c"], r["n_f"], r["on_c"], r["on_f"] = l.n_c, l.n_f, l.on_c, l.on_f
        r["coef_off"] = coef
        r["ocoef_off"] = ocoef
        coef += l.n_c + 7 * l.n_f
        ocoef += l.on_c + 7 * l.on_f
    segs = np.concatenate(chunks) if chunks else np.zeros(0, W.SEG_DTYPE)
    return recs, segs


def from_abi(recs, segs):
    """(locregs, segs) structured arrays -> oracle Locreg list (for feeding the
    oracle the same pattern the library built)."""
    out = []
    for r in recs:
        def lst(name):
            s = segs[int(r[name]):int(r[name]) + int(r["n" + name])]
            return np.stack([s["i1s"], s["i1e"], s["i2"], s["i3"]], axis=1).astype(np.int64) \
                if len(s) else np.zeros((0, 4), np.int64)
        out.append(Locreg(lo=tuple(int(v) for v in r["lo"]), dims=tuple(int(v) for v in r["dims"]),
                          ext=int(r["ext"]), cseg=lst("seg_c"), fseg=lst("seg_f"),
                          ocseg=lst("oseg_c"), ofseg=lst("oseg_f"),
                          center=tuple(float(v) for v in r["center"]), radius=float(r["radius"])))
    return out


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
