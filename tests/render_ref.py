"""Reference rendering of psi maps in numpy, written from the rule that
include/dd.h states for dd_render_maps (scale, colour-map anchors,
iso-lines, automatic range).  Shares no code with the library.

Also returns, per pixel, how far the float decisions (colour bin and level)
are from their boundaries, so that a comparison with the device rendering
can tell a pixel whose colour depends on the last bit of a logarithm (both
colours correct) from a wrong pixel."""
import numpy as np

ANCHORS = [(0, 0, 0, 0), (38, 32, 12, 96), (90, 118, 24, 132), (141, 200, 52, 84),
           (192, 244, 128, 32), (230, 250, 208, 64), (255, 255, 255, 232)]


def colour_table():
    tab = np.zeros((256, 3), dtype=np.uint8)
    for i in range(256):
        k = max(j for j in range(len(ANCHORS) - 1) if ANCHORS[j][0] <= i)
        b0, b1 = ANCHORS[k][0], ANCHORS[k + 1][0]
        for c in range(3):
            c0, c1 = float(ANCHORS[k][c + 1]), float(ANCHORS[k + 1][c + 1])
            x = c0 + (c1 - c0) * float(i - b0) / float(b1 - b0)
            tab[i, c] = int(np.floor(x + 0.5))
    return tab


def scale(v, lo, hi, log_scale):
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros_like(v)
    inside = (v > lo) & (v < hi)
    with np.errstate(all="ignore"):
        if log_scale:
            t[inside] = np.log(v[inside] / lo) / np.log(hi / lo)
        else:
            t[inside] = (v[inside] - lo) / (hi - lo)
    t[v >= hi] = 1.0
    t = np.where(np.isnan(t), 0.0, np.clip(t, 0.0, 1.0))
    return t


def render(psi, lo=0.0, hi=0.0, decades=6.0, log_scale=True, levels=0):
    """psi [n, h, w] -> (rgb [n, h, w, 3] uint8, margin [n, h, w]): margin is
    the smallest distance, in units of t, from a bin or level boundary of the
    decisions that made the pixel."""
    psi = np.asarray(psi, dtype=np.float64)
    n, h, w = psi.shape
    tab = colour_table()
    rgb = np.zeros((n, h, w, 3), dtype=np.uint8)
    margin = np.full((n, h, w), np.inf)
    for m in range(n):
        if lo == 0.0 and hi == 0.0:
            fin = psi[m][np.isfinite(psi[m])]
            mh = max(0.0, float(fin.max())) if fin.size else 0.0
            ml = max(mh * 10.0 ** (-decades), 2.0 ** -1022) if log_scale else 0.0
        else:
            ml, mh = lo, hi
        if not mh > ml:
            continue  # black
        t = scale(psi[m], ml, mh, log_scale)
        idx = np.minimum(255, np.floor(t * 256.0)).astype(np.int64)
        rgb[m] = tab[idx]
        inner = (t > 0) & (t < 1)
        f = t * 256.0
        margin[m] = np.where(inner, np.abs(f - np.round(f)) / 256.0, np.inf)
        if levels > 0:
            lv = np.minimum(levels - 1, np.floor(t * levels)).astype(np.int64)
            edge = np.zeros((h, w), dtype=bool)
            edge[:, :-1] |= lv[:, :-1] != lv[:, 1:]
            edge[:-1, :] |= lv[:-1, :] != lv[1:, :]
            rgb[m][edge] = 255
            g = t * levels
            lm = np.where(inner, np.abs(g - np.round(g)) / levels, np.inf)
            # a pixel's iso-line decision also depends on its neighbours' levels
            near = lm.copy()
            near[:, :-1] = np.minimum(near[:, :-1], lm[:, 1:])
            near[:-1, :] = np.minimum(near[:-1, :], lm[1:, :])
            margin[m] = np.minimum(margin[m], near)
    return rgb, margin
