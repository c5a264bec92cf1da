"""Shared helpers of the GPU parity tests (imported only by tests marked gpu)."""
import math

import numpy as np

LJ = [1.0, 1.0, 2.5]


def frel(F, Fref):
    """max_i |F_i - Fref_i| / F_rms(ref)."""
    frms = math.sqrt(np.mean(np.sum(Fref * Fref, axis=1)))
    return float(np.max(np.sqrt(np.sum((F - Fref) ** 2, axis=1))) / frms)


def by_tag(tag, *arrays):
    order = np.argsort(tag, kind="stable")
    return [a[order] for a in arrays]


def min_image_diff(a, b, L):
    d = a - b
    return d - L * np.rint(d / L)


def neighbor_sets_equal(orc, ctx, pos, L, r_cut, r_buff, which=None, bonds=None, sys=0):
    """Compare the GPU rows (as sets) with the oracle's brute-force sets."""
    nn, rows = ctx.neighbor_rows(sys)
    idx = np.arange(len(rows)) if which is None else np.asarray(which)
    off, ref = orc.neighbors(pos, L, r_cut, r_buff, which=idx, bonds=bonds)
    bad = []
    for q, i in enumerate(idx):
        got = np.sort(rows[i])
        want = ref[off[q]:off[q + 1]]
        if not np.array_equal(got, want):
            bad.append(int(i))
    return bad
