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
    """Compare the GPU rows (as sets of tags) with the oracle's brute-force
    sets over the input positions (input order = tag order).  `which` lists
    tags to check."""
    nn, rows = ctx.neighbor_rows(sys)
    o, n = ctx.offsets[sys], ctx.n_local[sys]
    tag = ctx.tag[o:o + n].cpu().numpy().astype(np.int64)
    row_of = np.empty(n, dtype=np.int64)
    row_of[tag] = np.arange(n)
    idx = np.arange(n) if which is None else np.asarray(which)
    off, ref = orc.neighbors(pos, L, r_cut, r_buff, which=idx, bonds=bonds)
    bad = []
    for q, t in enumerate(idx):
        got = np.sort(tag[rows[row_of[t]]])
        want = ref[off[q]:off[q + 1]]
        if not np.array_equal(got, want):
            bad.append(int(t))
    return bad
