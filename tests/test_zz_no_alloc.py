"""GPU: the allocation-free ghost selection + packing entry point
(pack_ghosts_noalloc, fixed device scratch) against pack_ghosts in
HOOMD_GHOST_SELECT mode through a context, byte for byte, on two calls in a
row -- the second with a smaller input, so that it runs over the scratch
left by the first -- and against the oracle's send lists."""
import numpy as np
import pytest

from paper_1412_3387_amd import inputs

pytestmark = pytest.mark.gpu
W = 2.9


@pytest.fixture(scope="module")
def B():
    from paper_1412_3387_amd import binding
    binding.lib()
    return binding


def _both(B, pos, vel, tag, lo, hi, fields, cap):
    import torch
    p = B.ModelParams(precision=B.MIXED)
    # an open frame one unit wider than the subdomain on each side: no
    # folding, no sorting, rows stay in input order
    lo_f = np.asarray(lo, dtype=np.float64) - 1.0
    L = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64) + 2.0
    ctx = B.Context([p], [dict(pos=pos, vel=vel, tag=tag, L=L, lo=lo_f, periodic=(0, 0, 0))])
    rec = {B.FIELD_POS | B.FIELD_TAG: 32, B.FIELD_POS | B.FIELD_VEL | B.FIELD_TAG: 56}[fields]
    dev = ctx.device
    out = []
    for which in ("ctx", "noalloc"):
        buf = torch.zeros(cap * rec, dtype=torch.uint8, device=dev)
        cnt = torch.full((26,), -1, dtype=torch.int32, device=dev)
        off = torch.full((26,), -1, dtype=torch.int32, device=dev)
        n = ctx.n_local[0]
        if which == "ctx":
            ctx.pack_ghosts(0, lo, hi, W, B.GHOST_SELECT, fields, buf, cap, cnt, off)
        else:
            B.pack_ghosts_noalloc(ctx.pos, ctx.vel, ctx.tag, n, lo, hi, W, fields, buf, cap, cnt, off,
                                  stream=ctx.stream.cuda_stream)
        torch.cuda.synchronize()
        out.append((buf.cpu().numpy(), cnt.cpu().numpy(), off.cpu().numpy()))
    ctx.check()
    ctx.close()
    return out, rec


def test_noalloc_matches_pack_ghosts_on_two_calls(orc, B):
    big = inputs.lj_subdomain_box(grid=3, cells=60)
    small = inputs.lj_subdomain_box(grid=3, cells=12)
    cases = [(big, 0, B.FIELD_POS | B.FIELD_VEL | B.FIELD_TAG),
             (small, 5, B.FIELD_POS | B.FIELD_TAG)]
    sizes = []
    for sd, s, fields in cases:
        loc = sd.local(s)
        sizes.append(len(loc))
        pos, vel = sd.full.pos[loc], sd.full.vel[loc]
        tag = loc.astype(np.int32)
        cap = 8 * len(loc)
        (a, b), rec = _both(B, pos, vel, tag, sd.lo(s), sd.hi(s), fields, cap)
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert np.array_equal(a[0], b[0])
        # and both equal the oracle's ordered send list
        m = orc.ghost_masks(pos, sd.lo(s), sd.hi(s), W)
        cnt, off, idx = orc.ghost_list(m)
        assert np.array_equal(b[1], cnt) and np.array_equal(b[2], off)
        recs = b[0][: len(idx) * rec]
        words = recs.view(np.float64).reshape(len(idx), rec // 8)
        assert np.array_equal(words[:, :3], pos[idx])
        if fields & B.FIELD_VEL:
            assert np.array_equal(words[:, 3:6], vel[idx])
        assert np.array_equal(recs.view(np.int32).reshape(len(idx), rec // 4)[:, -2], tag[idx])
        assert not b[0][len(idx) * rec:].any()
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_oversize_input(B):
    import torch
    z = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    cnt = torch.zeros(26, dtype=torch.int32, device="cuda")
    with pytest.raises(B.HoomdError) as e:
        B.pack_ghosts_noalloc(z, None, None, B.NOALLOC_MAX_ROWS + 1, (0, 0, 0), (1, 1, 1), 0.1,
                              B.FIELD_POS, None, 0, cnt, cnt)
    assert e.value.code == 1
