"""gi_trace_rays_noalloc (the entry point for callers that cannot allocate device memory)
against gi_trace_rays: closest and any hits bit-identical, on two calls in a row, the second
with fewer rays (and another context), so that what the first call left in the shared static
array cannot leak into the second."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2310_19855_amd import gi  # noqa: E402
from paper_2310_19855_amd import inputs as I  # noqa: E402


def _rays(n, lo, hi, seed, tmax):
    o, d = I.random_rays(n, lo, hi, seed=seed)
    o4 = torch.zeros((n, 4), dtype=torch.float32)
    d4 = torch.zeros((n, 4), dtype=torch.float32)
    o4[:, :3] = torch.from_numpy(o)
    o4[:, 3] = torch.from_numpy(np.asarray(tmax, np.float32))
    d4[:, :3] = torch.from_numpy(d)
    return o, d, o4.cuda(), d4.cuda()


def _both(ctx, o4, d4, any_hit):
    n = o4.shape[0]
    ref_tri = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    ref_t = torch.full((n,), 7.0, dtype=torch.float32, device="cuda")
    tri = torch.full((n,), 9, dtype=torch.int32, device="cuda")
    t = torch.full((n,), 9.0, dtype=torch.float32, device="cuda")
    ctx.trace_rays(o4, d4, ref_tri, ref_t, any_hit=any_hit)
    ctx.trace_rays_noalloc(o4, d4, tri, t, any_hit=any_hit)
    torch.cuda.synchronize()
    return (ref_tri.cpu().numpy().view(np.uint32), ref_t.cpu().numpy().view(np.uint32),
            tri.cpu().numpy().view(np.uint32), t.cpu().numpy().view(np.uint32))


def test_noalloc_trace_matches_trace_rays_twice_second_smaller():
    # first call: the ~1.0M-triangle field (a deep BVH whose walk spills), 300,000 rays, more
    # than one chunk of the static array
    field = I.field_scene()
    a = gi.Context(width=64, height=64, rays_per_probe=16)
    a.build_bvh(field)
    depth = int(a.dims()[10])
    assert 3 * depth + 1 > 16, "the field's walk must spill past the LDS part of the stack"
    n1 = 300_000
    o, d, o4, d4 = _rays(n1, [-40, 0.05, -40], [40, 10, 40], 41, np.full(n1, 3.0e38))
    rtri, rt, tri, t = _both(a, o4, d4, False)
    assert np.array_equal(tri, rtri) and np.array_equal(t, rt)
    assert (tri != 0xFFFFFFFF).mean() > 0.3
    # and the oracle's binary BVH on a sample of them
    osc = O.OracleScene(field)
    otri, ot = osc.closest(o[:20000], d[:20000])
    assert np.array_equal(tri[:20000], otri) and np.array_equal(t[:20000], ot.view(np.uint32))
    # any hit over finite segments, same rays
    tm = np.random.default_rng(6).uniform(0.1, 20.0, n1).astype(np.float32)
    o4[:, 3] = torch.from_numpy(tm).cuda()
    rtri, _, tri, _ = _both(a, o4, d4, True)
    assert np.array_equal(tri, rtri)

    # second call, right after: another context (the room), far fewer rays
    room = I.room_scene()
    b = gi.Context(width=32, height=32, rays_per_probe=4)
    b.build_bvh(room)
    n2 = 1000
    _, _, o4, d4 = _rays(n2, [0.1, 0.1, 0.1], [5.9, 2.9, 5.9], 43, np.full(n2, 3.0e38))
    rtri, rt, tri, t = _both(b, o4, d4, False)
    assert np.array_equal(tri, rtri) and np.array_equal(t, rt)
    assert (tri != 0xFFFFFFFF).all()     # closed room: every ray hits
    # and the first context again, on a ragged count below one wave
    _, _, o4, d4 = _rays(37, [-40, 0.05, -40], [40, 10, 40], 44, np.full(37, 3.0e38))
    rtri, rt, tri, t = _both(a, o4, d4, False)
    assert np.array_equal(tri, rtri) and np.array_equal(t, rt)
    a.close()
    b.close()


def test_noalloc_trace_arguments():
    ctx = gi.Context(width=32, height=32)
    z = torch.zeros((1, 4), dtype=torch.float32, device="cuda")
    tri = torch.zeros(1, dtype=torch.int32, device="cuda")
    t = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(gi.GIError, match="STATE"):
        ctx.trace_rays_noalloc(z, z, tri, t)          # no scene yet
    ctx.build_bvh(I.room_scene())
    e = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    ctx.trace_rays_noalloc(e, e, tri, t)              # no rays: nothing to do
    rc = gi.lib().gi_trace_rays_noalloc(ctx.h, None, None, 1, 0, None, None, None)
    assert rc == -1                                   # GI_ERR_INVALID_ARG
    ctx.close()
