"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Tolerances: images max-abs 1e-4 per channel over pixels whose compositing
decisions are not ambiguous in FP32 (flagged by the oracle, at most 0.1 %);
gradients per tensor |g - g_ref| <= 1e-3 |g_ref| + 1e-5 max |g_ref|; integer
work (bins, sort order, depth keys) bit-exact.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import native as N
from paper_2504_17954_amd import raster as R

pytestmark = pytest.mark.gpu
LOG2E = 1.4426950408889634


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    N.load()
    return torch.device("cuda:0")


def to_dev(planes, dev):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in planes.items()}


def c1_setup(seed_offset=0, width=128, height=128):
    w = I.c1(seed_offset)
    m = w.models[0]
    cam = I.look_at((0.0, -4.0, 0.0), width=width, height=height)
    return I.plain_planes(m), cam, O.Params(width, height)


def check_image(gpu, ref, what):
    """Max-abs 1e-4 per channel; each pixel may match the oracle's primary
    result or one of its ambiguous-branch alternatives; unresolvable pixels
    (more than two ambiguous decisions, ill-conditioned shading) are excluded
    and must stay below 0.1 % (at least 3 allowed on tiny images)."""
    err, excl, used = O.image_error(gpu, ref)
    npix = ref["flags"].size
    say(f"{what}: max-abs {err:.3e}, excluded {excl}/{npix}, matched an alternative {used}")
    assert excl <= max(3, 1e-3 * npix), excl
    assert err <= 1e-4, err


def check_grads(g_gpu, g_ref, what, exclude=None):
    for k in R.PLANES:
        a = g_gpu[k]
        b = g_ref[k]
        if exclude is not None:
            a = a[:, ~exclude]
            b = b[:, ~exclude]
        tol = 1e-3 * np.abs(b) + 1e-5 * np.abs(b).max() + 1e-30
        bad = np.abs(a - b) > tol
        worst = (np.abs(a - b) / tol).max() if b.size else 0
        say(f"{what} {k}: max|g| {np.abs(b).max():.3e}, outside {bad.sum()} / {b.size}, worst ratio {worst:.3f}")
        assert not bad.any(), (k, np.argwhere(bad)[:5])


# ------------------------------------------------------------------ project
def test_project_parity(dev):
    planes, cam, prm = c1_setup()
    say("project parity: c1 10k, 128x128")
    rnd = R.Renderer(R.Settings(128, 128))
    pd = to_dev(planes, dev)  # must outlive the launch: the batch holds raw pointers
    batch = rnd.make_batch(pd, None, R.default_edits(dev), R.camera_table([cam]), R.Jobs.single(10_000))
    rnd._ensure(batch)
    proj, _ = rnd._structs(batch)
    N.ivrgs_project(batch, R.Settings(128, 128).params(), proj, R._stream())
    rec = rnd.rec[:10_000].cpu().numpy()
    rect = rnd.rect[:10_000].cpu().numpy()
    # the row carries the rect too, and zeros in its spare words
    assert np.array_equal(rec[:, 12:14].view(np.uint32), rect.view(np.uint32))
    assert np.all(rec[:, [11, 14, 15]] == 0.0)
    ref = O.project(planes, cam, prm)
    kept = (rect[:, 0] != 0) | (rect[:, 1] != 0)
    valid = ref[:, 0] != 0
    assert np.all(valid[kept])
    z_ref = ref[:, 1].astype(np.float32)
    assert np.array_equal(rec[kept, 9].view(np.uint32), z_ref[kept].view(np.uint32))
    # the depth array carries the same key bits, and all-ones for culled records
    depth = rnd.depth[:10_000].cpu().numpy().view(np.uint32)
    assert np.array_equal(depth[kept], z_ref[kept].view(np.uint32))
    assert np.all(depth[~kept] == 0xFFFFFFFF)
    # screen mean within the error model the oracle uses for its decisions
    dm = ref[kept, 21]
    assert np.all(np.abs(rec[kept, 0] - ref[kept, 2]) <= dm)
    assert np.all(np.abs(rec[kept, 1] - ref[kept, 3]) <= dm)
    for col, field, scale in ((2, 7, -0.5 * LOG2E), (3, 8, -LOG2E), (4, 9, -0.5 * LOG2E)):
        want = scale * ref[kept, field]
        np.testing.assert_allclose(rec[kept, col], want, rtol=2e-4, atol=2e-6 * np.abs(want).max())
    np.testing.assert_array_equal(rec[kept, 5], planes["opacity"][0, kept])
    # colour within twice the oracle's FP32 error bound for it
    err = np.abs(rec[:, 6:9] - ref[:, 11:14]).max(1)
    bad = kept & (err > 2 * ref[:, 23])
    for i in np.flatnonzero(bad)[:10]:
        say(f"rgb mismatch {i}: gpu {rec[i, 6:9]} oracle {ref[i, 11:14]} nl {ref[i, 19]:.3e} "
            f"nh {ref[i, 20]:.3e} shade {planes['shade'][:, i]} normal {planes['normal'][:, i]} "
            f"mean {planes['mean'][:, i]} color {planes['color'][:, i]}")
    assert not bad.any(), int(bad.sum())
    # every Gaussian the oracle can see somewhere on screen is kept
    r = O.render(planes, cam, prm, want_maxw=True)
    assert np.all(kept[r["maxw"] > 0])


# ------------------------------------------------------------------ bin sort
def _bin_case(dev, width, height, rects, z, n_jobs=1, chunk=0):
    """Run ivrgs_bin_sort on synthetic records and compare with the
    definition: per (job, tile), ids of records whose rect covers it,
    ordered by (depth key bits, id)."""
    n = rects.shape[0]
    per = n // n_jobs
    s = R.Settings(width, height, sort_chunk=chunk)
    rnd = R.Renderer(s, capacity=1 << 21)
    jobs = R.Jobs.ranges([0] * n_jobs, [0] * n_jobs, [per] * n_jobs)
    planes = {k: torch.zeros((d, per), dtype=torch.float32, device=dev) for k, d in R.PLANE_DIMS.items()}
    batch = rnd.make_batch(planes, None, R.default_edits(dev), R.camera_table([I.look_at((0, -4, 0))]), jobs)
    rnd._ensure(batch)
    packed = np.stack([rects[:, 0] | (rects[:, 1] << 16), rects[:, 2] | (rects[:, 3] << 16)], 1)
    rec = np.zeros((n, 16), np.float32)
    rec[:, 9] = z
    rec[:, 12:14] = packed.astype(np.uint32).view(np.float32)  # the rect, also in the row
    rnd.rec[:n] = torch.from_numpy(rec).to(dev)
    rnd.rect[:n] = torch.from_numpy(packed.astype(np.uint32).view(np.int32)).to(dev)
    culled = (rects[:, 0] == 0) & (rects[:, 1] == 0) & (rects[:, 2] == 0) & (rects[:, 3] == 0)
    dbits = np.where(culled, np.uint32(0xFFFFFFFF), z.astype(np.float32).view(np.uint32))
    rnd.depth[:n] = torch.from_numpy(dbits.astype(np.uint32).view(np.int32)).to(dev)
    proj, bins = rnd._structs(batch)
    N.ivrgs_bin_sort(batch, s.params(), proj, bins, rnd.ws.data_ptr(), rnd.ws.numel(), R._stream())
    st = rnd.status.cpu().numpy()
    tpj = N.ivrgs_tiles_per_job(s.params())
    tx_n = (width + 15) // 16
    starts = rnd.tile_start[: n_jobs * tpj + 1].cpu().numpy().view(np.uint32)
    got = rnd.sorted[: int(starts[-1])].cpu().numpy().view(np.uint32)
    zb = z.astype(np.float32).view(np.uint32)
    total = 0
    for j in range(n_jobs):
        for t in range(tpj):
            tx, ty = t % tx_n, t // tx_n
            ids = np.arange(j * per, (j + 1) * per)
            rj = rects[ids]
            cov = (rj[:, 0] <= tx) & (tx < rj[:, 2]) & (rj[:, 1] <= ty) & (ty < rj[:, 3])
            sel = ids[cov]
            want = sel[np.lexsort((sel, zb[sel]))]
            g = j * tpj + t
            assert np.array_equal(got[starts[g]:starts[g + 1]], want), (j, t)
            total += want.size
    assert st[0] == total and st[1] == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_bin_sort_exact(dev, seed):
    say(f"bin_sort exact, synthetic records, seed {seed}")
    rng = np.random.default_rng(seed)
    n, W, H = 3000, 200, 120  # ragged tiles at the right and bottom
    tx_n, ty_n = 13, 8
    x0 = rng.integers(0, tx_n, n)
    y0 = rng.integers(0, ty_n, n)
    x1 = np.minimum(x0 + rng.integers(1, 5, n), tx_n)
    y1 = np.minimum(y0 + rng.integers(1, 5, n), ty_n)
    rects = np.stack([x0, y0, x1, y1], 1).astype(np.int64)
    culled = rng.random(n) < 0.1
    rects[culled] = 0
    # depth keys with deliberate exact ties and a narrow range
    z = rng.choice(np.linspace(2.5, 5.5, 700).astype(np.float32), n)
    _bin_case(dev, W, H, rects, z, n_jobs=1 if seed == 0 else 3)


@pytest.mark.parametrize("chunk", [0, 64, 512])
def test_bin_sort_many_chunks(dev, chunk):
    """Enough chunks that each wave of the scatter owns a whole chunk (64
    records per chunk), and the default chunk where waves share one."""
    say(f"bin_sort exact, 80k records, {chunk} records per chunk")
    rng = np.random.default_rng(3)
    n, W, H = 80_000, 200, 120
    tx_n, ty_n = 13, 8
    x0 = rng.integers(0, tx_n, n)
    y0 = rng.integers(0, ty_n, n)
    x1 = np.minimum(x0 + rng.integers(1, 4, n), tx_n)
    y1 = np.minimum(y0 + rng.integers(1, 4, n), ty_n)
    rects = np.stack([x0, y0, x1, y1], 1).astype(np.int64)
    rects[rng.random(n) < 0.05] = 0
    z = rng.choice(np.linspace(2.0, 6.0, 5000).astype(np.float32), n)
    _bin_case(dev, W, H, rects, z, chunk=chunk)


def test_bin_sort_large_tile(dev):
    """One tile holds more pairs than fit in LDS: the global-memory path."""
    say("bin_sort exact, 40k records on one tile")
    rng = np.random.default_rng(7)
    n = 40_000
    rects = np.tile(np.array([[0, 0, 1, 1]]), (n, 1))
    rects[::3] = [0, 0, 2, 1]
    z = (3.0 + rng.random(n) * 0.01).astype(np.float32)
    z[::50] = np.float32(3.001)
    _bin_case(dev, 32, 16, rects, z)


# ------------------------------------------------------------------- render
@pytest.mark.parametrize("px", [1, 2, 4])
def test_render_fwd_c1(dev, px):
    planes, cam, prm = c1_setup()
    say(f"render_fwd c1 vs oracle, px={px}")
    ref = O.render(planes, cam, prm)
    rnd = R.Renderer(R.Settings(128, 128, fwd_px=px))
    rgba = rnd.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(10_000),
                       edits_t=R.default_edits(dev))[0].cpu().numpy()
    check_image(rgba, ref, f"c1 fwd px={px}")


def test_render_fwd_px_bit_identical(dev):
    planes, cam, _ = c1_setup(1)
    imgs = []
    for px in (1, 2, 4):
        rnd = R.Renderer(R.Settings(128, 128, fwd_px=px))
        imgs.append(rnd.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(10_000),
                                edits_t=R.default_edits(dev)).cpu().numpy())
    assert np.array_equal(imgs[0], imgs[1]) and np.array_equal(imgs[0], imgs[2])


@pytest.mark.parametrize("W,H,seed", [(72, 40, 3), (33, 17, 4)])
def test_render_fwd_ragged(dev, W, H, seed):
    """Images that are not multiples of the tile, off-axis camera, bg colour."""
    m = I.small_scene(3000, 300 + seed, log_scale_mu=-3.2)
    planes = I.plain_planes(m)
    cam = I.look_at((1.5, -3.4, 1.2), width=W, height=H)
    prm = O.Params(W, H, bg=(0.2, 0.5, 0.9))
    say(f"render_fwd ragged {W}x{H}")
    ref = O.render(planes, cam, prm)
    rnd = R.Renderer(R.Settings(W, H, bg=(0.2, 0.5, 0.9)))
    rgba = rnd.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(m.n),
                       edits_t=R.default_edits(dev))[0].cpu().numpy()
    check_image(rgba, ref, f"ragged {W}x{H}")


def test_render_empty_and_culled(dev):
    """No Gaussians in view: background everywhere, A = 0."""
    m = I.small_scene(500, 9)
    planes = I.plain_planes(m)
    planes["mean"] = planes["mean"] + np.float32(20.0)  # far outside the frustum
    cam = I.look_at((0.0, -4.0, 0.0), width=48, height=32)
    s = R.Settings(48, 32, bg=(0.1, 0.2, 0.3))
    rnd = R.Renderer(s)
    rgba = rnd.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(m.n),
                       edits_t=R.default_edits(dev))[0].cpu().numpy()
    assert rnd.pairs() == 0
    np.testing.assert_array_equal(rgba[3], 0.0)
    for c, v in enumerate((0.1, 0.2, 0.3)):
        np.testing.assert_array_equal(rgba[c], np.float32(v))
    # zero Gaussians at all
    planes0 = {k: v[:, :0].copy() for k, v in planes.items()}
    rgba0 = rnd.forward(to_dev(planes0, dev), R.camera_table([cam]), R.Jobs.single(0),
                        edits_t=R.default_edits(dev))[0].cpu().numpy()
    np.testing.assert_array_equal(rgba0[3], 0.0)


def test_nonfinite_gaussians_are_culled(dev):
    planes, cam, prm = c1_setup(2, 64, 64)
    bad = {k: v.copy() for k, v in planes.items()}
    bad["mean"][0, 5] = np.nan
    bad["log_scale"][1, 6] = np.inf
    bad["shade"][3, 7] = np.nan
    keep = np.setdiff1d(np.arange(planes["mean"].shape[1]), [5, 6, 7])
    ref = O.render({k: v[:, keep] for k, v in planes.items()}, cam, prm)
    rnd = R.Renderer(R.Settings(64, 64))
    rgba = rnd.forward(to_dev(bad, dev), R.camera_table([cam]), R.Jobs.single(bad["mean"].shape[1]),
                       edits_t=R.default_edits(dev))[0].cpu().numpy()
    check_image(rgba, ref, "non-finite culled")
    # culled and counted: three Gaussians, once per projection
    assert rnd.nonfinite_count() == 3
    rnd.forward(to_dev(bad, dev), R.camera_table([cam, cam]), R.Jobs.views(bad["mean"].shape[1], [0, 1]),
                edits_t=R.default_edits(dev))
    assert rnd.nonfinite_count() == 3 + 6
    rnd.clear_nonfinite()
    rnd.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(planes["mean"].shape[1]),
                edits_t=R.default_edits(dev))
    assert rnd.nonfinite_count() == 0


def test_capacity_error_is_sticky_until_read(dev):
    """With the deferred check, an overflow in an earlier binning stays
    reported (with the largest requirement) after later binnings fit, until
    ivrgs_get_error reads and clears it."""
    planes, cam, prm = c1_setup()
    small = {k: v[:, :200].copy() for k, v in planes.items()}
    rnd = R.Renderer(R.Settings(128, 128), capacity=2000, check="defer")
    cams = R.camera_table([cam])
    rnd.forward(to_dev(planes, dev), cams, R.Jobs.single(10_000), edits_t=R.default_edits(dev))
    big = int(rnd.status[0].item())
    assert big > 2000
    rnd.forward(to_dev(small, dev), cams, R.Jobs.single(200), edits_t=R.default_edits(dev))
    small_pairs = int(rnd.status[0].item())
    assert small_pairs <= 2000 and int(rnd.status[1].item()) == 0
    bins = rnd._structs(None)[1]
    assert N.ivrgs_get_error(bins, R._stream()) == (N.DEV_E_CAPACITY, big)
    # read and cleared: now only the last (fitting) binning counts
    assert N.ivrgs_get_error(bins, R._stream()) == (0, small_pairs)
    assert rnd.verify() == small_pairs


def test_capacity_overflow_regrows(dev):
    planes, cam, prm = c1_setup()
    rnd = R.Renderer(R.Settings(128, 128), capacity=1000, check="sync")
    rgba = rnd.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(10_000),
                       edits_t=R.default_edits(dev))[0].cpu().numpy()
    assert rnd.capacity > 1000
    assert N.ivrgs_get_error(rnd._structs(None)[1], R._stream()) == (0, rnd.pairs())
    assert 1000 < rnd.verify() <= rnd.capacity
    ref = O.render(planes, cam, prm)
    check_image(rgba, ref, "after capacity regrow")
    # deferred mode reports the overflow instead of fixing it
    rnd2 = R.Renderer(R.Settings(128, 128), capacity=1000, check="defer")
    rnd2.forward(to_dev(planes, dev), R.camera_table([cam]), R.Jobs.single(10_000),
                 edits_t=R.default_edits(dev))
    err, need = N.ivrgs_get_error(rnd2._structs(None)[1], R._stream())
    assert err == N.DEV_E_CAPACITY and need == rnd.pairs()
    with pytest.raises(N.IvrgsError):
        rnd2.verify()


# ----------------------------------------------------------------- backward
def grad_exclusions(planes, cam, prm, edits=None, model_id=None):
    """Gaussians at a shading kink (|n.l| or |n.h| within 1e-5 of 0) or with
    |n.h| < 1e-3 (the beta < 1 lobe derivative is unbounded there)."""
    p = O.project(planes, cam, prm, edits=edits, model_id=model_id)
    return (np.abs(p[:, 19]) < 1e-5) | (np.abs(p[:, 20]) < 1e-3)


def upstream(ref, target_seed, shape):
    """L1 loss gradient from the oracle image, zero at ambiguous pixels."""
    tgt = np.random.default_rng(target_seed).uniform(0, 1, shape)
    dl = O.l1_loss_grad(ref["rgba"], tgt)
    dl[:, ref["flags"] != 0] = 0.0
    return dl


@pytest.mark.parametrize("px", [1, 2, 4])
def test_render_bwd_c1(dev, px):
    planes, cam, prm = c1_setup()
    say(f"render_bwd c1 vs oracle, bwd_px={px}")
    ref = O.render(planes, cam, prm)
    dl = upstream(ref, 2001, ref["rgba"].shape)
    g_ref, _ = O.backward(planes, cam, prm, dl)
    rnd = R.Renderer(R.Settings(128, 128, bwd_px=px))
    pd = to_dev(planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(10_000)
    rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
    g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                     edits_t=R.default_edits(dev))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    check_grads(g, g_ref, f"c1 bwd px={px}", exclude=grad_exclusions(planes, cam, prm))


BG = (0.3, 0.7, 0.15)


@pytest.mark.parametrize("px", [1, 2, 4])
def test_render_bwd_background(dev, px):
    """A coloured background puts T_final * bg into every alpha gradient (the
    colour behind each Gaussian includes it): C1 against the oracle at 1, 2
    and 4 pixels per lane."""
    w = I.c1(0)
    planes = I.plain_planes(w.models[0])
    cam = I.look_at((0.0, -4.0, 0.0), width=128, height=128)
    prm = O.Params(128, 128, bg=BG)
    say(f"render_bwd with background {BG}, bwd_px={px}")
    ref = O.render(planes, cam, prm)
    dl = upstream(ref, 2011, ref["rgba"].shape)
    g_ref, _ = O.backward(planes, cam, prm, dl)
    rnd = R.Renderer(R.Settings(128, 128, bg=BG, bwd_px=px))
    pd = to_dev(planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(10_000)
    rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
    check_image(rgba[0].cpu().numpy(), ref, f"c1 fwd bg px={px}")
    g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                     edits_t=R.default_edits(dev))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    check_grads(g, g_ref, f"c1 bwd bg px={px}", exclude=grad_exclusions(planes, cam, prm))


def test_render_bwd_background_segmented(dev):
    """Tile lists far longer than 128 records are cut into segments, and each
    segment's backward starts from the forward's checkpoint of (T, C): with a
    coloured background the colour behind a Gaussian must still include
    T_final * bg in every segment.  A dense cluster of 6000 Gaussians in a
    64x64 image gives lists of thousands of records."""
    m = I.small_scene(6000, 811, log_scale_mu=-3.3)
    m.planes["mean"] *= np.float32(0.8)
    planes = I.plain_planes(m)
    W = H = 64
    cam = I.look_at((0.2, -4.0, 0.3), width=W, height=H)
    prm = O.Params(W, H, bg=BG)
    ref = O.render(planes, cam, prm)
    dl = upstream(ref, 2012, ref["rgba"].shape)
    g_ref, _ = O.backward(planes, cam, prm, dl)
    rnd = R.Renderer(R.Settings(W, H, bg=BG))
    pd = to_dev(planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(m.n)
    rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
    starts = rnd.tile_start[:N.ivrgs_tiles_per_job(rnd.settings.params()) + 1].cpu().numpy()
    lens = np.diff(starts.astype(np.int64))
    say(f"segmented backward with background: longest list {lens.max()}, lists > 128: {(lens > 128).sum()}")
    assert lens.max() > 1024 and (lens > 128).sum() >= 12
    check_image(rgba[0].cpu().numpy(), ref, "cluster fwd bg")
    g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                     edits_t=R.default_edits(dev))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    check_grads(g, g_ref, "cluster bwd bg", exclude=grad_exclusions(planes, cam, prm))


def test_backward_overwrites_stale_gradients(dev):
    """One job over the whole set: the backward writes every Gaussian's
    gradient itself (no clearing pass), so buffers holding NaN come back
    equal to the oracle, with exact zeros for Gaussians it culls."""
    planes, cam, prm = c1_setup(seed_offset=3)
    planes = {k: v.copy() for k, v in planes.items()}
    planes["mean"][:, :50] = np.array([[0.0], [-10.0], [0.0]], np.float32)  # behind the camera: culled
    ref = O.render(planes, cam, prm)
    dl = upstream(ref, 2003, ref["rgba"].shape)
    g_ref, _ = O.backward(planes, cam, prm, dl)
    rnd = R.Renderer(R.Settings(128, 128))
    pd = to_dev(planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(10_000)
    rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
    stale = {k: torch.full((d, 10_000), float("nan"), device=dev) for k, d in R.PLANE_DIMS.items()}
    say("backward into NaN-filled gradient buffers, one job")
    g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                     edits_t=R.default_edits(dev), grads=stale)
    g = {k: v.cpu().numpy() for k, v in g.items()}
    for k in R.PLANES:
        assert np.isfinite(g[k]).all(), k
    culled = rnd.rect[:10_000].cpu().numpy().any(1) == 0
    assert culled[:50].all()
    for k in R.PLANES:
        assert np.all(g[k][:, culled] == 0.0), k
    check_grads(g, g_ref, "stale buffers", exclude=grad_exclusions(planes, cam, prm))


def test_autograd_function(dev):
    """loss.backward() through rasterize() equals the oracle gradient of the
    same L1 loss; the backward recomputes the bins when the renderer was
    reused by another forward in between."""
    m = I.small_scene(4000, 501, log_scale_mu=-3.3)
    planes = I.plain_planes(m)
    cam = I.look_at((0.3, -3.8, 1.0), width=96, height=80)
    prm = O.Params(96, 80)
    ref = O.render(planes, cam, prm)
    tgt = np.random.default_rng(5).uniform(0, 1, ref["rgba"].shape)
    # mask ambiguous pixels and entries where the L1 sign is within noise
    keep = (ref["flags"] == 0)[None] & (np.abs(ref["rgba"] - tgt) > 1e-3)
    dl = O.l1_loss_grad(ref["rgba"], tgt) * keep
    g_ref, _ = O.backward(planes, cam, prm, dl)
    pt = {k: v.requires_grad_(True) for k, v in to_dev(planes, dev).items()}
    rnd = R.Renderer(R.Settings(96, 80))
    cams, jobs = R.camera_table([cam]), R.Jobs.single(m.n)
    out = R.rasterize(pt, cams, jobs, rnd)[0]
    # another forward through the same renderer overwrites its buffers
    other = I.plain_planes(I.small_scene(1000, 502))
    rnd.forward(to_dev(other, dev), cams, R.Jobs.single(1000), edits_t=R.default_edits(dev))
    t = torch.from_numpy(tgt.astype(np.float32)).to(dev)
    mask = torch.from_numpy(keep).to(dev)
    loss = ((out - t).abs() * mask).sum() / out.numel()
    loss.backward()
    g = {k: pt[k].grad.cpu().numpy() for k in R.PLANES}
    check_grads(g, g_ref, "autograd", exclude=grad_exclusions(planes, cam, prm))


# ------------------------------------------------------------------ compose
def test_compose_parity(dev):
    ms = [I.small_scene(700 + 100 * k, 600 + k, log_scale_mu=-3.2) for k in range(3)]
    edits = I.c3_edits(ms, 77)
    rows = np.stack([e.row() for e in edits])
    say("compose parity: 3 models with edits")
    pl_ref, mid_ref = O.compose([m.planes for m in ms], rows)
    out, mid = R.compose([to_dev(m.planes, dev) for m in ms], edits)
    assert np.array_equal(mid.cpu().numpy(), mid_ref)
    for k in R.PLANES:
        a, b = out[k].cpu().numpy(), pl_ref[k]
        if k in ("mean", "log_scale", "quat", "normal", "color", "opacity"):
            assert np.array_equal(a, b), k
        else:  # lambda*k + b: one fused rounding on the GPU vs FP64 then FP32
            ulp = np.spacing(np.abs(b).astype(np.float32))
            assert np.all(np.abs(a - b) <= ulp), k
    # render the composed scene with per-model orbital lights
    cam = I.look_at((0.5, -3.9, 0.7), width=80, height=64)
    prm = O.Params(80, 64)
    ref = O.render(pl_ref, cam, prm, model_id=mid_ref, edits=rows)
    rnd = R.Renderer(R.Settings(80, 64))
    rgba = rnd.forward(out, R.camera_table([cam]), R.Jobs.single(mid.numel()), model_id=mid,
                       edits_t=R.edit_table(edits, dev))[0].cpu().numpy()
    check_image(rgba, ref, "composed render")
    dl = upstream(ref, 9, ref["rgba"].shape)
    g_ref, _ = O.backward(pl_ref, cam, prm, dl, model_id=mid_ref, edits=rows)
    g = rnd.backward(out, R.camera_table([cam]), R.Jobs.single(mid.numel()), torch.from_numpy(rgba[None]).to(dev),
                     torch.from_numpy(dl[None].astype(np.float32)).to(dev), model_id=mid,
                     edits_t=R.edit_table(edits, dev))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    check_grads(g, g_ref, "composed bwd",
                exclude=grad_exclusions(pl_ref, cam, prm, edits=rows, model_id=mid_ref))


# ------------------------------------------------- full-size sampled parity
def c2_scene(n=300_000):
    m = I.isosurface_model(n, I.SEED_SCENE + 2)
    return I.plain_planes(m)


@pytest.fixture(scope="module")
def c2_planes():
    return c2_scene()


def sample_pixels(W, H, count, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, W, count), rng.integers(0, H, count)], 1)


def windows(W, H, n, size, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        x0 = int(rng.integers(W // 4, 3 * W // 4 - size))
        y0 = int(rng.integers(H // 4, 3 * H // 4 - size))
        ys, xs = np.mgrid[y0:y0 + size, x0:x0 + size]
        out.append(np.stack([xs.reshape(-1), ys.reshape(-1)], 1))
    return np.unique(np.concatenate(out), axis=0)


@pytest.mark.parametrize("view", [0, 37])
def test_c2_fullsize_sampled(dev, c2_planes, view):
    """300k isosurface Gaussians at 800x800, the launch configuration the
    benchmark times: sampled pixels of the forward, and the backward of an
    upstream gradient supported on pixel windows (exact for every Gaussian,
    since pixels outside the windows carry no gradient on either side)."""
    W = H = 800
    cam = I.cameras_at(I.fibonacci_sphere(100)[view:view + 1], W, H)[0]
    prm = O.Params(W, H)
    say(f"c2 full size, view {view}: forward on sampled pixels")
    rnd = R.Renderer(R.Settings(W, H))
    pd = to_dev(c2_planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(c2_planes["mean"].shape[1])
    rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
    img = rgba[0].cpu().numpy()
    pix = sample_pixels(W, H, 3000, view)
    ref = O.render(c2_planes, cam, prm, pix=pix)
    check_image(img[:, pix[:, 1], pix[:, 0]].T, ref, f"c2 view {view} sampled")
    say(f"c2 full size, view {view}: backward on windows")
    win = windows(W, H, 6, 20, 100 + view)
    refw = O.render(c2_planes, cam, prm, pix=win)
    tgt = np.random.default_rng(view).uniform(0, 1, refw["rgba"].shape)
    keep = (refw["flags"] == 0)[:, None] & (np.abs(refw["rgba"] - tgt) > 1e-3)
    dlw = np.sign(refw["rgba"] - tgt) * keep / (4.0 * W * H)
    g_ref, _ = O.backward(c2_planes, cam, prm, dlw, pix=win)
    dl = np.zeros((1, 4, H, W), np.float32)
    dl[0, :, win[:, 1], win[:, 0]] = dlw.astype(np.float32)
    g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl).to(dev), edits_t=R.default_edits(dev))
    g = {k: v.cpu().numpy() for k, v in g.items()}
    touched = np.abs(np.concatenate([g_ref[k] for k in R.PLANES])).max(0) > 0
    say(f"c2 view {view}: {touched.sum()} Gaussians with gradient")
    excl = grad_exclusions(c2_planes, cam, prm) | ~touched
    check_grads(g, g_ref, f"c2 view {view} bwd", exclude=excl)
    # untouched Gaussians get exactly zero
    for k in R.PLANES:
        assert np.all(g[k][:, ~touched] == 0), k


@pytest.fixture(scope="module")
def c3_scene():
    w = I.c3()
    rows = np.stack([e.row() for e in w.edits])
    pl, mid = O.compose([m.planes for m in w.models], rows)
    return w, rows, pl, mid


@pytest.mark.parametrize("view", [0, 31])
def test_c3_fullsize_sampled(dev, c3_scene, view):
    """The composed forward in the launch configuration the benchmark times:
    8 nested-shell models of 150k Gaussians (1.2M) with per-model transfer-
    function and lighting edits (opacity scale up to 2, recolour, orbital
    lights, intensity), composed on the device, 1024x1024, 256 records per
    binning chunk; 3000 sampled pixels against the oracle's render of its
    own composition."""
    w, rows, pl, mid = c3_scene
    cam = w.cameras[view]
    W = H = 1024
    prm = O.Params(W, H)
    say(f"c3 full size, view {view}: compose + forward, 3000 sampled pixels")
    out, mid_d = R.compose([to_dev(m.planes, dev) for m in w.models], w.edits)
    assert np.array_equal(mid_d.cpu().numpy(), mid)
    rnd = R.Renderer(R.Settings(W, H, fwd_px=1, sort_chunk=256))
    rgba = rnd.forward(out, R.camera_table([cam]), R.Jobs.single(mid.size), model_id=mid_d,
                       edits_t=R.edit_table(w.edits, dev))
    img = rgba[0].cpu().numpy()
    say(f"c3 view {view}: {rnd.pairs()} pairs")
    pix = sample_pixels(W, H, 3000, 500 + view)
    ref = O.render(pl, cam, prm, model_id=mid, edits=rows, pix=pix)
    check_image(img[:, pix[:, 1], pix[:, 0]].T, ref, f"c3 view {view} sampled")


@pytest.mark.parametrize("n", [511, 512, 513, 1023, 1024, 1025, 4095, 4096, 4097, 8193, 600_001])
def test_bin_sort_chunk_and_segment_boundaries(dev, n):
    """List lengths around the binning chunk (512 records), the wave step (64)
    and the depth-sort segment (1024 records up to 2^19 records per job,
    4096 beyond: the last case), all on one tile."""
    say(f"bin_sort exact, {n} records on one tile")
    rng = np.random.default_rng(n)
    rects = np.tile(np.array([[0, 0, 1, 1]]), (n, 1))
    z = (2.0 + rng.random(n) * 3.0).astype(np.float32)
    z[::97] = np.float32(3.25)  # a run of exact ties
    _bin_case(dev, 16, 16, rects, z)


@pytest.mark.parametrize("pattern", ["all_equal", "top_byte", "low_byte", "mixed_exponents"])
def test_bin_sort_digit_patterns(dev, pattern):
    """Depth keys whose varying bits fall in different bytes (every digit
    pass, or none, of the radix sort is exercised), with ties resolved by id."""
    say(f"bin_sort exact, digit pattern {pattern}")
    rng = np.random.default_rng(11)
    n = 3000
    rects = np.tile(np.array([[0, 0, 2, 1]]), (n, 1))
    rects[::5] = [1, 0, 2, 1]
    if pattern == "all_equal":
        z = np.full(n, 3.0, np.float32)
    elif pattern == "top_byte":
        z = rng.choice(np.float32([2.0, 8.0, 32.0, 128.0]), n).astype(np.float32)
    elif pattern == "low_byte":
        base = np.float32(3.0).view(np.uint32)
        z = (base + rng.integers(0, 256, n).astype(np.uint32)).view(np.float32)
    else:
        z = (2.0 ** rng.uniform(-1, 10, n)).astype(np.float32)
    _bin_case(dev, 32, 16, rects, z)
