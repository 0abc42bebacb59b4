"""GPU parity of the auxiliary maps (Eq. 5 depth and normal maps; offset-
colour and shading maps of Sec. 4.3) and their backward, through the C ABI,
against the dense FP64 oracle and its autograd; and, at full size, the
property that compositing each Gaussian's colour as an attribute gives the
image itself.

Tolerances: maps within 1e-4 of the channel's largest attribute magnitude
(1e-4 of colour in [0, 1], scaled for depth); gradients within 1e-3 relative
plus 1e-5 of the largest magnitude; pixels with an ambiguous decision in the
C oracle are left out of the maps and carry no upstream gradient.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle import dense as D
from paper_2504_17954_amd import aux as AX
from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import native as N
from paper_2504_17954_amd import raster as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def check_grad(a, b, what):
    tol = 1e-3 * np.abs(b) + 1e-5 * np.abs(b).max() + 1e-30
    bad = np.abs(a - b) > tol
    say(f"  {what}: max|g| {np.abs(b).max():.3e}, outside {bad.sum()} / {b.size}, "
        f"worst {(np.abs(a - b) / tol).max():.3f}")
    assert not bad.any(), np.argwhere(bad)[:5]


def attributes(planes):
    n = planes["normal"]
    return np.concatenate([n / np.linalg.norm(n, axis=0, keepdims=True), planes["color"],
                           planes["shade"]]).astype(np.float32)


def device_rows(attr, dev):
    """Attribute planes [A, n] as the device rows the kernels take: [n, S]
    with S = A rounded up to a multiple of 4 (pad columns zero)."""
    A, n = attr.shape
    rows = np.zeros((n, (A + 3) // 4 * 4), np.float32)
    rows[:, :A] = attr.T
    return torch.from_numpy(rows).to(dev).requires_grad_(True)


def small(n, seed, width=40, height=32):
    m = I.small_scene(n, seed, log_scale_mu=-2.6)
    planes = I.plain_planes(m)
    cam = I.look_at((0.3, -3.6, 0.9), width=width, height=height)
    return planes, cam, O.Params(width, height)


@pytest.mark.parametrize("n,seed", [(150, 41), (400, 42)])
def test_aux_forward_and_backward_match_dense_oracle(dev, n, seed):
    planes, cam, prm = small(n, seed)
    attr = attributes(planes)
    say(f"aux maps, {n} Gaussians, 10 attributes")
    flags = O.render(planes, cam, prm)["flags"]
    ok = flags == 0
    pt = D.to_tensors(planes, requires_grad=True)
    at = torch.tensor(attr.astype(np.float64), requires_grad=True)
    _, _, _, ref = D.render(pt, cam.row(), prm, attr_t=at)
    G = np.random.default_rng(seed).normal(size=ref.shape) * ok[None]
    (ref * torch.from_numpy(G)).sum().backward()

    pd = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).requires_grad_(True) for k, v in planes.items()}
    ad = device_rows(attr, dev)
    rnd = R.Renderer(R.Settings(prm.width, prm.height))
    out = AX.render_aux(pd, ad, R.camera_table([cam]), R.Jobs.single(n), rnd, n_attr=len(attr))[0]
    got = out.detach().cpu().numpy()
    refn = ref.detach().numpy()
    scale = np.concatenate([[np.abs(refn[0]).max()], np.abs(attr).max(axis=1)])  # depth, then attributes
    err = np.abs(got - refn)[:, ok].max(axis=1)
    say(f"  map errors {np.array2string(err, precision=2)}")
    assert np.all(err <= 1e-4 * np.maximum(scale, 1.0))
    (out * torch.from_numpy(G.astype(np.float32)).to(dev)).sum().backward()
    check_grad(ad.grad.cpu().numpy()[:, :len(attr)].T, at.grad.numpy(), "d/dattr")
    for k in ("mean", "log_scale", "quat", "opacity"):
        check_grad(pd[k].grad.cpu().numpy(), pt[k].grad.numpy(), f"d/d{k}")


def test_colour_attribute_gives_the_image_at_full_size(dev):
    """300k Gaussians at 800x800 (the single-model configuration): with the
    shading passing the colour through, the colour maps equal the image."""
    m = I.isosurface_model(300_000, I.SEED_SCENE + 2, 0.0)
    planes = I.plain_planes(m)
    n = m.n
    planes["shade"] = np.tile(np.array([[1.0], [0.0], [0.0], [1.0]], np.float32), (1, n))
    cam = I.cameras_at(I.fibonacci_sphere(100), 800, 800)[7]
    pd = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in planes.items()}
    rnd = R.Renderer(R.Settings(800, 800), capacity=1 << 24, check="sync")
    cams = R.camera_table([cam])
    say("aux colour maps vs the image, 300k Gaussians, 800x800")
    img = rnd.forward(pd, cams, R.Jobs.single(n), edits_t=R.default_edits(dev))[0]
    ones = torch.ones((1, n), device=dev)
    attr = torch.cat([pd["color"], ones]).t().contiguous()
    aux = AX.render_aux(pd, attr, cams, R.Jobs.single(n), rnd)[0]
    d = (aux[1:4] - img[:3]).abs().max().item()
    da = (aux[4] - img[3]).abs().max().item()
    say(f"  colour max diff {d:.3e}, alpha max diff {da:.3e}")
    assert d <= 1e-5 and da <= 1e-5
    assert float(aux[0].max()) > 0.0


def test_invalid_attribute_count(dev):
    planes, cam, prm = small(20, 43)
    pd = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in planes.items()}
    with pytest.raises(ValueError):
        AX.render_aux(pd, torch.zeros((20, 16), device=dev), R.camera_table([cam]), R.Jobs.single(20),
                      R.Renderer(R.Settings(prm.width, prm.height)))
    with pytest.raises(ValueError):  # rows not padded to a multiple of 4
        AX.render_aux(pd, torch.zeros((20, 10), device=dev), R.camera_table([cam]), R.Jobs.single(20),
                      R.Renderer(R.Settings(prm.width, prm.height)))


def test_aux_two_jobs_with_overlapping_ranges(dev):
    """Two jobs in one batch (two cameras, overlapping Gaussian ranges): the
    maps of each job against the oracle of its camera and range, and the
    gradients, accumulated over the jobs, against the summed autograd."""
    n = 300
    planes, cam0, prm = small(n, 44)
    cam1 = I.look_at((-2.0, -3.0, 1.5), width=prm.width, height=prm.height)
    attr = attributes(planes)
    ranges = [(cam0, 0, n), (cam1, 80, n - 80)]
    pt = D.to_tensors(planes, requires_grad=True)
    at = torch.tensor(attr.astype(np.float64), requires_grad=True)
    refs, Gs, oks = [], [], []
    total = 0
    for j, (cam, b0, cnt) in enumerate(ranges):
        sub = {k: v[:, b0:b0 + cnt] for k, v in pt.items()}
        sub_np = {k: np.ascontiguousarray(v[:, b0:b0 + cnt]) for k, v in planes.items()}
        ok = O.render(sub_np, cam, prm)["flags"] == 0
        _, _, _, ref = D.render(sub, cam.row(), prm, attr_t=at[:, b0:b0 + cnt])
        G = np.random.default_rng(50 + j).normal(size=ref.shape) * ok[None]
        total = total + (ref * torch.from_numpy(G)).sum()
        refs.append(ref.detach().numpy())
        Gs.append(G)
        oks.append(ok)
    total.backward()
    say("aux maps, two jobs over overlapping ranges")
    pd = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).requires_grad_(True) for k, v in planes.items()}
    ad = device_rows(attr, dev)
    jobs = R.Jobs.ranges([0, 1], [r[1] for r in ranges], [r[2] for r in ranges])
    out = AX.render_aux(pd, ad, R.camera_table([cam0, cam1]), jobs, R.Renderer(R.Settings(prm.width, prm.height)),
                        n_attr=len(attr))
    for j in range(2):
        got = out[j].detach().cpu().numpy()
        scale = np.maximum(np.concatenate([[np.abs(refs[j][0]).max()], np.abs(attr).max(axis=1)]), 1.0)
        err = np.abs(got - refs[j])[:, oks[j]].max(axis=1)
        assert np.all(err <= 1e-4 * scale), (j, err)
    G = torch.from_numpy(np.stack(Gs).astype(np.float32)).to(dev)
    (out * G).sum().backward()
    check_grad(ad.grad.cpu().numpy()[:, :len(attr)].T, at.grad.numpy(), "d/dattr, two jobs")
    for k in ("mean", "log_scale", "quat", "opacity"):
        check_grad(pd[k].grad.cpu().numpy(), pt[k].grad.numpy(), f"d/d{k}, two jobs")


def test_maps_reuse_the_image_bins(dev):
    """Maps rendered from the same inputs as the image reuse its bins (no new
    binning, so the image's backward needs none either): images and maps
    equal those of two renderers that each bin for themselves, gradients
    equal up to the order of the atomic sums; an in-place change of a plane
    makes the next maps bin again."""
    n = 400
    planes, cam, prm = small(n, 45)
    attr = attributes(planes)
    cams, jobs, edits = R.camera_table([cam]), R.Jobs.single(n), R.default_edits(dev)
    G = torch.from_numpy(np.random.default_rng(9).normal(size=(1, 11, prm.height, prm.width))
                         .astype(np.float32)).to(dev)

    def run(shared):
        pd = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev).requires_grad_(True) for k, v in planes.items()}
        ad = device_rows(attr, dev)
        r1 = R.Renderer(R.Settings(prm.width, prm.height))
        r2 = r1 if shared else R.Renderer(R.Settings(prm.width, prm.height))
        rgba = R.rasterize(pd, cams, jobs, r1, edits_t=edits)
        gen = r1.generation
        maps = AX.render_aux(pd, ad, cams, jobs, r2, edits_t=edits, n_attr=len(attr))
        if shared:
            assert r1.generation == gen, "the maps binned again"
        (rgba.abs().sum() + (maps * G).sum()).backward()
        if shared:
            with torch.no_grad():
                pd["opacity"].mul_(0.5)
            AX.render_aux(pd, ad, cams, jobs, r1, edits_t=edits, n_attr=len(attr))
            assert r1.generation == gen + 1, "a changed plane must be binned again"
        return rgba.detach(), maps.detach(), {k: v.grad.cpu().numpy() for k, v in pd.items()}, ad.grad.cpu().numpy()

    say("maps reusing the image's bins")
    a, b = run(True), run(False)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    for k in a[2]:
        np.testing.assert_allclose(a[2][k], b[2][k], rtol=1e-5, atol=1e-6 * max(np.abs(b[2][k]).max(), 1e-30))
    np.testing.assert_allclose(a[3], b[3], rtol=1e-5, atol=1e-6 * np.abs(b[3]).max())


@pytest.mark.parametrize("n_attr", [0, 3, 10, 15])
def test_one_walk_image_and_maps_equal_the_two_walks(dev, n_attr):
    """ivrgs_render_fwd_aux against ivrgs_render_fwd (one pixel per lane)
    and ivrgs_render_aux_fwd on the same bins: the same image bit for bit,
    and the same maps (the same weights and additions in list order).  Two
    jobs over overlapping ranges, and a view of 30k Gaussians at 160x144
    whose lists are long enough to be cut for the backward (the checkpoints
    are then checked through a backward: identical gradients)."""
    for case in ("two_jobs", "long_lists"):
        if case == "two_jobs":
            n = 300
            planes, cam0, prm = small(n, 45)
            cam1 = I.look_at((-2.0, -3.0, 1.5), width=prm.width, height=prm.height)
            cams, jobs = [cam0, cam1], R.Jobs.ranges([0, 1], [0, 80], [n, n - 80])
            W, H = prm.width, prm.height
        else:
            m = I.small_scene(30_000, 812, log_scale_mu=-3.4)
            planes = I.plain_planes(m)
            n, W, H = m.n, 160, 144
            cams, jobs = [I.look_at((0.2, -3.0, 0.6), width=W, height=H)], R.Jobs.single(m.n)
        rng = np.random.default_rng(n_attr + 7)
        S = (n_attr + 3) // 4 * 4
        rows = np.zeros((n, S), np.float32)
        rows[:, :n_attr] = rng.normal(size=(n, n_attr))
        pd = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in planes.items()}
        ad = torch.from_numpy(rows).to(dev)
        cams_t = R.camera_table(cams, dev)
        edits = R.default_edits(dev)
        say(f"one walk vs two, {case}, n_attr={n_attr}")
        rnd = R.Renderer(R.Settings(W, H, fwd_px=1, bwd_px=1))
        img1, maps1 = rnd.forward_maps(pd, cams_t, jobs, ad, n_attr, edits)
        dl = torch.from_numpy(rng.normal(size=tuple(img1.shape)).astype(np.float32)).to(dev)
        g1 = rnd.backward(pd, cams_t, jobs, img1, dl, edits_t=edits)
        g1 = {k: v.clone() for k, v in g1.items()}
        img2 = rnd.forward(pd, cams_t, jobs, edits_t=edits)
        batch = rnd.make_batch(pd, None, edits, cams_t, jobs)
        proj, bins = rnd._structs(batch)
        maps2 = torch.empty_like(maps1)
        N.ivrgs_render_aux_fwd(batch, rnd.settings.params(), proj, bins, ad.data_ptr() if n_attr else None, n_attr,
                               maps2.data_ptr(), None)
        g2 = rnd.backward(pd, cams_t, jobs, img2, dl, edits_t=edits)
        torch.cuda.synchronize()
        assert torch.equal(img1, img2)
        err = (maps1 - maps2).abs().max().item()
        say(f"  image identical; maps max diff {err:.3e}")
        assert err <= 1e-6 * max(1.0, maps2.abs().max().item())
        for k in R.PLANES:  # float atomics: equal to rounding
            a, b = g1[k].cpu().numpy(), g2[k].cpu().numpy()
            assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 1e-5 * np.abs(b).max() + 1e-30), k
