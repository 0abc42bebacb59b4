"""GPU parity of the inverse-exploration gradients (Sec. 4.6) against the
oracle, through the C ABI: the per-model edit parameters (palette, opacity
scale, light magnitude lambda * k + b) from the composed set's gradients, and
the orbital light direction from the record gradients a backward leaves.

Tolerances: a float32 sum of n terms against the FP64 sum, 3e-5 of the sum of
the terms' magnitudes; sums of rendered gradients, the per-Gaussian gradient
tolerance (1e-3 relative + 1e-5 of the largest) carried through the sum; the
light direction, 1e-3 relative + 1e-5 of the largest component.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import raster as R

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def to_dev(planes, dev):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in planes.items()}


def abs_planes(d):
    return {k: np.abs(np.asarray(v, np.float64)) for k, v in d.items()}


def random_grads(total, seed):
    rng = np.random.default_rng(seed)
    return {k: rng.normal(size=(dm, total)).astype(np.float32) for k, dm in zip(R.PLANES, R.N.PLANE_DIMS)}


@pytest.mark.parametrize("sizes", [(1, 300_000, 257), (0, 5000), (70_001,)])
def test_compose_bwd_sums(dev, sizes):
    """Segmented sums over model slices, including an empty model, a single
    Gaussian and a slice longer than one pass of the grid-stride loop."""
    ms = [I.small_scene(n, 900 + i) if n else None for i, n in enumerate(sizes)]
    planes = [m.planes if m is not None else {k: np.zeros((d, 0), np.float32)
                                              for k, d in zip(R.PLANES, R.N.PLANE_DIMS)} for m in ms]
    total = sum(sizes)
    grads = random_grads(total, 31 + len(sizes))
    say(f"compose_bwd sums, model sizes {sizes}")
    rows = np.zeros((len(sizes), 16), np.float32)
    ref = O.compose_bwd(planes, rows, grads)
    mag = O.compose_bwd([abs_planes(p) for p in planes], rows, abs_planes(grads))
    g = R.compose_bwd([to_dev(p, dev) for p in planes], to_dev(grads, dev)).cpu().numpy()
    err = np.abs(g - ref)
    say(f"  max err {err.max():.3e}, worst ratio {(err / (3e-5 * mag + 1e-30)).max():.3f}")
    assert np.all(err <= 3e-5 * mag), np.argwhere(err > 3e-5 * mag)[:5]
    for i, n in enumerate(sizes):
        if n == 0:
            assert np.all(g[i] == 0.0)


def composed_scene(seed, width, height, headlight_first=True):
    ms = [I.small_scene(900 + 300 * k, 700 + k + seed, log_scale_mu=-3.2) for k in range(3)]
    rng = np.random.default_rng(seed)
    edits = []
    for k, m in enumerate(ms):
        e = I.identity_edit(m)
        e.palette = rng.uniform(0, 0.5, 3).astype(np.float32)
        e.opacity_scale = np.float32(rng.uniform(0.7, 1.3))
        e.shade_scale = rng.uniform(0.7, 1.3, 4).astype(np.float32)
        e.shade_bias = rng.uniform(-0.05, 0.05, 4).astype(np.float32)
        d = rng.normal(size=3) * rng.uniform(0.5, 2.0)  # unnormalised on purpose
        e.light_dir = d.astype(np.float32)
        e.headlight = headlight_first and k == 0
        edits.append(e)
    cam = I.look_at((0.5, -3.9, 0.7), width=width, height=height)
    return ms, edits, cam, O.Params(width, height)


def shading_kinks(planes, cam, prm, rows, mid):
    p = O.project(planes, cam, prm, edits=rows, model_id=mid)
    return (np.abs(p[:, 19]) < 1e-5) | (np.abs(p[:, 20]) < 1e-3)


@pytest.mark.parametrize("seed,W,H", [(0, 80, 64), (3, 61, 47)])
def test_edit_and_light_gradients_end_to_end(dev, seed, W, H):
    ms, edits, cam, prm = composed_scene(seed, W, H)
    rows = np.stack([e.row() for e in edits])
    pl_ref, mid_ref = O.compose([m.planes for m in ms], rows)
    # drop the Gaussians at a shading kink (a jump in the derivative that
    # float32 and FP64 may take on different sides), then compose again
    kinks = shading_kinks(pl_ref, cam, prm, rows, mid_ref)
    for m in ms:
        n = m.planes["mean"].shape[1]
        keep = ~kinks[:n]
        kinks = kinks[n:]
        m.planes = {k: np.ascontiguousarray(v[:, keep]) for k, v in m.planes.items()}
    pl_ref, mid_ref = O.compose([m.planes for m in ms], rows)
    assert not shading_kinks(pl_ref, cam, prm, rows, mid_ref).any()
    say(f"inverse gradients end to end, seed {seed}, {W}x{H}, {len(mid_ref)} Gaussians")
    ref = O.render(pl_ref, cam, prm, model_id=mid_ref, edits=rows)
    tgt = np.random.default_rng(seed + 7).uniform(0, 1, ref["rgba"].shape)
    dl = O.l1_loss_grad(ref["rgba"], tgt)
    dl[:, ref["flags"] != 0] = 0.0
    g_ref, grec_ref = O.backward(pl_ref, cam, prm, dl, model_id=mid_ref, edits=rows)
    e_ref = O.compose_bwd([m.planes for m in ms], rows, g_ref)
    l_ref = O.light_grad(pl_ref, cam, prm, grec_ref, model_id=mid_ref, edits=rows)

    out, mid = R.compose([to_dev(m.planes, dev) for m in ms], edits)
    et = R.edit_table(edits, dev)
    rnd = R.Renderer(R.Settings(W, H))
    cams, jobs = R.camera_table([cam]), R.Jobs.single(mid.numel())
    rgba = rnd.forward(out, cams, jobs, model_id=mid, edits_t=et)
    g = rnd.backward(out, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                     model_id=mid, edits_t=et)
    e_gpu = R.compose_bwd([to_dev(m.planes, dev) for m in ms], g).cpu().numpy()
    l_gpu = rnd.light_grad(out, cams, jobs, model_id=mid, edits_t=et).cpu().numpy()

    # per-Gaussian gradient tolerance carried through each sum
    tol_g = {k: 1e-3 * np.abs(g_ref[k]) + 1e-5 * np.abs(g_ref[k]).max() for k in R.PLANES}
    tol_e = O.compose_bwd([abs_planes(m.planes) for m in ms], rows, tol_g) + 1e-30
    err = np.abs(e_gpu - e_ref)
    say(f"  edit grads: max |g| {np.abs(e_ref).max():.3e}, worst ratio {(err / tol_e).max():.3f}")
    assert np.all(err <= tol_e), np.argwhere(err > tol_e)[:5]

    assert np.all(l_gpu[0] == 0.0) and np.all(l_ref[0] == 0.0)  # headlight model
    tol_l = 1e-3 * np.abs(l_ref) + 1e-5 * np.abs(l_ref).max()
    err = np.abs(l_gpu - l_ref)
    say(f"  light grads: max |g| {np.abs(l_ref).max():.3e}, worst ratio {(err / tol_l).max():.3f}")
    assert np.abs(l_ref[1:]).max() > 0.0
    assert np.all(err <= tol_l), (l_gpu, l_ref)
