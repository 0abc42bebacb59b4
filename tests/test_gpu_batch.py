"""Batched jobs, persistent render kernels, culling index lists and graph
capture, on the GPU through the C ABI."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_17954_amd import batch as B
from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import native as N
from paper_2504_17954_amd import raster as R
from test_gpu_parity import check_grads, check_image, grad_exclusions, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    N.load()
    return torch.device("cuda:0")


def c1():
    m = I.c1().models[0]
    return I.plain_planes(m), I.look_at((0.0, -4.0, 0.0), width=128, height=128)


def test_persistent_forward_bit_identical(dev):
    planes, cam = c1()
    pd = to_dev(planes, dev)
    out = []
    for flags in (0, N.FLAG_PERSISTENT):
        for per_cu in ((0,) if flags == 0 else (0, 1, 3)):
            rnd = R.Renderer(R.Settings(128, 128, flags=flags, persist_per_cu=per_cu))
            out.append(rnd.forward(pd, R.camera_table([cam]), R.Jobs.single(10_000),
                                   edits_t=R.default_edits(dev)).cpu().numpy())
    for o in out[1:]:
        assert np.array_equal(o, out[0])


def test_persistent_backward(dev):
    planes, cam = c1()
    prm = O.Params(128, 128)
    ref = O.render(planes, cam, prm)
    dl = O.l1_loss_grad(ref["rgba"], np.random.default_rng(3).uniform(0, 1, ref["rgba"].shape))
    dl[:, ref["flags"] != 0] = 0.0
    g_ref, _ = O.backward(planes, cam, prm, dl)
    rnd = R.Renderer(R.Settings(128, 128, flags=N.FLAG_PERSISTENT))
    pd = to_dev(planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(10_000)
    rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
    g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                     edits_t=R.default_edits(dev))
    check_grads({k: v.cpu().numpy() for k, v in g.items()}, g_ref, "persistent bwd",
                exclude=grad_exclusions(planes, cam, prm))


def test_split_backward_matches_whole_walks(dev):
    """Long tile lists are cut and their segments walked from the forward's
    checkpoints (one pixel per lane); the persistent launch walks every list
    whole.  Both equal the oracle gradient, and each other to rounding."""
    m = I.small_scene(30_000, 811, log_scale_mu=-3.4)
    planes = I.plain_planes(m)
    cam = I.look_at((0.2, -3.0, 0.6), width=96, height=96)
    prm = O.Params(96, 96)
    ref = O.render(planes, cam, prm)
    dl = O.l1_loss_grad(ref["rgba"], np.random.default_rng(12).uniform(0, 1, ref["rgba"].shape))
    dl[:, ref["flags"] != 0] = 0.0
    g_ref, _ = O.backward(planes, cam, prm, dl)
    pd = to_dev(planes, dev)
    cams, jobs = R.camera_table([cam]), R.Jobs.single(m.n)
    out = {}
    for name, flags in (("split", 0), ("whole", N.FLAG_PERSISTENT)):
        rnd = R.Renderer(R.Settings(96, 96, flags=flags))
        rgba = rnd.forward(pd, cams, jobs, edits_t=R.default_edits(dev))
        lens = np.diff(rnd.tile_start[:37].cpu().numpy().astype(np.int64))
        g = rnd.backward(pd, cams, jobs, rgba, torch.from_numpy(dl[None].astype(np.float32)).to(dev),
                         edits_t=R.default_edits(dev))
        out[name] = {k: v.cpu().numpy() for k, v in g.items()}
        say(f"{name}: longest tile list {lens.max()} (cut above 128, into up to 16 segments)")
        assert lens.max() > 16 * 128  # the longest lists take every cut
        check_grads(out[name], g_ref, f"{name} bwd", exclude=grad_exclusions(planes, cam, prm))
    for k in R.PLANES:
        a, b = out["split"][k], out["whole"][k]
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 1e-6 * np.abs(b).max()), k


def batched_setup(W=64, H=48, n_views=3):
    sizes = (300, 800, 1500)
    models = [I.small_scene(n, 700 + i, log_scale_mu=-3.0) for i, n in enumerate(sizes)]
    planes = {k: np.concatenate([I.plain_planes(m)[k] for m in models], 1) for k in R.PLANES}
    cams = I.cameras_at(I.fibonacci_sphere(n_views), W, H)
    return sizes, planes, cams


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_jobs(dev, persistent):
    """models x views jobs in one launch sequence: every image equals the
    job rendered alone (bit-identical) and the oracle; the gradient of a
    Gaussian seen by several views is the sum of the per-view oracle
    gradients."""
    W, H = 64, 48
    sizes, planes, cams = batched_setup(W, H)
    jobs = R.Jobs.models_by_views(sizes, len(cams))
    flags = N.FLAG_PERSISTENT if persistent else 0
    pd = to_dev(planes, dev)
    cams_t = R.camera_table(cams, dev)
    rnd = R.Renderer(R.Settings(W, H, flags=flags))
    rgba = rnd.forward(pd, cams_t, jobs, edits_t=R.default_edits(dev))
    imgs = rgba.cpu().numpy()
    starts = np.concatenate([[0], np.cumsum(sizes)])
    prm = O.Params(W, H)
    dl = np.zeros_like(imgs)
    g_ref = {k: np.zeros((d, planes["mean"].shape[1])) for k, d in zip(O.PLANES, O.DIMS)}
    excl = np.zeros(planes["mean"].shape[1], bool)
    for j, (cam_i, begin, count, _) in enumerate(jobs.host):
        sub = {k: v[:, begin:begin + count] for k, v in planes.items()}
        alone = R.Renderer(R.Settings(W, H)).forward(to_dev(sub, dev), R.camera_table([cams[cam_i]], dev),
                                                     R.Jobs.single(count), edits_t=R.default_edits(dev))
        assert np.array_equal(alone[0].cpu().numpy(), imgs[j]), j
        ref = O.render(sub, cams[cam_i], prm)
        check_image(imgs[j], ref, f"job {j}")
        d = np.random.default_rng(j).normal(size=ref["rgba"].shape) * (ref["flags"] == 0)[None] / imgs.size
        dl[j] = d
        gj, _ = O.backward(sub, cams[cam_i], prm, d)
        for k in O.PLANES:
            g_ref[k][:, begin:begin + count] += gj[k]
        excl[begin:begin + count] |= grad_exclusions(sub, cams[cam_i], prm)
    assert sorted(set(np.searchsorted(starts, jobs.host[:, 1], side="right") - 1)) == [0, 1, 2]
    g = rnd.backward(pd, cams_t, jobs, rgba, torch.from_numpy(dl.astype(np.float32)).to(dev),
                     edits_t=R.default_edits(dev))
    check_grads({k: v.cpu().numpy() for k, v in g.items()}, g_ref, f"batched bwd persistent={persistent}",
                exclude=excl)


def test_index_list_equals_subset(dev):
    """A job over an index list (culling survivors) renders exactly like the
    extracted subset."""
    planes, cam = c1()
    keep = np.flatnonzero(np.random.default_rng(4).random(10_000) < 0.6).astype(np.int32)
    pd = to_dev(planes, dev)
    idx = torch.from_numpy(keep).to(dev)
    cams = R.camera_table([cam])
    a = R.Renderer(R.Settings(128, 128)).forward(pd, cams, R.Jobs.single(keep.size), edits_t=R.default_edits(dev),
                                                  gauss_index=idx)
    sub = to_dev({k: np.ascontiguousarray(v[:, keep]) for k, v in planes.items()}, dev)
    b = R.Renderer(R.Settings(128, 128)).forward(sub, cams, R.Jobs.single(keep.size), edits_t=R.default_edits(dev))
    assert torch.equal(a, b)


def test_graph_replay_matches_eager(dev):
    """A captured batched step replays with the eager result: images
    bit-identical, gradients equal up to the order of float atomics; eager
    work runs between replays."""
    W, H = 64, 48
    sizes, planes, cams = batched_setup(W, H)
    jobs = R.Jobs.models_by_views(sizes, len(cams))
    pd = to_dev(planes, dev)
    targets = torch.rand((jobs.n_jobs, 4, H, W), device=dev)
    step = B.BatchStep(pd, R.camera_table(cams, dev), jobs, targets, B.batch_settings(W, H))
    g_eager = {k: v.clone() for k, v in step.step().items()}
    img_eager = step.rgba.clone()
    step.capture()
    for rep in range(3):
        step.rgba.zero_()
        for v in step.grads.values():
            v.fill_(7.0)
        _ = torch.randn(1000, device=dev).sum().item()  # unrelated eager work
        step.replay()
        torch.cuda.synchronize()
        assert torch.equal(step.rgba, img_eager), rep
        for k in R.PLANES:
            a, b = step.grads[k], g_eager[k]
            tol = 1e-5 * b.abs() + 1e-6 * b.abs().max() + 1e-30
            assert bool(((a - b).abs() <= tol).all()), (rep, k)
    step.verify()


# ------------------------------------------------------------------ culler
def bf16_round(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_ulp(x):
    a = np.abs(np.asarray(x, np.float32)).astype(np.float64)
    e = np.floor(np.log2(np.maximum(a, 1e-30)))
    return np.where(a > 0, 2.0 ** (e - 7), 2.0 ** -133)


def mlp_logit_bound(x16, W1, b1, W2, b2, w3, b3, x_amb=None):
    """FP64 reference logits of the BF16 MLP and, per Gaussian, the largest
    difference an FP32 evaluation in any summation order may show: one bf16
    ulp on each first-layer activation whose FP32 sum (17 terms) lies within
    its accumulation error of a bf16 rounding boundary, times that
    activation's largest effect on the logit, plus the FP32 accumulation
    error of the second layer and the output (gamma_n = n 2^-24 times the
    sums of magnitudes).  x_amb [n, 16] (optional): per input feature, the
    size of a bf16 rounding the kernel may take the other way (a feature it
    computes in FP32 that lies within a few FP32 ulps of a bf16 midpoint),
    propagated through the first layer."""
    W1, W2 = W1.astype(np.float64), W2.astype(np.float64)
    b1, b2, w3 = (np.asarray(v, np.float64) for v in (b1, b2, w3))
    v1 = x16.astype(np.float64) @ W1.T + b1
    e_in = 0.0 if x_amb is None else x_amb @ np.abs(W1).T
    e1 = 17 * 2.0 ** -24 * (np.abs(x16) @ np.abs(W1).T + np.abs(b1)) + e_in
    lo = bf16_round(np.maximum(v1 - e1, 0))
    hi = bf16_round(np.maximum(v1 + e1, 0))
    h1 = bf16_round(np.maximum(v1, 0)).astype(np.float64)
    reach = np.abs(W2).T @ np.abs(w3)
    amb = ((lo != hi) * np.maximum(bf16_ulp(lo), bf16_ulp(hi)) * reach[None, :]).sum(1)
    amb = amb + (np.asarray(e_in) * reach[None, :]).sum(1) if x_amb is not None else amb
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    g = 66 * 2.0 ** -24
    acc = g * ((np.abs(h1) @ np.abs(W2).T + np.abs(b2)) @ np.abs(w3)) + g * (np.abs(h2) @ np.abs(w3) + abs(b3))
    return h2 @ w3 + b3, amb + acc


def random_culler(dev, seed=0, threshold=0.0):
    from paper_2504_17954_amd import cull as CU
    torch.manual_seed(seed)
    m = CU.MLP().to(dev)
    mean = torch.zeros(10, device=dev)
    std = torch.ones(10, device=dev)
    return m, CU.pack(m, mean, std, threshold)


def test_cull_mlp_matches_reference(dev):
    """The BF16 matrix-core MLP equals the same network evaluated in FP64
    with BF16-rounded weights, inputs and first-layer activations, every
    logit within the bound of an FP32 evaluation (exercises the MFMA operand
    layouts)."""
    from paper_2504_17954_amd import cull as CU
    m = I.small_scene(5000, 801, log_scale_mu=-3.0)
    planes = I.plain_planes(m)
    cam = I.look_at((0.7, -3.1, 2.2), width=64, height=64)
    pd = to_dev(planes, dev)
    cams_t = R.camera_table([cam], dev)
    model, w = random_culler(dev, 3, threshold=-1e30)
    cu = CU.Culler(w, 5000)
    jobs = R.Jobs.single(5000)
    cu.run(pd, cams_t, jobs, 0, want_logits=True)
    got = cu.logits.cpu().numpy()
    # the unit direction to the camera is computed by the kernel in FP32 and
    # then rounded to bf16: the reference takes that rounding in the same
    # precision, with the kernel's operation order (camera centre -R^T t,
    # difference, squared length, reciprocal square root, product)
    f32 = np.float32
    Rm, tv = cam.R.astype(f32), cam.t.astype(f32)
    cpos = np.array([-(Rm[0, i] * tv[0] + Rm[1, i] * tv[1] + Rm[2, i] * tv[2]) for i in range(3)], f32)
    v = cpos[:, None] - planes["mean"].astype(f32)
    inv = f32(1) / np.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])
    d = (v * inv).T.astype(f32)
    x = np.concatenate([planes["mean"].T, planes["log_scale"].T, planes["opacity"].T, d], 1)
    x16 = np.zeros((5000, 16), np.float32)
    x16[:, :10] = bf16_round(x)
    # a direction component within 4 FP32 ulps of a bf16 midpoint may round
    # the other way in the kernel (its square root and division need not be
    # correctly rounded): one bf16 ulp of input there
    mid = (bf16_round(d) + np.float32(0.5) * bf16_ulp(d).astype(np.float32) * np.sign(d - bf16_round(d)))
    near = np.abs(d.astype(np.float64) - mid) <= 4 * np.spacing(np.abs(d)).astype(np.float64)
    x_amb = np.zeros((5000, 16))
    x_amb[:, 7:10] = near * bf16_ulp(d)
    w1 = w.w1.cpu().numpy().astype(np.int32).astype(np.uint32) << 16
    w2 = w.w2.cpu().numpy().astype(np.int32).astype(np.uint32) << 16
    W1 = (w1 & 0xFFFF0000).astype(np.uint32).view(np.float32)
    W2 = (w2 & 0xFFFF0000).astype(np.uint32).view(np.float32)
    ref, bound = mlp_logit_bound(x16, W1, w.b1.cpu().numpy(), W2, w.b2.cpu().numpy(), w.w3.cpu().numpy(),
                                 float(w.b3), x_amb)
    say(f"cull mlp: {int(near.any(1).sum())} Gaussians with a direction component at a bf16 midpoint")
    err = np.abs(got - ref)
    say(f"cull mlp: max err {err.max():.3e}, max |logit| {np.abs(ref).max():.3e}, "
        f"worst err / bound {(err / bound).max():.3f}")
    assert np.all(err <= bound), np.argsort(-(err / bound))[:5]
    assert jobs.device[0, 2].item() == 5000


def test_cull_compaction_and_fallback(dev):
    from paper_2504_17954_amd import cull as CU
    planes, cam = c1()
    pd = to_dev(planes, dev)
    cams_t = R.camera_table([cam], dev)
    _, w = random_culler(dev, 5)
    cu = CU.Culler(w, 10_000)
    jobs = R.Jobs.single(10_000)
    w.threshold = -1e30
    cu.run(pd, cams_t, jobs, 0, want_logits=True)
    logits = cu.logits.cpu().numpy()
    w.threshold = float(np.median(logits))
    idx = cu.run(pd, cams_t, jobs, 0)
    k = int(jobs.device[0, 2].item())
    want = np.flatnonzero(logits >= w.threshold)
    assert k == want.size
    assert np.array_equal(idx[:k].cpu().numpy(), want)
    # forced fallback: keep everything -> bit-identical to the plain render
    w.threshold = -1e30
    rnd = R.Renderer(R.Settings(128, 128))
    a = cu.render(rnd, pd, cams_t, jobs, 0).clone()
    b = R.Renderer(R.Settings(128, 128)).forward(pd, cams_t, R.Jobs.single(10_000), edits_t=R.default_edits(dev))
    assert torch.equal(a, b)


def test_maxw_labels_match_oracle(dev):
    """Culling labels from the rasterizer equal the oracle's max T*alpha >=
    1/255, except where the oracle's value is within FP32 noise of 1/255."""
    planes, cam = c1()
    pd = to_dev(planes, dev)
    _, maxw = R.Renderer(R.Settings(128, 128)).forward(pd, R.camera_table([cam], dev), R.Jobs.single(10_000),
                                                        edits_t=R.default_edits(dev), want_maxw=True)
    ref = O.render(planes, cam, O.Params(128, 128), want_maxw=True)
    g = maxw[:10_000].cpu().numpy()
    r = ref["maxw"]
    clear = np.abs(r - 1 / 255) > 1e-4 / 255
    assert np.array_equal((g >= 1 / 255)[clear], (r >= 1 / 255)[clear])
    both = (r > 0) & (g > 0)
    rel = np.abs(g[both] - r[both]) / r[both]
    assert np.quantile(rel, 0.999) <= 1e-3
