"""The regulariser kernels (ivrgs_reg_fwd / ivrgs_reg_bwd: normal
consistency with the pseudo-normal, offset-colour sparsity, bilateral
smoothness, opacity L1; Eq. 5-7, Sec. 4.3) against the FP64 oracle
(oracle/regularisers.py) on the same seeded float32 maps, through the C ABI.

Tolerances.  The kernel evaluates in FP32.  The valid-pixel count and the
validity mask are integer decisions on the same FP32 alpha values: exact.
The pseudo-normal's central differences are formed relative to themselves
(a Kahan-form determinant), so N~ is within a few hundred FP32 roundings:
2e-5 per component; pixels whose facing decision N~ . P is within 1e-4 of
0 (grazing) may take either side and are left out of that comparison.
Terms: 2e-5 absolute on the normal consistency (a mean of per-pixel values
each within the N~ bound), 1e-5 relative on the others (FP32 sums of at
most 256 terms per workgroup, FP64 across).  Gradients per tensor at the
usual bar |g - g_ref| <= 1e-3 |g_ref| + 1e-5 max |g_ref|; for the normal
gradient, pixels where || N/|N| - N~ || < 0.05 are left out: there its
direction is set by N~'s FP32 error over that length."""
import sys

import numpy as np
import pytest
import torch

from oracle import regularisers as G
from paper_2504_17954_amd import inputs as I
from paper_2504_17954_amd import losses as L
from paper_2504_17954_amd import native as N

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    N.load()
    return torch.device("cuda:0")


def run_gpu(dev, m, cam, gterm, keys=("normal", "delta_c", "shade", "opacity")):
    d = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in m.items()}
    H, W = m["alpha"].shape
    maps = N.ivrgs_reg_maps()
    maps.depth, maps.alpha, maps.target = d["depth"].data_ptr(), d["alpha"].data_ptr(), d["target"].data_ptr()
    for k in ("normal", "delta_c", "shade"):
        if k in keys:
            setattr(maps, k, d[k].data_ptr())
    if "opacity" in keys:
        maps.opacity, maps.n_gauss = d["opacity"].data_ptr(), d["opacity"].numel()
    maps.height, maps.width = H, W
    c = L.camera_struct(cam)
    ws = torch.empty(N.ivrgs_reg_workspace_size(maps), dtype=torch.uint8, device=dev)
    terms = torch.full((5,), float("nan"), device=dev)
    pn = torch.full((3, H, W), float("nan"), device=dev)
    s = torch.cuda.current_stream().cuda_stream
    N.ivrgs_reg_fwd(maps, c, terms.data_ptr(), pn.data_ptr(), ws.data_ptr(), ws.numel(), s)
    g = torch.tensor(gterm, dtype=torch.float32, device=dev)
    outs = {k: torch.full_like(d[k], float("nan")) for k in keys}
    gdepth = torch.full_like(d["depth"], float("nan"))
    N.ivrgs_reg_bwd(maps, c, terms.data_ptr(), g.data_ptr(),
                    *[outs[k].data_ptr() if k in outs else None for k in ("normal", "delta_c", "shade", "opacity")], s,
                    gdepth.data_ptr())
    torch.cuda.synchronize()
    assert bool((gdepth == 0).all())  # no gradient to the depth map: written as zeros
    return terms.cpu().numpy(), pn.cpu().numpy(), {k: v.cpu().numpy() for k, v in outs.items()}


def check_grad(g, ref, what, mask=None):
    if mask is not None:
        g, ref = g[..., mask], ref[..., mask]
    tol = 1e-3 * np.abs(ref) + 1e-5 * np.abs(ref).max() + 1e-30
    bad = np.abs(g - ref) > tol
    say(f"{what}: max |g - ref| {np.abs(g - ref).max():.3e} (max |ref| {np.abs(ref).max():.3e}), "
        f"{int(bad.sum())} outside")
    assert not bad.any()


@pytest.mark.parametrize("H,W,seed", [(37, 53, 1), (96, 130, 2), (800, 800, 3)])
def test_regularisers_match_oracle(dev, H, W, seed):
    cam = I.look_at((0.3, -3.5, 0.6), width=W, height=H)
    m = I.view_maps(H, W, seed, n_gauss=1000 + seed)
    gterm = [0.7, 1.3, -0.4, 2.0]
    terms, pn, g = run_gpu(dev, m, cam, gterm)
    ref = G.terms(m["depth"], m["alpha"], m["normal"], m["delta_c"], m["shade"], m["target"], m["opacity"], cam,
                  grad_terms=np.asarray(gterm))
    valid = ref["valid"]
    say(f"{H}x{W}: terms {terms[:4]} vs {ref['terms']}, valid {int(terms[4])} vs {ref['count']}")
    assert int(terms[4]) == ref["count"] and ref["count"] > 0
    # N~: zero at invalid pixels, within 2e-5 elsewhere (facing decision clear)
    assert np.all(pn[:, ~valid] == 0.0)
    ys, xs = np.nonzero(valid)
    P = np.stack([(xs + 0.5 - cam.cx) / cam.fx, (ys + 0.5 - cam.cy) / cam.fy, np.ones_like(xs, np.float64)])
    nc = np.asarray(cam.R, np.float64) @ ref["pseudo_normal"][:, ys, xs]  # back to camera space
    clear = np.abs((nc * P).sum(0)) / np.linalg.norm(P, axis=0) > 1e-4
    err = np.abs(pn[:, ys, xs] - ref["pseudo_normal"][:, ys, xs])[:, clear]
    say(f"pseudo-normal: max err {err.max():.3e} over {int(clear.sum())} pixels ({int((~clear).sum())} grazing)")
    assert err.max() <= 2e-5
    assert abs(terms[0] - ref["terms"][0]) <= 2e-5
    np.testing.assert_allclose(terms[1:4], ref["terms"][1:4], rtol=1e-5)
    # normal gradient away from pixels where N/|N| is within 0.05 of N~
    nrm = m["normal"].astype(np.float64)
    lgap = np.linalg.norm(nrm / np.linalg.norm(nrm, axis=0) - ref["pseudo_normal"], axis=0)
    keep = ~(valid & (lgap < 0.05))
    assert np.all(g["normal"][:, ~valid] == 0.0)
    check_grad(g["normal"], ref["grad_normal"], "grad normal", keep)
    check_grad(g["delta_c"], ref["grad_delta_c"], "grad delta-c")
    check_grad(g["shade"], ref["grad_shade"], "grad shade")
    check_grad(g["opacity"], ref["grad_opacity"], "grad opacity")


def test_regularisers_edge_cases(dev):
    H, W = 20, 24
    cam = I.look_at((0.0, -3.0, 0.0), width=W, height=H)
    m = I.view_maps(H, W, 9)
    # no valid pixel: the normal term and its gradient vanish
    m0 = dict(m, alpha=np.full((H, W), 0.5, np.float32))
    terms, pn, g = run_gpu(dev, m0, cam, [1.0, 1.0, 1.0, 1.0])
    assert terms[0] == 0.0 and terms[4] == 0.0
    assert np.all(pn == 0.0) and np.all(g["normal"] == 0.0)
    # absent maps drop their terms
    terms, _, g = run_gpu(dev, m, cam, [1.0, 1.0, 1.0, 1.0], keys=("normal",))
    assert np.all(terms[1:4] == 0.0) and terms[0] > 0.0
    # host validation: too small, shade without target, gradient without its map
    maps = N.ivrgs_reg_maps()
    maps.height, maps.width = 2, 24
    lib = N.load()
    assert lib.ivrgs_reg_fwd(N.ref(maps), N.ref(L.camera_struct(cam)), None, None, None, 0, None) == N.E_SHAPE
    maps.height = 20
    maps.shade = 1
    assert lib.ivrgs_reg_workspace_size(N.ref(maps)) == 0
    maps.shade = None
    assert lib.ivrgs_reg_bwd(N.ref(maps), N.ref(L.camera_struct(cam)), 1, 1, 1, None, None, None,
                             None, None) == N.E_INVALID


def test_editable_loss_regularisers_autograd(dev):
    """losses.regularisers as an autograd Function: the weighted terms'
    gradients equal the oracle's with the appendix weights as upstream."""
    H, W = 64, 72
    cam = I.look_at((0.3, -3.5, 0.6), width=W, height=H)
    m = I.view_maps(H, W, 4, n_gauss=500)
    d = {k: torch.from_numpy(v).to(dev) for k, v in m.items()}
    for k in ("normal", "delta_c", "shade", "opacity"):
        d[k].requires_grad_(True)
    t = L.regularisers(d["depth"], d["alpha"], cam, normal=d["normal"], delta_c=d["delta_c"], shade=d["shade"],
                       target=d["target"], opacity=d["opacity"])
    w = torch.tensor([L.W_REG, L.W_REG, L.W_REG, L.W_OPACITY], device=dev)
    (t * w).sum().backward()
    ref = G.terms(m["depth"], m["alpha"], m["normal"], m["delta_c"], m["shade"], m["target"], m["opacity"], cam,
                  grad_terms=np.array([L.W_REG, L.W_REG, L.W_REG, L.W_OPACITY]))
    np.testing.assert_allclose(t.detach().cpu().numpy()[1:], ref["terms"][1:], rtol=1e-5)
    nrm = m["normal"].astype(np.float64)
    lgap = np.linalg.norm(nrm / np.linalg.norm(nrm, axis=0) - ref["pseudo_normal"], axis=0)
    check_grad(d["normal"].grad.cpu().numpy(), ref["grad_normal"], "autograd normal",
               ~(ref["valid"] & (lgap < 0.05)))
    check_grad(d["shade"].grad.cpu().numpy(), ref["grad_shade"], "autograd shade")
    check_grad(d["opacity"].grad.cpu().numpy(), ref["grad_opacity"], "autograd opacity")
