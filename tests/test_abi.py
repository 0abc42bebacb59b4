"""The C-ABI library loads, exports every symbol of include/ivrgs.h, its
struct layouts match the binding, and host-side validation rejects bad
arguments before any launch (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2504_17954_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ivrgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ivrgs_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return N.load()


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert set(names) == set(N.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match(lib):
    for i, s in enumerate(N.STRUCTS):
        assert N.ivrgs_struct_size(i) == C.sizeof(s), s.__name__
    assert N.ivrgs_struct_size(99) == -1


def test_host_validation(lib):
    p = N.ivrgs_params()
    p.alpha_min, p.alpha_max, p.T_min, p.lowpass, p.z_near = 1 / 255, 0.99, 1e-4, 0.3, 0.2
    p.width, p.height, p.tile = 128, 96, 16
    assert N.ivrgs_tiles_per_job(p) == 8 * 6
    b = N.ivrgs_batch()
    b.n_models = 1
    # null batch / params / outputs are rejected without touching the device
    assert lib.ivrgs_project(None, N.ref(p), None, None) == N.E_INVALID
    assert lib.ivrgs_project(N.ref(b), N.ref(p), None, None) == N.E_INVALID
    assert lib.ivrgs_bin_sort(N.ref(b), N.ref(p), None, None, None, 0, None) == N.E_INVALID
    assert lib.ivrgs_render_fwd(N.ref(b), N.ref(p), None, None, None, None, None, 0, None) == N.E_INVALID
    assert lib.ivrgs_render_bwd(N.ref(b), N.ref(p), None, None, None, None, None, None, 0, None) == N.E_INVALID
    fake = C.c_void_p(256)  # non-null placeholder, never dereferenced
    assert lib.ivrgs_render_bwd_aux(N.ref(b), N.ref(p), None, None, None, None, None, 0, None, fake, None, None,
                                    None, 0, None) == N.E_INVALID  # no maps
    assert lib.ivrgs_render_bwd_aux(N.ref(b), N.ref(p), None, None, None, None, None, 16, fake, fake, None, None,
                                    None, 0, None) == N.E_INVALID  # more than 15 attributes
    assert lib.ivrgs_render_bwd_aux(N.ref(b), N.ref(p), None, None, None, None, C.c_void_p(260), 3, fake, fake,
                                    fake, None, None, 0, None) == N.E_INVALID  # unaligned rows
    assert lib.ivrgs_render_fwd_aux(N.ref(b), N.ref(p), None, None, None, 0, fake, fake, None, 0,
                                    None) == N.E_INVALID  # no projection or bins
    pd = N.ivrgs_params.from_buffer_copy(p)
    pd.flags = N.FLAG_DETERMINISTIC_BWD
    assert lib.ivrgs_render_bwd_aux(N.ref(b), N.ref(pd), None, None, None, None, None, 0, fake, fake, None, None,
                                    None, 0, None) == N.E_UNSUPPORTED
    assert lib.ivrgs_render_bwd_aux(N.ref(b), N.ref(p), None, None, None, None, None, 0, fake, fake, None, None,
                                    None, 0, None) == N.E_INVALID  # no batch contents, no outputs
    assert lib.ivrgs_compose(None, 0, None, None, None) == N.E_INVALID
    p2 = N.ivrgs_params.from_buffer_copy(p)
    p2.tile = 8
    assert lib.ivrgs_project(N.ref(b), N.ref(p2), None, None) == N.E_UNSUPPORTED
    p2.tile, p2.fwd_px = 16, 3
    assert lib.ivrgs_project(N.ref(b), N.ref(p2), None, None) == N.E_UNSUPPORTED
    p2.fwd_px, p2.width = 0, 0
    assert lib.ivrgs_project(N.ref(b), N.ref(p2), None, None) == N.E_SHAPE
    b.g.n = -1
    assert lib.ivrgs_project(N.ref(b), N.ref(p), None, None) == N.E_INVALID
    # workspace size is a host computation
    b.g.n = 0
    b.n_jobs, b.max_job_count, b.n_records = 2, 10, 20
    b.jobs = b.cameras = b.edits = 1  # non-null placeholders, never dereferenced
    b.n_jobs = 70_000  # beyond a grid dimension
    assert lib.ivrgs_project(N.ref(b), N.ref(p), None, None) == N.E_SHAPE
    b.n_jobs = 2
    ws = N.ivrgs_workspace_size(b, p, 1000)
    # two (key, id) arrays per record for the depth order, 10 gradient floats per record
    assert ws >= 4 * 4 * 20 + 10 * 4 * 20
    # the block entries of the binning (8 bytes each, capacity / 2 of them
    # besides a fixed part) and, per 256 of them, a part's block and 16 tile
    # counts (68 bytes) grow with the pair capacity
    big = N.ivrgs_workspace_size(b, p, 10 ** 6)
    d_ent = (10 ** 6 - 1000) // 2
    assert abs(big - ws - (8 * d_ent + 68 * d_ent / 256)) <= 1024
    assert N.ivrgs_workspace_size(b, p, -1) == 0
    assert lib.ivrgs_status_string(N.E_CAPACITY).decode().startswith("workspace")


def test_host_validation_of_ssim_and_error_query(lib):
    """The SSIM and L1 entry points and the device-error query check their
    arguments on the host: no device pointer is touched."""
    # workspace: 3 floats per valid window and channel plus one partial per 16x16 tile of windows
    assert N.ivrgs_ssim_workspace_size(4, 800, 800) == 4 * (3 * 4 * 790 * 790 + 4 * 50 * 50)
    assert N.ivrgs_ssim_workspace_size(1, 11, 11) == 4 * (3 + 1)
    for c, h, w in [(0, 32, 32), (2, 10, 40), (2, 40, 10), (-1, 20, 20)]:
        assert N.ivrgs_ssim_workspace_size(c, h, w) == 0
    P = C.c_void_p
    fake = P(256)  # non-null placeholder, never dereferenced
    assert lib.ivrgs_ssim_fwd(None, fake, 1, 20, 20, fake, fake, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_ssim_fwd(fake, fake, 1, 20, 20, fake, None, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_ssim_fwd(fake, fake, 1, 10, 20, fake, fake, 1 << 20, None) == N.E_SHAPE
    assert lib.ivrgs_ssim_fwd(fake, fake, 1, 20, 20, fake, fake, 16, None) == N.E_CAPACITY
    assert lib.ivrgs_ssim_bwd(fake, fake, 1, 20, 20, None, fake, fake, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_ssim_bwd(fake, fake, 1, 20, 5, fake, fake, fake, 1 << 20, None) == N.E_SHAPE
    assert lib.ivrgs_ssim_bwd(fake, fake, 1, 20, 20, fake, fake, fake, 16, None) == N.E_CAPACITY
    # the L1 term: one FP64 partial per workgroup slice of at least 4096 values, at most 1024
    assert N.ivrgs_l1_workspace_size(1) == 8
    assert N.ivrgs_l1_workspace_size(4096 * 3 + 1) == 8 * 4
    assert N.ivrgs_l1_workspace_size(10 ** 9) == 8 * 1024
    assert N.ivrgs_l1_workspace_size(0) == 0 and N.ivrgs_l1_workspace_size(-5) == 0
    assert lib.ivrgs_l1_fwd(None, fake, 10, fake, fake, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_l1_fwd(fake, fake, 10, None, fake, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_l1_fwd(fake, fake, 0, fake, fake, 1 << 20, None) == N.E_SHAPE
    assert lib.ivrgs_l1_fwd(fake, fake, 10 ** 6, fake, fake, 8, None) == N.E_CAPACITY
    assert lib.ivrgs_l1_bwd(fake, fake, 10, None, fake, None) == N.E_INVALID
    assert lib.ivrgs_l1_bwd(fake, fake, -1, fake, fake, None) == N.E_SHAPE
    # the photometric pass: the SSIM workspace plus one L1 partial per workgroup of windows
    assert N.ivrgs_photometric_workspace_size(4, 800, 800) == 4 * (3 * 4 * 790 * 790 + 2 * 4 * 50 * 50)
    assert N.ivrgs_photometric_workspace_size(2, 10, 40) == 0
    assert lib.ivrgs_photometric_fwd(None, fake, 1, 20, 20, fake, fake, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_photometric_fwd(fake, fake, 1, 20, 9, fake, fake, 1 << 20, None) == N.E_SHAPE
    assert lib.ivrgs_photometric_fwd(fake, fake, 1, 20, 20, fake, fake, 16, None) == N.E_CAPACITY
    assert lib.ivrgs_photometric_grad_dev(fake, fake, 1, 20, 20, None, fake, fake, 1 << 20, None) == N.E_INVALID
    assert lib.ivrgs_photometric_grad_dev(fake, fake, 1, 20, 20, fake, fake, fake, 16, None) == N.E_CAPACITY
    # the editable stage's attribute rows: 16-byte aligned rows, n = 0 a no-op
    assert lib.ivrgs_editable_attr_fwd(fake, fake, fake, -1, fake, None) == N.E_INVALID
    assert lib.ivrgs_editable_attr_fwd(None, fake, fake, 10, fake, None) == N.E_INVALID
    assert lib.ivrgs_editable_attr_fwd(fake, fake, fake, 10, P(260), None) == N.E_INVALID
    assert lib.ivrgs_editable_attr_fwd(None, None, None, 0, None, None) == N.OK
    assert lib.ivrgs_editable_attr_bwd(fake, 10, P(264), fake, fake, fake, None) == N.E_INVALID
    assert lib.ivrgs_editable_attr_bwd(fake, 10, fake, None, fake, fake, None) == N.E_INVALID
    assert lib.ivrgs_editable_attr_bwd(fake, -3, fake, fake, fake, fake, None) == N.E_INVALID
    out = C.c_int64(0)
    assert lib.ivrgs_get_error(None, None, C.cast(C.byref(out), P), None) == N.E_INVALID
    bins = N.ivrgs_bins(0, 0, 0, 0)  # no status word
    assert lib.ivrgs_get_error(N.ref(bins), None, C.cast(C.byref(out), P), None) == N.E_INVALID
    bins = N.ivrgs_bins(0, 0, 0, 256)
    assert lib.ivrgs_get_error(N.ref(bins), None, None, None) == N.E_INVALID


def test_host_validation_of_cull(lib):
    """ivrgs_cull rejects missing or misaligned weights on the host (the MLP
    loads four BF16 weights at a time, 8-byte aligned)."""
    P = C.c_void_p
    g = N.ivrgs_gaussians(0, *([256] * (len(N.PLANES) + 1)))  # empty set, non-null planes never read
    fake = P(256)  # non-null placeholder, never dereferenced: every call below fails its host checks
    w = N.ivrgs_culler(256, 256, 256, 256, 256, 0.0, 0.0)
    ws = N.ivrgs_cull_workspace_size(0)
    for bad in ("w1", "w2"):
        wb = N.ivrgs_culler.from_buffer_copy(w)
        setattr(wb, bad, 258)  # 2-byte aligned only
        assert lib.ivrgs_cull(N.ref(g), fake, 0, N.ref(wb), fake, fake, 0, None, fake, ws, None) == N.E_INVALID
    wn = N.ivrgs_culler.from_buffer_copy(w)
    wn.w3 = None
    assert lib.ivrgs_cull(N.ref(g), fake, 0, N.ref(wn), fake, fake, 0, None, fake, ws, None) == N.E_INVALID
