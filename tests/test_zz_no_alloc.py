"""ivrgs_bin_sort_noalloc (binning with its scratch in a static device
array, for callers that cannot allocate) against ivrgs_bin_sort with a
caller workspace, through the C ABI: tile lists, pair totals and status
words bit-identical on two calls in a row, the second with a smaller input;
a forward-only render over its bins identical to one over the workspace
bins; the host-side refusals (scratch too small, persistent launch)."""
import sys

import numpy as np
import pytest
import torch

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
    N.load()
    return torch.device("cuda:0")


def _bins(n_tiles, capacity, dev):
    tile_start = torch.full((n_tiles + 1,), -1, dtype=torch.int32, device=dev)
    sorted_ = torch.full((max(capacity, 1),), -1, dtype=torch.int32, device=dev)
    status = torch.zeros(8, dtype=torch.int64, device=dev)
    return tile_start, sorted_, status


def _compare(model, cam, width, height, dev, what):
    planes = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in I.plain_planes(model).items()}
    st = R.Settings(width, height, flags=N.FLAG_FWD_ONLY)
    rnd = R.Renderer(st, capacity=1 << 23)
    jobs = R.Jobs.single(model.n)
    cams_t = R.camera_table([cam], dev)
    batch = rnd.make_batch(planes, None, R.edit_table([I.identity_edit(model)], dev), cams_t, jobs)
    say(f"{what}: {model.n} Gaussians, {width}x{height}: project + ivrgs_bin_sort (workspace)")
    proj, bins_ws = rnd.project_and_bin(batch)
    p = st.params()
    s = torch.cuda.current_stream().cuda_stream
    n_tiles = N.ivrgs_tiles_per_job(p) * jobs.n_jobs
    tile_start, sorted_, status = _bins(n_tiles, rnd.capacity, dev)
    bins_na = N.ivrgs_bins(tile_start.data_ptr(), sorted_.data_ptr(), rnd.capacity, status.data_ptr())
    say(f"{what}: ivrgs_bin_sort_noalloc")
    N.ivrgs_bin_sort_noalloc(batch, p, proj, bins_na, s)
    torch.cuda.synchronize()
    ref_start = rnd.tile_start[: n_tiles + 1].cpu()
    total = int(ref_start[-1])
    assert total > 0
    assert torch.equal(tile_start.cpu(), ref_start), what
    assert torch.equal(sorted_[:total].cpu(), rnd.sorted[:total].cpu()), what
    assert torch.equal(status[:2].cpu(), rnd.status[:2].cpu()), what
    assert int(status[1]) == 0

    # a forward-only render needs no workspace; over either bins it is the same
    rgba_ws = torch.empty((1, 4, height, width), dtype=torch.float32, device=dev)
    rgba_na = torch.full_like(rgba_ws, float("nan"))
    N.ivrgs_render_fwd(batch, p, proj, bins_ws, rgba_ws.data_ptr(), None, None, 0, s)
    N.ivrgs_render_fwd(batch, p, proj, bins_na, rgba_na.data_ptr(), None, None, 0, s)
    torch.cuda.synchronize()
    assert torch.equal(rgba_na, rgba_ws), what
    say(f"{what}: {total} pairs, lists and image identical")
    return batch, proj, p, s


def test_noalloc_bin_sort_matches_workspace_twice(dev):
    big = I.isosurface_model(200_000, 1234)
    cam = I.look_at((0.5, -4.0, 1.0), width=800, height=800)
    _compare(big, cam, 800, 800, dev, "call 1")
    # second call, smaller input, ragged image: the array keeps the first
    # call's contents, which must not leak into the result
    small = I.small_scene(9_000, 77, log_scale_mu=-3.5)
    cam2 = I.look_at((-1.0, -3.5, 0.8), width=200, height=136)
    _compare(small, cam2, 200, 136, dev, "call 2")


def test_noalloc_refusals(dev):
    model = I.small_scene(2_000, 5)
    cam = I.look_at((0.0, -4.0, 0.0), width=64, height=64)
    batch, proj, p, s = _compare(model, cam, 64, 64, dev, "refusals setup")
    lib = N.load()
    tile_start, sorted_, status = _bins(N.ivrgs_tiles_per_job(p), 1 << 16, dev)
    bins = N.ivrgs_bins(tile_start.data_ptr(), sorted_.data_ptr(), 1 << 16, status.data_ptr())
    pp = N.ivrgs_params.from_buffer_copy(p)
    pp.flags = N.FLAG_PERSISTENT
    assert lib.ivrgs_bin_sort_noalloc(N.ref(batch), N.ref(pp), N.ref(proj), N.ref(bins), s) == N.E_UNSUPPORTED
    # more records than the scratch holds: refused on the host, nothing launched
    big = N.ivrgs_batch.from_buffer_copy(batch)
    big.n_records = N.NOALLOC_SCRATCH_BYTES // 16
    big.max_job_count = int(big.n_records)
    assert lib.ivrgs_bin_sort_noalloc(N.ref(big), N.ref(p), N.ref(proj), N.ref(bins), s) == N.E_CAPACITY
    torch.cuda.synchronize()
    assert int(status[0]) == 0 and int(status[1]) == 0
    assert torch.all(tile_start.cpu() == -1)
