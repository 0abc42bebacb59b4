"""ctypes binding of libivrgs.so: the C ABI of include/ivrgs.h, same names.

Argument marshalling only; every step of the rasterizer runs in the HIP
kernels of the library.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libivrgs.so")

PLANES = ("mean", "log_scale", "quat", "opacity", "normal", "color", "shade")
PLANE_DIMS = (3, 3, 4, 1, 3, 3, 4)

OK, E_INVALID, E_SHAPE, E_CAPACITY, E_HIP, E_UNSUPPORTED = range(6)
DEV_E_CAPACITY = 1
FLAG_PERSISTENT = 1
FLAG_COUNT_EVAL = 2
FLAG_FWD_ONLY = 4
FLAG_DETERMINISTIC_BWD = 8
EXPORTS = ("ivrgs_workspace_size", "ivrgs_tiles_per_job", "ivrgs_compose", "ivrgs_project",
           "ivrgs_bin_sort", "ivrgs_render_fwd", "ivrgs_render_bwd", "ivrgs_struct_size",
           "ivrgs_status_string", "ivrgs_timing_enable", "ivrgs_timing_read",
           "ivrgs_cull_workspace_size", "ivrgs_cull", "ivrgs_compose_bwd", "ivrgs_light_bwd",
           "ivrgs_compose_dev", "ivrgs_explore_state_words", "ivrgs_explore_step",
           "ivrgs_vq_workspace_size", "ivrgs_vq_fit", "ivrgs_vq_assign", "ivrgs_vq_compose",
           "ivrgs_sh_color", "ivrgs_sh_color_bwd", "ivrgs_render_aux_fwd", "ivrgs_render_aux_bwd",
           "ivrgs_get_error", "ivrgs_ssim_workspace_size", "ivrgs_ssim_fwd", "ivrgs_ssim_bwd",
           "ivrgs_vq_fit_batch_workspace_size", "ivrgs_vq_fit_batch", "ivrgs_photometric_grad",
           "ivrgs_reg_workspace_size", "ivrgs_reg_fwd", "ivrgs_reg_bwd", "ivrgs_bin_sort_noalloc",
           "ivrgs_l1_workspace_size", "ivrgs_l1_fwd", "ivrgs_l1_bwd", "ivrgs_editable_attr_fwd",
           "ivrgs_editable_attr_bwd", "ivrgs_render_bwd_aux",
           "ivrgs_photometric_workspace_size", "ivrgs_photometric_fwd", "ivrgs_photometric_grad_dev",
           "ivrgs_render_fwd_aux")
NOALLOC_SCRATCH_BYTES = 64 << 20
TIMING_KINDS = ("project", "tile_count", "scatter", "depth_sort", "render_fwd", "render_bwd",
                "project_bwd", "compose", "fill", "cull", "edit_bwd", "vq", "sh", "aux")


class ivrgs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in PLANES] + [("model_id", C.c_void_p)]


ivrgs_gaussians_mut = ivrgs_gaussians


class ivrgs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class ivrgs_model_edit(C.Structure):
    _fields_ = [("palette", C.c_float * 3), ("opacity_scale", C.c_float),
                ("shade_scale", C.c_float * 4), ("shade_bias", C.c_float * 4),
                ("light_dir", C.c_float * 3), ("headlight", C.c_int32)]


class ivrgs_job(C.Structure):
    _fields_ = [("camera", C.c_int32), ("gauss_begin", C.c_int32), ("gauss_count", C.c_int32),
                ("rec_begin", C.c_int32)]


class ivrgs_batch(C.Structure):
    _fields_ = [("g", ivrgs_gaussians), ("gauss_index", C.c_void_p), ("edits", C.c_void_p),
                ("n_models", C.c_int32), ("cameras", C.c_void_p), ("jobs", C.c_void_p),
                ("n_jobs", C.c_int32), ("max_job_count", C.c_int32), ("n_records", C.c_int64)]


class ivrgs_params(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("T_min", C.c_float),
                ("lowpass", C.c_float), ("z_near", C.c_float), ("bg", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32), ("tile", C.c_int32),
                ("flags", C.c_uint32), ("fwd_px", C.c_int32), ("bwd_px", C.c_int32),
                ("sort_chunk", C.c_int32), ("persist_per_cu", C.c_int32)]


class ivrgs_projected(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("rect", C.c_void_p), ("depth", C.c_void_p), ("nonfinite", C.c_void_p)]


class ivrgs_bins(C.Structure):
    _fields_ = [("tile_start", C.c_void_p), ("sorted", C.c_void_p), ("capacity", C.c_int64),
                ("status", C.c_void_p)]


class ivrgs_culler(C.Structure):
    _fields_ = [("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p),
                ("w3", C.c_void_p), ("b3", C.c_float), ("threshold", C.c_float)]


class ivrgs_explore_opts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("learn", C.c_uint32)]


class ivrgs_vq_model(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("normal", C.c_void_p), ("index", C.c_void_p),
                ("codebook", C.c_void_p), ("k", C.c_int32)]


class ivrgs_vq_book(C.Structure):
    _fields_ = [("values", C.c_void_p), ("n", C.c_int64), ("codebook", C.c_void_p), ("index", C.c_void_p)]


class ivrgs_reg_maps(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("alpha", C.c_void_p), ("normal", C.c_void_p), ("delta_c", C.c_void_p),
                ("shade", C.c_void_p), ("target", C.c_void_p), ("opacity", C.c_void_p), ("n_gauss", C.c_int64),
                ("height", C.c_int32), ("width", C.c_int32)]


STRUCTS = (ivrgs_gaussians, ivrgs_camera, ivrgs_model_edit, ivrgs_job, ivrgs_batch,
           ivrgs_params, ivrgs_projected, ivrgs_bins, ivrgs_culler, ivrgs_explore_opts, ivrgs_vq_model,
           ivrgs_vq_book, ivrgs_reg_maps)

_lib = None


class IvrgsError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise IvrgsError(f"{path} is missing: build it with "
                         f"`python -m paper_2504_17954_amd.build` (no CPU fallback exists)")
    # torch ships its own HIP runtime under the soname the library links
    # against; loading torch first makes the loader reuse that runtime, so
    # the library and torch's allocations share one.  Loaded the other way
    # round, the system runtime sits under torch and launches fail.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.ivrgs_workspace_size.argtypes = [P, P, C.c_int64]
    lib.ivrgs_workspace_size.restype = C.c_size_t
    lib.ivrgs_tiles_per_job.argtypes = [P]
    lib.ivrgs_tiles_per_job.restype = C.c_int32
    lib.ivrgs_compose.argtypes = [P, C.c_int32, P, P, P]
    lib.ivrgs_project.argtypes = [P, P, P, P]
    lib.ivrgs_bin_sort.argtypes = [P, P, P, P, P, C.c_size_t, P]
    lib.ivrgs_bin_sort_noalloc.argtypes = [P, P, P, P, P]
    lib.ivrgs_bin_sort_noalloc.restype = C.c_int
    lib.ivrgs_render_fwd.argtypes = [P, P, P, P, P, P, P, C.c_size_t, P]
    lib.ivrgs_render_bwd.argtypes = [P, P, P, P, P, P, P, P, C.c_size_t, P]
    for f in ("ivrgs_compose", "ivrgs_project", "ivrgs_bin_sort", "ivrgs_render_fwd",
              "ivrgs_render_bwd"):
        getattr(lib, f).restype = C.c_int
    lib.ivrgs_struct_size.argtypes = [C.c_int32]
    lib.ivrgs_struct_size.restype = C.c_int32
    lib.ivrgs_status_string.argtypes = [C.c_int]
    lib.ivrgs_status_string.restype = C.c_char_p
    lib.ivrgs_cull_workspace_size.argtypes = [C.c_int64]
    lib.ivrgs_cull_workspace_size.restype = C.c_size_t
    lib.ivrgs_cull.argtypes = [P, P, C.c_int32, P, P, P, C.c_int32, P, P, C.c_size_t, P]
    lib.ivrgs_cull.restype = C.c_int
    lib.ivrgs_compose_bwd.argtypes = [P, C.c_int32, P, P, P]
    lib.ivrgs_compose_bwd.restype = C.c_int
    lib.ivrgs_light_bwd.argtypes = [P, P, P, P, P, C.c_size_t, P]
    lib.ivrgs_light_bwd.restype = C.c_int
    lib.ivrgs_compose_dev.argtypes = [P, C.c_int32, P, P, P]
    lib.ivrgs_compose_dev.restype = C.c_int
    lib.ivrgs_explore_state_words.argtypes = [C.c_int32]
    lib.ivrgs_explore_state_words.restype = C.c_int64
    lib.ivrgs_explore_step.argtypes = [P, P, C.c_int32, P, P, P, P]
    lib.ivrgs_explore_step.restype = C.c_int
    lib.ivrgs_vq_workspace_size.argtypes = [C.c_int64, C.c_int32]
    lib.ivrgs_vq_workspace_size.restype = C.c_size_t
    lib.ivrgs_vq_fit.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P, P, P, C.c_size_t, P]
    lib.ivrgs_vq_fit.restype = C.c_int
    lib.ivrgs_vq_fit_batch_workspace_size.argtypes = [P, C.c_int32, C.c_int32]
    lib.ivrgs_vq_fit_batch_workspace_size.restype = C.c_size_t
    lib.ivrgs_vq_fit_batch.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, C.c_size_t, P]
    lib.ivrgs_vq_fit_batch.restype = C.c_int
    lib.ivrgs_vq_assign.argtypes = [P, C.c_int64, P, C.c_int32, P, P]
    lib.ivrgs_vq_assign.restype = C.c_int
    lib.ivrgs_vq_compose.argtypes = [P, C.c_int32, P, P, P]
    lib.ivrgs_vq_compose.restype = C.c_int
    lib.ivrgs_sh_color.argtypes = [P, C.c_int32, P, C.c_int64, P, P, P]
    lib.ivrgs_sh_color.restype = C.c_int
    lib.ivrgs_sh_color_bwd.argtypes = [P, C.c_int32, P, C.c_int64, P, P, P, P, P]
    lib.ivrgs_sh_color_bwd.restype = C.c_int
    lib.ivrgs_render_aux_fwd.argtypes = [P, P, P, P, P, C.c_int32, P, P]
    lib.ivrgs_render_aux_fwd.restype = C.c_int
    lib.ivrgs_render_aux_bwd.argtypes = [P, P, P, P, P, C.c_int32, P, P, P, P, P, C.c_size_t, P]
    lib.ivrgs_render_aux_bwd.restype = C.c_int
    lib.ivrgs_render_fwd_aux.argtypes = [P, P, P, P, P, C.c_int32, P, P, P, C.c_size_t, P]
    lib.ivrgs_render_fwd_aux.restype = C.c_int
    lib.ivrgs_render_bwd_aux.argtypes = [P, P, P, P, P, P, P, C.c_int32, P, P, P, P, P, C.c_size_t, P]
    lib.ivrgs_render_bwd_aux.restype = C.c_int
    lib.ivrgs_editable_attr_fwd.argtypes = [P, P, P, C.c_int64, P, P]
    lib.ivrgs_editable_attr_fwd.restype = C.c_int
    lib.ivrgs_editable_attr_bwd.argtypes = [P, C.c_int64, P, P, P, P, P]
    lib.ivrgs_editable_attr_bwd.restype = C.c_int
    I32 = C.c_int32
    lib.ivrgs_ssim_workspace_size.argtypes = [I32, I32, I32]
    lib.ivrgs_ssim_workspace_size.restype = C.c_size_t
    lib.ivrgs_ssim_fwd.argtypes = [P, P, I32, I32, I32, P, P, C.c_size_t, P]
    lib.ivrgs_ssim_fwd.restype = C.c_int
    lib.ivrgs_ssim_bwd.argtypes = [P, P, I32, I32, I32, P, P, P, C.c_size_t, P]
    lib.ivrgs_ssim_bwd.restype = C.c_int
    lib.ivrgs_photometric_grad.argtypes = [P, P, I32, I32, I32, C.c_float, P, P, C.c_size_t, P]
    lib.ivrgs_photometric_grad.restype = C.c_int
    lib.ivrgs_photometric_workspace_size.argtypes = [I32, I32, I32]
    lib.ivrgs_photometric_workspace_size.restype = C.c_size_t
    lib.ivrgs_photometric_fwd.argtypes = [P, P, I32, I32, I32, P, P, C.c_size_t, P]
    lib.ivrgs_photometric_fwd.restype = C.c_int
    lib.ivrgs_photometric_grad_dev.argtypes = [P, P, I32, I32, I32, P, P, P, C.c_size_t, P]
    lib.ivrgs_photometric_grad_dev.restype = C.c_int
    lib.ivrgs_l1_workspace_size.argtypes = [C.c_int64]
    lib.ivrgs_l1_workspace_size.restype = C.c_size_t
    lib.ivrgs_l1_fwd.argtypes = [P, P, C.c_int64, P, P, C.c_size_t, P]
    lib.ivrgs_l1_fwd.restype = C.c_int
    lib.ivrgs_l1_bwd.argtypes = [P, P, C.c_int64, P, P, P]
    lib.ivrgs_l1_bwd.restype = C.c_int
    lib.ivrgs_reg_workspace_size.argtypes = [P]
    lib.ivrgs_reg_workspace_size.restype = C.c_size_t
    lib.ivrgs_reg_fwd.argtypes = [P, P, P, P, P, C.c_size_t, P]
    lib.ivrgs_reg_fwd.restype = C.c_int
    lib.ivrgs_reg_bwd.argtypes = [P, P, P, P, P, P, P, P, P, P]
    lib.ivrgs_reg_bwd.restype = C.c_int
    lib.ivrgs_get_error.argtypes = [P, P, P, P]
    lib.ivrgs_get_error.restype = C.c_int
    lib.ivrgs_timing_enable.argtypes = [C.c_uint32]
    lib.ivrgs_timing_enable.restype = None
    lib.ivrgs_timing_read.argtypes = [P, P]
    lib.ivrgs_timing_read.restype = C.c_int32
    _lib = lib
    return lib


def check(status: int, what: str):
    if status != OK:
        msg = load().ivrgs_status_string(status).decode()
        raise IvrgsError(f"{what}: {msg} (status {status})")


def ref(x):
    return C.cast(C.byref(x), C.c_void_p)


def ivrgs_workspace_size(batch, params, capacity: int) -> int:
    return int(load().ivrgs_workspace_size(ref(batch), ref(params), C.c_int64(capacity)))


def ivrgs_tiles_per_job(params) -> int:
    return int(load().ivrgs_tiles_per_job(ref(params)))


def ivrgs_compose(models, n_models: int, edits, out, stream):
    arr_m = (ivrgs_gaussians * n_models)(*models)
    arr_e = (ivrgs_model_edit * n_models)(*edits)
    check(load().ivrgs_compose(C.cast(arr_m, C.c_void_p), n_models, C.cast(arr_e, C.c_void_p),
                               ref(out), stream), "ivrgs_compose")


def ivrgs_compose_bwd(models, n_models: int, grads, out_ptr, stream):
    arr_m = (ivrgs_gaussians * n_models)(*models)
    check(load().ivrgs_compose_bwd(C.cast(arr_m, C.c_void_p), n_models, ref(grads), out_ptr, stream),
          "ivrgs_compose_bwd")


def ivrgs_light_bwd(batch, params, proj, out_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_light_bwd(ref(batch), ref(params), ref(proj), out_ptr, ws_ptr, ws_bytes, stream),
          "ivrgs_light_bwd")


def ivrgs_compose_dev(models, n_models: int, edits_ptr, out, stream):
    arr_m = (ivrgs_gaussians * n_models)(*models)
    check(load().ivrgs_compose_dev(C.cast(arr_m, C.c_void_p), n_models, edits_ptr, ref(out), stream),
          "ivrgs_compose_dev")


def ivrgs_explore_state_words(n_models: int) -> int:
    return int(load().ivrgs_explore_state_words(n_models))


def ivrgs_explore_step(edit_grad_ptr, light_grad_ptr, n_models: int, opts, state_ptr, edits_ptr, stream):
    check(load().ivrgs_explore_step(edit_grad_ptr, light_grad_ptr, n_models, ref(opts), state_ptr, edits_ptr,
                                    stream), "ivrgs_explore_step")


def ivrgs_vq_workspace_size(n: int, k: int) -> int:
    return int(load().ivrgs_vq_workspace_size(C.c_int64(n), k))


def _book_array(books):
    arr = (ivrgs_vq_book * max(len(books), 1))(*books)
    return arr, C.cast(arr, C.c_void_p)


def ivrgs_vq_fit_batch_workspace_size(books, k: int) -> int:
    arr, ptr = _book_array(books)
    return int(load().ivrgs_vq_fit_batch_workspace_size(ptr, len(books), k))


def ivrgs_vq_fit_batch(books, k: int, iters: int, ws_ptr, ws_bytes, stream):
    arr, ptr = _book_array(books)
    check(load().ivrgs_vq_fit_batch(ptr, len(books), k, iters, ws_ptr, ws_bytes, stream), "ivrgs_vq_fit_batch")


def ivrgs_vq_fit(values_ptr, n: int, k: int, iters: int, codebook_ptr, index_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_vq_fit(values_ptr, C.c_int64(n), k, iters, codebook_ptr, index_ptr, ws_ptr, ws_bytes,
                              stream), "ivrgs_vq_fit")


def ivrgs_vq_assign(values_ptr, n: int, codebook_ptr, k: int, index_ptr, stream):
    check(load().ivrgs_vq_assign(values_ptr, C.c_int64(n), codebook_ptr, k, index_ptr, stream), "ivrgs_vq_assign")


def ivrgs_vq_compose(models, n_models: int, edits, out, stream):
    arr_m = (ivrgs_vq_model * n_models)(*models)
    arr_e = (ivrgs_model_edit * n_models)(*edits)
    check(load().ivrgs_vq_compose(C.cast(arr_m, C.c_void_p), n_models, C.cast(arr_e, C.c_void_p), ref(out),
                                  stream), "ivrgs_vq_compose")


def ivrgs_sh_color(sh_ptr, degree: int, mean_ptr, n: int, camera, color_ptr, stream):
    check(load().ivrgs_sh_color(sh_ptr, degree, mean_ptr, C.c_int64(n), ref(camera), color_ptr, stream),
          "ivrgs_sh_color")


def ivrgs_sh_color_bwd(sh_ptr, degree: int, mean_ptr, n: int, camera, grad_color_ptr, grad_sh_ptr, grad_mean_ptr,
                       stream):
    check(load().ivrgs_sh_color_bwd(sh_ptr, degree, mean_ptr, C.c_int64(n), ref(camera), grad_color_ptr,
                                    grad_sh_ptr, grad_mean_ptr, stream), "ivrgs_sh_color_bwd")


def ivrgs_render_aux_fwd(batch, params, proj, bins, attr_ptr, n_attr: int, aux_ptr, stream):
    check(load().ivrgs_render_aux_fwd(ref(batch), ref(params), ref(proj), ref(bins), attr_ptr, n_attr, aux_ptr,
                                      stream), "ivrgs_render_aux_fwd")


def ivrgs_render_aux_bwd(batch, params, proj, bins, attr_ptr, n_attr: int, aux_ptr, grad_aux_ptr, grad_attr_ptr,
                         grads, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_render_aux_bwd(ref(batch), ref(params), ref(proj), ref(bins), attr_ptr, n_attr, aux_ptr,
                                      grad_aux_ptr, grad_attr_ptr, ref(grads), ws_ptr, ws_bytes, stream),
          "ivrgs_render_aux_bwd")


def ivrgs_render_fwd_aux(batch, params, proj, bins, attr_ptr, n_attr: int, rgba_ptr, aux_ptr, ws_ptr, ws_bytes,
                         stream):
    check(load().ivrgs_render_fwd_aux(ref(batch), ref(params), ref(proj), ref(bins), attr_ptr, n_attr, rgba_ptr,
                                      aux_ptr, ws_ptr, ws_bytes, stream), "ivrgs_render_fwd_aux")


def ivrgs_render_bwd_aux(batch, params, proj, bins, rgba_ptr, dl_ptr, attr_ptr, n_attr: int, aux_ptr, grad_aux_ptr,
                         grad_attr_ptr, grads, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_render_bwd_aux(ref(batch), ref(params), ref(proj), ref(bins), rgba_ptr, dl_ptr, attr_ptr,
                                      n_attr, aux_ptr, grad_aux_ptr, grad_attr_ptr, ref(grads), ws_ptr, ws_bytes,
                                      stream), "ivrgs_render_bwd_aux")


def ivrgs_editable_attr_fwd(normal_ptr, color_ptr, shade_ptr, n: int, attr_ptr, stream):
    check(load().ivrgs_editable_attr_fwd(normal_ptr, color_ptr, shade_ptr, C.c_int64(n), attr_ptr, stream),
          "ivrgs_editable_attr_fwd")


def ivrgs_editable_attr_bwd(normal_ptr, n: int, grad_attr_ptr, grad_normal_ptr, grad_color_ptr, grad_shade_ptr,
                            stream):
    check(load().ivrgs_editable_attr_bwd(normal_ptr, C.c_int64(n), grad_attr_ptr, grad_normal_ptr, grad_color_ptr,
                                         grad_shade_ptr, stream), "ivrgs_editable_attr_bwd")


def ivrgs_get_error(bins, stream) -> tuple[int, int]:
    """(device error bits, pairs required) over every bin sort on these bins
    since the previous call: the OR of their bits and the largest count;
    clears the sticky words (waits for the stream)."""
    err, need = C.c_int64(0), C.c_int64(0)
    check(load().ivrgs_get_error(ref(bins), stream, C.cast(C.byref(err), C.c_void_p),
                                 C.cast(C.byref(need), C.c_void_p)), "ivrgs_get_error")
    return int(err.value), int(need.value)


def ivrgs_ssim_workspace_size(channels: int, height: int, width: int) -> int:
    return int(load().ivrgs_ssim_workspace_size(channels, height, width))


def ivrgs_ssim_fwd(x_ptr, y_ptr, channels: int, height: int, width: int, out_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_ssim_fwd(x_ptr, y_ptr, channels, height, width, out_ptr, ws_ptr, ws_bytes, stream),
          "ivrgs_ssim_fwd")


def ivrgs_ssim_bwd(x_ptr, y_ptr, channels: int, height: int, width: int, grad_mean_ptr, grad_x_ptr, ws_ptr,
                   ws_bytes, stream):
    check(load().ivrgs_ssim_bwd(x_ptr, y_ptr, channels, height, width, grad_mean_ptr, grad_x_ptr, ws_ptr,
                                ws_bytes, stream), "ivrgs_ssim_bwd")


def ivrgs_photometric_workspace_size(channels: int, height: int, width: int) -> int:
    return int(load().ivrgs_photometric_workspace_size(channels, height, width))


def ivrgs_photometric_fwd(x_ptr, y_ptr, channels: int, height: int, width: int, out_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_photometric_fwd(x_ptr, y_ptr, channels, height, width, out_ptr, ws_ptr, ws_bytes, stream),
          "ivrgs_photometric_fwd")


def ivrgs_photometric_grad_dev(x_ptr, y_ptr, channels: int, height: int, width: int, weights_ptr, grad_x_ptr,
                               ws_ptr, ws_bytes, stream):
    check(load().ivrgs_photometric_grad_dev(x_ptr, y_ptr, channels, height, width, weights_ptr, grad_x_ptr, ws_ptr,
                                            ws_bytes, stream), "ivrgs_photometric_grad_dev")


def ivrgs_photometric_grad(x_ptr, y_ptr, channels: int, height: int, width: int, lam: float, grad_x_ptr,
                           ws_ptr, ws_bytes, stream):
    check(load().ivrgs_photometric_grad(x_ptr, y_ptr, channels, height, width, lam, grad_x_ptr, ws_ptr,
                                        ws_bytes, stream), "ivrgs_photometric_grad")


def ivrgs_l1_workspace_size(n: int) -> int:
    return int(load().ivrgs_l1_workspace_size(n))


def ivrgs_l1_fwd(x_ptr, y_ptr, n: int, out_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_l1_fwd(x_ptr, y_ptr, n, out_ptr, ws_ptr, ws_bytes, stream), "ivrgs_l1_fwd")


def ivrgs_l1_bwd(x_ptr, y_ptr, n: int, grad_mean_ptr, grad_x_ptr, stream):
    check(load().ivrgs_l1_bwd(x_ptr, y_ptr, n, grad_mean_ptr, grad_x_ptr, stream), "ivrgs_l1_bwd")


def ivrgs_reg_workspace_size(maps) -> int:
    return int(load().ivrgs_reg_workspace_size(ref(maps)))


def ivrgs_reg_fwd(maps, camera, terms_ptr, pseudo_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_reg_fwd(ref(maps), ref(camera), terms_ptr, pseudo_ptr, ws_ptr, ws_bytes, stream),
          "ivrgs_reg_fwd")


def ivrgs_reg_bwd(maps, camera, terms_ptr, grad_terms_ptr, g_normal_ptr, g_dc_ptr, g_shade_ptr, g_op_ptr, stream,
                  g_depth_ptr=None):
    check(load().ivrgs_reg_bwd(ref(maps), ref(camera), terms_ptr, grad_terms_ptr, g_normal_ptr, g_dc_ptr,
                               g_shade_ptr, g_op_ptr, g_depth_ptr, stream), "ivrgs_reg_bwd")


def ivrgs_project(batch, params, proj, stream):
    check(load().ivrgs_project(ref(batch), ref(params), ref(proj), stream), "ivrgs_project")


def ivrgs_bin_sort(batch, params, proj, bins, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_bin_sort(ref(batch), ref(params), ref(proj), ref(bins), ws_ptr, ws_bytes,
                                stream), "ivrgs_bin_sort")


def ivrgs_bin_sort_noalloc(batch, params, proj, bins, stream):
    check(load().ivrgs_bin_sort_noalloc(ref(batch), ref(params), ref(proj), ref(bins), stream),
          "ivrgs_bin_sort_noalloc")


def ivrgs_render_fwd(batch, params, proj, bins, rgba_ptr, maxw_ptr, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_render_fwd(ref(batch), ref(params), ref(proj), ref(bins), rgba_ptr, maxw_ptr,
                                  ws_ptr, ws_bytes, stream), "ivrgs_render_fwd")


def ivrgs_render_bwd(batch, params, proj, bins, rgba_ptr, dl_ptr, grads, ws_ptr, ws_bytes, stream):
    check(load().ivrgs_render_bwd(ref(batch), ref(params), ref(proj), ref(bins), rgba_ptr, dl_ptr,
                                  ref(grads), ws_ptr, ws_bytes, stream), "ivrgs_render_bwd")


def ivrgs_struct_size(which: int) -> int:
    return int(load().ivrgs_struct_size(which))


TIMING_ALL = (1 << len(TIMING_KINDS)) - 1


def ivrgs_timing_enable(kinds=True):
    """Time the listed kernel kinds (names or a bit mask; True = all, False =
    off) and clear the sums."""
    if kinds is True:
        mask = TIMING_ALL
    elif kinds is False or kinds is None:
        mask = 0
    elif isinstance(kinds, int):
        mask = kinds
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << TIMING_KINDS.index(k)
    load().ivrgs_timing_enable(mask)


def ivrgs_timing_read() -> dict:
    """{kernel kind: (total ms, launches)} since the last enable (syncs)."""
    import numpy as np
    ms = np.zeros(len(TIMING_KINDS), np.float64)
    n = np.zeros(len(TIMING_KINDS), np.int64)
    load().ivrgs_timing_read(ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(TIMING_KINDS)}


def ivrgs_cull_workspace_size(n: int) -> int:
    return int(load().ivrgs_cull_workspace_size(C.c_int64(n)))


def ivrgs_cull(g, cams_ptr, camera: int, mlp, out_index_ptr, jobs_ptr, job: int, logit_ptr, ws_ptr, ws_bytes,
               stream):
    check(load().ivrgs_cull(ref(g), cams_ptr, camera, ref(mlp), out_index_ptr, jobs_ptr, job, logit_ptr, ws_ptr,
                            ws_bytes, stream), "ivrgs_cull")
